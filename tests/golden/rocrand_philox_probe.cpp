// Black-box reference for the oracle's Philox4x32-10: runs rocRAND's host
// engine (an independent implementation) for each (key, counter) read from
// stdin and prints the first block of four 32-bit outputs.
// Input lines: k0 k1 c0 c1 c2 c3 (decimal).  Output lines: o0 o1 o2 o3.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long subsequence = ((unsigned long long)c3 << 32) | c2;
        unsigned long long offset = (((unsigned long long)c1 << 32) | c0) * 4ull;
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
