// rewl_kernels.hip -- HIP kernels of replica-exchange Wang-Landau sampling for
// gfx950: one wavefront per walker, the walker's configuration, ln g~, H and
// visited flags staged in LDS for a whole segment.
//
// Paper references (Perera et al., arXiv:1411.4212):
//   Model, Eq. 1                H = -sum_{i<j} J_ij S_i.S_j, N = 2 L^3 on bcc
//   Sec. original WL            acceptance min(1, g~(E_A)/g~(E_B)); g~ *= f and
//                               H += 1 at the state after the move; flat when
//                               H(E) >= p <H>; f -> sqrt(f)
//   Sec. parallel scheme        windows with overlap o, m walkers per window,
//                               exchange acceptance min(1, g_i(E_A) g_j(E_B) /
//                               (g_i(E_B) g_j(E_A)))
//   Sec. simulation details     random site, arbitrary new direction; an
//                               exchange needs both replicas in the overlap
#include <hip/hip_runtime.h>

#include "rewl_device.h"
#include "rewl_internal.h"

namespace rewl {

using namespace dev;

enum { M_DET = REWL_MODE_FP64_DET, M_F64 = REWL_MODE_FP64, M_F32 = REWL_MODE_FP32_DE };

// ------------------------------------------------------------------ spins
// LDS / HBM spin element: double4 for the FP64 modes, float4 for FP32.
template <int MODE>
struct Spin;
template <>
struct Spin<M_DET> {
    using T = double;
    using V = double4;
};
template <>
struct Spin<M_F64> {
    using T = double;
    using V = double4;
};
template <>
struct Spin<M_F32> {
    using T = float;
    using V = float4;
};

struct WalkerLds {
    void *spins;
    double *lng;
    uint32_t *H;
    uint8_t *vis;
};

__device__ __forceinline__ WalkerLds carve_lds(unsigned char *base, const KArgs &a, int slot)
{
    const size_t per = (size_t)a.lds_spins_bytes + (size_t)a.lds_bins * 13u;
    const size_t per_al = (per + 15) & ~(size_t)15;
    unsigned char *p = base + per_al * (size_t)slot;
    WalkerLds w;
    w.spins = p;
    w.lng = (double *)(p + a.lds_spins_bytes);
    w.H = (uint32_t *)(p + a.lds_spins_bytes + (size_t)a.lds_bins * 8u);
    w.vis = (uint8_t *)(p + a.lds_spins_bytes + (size_t)a.lds_bins * 12u);
    return w;
}

// Per-wave lattice context: what a lane needs to find its neighbour slots.
template <int MODE>
struct LatCtx {
    int N, L, z;
    float invL;
    int lattice;
    // bcc: this lane's slots (lane, lane + 64)
    BccSlot s0, s1;
    bool has0, has1;
    // table lattice
    const int32_t *deg;
    const int32_t *nbr;
    const double *J;
    const BccSlot *slots;   // full slot table (DET sequential walk)
};

template <int MODE>
__device__ __forceinline__ void load_latctx(LatCtx<MODE> &c, const InstDesc &I, const KArgs &a, int lane)
{
    c.N = I.N;
    c.L = I.L;
    c.z = I.z;
    c.invL = I.L > 0 ? 1.0f / (float)I.L : 0.0f;
    c.lattice = I.lattice;
    c.slots = a.slots + I.slot_off;
    c.deg = a.tdeg ? a.tdeg + I.deg_off : nullptr;
    c.nbr = a.tnbr ? a.tnbr + I.tab_off : nullptr;
    c.J = a.tJ ? a.tJ + I.tab_off : nullptr;
    c.has0 = lane < I.z;
    c.has1 = lane + kWave < I.z;
    if (I.lattice == LAT_BCC) {
        BccSlot zero{};
        c.s0 = c.has0 ? c.slots[lane] : zero;
        c.s1 = c.has1 ? c.slots[lane + kWave] : zero;
    }
}

// Local field h_i = sum_j J_ij S_j.
//   DET: sequential over the neighbour list (list order), FP64, identical in
//        every lane.
//   F64 / F32: lane l gathers slots l and l+64, multiplies by J, and the
//        wavefront sums the partial fields.
template <int MODE>
__device__ __forceinline__ void local_field(const LatCtx<MODE> &c, const typename Spin<MODE>::V *S,
                                            int site, typename Spin<MODE>::T &hx,
                                            typename Spin<MODE>::T &hy, typename Spin<MODE>::T &hz)
{
    using T = typename Spin<MODE>::T;
    using V = typename Spin<MODE>::V;
    if constexpr (MODE == M_DET) {
        double ax = 0.0, ay = 0.0, az = 0.0;
        if (c.lattice == LAT_BCC) {
            for (int k = 0; k < c.z; ++k) {
                const BccSlot sl = c.slots[k];
                const int j = bcc_neighbour(site, c.L, c.invL, sl);
                const V s = S[j];
                ax = ax + sl.Jd * s.x;
                ay = ay + sl.Jd * s.y;
                az = az + sl.Jd * s.z;
            }
        } else {
            const int d = c.deg[site];
            for (int k = 0; k < d; ++k) {
                const int j = c.nbr[(int64_t)site * c.z + k];
                const double Jv = c.J[(int64_t)site * c.z + k];
                const V s = S[j];
                ax = ax + Jv * s.x;
                ay = ay + Jv * s.y;
                az = az + Jv * s.z;
            }
        }
        hx = ax;
        hy = ay;
        hz = az;
    } else {
        T px = 0, py = 0, pz = 0;
        const int lane = __lane_id();
        if (c.lattice == LAT_BCC) {
            if (c.has0) {
                const int j = bcc_neighbour(site, c.L, c.invL, c.s0);
                const V s = S[j];
                const T Jv = (MODE == M_F32) ? (T)c.s0.Jf : (T)c.s0.Jd;
                px = Jv * s.x;
                py = Jv * s.y;
                pz = Jv * s.z;
            }
            if (c.has1) {
                const int j = bcc_neighbour(site, c.L, c.invL, c.s1);
                const V s = S[j];
                const T Jv = (MODE == M_F32) ? (T)c.s1.Jf : (T)c.s1.Jd;
                px += Jv * s.x;
                py += Jv * s.y;
                pz += Jv * s.z;
            }
        } else {
            const int d = c.deg[site];
            for (int k = lane; k < d; k += kWave) {
                const int j = c.nbr[(int64_t)site * c.z + k];
                const T Jv = (T)c.J[(int64_t)site * c.z + k];
                const V s = S[j];
                px += Jv * s.x;
                py += Jv * s.y;
                pz += Jv * s.z;
            }
        }
        if constexpr (MODE == M_F32) {
            hx = wave_sum_f(px);
            hy = wave_sum_f(py);
            hz = wave_sum_f(pz);
        } else {
            hx = wave_sum_d(px);
            hy = wave_sum_d(py);
            hz = wave_sum_d(pz);
        }
    }
}

// Full energy E = -1/2 sum_i S_i . h_i.
//   DET: sites in index order, each site's field in list order, FP64.
//   other modes: lanes take sites lane, lane+64, ..., FP64 accumulation,
//   wavefront sum.
template <int MODE>
__device__ double full_energy(const LatCtx<MODE> &c, const typename Spin<MODE>::V *S)
{
    using V = typename Spin<MODE>::V;
    if constexpr (MODE == M_DET) {
        double acc = 0.0;
        for (int i = 0; i < c.N; ++i) {
            double hx, hy, hz;
            local_field<MODE>(c, S, i, hx, hy, hz);
            const V s = S[i];
            acc = acc + ((s.x * hx + s.y * hy) + s.z * hz);
        }
        return -0.5 * acc;
    } else {
        const int lane = __lane_id();
        double acc = 0.0;
        for (int i = lane; i < c.N; i += kWave) {
            double hx = 0.0, hy = 0.0, hz = 0.0;
            if (c.lattice == LAT_BCC) {
                for (int k = 0; k < c.z; ++k) {
                    const BccSlot sl = c.slots[k];
                    const int j = bcc_neighbour(i, c.L, c.invL, sl);
                    const V s = S[j];
                    hx += sl.Jd * (double)s.x;
                    hy += sl.Jd * (double)s.y;
                    hz += sl.Jd * (double)s.z;
                }
            } else {
                const int d = c.deg[i];
                for (int k = 0; k < d; ++k) {
                    const int j = c.nbr[(int64_t)i * c.z + k];
                    const double Jv = c.J[(int64_t)i * c.z + k];
                    const V s = S[j];
                    hx += Jv * (double)s.x;
                    hy += Jv * (double)s.y;
                    hz += Jv * (double)s.z;
                }
            }
            const V s = S[i];
            acc += ((double)s.x * hx + (double)s.y * hy) + (double)s.z * hz;
        }
        return -0.5 * wave_sum_d(acc);
    }
}

// Proposal direction in the spin type of the mode.
template <int MODE>
__device__ __forceinline__ void propose(uint32_t seed, uint32_t stream, uint64_t n, uint32_t tag,
                                        typename Spin<MODE>::T &x, typename Spin<MODE>::T &y,
                                        typename Spin<MODE>::T &z)
{
    if constexpr (MODE == M_F32) {
        sphere_f(seed, stream, n, tag, x, y, z);
    } else {
        sphere_d(seed, stream, n, tag, x, y, z);
    }
}

// Energy change of S_i -> S' given h_i:  -(S' - S_i) . h_i.
template <int MODE>
__device__ __forceinline__ double delta_e(typename Spin<MODE>::T nx, typename Spin<MODE>::T ny,
                                          typename Spin<MODE>::T nz, const typename Spin<MODE>::V &s,
                                          typename Spin<MODE>::T hx, typename Spin<MODE>::T hy,
                                          typename Spin<MODE>::T hz)
{
    if constexpr (MODE == M_F32) {
        const float d = __builtin_fmaf(nz - s.z, hz, __builtin_fmaf(ny - s.y, hy, (nx - s.x) * hx));
        return -(double)d;
    } else {
        return -(((nx - s.x) * hx + (ny - s.y) * hy) + (nz - s.z) * hz);
    }
}

// Copy a walker's configuration between HBM and LDS (all lanes).
template <int MODE>
__device__ __forceinline__ void copy_spins(typename Spin<MODE>::V *dst, const typename Spin<MODE>::V *src,
                                           int N)
{
    for (int i = __lane_id(); i < N; i += kWave) dst[i] = src[i];
}

// ------------------------------------------------------------------ init
// Start configuration, its energy, and the drive into the window: moves are
// accepted when the new energy lies in the window or strictly closer to it.
template <int MODE>
__global__ void __launch_bounds__(256) init_kernel(KArgs a)
{
    using T = typename Spin<MODE>::T;
    using V = typename Spin<MODE>::V;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int wave = threadIdx.x / kWave;
    const int lane = __lane_id();
    const int w = blockIdx.x * a.walkers_per_block + wave;
    if (w >= a.n_walkers) return;
    const WalkerDesc wd = a.wdesc[w];
    const InstDesc I = a.inst[wd.inst];
    WalkerLds L = carve_lds(lds_raw, a, wave);
    V *S = (V *)L.spins;
    LatCtx<MODE> c;
    load_latctx<MODE>(c, I, a, lane);

    for (int i = lane; i < I.N; i += kWave) {
        double x, y, z;
        if (I.init_off >= 0) {
            const double *p = a.init_spins + I.init_off + 3 * (int64_t)i;
            x = p[0];
            y = p[1];
            z = p[2];
        } else {
            sphere_d(a.seed, wd.stream, (uint64_t)i, TAG_INIT_CONFIG, x, y, z);
        }
        V v;
        v.x = (T)x;
        v.y = (T)y;
        v.z = (T)z;
        v.w = (T)0;
        S[i] = v;
    }
    wave_sync();

    double E = full_energy<MODE>(c, S);
    const double lo = (double)wd.lo, hi = (double)wd.hi;
    auto dist = [&](double e) {
        const double x = (e - I.Emin) * I.inv_de;
        return x < lo ? lo - x : (x >= hi ? x - hi : 0.0);
    };
    double x0 = (E - I.Emin) * I.inv_de;
    bool inside = (x0 >= lo && x0 < hi);
    const uint64_t cap = (uint64_t)10000 * (uint64_t)I.N;
    for (uint64_t n = 0; !inside && n < cap; ++n) {
        const U4 r = draw(a.seed, wd.stream, n, 0u, TAG_INIT_SITE);
        const int i = pick_site(r.x, I.N);
        T nx, ny, nz;
        propose<MODE>(a.seed, wd.stream, n, TAG_INIT_SPHERE, nx, ny, nz);
        T hx, hy, hz;
        local_field<MODE>(c, S, i, hx, hy, hz);
        const V si = S[i];
        const double Eb = E + delta_e<MODE>(nx, ny, nz, si, hx, hy, hz);
        const double xb = (Eb - I.Emin) * I.inv_de;
        const bool in_b = (xb >= lo && xb < hi);
        if (in_b || dist(Eb) < dist(E)) {
            V v;
            v.x = nx;
            v.y = ny;
            v.z = nz;
            v.w = (T)0;
            S[i] = v;
            E = Eb;
            inside = in_b;
        }
    }
    wave_sync();
    V *G = (V *)a.spins + I.cfg_off + (int64_t)wd.local * I.N;
    copy_spins<MODE>(G, S, I.N);
    if (lane == 0) {
        WalkerState st{};
        st.E = E;
        st.lnf = I.lnf_init;
        st.max_drift = 0.0;
        const double x = (E - I.Emin) * I.inv_de;
        st.bin = inside ? (int)floor(x) : wd.lo;
        st.cfg = wd.local;
        st.iter = 0;
        st.done = 0;
        st.nvis = 0;
        st.status = inside ? 0 : REWL_EINIT;
        a.state[w] = st;
    }
}

// ------------------------------------------------------------------ sweep
// One segment of I.seg_len trial moves for every walker, then the resync
// when due and the flatness test with the ln f update.
template <int MODE>
__global__ void __launch_bounds__(256) sweep_kernel(KArgs a)
{
    using T = typename Spin<MODE>::T;
    using V = typename Spin<MODE>::V;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int wave = threadIdx.x / kWave;
    const int lane = __lane_id();
    const int w = blockIdx.x * a.walkers_per_block + wave;
    if (w >= a.n_walkers) return;
    const WalkerDesc wd = a.wdesc[w];
    if (a.ictl[wd.inst].done) return;
    const InstDesc I = a.inst[wd.inst];
    WalkerState st = a.state[w];
    if (st.status != 0) return;
    WalkerLds L = carve_lds(lds_raw, a, wave);
    V *S = (V *)L.spins;
    LatCtx<MODE> c;
    load_latctx<MODE>(c, I, a, lane);

    const int nb = wd.hi - wd.lo;
    V *G = (V *)a.spins + I.cfg_off + (int64_t)st.cfg * I.N;
    copy_spins<MODE>(S, G, I.N);
    double *glng = a.lng + wd.bin_off;
    uint32_t *gH = a.hist + wd.bin_off;
    uint8_t *gvis = a.vis + wd.bin_off;
    for (int j = lane; j < nb; j += kWave) {
        L.lng[j] = glng[j];
        L.H[j] = gH[j];
        L.vis[j] = gvis[j];
    }
    wave_sync();

    const double Emin = I.Emin, inv = I.inv_de;
    const double lo = (double)wd.lo, hi = (double)wd.hi;
    const int ilo = wd.lo;
    double E = st.E;
    int bin = st.bin;
    const double lnf = st.lnf;
    const bool frozen = st.done != 0;
    const bool discovering = (st.iter == 0) && !frozen;
    double cur = L.lng[bin - ilo];
    uint64_t n = st.attempts;
    const uint64_t n_end = n + (uint64_t)I.seg_len;
    uint64_t acc_count = 0, oow = 0;
    rewl_trace_rec *trace = a.trace ? a.trace + (int64_t)w * a.trace_cap : nullptr;

    for (; n < n_end; ++n) {
        const U4 r = draw(a.seed, wd.stream, n, 0u, TAG_SITE);
        const int i = pick_site(r.x, I.N);
        const double u = u53(r.y, r.z);
        T nx, ny, nz;
        propose<MODE>(a.seed, wd.stream, n, TAG_SPHERE, nx, ny, nz);
        T hx, hy, hz;
        local_field<MODE>(c, S, i, hx, hy, hz);
        const V si = S[i];
        const double Eb = E + delta_e<MODE>(nx, ny, nz, si, hx, hy, hz);
        const double xb = (Eb - Emin) * inv;
        int bb = -1;
        bool outside = true;
        if (xb >= lo && xb < hi) {
            bb = (int)floor(xb);
            outside = false;
            if (!L.vis[bb - ilo]) {
                // first entry into a bin: during the first iteration its
                // initial guess is the current bin's estimate and H restarts;
                // afterwards the range is fixed
                if (discovering) {
                    L.lng[bb - ilo] = cur;
                    for (int j = lane; j < nb; j += kWave) L.H[j] = 0u;
                } else {
                    bb = -1;
                    outside = true;
                }
            }
        }
        bool accept = false;
        double lnb = 0.0;
        if (bb >= 0) {
            lnb = L.lng[bb - ilo];
            const double lr = cur - lnb;
            accept = (lr >= 0.0) || (u < exp_det(lr));
        }
        oow += outside ? 1u : 0u;
        if (accept) {
            V v;
            v.x = nx;
            v.y = ny;
            v.z = nz;
            v.w = (T)0;
            S[i] = v;
            E = Eb;
            bin = bb;
            cur = lnb;
            ++acc_count;
        }
        const int jb = bin - ilo;
        if (!frozen) {
            cur = cur + lnf;
            L.lng[jb] = cur;
            L.H[jb] = L.H[jb] + 1u;
        }
        L.vis[jb] = 1;
        if (trace && n < (uint64_t)a.trace_cap && lane == 0) {
            rewl_trace_rec rec;
            rec.site = (uint32_t)i;
            rec.flags = (accept ? 1u : 0u) | (outside ? 2u : 0u);
            rec.E = E;
            rec.bin = bin;
            rec.attempt_lo = (uint32_t)n;
            trace[n] = rec;
        }
    }
    wave_sync();

    // resync: recompute E from scratch when the attempt count crossed a
    // multiple of the resync interval during this segment
    if (I.resync > 0 && (n / (uint64_t)I.resync) != (st.attempts / (uint64_t)I.resync)) {
        const double ef = full_energy<MODE>(c, S);
        const double d = fabs(ef - E);
        if (d > st.max_drift) st.max_drift = d;
        E = ef;
        const double x = (ef - Emin) * inv;
        bin = x < lo ? wd.lo : (x >= hi ? wd.hi - 1 : (int)floor(x));
    }

    // flatness over visited bins (integer test), then the ln f update
    int nvis = 0;
    unsigned long long sumH = 0;
    uint32_t minH = 0xFFFFFFFFu;
    for (int j = lane; j < nb; j += kWave) {
        if (L.vis[j]) {
            nvis += 1;
            sumH += L.H[j];
            minH = L.H[j] < minH ? L.H[j] : minH;
        }
    }
    nvis = wave_sum_i(nvis);
    sumH = wave_sum_u64(sumH);
    minH = wave_min_u32(minH);
    if (!frozen) {
        bool flat = false;
        if (nvis > st.nvis) {
            flat = false;
        } else if (nvis > 0 && sumH > 0) {
            flat = (unsigned long long)I.flat_den * (unsigned long long)minH * (unsigned long long)nvis >=
                   (unsigned long long)I.flat_num * sumH;
        }
        st.nvis = nvis;
        if (flat) {
            if (st.lnf <= I.lnf_final) {
                st.done = 1;
            } else {
                st.lnf = st.lnf * 0.5;
                st.iter += 1;
                for (int j = lane; j < nb; j += kWave) L.H[j] = 0u;
            }
        }
    } else {
        st.nvis = nvis;
    }
    wave_sync();

    copy_spins<MODE>(G, S, I.N);
    for (int j = lane; j < nb; j += kWave) {
        glng[j] = L.lng[j];
        gH[j] = L.H[j];
        gvis[j] = L.vis[j];
    }
    if (lane == 0) {
        st.E = E;
        st.bin = bin;
        st.attempts = n;
        st.accepts += acc_count;
        st.oow += oow;
        if (!isfinite(E) || !isfinite(cur)) st.status = REWL_ENUMERIC;
        a.state[w] = st;
    }
}

// ------------------------------------------------------------------ exchange
// One replica-exchange step for every instance not yet done: window pairs
// (k, k+1) with k of the parity of the step counter; the m walkers of window
// k are paired with those of window k+1 by a Fisher-Yates permutation; a pair
// may swap only if each energy lies in the other's window on a bin that
// walker has visited; the swap moves configuration, energy and bin.  Then
// the instance's done flag is recomputed.
__global__ void __launch_bounds__(64) exchange_kernel(KArgs a)
{
    __shared__ int perm_all[kWave][REWL_MAX_WALKERS_PER_WINDOW];
    __shared__ int all_done;
    const int ii = blockIdx.x;
    if (ii >= a.n_inst) return;
    if (a.ictl[ii].done) return;
    const InstDesc I = a.inst[ii];
    const int tid = threadIdx.x;
    const uint64_t t = (uint64_t)a.t;
    const int m = I.m;
    int *perm = perm_all[tid];
    for (int k = (int)(t & 1u) + 2 * tid; k + 1 < I.h; k += 2 * kWave) {
        for (int r = 0; r < m; ++r) perm[r] = r;
        for (int i = m - 1; i >= 1; --i) {
            const U4 rr = draw(a.seed, (uint32_t)ii, t, ((uint32_t)k << 16) | (uint32_t)i, TAG_PERM);
            const int j = (int)__umulhi(rr.x, (uint32_t)(i + 1));
            const int tmp = perm[i];
            perm[i] = perm[j];
            perm[j] = tmp;
        }
        for (int r = 0; r < m; ++r) {
            const int wa = I.walker_base + k * m + r;
            const int wb = I.walker_base + (k + 1) * m + perm[r];
            const WalkerDesc da = a.wdesc[wa], db = a.wdesc[wb];
            WalkerState *sa = a.state + wa;
            WalkerState *sb = a.state + wb;
            a.xatt[I.xstat_off + k] += 1ull;
            const double Ea = sa->E, Eb = sb->E;
            const double xa = (Ea - I.Emin) * I.inv_de;
            const double xb = (Eb - I.Emin) * I.inv_de;
            if (!(xa >= (double)db.lo && xa < (double)db.hi)) continue;
            if (!(xb >= (double)da.lo && xb < (double)da.hi)) continue;
            const int ba = (int)floor(xa), bbn = (int)floor(xb);
            if (!a.vis[db.bin_off + (ba - db.lo)] || !a.vis[da.bin_off + (bbn - da.lo)]) continue;
            const U4 rr = draw(a.seed, (uint32_t)ii, t, ((uint32_t)k << 16) | (uint32_t)r, TAG_EXCH);
            const double u = u53(rr.x, rr.y);
            const int bina = sa->bin, binb = sb->bin;
            // stored bins (a resync may have clamped them) must lie in the
            // other window as well
            if (bina < db.lo || bina >= db.hi || binb < da.lo || binb >= da.hi) continue;
            const double lga_a = a.lng[da.bin_off + (bina - da.lo)];
            const double lga_b = a.lng[da.bin_off + (binb - da.lo)];
            const double lgb_b = a.lng[db.bin_off + (binb - db.lo)];
            const double lgb_a = a.lng[db.bin_off + (bina - db.lo)];
            const double lr = (lga_a - lga_b) + (lgb_b - lgb_a);
            if (!((lr >= 0.0) || (u < exp_det(lr)))) continue;
            a.xacc[I.xstat_off + k] += 1ull;
            const int tc = sa->cfg;
            sa->cfg = sb->cfg;
            sb->cfg = tc;
            sa->E = Eb;
            sb->E = Ea;
            sa->bin = binb;
            sb->bin = bina;
        }
    }
    if (tid == 0) all_done = 1;
    __syncthreads();
    for (int w = tid; w < I.n_walkers; w += kWave)
        if (!a.state[I.walker_base + w].done) all_done = 0;
    __syncthreads();
    if (tid == 0 && all_done) a.ictl[ii].done = 1;
}

// ------------------------------------------------------------------ launchers
static size_t lds_bytes(const KArgs &a, size_t per_walker)
{
    return ((per_walker + 15) & ~(size_t)15) * (size_t)a.walkers_per_block;
}

int launch_init(const KArgs &a, int mode, hipStream_t s, size_t per_walker)
{
    const int wpb = a.walkers_per_block;
    const dim3 grid((a.n_walkers + wpb - 1) / wpb), block(kWave * wpb);
    const size_t lds = lds_bytes(a, per_walker);
    switch (mode) {
    case M_DET: hipLaunchKernelGGL(init_kernel<M_DET>, grid, block, lds, s, a); break;
    case M_F64: hipLaunchKernelGGL(init_kernel<M_F64>, grid, block, lds, s, a); break;
    case M_F32: hipLaunchKernelGGL(init_kernel<M_F32>, grid, block, lds, s, a); break;
    default: return REWL_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? REWL_OK : REWL_EDEVICE;
}

int launch_sweep(const KArgs &a, int mode, hipStream_t s, size_t per_walker)
{
    const int wpb = a.walkers_per_block;
    const dim3 grid((a.n_walkers + wpb - 1) / wpb), block(kWave * wpb);
    const size_t lds = lds_bytes(a, per_walker);
    switch (mode) {
    case M_DET: hipLaunchKernelGGL(sweep_kernel<M_DET>, grid, block, lds, s, a); break;
    case M_F64: hipLaunchKernelGGL(sweep_kernel<M_F64>, grid, block, lds, s, a); break;
    case M_F32: hipLaunchKernelGGL(sweep_kernel<M_F32>, grid, block, lds, s, a); break;
    default: return REWL_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? REWL_OK : REWL_EDEVICE;
}

int launch_exchange(const KArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(exchange_kernel, dim3(a.n_inst), dim3(kWave), 0, s, a);
    return hipGetLastError() == hipSuccess ? REWL_OK : REWL_EDEVICE;
}

}  // namespace rewl
