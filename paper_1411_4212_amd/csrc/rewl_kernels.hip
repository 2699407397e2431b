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
#include "rewl_mlp_device.h"

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

// Per-walker LDS: spins | ln g (FP64) | H (u32) | visited (u8) | look-ahead
// batch of 64 trial moves (fast kernel).  When the fast kernel reads the
// configuration from HBM, only ln g of the window is staged (8 bytes per
// bin): H stays in HBM (see fast_segment).
constexpr size_t kBatchBytes = 64 * (32 + 4 + 4 + 8 + 16);

__device__ __forceinline__ size_t lds_core_bytes(const KArgs &a)
{
    return ((size_t)a.lds_spins_bytes + (size_t)a.lds_bins * (size_t)a.lds_bin_bytes + 15) & ~(size_t)15;
}

__device__ __forceinline__ WalkerLds carve_lds(unsigned char *base, const KArgs &a, int slot)
{
    const size_t per_al = lds_core_bytes(a) + kBatchBytes;
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
    // storage order of the configuration these functions read: -1 for one
    // staged in LDS (site order), the instance's layout for one in HBM
    int lay, lgk;
    __device__ __forceinline__ int at(int i) const { return spin_slot(i, lay, lgk); }
    int coord;              // the walk's coordinate: 0 energy, 1 M_z
};

template <int MODE>
__device__ __forceinline__ void load_latctx(LatCtx<MODE> &c, const InstDesc &I, const KArgs &a, int lane)
{
    c.N = I.N;
    c.L = I.L;
    c.z = I.z;
    c.invL = I.L > 0 ? 1.0f / (float)I.L : 0.0f;
    c.lattice = I.lattice;
    c.lay = -1;
    c.lgk = I.lg_L;
    c.coord = I.coord;
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
                const V s = S[c.at(j)];
                ax = ax + sl.Jd * s.x;
                ay = ay + sl.Jd * s.y;
                az = az + sl.Jd * s.z;
            }
        } else {
            const int d = c.deg[site];
            for (int k = 0; k < d; ++k) {
                const int j = c.nbr[(int64_t)site * c.z + k];
                const double Jv = c.J[(int64_t)site * c.z + k];
                const V s = S[c.at(j)];
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
                const V s = S[c.at(j)];
                const T Jv = (MODE == M_F32) ? (T)c.s0.Jf : (T)c.s0.Jd;
                px = Jv * s.x;
                py = Jv * s.y;
                pz = Jv * s.z;
            }
            if (c.has1) {
                const int j = bcc_neighbour(site, c.L, c.invL, c.s1);
                const V s = S[c.at(j)];
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
                const V s = S[c.at(j)];
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
            const V s = S[c.at(i)];
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
                    const V s = S[c.at(j)];
                    hx += sl.Jd * (double)s.x;
                    hy += sl.Jd * (double)s.y;
                    hz += sl.Jd * (double)s.z;
                }
            } else {
                const int d = c.deg[i];
                for (int k = 0; k < d; ++k) {
                    const int j = c.nbr[(int64_t)i * c.z + k];
                    const double Jv = c.J[(int64_t)i * c.z + k];
                    const V s = S[c.at(j)];
                    hx += Jv * (double)s.x;
                    hy += Jv * (double)s.y;
                    hz += Jv * (double)s.z;
                }
            }
            const V s = S[c.at(i)];
            acc += ((double)s.x * hx + (double)s.y * hy) + (double)s.z * hz;
        }
        return -0.5 * wave_sum_d(acc);
    }
}

// The walk's coordinate over a whole configuration: the energy, or
// M_z = sum_i S_i^z (DET: FP64 in site order; other modes: lane partial sums
// in FP64, then the wavefront sum).
template <int MODE>
__device__ double full_value(const LatCtx<MODE> &c, const typename Spin<MODE>::V *S)
{
    if (!c.coord) return full_energy<MODE>(c, S);
    if constexpr (MODE == M_DET) {
        double m = 0.0;
        for (int i = 0; i < c.N; ++i) m = m + (double)S[c.at(i)].z;
        return m;
    } else {
        double m = 0.0;
        for (int i = __lane_id(); i < c.N; i += kWave) m += (double)S[c.at(i)].z;
        return wave_sum_d(m);
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

// Change of the walk's coordinate when S_i becomes S' = (nx, ny, nz): dE
// from the local field, or nz - S_i^z for M_z.
template <int MODE>
__device__ __forceinline__ double move_delta(const LatCtx<MODE> &c, const typename Spin<MODE>::V *S, int i,
                                             typename Spin<MODE>::T nx, typename Spin<MODE>::T ny,
                                             typename Spin<MODE>::T nz, const typename Spin<MODE>::V &si)
{
    using T = typename Spin<MODE>::T;
    if (c.coord) return (double)(nz - si.z);
    T hx, hy, hz;
    local_field<MODE>(c, S, i, hx, hy, hz);
    return delta_e<MODE>(nx, ny, nz, si, hx, hy, hz);
}

// Copy a walker's configuration from HBM (instance layout) into LDS (site
// order), and back (all lanes).
template <int MODE>
__device__ __forceinline__ void spins_to_lds(typename Spin<MODE>::V *S, const typename Spin<MODE>::V *G,
                                             const InstDesc &I)
{
    for (int i = __lane_id(); i < I.N; i += kWave) S[i] = G[spin_slot(i, I.layout, I.lg_L)];
}
template <int MODE>
__device__ __forceinline__ void spins_to_hbm(typename Spin<MODE>::V *G, const typename Spin<MODE>::V *S,
                                             const InstDesc &I)
{
    for (int i = __lane_id(); i < I.N; i += kWave) G[spin_slot(i, I.layout, I.lg_L)] = S[i];
}

// ------------------------------------------------------------------ init
// Start configuration, its energy, and the drive into the window: moves are
// accepted when the new energy lies in the window or strictly closer to it.
template <int MODE, bool LDS_SPINS>
__global__ void __launch_bounds__(256) init_kernel(KArgs a)
{
    using T = typename Spin<MODE>::T;
    using V = typename Spin<MODE>::V;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = __lane_id();
    const int w = blockIdx.x * a.walkers_per_block + wave;
    if (w >= a.n_walkers) return;
    const WalkerDesc wd = a.wdesc[w];
    const InstDesc I = a.inst[wd.inst];
    WalkerLds L = carve_lds(lds_raw, a, wave);
    V *G = (V *)a.spins + I.cfg_off + (int64_t)wd.local * I.N;
    V *S = LDS_SPINS ? (V *)L.spins : G;
    LatCtx<MODE> c;
    load_latctx<MODE>(c, I, a, lane);
    if (!LDS_SPINS) c.lay = I.layout;

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
        S[c.at(i)] = v;
    }
    wave_sync();

    double E = full_value<MODE>(c, S);
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
        const V si = S[c.at(i)];
        const double Eb = E + move_delta<MODE>(c, S, i, nx, ny, nz, si);
        const double xb = (Eb - I.Emin) * I.inv_de;
        const bool in_b = (xb >= lo && xb < hi);
        if (in_b || dist(Eb) < dist(E)) {
            V v;
            v.x = nx;
            v.y = ny;
            v.z = nz;
            v.w = (T)0;
            S[c.at(i)] = v;
            E = Eb;
            inside = in_b;
        }
    }
    wave_sync();
    if (LDS_SPINS) spins_to_hbm<MODE>(G, S, I);
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
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
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
    spins_to_lds<MODE>(S, G, I);
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
        const V si = S[i];
        const double Eb = E + move_delta<MODE>(c, S, i, nx, ny, nz, si);
        const double xb = (Eb - Emin) * inv;
        int bb = -1;
        bool outside = true;
        bool newbin = false;
        double lnb = 0.0;
        if (xb >= lo && xb < hi) {
            bb = (int)floor(xb);
            outside = false;
            if (L.vis[bb - ilo]) {
                lnb = L.lng[bb - ilo];
            } else if (discovering) {
                // a bin not visited yet, during the first iteration: it
                // still holds the initial guess ln g~ = 0; it joins the
                // range (and H restarts) when the walker enters it
                newbin = true;
                lnb = L.lng[bb - ilo];
            } else {
                // afterwards the range is fixed
                bb = -1;
                outside = true;
            }
        }
        bool accept = false;
        if (bb >= 0) {
            const double lr = cur - lnb;
            accept = (lr >= 0.0) || (u < exp_det(lr));
        }
        oow += outside ? 1u : 0u;
        if (accept && newbin) {
            for (int j = lane; j < nb; j += kWave) L.H[j] = 0u;
        }
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
        const double ef = full_value<MODE>(c, S);
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
        if (flat && I.share) {
            // the window's walkers advance together (exchange_instance merges)
            st.ready = 1;
        } else if (flat) {
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

    spins_to_hbm<MODE>(G, S, I);
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
// Window sharing (the multiple-walker refinement of the parallel scheme): a
// walker whose histogram is flat keeps walking at its ln f until every walker
// of its window is flat; then every bin's ln g~ becomes the mean over the
// walkers that visited it (summed in walker order, then divided by their
// count), every walker takes that estimate and the union of the visited bins,
// H restarts, and ln f halves for all (or all finish, when the iteration ran
// at ln f <= ln f_final).  The walkers of a window make the same number of
// moves at the same ln f, so their estimates carry the same total and are
// averaged without shifts.  Lane j takes bins j, j + 64, ...
__device__ void merge_windows(const KArgs &a, const InstDesc &I)
{
    const int lane = __lane_id();
    const int m = I.m;
    for (int k = 0; k < I.h; ++k) {
        const int w0 = I.walker_base + k * m;
        bool waiting = false;
        for (int r = lane; r < m; r += kWave) {
            const WalkerState &s = a.state[w0 + r];
            waiting |= !(s.ready != 0 && s.done == 0);
        }
        if (__builtin_amdgcn_ballot_w64(waiting) != 0ull) continue;
        const WalkerDesc d0 = a.wdesc[w0];
        const int nb = d0.hi - d0.lo;
        const bool finish = a.state[w0].lnf <= I.lnf_final;
        int nvis = 0;
        for (int j = lane; j < nb; j += kWave) {
            double sum = 0.0;
            int cnt = 0;
            for (int r = 0; r < m; ++r) {
                const int64_t o = a.wdesc[w0 + r].bin_off + j;
                if (a.vis[o]) {
                    sum = sum + a.lng[o];
                    cnt += 1;
                }
            }
            if (cnt > 0) {
                const double mean = sum / (double)cnt;
                for (int r = 0; r < m; ++r) {
                    const int64_t o = a.wdesc[w0 + r].bin_off + j;
                    a.lng[o] = mean;
                    a.vis[o] = 1;
                }
                nvis += 1;
            }
            if (!finish)
                for (int r = 0; r < m; ++r) a.hist[a.wdesc[w0 + r].bin_off + j] = 0u;
        }
        nvis = wave_sum_i(nvis);
        for (int r = lane; r < m; r += kWave) {
            WalkerState *s = a.state + w0 + r;
            s->ready = 0;
            s->nvis = nvis;
            if (finish) {
                s->done = 1;
            } else {
                s->lnf = s->lnf * 0.5;
                s->iter += 1;
            }
        }
    }
    // the exchange below reads what other lanes stored
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// One replica-exchange step of instance ii at step t, by one wavefront:
// window pairs (k, k+1) with k of the parity of t; the m walkers of window k
// are paired with those of window k+1 by a Fisher-Yates permutation (lane r
// holds entry r); a pair may swap only if each energy lies in the other's
// window on a bin that walker has visited; the swap moves configuration,
// energy and bin.  Lanes r < m decide the m pairs of a window pair at once
// (they touch disjoint walkers).  Then the instance's done flag is
// recomputed.  With window sharing, merge_windows runs first.
__device__ void exchange_instance(const KArgs &a, int ii, uint64_t t)
{
    const int lane = __lane_id();
    const InstDesc I = a.inst[ii];
    const int m = I.m;
    if (I.share) merge_windows(a, I);
    for (int k = (int)(t & 1u); k + 1 < I.h; k += 2) {
        int pr = lane;
        for (int i = m - 1; i >= 1; --i) {
            const U4 rr = draw(a.seed, (uint32_t)ii, t, ((uint32_t)k << 16) | (uint32_t)i, TAG_PERM);
            const int j = (int)__umulhi(rr.x, (uint32_t)(i + 1));
            const int pi = __shfl(pr, i, kWave), pj = __shfl(pr, j, kWave);
            pr = (lane == i) ? pj : ((lane == j) ? pi : pr);
        }
        bool swapped = false;
        if (lane < m) {
            const int r = lane;
            const int wa = I.walker_base + k * m + r;
            const int wb = I.walker_base + (k + 1) * m + pr;
            const WalkerDesc da = a.wdesc[wa], db = a.wdesc[wb];
            WalkerState *sa = a.state + wa;
            WalkerState *sb = a.state + wb;
            const double Ea = sa->E, Eb = sb->E;
            const double xa = (Ea - I.Emin) * I.inv_de;
            const double xb = (Eb - I.Emin) * I.inv_de;
            bool ok = (xa >= (double)db.lo && xa < (double)db.hi) && (xb >= (double)da.lo && xb < (double)da.hi);
            const int bina = sa->bin, binb = sb->bin;
            // the stored bins (the ones the swap installs and the ratio
            // reads) must lie in the other window, on a bin the receiving
            // walker has visited
            ok = ok && !(bina < db.lo || bina >= db.hi || binb < da.lo || binb >= da.hi);
            if (ok) ok = a.vis[db.bin_off + (bina - db.lo)] && a.vis[da.bin_off + (binb - da.lo)];
            if (ok) {
                const U4 rr = draw(a.seed, (uint32_t)ii, t, ((uint32_t)k << 16) | (uint32_t)r, TAG_EXCH);
                const double u = u53(rr.x, rr.y);
                const double lga_a = a.lng[da.bin_off + (bina - da.lo)];
                const double lga_b = a.lng[da.bin_off + (binb - da.lo)];
                const double lgb_b = a.lng[db.bin_off + (binb - db.lo)];
                const double lgb_a = a.lng[db.bin_off + (bina - db.lo)];
                const double lr = (lga_a - lga_b) + (lgb_b - lgb_a);
                if ((lr >= 0.0) || (u < exp_det(lr))) {
                    swapped = true;
                    const int tc = sa->cfg;
                    sa->cfg = sb->cfg;
                    sb->cfg = tc;
                    sa->E = Eb;
                    sb->E = Ea;
                    sa->bin = binb;
                    sb->bin = bina;
                }
            }
        }
        const unsigned long long nacc = (unsigned long long)__popcll(__builtin_amdgcn_ballot_w64(swapped));
        if (lane == 0) {
            __hip_atomic_fetch_add(a.xatt + I.xstat_off + k, (unsigned long long)m, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(a.xacc + I.xstat_off + k, nacc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // round trips of configurations between the lowest and the highest
    // window (the replica diffusion the paper follows in its Fig. 1): a
    // half trip is counted when a configuration held in an extreme window
    // last visited the other extreme
    if (I.h >= 2) {
        // the swaps above were stored by other lanes of this wavefront
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        for (int j = lane; j < 2 * m; j += kWave) {
            const int win = j < m ? 0 : I.h - 1;
            const int w = I.walker_base + win * m + (j < m ? j : j - m);
            const int c = a.state[w].cfg;
            uint32_t *e = a.rtrip + I.walker_base + c;
            const uint32_t ext = j < m ? 1u : 2u;
            const uint32_t v = *e;
            if ((v & 3u) != ext) *e = ((v & ~3u) + ((v & 3u) ? 4u : 0u)) | ext;
        }
    }
    bool running = false;
    for (int w = lane; w < I.n_walkers; w += kWave) running |= (a.state[I.walker_base + w].done == 0);
    const bool all_done = __builtin_amdgcn_ballot_w64(running) == 0ull;
    if (lane == 0 && all_done) a.ictl[ii].done = 1;
}

__global__ void __launch_bounds__(64) exchange_kernel(KArgs a)
{
    const int ii = blockIdx.x;
    if (ii >= a.n_inst) return;
    if (a.ictl[ii].done) return;
    exchange_instance(a, ii, (uint64_t)a.t);
}


// ------------------------------------------------------------------ fast sweep
// The same segment as sweep_kernel for the FP32_DE and FP64 modes on bcc
// lattices, organised for one wavefront:
//  * every 64 trial moves, lane j draws the random numbers of move n0 + j
//    (site, acceptance uniform as ln u, proposal) into an LDS batch: these do
//    not depend on the walk;
//  * the wavefront then treats GW moves at a time (a pass): lane group g
//    gathers the neighbours of move g's site and computes dE of its move from
//    the current spins.  GW = 4 (16 lanes per move) when the configuration is
//    in LDS; GW = 16 (4 lanes per move) when it is read from HBM, so that one
//    round trip to memory serves 16 moves and the learned proposal's MFMA
//    evaluation fills its 16 columns.  The field sum has one fixed order for
//    both widths: 16 partial chains (chain c sums slots c, c+16, ... with
//    FMA), combined pairwise within quads of chains, then across quads as
//    (B0 + B3) + (B2 + B1); with GW = 4 a chain is a lane and the
//    combination DPP row operations, with GW = 16 a lane holds four chains.
//    The walk is therefore the same bit for bit at either width;
//  * the moves are then decided one after the other; an accepted move that
//    changes a spin of a later move's neighbourhood (or its own site) marks
//    the pass stale and the remaining moves' fields are recomputed from the
//    updated spins, so every decision uses exactly the current configuration
//    (with GW = 16 the test is geometric: the minimum-image distance between
//    the two sites is within the stencil's largest shell, which for bcc
//    shells holds exactly for the neighbours and the site itself);
//  * u < g(E_A)/g(E_B) is tested as ln u < ln g(E_A) - ln g(E_B);
//  * unvisited bins hold NaN in the LDS copy of ln g, so the move loop reads
//    one LDS word for the proposed bin and writes no visited flags.
// Neighbour indices: for L a power of two the site index is the bit field
// (x | y << k | z << 2k | s << 3k) and a neighbour is a field-wise addition
// modulo L (carry-free SWAR add); otherwise coordinates are packed in 8-bit
// fields and wrapped by a packed compare-subtract.
template <int CTRL>
__device__ __forceinline__ float rowsum_step_f(float v) { return v + dpp_f<CTRL>(v); }
template <int CTRL>
__device__ __forceinline__ double rowsum_step_d(double v) { return v + dpp_d<CTRL>(v); }

template <typename T>
__device__ __forceinline__ T row_sum16(T v)
{
    if constexpr (sizeof(T) == 4) {
        v = rowsum_step_f<0xB1>(v);
        v = rowsum_step_f<0x4E>(v);
        v = rowsum_step_f<0x124>(v);
        v = rowsum_step_f<0x128>(v);
    } else {
        v = rowsum_step_d<0xB1>(v);
        v = rowsum_step_d<0x4E>(v);
        v = rowsum_step_d<0x124>(v);
        v = rowsum_step_d<0x128>(v);
    }
    return v;
}

// The same sum as row_sum16 when one lane holds four chains: p[c] is chain
// 4j + c of the 16 (j = the lane within its quad).  Within the lane the
// chains combine as (p0 + p1) + (p2 + p3), the first two levels of
// row_sum16; across the quad B_j + B_{j-1}, then + the pair two lanes over:
// the row_ror:4 and row_ror:8 steps, in which lane l adds lane l - 4 and
// l - 8 of its row.  Lane 0 of the quad then holds (B0 + B3) + (B2 + B1),
// bit for bit the value row_sum16 leaves in lane 0 of a row.
template <int CTRL>
__device__ __forceinline__ float quadstep_f(float v) { return v + dpp_f<CTRL>(v); }
template <int CTRL>
__device__ __forceinline__ double quadstep_d(double v) { return v + dpp_d<CTRL>(v); }

template <typename T>
__device__ __forceinline__ T quad_combine(const T (&p)[4])
{
    T b = (p[0] + p[1]) + (p[2] + p[3]);
    if constexpr (sizeof(T) == 4) {
        b = quadstep_f<0x93>(b);   // quad_perm [3,0,1,2]: lane j adds lane j-1
        b = quadstep_f<0x4E>(b);   // quad_perm [2,3,0,1]: lane j adds lane j-2
    } else {
        b = quadstep_d<0x93>(b);
        b = quadstep_d<0x4E>(b);
    }
    return b;
}

template <typename T>
__device__ __forceinline__ T readlane_t(T v, int l)
{
    if constexpr (sizeof(T) == 4) return readlane_f(v, l);
    else return readlane_d(v, l);
}

__device__ __forceinline__ double uniform_d(double v)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c)
{
    if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}

struct FastLat {
    int L, k, L3, pow2;
    uint32_t M, Hm;          // SWAR masks: field bits below the top bit / top bits
};

// One segment of walker w by the calling wavefront, in LDS slot `wave`.
template <int MODE, int Q, bool POW2, bool LDS_SPINS, bool LEARNED>
__device__ __forceinline__ void fast_segment(const KArgs &a, const int w, const int wave, unsigned char *lds_raw)
{
    using T = typename Spin<MODE>::T;
    using V = typename Spin<MODE>::V;
    const int lane = __lane_id();
    const WalkerDesc wd = a.wdesc[w];
    if (a.ictl[wd.inst].done) return;
    const InstDesc I = a.inst[wd.inst];
    WalkerState st = a.state[w];
    if (st.status != 0) return;
    WalkerLds Ld = carve_lds(lds_raw, a, wave);
    unsigned char *bbase = (unsigned char *)lds_raw +
                           (lds_core_bytes(a) + kBatchBytes) * (size_t)wave + lds_core_bytes(a);
    V *b_prop = (V *)bbase;
    int32_t *b_site = (int32_t *)(bbase + 64 * sizeof(V));
    int32_t *b_code = b_site + 64;
    double *b_lnu = (double *)(b_code + 64);
    float4 *b_ul = (float4 *)(b_lnu + 64);      // learned proposal: (u_mix, u_w, u_phi, -)

    const int N = I.N;
    const int nb = wd.hi - wd.lo;
    const int ilo = wd.lo;
    // spins in LDS for the segment, or read and written in place in HBM
    V *G = (V *)a.spins + I.cfg_off + (int64_t)st.cfg * N;
    V *S = LDS_SPINS ? (V *)Ld.spins : G;
    if (LDS_SPINS) spins_to_lds<MODE>(S, G, I);
    double *glng = a.lng + wd.bin_off;
    uint32_t *gH = a.hist + wd.bin_off;
    uint8_t *gvis = a.vis + wd.bin_off;
    const double qnan = __longlong_as_double(0x7ff8000000000000ll);
    // With the configuration in HBM the walker's H stays in HBM too: the
    // move loop counts the visits to the bin it is in (hcur) and adds them
    // to H when it leaves the bin; only ln g of the window is staged.
    constexpr bool H_HBM = !LDS_SPINS;
    for (int j = lane; j < nb; j += kWave) {
        Ld.lng[j] = (gvis[j] || j == st.bin - ilo) ? glng[j] : qnan;
        if constexpr (!H_HBM) Ld.H[j] = gH[j];
    }

    // lattice constants and this lane's neighbour slots
    FastLat fl;
    fl.L = I.L;
    fl.pow2 = POW2 ? 1 : ((I.L & (I.L - 1)) == 0);
    fl.k = 31 - __clz(I.L);
    fl.L3 = I.L * I.L * I.L;
    {
        uint32_t one = 1u | (1u << fl.k) | (1u << (2 * fl.k));
        uint32_t full = (uint32_t)fl.L3 - 1u;
        fl.Hm = (one << (fl.k - 1)) & full;
        fl.M = full & ~fl.Hm;
    }
    // moves per pass, lanes per move, partial chains per lane (see above)
    constexpr int GW = (!LDS_SPINS && Q >= 4) ? 16 : 4;
    constexpr int GL = 64 / GW;
    constexpr int NC = 16 / GL;
    const int grp = lane / GL, r = lane % GL;
    // slot (c, q) of this lane is entry k = 16 q + NC r + c of the fast slot
    // table (neighbours grouped by memory row; see the API's table set-up):
    // chain NC r + c of the 16-chain order.  With one chain per lane the SWAR
    // offsets are kept split (low bits / top bit of each field); with four,
    // whole.
    uint32_t offM[2][NC][Q], offH[2][NC][Q];
    uint32_t flipm = 0;            // bit c Q + q: neighbour on the other sublattice
    T Jq[NC][Q];
    int d2max = 0;                 // largest squared stencil length, half-cell units
    {
        const BccSlot *slots = a.slots + I.fslot_off;
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int k = q * 16 + r * NC + c;
                const BccSlot sl = slots[k];
                Jq[c][q] = sl.real ? ((MODE == M_F32) ? (T)sl.Jf : (T)sl.Jd) : (T)0;
                if (sl.flip) flipm |= 1u << (c * Q + q);
                if (sl.real) {
                    const int vx = 2 * sl.d[0][0] + sl.flip, vy = 2 * sl.d[0][1] + sl.flip,
                              vz = 2 * sl.d[0][2] + sl.flip;
                    const int d2 = vx * vx + vy * vy + vz * vz;
                    d2max = d2 > d2max ? d2 : d2max;
                }
#pragma unroll
                for (int sb = 0; sb < 2; ++sb) {
                    const uint32_t ox = (uint32_t)((sl.d[sb][0] + fl.L) % fl.L);
                    const uint32_t oy = (uint32_t)((sl.d[sb][1] + fl.L) % fl.L);
                    const uint32_t oz = (uint32_t)((sl.d[sb][2] + fl.L) % fl.L);
                    if (fl.pow2) {
                        const uint32_t off = ox | (oy << fl.k) | (oz << (2 * fl.k));
                        offM[sb][c][q] = NC == 1 ? (off & fl.M) : off;
                        offH[sb][c][q] = NC == 1 ? (off & fl.Hm) : 0u;
                    } else {
                        offM[sb][c][q] = ox | (oy << 8) | (oz << 16);
                        offH[sb][c][q] = 0;
                    }
                }
            }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {                       // wave maximum
            const int v = __shfl_xor(d2max, o, kWave);
            d2max = v > d2max ? v : d2max;
        }
    }
    wave_sync();

    const double inv = I.inv_de;
    const double emin_inv = I.Emin * inv;
    const double lo = (double)wd.lo, hi = (double)wd.hi;
    double E = st.E;
    int bin = st.bin;
    const double lnf = st.lnf;
    const bool frozen = st.done != 0;
    const bool discovering = (st.iter == 0) && !frozen;
    const double lnf_add = frozen ? 0.0 : lnf;
    const uint32_t h_add = frozen ? 0u : 1u;
    // ln g and H of the current bin live in registers while the walker
    // stays in it; LDS holds them again once it leaves and at the end
    double cur = uniform_d(Ld.lng[bin - ilo]);
    uint32_t hcur = H_HBM ? 0u : (uint32_t)__builtin_amdgcn_readfirstlane((int)Ld.H[bin - ilo]);
    const uint64_t n_begin = st.attempts;
    const uint64_t n_end = n_begin + (uint64_t)I.seg_len;
    uint64_t acc_count = 0, oow = 0;
    rewl_trace_rec *trace = a.trace ? a.trace + (int64_t)w * a.trace_cap : nullptr;
    const uint32_t wrapC = 0x00808080u - 0x00010101u * (uint32_t)fl.L;   // 128 - L per 8-bit field

    int nidx[NC == 1 ? Q : 1];
    // the site and proposal of this lane's group move, kept in registers so
    // that an accepted move needs no LDS round trip to write its spin or to
    // find the later moves it invalidates
    int mv_site = 0;
    int mhx = 0, mhy = 0, mhz = 0;            // half-cell coordinates of that site (GW = 16)
    V mv_prop{};
    T dEv = 0;
    T hx_k = 0, hy_k = 0, hz_k = 0;          // this lane's group field (harvest)
    V si_k{};
    float lnqr_v = 0.f;                        // learned: ln q(S_i) - ln q(S'), lane = move
    float psx = 0.f, psy = 0.f, psz = 0.f;     // learned: proposal of move p + lane
    const float inv_hs = I.inv_hs, e_w = wd.e_w;
    mlp::Lane Wl;
    if constexpr (LEARNED) Wl = ((const mlp::Lane *)a.mlp)[lane];
    const bool harvesting = a.harvest != nullptr && !LEARNED;
    uint64_t hcount = st.harvested;
    const int twoL = 2 * fl.L;
    // storage order of the configuration in HBM (LDS holds site order)
    const int lay = I.layout, lgk = I.lg_L;
    // half-cell coordinates (2x + s, 2y + s, 2z + s) of a move's site from its code
    auto halfcell = [&](int code, int &hx_, int &hy_, int &hz_) {
        int x, y, zc, sb;
        if (POW2 || fl.pow2) {
            x = code & (fl.L - 1);
            y = (code >> fl.k) & (fl.L - 1);
            zc = (code >> (2 * fl.k)) & (fl.L - 1);
            sb = code >> (3 * fl.k);
        } else {
            x = code & 0xFF;
            y = (code >> 8) & 0xFF;
            zc = (code >> 16) & 0xFF;
            sb = code >> 24;
        }
        hx_ = 2 * x + sb;
        hy_ = 2 * y + sb;
        hz_ = 2 * zc + sb;
    };
    // gather + field + dE of the move held by this lane's group (batch slot p + grp)
    auto fields = [&](int p) {
        const int e = p + grp;
        const int code = b_code[e];
        const int site = b_site[e];
        // the site's own spin and the proposal are read with the gather
        const V si = S[LDS_SPINS ? site : spin_slot(site, lay, lgk)];
        const V pr = b_prop[e];
        mv_site = site;
        mv_prop = pr;
        if constexpr (NC > 1) halfcell(code, mhx, mhy, mhz);
        T px[NC], py[NC], pz[NC];
        T gx[NC][Q], gy[NC][Q], gz[NC][Q];
#pragma unroll
        for (int c = 0; c < NC; ++c) px[c] = py[c] = pz[c] = (T)0;
        const int sb = (POW2 || fl.pow2) ? (code >> (3 * fl.k)) : (code >> 24);
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                int j;
                const int t = sb ^ (int)((flipm >> (c * Q + q)) & 1u);
                if (POW2 || fl.pow2) {
                    const uint32_t aa = (uint32_t)code & (uint32_t)(fl.L3 - 1);
                    const uint32_t o = sb ? offM[1][c][q] : offM[0][c][q];
                    uint32_t om, oh;
                    if constexpr (NC == 1) {
                        om = o;
                        oh = sb ? offH[1][c][q] : offH[0][c][q];
                    } else {
                        om = o & fl.M;
                        oh = o & fl.Hm;
                    }
                    const uint32_t cell = ((aa & fl.M) + om) ^ (aa & fl.Hm) ^ oh;
                    // site order in LDS; in HBM the storage order (spin_slot)
                    j = (LDS_SPINS || lay < 0) ? (int)(cell | ((uint32_t)t << (3 * fl.k)))
                                               : (int)((cell << 1) | (uint32_t)t);
                } else {
                    uint32_t sum = ((uint32_t)code & 0x00FFFFFFu) + (sb ? offM[1][c][q] : offM[0][c][q]);
                    const uint32_t gt = ((sum + wrapC) >> 7) & 0x00010101u;
                    sum -= gt * (uint32_t)fl.L;
                    // L not a power of two: HBM holds site order (layout -1)
                    j = (int)(sum & 0xFF) + fl.L * ((int)((sum >> 8) & 0xFF) + fl.L * ((int)(sum >> 16) + fl.L * t));
                }
                if constexpr (NC == 1) nidx[q] = j;
                const V s = S[j];
                gx[c][q] = s.x;
                gy[c][q] = s.y;
                gz[c][q] = s.z;
            }
        // all of this lane's neighbour loads are issued above, before the
        // first sum below waits for one: the pass pays one memory latency,
        // not one per slot.  The scheduling barrier keeps the compiler from
        // moving each sum up to its load (which it does under register
        // pressure, leaving a full memory wait after every load).
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                px[c] = fma_t<T>(Jq[c][q], gx[c][q], px[c]);
                py[c] = fma_t<T>(Jq[c][q], gy[c][q], py[c]);
                pz[c] = fma_t<T>(Jq[c][q], gz[c][q], pz[c]);
            }
        T hx, hy, hz;
        if constexpr (NC == 1) {
            hx = row_sum16(px[0]);
            hy = row_sum16(py[0]);
            hz = row_sum16(pz[0]);
        } else {
            hx = quad_combine(px);
            hy = quad_combine(py);
            hz = quad_combine(pz);
        }
        hx_k = hx;
        hy_k = hy;
        hz_k = hz;
        si_k = si;
        if constexpr (!LEARNED) {
            if constexpr (MODE == M_F32) {
                dEv = -__builtin_fmaf(pr.z - si.z, hz, __builtin_fmaf(pr.y - si.y, hy, (pr.x - si.x) * hx));
            } else {
                dEv = -(((pr.x - si.x) * hx + (pr.y - si.y) * hy) + (pr.z - si.z) * hz);
            }
        } else {
            // lane m < GW takes move p + m: its field and current spin from the
            // first lane of group m
            float hm0, hm1, hm2, sm0, sm1, sm2;
            if constexpr (GW == 4) {
                const int mv = lane & 3;
                auto pick = [&](float v) {
                    const float v0 = readlane_f(v, 0), v1 = readlane_f(v, 16), v2 = readlane_f(v, 32),
                                v3 = readlane_f(v, 48);
                    return (mv & 2) ? ((mv & 1) ? v3 : v2) : ((mv & 1) ? v1 : v0);
                };
                hm0 = pick((float)hx);
                hm1 = pick((float)hy);
                hm2 = pick((float)hz);
                sm0 = pick((float)si.x);
                sm1 = pick((float)si.y);
                sm2 = pick((float)si.z);
            } else {
                const int src = GL * (lane & 15);
                hm0 = __shfl((float)hx, src, kWave);
                hm1 = __shfl((float)hy, src, kWave);
                hm2 = __shfl((float)hz, src, kWave);
                sm0 = __shfl((float)si.x, src, kWave);
                sm1 = __shfl((float)si.y, src, kWave);
                sm2 = __shfl((float)si.z, src, kWave);
            }
            const mlp::bf16x8 xb = mlp::input_operand(hm0 * inv_hs, hm1 * inv_hs, hm2 * inv_hs, e_w, lane < GW);
            const mlp::f32x4 o = mlp::forward(Wl, xb);
            float out[12];
            mlp::gather_outputs(o, out);
            if (lane < GW) {
                const mlp::Mix mx = mlp::mixture(out);
                const float4 uu = b_ul[p + lane];
                const V ud = b_prop[p + lane];
                mlp::sample(mx, uu.x, uu.y, uu.z, (float)ud.x, (float)ud.y, (float)ud.z, psx, psy, psz);
                lnqr_v = mlp::log_q(mx, sm0, sm1, sm2) - mlp::log_q(mx, psx, psy, psz);
                dEv = (T)(-__builtin_fmaf(psz - sm2, hm2, __builtin_fmaf(psy - sm1, hm1, (psx - sm0) * hm0)));
            }
        }
    };

    int my_site = 0;
    int b_code_reg = 0;
    double my_lnu = 0.0;
    for (uint64_t n0 = n_begin; n0 < n_end; n0 += 64) {
        // draw the random numbers of moves n0 .. n0+63, one per lane
        {
            const uint64_t nn = n0 + (uint64_t)lane;
            const U4 rr = draw(a.seed, wd.stream, nn, 0u, TAG_SITE);
            const int site = pick_site(rr.x, N);
            const double u = u53(rr.y, rr.z);
            T px, py, pz;
            propose<MODE>(a.seed, wd.stream, nn, TAG_SPHERE, px, py, pz);
            int code = site;
            if (!fl.pow2) {
                int x, y, zc;
                int qv = divmod_small(site, fl.L, 1.0f / (float)fl.L, x);
                qv = divmod_small(qv, fl.L, 1.0f / (float)fl.L, y);
                const int sb = divmod_small(qv, fl.L, 1.0f / (float)fl.L, zc);
                code = x | (y << 8) | (zc << 16) | (sb << 24);
            }
            V pv;
            pv.x = px;
            pv.y = py;
            pv.z = pz;
            pv.w = (T)0;
            b_prop[lane] = pv;
            b_site[lane] = site;
            b_code[lane] = code;
            b_code_reg = code;
            my_site = site;
            my_lnu = log(u);
            if constexpr (LEARNED) {
                const U4 ru = draw(a.seed, wd.stream, nn, 0u, TAG_LEARNED);
                b_ul[lane] = make_float4((float)(ru.x >> 8) * (1.0f / 16777216.0f),
                                         ((float)(ru.y >> 8) + 0.5f) * (1.0f / 16777216.0f),
                                         (float)(ru.z >> 8) * (1.0f / 16777216.0f), 0.f);
            }
        }
        wave_sync();
        const int nvalid = __builtin_amdgcn_readfirstlane((int)((n_end - n0) < 64 ? (n_end - n0) : 64));
        // moves of this batch that go to the trace (uniform)
        const int ntr = (trace == nullptr || n0 >= (uint64_t)a.trace_cap)
                            ? 0
                            : __builtin_amdgcn_readfirstlane((int)((uint64_t)a.trace_cap - n0 < 64 ? (uint64_t)a.trace_cap - n0 : 64));
        for (int p = 0; p < nvalid; p += GW) {
            fields(p);
            bool stale = false;
            const int gmax = (nvalid - p) < GW ? (nvalid - p) : GW;
            for (int g = 0; g < gmax; ++g) {
                if (stale) {
                    fields(p);
                    stale = false;
                }
                const uint64_t n = n0 + (uint64_t)(p + g);
                const double dE = (double)readlane_t<T>(dEv, LEARNED ? g : GL * g);
                const double lnqr = LEARNED ? (double)readlane_f(lnqr_v, g) : 0.0;
                if (harvesting && (n % (uint64_t)a.harvest_every) == 0 && hcount < (uint64_t)a.harvest_cap) {
                    // training record of this move, taken before the move
                    const float rx = readlane_f((float)hx_k, GL * g), ry = readlane_f((float)hy_k, GL * g),
                                rz = readlane_f((float)hz_k, GL * g);
                    const float sx = readlane_f((float)si_k.x, GL * g), sy = readlane_f((float)si_k.y, GL * g),
                                sz = readlane_f((float)si_k.z, GL * g);
                    if (lane == 0) {
                        float4 *rec = (float4 *)(a.harvest + ((int64_t)w * a.harvest_cap + (int64_t)hcount) * 8);
                        rec[0] = make_float4(rx * inv_hs, ry * inv_hs, rz * inv_hs, e_w);
                        rec[1] = make_float4(sx, sy, sz, 0.f);
                    }
                    ++hcount;
                }
                const int site = __builtin_amdgcn_readlane(my_site, p + g);
                const double lnu = readlane_d(my_lnu, p + g);
                const double Eb = E + dE;
                const double xb = __builtin_fma(Eb, inv, -emin_inv);
                // ln g and H of the proposed bin, read without a branch: a
                // proposal outside the window reads the current bin instead
                const bool inwin = (xb >= lo) && (xb < hi);
                const int bb = (int)(inwin ? xb : (double)bin);   // xb >= lo >= 0: truncation is the floor
                const double lnb_m = Ld.lng[bb - ilo];
                const uint32_t hb_m = H_HBM ? 0u : Ld.H[bb - ilo];
                const bool same = bb == bin;
                double lnb = same ? cur : lnb_m;
                uint32_t hb = same ? hcur : hb_m;
                bool outside = !inwin;
                bool newbin = false;
                if (inwin && __builtin_isnan(lnb)) {
                    // a bin not visited yet: during the first iteration it
                    // holds the initial guess ln g~ = 0 and joins the range
                    // when the walker enters it; afterwards the range is
                    // fixed
                    if (discovering) {
                        lnb = 0.0;
                        newbin = true;
                    } else {
                        outside = true;
                    }
                }
                // ln u < 0 always, so ln u < lr also covers lr >= 0; the q-ratio
                // term only exists with the learned proposal
                const double lr = LEARNED ? (cur - lnb) + lnqr : (cur - lnb);
                const bool accept = !outside && (lnu < lr);
                oow += outside ? 1u : 0u;
                if (accept && newbin) {
                    // the range grew: the histogram restarts (the new bin's
                    // ln g~ rides in `cur` until the walker leaves it)
                    if constexpr (H_HBM) {
                        for (int j = lane; j < nb; j += kWave) gH[j] = 0u;
                        // the cleared counts land before any later addition
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    } else {
                        for (int j = lane; j < nb; j += kWave) Ld.H[j] = 0u;
                    }
                    hb = 0u;
                    hcur = 0u;
                }
                if (accept && bb != bin) {
                    // leave the current bin: its ln g back to LDS, its H to
                    // LDS or (added) to HBM
                    Ld.lng[bin - ilo] = cur;
                    if constexpr (H_HBM) {
                        if (lane == 0 && hcur != 0u)
                            __hip_atomic_fetch_add(gH + (bin - ilo), hcur, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                    } else {
                        Ld.H[bin - ilo] = hcur;
                    }
                    hcur = hb;
                }
                if (accept) {
                    if constexpr (LEARNED) {
                        if (lane == g) {
                            V v;
                            v.x = (T)psx;
                            v.y = (T)psy;
                            v.z = (T)psz;
                            v.w = (T)0;
                            S[LDS_SPINS ? site : spin_slot(site, lay, lgk)] = v;
                        }
                    } else {
                        if (lane == GL * g) S[LDS_SPINS ? site : spin_slot(site, lay, lgk)] = mv_prop;
                    }
                    // one lane stored the spin; other lanes of this wavefront
                    // gather it for later moves
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                    E = Eb;
                    bin = bb;
                    cur = lnb;
                    ++acc_count;
                    // later moves of this pass whose neighbourhood or site changed
                    bool hit;
                    if constexpr (NC == 1) {
                        hit = (grp > g) && (mv_site == site);
                        const int sslot = LDS_SPINS ? site : spin_slot(site, lay, lgk);
#pragma unroll
                        for (int q = 0; q < Q; ++q) hit |= (grp > g) && (nidx[q] == sslot);
                    } else {
                        int ax, ay, az;
                        halfcell(__builtin_amdgcn_readlane(b_code_reg, p + g), ax, ay, az);
                        int dx = mhx - ax, dy = mhy - ay, dz = mhz - az;
                        dx += dx < -fl.L ? twoL : (dx >= fl.L ? -twoL : 0);
                        dy += dy < -fl.L ? twoL : (dy >= fl.L ? -twoL : 0);
                        dz += dz < -fl.L ? twoL : (dz >= fl.L ? -twoL : 0);
                        hit = (grp > g) && (dx * dx + dy * dy + dz * dz <= d2max);
                    }
                    stale = __builtin_amdgcn_ballot_w64(hit) != 0ull;
                }
                // a finished walker adds +0: every ln g value stays as it is
                // (a -0 would turn into +0, the same number)
                cur = cur + lnf_add;
                hcur = hcur + h_add;
                if (p + g < ntr) {
                    // every lane stores the same (uniform) record
                    rewl_trace_rec rec;
                    rec.site = (uint32_t)site;
                    rec.flags = (accept ? 1u : 0u) | (outside ? 2u : 0u);
                    rec.E = E;
                    rec.bin = bin;
                    rec.attempt_lo = (uint32_t)n;
                    trace[n] = rec;
                }
            }
        }
        wave_sync();
    }
    const uint64_t n = n_end;
    Ld.lng[bin - ilo] = cur;
    if constexpr (H_HBM) {
        if (lane == 0 && hcur != 0u)
            __hip_atomic_fetch_add(gH + (bin - ilo), hcur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        // the additions are complete before the flatness test reads H
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    } else {
        Ld.H[bin - ilo] = hcur;
    }
    wave_sync();

    // resync when due (lane-parallel FP64 energy)
    LatCtx<MODE> c;
    load_latctx<MODE>(c, I, a, lane);
    if (!LDS_SPINS) c.lay = lay;
    if (I.resync > 0 && (n / (uint64_t)I.resync) != (n_begin / (uint64_t)I.resync)) {
        const double ef = full_value<MODE>(c, S);
        const double d = fabs(ef - E);
        if (d > st.max_drift) st.max_drift = d;
        E = ef;
        const double x = (ef - I.Emin) * inv;
        bin = x < lo ? wd.lo : (x >= hi ? wd.hi - 1 : (int)floor(x));
    }

    // flatness over visited bins, then the ln f update
    int nvis = 0;
    unsigned long long sumH = 0;
    uint32_t minH = 0xFFFFFFFFu;
    for (int j = lane; j < nb; j += kWave) {
        if (!__builtin_isnan(Ld.lng[j])) {
            const uint32_t hj = H_HBM ? gH[j] : Ld.H[j];
            nvis += 1;
            sumH += hj;
            minH = hj < minH ? hj : minH;
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
        if (flat && I.share) {
            st.ready = 1;
        } else if (flat) {
            if (st.lnf <= I.lnf_final) {
                st.done = 1;
            } else {
                st.lnf = st.lnf * 0.5;
                st.iter += 1;
                for (int j = lane; j < nb; j += kWave) {
                    if constexpr (H_HBM) gH[j] = 0u;
                    else Ld.H[j] = 0u;
                }
            }
        }
    } else {
        st.nvis = nvis;
    }
    wave_sync();

    if (LDS_SPINS) spins_to_hbm<MODE>(G, S, I);
    for (int j = lane; j < nb; j += kWave) {
        const double v = Ld.lng[j];
        const bool vis = !__builtin_isnan(v);
        glng[j] = vis ? v : 0.0;
        if constexpr (!H_HBM) gH[j] = Ld.H[j];
        gvis[j] = vis ? 1 : 0;
    }
    if (lane == 0) {
        st.E = E;
        st.bin = bin;
        st.attempts = n;
        st.accepts += acc_count;
        st.oow += oow;
        st.harvested = hcount;
        if (!isfinite(E) || !isfinite(cur)) st.status = REWL_ENUMERIC;
        a.state[w] = st;
    }
}

template <int MODE, int Q, bool POW2, bool LDS_SPINS, bool LEARNED>
__global__ void __launch_bounds__(256) sweep_fast_kernel(KArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int w = blockIdx.x * a.walkers_per_block + wave;
    if (w >= a.n_walkers) return;
    fast_segment<MODE, Q, POW2, LDS_SPINS, LEARNED>(a, w, wave, lds_raw);
}

// ------------------------------------------------------------------ persistent
// Every instance runs up to p_max_rounds rounds (a segment of each of its
// walkers, then its exchange step) in one launch, independently of the
// other instances.  Wavefronts take walkers from a bounded multi-producer
// multi-consumer queue; the last walker of an instance to finish a round
// runs that instance's exchange and queues the instance's walkers for the
// next round (or marks the instance stopped).  A wavefront waits only while
// the queue is empty, and the walkers it waits for are held by running
// wavefronts, so no launch shape can deadlock.  Every wait is bounded: past
// the limit the wavefront raises `error`, sets all_done and leaves, so the
// grid always drains (the limit, in polls of at least ~50 ns, is set by the
// host well above the longest segment).  Synchronisation is release/acquire at agent scope
// (the L2 caches of the chip are not coherent with each other).  Every
// branch and loop of the persistent loop is wave-uniform: values that steer
// it are broadcast with readfirstlane, since the segment's wavefront-level
// operations (DPP sums, readlane, ballots) need all 64 lanes active.

__device__ __forceinline__ uint32_t ld_acq(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_acq64(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel64(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t add_acqrel(uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void persist_abort(const KArgs &a)
{
    st_rel(&a.pctl->error, 1u);
    st_rel(&a.pctl->all_done, 1u);
}

// The queue operations below are called by the whole wavefront and keep
// every branch and loop wave-uniform (values broadcast with readfirstlane,
// readiness of several slots combined with a ballot).

// Next walker, or -1 when all is done.
__device__ int persist_pop(const KArgs &a)
{
    const int lane = __lane_id();
    uint32_t t = 0;
    if (lane == 0) t = add_acqrel(&a.pctl->head, 1u);
    t = (uint32_t)__builtin_amdgcn_readfirstlane((int)t);
    unsigned long long *slot = a.p_slots + (t & a.p_mask);
    for (uint64_t it = 0;; ++it) {
        const unsigned long long v = ld_acq64(slot);
        const uint32_t seq = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
        if (seq == t + 1u) {
            const int w = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
            if (lane == 0) st_rel64(slot, (unsigned long long)(t + a.p_mask + 1u) << 32);
            return w;
        }
        const uint32_t done = (uint32_t)__builtin_amdgcn_readfirstlane((int)ld_acq(&a.pctl->all_done));
        if (done) return -1;
        if (it >= a.p_spin_limit) {
            if (lane == 0) persist_abort(a);
            return -1;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// Queue walkers base .. base + n - 1.
__device__ void persist_push_range(const KArgs &a, int base, int n)
{
    const int lane = __lane_id();
    uint32_t p0 = 0;
    if (lane == 0) p0 = __hip_atomic_fetch_add(&a.pctl->tail, (uint32_t)n, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    p0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)p0);
    for (int c0 = 0; c0 < n; c0 += kWave) {
        const bool active = c0 + lane < n;
        const uint32_t p = p0 + (uint32_t)(c0 + lane);
        unsigned long long *slot = a.p_slots + (p & a.p_mask);
        bool ready = false;
        for (uint64_t it = 0;; ++it) {
            const bool ok = !active || (uint32_t)(ld_acq64(slot) >> 32) == p;
            if (__builtin_amdgcn_ballot_w64(!ok) == 0ull) {
                ready = true;
                break;
            }
            const uint32_t done = (uint32_t)__builtin_amdgcn_readfirstlane((int)ld_acq(&a.pctl->all_done));
            if (done || it >= a.p_spin_limit) break;
            __builtin_amdgcn_s_sleep(2);
        }
        if (!ready) {
            if (lane == 0) persist_abort(a);
            return;
        }
        if (active) st_rel64(slot, ((unsigned long long)(p + 1u) << 32) | (uint32_t)(base + c0 + lane));
    }
}

template <int MODE, int Q, bool POW2, bool LDS_SPINS, bool LEARNED>
__global__ void __launch_bounds__(256) persistent_kernel(KArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = __lane_id();
    for (;;) {
        const int w = persist_pop(a);
        if (w < 0) break;
        if (w >= a.n_walkers) {
            if (lane == 0) persist_abort(a);
            break;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        fast_segment<MODE, Q, POW2, LDS_SPINS, LEARNED>(a, w, wave, lds_raw);
        wave_sync();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        // every control value wave-uniform (loads land in vector registers)
        const int ii = __builtin_amdgcn_readfirstlane(a.wdesc[w].inst);
        const int nw = __builtin_amdgcn_readfirstlane(a.inst[ii].n_walkers);
        const int wbase = __builtin_amdgcn_readfirstlane(a.inst[ii].walker_base);
        // arrivals are counted without reset: the nw-th arrival of a round
        // leaves a multiple of nw
        uint32_t prev = 0;
        if (lane == 0) prev = add_acqrel(a.p_arrive + ii, 1u);
        prev = (uint32_t)__builtin_amdgcn_readfirstlane((int)prev);
        if ((prev + 1u) % (uint32_t)nw != 0u) continue;
        // last walker of instance ii in this round: exchange, then the next round
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        uint32_t r = 0;
        if (lane == 0) r = add_acqrel(a.p_rounds + ii, 1u);
        r = (uint32_t)__builtin_amdgcn_readfirstlane((int)r);
        exchange_instance(a, ii, (uint64_t)a.t + r);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int done_i = __builtin_amdgcn_readfirstlane(a.ictl[ii].done);
        const bool stop = done_i != 0 || (int32_t)(r + 1u) >= a.p_max_rounds;
        if (!stop) {
            persist_push_range(a, wbase, nw);
        } else {
            uint32_t f = 0;
            if (lane == 0) f = add_acqrel(&a.pctl->finished, 1u);
            f = (uint32_t)__builtin_amdgcn_readfirstlane((int)f);
            if (f + 1u == (uint32_t)a.n_inst && lane == 0) st_rel(&a.pctl->all_done, 1u);
        }
    }
}

// Queue set-up for a persistent launch (one block): walkers of instances
// not yet done are queued, done instances count as finished.
__global__ void __launch_bounds__(256) persistent_prep_kernel(KArgs a)
{
    __shared__ int n_active;
    __shared__ int n_done;
    const int tid = threadIdx.x;
    if (tid == 0) {
        int q = 0, d = 0;
        for (int i = 0; i < a.n_inst; ++i) {
            if (a.ictl[i].done) {
                ++d;
            } else {
                q += a.inst[i].n_walkers;
            }
        }
        n_active = q;
        n_done = d;
    }
    __syncthreads();
    for (int i = tid; i < a.n_inst; i += blockDim.x) {
        a.p_arrive[i] = 0u;
        a.p_rounds[i] = 0u;
    }
    // queued walkers in instance order
    if (tid == 0) {
        int q = 0;
        for (int i = 0; i < a.n_inst; ++i) {
            if (a.ictl[i].done) continue;
            const int b = a.inst[i].walker_base;
            for (int w = 0; w < a.inst[i].n_walkers; ++w, ++q)
                a.p_slots[q] = ((unsigned long long)(q + 1) << 32) | (uint32_t)(b + w);
        }
    }
    for (uint32_t j = (uint32_t)n_active + tid; j <= a.p_mask; j += blockDim.x)
        a.p_slots[j] = (unsigned long long)j << 32;
    if (tid == 0) {
        a.pctl->head = 0u;
        a.pctl->tail = (uint32_t)n_active;
        a.pctl->finished = (uint32_t)n_done;
        a.pctl->all_done = (n_done == a.n_inst || a.p_max_rounds <= 0) ? 1u : 0u;
        a.pctl->error = 0u;
    }
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
    if (a.spins_in_lds) {
        switch (mode) {
        case M_DET: hipLaunchKernelGGL((init_kernel<M_DET, true>), grid, block, lds, s, a); break;
        case M_F64: hipLaunchKernelGGL((init_kernel<M_F64, true>), grid, block, lds, s, a); break;
        case M_F32: hipLaunchKernelGGL((init_kernel<M_F32, true>), grid, block, lds, s, a); break;
        default: return REWL_EINVAL;
        }
    } else {
        switch (mode) {
        case M_F64: hipLaunchKernelGGL((init_kernel<M_F64, false>), grid, block, lds, s, a); break;
        case M_F32: hipLaunchKernelGGL((init_kernel<M_F32, false>), grid, block, lds, s, a); break;
        default: return REWL_EINVAL;
        }
    }
    return hipGetLastError() == hipSuccess ? REWL_OK : REWL_EDEVICE;
}

int launch_sweep(const KArgs &a, int mode, hipStream_t s, size_t per_walker)
{
    const int wpb = a.walkers_per_block;
    const dim3 grid((a.n_walkers + wpb - 1) / wpb), block(kWave * wpb);
    const size_t lds = lds_bytes(a, per_walker);
    if (a.fast_q > 0 && mode != M_DET) {
#define REWL_FAST(M, Qv, P2)                                                                          \
    do {                                                                                              \
        if (a.mlp && M == M_F32) {                                                                    \
            if (a.spins_in_lds)                                                                       \
                hipLaunchKernelGGL((sweep_fast_kernel<M_F32, Qv, P2, true, true>), grid, block, lds, s, a);  \
            else                                                                                      \
                hipLaunchKernelGGL((sweep_fast_kernel<M_F32, Qv, P2, false, true>), grid, block, lds, s, a); \
        } else if (a.spins_in_lds) {                                                                  \
            hipLaunchKernelGGL((sweep_fast_kernel<M, Qv, P2, true, false>), grid, block, lds, s, a);  \
        } else {                                                                                      \
            hipLaunchKernelGGL((sweep_fast_kernel<M, Qv, P2, false, false>), grid, block, lds, s, a); \
        }                                                                                             \
    } while (0)
#define REWL_FAST_Q(M, P2)                          \
    switch (a.fast_q) {                             \
    case 1: REWL_FAST(M, 1, P2); break;             \
    case 4: REWL_FAST(M, 4, P2); break;             \
    case 8: REWL_FAST(M, 8, P2); break;             \
    default: return REWL_EINVAL;                    \
    }
        if (mode == M_F32) {
            if (a.all_pow2) { REWL_FAST_Q(M_F32, true) } else { REWL_FAST_Q(M_F32, false) }
        } else {
            if (a.all_pow2) { REWL_FAST_Q(M_F64, true) } else { REWL_FAST_Q(M_F64, false) }
        }
#undef REWL_FAST_Q
#undef REWL_FAST
        return hipGetLastError() == hipSuccess ? REWL_OK : REWL_EDEVICE;
    }
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

template <int MODE, int Q, bool POW2, bool LDS_SPINS, bool LEARNED>
static int launch_persist_t(const KArgs &a, hipStream_t s, size_t lds, int n_cu, int max_blocks, int *grid_out)
{
    const int wpb = a.walkers_per_block;
    const auto kern = persistent_kernel<MODE, Q, POW2, LDS_SPINS, LEARNED>;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kWave * wpb, lds) != hipSuccess || per_cu < 1)
        return REWL_EUNSUPPORTED;
    const int need = (a.n_walkers + wpb - 1) / wpb;
    int grid = std::max(1, std::min(need, per_cu * n_cu));
    if (max_blocks > 0) grid = std::min(grid, max_blocks);
    *grid_out = grid;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWave * wpb), lds, s, a);
    return hipGetLastError() == hipSuccess ? REWL_OK : REWL_EDEVICE;
}

int launch_persistent(const KArgs &a, int mode, hipStream_t s, size_t per_walker, int n_cu, int max_blocks,
                      int *grid_out)
{
    if (a.fast_q <= 0 || mode == M_DET) return REWL_EUNSUPPORTED;
    hipLaunchKernelGGL(persistent_prep_kernel, dim3(1), dim3(256), 0, s, a);
    if (hipGetLastError() != hipSuccess) return REWL_EDEVICE;
    const size_t lds = lds_bytes(a, per_walker);
#define REWL_PERS(M, Qv, P2)                                                                              \
    do {                                                                                                  \
        if (a.mlp && M == M_F32)                                                                          \
            return a.spins_in_lds ? launch_persist_t<M_F32, Qv, P2, true, true>(a, s, lds, n_cu, max_blocks, grid_out)   \
                                  : launch_persist_t<M_F32, Qv, P2, false, true>(a, s, lds, n_cu, max_blocks, grid_out); \
        return a.spins_in_lds ? launch_persist_t<M, Qv, P2, true, false>(a, s, lds, n_cu, max_blocks, grid_out)          \
                              : launch_persist_t<M, Qv, P2, false, false>(a, s, lds, n_cu, max_blocks, grid_out);        \
    } while (0)
#define REWL_PERS_Q(M, P2)                  \
    switch (a.fast_q) {                     \
    case 1: REWL_PERS(M, 1, P2);            \
    case 4: REWL_PERS(M, 4, P2);            \
    case 8: REWL_PERS(M, 8, P2);            \
    default: return REWL_EINVAL;            \
    }
    if (mode == M_F32) {
        if (a.all_pow2) { REWL_PERS_Q(M_F32, true) } else { REWL_PERS_Q(M_F32, false) }
    } else {
        if (a.all_pow2) { REWL_PERS_Q(M_F64, true) } else { REWL_PERS_Q(M_F64, false) }
    }
#undef REWL_PERS_Q
#undef REWL_PERS
}

}  // namespace rewl
