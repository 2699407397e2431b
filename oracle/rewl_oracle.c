/*
 * rewl_oracle.c -- plain, slow, FP64 CPU oracle of replica-exchange
 * Wang-Landau (REWL) sampling for the classical Heisenberg model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code with the GPU path.
 *
 * What it computes, and where the paper defines it:
 *   - Hamiltonian H = -sum_{i<j} J_ij S_i.S_j, |S_i| = 1          (Model, Eq. 1)
 *   - bcc lattice, two spins per cubic cell, N = 2 L^3            (Model)
 *   - restricted range [E_min, E_max], bin width dE               (Model; Sec. original WL)
 *   - WL: ln g~ = 0, H = 0, accept min(1, g~(E_A)/g~(E_B)),
 *     update ln g~ and H at the state the walker is in afterwards,
 *     flat if H(E) >= p <H>, then ln f -> ln f / 2, stop at f_min (Sec. original WL)
 *   - h overlapping windows with overlap ratio o, m walkers/window,
 *     each walker its own ln g~, H and ln f                        (Sec. parallel scheme)
 *   - replica exchange between adjacent windows, acceptance
 *     min(1, g_i(E_A) g_j(E_B) / (g_i(E_B) g_j(E_A))), possible only
 *     if both replicas lie in the overlap                          (Sec. parallel scheme; Sec. simulation details)
 *   - trial move: random site, new direction uniform on the sphere (Sec. simulation details)
 *   - optional: the walk over another coordinate, the magnetisation M_z
 *     instead of E                                                 (Sec. original WL)
 *   - optional: the walkers of a window sharing ln g~ (the multiple-walker
 *     refinement of the parallel scheme)                           (Sec. parallel scheme)
 *
 * Readings where the paper is silent (documented with the design):
 *   flatness is taken over the bins the walker has visited; a check in a
 *   segment that first visited a bin is not flat; out-of-window proposals are
 *   rejected; walkers start from a given configuration and are driven into
 *   their window; exchanges alternate even/odd window pairs with a random
 *   pairing of the m walkers; a walker whose last iteration is flat freezes
 *   its ln g~ and H but keeps walking and exchanging.
 *
 * Everything is sequential and in plain FP64 arithmetic (built with
 * -ffp-contract=off).  Loops over walkers within a segment run on several
 * threads; each walker owns its configuration during a segment and draws its
 * random numbers from its own counter-based stream, so the result does not
 * depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ESTATE (-2)
#define ORC_EINIT (-5)

/* Philox stream tags (the fourth counter word). */
#define TAG_SITE 0u
#define TAG_SPHERE 1u
#define TAG_INIT_SITE 2u
#define TAG_INIT_SPHERE 3u
#define TAG_EXCH 4u
#define TAG_PERM 5u
#define TAG_INIT_CONFIG 6u
#define TAG_LEARNED 7u

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers:
 * as easy as 1, 2, 3", SC'11).  Ten rounds of the 4x32 S-box with the
 * published multipliers and Weyl key increments.                      */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint32_t seed, uint32_t stream, uint64_t n, uint32_t word2, uint32_t tag,
                 uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)n, (uint32_t)(n >> 32), word2, tag};
    uint32_t key[2] = {seed, stream};
    orc_philox4x32_10(ctr, key, out);
}

/* uniform double in [0,1) with 53 random bits from two words */
static double u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

/* site index uniform on 0..N-1 by a multiply-shift of one word */
static int pick_site(uint32_t w, int N)
{
    return (int)(((uint64_t)w * (uint64_t)(uint32_t)N) >> 32);
}

/* Uniform direction on the unit sphere: Marsaglia (1972).  Draw v1, v2
 * uniform on [-1,1) until s = v1^2 + v2^2 < 1, then
 * S = (2 v1 sqrt(1-s), 2 v2 sqrt(1-s), 1 - 2 s).  Each Philox block gives
 * two tries; blocks are numbered by the third counter word.  After 64 blocks
 * without success (probability ~1e-86) the direction +z is used.         */
void orc_sphere(uint32_t seed, uint32_t stream, uint64_t n, uint32_t tag, double out[3])
{
    for (uint32_t blk = 0; blk < 64; ++blk) {
        uint32_t r[4];
        draw(seed, stream, n, blk, tag, r);
        for (int t = 0; t < 2; ++t) {
            double v1 = (double)(int32_t)r[2 * t] * (1.0 / 2147483648.0);
            double v2 = (double)(int32_t)r[2 * t + 1] * (1.0 / 2147483648.0);
            double s = v1 * v1 + v2 * v2;
            if (s < 1.0) {
                double q = sqrt(1.0 - s);
                out[0] = (2.0 * v1) * q;
                out[1] = (2.0 * v2) * q;
                out[2] = 1.0 - 2.0 * s;
                return;
            }
        }
    }
    out[0] = 0.0; out[1] = 0.0; out[2] = 1.0;
}

/* exp(x) for x <= 0, used only to compare against a uniform number in the
 * acceptance tests.  Cody-Waite reduction x = k ln2 + r with ln 2 split in a
 * 32-bit head and a tail, |r| <= ln2/2, then the degree-13 Taylor polynomial
 * of e^r (truncation error < 1e-17) in Horner form, then the exact scaling
 * by 2^k.  Returns 0 below -700.                                          */
double orc_exp_det(double x)
{
    if (x > 0.0) x = 0.0;
    if (x < -700.0) return 0.0;
    const double ln2_hi = 0x1.62e42ff000000p-1;
    const double ln2_lo = -0x1.718432a1b0e26p-35;
    const double inv_ln2 = 0x1.71547652b82fep+0;
    double kd = floor(x * inv_ln2 + 0.5);
    double r = (x - kd * ln2_hi) - kd * ln2_lo;
    double p = 1.0 / 6227020800.0;          /* 1/13! */
    p = p * r + 1.0 / 479001600.0;          /* 1/12! */
    p = p * r + 1.0 / 39916800.0;           /* 1/11! */
    p = p * r + 1.0 / 3628800.0;            /* 1/10! */
    p = p * r + 1.0 / 362880.0;             /* 1/9!  */
    p = p * r + 1.0 / 40320.0;              /* 1/8!  */
    p = p * r + 1.0 / 5040.0;               /* 1/7!  */
    p = p * r + 1.0 / 720.0;                /* 1/6!  */
    p = p * r + 1.0 / 120.0;                /* 1/5!  */
    p = p * r + 1.0 / 24.0;                 /* 1/4!  */
    p = p * r + 1.0 / 6.0;                  /* 1/3!  */
    p = p * r + 0.5;                        /* 1/2!  */
    p = p * r + 1.0;
    p = p * r + 1.0;
    int k = (int)kd;                        /* -1010 <= k <= 0 */
    uint64_t bits = (uint64_t)(int64_t)(k + 1023) << 52;
    double scale;
    memcpy(&scale, &bits, sizeof scale);
    return p * scale;
}

/* ------------------------------------------------------------------ */
/* Lattice: per-site neighbour lists with couplings.                   */
/* ------------------------------------------------------------------ */
typedef struct {
    int N;
    int zmax;       /* row stride of nbr/Jn */
    int *deg;       /* [N] */
    int *nbr;       /* [N*zmax] */
    double *Jn;     /* [N*zmax] */
} olat;

static void lat_free(olat *l)
{
    free(l->deg); free(l->nbr); free(l->Jn);
    memset(l, 0, sizeof *l);
}

/* bcc shells.  Sites sit at half-cell coordinates (2x+s, 2y+s, 2z+s) with
 * sublattice s in {0,1}; lattice vectors are integer triples of equal
 * parity.  Shell n collects the vectors of the n-th smallest length; within
 * a shell the vectors are taken in ascending lexicographic (dx,dy,dz) order.
 * Returns the number of vectors written (<= cap), -1 if cap is too small.  */
int orc_bcc_shells(int n_shells, int *dx, int *dy, int *dz, int *shell, int cap)
{
    int d2s[64];
    int nd = 0;
    /* collect distinct squared lengths (vectors up to |component| 6) */
    for (int a = -6; a <= 6; ++a)
        for (int b = -6; b <= 6; ++b)
            for (int c = -6; c <= 6; ++c) {
                if (a == 0 && b == 0 && c == 0) continue;
                if (((a ^ b) & 1) || ((a ^ c) & 1)) continue;
                int d2 = a * a + b * b + c * c;
                int seen = 0;
                for (int q = 0; q < nd; ++q) if (d2s[q] == d2) seen = 1;
                if (!seen && nd < 64) d2s[nd++] = d2;
            }
    /* sort ascending (insertion sort) */
    for (int i = 1; i < nd; ++i) {
        int v = d2s[i], j = i - 1;
        while (j >= 0 && d2s[j] > v) { d2s[j + 1] = d2s[j]; --j; }
        d2s[j + 1] = v;
    }
    if (n_shells > nd || n_shells > 12) return -1;   /* |component| 6 covers 12 shells safely */
    int cnt = 0;
    for (int n = 0; n < n_shells; ++n)
        for (int a = -6; a <= 6; ++a)
            for (int b = -6; b <= 6; ++b)
                for (int c = -6; c <= 6; ++c) {
                    if (a == 0 && b == 0 && c == 0) continue;
                    if (((a ^ b) & 1) || ((a ^ c) & 1)) continue;
                    if (a * a + b * b + c * c != d2s[n]) continue;
                    if (cnt >= cap) return -1;
                    dx[cnt] = a; dy[cnt] = b; dz[cnt] = c; shell[cnt] = n;
                    ++cnt;
                }
    return cnt;
}

static int wrap(int v, int L) { v %= L; return v < 0 ? v + L : v; }

/* site index of (sublattice s, cell x, y, z) */
int orc_bcc_site(int L, int s, int x, int y, int z)
{
    return ((s * L + z) * L + y) * L + x;
}

static int lat_build_bcc(olat *l, int L, int n_shells, const double *J)
{
    int dx[1024], dy[1024], dz[1024], sh[1024];
    int z = orc_bcc_shells(n_shells, dx, dy, dz, sh, 1024);
    if (z <= 0 || L < 1) return ORC_EINVAL;
    int N = 2 * L * L * L;
    l->N = N; l->zmax = z;
    l->deg = (int *)malloc(sizeof(int) * (size_t)N);
    l->nbr = (int *)malloc(sizeof(int) * (size_t)N * (size_t)z);
    l->Jn = (double *)malloc(sizeof(double) * (size_t)N * (size_t)z);
    for (int s = 0; s < 2; ++s)
        for (int cz = 0; cz < L; ++cz)
            for (int cy = 0; cy < L; ++cy)
                for (int cx = 0; cx < L; ++cx) {
                    int i = orc_bcc_site(L, s, cx, cy, cz);
                    l->deg[i] = z;
                    for (int k = 0; k < z; ++k) {
                        int t = s ^ (dx[k] & 1);
                        /* half-cell coordinate 2c+s moves by d; new cell = (2c+s+d-t)/2 */
                        int nx = wrap(cx + (s + dx[k] - t) / 2, L);
                        int ny = wrap(cy + (s + dy[k] - t) / 2, L);
                        int nz = wrap(cz + (s + dz[k] - t) / 2, L);
                        l->nbr[(size_t)i * z + k] = orc_bcc_site(L, t, nx, ny, nz);
                        l->Jn[(size_t)i * z + k] = J[sh[k]];
                    }
                }
    return ORC_OK;
}

/* Explicit couplings: pair p adds J[p] to the lists of both ends, in the
 * order given. */
static int lat_build_explicit(olat *l, int N, int64_t n_pairs, const int32_t *pi,
                              const int32_t *pj, const double *pJ)
{
    if (N < 1) return ORC_EINVAL;
    int *deg = (int *)calloc((size_t)N, sizeof(int));
    for (int64_t p = 0; p < n_pairs; ++p) {
        if (pi[p] < 0 || pi[p] >= N || pj[p] < 0 || pj[p] >= N || pi[p] == pj[p]) {
            free(deg);
            return ORC_EINVAL;
        }
        deg[pi[p]]++; deg[pj[p]]++;
    }
    int zmax = 1;
    for (int i = 0; i < N; ++i) if (deg[i] > zmax) zmax = deg[i];
    l->N = N; l->zmax = zmax;
    l->deg = (int *)calloc((size_t)N, sizeof(int));
    l->nbr = (int *)calloc((size_t)N * (size_t)zmax, sizeof(int));
    l->Jn = (double *)calloc((size_t)N * (size_t)zmax, sizeof(double));
    for (int64_t p = 0; p < n_pairs; ++p) {
        int a = pi[p], b = pj[p];
        l->nbr[(size_t)a * zmax + l->deg[a]] = b; l->Jn[(size_t)a * zmax + l->deg[a]] = pJ[p]; l->deg[a]++;
        l->nbr[(size_t)b * zmax + l->deg[b]] = a; l->Jn[(size_t)b * zmax + l->deg[b]] = pJ[p]; l->deg[b]++;
    }
    free(deg);
    return ORC_OK;
}

/* h_i = sum_j J_ij S_j over i's neighbour list, in list order */
static void local_field(const olat *l, const double *S, int i, double h[3])
{
    double hx = 0.0, hy = 0.0, hz = 0.0;
    const int *nb = l->nbr + (size_t)i * l->zmax;
    const double *J = l->Jn + (size_t)i * l->zmax;
    for (int k = 0; k < l->deg[i]; ++k) {
        const double *s = S + 3 * (size_t)nb[k];
        hx = hx + J[k] * s[0];
        hy = hy + J[k] * s[1];
        hz = hz + J[k] * s[2];
    }
    h[0] = hx; h[1] = hy; h[2] = hz;
}

/* E = -1/2 sum_i S_i . h_i  (every bond counted from both ends) */
static double full_energy(const olat *l, const double *S)
{
    double acc = 0.0;
    for (int i = 0; i < l->N; ++i) {
        double h[3];
        local_field(l, S, i, h);
        const double *s = S + 3 * (size_t)i;
        acc = acc + ((s[0] * h[0] + s[1] * h[1]) + s[2] * h[2]);
    }
    return -0.5 * acc;
}

/* energy change of S_i -> Sn given the local field h at i */
static double delta_e(const double *Sold, const double *Sn, const double h[3])
{
    return -(((Sn[0] - Sold[0]) * h[0] + (Sn[1] - Sold[1]) * h[1]) + (Sn[2] - Sold[2]) * h[2]);
}

/* ------------------------------------------------------------------ */
/* Windows (parallel scheme): h windows of equal width on a global bin  */
/* grid of B bins, neighbours overlapping by the ratio o.               */
/* ------------------------------------------------------------------ */
static int round_half_up(double x) { return (int)floor(x + 0.5); }

int orc_window_bins(int B, int h, double o, int k, int *lo, int *hi)
{
    if (B < 1 || h < 1 || k < 0 || k >= h || !(o >= 0.0) || !(o < 1.0)) return ORC_EINVAL;
    int wb = round_half_up((double)B / (1.0 + (double)(h - 1) * (1.0 - o)));
    if (wb < 1) wb = 1;
    if (wb > B) wb = B;
    int l = (h == 1) ? 0 : round_half_up((double)k * (double)(B - wb) / (double)(h - 1));
    *lo = l; *hi = l + wb;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Oracle context.                                                     */
/* ------------------------------------------------------------------ */
typedef struct {
    uint32_t stream;       /* global walker id: second Philox key word */
    int win, rep;          /* window index, walker index within window */
    int lo, hi;            /* window bins [lo, hi) */
    int cfg;               /* configuration this walker carries */
    double E;
    int bin;
    double lnf;
    int iter;
    int done;
    uint64_t attempts, accepts, oow;
    int nvis_prev;
    int ready;             /* window sharing: flat in this iteration, waiting for the window */
    double *lng;           /* [hi-lo] */
    uint32_t *H;           /* [hi-lo] */
    uint8_t *vis;          /* [hi-lo] */
    double max_drift;
} owalker;

typedef struct {
    olat lat;
    int L;
    double Emin, Emax, inv_de;
    int B, h, m;
    double overlap;
    int flat_num, flat_den;
    double lnf_init, lnf_final;
    int64_t seg_len, resync;
    uint32_t seed;
    int W;                 /* = h*m walkers */
    owalker *w;
    double *spins;         /* [W][N][3] configurations */
    int64_t t;             /* exchange step counter */
    uint32_t stream_base;  /* global id of walker 0 (several runs in one batch) */
    uint32_t instance;     /* second key word of the exchange stream */
    int inited;
    int n_threads;
    uint64_t *xatt, *xacc; /* [h-1] exchange attempts / accepts per window pair */
    /* trace */
    int64_t trace_cap;
    unsigned char *trace;  /* [W][trace_cap] records of 24 bytes */
    int check_energy;      /* test mode: full recompute after every accept */
    double max_check_err;
    /* learned proposal (NULL: uniform new direction) */
    double *mlp;           /* [ORC_MLP_PARAMS] FP64 parameters */
    double hs;             /* largest sum of |J| over a site's neighbours */
    /* drive into the window: per-attempt records (test mode) */
    int64_t drive_cap;
    unsigned char *drive;  /* [W][drive_cap] records of 24 bytes */
    int64_t *drive_len;    /* [W] */
    /* replica round trips, per configuration: (half trips << 2) | last
     * extreme window visited (1 lowest, 2 highest, 0 none yet) */
    uint32_t *rtrip;
    int share;             /* walkers of a window advance together and share ln g */
    int coord;             /* the walk's coordinate: 0 energy, 1 magnetisation M_z */
} octx;

/* The coordinate the walk bins (Sec. original WL: the density of states may
 * be taken over another order parameter instead of E): the energy of Eq. 1,
 * or the magnetisation along z, M_z = sum_i S_i^z, summed in site order.   */
static double full_coord(const octx *c, const double *S)
{
    if (!c->coord) return full_energy(&c->lat, S);
    double m = 0.0;
    for (int i = 0; i < c->lat.N; ++i) m = m + S[3 * (size_t)i + 2];
    return m;
}

/* change of the coordinate when S_i becomes Sn (h: the local field at i) */
static double coord_delta(const octx *c, const double *Sold, const double *Sn, const double h[3])
{
    if (c->coord) return Sn[2] - Sold[2];
    return delta_e(Sold, Sn, h);
}

typedef struct {
    uint32_t site;
    uint32_t flags;        /* bit0 accepted, bit1 proposal out of window */
    double E;              /* energy after the attempt */
    int32_t bin;           /* bin after the attempt */
    uint32_t attempt_lo;
} otrace;

static double *cfg_spins(octx *c, int cfg) { return c->spins + (size_t)cfg * 3 * (size_t)c->lat.N; }

/* bin coordinate; returns 1 and the bin if lo <= x < hi */
static int in_window(const octx *c, double E, int lo, int hi, int *bin)
{
    double x = (E - c->Emin) * c->inv_de;
    if (x >= (double)lo && x < (double)hi) {
        *bin = (int)floor(x);
        return 1;
    }
    return 0;
}

static double window_distance(const octx *c, double E, int lo, int hi)
{
    double x = (E - c->Emin) * c->inv_de;
    if (x < (double)lo) return (double)lo - x;
    if (x >= (double)hi) return x - (double)hi;
    return 0.0;
}

octx *orc_create_bcc(int L, int n_shells, const double *J)
{
    octx *c = (octx *)calloc(1, sizeof(octx));
    if (lat_build_bcc(&c->lat, L, n_shells, J) != ORC_OK) { free(c); return NULL; }
    c->L = L;
    return c;
}

octx *orc_create_explicit(int N, int64_t n_pairs, const int32_t *pi, const int32_t *pj,
                          const double *pJ)
{
    octx *c = (octx *)calloc(1, sizeof(octx));
    if (lat_build_explicit(&c->lat, N, n_pairs, pi, pj, pJ) != ORC_OK) { free(c); return NULL; }
    c->L = 0;
    return c;
}

static void free_walkers(octx *c)
{
    if (c->w) {
        for (int i = 0; i < c->W; ++i) { free(c->w[i].lng); free(c->w[i].H); free(c->w[i].vis); }
        free(c->w);
    }
    c->w = NULL;
    free(c->spins); c->spins = NULL;
    free(c->xatt); free(c->xacc); c->xatt = c->xacc = NULL;
    free(c->rtrip); c->rtrip = NULL;
}

void orc_destroy(octx *c)
{
    if (!c) return;
    free_walkers(c);
    free(c->trace);
    free(c->drive);
    free(c->drive_len);
    free(c->mlp);
    lat_free(&c->lat);
    free(c);
}

int orc_num_sites(const octx *c) { return c->lat.N; }
int orc_max_degree(const octx *c) { return c->lat.zmax; }

/* neighbour list of site i (for tests) */
int orc_neighbours(const octx *c, int i, int32_t *nbr, double *J, int cap)
{
    if (i < 0 || i >= c->lat.N) return ORC_EINVAL;
    int d = c->lat.deg[i];
    for (int k = 0; k < d && k < cap; ++k) {
        nbr[k] = c->lat.nbr[(size_t)i * c->lat.zmax + k];
        J[k] = c->lat.Jn[(size_t)i * c->lat.zmax + k];
    }
    return d;
}

double orc_energy(const octx *c, const double *spins) { return full_energy(&c->lat, spins); }

void orc_local_field(const octx *c, const double *spins, int i, double h[3])
{
    local_field(&c->lat, spins, i, h);
}

int orc_set_windows(octx *c, double Emin, double Emax, int B, int h, double o, int m)
{
    if (!(Emax > Emin) || B < 1 || h < 1 || m < 1 || !(o >= 0.0) || !(o < 1.0)) return ORC_EINVAL;
    c->Emin = Emin; c->Emax = Emax; c->B = B; c->h = h; c->overlap = o; c->m = m;
    c->inv_de = (double)B / (Emax - Emin);
    return ORC_OK;
}

int orc_set_schedule(octx *c, int flat_num, int flat_den, double lnf_init, double lnf_final,
                     int64_t seg_len, int64_t resync)
{
    if (flat_num < 0 || flat_den < 1 || flat_num > flat_den || !(lnf_init > 0.0) ||
        !(lnf_final > 0.0) || seg_len < 1 || resync < 0)
        return ORC_EINVAL;
    c->flat_num = flat_num; c->flat_den = flat_den;
    c->lnf_init = lnf_init; c->lnf_final = lnf_final;
    c->seg_len = seg_len; c->resync = resync;
    return ORC_OK;
}

void orc_set_threads(octx *c, int n) { c->n_threads = n; }

/* place this run inside a batch: walker w uses stream base+w, exchanges use
 * the instance number as their key word */
void orc_set_ids(octx *c, uint32_t stream_base, uint32_t instance)
{
    c->stream_base = stream_base;
    c->instance = instance;
}
void orc_set_check_energy(octx *c, int on) { c->check_energy = on; }
double orc_max_check_err(const octx *c) { return c->max_check_err; }

int orc_set_trace(octx *c, int64_t cap)
{
    free(c->trace);
    c->trace = NULL;
    c->trace_cap = cap > 0 ? cap : 0;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Acceptance functions (the ones the walkers use).                    */
/* ------------------------------------------------------------------ */

/* Wang-Landau: ln of g~(E_A)/g~(E_B) */
static double wl_log_ratio(double lng_a, double lng_b) { return lng_a - lng_b; }

/* replica exchange: ln of g_i(E_A) g_j(E_B) / (g_i(E_B) g_j(E_A)) */
static double re_log_ratio(double lngi_a, double lngi_b, double lngj_b, double lngj_a)
{
    return (lngi_a - lngi_b) + (lngj_b - lngj_a);
}

/* accept with probability min(1, e^lr) given a uniform u in [0,1) */
static int metropolis(double lr, double u) { return lr >= 0.0 || u < orc_exp_det(lr); }

double orc_wl_accept_prob(double lng_a, double lng_b)
{
    double lr = wl_log_ratio(lng_a, lng_b);
    return lr >= 0.0 ? 1.0 : orc_exp_det(lr);
}

/* Wang-Landau acceptance with an asymmetric proposal q(.|x) whose input x
 * does not depend on the moved spin: ln of g(E_A) q(S_i|x) / (g(E_B) q(S'|x)) */
static double wl_log_ratio_q(double lng_a, double lng_b, double lnq_old, double lnq_new)
{
    return (lng_a - lng_b) + (lnq_old - lnq_new);
}

double orc_wl_accept_prob_q(double lng_a, double lng_b, double lnq_old, double lnq_new)
{
    double lr = wl_log_ratio_q(lng_a, lng_b, lnq_old, lnq_new);
    return lr >= 0.0 ? 1.0 : orc_exp_det(lr);
}

double orc_re_accept_prob(double lngi_a, double lngi_b, double lngj_b, double lngj_a)
{
    double lr = re_log_ratio(lngi_a, lngi_b, lngj_b, lngj_a);
    return lr >= 0.0 ? 1.0 : orc_exp_det(lr);
}

/* ------------------------------------------------------------------ */
/* Learned proposal (an extension; the paper's move is a uniform new    */
/* direction).  Wang-Landau with an asymmetric proposal q(.|x) whose    */
/* input x does not involve the moved spin stays exact when the         */
/* acceptance carries q(S_i|x) / q(S'|x) (the Metropolis-Hastings form  */
/* of the acceptance of the original WL algorithm).                     */
/*                                                                      */
/* x = (h_i / h_s, e_w): the local field (which never contains S_i)     */
/* scaled by h_s = the largest sum of |J| over a site's neighbours, and */
/* the walker's window-centre energy per spin in units of h_s / 2.      */
/* A 4-64-64-12 perceptron with ReLU gives, per component c = 0..2,     */
/* v_c (3 values) and a logit a_c:  kappa_c = clip(|v_c|, 1e-3, 1e3),   */
/* mu_c = v_c / |v_c|, alpha = softmax(a), and                          */
/*   q(s) = eps/(4 pi) + (1 - eps) sum_c alpha_c f(s; mu_c, kappa_c),   */
/*   f(s; mu, k) = k / (2 pi (1 - e^{-2k})) exp(k (mu.s - 1)),          */
/* the von Mises-Fisher density on the unit sphere, eps = 0.05.         */
/* Parameters: W1[64][4], b1[64], W2[64][64], b2[64], W3[12][64], b3[12]. */
/* ------------------------------------------------------------------ */
#define ORC_MLP_PARAMS (64 * 4 + 64 + 64 * 64 + 64 + 12 * 64 + 12)
#define MLP_EPS 0.05
#define MLP_KMIN 1e-3
#define MLP_KMAX 1e3

typedef struct {
    double mu[3][3];
    double kappa[3];
    double alpha[3];
} omix;

static void mlp_forward(const double *th, const double x[4], double out[12])
{
    const double *W1 = th, *b1 = W1 + 64 * 4, *W2 = b1 + 64, *b2 = W2 + 64 * 64;
    const double *W3 = b2 + 64, *b3 = W3 + 12 * 64;
    double a1[64], a2[64];
    for (int i = 0; i < 64; ++i) {
        double z = b1[i];
        for (int k = 0; k < 4; ++k) z = z + W1[i * 4 + k] * x[k];
        a1[i] = z > 0.0 ? z : 0.0;
    }
    for (int i = 0; i < 64; ++i) {
        double z = b2[i];
        for (int k = 0; k < 64; ++k) z = z + W2[i * 64 + k] * a1[k];
        a2[i] = z > 0.0 ? z : 0.0;
    }
    for (int i = 0; i < 12; ++i) {
        double z = b3[i];
        for (int k = 0; k < 64; ++k) z = z + W3[i * 64 + k] * a2[k];
        out[i] = z;
    }
}

static void mlp_mixture(const double out[12], omix *m)
{
    double amax = out[3];
    if (out[7] > amax) amax = out[7];
    if (out[11] > amax) amax = out[11];
    double e[3], es = 0.0;
    for (int c = 0; c < 3; ++c) { e[c] = exp(out[4 * c + 3] - amax); es += e[c]; }
    for (int c = 0; c < 3; ++c) {
        const double vx = out[4 * c], vy = out[4 * c + 1], vz = out[4 * c + 2];
        const double r = sqrt(vx * vx + vy * vy + vz * vz);
        double k = r;
        if (k < MLP_KMIN) k = MLP_KMIN;
        if (k > MLP_KMAX) k = MLP_KMAX;
        m->kappa[c] = k;
        m->alpha[c] = e[c] / es;
        if (r > 0.0) {
            m->mu[c][0] = vx / r; m->mu[c][1] = vy / r; m->mu[c][2] = vz / r;
        } else {
            m->mu[c][0] = 0.0; m->mu[c][1] = 0.0; m->mu[c][2] = 1.0;
        }
    }
}

/* ln q(s) of the mixture */
static double mix_log_q(const omix *m, const double s[3])
{
    double t = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double k = m->kappa[c];
        const double w = m->mu[c][0] * s[0] + m->mu[c][1] * s[1] + m->mu[c][2] * s[2];
        const double lnf = log(k) - log(2.0 * M_PI) - log(-expm1(-2.0 * k)) + k * (w - 1.0);
        t += m->alpha[c] * exp(lnf);
    }
    return log(MLP_EPS / (4.0 * M_PI) + (1.0 - MLP_EPS) * t);
}

/* One draw from q: with probability eps the given uniform direction, else
 * a component by its weight, then w = mu.s by inverting the vMF marginal
 * CDF of w, F(w) = (e^{k(w-1)} - e^{-2k}) / (1 - e^{-2k}), and a uniform
 * azimuth about mu (two unit vectors orthogonal to mu complete the frame).  */
static void mix_sample(const omix *m, double u_mix, double u_w, double u_phi, const double uni[3],
                       double s[3])
{
    if (u_mix < MLP_EPS) { s[0] = uni[0]; s[1] = uni[1]; s[2] = uni[2]; return; }
    const double um = (u_mix - MLP_EPS) / (1.0 - MLP_EPS);
    int c = 2;
    if (um < m->alpha[0]) c = 0;
    else if (um < m->alpha[0] + m->alpha[1]) c = 1;
    const double k = m->kappa[c];
    const double *mu = m->mu[c];
    double w = 1.0 + log(u_w + (1.0 - u_w) * exp(-2.0 * k)) / k;
    if (w > 1.0) w = 1.0;
    if (w < -1.0) w = -1.0;
    /* e1: the coordinate axis least aligned with mu, made orthogonal to it */
    int ax = 0;
    if (fabs(mu[1]) < fabs(mu[ax])) ax = 1;
    if (fabs(mu[2]) < fabs(mu[ax])) ax = 2;
    double e1[3] = {0.0, 0.0, 0.0};
    e1[ax] = 1.0;
    const double d = mu[ax];
    for (int q = 0; q < 3; ++q) e1[q] -= d * mu[q];
    const double n1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int q = 0; q < 3; ++q) e1[q] /= n1;
    const double e2[3] = {mu[1] * e1[2] - mu[2] * e1[1], mu[2] * e1[0] - mu[0] * e1[2],
                          mu[0] * e1[1] - mu[1] * e1[0]};
    const double phi = 2.0 * M_PI * u_phi;
    const double rt = sqrt(1.0 - w * w > 0.0 ? 1.0 - w * w : 0.0);
    for (int q = 0; q < 3; ++q) s[q] = w * mu[q] + rt * (cos(phi) * e1[q] + sin(phi) * e2[q]);
}

/* set (or with NULL clear) the learned proposal's parameters */
int orc_set_proposal_mlp(octx *c, const double *theta)
{
    free(c->mlp);
    c->mlp = NULL;
    if (!theta) return ORC_OK;
    c->mlp = (double *)malloc(sizeof(double) * ORC_MLP_PARAMS);
    memcpy(c->mlp, theta, sizeof(double) * ORC_MLP_PARAMS);
    return ORC_OK;
}

int orc_mlp_param_count(void) { return ORC_MLP_PARAMS; }

/* ln q(s | x) and one draw, for tests: x[4], s[3]; u = (u_mix, u_w, u_phi),
 * uni[3] the direction used on the uniform branch */
double orc_mlp_log_q(const double *theta, const double x[4], const double s[3])
{
    double out[12];
    omix m;
    mlp_forward(theta, x, out);
    mlp_mixture(out, &m);
    return mix_log_q(&m, s);
}

void orc_mlp_sample(const double *theta, const double x[4], const double u[3], const double uni[3],
                    double s[3])
{
    double out[12];
    omix m;
    mlp_forward(theta, x, out);
    mlp_mixture(out, &m);
    mix_sample(&m, u[0], u[1], u[2], uni, s);
}

/* ------------------------------------------------------------------ */
/* Walkers.                                                            */
/* ------------------------------------------------------------------ */

/* Drive a walker from its starting configuration into its window:
 * propose plain moves, accept a move if it lands in the window or strictly
 * closer to it, stop on entry.  Fails after 10^4 N proposals.             */
typedef struct {
    uint32_t attempt;
    uint32_t flags;        /* bit0 accepted, bit1 the proposal lies in the window */
    double E;              /* energy before the attempt */
    double Eb;             /* proposed energy */
} odrive;

static int drive_into_window(octx *c, owalker *w)
{
    double *S = cfg_spins(c, w->cfg);
    int N = c->lat.N;
    int b;
    size_t widx = (size_t)(w - c->w);
    if (c->drive_len) c->drive_len[widx] = 0;
    if (in_window(c, w->E, w->lo, w->hi, &b)) { w->bin = b; return ORC_OK; }
    uint64_t cap = (uint64_t)10000 * (uint64_t)N;
    for (uint64_t n = 0; n < cap; ++n) {
        uint32_t r[4];
        draw(c->seed, w->stream, n, 0u, TAG_INIT_SITE, r);
        int i = pick_site(r[0], N);
        double sn[3], h[3];
        orc_sphere(c->seed, w->stream, n, TAG_INIT_SPHERE, sn);
        local_field(&c->lat, S, i, h);
        double Eb = w->E + coord_delta(c, S + 3 * (size_t)i, sn, h);
        int inside = in_window(c, Eb, w->lo, w->hi, &b);
        int acc = inside || window_distance(c, Eb, w->lo, w->hi) < window_distance(c, w->E, w->lo, w->hi);
        if (c->drive && n < (uint64_t)c->drive_cap) {
            odrive *d = (odrive *)(c->drive + (widx * (size_t)c->drive_cap + (size_t)n) * sizeof(odrive));
            d->attempt = (uint32_t)n;
            d->flags = (uint32_t)acc | ((uint32_t)inside << 1);
            d->E = w->E;
            d->Eb = Eb;
            c->drive_len[widx] = (int64_t)n + 1;
        }
        if (acc) {
            S[3 * (size_t)i] = sn[0]; S[3 * (size_t)i + 1] = sn[1]; S[3 * (size_t)i + 2] = sn[2];
            w->E = Eb;
            if (inside) { w->bin = b; return ORC_OK; }
        }
    }
    return ORC_EINIT;
}

/* record the first `cap` attempts of each walker's drive into its window at
 * the next orc_init (test mode; 0 turns it off) */
int orc_set_drive_trace(octx *c, int64_t cap)
{
    free(c->drive);
    free(c->drive_len);
    c->drive = NULL;
    c->drive_len = NULL;
    c->drive_cap = cap > 0 ? cap : 0;
    return ORC_OK;
}

/* walker's drive records: returns how many were written (<= cap) */
int64_t orc_read_drive(const octx *c, int walker, void *out, int64_t cap)
{
    if (!c->drive || walker < 0 || walker >= c->W) return ORC_EINVAL;
    int64_t n = c->drive_len[walker] < cap ? c->drive_len[walker] : cap;
    memcpy(out, c->drive + (size_t)walker * (size_t)c->drive_cap * sizeof(odrive), (size_t)n * sizeof(odrive));
    return n;
}

int orc_init(octx *c, uint32_t seed, const double *init_spins)
{
    if (c->B < 1 || c->seg_len < 1) return ORC_ESTATE;
    free_walkers(c);
    int N = c->lat.N;
    c->seed = seed;
    c->W = c->h * c->m;
    c->t = 0;
    c->w = (owalker *)calloc((size_t)c->W, sizeof(owalker));
    c->spins = (double *)malloc(sizeof(double) * 3 * (size_t)N * (size_t)c->W);
    c->xatt = (uint64_t *)calloc((size_t)(c->h > 1 ? c->h - 1 : 1), sizeof(uint64_t));
    c->xacc = (uint64_t *)calloc((size_t)(c->h > 1 ? c->h - 1 : 1), sizeof(uint64_t));
    if (c->trace_cap > 0) {
        free(c->trace);
        c->trace = (unsigned char *)calloc((size_t)c->W * (size_t)c->trace_cap, sizeof(otrace));
    }
    free(c->drive);
    free(c->drive_len);
    c->drive = NULL;
    c->drive_len = NULL;
    if (c->drive_cap > 0) {
        c->drive = (unsigned char *)calloc((size_t)c->W * (size_t)c->drive_cap, sizeof(odrive));
        c->drive_len = (int64_t *)calloc((size_t)c->W, sizeof(int64_t));
    }
    c->rtrip = (uint32_t *)calloc((size_t)c->W, sizeof(uint32_t));
    /* h_s: the largest sum of |J| over one site's neighbours */
    c->hs = 0.0;
    for (int i = 0; i < N; ++i) {
        double a = 0.0;
        for (int k = 0; k < c->lat.deg[i]; ++k) a += fabs(c->lat.Jn[(size_t)i * c->lat.zmax + k]);
        if (a > c->hs) c->hs = a;
    }
    int status = ORC_OK;
    for (int wi = 0; wi < c->W; ++wi) {
        owalker *w = &c->w[wi];
        w->stream = c->stream_base + (uint32_t)wi;
        w->win = wi / c->m;
        w->rep = wi % c->m;
        orc_window_bins(c->B, c->h, c->overlap, w->win, &w->lo, &w->hi);
        int nb = w->hi - w->lo;
        w->lng = (double *)calloc((size_t)nb, sizeof(double));      /* ln g~ = 0 */
        w->H = (uint32_t *)calloc((size_t)nb, sizeof(uint32_t));    /* H = 0 */
        w->vis = (uint8_t *)calloc((size_t)nb, sizeof(uint8_t));
        w->lnf = c->lnf_init;
        w->cfg = wi;
        double *S = cfg_spins(c, wi);
        for (int i = 0; i < N; ++i) {
            if (init_spins) {
                S[3 * i] = init_spins[3 * i]; S[3 * i + 1] = init_spins[3 * i + 1]; S[3 * i + 2] = init_spins[3 * i + 2];
            } else {
                /* an arbitrary start: every spin uniform on the sphere */
                orc_sphere(seed, w->stream, (uint64_t)i, TAG_INIT_CONFIG, S + 3 * (size_t)i);
            }
        }
        w->E = full_coord(c, S);
    }
    #pragma omp parallel for schedule(static) num_threads(c->n_threads > 0 ? c->n_threads : omp_get_max_threads())
    for (int wi = 0; wi < c->W; ++wi) {
        int st = drive_into_window(c, &c->w[wi]);
        if (st != ORC_OK) {
            #pragma omp critical
            status = st;
        }
    }
    c->inited = (status == ORC_OK);
    return status;
}

/* One Wang-Landau trial move of walker w (steps in the order of the
 * original algorithm: propose, evaluate E_B, accept with min(1, g_A/g_B),
 * times q(S_i|x)/q(S'|x) with the learned proposal, then multiply g~ and
 * increment H at the current state).                                    */
static void wl_attempt(octx *c, owalker *w)
{
    int N = c->lat.N;
    double *S = cfg_spins(c, w->cfg);
    uint64_t n = w->attempts;
    uint32_t r[4];
    draw(c->seed, w->stream, n, 0u, TAG_SITE, r);
    int i = pick_site(r[0], N);
    double u = u53(r[1], r[2]);
    double sn[3], h[3];
    orc_sphere(c->seed, w->stream, n, TAG_SPHERE, sn);
    local_field(&c->lat, S, i, h);
    double *si = S + 3 * (size_t)i;
    double lnq_ratio = 0.0;
    if (c->mlp) {
        /* x from the field at i (S_i is not part of it), so q(.|x) is the
         * same before and after the move */
        const double ec = c->Emin + 0.5 * (double)(w->lo + w->hi) * ((c->Emax - c->Emin) / (double)c->B);
        double x[4] = {h[0] / c->hs, h[1] / c->hs, h[2] / c->hs, ec / ((double)N * 0.5 * c->hs)};
        double out[12];
        omix m;
        mlp_forward(c->mlp, x, out);
        mlp_mixture(out, &m);
        uint32_t ru[4];
        draw(c->seed, w->stream, n, 0u, TAG_LEARNED, ru);
        const double u_mix = (double)(ru[0] >> 8) * (1.0 / 16777216.0);
        const double u_w = ((double)(ru[1] >> 8) + 0.5) * (1.0 / 16777216.0);
        const double u_phi = (double)(ru[2] >> 8) * (1.0 / 16777216.0);
        double uni[3] = {sn[0], sn[1], sn[2]};
        mix_sample(&m, u_mix, u_w, u_phi, uni, sn);
        lnq_ratio = mix_log_q(&m, si) - mix_log_q(&m, sn);
    }
    double Eb = w->E + coord_delta(c, si, sn, h);
    int bb;
    int acc = 0, outside = 0, newbin = 0;
    double lnb = 0.0;
    if (in_window(c, Eb, w->lo, w->hi, &bb)) {
        if (w->vis[bb - w->lo]) {
            lnb = w->lng[bb - w->lo];
        } else if (w->iter == 0 && !w->done) {
            /* A bin not yet visited, during the first iteration: the walker
             * is still discovering its range.  The bin still holds the
             * initial guess g~ = 1 (ln g~ = 0); it joins the range, and the
             * histogram restarts, when the walker enters it. */
            newbin = 1;
            lnb = w->lng[bb - w->lo];
        } else {
            /* after the first iteration the range is fixed */
            outside = 1;
        }
        if (!outside) {
            double lr = wl_log_ratio(w->lng[w->bin - w->lo], lnb) + lnq_ratio;
            acc = metropolis(lr, u);
        }
    } else {
        outside = 1;
    }
    if (outside) w->oow++;
    if (acc) {
        if (newbin) memset(w->H, 0, sizeof(uint32_t) * (size_t)(w->hi - w->lo));
        si[0] = sn[0]; si[1] = sn[1]; si[2] = sn[2];
        w->E = Eb;
        w->bin = bb;
        w->accepts++;
        if (c->check_energy) {
            double ef = full_coord(c, S);
            double err = fabs(ef - w->E);
            if (err > c->max_check_err) c->max_check_err = err;
        }
    }
    int j = w->bin - w->lo;
    if (!w->done) {
        w->lng[j] = w->lng[j] + w->lnf;
        w->H[j] = w->H[j] + 1u;
    }
    w->vis[j] = 1;
    if (c->trace && n < (uint64_t)c->trace_cap) {
        size_t widx = (size_t)(w - c->w);
        otrace *tr = (otrace *)(c->trace + (widx * (size_t)c->trace_cap + (size_t)n) * sizeof(otrace));
        tr->site = (uint32_t)i;
        tr->flags = (uint32_t)acc | ((uint32_t)outside << 1);
        tr->E = w->E;
        tr->bin = w->bin;
        tr->attempt_lo = (uint32_t)n;
    }
    w->attempts = n + 1;
}

/* Full-energy resynchronisation, done at the end of a segment in which the
 * walker's attempt count crossed a multiple of the resync interval.        */
static void maybe_resync(octx *c, owalker *w, uint64_t before)
{
    if (c->resync <= 0) return;
    uint64_t R = (uint64_t)c->resync;
    if (w->attempts / R == before / R) return;
    double ef = full_coord(c, cfg_spins(c, w->cfg));
    double d = fabs(ef - w->E);
    if (d > w->max_drift) w->max_drift = d;
    w->E = ef;
    double x = (ef - c->Emin) * c->inv_de;
    int b;
    if (x < (double)w->lo) b = w->lo;
    else if (x >= (double)w->hi) b = w->hi - 1;
    else b = (int)floor(x);
    w->bin = b;
}

/* Flatness over visited bins: flat iff den * min H * n_vis >= num * sum H,
 * i.e. min H >= p <H> with p = num/den; not flat if the segment visited a
 * new bin.  On a flat histogram: stop if ln f <= ln f_final, else halve
 * ln f (f -> sqrt f), reset H, keep ln g~.                               */
static void flatness_check(octx *c, owalker *w)
{
    if (w->done) return;
    int nb = w->hi - w->lo;
    int nvis = 0;
    uint64_t sum = 0;
    uint32_t mn = 0xFFFFFFFFu;
    for (int j = 0; j < nb; ++j) {
        if (!w->vis[j]) continue;
        nvis++;
        sum += w->H[j];
        if (w->H[j] < mn) mn = w->H[j];
    }
    int flat = 0;
    if (nvis > w->nvis_prev) {
        flat = 0;
    } else if (nvis > 0 && sum > 0) {
        flat = (uint64_t)c->flat_den * (uint64_t)mn * (uint64_t)nvis >= (uint64_t)c->flat_num * sum;
    }
    w->nvis_prev = nvis;
    if (!flat) return;
    if (c->share) {
        /* the window's walkers advance together (see window_merge) */
        w->ready = 1;
        return;
    }
    if (w->lnf <= c->lnf_final) {
        w->done = 1;
        return;
    }
    w->lnf = w->lnf * 0.5;
    w->iter++;
    memset(w->H, 0, sizeof(uint32_t) * (size_t)nb);
}

/* Several walkers per window sharing their estimate (the multiple-walker
 * form of the parallel scheme, refined in the REWL literature the paper
 * cites): a walker whose histogram is flat keeps walking at its ln f until
 * every walker of its window is flat; then each bin's ln g~ becomes the
 * mean over the walkers that visited it (walkers taken in order), every
 * walker gets that estimate and the union of the visited bins, H restarts,
 * and ln f halves for all of them (or all finish, when the iteration ran at
 * ln f <= ln f_final).  All walkers of a window do the same number of moves
 * at the same ln f, so their estimates carry the same total and are
 * averaged without shifts. */
static void window_merge(octx *c)
{
    int m = c->m;
    for (int k = 0; k < c->h; ++k) {
        owalker *w0 = &c->w[k * m];
        int all = 1;
        for (int r = 0; r < m; ++r) all &= c->w[k * m + r].ready && !c->w[k * m + r].done;
        if (!all) continue;
        int nb = w0->hi - w0->lo;
        int nvis = 0;
        for (int j = 0; j < nb; ++j) {
            double sum = 0.0;
            int cnt = 0;
            for (int r = 0; r < m; ++r) {
                owalker *w = &c->w[k * m + r];
                if (w->vis[j]) { sum = sum + w->lng[j]; cnt++; }
            }
            if (cnt == 0) continue;
            double mean = sum / (double)cnt;
            for (int r = 0; r < m; ++r) {
                owalker *w = &c->w[k * m + r];
                w->lng[j] = mean;
                w->vis[j] = 1;
            }
            nvis++;
        }
        int finish = w0->lnf <= c->lnf_final;
        for (int r = 0; r < m; ++r) {
            owalker *w = &c->w[k * m + r];
            w->ready = 0;
            w->nvis_prev = nvis;
            if (finish) {
                w->done = 1;
            } else {
                w->lnf = w->lnf * 0.5;
                w->iter++;
                memset(w->H, 0, sizeof(uint32_t) * (size_t)nb);
            }
        }
    }
}

/* the walk's coordinate: 0 energy (default), 1 magnetisation M_z (before
 * orc_init; windows and bins are then over M_z) */
int orc_set_coordinate(octx *c, int coord)
{
    if (coord != 0 && coord != 1) return ORC_EINVAL;
    c->coord = coord;
    return ORC_OK;
}

/* turn window sharing on or off (before orc_init) */
int orc_set_share(octx *c, int on)
{
    c->share = on ? 1 : 0;
    return ORC_OK;
}

/* Replica exchange between windows k and k+1 for all k of the parity of the
 * step counter.  The m walkers of window k are paired with those of window
 * k+1 through a random permutation (Fisher-Yates); a pair can swap only if
 * both energies lie in both windows; the swap exchanges configurations.  */
static void exchange_step(octx *c)
{
    int m = c->m;
    int *perm = (int *)malloc(sizeof(int) * (size_t)m);
    uint64_t t = (uint64_t)c->t;
    for (int k = (int)(t & 1u); k + 1 < c->h; k += 2) {
        for (int r = 0; r < m; ++r) perm[r] = r;
        for (int i = m - 1; i >= 1; --i) {
            uint32_t rr[4];
            draw(c->seed, c->instance, t, ((uint32_t)k << 16) | (uint32_t)i, TAG_PERM, rr);
            int j = (int)(((uint64_t)rr[0] * (uint64_t)(uint32_t)(i + 1)) >> 32);
            int tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
        }
        for (int r = 0; r < m; ++r) {
            owalker *a = &c->w[k * m + r];
            owalker *b = &c->w[(k + 1) * m + perm[r]];
            int ba_in_b, bb_in_a;
            c->xatt[k]++;
            if (!in_window(c, a->E, b->lo, b->hi, &ba_in_b)) continue;
            if (!in_window(c, b->E, a->lo, a->hi, &bb_in_a)) continue;
            /* the bins the walkers hold (which a resync may have clamped),
             * which the swap hands over and the ratio reads, must lie in the
             * other window, and each walker's estimate must exist at the bin
             * it receives */
            if (a->bin < b->lo || a->bin >= b->hi || b->bin < a->lo || b->bin >= a->hi) continue;
            if (!b->vis[a->bin - b->lo] || !a->vis[b->bin - a->lo]) continue;
            uint32_t rr[4];
            draw(c->seed, c->instance, t, ((uint32_t)k << 16) | (uint32_t)r, TAG_EXCH, rr);
            double u = u53(rr[0], rr[1]);
            double lr = re_log_ratio(a->lng[a->bin - a->lo], a->lng[b->bin - a->lo],
                                     b->lng[b->bin - b->lo], b->lng[a->bin - b->lo]);
            if (!metropolis(lr, u)) continue;
            c->xacc[k]++;
            int tc = a->cfg; a->cfg = b->cfg; b->cfg = tc;
            double te = a->E; a->E = b->E; b->E = te;
            int tb = a->bin; a->bin = b->bin; b->bin = tb;
        }
    }
    free(perm);
    /* Replica diffusion (the round trips of Fig. 1 of the results): a
     * configuration now held by a walker of the lowest window whose last
     * extreme window was the highest one (or the reverse) has made one more
     * half trip. */
    if (c->h >= 2) {
        for (int e = 0; e < 2; ++e) {
            const int win = e == 0 ? 0 : c->h - 1;
            const uint32_t ext = e == 0 ? 1u : 2u;
            for (int r = 0; r < m; ++r) {
                uint32_t *v = &c->rtrip[c->w[win * m + r].cfg];
                uint32_t last = *v & 3u, trips = *v >> 2;
                if (last == ext) continue;
                if (last != 0u) trips += 1u;
                *v = (trips << 2) | ext;
            }
        }
    }
}

int orc_all_done(const octx *c)
{
    for (int i = 0; i < c->W; ++i) if (!c->w[i].done) return 0;
    return 1;
}

/* Run up to n_segments segments; each is seg_len trial moves per walker,
 * then resync (when due) and the flatness test per walker, then one exchange
 * step.  Returns the number of segments run; stops early once every walker
 * is done.                                                               */
int64_t orc_run(octx *c, int64_t n_segments)
{
    if (!c->inited) return ORC_ESTATE;
    int64_t done_segs = 0;
    for (int64_t s = 0; s < n_segments; ++s) {
        if (orc_all_done(c)) break;
        #pragma omp parallel for schedule(static) num_threads(c->n_threads > 0 ? c->n_threads : omp_get_max_threads())
        for (int wi = 0; wi < c->W; ++wi) {
            owalker *w = &c->w[wi];
            uint64_t before = w->attempts;
            for (int64_t a = 0; a < c->seg_len; ++a) wl_attempt(c, w);
            maybe_resync(c, w, before);
            flatness_check(c, w);
        }
        if (c->share) window_merge(c);
        exchange_step(c);
        c->t++;
        done_segs++;
    }
    return done_segs;
}

/* one exchange step on its own (tests) */
int orc_exchange(octx *c)
{
    if (!c->inited) return ORC_ESTATE;
    if (c->share) window_merge(c);
    exchange_step(c);
    c->t++;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Read-out.                                                           */
/* ------------------------------------------------------------------ */
int orc_num_walkers(const octx *c) { return c->W; }

int orc_window(const octx *c, int walker, int *lo, int *hi)
{
    if (walker < 0 || walker >= c->W) return ORC_EINVAL;
    *lo = c->w[walker].lo; *hi = c->w[walker].hi;
    return ORC_OK;
}

int orc_read_lng(const octx *c, int walker, double *out, int cap)
{
    if (walker < 0 || walker >= c->W) return ORC_EINVAL;
    const owalker *w = &c->w[walker];
    int nb = w->hi - w->lo;
    for (int j = 0; j < nb && j < cap; ++j) out[j] = w->lng[j];
    return nb;
}

int orc_read_hist(const octx *c, int walker, uint32_t *out, uint8_t *vis, int cap)
{
    if (walker < 0 || walker >= c->W) return ORC_EINVAL;
    const owalker *w = &c->w[walker];
    int nb = w->hi - w->lo;
    for (int j = 0; j < nb && j < cap; ++j) { out[j] = w->H[j]; if (vis) vis[j] = w->vis[j]; }
    return nb;
}

/* walker state: E, lnf, max_drift as doubles; bin, iter, done, cfg, nvis as
 * ints; attempts, accepts, out-of-window as u64 */
int orc_read_walker(const octx *c, int walker, double *d3, int32_t *i5, uint64_t *u3)
{
    if (walker < 0 || walker >= c->W) return ORC_EINVAL;
    const owalker *w = &c->w[walker];
    d3[0] = w->E; d3[1] = w->lnf; d3[2] = w->max_drift;
    i5[0] = w->bin; i5[1] = w->iter; i5[2] = w->done; i5[3] = w->cfg; i5[4] = w->nvis_prev;
    u3[0] = w->attempts; u3[1] = w->accepts; u3[2] = w->oow;
    return ORC_OK;
}

int orc_read_config(const octx *c, int cfg, double *out)
{
    if (cfg < 0 || cfg >= c->W) return ORC_EINVAL;
    memcpy(out, c->spins + (size_t)cfg * 3 * (size_t)c->lat.N, sizeof(double) * 3 * (size_t)c->lat.N);
    return ORC_OK;
}

int orc_read_exchange_stats(const octx *c, uint64_t *att, uint64_t *acc)
{
    for (int k = 0; k + 1 < c->h; ++k) { att[k] = c->xatt[k]; acc[k] = c->xacc[k]; }
    return c->h - 1;
}

int64_t orc_step_counter(const octx *c) { return c->t; }

int orc_read_trace(const octx *c, int walker, void *out, int64_t cap)
{
    if (!c->trace || walker < 0 || walker >= c->W) return ORC_EINVAL;
    int64_t n = cap < c->trace_cap ? cap : c->trace_cap;
    memcpy(out, c->trace + (size_t)walker * (size_t)c->trace_cap * sizeof(otrace), (size_t)n * sizeof(otrace));
    return (int)n;
}

/* half trips per configuration (see the exchange step) */
int orc_read_round_trips(const octx *c, uint32_t *out, int cap)
{
    if (!c->rtrip) return ORC_ESTATE;
    for (int i = 0; i < c->W && i < cap; ++i) out[i] = c->rtrip[i] >> 2;
    return c->W;
}

/* Replace a walker's ln g~ (and its visited bins, NULL = all) over its
 * window, e.g. to run with fixed weights; the bins count as seen by the
 * flatness test's new-bin rule.  A bin marked not visited holds the initial
 * guess ln g~ = 0. */
int orc_write_lng(octx *c, int walker, const double *lng, const uint8_t *vis, int cap)
{
    if (!c->inited || walker < 0 || walker >= c->W || !lng) return ORC_EINVAL;
    owalker *w = &c->w[walker];
    int nb = w->hi - w->lo;
    int nvis = 0;
    for (int j = 0; j < nb && j < cap; ++j) {
        w->vis[j] = vis ? (vis[j] != 0) : 1;
        w->lng[j] = w->vis[j] ? lng[j] : 0.0;
    }
    w->vis[w->bin - w->lo] = 1;
    for (int j = 0; j < nb; ++j) nvis += w->vis[j];
    w->nvis_prev = nvis;
    return ORC_OK;
}

/* Test mode: add `delta` to a walker's running energy, as an accumulated
 * rounding drift would; the next resync must undo it. */
int orc_shift_energy(octx *c, int walker, double delta)
{
    if (!c->inited || walker < 0 || walker >= c->W) return ORC_EINVAL;
    c->w[walker].E += delta;
    return ORC_OK;
}
