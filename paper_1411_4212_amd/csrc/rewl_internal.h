// rewl_internal.h -- layouts shared by the librewl host code and its kernels.
#pragma once

#include <stdint.h>
#include <hip/hip_runtime.h>
#include "../../include/rewl.h"

namespace rewl {

enum Lattice : int32_t { LAT_BCC = 0, LAT_TABLE = 1 };

// Philox stream tags: the fourth counter word of every draw.
enum Tag : uint32_t {
    TAG_SITE = 0,          // site choice and acceptance uniform of a trial move
    TAG_SPHERE = 1,        // proposal direction of a trial move
    TAG_INIT_SITE = 2,     // drive into the window: site
    TAG_INIT_SPHERE = 3,   // drive into the window: direction
    TAG_EXCH = 4,          // replica-exchange acceptance uniform
    TAG_PERM = 5,          // pairing permutation of an exchange step
    TAG_INIT_CONFIG = 6,   // random initial configuration
    TAG_LEARNED = 7        // learned proposal: mixture choice, w and azimuth uniforms
};

// Read-only description of one REWL instance.
struct InstDesc {
    int32_t N, L, lattice, z;          // sites, cells per edge, lattice kind, neighbours/site
    int32_t h, m, B, walker_base;      // windows, walkers/window, global bins, first walker
    int32_t n_walkers, slot_off, flat_num, flat_den;
    int32_t xstat_off, nb_max, deg_off;   // deg_off: first entry in the degree table
    float inv_hs;                         // 1 / sum_n z_n |J_n| (learned-proposal features)
    int32_t share;                        // 1: the walkers of a window share ln g (merged when all are flat)
    int32_t fslot_off;                    // the fast sweep's 16 Q slots, grouped by memory row
    int32_t layout;                       // storage order of a configuration in HBM (spin_slot): -1 or 0
    int32_t lg_L;                         // log2 L when L is a power of two, else 0
    int32_t coord;                        // the walk's coordinate: 0 energy, 1 magnetisation M_z
    int32_t pad_coord;
    double Emin, inv_de, lnf_final, lnf_init;
    int64_t seg_len, resync;
    int64_t cfg_off;                   // spin element offset of configuration 0
    int64_t tab_off;                   // element offset in the neighbour table
    int64_t init_off;                  // double offset of the caller's start spins, -1 = random
};

// Read-only description of one walker.
struct WalkerDesc {
    int32_t inst, win, lo, hi;         // instance, window, window bins [lo, hi)
    int64_t bin_off;                   // element offset of its window in LNG/HIST/VISITED
    uint32_t stream;                   // global walker id: second Philox key word
    int32_t local;                     // index within its instance
    float e_w;                         // window centre energy per spin / (h_s / 2)
    int32_t pad;
};

// Dynamic per-walker state (device).
struct WalkerState {
    double E, lnf, max_drift;
    int32_t bin, cfg, iter, done, nvis, status;
    int32_t ready;                     // window sharing: flat in this iteration, waiting for its window
    int32_t pad_ready;
    uint64_t attempts, accepts, oow;
    uint64_t harvested;                // training records written
};

// One bcc neighbour slot: cell displacement for a site on sublattice 0 and
// on sublattice 1, whether the neighbour is on the other sublattice, and
// the shell's coupling.
struct BccSlot {
    int8_t d[2][3];
    uint8_t flip;
    uint8_t real;      // fast-sweep tables: 1 for a neighbour, 0 for a padding slot (J = 0)
    float Jf;
    double Jd;
};

// Per-instance control words (device, CONTROL buffer).
struct InstControl {
    int32_t done;
    int32_t pad;
};

// Work queue of the persistent kernel (CONTROL buffer).  A slot holds
// (sequence << 32 | walker); slot j starts with sequence j (empty).  A
// producer of ticket p waits for sequence p, writes (p + 1, walker); the
// consumer of ticket p waits for p + 1 and leaves p + capacity.
struct PersistCtl {
    uint32_t head, tail;       // consumer / producer tickets
    uint32_t finished;         // instances that have stopped
    uint32_t all_done;         // set once every instance has stopped
    uint32_t error;            // a bounded wait ran out
    uint32_t pad[11];
};

struct KArgs {
    void *spins;
    WalkerState *state;
    double *lng;
    uint32_t *hist;
    uint8_t *vis;
    const InstDesc *inst;
    const WalkerDesc *wdesc;
    const BccSlot *slots;
    const int32_t *tdeg;
    const int32_t *tnbr;
    const double *tJ;
    const double *init_spins;
    InstControl *ictl;
    unsigned long long *xatt;
    unsigned long long *xacc;
    uint32_t *rtrip;           // per configuration: (half trips << 2) | last extreme window (1 low, 2 high)
    rewl_trace_rec *trace;
    int64_t trace_cap;
    int64_t t;                 // exchange step counter
    uint32_t seed;
    int32_t n_walkers;
    int32_t n_inst;
    int32_t walkers_per_block;
    int32_t lds_spins_bytes;   // bytes of LDS for spins per walker slot
    int32_t lds_bins;          // window bins per walker slot in LDS
    int32_t lds_bin_bytes;     // LDS bytes per bin: 13 (ln g, H, visited) or 8 (ln g only)
    int32_t fast_q;            // >0: fast sweep kernel with this many neighbour slots per lane
    int32_t all_pow2;          // every instance has L a power of two
    int32_t spins_in_lds;      // 1: configurations staged in LDS; 0: read in place from HBM
    int32_t harvest_every;     // record every k-th move
    const void *mlp;           // packed learned-proposal network (nullptr: uniform proposal)
    float *harvest;            // training records [walker][harvest_cap][8] (nullptr: off)
    int64_t harvest_cap;
    // persistent kernel
    PersistCtl *pctl;
    uint32_t *p_arrive;        // per instance: walker arrivals in this launch
    uint32_t *p_rounds;        // per instance: rounds completed in this launch
    unsigned long long *p_slots;
    uint32_t p_mask;           // queue capacity - 1 (power of two >= walkers)
    int32_t p_max_rounds;
    uint64_t p_spin_limit;     // polls before a wait gives up
};

// Storage slot of site i (site order ((s L + z) L + y) L + x) in a
// configuration held in HBM.  layout < 0: the site order itself.  layout = 0
// (bcc, L = 2^k): cells in site order with the two sublattice sites of a cell
// side by side, slot = 2 (i mod L^3) + s, so that the two sublattices' rows
// of a move's stencil share cache lines.
__host__ __device__ inline int spin_slot(int i, int layout, int k)
{
    if (layout < 0) return i;
    const uint32_t u = (uint32_t)i, c = u & ((1u << (3 * k)) - 1u);
    return (int)((c << 1) | (u >> (3 * k)));
}

constexpr int kWave = 64;

// Record an error for rewl_last_error() and return `code`.
rewl_status report_error(rewl_status code, const char *msg);

int launch_mlp_pack(const float *dev_params, void *dev_packed, hipStream_t s);

// Kernel launchers (rewl_kernels.hip).
int launch_init(const KArgs &a, int mode, hipStream_t s, size_t lds_per_walker);
int launch_sweep(const KArgs &a, int mode, hipStream_t s, size_t lds_per_walker);
int launch_exchange(const KArgs &a, hipStream_t s);
// Persistent form: every instance runs up to a.p_max_rounds rounds
// (segment + exchange) in one launch; `n_cu` compute units.
int launch_persistent(const KArgs &a, int mode, hipStream_t s, size_t lds_per_walker, int n_cu,
                      int max_blocks, int *grid_out);

}  // namespace rewl
