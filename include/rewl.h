/*
 * rewl.h -- C ABI of librewl: replica-exchange Wang-Landau (REWL) sampling of
 * the classical Heisenberg model on MI355X (gfx950).
 *
 * The calls follow the paper's statement of the problem (Perera, Li,
 * Eisenbach, Vogel, Landau, "Replica-exchange Wang-Landau sampling: pushing
 * the limits of Monte Carlo simulations in materials sciences"):
 *   - a Hamiltonian H = -sum_{i<j} J_ij S_i.S_j with unit spins   (Model, Eq. 1)
 *   - a bcc lattice of L^3 cells, N = 2 L^3 spins, couplings by
 *     neighbour shell                                             (Model)
 *   - a restricted global range [E_min, E_max] and bin width     (Model; Sec. original WL)
 *   - h windows overlapping by the ratio o, m walkers each        (Sec. parallel scheme)
 *   - replica exchange between adjacent windows after a fixed
 *     number of trial moves                                       (Sec. parallel scheme; Sec. simulation details)
 *   - flatness fraction p and final modification factor f_min    (Sec. original WL; Sec. simulation details)
 * and return the g~(E) fragments of every walker (Sec. parallel scheme).
 *
 * Conventions
 *   - Every call returns REWL_OK (0) or a negative REWL_E* code; the text of
 *     the last error of the calling thread is rewl_last_error().  No C++
 *     exception crosses this interface.
 *   - Call order: rewl_create -> rewl_add_instance + rewl_set_lattice_* +
 *     rewl_set_windows + rewl_set_schedule for every instance ->
 *     rewl_query_sizes -> rewl_bind_buffers -> rewl_init_walkers ->
 *     rewl_run / rewl_exchange / rewl_poll -> rewl_read_*.  A call out of
 *     order returns REWL_ESTATE.
 *   - Host arrays passed in are copied during the call; the caller keeps
 *     ownership.  Device buffers are allocated by the caller (for instance
 *     as PyTorch tensors) with the sizes rewl_query_sizes reports, must be
 *     256-byte aligned and must outlive the context.  The library itself
 *     never allocates device memory.
 *   - Work is enqueued on the HIP stream given to rewl_create.  rewl_run and
 *     rewl_exchange return before the GPU finishes; rewl_poll, rewl_read_*
 *     and rewl_init_walkers synchronise that stream.  A kernel fault shows up
 *     at the next synchronising call as REWL_EDEVICE.
 *   - Energies are in units of the couplings (k_B = 1).  Bins are global
 *     indices on [E_min, E_max) with bin(E) = floor((E - E_min) * B /
 *     (E_max - E_min)); windows are half-open bin ranges [lo, hi).
 *   - Random numbers: Philox4x32-10 with key (seed, walker id) and counter
 *     (attempt low word, attempt high word, draw, stream tag), so a run is
 *     reproducible from its seed.
 */
#ifndef REWL_H
#define REWL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rewl_ctx rewl_ctx;
typedef int32_t rewl_status;

enum {
    REWL_OK = 0,
    REWL_EINVAL = -1,       /* bad argument */
    REWL_ESTATE = -2,       /* call out of order */
    REWL_EDEVICE = -3,      /* HIP runtime error or kernel fault */
    REWL_ERANGE = -4,       /* a size exceeds a documented limit */
    REWL_EINIT = -5,        /* a walker could not be driven into its window */
    REWL_ENUMERIC = -6,     /* non-finite ln g or energy detected */
    REWL_ECORRUPT = -7,     /* checkpoint damaged or from another configuration */
    REWL_EUNSUPPORTED = -8  /* combination not implemented */
};

/* Arithmetic modes of the trial-move kernel.
 *  FP64_DET  all arithmetic in FP64 in the canonical sequential order (local
 *            field summed over the neighbour list in list order), so the
 *            trajectory is reproducible bit for bit; spins FP64 in LDS.
 *  FP64      FP64 spins and local field, lanes gather neighbours in
 *            parallel and sum them with a wavefront reduction.
 *  FP32_DE   FP32 spins, local field and energy change; the running energy,
 *            ln g, bins and the periodic full-energy resync stay FP64.       */
enum { REWL_MODE_FP64_DET = 0, REWL_MODE_FP64 = 1, REWL_MODE_FP32_DE = 2 };

/* Device buffers the caller allocates (indices into the size/pointer arrays). */
enum {
    REWL_BUF_SPINS = 0,     /* configurations, one per walker              */
    REWL_BUF_STATE = 1,     /* per-walker dynamic state                    */
    REWL_BUF_LNG = 2,       /* ln g~ per walker window bin, FP64           */
    REWL_BUF_HIST = 3,      /* H per walker window bin, uint32             */
    REWL_BUF_VISITED = 4,   /* visited flag per walker window bin, uint8   */
    REWL_BUF_PARAMS = 5,    /* read-only lattice / window tables           */
    REWL_BUF_CONTROL = 6,   /* per-instance flags and exchange counters    */
    REWL_NBUF = 7
};

/* Limits. */
#define REWL_MAX_DEGREE 128          /* neighbours per site                     */
#define REWL_MAX_SHELLS 8            /* bcc shells                               */
#define REWL_MAX_WALKERS_PER_WINDOW 64
#define REWL_MAX_WINDOW_BINS 4096

/* Per-walker state as read back by rewl_read_walker_state. */
typedef struct {
    double E;                /* running energy of the configuration held     */
    double lnf;              /* current ln f                                 */
    double max_drift;        /* largest |E_running - E_full| seen at resync  */
    int32_t bin;             /* global bin of E                              */
    int32_t config;          /* index of the configuration held (in instance) */
    int32_t iteration;       /* number of ln f halvings so far               */
    int32_t done;            /* 1 once the iteration with ln f <= ln f_final was flat */
    int32_t n_visited;       /* bins visited so far                          */
    int32_t window;          /* window index                                 */
    uint64_t attempts;       /* trial moves made                             */
    uint64_t accepts;        /* trial moves accepted                         */
    uint64_t rejected_outside; /* proposals outside the window or range      */
} rewl_walker_state;

/* One trial move of the per-attempt trace (rewl_set_trace). 24 bytes. */
typedef struct {
    uint32_t site;
    uint32_t flags;          /* bit0 accepted, bit1 proposal outside window  */
    double E;                /* energy after the move                        */
    int32_t bin;             /* bin after the move                           */
    uint32_t attempt_lo;     /* low word of the attempt number               */
} rewl_trace_rec;

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the null stream), in arithmetic mode `mode`. */
rewl_status rewl_create(rewl_ctx **out, int32_t device, void *hip_stream, int32_t mode);

/* Destroy a context (NULL-safe).  Does not free caller-owned buffers. */
void rewl_destroy(rewl_ctx *ctx);

/* Add one independent REWL run; its index is written to *instance_id_out.
 * A context may hold many instances of different sizes (batched runs). */
rewl_status rewl_add_instance(rewl_ctx *ctx, int32_t *instance_id_out);

/* Periodic bcc lattice of L^3 cells (N = 2 L^3 spins, Model section) with
 * couplings J[n] on the n-th neighbour shell, n < n_shells <= 8; shell n
 * holds the lattice vectors of the n-th smallest length.  Site index
 * ((s L + z) L + y) L + x for sublattice s and cell (x, y, z).  Requires
 * that no two neighbours of a site coincide under the periodic wrap. */
rewl_status rewl_set_lattice_bcc(rewl_ctx *ctx, int32_t inst, int32_t L, int32_t n_shells,
                                 const double *J);

/* Arbitrary couplings (Model, Eq. 1): pair p couples spins i[p] and j[p]
 * with J[p]; each site's neighbour list is built in pair order.  Intended for
 * small test systems (spins read from global memory for the neighbours). */
rewl_status rewl_set_couplings_explicit(rewl_ctx *ctx, int32_t inst, int32_t N, int64_t n_pairs,
                                        const int32_t *i, const int32_t *j, const double *J);

/* Global range [E_min, E_max) on n_global_bins bins, split into n_windows
 * windows of equal width overlapping by the ratio `overlap` (parallel
 * scheme): w = round(B / (1 + (h-1)(1-o))) bins per window, window k starts
 * at round(k (B - w)/(h - 1)), round(x) = floor(x + 1/2).  Each window holds
 * walkers_per_window walkers. */
rewl_status rewl_set_windows(rewl_ctx *ctx, int32_t inst, double E_min, double E_max,
                             int32_t n_global_bins, int32_t n_windows, double overlap,
                             int32_t walkers_per_window);

/* Wang-Landau schedule (Sec. original WL): flat iff min H >= (flat_num /
 * flat_den) <H> over visited bins; ln f starts at lnf_init and halves on every
 * flat histogram; a walker is done when the iteration with ln f <= lnf_final
 * is flat.  exchange_interval trial moves per walker form one segment; the
 * flatness test and one replica-exchange step follow every segment.  The
 * energy is recomputed from scratch at the end of every segment in which the
 * walker's attempt count crosses a multiple of resync_interval (0 = never). */
rewl_status rewl_set_schedule(rewl_ctx *ctx, int32_t inst, int32_t flat_num, int32_t flat_den,
                              double lnf_init, double lnf_final, int64_t exchange_interval,
                              int64_t resync_interval);

/* Window sharing (before rewl_query_sizes; default off): the m walkers of a
 * window advance through the iterations together.  A walker whose histogram
 * is flat keeps walking at its ln f until every walker of its window is flat;
 * at the next exchange step each bin's ln g~ becomes the mean over the
 * walkers that visited it (summed in walker order), every walker takes that
 * estimate and the union of the visited bins, H restarts and ln f halves for
 * all of them (or all finish).  This is the multiple-walker refinement of the
 * parallel scheme from the replica-exchange Wang-Landau literature the paper
 * cites (Sec. parallel scheme, several walkers per window); off, each walker
 * proceeds independently, as the paper's own runs do.  on: 0 or 1, else
 * REWL_EINVAL; REWL_ESTATE after rewl_query_sizes. */
rewl_status rewl_set_window_sharing(rewl_ctx *ctx, int32_t inst, int32_t on);

/* The walk's coordinate (before rewl_query_sizes; default 0): 0 = the energy
 * of Eq. 1; 1 = the magnetisation along z, M_z = sum_i S_i^z (Sec. original
 * WL: the density of states may be taken over another order parameter).
 * With 1, rewl_set_windows' E_min, E_max and bins are over M_z, every E in the
 * walker state and trace holds M_z, and the walk runs in the generic sweep
 * kernel (a context with such an instance has no fast sweep, persistent
 * form or learned proposal: those calls return REWL_EUNSUPPORTED).
 * coord outside {0, 1}: REWL_EINVAL; after rewl_query_sizes: REWL_ESTATE. */
rewl_status rewl_set_coordinate(rewl_ctx *ctx, int32_t inst, int32_t coord);

/* Launch shape of the trial-move kernel (after rewl_query_sizes).
 * walkers_per_block: 1..4 walkers (one wavefront each) per workgroup
 * (several workgroups share a compute unit when LDS allows).
 * residency: 0 = automatic (configurations in LDS when a configuration, its
 * window and the look-ahead batch fit in 160 KB, else read and written in
 * place in HBM), 1 = LDS, 2 = HBM (FP32_DE / FP64 modes on bcc lattices).
 * Fails with REWL_EUNSUPPORTED when the shape does not fit, leaving the
 * previous shape in place. */
rewl_status rewl_set_launch(rewl_ctx *ctx, int32_t walkers_per_block, int32_t residency);

/* Grid cap of rewl_run_persistent calls that pass max_blocks = 0: at most
 * max_blocks blocks (0 = every block that can be resident).  Set by the
 * autotuner's persistent form; rewl_set_launch clears it.  Negative:
 * REWL_EINVAL. */
rewl_status rewl_set_grid_cap(rewl_ctx *ctx, int32_t max_blocks);

/* The grid cap in use (rewl_set_grid_cap).  Null argument: REWL_EINVAL. */
rewl_status rewl_get_grid_cap(rewl_ctx *ctx, int32_t *max_blocks);

/* The launch shape in use: walkers per block, 1 if configurations are staged
 * in LDS, and LDS bytes per workgroup. */
rewl_status rewl_get_launch(rewl_ctx *ctx, int32_t *walkers_per_block, int32_t *spins_in_lds,
                            int64_t *lds_bytes_per_block);

/* Launch-shape autotuner.  Times `segments` segments (rewl_run, or one
 * rewl_run_persistent call if persistent != 0) for every walkers-per-block
 * count in {1, 2, 4} and residency in {LDS, HBM} that the context can use.
 * In the persistent form each shape is timed first with every resident
 * block, then with the grid halved, a quarter, ... (down to 1/16) for as
 * long as each step is faster than the one before (where the memory system
 * saturates, fewer walkers in flight can be faster).  The walk's state is
 * restored before each trial and at the end, so that the walk itself is
 * unchanged; then the fastest shape and, in the persistent form, its grid
 * cap (rewl_set_grid_cap) are applied.  entries[] (may be NULL) receives up
 * to cap trials (at most 30), *n_out (may be NULL) their number.
 * Synchronises the stream; walkers must be initialised.  Needs host memory
 * for one copy of the device buffers. */
typedef struct {
    int32_t walkers_per_block;
    int32_t residency;         /* 1: configurations in LDS, 2: in HBM        */
    int32_t persistent;        /* 1: timed with rewl_run_persistent          */
    int32_t status;            /* REWL_OK, or why the shape was not usable   */
    double ms_per_segment;     /* < 0 when not usable                        */
    int32_t max_blocks;        /* persistent grid cap of the trial, 0 = none */
    int32_t pad;
} rewl_tune_entry;

rewl_status rewl_autotune(rewl_ctx *ctx, int32_t segments, int32_t persistent, rewl_tune_entry *entries,
                          int32_t cap, int32_t *n_out);

/* 64-bit digest of everything that fixes the meaning of the context's
 * buffers (mode, sizes, instance and lattice tables): equal digests mean
 * interchangeable checkpoints and launch-shape choices. */
rewl_status rewl_fingerprint(rewl_ctx *ctx, uint64_t *digest_out);

/* Byte sizes of the REWL_NBUF device buffers the caller must provide. */
rewl_status rewl_query_sizes(rewl_ctx *ctx, size_t *bytes_out /* [REWL_NBUF] */);

/* Hand the library its device buffers (caller-owned, 256-byte aligned) and
 * upload the read-only tables.  Synchronises the stream. */
rewl_status rewl_bind_buffers(rewl_ctx *ctx, void *const *dev_ptrs /* [REWL_NBUF] */);

/* Start every walker: ln g~ = 0, H = 0, ln f = lnf_init (Sec. original WL);
 * configuration = init_spins (N*3 doubles per instance, concatenated in
 * instance order) or, if NULL, every spin uniform on the sphere; then each
 * walker is driven into its window by moves accepted when they enter the
 * window or come strictly closer to it (at most 10^4 N moves, else
 * REWL_EINIT).  Synchronises the stream. */
rewl_status rewl_init_walkers(rewl_ctx *ctx, uint64_t seed, const double *init_spins);

/* Enqueue n_segments segments: exchange_interval trial moves per walker,
 * the resync when due and the flatness test, then one replica-exchange step
 * (Sec. parallel scheme).  Instances whose walkers are all done are skipped.
 * Asynchronous. */
rewl_status rewl_run(rewl_ctx *ctx, int64_t n_segments);

/* The same walk as rewl_run(ctx, max_rounds) in ONE persistent launch
 * (FP64 and FP32_DE modes on bcc lattices): each instance advances on its
 * own, a round being a segment of each of its walkers followed by its
 * exchange step, until it is done or has run max_rounds rounds; instances of
 * uneven size therefore never wait for each other.  Wavefronts take walkers
 * from a device work queue, and the last walker of an instance to finish a
 * round runs the exchange.  The results are bit-identical to rewl_run's.
 * The grid is as many blocks (of rewl_set_launch's walkers per block) as
 * are resident at once, at most one walker per wavefront, and at most
 * max_blocks if max_blocks > 0 (max_blocks = 0: the rewl_set_grid_cap cap,
 * if any); *grid_out (may be NULL) receives it.  Synchronises the stream;
 * REWL_EDEVICE if a bounded device wait ran out, REWL_ERANGE if
 * max_rounds * walkers >= 2^31 - queue capacity, REWL_EUNSUPPORTED in
 * FP64_DET mode or on explicit couplings. */
rewl_status rewl_run_persistent(rewl_ctx *ctx, int64_t max_rounds, int32_t max_blocks, int32_t *grid_out);

/* Enqueue the trial-move part of one segment only: exchange_interval trial
 * moves per walker, the resync when due and the flatness test, without the
 * exchange step (rewl_run = rewl_sweep + rewl_exchange, repeated).
 * Asynchronous. */
rewl_status rewl_sweep(rewl_ctx *ctx);

/* Enqueue one replica-exchange step on its own.  Asynchronous. */
rewl_status rewl_exchange(rewl_ctx *ctx);

/* Synchronise and report whether every instance is done. */
rewl_status rewl_poll(rewl_ctx *ctx, int32_t *all_done_out);

/* Read-out (synchronising).  inst = instance, walker = index within it
 * (walker w belongs to window w / m).  rewl_read_lng / rewl_read_hist /
 * rewl_read_visited copy min(cap, hi - lo) entries of the walker's window
 * and return that count through *n_out. */
rewl_status rewl_read_lng(rewl_ctx *ctx, int32_t inst, int32_t walker, double *out, int32_t cap,
                          int32_t *n_out);
rewl_status rewl_read_hist(rewl_ctx *ctx, int32_t inst, int32_t walker, uint32_t *out,
                           int32_t cap, int32_t *n_out);
rewl_status rewl_read_visited(rewl_ctx *ctx, int32_t inst, int32_t walker, uint8_t *out,
                              int32_t cap, int32_t *n_out);
rewl_status rewl_read_walker_state(rewl_ctx *ctx, int32_t inst, int32_t walker,
                                   rewl_walker_state *out);
/* Overwrite a walker's ln g~ (and visited flags; NULL = all visited) for its
 * window, min(cap, hi - lo) entries from `lng` (host); a bin marked not
 * visited holds the initial guess ln g~ = 0.  With ln f ~ 0 and a flatness
 * fraction of 1 this runs a fixed-weight (multicanonical) walk; it also
 * restores a saved estimate.  Synchronises the stream. */
rewl_status rewl_write_lng(rewl_ctx *ctx, int32_t inst, int32_t walker, const double *lng,
                           const uint8_t *visited, int32_t cap);

/* configuration `config` of instance inst as N*3 doubles */
rewl_status rewl_read_config(rewl_ctx *ctx, int32_t inst, int32_t config, double *out,
                             int64_t cap);
rewl_status rewl_read_window(rewl_ctx *ctx, int32_t inst, int32_t win, int32_t *lo_bin,
                             int32_t *hi_bin);
/* exchange attempts / accepts of the window pairs (k, k+1), k < h-1 */
rewl_status rewl_read_exchange_stats(rewl_ctx *ctx, int32_t inst, uint64_t *attempts,
                                     uint64_t *accepts, int32_t cap);
/* number of exchange steps made so far */
rewl_status rewl_read_step(rewl_ctx *ctx, int64_t *step_out);

/* Record the first `capacity` trial moves of every walker into the device
 * buffer dev_records (caller-owned, capacity * total walkers records of
 * rewl_trace_rec, walker-major in instance order); NULL switches recording
 * off.  Call before rewl_init_walkers. */
rewl_status rewl_set_trace(rewl_ctx *ctx, void *dev_records, int64_t capacity);

/* ------------------------------------------------------------------------
 * Learned proposal (an extension; the paper's trial move is a uniform new
 * direction, Sec. simulation details).  The new direction is drawn from a
 * mixture of three von Mises-Fisher densities and an eps = 0.05 uniform
 * part, q(s|x), whose parameters an MLP 4 -> 64 -> 64 -> 12 (ReLU) computes
 * from x = (h / h_s, e_w): h the local field at the site (without the site's
 * own spin), h_s = sum_n z_n |J_n|, e_w the window centre energy per spin in
 * units of h_s / 2.  Acceptance min(1, g(E_A) q(S_i|x) / (g(E_B) q(S'|x)))
 * keeps the Wang-Landau walk exact.  Inference uses BF16 MFMA with FP32
 * accumulation; training FP32.  Parameters: one FP32 vector of
 * rewl_mlp_param_count() values in the order W1[64][4], b1[64], W2[64][64],
 * b2[64], W3[12][64], b3[12]; outputs 4c..4c+3 are (v_c, a_c) of component c
 * with kappa_c = clip(|v_c|, 1e-3, 1e3), mu_c = v_c/|v_c|, alpha = softmax(a).
 * Training records are 8 floats: x0..x3, s0..s2 (unit spin), unused.
 * ------------------------------------------------------------------------ */
int32_t rewl_mlp_param_count(void);

/* Bytes of the packed (per-lane BF16 MFMA layout) network. */
size_t rewl_mlp_packed_bytes(void);

/* Device workspace bytes for rewl_mlp_train (batch) or rewl_mlp_loss_grad (n). */
rewl_status rewl_mlp_workspace_bytes(int64_t max_batch, size_t *bytes);

/* Pack FP32 parameters (device) into the inference layout (device). */
rewl_status rewl_mlp_pack(const float *dev_params, void *dev_packed, void *hip_stream);

/* Evaluate the packed network on n inputs (device arrays): x[n][4], s[n][3],
 * uniforms u[n][3] = (u_mix, u_w, u_phi) in [0,1) (u_w > 0), uniform
 * directions udir[n][3]; writes ln q(s|x), a draw s' ~ q(.|x) and ln q(s'|x). */
rewl_status rewl_mlp_eval(const void *dev_packed, const float *dev_x, const float *dev_s,
                          const float *dev_u, const float *dev_udir, float *dev_lnq_s,
                          float *dev_sample, float *dev_lnq_sample, int64_t n, void *hip_stream);

/* Mean negative log-likelihood of n records and its gradient (device),
 * FP32, summed in a fixed order (deterministic).  Synchronises the stream. */
rewl_status rewl_mlp_loss_grad(const float *dev_records, int64_t n, const float *dev_params,
                               float *dev_grad, double *loss_out, void *dev_workspace,
                               void *hip_stream);

/* Adam (lr, beta 0.9/0.999) on minibatches of `batch` records drawn with
 * replacement by Philox(seed); epochs x (n / batch) steps; parameters updated
 * in place (device); loss_per_epoch (host, optional) gets each epoch's mean
 * minibatch loss.  Synchronises the stream. */
rewl_status rewl_mlp_train(const float *dev_records, int64_t n, int32_t epochs, int32_t batch,
                           float lr, uint64_t seed, float *dev_params, void *dev_workspace,
                           float *loss_per_epoch, void *hip_stream);

/* rewl_mlp_train without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The workspace is a file-scope
 * device array of the library, one per GPU (2.8 MB, minibatches of at most
 * 8192 records; a larger batch returns REWL_ERANGE); the calling thread's
 * current device is used, and hip_stream must belong to it.  The call
 * allocates nothing.  Calls that overlap on one GPU share that array and
 * race: serialise them (one stream, or synchronise between calls).  The
 * results equal rewl_mlp_train's bit for bit. */
rewl_status rewl_mlp_train_static(const float *dev_records, int64_t n, int32_t epochs, int32_t batch,
                                  float lr, uint64_t seed, float *dev_params, float *loss_per_epoch,
                                  void *hip_stream);

/* Proposal of a context: kind 0 = uniform direction, 1 = learned (FP32
 * parameters on the device, packed into the context).  FP32_DE mode, bcc
 * lattices. */
rewl_status rewl_set_proposal(rewl_ctx *ctx, int32_t kind, const float *dev_params);

/* Record (x, S_i) of every every_k-th trial move (before the move) into
 * dev_records[walker][capacity_per_walker][8] (device, caller-owned, walker
 * global index in instance order); NULL switches recording off.  Uniform
 * proposal, fast kernel.  rewl_read_harvest_counts gives records per walker. */
rewl_status rewl_set_harvest(rewl_ctx *ctx, float *dev_records, int64_t capacity_per_walker,
                             int32_t every_k);
rewl_status rewl_read_harvest_counts(rewl_ctx *ctx, int64_t *counts, int32_t cap);

/* Checkpoint / restore.  rewl_save writes every device buffer of the
 * context (configurations, ln g, H, visited flags, walker states, tables,
 * the packed learned network, exchange counters) plus the exchange step,
 * seed and proposal kind to `path` (host file, overwritten), after
 * synchronising the stream.  rewl_load needs a context configured with the
 * same instances, mode and launch-independent layout and with buffers bound;
 * it restores that state, after which rewl_run continues exactly as the
 * saved context would have (bit-identical in every mode, since all random
 * numbers are functions of (seed, walker, attempt count)).  Harvest and trace
 * targets are not part of the state.  Errors: REWL_EINVAL (file cannot be
 * opened, read or written), REWL_ECORRUPT (bad magic, short file, or a
 * fingerprint of the configuration that differs from this context's). */
rewl_status rewl_save(rewl_ctx *ctx, const char *path);
rewl_status rewl_load(rewl_ctx *ctx, const char *path);

/* Replica diffusion (the paper's Fig. 1, Sec. results): for each of the
 * instance's configurations (index = the `config` field of the walker
 * states), the number of half round trips between the lowest and the
 * highest window, counted at exchange steps (a configuration held by a
 * walker of an extreme window whose last extreme visited was the other
 * one).  half_trips: host, min(cap, walkers of the instance) entries.
 * Synchronises the stream. */
rewl_status rewl_read_round_trips(rewl_ctx *ctx, int32_t inst, uint32_t *half_trips, int32_t cap);

/* Totals over all walkers of the context (synchronising). */
rewl_status rewl_total_attempts(rewl_ctx *ctx, uint64_t *attempts, uint64_t *accepts);

/* Human-readable text of the calling thread's last error. */
const char *rewl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* REWL_H */
