// rewl_api.cpp -- host side of librewl: configuration, validation, device
// buffer layout, kernel launches and read-out.  See include/rewl.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rewl_internal.h"

using namespace rewl;

namespace {

thread_local std::string g_last_error;

rewl_status fail(rewl_status code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(REWL_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

struct InstanceCfg {
    bool has_lattice = false, has_windows = false, has_schedule = false;
    int32_t lattice = LAT_BCC;
    int32_t L = 0, N = 0;
    std::vector<double> Jshell;
    std::vector<int32_t> pi, pj;
    std::vector<double> pJ;
    double Emin = 0, Emax = 0, overlap = 0;
    int32_t B = 0, h = 0, m = 0;
    int32_t flat_num = 0, flat_den = 1;
    double lnf_init = 1.0, lnf_final = 1e-8;
    int64_t seg = 0, resync = 0;
    int32_t share = 0;
    int32_t coord = 0;
    // derived
    int32_t z = 0;
    std::vector<int32_t> lo, hi;
};

int round_half_up(double x) { return (int)std::floor(x + 0.5); }



// The fast sweep's neighbour slots: 16 Q entries, slot k read by lane group
// member (k mod 16) / 4 in column (k / 16, k mod 4) -- one load instruction
// per column.  Neighbours in one memory row of the configuration (same
// sublattice and the same y and z cell offsets, consecutive x cells) are put
// into one column, so that one instruction touches each cache line of the
// stencil once; rows longer than a column are split.  Columns are filled
// first-fit in order of decreasing row length; padding slots carry J = 0 and
// point at the site itself (a line the move reads anyway).  If the rows do
// not fit, the shell order is kept.
std::vector<BccSlot> fast_slot_table(const BccSlot *sl, int z, int Q)
{
    const int ncol = 4 * Q;
    BccSlot pad{};
    std::vector<BccSlot> out((size_t)16 * Q, pad);
    // rows keyed by (flip, dz, dy) of the sublattice-0 displacement, cells by x
    std::vector<std::vector<int>> rows;
    std::vector<std::array<int, 3>> keys;
    for (int k = 0; k < z; ++k) {
        const std::array<int, 3> key = {sl[k].flip, sl[k].d[0][2], sl[k].d[0][1]};
        size_t r = 0;
        while (r < keys.size() && keys[r] != key) ++r;
        if (r == keys.size()) {
            keys.push_back(key);
            rows.emplace_back();
        }
        rows[r].push_back(k);
    }
    std::vector<std::vector<int>> pieces;
    for (auto &row : rows) {
        std::stable_sort(row.begin(), row.end(), [&](int a, int b) { return sl[a].d[0][0] < sl[b].d[0][0]; });
        for (size_t i = 0; i < row.size(); i += 4)
            pieces.emplace_back(row.begin() + i, row.begin() + std::min(row.size(), i + 4));
    }
    std::stable_sort(pieces.begin(), pieces.end(),
                     [](const std::vector<int> &a, const std::vector<int> &b) { return a.size() > b.size(); });
    std::vector<std::vector<int>> cols;
    for (const auto &pc : pieces) {
        size_t c = 0;
        while (c < cols.size() && cols[c].size() + pc.size() > 4) ++c;
        if (c == cols.size()) cols.emplace_back();
        cols[c].insert(cols[c].end(), pc.begin(), pc.end());
    }
    if ((int)cols.size() > ncol) {
        for (int k = 0; k < z; ++k) {
            out[k] = sl[k];
            out[k].real = 1;
        }
        return out;
    }
    for (size_t c = 0; c < cols.size(); ++c)
        for (size_t r = 0; r < cols[c].size(); ++r) {
            const size_t k = 16 * (c / 4) + 4 * r + (c % 4);
            out[k] = sl[cols[c][r]];
            out[k].real = 1;
        }
    return out;
}

// bcc lattice vectors in half-cell units (integer triples of equal parity),
// grouped in shells of increasing length, lexicographic within a shell.
struct ShellVec {
    int dx, dy, dz, shell;
};

std::vector<ShellVec> bcc_shell_vectors(int n_shells)
{
    std::vector<std::array<int, 4>> all;   // d2, dx, dy, dz
    for (int a = -5; a <= 5; ++a)
        for (int b = -5; b <= 5; ++b)
            for (int c = -5; c <= 5; ++c) {
                if (a == 0 && b == 0 && c == 0) continue;
                if ((a & 1) != (b & 1) || (a & 1) != (c & 1)) continue;
                all.push_back({a * a + b * b + c * c, a, b, c});
            }
    std::sort(all.begin(), all.end());
    std::vector<ShellVec> out;
    int shell = -1, last_d2 = -1;
    for (const auto &v : all) {
        if (v[0] != last_d2) {
            ++shell;
            last_d2 = v[0];
        }
        if (shell >= n_shells) break;
        out.push_back({v[1], v[2], v[3], shell});
    }
    return out;
}

}  // namespace

rewl_status rewl::report_error(rewl_status code, const char *msg) { return fail(code, msg); }

struct rewl_ctx {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    int32_t mode = 0;
    std::vector<InstanceCfg> inst;
    int stage = 0;   // 0 configuring, 1 sized, 2 bound, 3 initialised
    size_t sizes[REWL_NBUF] = {};
    void *buf[REWL_NBUF] = {};
    // host copies of the tables
    std::vector<InstDesc> idesc;
    std::vector<WalkerDesc> wdesc;
    std::vector<BccSlot> slots;
    std::vector<int32_t> tdeg, tnbr;
    std::vector<double> tJ;
    std::vector<double> init_host;
    // PARAMS layout (byte offsets)
    size_t off_inst = 0, off_wdesc = 0, off_slots = 0, off_tdeg = 0, off_tnbr = 0, off_tJ = 0,
           off_init = 0;
    // CONTROL layout
    size_t off_ictl = 0, off_xatt = 0, off_xacc = 0, off_rtrip = 0;
    size_t off_pctl = 0, off_parr = 0, off_prnd = 0, off_pslots = 0;
    uint32_t p_cap = 0;
    int32_t last_grid = 0;
    int32_t grid_cap = 0;        // persistent grid cap for max_blocks = 0 (0: none)
    int32_t n_walkers = 0, n_xstat = 0;
    int64_t total_bins = 0, total_spins = 0;
    int32_t lds_spins_bytes = 0, lds_bins = 0;
    size_t lds_per_walker = 0;
    int32_t max_N = 0;
    int32_t residency_req = 0;   // 0 auto, 1 LDS, 2 HBM
    int32_t wpb_req = 1;
    int32_t spins_in_lds = 1;
    size_t off_mlp = 0;          // packed learned-proposal network in PARAMS
    int32_t proposal = 0;        // 0 uniform, 1 learned
    float *harvest = nullptr;
    int64_t harvest_cap = 0;
    int32_t harvest_every = 1;
    int32_t wpb = 1;
    int32_t fast_q = 0;
    int32_t all_pow2 = 0;
    uint32_t seed = 0;
    int64_t t = 0;
    rewl_trace_rec *trace = nullptr;
    int64_t trace_cap = 0;
};

namespace {

size_t spin_bytes(int mode) { return mode == REWL_MODE_FP32_DE ? 16 : 32; }
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

rewl_status check_inst(rewl_ctx *c, int32_t inst)
{
    if (!c) return fail(REWL_EINVAL, "null context");
    if (inst < 0 || inst >= (int32_t)c->inst.size()) return fail(REWL_EINVAL, "bad instance index");
    if (c->stage != 0) return fail(REWL_ESTATE, "instances can only be configured before rewl_query_sizes");
    return REWL_OK;
}

KArgs make_args(rewl_ctx *c)
{
    KArgs a{};
    unsigned char *P = (unsigned char *)c->buf[REWL_BUF_PARAMS];
    unsigned char *Cb = (unsigned char *)c->buf[REWL_BUF_CONTROL];
    a.spins = c->buf[REWL_BUF_SPINS];
    a.state = (WalkerState *)c->buf[REWL_BUF_STATE];
    a.lng = (double *)c->buf[REWL_BUF_LNG];
    a.hist = (uint32_t *)c->buf[REWL_BUF_HIST];
    a.vis = (uint8_t *)c->buf[REWL_BUF_VISITED];
    a.inst = (const InstDesc *)(P + c->off_inst);
    a.wdesc = (const WalkerDesc *)(P + c->off_wdesc);
    a.slots = c->slots.empty() ? nullptr : (const BccSlot *)(P + c->off_slots);
    a.tdeg = c->tdeg.empty() ? nullptr : (const int32_t *)(P + c->off_tdeg);
    a.tnbr = c->tnbr.empty() ? nullptr : (const int32_t *)(P + c->off_tnbr);
    a.tJ = c->tJ.empty() ? nullptr : (const double *)(P + c->off_tJ);
    a.init_spins = c->init_host.empty() ? nullptr : (const double *)(P + c->off_init);
    a.ictl = (InstControl *)(Cb + c->off_ictl);
    a.xatt = (unsigned long long *)(Cb + c->off_xatt);
    a.xacc = (unsigned long long *)(Cb + c->off_xacc);
    a.rtrip = (uint32_t *)(Cb + c->off_rtrip);
    a.pctl = (PersistCtl *)(Cb + c->off_pctl);
    a.p_arrive = (uint32_t *)(Cb + c->off_parr);
    a.p_rounds = (uint32_t *)(Cb + c->off_prnd);
    a.p_slots = (unsigned long long *)(Cb + c->off_pslots);
    a.p_mask = c->p_cap - 1u;
    a.p_max_rounds = 0;
    a.trace = c->trace;
    a.trace_cap = c->trace_cap;
    a.t = c->t;
    a.seed = c->seed;
    a.n_walkers = c->n_walkers;
    a.n_inst = (int32_t)c->inst.size();
    a.walkers_per_block = c->wpb;
    a.lds_spins_bytes = c->spins_in_lds ? c->lds_spins_bytes : 0;
    a.spins_in_lds = c->spins_in_lds;
    a.mlp = c->proposal == 1 ? (const void *)(P + c->off_mlp) : nullptr;
    a.harvest = c->harvest;
    a.harvest_cap = c->harvest_cap;
    a.harvest_every = c->harvest_every;
    a.lds_bins = c->lds_bins;
    a.lds_bin_bytes = c->spins_in_lds ? 13 : 8;
    a.fast_q = c->fast_q;
    a.all_pow2 = c->all_pow2;
    return a;
}

// Where configurations live during a segment and how many walkers share a
// workgroup: LDS when the configuration, its window and the look-ahead batch
// fit in 160 KB, otherwise in place in HBM (fast kernel only).
rewl_status plan_launch(rewl_ctx *c)
{
    // spins in LDS: spins, ln g, H and visited flags (13 B per bin); spins
    // in HBM (fast kernel): ln g only (8 B per bin), H stays in HBM
    const size_t bins = ((size_t)c->lds_bins * 8u + 15) & ~(size_t)15;
    const size_t batch = 64 * 64;
    const size_t with_spins = (((size_t)c->lds_spins_bytes + (size_t)c->lds_bins * 13u + 15) & ~(size_t)15) + batch;
    const size_t without = bins + batch;
    const size_t cap = 160 * 1024;
    bool in_lds;
    if (c->residency_req == 1) in_lds = true;
    else if (c->residency_req == 2) in_lds = false;
    else in_lds = with_spins <= cap || c->fast_q == 0;
    if (!in_lds && c->fast_q == 0)
        return fail(REWL_EUNSUPPORTED, "spins in HBM need the fast kernel (FP32_DE/FP64 mode, bcc lattice)");
    const size_t per = in_lds ? with_spins : without;
    if (per * (size_t)c->wpb_req > cap)
        return fail(REWL_EUNSUPPORTED, "walkers per block x LDS per walker exceeds 160 KB");
    c->spins_in_lds = in_lds ? 1 : 0;
    c->lds_per_walker = per;
    c->wpb = c->wpb_req;
    return REWL_OK;
}

// Build the read-only tables and compute buffer sizes.
rewl_status finalize(rewl_ctx *c)
{
    if (c->inst.empty()) return fail(REWL_ESTATE, "no instance added");
    c->idesc.clear();
    c->wdesc.clear();
    c->slots.clear();
    c->tdeg.clear();
    c->tnbr.clear();
    c->tJ.clear();
    int64_t bin_off = 0, cfg_off = 0;
    int32_t walker_base = 0, xstat = 0;
    int32_t max_N = 0, max_nb = 0;
    for (size_t ii = 0; ii < c->inst.size(); ++ii) {
        InstanceCfg &q = c->inst[ii];
        if (!q.has_lattice || !q.has_windows || !q.has_schedule)
            return fail(REWL_ESTATE, "instance " + std::to_string(ii) +
                                         " needs lattice, windows and schedule");
        InstDesc d{};
        d.N = q.N;
        d.L = q.L;
        d.lattice = q.lattice;
        d.h = q.h;
        d.m = q.m;
        d.B = q.B;
        d.walker_base = walker_base;
        d.n_walkers = q.h * q.m;
        d.flat_num = q.flat_num;
        d.flat_den = q.flat_den;
        d.xstat_off = xstat;
        d.Emin = q.Emin;
        d.inv_de = (double)q.B / (q.Emax - q.Emin);
        d.lnf_final = q.lnf_final;
        d.lnf_init = q.lnf_init;
        d.seg_len = q.seg;
        d.resync = q.resync;
        d.share = q.share;
        d.coord = q.coord;
        d.layout = -1;
        d.lg_L = 0;
        if (q.lattice == LAT_BCC && (q.L & (q.L - 1)) == 0) {
            // sublattices interleaved per cell: on the L=32 eight-shell
            // workload 7 % faster than the site order, and 1-4 % ahead of
            // bricks of 2, 4 and 8 cells per edge (measured, not kept)
            while ((1 << d.lg_L) < q.L) ++d.lg_L;
            d.layout = 0;
        }
        d.cfg_off = cfg_off;
        d.init_off = -1;
        if (q.lattice == LAT_BCC) {
            std::vector<ShellVec> v = bcc_shell_vectors((int)q.Jshell.size());
            d.z = (int32_t)v.size();
            d.slot_off = (int32_t)c->slots.size();
            // every neighbour of a site must be a distinct other site
            std::vector<int> seen;
            for (int s = 0; s < 2; ++s) {
                seen.clear();
                for (const ShellVec &sv : v) {
                    const int t = s ^ (sv.dx & 1);
                    auto w = [&](int base, int dd) {
                        int x = (base + (s + dd - t) / 2) % q.L;
                        return x < 0 ? x + q.L : x;
                    };
                    const int idx = ((t * q.L + w(0, sv.dz)) * q.L + w(0, sv.dy)) * q.L + w(0, sv.dx);
                    if (idx == s * q.L * q.L * q.L) return fail(REWL_EINVAL, "lattice too small: a neighbour wraps onto the site");
                    if (std::find(seen.begin(), seen.end(), idx) != seen.end())
                        return fail(REWL_EINVAL, "lattice too small: two neighbours coincide under the periodic wrap");
                    seen.push_back(idx);
                }
            }
            for (const ShellVec &sv : v) {
                BccSlot sl{};
                const int dd[3] = {sv.dx, sv.dy, sv.dz};
                for (int s = 0; s < 2; ++s) {
                    const int t = s ^ (sv.dx & 1);
                    for (int k = 0; k < 3; ++k) sl.d[s][k] = (int8_t)((s + dd[k] - t) / 2);
                }
                sl.flip = (uint8_t)(sv.dx & 1);
                sl.Jd = q.Jshell[sv.shell];
                sl.Jf = (float)sl.Jd;
                c->slots.push_back(sl);
            }
        } else {
            std::vector<int32_t> deg(q.N, 0);
            for (size_t p = 0; p < q.pi.size(); ++p) {
                deg[q.pi[p]]++;
                deg[q.pj[p]]++;
            }
            int zmax = 1;
            for (int i = 0; i < q.N; ++i) zmax = std::max(zmax, deg[i]);
            if (zmax > REWL_MAX_DEGREE) return fail(REWL_ERANGE, "a site has more than 128 neighbours");
            d.z = zmax;
            d.tab_off = (int64_t)c->tnbr.size();
            d.deg_off = (int32_t)c->tdeg.size();
            const size_t base = c->tnbr.size();
            c->tnbr.resize(base + (size_t)q.N * zmax, 0);
            c->tJ.resize(base + (size_t)q.N * zmax, 0.0);
            std::vector<int32_t> fill(q.N, 0);
            for (size_t p = 0; p < q.pi.size(); ++p) {
                const int a = q.pi[p], b = q.pj[p];
                c->tnbr[base + (size_t)a * zmax + fill[a]] = b;
                c->tJ[base + (size_t)a * zmax + fill[a]] = q.pJ[p];
                fill[a]++;
                c->tnbr[base + (size_t)b * zmax + fill[b]] = a;
                c->tJ[base + (size_t)b * zmax + fill[b]] = q.pJ[p];
                fill[b]++;
            }
            c->tdeg.insert(c->tdeg.end(), deg.begin(), deg.end());
        }
        if (d.z > REWL_MAX_DEGREE) return fail(REWL_ERANGE, "more than 128 neighbours per site");
        {
            // h_s = sum of |J| over a site's neighbours (largest over sites)
            double hs = 0.0;
            if (q.lattice == LAT_BCC) {
                for (int k = 0; k < d.z; ++k) hs += std::fabs(c->slots[d.slot_off + k].Jd);
            } else {
                std::vector<double> acc(q.N, 0.0);
                for (size_t p = 0; p < q.pi.size(); ++p) {
                    acc[q.pi[p]] += std::fabs(q.pJ[p]);
                    acc[q.pj[p]] += std::fabs(q.pJ[p]);
                }
                for (double v : acc) hs = std::max(hs, v);
            }
            d.inv_hs = hs > 0.0 ? (float)(1.0 / hs) : 0.f;
        }
        // windows
        q.lo.assign(q.h, 0);
        q.hi.assign(q.h, 0);
        int wb = round_half_up((double)q.B / (1.0 + (double)(q.h - 1) * (1.0 - q.overlap)));
        wb = std::max(1, std::min(wb, q.B));
        int nb_max = 0;
        for (int k = 0; k < q.h; ++k) {
            const int l = q.h == 1 ? 0 : round_half_up((double)k * (double)(q.B - wb) / (double)(q.h - 1));
            q.lo[k] = l;
            q.hi[k] = l + wb;
            nb_max = std::max(nb_max, wb);
        }
        if (nb_max > REWL_MAX_WINDOW_BINS) return fail(REWL_ERANGE, "more than 4096 bins per window");
        d.nb_max = nb_max;
        for (int k = 0; k < q.h; ++k)
            for (int r = 0; r < q.m; ++r) {
                WalkerDesc wd{};
                wd.inst = (int32_t)ii;
                wd.win = k;
                wd.lo = q.lo[k];
                wd.hi = q.hi[k];
                wd.bin_off = bin_off;
                wd.stream = (uint32_t)(walker_base + k * q.m + r);
                wd.local = k * q.m + r;
                {
                    const double de = (q.Emax - q.Emin) / (double)q.B;
                    const double ec = q.Emin + 0.5 * (double)(q.lo[k] + q.hi[k]) * de;
                    const double hs = d.inv_hs > 0.f ? 1.0 / (double)d.inv_hs : 1.0;
                    wd.e_w = (float)(ec / ((double)q.N * 0.5 * hs));
                }
                bin_off += wd.hi - wd.lo;
                c->wdesc.push_back(wd);
            }
        walker_base += q.h * q.m;
        xstat += std::max(q.h - 1, 1);
        cfg_off += (int64_t)q.N * q.h * q.m;
        max_N = std::max(max_N, q.N);
        max_nb = std::max(max_nb, nb_max);
        c->idesc.push_back(d);
    }
    // lattice-table offsets of the degree array: fix up after the loop
    c->n_walkers = walker_base;
    c->n_xstat = xstat;
    c->total_bins = bin_off;
    c->total_spins = cfg_off;
    c->max_N = max_N;
    c->lds_spins_bytes = (int32_t)(((size_t)max_N * spin_bytes(c->mode) + 15) & ~(size_t)15);
    c->lds_bins = (max_nb + 15) & ~15;
    // the fast kernel covers bcc lattices with L a power of two or L <= 64
    c->fast_q = 0;
    if (c->mode != REWL_MODE_FP64_DET) {
        bool ok = true, p2 = true;
        int zmax = 0;
        for (size_t ii = 0; ii < c->inst.size(); ++ii) {
            const InstanceCfg &q = c->inst[ii];
            const bool pow2 = (q.L & (q.L - 1)) == 0;
            // the fast sweep walks in energy only
            ok &= q.lattice == LAT_BCC && q.L >= 4 && (pow2 || q.L <= 64) && q.coord == 0;
            p2 &= pow2;
            zmax = std::max(zmax, c->idesc[ii].z);
        }
        if (ok) c->fast_q = zmax <= 16 ? 1 : (zmax <= 64 ? 4 : 8);
        c->all_pow2 = p2 ? 1 : 0;
    }
    if (c->fast_q > 0) {
        for (size_t ii = 0; ii < c->inst.size(); ++ii) {
            InstDesc &d = c->idesc[ii];
            d.fslot_off = (int32_t)c->slots.size();
            const std::vector<BccSlot> f = fast_slot_table(&c->slots[d.slot_off], d.z, c->fast_q);
            c->slots.insert(c->slots.end(), f.begin(), f.end());
        }
    }
    {
        rewl_status st = plan_launch(c);
        if (st) return st;
    }
    size_t o = 0;
    c->off_inst = o;
    o = align256(o + sizeof(InstDesc) * c->idesc.size());
    c->off_wdesc = o;
    o = align256(o + sizeof(WalkerDesc) * c->wdesc.size());
    c->off_slots = o;
    o = align256(o + sizeof(BccSlot) * c->slots.size());
    c->off_tdeg = o;
    o = align256(o + sizeof(int32_t) * c->tdeg.size());
    c->off_tnbr = o;
    o = align256(o + sizeof(int32_t) * c->tnbr.size());
    c->off_tJ = o;
    o = align256(o + sizeof(double) * c->tJ.size());
    c->off_mlp = o;
    o = align256(o + rewl_mlp_packed_bytes());
    c->off_init = o;
    int64_t init_doubles = 0;
    for (auto &q : c->inst) init_doubles += 3 * (int64_t)q.N;
    o = align256(o + sizeof(double) * (size_t)init_doubles);
    c->sizes[REWL_BUF_PARAMS] = std::max<size_t>(o, 256);

    c->sizes[REWL_BUF_SPINS] = align256(spin_bytes(c->mode) * (size_t)c->total_spins);
    c->sizes[REWL_BUF_STATE] = align256(sizeof(WalkerState) * (size_t)c->n_walkers);
    c->sizes[REWL_BUF_LNG] = align256(sizeof(double) * (size_t)c->total_bins);
    c->sizes[REWL_BUF_HIST] = align256(sizeof(uint32_t) * (size_t)c->total_bins);
    c->sizes[REWL_BUF_VISITED] = align256((size_t)c->total_bins);
    size_t oc = 0;
    c->off_ictl = oc;
    oc = align256(oc + sizeof(InstControl) * c->inst.size());
    c->off_xatt = oc;
    oc = align256(oc + sizeof(unsigned long long) * (size_t)c->n_xstat);
    c->off_xacc = oc;
    oc = align256(oc + sizeof(unsigned long long) * (size_t)c->n_xstat);
    c->off_rtrip = oc;
    oc = align256(oc + sizeof(uint32_t) * (size_t)c->n_walkers);
    // persistent-kernel queue: capacity a power of two above every walker
    // plus every wavefront that may hold a ticket
    c->p_cap = 256;
    while (c->p_cap < 2u * (uint32_t)c->n_walkers + 256u) c->p_cap <<= 1;
    c->off_pctl = oc;
    oc = align256(oc + sizeof(PersistCtl));
    c->off_parr = oc;
    oc = align256(oc + sizeof(uint32_t) * c->inst.size());
    c->off_prnd = oc;
    oc = align256(oc + sizeof(uint32_t) * c->inst.size());
    c->off_pslots = oc;
    oc = align256(oc + sizeof(unsigned long long) * (size_t)c->p_cap);
    c->sizes[REWL_BUF_CONTROL] = oc;
    return REWL_OK;
}

rewl_status sync_check(rewl_ctx *c)
{
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(REWL_EDEVICE, std::string("stream: ") + hipGetErrorString(e));
    return REWL_OK;
}

rewl_status check_walker(rewl_ctx *c, int32_t inst, int32_t walker, int *gw)
{
    if (!c) return fail(REWL_EINVAL, "null context");
    if (c->stage < 3) return fail(REWL_ESTATE, "walkers not initialised");
    if (inst < 0 || inst >= (int32_t)c->inst.size()) return fail(REWL_EINVAL, "bad instance index");
    const InstDesc &d = c->idesc[inst];
    if (walker < 0 || walker >= d.n_walkers) return fail(REWL_EINVAL, "bad walker index");
    *gw = d.walker_base + walker;
    return REWL_OK;
}

}  // namespace

extern "C" {

const char *rewl_last_error(void) { return g_last_error.c_str(); }

rewl_status rewl_create(rewl_ctx **out, int32_t device, void *hip_stream, int32_t mode)
{
    if (!out) return fail(REWL_EINVAL, "null output pointer");
    *out = nullptr;
    if (mode < REWL_MODE_FP64_DET || mode > REWL_MODE_FP32_DE) return fail(REWL_EINVAL, "unknown mode");
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(REWL_EINVAL, "bad device index");
    rewl_ctx *c = new (std::nothrow) rewl_ctx();
    if (!c) return fail(REWL_EINVAL, "out of host memory");
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->mode = mode;
    *out = c;
    return REWL_OK;
}

void rewl_destroy(rewl_ctx *ctx) { delete ctx; }

rewl_status rewl_add_instance(rewl_ctx *ctx, int32_t *instance_id_out)
{
    if (!ctx || !instance_id_out) return fail(REWL_EINVAL, "null argument");
    if (ctx->stage != 0) return fail(REWL_ESTATE, "cannot add instances after rewl_query_sizes");
    ctx->inst.emplace_back();
    *instance_id_out = (int32_t)ctx->inst.size() - 1;
    return REWL_OK;
}

rewl_status rewl_set_lattice_bcc(rewl_ctx *ctx, int32_t inst, int32_t L, int32_t n_shells, const double *J)
{
    rewl_status st = check_inst(ctx, inst);
    if (st) return st;
    if (L < 2 || L > 256) return fail(REWL_EINVAL, "L must be in [2, 256]");
    if (n_shells < 1 || n_shells > REWL_MAX_SHELLS || !J) return fail(REWL_EINVAL, "1..8 shells with couplings required");
    for (int i = 0; i < n_shells; ++i)
        if (!std::isfinite(J[i])) return fail(REWL_EINVAL, "non-finite coupling");
    const int64_t N = 2ll * L * L * L;
    if (N > (1 << 22)) return fail(REWL_ERANGE, "too many sites");
    InstanceCfg &q = ctx->inst[inst];
    q.lattice = LAT_BCC;
    q.L = L;
    q.N = (int32_t)N;
    q.Jshell.assign(J, J + n_shells);
    q.has_lattice = true;
    return REWL_OK;
}

rewl_status rewl_set_couplings_explicit(rewl_ctx *ctx, int32_t inst, int32_t N, int64_t n_pairs,
                                        const int32_t *i, const int32_t *j, const double *J)
{
    rewl_status st = check_inst(ctx, inst);
    if (st) return st;
    if (N < 1 || N > (1 << 22)) return fail(REWL_EINVAL, "N out of range");
    if (n_pairs < 0 || (n_pairs > 0 && (!i || !j || !J))) return fail(REWL_EINVAL, "bad pair arrays");
    for (int64_t p = 0; p < n_pairs; ++p) {
        if (i[p] < 0 || i[p] >= N || j[p] < 0 || j[p] >= N || i[p] == j[p])
            return fail(REWL_EINVAL, "pair index out of range or self-coupling");
        if (!std::isfinite(J[p])) return fail(REWL_EINVAL, "non-finite coupling");
    }
    InstanceCfg &q = ctx->inst[inst];
    q.lattice = LAT_TABLE;
    q.L = 0;
    q.N = N;
    q.pi.assign(i, i + n_pairs);
    q.pj.assign(j, j + n_pairs);
    q.pJ.assign(J, J + n_pairs);
    q.has_lattice = true;
    return REWL_OK;
}

rewl_status rewl_set_windows(rewl_ctx *ctx, int32_t inst, double E_min, double E_max,
                             int32_t n_global_bins, int32_t n_windows, double overlap,
                             int32_t walkers_per_window)
{
    rewl_status st = check_inst(ctx, inst);
    if (st) return st;
    if (!std::isfinite(E_min) || !std::isfinite(E_max) || !(E_max > E_min))
        return fail(REWL_EINVAL, "need finite E_min < E_max");
    if (n_global_bins < 1 || n_windows < 1 || walkers_per_window < 1)
        return fail(REWL_EINVAL, "bins, windows and walkers must be positive");
    if (walkers_per_window > REWL_MAX_WALKERS_PER_WINDOW) return fail(REWL_ERANGE, "more than 64 walkers per window");
    if (n_windows > 65535) return fail(REWL_ERANGE, "more than 65535 windows");
    if (!(overlap >= 0.0) || !(overlap < 1.0)) return fail(REWL_EINVAL, "overlap must be in [0, 1)");
    InstanceCfg &q = ctx->inst[inst];
    q.Emin = E_min;
    q.Emax = E_max;
    q.B = n_global_bins;
    q.h = n_windows;
    q.overlap = overlap;
    q.m = walkers_per_window;
    q.has_windows = true;
    return REWL_OK;
}

rewl_status rewl_set_schedule(rewl_ctx *ctx, int32_t inst, int32_t flat_num, int32_t flat_den,
                              double lnf_init, double lnf_final, int64_t exchange_interval,
                              int64_t resync_interval)
{
    rewl_status st = check_inst(ctx, inst);
    if (st) return st;
    if (flat_den < 1 || flat_num < 0 || flat_num > flat_den) return fail(REWL_EINVAL, "need 0 <= flat_num <= flat_den, flat_den >= 1");
    if (!(lnf_init > 0.0) || !(lnf_final > 0.0) || !std::isfinite(lnf_init)) return fail(REWL_EINVAL, "ln f values must be positive");
    if (exchange_interval < 1 || resync_interval < 0) return fail(REWL_EINVAL, "bad intervals");
    InstanceCfg &q = ctx->inst[inst];
    q.flat_num = flat_num;
    q.flat_den = flat_den;
    q.lnf_init = lnf_init;
    q.lnf_final = lnf_final;
    q.seg = exchange_interval;
    q.resync = resync_interval;
    q.has_schedule = true;
    return REWL_OK;
}

rewl_status rewl_set_window_sharing(rewl_ctx *ctx, int32_t inst, int32_t on)
{
    rewl_status st = check_inst(ctx, inst);
    if (st) return st;
    if (on != 0 && on != 1) return fail(REWL_EINVAL, "window sharing is 0 (off) or 1 (on)");
    ctx->inst[inst].share = on;
    return REWL_OK;
}

rewl_status rewl_set_coordinate(rewl_ctx *ctx, int32_t inst, int32_t coord)
{
    rewl_status st = check_inst(ctx, inst);
    if (st) return st;
    if (coord != 0 && coord != 1) return fail(REWL_EINVAL, "coordinate is 0 (energy) or 1 (magnetisation M_z)");
    ctx->inst[inst].coord = coord;
    return REWL_OK;
}

rewl_status rewl_query_sizes(rewl_ctx *ctx, size_t *bytes_out)
{
    if (!ctx || !bytes_out) return fail(REWL_EINVAL, "null argument");
    if (ctx->stage == 0) {
        rewl_status st = finalize(ctx);
        if (st) return st;
        ctx->stage = 1;
    }
    for (int b = 0; b < REWL_NBUF; ++b) bytes_out[b] = ctx->sizes[b];
    return REWL_OK;
}

rewl_status rewl_bind_buffers(rewl_ctx *ctx, void *const *dev_ptrs)
{
    if (!ctx || !dev_ptrs) return fail(REWL_EINVAL, "null argument");
    if (ctx->stage < 1) return fail(REWL_ESTATE, "call rewl_query_sizes first");
    for (int b = 0; b < REWL_NBUF; ++b) {
        if (!dev_ptrs[b]) return fail(REWL_EINVAL, "null device buffer " + std::to_string(b));
        if (((uintptr_t)dev_ptrs[b]) & 255) return fail(REWL_EINVAL, "device buffer not 256-byte aligned");
        ctx->buf[b] = dev_ptrs[b];
    }
    ctx->stage = 2;
    return REWL_OK;
}

rewl_status rewl_set_trace(rewl_ctx *ctx, void *dev_records, int64_t capacity)
{
    if (!ctx) return fail(REWL_EINVAL, "null context");
    if (capacity < 0) return fail(REWL_EINVAL, "negative capacity");
    ctx->trace = (rewl_trace_rec *)dev_records;
    ctx->trace_cap = dev_records ? capacity : 0;
    return REWL_OK;
}

rewl_status rewl_init_walkers(rewl_ctx *ctx, uint64_t seed, const double *init_spins)
{
    if (!ctx) return fail(REWL_EINVAL, "null context");
    if (ctx->stage < 2) return fail(REWL_ESTATE, "bind buffers first");
    HIP_TRY(hipSetDevice(ctx->device));
    ctx->seed = (uint32_t)seed;
    ctx->t = 0;
    ctx->init_host.clear();
    int64_t off = 0;
    for (size_t ii = 0; ii < ctx->inst.size(); ++ii) {
        const int N = ctx->inst[ii].N;
        if (init_spins) {
            for (int64_t k = 0; k < 3 * (int64_t)N; ++k) {
                const double v = init_spins[off + k];
                if (!std::isfinite(v)) return fail(REWL_EINVAL, "non-finite initial spin");
                ctx->init_host.push_back(v);
            }
            ctx->idesc[ii].init_off = off;
        } else {
            ctx->idesc[ii].init_off = -1;
        }
        off += 3 * (int64_t)N;
    }
    unsigned char *P = (unsigned char *)ctx->buf[REWL_BUF_PARAMS];
    hipStream_t s = ctx->stream;
    HIP_TRY(hipMemcpyAsync(P + ctx->off_inst, ctx->idesc.data(), sizeof(InstDesc) * ctx->idesc.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(P + ctx->off_wdesc, ctx->wdesc.data(), sizeof(WalkerDesc) * ctx->wdesc.size(), hipMemcpyHostToDevice, s));
    if (!ctx->slots.empty())
        HIP_TRY(hipMemcpyAsync(P + ctx->off_slots, ctx->slots.data(), sizeof(BccSlot) * ctx->slots.size(), hipMemcpyHostToDevice, s));
    if (!ctx->tdeg.empty())
        HIP_TRY(hipMemcpyAsync(P + ctx->off_tdeg, ctx->tdeg.data(), sizeof(int32_t) * ctx->tdeg.size(), hipMemcpyHostToDevice, s));
    if (!ctx->tnbr.empty()) {
        HIP_TRY(hipMemcpyAsync(P + ctx->off_tnbr, ctx->tnbr.data(), sizeof(int32_t) * ctx->tnbr.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(P + ctx->off_tJ, ctx->tJ.data(), sizeof(double) * ctx->tJ.size(), hipMemcpyHostToDevice, s));
    }
    if (!ctx->init_host.empty())
        HIP_TRY(hipMemcpyAsync(P + ctx->off_init, ctx->init_host.data(), sizeof(double) * ctx->init_host.size(), hipMemcpyHostToDevice, s));
    for (int b : {REWL_BUF_STATE, REWL_BUF_LNG, REWL_BUF_HIST, REWL_BUF_VISITED, REWL_BUF_CONTROL})
        HIP_TRY(hipMemsetAsync(ctx->buf[b], 0, ctx->sizes[b], s));
    KArgs a = make_args(ctx);
    int rc = launch_init(a, ctx->mode, s, ctx->lds_per_walker);
    if (rc) return fail(rc, "init kernel launch failed");
    rewl_status st = sync_check(ctx);
    if (st) return st;
    std::vector<WalkerState> ws(ctx->n_walkers);
    HIP_TRY(hipMemcpy(ws.data(), ctx->buf[REWL_BUF_STATE], sizeof(WalkerState) * ws.size(), hipMemcpyDeviceToHost));
    for (int w = 0; w < ctx->n_walkers; ++w)
        if (ws[w].status != 0)
            return fail(REWL_EINIT, "walker " + std::to_string(w) + " could not be driven into its window");
    ctx->stage = 3;
    return REWL_OK;
}

rewl_status rewl_run(rewl_ctx *ctx, int64_t n_segments)
{
    if (!ctx) return fail(REWL_EINVAL, "null context");
    if (ctx->stage < 3) return fail(REWL_ESTATE, "initialise walkers first");
    if (n_segments < 0) return fail(REWL_EINVAL, "negative segment count");
    for (int64_t k = 0; k < n_segments; ++k) {
        KArgs a = make_args(ctx);
        int rc = launch_sweep(a, ctx->mode, ctx->stream, ctx->lds_per_walker);
        if (rc) return fail(rc, "sweep kernel launch failed");
        rc = launch_exchange(a, ctx->stream);
        if (rc) return fail(rc, "exchange kernel launch failed");
        ctx->t += 1;
    }
    return REWL_OK;
}

rewl_status rewl_run_persistent(rewl_ctx *ctx, int64_t max_rounds, int32_t max_blocks, int32_t *grid_out)
{
    if (!ctx) return fail(REWL_EINVAL, "null context");
    if (ctx->stage < 3) return fail(REWL_ESTATE, "initialise walkers first");
    if (max_rounds < 0 || max_blocks < 0) return fail(REWL_EINVAL, "negative round or block count");
    if (ctx->mode == REWL_MODE_FP64_DET || ctx->fast_q <= 0)
        return fail(REWL_EUNSUPPORTED, "the persistent kernel needs FP64 or FP32_DE mode on bcc lattices");
    if ((double)max_rounds * (double)ctx->n_walkers + 2.0 * ctx->p_cap >= 2147483648.0)
        return fail(REWL_ERANGE, "too many rounds for one persistent launch; split the call");
    if (max_rounds == 0) {
        if (grid_out) *grid_out = 0;
        return REWL_OK;
    }
    int n_cu = 0;
    HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    KArgs a = make_args(ctx);
    a.p_max_rounds = (int32_t)max_rounds;
    // a legitimate wait lasts at most one segment of another walker plus an
    // exchange: about seg_len trial moves of at most ~10 us each
    int64_t seg_max = 1;
    for (auto &d : ctx->idesc) seg_max = std::max<int64_t>(seg_max, d.seg_len);
    a.p_spin_limit = (uint64_t)std::min<int64_t>(std::max<int64_t>(512 * seg_max, int64_t(1) << 22), int64_t(1) << 32);
    int grid = 0;
    if (max_blocks == 0) max_blocks = ctx->grid_cap;
    int rc = launch_persistent(a, ctx->mode, ctx->stream, ctx->lds_per_walker, n_cu, max_blocks, &grid);
    if (rc) return fail(rc, "persistent kernel launch failed");
    ctx->last_grid = grid;
    if (grid_out) *grid_out = grid;
    rewl_status st = sync_check(ctx);
    if (st) return st;
    PersistCtl pc{};
    HIP_TRY(hipMemcpy(&pc, (unsigned char *)ctx->buf[REWL_BUF_CONTROL] + ctx->off_pctl, sizeof pc,
                      hipMemcpyDeviceToHost));
    if (pc.error) return fail(REWL_EDEVICE, "persistent kernel: a bounded wait ran out");
    if (!pc.all_done) return fail(REWL_EDEVICE, "persistent kernel ended before every instance stopped");
    ctx->t += max_rounds;
    return REWL_OK;
}

rewl_status rewl_set_launch(rewl_ctx *ctx, int32_t walkers_per_block, int32_t residency)
{
    if (!ctx) return fail(REWL_EINVAL, "null context");
    if (ctx->stage < 1) return fail(REWL_ESTATE, "call rewl_query_sizes first");
    if (walkers_per_block < 1 || walkers_per_block > 4) return fail(REWL_EINVAL, "walkers per block must be 1..4");
    if (residency < 0 || residency > 2) return fail(REWL_EINVAL, "residency must be 0 (auto), 1 (LDS) or 2 (HBM)");
    const int32_t old_w = ctx->wpb_req, old_r = ctx->residency_req;
    ctx->wpb_req = walkers_per_block;
    ctx->residency_req = residency;
    rewl_status st = plan_launch(ctx);
    if (st) {
        ctx->wpb_req = old_w;
        ctx->residency_req = old_r;
        plan_launch(ctx);
        return st;
    }
    ctx->grid_cap = 0;
    return REWL_OK;
}

rewl_status rewl_set_grid_cap(rewl_ctx *ctx, int32_t max_blocks)
{
    if (!ctx) return fail(REWL_EINVAL, "null context");
    if (max_blocks < 0) return fail(REWL_EINVAL, "negative grid cap");
    ctx->grid_cap = max_blocks;
    return REWL_OK;
}

rewl_status rewl_get_grid_cap(rewl_ctx *ctx, int32_t *max_blocks)
{
    if (!ctx || !max_blocks) return fail(REWL_EINVAL, "null argument");
    *max_blocks = ctx->grid_cap;
    return REWL_OK;
}

rewl_status rewl_get_launch(rewl_ctx *ctx, int32_t *walkers_per_block, int32_t *spins_in_lds,
                            int64_t *lds_bytes_per_block)
{
    if (!ctx || !walkers_per_block || !spins_in_lds || !lds_bytes_per_block) return fail(REWL_EINVAL, "null argument");
    if (ctx->stage < 1) return fail(REWL_ESTATE, "call rewl_query_sizes first");
    *walkers_per_block = ctx->wpb;
    *spins_in_lds = ctx->spins_in_lds;
    *lds_bytes_per_block = (int64_t)(((ctx->lds_per_walker + 15) & ~(size_t)15) * (size_t)ctx->wpb);
    return REWL_OK;
}

rewl_status rewl_set_proposal(rewl_ctx *ctx, int32_t kind, const float *dev_params)
{
    if (!ctx) return fail(REWL_EINVAL, "null context");
    if (ctx->stage < 2) return fail(REWL_ESTATE, "bind buffers first");
    if (kind == 0) {
        ctx->proposal = 0;
        return REWL_OK;
    }
    if (kind != 1 || !dev_params) return fail(REWL_EINVAL, "kind must be 0 (uniform) or 1 (learned, with parameters)");
    if (ctx->mode != REWL_MODE_FP32_DE || ctx->fast_q == 0)
        return fail(REWL_EUNSUPPORTED, "the learned proposal runs in FP32_DE mode on bcc lattices");
    if (ctx->harvest) return fail(REWL_EUNSUPPORTED, "harvesting records needs the uniform proposal");
    int rc = launch_mlp_pack(dev_params, (unsigned char *)ctx->buf[REWL_BUF_PARAMS] + ctx->off_mlp, ctx->stream);
    if (rc) return fail(rc, "pack kernel launch failed");
    ctx->proposal = 1;
    return REWL_OK;
}

rewl_status rewl_set_harvest(rewl_ctx *ctx, float *dev_records, int64_t capacity_per_walker, int32_t every_k)
{
    if (!ctx) return fail(REWL_EINVAL, "null context");
    if (ctx->stage < 1) return fail(REWL_ESTATE, "call rewl_query_sizes first");
    if (!dev_records) {
        ctx->harvest = nullptr;
        ctx->harvest_cap = 0;
        return REWL_OK;
    }
    if (capacity_per_walker < 1 || every_k < 1) return fail(REWL_EINVAL, "capacity and interval must be positive");
    if (ctx->fast_q == 0 || ctx->proposal != 0)
        return fail(REWL_EUNSUPPORTED, "harvesting needs the fast kernel and the uniform proposal");
    ctx->harvest = dev_records;
    ctx->harvest_cap = capacity_per_walker;
    ctx->harvest_every = every_k;
    return REWL_OK;
}

rewl_status rewl_read_harvest_counts(rewl_ctx *ctx, int64_t *counts, int32_t cap)
{
    if (!ctx || !counts) return fail(REWL_EINVAL, "null argument");
    if (ctx->stage < 3) return fail(REWL_ESTATE, "walkers not initialised");
    rewl_status st = sync_check(ctx);
    if (st) return st;
    std::vector<WalkerState> ws(ctx->n_walkers);
    HIP_TRY(hipMemcpy(ws.data(), ctx->buf[REWL_BUF_STATE], sizeof(WalkerState) * ws.size(), hipMemcpyDeviceToHost));
    for (int w = 0; w < ctx->n_walkers && w < cap; ++w) counts[w] = (int64_t)ws[w].harvested;
    return REWL_OK;
}

rewl_status rewl_sweep(rewl_ctx *ctx)
{
    if (!ctx) return fail(REWL_EINVAL, "null context");
    if (ctx->stage < 3) return fail(REWL_ESTATE, "initialise walkers first");
    KArgs a = make_args(ctx);
    int rc = launch_sweep(a, ctx->mode, ctx->stream, ctx->lds_per_walker);
    if (rc) return fail(rc, "sweep kernel launch failed");
    return REWL_OK;
}

rewl_status rewl_exchange(rewl_ctx *ctx)
{
    if (!ctx) return fail(REWL_EINVAL, "null context");
    if (ctx->stage < 3) return fail(REWL_ESTATE, "initialise walkers first");
    KArgs a = make_args(ctx);
    int rc = launch_exchange(a, ctx->stream);
    if (rc) return fail(rc, "exchange kernel launch failed");
    ctx->t += 1;
    return REWL_OK;
}

rewl_status rewl_poll(rewl_ctx *ctx, int32_t *all_done_out)
{
    if (!ctx || !all_done_out) return fail(REWL_EINVAL, "null argument");
    if (ctx->stage < 3) return fail(REWL_ESTATE, "initialise walkers first");
    rewl_status st = sync_check(ctx);
    if (st) return st;
    std::vector<InstControl> ic(ctx->inst.size());
    HIP_TRY(hipMemcpy(ic.data(), (unsigned char *)ctx->buf[REWL_BUF_CONTROL] + ctx->off_ictl,
                      sizeof(InstControl) * ic.size(), hipMemcpyDeviceToHost));
    int all = 1;
    for (auto &x : ic) all &= (x.done != 0);
    *all_done_out = all;
    return REWL_OK;
}

static rewl_status read_bins(rewl_ctx *ctx, int32_t inst, int32_t walker, int buf, size_t esz,
                             void *out, int32_t cap, int32_t *n_out)
{
    int gw;
    rewl_status st = check_walker(ctx, inst, walker, &gw);
    if (st) return st;
    if (!out || cap < 0) return fail(REWL_EINVAL, "bad output buffer");
    st = sync_check(ctx);
    if (st) return st;
    const WalkerDesc &wd = ctx->wdesc[gw];
    const int32_t nb = wd.hi - wd.lo;
    const int32_t n = std::min(nb, cap);
    HIP_TRY(hipMemcpy(out, (unsigned char *)ctx->buf[buf] + esz * (size_t)wd.bin_off, esz * (size_t)n,
                      hipMemcpyDeviceToHost));
    if (n_out) *n_out = n;
    return REWL_OK;
}

rewl_status rewl_read_lng(rewl_ctx *ctx, int32_t inst, int32_t walker, double *out, int32_t cap, int32_t *n_out)
{
    return read_bins(ctx, inst, walker, REWL_BUF_LNG, sizeof(double), out, cap, n_out);
}

rewl_status rewl_read_hist(rewl_ctx *ctx, int32_t inst, int32_t walker, uint32_t *out, int32_t cap, int32_t *n_out)
{
    return read_bins(ctx, inst, walker, REWL_BUF_HIST, sizeof(uint32_t), out, cap, n_out);
}

rewl_status rewl_read_visited(rewl_ctx *ctx, int32_t inst, int32_t walker, uint8_t *out, int32_t cap, int32_t *n_out)
{
    return read_bins(ctx, inst, walker, REWL_BUF_VISITED, 1, out, cap, n_out);
}

rewl_status rewl_write_lng(rewl_ctx *ctx, int32_t inst, int32_t walker, const double *lng,
                           const uint8_t *visited, int32_t cap)
{
    int gw;
    rewl_status st = check_walker(ctx, inst, walker, &gw);
    if (st) return st;
    if (!lng || cap < 0) return fail(REWL_EINVAL, "bad input");
    st = sync_check(ctx);
    if (st) return st;
    const WalkerDesc &wd = ctx->wdesc[gw];
    const int32_t n = std::min(wd.hi - wd.lo, cap);
    for (int32_t j = 0; j < n; ++j)
        if (!std::isfinite(lng[j])) return fail(REWL_EINVAL, "non-finite ln g");
    std::vector<uint8_t> vis(n, 1);
    if (visited) vis.assign(visited, visited + n);
    // a bin marked not visited holds the initial guess ln g~ = 0
    std::vector<double> val(lng, lng + n);
    for (int32_t j = 0; j < n; ++j)
        if (!vis[j]) val[j] = 0.0;
    HIP_TRY(hipMemcpy((double *)ctx->buf[REWL_BUF_LNG] + wd.bin_off, val.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy((uint8_t *)ctx->buf[REWL_BUF_VISITED] + wd.bin_off, vis.data(), n, hipMemcpyHostToDevice));
    return REWL_OK;
}

rewl_status rewl_read_walker_state(rewl_ctx *ctx, int32_t inst, int32_t walker, rewl_walker_state *out)
{
    int gw;
    rewl_status st = check_walker(ctx, inst, walker, &gw);
    if (st) return st;
    if (!out) return fail(REWL_EINVAL, "null output");
    st = sync_check(ctx);
    if (st) return st;
    WalkerState ws;
    HIP_TRY(hipMemcpy(&ws, (WalkerState *)ctx->buf[REWL_BUF_STATE] + gw, sizeof ws, hipMemcpyDeviceToHost));
    out->E = ws.E;
    out->lnf = ws.lnf;
    out->max_drift = ws.max_drift;
    out->bin = ws.bin;
    out->config = ws.cfg;
    out->iteration = ws.iter;
    out->done = ws.done;
    out->n_visited = ws.nvis;
    out->window = ctx->wdesc[gw].win;
    out->attempts = ws.attempts;
    out->accepts = ws.accepts;
    out->rejected_outside = ws.oow;
    if (ws.status == REWL_ENUMERIC) return fail(REWL_ENUMERIC, "non-finite energy or ln g");
    return REWL_OK;
}

rewl_status rewl_read_config(rewl_ctx *ctx, int32_t inst, int32_t config, double *out, int64_t cap)
{
    if (!ctx || !out) return fail(REWL_EINVAL, "null argument");
    if (ctx->stage < 3) return fail(REWL_ESTATE, "walkers not initialised");
    if (inst < 0 || inst >= (int32_t)ctx->inst.size()) return fail(REWL_EINVAL, "bad instance index");
    const InstDesc &d = ctx->idesc[inst];
    if (config < 0 || config >= d.n_walkers) return fail(REWL_EINVAL, "bad configuration index");
    if (cap < 3 * (int64_t)d.N) return fail(REWL_EINVAL, "output too small");
    rewl_status st = sync_check(ctx);
    if (st) return st;
    const size_t sb = spin_bytes(ctx->mode);
    std::vector<unsigned char> tmp(sb * (size_t)d.N);
    HIP_TRY(hipMemcpy(tmp.data(), (unsigned char *)ctx->buf[REWL_BUF_SPINS] + sb * (size_t)(d.cfg_off + (int64_t)config * d.N),
                      tmp.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < d.N; ++i) {
        const size_t j = (size_t)spin_slot(i, d.layout, d.lg_L);
        for (int k = 0; k < 3; ++k)
            out[3 * (size_t)i + k] = sb == 16 ? (double)((const float *)tmp.data())[4 * j + k]
                                              : ((const double *)tmp.data())[4 * j + k];
    }
    return REWL_OK;
}

rewl_status rewl_read_window(rewl_ctx *ctx, int32_t inst, int32_t win, int32_t *lo_bin, int32_t *hi_bin)
{
    if (!ctx || !lo_bin || !hi_bin) return fail(REWL_EINVAL, "null argument");
    if (ctx->stage < 1) return fail(REWL_ESTATE, "call rewl_query_sizes first");
    if (inst < 0 || inst >= (int32_t)ctx->inst.size()) return fail(REWL_EINVAL, "bad instance index");
    const InstanceCfg &q = ctx->inst[inst];
    if (win < 0 || win >= q.h) return fail(REWL_EINVAL, "bad window index");
    *lo_bin = q.lo[win];
    *hi_bin = q.hi[win];
    return REWL_OK;
}

rewl_status rewl_read_exchange_stats(rewl_ctx *ctx, int32_t inst, uint64_t *attempts, uint64_t *accepts, int32_t cap)
{
    if (!ctx || !attempts || !accepts) return fail(REWL_EINVAL, "null argument");
    if (ctx->stage < 3) return fail(REWL_ESTATE, "walkers not initialised");
    if (inst < 0 || inst >= (int32_t)ctx->inst.size()) return fail(REWL_EINVAL, "bad instance index");
    rewl_status st = sync_check(ctx);
    if (st) return st;
    const InstDesc &d = ctx->idesc[inst];
    const int n = std::min(cap, std::max(d.h - 1, 0));
    unsigned char *Cb = (unsigned char *)ctx->buf[REWL_BUF_CONTROL];
    if (n > 0) {
        HIP_TRY(hipMemcpy(attempts, Cb + ctx->off_xatt + 8 * (size_t)d.xstat_off, 8 * (size_t)n, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(accepts, Cb + ctx->off_xacc + 8 * (size_t)d.xstat_off, 8 * (size_t)n, hipMemcpyDeviceToHost));
    }
    return REWL_OK;
}

rewl_status rewl_read_step(rewl_ctx *ctx, int64_t *step_out)
{
    if (!ctx || !step_out) return fail(REWL_EINVAL, "null argument");
    *step_out = ctx->t;
    return REWL_OK;
}

rewl_status rewl_read_round_trips(rewl_ctx *ctx, int32_t inst, uint32_t *half_trips, int32_t cap)
{
    if (!ctx || !half_trips || cap < 0) return fail(REWL_EINVAL, "bad argument");
    if (ctx->stage < 3) return fail(REWL_ESTATE, "walkers not initialised");
    if (inst < 0 || inst >= (int32_t)ctx->inst.size()) return fail(REWL_EINVAL, "bad instance index");
    rewl_status st = sync_check(ctx);
    if (st) return st;
    const InstDesc &d = ctx->idesc[inst];
    const int32_t n = std::min(d.n_walkers, cap);
    std::vector<uint32_t> v(n);
    HIP_TRY(hipMemcpy(v.data(), (unsigned char *)ctx->buf[REWL_BUF_CONTROL] + ctx->off_rtrip + 4 * (size_t)d.walker_base,
                      4 * (size_t)n, hipMemcpyDeviceToHost));
    for (int32_t k = 0; k < n; ++k) half_trips[k] = v[k] >> 2;
    return REWL_OK;
}

rewl_status rewl_total_attempts(rewl_ctx *ctx, uint64_t *attempts, uint64_t *accepts)
{
    if (!ctx || !attempts || !accepts) return fail(REWL_EINVAL, "null argument");
    if (ctx->stage < 3) return fail(REWL_ESTATE, "walkers not initialised");
    rewl_status st = sync_check(ctx);
    if (st) return st;
    std::vector<WalkerState> ws(ctx->n_walkers);
    HIP_TRY(hipMemcpy(ws.data(), ctx->buf[REWL_BUF_STATE], sizeof(WalkerState) * ws.size(), hipMemcpyDeviceToHost));
    uint64_t at = 0, ac = 0;
    for (auto &w : ws) {
        at += w.attempts;
        ac += w.accepts;
    }
    *attempts = at;
    *accepts = ac;
    return REWL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- checkpoints

namespace {

struct CkptHeader {
    char magic[8];
    uint32_t version;
    int32_t mode;
    uint64_t fingerprint;
    uint32_t seed;
    int32_t proposal;
    int64_t t;
    uint64_t sizes[REWL_NBUF];
};
constexpr char kCkptMagic[8] = {'R', 'E', 'W', 'L', 'C', 'K', 'P', '1'};

uint64_t fnv1a(uint64_t h, const void *p, size_t n)
{
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Everything that fixes the meaning of the device buffers: mode, buffer
// sizes and the host copies of the instance, walker and lattice tables.
uint64_t fingerprint(const rewl_ctx *c)
{
    uint64_t h = 14695981039346656037ull;
    h = fnv1a(h, &c->mode, sizeof c->mode);
    h = fnv1a(h, c->sizes, sizeof c->sizes);
    h = fnv1a(h, c->idesc.data(), c->idesc.size() * sizeof(InstDesc));
    h = fnv1a(h, c->wdesc.data(), c->wdesc.size() * sizeof(WalkerDesc));
    h = fnv1a(h, c->slots.data(), c->slots.size() * sizeof(BccSlot));
    h = fnv1a(h, c->tdeg.data(), c->tdeg.size() * sizeof(int32_t));
    h = fnv1a(h, c->tnbr.data(), c->tnbr.size() * sizeof(int32_t));
    h = fnv1a(h, c->tJ.data(), c->tJ.size() * sizeof(double));
    return h;
}

constexpr size_t kCkptChunk = size_t(64) << 20;

struct FileCloser {
    FILE *f;
    ~FileCloser()
    {
        if (f) fclose(f);
    }
};

}  // namespace

extern "C" {

rewl_status rewl_save(rewl_ctx *ctx, const char *path)
{
    if (!ctx || !path) return fail(REWL_EINVAL, "null argument");
    if (ctx->stage < 3) return fail(REWL_ESTATE, "initialise walkers first");
    rewl_status st = sync_check(ctx);
    if (st) return st;
    CkptHeader hd{};
    memcpy(hd.magic, kCkptMagic, 8);
    hd.version = 1;
    hd.mode = ctx->mode;
    hd.fingerprint = fingerprint(ctx);
    hd.seed = ctx->seed;
    hd.proposal = ctx->proposal;
    hd.t = ctx->t;
    for (int b = 0; b < REWL_NBUF; ++b) hd.sizes[b] = ctx->sizes[b];
    FileCloser fc{fopen(path, "wb")};
    if (!fc.f) return fail(REWL_EINVAL, std::string("cannot open checkpoint for writing: ") + path);
    if (fwrite(&hd, sizeof hd, 1, fc.f) != 1) return fail(REWL_EINVAL, "checkpoint write failed");
    std::vector<unsigned char> tmp;
    for (int b = 0; b < REWL_NBUF; ++b) {
        for (size_t off = 0; off < ctx->sizes[b]; off += kCkptChunk) {
            const size_t n = std::min(kCkptChunk, ctx->sizes[b] - off);
            tmp.resize(n);
            HIP_TRY(hipMemcpy(tmp.data(), (unsigned char *)ctx->buf[b] + off, n, hipMemcpyDeviceToHost));
            if (fwrite(tmp.data(), 1, n, fc.f) != n) return fail(REWL_EINVAL, "checkpoint write failed");
        }
    }
    if (fflush(fc.f) != 0) return fail(REWL_EINVAL, "checkpoint write failed");
    return REWL_OK;
}

rewl_status rewl_load(rewl_ctx *ctx, const char *path)
{
    if (!ctx || !path) return fail(REWL_EINVAL, "null argument");
    if (ctx->stage < 2) return fail(REWL_ESTATE, "bind buffers before loading a checkpoint");
    rewl_status st = sync_check(ctx);
    if (st) return st;
    FileCloser fc{fopen(path, "rb")};
    if (!fc.f) return fail(REWL_EINVAL, std::string("cannot open checkpoint: ") + path);
    CkptHeader hd{};
    if (fread(&hd, sizeof hd, 1, fc.f) != 1) return fail(REWL_ECORRUPT, "checkpoint too short");
    if (memcmp(hd.magic, kCkptMagic, 8) != 0 || hd.version != 1)
        return fail(REWL_ECORRUPT, "not a checkpoint of this library version");
    if (hd.mode != ctx->mode) return fail(REWL_ECORRUPT, "checkpoint was written in another arithmetic mode");
    for (int b = 0; b < REWL_NBUF; ++b)
        if (hd.sizes[b] != ctx->sizes[b]) return fail(REWL_ECORRUPT, "checkpoint buffer sizes differ from this context");
    if (hd.fingerprint != fingerprint(ctx))
        return fail(REWL_ECORRUPT, "checkpoint belongs to a different configuration");
    if (hd.proposal != 0 && hd.proposal != 1) return fail(REWL_ECORRUPT, "bad proposal kind in checkpoint");
    // read everything before touching the device, so that a short file
    // leaves the context as it was
    std::vector<std::vector<unsigned char>> data(REWL_NBUF);
    for (int b = 0; b < REWL_NBUF; ++b) {
        data[b].resize(ctx->sizes[b]);
        if (ctx->sizes[b] && fread(data[b].data(), 1, ctx->sizes[b], fc.f) != ctx->sizes[b])
            return fail(REWL_ECORRUPT, "checkpoint truncated");
    }
    unsigned char extra;
    if (fread(&extra, 1, 1, fc.f) != 0) return fail(REWL_ECORRUPT, "trailing bytes in checkpoint");
    for (int b = 0; b < REWL_NBUF; ++b)
        if (ctx->sizes[b])
            HIP_TRY(hipMemcpy(ctx->buf[b], data[b].data(), ctx->sizes[b], hipMemcpyHostToDevice));
    ctx->seed = hd.seed;
    ctx->proposal = hd.proposal;
    ctx->t = hd.t;
    ctx->stage = 3;
    return REWL_OK;
}


rewl_status rewl_fingerprint(rewl_ctx *ctx, uint64_t *digest_out)
{
    if (!ctx || !digest_out) return fail(REWL_EINVAL, "null argument");
    if (ctx->stage < 1) return fail(REWL_ESTATE, "call rewl_query_sizes first");
    *digest_out = fingerprint(ctx);
    return REWL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- autotuner

namespace {

struct Snapshot {
    std::vector<std::vector<unsigned char>> buf;
    int64_t t = 0;
};

rewl_status take_snapshot(rewl_ctx *c, Snapshot &sn)
{
    rewl_status st = sync_check(c);
    if (st) return st;
    sn.buf.assign(REWL_NBUF, {});
    for (int b = 0; b < REWL_NBUF; ++b) {
        sn.buf[b].resize(c->sizes[b]);
        if (c->sizes[b]) HIP_TRY(hipMemcpy(sn.buf[b].data(), c->buf[b], c->sizes[b], hipMemcpyDeviceToHost));
    }
    sn.t = c->t;
    return REWL_OK;
}

rewl_status restore_snapshot(rewl_ctx *c, const Snapshot &sn)
{
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int b = 0; b < REWL_NBUF; ++b)
        if (c->sizes[b]) HIP_TRY(hipMemcpy(c->buf[b], sn.buf[b].data(), c->sizes[b], hipMemcpyHostToDevice));
    c->t = sn.t;
    return REWL_OK;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

extern "C" {

rewl_status rewl_autotune(rewl_ctx *ctx, int32_t segments, int32_t persistent, rewl_tune_entry *entries,
                          int32_t cap, int32_t *n_out)
{
    if (!ctx) return fail(REWL_EINVAL, "null context");
    if (ctx->stage < 3) return fail(REWL_ESTATE, "initialise walkers first");
    if (segments < 1 || cap < 0) return fail(REWL_EINVAL, "need segments >= 1 and cap >= 0");
    if (persistent && (ctx->mode == REWL_MODE_FP64_DET || ctx->fast_q <= 0))
        return fail(REWL_EUNSUPPORTED, "the persistent kernel needs FP64 or FP32_DE mode on bcc lattices");
    Snapshot sn;
    rewl_status st = take_snapshot(ctx, sn);
    if (st) return st;
    const int32_t old_w = ctx->wpb_req, old_r = ctx->residency_req, old_cap = ctx->grid_cap;
    ctx->grid_cap = 0;
    EventPair ev;
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    // persistent form: each shape first with every resident block, then with
    // the grid halved again and again (at most kHalvings times) while that
    // keeps getting faster
    constexpr int kHalvings = 4;
    int32_t cap_blocks = 0;       // grid cap of the current trial (persistent form)
    int32_t grid_full = 0;        // grid the uncapped trial of the same shape launched
    bool keep = false;            // the shape's last trial was timed and faster than the one before
    double shape_ms = -1.0;       // time of the shape's last timed trial
    auto run = [&](int32_t n) -> rewl_status {
        if (persistent) {
            int32_t g = 0;
            rewl_status s = rewl_run_persistent(ctx, n, cap_blocks, &g);
            if (!s && cap_blocks == 0) grid_full = g;
            return s;
        }
        return rewl_run(ctx, n);
    };
    int32_t n = 0, best_w = 0, best_r = 0, best_cap = 0;
    double best = -1.0;
    const int wpbs[3] = {1, 2, 4};
    for (int r = 1; r <= 2; ++r) {
        for (int kk = 0; kk < (persistent ? 3 * (1 + kHalvings) : 3); ++kk) {
            const int k = persistent ? kk / (1 + kHalvings) : kk;
            const int halvings = persistent ? kk % (1 + kHalvings) : 0;
            if (halvings > 0) {
                if (!keep || (grid_full >> halvings) < 1) continue;
                cap_blocks = grid_full >> halvings;
            } else {
                cap_blocks = 0;
                grid_full = 0;
                shape_ms = -1.0;
            }
            keep = false;
            rewl_tune_entry e{};
            e.walkers_per_block = wpbs[k];
            e.residency = r;
            e.persistent = persistent ? 1 : 0;
            e.ms_per_segment = -1.0;
            e.max_blocks = cap_blocks;
            ctx->wpb_req = wpbs[k];
            ctx->residency_req = r;
            e.status = plan_launch(ctx);
            if (e.status == REWL_OK) {
                // one untimed segment (code and cache warm-up), then the trial
                st = restore_snapshot(ctx, sn);
                if (!st) st = run(1);
                if (!st) st = restore_snapshot(ctx, sn);
                if (!st) {
                    if (hipEventRecord(ev.a, ctx->stream) != hipSuccess) st = REWL_EDEVICE;
                }
                if (!st) st = run(segments);
                if (!st) {
                    if (hipEventRecord(ev.b, ctx->stream) != hipSuccess || hipEventSynchronize(ev.b) != hipSuccess)
                        st = REWL_EDEVICE;
                }
                if (!st) st = sync_check(ctx);
                if (st == REWL_EUNSUPPORTED) {
                    // the shape plans but cannot launch (no resident block)
                    e.status = st;
                    st = restore_snapshot(ctx, sn);
                    if (st) return st;
                    if (entries && n < cap) entries[n] = e;
                    ++n;
                    continue;
                }
                if (st) {
                    // a failed trial leaves the walk restored and the old shape
                    ctx->wpb_req = old_w;
                    ctx->residency_req = old_r;
                    ctx->grid_cap = old_cap;
                    plan_launch(ctx);
                    rewl_status st2 = restore_snapshot(ctx, sn);
                    return st2 ? st2 : st;
                }
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
                e.ms_per_segment = (double)ms / segments;
                keep = shape_ms < 0.0 || e.ms_per_segment < shape_ms;
                shape_ms = e.ms_per_segment;
                if (best < 0.0 || e.ms_per_segment < best) {
                    best = e.ms_per_segment;
                    best_w = wpbs[k];
                    best_r = r;
                    best_cap = cap_blocks;
                }
            }
            if (entries && n < cap) entries[n] = e;
            ++n;
        }
    }
    st = restore_snapshot(ctx, sn);
    if (st) return st;
    if (best < 0.0) {
        ctx->wpb_req = old_w;
        ctx->residency_req = old_r;
        ctx->grid_cap = old_cap;
        plan_launch(ctx);
        return fail(REWL_EUNSUPPORTED, "no launch shape is usable for this context");
    }
    ctx->wpb_req = best_w;
    ctx->residency_req = best_r;
    ctx->grid_cap = persistent ? best_cap : old_cap;
    st = plan_launch(ctx);
    if (st) return st;
    if (n_out) *n_out = std::min(n, cap);
    return REWL_OK;
}

}  // extern "C"
