"""Python binding of librewl (argument marshalling only).

Every ``rewl_*`` function of ``include/rewl.h`` is exposed here under the
same name; each raises :class:`RewlError` on a negative status.  All
computation happens in the HIP kernels of ``librewl.so``; there is no CPU
fallback, and importing this module fails if the library is not built.

PyTorch supplies device memory and the stream: :class:`Run` allocates the
buffers ``rewl_query_sizes`` asks for as ``torch.uint8`` tensors on the GPU
and passes their addresses.
"""
import ctypes as C
import os

import numpy as np
# torch first: its bundled HIP runtime then satisfies librewl's
# libamdhip64.so.7 / libhsa-runtime64.so.1 dependencies, so the process holds
# one HIP runtime and torch's device pointers and streams are valid in ours.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librewl.so")

REWL_OK = 0
MODE_FP64_DET, MODE_FP64, MODE_FP32_DE = 0, 1, 2
MODES = {"fp64_det": MODE_FP64_DET, "fp64": MODE_FP64, "fp32_de": MODE_FP32_DE}
NBUF = 7
BUF_NAMES = ["spins", "state", "lng", "hist", "visited", "params", "control"]

TRACE_DTYPE = np.dtype([("site", "<u4"), ("flags", "<u4"), ("E", "<f8"),
                        ("bin", "<i4"), ("attempt_lo", "<u4")])


class rewl_walker_state(C.Structure):
    _fields_ = [("E", C.c_double), ("lnf", C.c_double), ("max_drift", C.c_double),
                ("bin", C.c_int32), ("config", C.c_int32), ("iteration", C.c_int32),
                ("done", C.c_int32), ("n_visited", C.c_int32), ("window", C.c_int32),
                ("attempts", C.c_uint64), ("accepts", C.c_uint64),
                ("rejected_outside", C.c_uint64)]


class rewl_tune_entry(C.Structure):
    _fields_ = [("walkers_per_block", C.c_int32), ("residency", C.c_int32), ("persistent", C.c_int32),
                ("status", C.c_int32), ("ms_per_segment", C.c_double), ("max_blocks", C.c_int32),
                ("pad", C.c_int32)]


class RewlError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__("%s failed (%d): %s" % (fn, code, msg))
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError("librewl.so is not built; run __graft_entry__.build() "
                      "(or python paper_1411_4212_amd/build.py) first")

_lib = C.CDLL(LIB_PATH)

_P = C.POINTER
_vp, _i32, _i64, _u64, _dbl, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double, C.c_size_t
_SIGS = {
    "rewl_create": [_P(_vp), _i32, _vp, _i32],
    "rewl_add_instance": [_vp, _P(_i32)],
    "rewl_set_lattice_bcc": [_vp, _i32, _i32, _i32, _P(_dbl)],
    "rewl_set_couplings_explicit": [_vp, _i32, _i32, _i64, _P(_i32), _P(_i32), _P(_dbl)],
    "rewl_set_windows": [_vp, _i32, _dbl, _dbl, _i32, _i32, _dbl, _i32],
    "rewl_set_schedule": [_vp, _i32, _i32, _i32, _dbl, _dbl, _i64, _i64],
    "rewl_set_window_sharing": [_vp, _i32, _i32],
    "rewl_set_coordinate": [_vp, _i32, _i32],
    "rewl_query_sizes": [_vp, _P(_sz)],
    "rewl_bind_buffers": [_vp, _P(_vp)],
    "rewl_init_walkers": [_vp, _u64, _P(_dbl)],
    "rewl_run": [_vp, _i64],
    "rewl_sweep": [_vp],
    "rewl_exchange": [_vp],
    "rewl_poll": [_vp, _P(_i32)],
    "rewl_read_lng": [_vp, _i32, _i32, _P(_dbl), _i32, _P(_i32)],
    "rewl_read_hist": [_vp, _i32, _i32, _P(C.c_uint32), _i32, _P(_i32)],
    "rewl_read_visited": [_vp, _i32, _i32, _P(C.c_uint8), _i32, _P(_i32)],
    "rewl_read_walker_state": [_vp, _i32, _i32, _P(rewl_walker_state)],
    "rewl_read_config": [_vp, _i32, _i32, _P(_dbl), _i64],
    "rewl_write_lng": [_vp, _i32, _i32, _P(_dbl), _P(C.c_uint8), _i32],
    "rewl_save": [_vp, C.c_char_p],
    "rewl_read_round_trips": [_vp, _i32, _P(C.c_uint32), _i32],
    "rewl_run_persistent": [_vp, _i64, _i32, _P(_i32)],
    "rewl_autotune": [_vp, _i32, _i32, _P(rewl_tune_entry), _i32, _P(_i32)],
    "rewl_fingerprint": [_vp, _P(_u64)],
    "rewl_load": [_vp, C.c_char_p],
    "rewl_read_window": [_vp, _i32, _i32, _P(_i32), _P(_i32)],
    "rewl_read_exchange_stats": [_vp, _i32, _P(_u64), _P(_u64), _i32],
    "rewl_read_step": [_vp, _P(_i64)],
    "rewl_set_trace": [_vp, _vp, _i64],
    "rewl_set_launch": [_vp, _i32, _i32],
    "rewl_set_grid_cap": [_vp, _i32],
    "rewl_get_grid_cap": [_vp, _P(_i32)],
    "rewl_set_proposal": [_vp, _i32, _vp],
    "rewl_set_harvest": [_vp, _vp, _i64, _i32],
    "rewl_read_harvest_counts": [_vp, _P(_i64), _i32],
    "rewl_mlp_workspace_bytes": [_i64, _P(_sz)],
    "rewl_mlp_pack": [_vp, _vp, _vp],
    "rewl_mlp_eval": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp],
    "rewl_mlp_loss_grad": [_vp, _i64, _vp, _vp, _P(C.c_double), _vp, _vp],
    "rewl_mlp_train": [_vp, _i64, _i32, _i32, C.c_float, _u64, _vp, _vp, _P(C.c_float), _vp],
    "rewl_mlp_train_static": [_vp, _i64, _i32, _i32, C.c_float, _u64, _vp, _P(C.c_float), _vp],
    "rewl_get_launch": [_vp, _P(_i32), _P(_i32), _P(_i64)],
    "rewl_total_attempts": [_vp, _P(_u64), _P(_u64)],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int32
_lib.rewl_mlp_param_count.argtypes = []
_lib.rewl_mlp_param_count.restype = C.c_int32
_lib.rewl_mlp_packed_bytes.argtypes = []
_lib.rewl_mlp_packed_bytes.restype = C.c_size_t
_lib.rewl_destroy.argtypes = [_vp]
_lib.rewl_destroy.restype = None
_lib.rewl_last_error.argtypes = []
_lib.rewl_last_error.restype = C.c_char_p

EXPORTED = list(_SIGS) + ["rewl_destroy", "rewl_last_error", "rewl_mlp_param_count",
                          "rewl_mlp_packed_bytes"]


def rewl_last_error():
    return _lib.rewl_last_error().decode()


def _call(name, *args):
    rc = getattr(_lib, name)(*args)
    if rc != REWL_OK:
        raise RewlError(name, rc, rewl_last_error())
    return rc


def _dp(a):
    return a.ctypes.data_as(_P(_dbl))


def rewl_create(device, stream_ptr, mode):
    h = _vp()
    _call("rewl_create", C.byref(h), device, _vp(stream_ptr), mode)
    return h


def rewl_destroy(ctx):
    _lib.rewl_destroy(ctx)


def rewl_add_instance(ctx):
    i = _i32()
    _call("rewl_add_instance", ctx, C.byref(i))
    return i.value


def rewl_set_lattice_bcc(ctx, inst, L, J):
    J = np.ascontiguousarray(J, dtype=np.float64)
    _call("rewl_set_lattice_bcc", ctx, inst, L, len(J), _dp(J))


def rewl_set_couplings_explicit(ctx, inst, N, i, j, J):
    i = np.ascontiguousarray(i, dtype=np.int32)
    j = np.ascontiguousarray(j, dtype=np.int32)
    J = np.ascontiguousarray(J, dtype=np.float64)
    _call("rewl_set_couplings_explicit", ctx, inst, N, len(i), i.ctypes.data_as(_P(_i32)),
          j.ctypes.data_as(_P(_i32)), _dp(J))


def rewl_set_windows(ctx, inst, E_min, E_max, n_bins, n_windows, overlap, walkers_per_window):
    _call("rewl_set_windows", ctx, inst, E_min, E_max, n_bins, n_windows, overlap,
          walkers_per_window)


def rewl_set_schedule(ctx, inst, flat_num, flat_den, lnf_init, lnf_final, exchange_interval,
                      resync_interval):
    _call("rewl_set_schedule", ctx, inst, flat_num, flat_den, lnf_init, lnf_final,
          exchange_interval, resync_interval)


def rewl_set_window_sharing(ctx, inst, on):
    _call("rewl_set_window_sharing", ctx, inst, 1 if on else 0)


def rewl_set_coordinate(ctx, inst, coord):
    _call("rewl_set_coordinate", ctx, inst, {"E": 0, "Mz": 1}[coord] if isinstance(coord, str) else coord)


def rewl_query_sizes(ctx):
    out = (_sz * NBUF)()
    _call("rewl_query_sizes", ctx, out)
    return [int(x) for x in out]


def rewl_bind_buffers(ctx, ptrs):
    arr = (_vp * NBUF)(*[_vp(p) for p in ptrs])
    _call("rewl_bind_buffers", ctx, arr)


def rewl_init_walkers(ctx, seed, init_spins=None):
    if init_spins is None:
        _call("rewl_init_walkers", ctx, seed, None)
    else:
        s = np.ascontiguousarray(init_spins, dtype=np.float64)
        _call("rewl_init_walkers", ctx, seed, _dp(s))


def rewl_run(ctx, n_segments):
    _call("rewl_run", ctx, n_segments)


def rewl_sweep(ctx):
    _call("rewl_sweep", ctx)


def rewl_exchange(ctx):
    _call("rewl_exchange", ctx)


def rewl_poll(ctx):
    d = _i32()
    _call("rewl_poll", ctx, C.byref(d))
    return bool(d.value)


def _read_bins(name, ctx, inst, walker, cap, dtype, ct):
    out = np.zeros(cap, dtype=dtype)
    n = _i32()
    _call(name, ctx, inst, walker, out.ctypes.data_as(_P(ct)), cap, C.byref(n))
    return out[: n.value]


def rewl_read_lng(ctx, inst, walker, cap=4096):
    return _read_bins("rewl_read_lng", ctx, inst, walker, cap, np.float64, _dbl)


def rewl_read_hist(ctx, inst, walker, cap=4096):
    return _read_bins("rewl_read_hist", ctx, inst, walker, cap, np.uint32, C.c_uint32)


def rewl_read_visited(ctx, inst, walker, cap=4096):
    return _read_bins("rewl_read_visited", ctx, inst, walker, cap, np.uint8, C.c_uint8)


def rewl_read_walker_state(ctx, inst, walker):
    st = rewl_walker_state()
    _call("rewl_read_walker_state", ctx, inst, walker, C.byref(st))
    return {f: getattr(st, f) for f, _ in rewl_walker_state._fields_}


def rewl_write_lng(ctx, inst, walker, lng, visited=None):
    lng = np.ascontiguousarray(lng, dtype=np.float64)
    if visited is None:
        _call("rewl_write_lng", ctx, inst, walker, _dp(lng), None, len(lng))
    else:
        v = np.ascontiguousarray(visited, dtype=np.uint8)
        _call("rewl_write_lng", ctx, inst, walker, _dp(lng), v.ctypes.data_as(_P(C.c_uint8)), len(lng))


def rewl_run_persistent(ctx, max_rounds, max_blocks=0):
    g = _i32(0)
    _call("rewl_run_persistent", ctx, max_rounds, max_blocks, C.byref(g))
    return g.value


def rewl_autotune(ctx, segments, persistent=False):
    arr = (rewl_tune_entry * 32)()
    n = _i32(0)
    _call("rewl_autotune", ctx, segments, 1 if persistent else 0, arr, 32, C.byref(n))
    return [{f: getattr(arr[k], f) for f, _ in rewl_tune_entry._fields_ if f != "pad"} for k in range(n.value)]


def rewl_fingerprint(ctx):
    d = _u64(0)
    _call("rewl_fingerprint", ctx, C.byref(d))
    return d.value


def rewl_read_round_trips(ctx, inst, n):
    out = np.zeros(n, dtype=np.uint32)
    _call("rewl_read_round_trips", ctx, inst, out.ctypes.data_as(_P(C.c_uint32)), n)
    return out


def rewl_save(ctx, path):
    _call("rewl_save", ctx, os.fsencode(path))


def rewl_load(ctx, path):
    _call("rewl_load", ctx, os.fsencode(path))


def rewl_read_config(ctx, inst, config, N):
    out = np.zeros(3 * N)
    _call("rewl_read_config", ctx, inst, config, _dp(out), 3 * N)
    return out.reshape(N, 3)


def rewl_read_window(ctx, inst, win):
    lo, hi = _i32(), _i32()
    _call("rewl_read_window", ctx, inst, win, C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def rewl_read_exchange_stats(ctx, inst, n_pairs):
    att = np.zeros(max(n_pairs, 1), dtype=np.uint64)
    acc = np.zeros(max(n_pairs, 1), dtype=np.uint64)
    _call("rewl_read_exchange_stats", ctx, inst, att.ctypes.data_as(_P(_u64)),
          acc.ctypes.data_as(_P(_u64)), n_pairs)
    return att[:n_pairs], acc[:n_pairs]


def rewl_read_step(ctx):
    s = _i64()
    _call("rewl_read_step", ctx, C.byref(s))
    return s.value


def rewl_set_trace(ctx, dev_ptr, capacity):
    _call("rewl_set_trace", ctx, _vp(dev_ptr) if dev_ptr else None, capacity)


def rewl_set_launch(ctx, walkers_per_block, residency=0):
    _call("rewl_set_launch", ctx, walkers_per_block, residency)


def rewl_set_grid_cap(ctx, max_blocks):
    _call("rewl_set_grid_cap", ctx, max_blocks)


def rewl_get_grid_cap(ctx):
    g = _i32()
    _call("rewl_get_grid_cap", ctx, C.byref(g))
    return g.value


def rewl_get_launch(ctx):
    w, r, b = _i32(), _i32(), _i64()
    _call("rewl_get_launch", ctx, C.byref(w), C.byref(r), C.byref(b))
    return dict(walkers_per_block=w.value, spins_in_lds=bool(r.value), lds_bytes_per_block=b.value)


def rewl_set_proposal(ctx, kind, dev_params_ptr=None):
    _call("rewl_set_proposal", ctx, kind, _vp(dev_params_ptr) if dev_params_ptr else None)


def rewl_set_harvest(ctx, dev_records_ptr, capacity_per_walker, every_k):
    _call("rewl_set_harvest", ctx, _vp(dev_records_ptr) if dev_records_ptr else None,
          capacity_per_walker, every_k)


def rewl_read_harvest_counts(ctx, n_walkers):
    out = np.zeros(n_walkers, dtype=np.int64)
    _call("rewl_read_harvest_counts", ctx, out.ctypes.data_as(_P(_i64)), n_walkers)
    return out


def rewl_mlp_param_count():
    return int(_lib.rewl_mlp_param_count())


def rewl_mlp_packed_bytes():
    return int(_lib.rewl_mlp_packed_bytes())


def rewl_mlp_workspace_bytes(max_batch):
    b = _sz()
    _call("rewl_mlp_workspace_bytes", max_batch, C.byref(b))
    return b.value


def rewl_mlp_pack(dev_params, dev_packed, stream=0):
    _call("rewl_mlp_pack", _vp(dev_params), _vp(dev_packed), _vp(stream))


def rewl_mlp_eval(dev_packed, dev_x, dev_s, dev_u, dev_udir, dev_lnq_s, dev_sample, dev_lnq_sample,
                  n, stream=0):
    _call("rewl_mlp_eval", _vp(dev_packed), _vp(dev_x), _vp(dev_s), _vp(dev_u), _vp(dev_udir),
          _vp(dev_lnq_s), _vp(dev_sample), _vp(dev_lnq_sample), n, _vp(stream))


def rewl_mlp_loss_grad(dev_records, n, dev_params, dev_grad, dev_workspace, stream=0):
    loss = C.c_double()
    _call("rewl_mlp_loss_grad", _vp(dev_records), n, _vp(dev_params), _vp(dev_grad), C.byref(loss),
          _vp(dev_workspace), _vp(stream))
    return loss.value


def rewl_mlp_train(dev_records, n, epochs, batch, lr, seed, dev_params, dev_workspace, stream=0):
    losses = np.zeros(max(epochs, 1), dtype=np.float32)
    _call("rewl_mlp_train", _vp(dev_records), n, epochs, batch, lr, seed, _vp(dev_params),
          _vp(dev_workspace), losses.ctypes.data_as(_P(C.c_float)), _vp(stream))
    return losses[:epochs]


def rewl_mlp_train_static(dev_records, n, epochs, batch, lr, seed, dev_params, stream=0):
    losses = np.zeros(max(epochs, 1), dtype=np.float32)
    _call("rewl_mlp_train_static", _vp(dev_records), n, epochs, batch, lr, seed, _vp(dev_params),
          losses.ctypes.data_as(_P(C.c_float)), _vp(stream))
    return losses[:epochs]


def rewl_total_attempts(ctx):
    a, b = _u64(), _u64()
    _call("rewl_total_attempts", ctx, C.byref(a), C.byref(b))
    return a.value, b.value


class Run:
    """One context with its torch-owned device buffers.

    instances: list of dicts with keys
      lattice: ("bcc", L, J) or ("explicit", N, i, j, J)
      windows: (E_min, E_max, n_bins, n_windows, overlap, walkers_per_window)
      schedule: (flat_num, flat_den, lnf_init, lnf_final, exchange_interval, resync_interval)
      share: optional, True for window sharing (rewl_set_window_sharing)
      coord: optional, "E" (default) or "Mz" (rewl_set_coordinate)
    """

    def __init__(self, instances, mode="fp64_det", device=0, stream=None, trace_cap=0,
                 walkers_per_block=1, residency=0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.mode = MODES[mode] if isinstance(mode, str) else int(mode)
        self.ctx = rewl_create(device, self.stream.cuda_stream, self.mode)
        self.inst = []
        for d in instances:
            i = rewl_add_instance(self.ctx)
            lat = d["lattice"]
            if lat[0] == "bcc":
                rewl_set_lattice_bcc(self.ctx, i, lat[1], lat[2])
                N = 2 * lat[1] ** 3
            else:
                rewl_set_couplings_explicit(self.ctx, i, lat[1], lat[2], lat[3], lat[4])
                N = lat[1]
            rewl_set_windows(self.ctx, i, *d["windows"])
            rewl_set_schedule(self.ctx, i, *d["schedule"])
            if d.get("share"):
                rewl_set_window_sharing(self.ctx, i, True)
            if d.get("coord", "E") != "E":
                rewl_set_coordinate(self.ctx, i, d["coord"])
            self.inst.append(dict(N=N, h=d["windows"][3], m=d["windows"][5]))
        self.sizes = rewl_query_sizes(self.ctx)
        self.bufs = [torch.empty(max(s, 256), dtype=torch.uint8, device=self.device)
                     for s in self.sizes]
        rewl_bind_buffers(self.ctx, [b.data_ptr() for b in self.bufs])
        if walkers_per_block != 1 or residency != 0:
            rewl_set_launch(self.ctx, walkers_per_block, residency)
        self.n_walkers = sum(q["h"] * q["m"] for q in self.inst)
        self.trace_cap = trace_cap
        self.trace_buf = None
        if trace_cap:
            self.trace_buf = torch.zeros(self.n_walkers * trace_cap * TRACE_DTYPE.itemsize,
                                         dtype=torch.uint8, device=self.device)
            rewl_set_trace(self.ctx, self.trace_buf.data_ptr(), trace_cap)

    def close(self):
        if getattr(self, "ctx", None):
            rewl_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, seed, init_spins=None):
        rewl_init_walkers(self.ctx, seed, init_spins)

    def run(self, n_segments):
        rewl_run(self.ctx, n_segments)

    def sweep(self):
        rewl_sweep(self.ctx)

    def exchange(self):
        rewl_exchange(self.ctx)

    def poll(self):
        return rewl_poll(self.ctx)

    def run_to_convergence(self, max_segments=10 ** 9, chunk=256):
        done = 0
        while done < max_segments:
            n = min(chunk, max_segments - done)
            self.run(n)
            done += n
            if self.poll():
                break
        return done

    def window(self, inst, walker):
        return rewl_read_window(self.ctx, inst, walker // self.inst[inst]["m"])

    def lng(self, inst, walker):
        return rewl_read_lng(self.ctx, inst, walker)

    def hist(self, inst, walker):
        return rewl_read_hist(self.ctx, inst, walker)

    def visited(self, inst, walker):
        return rewl_read_visited(self.ctx, inst, walker).astype(bool)

    def walker(self, inst, walker):
        return rewl_read_walker_state(self.ctx, inst, walker)

    def write_lng(self, inst, walker, lng, visited=None):
        rewl_write_lng(self.ctx, inst, walker, lng, visited)

    def run_persistent(self, max_rounds, max_blocks=0):
        """All instances advance up to max_rounds rounds in one launch;
        returns the grid size used."""
        return rewl_run_persistent(self.ctx, max_rounds, max_blocks)

    def autotune(self, segments=2, persistent=False, cache=None):
        """Choose walkers per block and residency (and, for the persistent
        kernel, a grid cap) by timing; the walk's state is restored, so
        results do not change.  With `cache` (a JSON file path) a shape
        chosen earlier for the same configuration digest is applied without
        timing.  Returns the trials (empty when cached)."""
        import json
        key = "%016x/%s" % (rewl_fingerprint(self.ctx), "persistent" if persistent else "run")
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                w, r = table[key][:2]
                rewl_set_launch(self.ctx, w, r)
                if persistent and len(table[key]) > 2:
                    rewl_set_grid_cap(self.ctx, table[key][2])
                return []
        trials = rewl_autotune(self.ctx, segments, persistent)
        if cache:
            lc = rewl_get_launch(self.ctx)
            table[key] = [lc["walkers_per_block"], 1 if lc["spins_in_lds"] else 2]
            if persistent:
                table[key].append(rewl_get_grid_cap(self.ctx))
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1)
            os.replace(tmp, cache)
        return trials

    def round_trips(self, inst):
        """Half round trips (lowest <-> highest window) per configuration."""
        return rewl_read_round_trips(self.ctx, inst, self.inst[inst]["h"] * self.inst[inst]["m"])

    def save(self, path):
        rewl_save(self.ctx, path)

    def load(self, path):
        rewl_load(self.ctx, path)

    def config(self, inst, cfg):
        return rewl_read_config(self.ctx, inst, cfg, self.inst[inst]["N"])

    def exchange_stats(self, inst):
        return rewl_read_exchange_stats(self.ctx, inst, self.inst[inst]["h"] - 1)

    def step(self):
        return rewl_read_step(self.ctx)

    def total_attempts(self):
        return rewl_total_attempts(self.ctx)

    def set_proposal(self, params=None):
        """params: torch float32 tensor on the device (learned) or None (uniform)."""
        if params is None:
            rewl_set_proposal(self.ctx, 0, None)
        else:
            self._mlp_params = params
            rewl_set_proposal(self.ctx, 1, params.data_ptr())

    def set_harvest(self, capacity_per_walker, every_k):
        self.harvest_cap = capacity_per_walker
        self.harvest_buf = self.torch.zeros(self.n_walkers * capacity_per_walker * 8,
                                            dtype=self.torch.float32, device=self.device)
        rewl_set_harvest(self.ctx, self.harvest_buf.data_ptr(), capacity_per_walker, every_k)

    def harvested(self):
        """All harvested records as a (n, 8) float32 device tensor."""
        counts = rewl_read_harvest_counts(self.ctx, self.n_walkers)
        recs = self.harvest_buf.view(self.n_walkers, self.harvest_cap, 8)
        parts = [recs[w, :int(c)] for w, c in enumerate(counts) if c > 0]
        return self.torch.cat(parts) if parts else recs[:0, 0]

    def set_launch(self, walkers_per_block, residency=0):
        rewl_set_launch(self.ctx, walkers_per_block, residency)

    def grid_cap(self):
        """Grid cap of run_persistent calls with max_blocks = 0 (0: none)."""
        return rewl_get_grid_cap(self.ctx)

    def set_grid_cap(self, max_blocks):
        rewl_set_grid_cap(self.ctx, max_blocks)

    def launch(self):
        return rewl_get_launch(self.ctx)

    def trace(self, walker_global):
        self.torch.cuda.synchronize(self.device)
        raw = self.trace_buf.cpu().numpy().view(TRACE_DTYPE)
        return raw[walker_global * self.trace_cap:(walker_global + 1) * self.trace_cap]
