"""CPU oracle for replica-exchange Wang-Landau sampling (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It is a plain, slow FP64
implementation written from the paper (Model; Sec. "original Wang-Landau";
Sec. "parallel scheme"; Sec. "simulation details") and shares no code with the
GPU path.  The C core is ``rewl_oracle.c``; this module only marshals
arguments.
"""
import ctypes as C
import os

import numpy as np

from .build import LIB, build_oracle

_lib = None

TRACE_DTYPE = np.dtype([("site", "<u4"), ("flags", "<u4"), ("E", "<f8"),
                        ("bin", "<i4"), ("attempt_lo", "<u4")])
# drive into the window: flags bit 0 accepted, bit 1 proposal inside the window
DRIVE_DTYPE = np.dtype([("attempt", "<u4"), ("flags", "<u4"), ("E", "<f8"), ("Eb", "<f8")])


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("REWL_ORACLE_LIB", LIB)
        if path == LIB and not os.path.exists(LIB):
            build_oracle()
        L = C.CDLL(path)
        vp, i32, i64, u32, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double
        P = C.POINTER
        L.orc_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.orc_sphere.argtypes = [u32, u32, C.c_uint64, u32, P(dbl)]
        L.orc_exp_det.argtypes = [dbl]
        L.orc_exp_det.restype = dbl
        L.orc_bcc_shells.argtypes = [i32, P(i32), P(i32), P(i32), P(i32), i32]
        L.orc_bcc_site.argtypes = [i32, i32, i32, i32, i32]
        L.orc_window_bins.argtypes = [i32, i32, dbl, i32, P(i32), P(i32)]
        L.orc_create_bcc.argtypes = [i32, i32, P(dbl)]
        L.orc_create_bcc.restype = vp
        L.orc_create_explicit.argtypes = [i32, i64, P(i32), P(i32), P(dbl)]
        L.orc_create_explicit.restype = vp
        L.orc_destroy.argtypes = [vp]
        L.orc_num_sites.argtypes = [vp]
        L.orc_max_degree.argtypes = [vp]
        L.orc_neighbours.argtypes = [vp, i32, P(i32), P(dbl), i32]
        L.orc_energy.argtypes = [vp, P(dbl)]
        L.orc_energy.restype = dbl
        L.orc_local_field.argtypes = [vp, P(dbl), i32, P(dbl)]
        L.orc_set_windows.argtypes = [vp, dbl, dbl, i32, i32, dbl, i32]
        L.orc_set_schedule.argtypes = [vp, i32, i32, dbl, dbl, i64, i64]
        L.orc_set_threads.argtypes = [vp, i32]
        L.orc_set_ids.argtypes = [vp, u32, u32]
        L.orc_set_check_energy.argtypes = [vp, i32]
        L.orc_max_check_err.argtypes = [vp]
        L.orc_max_check_err.restype = dbl
        L.orc_set_trace.argtypes = [vp, i64]
        L.orc_wl_accept_prob.argtypes = [dbl, dbl]
        L.orc_wl_accept_prob.restype = dbl
        L.orc_wl_accept_prob_q.argtypes = [dbl, dbl, dbl, dbl]
        L.orc_wl_accept_prob_q.restype = dbl
        L.orc_re_accept_prob.argtypes = [dbl, dbl, dbl, dbl]
        L.orc_re_accept_prob.restype = dbl
        L.orc_init.argtypes = [vp, u32, P(dbl)]
        L.orc_run.argtypes = [vp, i64]
        L.orc_run.restype = i64
        L.orc_exchange.argtypes = [vp]
        L.orc_all_done.argtypes = [vp]
        L.orc_num_walkers.argtypes = [vp]
        L.orc_window.argtypes = [vp, i32, P(i32), P(i32)]
        L.orc_read_lng.argtypes = [vp, i32, P(dbl), i32]
        L.orc_read_hist.argtypes = [vp, i32, P(C.c_uint32), P(C.c_uint8), i32]
        L.orc_read_walker.argtypes = [vp, i32, P(dbl), P(i32), P(C.c_uint64)]
        L.orc_read_config.argtypes = [vp, i32, P(dbl)]
        L.orc_read_exchange_stats.argtypes = [vp, P(C.c_uint64), P(C.c_uint64)]
        L.orc_step_counter.argtypes = [vp]
        L.orc_step_counter.restype = i64
        L.orc_read_trace.argtypes = [vp, i32, vp, i64]
        L.orc_set_proposal_mlp.argtypes = [vp, P(dbl)]
        L.orc_mlp_param_count.argtypes = []
        L.orc_mlp_log_q.argtypes = [P(dbl), P(dbl), P(dbl)]
        L.orc_mlp_log_q.restype = dbl
        L.orc_mlp_sample.argtypes = [P(dbl), P(dbl), P(dbl), P(dbl), P(dbl)]
        L.orc_set_drive_trace.argtypes = [vp, i64]
        L.orc_read_drive.argtypes = [vp, i32, vp, i64]
        L.orc_read_drive.restype = i64
        L.orc_read_round_trips.argtypes = [vp, P(C.c_uint32), i32]
        L.orc_write_lng.argtypes = [vp, i32, P(dbl), P(C.c_uint8), i32]
        L.orc_shift_energy.argtypes = [vp, i32, dbl]
        L.orc_set_share.argtypes = [vp, i32]
        L.orc_set_coordinate.argtypes = [vp, i32]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def sphere(seed, stream, n, tag=1):
    out = np.zeros(3)
    lib().orc_sphere(seed, stream, n, tag, _p(out, C.c_double))
    return out


def exp_det(x):
    return lib().orc_exp_det(float(x))


def wl_accept_prob(lng_a, lng_b):
    return lib().orc_wl_accept_prob(float(lng_a), float(lng_b))


def wl_accept_prob_q(lng_a, lng_b, lnq_old, lnq_new):
    return lib().orc_wl_accept_prob_q(float(lng_a), float(lng_b), float(lnq_old), float(lnq_new))


def re_accept_prob(lngi_a, lngi_b, lngj_b, lngj_a):
    return lib().orc_re_accept_prob(float(lngi_a), float(lngi_b), float(lngj_b), float(lngj_a))


def mlp_log_q(theta, x, s):
    """ln q(s | x) of the learned proposal with FP64 parameters theta."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    ss = np.ascontiguousarray(s, dtype=np.float64)
    return lib().orc_mlp_log_q(_p(th, C.c_double), _p(xx, C.c_double), _p(ss, C.c_double))


def mlp_sample(theta, x, u, uni):
    """One draw of the learned proposal for uniforms u = (u_mix, u_w, u_phi)
    and the direction `uni` used on its uniform branch."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    un = np.ascontiguousarray(uni, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_mlp_sample(_p(th, C.c_double), _p(xx, C.c_double), _p(uu, C.c_double),
                         _p(un, C.c_double), _p(out, C.c_double))
    return out


def bcc_shells(n_shells):
    cap = 4096
    dx, dy, dz, sh = (np.zeros(cap, dtype=np.int32) for _ in range(4))
    n = lib().orc_bcc_shells(n_shells, _p(dx, C.c_int32), _p(dy, C.c_int32), _p(dz, C.c_int32),
                             _p(sh, C.c_int32), cap)
    if n < 0:
        raise ValueError("too many shells")
    return np.stack([dx[:n], dy[:n], dz[:n]], axis=1), sh[:n]


def window_bins(B, h, o, k):
    lo, hi = C.c_int32(), C.c_int32()
    st = lib().orc_window_bins(B, h, o, k, C.byref(lo), C.byref(hi))
    if st != 0:
        raise ValueError("bad window arguments")
    return lo.value, hi.value


class OracleError(RuntimeError):
    pass


class Oracle:
    """One REWL run on the CPU: lattice + windows + schedule + walkers."""

    def __init__(self, *, L=None, J=None, explicit=None):
        L_ = lib()
        if explicit is not None:
            N, pi, pj, pJ = explicit
            pi = np.ascontiguousarray(pi, dtype=np.int32)
            pj = np.ascontiguousarray(pj, dtype=np.int32)
            pJ = np.ascontiguousarray(pJ, dtype=np.float64)
            self._c = L_.orc_create_explicit(int(N), len(pi), _p(pi, C.c_int32), _p(pj, C.c_int32),
                                             _p(pJ, C.c_double))
        else:
            Jarr = np.ascontiguousarray(J, dtype=np.float64)
            self._c = L_.orc_create_bcc(int(L), len(Jarr), _p(Jarr, C.c_double))
        if not self._c:
            raise OracleError("invalid lattice")
        self.N = L_.orc_num_sites(self._c)

    def __del__(self):
        c = getattr(self, "_c", None)
        if c:
            lib().orc_destroy(c)
            self._c = None

    def neighbours(self, i):
        cap = lib().orc_max_degree(self._c)
        nb = np.zeros(cap, dtype=np.int32)
        Jn = np.zeros(cap)
        d = lib().orc_neighbours(self._c, i, _p(nb, C.c_int32), _p(Jn, C.c_double), cap)
        return nb[:d], Jn[:d]

    def energy(self, spins):
        s = np.ascontiguousarray(spins, dtype=np.float64).reshape(-1, 3)
        return lib().orc_energy(self._c, _p(s, C.c_double))

    def local_field(self, spins, i):
        s = np.ascontiguousarray(spins, dtype=np.float64).reshape(-1, 3)
        h = np.zeros(3)
        lib().orc_local_field(self._c, _p(s, C.c_double), int(i), _p(h, C.c_double))
        return h

    def set_windows(self, E_min, E_max, n_bins, n_windows, overlap, walkers_per_window):
        st = lib().orc_set_windows(self._c, E_min, E_max, n_bins, n_windows, overlap,
                                   walkers_per_window)
        if st:
            raise OracleError("set_windows: %d" % st)
        self.h, self.m = n_windows, walkers_per_window

    def set_schedule(self, flat_num, flat_den, lnf_init, lnf_final, exchange_interval,
                     resync_interval):
        st = lib().orc_set_schedule(self._c, flat_num, flat_den, lnf_init, lnf_final,
                                    exchange_interval, resync_interval)
        if st:
            raise OracleError("set_schedule: %d" % st)

    def set_threads(self, n):
        lib().orc_set_threads(self._c, n)

    def set_ids(self, stream_base, instance):
        lib().orc_set_ids(self._c, stream_base, instance)

    def set_check_energy(self, on=True):
        lib().orc_set_check_energy(self._c, 1 if on else 0)

    def max_check_err(self):
        return lib().orc_max_check_err(self._c)

    def set_trace(self, cap):
        lib().orc_set_trace(self._c, cap)
        self.trace_cap = cap

    def set_proposal(self, theta=None):
        """Learned proposal with FP64 parameters theta (None: uniform)."""
        if theta is None:
            lib().orc_set_proposal_mlp(self._c, None)
            return
        th = np.ascontiguousarray(theta, dtype=np.float64)
        if th.size != lib().orc_mlp_param_count():
            raise OracleError("expected %d parameters" % lib().orc_mlp_param_count())
        lib().orc_set_proposal_mlp(self._c, _p(th, C.c_double))

    def set_coordinate(self, coord):
        """The walk's coordinate: "E" (energy, default) or "Mz" (magnetisation
        along z); before init.  Windows and bins are then over that value."""
        code = {"E": 0, "Mz": 1}[coord]
        if lib().orc_set_coordinate(self._c, code) != 0:
            raise OracleError("bad coordinate")

    def set_share(self, on=True):
        """Walkers of a window advance through the iterations together and
        share their ln g (before init)."""
        lib().orc_set_share(self._c, 1 if on else 0)

    def set_drive_trace(self, cap):
        lib().orc_set_drive_trace(self._c, cap)
        self.drive_cap = cap

    def drive(self, w):
        out = np.zeros(self.drive_cap, dtype=DRIVE_DTYPE)
        n = lib().orc_read_drive(self._c, w, out.ctypes.data_as(C.c_void_p), self.drive_cap)
        if n < 0:
            raise OracleError("no drive trace")
        return out[:n]

    def round_trips(self):
        out = np.zeros(self.W, dtype=np.uint32)
        n = lib().orc_read_round_trips(self._c, _p(out, C.c_uint32), self.W)
        if n < 0:
            raise OracleError("round trips: %d" % n)
        return out

    def write_lng(self, w, lng, visited=None):
        lg = np.ascontiguousarray(lng, dtype=np.float64)
        if visited is None:
            st = lib().orc_write_lng(self._c, w, _p(lg, C.c_double), None, lg.size)
        else:
            vi = np.ascontiguousarray(visited, dtype=np.uint8)
            st = lib().orc_write_lng(self._c, w, _p(lg, C.c_double), _p(vi, C.c_uint8), lg.size)
        if st:
            raise OracleError("write_lng: %d" % st)

    def shift_energy(self, w, delta):
        st = lib().orc_shift_energy(self._c, w, float(delta))
        if st:
            raise OracleError("shift_energy: %d" % st)

    def init(self, seed, init_spins=None):
        if init_spins is not None:
            s = np.ascontiguousarray(init_spins, dtype=np.float64).reshape(-1, 3)
            st = lib().orc_init(self._c, seed, _p(s, C.c_double))
        else:
            st = lib().orc_init(self._c, seed, None)
        if st:
            raise OracleError("init failed: %d" % st)
        self.W = lib().orc_num_walkers(self._c)

    def run(self, n_segments):
        r = lib().orc_run(self._c, n_segments)
        if r < 0:
            raise OracleError("run: %d" % r)
        return r

    def run_to_convergence(self, max_segments=10**9, chunk=64):
        total = 0
        while total < max_segments and not self.all_done():
            total += self.run(min(chunk, max_segments - total))
        return total

    def exchange(self):
        st = lib().orc_exchange(self._c)
        if st:
            raise OracleError("exchange: %d" % st)

    def all_done(self):
        return bool(lib().orc_all_done(self._c))

    def window(self, w):
        lo, hi = C.c_int32(), C.c_int32()
        lib().orc_window(self._c, w, C.byref(lo), C.byref(hi))
        return lo.value, hi.value

    def lng(self, w):
        lo, hi = self.window(w)
        out = np.zeros(hi - lo)
        lib().orc_read_lng(self._c, w, _p(out, C.c_double), hi - lo)
        return out

    def hist(self, w):
        lo, hi = self.window(w)
        H = np.zeros(hi - lo, dtype=np.uint32)
        vis = np.zeros(hi - lo, dtype=np.uint8)
        lib().orc_read_hist(self._c, w, _p(H, C.c_uint32), _p(vis, C.c_uint8), hi - lo)
        return H, vis.astype(bool)

    def walker(self, w):
        d = np.zeros(3)
        i = np.zeros(5, dtype=np.int32)
        u = np.zeros(3, dtype=np.uint64)
        lib().orc_read_walker(self._c, w, _p(d, C.c_double), _p(i, C.c_int32), _p(u, C.c_uint64))
        return dict(E=d[0], lnf=d[1], max_drift=d[2], bin=int(i[0]), iter=int(i[1]),
                    done=bool(i[2]), cfg=int(i[3]), nvis=int(i[4]), attempts=int(u[0]),
                    accepts=int(u[1]), out_of_window=int(u[2]))

    def config(self, cfg):
        out = np.zeros((self.N, 3))
        lib().orc_read_config(self._c, cfg, _p(out, C.c_double))
        return out

    def exchange_stats(self):
        n = max(self.h - 1, 1)
        att = np.zeros(n, dtype=np.uint64)
        acc = np.zeros(n, dtype=np.uint64)
        lib().orc_read_exchange_stats(self._c, _p(att, C.c_uint64), _p(acc, C.c_uint64))
        return att[: self.h - 1], acc[: self.h - 1]

    def step_counter(self):
        return lib().orc_step_counter(self._c)

    def trace(self, w):
        out = np.zeros(self.trace_cap, dtype=TRACE_DTYPE)
        n = lib().orc_read_trace(self._c, w, out.ctypes.data_as(C.c_void_p), self.trace_cap)
        if n < 0:
            raise OracleError("no trace")
        return out[:n]
