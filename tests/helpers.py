"""Shared test helpers: build the oracle or the GPU path from one workload
description (paper_1411_4212_amd.workloads)."""
import numpy as np


def oracle_from(cfg, threads=4, trace=0, check_energy=False):
    import oracle
    lat = cfg["lattice"]
    if lat[0] == "bcc":
        o = oracle.Oracle(L=lat[1], J=lat[2])
    else:
        o = oracle.Oracle(explicit=(lat[1], lat[2], lat[3], lat[4]))
    o.set_windows(*cfg["windows"])
    o.set_schedule(*cfg["schedule"])
    o.set_threads(threads)
    if trace:
        o.set_trace(trace)
    if check_energy:
        o.set_check_energy(True)
    if cfg.get("share"):
        o.set_share(True)
    if cfg.get("coord", "E") != "E":
        o.set_coordinate(cfg["coord"])
    o.init(cfg["seed"])
    return o


def gpu_from(cfgs, mode, trace=0, seed=None, walkers_per_block=1, residency=0):
    import numpy as np
    from paper_1411_4212_amd.rewl import Run
    from paper_1411_4212_amd.workloads import init_spins
    if isinstance(cfgs, dict):
        cfgs = [cfgs]
    r = Run([dict(lattice=c["lattice"], windows=c["windows"], schedule=c["schedule"],
                  share=c.get("share", False), coord=c.get("coord", "E")) for c in cfgs], mode=mode, trace_cap=trace, walkers_per_block=walkers_per_block,
            residency=residency)
    starts = [init_spins(c) for c in cfgs]
    if all(s is None for s in starts):
        init = None
    else:
        init = np.concatenate([s if s is not None else _random_unit(c) for s, c in zip(starts, cfgs)])
    r.init(cfgs[0]["seed"] if seed is None else seed, init)
    return r


def _random_unit(cfg):
    raise ValueError("mixing random and given starts is not supported in tests")


def joined_lng(read_lng, read_vis, window, h, m):
    """Combine walkers per window and join windows (oracle analysis)."""
    from oracle.analysis import combine_walkers, join_windows
    frags = []
    for k in range(h):
        ws = range(k * m, (k + 1) * m)
        lo, hi = window(k * m)
        lg, vis = combine_walkers([read_lng(w) for w in ws], [read_vis(w) for w in ws])
        frags.append((lo, hi, lg, vis))
    return join_windows(frags)


def bits(x):
    return np.asarray(x, dtype=np.float64).view(np.uint64)


def wl_truth_bound(ref_mean, truth, margin=0.1):
    """Bound on a Wang-Landau mean's distance from the fixed-weight ln g:
    the oracle's own Wang-Landau mean's largest distance from it (the
    estimator's error at the final ln f, largest at the lowest bin of a range
    reaching towards the ordered state) plus `margin`."""
    from oracle.analysis import normalise
    a, b = np.asarray(ref_mean, dtype=float), np.asarray(truth, dtype=float)
    ok = np.isfinite(a) & np.isfinite(b)
    return float(np.max(np.abs(normalise(a, ok)[ok] - normalise(b, ok)[ok]))) + margin


_progress_writer = None


def set_progress_writer(fn):
    global _progress_writer
    _progress_writer = fn


def progress(*a):
    """A progress line of a long GPU test.  It reaches the terminal even while
    pytest captures the test's output (tests/conftest.py installs the
    writer): a run that prints nothing for minutes looks hung."""
    msg = " ".join(str(x) for x in a)
    if _progress_writer is not None:
        _progress_writer(msg)
    else:
        print(msg, flush=True)
