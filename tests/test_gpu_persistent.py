"""Persistent batched kernel (rewl_run_persistent): one launch in which
every instance advances on its own must reproduce, bit for bit, the
launch-per-segment walk (rewl_run) on the same inputs: ln g, H, visited
flags, walker states, configurations and exchange counters.  Covered:
uneven instances (L, windows, walkers per window), instances that finish
inside the launch, walkers per block 1/3/4, spins in LDS and in HBM, FP64
and FP32_DE, the learned proposal, and the 64-instance batched workload."""
import sys

import numpy as np
import pytest

from helpers import bits, gpu_from, progress

pytestmark = pytest.mark.gpu


_say = progress


def _uneven():
    mk = lambda L, J, win, sched, seed=5: dict(lattice=("bcc", L, J), windows=win, schedule=sched, seed=seed)
    return [
        mk(4, [1.0, 0.5], (-600.0, -100.0, 60, 3, 0.75, 2), (4, 5, 1.0, 2.0 ** -12, 5000, 12800)),
        # finishes inside the launch
        mk(4, [1.0, 0.5], (-100.0, 0.0, 4, 1, 0.75, 1), (1, 10, 1.0, 0.5, 3000, 12800)),
        mk(6, [1.0, 0.6, -0.05, -0.1], (-1500.0, -300.0, 120, 4, 0.75, 3), (4, 5, 1.0, 2.0 ** -12, 5000, 43200)),
        mk(8, [1.0, 0.6, -0.05, -0.1], (-3500.0, -500.0, 200, 5, 0.75, 2), (4, 5, 1.0, 2.0 ** -12, 5000, 102400)),
    ]


def _snapshot(g, cfgs):
    out = []
    for i, c in enumerate(cfgs):
        h, m = c["windows"][3], c["windows"][5]
        for w in range(h * m):
            st = g.walker(i, w)
            out.append((bits(g.lng(i, w)).tolist(), g.hist(i, w).tolist(), g.visited(i, w).tolist(),
                        {k: (bits(v).item() if isinstance(v, float) else v) for k, v in st.items()}))
            out.append(bits(g.config(i, st["config"])).tolist())
        out.append(np.asarray(g.exchange_stats(i)).tolist())
    return out


def _diff(a, b, cfgs):
    """First differences between two contexts, per instance and walker."""
    out = []
    for i, c in enumerate(cfgs):
        h, m = c["windows"][3], c["windows"][5]
        for w in range(h * m):
            sa, sb = a.walker(i, w), b.walker(i, w)
            keys = [k for k in sa if sa[k] != sb[k]]
            parts = [n for n, fa, fb in (("lng", a.lng, b.lng), ("hist", a.hist, b.hist), ("vis", a.visited, b.visited))
                     if not np.array_equal(np.asarray(fa(i, w)).view(np.uint8), np.asarray(fb(i, w)).view(np.uint8))]
            if keys or parts:
                out.append("inst %d walker %d: state %s %s a=%s b=%s" % (
                    i, w, keys, parts, {k: sa[k] for k in keys}, {k: sb[k] for k in keys}))
        xa, xb = np.asarray(a.exchange_stats(i)), np.asarray(b.exchange_stats(i))
        if not np.array_equal(xa, xb):
            out.append("inst %d exchange stats a=%s b=%s" % (i, xa.tolist(), xb.tolist()))
    return out


def _compare(cfgs, mode, rounds, wpb=1, residency=0, params=None, chunks=1, max_blocks=0):
    a = gpu_from(cfgs, mode, walkers_per_block=wpb, residency=residency)
    b = gpu_from(cfgs, mode, walkers_per_block=wpb, residency=residency)
    if params is not None:
        a.set_proposal(params)
        b.set_proposal(params)
    a.run(rounds)
    for _ in range(chunks):
        grid = b.run_persistent(rounds // chunks, max_blocks)
    _say("persistent", mode, "wpb", wpb, "residency", residency, "grid", grid, "rounds", rounds, "chunks", chunks)
    assert a.step() == b.step() == rounds
    d = _diff(a, b, cfgs)
    for line in d[:20]:
        _say(line)
    assert not d
    assert _snapshot(a, cfgs) == _snapshot(b, cfgs)
    return a, b


@pytest.mark.parametrize("max_blocks", [1, 2, 8, 0])
def test_persistent_grid_sizes(max_blocks):
    """One wavefront for everything up to one per walker."""
    _compare(_uneven(), "fp32_de", 8, 1, 0, max_blocks=max_blocks)


def test_persistent_single_rounds_equal_launch_per_segment():
    """One round per persistent launch: the round itself (queue, last-walker
    exchange) without cross-round ordering."""
    _compare(_uneven(), "fp32_de", 6, 1, 0, chunks=6)


@pytest.mark.parametrize("mode,wpb,residency", [("fp32_de", 1, 0), ("fp32_de", 4, 0), ("fp32_de", 3, 2),
                                                ("fp64", 1, 0), ("fp64", 2, 2)])
def test_persistent_equals_launch_per_segment(mode, wpb, residency):
    cfgs = _uneven()
    a, b = _compare(cfgs, mode, 24, wpb, residency)
    # the small instance stopped inside the launch; the others did not
    assert a.walker(1, 0)["done"] == 1
    # continuing both ways after the persistent launch stays identical
    a.run(3)
    b.run(3)
    assert _snapshot(a, cfgs) == _snapshot(b, cfgs)


def test_persistent_learned_proposal():
    from paper_1411_4212_amd import learned
    import torch
    params = learned.init_params(7, torch.device("cuda", 0))
    _compare(_uneven(), "fp32_de", 6, 2, 0, params=params)


def test_persistent_batched_workload():
    from paper_1411_4212_amd.workloads import batched
    cfgs = [dict(c, schedule=c["schedule"][:4] + (2000,) + c["schedule"][5:]) for c in batched(64)]
    _compare(cfgs, "fp32_de", 3, 1, 0)


def test_persistent_rejects_det_mode_and_zero_rounds():
    from paper_1411_4212_amd.rewl import RewlError
    g = gpu_from(_uneven()[:1], "fp64_det")
    with pytest.raises(RewlError) as e:
        g.run_persistent(2)
    assert e.value.code == -8
    f = gpu_from(_uneven()[:1], "fp32_de")
    assert f.run_persistent(0) == 0
    assert f.step() == 0
