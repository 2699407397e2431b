"""Window sharing on the GPU (rewl_set_window_sharing) through the C ABI.

* FP64 deterministic mode against the oracle with the same option: the whole
  run to convergence (merges, ln f halvings, exchanges) reproduces the
  oracle bit for bit: trajectories, ln g~, H, visited flags, states,
  configurations.
* The merge in the persistent batched kernel and with H kept in HBM equals
  the launch-per-segment walk bit for bit (FP32_DE); the window's walkers
  advance through the iterations together and finish with one ln g~.
"""
import sys

import numpy as np
import pytest

from helpers import bits, gpu_from, oracle_from, progress
from test_gpu_parity import _compare_state, _compare_trace
from test_gpu_persistent import _compare

pytestmark = pytest.mark.gpu

WL = dict(lattice=("bcc", 4, [1.0, 0.5]), windows=(-400.0, -100.0, 30, 2, 0.75, 3),
          schedule=(4, 5, 1.0, 2.0 ** -8, 5000, 12800), seed=11, share=True)


_say = progress


def _windows_identical(g, inst, h, m):
    for k in range(h):
        ref = bits(g.lng(inst, k * m))
        for w in range(k * m, (k + 1) * m):
            s = g.walker(inst, w)
            # iterations advance together; once done, ln g~ is the window's
            assert s["iteration"] == g.walker(inst, k * m)["iteration"], (inst, w)
            assert s["done"] == g.walker(inst, k * m)["done"], (inst, w)
            if s["done"]:
                assert np.array_equal(bits(g.lng(inst, w)), ref), (inst, w)
                assert np.array_equal(g.visited(inst, w), g.visited(inst, k * m)), (inst, w)


def test_det_share_bit_exact_to_convergence():
    cap = 5000
    o = oracle_from(WL, trace=cap)
    n = o.run_to_convergence(max_segments=3000, chunk=1)
    assert o.all_done()
    _say("share det: oracle done after", n, "segments; gpu")
    g = gpu_from(WL, "fp64_det", trace=cap)
    g.run(n)
    assert g.poll()
    h, m = WL["windows"][3], WL["windows"][5]
    for w in range(h * m):
        _compare_trace(o, g, w, w, cap)
    _compare_state(o, g)
    _windows_identical(g, 0, h, m)
    ao, co = o.exchange_stats()
    ag, cg = g.exchange_stats(0)
    assert np.array_equal(ao, ag) and np.array_equal(co, cg)


def _shared_workloads():
    mk = lambda L, J, win, sched, seed=5: dict(lattice=("bcc", L, J), windows=win, schedule=sched,
                                              seed=seed, share=True)
    return [
        dict(WL, schedule=(4, 5, 1.0, 2.0 ** -10, 5000, 12800)),
        mk(6, [1.0, 0.6, -0.05, -0.1], (-1500.0, -1380.0, 40, 2, 0.75, 4), (4, 5, 1.0, 2.0 ** -10, 5000, 43200)),
        # sharing off beside it
        dict(mk(4, [1.0, 0.5], (-600.0, -100.0, 60, 3, 0.75, 2), (4, 5, 1.0, 2.0 ** -12, 5000, 12800)),
             share=False),
    ]


@pytest.mark.parametrize("residency", [0, 2])
def test_share_persistent_equals_launch_per_segment(residency):
    cfgs = _shared_workloads()
    a, b = _compare(cfgs, "fp32_de", 160, 1, residency)
    for i, c in enumerate(cfgs[:2]):
        h, m = c["windows"][3], c["windows"][5]
        assert max(a.walker(i, w)["iteration"] for w in range(h * m)) >= 2, i
        _windows_identical(a, i, h, m)
