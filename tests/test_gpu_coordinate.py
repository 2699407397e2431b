"""The walk over the magnetisation M_z = sum_i S_i^z (rewl_set_coordinate)
through the C ABI.

* FP64 deterministic mode against the oracle with the same coordinate, bit
  for bit: per-move traces, ln g~, H, visited flags, states and
  configurations, on bcc L=4 (two windows, exchanges) and, run to the end,
  on a four-spin chain.
* FP64 and FP32_DE modes against the closed form: over N spins M_z is a sum
  of N independent U(-1, 1) (each S^z of a uniform unit vector is uniform),
  so ln g over M_z bins is ln of Irwin-Hall bin masses; the mean of 32
  independent runs lies within 0.05 of it on every bin (the oracle meets the
  same closed form to 0.02; tests/test_oracle_coordinate.py).
* A context with such an instance refuses the fast-only calls.
"""
import sys

import numpy as np
import pytest

from helpers import gpu_from, oracle_from, progress
from test_gpu_parity import _compare_state, _compare_trace
from test_oracle_coordinate import _exact_lng

pytestmark = pytest.mark.gpu

BCC = dict(lattice=("bcc", 4, [1.0, 0.5]), windows=(-24.0, 24.0, 24, 2, 0.75, 2),
           schedule=(4, 5, 1.0, 2.0 ** -8, 3000, 1280), seed=7, coord="Mz")


def _chain(N=4, seed=100):
    return dict(lattice=("explicit", N, list(range(N - 1)), list(range(1, N)), [1.0] * (N - 1)),
                windows=(-float(N), float(N), 16, 1, 0.75, 2),
                schedule=(4, 5, 1.0, 2.0 ** -12, 20000, 0), seed=seed, coord="Mz")


_say = progress


def test_det_mz_walk_bit_exact_bcc():
    cap = 9000
    o = oracle_from(BCC, trace=cap)
    g = gpu_from(BCC, "fp64_det", trace=cap)
    _compare_state(o, g)
    o.run(3)
    g.run(3)
    for w in range(4):
        _compare_trace(o, g, w, w, cap)
    _compare_state(o, g)
    ao, co = o.exchange_stats()
    ag, cg = g.exchange_stats(0)
    assert np.array_equal(ao, ag) and np.array_equal(co, cg)


def test_det_mz_walk_bit_exact_to_convergence():
    cfg = _chain()
    o = oracle_from(cfg, trace=4000)
    n = o.run_to_convergence(max_segments=20000, chunk=1)
    assert o.all_done()
    g = gpu_from(cfg, "fp64_det", trace=4000)
    g.run(n)
    assert g.poll()
    for w in range(2):
        _compare_trace(o, g, w, w, 4000)
    _compare_state(o, g)


@pytest.mark.parametrize("mode", ["fp64", "fp32_de"])
def test_mz_walk_matches_irwin_hall(mode):
    from oracle.analysis import combine_walkers, normalise
    N, R = 4, 32
    cfg = _chain(N)
    g = gpu_from([cfg] * R, mode)
    g.run_to_convergence(max_segments=40000, chunk=256)
    assert g.poll()
    runs = []
    for i in range(R):
        lg, vis = combine_walkers([g.lng(i, w) for w in range(2)], [g.visited(i, w) for w in range(2)])
        assert np.all(vis)
        runs.append(normalise(lg))
    d = np.mean(runs, axis=0) - normalise(_exact_lng(N, -N, N, 16))
    _say(mode, "Mz vs Irwin-Hall", np.round(d, 3))
    assert np.max(np.abs(d)) < 0.05


def test_mz_context_refuses_fast_only_calls():
    from paper_1411_4212_amd import learned
    from paper_1411_4212_amd.rewl import RewlError
    import torch
    g = gpu_from(BCC, "fp32_de")
    assert g.launch()["spins_in_lds"]
    with pytest.raises(RewlError):
        g.run_persistent(1)
    with pytest.raises(RewlError):
        g.set_proposal(learned.init_params(3, torch.device("cuda", 0)))


def test_det_mz_walk_with_window_sharing_bit_exact():
    """The two variants together: an M_z walk whose window walkers share ln g~
    (bcc L=4, two windows x 2 walkers, to convergence) equals the oracle bit
    for bit."""
    cfg = dict(BCC, schedule=(4, 5, 1.0, 2.0 ** -6, 3000, 1280), share=True)
    o = oracle_from(cfg, trace=3000)
    n = o.run_to_convergence(max_segments=4000, chunk=1)
    assert o.all_done()
    _say("Mz + sharing: oracle done after", n, "segments")
    g = gpu_from(cfg, "fp64_det", trace=3000)
    g.run(n)
    assert g.poll()
    for w in range(4):
        _compare_trace(o, g, w, w, 3000)
    _compare_state(o, g)
