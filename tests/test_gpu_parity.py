"""GPU path vs the CPU oracle through the C ABI.

Deterministic FP64 mode: trajectories (site, accept bit, energy, bin of every
trial move), ln g~, H, visited flags, walker states and configurations are
compared bit for bit on the same Philox seed.
"""
import sys

import numpy as np
import pytest

from helpers import bits, gpu_from, oracle_from, progress

pytestmark = pytest.mark.gpu


_say = progress


def _compare_state(o, g, inst=0, walkers=None, check_config=True):
    W = o.W if walkers is None else walkers
    for w in range(W):
        so, sg = o.walker(w), g.walker(inst, w)
        assert bits(so["E"]) == bits(sg["E"]), (w, so["E"], sg["E"])
        assert so["bin"] == sg["bin"], w
        assert so["lnf"] == sg["lnf"] and so["iter"] == sg["iteration"], w
        assert so["done"] == bool(sg["done"]), w
        assert so["cfg"] == sg["config"], w
        assert so["attempts"] == sg["attempts"] and so["accepts"] == sg["accepts"], w
        assert so["out_of_window"] == sg["rejected_outside"], w
        assert so["nvis"] == sg["n_visited"], w
        assert np.array_equal(bits(o.lng(w)), bits(g.lng(inst, w))), w
        Ho, vo = o.hist(w)
        assert np.array_equal(Ho, g.hist(inst, w)), w
        assert np.array_equal(vo, g.visited(inst, w)), w
        if check_config:
            c = so["cfg"]
            assert np.array_equal(bits(o.config(c)), bits(g.config(inst, c))), w


def _compare_trace(o, g, w_local, w_global, n):
    to, tg = o.trace(w_local)[:n], g.trace(w_global)[:n]
    assert np.array_equal(to["site"], tg["site"]), w_local
    assert np.array_equal(to["flags"], tg["flags"]), w_local
    assert np.array_equal(to["bin"], tg["bin"]), w_local
    assert np.array_equal(bits(to["E"]), bits(tg["E"])), w_local


def test_det_c1_trajectories_bit_exact():
    """bcc L=4 workload: three segments (3e4 moves per walker, with two
    exchange steps and flatness tests) reproduce the oracle bit for bit."""
    from paper_1411_4212_amd.workloads import c1
    cfg = c1()
    cap = 30000
    _say("c1 det: oracle")
    o = oracle_from(cfg, trace=cap)
    _say("c1 det: gpu init")
    g = gpu_from(cfg, "fp64_det", trace=cap)
    _compare_state(o, g)
    o.run(3)
    _say("c1 det: gpu run 3 segments")
    g.run(3)
    for w in range(4):
        _compare_trace(o, g, w, w, cap)
    _compare_state(o, g)


def test_det_c1_long_run_bit_exact():
    """2000 segments (2e7 moves per walker): windows 1-3 finish all eleven
    ln f stages, window 0 is still discovering its range; every ln g~, H,
    state and configuration agrees bit for bit, and so do the exchange
    counts."""
    from paper_1411_4212_amd.workloads import c1
    cfg = c1()
    o = oracle_from(cfg)
    o.run(2000)
    _say("c1 det long: gpu 2000 segments")
    g = gpu_from(cfg, "fp64_det")
    g.run(2000)
    assert g.step() == o.step_counter() == 2000
    _compare_state(o, g)
    ao, co = o.exchange_stats()
    ag, cg = g.exchange_stats(0)
    assert np.array_equal(ao, ag) and np.array_equal(co, cg)
    assert sum(o.walker(w)["done"] for w in range(4)) >= 2


@pytest.mark.parametrize("which", ["two_spins", "open_chain"])
def test_det_explicit_bit_exact(which):
    """Explicit-coupling systems (neighbour table path): converge to the end
    on both sides with identical results."""
    from paper_1411_4212_amd import workloads
    cfg = getattr(workloads, which)()
    cfg = dict(cfg, schedule=cfg["schedule"][:3] + (2.0 ** -8,) + (20000, 0))
    o = oracle_from(cfg, trace=5000)
    o.run_to_convergence(max_segments=5000)
    _say(which, "det: gpu")
    g = gpu_from(cfg, "fp64_det", trace=5000)
    g.run_to_convergence(max_segments=5000, chunk=64)
    assert o.all_done()
    h, m = cfg["windows"][3], cfg["windows"][5]
    for w in range(h * m):
        _compare_trace(o, g, w, w, 5000)
    _compare_state(o, g)
