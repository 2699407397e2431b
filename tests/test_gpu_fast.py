"""Fast GPU modes (FP32_DE and FP64 with the look-ahead kernel): invariants
that hold for any trajectory, checked through the C ABI."""
import sys

import numpy as np
import pytest

from helpers import gpu_from, progress

pytestmark = pytest.mark.gpu


_say = progress


@pytest.mark.parametrize("mode", ["fp32_de", "fp64"])
@pytest.mark.parametrize("which", ["c1", "c2"])
def test_fast_invariants(mode, which):
    """After 12 segments: every walker made exactly 12 x 1e4 moves, its
    running energy equals the full energy of the configuration it holds
    (FP64 oracle energy function) up to the mode's rounding drift, its bin is
    the bin of that energy and lies in its window, the configurations are a
    permutation, ln f = 2^-iteration, and visited bins carry H or ln g."""
    import oracle
    from paper_1411_4212_amd import workloads
    cfg = getattr(workloads, which)()
    _say(which, mode)
    g = gpu_from(cfg, mode)
    g.run(12)
    lat = cfg["lattice"]
    o = oracle.Oracle(L=lat[1], J=lat[2])
    Emin, Emax, B = cfg["windows"][:3]
    inv = B / (Emax - Emin)
    W = g.n_walkers
    cfgs = []
    tol = 2e-3 if mode == "fp32_de" else 1e-8
    for w in range(W):
        st = g.walker(0, w)
        assert st["attempts"] == 12 * cfg["schedule"][4]
        assert 0 < st["accepts"] < st["attempts"]
        assert st["lnf"] == 2.0 ** -st["iteration"]
        S = g.config(0, st["config"])
        assert np.allclose(np.linalg.norm(S, axis=1), 1.0, atol=1e-6 if mode == "fp32_de" else 1e-14)
        Ef = o.energy(S)
        assert abs(Ef - st["E"]) <= tol * (1 + abs(Ef)) ** 0.5 * 10, (w, Ef, st["E"])
        lo, hi = g.window(0, w)
        assert lo <= st["bin"] < hi
        assert st["bin"] == int(np.floor((st["E"] - Emin) * inv)) or abs(
            (st["E"] - Emin) * inv - round((st["E"] - Emin) * inv)) < 1e-9
        vis = g.visited(0, w)
        assert vis[st["bin"] - lo]
        assert vis.sum() == st["n_visited"]
        cfgs.append(st["config"])
    assert sorted(cfgs) == list(range(W))
    att, acc = g.exchange_stats(0)
    assert att.sum() > 0


def test_fast_matches_oracle_early_trajectory():
    """FP64 fast mode makes the same decisions as the oracle while rounding
    differences stay below the bin and acceptance resolution: the first 200
    moves of every C1 walker (same Philox streams) agree in site, accept bit
    and bin with the oracle's trajectory."""
    from helpers import oracle_from
    from paper_1411_4212_amd import workloads
    cfg = workloads.c1()
    o = oracle_from(cfg, trace=200)
    o.run(1)
    g = gpu_from(cfg, "fp64", trace=200)
    g.run(1)
    agree = 0
    for w in range(4):
        to, tg = o.trace(w), g.trace(w)
        assert np.array_equal(to["site"], tg["site"])
        same = (to["flags"] == tg["flags"]) & (to["bin"] == tg["bin"])
        k = int(np.argmin(same)) if not same.all() else len(same)
        agree += k
        assert k >= 150, (w, k)
    assert agree >= 700


@pytest.mark.parametrize("mode", ["fp32_de", "fp64"])
def test_launch_shapes_bit_identical(mode):
    """Configurations in LDS or read in place from HBM, one or four walkers
    per workgroup: the same arithmetic on the same streams, so every state,
    ln g and configuration agrees bit for bit after 6 segments."""
    from paper_1411_4212_amd import workloads
    from helpers import bits
    cfg = workloads.c2()
    runs = []
    for wpb, res in [(1, 1), (1, 2), (3, 1), (4, 2)]:
        _say("c2", mode, "wpb", wpb, "residency", res)
        g = gpu_from(cfg, mode, walkers_per_block=wpb, residency=res)
        assert g.launch()["walkers_per_block"] == wpb
        assert g.launch()["spins_in_lds"] == (res == 1)
        g.run(6)
        runs.append(g)
    ref = runs[0]
    for g in runs[1:]:
        for w in range(ref.n_walkers):
            a, b = ref.walker(0, w), g.walker(0, w)
            assert a == b, w
            assert np.array_equal(bits(ref.lng(0, w)), bits(g.lng(0, w))), w
            assert np.array_equal(ref.hist(0, w), g.hist(0, w)), w
        for c in range(0, ref.n_walkers, 17):
            assert np.array_equal(bits(ref.config(0, c)), bits(g.config(0, c))), c


def test_hbm_L32_invariants():
    """bcc L=32 (65536 spins, configurations in HBM) with the eight-shell
    couplings, a slice of 2 windows per instance start from the ferromagnet:
    two segments later every walker's running energy equals the FP64 energy
    of its configuration (oracle energy function) within FP32 drift."""
    import oracle
    from paper_1411_4212_amd import workloads
    cfg = workloads.c5()
    Emin, Emax, B, h, o, m = cfg["windows"]
    # the two lowest windows of the full layout
    wl = round(B / (1 + (h - 1) * (1 - o)))
    lo1 = round((B - wl) / (h - 1))
    de = (Emax - Emin) / B
    sub = dict(cfg, windows=(Emin, Emin + (lo1 + wl) * de, lo1 + wl, 2, o, 4))
    _say("L32 hbm")
    g = gpu_from(sub, "fp32_de")
    assert not g.launch()["spins_in_lds"]
    g.run(2)
    lat = cfg["lattice"]
    orc = oracle.Oracle(L=lat[1], J=lat[2])
    for w in range(g.n_walkers):
        st = g.walker(0, w)
        assert st["attempts"] == 2 * cfg["schedule"][4]
        S = g.config(0, st["config"])
        Ef = orc.energy(S)
        assert abs(Ef - st["E"]) < 0.05, (w, Ef, st["E"])
        lo, hi = g.window(0, w)
        assert lo <= st["bin"] < hi


@pytest.mark.parametrize("L,shells,learned", [(8, 8, False), (6, 4, False), (6, 8, False), (8, 8, True),
                                              (6, 8, True), (8, 4, True)])
def test_pass_widths_bit_identical(L, shells, learned):
    """The fast sweep decides 4 moves per pass with the configuration in LDS
    and 16 per pass when it reads it from HBM (four lanes per move, the same
    16-chain field sum).  Both forms, on four- and eight-shell lattices with
    L a power of two or not, with the uniform and the learned proposal, give
    the same walk bit for bit: states, ln g, H and configurations after 4
    segments, for FP32_DE (and FP64 with the uniform proposal)."""
    from paper_1411_4212_amd import learned as lrn, workloads
    from helpers import bits
    J = workloads.J8 if shells == 8 else workloads.J_C2
    Emin, Emax = workloads.paper_cut(L, J)
    cfg = dict(lattice=("bcc", L, list(J)), windows=(Emin, Emax, 400, 4, 0.75, 4),
               schedule=(4, 5, 1.0, 2.0 ** -20, 4000, 100 * 2 * L ** 3), seed=5)
    modes = ["fp32_de"] if learned else ["fp32_de", "fp64"]
    for mode in modes:
        runs = []
        for res in (1, 2):
            _say("pass widths", L, shells, "learned" if learned else "uniform", mode, "residency", res)
            g = gpu_from(cfg, mode, residency=res)
            assert g.launch()["spins_in_lds"] == (res == 1)
            if learned:
                import torch
                g.set_proposal(lrn.init_params(7, torch.device("cuda", 0)))
            g.run(4)
            runs.append(g)
        a, b = runs
        for w in range(a.n_walkers):
            assert a.walker(0, w) == b.walker(0, w), (mode, w)
            assert np.array_equal(bits(a.lng(0, w)), bits(b.lng(0, w))), (mode, w)
            assert np.array_equal(a.hist(0, w), b.hist(0, w)), (mode, w)
        for c in range(0, a.n_walkers, 5):
            assert np.array_equal(bits(a.config(0, c)), bits(b.config(0, c))), (mode, c)
        acc = sum(a.walker(0, w)["accepts"] for w in range(a.n_walkers))
        assert acc > 0
