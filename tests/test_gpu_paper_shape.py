"""The paper's largest run in shape on the GPU (Sec. results: L = 40, 893
windows at overlap 0.75, one walker each; bcc with couplings J = (1, 0.5),
128,000 spins, configurations in HBM, ferromagnetic start).

After two segments of the look-ahead kernel, for every walker:
  * each window's bin range is the one the oracle's window placement gives
    for this bin count, window count and overlap;
  * the running energy equals the oracle's full FP64 energy of the
    configuration the walker holds (to the FP32 energy-change bound);
  * the current bin lies in the walker's window and every spin is a unit
    vector; the configurations are a permutation of the walkers;
and the same walk in one persistent launch is bit-identical."""
import numpy as np
import pytest

from helpers import bits, progress

pytestmark = pytest.mark.gpu
_say = progress


def test_paper_shape_L40_energies_windows_and_persistent():
    import oracle
    from paper_1411_4212_amd.rewl import Run
    from paper_1411_4212_amd import workloads
    wl = workloads.paper_l40()
    Emin, Emax, B, h, ov, m = wl["windows"]
    assert (h, m) == (893, 1)
    L, J = wl["lattice"][1], wl["lattice"][2]
    W = h * m

    def build():
        r = Run([dict(lattice=wl["lattice"], windows=wl["windows"], schedule=wl["schedule"])], mode="fp32_de")
        r.init(wl["seed"], workloads.init_spins(wl))
        return r

    _say("L=40 paper shape: %d walkers, %d bins, %d spins" % (W, B, 2 * L ** 3))
    g = build()
    g.run(2)
    _say("L=40: two segments done (per-segment launches)")
    p = build()
    grid = p.run_persistent(2)
    _say("L=40: two rounds done (persistent, grid %d)" % grid)
    o = oracle.Oracle(L=L, J=J)
    seg = wl["schedule"][4]
    configs = []
    worst = 0.0
    for w in range(W):
        st = g.walker(0, w)
        configs.append(st["config"])
        assert st == p.walker(0, w), w
        lo, hi = g.window(0, w)
        assert (lo, hi) == oracle.window_bins(B, h, ov, w // m), w
        assert lo <= st["bin"] < hi
        assert st["attempts"] == 2 * seg or st["done"]
        S = g.config(0, st["config"])
        assert np.allclose(np.linalg.norm(S, axis=1), 1.0, atol=1e-5)
        assert np.array_equal(bits(S), bits(p.config(0, st["config"])))
        Ef = o.energy(S)
        assert abs(Ef - st["E"]) <= 2e-2 * (1 + abs(Ef)) ** 0.5, (w, Ef, st["E"])
        worst = max(worst, abs(Ef - st["E"]))
        assert np.array_equal(bits(g.lng(0, w)), bits(p.lng(0, w)))
        if w % 128 == 0 or w == W - 1:
            _say("walker %3d window (%d, %d) bin %d E %.4f full %.4f" % (w, lo, hi, st["bin"], st["E"], Ef))
    assert sorted(configs) == list(range(W))
    _say("L=40: max |E - full energy| over %d walkers %.2e" % (W, worst))
    g.close()
    p.close()
