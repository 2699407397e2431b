"""Input recipes (paper_1411_4212_amd/workloads.py): sizes and bin widths
of the named workloads stay within the library's documented limits and
follow the readings they state."""
import math

import pytest


def _per_window(c):
    Emin, Emax, B, h, o, m = c["windows"]
    return int(math.floor(B / (1 + (h - 1) * (1 - o)) + 0.5))


@pytest.mark.parametrize("name", ["c1", "c2", "c2_l6", "c4", "c5", "paper_l40"])
def test_workload_limits(name):
    from paper_1411_4212_amd import workloads
    c = getattr(workloads, name)()
    Emin, Emax, B, h, o, m = c["windows"]
    assert Emin < Emax and B >= h and 1 <= m <= 64
    assert _per_window(c) <= 4096
    assert len(c["lattice"][2]) <= 8


def test_bin_widths():
    from paper_1411_4212_amd import workloads as W
    width = lambda c: (c["windows"][1] - c["windows"][0]) / c["windows"][2]
    assert abs(width(W.c2()) - 2.22) < 0.01
    assert abs(width(W.c2_l6()) - 2.22) < 0.01
    assert abs(width(W.c4()) - 3.0) < 0.01
    assert abs(width(W.c5()) - 4.0) < 0.01
    assert _per_window(W.c1()) == 100
    assert _per_window(W.paper_l40()) == 100 and W.paper_l40()["windows"][3] == 893


def test_paper_cut_fractions():
    """E_min = E_lo + span/28 and E_max = E_lo + 5 span/7 of the quench span."""
    from paper_1411_4212_amd import workloads as W
    lo, hi = W.KNOWN_SPANS_L8[tuple(W.J_C2)]
    Emin, Emax = W.paper_cut(8, W.J_C2)
    span = hi - lo
    assert abs(Emin - (lo + span / 28)) < 1e-9 and abs(Emax - (lo + 5 * span / 7)) < 1e-9
    # extensive scaling to other sizes
    Emin6, Emax6 = W.paper_cut(6, W.J_C2)
    assert abs(Emin6 / (2 * 6 ** 3) - Emin / 1024) < 1e-12


def test_weak_scaling_layout():
    """Fixed window width and overlap, windows growing with the lattice (Sec.
    results): the width taken from the L = 40 range and 893 windows gives 893
    windows at L = 40 and the paper's 11 at L = 10; every layout covers the
    paper's cut of its range, with 100 bins per window."""
    from paper_1411_4212_amd import weak_scaling as ws
    from paper_1411_4212_amd import workloads as W
    assert ws.layout(10)["h"] == 11
    assert ws.layout(40)["h"] == 893
    prev = 0
    for L in (10, 20, 30, 40, 50):
        lay = ws.layout(L)
        lo, hi = W.paper_cut(L, list(ws.J_PAPER_SHAPE))
        assert lay["E_min"] == lo and lay["E_max"] >= hi - 1e-6
        # one window fewer would not cover the range
        W_ = lay["width"]
        assert W_ * (1 + (lay["h"] - 2) * (1 - ws.OVERLAP)) < hi - lo
        assert lay["bins"] == round(100 * (1 + (lay["h"] - 1) * (1 - ws.OVERLAP)))
        assert lay["h"] > prev
        prev = lay["h"]
    # the L = 40 layout is the paper-shaped workload's
    c = W.paper_l40()
    lay = ws.layout(40)
    assert (lay["bins"], lay["h"]) == (c["windows"][2], c["windows"][3])
    assert abs(lay["E_max"] - c["windows"][1]) < 1e-6 * abs(c["windows"][1] - c["windows"][0])
    s = ws.layout(10, serial=True)
    assert (s["h"], s["bins"]) == (1, 350)


def test_scan_workload_for_convergence_runs():
    """converge's scan_L<n> workload is the weak-scaling layout at 3 J bins:
    the same windows (893 at L = 40), about 3 J per bin, one walker per
    window, the ferromagnetic start; named workloads pass through."""
    from paper_1411_4212_amd import weak_scaling as ws
    from paper_1411_4212_amd import workloads as W
    from paper_1411_4212_amd.converge import workload_config
    c = workload_config("scan_L40")
    lay = ws.layout(40, bin_width=3)
    Emin, Emax, B, h, o, m = c["windows"]
    assert (h, m, o) == (893, 1, ws.OVERLAP) and B == lay["bins"]
    assert (Emin, Emax) == (lay["E_min"], lay["E_max"])
    assert abs((Emax - Emin) / B - 3.0) < 0.05
    assert c["lattice"] == ("bcc", 40, [1.0, 0.5]) and c["init"] == "ferro"
    assert W.init_spins(c).shape == (2 * 40 ** 3, 3)
    assert c["schedule"][3] == 2.0 ** -20
    assert workload_config("c4") == W.c4()


def test_weak_scaling_summary():
    """Quantiles count an unfinished window as infinitely slow; the tenths
    split the window index range evenly."""
    from paper_1411_4212_amd.weak_scaling import summarize
    first = [None, None, 300, 100, 200, 400, 500, 600, 700, 800]
    s = summarize(first)
    assert s["finished"] == 8 and s["walkers"] == 10
    q = s["moves_quantiles"]
    # sorted: 100 .. 800, inf, inf; qX is the ceil(X % of 10)-th smallest
    assert q["q10"] == 100 and q["q50"] == 500 and q["q75"] == 800
    assert q["q100"] is None
    assert s["finished_per_tenth"] == [0, 0, 1, 1, 1, 1, 1, 1, 1, 1]
    assert s["median_of_finished"] == 450
    s = summarize([None] * 3)
    assert s["finished"] == 0 and s["moves_quantiles"]["q5"] is None and s["median_of_finished"] is None
    assert summarize([5])["moves_quantiles"]["q100"] == 5
