"""Statistical parity of the fast GPU modes with the FP64 oracle.

Reference: tests/golden/ref_parity_L4.json, written by
tests/golden/make_reference.py from many independent oracle runs of one
small workload.  Here the same workload runs as many independent instances
in one GPU context (distinct Philox streams), and the mean normalised
joined ln g is compared with the oracle's mean:
  * max |Delta ln g| <= 0.02 over all bins (each mean normalised to zero);
  * every bin's Delta within 5 standard errors of the two means (the
    paper's Delta-versus-sigma accuracy check over independent runs);
  * the specific-heat peak temperature of the two means within 0.5%.
"""
import json
import os
import sys

import numpy as np
import pytest

from helpers import gpu_from

pytestmark = pytest.mark.gpu
REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ref_parity_L4.json")
RUNS = 256


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode", ["fp32_de", "fp64"])
def test_statistical_parity_L4(mode):
    from oracle.analysis import combine_walkers, cv_peak, join_windows, normalise
    ref = json.load(open(REF))
    wl = ref["workload"]
    cfg = dict(lattice=tuple(wl["lattice"]), windows=tuple(wl["windows"]),
               schedule=tuple(wl["schedule"]), seed=77)
    _say("statistical parity", mode, RUNS, "instances")
    g = gpu_from([cfg] * RUNS, mode)
    g.run_to_convergence(max_segments=20000, chunk=64)
    assert g.poll()
    h, m = cfg["windows"][3], cfg["windows"][5]
    runs = []
    for inst in range(RUNS):
        frags = []
        for k in range(h):
            ws = range(k * m, (k + 1) * m)
            lo, hi = g.window(inst, k * m)
            lg, vis = combine_walkers([g.lng(inst, w) for w in ws], [g.visited(inst, w) for w in ws])
            frags.append((lo, hi, lg, vis))
        _, lg, _ = join_windows(frags)
        runs.append(normalise(lg))
    A = np.array(runs)
    mean_g = np.nanmean(A, axis=0)
    mean_r = np.array(ref["mean_lng"])
    ok = np.isfinite(mean_g) & np.isfinite(mean_r)
    assert ok.sum() >= 0.9 * len(mean_r)
    dg = normalise(mean_g, ok)
    dr = normalise(mean_r, ok)
    delta = dg - dr
    se = np.sqrt(np.nanstd(A, axis=0, ddof=1) ** 2 / RUNS + np.array(ref["std_lng"]) ** 2 / ref["runs"])
    z = np.abs(delta[ok]) / se[ok]
    np.set_printoptions(precision=3, suppress=True, linewidth=200)
    _say("delta", delta[ok])
    _say("z    ", z)
    _say("se   ", se[ok])
    _say("max|delta| %.4f  max z %.2f" % (np.nanmax(np.abs(delta[ok])), z.max()))
    assert np.nanmax(np.abs(delta[ok])) <= 0.02
    assert z.max() <= 5.0
    Emin, Emax, B = cfg["windows"][:3]
    Ec = Emin + (np.arange(B) + 0.5) * (Emax - Emin) / B
    tg = cv_peak(Ec[ok], dg[ok], 1.0, 8.0)[0]
    tr = cv_peak(Ec[ok], dr[ok], 1.0, 8.0)[0]
    _say("C_V peak gpu %.4f oracle %.4f" % (tg, tr))
    assert abs(tg - tr) / tr <= 0.005
