"""ln g parity with the oracle at the hot path's real shapes.

The larger workloads run the fast sweep with four neighbour slots per lane
(four shells, z = 50) and eight (eight shells, z = 112).  These tests run
those shapes on bcc L=6 (432 spins; L not a power of two, so the packed
coordinate path of the neighbour index), over 40 bins in the lower half of
the spectrum, where the oracle converges (tests/golden, written by
make_reference.py from the CPU oracle only):

* fixed-weight (multicanonical) walks with the oracle reference's weights:
  the stationary histogram gives ln g = ln g~ + ln H with no Wang-Landau
  modification error, so the GPU kernel's Markov chain is compared with the
  oracle's directly, in FP32_DE, FP64 and the persistent batched kernel
  (H counted after a burn-in of 40 segments: the walkers enter their windows
  from above, and the entry transient would weigh the top bins);
* Wang-Landau runs to ln f = 2^-16 (FP32_DE) against the oracle's
  Wang-Landau mean over 64 runs (parity bars), and against the fixed-weight
  ln g (reported; a Wang-Landau mean, the oracle's included, differs from it
  by a smooth tilt of a few hundredths at this final ln f; bounded by the
  oracle's own Wang-Landau mean's distance from it plus 0.1).

Bars: every bin within 5 combined standard errors, |Delta| <= 0.02 on every
bin whose combined standard error is at most 0.004, the specific-heat peak
within 0.5 % (Sec. results and discussion compares Delta with sigma over
independent runs).  Each test prints the FP32_DE-versus-oracle error.
"""
import json
import os
import sys

import numpy as np
import pytest

from helpers import gpu_from, wl_truth_bound, progress

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SHAPES = ["z50_L6", "z112_L6"]


_say = progress


def _truth(name):
    return json.load(open(os.path.join(GOLD, "truth_%s.json" % name)))


def _cfg(name, seed=31):
    wl = _truth(name)["workload"]
    return dict(lattice=tuple(wl["lattice"]), windows=tuple(wl["windows"]),
                schedule=tuple(wl["schedule"]), seed=seed)


def _check(tag, cfg, mean_g, se_g, mean_r, se_r, loose=None):
    from oracle.analysis import cv_peak, normalise
    ok = np.isfinite(mean_g) & np.isfinite(mean_r)
    assert ok.sum() >= 0.9 * len(mean_r)
    dg, dr = normalise(mean_g, ok), normalise(mean_r, ok)
    delta = dg - dr
    se = np.sqrt(se_g ** 2 + se_r ** 2)
    z = np.abs(delta[ok]) / se[ok]
    tight = ok & (se <= 0.004)
    np.set_printoptions(precision=3, suppress=True, linewidth=200)
    _say(tag, "delta", delta[ok])
    _say(tag, "z    ", z)
    _say("%s: max|delta| %.4f (bins with se <= 0.004: %d, max|delta| there %.4f) max z %.2f"
         % (tag, np.nanmax(np.abs(delta[ok])), tight.sum(),
            np.abs(delta[tight]).max() if tight.any() else 0.0, z.max()))
    if loose is not None:
        # a Wang-Landau mean against the fixed-weight ln g: the estimator's
        # own error at this final ln f, bounded by the oracle's Wang-Landau
        # mean's distance from the same reference plus a margin
        _say("%s: bound %.3f" % (tag, loose))
        assert np.nanmax(np.abs(delta[ok])) <= loose
        return np.nanmax(np.abs(delta[ok]))
    assert z.max() <= 5.0
    if tight.any():
        assert np.abs(delta[tight]).max() <= 0.02
    Emin, Emax, B = cfg["windows"][:3]
    Ec = Emin + (np.arange(B) + 0.5) * (Emax - Emin) / B
    tg, tr = cv_peak(Ec[ok], dg[ok], 0.3, 6.0)[0], cv_peak(Ec[ok], dr[ok], 0.3, 6.0)[0]
    _say("%s: C_V peak %.4f vs %.4f" % (tag, tg, tr))
    assert abs(tg - tr) / tr <= 0.005


def _join_offset(frags, B):
    acc = np.zeros(B)
    cnt = np.zeros(B)
    for lo, lg in frags:
        idx = np.arange(lo, lo + len(lg))
        okk = np.isfinite(lg)
        both = okk & (cnt[idx] > 0)
        off = np.mean(acc[idx][both] / cnt[idx][both] - lg[both]) if both.any() else 0.0
        acc[idx[okk]] += lg[okk] + off
        cnt[idx[okk]] += 1
    out = np.full(B, np.nan)
    out[cnt > 0] = acc[cnt > 0] / cnt[cnt > 0]
    return out


@pytest.mark.parametrize("name", SHAPES)
@pytest.mark.parametrize("form", ["fp32_de", "fp64", "persistent"])
def test_fixed_weight_chain_matches_oracle(name, form):
    from oracle.analysis import normalise
    t = _truth(name)
    W = np.array(t["weights"])
    cfg = _cfg(name)
    fixed = dict(cfg, schedule=(1, 1, 1e-300, 1e-300, cfg["schedule"][4], cfg["schedule"][5]))
    B, h, m = cfg["windows"][2], cfg["windows"][3], cfg["windows"][5]
    R, segments = 32, 160
    _say("fixed-weight", name, form, R, "instances x", segments, "segments")
    g = gpu_from([fixed] * R, "fp64" if form == "fp64" else "fp32_de")
    for i in range(R):
        for w in range(h * m):
            lo, hi = g.window(i, w)
            g.write_lng(i, w, W[lo:hi])
    burn = 40
    step = (lambda n: g.run_persistent(n)) if form == "persistent" else (lambda n: g.run(n))
    # burn-in: the walkers enter their windows from above (the random start is
    # hotter than the range); H counted from here on
    step(burn)
    H0 = [[g.hist(i, w).astype(np.float64) for w in range(h * m)] for i in range(R)]
    for _ in range(segments // 40):
        step(40)
        g.poll()
        _say("  %s: 40 segments" % form)
    assert g.step() == segments + burn
    est = []
    for i in range(R):
        frags = []
        for k in range(h):
            lo, hi = g.window(i, k * m)
            Hs = sum(g.hist(i, w).astype(np.float64) - H0[i][w] for w in range(k * m, (k + 1) * m))
            frags.append((lo, np.where(Hs > 0, W[lo:hi] + np.log(np.maximum(Hs, 1.0)), np.nan)))
        est.append(normalise(_join_offset(frags, B)))
    A = np.array(est)
    mean_g = np.nanmean(A, axis=0)
    se_g = np.nanstd(A, axis=0, ddof=1) / np.sqrt(np.isfinite(A).sum(0))
    _check("%s fixed-weight %s vs oracle" % (name, form), cfg, mean_g, se_g, np.array(t["lng"]),
           np.array(t["se"]))


@pytest.mark.parametrize("name", SHAPES)
def test_wang_landau_fp32_de_matches_oracle(name):
    """128 independent FP32_DE Wang-Landau runs to ln f = 2^-16: the mean
    normalised joined ln g against the oracle's fixed-weight ln g and, when
    present, the oracle's Wang-Landau mean."""
    from oracle.analysis import combine_walkers, join_windows, normalise
    t = _truth(name)
    cfg = _cfg(name)
    R = 128
    g = gpu_from([cfg] * R, "fp32_de")
    seg = 0
    while seg < 20000:
        g.run(64)
        seg += 64
        done = g.poll()
        if seg % 256 == 0 or done:
            _say("%s WL: %d segments%s" % (name, seg, " (all done)" if done else ""))
        if done:
            break
    assert g.poll()
    h, m = cfg["windows"][3], cfg["windows"][5]
    runs = []
    for i in range(R):
        frags = []
        for k in range(h):
            ws = range(k * m, (k + 1) * m)
            lo, hi = g.window(i, k * m)
            lg, vis = combine_walkers([g.lng(i, w) for w in ws], [g.visited(i, w) for w in ws])
            frags.append((lo, hi, lg, vis))
        _, lg, _ = join_windows(frags)
        runs.append(normalise(lg))
    A = np.array(runs)
    mean_g = np.nanmean(A, axis=0)
    se_g = np.nanstd(A, axis=0, ddof=1) / np.sqrt(np.isfinite(A).sum(0))
    r = json.load(open(os.path.join(GOLD, "ref_parity_%s.json" % name)))
    _check("%s WL fp32_de vs oracle fixed-weight" % name, cfg, mean_g, se_g, np.array(t["lng"]),
           np.array(t["se"]), loose=wl_truth_bound(r["mean_lng"], t["lng"]))
    _check("%s WL fp32_de vs oracle WL" % name, cfg, mean_g, se_g, np.array(r["mean_lng"]),
           np.array(r["std_lng"]) / np.sqrt(r["runs"]))
