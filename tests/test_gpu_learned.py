"""Learned proposal in the REWL walk (FP32_DE mode) through the C ABI.

The uniform proposal is the reference: a walk with the learned proposal must
reproduce the oracle's ln g, because the exact q-ratio enters the
acceptance.  Two oracle references per workload (tests/golden, written by
make_reference.py from the CPU oracle only):

* the Wang-Landau estimator's mean over many oracle runs (uniform proposal),
  with its run-to-run spread;
* for the range that reaches down towards the ordered state, ln g from a
  fixed-weight oracle run, which carries no Wang-Landau modification error:
  fixed-weight walks on the GPU are held to it at the parity bars, while a
  Wang-Landau mean (the oracle's as well) differs from it by a smooth tilt
  of a few hundredths, the estimator's own error at ln f = 2^-18; that
  difference is reported and bounded by the oracle's own Wang-Landau
  mean's distance from it plus 0.1 (that distance is about 0.18 at the
  lowest bin of the low range, a few hundredths elsewhere).

Workloads: bcc L=4, J = (1, 0.5), 2 windows x 8 walkers, on the middle of
the spectrum [-400, -100) (30 bins) and on [-550, -50) (40 bins), whose
lowest bins lie at 4.3 J per spin against the ferromagnet's 5.5.

Bars (the paper's accuracy check compares Delta with sigma over independent
runs, Sec. results and discussion): every bin within 5 combined standard
errors; |Delta| <= 0.02 on every bin whose combined standard error is at
most 0.004 (where 0.02 is five of them); the specific-heat peak within 0.5%.
"""
import json
import os
import sys

import numpy as np
import pytest

from helpers import gpu_from, wl_truth_bound, progress

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
REF = {"L4_mid": "ref_parity_L4.json", "L4_low": "ref_parity_L4_low.json"}
TRUTH = {"L4_low": "truth_L4_low.json"}


_say = progress


def _ref(name):
    return json.load(open(os.path.join(GOLD, REF[name])))


def _workload(name, seed=77):
    wl = _ref(name)["workload"]
    return dict(lattice=tuple(wl["lattice"]), windows=tuple(wl["windows"]),
                schedule=tuple(wl["schedule"]), seed=seed)


def _harvest_and_train(cfg, segments_skip=60, segments_harvest=30, epochs=6):
    """Plain walk, harvest (x, S_i) every 4th move once ln g is roughly
    converged, train the MLP on the device."""
    from paper_1411_4212_amd import learned
    g = gpu_from([cfg] * 4, "fp32_de")
    g.run(segments_skip)
    seg = cfg["schedule"][4]
    g.set_harvest(segments_harvest * seg // 4 + 1, 4)
    g.run(segments_harvest)
    recs = g.harvested()
    params = learned.init_params(3, recs.device)
    losses = learned.train(recs, params, epochs=epochs, batch=4096, lr=2e-3, seed=5)
    _say("records", recs.shape[0], "loss", losses)
    return params, recs


def _wl_runs(cfg, runs, params=None, tag=""):
    """`runs` independent instances to convergence; per run the joined,
    normalised ln g, and the acceptance of every walker."""
    from oracle.analysis import combine_walkers, join_windows, normalise
    g = gpu_from([cfg] * runs, "fp32_de")
    if params is not None:
        g.set_proposal(params)
    seg = 0
    while seg < 20000:
        g.run(64)
        seg += 64
        done = g.poll()
        if seg % 256 == 0 or done:
            _say("%s: %d segments%s" % (tag, seg, " (all done)" if done else ""))
        if done:
            break
    assert g.poll()
    h, m = cfg["windows"][3], cfg["windows"][5]
    out, acc = [], []
    for inst in range(runs):
        frags = []
        for k in range(h):
            ws = range(k * m, (k + 1) * m)
            lo, hi = g.window(inst, k * m)
            lg, vis = combine_walkers([g.lng(inst, w) for w in ws], [g.visited(inst, w) for w in ws])
            frags.append((lo, hi, lg, vis))
        _, lg, _ = join_windows(frags)
        out.append(normalise(lg))
        for w in range(h * m):
            st = g.walker(inst, w)
            acc.append(st["accepts"] / st["attempts"])
    return np.array(out), float(np.mean(acc))


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
    tg, tr = cv_peak(Ec[ok], dg[ok], 1.0, 8.0)[0], cv_peak(Ec[ok], dr[ok], 1.0, 8.0)[0]
    _say("%s: C_V peak %.4f vs %.4f" % (tag, tg, tr))
    assert abs(tg - tr) / tr <= 0.005
    return np.nanmax(np.abs(delta[ok]))


def test_harvest_records():
    """Records: one every k-th move, unit spins, |h / h_s| <= 1, and the
    window feature e_w = centre energy / (N h_s / 2) of the walker's window."""
    cfg = _workload("L4_mid")
    g = gpu_from(cfg, "fp32_de")
    g.set_harvest(60000, 10)
    g.run(2)
    from paper_1411_4212_amd.rewl import rewl_read_harvest_counts
    counts = rewl_read_harvest_counts(g.ctx, g.n_walkers)
    seg = cfg["schedule"][4]
    assert np.all(counts == 2 * seg // 10)
    recs = g.harvest_buf.view(g.n_walkers, 60000, 8).cpu().numpy()
    Emin, Emax, B, h, o, m = cfg["windows"]
    hs = 8 * 1.0 + 6 * 0.5
    N = 128
    for w in range(g.n_walkers):
        r = recs[w, :counts[w]]
        assert np.allclose(np.linalg.norm(r[:, 4:7], axis=1), 1.0, atol=1e-5)
        assert np.all(np.linalg.norm(r[:, :3], axis=1) <= 1.0 + 1e-5)
        lo, hi = g.window(0, w)
        ec = Emin + 0.5 * (lo + hi) * (Emax - Emin) / B
        assert np.allclose(r[:, 3], ec / (N * hs / 2), rtol=1e-6)


@pytest.mark.parametrize("name", ["L4_mid", "L4_low"])
def test_learned_walk_statistical_parity(name):
    """Train on records of the plain walk, then run 256 independent learned
    walks: on the middle range their mean normalised ln g matches the
    oracle's Wang-Landau mean within the bars above.  On the low range the
    Wang-Landau estimator's own error at the final ln f (the oracle's mean
    lies 0.18 from the fixed-weight ln g at the lowest bin) depends on the
    walk's dynamics, which the proposal changes, so two Wang-Landau means
    need not agree there within their spreads: the learned mean is held to
    the fixed-weight ln g within the oracle's own distance plus 0.1, and the
    proposal's parity on that range is the fixed-weight test below;
    the learned proposal accepts more often than the uniform one, both
    measured over whole runs to convergence on the same schedule (uniform
    walks on these ranges are held to the parity bars in
    test_gpu_statistical)."""
    ref = _ref(name)
    cfg = _workload(name)
    params, _ = _harvest_and_train(cfg)
    A, acc_l = _wl_runs(cfg, 256, params, "learned " + name)
    _, acc_u = _wl_runs(cfg, 32, None, "uniform " + name)
    mean_r = np.array(ref["mean_lng"])
    se_r = np.array(ref["std_lng"]) / np.sqrt(ref["runs"])
    mean_g = np.nanmean(A, axis=0)
    se_g = np.nanstd(A, axis=0, ddof=1) / np.sqrt(np.isfinite(A).sum(0))
    if name not in TRUTH:
        _check("%s learned vs oracle WL" % name, cfg, mean_g, se_g, mean_r, se_r)
    else:
        t = json.load(open(os.path.join(GOLD, TRUTH[name])))
        _check("%s learned vs truth" % name, cfg, mean_g, se_g, np.array(t["lng"]), np.array(t["se"]),
               loose=wl_truth_bound(mean_r, t["lng"]))
    _say("acceptance learned %.3f uniform %.3f (same schedule, to convergence)" % (acc_l, acc_u))
    assert acc_l > acc_u


def _fixed_weight_lng(cfg, W, params, R, segments):
    """ln g from fixed-weight walks of R instances (ln f = 1e-300, flatness
    1: the weights never change, H only accumulates): per instance and
    window, W + ln H over the walkers' summed histogram, windows joined by
    the mean offset over shared bins."""
    from oracle.analysis import normalise
    fixed = dict(cfg, schedule=(1, 1, 1e-300, 1e-300, cfg["schedule"][4], cfg["schedule"][5]))
    h, m, B = cfg["windows"][3], cfg["windows"][5], cfg["windows"][2]
    g = gpu_from([fixed] * R, "fp32_de")
    for i in range(R):
        for w in range(h * m):
            lo, hi = g.window(i, w)
            g.write_lng(i, w, W[lo:hi])
    if params is not None:
        g.set_proposal(params)
    # burn-in (the walkers enter their windows from above), then count
    g.run(20)
    H0 = [[g.hist(i, w).astype(np.float64) for w in range(h * m)] for i in range(R)]
    done = 0
    while done < segments:
        n = min(20, segments - done)
        g.run(n)
        g.poll()
        done += n
        _say("fixed weight: %d of %d segments" % (done, segments))
    out = []
    for i in range(R):
        acc = np.zeros(B)
        cnt = np.zeros(B)
        for k in range(h):
            lo, hi = g.window(i, k * m)
            Hs = sum(g.hist(i, w).astype(np.float64) - H0[i][w] for w in range(k * m, (k + 1) * m))
            lg = np.where(Hs > 0, W[lo:hi] + np.log(np.maximum(Hs, 1.0)), np.nan)
            idx = np.arange(lo, hi)
            have = cnt[idx] > 0
            okk = np.isfinite(lg)
            both = have & okk
            off = np.mean(acc[idx][both] / cnt[idx][both] - lg[both]) if both.any() else 0.0
            acc[idx[okk]] += lg[okk] + off
            cnt[idx[okk]] += 1
        est = np.full(B, np.nan)
        est[cnt > 0] = acc[cnt > 0] / cnt[cnt > 0]
        out.append(normalise(est))
    return np.array(out)


def test_learned_fixed_weight_walk_matches_truth():
    """Fixed-weight (multicanonical) walks on the low range with the oracle
    truth's weights: the stationary histogram gives ln g = ln g~ + ln H with
    no Wang-Landau modification error, so this isolates the Markov kernel.
    Both the learned and the uniform proposal must reproduce the oracle's
    fixed-weight ln g within 5 standard errors per bin (and 0.02 where the
    errors allow)."""
    t = json.load(open(os.path.join(GOLD, TRUTH["L4_low"])))
    W = np.array(t["weights"])
    cfg = _workload("L4_low")
    params, _ = _harvest_and_train(cfg, segments_skip=40, segments_harvest=10, epochs=3)
    R = 32
    for kind, p in (("uniform", None), ("learned", params)):
        X = _fixed_weight_lng(cfg, W, p, R, 60)
        mean_g = np.nanmean(X, axis=0)
        se_g = np.nanstd(X, axis=0, ddof=1) / np.sqrt(np.isfinite(X).sum(0))
        _check("fixed-weight %s vs truth" % kind, cfg, mean_g, se_g, np.array(t["lng"]),
               np.array(t["se"]))


def test_learned_fixed_weight_walk_unbiased():
    """Fixed-weight walk on the middle range: every walker's ln g~ is set to
    the oracle's reference ln g (ln f = 1e-300, flatness fraction 1, so the
    weights never change and H is never reset); the stationary histogram is
    then H(E) ~ g(E) / g~(E).  The residual ln H of walks with the learned
    proposal (any q, through the exact q-ratio) must equal that of the
    uniform proposal bin by bin: z <= 5 from the spread over 32 independent
    instances, and |mean difference| <= 0.03."""
    ref = _ref("L4_mid")
    mean_r = np.array(ref["mean_lng"])
    cfg = _workload("L4_mid")
    params, _ = _harvest_and_train(cfg, segments_skip=40, segments_harvest=10, epochs=3)
    fixed = dict(cfg, schedule=(1, 1, 1e-300, 1e-300, cfg["schedule"][4], cfg["schedule"][5]))
    R = 32
    h, m = cfg["windows"][3], cfg["windows"][5]
    res = {}
    for kind in ("plain", "learned"):
        g = gpu_from([fixed] * R, "fp32_de")
        for i in range(R):
            for w in range(h * m):
                lo, hi = g.window(i, w)
                g.write_lng(i, w, mean_r[lo:hi])
        if kind == "learned":
            g.set_proposal(params)
        g.run(30)
        per = []
        for i in range(R):
            row = []
            for k in range(h):
                Hs = sum(g.hist(i, w).astype(np.float64) for w in range(k * m, (k + 1) * m))
                lh = np.log(np.maximum(Hs, 1.0))
                row.append(lh - lh.mean())
            per.append(np.concatenate(row))
        res[kind] = np.array(per)
        _say(kind, "residual ln H range %.3f" % (res[kind].mean(0).max() - res[kind].mean(0).min()))
    a, b = res["plain"], res["learned"]
    d = b.mean(0) - a.mean(0)
    se = np.sqrt(a.var(0, ddof=1) / R + b.var(0, ddof=1) / R)
    z = np.abs(d) / np.maximum(se, 1e-12)
    np.set_printoptions(precision=3, suppress=True, linewidth=200)
    _say("diff", d)
    _say("z   ", z)
    assert z.max() <= 5.0
    assert np.abs(d).max() <= 0.03
