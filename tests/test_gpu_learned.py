"""Learned proposal in the REWL walk (FP32_DE mode) through the C ABI.

The uniform proposal is the reference: a walk with the learned proposal must
reproduce the oracle's (uniform-proposal) ln g within the same statistical
bounds, because the exact q-ratio enters the acceptance."""
import json
import os
import sys

import numpy as np
import pytest

from helpers import gpu_from

pytestmark = pytest.mark.gpu
REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ref_parity_L4.json")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _workload(seed=77):
    wl = json.load(open(REF))["workload"]
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


def test_harvest_records():
    """Records: one every k-th move, unit spins, |h / h_s| <= 1, and the
    window feature e_w = centre energy / (N h_s / 2) of the walker's window."""
    cfg = _workload()
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


def test_learned_walk_statistical_parity_and_gain():
    """Train on records of the plain walk, then run 128 independent learned
    walks: their mean normalised ln g matches the oracle reference within
    0.02 and 5 standard errors per bin, the specific-heat peak within 0.5%,
    and the acceptance rate exceeds the uniform proposal's."""
    from oracle.analysis import combine_walkers, cv_peak, join_windows, normalise
    ref = json.load(open(REF))
    cfg = _workload()
    params, _ = _harvest_and_train(cfg)
    RUNS = 256
    g = gpu_from([cfg] * RUNS, "fp32_de")
    g.set_proposal(params)
    g.run_to_convergence(max_segments=20000, chunk=64)
    assert g.poll()
    h, m = cfg["windows"][3], cfg["windows"][5]
    runs = []
    acc_l = []
    for inst in range(RUNS):
        frags = []
        for k in range(h):
            ws = range(k * m, (k + 1) * m)
            lo, hi = g.window(inst, k * m)
            lg, vis = combine_walkers([g.lng(inst, w) for w in ws], [g.visited(inst, w) for w in ws])
            frags.append((lo, hi, lg, vis))
        _, lg, _ = join_windows(frags)
        runs.append(normalise(lg))
        for w in range(h * m):
            st = g.walker(inst, w)
            acc_l.append(st["accepts"] / st["attempts"])
    A = np.array(runs)
    mean_g = np.nanmean(A, axis=0)
    mean_r = np.array(ref["mean_lng"])
    ok = np.isfinite(mean_g) & np.isfinite(mean_r)
    dg, dr = normalise(mean_g, ok), normalise(mean_r, ok)
    delta = dg - dr
    se = np.sqrt(np.nanstd(A, axis=0, ddof=1) ** 2 / RUNS + np.array(ref["std_lng"]) ** 2 / ref["runs"])
    z = np.abs(delta[ok]) / se[ok]
    np.set_printoptions(precision=3, suppress=True, linewidth=200)
    _say("delta", delta[ok])
    _say("z    ", z)
    _say("se   ", se[ok])
    _say("learned: max|delta| %.4f max z %.2f" % (np.nanmax(np.abs(delta[ok])), z.max()))
    assert np.nanmax(np.abs(delta[ok])) <= 0.02
    assert z.max() <= 5.0
    Emin, Emax, B = cfg["windows"][:3]
    Ec = Emin + (np.arange(B) + 0.5) * (Emax - Emin) / B
    tg, tr = cv_peak(Ec[ok], dg[ok], 1.0, 8.0)[0], cv_peak(Ec[ok], dr[ok], 1.0, 8.0)[0]
    _say("C_V peak learned %.4f oracle %.4f" % (tg, tr))
    assert abs(tg - tr) / tr <= 0.005
    # acceptance of the plain walk on the same workload
    p = gpu_from([cfg] * 8, "fp32_de")
    p.run(40)
    acc_p = [p.walker(i, w)["accepts"] / p.walker(i, w)["attempts"] for i in range(8) for w in range(h * m)]
    _say("acceptance learned %.3f plain %.3f" % (np.mean(acc_l), np.mean(acc_p)))
    assert np.mean(acc_l) > np.mean(acc_p)


def test_learned_fixed_weight_walk_unbiased():
    """Fixed-weight (multicanonical) walk: every walker's ln g~ is set to the
    oracle's reference ln g (ln f = 1e-300, flatness fraction 1, so the
    weights never change and H is never reset); the stationary histogram is
    then H(E) ~ g(E) / g~(E).  The residual ln H of walks with the learned
    proposal (any q, through the exact q-ratio) must equal that of the
    uniform proposal bin by bin: z <= 5 from the spread over 32 independent
    instances, and |mean difference| <= 0.03."""
    ref = json.load(open(REF))
    mean_r = np.array(ref["mean_lng"])
    cfg = _workload()
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
