"""Pins of the oracle's window sharing (the multiple-walker refinement of the
parallel scheme: walkers of a window advance together and share ln g~).

* One walker per window: sharing changes nothing (the merge of a single
  walker is that walker), so trajectories, ln g~, H and states are bit for
  bit those of the independent walkers of the paper's scheme.
* Conservation: every trial move adds the current ln f to exactly one bin of
  the walker's ln g~ (Sec. original WL), so a walker's sum over bins is the
  sum of ln f over its moves.  When all walkers of a window have visited the
  same bins, a per-bin mean over them keeps that sum (all made the same moves
  at the same ln f); this holds at every step from a start on which every bin
  counts as visited.
* After every merge the window's walkers hold the same ln g~, visited set,
  ln f and iteration count, and iterations advance together.

None of the expected values is taken from the oracle itself.
"""
import numpy as np
import pytest

from helpers import oracle_from

WL = dict(lattice=("bcc", 4, [1.0, 0.5]), windows=(-400.0, -100.0, 30, 2, 0.75, 3),
          schedule=(4, 5, 1.0, 2.0 ** -6, 5000, 12800), seed=11)


def _state(o, w):
    s = o.walker(w)
    return (s["E"], s["bin"], s["lnf"], s["iter"], s["done"], s["cfg"], s["attempts"], s["accepts"],
            s["nvis"])


def test_single_walker_windows_unchanged(oracle_mod):
    cfg = dict(WL, windows=WL["windows"][:5] + (1,))
    a = oracle_from(cfg, trace=4000)
    b = oracle_from(dict(cfg, share=True), trace=4000)
    for _ in range(6):
        a.run(25)
        b.run(25)
        for w in range(a.W):
            assert _state(a, w) == _state(b, w)
            assert np.array_equal(a.lng(w).view(np.uint64), b.lng(w).view(np.uint64))
            assert np.array_equal(a.hist(w)[0], b.hist(w)[0])
    assert max(a.walker(w)["iter"] for w in range(a.W)) >= 2
    for w in range(a.W):
        ta, tb = a.trace(w), b.trace(w)
        assert np.array_equal(ta["site"], tb["site"]) and np.array_equal(ta["flags"], tb["flags"])


def test_sum_of_lng_is_conserved_by_merges(oracle_mod):
    o = oracle_from(dict(WL, share=True))
    h, m = WL["windows"][3], WL["windows"][5]
    seg = WL["schedule"][4]
    for w in range(o.W):
        lo, hi = o.window(w)
        o.write_lng(w, np.zeros(hi - lo), np.ones(hi - lo, dtype=np.uint8))
    expect = np.zeros(o.W)
    merges = 0
    for _ in range(400):
        if o.all_done():
            break
        lnf_before = np.array([o.walker(w)["lnf"] for w in range(o.W)])
        it_before = np.array([o.walker(w)["iter"] for w in range(o.W)])
        running = np.array([not o.walker(w)["done"] for w in range(o.W)])
        o.run(1)
        # done walkers keep walking (and exchanging) without updating ln g~
        expect += np.where(running, seg * lnf_before, 0.0)
        for w in range(o.W):
            got = float(np.sum(o.lng(w)))
            assert abs(got - expect[w]) <= 1e-9 * max(1.0, expect[w]), (w, got, expect[w])
        it_after = np.array([o.walker(w)["iter"] for w in range(o.W)])
        for k in range(h):
            ws = range(k * m, (k + 1) * m)
            # iterations advance together, for the whole window at once
            assert len({int(it_after[w] - it_before[w]) for w in ws}) == 1
            if it_after[k * m] > it_before[k * m]:
                merges += 1
                ref = o.lng(k * m).view(np.uint64)
                for w in ws:
                    assert np.array_equal(o.lng(w).view(np.uint64), ref)
                    assert np.array_equal(o.hist(w)[1], o.hist(k * m)[1])
                    assert o.walker(w)["lnf"] == o.walker(k * m)["lnf"]
                    assert int(o.hist(w)[0].sum()) == 0
    assert merges >= 2 * h


def test_shared_windows_converge_together(oracle_mod):
    o = oracle_from(dict(WL, share=True))
    n = o.run_to_convergence(max_segments=3000)
    assert o.all_done(), n
    h, m = WL["windows"][3], WL["windows"][5]
    for k in range(h):
        ws = list(range(k * m, (k + 1) * m))
        ref = o.lng(ws[0]).view(np.uint64)
        for w in ws:
            s = o.walker(w)
            assert s["done"] and s["lnf"] == o.walker(ws[0])["lnf"] and s["iter"] == o.walker(ws[0])["iter"]
            assert np.array_equal(o.lng(w).view(np.uint64), ref)
