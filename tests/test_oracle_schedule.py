"""Pins of the oracle's Wang-Landau schedule (Sec. original WL algorithm: the
histogram update, the flatness test, the halving of ln f and the stopping rule).

The oracle is stepped one segment at a time with a full per-attempt trace.
Each check is an invariant of the method rather than a second copy of the
oracle's code:

- every attempt adds exactly one count to H at the walker's bin after the
  move, accepted or not, so H at the end of a segment is H at its start plus
  the histogram of the traced bins;
- a flat histogram halves ln f exactly and empties H; a walker finishes on the
  flat histogram of an iteration run at ln f <= ln f_final and then keeps its
  ln g and H;
- flat means min H >= p <H> over the visited bins (the paper's definition, in
  real arithmetic, against the oracle's integer form): no advance is missed
  and none is taken early; a segment that visits a new bin is not flat;
- p = 0 makes every segment without a new bin flat.
"""
import math

import numpy as np

CHAIN = (4, [0, 1, 2], [1, 2, 3], [1.0, 1.0, 1.0])   # open chain, E in [-3, 3]


def _stepper(oracle_mod, flat_num, flat_den, lnf_final, segments, seg=1000, B=36, h=3, m=2,
             seed=5):
    # the range reaches past the chain's |E| <= 3, so the outer bins of the
    # end windows are never visited: flatness must ignore them
    o = oracle_mod.Oracle(explicit=CHAIN)
    o.set_windows(-3.6, 3.6, B, h, 0.75, m)
    o.set_schedule(flat_num, flat_den, 1.0, lnf_final, seg, 0)
    o.set_threads(1)
    o.set_trace(segments * seg)
    o.init(seed)
    snaps = []

    def snap():
        out = []
        for w in range(o.W):
            H, vis = o.hist(w)
            out.append(dict(st=o.walker(w), H=H.astype(np.int64), vis=vis, lng=o.lng(w).copy(),
                            lo=o.window(w)[0]))
        return out

    snaps.append(snap())
    for _ in range(segments):
        o.run(1)
        snaps.append(snap())
    traces = [o.trace(w) for w in range(o.W)]
    return o, snaps, traces, seg


def _segment_bins(trace, a0, a1, lo, nb):
    rec = trace[a0:a1]
    assert len(rec) == a1 - a0
    assert np.array_equal(rec["attempt_lo"], np.arange(a0, a1, dtype=np.uint64).astype(np.uint32))
    return np.bincount(rec["bin"] - lo, minlength=nb)


def _flat_by_definition(H, vis, p):
    Hv = H[vis].astype(np.float64)
    return vis.any() and Hv.sum() > 0 and Hv.min() >= p * Hv.mean()


def test_histogram_flatness_and_lnf_schedule(oracle_mod):
    p = 0.8
    o, snaps, traces, seg = _stepper(oracle_mod, 4, 5, 2.0 ** -5, segments=240)
    advances = finishes = quiet = 0
    for s in range(len(snaps) - 1):
        for w in range(o.W):
            a, b = snaps[s][w], snaps[s + 1][w]
            sa, sb = a["st"], b["st"]
            nb = len(a["H"])
            if sa["done"]:
                # a finished walker keeps its ln g and H
                assert sb["done"]
                assert np.array_equal(a["lng"].view(np.uint64), b["lng"].view(np.uint64))
                assert np.array_equal(a["H"], b["H"])
                continue
            assert sb["attempts"] - sa["attempts"] == seg
            counts = _segment_bins(traces[w], sa["attempts"], sb["attempts"], a["lo"], nb)
            new_bins = bool((b["vis"] & ~a["vis"]).any())
            assert not (a["vis"] & ~b["vis"]).any()          # visited only grows
            assert b["vis"][counts > 0].all()                 # every traced bin is visited
            if sb["iter"] == sa["iter"] + 1:
                # flat: ln f halves exactly, H empties, and the histogram the
                # segment ended with was flat by the definition
                advances += 1
                assert not new_bins
                assert sb["lnf"] == sa["lnf"] / 2 and not sb["done"]
                assert not b["H"].any()
                if sa["iter"] >= 1:
                    assert _flat_by_definition(a["H"] + counts, b["vis"], p)
            elif sb["done"]:
                finishes += 1
                assert sb["iter"] == sa["iter"] and sa["lnf"] <= 2.0 ** -5
                assert sb["lnf"] == sa["lnf"] and not new_bins
                assert np.array_equal(b["H"], a["H"] + counts)
                assert _flat_by_definition(b["H"], b["vis"], p)
            else:
                assert sb["iter"] == sa["iter"] and sb["lnf"] == sa["lnf"]
                if sa["iter"] >= 1:
                    # range fixed after iteration 0: plain accumulation, and no
                    # flat histogram was passed over
                    quiet += 1
                    assert not new_bins
                    assert np.array_equal(b["H"], a["H"] + counts)
                    assert not _flat_by_definition(b["H"], b["vis"], p)
    # the schedule actually ran through its steps, with bins left unvisited
    assert advances >= o.W * 3 and finishes >= 1 and quiet > 0
    assert any(not d["vis"].all() for d in snaps[-1])


def test_lnf_equals_initial_halved_per_iteration(oracle_mod):
    o, snaps, _, _ = _stepper(oracle_mod, 4, 5, 2.0 ** -5, segments=120)
    for sn in snaps:
        for d in sn:
            st = d["st"]
            assert st["lnf"] == 2.0 ** -st["iter"]
            assert st["iter"] <= 5


def test_p_zero_every_segment_without_new_bins_is_flat(oracle_mod):
    """flat_num = 0 (p = 0): min H >= 0 always holds, so a segment advances
    exactly when it found no new bin; with ln f_final = 2^-3 a walker is done
    after four such segments: iterations 0-2 halve ln f down to 2^-3, and the
    flat histogram of iteration 3 (run at ln f = 2^-3) finishes it."""
    o, snaps, traces, seg = _stepper(oracle_mod, 0, 5, 2.0 ** -3, segments=40)
    for w in range(o.W):
        quiet_segments = 0
        for s in range(len(snaps) - 1):
            a, b = snaps[s][w], snaps[s + 1][w]
            if a["st"]["done"]:
                break
            new_bins = bool((b["vis"] & ~a["vis"]).any())
            if new_bins:
                assert b["st"]["iter"] == a["st"]["iter"] and not b["st"]["done"]
            else:
                quiet_segments += 1
                assert b["st"]["iter"] == a["st"]["iter"] + 1 or b["st"]["done"]
        assert snaps[-1][w]["st"]["done"]
        assert quiet_segments == 4
        assert snaps[-1][w]["st"]["iter"] == 3


def test_exchange_step_against_its_definition(oracle_mod):
    """Replica exchange (Sec. parallel scheme), one walker per window so the
    pairing is fixed: a step of parity t pairs windows (k, k+1) with
    k = t mod 2.  A pair may swap only when each walker's bin lies in the other
    window and was visited there; it swaps with probability
    min(1, g_i(E_X) g_j(E_Y) / (g_i(E_Y) g_j(E_X))); a swap exchanges the
    configuration, E and bin exactly and leaves every ln g and H alone.
    Certain swaps (ratio >= 1) must happen, impossible ones must not, and the
    others must happen at the predicted rate (binomial, 4 sigma)."""
    N = 12
    o = oracle_mod.Oracle(explicit=(N, list(range(N - 1)), list(range(1, N)), [1.0] * (N - 1)))
    o.set_windows(-11.0, 11.0, 120, 3, 0.75, 1)
    # short segments and no flatness bar (p = 0): the first iteration ends at
    # the first segment that finds no new bin, before a walker has seen its
    # whole window, so pairs whose bins lie in the other window but were
    # never visited there occur
    o.set_schedule(0, 10, 1.0, 2.0 ** -30, 10, 0)
    o.set_threads(1)
    o.init(11)
    wins = [o.window(w) for w in range(3)]
    certain = impossible = unvisited = 0
    p_sum = p_var = swaps = 0.0
    n_prob = 0
    for _ in range(3000):
        o.run(1)
        t = o.step_counter()
        pre = [o.walker(w) for w in range(3)]
        lng = [o.lng(w).copy() for w in range(3)]
        hist = [o.hist(w) for w in range(3)]
        att0, acc0 = o.exchange_stats()
        o.exchange()
        post = [o.walker(w) for w in range(3)]
        att1, acc1 = o.exchange_stats()
        for w in range(3):
            assert np.array_equal(o.lng(w).view(np.uint64), lng[w].view(np.uint64))
            assert np.array_equal(o.hist(w)[0], hist[w][0])
        i = t % 2
        j = i + 1
        rest = [w for w in range(3) if w not in (i, j)]
        for w in rest:
            assert (post[w]["cfg"], post[w]["E"], post[w]["bin"]) == (pre[w]["cfg"], pre[w]["E"], pre[w]["bin"])
        swapped = post[i]["cfg"] == pre[j]["cfg"]
        key = lambda s: (s["cfg"], s["E"], s["bin"])
        if swapped:
            assert key(post[i]) == key(pre[j]) and key(post[j]) == key(pre[i])
        else:
            assert key(post[i]) == key(pre[i]) and key(post[j]) == key(pre[j])
        assert att1[i] == att0[i] + 1 and acc1[i] == acc0[i] + int(swapped)
        (li, hi_), (lj, hj) = wins[i], wins[j]
        a, b = pre[i]["bin"], pre[j]["bin"]
        in_range = lj <= a < hj and li <= b < hi_
        feasible = in_range and hist[j][1][a - lj] and hist[i][1][b - li]
        unvisited += in_range and not feasible
        if not feasible:
            impossible += 1
            assert not swapped
            continue
        lnP = (lng[i][a - li] - lng[i][b - li]) + (lng[j][b - lj] - lng[j][a - lj])
        if lnP >= 0:
            certain += 1
            assert swapped
        else:
            p = math.exp(lnP)
            n_prob += 1
            p_sum += p
            p_var += p * (1 - p)
            swaps += swapped
    assert certain > 50 and impossible > 100 and unvisited > 100 and n_prob > 200
    assert abs(swaps - p_sum) <= 4 * math.sqrt(p_var) + 1
