"""Weak scaling of REWL on one GPU: trial moves needed to finish the first
Wang-Landau iteration as the lattice grows, the energy windows keeping a fixed
width and overlap (Sec. results, the weak-scaling figure).

The paper grows the number of windows with the system: at L = 40 its range
holds 893 windows of a fixed width at o = 0.75, so the width is the range
divided by 1 + 892 (1 - o) = 224.  `layout(L)` applies that width, taken from
the L = 40 range, to every L; that gives 11 windows at L = 10, as in the paper.
One walker per window, as there.  The quantity measured per window is the
number of trial moves a walker needs until its first flat histogram; the
parallel run's time is the slowest window's.  A serial run (one walker over
the whole range of the same bins) is the comparison, affordable only at small L.

    python -m paper_1411_4212_amd.weak_scaling --sizes 10,20,30,40 --cap 20000000
"""
import argparse
import json
import math
import sys
import time

import numpy as np

J_PAPER_SHAPE = (1.0, 0.5)        # nearest and next-nearest shells (synthetic)
L_REF, H_REF = 40, 893            # the paper's largest run
OVERLAP = 0.75
BINS_PER_WINDOW = 100


def window_width(J=J_PAPER_SHAPE):
    """Energy width of one window: the L = 40 range over 1 + (H_REF - 1)(1 - o)."""
    from .workloads import paper_cut
    lo, hi = paper_cut(L_REF, list(J))
    return (hi - lo) / (1 + (H_REF - 1) * (1 - OVERLAP))


def layout(L, J=J_PAPER_SHAPE, serial=False, bin_width=None):
    """Windows for a lattice of side L at the fixed window width: h windows
    (the smallest count whose union covers the paper's cut of the range),
    BINS_PER_WINDOW bins each, or bins of about bin_width J when given.  The
    range starts at the cut's lower end and ends where the h-th window ends.
    serial=True puts the same bins in one window with one walker."""
    from .workloads import paper_cut
    lo, hi = paper_cut(L, list(J))
    W = window_width(J)
    h = int(math.ceil(((hi - lo) / W - 1) / (1 - OVERLAP) - 1e-9)) + 1
    span = W * (1 + (h - 1) * (1 - OVERLAP))
    per = BINS_PER_WINDOW if bin_width is None else int(round(W / bin_width))
    B = int(round(per * (1 + (h - 1) * (1 - OVERLAP))))
    if serial:
        return dict(E_min=lo, E_max=lo + span, bins=B, h=1, m=1, width=W)
    return dict(E_min=lo, E_max=lo + span, bins=B, h=h, m=1, width=W)


def summarize(first):
    """Per-window move counts at the first flat histogram (None = not within
    the cap) -> quantiles over all windows, an unfinished window counting as
    infinitely slow ("qX": moves by which X % of the windows had finished,
    None if they had not), and finished windows per tenth of the window
    index (low to high energy)."""
    nw = len(first)
    allm = np.sort(np.array([np.inf if f is None else f for f in first], dtype=float))
    quant = {}
    for q in (5, 10, 25, 50, 75, 100):
        v = float(allm[max(int(math.ceil(q / 100.0 * nw)) - 1, 0)])
        quant["q%d" % q] = v if np.isfinite(v) else None
    tenth = [0] * 10
    for w in range(nw):
        if first[w] is not None:
            tenth[min(10 * w // nw, 9)] += 1
    done = [f for f in first if f is not None]
    return dict(finished=len(done), walkers=nw, moves_quantiles=quant, finished_per_tenth=tenth,
                median_of_finished=float(np.median(done)) if done else None)


def run_one(L, serial=False, cap_moves=2 * 10 ** 7, seg=10000, poll_segments=10, seed=0,
            J=J_PAPER_SHAPE, bin_width=None, proposal="uniform", harvest_segments=2,
            max_records=10 ** 7, log=None):
    """Run REWL (or the serial walk) from the ferromagnet until every window
    has finished its first WL iteration or cap_moves trial moves per walker
    have run.  Returns per-window move counts at the first flat histogram
    (to within poll_segments * seg moves; None where the cap came first).
    proposal="learned": the first harvest_segments segments are the plain
    walk, recording (field, spin) pairs of every k-th move (at most about
    max_records), on which the network is trained on the device; the walk
    then continues with the learned proposal.  Those segments count as moves
    of the walk."""
    import torch
    from .rewl import Run, rewl_set_harvest
    from . import learned
    lay = layout(L, J, serial, bin_width)
    N = 2 * L ** 3
    cfg = dict(lattice=("bcc", L, list(J)),
               windows=(lay["E_min"], lay["E_max"], lay["bins"], lay["h"], OVERLAP, lay["m"]),
               schedule=(4, 5, 1.0, 2.0 ** -20, seg, 100 * N))
    r = Run([cfg], mode="fp32_de")
    S = np.zeros((N, 3))
    S[:, 2] = 1.0
    t_init = time.perf_counter()
    r.init(seed, S)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t_init
    nw = r.n_walkers
    first = [None] * nw
    t0 = time.perf_counter()
    moves = 0
    info = {}

    def note_finished():
        for w in range(nw):
            if first[w] is None and r.walker(0, w)["iteration"] >= 1:
                first[w] = moves

    if proposal == "learned":
        every = max(1, -(-harvest_segments * seg * nw // max_records))
        r.set_harvest(harvest_segments * seg // every + 1, every)
        r.run(harvest_segments)
        moves += harvest_segments * seg
        recs = r.harvested()
        rewl_set_harvest(r.ctx, None, 0, 1)
        params = learned.init_params(1, recs.device)
        losses = learned.train(recs, params, epochs=4, batch=4096, lr=2e-3, seed=3)
        r.set_proposal(params)
        torch.cuda.synchronize()
        info = dict(records=int(recs.shape[0]), loss=[round(float(x), 4) for x in losses],
                    harvest_train_seconds=round(time.perf_counter() - t0, 2))
        del recs
        r.harvest_buf = None
        note_finished()
    next_log = 10 ** 7
    while moves < cap_moves and not all(f is not None for f in first):
        r.run(poll_segments)
        moves += poll_segments * seg
        note_finished()
        if log and moves >= next_log:
            log("L=%d %s: %.3g moves, %d of %d windows finished, %.0f s"
                % (L, proposal, moves, sum(f is not None for f in first), nw, time.perf_counter() - t0))
            next_log += 10 ** 7
    seconds = time.perf_counter() - t0
    launch = r.launch()
    acc = sum(r.walker(0, w)["accepts"] for w in range(nw)) / max(1, sum(r.walker(0, w)["attempts"] for w in range(nw)))
    r.close()
    return dict(L=L, N=N, serial=serial, proposal=proposal, windows=lay["h"], bins=lay["bins"],
                window_width=round(lay["width"], 2), cap_moves=cap_moves,
                resolution_moves=poll_segments * seg, **summarize(first), first_moves=first,
                acceptance=round(acc, 4), seconds=round(seconds, 2), init_seconds=round(t_init, 2),
                spins_in_lds=bool(launch["spins_in_lds"]), **info)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="10,20,30,40")
    ap.add_argument("--serial-sizes", default="10")
    ap.add_argument("--cap", type=int, default=2 * 10 ** 7, help="trial moves per walker")
    ap.add_argument("--serial-cap", type=int, default=5 * 10 ** 7)
    ap.add_argument("--poll", type=int, default=10, help="segments between reads of the walker states")
    ap.add_argument("--bin-width", type=float, default=None, help="bin width in J (default: 100 bins per window)")
    ap.add_argument("--proposal", choices=("uniform", "learned"), default="uniform")
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)
    for L in [int(x) for x in args.serial_sizes.split(",") if x]:
        print(json.dumps(run_one(L, serial=True, cap_moves=args.serial_cap, poll_segments=args.poll,
                                 bin_width=args.bin_width, proposal=args.proposal, seed=args.seed,
                                 log=log)), flush=True)
    for L in [int(x) for x in args.sizes.split(",") if x]:
        print(json.dumps(run_one(L, cap_moves=args.cap, poll_segments=args.poll, bin_width=args.bin_width,
                                 proposal=args.proposal, seed=args.seed, log=log)), flush=True)


if __name__ == "__main__":
    sys.exit(main())
