"""Time to converged ln g with the uniform and with the learned proposal
(the second half of the benchmark metric): wall-clock from the first sweep
until every walker has finished its last ln f iteration, and the error of
the joined ln g.  Library function plus a command line:

    python -m paper_1411_4212_amd.converge --workload c4 --cap 600

The learned run starts like the plain one; once the median walker has
reached ln f <= 2^-harvest_iter (with harvest_iter <= 0: right after the
start, while the walkers sit at the low end of their windows) it records
(x, S_i) of every k-th move for a few segments, trains the network on the
device, switches to the learned proposal and continues to the end.  Its
time includes harvest and training.
Progress goes to stdout as one JSON line per chunk.
"""
import argparse
import json
import math
import sys
import time

import numpy as np


def _progress(r):
    st = [r.walker(i, w) for i in range(len(r.inst)) for w in range(r.inst[i]["h"] * r.inst[i]["m"])]
    lnf = np.array([s["lnf"] for s in st])
    done = np.array([s["done"] for s in st])
    att = sum(s["attempts"] for s in st)
    acc = sum(s["accepts"] for s in st)
    it = np.array([s["iteration"] for s in st])
    hist = np.bincount(it, minlength=int(it.max()) + 1)
    return dict(max_lnf=float(lnf.max()), min_iter=int(round(-math.log2(lnf.max()))),
                done_frac=float(done.mean()), attempts=int(att), acceptance=acc / max(att, 1),
                iter_hist=hist.tolist())


def run(cfg, proposal="uniform", cap_s=600.0, rounds=256, harvest_iter=8, harvest_segments=4,
        harvest_every=16, epochs=4, seed=None, tag=""):
    import torch
    from . import analysis, learned, workloads
    from .rewl import Run
    r = Run([dict(lattice=cfg["lattice"], windows=cfg["windows"], schedule=cfg["schedule"])], mode="fp32_de")
    r.init(cfg["seed"] if seed is None else seed, workloads.init_spins(cfg))
    dev = torch.device("cuda", 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phase = "plain"
    info = {}
    done = False
    done_at = np.full(r.n_walkers, np.nan)

    def switch():
        # harvest (field, spin) pairs of the plain walk, train, switch
        th = time.perf_counter()
        seg = cfg["schedule"][4]
        cap = harvest_segments * seg // harvest_every + 1
        r.set_harvest(cap, harvest_every)
        r.run(harvest_segments)
        recs = r.harvested()
        from .rewl import rewl_set_harvest
        rewl_set_harvest(r.ctx, None, 0, 1)
        params = learned.init_params(1, dev)
        losses = learned.train(recs, params, epochs=epochs, batch=4096, lr=2e-3, seed=3)
        r.set_proposal(params)
        torch.cuda.synchronize()
        out = dict(records=int(recs.shape[0]), loss=[round(float(x), 4) for x in losses],
                   harvest_train_s=round(time.perf_counter() - th, 2))
        print(json.dumps(dict(tag=tag, event="switched to learned proposal", **out)), flush=True)
        del recs
        r.harvest_buf = None
        return out

    if proposal == "learned" and harvest_iter <= 0:
        # right after the start: the walkers have just entered their windows
        # from below (ferromagnetic start), so the records cover the low end
        info = switch()
        phase = "learned"
    while True:
        r.run_persistent(rounds)
        done = bool(r.poll())
        p = _progress(r)
        el = time.perf_counter() - t0
        dn = np.array([r.walker(0, w)["done"] for w in range(r.n_walkers)], dtype=bool)
        done_at[dn & np.isnan(done_at)] = el
        print(json.dumps(dict(tag=tag, proposal=proposal, phase=phase, seconds=round(el, 2), **p)), flush=True)
        if done or el > cap_s:
            break
        its = np.repeat(np.arange(len(p["iter_hist"])), p["iter_hist"])
        if proposal == "learned" and phase == "plain" and np.median(its) >= harvest_iter:
            info = switch()
            phase = "learned"
    seconds = time.perf_counter() - t0
    states = [r.walker(0, w) for w in range(r.n_walkers)]
    order = sorted(range(r.n_walkers), key=lambda w: states[w]["iteration"])[:12]
    slow = []
    for w in order:
        h_ = r.hist(0, w)
        v_ = r.visited(0, w).astype(bool)
        slow.append(dict(walker=w, window=states[w]["window"], iteration=states[w]["iteration"],
                         n_visited=states[w]["n_visited"], bins=int(v_.size), bin=states[w]["bin"],
                         H_min=int(h_[v_].min()) if v_.any() else 0,
                         H_mean=float(h_[v_].mean()) if v_.any() else 0.0))
    print(json.dumps(dict(tag=tag, slowest_walkers=slow)), flush=True)
    try:
        bins, lng = analysis.run_lng(r, 0)
    except ValueError as e:          # windows not yet joinable
        print(json.dumps(dict(tag=tag, join_failed=str(e))), flush=True)
        bins = np.arange(cfg["windows"][2])
        lng = np.full(cfg["windows"][2], np.nan)
    # per-window combined ln g of the windows whose walkers are all done
    inst = r.inst[0]
    frags = {}
    for k in range(inst["h"]):
        ws = range(k * inst["m"], (k + 1) * inst["m"])
        if all(r.walker(0, w)["done"] for w in ws):
            lg_k, vis_k = analysis.combine_walkers([r.lng(0, w) for w in ws], [r.visited(0, w) for w in ws])
            frags["win%03d" % k] = np.where(vis_k, lg_k, np.nan)
    fr = {}
    m_ = inst["m"]
    fr["window_done_s"] = [None if np.isnan(done_at[k * m_:(k + 1) * m_]).any()
                           else round(float(done_at[k * m_:(k + 1) * m_].max()), 1) for k in range(inst["h"])]
    for q in (50, 75, 90, 100):
        k = int(math.ceil(q / 100.0 * r.n_walkers))
        srt = np.sort(done_at)
        fr["t_done_%d%%" % q] = None if np.isnan(srt[k - 1]) else round(float(srt[k - 1]), 1)
    res = dict(tag=tag, proposal=proposal, seconds=seconds, done=done, **fr, **_progress(r), **info)
    r.close()
    return res, bins, lng, frags


def race(cfg, proposal="uniform", R=64, chunk=8, cap_s=600.0, harvest_iter=6, harvest_segments=2,
         harvest_every=4, epochs=4, seed=11, log=None, max_records=10_000_000):
    """R independent REWL runs of one workload in one context, run to the
    end by the persistent kernel; the wall-clock time at which each run's
    last walker finished its final ln f iteration (the paper's stopping
    rule: f has reached f_min), and each run's joined ln g.

    With proposal="learned" the runs start with the uniform proposal; once
    the median walker has reached ln f <= 2^-harvest_iter, (x, S_i) of every
    harvest_every-th move is recorded for harvest_segments segments, the
    network is trained on the device, and the runs continue with the learned
    proposal.  Harvest and training are inside the measured time; the
    harvest takes every k-th move with k at least harvest_every and large
    enough to keep the records under max_records."""
    import torch
    from . import analysis, learned, workloads
    from .rewl import Run, rewl_set_harvest
    r = Run([dict(lattice=cfg["lattice"], windows=cfg["windows"], schedule=cfg["schedule"])] * R,
            mode="fp32_de")
    init = workloads.init_spins(cfg)
    r.init(seed, None if init is None else np.concatenate([init] * R))
    dev = torch.device("cuda", 0)
    nw = r.inst[0]["h"] * r.inst[0]["m"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phase = "plain" if proposal == "learned" else proposal
    done_at = np.full(R, np.nan)
    info = {}
    rounds = 0
    while True:
        r.run_persistent(chunk)
        rounds += chunk
        all_done = bool(r.poll())
        el = time.perf_counter() - t0
        st = [[r.walker(i, w) for w in range(nw)] for i in range(R)]
        for i in range(R):
            if np.isnan(done_at[i]) and all(s["done"] for s in st[i]):
                done_at[i] = el
        if log:
            log("%s: %d rounds, %.1f s, %d of %d runs done" % (proposal, rounds, el, np.isfinite(done_at).sum(), R))
        if all_done or el > cap_s:
            break
        its = np.array([s["iteration"] for row in st for s in row])
        if proposal == "learned" and phase == "plain" and np.median(its) >= harvest_iter:
            th = time.perf_counter()
            seg = cfg["schedule"][4]
            # about 1e7 records at most (what the network needs; long segments
            # would otherwise make training the larger cost)
            every = max(harvest_every, -(-harvest_segments * seg * r.n_walkers // max_records))
            r.set_harvest(harvest_segments * seg // every + 1, every)
            r.run(harvest_segments)
            recs = r.harvested()
            rewl_set_harvest(r.ctx, None, 0, 1)
            params = learned.init_params(1, dev)
            losses = learned.train(recs, params, epochs=epochs, batch=4096, lr=2e-3, seed=3)
            r.set_proposal(params)
            torch.cuda.synchronize()
            info = dict(records=int(recs.shape[0]), loss=[round(float(x), 4) for x in losses],
                        harvest_train_s=round(time.perf_counter() - th, 2), switched_at_s=round(el, 2))
            del recs
            r.harvest_buf = None
            phase = "learned"
    lngs = []
    for i in range(R):
        try:
            lngs.append(analysis.run_lng(r, i)[1])
        except ValueError:
            lngs.append(np.full(cfg["windows"][2], np.nan))
    att = sum(s["attempts"] for row in st for s in row)
    acc = sum(s["accepts"] for row in st for s in row)
    r.close()
    return dict(proposal=proposal, runs=R, done_at=done_at, seconds=time.perf_counter() - t0,
                acceptance=acc / max(att, 1), attempts=int(att), **info), np.array(lngs)


def workload_config(name):
    """A workloads.py configuration by name, or "scan_L<n>": the layout of the
    weak-scaling scan for bcc side n (J = (1, 0.5), windows of the fixed
    width at overlap 0.75, 3 J bins, one walker per window, exchange every
    1e4 moves, ferromagnetic start, ln f from 1 to 2^-20)."""
    from . import workloads
    if name.startswith("scan_L"):
        from .weak_scaling import OVERLAP, layout
        L = int(name[len("scan_L"):])
        lay = layout(L, bin_width=3)
        return dict(name=name, lattice=("bcc", L, [1.0, 0.5]),
                    windows=(lay["E_min"], lay["E_max"], lay["bins"], lay["h"], OVERLAP, 1),
                    schedule=(4, 5, 1.0, 2.0 ** -20, 10000, 100 * 2 * L ** 3), seed=0, init="ferro")
    return getattr(workloads, name)()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c4",
                    help="a workloads.py configuration (c4, c5, ...), or scan_L<n>: the weak-scaling "
                         "layout for bcc side n (one walker per window, 3 J bins, ferromagnetic start)")
    ap.add_argument("--cap", type=float, default=600.0, help="seconds per run")
    ap.add_argument("--lnf-final-exp", type=int, default=20, help="run to ln f = 2^-this")
    ap.add_argument("--proposals", default="uniform,learned")
    ap.add_argument("--seeds", default="0")
    ap.add_argument("--harvest-iter", type=int, default=8,
                    help="learned runs: harvest once the median walker is at ln f <= 2^-this "
                         "(<= 0: right after the start)")
    ap.add_argument("--harvest-segments", type=int, default=4)
    ap.add_argument("--harvest-every", type=int, default=16)
    ap.add_argument("--rounds", type=int, default=256, help="rounds per persistent launch")
    ap.add_argument("--out", default=None, help="write the joined ln g of every run (npz)")
    args = ap.parse_args()
    cfg = workload_config(args.workload)
    s = list(cfg["schedule"])
    s[3] = 2.0 ** -args.lnf_final_exp
    cfg["schedule"] = tuple(s)
    results, curves = [], {}
    for seed in [int(x) for x in args.seeds.split(",")]:
        for prop in args.proposals.split(","):
            tag = "%s/seed%d" % (prop, seed)
            res, bins, lng, frags = run(cfg, prop, args.cap, rounds=args.rounds, harvest_iter=args.harvest_iter,
                                        harvest_segments=args.harvest_segments,
                                        harvest_every=args.harvest_every, seed=seed, tag=tag)
            results.append(res)
            curves[tag] = lng
            for k, v in frags.items():
                curves[tag + "/" + k] = v
            print(json.dumps(dict(result=res)), flush=True)
    keys = [k for k in curves if k.count("/") == 1]
    for i in range(len(keys)):
        for j in range(i + 1, len(keys)):
            a, b = curves[keys[i]], curves[keys[j]]
            ok = np.isfinite(a) & np.isfinite(b)
            d = (a - a[ok].mean()) - (b - b[ok].mean())
            print(json.dumps(dict(compare=[keys[i], keys[j]], max_abs_dlng=float(np.abs(d[ok]).max()),
                                  rms_dlng=float(np.sqrt(np.mean(d[ok] ** 2))), bins=int(ok.sum()))), flush=True)
    if args.out:
        np.savez(args.out, **{k.replace("/", "__"): v for k, v in curves.items()})


if __name__ == "__main__":
    sys.exit(main())
