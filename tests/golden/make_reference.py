"""Write the oracle references of the GPU statistical parity tests.

Calls only the CPU oracle.  Two kinds of reference, per workload:

* ``wl``: the mean normalised joined ln g (and its spread) over many
  independent REWL runs (each run's walkers combined per window, windows
  joined where the slopes of ln g coincide, the result normalised to zero
  mean); run r uses seed 1000 + r.  This is the Wang-Landau estimator itself,
  with its run-to-run spread (the paper's accuracy check compares Delta with
  sigma over independent runs, Sec. results and discussion).

* ``truth``: ln g from a fixed-weight (multicanonical) run, which has no
  Wang-Landau modification error.  With the weights 1/g~ frozen, the walk is
  an ordinary Markov chain whose stationary histogram is H(E) ~ g(E)/g~(E)
  (the flat-histogram idea of Sec. original WL), so ln g = ln g~ + ln H up to
  a constant per window.  The weights come from a few short WL runs of the
  oracle; H is accumulated in batches (the first eighth discarded as a
  burn-in), whose spread gives the standard error.  Windows are joined by the
  mean offset over the bins both cover.

Usage:
  python tests/golden/make_reference.py wl <workload> [runs] [threads] [output file]
  python tests/golden/make_reference.py truth <workload> [batches] [segments_per_batch] [threads]

Workloads (bcc, o = 0.75, flatness 0.8, ln f 1 -> final, resync every 100 N):
  L4_mid  L=4, J = (1, 0.5), E in [-400, -100) on 30 bins, 2 windows x 8
          walkers, ln f -> 2^-18, 2e5 moves per segment (ref_parity_L4.json)
  L4_low  the same lattice on [-550, -50) with 40 bins, reaching down to
          about 4.3 J per spin against the ferromagnet's 5.5
          (ref_parity_L4_low.json, truth_L4_low.json)
  z50_L6  bcc L=6 (432 spins), J = (1, 0.6, -0.05, -0.1) (z = 50), E in
          [-1500, -1380) on 40 bins of 3 J (ferromagnet -1857.6; canonical
          temperatures about 0.85 to 1.1, so ln g changes by about 3 per
          bin), 2 windows x 4 walkers, ln f -> 2^-16, 1e5 moves per segment
          (ref_parity_z50_L6.json, truth_z50_L6.json)
  z112_L6 bcc L=6, eight shells J_n = e^{-0.6 (n-1)} (-1)^[n>5] (z = 112),
          E in [-3380, -3200) on 40 bins of 4.5 J (ferromagnet -3949.7;
          temperatures about 1.5 to 1.9), the same layout and schedule
          (ref_parity_z112_L6.json, truth_z112_L6.json)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_1411_4212_amd.workloads import J8, J_C2  # noqa: E402  (input parameters only)

WORKLOADS = {
    "L4_mid": dict(lattice=("bcc", 4, [1.0, 0.5]), windows=(-400.0, -100.0, 30, 2, 0.75, 8),
                   schedule=(4, 5, 1.0, 2.0 ** -18, 200000, 12800)),
    "L4_low": dict(lattice=("bcc", 4, [1.0, 0.5]), windows=(-550.0, -50.0, 40, 2, 0.75, 8),
                   schedule=(4, 5, 1.0, 2.0 ** -18, 200000, 12800)),
    # the shapes of the larger workloads on a lattice the oracle converges:
    # four shells (z = 50) and eight shells (z = 112) on bcc L=6 (a lattice
    # size that is not a power of two), each over 40 bins from the bottom of
    # the paper's range cut upwards
    "z50_L6": dict(lattice=("bcc", 6, list(J_C2)),
                   windows=(-1500.0, -1380.0, 40, 2, 0.75, 4),
                   schedule=(4, 5, 1.0, 2.0 ** -16, 100000, 43200)),
    "z112_L6": dict(lattice=("bcc", 6, list(J8)),
                    windows=(-3380.0, -3200.0, 40, 2, 0.75, 4),
                    schedule=(4, 5, 1.0, 2.0 ** -16, 100000, 43200)),
}
WL_OUT = {"L4_mid": "ref_parity_L4.json", "L4_low": "ref_parity_L4_low.json",
          "z50_L6": "ref_parity_z50_L6.json", "z112_L6": "ref_parity_z112_L6.json"}
TRUTH_OUT = {"L4_low": "truth_L4_low.json", "L4_mid": "truth_L4_mid.json",
             "z50_L6": "truth_z50_L6.json", "z112_L6": "truth_z112_L6.json"}


def _oracle(wl, threads):
    import oracle
    lat = wl["lattice"]
    o = oracle.Oracle(L=lat[1], J=lat[2])
    o.set_windows(*wl["windows"])
    o.set_threads(threads)
    return o


def _joined(o, h, m):
    from oracle.analysis import combine_walkers, join_windows
    frags = []
    for k in range(h):
        ws = range(k * m, (k + 1) * m)
        lo, hi = o.window(k * m)
        lg, vis = combine_walkers([o.lng(w) for w in ws], [o.hist(w)[1] for w in ws])
        frags.append((lo, hi, lg, vis))
    _, lg, _ = join_windows(frags)
    return lg


def wl_run(wl, seed, threads, schedule=None):
    from oracle.analysis import normalise
    o = _oracle(wl, threads)
    o.set_schedule(*(schedule or wl["schedule"]))
    o.init(seed)
    o.run_to_convergence(max_segments=100000)
    return normalise(_joined(o, wl["windows"][3], wl["windows"][5]))


def join_by_offset(frags, B):
    """frags: list of (lo, ln g over [lo, hi) with NaN where absent).  Each
    window is shifted onto the union of the previous ones by the mean offset
    over the bins both cover; the covered bins are averaged."""
    acc = np.zeros(B)
    cnt = np.zeros(B)
    for lo, lg in frags:
        idx = np.arange(lo, lo + len(lg))
        ok = np.isfinite(lg)
        have = cnt[idx] > 0
        both = ok & have
        off = 0.0
        if both.any():
            off = np.mean(acc[idx][both] / cnt[idx][both] - lg[both])
        acc[idx[ok]] += lg[ok] + off
        cnt[idx[ok]] += 1
    out = np.full(B, np.nan)
    out[cnt > 0] = acc[cnt > 0] / cnt[cnt > 0]
    return out


def _fixed_weight_pass(wl, W, batches, seg_per_batch, threads, seed):
    """One fixed-weight run with weights W (global bins): per window, the
    histogram summed over its walkers, in batches."""
    Emin, Emax, B, h, o_, m = wl["windows"]
    sch = wl["schedule"]
    o = _oracle(wl, threads)
    o.set_schedule(1, 1, 1e-300, 1e-300, sch[4], sch[5])
    o.init(seed)
    for w in range(h * m):
        lo, hi = o.window(w)
        wv = W[lo:hi]
        o.write_lng(w, np.where(np.isfinite(wv), wv, 0.0), np.isfinite(wv).astype(np.uint8))
    prev = [o.hist(w)[0].astype(np.float64) for w in range(h * m)]
    wins = [o.window(k * m) for k in range(h)]
    Hb = []
    for b in range(batches):
        o.run(seg_per_batch)
        row = []
        for k in range(h):
            lo, hi = wins[k]
            Hk = np.zeros(hi - lo)
            for w in range(k * m, (k + 1) * m):
                cur = o.hist(w)[0].astype(np.float64)
                Hk += cur - prev[w]
                prev[w] = cur
            row.append(Hk)
        Hb.append(row)
        print("batch %d/%d" % (b + 1, batches), flush=True)
    attempts = sum(o.walker(w)["attempts"] for w in range(h * m))
    return wins, Hb, attempts


def _estimate(W, wins, Hs, B):
    frags = []
    for (lo, hi), Hk in zip(wins, Hs):
        frags.append((lo, np.where(Hk > 0, W[lo:hi] + np.log(np.maximum(Hk, 1.0)), np.nan)))
    return join_by_offset(frags, B)


def truth(wl, batches, seg_per_batch, threads):
    """Fixed-weight estimate of ln g (see the module docstring): weights from
    four short Wang-Landau runs (ln f -> 2^-12), refined by one fixed-weight
    pass, then the measured pass; its batches, each aligned to the total by
    the mean offset over the bins both cover, give the standard error.  Each
    pass starts from walkers just driven into their windows (from above, the
    random start being hotter than the range), so the first eighth of its
    batches is a burn-in and does not count."""
    from oracle.analysis import normalise
    B, h, m = wl["windows"][2], wl["windows"][3], wl["windows"][5]
    sch = wl["schedule"]
    short = (sch[0], sch[1], sch[2], 2.0 ** -12, sch[4], sch[5])
    W = np.nanmean([wl_run(wl, 7000 + r, threads, short) for r in range(4)], axis=0)
    wins, Hb, _ = _fixed_weight_pass(wl, W, max(batches // 4, 2), seg_per_batch, threads, 8000)
    Hb = Hb[max(len(Hb) // 8, 1):]
    W1 = _estimate(W, wins, [sum(r[k] for r in Hb) for k in range(h)], B)
    W1 = np.where(np.isfinite(W1), W1, W)
    wins, Hb, attempts = _fixed_weight_pass(wl, W1, batches, seg_per_batch, threads, 8001)
    Hb = Hb[max(len(Hb) // 8, 1):]
    est = normalise(_estimate(W1, wins, [sum(r[k] for r in Hb) for k in range(h)], B))
    per = []
    for r in Hb:
        e = _estimate(W1, wins, r, B)
        ok = np.isfinite(e) & np.isfinite(est)
        per.append(e - np.mean(e[ok] - est[ok]))
    A = np.array(per)
    n = np.isfinite(A).sum(0)
    se = np.nanstd(A, axis=0, ddof=1) / np.sqrt(n)
    return est, se, attempts, W1


def main():
    from oracle.analysis import cv_peak
    kind, name = sys.argv[1], sys.argv[2]
    wl = WORKLOADS[name]
    Emin, Emax, B = wl["windows"][:3]
    Ec = Emin + (np.arange(B) + 0.5) * (Emax - Emin) / B
    if kind == "truth":
        batches = int(sys.argv[3]) if len(sys.argv) > 3 else 32
        spb = int(sys.argv[4]) if len(sys.argv) > 4 else 40
        threads = int(sys.argv[5]) if len(sys.argv) > 5 else 8
        t0 = time.time()
        est, se, attempts, W = truth(wl, batches, spb, threads)
        doc = {"_source": "tests/golden/make_reference.py truth %s (CPU oracle only)" % name,
               "workload": wl, "batches": batches, "segments_per_batch": spb,
               "attempts": int(attempts), "lng": est.tolist(), "se": se.tolist(),
               "weights": W.tolist(), "cv_peak_T": cv_peak(Ec, est, 1.0, 8.0)[0]}
        out = os.path.join(HERE, TRUTH_OUT[name])
        with open(out + ".tmp", "w") as f:
            json.dump(doc, f, indent=1)
        os.replace(out + ".tmp", out)
        print("truth %s: %d attempts, %.0f s, max se %.4f" % (name, attempts, time.time() - t0,
                                                             np.nanmax(se)))
        return
    runs = int(sys.argv[3]) if len(sys.argv) > 3 else 256
    threads = int(sys.argv[4]) if len(sys.argv) > 4 else 8
    out = os.path.join(HERE, sys.argv[5] if len(sys.argv) > 5 else WL_OUT[name])
    all_lg, peaks = [], []
    t0 = time.time()
    for r in range(runs):
        lg = wl_run(wl, 1000 + r, threads)
        all_lg.append(lg)
        peaks.append(cv_peak(Ec, lg, 1.0, 8.0)[0])
        if (r + 1) % 8 == 0 or r + 1 == runs:
            A = np.array(all_lg)
            mean = np.nanmean(A, axis=0)
            mean = mean - np.nanmean(mean)
            doc = {
                "_source": "tests/golden/make_reference.py wl %s (CPU oracle only)" % name,
                "workload": wl, "runs": len(all_lg), "seeds": [1000, 1000 + len(all_lg) - 1],
                "mean_lng": mean.tolist(), "std_lng": np.nanstd(A, axis=0, ddof=1).tolist(),
                "finite_runs": np.isfinite(A).sum(0).tolist(),
                "cv_peak_T_of_mean": cv_peak(Ec, mean, 1.0, 8.0)[0],
                "cv_peak_T_runs": peaks,
                "run_lng": [[None if not np.isfinite(v) else round(float(v), 6) for v in r] for r in all_lg],
            }
            with open(out + ".tmp", "w") as f:
                json.dump(doc, f, indent=1)
            os.replace(out + ".tmp", out)
            print("runs %d  %.0fs  peak(mean) %.4f" % (len(all_lg), time.time() - t0,
                                                       doc["cv_peak_T_of_mean"]), flush=True)


if __name__ == "__main__":
    main()
