"""Write tests/golden/ref_parity_L4.json: the oracle's mean normalised ln g
(and its spread) over many independent REWL runs of one small workload,
the reference of the GPU statistical parity test.

Calls only the CPU oracle.  Usage: python tests/golden/make_reference.py [runs] [threads]

Workload: bcc L=4 (128 spins), J = (1, 0.5), E in [-400, -100) on 30 bins
(the middle of the spectrum, so that every bin is well sampled and the
run-to-run spread of ln g stays near 0.02-0.05), 2 windows (o = 0.75) x 8
walkers, flatness 0.8, ln f 1 -> 2^-18, 2e5 moves per segment, resync every
100 N moves; run r uses seed 1000 + r.  The specific heat of this range
peaks near T = 2.8.
Each run's walkers are combined per window and the windows joined where the
slopes of ln g coincide; the joined ln g is normalised to zero mean.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

WORKLOAD = dict(lattice=("bcc", 4, [1.0, 0.5]), windows=(-400.0, -100.0, 30, 2, 0.75, 8),
                schedule=(4, 5, 1.0, 2.0 ** -18, 200000, 12800))
OUT = os.path.join(HERE, "ref_parity_L4.json")


def one_run(seed, threads):
    import oracle
    from oracle.analysis import combine_walkers, join_windows, normalise
    lat = WORKLOAD["lattice"]
    o = oracle.Oracle(L=lat[1], J=lat[2])
    o.set_windows(*WORKLOAD["windows"])
    o.set_schedule(*WORKLOAD["schedule"])
    o.set_threads(threads)
    o.init(seed)
    o.run_to_convergence(max_segments=100000)
    h, m = WORKLOAD["windows"][3], WORKLOAD["windows"][5]
    frags = []
    for k in range(h):
        ws = range(k * m, (k + 1) * m)
        lo, hi = o.window(k * m)
        lg, vis = combine_walkers([o.lng(w) for w in ws], [o.hist(w)[1] for w in ws])
        frags.append((lo, hi, lg, vis))
    _, lg, _ = join_windows(frags)
    return normalise(lg)


def main():
    runs = int(sys.argv[1]) if len(sys.argv) > 1 else 256
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else 8
    from oracle.analysis import cv_peak
    Emin, Emax, B = WORKLOAD["windows"][:3]
    Ec = Emin + (np.arange(B) + 0.5) * (Emax - Emin) / B
    all_lg, peaks = [], []
    t0 = time.time()
    for r in range(runs):
        lg = one_run(1000 + r, threads)
        all_lg.append(lg)
        peaks.append(cv_peak(Ec, lg, 1.0, 8.0)[0])
        if (r + 1) % 8 == 0 or r + 1 == runs:
            A = np.array(all_lg)
            mean = np.nanmean(A, axis=0)
            mean = mean - np.nanmean(mean)
            doc = {
                "_source": "tests/golden/make_reference.py (CPU oracle only)",
                "workload": WORKLOAD, "runs": len(all_lg), "seeds": [1000, 1000 + len(all_lg) - 1],
                "mean_lng": mean.tolist(), "std_lng": np.nanstd(A, axis=0, ddof=1).tolist(),
                "finite_runs": np.isfinite(A).sum(0).tolist(),
                "cv_peak_T_of_mean": cv_peak(Ec, mean, 1.0, 8.0)[0],
                "cv_peak_T_runs": peaks,
            }
            with open(OUT + ".tmp", "w") as f:
                json.dump(doc, f, indent=1)
            os.replace(OUT + ".tmp", OUT)
            print("runs %d  %.0fs  peak(mean) %.4f" % (len(all_lg), time.time() - t0,
                                                       doc["cv_peak_T_of_mean"]), flush=True)


if __name__ == "__main__":
    main()
