"""Write data/batched_instances.json: the 64 independent instances of the
batched workload (inputs only).

Instance w: L = (6, 8, 10, 12)[w mod 4]; four shell couplings
J_n = -0.2 + 1.2 u_n with u from numpy's Philox generator (key 3, one
stream per instance); h = 8 + (w mod 25) windows, m = 4 + (w mod 5) walkers,
100 bins per window, o = 0.75; energy range cut from the quench span like
the other bcc workloads.  Usage: python paper_1411_4212_amd/make_batched.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def main():
    from paper_1411_4212_amd.workloads import energy_span
    out = []
    for w in range(64):
        bg = np.random.Generator(np.random.Philox(key=3, counter=[w, 0, 0, 0]))
        J = [float(-0.2 + 1.2 * u) for u in bg.random(4)]
        L = (6, 8, 10, 12)[w % 4]
        Lq = min(L, 8)
        lo, hi = energy_span(Lq, tuple(J), n_starts=2, iters=800)
        scale = (2 * L ** 3) / (2 * Lq ** 3)
        lo, hi = lo * scale, hi * scale
        span = hi - lo
        out.append(dict(L=L, J=J, h=8 + w % 25, m=4 + w % 5,
                        E_min=lo + span / 28.0, E_max=lo + 5.0 * span / 7.0))
        print(w, L, ["%.3f" % j for j in J], "%.1f %.1f" % (out[-1]["E_min"], out[-1]["E_max"]), flush=True)
    os.makedirs(os.path.join(HERE, "data"), exist_ok=True)
    with open(os.path.join(HERE, "data", "batched_instances.json"), "w") as f:
        json.dump({"_source": "paper_1411_4212_amd/make_batched.py", "instances": out}, f, indent=1)


if __name__ == "__main__":
    main()
