"""Pins of the oracle's walk over another coordinate: the magnetisation
M_z = sum_i S_i^z in place of the energy (the paper notes that the density of
states may be taken over other order parameters, Sec. original WL).

* Closed form.  With S_i uniform on the sphere, each S_i^z is uniform on
  [-1, 1] (Archimedes), so the density of M_z over N spins is that of a sum of
  N independent U(-1, 1): y = (M + N) / 2 follows the Irwin-Hall law with
  CDF F(y) = sum_{k <= y} (-1)^k C(N, k) (y - k)^N / N!.  A converged
  Wang-Landau walk over M_z reproduces ln of its bin masses, whatever the
  couplings (here an open chain, so E and M_z differ).
* The running coordinate equals sum_i S_i^z of the walker's configuration,
  computed here from the configuration itself, after every segment, and the
  incremental updates agree with full recomputes along the trajectory.

None of the expected values is taken from the oracle itself.
"""
from math import comb, factorial

import numpy as np
import pytest

from helpers import oracle_from


def _irwin_hall_cdf(y, N):
    if y <= 0:
        return 0.0
    if y >= N:
        return 1.0
    return sum((-1) ** k * comb(N, k) * (y - k) ** N for k in range(int(np.floor(y)) + 1)) / factorial(N)


def _exact_lng(N, lo, hi, B):
    edges = np.linspace(lo, hi, B + 1)
    F = np.array([_irwin_hall_cdf((e + N) / 2.0, N) for e in edges])
    return np.log(np.diff(F))


@pytest.mark.parametrize("N", [2, 4])
def test_mz_walk_matches_irwin_hall(oracle_mod, N):
    from oracle.analysis import normalise
    B = 16
    runs = []
    for seed in range(6):
        cfg = dict(lattice=("explicit", N, list(range(N - 1)), list(range(1, N)), [1.0] * (N - 1)),
                   windows=(-float(N), float(N), B, 1, 0.75, 2),
                   schedule=(4, 5, 1.0, 2.0 ** -14, 20000, 0), seed=100 + seed, coord="Mz")
        o = oracle_from(cfg, threads=2)
        o.run_to_convergence(max_segments=20000)
        assert o.all_done()
        from oracle.analysis import combine_walkers
        lg, vis = combine_walkers([o.lng(w) for w in range(2)], [o.hist(w)[1] for w in range(2)])
        assert np.all(vis)
        runs.append(normalise(lg))
    mean = np.mean(runs, axis=0)
    exact = normalise(_exact_lng(N, -N, N, B))
    d = mean - exact
    # the outermost bins hold ln-masses far below the centre (N = 4: -7.8);
    # six runs to ln f = 2^-14 resolve every bin to a few hundredths
    assert np.max(np.abs(d)) < 0.08, np.round(d, 3)


def test_mz_running_value_is_the_configurations_sum(oracle_mod):
    cfg = dict(lattice=("bcc", 4, [1.0, 0.5]), windows=(-24.0, 24.0, 24, 2, 0.75, 2),
               schedule=(4, 5, 1.0, 2.0 ** -6, 3000, 0), seed=7, coord="Mz")
    o = oracle_from(cfg, threads=2, check_energy=True)
    for _ in range(20):
        o.run(1)
        for w in range(o.W):
            s = o.walker(w)
            mz = float(np.sum(o.config(s["cfg"])[:, 2]))
            assert abs(mz - s["E"]) < 1e-9, (w, mz, s["E"])
            lo, hi = o.window(w)
            assert lo <= s["bin"] < hi and s["bin"] == int(np.floor((s["E"] + 24.0) / 2.0))
    assert o.max_check_err() < 1e-9
    assert sum(o.walker(w)["accepts"] for w in range(o.W)) > 1000
