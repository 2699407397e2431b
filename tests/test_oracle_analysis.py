"""Pins of the oracle's post-processing (joining fragments, thermodynamics)
against constructions with known answers."""
import math

import numpy as np
from scipy import optimize, stats


def test_join_recovers_function_up_to_constant():
    """Fragments of one smooth ln g with arbitrary per-window offsets (the
    constant each walker's ln g~ carries) join back to the function up to a
    single constant (joining where slopes coincide, Sec. parallel scheme)."""
    from oracle.analysis import join_windows
    B = 200
    E = np.arange(B)
    f = 40.0 - ((E - 80.0) / 30.0) ** 2 + 0.001 * E ** 1.5
    rng = np.random.default_rng(0)
    frags = []
    for lo in range(0, 151, 25):
        hi = lo + 50
        vis = np.ones(hi - lo, dtype=bool)
        frags.append((lo, hi, f[lo:hi] + rng.normal(scale=100.0), vis))
    bins, lg, joins = join_windows(frags)
    assert bins[0] == 0 and bins[-1] == 199
    d = lg - f
    assert np.nanmax(d) - np.nanmin(d) < 1e-9
    # the join point is an interior overlap bin
    for k, b in enumerate(joins):
        lo_next = frags[k + 1][0]
        hi_cur = frags[k][1]
        assert lo_next + 1 <= b <= hi_cur - 2


def test_join_picks_best_slope_match():
    """With a kink in one fragment the join moves to where slopes agree."""
    from oracle.analysis import join_windows
    E = np.arange(60, dtype=float)
    f = 0.5 * E
    a = f[0:40].copy()
    b = f[20:60].copy()
    b[:12] += 0.3 * (12 - np.arange(12)) ** 2      # window k+1 distorted at its low end
    frags = [(0, 40, a, np.ones(40, bool)), (20, 60, b, np.ones(40, bool))]
    _, lg, joins = join_windows(frags)
    assert joins[0] >= 32
    assert np.allclose(lg[joins[0]:] - f[joins[0]:], 0.0, atol=1e-12)


def test_thermo_exact_chain():
    """<E>(T) from exact binned Irwin-Hall g of an open chain equals the
    closed form -(N-1)J(coth(bJ) - 1/(bJ)) to binning accuracy
    (Sec. background, <E> = sum g E e^{-E/T} / Z)."""
    from oracle.analysis import thermo
    n, J, B = 6, 1.0, 600
    edges = np.linspace(-n, n, B + 1)
    ih = stats.irwinhall(n)
    mass = ih.cdf((n - edges[:-1]) / 2) - ih.cdf((n - edges[1:]) / 2)
    lg = np.where(mass > 0, np.log(np.maximum(mass, 1e-300)), -np.inf)
    lg[mass <= 0] = np.nan
    Ec = 0.5 * (edges[:-1] + edges[1:])
    T = np.linspace(0.3, 10.0, 30)
    U, C = thermo(Ec, lg, T)
    b = J / T
    Uex = -n * J * (1 / np.tanh(b) - 1 / b)
    Cex = n * (1 - b ** 2 / np.sinh(b) ** 2)
    assert np.max(np.abs(U - Uex)) < 2e-3
    assert np.max(np.abs(C - Cex)) < 5e-3


def test_cv_peak_schottky():
    """Two levels, degeneracies 1 (E=0) and G (E=1): C = G b^2 e^-b /(1+G e^-b)^2
    with b = 1/T; the peak found by the analysis matches a root of dC/dT."""
    from oracle.analysis import cv_peak
    G = 50.0
    E = np.array([0.0, 1.0])
    lg = np.array([0.0, math.log(G)])

    def C(T):
        b = 1.0 / T
        return G * b * b * math.exp(-b) / (1 + G * math.exp(-b)) ** 2

    Tstar = optimize.minimize_scalar(lambda T: -C(T), bounds=(0.05, 2.0), method="bounded",
                                     options={"xatol": 1e-10}).x
    Tp, Cp = cv_peak(E, lg, 0.05, 2.0)
    assert abs(Tp - Tstar) / Tstar < 1e-4
    assert abs(Cp - C(Tstar)) < 1e-6


def test_combine_walkers_offsets():
    from oracle.analysis import combine_walkers
    f = np.linspace(0, 5, 30)
    v = np.ones(30, bool)
    v2 = v.copy()
    v2[:3] = False
    out, vis = combine_walkers([f + 3.0, f - 7.0, f + 0.5], [v, v2, v])
    assert vis.all()
    assert np.allclose(out - f, 3.0)
