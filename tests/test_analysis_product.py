"""The product-side read-out post-processing (paper_1411_4212_amd.analysis)
agrees with the oracle's independent implementation on random fragments."""
import numpy as np


def _fragments(rng, h=4, width=40, step=10, holes=True):
    truth = np.cumsum(rng.normal(0.5, 0.3, size=width + step * (h - 1)))
    frags = []
    for k in range(h):
        lo = k * step
        vis = np.ones(width, dtype=bool)
        if holes:
            vis[rng.integers(0, width, size=3)] = False
            vis[1:-1] = vis[1:-1]
        lg = truth[lo:lo + width] + rng.normal(0, 0.05, size=width) + rng.normal(0, 5)
        frags.append((lo, lo + width, np.where(vis, lg, 0.0), vis))
    return frags


def test_combine_matches_oracle():
    from oracle.analysis import combine_walkers as oc
    from paper_1411_4212_amd.analysis import combine_walkers as pc
    rng = np.random.default_rng(3)
    for _ in range(20):
        W, B = 8, 50
        lngs = rng.normal(size=(W, B)) + rng.normal(0, 10, size=(W, 1))
        vis = rng.random((W, B)) < 0.8
        a, va = oc(list(lngs), list(vis))
        b, vb = pc(list(lngs), list(vis))
        assert np.array_equal(va, vb)
        assert np.allclose(a[va], b[vb], rtol=0, atol=1e-12)


def test_join_matches_oracle():
    from oracle.analysis import join_windows as oj
    from paper_1411_4212_amd.analysis import join_windows as pj
    rng = np.random.default_rng(5)
    for _ in range(20):
        frags = _fragments(rng)
        b1, g1, j1 = oj(frags)
        b2, g2, j2 = pj(frags)
        assert j1 == j2
        assert np.array_equal(np.isnan(g1), np.isnan(g2))
        ok = ~np.isnan(g1)
        assert np.allclose(g1[ok], g2[ok], rtol=0, atol=1e-10)


def test_cv_peak_matches_oracle():
    from oracle.analysis import cv_peak as ocv
    from paper_1411_4212_amd.analysis import cv_peak as pcv
    # two-level system on a coarse grid: Schottky peak
    E = np.array([0.0, 1.0])
    lng = np.array([0.0, np.log(3.0)])
    t1 = ocv(E, lng, 0.1, 3.0)[0]
    t2 = pcv(E, lng, 0.1, 3.0)[0]
    assert abs(t1 - t2) / t1 < 1e-3
