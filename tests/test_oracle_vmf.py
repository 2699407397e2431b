"""Pins of the FP64 learned-proposal reference (oracle/vmf_mlp.py)."""
import math

import numpy as np

from oracle import vmf_mlp as V


def _sphere_grid(nt=1200, nphi=2400):
    t = (np.arange(nt) + 0.5) * np.pi / nt
    p = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    T, P = np.meshgrid(t, p, indexing="ij")
    S = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], axis=-1).reshape(-1, 3)
    wts = (np.sin(T) * (np.pi / nt) * (2 * np.pi / nphi)).ravel()
    return S, wts


def test_density_integrates_to_one():
    """The mixture q is a probability density on S^2: a fine quadrature of
    q over the sphere is 1 for random networks and inputs (including very
    small and very large kappa)."""
    S, wts = _sphere_grid()
    rng = np.random.default_rng(0)
    for trial in range(4):
        theta = V.init_params(trial)
        X = rng.normal(size=(1, 4))
        out, _ = V.forward(theta, X)
        if trial == 3:
            out = out.copy()
            out[0, 0:3] = [0.0, 0.0, 1e-5]       # kappa clipped at the floor
            out[0, 4:7] = [0.0, 30.0, 0.0]       # concentrated
        lq = V.log_q(np.repeat(out, len(S), axis=0), S)
        assert abs(np.sum(np.exp(lq) * wts) - 1.0) < 1e-4


def test_vmf_mean_cosine_langevin():
    """For one vMF component, E[mu.s] = coth(k) - 1/k (Langevin function)."""
    S, wts = _sphere_grid(2000, 40)
    mu = np.array([0.0, 0.0, 1.0])
    for k in (0.3, 2.0, 15.0):
        f = np.exp(V.vmf_log_density(S, mu, np.full(len(S), k)))
        m = np.sum(f * S[:, 2] * wts) / np.sum(f * wts)
        assert abs(m - (1 / math.tanh(k) - 1 / k)) < 1e-5


def test_gradient_matches_finite_differences():
    """Analytic backprop of the mean NLL equals central differences."""
    rng = np.random.default_rng(3)
    theta = V.init_params(7) * 0.7
    X = rng.normal(size=(16, 4))
    S = rng.normal(size=(16, 3))
    S /= np.linalg.norm(S, axis=1, keepdims=True)
    L, g = V.loss_grad(theta, X, S)
    assert abs(L - V.loss(theta, X, S)) < 1e-12
    idx = rng.choice(V.N_PARAMS, size=60, replace=False)
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = 1e-6
        fd = (V.loss(theta + e, X, S) - V.loss(theta - e, X, S)) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * (1 + abs(fd)), (i, fd, g[i])


def test_sampler_follows_density():
    """Directions drawn by the inverse-CDF sampler follow q: chi-square over
    60 equal-area cells (z bands x azimuth sectors)."""
    from scipy import stats
    rng = np.random.default_rng(11)
    theta = V.init_params(5)
    out, _ = V.forward(theta, rng.normal(size=(1, 4)) * 2)
    n = 200000
    O = np.repeat(out, n, axis=0)
    su = rng.normal(size=(n, 3))
    su /= np.linalg.norm(su, axis=1, keepdims=True)
    s = V.sample(O, rng.random(n), rng.random(n), rng.random(n), su)
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0)
    nz, nphi = 6, 10

    def cell(v):
        zi = np.minimum(((v[:, 2] + 1) / 2 * nz).astype(int), nz - 1)
        pi = np.minimum(((np.arctan2(v[:, 1], v[:, 0]) + np.pi) / (2 * np.pi) * nphi).astype(int), nphi - 1)
        return zi * nphi + pi

    obs = np.bincount(cell(s), minlength=nz * nphi)
    G, wts = _sphere_grid(600, 1200)
    q = np.exp(V.log_q(np.repeat(out, len(G), axis=0), G)) * wts
    exp = np.bincount(cell(G), weights=q, minlength=nz * nphi) * n
    chi2 = np.sum((obs - exp) ** 2 / exp)
    assert stats.chi2.sf(chi2, nz * nphi - 1) > 1e-4
