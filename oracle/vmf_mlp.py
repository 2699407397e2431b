"""FP64 reference of the learned proposal (TEST INFRASTRUCTURE).

The proposal is not part of the paper; the paper's trial move is a uniform
new direction (Sec. simulation details).  A learned proposal keeps the
sampling exact because Wang-Landau acceptance with an asymmetric proposal
q uses min(1, g(E_A) q(S_i|x) / (g(E_B) q(S'|x))) (the Metropolis-Hastings
form of the acceptance of Sec. original WL), with x independent of the
moved spin.

Model: x = (h / h_s, e_w) with h the local field at the site (which does not
contain the site's own spin), h_s = sum_n z_n |J_n| and e_w the window's
centre energy per spin in units of h_s / 2.  MLP 4 -> 64 -> 64 -> 12 with ReLU;
outputs (v_c in R^3, a_c) for c = 0, 1, 2.  kappa_c = clip(|v_c|, 1e-3, 1e3),
mu_c = v_c / |v_c|, alpha = softmax(a).  Density on the unit sphere
  q(s) = eps / (4 pi) + (1 - eps) sum_c alpha_c f(s; mu_c, kappa_c),
  f(s; mu, k) = k / (2 pi (1 - e^{-2k})) exp(k (mu.s - 1))    (von Mises-Fisher, p = 3)
with eps = 0.05.  Sampling: with probability eps a uniform direction, else
component c with probability alpha_c and w = mu.s from the inverse CDF
w = 1 + ln(u + (1 - u) e^{-2k}) / k, azimuth uniform about mu.

Parameters are one flat FP64 vector in the order W1[64,4], b1[64], W2[64,64],
b2[64], W3[12,64], b3[12] (5260 values).
"""
import numpy as np

EPS = 0.05
K_MIN, K_MAX = 1e-3, 1e3
SHAPES = [("W1", (64, 4)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (12, 64)),
          ("b3", (12,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def init_params(seed=0):
    """He-uniform weights, zero biases (numpy generator with `seed`)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in SHAPES:
        if name.startswith("W"):
            fan_in = shp[1]
            lim = np.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, size=shp).ravel())
        else:
            parts.append(np.zeros(shp))
    return np.concatenate(parts)


def forward(theta, X):
    p = unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ p["W2"].T + p["b2"]
    a2 = np.maximum(z2, 0.0)
    out = a2 @ p["W3"].T + p["b3"]
    return out, (X, z1, a1, z2, a2)


def mixture(out):
    """kappa [n,3], mu [n,3,3], alpha [n,3], |v| [n,3] from outputs [n,12]."""
    v = out.reshape(-1, 3, 4)[:, :, :3]
    a = out.reshape(-1, 3, 4)[:, :, 3]
    r = np.linalg.norm(v, axis=2)
    kappa = np.clip(r, K_MIN, K_MAX)
    mu = v / np.maximum(r, 1e-300)[:, :, None]
    am = a - a.max(axis=1, keepdims=True)
    alpha = np.exp(am) / np.exp(am).sum(axis=1, keepdims=True)
    return kappa, mu, alpha, r


def vmf_log_density(s, mu, kappa):
    """ln f(s; mu, kappa) for unit vectors, broadcast over leading axes."""
    w = np.sum(mu * s, axis=-1)
    return (np.log(kappa) - np.log(2.0 * np.pi) - np.log(-np.expm1(-2.0 * kappa))
            + kappa * (w - 1.0))


def log_q(out, S):
    """ln q(S | outputs) for S [n,3]."""
    kappa, mu, alpha, _ = mixture(out)
    f = np.exp(vmf_log_density(S[:, None, :], mu, kappa))
    q = EPS / (4.0 * np.pi) + (1.0 - EPS) * np.sum(alpha * f, axis=1)
    return np.log(q)


def loss(theta, X, S):
    out, _ = forward(theta, X)
    return float(-np.mean(log_q(out, S)))


def loss_grad(theta, X, S):
    """Mean negative log-likelihood and its gradient (analytic backprop)."""
    p = unpack(theta)
    out, (X, z1, a1, z2, a2) = forward(theta, X)
    n = X.shape[0]
    v = out.reshape(n, 3, 4)[:, :, :3]
    kappa, mu, alpha, r = mixture(out)
    w = np.sum(mu * S[:, None, :], axis=2)
    lf = vmf_log_density(S[:, None, :], mu, kappa)
    f = np.exp(lf)
    F = np.sum(alpha * f, axis=1)
    Q = EPS / (4.0 * np.pi) + (1.0 - EPS) * F
    L = float(-np.mean(np.log(Q)))
    coef = -(1.0 - EPS) / Q / n                       # dL/dp_c with p_c = alpha_c f_c
    # logits: d(sum alpha f)/da_k = alpha_k (f_k - F)
    d_a = coef[:, None] * alpha * (f - F[:, None])
    # directions: d ln f / dv
    inside = (r > K_MIN) & (r < K_MAX)
    rr = np.maximum(r, 1e-300)
    e2 = np.exp(-2.0 * kappa)
    dlnf_dk = 1.0 / kappa - 2.0 * e2 / (-np.expm1(-2.0 * kappa)) + (w - 1.0)
    # d mu / dv applied to s: (s - (mu.s) mu) / r
    dmu_s = (S[:, None, :] - w[:, :, None] * mu) / rr[:, :, None]
    dlnf_dv = (kappa[:, :, None] * dmu_s
               + np.where(inside, dlnf_dk, 0.0)[:, :, None] * mu)
    d_v = (coef[:, None] * alpha * f)[:, :, None] * dlnf_dv
    d_out = np.concatenate([d_v, d_a[:, :, None]], axis=2).reshape(n, 12)
    g = {}
    g["W3"] = d_out.T @ a2
    g["b3"] = d_out.sum(0)
    d_a2 = d_out @ p["W3"]
    d_z2 = d_a2 * (z2 > 0)
    g["W2"] = d_z2.T @ a1
    g["b2"] = d_z2.sum(0)
    d_a1 = d_z2 @ p["W2"]
    d_z1 = d_a1 * (z1 > 0)
    g["W1"] = d_z1.T @ X
    g["b1"] = d_z1.sum(0)
    grad = np.concatenate([g[name].ravel() for name, _ in SHAPES])
    return L, grad


def tangent_basis(mu):
    """Two unit vectors orthogonal to mu (and to each other): e1 from the
    coordinate axis least aligned with mu."""
    mu = np.atleast_2d(mu)
    ax = np.argmin(np.abs(mu), axis=1)
    t = np.zeros_like(mu)
    t[np.arange(len(mu)), ax] = 1.0
    e1 = t - np.sum(t * mu, axis=1, keepdims=True) * mu
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(mu, e1)
    return e1, e2


def sample(out, u_mix, u_w, u_phi, s_uniform):
    """Draw one direction per row: uniform (given) with probability eps, else
    component c (alpha) with w from the vMF inverse CDF and azimuth 2 pi u_phi."""
    kappa, mu, alpha, _ = mixture(out)
    n = out.shape[0]
    cum = np.cumsum(alpha, axis=1)
    um = (u_mix - EPS) / (1.0 - EPS)
    c = np.minimum(np.sum(um[:, None] >= cum, axis=1), 2)
    k = kappa[np.arange(n), c]
    m = mu[np.arange(n), c]
    w = 1.0 + np.log(u_w + (1.0 - u_w) * np.exp(-2.0 * k)) / k
    w = np.clip(w, -1.0, 1.0)
    e1, e2 = tangent_basis(m)
    phi = 2.0 * np.pi * u_phi
    rt = np.sqrt(np.maximum(1.0 - w * w, 0.0))
    s = w[:, None] * m + rt[:, None] * (np.cos(phi)[:, None] * e1 + np.sin(phi)[:, None] * e2)
    return np.where((u_mix < EPS)[:, None], s_uniform, s)
