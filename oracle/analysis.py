"""Post-processing of ln g fragments (TEST INFRASTRUCTURE, FP64 numpy).

* Walkers of one window are combined by aligning each to the first walker by
  the mean offset over the bins both visited, then averaging (the paper runs
  several walkers per window to reduce statistical error; Sec. "parallel
  scheme").
* Adjacent windows are joined where the slopes d ln g / dE best coincide
  (Sec. "parallel scheme"): for each overlap the join bin is the interior
  overlap bin (each window's first and last bin excluded) minimising
  |slope_k - slope_{k+1}|, slopes by central differences, ties to the lowest
  bin; window k+1 is shifted to match window k there, window k is used up to
  and including that bin and window k+1 above it.
* Thermodynamics from g(E) (Sec. "background in statistical mechanics"):
  Z = sum_E g(E) exp(-E/T), <E>, C_V = (<E^2> - <E>^2)/T^2 with k_B = 1 and E
  at bin centres, evaluated with log-sum-exp.
"""
import numpy as np


def combine_walkers(lngs, visited):
    """lngs, visited: lists of equal-length arrays for the walkers of one
    window.  Returns (mean ln g, visited-by-any mask)."""
    base = np.asarray(lngs[0], dtype=np.float64)
    vbase = np.asarray(visited[0], dtype=bool)
    acc = np.where(vbase, base, 0.0)
    cnt = vbase.astype(np.float64)
    for lg, vi in zip(lngs[1:], visited[1:]):
        lg = np.asarray(lg, dtype=np.float64)
        vi = np.asarray(vi, dtype=bool)
        common = vi & vbase
        if not common.any():
            continue
        off = np.mean(base[common] - lg[common])
        acc += np.where(vi, lg + off, 0.0)
        cnt += vi
    vis = cnt > 0
    out = np.full(base.shape, np.nan)
    out[vis] = acc[vis] / cnt[vis]
    return out, vis


def join_windows(fragments):
    """fragments: list of (lo, hi, lng[hi-lo], visited[hi-lo]) for windows in
    ascending order.  Returns (bins, lng) over [lo_0, hi_last) with NaN where
    no window has data, and the list of join bins."""
    lo0 = fragments[0][0]
    hi_end = fragments[-1][1]
    glob = np.full(hi_end - lo0, np.nan)
    lo, hi, lg, vi = fragments[0]
    cur = np.where(vi, np.asarray(lg, dtype=np.float64), np.nan)
    glob[lo - lo0:hi - lo0] = cur
    cur_lo, cur_hi = lo, hi
    joins = []
    for (nlo, nhi, nlg, nvi) in fragments[1:]:
        nxt = np.where(nvi, np.asarray(nlg, dtype=np.float64), np.nan)
        best, bstar = None, None
        for b in range(nlo + 1, cur_hi - 1):      # interior overlap bins
            if b - 1 < cur_lo or b + 1 >= nhi:
                continue
            a = glob[b - 1 - lo0:b + 2 - lo0]
            c = nxt[b - 1 - nlo:b + 2 - nlo]
            if np.isnan(a).any() or np.isnan(c).any():
                continue
            s1 = 0.5 * (a[2] - a[0])
            s2 = 0.5 * (c[2] - c[0])
            d = abs(s1 - s2)
            if best is None or d < best:
                best, bstar = d, b
        if bstar is None:
            raise ValueError("windows [%d,%d) and [%d,%d) share no usable overlap"
                             % (cur_lo, cur_hi, nlo, nhi))
        shift = glob[bstar - lo0] - nxt[bstar - nlo]
        nxt = nxt + shift
        glob[bstar + 1 - lo0:nhi - lo0] = nxt[bstar + 1 - nlo:]
        joins.append(bstar)
        cur_lo, cur_hi = nlo, nhi
    return np.arange(lo0, hi_end), glob, joins


def normalise(lng, mask=None):
    """Subtract the mean over the compared (finite) bins."""
    lng = np.asarray(lng, dtype=np.float64)
    m = np.isfinite(lng) if mask is None else (mask & np.isfinite(lng))
    out = np.full(lng.shape, np.nan)
    out[m] = lng[m] - lng[m].mean()
    return out


def thermo(E, lng, T):
    """<E>(T) and C_V(T) from ln g at energies E (finite entries only)."""
    E = np.asarray(E, dtype=np.float64)
    lng = np.asarray(lng, dtype=np.float64)
    m = np.isfinite(lng)
    E, lng = E[m], lng[m]
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    x = lng[None, :] - E[None, :] / T[:, None]
    xm = x.max(axis=1, keepdims=True)
    w = np.exp(x - xm)
    Z = w.sum(axis=1)
    U = (w * E[None, :]).sum(axis=1) / Z
    U2 = (w * (E[None, :] ** 2)).sum(axis=1) / Z
    C = (U2 - U * U) / (T * T)
    return U, C


def cv_peak(E, lng, T_lo, T_hi, n_coarse=400, rel_step=1e-4):
    """Temperature of the C_V maximum: coarse scan, then a fine scan with
    spacing rel_step*T around the coarse maximum, then a parabola through the
    three highest fine points."""
    Tc = np.linspace(T_lo, T_hi, n_coarse)
    _, C = thermo(E, lng, Tc)
    i = int(np.argmax(C))
    i0, i1 = max(i - 1, 0), min(i + 1, n_coarse - 1)
    step = rel_step * Tc[i]
    Tf = np.arange(Tc[i0], Tc[i1] + step, step)
    _, Cf = thermo(E, lng, Tf)
    j = int(np.argmax(Cf))
    if j == 0 or j == len(Tf) - 1:
        return float(Tf[j]), float(Cf[j])
    c0, c1, c2 = Cf[j - 1], Cf[j], Cf[j + 1]
    den = c0 - 2.0 * c1 + c2
    off = 0.0 if den == 0 else 0.5 * (c0 - c2) / den
    return float(Tf[j] + off * step), float(c1)
