"""Read-out post-processing of the ln g~ fragments the walkers return
(Sec. "The parallel scheme"): walkers of a window are combined, adjacent
windows are joined where the slopes of ln g (the inverse microcanonical
temperatures) agree, and thermodynamics follow from the joined g(E)
(Sec. "Background in statistical mechanics").  Host-side numpy, FP64.

Definitions (the same readings the test oracle uses, implemented here on
their own):
  * combine: each walker of a window is shifted by the mean of
    (ln g_0 - ln g_w) over the bins both it and walker 0 visited, and the
    shifted values are averaged bin by bin over the walkers that visited it;
  * join: between windows k and k+1 the join bin b is the bin of the overlap
    (excluding each window's first and last bin) with the bin and both its
    neighbours known in both fragments that minimises |slope_k(b) - slope_{k+1}(b)|, slopes by
    central differences, ties to the lowest b; window k+1 is shifted to agree
    with the joined curve at b and supplies the bins above b;
  * thermodynamics with k_B = 1 and energies at bin centres.
"""
import numpy as np


def combine_walkers(lngs, visited):
    L = np.asarray(lngs, dtype=np.float64)
    V = np.asarray(visited, dtype=bool)
    common = V & V[0]
    n_common = common.sum(axis=1)
    diff = np.where(common, L[0] - L, 0.0).sum(axis=1)
    off = np.divide(diff, n_common, out=np.zeros_like(diff), where=n_common > 0)
    use = V & (n_common > 0)[:, None]
    use[0] = V[0]
    num = np.where(use, L + off[:, None], 0.0).sum(axis=0)
    cnt = use.sum(axis=0)
    vis = cnt > 0
    out = np.full(L.shape[1], np.nan)
    out[vis] = num[vis] / cnt[vis]
    return out, vis


def _slopes(y):
    s = np.full(y.shape, np.nan)
    s[1:-1] = 0.5 * (y[2:] - y[:-2])
    return s


def join_windows(fragments):
    """fragments: [(lo, hi, lng, visited)] in ascending window order.
    Returns (global bin indices, joined ln g with NaN where unknown, join bins)."""
    lo0, hi_end = fragments[0][0], fragments[-1][1]
    out = np.full(hi_end - lo0, np.nan)
    lo, hi, lg, vi = fragments[0]
    out[lo - lo0:hi - lo0] = np.where(vi, lg, np.nan)
    prev_lo, prev_hi = lo, hi
    joins = []
    for lo, hi, lg, vi in fragments[1:]:
        nxt = np.where(vi, np.asarray(lg, dtype=np.float64), np.nan)
        a0, a1 = max(lo + 1, prev_lo + 1), min(prev_hi - 1, hi - 1)
        if a1 <= a0:
            raise ValueError("windows [%d,%d) and [%d,%d) do not overlap" % (prev_lo, prev_hi, lo, hi))
        b = np.arange(a0, a1)
        s_prev = _slopes(out)[b - lo0]
        s_next = _slopes(nxt)[b - lo]
        d = np.abs(s_prev - s_next)
        d[~(np.isfinite(out[b - lo0]) & np.isfinite(nxt[b - lo]))] = np.nan
        if not np.isfinite(d).any():
            raise ValueError("windows [%d,%d) and [%d,%d) share no usable overlap" % (prev_lo, prev_hi, lo, hi))
        bstar = int(b[np.nanargmin(np.where(np.isfinite(d), d, np.nan))])
        nxt = nxt + (out[bstar - lo0] - nxt[bstar - lo])
        out[bstar + 1 - lo0:hi - lo0] = nxt[bstar + 1 - lo:]
        joins.append(bstar)
        prev_lo, prev_hi = lo, hi
    return np.arange(lo0, hi_end), out, joins


def normalise(lng, mask=None):
    lng = np.asarray(lng, dtype=np.float64)
    m = np.isfinite(lng) if mask is None else (np.asarray(mask, dtype=bool) & np.isfinite(lng))
    return lng - lng[m].mean()


def run_lng(run, inst):
    """Joined, normalised ln g of instance `inst` of a Run, on the global bins."""
    h, m = run.inst[inst]["h"], run.inst[inst]["m"]
    frags = []
    for k in range(h):
        ws = range(k * m, (k + 1) * m)
        lo, hi = run.window(inst, k * m)
        lg, vis = combine_walkers([run.lng(inst, w) for w in ws], [run.visited(inst, w) for w in ws])
        frags.append((lo, hi, lg, vis))
    bins, lg, _ = join_windows(frags)
    return bins, normalise(lg)


def thermodynamics(E, lng, T):
    """<E>, C_V at temperatures T from ln g on energies E (NaN bins ignored)."""
    E = np.asarray(E, dtype=np.float64)
    lng = np.asarray(lng, dtype=np.float64)
    ok = np.isfinite(lng)
    E, lng = E[ok], lng[ok]
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    a = lng[None, :] - E[None, :] / T[:, None]
    w = np.exp(a - a.max(axis=1, keepdims=True))
    w /= w.sum(axis=1, keepdims=True)
    U = (w * E).sum(axis=1)
    C = ((w * E * E).sum(axis=1) - U * U) / (T * T)
    return U, C


def cv_peak(E, lng, T_lo, T_hi, n=2000):
    """Temperature and height of the specific-heat maximum on [T_lo, T_hi]:
    grid search, then a parabola through the best point and its neighbours."""
    T = np.linspace(T_lo, T_hi, n)
    _, C = thermodynamics(E, lng, T)
    i = int(np.argmax(C))
    if 0 < i < n - 1:
        y0, y1, y2 = C[i - 1], C[i], C[i + 1]
        den = y0 - 2 * y1 + y2
        if den < 0:
            dx = 0.5 * (y0 - y2) / den
            return T[i] + dx * (T[1] - T[0]), y1 - 0.25 * (y0 - y2) * dx
    return T[i], C[i]
