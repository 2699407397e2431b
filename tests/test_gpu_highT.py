"""Closed-form check of the fast GPU path on the L=8 four-shell lattice,
independent of the oracle.  At infinite temperature the spins are
independent: <E> = 0, Var E = N sum_n z_n J_n^2 / 6 (since
<(S_i.S_j)^2> = 1/3), and the third cumulant comes from bond triangles
only, kappa_3 = -(2/3) sum_triangles J_a J_b J_c (since
<(S1.S2)(S2.S3)(S3.S1)> = 1/9).  Near E = 0 the density of states follows
the Edgeworth form ln g = -x^2/2 + (gamma/6)(x^3 - 3x) + const, x = E/sigma,
gamma = kappa_3 / sigma^3, up to O(1/N).  A converged walk over [-300, 300)
J (about +-7 sigma) must reproduce the curvature (3 %), the slope at E = 0
and the cubic coefficient of a cubic fit."""
import sys

import numpy as np
import pytest

from helpers import gpu_from, progress

pytestmark = pytest.mark.gpu


def _cumulants(L, J):
    """Var E and kappa_3 at infinite temperature for the bcc lattice."""
    from paper_1411_4212_amd.workloads import _bcc_tables
    nbr, Jz = _bcc_tables(L, list(J))
    N = nbr.shape[0]
    adj = [dict() for _ in range(N)]
    var = 0.0
    for i in range(N):
        for k in range(nbr.shape[1]):
            j = int(nbr[i, k])
            if i < j:
                adj[i][j] = Jz[k]
                adj[j][i] = Jz[k]
                var += Jz[k] ** 2 / 3.0
    tri = 0.0
    for i in range(N):
        for j, a in adj[i].items():
            if j <= i:
                continue
            for k, b in adj[j].items():
                if k > j and k in adj[i]:
                    tri += a * b * adj[i][k]
    return var, -(2.0 / 3.0) * tri


@pytest.mark.parametrize("mode", ["fp32_de", "fp64"])
def test_edgeworth_dos_near_zero_energy(mode):
    from paper_1411_4212_amd.analysis import run_lng
    from paper_1411_4212_amd.workloads import J_C2
    N = 1024
    var, k3 = _cumulants(8, J_C2)
    z = np.array([8, 6, 12, 24])
    assert abs(var - N * float(np.sum(z * np.array(J_C2) ** 2)) / 6.0) < 1e-6 * var
    sigma = np.sqrt(var)
    gamma = k3 / sigma ** 3
    cfg = dict(lattice=("bcc", 8, list(J_C2)), windows=(-300.0, 300.0, 120, 2, 0.75, 4),
               schedule=(4, 5, 1.0, 2.0 ** -14, 20000, 100 * N), seed=13)
    g = gpu_from(cfg, mode)
    segs = 0
    while segs < 4000:
        g.run(64)
        segs += 64
        done = g.poll()
        progress("edgeworth %s: %d segments%s" % (mode, segs, " (all done)" if done else ""))
        if done:
            break
    assert g.poll(), "not converged in %d segments" % segs
    bins, lg = run_lng(g, 0)
    E = -300.0 + (bins + 0.5) * 5.0
    m = np.isfinite(lg) & (np.abs(E) < 200)
    x = E[m] / sigma
    c3, c2, c1, _ = np.polyfit(x, lg[m], 3)
    print(mode, "segments", segs, "curvature %.4f (-1)  slope %.4f (%.4f)  cubic %.5f (%.5f)"
          % (2 * c2, c1, -gamma / 2, c3, gamma / 6), flush=True)
    sys.stdout.flush()
    assert abs(2 * c2 + 1.0) < 0.03
    assert abs(c1 + gamma / 2) < 0.04
    assert abs(c3 - gamma / 6) < 0.006
