"""Closed-form check of the fast GPU path on the L=8 four-shell lattice,
independent of the oracle: at infinite temperature the spins are
independent, <E> = 0 and Var E = N sum_n z_n J_n^2 / 6 (since
<(S_i.S_j)^2> = 1/3), so near E = 0 the density of states is Gaussian to
O(1/N): d ln g/dE = -E / Var E.  A converged walk over [-300, 300) J (about
+-7 standard deviations) must reproduce that curvature within 3 % and a
zero slope at E = 0."""
import sys

import numpy as np
import pytest

from helpers import gpu_from

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["fp32_de", "fp64"])
def test_gaussian_dos_near_zero_energy(mode):
    from paper_1411_4212_amd.analysis import run_lng
    from paper_1411_4212_amd.workloads import J_C2
    N = 1024
    cfg = dict(lattice=("bcc", 8, list(J_C2)), windows=(-300.0, 300.0, 120, 2, 0.75, 4),
               schedule=(4, 5, 1.0, 2.0 ** -14, 20000, 100 * N), seed=13)
    g = gpu_from(cfg, mode)
    segs = g.run_to_convergence(max_segments=4000, chunk=64)
    assert g.poll(), "not converged in %d segments" % segs
    bins, lg = run_lng(g, 0)
    E = -300.0 + (bins + 0.5) * 5.0
    z = np.array([8, 6, 12, 24])
    var = N * float(np.sum(z * np.array(J_C2) ** 2)) / 6.0
    m = np.isfinite(lg) & (np.abs(E) < 200)
    a, b, _ = np.polyfit(E[m], lg[m], 2)
    print(mode, "segments", segs, "curvature*Var %.4f  slope*sigma %.4f" % (2 * a * var, b * np.sqrt(var)),
          flush=True)
    sys.stdout.flush()
    assert abs(2 * a * var + 1.0) < 0.03
    assert abs(b * np.sqrt(var)) < 0.03
