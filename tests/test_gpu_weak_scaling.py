"""The weak-scaling measurement on the GPU (Sec. results, weak-scaling
figure: trial moves until each window's first flat histogram, windows of a
fixed width and overlap): bcc L=30, J = (1, 0.5), 375 windows of 3 J bins,
one walker each, ferromagnetic start.

What the trained network gains here: with the learned proposal (trained on
the device on the first two segments of the plain walk, then used for the
rest) at least 95 % of the windows finish their first iteration within 1e7
moves per walker; the uniform walk finishes at most 80 % by then.  Measured
on two seeds: 100 % against a uniform median of 5.8e6 and q75 of 2.4e7
moves, i.e. between half and three quarters."""
import pytest

from helpers import progress

pytestmark = pytest.mark.gpu


def test_learned_proposal_finishes_the_first_iteration_sooner():
    from paper_1411_4212_amd.weak_scaling import run_one
    cap = 10 ** 7
    res = {}
    for prop in ("learned", "uniform"):
        progress("weak scaling L=30, %s proposal, cap %.0e moves per walker" % (prop, cap))
        r = run_one(30, cap_moves=cap, bin_width=3, proposal=prop, log=progress)
        frac = r["finished"] / r["walkers"]
        progress("%s: %d of %d windows finished, quantiles %s, acceptance %.3f, %.1f s"
                 % (prop, r["finished"], r["walkers"], r["moves_quantiles"], r["acceptance"], r["seconds"]))
        assert r["walkers"] == 375
        res[prop] = frac
    assert res["learned"] >= 0.95
    assert res["uniform"] <= 0.80
