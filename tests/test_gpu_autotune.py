"""Launch-shape autotuner (rewl_autotune): it times every usable walkers-
per-block / residency shape (the persistent form each also at halved
grids while that is faster), restores the walk's state around each trial,
and applies the fastest; the walk that follows is bit-identical to one
that never tuned (the shape and grid do not change results).  A JSON cache
keyed by the configuration digest reapplies the choice without timing."""
import os
import sys

import numpy as np
import pytest

from helpers import bits, gpu_from, progress

pytestmark = pytest.mark.gpu


_say = progress


def _cfgs():
    mk = lambda L, J, win, seed=4: dict(lattice=("bcc", L, J), windows=win,
                                       schedule=(4, 5, 1.0, 2.0 ** -10, 3000, 2 * L ** 3 * 100), seed=seed)
    return [mk(4, [1.0, 0.5], (-600.0, -100.0, 60, 3, 0.75, 2)),
            mk(6, [1.0, 0.6, -0.05, -0.1], (-1500.0, -300.0, 120, 4, 0.75, 3)),
            mk(8, [1.0, 0.6, -0.05, -0.1], (-3500.0, -500.0, 200, 5, 0.75, 2))]


def _state(g, cfgs):
    out = []
    for i, c in enumerate(cfgs):
        for w in range(c["windows"][3] * c["windows"][5]):
            out.append((bits(g.lng(i, w)).tolist(), g.hist(i, w).tolist(), sorted(g.walker(i, w).items())))
    return out


@pytest.mark.parametrize("persistent", [False, True])
def test_autotune_restores_state_and_applies_fastest(persistent, tmp_path):
    cfgs = _cfgs()
    ref = gpu_from(cfgs, "fp32_de")
    ref.run(2)
    g = gpu_from(cfgs, "fp32_de")
    g.run(2)
    before = _state(g, cfgs)
    cache = str(tmp_path / "tune.json")
    trials = g.autotune(segments=2, persistent=persistent, cache=cache)
    _say("trials", trials, "chosen", g.launch())
    full = [t for t in trials if t["max_blocks"] == 0]
    assert len(full) == 6
    if persistent:
        # each usable shape is also timed at half its grid, and halved again
        # (to 1/16 at most) while each step was faster than the one before
        for f in full:
            shape = [t for t in trials if (t["walkers_per_block"], t["residency"]) ==
                     (f["walkers_per_block"], f["residency"])]
            assert shape[0] is f
            if f["status"] != 0:
                assert len(shape) == 1
                continue
            assert 2 <= len(shape) <= 5
            caps = [t["max_blocks"] for t in shape[1:]]
            assert all(c2 == c1 // 2 for c1, c2 in zip(caps, caps[1:]))
            ms = [t["ms_per_segment"] for t in shape]
            assert all(ms[i] < ms[i - 1] for i in range(1, len(ms) - 1))
            assert len(shape) == 5 or ms[-1] >= ms[-2] or caps[-1] // 2 < 1
    else:
        assert len(trials) == 6
    ok = [t for t in trials if t["status"] == 0]
    assert ok and all(t["ms_per_segment"] > 0 for t in ok)
    best = min(ok, key=lambda t: t["ms_per_segment"])
    lc = g.launch()
    assert lc["walkers_per_block"] == best["walkers_per_block"]
    assert lc["spins_in_lds"] == (best["residency"] == 1)
    assert g.grid_cap() == best["max_blocks"]
    assert _state(g, cfgs) == before
    assert g.step() == ref.step()
    ref.run(3)
    if persistent:
        g.run_persistent(3)
    else:
        g.run(3)
    assert _state(g, cfgs) == _state(ref, cfgs)
    # a second context with the same configuration takes the cached shape
    h = gpu_from(cfgs, "fp32_de")
    assert h.autotune(segments=2, persistent=persistent, cache=cache) == []
    assert h.launch() == lc
    assert h.grid_cap() == g.grid_cap()
    # a grid cap leaves results unchanged; rewl_set_launch clears it
    if persistent:
        full_grid = ref.run_persistent(2)
        h.set_grid_cap(max(1, full_grid // 3))
        h.run(5)
        assert h.run_persistent(2) <= max(1, full_grid // 3)
        assert _state(h, cfgs) == _state(ref, cfgs)
        h.set_launch(lc["walkers_per_block"], 1 if lc["spins_in_lds"] else 2)
        assert h.grid_cap() == 0
    assert os.path.exists(cache)
