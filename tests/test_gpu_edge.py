"""Ragged, degenerate and maximum-size inputs through the C ABI.

* Several instances of different lattice size (L a power of two and not),
  window counts, walkers per window, odd bin counts and segment lengths that
  are not multiples of the 64-move batch, in ONE GPU context, against the
  oracle run instance by instance (walker ids and instance index set to the
  GPU's): bit-exact in the deterministic mode, trajectories included.
* Degenerate cases: one window (no exchange partner), one walker, segments
  of a single move, zero segments, a window of one bin.
* Documented maxima: 64 walkers per window and 4096 bins per window run and
  match the oracle; one more of either is rejected with REWL_ERANGE.
"""
import sys

import numpy as np
import pytest

from helpers import bits, gpu_from, progress

pytestmark = pytest.mark.gpu


_say = progress


def _oracle_for(cfg, seed, stream_base, instance, trace=0):
    import oracle
    lat = cfg["lattice"]
    o = oracle.Oracle(L=lat[1], J=lat[2])
    o.set_windows(*cfg["windows"])
    o.set_schedule(*cfg["schedule"])
    o.set_threads(4)
    o.set_ids(stream_base, instance)
    if trace:
        o.set_trace(trace)
    o.init(seed)
    return o


def _compare(o, g, inst, W):
    for w in range(W):
        so, sg = o.walker(w), g.walker(inst, w)
        assert bits(so["E"]) == bits(sg["E"]), (inst, w)
        assert so["bin"] == sg["bin"] and so["cfg"] == sg["config"], (inst, w)
        assert so["lnf"] == sg["lnf"] and so["iter"] == sg["iteration"], (inst, w)
        assert so["attempts"] == sg["attempts"] and so["accepts"] == sg["accepts"], (inst, w)
        assert so["out_of_window"] == sg["rejected_outside"], (inst, w)
        assert np.array_equal(bits(o.lng(w)), bits(g.lng(inst, w))), (inst, w)
        Ho, vo = o.hist(w)
        assert np.array_equal(Ho, g.hist(inst, w)) and np.array_equal(vo, g.visited(inst, w)), (inst, w)
        c = so["cfg"]
        assert np.array_equal(bits(o.config(c)), bits(g.config(inst, c))), (inst, w)
    ao, co = o.exchange_stats()
    ag, cg = g.exchange_stats(inst)
    assert np.array_equal(ao, ag) and np.array_equal(co, cg), inst


RAGGED = [
    dict(lattice=("bcc", 4, [1.0, 0.5]), windows=(-600.0, -100.0, 61, 3, 0.75, 2),
         schedule=(4, 5, 1.0, 2.0 ** -6, 1037, 12800)),
    dict(lattice=("bcc", 6, [1.0, 0.6, -0.05, -0.1]), windows=(-1500.0, -300.0, 50, 2, 0.75, 3),
         schedule=(4, 5, 1.0, 2.0 ** -6, 777, 43200)),
    # one window, one walker, one batch per segment, large ln f steps
    dict(lattice=("bcc", 4, [1.0, 0.5]), windows=(-500.0, -300.0, 7, 1, 0.75, 1),
         schedule=(1, 2, 1.0, 0.25, 64, 12800)),
]


def test_det_ragged_instances_bit_exact():
    seed = 21
    cfgs = [dict(c, seed=seed) for c in RAGGED]
    cap = 2500
    g = gpu_from(cfgs, "fp64_det", trace=cap)
    g.run(6)
    base = 0
    for i, c in enumerate(cfgs):
        W = c["windows"][3] * c["windows"][5]
        o = _oracle_for(c, seed, base, i, trace=cap)
        o.run(6)
        _say("instance", i, "walkers", W)
        _compare(o, g, i, W)
        for w in range(W):
            n = min(cap, 6 * c["schedule"][4])
            to, tg = o.trace(w)[:n], g.trace(base + w)[:n]
            assert np.array_equal(to["site"], tg["site"]) and np.array_equal(to["flags"], tg["flags"])
            assert np.array_equal(bits(to["E"]), bits(tg["E"])) and np.array_equal(to["bin"], tg["bin"])
        base += W


@pytest.mark.parametrize("mode", ["fp32_de", "fp64"])
def test_fast_ragged_instances_invariants(mode):
    """The look-ahead kernel on the ragged instances (non-power-of-two L,
    partial batches): exact move counts, running energy = full energy of
    the held configuration, bins inside the windows, configurations a
    permutation per instance; and the same walk in one persistent launch."""
    import oracle
    cfgs = [dict(c, seed=5) for c in RAGGED]
    g = gpu_from(cfgs, mode)
    g.run(8)
    p = gpu_from(cfgs, mode)
    p.run_persistent(8)
    tol = 2e-3 if mode == "fp32_de" else 1e-9
    for i, c in enumerate(cfgs):
        lat = c["lattice"]
        o = oracle.Oracle(L=lat[1], J=lat[2])
        W = c["windows"][3] * c["windows"][5]
        used = []
        for w in range(W):
            st = g.walker(i, w)
            assert st["attempts"] == 8 * c["schedule"][4] or st["done"]
            S = g.config(i, st["config"])
            Ef = o.energy(S)
            assert abs(Ef - st["E"]) <= tol * 10 * (1 + abs(Ef)) ** 0.5, (i, w, Ef, st["E"])
            lo, hi = g.window(i, w)
            assert lo <= st["bin"] < hi
            used.append(st["config"])
            assert st == p.walker(i, w)
            assert np.array_equal(bits(g.lng(i, w)), bits(p.lng(i, w)))
        assert sorted(used) == list(range(W))


def test_degenerate_calls():
    from paper_1411_4212_amd.rewl import RewlError
    cfg = dict(RAGGED[0], seed=3)
    g = gpu_from(cfg, "fp32_de")
    before = [g.walker(0, w) for w in range(6)]
    g.run(0)
    assert g.step() == 0 and [g.walker(0, w) for w in range(6)] == before
    assert g.run_persistent(0) == 0
    # single-move segments
    one = gpu_from(dict(cfg, schedule=(4, 5, 1.0, 2.0 ** -6, 1, 12800)), "fp32_de")
    one.run(3)
    assert all(one.walker(0, w)["attempts"] == 3 for w in range(6))
    # a window of a single bin: every in-window move stays in it
    tiny = dict(lattice=("bcc", 4, [1.0, 0.5]), windows=(-400.0, -390.0, 1, 1, 0.75, 2),
                schedule=(4, 5, 1.0, 0.5, 500, 12800), seed=3)
    t = gpu_from(tiny, "fp64_det")
    t.run(2)
    for w in range(2):
        st = t.walker(0, w)
        assert st["bin"] == 0 and t.visited(0, w)[0] == 1
    with pytest.raises(RewlError):
        g.run(-1)


def test_maximum_sizes():
    """64 walkers in a window and 4096 bins in a window run bit-exact
    against the oracle; 65 walkers or 4097 bins are rejected."""
    from paper_1411_4212_amd.rewl import RewlError, Run
    seed = 8
    big = dict(lattice=("bcc", 4, [1.0, 0.5]), windows=(-600.0, -100.0, 4096, 1, 0.75, 64),
               schedule=(4, 5, 1.0, 2.0 ** -6, 300, 12800), seed=seed)
    g = gpu_from(big, "fp64_det")
    g.run(2)
    o = _oracle_for(big, seed, 0, 0)
    o.run(2)
    _compare(o, g, 0, 64)
    for win in [(-600.0, -100.0, 4097, 1, 0.75, 1), (-600.0, -100.0, 100, 1, 0.75, 65)]:
        with pytest.raises(RewlError) as e:
            Run([dict(lattice=("bcc", 4, [1.0, 0.5]), windows=win,
                      schedule=(4, 5, 1.0, 0.5, 100, 12800))], mode="fp32_de")
        assert e.value.code == -4, win


def test_round_trips_match_host_count():
    """Half round trips per configuration, counted on the device at every
    exchange step, equal a host recount from the walker states read after
    each step (which configuration sits in the lowest / highest window)."""
    cfg = dict(lattice=("bcc", 4, [1.0, 0.5]), windows=(-600.0, -100.0, 60, 4, 0.75, 2),
               schedule=(4, 5, 1.0, 2.0 ** -20, 2000, 12800), seed=17)
    g = gpu_from(cfg, "fp32_de")
    h, m = 4, 2
    W = h * m
    last = np.zeros(W, dtype=np.int64)
    half = np.zeros(W, dtype=np.int64)
    for _ in range(40):
        g.run(1)
        cf = [g.walker(0, w)["config"] for w in range(W)]
        for win, ext in ((0, 1), (h - 1, 2)):
            for r in range(m):
                c = cf[win * m + r]
                if last[c] != ext:
                    if last[c]:
                        half[c] += 1
                    last[c] = ext
    dev = g.round_trips(0)
    _say("half trips", dev.tolist())
    assert np.array_equal(dev.astype(np.int64), half)
    assert half.sum() > 0


def test_round_trips_det_equal_oracle():
    """Deterministic FP64 mode: the device's half-trip count per
    configuration equals the oracle's, bit for bit, after 300 segments with
    an exchange step each (same Philox seed, so the same swaps)."""
    from helpers import oracle_from
    cfg = dict(lattice=("bcc", 4, [1.0, 0.5]), windows=(-560.0, 160.0, 60, 4, 0.75, 2),
               schedule=(4, 5, 1.0, 2.0 ** -6, 1500, 0), seed=21)
    o = oracle_from(cfg)
    o.run(300)
    g = gpu_from(cfg, "fp64_det")
    g.run(300)
    dev = g.round_trips(0).astype(np.int64)
    ref = o.round_trips().astype(np.int64)
    _say("half trips det", dev.tolist(), ref.tolist())
    assert np.array_equal(dev, ref)
    assert ref.sum() >= 4
