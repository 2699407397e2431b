"""Pins of the oracle's walker bookkeeping and of its learned-proposal walk.

* The drive into the window (a reading of the paper's arbitrary initial
  configuration, Sec. original WL): from the per-attempt drive records, a move
  is accepted exactly when its energy lies in the window or strictly closer to
  it, the distance falls at every accepted move, and the drive stops at the
  first entry.
* The energy resync: after a segment in which the attempt count crossed a
  multiple of the resync interval, E is the full energy of the walker's
  configuration (brute force over the geometric couplings of Eq. 1) and the
  bin is the clamp of that energy's bin into the window, even after the
  running energy was pushed off by a planted drift.
* Replica round trips (the replica diffusion of Fig. 1): the oracle's count
  per configuration equals the count by definition from the window that
  holds each configuration after every exchange step.
* The learned proposal: its C implementation equals the FP64 numpy reference
  (itself pinned by quadrature and a chi-square test), and a walk with it
  keeps the exact answers: a fixed-weight walk of two spins with the exact
  weights has a flat energy histogram (g is uniform on [-J, J]), and the
  Wang-Landau estimate of that g is flat.

None of the expected values is taken from the oracle itself.
"""
import numpy as np
import pytest


def _bcc_coupling_matrix(L, J):
    """Dense J_ij of the periodic bcc lattice from geometry (half-cell
    coordinates, minimum image), independent of the oracle's tables."""
    N = 2 * L ** 3
    pos = np.zeros((N, 3), dtype=np.int64)
    for s in range(2):
        for z in range(L):
            for y in range(L):
                for x in range(L):
                    pos[((s * L + z) * L + y) * L + x] = (2 * x + s, 2 * y + s, 2 * z + s)
    d = pos[:, None, :] - pos[None, :, :]
    d = (d + L) % (2 * L) - L
    d2 = (d ** 2).sum(-1)
    shell_d2 = [3, 4, 8, 11, 12, 16, 19, 20][: len(J)]
    M = np.zeros((N, N))
    for n, s2 in enumerate(shell_d2):
        M[d2 == s2] = J[n]
    return M


def _energy(M, S):
    return -0.5 * float(np.sum(S * (M @ S)))


def _dist(x, lo, hi):
    return lo - x if x < lo else (x - hi if x >= hi else 0.0)


def test_drive_into_window_rule(oracle_mod):
    """Every recorded drive attempt: accepted iff the proposed energy is in
    the window or strictly closer to it; the energy chain follows the
    accepted moves; the distance strictly falls at each accepted move; the
    drive ends on the first entry and the walker then sits in its bin."""
    L, J = 4, [1.0, 0.5]
    Emin, Emax, B, h = -1024.0, 1024.0, 175, 4
    o = oracle_mod.Oracle(L=L, J=J)
    o.set_windows(Emin, Emax, B, h, 0.75, 2)
    o.set_schedule(4, 5, 1.0, 2.0 ** -10, 1000, 0)
    o.set_threads(2)
    o.set_drive_trace(200000)
    # the ferromagnet lies below windows 1..3: those walkers must be driven
    ferro = np.tile([0.0, 0.0, 1.0], (o.N, 1))
    o.init(4, ferro)
    inv = B / (Emax - Emin)
    M = _bcc_coupling_matrix(L, J)
    driven = 0
    for w in range(o.W):
        lo, hi = o.window(w)
        rec = o.drive(w)
        st = o.walker(w)
        if len(rec) == 0:
            # started inside its window
            assert lo <= (_energy(M, ferro) - Emin) * inv < hi
            continue
        driven += 1
        assert len(rec) < 200000
        assert np.array_equal(rec["attempt"], np.arange(len(rec), dtype=np.uint32))
        E = _energy(M, ferro)
        assert abs(rec["E"][0] - E) < 1e-9
        for k, r in enumerate(rec):
            assert r["E"] == E or k == 0
            xa, xb = (r["E"] - Emin) * inv, (r["Eb"] - Emin) * inv
            inside = lo <= xb < hi
            assert bool(r["flags"] & 2) == inside
            expect = inside or _dist(xb, lo, hi) < _dist(xa, lo, hi)
            assert bool(r["flags"] & 1) == expect
            if expect:
                assert _dist(xb, lo, hi) < _dist(xa, lo, hi) or inside
                E = r["Eb"]
            if inside:
                assert k == len(rec) - 1      # stops on the first entry
        assert rec["flags"][-1] & 3 == 3
        assert st["E"] == rec["Eb"][-1]
        assert st["bin"] == int(np.floor((st["E"] - Emin) * inv))
        assert abs(_energy(M, o.config(st["cfg"])) - st["E"]) < 1e-8
    assert driven >= 3


def test_resync_restores_full_energy_and_clamps_bin(oracle_mod):
    """Walkers whose running energy was moved by a planted drift to an edge
    of the window (so that they keep walking, but with the true energy off
    by the drift) walk one segment; the resync at its end (interval = one
    segment) sets E to the full energy of the configuration and the bin to
    its clamp into the window.  Without a resync the drift stays."""
    L, J = 4, [1.0, 0.5]
    Emin, Emax, B = -420.0, -320.0, 10
    inv = B / (Emax - Emin)
    M = _bcc_coupling_matrix(L, J)
    seg = 10000
    for resync in (seg, 0):
        o = oracle_mod.Oracle(L=L, J=J)
        o.set_windows(Emin, Emax, B, 1, 0.75, 8)
        o.set_schedule(4, 5, 1.0, 2.0 ** -10, seg, resync)
        o.set_threads(2)
        o.init(9)
        o.run(1)
        shifts = []
        for w in range(8):
            E = o.walker(w)["E"]
            d = (Emax - 2.0 - E) if w % 2 == 0 else (Emin + 2.0 - E)
            o.shift_energy(w, d)
            shifts.append(d)
        o.run(1)
        clamped = 0
        for w, d in enumerate(shifts):
            st = o.walker(w)
            lo, hi = o.window(w)
            Ef = _energy(M, o.config(st["cfg"]))
            if resync:
                assert abs(st["E"] - Ef) < 1e-9 * (1.0 + abs(Ef))
                assert st["E"] == o.energy(o.config(st["cfg"]))
                x = (st["E"] - Emin) * inv
                want = lo if x < lo else (hi - 1 if x >= hi else int(np.floor(x)))
                clamped += not (lo <= x < hi)
                assert st["bin"] == want
                assert st["max_drift"] >= abs(d) * (1 - 1e-9)
            else:
                assert abs((st["E"] - Ef) - d) < 1e-6
        if resync:
            assert clamped >= 2


def test_round_trips_by_definition(oracle_mod):
    """A half trip is counted when a configuration reaches one extreme window
    after it was last in the other; the oracle's per-configuration counts
    equal that count taken from the window of each configuration after every
    exchange step."""
    o = oracle_mod.Oracle(L=4, J=[1.0, 0.5])
    h, m = 4, 2
    o.set_windows(-560.0, 160.0, 60, h, 0.75, m)
    o.set_schedule(4, 5, 1.0, 2.0 ** -6, 1500, 0)
    o.set_threads(2)
    o.init(21)
    W = h * m
    last = np.zeros(W, dtype=np.int64)      # 0 none, 1 lowest, 2 highest
    trips = np.zeros(W, dtype=np.int64)
    for _ in range(300):
        o.run(1)
        where = np.empty(W, dtype=np.int64)
        for w in range(W):
            where[o.walker(w)["cfg"]] = w // m
        for c in range(W):
            ext = 1 if where[c] == 0 else (2 if where[c] == h - 1 else 0)
            if ext and last[c] != ext:
                trips[c] += last[c] != 0
                last[c] = ext
    got = o.round_trips()
    assert np.array_equal(got, trips)
    assert trips.sum() >= 4


# ---------------------------------------------------------------- learned
def _theta(scale=3.0, seed=3):
    from oracle import vmf_mlp as V
    th = V.init_params(seed)
    th[64 * 4 + 64 + 64 * 64 + 64:] *= scale     # output layer: concentrations ~1..10
    return th


def test_learned_proposal_matches_fp64_reference(oracle_mod):
    """ln q and the sampler of the oracle's C code equal the numpy FP64
    reference (pinned by quadrature and chi-square in test_oracle_vmf)."""
    from oracle import vmf_mlp as V
    th = _theta()
    rng = np.random.default_rng(1)
    for _ in range(64):
        x = rng.normal(size=4)
        s = rng.normal(size=3)
        s /= np.linalg.norm(s)
        out, _ = V.forward(th, x[None])
        assert abs(oracle_mod.mlp_log_q(th, x, s) - V.log_q(out, s[None])[0]) < 1e-12
        u = rng.random(3)
        uni = rng.normal(size=3)
        uni /= np.linalg.norm(uni)
        ref = V.sample(out, u[:1], u[1:2], u[2:], uni[None])[0]
        assert np.abs(oracle_mod.mlp_sample(th, x, u, uni) - ref).max() < 1e-12


def _two_spins(oracle_mod, B, m, schedule, theta):
    o = oracle_mod.Oracle(explicit=(2, [0], [1], [1.0]))
    o.set_windows(-1.0, 1.0, B, 1, 0.75, m)
    o.set_schedule(*schedule)
    o.set_threads(m)
    o.set_proposal(theta)
    o.init(5)
    return o


def test_learned_fixed_weight_walk_is_exact(oracle_mod):
    """Two spins, the exact weights (g uniform on [-J, J], so ln g~ = 0) held
    fixed: with the learned proposal the stationary histogram of E is flat.
    Each bin's share is compared with 1/B against the spread over batches."""
    B, m = 16, 4
    o = _two_spins(oracle_mod, B, m, (1, 1, 1e-300, 1e-300, 50000, 0), _theta())
    for w in range(m):
        o.write_lng(w, np.zeros(B))
    prev = np.zeros(B)
    shares = []
    for _ in range(12):
        o.run(4)
        H = sum(o.hist(w)[0].astype(np.float64) for w in range(m))
        d = H - prev
        prev = H
        shares.append(d / d.sum())
    A = np.array(shares)
    mean = A.mean(0)
    se = A.std(0, ddof=1) / np.sqrt(len(A))
    z = np.abs(mean - 1.0 / B) / se
    assert z.max() < 5.0
    assert np.abs(mean * B - 1.0).max() < 0.02
    acc = np.mean([o.walker(w)["accepts"] / o.walker(w)["attempts"] for w in range(m)])
    assert 0.05 < acc < 0.95


def test_learned_wang_landau_two_spins_flat(oracle_mod):
    """The Wang-Landau estimate of the two-spin g with the learned proposal is
    flat: each walker's normalised ln g within 0.06, the walkers' mean within
    0.04 (a poorer proposal than the uniform one, hence a larger spread)."""
    from oracle.analysis import normalise
    B, m = 16, 4
    o = _two_spins(oracle_mod, B, m, (4, 5, 1.0, 2.0 ** -14, 50000, 0), _theta())
    o.run_to_convergence(max_segments=4000)
    assert o.all_done()
    lg = np.array([normalise(o.lng(w)) for w in range(m)])
    assert np.abs(lg).max() <= 0.06
    assert np.abs(normalise(lg.mean(0))).max() <= 0.04
