"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test names what it pins.  None of them compares the oracle with itself:
expected values come from the paper's printed numbers, closed forms, an
independent implementation run as a black box, or brute force.
"""
import json
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


# ---------------------------------------------------------------- Philox
def _rocrand_probe():
    exe = os.path.join("/tmp", "rewl_rocrand_philox_probe")
    src = os.path.join(GOLDEN, "rocrand_philox_probe.cpp")
    if not os.path.exists(exe) or os.path.getmtime(exe) < os.path.getmtime(src):
        hipcc = shutil.which("hipcc")
        if hipcc is None:
            pytest.skip("hipcc not available to build the rocRAND reference")
        subprocess.check_call([hipcc, "-O1", "-o", exe, src], cwd="/tmp")
    return exe


def test_philox_matches_rocrand_black_box(oracle_mod):
    """Philox4x32-10: oracle == rocRAND's independent engine, random inputs."""
    exe = _rocrand_probe()
    rng = np.random.default_rng(1234)
    rows = []
    for _ in range(200):
        k = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        c[1] %= 2**30   # rocRAND's offset argument is counted in words (x4)
        rows.append((k, c))
    inp = "".join("%d %d %d %d %d %d\n" % (k[0], k[1], c[0], c[1], c[2], c[3]) for k, c in rows)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(x) for x in line.split()] for line in out.strip().splitlines()])
    got = np.array([oracle_mod.philox(c, k) for k, c in rows], dtype=np.int64)
    assert ref.shape == got.shape
    assert np.array_equal(ref, got)


def test_philox_bits_uniform(oracle_mod):
    words = np.concatenate([oracle_mod.philox([i, 0, 3, 1], [0, 5]) for i in range(4000)])
    bits = ((words[:, None] >> np.arange(32)) & 1).astype(float)
    # every bit position has mean 1/2 within 5 sigma
    assert np.all(np.abs(bits.mean(0) - 0.5) < 5 * 0.5 / math.sqrt(len(words)))


# ---------------------------------------------------------------- sphere
def test_sphere_uniform(oracle_mod):
    """Marsaglia's method: |S| = 1, and z uniform on [-1,1] (Archimedes'
    hat-box theorem), azimuth uniform, components mean 0 and variance 1/3."""
    from scipy import stats
    S = np.array([oracle_mod.sphere(0, 7, n) for n in range(20000)])
    assert np.allclose(np.linalg.norm(S, axis=1), 1.0, atol=1e-15)
    assert stats.kstest(S[:, 2], stats.uniform(loc=-1, scale=2).cdf).pvalue > 1e-3
    phi = np.arctan2(S[:, 1], S[:, 0])
    assert stats.kstest(phi, stats.uniform(loc=-np.pi, scale=2 * np.pi).cdf).pvalue > 1e-3
    assert np.all(np.abs(S.mean(0)) < 5 * math.sqrt(1 / 3 / len(S)))
    assert np.allclose((S ** 2).mean(0), 1 / 3, atol=0.01)


# ---------------------------------------------------------------- exp
def test_exp_det_accuracy(oracle_mod):
    xs = np.concatenate([-np.logspace(-12, np.log10(699), 3000), [0.0, -1e-300, -0.5, -1.0]])
    for x in xs:
        ref = math.exp(x)
        got = oracle_mod.exp_det(x)
        assert abs(got - ref) <= 4e-16 * ref + 1e-300, (x, got, ref)
    assert oracle_mod.exp_det(-800.0) == 0.0


# ---------------------------------------------------------------- lattice
def test_bcc_shell_table(oracle_mod):
    """bcc shells from lattice geometry: squared lengths (half-cell units)
    3,4,8,11,12,16,19,20 with 8,6,12,24,8,6,24,24 members (nearest and next
    nearest are the first two; Model section)."""
    d, sh = oracle_mod.bcc_shells(8)
    assert np.bincount(sh).tolist() == [8, 6, 12, 24, 8, 6, 24, 24]
    d2 = (d ** 2).sum(1)
    for n, expect in enumerate([3, 4, 8, 11, 12, 16, 19, 20]):
        assert np.all(d2[sh == n] == expect)
    # lexicographic order within each shell
    for n in range(8):
        rows = [tuple(r) for r in d[sh == n]]
        assert rows == sorted(rows)


def _bcc_positions(L):
    pos = np.zeros((2 * L ** 3, 3), dtype=np.int64)
    for s in range(2):
        for z in range(L):
            for y in range(L):
                for x in range(L):
                    i = ((s * L + z) * L + y) * L + x
                    pos[i] = (2 * x + s, 2 * y + s, 2 * z + s)
    return pos


@pytest.mark.parametrize("L,J", [(4, [1.0, 0.5]), (5, [1.0, 0.6, -0.05, -0.1]),
                                 (6, [1.0, 0.55, 0.3, 0.17, 0.09, -0.05, -0.03, -0.015])])
def test_bcc_neighbours_geometric(oracle_mod, L, J):
    """Neighbour lists equal the brute-force set of sites at the shell
    distances under periodic minimum image, with the shell's coupling; the
    relation is symmetric; N = 2 L^3 (Model section)."""
    o = oracle_mod.Oracle(L=L, J=J)
    N = 2 * L ** 3
    assert o.N == N
    pos = _bcc_positions(L)
    shell_d2 = [3, 4, 8, 11, 12, 16, 19, 20][: len(J)]
    rng = np.random.default_rng(L)
    for i in rng.choice(N, size=min(N, 40), replace=False):
        dvec = pos - pos[i]
        dvec = (dvec + L) % (2 * L) - L       # minimum image in half-cell units
        d2 = (dvec ** 2).sum(1)
        nb, Jn = o.neighbours(int(i))
        assert len(nb) == len(set(nb.tolist()))
        expect = {}
        for n, s2 in enumerate(shell_d2):
            for j in np.nonzero(d2 == s2)[0]:
                expect[int(j)] = J[n]
        assert set(nb.tolist()) == set(expect)
        for j, Jv in zip(nb.tolist(), Jn.tolist()):
            assert Jv == expect[j]
            assert int(i) in o.neighbours(j)[0].tolist()


def test_energy_bruteforce_and_ferro(oracle_mod):
    """E = -sum_{i<j} J_ij S_i.S_j (Model, Eq. 1) by brute force over all pairs
    with geometric neighbour detection; the ferromagnet has E = -N/2 sum z_n J_n."""
    L, J = 4, [1.0, 0.5]
    o = oracle_mod.Oracle(L=L, J=J)
    N = o.N
    rng = np.random.default_rng(5)
    S = rng.normal(size=(N, 3))
    S /= np.linalg.norm(S, axis=1, keepdims=True)
    pos = _bcc_positions(L)
    E = 0.0
    for i in range(N):
        dvec = (pos[i + 1:] - pos[i] + L) % (2 * L) - L
        d2 = (dvec ** 2).sum(1)
        Jij = np.where(d2 == 3, J[0], np.where(d2 == 4, J[1], 0.0))
        E -= np.sum(Jij * (S[i + 1:] @ S[i]))
    assert abs(o.energy(S) - E) < 1e-9
    ferro = np.tile([0.0, 0.0, 1.0], (N, 1))
    assert o.energy(ferro) == -0.5 * N * (8 * 1.0 + 6 * 0.5)


def test_explicit_chain_energy(oracle_mod):
    N = 6
    pi = np.arange(N - 1)
    o = oracle_mod.Oracle(explicit=(N, pi, pi + 1, np.full(N - 1, 1.3)))
    rng = np.random.default_rng(0)
    S = rng.normal(size=(N, 3))
    S /= np.linalg.norm(S, axis=1, keepdims=True)
    E = -1.3 * sum(S[k] @ S[k + 1] for k in range(N - 1))
    assert abs(o.energy(S) - E) < 1e-12
    h = o.local_field(S, 2)
    assert np.allclose(h, 1.3 * (S[1] + S[3]), atol=1e-15)


# ---------------------------------------------------------------- windows
def test_window_arithmetic_matches_paper(oracle_mod):
    """Window layout (parallel scheme): with the paper's L=10 run (380 eV,
    h=11, o=0.75) the window width is the printed 108.57 eV, and keeping that
    width and overlap for L=40 (24320 eV) needs the printed 893 windows."""
    g = json.load(open(os.path.join(GOLDEN, "paper_windows.json")))
    a = g["l10"]
    rng_e = a["E_max"] - a["E_min"]
    B = 3500                      # bin width 380/3500 eV
    lo0, hi0 = oracle_mod.window_bins(B, a["h"], a["overlap"], 0)
    lo1, hi1 = oracle_mod.window_bins(B, a["h"], a["overlap"], 1)
    lok, hik = oracle_mod.window_bins(B, a["h"], a["overlap"], a["h"] - 1)
    de = rng_e / B
    width = (hi0 - lo0) * de
    assert abs(width - g["window_width_printed"]) < 0.005
    assert abs((lo1 - lo0) * de - (1 - a["overlap"]) * width) < 1e-9
    assert lo0 == 0 and hik == B
    b = g["l40"]
    span = b["E_max"] - b["E_min"]
    h40 = 1 + (span / width - 1) / (1 - b["overlap"])
    assert round(h40) == b["h_printed"]
    B40 = int(round(span / de))
    lo, hi = oracle_mod.window_bins(B40, b["h_printed"], b["overlap"], 0)
    assert abs((hi - lo) * de - width) < 1e-6
    lo, hi = oracle_mod.window_bins(B40, b["h_printed"], b["overlap"], b["h_printed"] - 1)
    assert hi == B40
    m = g["model_sizes"]
    for L, N in zip(m["L"], m["N"]):
        assert oracle_mod.Oracle(L=L, J=[1.0]).N == N if L <= 10 else 2 * L ** 3 == N


def test_window_bins_configs(oracle_mod):
    assert [oracle_mod.window_bins(175, 4, 0.75, k) for k in range(4)] == \
        [(0, 100), (25, 125), (50, 150), (75, 175)]
    w = [oracle_mod.window_bins(2000, 16, 0.75, k) for k in range(16)]
    assert all(hi - lo == 421 for lo, hi in w)
    assert w[0][0] == 0 and w[-1][1] == 2000
    for (lo, hi), (lo2, hi2) in zip(w, w[1:]):
        assert 0.74 < (hi - lo2) / 421 < 0.76


# ---------------------------------------------------------------- acceptance
def _icosahedron():
    p = (1 + 5 ** 0.5) / 2
    v = []
    for a in (-1, 1):
        for b in (-1, 1):
            v += [(0, a, b * p), (a, b * p, 0), (b * p, 0, a)]
    v = np.array(v, dtype=float)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("n_spins", [2, 3, 4])
def test_detailed_balance_exhaustive(oracle_mod, n_spins):
    """Exhaustive detailed balance on n spins with directions restricted to
    the 12 icosahedron vertices: with frozen random ln g~ per bin, the move
    'random site, new direction uniform on the set' accepted by the oracle's
    Wang-Landau acceptance satisfies pi(X) T(X,Y) = pi(Y) T(Y,X) for
    pi ~ 1/g~(E) (Sec. original WL, acceptance min(1, g~(E_A)/g~(E_B)))."""
    D = _icosahedron()
    nd = len(D)
    pairs = [(k, k + 1, 1.0 - 0.3 * k) for k in range(n_spins - 1)]
    if n_spins >= 3:
        pairs.append((0, n_spins - 1, -0.45))
    o = oracle_mod.Oracle(explicit=(n_spins, [p[0] for p in pairs], [p[1] for p in pairs],
                                    [p[2] for p in pairs]))
    idx = np.array(np.meshgrid(*[np.arange(nd)] * n_spins, indexing="ij")).reshape(n_spins, -1).T
    E = np.array([o.energy(D[s]) for s in idx])
    Emin, Emax, B = E.min() - 1e-9, E.max() + 1e-9, 9
    bins = np.floor((E - Emin) * (B / (Emax - Emin))).astype(int)
    rng = np.random.default_rng(n_spins)
    lng = rng.normal(scale=2.0, size=B)
    P = np.array([[oracle_mod.wl_accept_prob(lng[a], lng[b]) for b in range(B)] for a in range(B)])
    logpi = -lng[bins]
    nS = len(idx)
    pw = nd ** np.arange(n_spins)
    code = idx @ pw                      # state X has code X (meshgrid order)
    assert np.array_equal(np.sort(code), np.arange(nS))
    pos = np.empty(nS, dtype=np.int64)
    pos[code] = np.arange(nS)
    worst = 0.0
    T = np.zeros((nS, nS)) if n_spins <= 3 else None
    for i in range(n_spins):
        for d in range(nd):
            Ynew = idx.copy()
            Ynew[:, i] = d
            Y = pos[Ynew @ pw]
            pf = P[bins, bins[Y]]
            pb = P[bins[Y], bins]
            worst = max(worst, np.max(np.abs((logpi + np.log(pf)) - (logpi[Y] + np.log(pb)))))
            if T is not None:
                np.add.at(T, (np.arange(nS), Y), pf / (n_spins * nd))
    assert worst < 1e-12
    if n_spins <= 3:
        T[np.arange(nS), np.arange(nS)] += 1.0 - T.sum(1)
        pi = np.exp(logpi - logpi.max())
        pi /= pi.sum()
        assert np.max(np.abs(pi @ T - pi)) < 1e-12 * pi.max() * 10


def test_detailed_balance_replica_exchange(oracle_mod):
    """Replica exchange (Sec. parallel scheme): for two walkers with
    different frozen ln g~, the swap acceptance satisfies detailed balance
    for the product weight 1/(g_i(E_X) g_j(E_Y))."""
    rng = np.random.default_rng(9)
    lgi = rng.normal(scale=3, size=12)
    lgj = rng.normal(scale=3, size=12)
    for a in range(12):
        for b in range(12):
            # walker i holds energy bin a, walker j bin b
            p_fwd = oracle_mod.re_accept_prob(lgi[a], lgi[b], lgj[b], lgj[a])
            p_bwd = oracle_mod.re_accept_prob(lgi[b], lgi[a], lgj[a], lgj[b])
            lhs = -(lgi[a] + lgj[b]) + math.log(p_fwd)
            rhs = -(lgi[b] + lgj[a]) + math.log(p_bwd)
            assert abs(lhs - rhs) < 1e-12
            assert 0.0 < p_fwd <= 1.0


# ---------------------------------------------------------------- runs
def _explicit_run(oracle_mod, N, pairs, Erange, B, h, m, lnf_final, seed=1, seg=2000):
    pi, pj, pJ = zip(*pairs)
    o = oracle_mod.Oracle(explicit=(N, pi, pj, pJ))
    o.set_windows(Erange[0], Erange[1], B, h, 0.75, m)
    o.set_schedule(4, 5, 1.0, lnf_final, seg, 0)
    o.set_threads(4)
    o.init(seed)
    o.run_to_convergence(max_segments=200000)
    assert o.all_done()
    return o


def _joined(oracle_mod, o):
    from oracle.analysis import combine_walkers, join_windows
    frags = []
    for k in range(o.h):
        ws = range(k * o.m, (k + 1) * o.m)
        lo, hi = o.window(k * o.m)
        lg, vis = combine_walkers([o.lng(w) for w in ws], [o.hist(w)[1] for w in ws])
        frags.append((lo, hi, lg, vis))
    return join_windows(frags)


def test_two_spin_dos_is_uniform(oracle_mod):
    """Two spins: E = -J S1.S2 with S1.S2 uniform on [-1,1] (Archimedes), so
    g(E) is flat on [-J, J]; the normalised REWL ln g must be flat within
    0.02 in every bin."""
    from oracle.analysis import normalise
    o = _explicit_run(oracle_mod, 2, [(0, 1, 1.0)], (-1.0, 1.0), 40, 2, 2, 2.0 ** -18,
                      seg=400000)
    bins, lg, _ = _joined(oracle_mod, o)
    assert np.isfinite(lg).all()
    assert np.max(np.abs(normalise(lg))) <= 0.02


def test_open_chain_dos_irwin_hall_and_energy(oracle_mod):
    """Open Heisenberg chain of N spins: E = -J sum_k c_k with c_k iid
    uniform on [-1,1], so g is the density of a shifted, scaled Irwin-Hall
    sum of N-1 terms; the bin integrals fix ln g.  U(T) from the closed form
    Z ~ (sinh(bJ)/(bJ))^(N-1): U = -(N-1) J (coth(bJ) - 1/(bJ)).  Compared on
    bins whose exact mass is not tiny."""
    from scipy import stats
    from oracle.analysis import normalise, thermo
    N, J = 5, 1.0
    n = N - 1
    Emin, Emax, B = -4.0, 4.0, 64
    o = _explicit_run(oracle_mod, N, [(k, k + 1, J) for k in range(n)], (Emin, Emax), B, 3, 2,
                      2.0 ** -18, seg=200000)
    bins, lg, _ = _joined(oracle_mod, o)
    edges = Emin + (Emax - Emin) * np.arange(B + 1) / B
    # E = -J(2 IH - n)  ->  IH = (n - E/J)/2 ; mass of bin [e0,e1]
    ih = stats.irwinhall(n)
    mass = ih.cdf((n - edges[:-1] / J) / 2) - ih.cdf((n - edges[1:] / J) / 2)
    ok = mass > 1e-4 * mass.max()
    ref = normalise(np.log(mass), ok)
    got = normalise(lg, ok)
    assert np.nanmax(np.abs(got[ok] - ref[ok])) <= 0.05
    # thermodynamics (k_B = 1) at temperatures where the binning is fine
    T = np.linspace(0.6, 5.0, 12)
    Ec = 0.5 * (edges[:-1] + edges[1:])
    U, _ = thermo(Ec, lg, T)
    b = J / T
    Uex = -n * J * (1 / np.tanh(b) - 1 / b)
    assert np.max(np.abs(U - Uex)) < 0.03 * n


def test_incremental_energy_equals_full(oracle_mod):
    """Running energy (E += dE per accepted move) equals a full recompute
    after every accepted move, to rounding."""
    o = oracle_mod.Oracle(L=4, J=[1.0, 0.5])
    o.set_windows(-1024.0, 1024.0, 175, 4, 0.75, 1)
    o.set_schedule(4, 5, 1.0, 2.0 ** -10, 2000, 0)
    o.set_check_energy(True)
    o.set_threads(1)
    o.init(3)
    o.run(3)
    assert 0.0 < o.max_check_err() < 1e-9
    for w in range(4):
        st = o.walker(w)
        assert abs(o.energy(o.config(st["cfg"])) - st["E"]) < 1e-9


def test_schedule_and_thread_independence(oracle_mod):
    """ln f = 2^-k after k flat iterations (f -> sqrt f, ln f0 = 1); results
    do not depend on the thread count; exchanges permute configurations."""
    runs = []
    for th in (1, 4):
        o = oracle_mod.Oracle(L=4, J=[1.0, 0.5])
        o.set_windows(-600.0, 0.0, 60, 3, 0.75, 2)
        o.set_schedule(4, 5, 1.0, 2.0 ** -6, 4000, 50000)
        o.set_threads(th)
        o.init(11)
        o.run(300)
        runs.append(o)
    a, b = runs
    for w in range(a.W):
        sa, sb = a.walker(w), b.walker(w)
        assert sa == sb
        assert np.array_equal(a.lng(w), b.lng(w))
        assert sa["lnf"] == 2.0 ** -sa["iter"]
    assert max(a.walker(w)["iter"] for w in range(a.W)) >= 2
    cfgs = sorted(a.walker(w)["cfg"] for w in range(a.W))
    assert cfgs == list(range(a.W))
    att, acc = a.exchange_stats()
    assert att.sum() > 0 and acc.sum() > 0


def test_detailed_balance_learned_proposal(oracle_mod):
    """Exhaustive detailed balance for an asymmetric proposal: 3 spins on the
    icosahedron directions, the new direction drawn from a categorical q that
    depends on the site's neighbour field (not on the moved spin), accepted
    by the oracle's q-ratio acceptance; pi ~ 1/g~(E) is reversible."""
    D = _icosahedron()
    nd = len(D)
    n = 3
    pairs = [(0, 1, 1.0), (1, 2, 0.7), (0, 2, -0.45)]
    o = oracle_mod.Oracle(explicit=(n, [p[0] for p in pairs], [p[1] for p in pairs],
                                    [p[2] for p in pairs]))
    idx = np.array(np.meshgrid(*[np.arange(nd)] * n, indexing="ij")).reshape(n, -1).T
    E = np.array([o.energy(D[s]) for s in idx])
    Emin, Emax, B = E.min() - 1e-9, E.max() + 1e-9, 7
    bins = np.floor((E - Emin) * (B / (Emax - Emin))).astype(int)
    rng = np.random.default_rng(2)
    lng = rng.normal(scale=2.0, size=B)
    pw = nd ** np.arange(n)
    worst = 0.0
    for X in range(len(idx)):
        S = D[idx[X]]
        for i in range(n):
            h = o.local_field(S, i)
            logits = 2.5 * (D @ h)             # favours directions along the field
            lq = logits - np.log(np.sum(np.exp(logits)))
            for d in range(nd):
                Yi = idx[X].copy()
                Yi[i] = d
                Y = int(Yi @ pw)
                old = idx[X][i]
                pf = oracle_mod.wl_accept_prob_q(lng[bins[X]], lng[bins[Y]], lq[old], lq[d])
                pb = oracle_mod.wl_accept_prob_q(lng[bins[Y]], lng[bins[X]], lq[d], lq[old])
                fwd = -lng[bins[X]] + lq[d] + np.log(pf)
                bwd = -lng[bins[Y]] + lq[old] + np.log(pb)
                worst = max(worst, abs(fwd - bwd))
    assert worst < 1e-12
