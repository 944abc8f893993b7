"""Pins of the CPU oracle against facts that do not come from the oracle
itself: closed forms of the Heisenberg model, exact invariants, brute-force
properties and an independent Philox implementation (rocRAND's).

Paper passages: Eq. 1-2 (section "Classical spin Hamiltonian") for the energy;
Eq. 4 and the MCS definition (section "Monte Carlo Metropolis algorithm") for
the dynamics; the per-MCS history of energy and magnetisation (section
"VEGAS software package").
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from _stats import block_mean_se, langevin, langevin_var, after_burn_in

EXACT, F32MAP = oracle.PROPOSAL_EXACT, oracle.PROPOSAL_F32MAP


# ---------------------------------------------------------------- P13 Philox
def _rocrand_words(ctr, key):
    exe = "/tmp/hsim_philox_rocrand_ref"
    src = os.path.join(os.path.dirname(__file__), "philox_rocrand_ref.cpp")
    if not os.path.exists(exe) or os.path.getmtime(exe) < os.path.getmtime(src):
        subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-O1", "-o", exe, src],
                              cwd="/tmp")
    lines = "".join("%x %x %x %x %x %x\n" % (*c, *key) for c in ctr)
    out = subprocess.run([exe], input=lines, capture_output=True, text=True, check=True).stdout
    return np.array([[int(w, 16) for w in ln.split()] for ln in out.strip().splitlines()],
                    dtype=np.uint32)


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not found")
def test_p13_philox_matches_rocrand():
    """Philox4x32-10 words equal those of rocRAND's engine (an implementation
    that shares nothing with the oracle) on edge and random counters/keys."""
    rng_words = synth.splitmix64(13, 6 * 200, tag=1).astype(np.uint64)
    ctrs = (rng_words[:800] & np.uint64(0xFFFFFFFF)).astype(np.uint32).reshape(200, 4)
    ctrs[0] = 0
    ctrs[1] = 0xFFFFFFFF
    ctrs[2] = [0xFFFFFFFF, 0xFFFFFFFF, 0, 0]
    for key in ([0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [0x12345678, 0x9ABCDEF0]):
        ref = _rocrand_words(ctrs, key)
        got = oracle.philox(ctrs, key)
        assert np.array_equal(ref, got)


def test_uniform_maps_exact_and_open():
    """u53 and u24 are odd multiples of 2^-53 / 2^-24 strictly inside (0, 1)."""
    assert oracle.u53(0, 0) == 2.0 ** -53
    assert oracle.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert oracle.u24(0) == 2.0 ** -24
    assert oracle.u24(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    # u24 is exactly representable in single precision
    for w in (0, 1, 511, 512, 0x80000000, 0xFFFFFFFF, 0x12345678):
        u = oracle.u24(w)
        assert float(np.float32(u)) == u
        assert float(np.float32(2.0 * u - 1.0)) == 2.0 * u - 1.0


def _sphere_points(n, mode):
    pts = np.empty((n, 3))
    for i in range(n):
        if mode == "exact":
            pts[i], _ = oracle.sphere_exact(7, i, 3, 1)
        else:
            pts[i], _ = oracle.sphere_f32map(7, i, 3, 1)
    return pts


@pytest.mark.parametrize("mode", ["exact", "f32map"])
def test_trial_moves_uniform_on_sphere(mode):
    """Both proposal maps give unit vectors whose moments match the uniform
    distribution on S^2 (Archimedes: z uniform on [-1, 1]; E[x^2] = 1/3)."""
    pts = _sphere_points(20000, mode)
    n = pts.shape[0]
    assert np.allclose(np.linalg.norm(pts, axis=1), 1.0, atol=1e-14)
    se = 1.0 / np.sqrt(n)
    for c in range(3):
        assert abs(pts[:, c].mean()) < 4.5 * se * np.sqrt(1 / 3)
        assert abs((pts[:, c] ** 2).mean() - 1 / 3) < 4.5 * se * np.sqrt(4 / 45)
    counts, _ = np.histogram(pts[:, 2], bins=20, range=(-1, 1))
    chi2 = ((counts - n / 20) ** 2 / (n / 20)).sum()
    assert chi2 < 45.0          # 19 dof, p ~ 1e-3
    phi = np.arctan2(pts[:, 1], pts[:, 0])
    counts, _ = np.histogram(phi, bins=20, range=(-np.pi, np.pi))
    assert ((counts - n / 20) ** 2 / (n / 20)).sum() < 45.0


def test_marsaglia_attempts_geometric():
    """Rejection rate of the exact map is 1 - pi/4."""
    att = np.array([oracle.sphere_exact(5, i, 0, 0)[1] for i in range(20000)])
    acc1 = np.mean(att == 1)
    assert abs(acc1 - np.pi / 4) < 4.5 * np.sqrt(0.17 / att.size)


# ------------------------------------------------------------ validation
def _lat_copy(lat, **kw):
    d = dict(n=lat.n, row_ptr=lat.row_ptr.copy(), col=lat.col.copy(), J=lat.J.copy(),
             k=None if lat.k is None else lat.k.copy(),
             axis=None if lat.axis is None else lat.axis.copy(),
             ndir=None if lat.ndir is None else lat.ndir.copy())
    d.update(kw)
    return synth.Lattice(**d)


def test_validation_rejects_bad_input():
    lat = synth.sc_periodic(4)
    assert oracle.validate(lat) == 0
    bad = _lat_copy(lat)
    bad.J[0] = 2.0                                   # asymmetric constant
    assert oracle.validate(bad) == -3
    bad = _lat_copy(lat)
    bad.col[0] = 0                                   # self loop at site 0
    assert oracle.validate(bad) == -2
    bad = _lat_copy(lat)
    bad.col[1] = bad.col[0]                          # duplicate link
    assert oracle.validate(bad) == -2
    bad = _lat_copy(lat)
    bad.col[0] = lat.n                               # out of range
    assert oracle.validate(bad) == -2
    bad = _lat_copy(lat, k=np.full(lat.n, np.nan))
    assert oracle.validate(bad) == -3
    bad = _lat_copy(lat, axis=np.tile([0.0, 0.0, 1.1], (lat.n, 1)))
    assert oracle.validate(bad) == -3


# ------------------------------------------------------------ P8 colouring
def _bfs_order(lat):
    """Breadth-first visiting order: components by lowest index, neighbours
    queued in CSR order."""
    from collections import deque
    seen = np.zeros(lat.n, dtype=bool)
    order = []
    for root in range(lat.n):
        if seen[root]:
            continue
        seen[root] = True
        q = deque([root])
        while q:
            i = q.popleft()
            order.append(i)
            for j in lat.col[lat.row_ptr[i]:lat.row_ptr[i + 1]]:
                if not seen[j]:
                    seen[j] = True
                    q.append(int(j))
    return order


def _greedy_property(lat, c):
    """Every site of colour c has, among the neighbours visited before it,
    every colour < c (the colour is the smallest free one)."""
    rank = np.empty(lat.n, dtype=np.int64)
    rank[_bfs_order(lat)] = np.arange(lat.n)
    for i in range(lat.n):
        nb = lat.col[lat.row_ptr[i]:lat.row_ptr[i + 1]]
        earlier = set(int(c[j]) for j in nb if rank[j] < rank[i])
        if any(cc not in earlier for cc in range(c[i])):
            return False
    return True


def test_p8_colouring():
    """No link joins two sites of one colour; every colour is the smallest
    free one in breadth-first order; connected bipartite graphs (even periodic
    SC, trees, the sphere cut) get exactly two colours, the SC ones by parity;
    odd cycles and cliques need 3 and 5."""
    sc = synth.sc_periodic(8)
    c, nc = oracle.greedy_colour(sc)
    assert nc == 2 and np.array_equal(c, (sc.pos.sum(axis=1) % 2).astype(np.int32))
    for lat, expect in ((synth.diluted_film(17, 3, seed=5), None),
                        (synth.diluted_film(16, 3, seed=5), None),
                        (synth.random_tree(300, seed=2), 2),
                        (synth.core_shell_ball(R=8, Rc=5), 2),
                        (synth.sc_periodic(6, 4, 8), 2),
                        (synth.from_bonds(3, [0, 1, 0], [1, 2, 2], [1.0, 1.0, 1.0]), 3),
                        (synth.from_bonds(5, *np.triu_indices(5, 1), np.ones(10)), 5)):
        c, nc = oracle.greedy_colour(lat)
        assert oracle.count_conflicts(lat, c) == 0
        assert _greedy_property(lat, c)
        if expect is not None:
            assert nc == expect
    odd = synth.sc_periodic(5, 5, 3)
    c, nc = oracle.greedy_colour(odd)
    assert nc >= 3 and oracle.count_conflicts(odd, c) == 0


def test_p8_conflicting_colouring_rejected():
    lat = synth.sc_periodic(4)
    with pytest.raises(ValueError):
        oracle.run(lat, [1.0], [0.0], 1, seed=0, colour=np.zeros(lat.n, dtype=np.int32))


# ------------------------------------------------------------ P1 Langevin
@pytest.mark.parametrize("proposal", [EXACT, F32MAP])
@pytest.mark.parametrize("x", [0.1, 0.5, 1.0, 2.0, 5.0, 10.0])
def test_p1_langevin(x, proposal):
    """Isolated spins in a field B along z at T = 1: <S_z> = L(x),
    <E>/N = -B L(x), Var(S_z) = 1/x^2 - 1/sinh^2 x (which is also
    d<M_z>/dB / (beta N), the fluctuation estimator), <S_z^2> = 1 - 2L/x."""
    N, M = 4096, 240
    lat = synth.isolated(N)
    r = oracle.run(lat, [1.0], [x], M, seed=101, init="random", proposal=proposal)
    h = after_burn_in(r["history"][0], 1 / 6)
    m, se = block_mean_se(h[:, 3] / N)
    assert abs(m - langevin(x)) <= 4 * se + 1e-12
    e, se_e = block_mean_se(h[:, 0] / N)
    assert abs(e + x * langevin(x)) <= 4 * se_e + 1e-12
    # the final state holds N independent spins: their sample variance
    sz = r["spins"][:, 2]
    dev2 = (sz - langevin(x)) ** 2
    assert abs(dev2.mean() - langevin_var(x)) <= 4 * dev2.std() / np.sqrt(N)
    sz2 = sz ** 2
    assert abs(sz2.mean() - (1 - 2 * langevin(x) / x)) <= 4 * sz2.std() / np.sqrt(N)


# --------------------------------------------------- P2 isolated anisotropic
def _mu_moments(a, b):
    Z = integrate.quad(lambda u: np.exp(a * u * u + b * u), -1, 1)[0]
    m1 = integrate.quad(lambda u: u * np.exp(a * u * u + b * u), -1, 1)[0] / Z
    m2 = integrate.quad(lambda u: u * u * np.exp(a * u * u + b * u), -1, 1)[0] / Z
    return m1, m2


@pytest.mark.parametrize("a,b", [(2.0, 0.0), (-1.5, 0.0), (4.0, 0.0), (3.0, 1.0), (1.0, -2.0)])
def test_p2_isolated_anisotropic(a, b):
    """Isolated spins with per-site random easy axes e_i (k = a, T = 1) and a
    field b along e_i: mu = S.e has density exp(a mu^2 + b mu) on [-1, 1]."""
    N, M = 4096, 240
    axes = synth.unit_vectors(3, N, tag=5)
    lat = synth.isolated(N, k=np.full(N, a), axis=axes, ndir=axes)
    r = oracle.run(lat, [1.0], [b], M, seed=202, init="random")
    m1, m2 = _mu_moments(a, b)
    if b == 0.0:   # closed form of the zero-field second moment
        Z = integrate.quad(lambda u: np.exp(a * u * u), -1, 1)[0]
        assert abs(m2 - (np.exp(a) / (a * Z) - 1 / (2 * a))) < 1e-10
    h = after_burn_in(r["history"][0], 1 / 6)
    e, se = block_mean_se(h[:, 0] / N)
    assert abs(e - (-b * m1 - a * m2)) <= 4 * se
    mu = np.einsum("ij,ij->i", r["spins"], axes)
    assert abs(mu.mean() - m1) <= 4 * mu.std() / np.sqrt(N)
    assert abs((mu ** 2).mean() - m2) <= 4 * (mu ** 2).std() / np.sqrt(N)


# ------------------------------------------------------ P3 trees and chains
def test_p3_tree_energy():
    """On a tree the bond variables are independent (Fisher 1964):
    <E> = -sum_b J_b L(beta J_b), for constants of either sign."""
    lat = synth.random_tree(300, seed=9)
    _, _, Jb = lat.bonds()
    for T in (0.5, 2.0):
        r = oracle.run(lat, [T], [0.0], 3000, seed=303, init="random")
        h = after_burn_in(r["history"][0])
        e, se = block_mean_se(h[:, 0])
        exact = -np.sum(Jb * langevin(Jb / T))
        assert abs(e - exact) <= 4 * se, (T, e, exact, se)


def test_p3_open_chain_magnetisation():
    """Open uniform chain: <|M|^2> = N + 2 sum_r (N - r) u^r, u = L(beta J),
    and <E> = -(N-1) J u."""
    N, T = 48, 0.5
    lat = synth.open_chain(N, J=1.0)
    r = oracle.run(lat, [T], [0.0], 24000, seed=404, init="random")
    h = after_burn_in(r["history"][0], 0.1)
    u = float(langevin(1.0 / T))
    rr = np.arange(1, N)
    m2_exact = N + 2 * np.sum((N - rr) * u ** rr)
    m2, se = block_mean_se((h[:, 1:4] ** 2).sum(axis=1))
    assert abs(m2 - m2_exact) <= 4 * se, (m2, m2_exact, se)
    e, se_e = block_mean_se(h[:, 0])
    assert abs(e + (N - 1) * u) <= 4 * se_e


# --------------------------------------------------------------- P4 beta = 0
def test_p4_infinite_temperature():
    """T = inf: every move is accepted; spins are fresh uniform points each
    MCS, so <|M|^2> = N, <E> = -sum k/3 and
    Var(E) = sum_b J_b^2/3 + B^2 N/3 + (4/45) sum_i k_i^2."""
    lat = synth.diluted_film(12, 3, seed=8)
    lat.k = 2.0 * synth.uniform01(8, lat.n, tag=9)
    lat.axis = synth.unit_vectors(8, lat.n, tag=10)
    Bf = 0.7
    M = 4000
    r = oracle.run(lat, [np.inf], [Bf], M, seed=505, init="random")
    h = r["history"][0]
    assert np.all(h[:, 4] == lat.n)
    N = lat.n
    _, _, Jb = lat.bonds()
    m2 = (h[:, 1:4] ** 2).sum(axis=1)
    assert abs(m2.mean() - N) <= 4 * m2.std() / np.sqrt(M)
    E = h[:, 0]
    assert abs(E.mean() + lat.k.sum() / 3) <= 4 * E.std() / np.sqrt(M)
    var_exact = np.sum(Jb ** 2) / 3 + Bf ** 2 * N / 3 + 4 / 45 * np.sum(lat.k ** 2)
    assert abs(E.var(ddof=1) - var_exact) <= 4 * var_exact * np.sqrt(2 / (M - 1))


# ---------------------------------------------------------- P5 high T
@pytest.mark.parametrize("T", [10.0, 20.0, 50.0])
def test_p5_high_temperature(T):
    """High-T series of the SC ferromagnet (J = 1, each bond once):
    E/N = -1/T + O(T^-3); Curie law 3 <M_z^2>/N = 1 + 2/T + O(T^-2)."""
    lat = synth.sc_periodic(8)
    N = lat.n
    r = oracle.run(lat, [T], [0.0], 3000, seed=606, init="random")
    h = after_burn_in(r["history"][0], 0.1)
    e, se = block_mean_se(h[:, 0] / N)
    assert abs(e + 1 / T) <= 4 * se + 2 / T ** 3, (e, se)
    c, se_c = block_mean_se(3 * h[:, 3] ** 2 / N)
    assert abs(c - (1 + 2 / T)) <= 4 * se_c + 4 / T ** 2, (c, se_c)


# ---------------------------------------------------------- P6 ground state
def test_p6_zero_temperature_cold_start():
    """T = 0 from the aligned state with k, B >= 0 along z: nothing is ever
    accepted and E stays at the full energy -N (3J + k + B)."""
    lat = synth.sc_periodic(8)
    lat.k = np.full(lat.n, 0.1)
    r = oracle.run(lat, [0.0, 0.0], [0.5, 0.25], 10, seed=707, init="cold")
    h = r["history"]
    assert np.all(h[..., 4] == 0)
    assert np.all(r["spins"] == np.array([0.0, 0.0, 1.0]))
    for s, Bf in enumerate((0.5, 0.25)):
        ef = oracle.energy(lat, Bf, r["spins"])["E"]
        assert np.all(h[s, :, 0] == ef)
        assert abs(ef + lat.n * (3 + 0.1 + Bf)) <= 1e-12 * lat.n * 3.6
        assert np.all(h[s, :, 3] == lat.n)


def _watson_sum(L):
    q = 2 * np.pi * np.arange(L) / L
    qx, qy, qz = np.meshgrid(q, q, q, indexing="ij")
    g = (np.cos(qx) + np.cos(qy) + np.cos(qz)) / 3
    d = 1 - g
    d[0, 0, 0] = np.inf
    return np.sum(1 / d) / L ** 3


def test_p6_low_temperature_spin_waves():
    """Harmonic limit of the SC ferromagnet (k = B = 0), cold start:
    E/N + 3 = T (1 - 1/N) + O(T^2) (2N - 2 quadratic modes) and
    1 - <|M|>/N = T W_L / 6 + O(T^2), W_L the lattice sum over q != 0 of
    1/(1 - (cos qx + cos qy + cos qz)/3)/N.  Slopes from a quadratic fit."""
    L = 6
    lat = synth.sc_periodic(L)
    N = lat.n
    Ts = np.array([0.05, 0.1, 0.2])
    e_dev, m_dev, e_se, m_se = [], [], [], []
    for j, T in enumerate(Ts):
        r = oracle.run(lat, [T], [0.0], 12000, seed=808 + j, init="cold")
        h = after_burn_in(r["history"][0], 0.25)
        e, se = block_mean_se(h[:, 0] / N + 3)
        m, sm = block_mean_se(1 - np.linalg.norm(h[:, 1:4], axis=1) / N)
        e_dev.append(e); e_se.append(se); m_dev.append(m); m_se.append(sm)
    A = np.stack([Ts, Ts ** 2], axis=1)
    a_e = np.linalg.lstsq(A, np.array(e_dev), rcond=None)[0][0]
    a_m = np.linalg.lstsq(A, np.array(m_dev), rcond=None)[0][0]
    assert abs(a_e - (1 - 1 / N)) < 0.08, a_e
    assert abs(a_m - _watson_sum(L) / 6) < 0.1 * _watson_sum(L) / 6, (a_m, _watson_sum(L) / 6)


def test_watson_sum_values():
    """The lattice sum converges to Watson's integral 1.516386... as L grows."""
    w = [_watson_sum(L) for L in (8, 32, 64)]
    assert abs(w[0] - 1.347634) < 1e-6
    assert w[0] < w[1] < w[2] < 1.516387


# ------------------------------------------------- P7 incremental vs full
def test_p7_incremental_energy_matches_full_recompute():
    lat = synth.sc_periodic(8)
    T = synth.cooling_schedule(20)[:4]
    r = oracle.run(lat, T, 0.0, 250, seed=0, init="random", full_energy=True)
    assert r["max_incr_err"] <= 1e-12
    lat.k = 0.3 * synth.uniform01(1, lat.n, tag=2)
    lat.axis = synth.unit_vectors(1, lat.n, tag=3)
    r = oracle.run(lat, [1.0, 0.7], [0.4, -0.3], 4, seed=1, init="random",
                   check_every_update=True, full_energy=True)
    assert 0 < r["max_update_err"] <= 1e-13
    assert r["max_incr_err"] <= 1e-13


# ------------------------------------------------ P9 order inside a class
def test_p9_order_inside_class_is_irrelevant():
    lat = synth.diluted_film(11, 3, seed=4)
    perm = np.argsort(synth.uniform01(99, lat.n, tag=7))
    a = oracle.run(lat, [1.0, 0.5], [0.1, 0.0], 30, seed=12, init="random")
    b = oracle.run(lat, [1.0, 0.5], [0.1, 0.0], 30, seed=12, init="random", order=perm)
    assert np.array_equal(a["spins"], b["spins"])
    assert np.array_equal(a["history"][..., 1:], b["history"][..., 1:])
    assert np.allclose(a["history"][..., 0], b["history"][..., 0], rtol=1e-12, atol=0)


# ------------------------------------------------------- history contents
def test_history_bookkeeping_and_resume():
    """n_acc equals the accept trace; M equals the spin sum; resuming from a
    stored state at step s reproduces the uninterrupted run bit for bit."""
    lat = synth.sc_periodic(4)
    T = [2.0, 1.0, 0.5, 0.25]
    full = oracle.run(lat, T, 0.0, 20, seed=21, init="random", trace_accepts=True)
    acc = full["accept"].reshape(4, 20, lat.n)
    assert np.array_equal(full["history"][..., 4], acc.sum(axis=2))
    assert np.allclose(full["history"][-1, -1, 1:4], full["spins"].sum(axis=0), rtol=0,
                       atol=1e-12)
    first = oracle.run(lat, T[:2], 0.0, 20, seed=21, init="random")
    second = oracle.run(lat, T[2:], 0.0, 20, seed=21, init="given", spins=first["spins"],
                        first_step=2)
    assert np.array_equal(second["spins"], full["spins"])
    assert np.array_equal(second["history"], full["history"][2:])


def test_random_start_uses_reserved_counter():
    lat = synth.isolated(16)
    r = oracle.run(lat, [1.0], [0.0], 0, seed=77, init="random", replica=3)
    for i in (0, 5, 15):
        p, _ = oracle.sphere_exact(77, i, 0xFFFFFFFF, 3)
        assert np.array_equal(r["spins"][i], p)


# ------------------------------------------------------------ P11 gradients
def test_p11_gradients_match_central_differences():
    """E is at most quadratic in any one variable, so central differences are
    exact up to rounding."""
    lat = synth.gradient_lattice(L=5, seed=4)
    S = synth.random_spins(3, lat.n)
    Bf = 0.5
    gS, gJ, gk, gB = oracle.energy_grad(lat, Bf, S)
    h = 1e-3
    E = lambda l, b, s: oracle.energy(l, b, s)["E"]
    rng = synth.uniform01(5, 64, tag=1)
    for t in range(16):
        i, c = int(rng[t] * lat.n), t % 3
        Sp, Sm = S.copy(), S.copy()
        Sp[i, c] += h
        Sm[i, c] -= h
        fd = (E(lat, Bf, Sp) - E(lat, Bf, Sm)) / (2 * h)
        assert abs(fd - gS[i, c]) <= 1e-10 * max(1.0, abs(fd))
    _, _, Jb = lat.bonds()
    for t in range(16):
        b = int(rng[16 + t] * Jb.size)
        Jp, Jm = Jb.copy(), Jb.copy()
        Jp[b] += h
        Jm[b] -= h
        fd = (E(lat.with_bond_J(Jp), Bf, S) - E(lat.with_bond_J(Jm), Bf, S)) / (2 * h)
        assert abs(fd - gJ[b]) <= 1e-10 * max(1.0, abs(fd))
    for t in range(16):
        i = int(rng[32 + t] * lat.n)
        lp, lm = _lat_copy(lat), _lat_copy(lat)
        lp.k[i] += h
        lm.k[i] -= h
        fd = (E(lp, Bf, S) - E(lm, Bf, S)) / (2 * h)
        assert abs(fd - gk[i]) <= 1e-10 * max(1.0, abs(fd))
    fd = (E(lat, Bf + h, S) - E(lat, Bf - h, S)) / (2 * h)
    assert abs(fd - gB) <= 1e-10 * max(1.0, abs(fd))
    # dE/dB is minus the field-direction projection of the magnetisation
    assert abs(gB + S[:, 2].sum()) <= 1e-12 * lat.n
