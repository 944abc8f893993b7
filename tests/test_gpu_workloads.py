"""The five workloads on the GPU, at (or close to) their full sizes, checked
against the CPU oracle on sampled outputs, on statistics, or on properties that
hold at any size.  All calls go through the C-ABI."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1803_07030_amd import hsim
from _ties import check_one_mcs
from _stats import block_mean_se, langevin_var
from _fp32 import grad_bounds

pytestmark = pytest.mark.gpu


def _start_fp32(lat, seed, rep):
    """The random start of replica rep, computed by the oracle in double and
    rounded to single precision (what the FP32 path starts from)."""
    r = oracle.run(lat, [1.0], [0.0], 0, seed=seed, replica=rep, init="random")
    return r["spins"].astype(np.float32).astype(np.float64)


# ------------------------------------------------------------------ C1
@pytest.mark.parametrize("launch", [hsim.LAUNCH_PLAIN, hsim.LAUNCH_GRAPH, hsim.LAUNCH_PERSISTENT])
def test_c1_full_size_start_and_one_mcs(launch):
    """SC 64^3, K = 0.1 z, 64 replicas at T = 0.1..3.0, FP32, replica-lane
    layout, in the launch modes bench.py times: the device's random start
    equals the oracle's (rounded to single precision) bit for bit, and one MCS
    agrees site by site on sampled replicas."""
    lat = synth.sc_periodic(64)
    lat.k = np.full(lat.n, 0.1)
    R, seed = 64, 1
    T = synth.replica_temperatures(R, 0.1, 3.0)
    plan = hsim.Plan(lat)
    b = hsim.Batch([plan] * R, seed=seed, precision=hsim.FP32, layout=hsim.LAYOUT_REPLICA).bind(1, 1)
    assert b.layout == "replica"
    b.init_spins(hsim.INIT_RANDOM)
    torch.cuda.synchronize()
    sampled = (0, 31, 63)
    starts = {r: _start_fp32(lat, seed, r) for r in sampled}
    for r in sampled:
        assert np.array_equal(b.spins_user(r).cpu().numpy(), starts[r])
    b.run(T[:, None], 0.0, launch=launch)
    torch.cuda.synchronize()
    assert b.status() == 0
    h = b.history.cpu().numpy()
    colour = plan.colouring()
    for r in sampled:
        got = b.spins_user(r).cpu().numpy()
        check_one_mcs(lat, colour, starts[r], T[r], 0.0, seed, r, got, spin_tol=2e-6)
        assert abs(h[r, 0, 0, 4] - np.sum(np.any(got != starts[r], axis=1))) == 0
        ef = oracle.energy(lat, 0.0, got)["E"]
        assert abs(h[r, 0, 0, 0] - ef) <= 1e-5 * 3 * lat.n


# --------------------------------------------------------- FP32 statistics
def test_fp32_statistics_match_oracle_sampler():
    """FP32 replica-lane chains vs independent FP64 oracle chains (other
    replica ids): per-temperature <E>/N, <|M|>/N and acceptance within 4
    combined standard errors (block means, then the spread of replicas)."""
    lat = synth.sc_periodic(8)
    lat.k = np.full(lat.n, 0.1)
    N = lat.n
    temps = [0.6, 1.0, 2.0, 3.0]
    per = 4
    T = np.repeat(temps, per)
    R, M = T.size, 3000
    plan = hsim.Plan(lat)
    b = hsim.Batch([plan] * R, seed=5, precision=hsim.FP32, layout=hsim.LAYOUT_REPLICA).bind(1, M)
    b.init_spins(hsim.INIT_COLD_Z)
    b.run(T[:, None], 0.0, launch=hsim.LAUNCH_GRAPH)
    torch.cuda.synchronize()
    hg = b.history.cpu().numpy()[:, 0, M // 5:, :]
    jobs = [dict(lat=lat, T=[t], B=[0.0], mcs_per_step=M, seed=5, replica=1000 + i, init="cold")
            for i, t in enumerate(T)]
    res, _ = oracle.run_replicas(jobs)
    ho = np.stack([x["history"][0, M // 5:, :] for x in res])

    def obs(h):
        return {"E": h[..., 0] / N, "absM": np.linalg.norm(h[..., 1:4], axis=-1) / N,
                "acc": h[..., 4] / N}

    og, oo = obs(hg), obs(ho)
    worst = 0.0
    for ti, t in enumerate(temps):
        sl = slice(ti * per, (ti + 1) * per)
        for key in og:
            mg = [block_mean_se(x) for x in og[key][sl]]
            mo = [block_mean_se(x) for x in oo[key][sl]]
            mu_g, se_g = np.mean([m for m, _ in mg]), np.sqrt(np.sum([s ** 2 for _, s in mg])) / per
            mu_o, se_o = np.mean([m for m, _ in mo]), np.sqrt(np.sum([s ** 2 for _, s in mo])) / per
            z = abs(mu_g - mu_o) / np.sqrt(se_g ** 2 + se_o ** 2 + 1e-30)
            worst = max(worst, z)
            assert z <= 4.0, (t, key, mu_g, mu_o, se_g, se_o)
    assert worst <= 4.0


# ------------------------------------------------------------------ C2
def test_c2_sphere_full_size():
    """Core/shell sphere R = 20 (33,401 sites; 2 colours), 32 seeds, FP32,
    lane width 32: the accept count of the first MCS from the aligned start at
    B = +2 matches the oracle's on sampled seeds (up to near-tie decisions); a
    short field sweep keeps unit spins, a magnetisation equal to the spin sum
    and an incremental energy that matches a double-precision recompute."""
    lat = synth.core_shell_ball()
    plan = hsim.Plan(lat)
    assert plan.info.n_colours == 2
    R = 32
    ids = np.arange(R, dtype=np.uint32)
    B_sweep = np.array([2.0, 1.0, 0.0, -1.0, -2.0])
    b = hsim.Batch([plan] * R, seed=2, replica_ids=ids, precision=hsim.FP32,
                   layout=hsim.LAYOUT_REPLICA).bind(len(B_sweep), 40)
    b.init_spins(hsim.INIT_COLD_Z)
    cold = np.tile([0.0, 0.0, 1.0], (lat.n, 1))
    # first step only, then compare one MCS
    b.run(np.full((R, 1), 0.1), B_sweep[:1][None, :].repeat(R, 0), recompute_every=10)
    torch.cuda.synchronize()
    h = b.history.cpu().numpy()
    assert b.status() == 0
    # the first MCS from the aligned start, site by site (a second batch
    # stopped after one MCS gives the spins)
    one = hsim.Batch([plan] * R, seed=2, replica_ids=ids, precision=hsim.FP32,
                     layout=hsim.LAYOUT_REPLICA).bind(1, 1)
    one.init_spins(hsim.INIT_COLD_Z)
    one.run(np.full((R, 1), 0.1), np.full((R, 1), 2.0), recompute_every=10)
    torch.cuda.synchronize()
    colour = plan.colouring()
    for r in (0, 17):
        got = one.spins_user(r).cpu().numpy()
        check_one_mcs(lat, colour, cold, 0.1, 2.0, 2, r, got, spin_tol=2e-6)
        assert int(h[r, 0, 0, 4]) == int(np.sum(np.any(got != cold, axis=1)))
    b.run(np.full((R, 4), 0.1), B_sweep[1:][None, :].repeat(R, 0), first_step=1,
          recompute_every=10)
    torch.cuda.synchronize()
    assert b.status() == 0
    h = b.history.cpu().numpy()
    for r in (0, 9, 31):
        s = b.spins_user(r).cpu().numpy()
        assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=2e-6)
        assert np.allclose(h[r, -1, -1, 1:4], s.sum(axis=0), rtol=0, atol=1e-6 * lat.n)
        e = oracle.energy(lat, -2.0, s)
        assert abs(h[r, -1, -1, 0] - e["E"]) <= 1e-5 * e["scale"]
    assert np.all(h[:, 0, -1, 3] > 0)
    del cold


# ------------------------------------------------------------------ C3
def test_c3_uneven_film_batch_fp64_bit_exact():
    """An uneven batch of diluted films (odd and even L: 2 to 6 colours, one
    batch, site layout, FP64): every film equals its own oracle run bit for
    bit."""
    films = [synth.diluted_film(L, d, seed=100 + i)
             for i, (L, d) in enumerate([(16, 2), (17, 3), (23, 5), (30, 2), (19, 4), (40, 3)])]
    plans = [hsim.Plan(f) for f in films]
    Ts = np.array([0.3, 0.9, 1.4, 2.0, 0.6, 1.1])
    b = hsim.Batch(plans, seed=3, precision=hsim.FP64_EXACT, layout=hsim.LAYOUT_SITE).bind(1, 6)
    b.init_spins(hsim.INIT_COLD_Z)
    b.run(Ts[:, None], 0.0)
    torch.cuda.synchronize()
    H = b.history.cpu().numpy()
    for r, f in enumerate(films):
        ref = oracle.run(f, [Ts[r]], [0.0], 6, seed=3, replica=r, init="cold")
        assert np.array_equal(b.spins_user(r).cpu().numpy(), ref["spins"])
        assert np.array_equal(H[r][..., 4], ref["history"][..., 4])


def test_c3_groups_on_two_streams_change_nothing():
    """Films with trailing colour classes and films without run as two groups
    on the batch's two streams (plain and graph launches); with per-MCS
    outputs bound the same batch interleaves both groups on the caller's
    stream, and each group alone is a batch of its own: spins and history
    bit-identical in all of them."""
    films, Ts = synth.film_batch()
    order = np.argsort([f.n for f in films], kind="stable")[:24]
    plans = {int(f): hsim.Plan(films[f]) for f in order}
    pick = [int(f) for f in order]
    tail = [f for f in pick if plans[f].info.n_colours > 2]
    rest = [f for f in pick if plans[f].info.n_colours <= 2]
    assert tail and rest
    M = 6
    T = np.array([Ts[f] for f in pick])[:, None] * np.ones((1, 2))

    def run(fs, launch, outputs=False):
        b = hsim.Batch([plans[f] for f in fs], seed=7, replica_ids=np.array(fs, dtype=np.uint32),
                       precision=hsim.FP32, layout=hsim.LAYOUT_SITE).bind(2, M)
        if outputs:
            b.bind_outputs(snapshots=True)
        b.init_spins(hsim.INIT_RANDOM)
        idx = [pick.index(f) for f in fs]
        b.run(T[idx], 0.2, recompute_every=3, launch=launch)
        torch.cuda.synchronize()
        assert b.status() == 0
        return {f: (b.spins_user(k).cpu().numpy(), b.history.cpu().numpy()[k]) for k, f in enumerate(fs)}

    ref = run(pick, hsim.LAUNCH_PLAIN)
    for got in (run(pick, hsim.LAUNCH_GRAPH), run(pick, hsim.LAUNCH_PLAIN, outputs=True),
                {**run(tail, hsim.LAUNCH_PLAIN), **run(rest, hsim.LAUNCH_GRAPH)}):
        for f in pick:
            assert np.array_equal(got[f][0], ref[f][0]), f
            assert np.array_equal(got[f][1], ref[f][1]), f


def test_c3_full_batch_fp32():
    """All 256 films (8.6M sites) in one site-layout batch, FP32, graph
    launch: unit spins, incremental vs full energy and one-MCS site agreement
    on sampled films."""
    films, Ts = synth.film_batch()
    plans = [hsim.Plan(f) for f in films]
    b = hsim.Batch(plans, seed=3, precision=hsim.FP32, layout=hsim.LAYOUT_SITE).bind(1, 1)
    assert b.info.total_sites == sum(f.n for f in films)
    b.init_spins(hsim.INIT_COLD_Z)
    b.run(Ts[:, None], 0.0, launch=hsim.LAUNCH_GRAPH)
    torch.cuda.synchronize()
    assert b.status() == 0
    h = b.history.cpu().numpy()
    for r in (0, 77, 255):
        f = films[r]
        got = b.spins_user(r).cpu().numpy()
        start = np.tile([0.0, 0.0, 1.0], (f.n, 1))
        check_one_mcs(f, plans[r].colouring(), start, Ts[r], 0.0, 3, r, got, spin_tol=2e-6)
        e = oracle.energy(f, 0.0, got)
        assert abs(h[r, 0, 0, 0] - e["E"]) <= 1e-5 * e["scale"]


# ------------------------------------------------------------------ C4
def test_c4_energy_gradients_full_size():
    """SC 32^3 with per-bond J ~ N(1, 0.1), per-site K and axes, B = 0.5 z;
    a batch of 1024 configurations: FP32 energies of sampled configurations
    and the weighted gradients against the FP64 oracle element by element;
    FP64 gradients against FP64 central differences of the device's own
    energy on 64 sampled coordinates per family (spin components, bond
    constants, anisotropy constants) and dE/dB, over 8 configurations."""
    from paper_1803_07030_amd.energy import heisenberg_energy
    lat = synth.gradient_lattice(L=32, seed=4)
    plan = hsim.Plan(lat)
    Bn = 1024
    S = synth.random_spins(44, lat.n, batch=Bn).astype(np.float32)
    _, _, Jb = lat.bonds()
    dev = "cuda"
    St = torch.tensor(S.transpose(0, 2, 1).copy(), device=dev, requires_grad=True)
    Jt = torch.tensor(Jb, dtype=torch.float32, device=dev, requires_grad=True)
    kt = torch.tensor(lat.k, dtype=torch.float32, device=dev, requires_grad=True)
    Bt = torch.tensor(0.5, dtype=torch.float64, device=dev, requires_grad=True)
    ax = torch.tensor(lat.axis.T.copy(), dtype=torch.float32, device=dev)
    E = heisenberg_energy(St, Jt, kt, Bt, plan, ax)
    w = torch.zeros(Bn, dtype=torch.float64, device=dev)
    picked = [0, 5, 100, 511, 512, 900, 1000, 1023]
    w[picked] = torch.linspace(0.5, 1.5, len(picked), dtype=torch.float64, device=dev)
    (E * w).sum().backward()
    Sd = S.astype(np.float64)
    Jf = Jb.astype(np.float32).astype(np.float64)
    lat32 = lat.with_bond_J(Jf)
    lat32.k = lat.k.astype(np.float32).astype(np.float64)
    lat32.axis = lat.axis.astype(np.float32).astype(np.float64)
    gJ_ref = np.zeros(Jb.size)
    gk_ref = np.zeros(lat.n)
    gB_ref = 0.0
    wv = w.cpu().numpy()
    bS, bJ, bk, _ = grad_bounds(lat32, 0.5, wv)    # tests/_fp32.py
    for i, c in enumerate(picked):
        e = oracle.energy(lat32, 0.5, Sd[c])
        assert abs(E[c].item() - e["E"]) <= 2e-6 * e["scale"]
        gS, gJ, gk, gB = oracle.energy_grad(lat32, 0.5, Sd[c], g=float(w[c]))
        gs = St.grad[c].detach().cpu().numpy().T
        r = np.abs(gs - gS) / (bS[:, None] * wv[c])
        assert r.max() <= 1.0, (c, float(r.max()))
        gJ_ref += gJ
        gk_ref += gk
        gB_ref += gB
    dJ = np.max(np.abs(Jt.grad.cpu().numpy() - gJ_ref))
    dk = np.max(np.abs(kt.grad.cpu().numpy() - gk_ref))
    assert dJ <= bJ, (float(dJ), bJ)
    assert dk <= bk, (float(dk), bk)
    assert abs(Bt.grad.item() - gB_ref) <= 1e-7 * lat.n * len(picked)
    unpicked = np.setdiff1d(np.arange(Bn), picked)[:4]
    assert float(St.grad[unpicked].abs().max()) == 0.0
    # FP64 mode: gradients vs central differences of the device energy, on 64
    # sampled coordinates of each family (spin components, bonds, sites) and
    # dE/dB, over 8 configurations with weights.  E is a polynomial of degree
    # <= 2 in every single coordinate, so a central difference is exact up to
    # rounding for any step; h = 0.25 keeps the rounding of the differences
    # (about 1e-16 |E| / h) far below the tolerance.
    nc = 8
    S64 = torch.tensor(Sd[:nc].transpose(0, 2, 1).copy(), device=dev, requires_grad=True)
    J64 = torch.tensor(Jb, device=dev, requires_grad=True)
    k64 = torch.tensor(lat.k, device=dev, requires_grad=True)
    ax64 = torch.tensor(lat.axis.T.copy(), device=dev)
    B64 = torch.tensor(0.5, dtype=torch.float64, device=dev, requires_grad=True)
    w64 = torch.linspace(0.5, 1.5, nc, dtype=torch.float64, device=dev)
    (heisenberg_energy(S64, J64, k64, B64, plan, ax64) * w64).sum().backward()
    h = 0.25

    def weighted(Sx, Jx, kx, Bx):
        with torch.no_grad():
            return float((heisenberg_energy(Sx, Jx, kx, Bx, plan, ax64) * w64).sum())

    base = [S64.detach(), J64.detach(), k64.detach(), B64.detach()]
    rng = np.random.default_rng(4)
    picks = {0: [(int(rng.integers(nc)), int(rng.integers(3)), int(rng.integers(lat.n)))
                 for _ in range(64)],
             1: [(int(x),) for x in rng.choice(Jb.size, 64, replace=False)],
             2: [(int(x),) for x in rng.choice(lat.n, 64, replace=False)],
             3: [()]}
    grads = [S64.grad, J64.grad, k64.grad, B64.grad]
    for fam, idxs in picks.items():
        for idx in idxs:
            plus = [t.clone() for t in base]
            minus = [t.clone() for t in base]
            plus[fam][idx] += h
            minus[fam][idx] -= h
            fd = (weighted(*plus) - weighted(*minus)) / (2 * h)
            g = grads[fam][idx].item()
            assert abs(fd - g) <= 1e-9 * max(1.0, abs(fd)), (fam, idx, fd, g)
