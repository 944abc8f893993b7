"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Double-precision validation mode: the accept/reject sequence and the spins are
bit-exact and the energies agree to 1e-12 of the energy scale (the two sides
sum the per-MCS energy changes in different orders).  Single-precision
production mode: one MCS from a shared state agrees site by site, a decision
differing only within single-precision error of its tie or after a differing
neighbour of an earlier colour (tests/_ties.py); different layouts and launch
modes give bit-identical spins.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1803_07030_amd import hsim
from _ties import check_one_mcs
from _fp32 import grad_bounds

pytestmark = pytest.mark.gpu


def _fp64_run(lat, T, B, M, seed, layout, init="random", given=None, trace=True):
    plan = hsim.Plan(lat)
    b = hsim.Batch([plan], seed=seed, precision=hsim.FP64_EXACT, layout=layout).bind(len(T), M)
    if init == "random":
        b.init_spins(hsim.INIT_RANDOM)
    elif init == "cold":
        b.init_spins(hsim.INIT_COLD_Z)
    else:
        b.init_spins(hsim.INIT_GIVEN, given)
    tr = b.new_trace(len(T)) if trace else None
    b.run(T, B, trace=tr, launch=hsim.LAUNCH_PLAIN)
    torch.cuda.synchronize()
    assert b.status() == 0
    acc = None if tr is None else hsim.unpack_trace(tr, lat.n)[0]
    return b, acc, b.history.cpu().numpy()[0], b.spins_user(0).cpu().numpy()


def _energy_scale(lat):
    return np.abs(lat.J).sum() / 2 + (0 if lat.k is None else np.abs(lat.k).sum()) + lat.n


@pytest.mark.parametrize("layout", [hsim.LAYOUT_BLOCK, hsim.LAYOUT_SITE])
def test_fp64_c0_parity_100_mcs(layout):
    """SC 8^3, J = 1, random start (seed 0), the 20-temperature cooling
    schedule with 5 MCS each: 100 MCS, bit-exact accepts and spins."""
    lat = synth.sc_periodic(8)
    T = synth.cooling_schedule(20)
    M = 5
    b, acc, h, s = _fp64_run(lat, T, 0.0, M, 0, layout)
    assert b.layout == {hsim.LAYOUT_BLOCK: "block", hsim.LAYOUT_SITE: "site"}[layout]
    ref = oracle.run(lat, T, 0.0, M, seed=0, init="random", trace_accepts=True)
    assert np.array_equal(acc, ref["accept"].astype(bool))
    assert np.array_equal(s, ref["spins"])
    assert np.array_equal(h[..., 4], ref["history"][..., 4])
    sc = _energy_scale(lat)
    assert np.max(np.abs(h[..., 0] - ref["history"][..., 0])) <= 1e-12 * sc
    assert np.max(np.abs(h[..., 1:4] - ref["history"][..., 1:4])) <= 1e-12 * lat.n


def test_fp64_c0_single_temperature_100_mcs():
    lat = synth.sc_periodic(8)
    b, acc, h, s = _fp64_run(lat, [3.0], 0.0, 100, 0, hsim.LAYOUT_BLOCK)
    ref = oracle.run(lat, [3.0], 0.0, 100, seed=0, init="random", trace_accepts=True)
    assert np.array_equal(acc, ref["accept"].astype(bool))
    assert np.array_equal(s, ref["spins"])
    assert np.max(np.abs(h[..., 0] - ref["history"][..., 0]) / np.abs(ref["history"][..., 0])) <= 1e-12


def test_fp64_full_c0_run():
    """The whole workload: 20 temperatures x 1000 MCS, block layout."""
    lat = synth.sc_periodic(8)
    T = synth.cooling_schedule(20)
    b, _, h, s = _fp64_run(lat, T, 0.0, 1000, 0, hsim.LAYOUT_BLOCK, trace=False)
    ref = oracle.run(lat, T, 0.0, 1000, seed=0, init="random")
    assert ref["near_ties"] == 0
    assert np.array_equal(h[..., 4], ref["history"][..., 4])
    assert np.array_equal(s, ref["spins"])
    assert np.max(np.abs(h[..., 0] - ref["history"][..., 0])) <= 1e-12 * _energy_scale(lat)


@pytest.mark.parametrize("kind", ["sc6", "isolated", "sc10", "sc14"])
def test_fp64_block_layout_class_sizes(kind):
    """The double-precision block kernel bounded at 256 threads draws a
    site's acceptance word and trial point ahead of the colour phases when
    there are at most two classes of at most one site per thread: SC 6^3
    (two classes of 108 sites) and 200 isolated spins (one class).  The
    kernel bounded at 1024 threads draws in the phases: SC 10^3 (two classes
    of 500, a 512-thread block) and SC 14^3 (classes of 1372 sites, more
    than a block's 1024 threads).  Per-site anisotropy, field steps of both
    signs; accepts and spins bit-exact."""
    if kind == "isolated":
        lat = synth.isolated(200)
    else:
        lat = synth.sc_periodic({"sc6": 6, "sc10": 10, "sc14": 14}[kind])
    lat.k = 0.4 * synth.uniform01(21, lat.n, tag=1) - 0.1
    lat.axis = synth.unit_vectors(21, lat.n, tag=2)
    T = [2.0, 0.5, 0.0]
    B = [0.3, -0.4, 0.1]
    M = 8
    b, acc, h, s = _fp64_run(lat, T, B, M, 21, hsim.LAYOUT_BLOCK)
    assert b.layout == "block"
    ref = oracle.run(lat, T, B, M, seed=21, init="random", trace_accepts=True)
    assert np.array_equal(acc, ref["accept"].astype(bool))
    assert np.array_equal(s, ref["spins"])
    assert np.array_equal(h[..., 4], ref["history"][..., 4])
    assert np.max(np.abs(h[..., 0] - ref["history"][..., 0])) <= 1e-12 * _energy_scale(lat)


@pytest.mark.parametrize("layout", [hsim.LAYOUT_BLOCK, hsim.LAYOUT_SITE])
def test_fp64_irregular_lattice_with_all_terms(layout):
    """Film with vacancies (odd L: 5 colours), random per-bond J, per-site k
    and axes, per-site field directions, field steps of both signs."""
    lat = synth.diluted_film(13, 3, seed=6)
    lat.k = 0.5 * synth.uniform01(6, lat.n, tag=1) - 0.1
    lat.axis = synth.unit_vectors(6, lat.n, tag=2)
    lat.ndir = synth.unit_vectors(6, lat.n, tag=3)
    T = [2.0, 1.0, 0.3, 0.0]
    B = [0.5, -0.7, 0.2, 1.0]
    M = 6
    _, acc, h, s = _fp64_run(lat, T, B, M, 77, layout)
    ref = oracle.run(lat, T, B, M, seed=77, init="random", trace_accepts=True)
    assert np.array_equal(acc, ref["accept"].astype(bool))
    assert np.array_equal(s, ref["spins"])
    assert np.max(np.abs(h[..., 0] - ref["history"][..., 0])) <= 1e-12 * _energy_scale(lat)


def test_fp64_resume_is_bit_exact():
    lat = synth.sc_periodic(6)
    T = synth.cooling_schedule(6, 2.0, 0.5)
    plan = hsim.Plan(lat)
    b = hsim.Batch([plan], seed=9, precision=hsim.FP64_EXACT).bind(6, 7)
    b.init_spins(hsim.INIT_RANDOM)
    b.run(T[:3], 0.0)
    b.run(T[3:], 0.0, first_step=3)
    torch.cuda.synchronize()
    ref = oracle.run(lat, T, 0.0, 7, seed=9, init="random")
    assert np.array_equal(b.spins_user(0).cpu().numpy(), ref["spins"])
    assert np.array_equal(b.history.cpu().numpy()[0][..., 4], ref["history"][..., 4])


def test_fp64_multi_replica_site_layout():
    """Different lattices and replica ids in one batch: each replica equals
    its own oracle run (counter word 2 = replica id)."""
    lats = [synth.sc_periodic(4), synth.diluted_film(9, 2, seed=1), synth.random_tree(70, seed=4)]
    plans = [hsim.Plan(l) for l in lats]
    ids = [3, 11, 40]
    T = np.array([[1.5, 0.7], [0.9, 0.4], [2.0, 1.0]])
    b = hsim.Batch(plans, seed=5, replica_ids=ids, precision=hsim.FP64_EXACT,
                   layout=hsim.LAYOUT_SITE).bind(2, 4)
    b.init_spins(hsim.INIT_RANDOM)
    b.run(T, 0.25)
    torch.cuda.synchronize()
    H = b.history.cpu().numpy()
    for r, lat in enumerate(lats):
        ref = oracle.run(lat, T[r], 0.25, 4, seed=5, replica=ids[r], init="random")
        assert np.array_equal(b.spins_user(r).cpu().numpy(), ref["spins"])
        assert np.array_equal(H[r][..., 4], ref["history"][..., 4])


# ------------------------------------------------------------------ FP32
def _fp32_lattice():
    lat = synth.diluted_film(17, 3, seed=2)      # 5 colour classes, random J
    lat.k = np.full(lat.n, 0.05)
    return lat


def _fp32_spins(batch, rep):
    return batch.spins_user(rep).cpu().numpy()


@pytest.mark.parametrize("lat_kind", ["film", "sc_site_params"])
def test_fp32_layouts_and_launches_bit_identical(lat_kind):
    """The same replicas in the site, block and replica layouts and in the
    plain, graph and persistent launches give bit-identical spins; history
    is identical between launch modes of one layout."""
    if lat_kind == "film":
        lat = _fp32_lattice()
    else:
        lat = synth.sc_periodic(10)
        lat.k = 0.3 * synth.uniform01(3, lat.n, tag=1)
        lat.axis = synth.unit_vectors(3, lat.n, tag=2)
        lat.ndir = synth.unit_vectors(3, lat.n, tag=3)
    plan = hsim.Plan(lat)
    R, M = 20, 12
    T = np.linspace(0.3, 2.5, R)[:, None] * np.ones((1, 2))
    B = np.linspace(-0.5, 0.5, R)[:, None] * np.ones((1, 2))
    out = {}
    for name, layout, launch in (("site", hsim.LAYOUT_SITE, hsim.LAUNCH_PLAIN),
                                 ("site_graph", hsim.LAYOUT_SITE, hsim.LAUNCH_GRAPH),
                                 ("block", hsim.LAYOUT_BLOCK, hsim.LAUNCH_PLAIN),
                                 ("rep", hsim.LAYOUT_REPLICA, hsim.LAUNCH_PLAIN),
                                 ("rep_graph", hsim.LAYOUT_REPLICA, hsim.LAUNCH_GRAPH),
                                 ("rep_persist", hsim.LAYOUT_REPLICA, hsim.LAUNCH_PERSISTENT)):
        b = hsim.Batch([plan] * R, seed=21, precision=hsim.FP32, layout=layout).bind(2, M)
        b.init_spins(hsim.INIT_RANDOM)
        b.run(T, B, recompute_every=5, launch=launch)
        torch.cuda.synchronize()
        assert b.status() == 0, name
        out[name] = (np.stack([_fp32_spins(b, r) for r in range(R)]), b.history.cpu().numpy())
    ref_s = out["site"][0]
    for name, (s, _) in out.items():
        assert np.array_equal(s, ref_s), name
    assert np.array_equal(out["site"][1], out["site_graph"][1])
    assert np.array_equal(out["rep"][1], out["rep_graph"][1])
    assert np.array_equal(out["rep"][1], out["rep_persist"][1])
    # all layouts: same accept counts, M within rounding, E within FP32 drift
    for name, (_, h) in out.items():
        assert np.array_equal(h[..., 4], out["site"][1][..., 4]), name
        assert np.allclose(h[..., 1:4], out["site"][1][..., 1:4], rtol=0, atol=1e-9 * lat.n)
        assert np.allclose(h[..., 0], out["site"][1][..., 0], rtol=0, atol=1e-9 * lat.n)


@pytest.mark.parametrize("layout", [hsim.LAYOUT_SITE, hsim.LAYOUT_REPLICA, hsim.LAYOUT_BLOCK])
def test_fp32_one_mcs_matches_oracle_site_by_site(layout):
    """One MCS from a shared start state: the single-precision kernels take
    the same decisions as the oracle (which evaluates the same proposal map in
    double) except where the two are within single-precision rounding of a
    tie, and the new spins agree to single-precision accuracy."""
    lat = synth.sc_periodic(12)
    lat.k = 0.2 * synth.uniform01(8, lat.n, tag=1)
    lat.axis = synth.unit_vectors(8, lat.n, tag=2)
    R = 16
    start = synth.random_spins(4, lat.n, batch=R).astype(np.float32).astype(np.float64)
    plan = hsim.Plan(lat)
    T = np.linspace(0.4, 3.0, R)
    b = hsim.Batch([plan] * R, seed=33, precision=hsim.FP32, layout=layout).bind(1, 1)
    b.init_spins(hsim.INIT_GIVEN, start.reshape(-1, 3))
    b.run(T[:, None], 0.3)
    torch.cuda.synchronize()
    colour = plan.colouring()
    for r in range(R):
        check_one_mcs(lat, colour, start[r], T[r], 0.3, 33, r, _fp32_spins(b, r), spin_tol=2e-6)


def test_fp32_energy_history_consistent():
    """Incremental FP32 energy vs a full recompute of the final state."""
    lat = _fp32_lattice()
    plan = hsim.Plan(lat)
    R = 8
    b = hsim.Batch([plan] * R, seed=3, precision=hsim.FP32, layout=hsim.LAYOUT_SITE).bind(1, 99)
    b.init_spins(hsim.INIT_RANDOM)
    b.run(np.linspace(0.5, 2.0, R)[:, None], 0.1, recompute_every=0)
    torch.cuda.synchronize()
    h = b.history.cpu().numpy()
    for r in range(R):
        s = _fp32_spins(b, r)
        ef = oracle.energy(lat, 0.1, s)["E"]
        assert abs(h[r, 0, -1, 0] - ef) <= 1e-5 * _energy_scale(lat)
        assert np.allclose(h[r, 0, -1, 1:4], s.sum(axis=0), rtol=0, atol=1e-9 * lat.n)
        assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=2e-6)


# ------------------------------------------------------------ energy / grads
@pytest.mark.parametrize("kind", ["sc9", "deg8"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_energy_and_gradients_match_oracle(dtype, kind):
    """Energies and every gradient against the oracle: SC 9^3 (padded rows
    of 6, three tiles, the last one ragged) and a random graph of degree up
    to 8 (rows of 8, two tiles)."""
    from paper_1803_07030_amd.energy import heisenberg_energy
    if kind == "sc9":
        lat = synth.gradient_lattice(L=9, seed=4)
        lat.ndir = synth.unit_vectors(4, lat.n, tag=9)
    else:
        lat = _degree8_lattice()
    plan = hsim.Plan(lat)
    Bn = 8
    S = synth.random_spins(12, lat.n, batch=Bn)                     # [b, n, 3]
    _, _, Jb = lat.bonds()
    dev = "cuda"
    St = torch.tensor(S.transpose(0, 2, 1).copy(), dtype=dtype, device=dev, requires_grad=True)
    Jt = torch.tensor(Jb, dtype=dtype, device=dev, requires_grad=True)
    kt = torch.tensor(lat.k, dtype=dtype, device=dev, requires_grad=True)
    Bt = torch.tensor(0.5, dtype=torch.float64, device=dev, requires_grad=True)
    ax = torch.tensor(lat.axis.T.copy(), dtype=dtype, device=dev)
    nd = torch.tensor(lat.ndir.T.copy(), dtype=dtype, device=dev)
    E = heisenberg_energy(St, Jt, kt, Bt, plan, ax, nd)
    w = torch.linspace(0.5, 1.5, Bn, dtype=torch.float64, device=dev)
    (E * w).sum().backward()
    tol = 1e-12 if dtype == torch.float64 else 2e-6
    Sl = S.astype(np.float32).astype(np.float64) if dtype == torch.float32 else S
    gS_ref = np.zeros_like(S)
    gJ_ref = np.zeros(Jb.size)
    gk_ref = np.zeros(lat.n)
    gB_ref = 0.0
    for b_ in range(Bn):
        e = oracle.energy(lat, 0.5, Sl[b_])
        sc = e["scale"]
        assert abs(E[b_].item() - e["E"]) <= tol * sc
        gS, gJ, gk, gB = oracle.energy_grad(lat, 0.5, Sl[b_], g=float(w[b_]))
        gS_ref[b_] = gS
        gJ_ref += gJ
        gk_ref += gk
        gB_ref += gB
    gs = St.grad.detach().cpu().numpy().transpose(0, 2, 1)
    dJ = np.abs(Jt.grad.cpu().numpy() - gJ_ref)
    dk = np.abs(kt.grad.cpu().numpy() - gk_ref)
    dB = abs(Bt.grad.item() - gB_ref)
    if dtype == torch.float64:
        assert np.max(np.abs(gs - gS_ref)) <= tol * 20
        assert np.max(dJ) <= tol * 20 * Bn
        assert np.max(dk) <= tol * 20 * Bn
        assert dB <= tol * lat.n * Bn
    else:
        # element by element, within the single-precision bounds of tests/_fp32.py
        bS, bJ, bk, bB = grad_bounds(lat, 0.5, w.cpu().numpy())
        wv = w.cpu().numpy()
        r = np.abs(gs - gS_ref) / (bS[None, :, None] * wv[:, None, None])
        assert r.max() <= 1.0, float(r.max())
        assert np.max(dJ) <= bJ, (float(np.max(dJ)), bJ)
        assert np.max(dk) <= bk, (float(np.max(dk)), bk)
        assert dB <= bB, (dB, bB)


def _degree8_lattice(n=400, seed=11):
    """Random graph with degrees up to 8 (many odd), per-bond J, per-site K,
    axes and field directions: padded rows of width 8, half rows of 4."""
    rng = np.random.default_rng(seed)
    deg = np.zeros(n, dtype=np.int64)
    pairs = set()
    for _ in range(8 * n):
        a, b = (int(x) for x in rng.integers(0, n, 2))
        if a == b or deg[a] >= 8 or deg[b] >= 8 or (min(a, b), max(a, b)) in pairs:
            continue
        pairs.add((min(a, b), max(a, b)))
        deg[a] += 1
        deg[b] += 1
    bi, bj = (np.array(x) for x in zip(*sorted(pairs)))
    lat = synth.from_bonds(n, bi, bj, rng.uniform(-1.0, 1.5, bi.size), name="deg8")
    lat.k = rng.uniform(0.0, 0.3, n)
    lat.axis = synth.unit_vectors(seed, n, tag=1)
    lat.ndir = synth.unit_vectors(seed, n, tag=2)
    assert lat.degree.max() == 8 and np.any(lat.degree % 2 == 1)
    return lat


@pytest.mark.parametrize("kind", ["film", "deg8", "isolated", "chain"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_energy_forward_from_half_rows(kind, dtype):
    """The forward reads each bond once, from half rows that an Euler
    orientation of the bonds gives each site (at most ceil(deg/2) of them);
    with odd degrees and rows of up to 8 entries its energies equal the
    oracle's (FP64: 1e-12 of the scale; FP32: 2e-6 of the scale)."""
    from paper_1803_07030_amd.energy import heisenberg_energy
    if kind == "film":
        lat = synth.diluted_film(21, 5, seed=12)
        lat.ndir = synth.unit_vectors(12, lat.n, tag=3)
    elif kind == "deg8":
        lat = _degree8_lattice()
    else:
        # no bonds (every half-row slot empty), or an open chain (the ends
        # have odd degree)
        lat = synth.isolated(300) if kind == "isolated" else synth.open_chain(301)
        lat.k = synth.uniform01(14, lat.n, tag=1)
        lat.axis = synth.unit_vectors(14, lat.n, tag=2)
        lat.ndir = synth.unit_vectors(14, lat.n, tag=3)
    plan = hsim.Plan(lat)
    nbatch = 40
    S = synth.random_spins(13, lat.n, batch=nbatch)
    if dtype == torch.float32:
        S = S.astype(np.float32).astype(np.float64)
    _, _, Jb = lat.bonds()
    dev = "cuda"
    St = torch.tensor(S.transpose(0, 2, 1).copy(), dtype=dtype, device=dev)
    J = torch.tensor(Jb, dtype=dtype, device=dev)
    k = torch.tensor(lat.k, dtype=dtype, device=dev)
    ax = torch.tensor(lat.axis.T.copy(), dtype=dtype, device=dev)
    nd = torch.tensor(lat.ndir.T.copy(), dtype=dtype, device=dev)
    B = torch.tensor(0.7, dtype=torch.float64, device=dev)
    E = heisenberg_energy(St, J, k, B, plan, ax, nd).cpu().numpy()
    tol = 1e-12 if dtype == torch.float64 else 2e-6
    for b_ in range(nbatch):
        e = oracle.energy(lat, 0.7, S[b_])
        assert abs(E[b_] - e["E"]) <= tol * e["scale"], (b_, E[b_], e["E"])


@pytest.mark.parametrize("layout", [hsim.LAYOUT_SITE, hsim.LAYOUT_REPLICA])
def test_phase_timing_counts_and_leaves_results_unchanged(layout):
    """Sampled timing of the colour-phase launches (every 3rd MCS of a plain
    run, graph requests fall back to plain) counts one launch per colour of
    each sampled MCS and that colour's updates, and changes no result."""
    lat = synth.sc_periodic(10)
    plan = hsim.Plan(lat)
    ncol = int(plan.info.n_colours)
    sizes = list(plan.info.colour_size)[:ncol]
    R, M, every = 20, 11, 3
    T = np.linspace(0.3, 2.5, R)[:, None]
    res = {}
    for timed in (False, True):
        b = hsim.Batch([plan] * R, seed=5, precision=hsim.FP32, layout=layout).bind(1, M)
        b.init_spins(hsim.INIT_RANDOM)
        if timed:
            b.time_phases(every)
        b.run(T, 0.2, recompute_every=4, launch=hsim.LAUNCH_GRAPH)
        torch.cuda.synchronize()
        assert b.status() == 0
        ms, n, upd = b.phase_times()
        sampled = len(range(0, M, every))
        if timed:
            assert n == sampled * ncol
            assert upd == sampled * R * sum(sizes)
            assert ms > 0.0
            assert b.phase_times() == (0.0, 0, 0)          # read-out clears
        else:
            assert (ms, n, upd) == (0.0, 0, 0)
        res[timed] = (np.stack([_fp32_spins(b, r) for r in range(R)]), b.history.cpu().numpy())
    assert np.array_equal(res[False][0], res[True][0])
    assert np.array_equal(res[False][1], res[True][1])
