"""Edge cases of the GPU path (through the C-ABI): the autotuner leaves
results, outputs and adaptive widths as an untuned run gives them; the
replica layout with more than 64 replicas (two lane columns); lattices with
a site of more than 8 neighbours (the CSR walk instead of padded rows);
lattices without sites, alone and beside others; and the temperature limits
T = 0 (downhill moves only) and T = infinity (every trial accepted)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1803_07030_amd import hsim
from _ties import check_one_mcs

pytestmark = pytest.mark.gpu


def _user(b, R):
    return np.stack([b.spins_user(r).cpu().numpy() for r in range(R)])


# ------------------------------------------------------------------ autotune
@pytest.mark.parametrize("layout", [hsim.LAYOUT_REPLICA, hsim.LAYOUT_SITE], ids=["replica", "site"])
def test_autotune_keeps_results_outputs_and_widths(layout, tmp_path):
    """A run that stops, autotunes and goes on with the tuned choice equals a
    plain run: spins, snapshots, accept counts and adaptive widths bit for
    bit; energies, magnetisations and per-type magnetisations within
    rounding (a different tile shape groups the sums differently).  A second
    batch takes the choice from the cache."""
    lat = synth.sc_periodic(8)
    lat.k = np.full(lat.n, 0.1)
    types = (np.arange(lat.n) % 2).astype(np.int32)
    plan = hsim.Plan(lat)
    plan.set_types(types)
    R, S, M = 24, 4, 5
    T = np.linspace(0.4, 2.2, R)[:, None] * np.ones((1, S))
    pols = [(hsim.POLICY_ADAPTIVE, 0.5), (hsim.POLICY_SMALL_STEP, 0.3)]
    cache = str(tmp_path / "tune.txt")

    def run(tune):
        b = hsim.Batch([plan] * R, seed=12, precision=hsim.FP32, layout=layout).bind(S, M)
        b.set_policies(pols)
        b.bind_outputs(type_mag_types=2, snapshots=True)
        b.init_spins(hsim.INIT_RANDOM)
        b.run(T[:, :2], 0.05, recompute_every=5, launch=hsim.LAUNCH_PLAIN)
        if tune:
            b.autotune(cache_path=cache, trial_mcs=4)
        b.run(T[:, 2:], 0.05, first_step=2, recompute_every=5,
              launch=hsim.LAUNCH_AUTO if tune else hsim.LAUNCH_PLAIN)
        torch.cuda.synchronize()
        assert b.status() == 0
        return (_user(b, R), b.history.cpu().numpy(), b.type_mag.cpu().numpy(),
                b.snapshots.cpu().numpy(), b.sigma())

    ref = run(False)
    N = lat.n
    for attempt in range(2):          # tuned, then read from the cache
        got = run(True)
        assert np.array_equal(got[0], ref[0])                     # spins
        assert np.array_equal(got[3], ref[3])                     # snapshots
        assert np.array_equal(got[4], ref[4])                     # widths
        assert np.array_equal(got[1][..., 4], ref[1][..., 4])     # accepts
        assert np.allclose(got[1][..., :4], ref[1][..., :4], rtol=0, atol=1e-9 * N)
        assert np.allclose(got[2], ref[2], rtol=0, atol=1e-9 * N)
    with open(cache) as f:
        assert len(f.read().split()) == 5


def test_autotune_without_policies_matches_plain():
    """Replica layout with the persistent launch among the candidates."""
    lat = synth.sc_periodic(8)
    plan = hsim.Plan(lat)
    R, M = 64, 6
    T = np.linspace(0.5, 2.5, R)[:, None] * np.ones((1, 2))
    out = []
    for tune in (False, True):
        b = hsim.Batch([plan] * R, seed=4, precision=hsim.FP32, layout=hsim.LAYOUT_REPLICA).bind(2, M)
        b.init_spins(hsim.INIT_RANDOM)
        if tune:
            b.autotune(trial_mcs=6)
        b.run(T, 0.1, recompute_every=3, launch=hsim.LAUNCH_AUTO if tune else hsim.LAUNCH_PLAIN)
        torch.cuda.synchronize()
        assert b.status() == 0
        out.append((_user(b, R), b.history.cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1][..., 4], out[1][1][..., 4])
    assert np.allclose(out[0][1], out[1][1], rtol=0, atol=1e-9 * lat.n)


@pytest.mark.parametrize("case", ["replicas", "films", "fp64"])
def test_choose_layout_returns_a_usable_layout(case):
    """hsim_choose_layout times the layouts a batch can use and returns one of
    them: never the replica layout for uneven lattices or double precision;
    a batch built with its choice gives the same spins as one built with
    HSIM_LAYOUT_AUTO."""
    if case == "replicas":
        lats = [synth.sc_periodic(12)] * 32
        prec = hsim.FP32
    elif case == "films":
        films, _ = synth.film_batch()
        order = np.argsort([f.n for f in films], kind="stable")[:12]
        lats = [films[f] for f in order]
        prec = hsim.FP32
    else:
        lats = [synth.sc_periodic(8)] * 4
        prec = hsim.FP64_EXACT
    plans = [hsim.Plan(lat) for lat in lats]
    R, M = len(plans), 5
    T = np.linspace(0.4, 2.0, R)
    lay = hsim.Batch.choose_layout(plans, 9, T, 0.2, precision=prec, trial_mcs=5)
    allowed = {hsim.LAYOUT_SITE, hsim.LAYOUT_BLOCK} | ({hsim.LAYOUT_REPLICA} if case == "replicas" else set())
    assert lay in allowed, (case, lay)
    out = []
    for layout in (hsim.LAYOUT_AUTO, lay):
        b = hsim.Batch(plans, seed=9, precision=prec, layout=layout).bind(1, M)
        b.init_spins(hsim.INIT_RANDOM)
        b.run(T[:, None], 0.2, launch=hsim.LAUNCH_PLAIN)
        torch.cuda.synchronize()
        assert b.status() == 0
        out.append([b.spins_user(r).cpu().numpy() for r in range(R)])
    for r in range(R):
        assert np.array_equal(out[0][r], out[1][r]), (case, r)


@pytest.mark.parametrize("R", [64, 20], ids=["64-lane rows", "32-lane rows"])
def test_tile_shapes_and_store_policies_give_identical_spins(R):
    """Every tile shape (4, 8, 32 sites per wave) and store policy (whole
    rows, accepted moves only) the tuner may pick, in plain, graph and
    persistent launches: bit-identical spins and accept counts; energies and
    magnetisations within rounding (sums grouped by tiles)."""
    lat = synth.sc_periodic(16)
    lat.k = 0.2 * synth.uniform01(5, lat.n, tag=1)
    lat.axis = synth.unit_vectors(5, lat.n, tag=2)
    plan = hsim.Plan(lat)
    M = 12
    T = np.linspace(0.3, 2.8, R)[:, None]
    ref = None
    for spw in (4, 8, 32):
        for masked in (0, 1):
            for launch in (hsim.LAUNCH_PLAIN, hsim.LAUNCH_GRAPH, hsim.LAUNCH_PERSISTENT):
                b = hsim.Batch([plan] * R, seed=9, precision=hsim.FP32,
                               layout=hsim.LAYOUT_REPLICA).bind(1, M)
                b.set_shape(spw, masked)
                assert (b.info.sites_per_wave, b.info.masked_store) == (spw, masked)
                b.init_spins(hsim.INIT_RANDOM)
                b.run(T, 0.15, recompute_every=5, launch=launch)
                torch.cuda.synchronize()
                assert b.status() == 0
                got = (_user(b, R), b.history.cpu().numpy())
                if ref is None:
                    ref = got
                    continue
                assert np.array_equal(got[0], ref[0]), (spw, masked, launch)
                assert np.array_equal(got[1][..., 4], ref[1][..., 4]), (spw, masked, launch)
                assert np.allclose(got[1], ref[1], rtol=0, atol=1e-9 * lat.n), (spw, masked, launch)


@pytest.mark.parametrize("spw,R", [(8, 64), (32, 64), (4, 100)])
def test_tile_dispatch_order_changes_nothing(spw, R):
    """The replica layout's tile dispatch order (tiles one plane of the class
    apart started together; explicit plane strides and the derived one) in
    plain, graph and persistent launches, with 64-lane rows and with two
    lane columns (R = 100): spins and history bit-identical to tiles in order
    (records are kept per tile)."""
    lat = synth.sc_periodic(24)
    lat.k = np.full(lat.n, 0.1)
    plan = hsim.Plan(lat)
    M = 8
    T = np.linspace(0.3, 2.8, R)[:, None]
    ref = None
    for order in (0, 288, 96, -1):
        for launch in (hsim.LAUNCH_PLAIN, hsim.LAUNCH_GRAPH, hsim.LAUNCH_PERSISTENT):
            b = hsim.Batch([plan] * R, seed=12, precision=hsim.FP32,
                           layout=hsim.LAYOUT_REPLICA).bind(1, M)
            b.set_shape(spw, 0)
            b.set_order(order)
            b.init_spins(hsim.INIT_RANDOM)
            b.run(T, 0.1, recompute_every=3, launch=launch)
            torch.cuda.synchronize()
            assert b.status() == 0
            got = (_user(b, R), b.history.cpu().numpy())
            if ref is None:
                ref = got
                continue
            assert np.array_equal(got[0], ref[0]), (order, launch)
            assert np.array_equal(got[1], ref[1]), (order, launch)


# ------------------------------------------------ more than 64 replicas
def test_replica_layout_two_lane_columns():
    """R = 100 (128 lanes): the same spins as the site layout after 8 MCS in
    every launch mode, history within rounding, and one MCS from a shared
    start against the oracle for replicas on both sides of lane 64."""
    lat = synth.sc_periodic(10)
    lat.k = 0.2 * synth.uniform01(6, lat.n, tag=1)
    plan = hsim.Plan(lat)
    R, M = 100, 8
    T = np.linspace(0.3, 3.0, R)[:, None]
    B = np.linspace(-0.4, 0.4, R)[:, None]
    out = {}
    for name, layout, launch in (("site", hsim.LAYOUT_SITE, hsim.LAUNCH_PLAIN),
                                 ("rep", hsim.LAYOUT_REPLICA, hsim.LAUNCH_PLAIN),
                                 ("rep_graph", hsim.LAYOUT_REPLICA, hsim.LAUNCH_GRAPH),
                                 ("rep_persist", hsim.LAYOUT_REPLICA, hsim.LAUNCH_PERSISTENT)):
        b = hsim.Batch([plan] * R, seed=17, precision=hsim.FP32, layout=layout).bind(1, M)
        b.init_spins(hsim.INIT_RANDOM)
        b.run(T, B, recompute_every=4, launch=launch)
        torch.cuda.synchronize()
        assert b.status() == 0, name
        out[name] = (_user(b, R), b.history.cpu().numpy())
    s0, h0 = out["site"]
    for name, (s, h) in out.items():
        assert np.array_equal(s, s0), name
        assert np.array_equal(h[..., 4], h0[..., 4]), name
        assert np.allclose(h[..., :4], h0[..., :4], rtol=0, atol=1e-9 * lat.n), name
    # the history's magnetisation is the sum of the final spins
    for r in (0, 63, 64, 99):
        assert np.allclose(out["rep"][1][r, 0, -1, 1:4], s0[r].sum(axis=0), rtol=0, atol=1e-9 * lat.n)

    start = synth.random_spins(2, lat.n, batch=R).astype(np.float32).astype(np.float64)
    b = hsim.Batch([plan] * R, seed=5, precision=hsim.FP32, layout=hsim.LAYOUT_REPLICA).bind(1, 1)
    b.init_spins(hsim.INIT_GIVEN, start.reshape(-1, 3))
    b.run(T, B, launch=hsim.LAUNCH_PLAIN)
    torch.cuda.synchronize()
    colour = plan.colouring()
    for r in (0, 1, 63, 64, 65, 99):
        check_one_mcs(lat, colour, start[r], T[r, 0], B[r, 0], 5, r, b.spins_user(r).cpu().numpy(),
                      spin_tol=8e-6)


# ---------------------------------------------- sites of high degree
def _hub_lattice(n=300, hub_deg=40, seed=3):
    """A ring with random J plus site 0 linked to hub_deg ring sites."""
    bi = np.arange(n)
    bj = (bi + 1) % n
    extra = np.linspace(2, n - 2, hub_deg).astype(np.int64)
    bi = np.concatenate([bi, np.zeros(hub_deg, dtype=np.int64)])
    bj = np.concatenate([bj, extra])
    bJ = 0.5 + synth.uniform01(seed, bi.size, tag=1)
    lat = synth.from_bonds(n, bi, bj, bJ)
    lat.k = 0.2 * synth.uniform01(seed, n, tag=2)
    lat.axis = synth.unit_vectors(seed, n, tag=3)
    assert lat.degree.max() == hub_deg + 2
    return lat


@pytest.mark.parametrize("layout", [hsim.LAYOUT_SITE, hsim.LAYOUT_BLOCK], ids=["site", "block"])
def test_fp64_bit_exact_with_a_hub_site(layout):
    lat = _hub_lattice()
    plan = hsim.Plan(lat)
    T = synth.cooling_schedule(10, 2.5, 0.2)
    b = hsim.Batch([plan], seed=6, precision=hsim.FP64_EXACT, layout=layout).bind(10, 6)
    b.init_spins(hsim.INIT_RANDOM)
    tr = b.new_trace(10)
    b.run(T, 0.3, trace=tr, recompute_every=4, launch=hsim.LAUNCH_PLAIN)
    torch.cuda.synchronize()
    assert b.status() == 0
    ref = oracle.run(lat, T, 0.3, 6, seed=6, init="random", recompute_every=4, trace_accepts=True)
    assert np.array_equal(hsim.unpack_trace(tr, lat.n)[0], ref["accept"].astype(bool))
    assert np.array_equal(b.spins_user(0).cpu().numpy(), ref["spins"])
    h = b.history.cpu().numpy()[0]
    assert np.array_equal(h[..., 4], ref["history"][..., 4])
    scale = np.abs(lat.J).sum() / 2 + np.abs(lat.k).sum() + 0.3 * lat.n
    assert np.max(np.abs(h[..., 0] - ref["history"][..., 0])) <= 1e-12 * scale


def _padded_tiles_lattice():
    """Isolated sites, then an open chain, then a periodic SC 6^3 block (one
    lattice, rows padded to 6 slots): the site layout's tiles of 256 sites of
    a class use 0, 2 or 6 slots, and some mix two parts."""
    n_iso, n_chain = 700, 400
    sc = synth.sc_periodic(6)
    si, sj, sJ = sc.bonds()
    ci = np.arange(n_chain - 1) + n_iso
    bi = np.concatenate([ci, si + n_iso + n_chain])
    bj = np.concatenate([ci + 1, sj + n_iso + n_chain])
    rng = np.random.default_rng(17)
    bJ = rng.uniform(0.5, 1.5, bi.size)
    n = n_iso + n_chain + sc.n
    lat = synth.from_bonds(n, bi, bj, bJ, name="padded_tiles")
    lat.k = rng.uniform(0.0, 0.3, n)
    lat.axis = synth.unit_vectors(17, n, tag=1)
    return lat


def test_fp64_bit_exact_with_tiles_of_every_row_width():
    """Site layout: slots past a tile's largest degree are read at the tile's
    first site (its padding entry); accepts and spins stay bit-exact with the
    oracle for tiles whose sites use 0, 2 and 6 slots."""
    lat = _padded_tiles_lattice()
    assert lat.degree.max() == 6 and (lat.degree == 0).sum() == 700
    plan = hsim.Plan(lat)
    T = synth.cooling_schedule(6, 2.5, 0.2)
    b = hsim.Batch([plan], seed=8, precision=hsim.FP64_EXACT, layout=hsim.LAYOUT_SITE).bind(6, 5)
    b.init_spins(hsim.INIT_RANDOM)
    tr = b.new_trace(6)
    b.run(T, 0.3, trace=tr, recompute_every=3, launch=hsim.LAUNCH_PLAIN)
    torch.cuda.synchronize()
    assert b.status() == 0
    ref = oracle.run(lat, T, 0.3, 5, seed=8, init="random", recompute_every=3, trace_accepts=True)
    assert np.array_equal(hsim.unpack_trace(tr, lat.n)[0], ref["accept"].astype(bool))
    assert np.array_equal(b.spins_user(0).cpu().numpy(), ref["spins"])


def test_fp32_hub_site_layouts_identical_and_match_oracle():
    lat = _hub_lattice()
    plan = hsim.Plan(lat)
    R, M = 64, 6
    T = np.linspace(0.3, 2.5, R)[:, None]
    out = {}
    for name, layout, launch in (("site", hsim.LAYOUT_SITE, hsim.LAUNCH_PLAIN),
                                 ("block", hsim.LAYOUT_BLOCK, hsim.LAUNCH_PLAIN),
                                 ("rep", hsim.LAYOUT_REPLICA, hsim.LAUNCH_PLAIN),
                                 ("rep_persist", hsim.LAYOUT_REPLICA, hsim.LAUNCH_PERSISTENT)):
        b = hsim.Batch([plan] * R, seed=8, precision=hsim.FP32, layout=layout).bind(1, M)
        b.init_spins(hsim.INIT_RANDOM)
        b.run(T, 0.2, launch=launch)
        torch.cuda.synchronize()
        assert b.status() == 0, name
        out[name] = _user(b, R)
    for name, s in out.items():
        assert np.array_equal(s, out["site"]), name
    start = synth.random_spins(9, lat.n, batch=R).astype(np.float32).astype(np.float64)
    b = hsim.Batch([plan] * R, seed=8, precision=hsim.FP32, layout=hsim.LAYOUT_REPLICA).bind(1, 1)
    b.init_spins(hsim.INIT_GIVEN, start.reshape(-1, 3))
    b.run(T, 0.2, launch=hsim.LAUNCH_PLAIN)
    torch.cuda.synchronize()
    colour = plan.colouring()
    for r in range(0, R, 9):
        check_one_mcs(lat, colour, start[r], T[r, 0], 0.2, 8, r, b.spins_user(r).cpu().numpy(),
                      spin_tol=8e-6)


# ---------------------------------------------- lattices without sites
@pytest.mark.parametrize("prec,layout", [(hsim.FP64_EXACT, hsim.LAYOUT_SITE),
                                         (hsim.FP64_EXACT, hsim.LAYOUT_BLOCK),
                                         (hsim.FP32, hsim.LAYOUT_REPLICA)],
                         ids=["fp64_site", "fp64_block", "fp32_replica"])
def test_empty_lattice(prec, layout):
    empty = hsim.Plan(synth.isolated(0))
    R = 20 if layout == hsim.LAYOUT_REPLICA else 2
    for launch in (hsim.LAUNCH_PLAIN, hsim.LAUNCH_GRAPH, hsim.LAUNCH_AUTO):
        b = hsim.Batch([empty] * R, seed=1, precision=prec, layout=layout).bind(2, 3)
        b.history.fill_(7.0)
        b.init_spins(hsim.INIT_RANDOM)
        b.run([1.0, 0.5], 0.2, launch=launch)
        torch.cuda.synchronize()
        assert b.status() == 0
        assert torch.count_nonzero(b.history).item() == 0
        assert b.spins_user(R - 1).shape == (0, 3)


@pytest.mark.parametrize("layout", [hsim.LAYOUT_SITE, hsim.LAYOUT_BLOCK], ids=["site", "block"])
def test_empty_lattice_beside_others(layout):
    """A batch [empty, SC 4^3, empty, film]: the lattices with sites equal
    their own oracle runs bit for bit; the empty ones record zeros."""
    lats = [synth.isolated(0), synth.sc_periodic(4), synth.isolated(0), synth.diluted_film(7, 2, seed=3)]
    plans = [hsim.Plan(l) for l in lats]
    T = np.array([[1.0, 0.5]] * 4)
    b = hsim.Batch(plans, seed=2, precision=hsim.FP64_EXACT, layout=layout).bind(2, 4)
    b.history.fill_(7.0)
    b.bind_outputs(type_mag_types=1)
    b.init_spins(hsim.INIT_RANDOM)
    b.run(T, 0.1, recompute_every=3, launch=hsim.LAUNCH_PLAIN)
    torch.cuda.synchronize()
    assert b.status() == 0
    H = b.history.cpu().numpy()
    tm = b.type_mag.cpu().numpy()
    for r, lat in enumerate(lats):
        if lat.n == 0:
            assert np.all(H[r] == 0) and np.all(tm[r] == 0)
            continue
        ref = oracle.run(lat, T[r], 0.1, 4, seed=2, replica=r, init="random", recompute_every=3)
        assert np.array_equal(b.spins_user(r).cpu().numpy(), ref["spins"])
        assert np.array_equal(H[r][..., 4], ref["history"][..., 4])
        assert np.allclose(tm[r][..., 0, :], ref["history"][..., 1:4], rtol=0, atol=1e-12 * lat.n)


def test_energy_of_an_empty_lattice():
    from paper_1803_07030_amd.energy import heisenberg_energy
    plan = hsim.Plan(synth.isolated(0))
    for dt in (torch.float64, torch.float32):
        S = torch.zeros((3, 3, 0), dtype=dt, device="cuda", requires_grad=True)
        J = torch.zeros(0, dtype=dt, device="cuda")
        k = torch.zeros(0, dtype=dt, device="cuda")
        ax = torch.zeros((3, 0), dtype=dt, device="cuda")
        Bt = torch.tensor(0.7, dtype=torch.float64, device="cuda", requires_grad=True)
        E = heisenberg_energy(S, J, k, Bt, plan, ax, None)
        E.sum().backward()
        assert torch.count_nonzero(E).item() == 0
        assert Bt.grad.item() == 0.0


# ------------------------------------------------------ temperature limits
def test_zero_and_infinite_temperature_replica_layout():
    """One MCS from a shared start, replicas at T = 0, T = infinity and
    finite T in one replica-layout batch: at T = infinity every trial is
    taken (the spins are the oracle's trial spins); at T = 0 only downhill
    moves are taken; both against the oracle site by site."""
    lat = synth.sc_periodic(8)
    lat.k = np.full(lat.n, 0.3)
    plan = hsim.Plan(lat)
    R = 64
    T = np.where(np.arange(R) % 3 == 0, 0.0, np.where(np.arange(R) % 3 == 1, np.inf, 1.0))
    start = synth.random_spins(14, lat.n, batch=R).astype(np.float32).astype(np.float64)
    for launch in (hsim.LAUNCH_PLAIN, hsim.LAUNCH_PERSISTENT):
        b = hsim.Batch([plan] * R, seed=3, precision=hsim.FP32, layout=hsim.LAYOUT_REPLICA).bind(1, 1)
        b.init_spins(hsim.INIT_GIVEN, start.reshape(-1, 3))
        b.run(T[:, None], 0.25, launch=launch)
        torch.cuda.synchronize()
        assert b.status() == 0
        h = b.history.cpu().numpy()
        colour = plan.colouring()
        for r in range(6):
            got = b.spins_user(r).cpu().numpy()
            check_one_mcs(lat, colour, start[r], T[r], 0.25, 3, r, got, spin_tol=8e-6)
            if np.isinf(T[r]):
                assert np.all(np.any(got != start[r], axis=1)) and h[r, 0, 0, 4] == lat.n


# ------------------------------------------- planar spin rows (large arrays)
def test_replica_layout_planar_rows_for_arrays_over_2gib():
    """SC 142^3 (2.86M sites) with 64 replicas: the spin array passes 2 GiB,
    so the replica layout keeps each component in a plane of its own; two
    MCS give the same spins as the site layout, bit for bit."""
    lat = synth.sc_periodic(142)
    lat.k = np.full(lat.n, 0.1)
    assert 3 * lat.n * 64 * 4 >= 1 << 31
    plan = hsim.Plan(lat)
    R = 64
    T = np.linspace(0.2, 2.8, R)[:, None]
    out = {}
    for name, layout in (("rep", hsim.LAYOUT_REPLICA), ("site", hsim.LAYOUT_SITE)):
        b = hsim.Batch([plan] * R, seed=23, precision=hsim.FP32, layout=layout).bind(1, 2)
        b.init_spins(hsim.INIT_RANDOM)
        b.run(T, 0.0, launch=hsim.LAUNCH_PLAIN)
        torch.cuda.synchronize()
        assert b.status() == 0, name
        out[name] = [b.spins_user(r).cpu().numpy() for r in (0, 37, 63)]
        h = b.history.cpu().numpy()
        out[name + "_acc"] = h[..., 4]
        del b
        torch.cuda.empty_cache()
    for x, y in zip(out["rep"], out["site"]):
        assert np.array_equal(x, y)
    assert np.array_equal(out["rep_acc"], out["site_acc"])


# ---------------------------------------------- tile sizes of the replica layout
@pytest.mark.parametrize("L", [48, 56, 64], ids=["sc48", "sc56", "sc64"])
def test_replica_tiles_of_every_size_match_the_site_layout(L):
    """The replica layout sizes its tiles to the lattice (4, 8 or 32 sites
    per wave: on a 256-CU GPU SC 48^3 with 64 replicas takes 8, SC 56^3 and
    the SC 64^3 headline take 32; the smaller lattices of other tests take 4):
    spins and accept counts equal the site layout's after 3 MCS."""
    lat = synth.sc_periodic(L)
    lat.k = np.full(lat.n, 0.1)
    plan = hsim.Plan(lat)
    R = 64
    T = np.linspace(0.2, 2.8, R)[:, None]
    out = {}
    for name, layout in (("rep", hsim.LAYOUT_REPLICA), ("site", hsim.LAYOUT_SITE)):
        b = hsim.Batch([plan] * R, seed=31, precision=hsim.FP32, layout=layout).bind(1, 3)
        b.init_spins(hsim.INIT_RANDOM)
        b.run(T, 0.1, launch=hsim.LAUNCH_PLAIN)
        torch.cuda.synchronize()
        assert b.status() == 0, name
        out[name] = ([b.spins_user(r).cpu().numpy() for r in (0, 31, 63)], b.history.cpu().numpy())
    for x, y in zip(out["rep"][0], out["site"][0]):
        assert np.array_equal(x, y)
    assert np.array_equal(out["rep"][1][..., 4], out["site"][1][..., 4])
    assert np.allclose(out["rep"][1][..., :4], out["site"][1][..., :4], rtol=0, atol=1e-9 * lat.n)


# ----------------------------------------------- energy backward, partial outputs
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_energy_backward_with_some_outputs_null(dtype):
    """Any output of the backward may be NULL: dE/dB alone, dE/dS alone and
    (dE/dJ, dE/dk) alone equal the same outputs of the full call."""
    lat = synth.gradient_lattice(L=9, seed=5)
    plan = hsim.Plan(lat)
    nb = 37
    prec = hsim.FP64_EXACT if dtype == torch.float64 else hsim.FP32
    S = torch.tensor(synth.random_spins(3, lat.n, batch=nb).transpose(0, 2, 1).copy(), dtype=dtype,
                     device="cuda")
    _, _, Jb = lat.bonds()
    J = torch.tensor(Jb, dtype=dtype, device="cuda")
    k = torch.tensor(lat.k, dtype=dtype, device="cuda")
    ax = torch.tensor(lat.axis.T.copy(), dtype=dtype, device="cuda")
    gE = torch.linspace(0.5, 1.5, nb, dtype=torch.float64, device="cuda")

    def call(want):
        out = dict(gS=torch.full_like(S, 7.0), gJ=torch.full_like(J, 7.0), gk=torch.full_like(k, 7.0),
                   gB=torch.full((1,), 7.0, dtype=torch.float64, device="cuda"))
        args = {name: (out[name] if name in want else None) for name in out}
        hsim.hsim_energy_backward(plan.handle, nb, prec, S, J, k, ax, 0.4, None, gE, **args)
        torch.cuda.synchronize()
        return {name: out[name].cpu().numpy() for name in want}

    full = call(("gS", "gJ", "gk", "gB"))
    for want in (("gB",), ("gS",), ("gJ", "gk")):
        part = call(want)
        for name in want:
            assert np.array_equal(part[name], full[name]), (want, name)


@pytest.mark.parametrize("R", [1, 33], ids=["one replica", "33 replicas"])
def test_replica_layout_with_mostly_idle_lanes(R):
    """One replica (31 idle lanes of a 32-lane row) and 33 replicas (31 idle
    lanes of a 64-lane row): spins, accept counts and the adaptive widths of
    a policy run equal the site layout's."""
    lat = synth.diluted_film(13, 3, seed=7)
    lat.k = np.full(lat.n, 0.05)
    types = (np.arange(lat.n) % 2).astype(np.int32)
    plan = hsim.Plan(lat)
    plan.set_types(types)
    T = np.linspace(0.5, 2.0, R)[:, None] * np.ones((1, 2))
    out = {}
    for name, layout in (("rep", hsim.LAYOUT_REPLICA), ("site", hsim.LAYOUT_SITE)):
        b = hsim.Batch([plan] * R, seed=19, precision=hsim.FP32, layout=layout).bind(2, 6)
        b.set_policies([(hsim.POLICY_ADAPTIVE, 0.7), (hsim.POLICY_RANDOM, 0.0)])
        b.init_spins(hsim.INIT_RANDOM)
        b.run(T, 0.1, launch=hsim.LAUNCH_PLAIN)
        torch.cuda.synchronize()
        assert b.status() == 0, name
        out[name] = (_user(b, R), b.history.cpu().numpy()[..., 4], b.sigma())
    assert np.array_equal(out["rep"][0], out["site"][0])
    assert np.array_equal(out["rep"][1], out["site"][1])
    assert np.array_equal(out["rep"][2], out["site"][2])


# ---------------------------------------------- failure paths
@pytest.mark.parametrize("layout,launch", [(hsim.LAYOUT_REPLICA, hsim.LAUNCH_PLAIN),
                                           (hsim.LAYOUT_REPLICA, hsim.LAUNCH_PERSISTENT),
                                           (hsim.LAYOUT_SITE, hsim.LAUNCH_GRAPH),
                                           (hsim.LAYOUT_BLOCK, hsim.LAUNCH_PLAIN)])
def test_nan_energy_change_reports_numeric(layout, launch):
    """A NaN field intensity staged by the debug flag makes every energy change
    NaN: no move is taken, the device status reads HSIM_E_NUMERIC once (the
    read clears it), and a normal run afterwards is clean."""
    lat = synth.sc_periodic(8)
    prec = hsim.FP64_EXACT if layout == hsim.LAYOUT_BLOCK else hsim.FP32
    R = 1 if layout == hsim.LAYOUT_BLOCK else 32
    b = hsim.Batch([hsim.Plan(lat)] * R, seed=1, precision=prec, layout=layout).bind(2, 8)
    b.init_spins(hsim.INIT_COLD_Z)
    b.run(np.full((R, 1), 1.0), 0.3, launch=launch, debug_flags=hsim.RUN_DEBUG_NAN_FIELD)
    torch.cuda.synchronize()
    assert b.status() == -8                     # HSIM_E_NUMERIC
    assert b.status() == 0                      # cleared by the read
    h = b.history.cpu().numpy()
    assert np.all(h[:, 0, :, 4] == 0)           # nothing accepted
    assert np.all(b.spins_user(0).cpu().numpy() == np.tile([0.0, 0.0, 1.0], (lat.n, 1)))
    b.run(np.full((R, 1), 1.0), 0.3, first_step=1, launch=launch)
    torch.cuda.synchronize()
    assert b.status() == 0
    assert np.all(np.isfinite(b.history.cpu().numpy()[:, 1]))


def test_persistent_barrier_wait_cap_reports_timeout():
    """With the debug flag every device barrier wait of the persistent launch
    gives up after one polling round: the first wait that has to wait
    releases all later ones, the launch drains, and the device status reads
    HSIM_E_TIMEOUT; a normal run afterwards is clean."""
    lat = synth.sc_periodic(32)
    R = 64
    b = hsim.Batch([hsim.Plan(lat)] * R, seed=1, precision=hsim.FP32,
                   layout=hsim.LAYOUT_REPLICA).bind(1, 20)
    b.init_spins(hsim.INIT_COLD_Z)
    b.run(np.full((R, 1), 1.0), 0.0, launch=hsim.LAUNCH_PERSISTENT,
          debug_flags=hsim.RUN_DEBUG_WAIT_CAP)
    torch.cuda.synchronize()
    assert b.status() == -7                     # HSIM_E_TIMEOUT
    assert b.status() == 0
    b.init_spins(hsim.INIT_COLD_Z)
    b.run(np.full((R, 1), 1.0), 0.0, launch=hsim.LAUNCH_PERSISTENT)
    torch.cuda.synchronize()
    assert b.status() == 0


# --------------------------------------------- accept trace, replica layout
@pytest.mark.parametrize("case", ["sc_r20", "sc_r64", "hub_r64"])
def test_replica_layout_accept_trace_equals_site_layout(case):
    """The accept bitmap of a replica-layout run (plain, graph and a
    persistent request, which runs as plain launches) equals the site
    layout's bit for bit over 2 steps x 6 MCS: rows of 32 lanes (R = 20), 64
    lanes (R = 64) and the generic row walk (a site of degree 42).  With
    update policies the replica layout refuses a trace."""
    if case == "hub_r64":
        lat = _hub_lattice()
    else:
        lat = synth.sc_periodic(10)
        lat.k = 0.2 * synth.uniform01(7, lat.n, tag=1)
        lat.axis = synth.unit_vectors(7, lat.n, tag=2)
    R = 20 if case == "sc_r20" else 64
    plan = hsim.Plan(lat)
    S, M = 2, 6
    T = np.linspace(0.3, 2.5, R)[:, None] * np.ones((1, S))
    Bf = np.linspace(-0.4, 0.4, R)[:, None] * np.ones((1, S))
    out = {}
    for name, layout, launch in (("site", hsim.LAYOUT_SITE, hsim.LAUNCH_PLAIN),
                                 ("rep", hsim.LAYOUT_REPLICA, hsim.LAUNCH_PLAIN),
                                 ("rep_graph", hsim.LAYOUT_REPLICA, hsim.LAUNCH_GRAPH),
                                 ("rep_persist", hsim.LAYOUT_REPLICA, hsim.LAUNCH_PERSISTENT)):
        b = hsim.Batch([plan] * R, seed=17, precision=hsim.FP32, layout=layout).bind(S, M)
        b.init_spins(hsim.INIT_RANDOM)
        tr = b.new_trace(S)
        b.run(T, Bf, recompute_every=3, launch=launch, trace=tr)
        torch.cuda.synchronize()
        assert b.status() == 0, name
        out[name] = (tr.cpu().numpy(), b.history.cpu().numpy())
    acc = hsim.unpack_trace(torch.from_numpy(out["site"][0]), lat.n)
    assert acc.sum() > 0
    for name, (tr, h) in out.items():
        assert np.array_equal(tr, out["site"][0]), name
        # the bitmap counts the history's accepted moves
        got = hsim.unpack_trace(torch.from_numpy(tr), lat.n)
        assert np.array_equal(got.sum(axis=-1).reshape(R, S, M), h[..., 4]), name
    b = hsim.Batch([plan] * R, seed=17, precision=hsim.FP32, layout=hsim.LAYOUT_REPLICA).bind(1, 2)
    b.set_policies([(hsim.POLICY_SMALL_STEP, 0.3)])
    with pytest.raises(hsim.HsimError):
        b.run(T[:, :1], 0.0, trace=b.new_trace(1))
