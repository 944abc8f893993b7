"""Cubic anisotropy (Eq. 3) and per-site spin norms on the GPU (through the
C-ABI) against the oracle: FP64 bit-exact trajectories for 100 MCS (with the
random move and with update policies), FP32 one-MCS site-by-site agreement in
both replica-lane paths, layout and launch identity, the device's starts,
and the energy and its gradient."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1803_07030_amd import hsim
from _ties import check_one_mcs

pytestmark = pytest.mark.gpu


def _lattice(L=8, seed=21):
    lat = synth.sc_periodic(L)
    lat.k = 0.3 * synth.uniform01(seed, lat.n, tag=1)
    lat.axis = synth.unit_vectors(seed, lat.n, tag=2)
    lat.kc = 1.2 * synth.uniform01(seed, lat.n, tag=3) - 0.6
    lat.norm = 0.5 + 1.5 * synth.uniform01(seed, lat.n, tag=4)
    return lat


def _scale(lat):
    return (np.abs(lat.J).sum() / 2 + np.abs(lat.k).sum() * 4 + np.abs(lat.kc).sum() * 16 +
            lat.n * 4)


@pytest.mark.parametrize("layout", [hsim.LAYOUT_BLOCK, hsim.LAYOUT_SITE])
@pytest.mark.parametrize("pols", [None, [(hsim.POLICY_SMALL_STEP, 0.4), (hsim.POLICY_ADAPTIVE, 0.5)]],
                         ids=["random", "policies"])
def test_fp64_bit_exact_with_cubic_and_norms(layout, pols):
    lat = _lattice()
    types = None if pols is None else (np.arange(lat.n) % 2).astype(np.int32)
    T = synth.cooling_schedule(20)
    B = np.full(20, 0.2)
    plan = hsim.Plan(lat)
    if types is not None:
        plan.set_types(types)
    b = hsim.Batch([plan], seed=0, precision=hsim.FP64_EXACT, layout=layout).bind(20, 5)
    if pols is not None:
        b.set_policies(pols)
    b.init_spins(hsim.INIT_RANDOM)
    tr = b.new_trace(20)
    b.run(T, B, trace=tr, launch=hsim.LAUNCH_PLAIN)
    torch.cuda.synchronize()
    assert b.status() == 0
    acc = hsim.unpack_trace(tr, lat.n)[0]
    h = b.history.cpu().numpy()[0]
    s = b.spins_user(0).cpu().numpy()
    ref = oracle.run(lat, T, B, 5, seed=0, init="random", trace_accepts=True, policies=pols,
                     site_type=types)
    assert np.array_equal(acc, ref["accept"].astype(bool))
    assert np.array_equal(s, ref["spins"])
    assert np.array_equal(h[..., 4], ref["history"][..., 4])
    assert np.max(np.abs(h[..., 0] - ref["history"][..., 0])) <= 1e-12 * _scale(lat)
    assert np.max(np.abs(h[..., 1:4] - ref["history"][..., 1:4])) <= 1e-12 * lat.n * 2
    if pols is not None:
        assert b.sigma()[0] == ref["sigma"]


@pytest.mark.parametrize("R", [64, 20], ids=["64-lane rows", "32-lane rows"])
def test_fp32_replica_lane_one_mcs_with_cubic_and_norms(R):
    lat = _lattice(12, seed=8)
    start = synth.random_spins(4, lat.n, batch=R) * lat.norm[None, :, None]
    start = start.astype(np.float32).astype(np.float64)
    plan = hsim.Plan(lat)
    T = np.linspace(0.4, 3.0, R)
    b = hsim.Batch([plan] * R, seed=33, precision=hsim.FP32, layout=hsim.LAYOUT_REPLICA).bind(1, 1)
    assert b.layout == "replica"
    b.init_spins(hsim.INIT_GIVEN, start.reshape(-1, 3))
    b.run(T[:, None], 0.3, launch=hsim.LAUNCH_PLAIN)
    torch.cuda.synchronize()
    assert b.status() == 0
    colour = plan.colouring()
    for r in range(0, R, 3):
        check_one_mcs(lat, colour, start[r], T[r], 0.3, 33, r, b.spins_user(r).cpu().numpy(),
                      spin_tol=8e-6)


def test_fp32_layouts_identical_and_starts_with_norms():
    """Site, block and replica layouts (plain, graph, and a persistent
    request run as plain) give bit-identical spins; the random start is the
    oracle's start rounded to single precision; every spin keeps its length."""
    lat = synth.diluted_film(17, 3, seed=2)
    lat.kc = np.full(lat.n, 0.4)
    lat.norm = np.where(np.arange(lat.n) % 3 == 0, 2.0, 0.75)
    plan = hsim.Plan(lat)
    R, M = 20, 10
    T = np.linspace(0.3, 2.5, R)[:, None]
    out = {}
    for name, layout, launch in (("site", hsim.LAYOUT_SITE, hsim.LAUNCH_PLAIN),
                                 ("block", hsim.LAYOUT_BLOCK, hsim.LAUNCH_PLAIN),
                                 ("rep", hsim.LAYOUT_REPLICA, hsim.LAUNCH_GRAPH),
                                 ("rep_persist", hsim.LAYOUT_REPLICA, hsim.LAUNCH_PERSISTENT)):
        b = hsim.Batch([plan] * R, seed=21, precision=hsim.FP32, layout=layout).bind(1, M)
        b.init_spins(hsim.INIT_RANDOM)
        if name == "site":
            for r in (0, 7):
                ref = oracle.run(lat, [1.0], [0.0], 0, seed=21, replica=r, init="random")
                assert np.array_equal(b.spins_user(r).cpu().numpy(),
                                      ref["spins"].astype(np.float32).astype(np.float64))
        b.run(T, 0.1, launch=launch)
        torch.cuda.synchronize()
        assert b.status() == 0, name
        out[name] = np.stack([b.spins_user(r).cpu().numpy() for r in range(R)])
    for name, s in out.items():
        assert np.array_equal(s, out["site"]), name
    assert np.allclose(np.linalg.norm(out["site"], axis=2), lat.norm[None, :], rtol=2e-6)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_energy_and_gradient_with_cubic(dtype):
    from paper_1803_07030_amd.energy import heisenberg_energy
    lat = synth.gradient_lattice(L=9, seed=4)
    lat.kc = 0.8 * synth.uniform01(4, lat.n, tag=7) - 0.4
    plan = hsim.Plan(lat)
    Bn = 4
    S = synth.random_spins(12, lat.n, batch=Bn) * 1.3
    _, _, Jb = lat.bonds()
    St = torch.tensor(S.transpose(0, 2, 1).copy(), dtype=dtype, device="cuda", requires_grad=True)
    Jt = torch.tensor(Jb, dtype=dtype, device="cuda")
    kt = torch.tensor(lat.k, dtype=dtype, device="cuda")
    Bt = torch.tensor(0.5, dtype=torch.float64, device="cuda")
    ax = torch.tensor(lat.axis.T.copy(), dtype=dtype, device="cuda")
    E = heisenberg_energy(St, Jt, kt, Bt, plan, ax, None)
    E.sum().backward()
    tol = 1e-12 if dtype == torch.float64 else 4e-6
    Sl = S.astype(np.float32).astype(np.float64) if dtype == torch.float32 else S
    gs = St.grad.detach().cpu().numpy().transpose(0, 2, 1)
    for b_ in range(Bn):
        e = oracle.energy(lat, 0.5, Sl[b_])
        assert abs(E[b_].item() - e["E"]) <= tol * e["scale"]
        gS, _, _, _ = oracle.energy_grad(lat, 0.5, Sl[b_])
        assert np.max(np.abs(gs[b_] - gS)) <= tol * 40
