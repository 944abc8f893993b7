"""Update policies on the GPU (through the C-ABI) against the oracle.

Double-precision validation mode: for every policy (spin flip, small step,
Gaussian, Hinzke-Nowak, adaptive) and for a lattice whose site types use
different policies, the accept/reject sequence, the spins and the adaptive
width are bit-exact against the oracle for 100 MCS, with energies within
1e-12 of the energy scale.  Single precision: one MCS agrees site by site with
the oracle's evaluation of the same proposal map except at near ties, in both
replica-lane paths (64-lane rows and 32-lane rows); layouts and launch modes
give bit-identical spins, history and widths; the adaptive width holds the
acceptance at one half.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1803_07030_amd import hsim
from _ties import check_one_mcs

pytestmark = pytest.mark.gpu

POLS = [(hsim.POLICY_FLIP, 0.0), (hsim.POLICY_SMALL_STEP, 0.4), (hsim.POLICY_GAUSSIAN, 0.3),
        (hsim.POLICY_HN, 0.5), (hsim.POLICY_ADAPTIVE, 0.5)]
POL_IDS = ["flip", "small_step", "gaussian", "hn", "adaptive"]


def _lattice_with_terms(L=8):
    lat = synth.sc_periodic(L)
    lat.k = 0.3 * synth.uniform01(21, lat.n, tag=1)
    lat.axis = synth.unit_vectors(21, lat.n, tag=2)
    return lat


def _scale(lat):
    return np.abs(lat.J).sum() / 2 + (0 if lat.k is None else np.abs(lat.k).sum()) + lat.n


def _fp64_policy_run(lat, pols, types, layout, T, B, M, seed=0):
    plan = hsim.Plan(lat)
    if types is not None:
        plan.set_types(types)
    b = hsim.Batch([plan], seed=seed, precision=hsim.FP64_EXACT, layout=layout).bind(len(T), M)
    b.set_policies(pols)
    b.init_spins(hsim.INIT_RANDOM)
    tr = b.new_trace(len(T))
    b.run(T, B, trace=tr, launch=hsim.LAUNCH_PLAIN)
    torch.cuda.synchronize()
    assert b.status() == 0
    acc = hsim.unpack_trace(tr, lat.n)[0]
    return b, acc, b.history.cpu().numpy()[0], b.spins_user(0).cpu().numpy()


def _check_fp64(lat, b, acc, h, s, ref):
    assert np.array_equal(acc, ref["accept"].astype(bool))
    assert np.array_equal(s, ref["spins"])
    assert np.array_equal(h[..., 4], ref["history"][..., 4])
    assert np.max(np.abs(h[..., 0] - ref["history"][..., 0])) <= 1e-12 * _scale(lat)
    assert np.max(np.abs(h[..., 1:4] - ref["history"][..., 1:4])) <= 1e-12 * lat.n
    if ref["sigma"] is not None:
        assert b.sigma()[0] == ref["sigma"]


@pytest.mark.parametrize("layout", [hsim.LAYOUT_BLOCK, hsim.LAYOUT_SITE])
@pytest.mark.parametrize("pol", POLS, ids=POL_IDS)
def test_fp64_policy_bit_exact_100_mcs(layout, pol):
    """SC 8^3 with per-site anisotropy, a field, the 20-temperature cooling
    schedule x 5 MCS from a random start: bit-exact for every policy."""
    lat = _lattice_with_terms()
    T = synth.cooling_schedule(20)
    B = np.full(20, 0.2)
    b, acc, h, s = _fp64_policy_run(lat, [pol], None, layout, T, B, 5)
    ref = oracle.run(lat, T, B, 5, seed=0, init="random", trace_accepts=True, policies=[pol])
    _check_fp64(lat, b, acc, h, s, ref)


@pytest.mark.parametrize("layout", [hsim.LAYOUT_BLOCK, hsim.LAYOUT_SITE])
def test_fp64_policy_per_site_type(layout):
    """Three site types (random, flip, adaptive) in one lattice: bit-exact,
    including the adaptive width; flip sites of the random start keep their
    axis."""
    lat = _lattice_with_terms()
    types = (np.arange(lat.n) % 3).astype(np.int32)
    pols = [(hsim.POLICY_RANDOM, 0.0), (hsim.POLICY_FLIP, 0.0), (hsim.POLICY_ADAPTIVE, 0.8)]
    T = synth.cooling_schedule(20)
    B = np.full(20, 0.1)
    b, acc, h, s = _fp64_policy_run(lat, pols, types, layout, T, B, 5)
    ref = oracle.run(lat, T, B, 5, seed=0, init="random", trace_accepts=True, policies=pols,
                     site_type=types)
    _check_fp64(lat, b, acc, h, s, ref)


def test_fp64_adaptive_multi_replica_resume():
    """Three replicas (ids 5, 9, 2) with the adaptive move, run in two calls:
    each replica's spins and width match its own oracle chain bit for bit."""
    lat = _lattice_with_terms(6)
    plan = hsim.Plan(lat)
    ids = [5, 9, 2]
    T = np.array([[0.6, 1.2], [1.0, 0.8], [2.0, 0.3]])
    b = hsim.Batch([plan] * 3, seed=12, replica_ids=ids, precision=hsim.FP64_EXACT,
                   layout=hsim.LAYOUT_SITE).bind(2, 7)
    b.set_policies([(hsim.POLICY_ADAPTIVE, 2.0)], sigma_min=0.05, sigma_max=3.0)
    b.init_spins(hsim.INIT_COLD_Z)
    b.run(T[:, :1], 0.0, first_step=0, launch=hsim.LAUNCH_GRAPH)
    b.run(T[:, 1:], 0.0, first_step=1, launch=hsim.LAUNCH_PLAIN)
    torch.cuda.synchronize()
    assert b.status() == 0
    sig = b.sigma()
    for r, rid in enumerate(ids):
        ref = oracle.run(lat, T[r], [0.0, 0.0], 7, seed=12, replica=rid, init="cold",
                         policies=[(oracle.POLICY_ADAPTIVE, 2.0)], sigma_min=0.05, sigma_max=3.0)
        assert np.array_equal(b.spins_user(r).cpu().numpy(), ref["spins"])
        assert sig[r] == ref["sigma"]


@pytest.mark.parametrize("R", [64, 20], ids=["64-lane rows", "32-lane rows"])
@pytest.mark.parametrize("pol", POLS, ids=POL_IDS)
def test_fp32_replica_lane_one_mcs_matches_oracle(R, pol):
    """One MCS from a shared start: the replica-lane kernel under each policy
    decides as the oracle's double-precision evaluation of the same map except
    at near ties and their later neighbours (tests/_ties.py); accepted spins
    agree to single-precision accuracy."""
    lat = synth.sc_periodic(12)
    lat.k = 0.2 * synth.uniform01(8, lat.n, tag=1)
    lat.axis = synth.unit_vectors(8, lat.n, tag=2)
    start = synth.random_spins(4, lat.n, batch=R).astype(np.float32).astype(np.float64)
    plan = hsim.Plan(lat)
    T = np.linspace(0.4, 3.0, R)
    b = hsim.Batch([plan] * R, seed=33, precision=hsim.FP32, layout=hsim.LAYOUT_REPLICA).bind(1, 1)
    assert b.layout == "replica"
    b.set_policies([pol])
    b.init_spins(hsim.INIT_GIVEN, start.reshape(-1, 3))
    b.run(T[:, None], 0.3, launch=hsim.LAUNCH_PLAIN)
    torch.cuda.synchronize()
    assert b.status() == 0
    h = b.history.cpu().numpy()
    colour = plan.colouring()
    for r in range(0, R, 3):
        got = b.spins_user(r).cpu().numpy()
        check_one_mcs(lat, colour, start[r], T[r], 0.3, 33, r, got, policies=[pol])
        assert h[r, 0, 0, 4] == np.sum(np.any(got != start[r], axis=1))


def test_fp32_layouts_and_launches_bit_identical_with_policies():
    """Two site types (Hinzke-Nowak, adaptive) on a 5-colour film: the site,
    block and replica layouts in plain and graph launches (and a persistent
    request, which runs as plain launches) give bit-identical spins and
    widths, and identical history between launch modes of one layout."""
    lat = synth.diluted_film(17, 3, seed=2)
    lat.k = np.full(lat.n, 0.05)
    types = (np.arange(lat.n) % 2).astype(np.int32)
    plan = hsim.Plan(lat)
    plan.set_types(types)
    pols = [(hsim.POLICY_HN, 0.6), (hsim.POLICY_ADAPTIVE, 0.4)]
    R, M = 20, 12
    T = np.linspace(0.3, 2.5, R)[:, None] * np.ones((1, 2))
    out = {}
    for name, layout, launch in (("site", hsim.LAYOUT_SITE, hsim.LAUNCH_PLAIN),
                                 ("site_graph", hsim.LAYOUT_SITE, hsim.LAUNCH_GRAPH),
                                 ("block", hsim.LAYOUT_BLOCK, hsim.LAUNCH_PLAIN),
                                 ("rep", hsim.LAYOUT_REPLICA, hsim.LAUNCH_PLAIN),
                                 ("rep_graph", hsim.LAYOUT_REPLICA, hsim.LAUNCH_GRAPH),
                                 ("rep_persist", hsim.LAYOUT_REPLICA, hsim.LAUNCH_PERSISTENT)):
        b = hsim.Batch([plan] * R, seed=21, precision=hsim.FP32, layout=layout).bind(2, M)
        b.set_policies(pols)
        b.init_spins(hsim.INIT_RANDOM)
        b.run(T, 0.1, recompute_every=5, launch=launch)
        torch.cuda.synchronize()
        assert b.status() == 0, name
        out[name] = (np.stack([b.spins_user(r).cpu().numpy() for r in range(R)]),
                     b.history.cpu().numpy(), b.sigma())
    ref_s, _, ref_sig = out["site"]
    for name, (s, h, sig) in out.items():
        assert np.array_equal(s, ref_s), name
        assert np.array_equal(sig, ref_sig), name
        assert np.array_equal(h[..., 4], out["site"][1][..., 4]), name
    assert np.array_equal(out["site"][1], out["site_graph"][1])
    assert np.array_equal(out["rep"][1], out["rep_graph"][1])
    assert np.array_equal(out["rep"][1], out["rep_persist"][1])
    assert np.all((ref_sig >= hsim.SIGMA_MIN) & (ref_sig <= hsim.SIGMA_MAX))


def test_fp32_adaptive_holds_half_acceptance():
    """SC 16^3, 64 replicas at T = 0.5..1.3 (where the random move accepts
    well under one half), adaptive move from sigma = 3: after 100 MCS every
    replica accepts one half of its moves (within 3 points)."""
    lat = synth.sc_periodic(16)
    R, M = 64, 200
    T = np.linspace(0.5, 1.3, R)
    plan = hsim.Plan(lat)
    b = hsim.Batch([plan] * R, seed=7, precision=hsim.FP32, layout=hsim.LAYOUT_REPLICA).bind(1, M)
    b.set_policies([(hsim.POLICY_ADAPTIVE, 3.0)])
    b.init_spins(hsim.INIT_COLD_Z)
    b.run(T[:, None], 0.0, launch=hsim.LAUNCH_GRAPH)
    torch.cuda.synchronize()
    assert b.status() == 0
    acc = b.history.cpu().numpy()[:, 0, M // 2:, 4].mean(axis=1) / lat.n
    assert np.all(np.abs(acc - 0.5) < 0.03), acc
    sig = b.sigma()
    assert np.all((sig > hsim.SIGMA_MIN) & (sig < hsim.SIGMA_MAX))
    # widths shrink as the temperature falls
    assert np.corrcoef(T, sig)[0, 1] > 0.9
