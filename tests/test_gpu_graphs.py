"""Graph launches through the C-ABI.

  * GRAPH mode keeps its instantiated graph across calls: a run split into
    several GRAPH calls (the graph captured by the first and replayed by the
    later ones), with a rebind and new optional outputs in between, gives the
    spins and history of plain launches bit for bit.
  * A caller may record hsim_batch_run itself into a graph of its own (here a
    torch CUDA graph, runs made in AUTO mode and as one persistent launch):
    the schedule travels inside the recorded work, and every replay, with
    eager work and synchronisation between replays, equals the same run made
    eagerly in the same mode bit for bit (and, for the persistent launch, the
    plain launches' spins and accept counts, with energies and
    magnetisations within rounding).
"""
import numpy as np
import pytest
import torch

import synth
from paper_1803_07030_amd import hsim

pytestmark = pytest.mark.gpu


def _spins(b):
    return np.stack([b.spins_user(r).cpu().numpy() for r in range(b.R)])


@pytest.mark.parametrize("layout", [hsim.LAYOUT_REPLICA, hsim.LAYOUT_SITE])
def test_graph_reused_across_calls_equals_plain(layout):
    lat = synth.sc_periodic(10)
    lat.k = np.full(lat.n, 0.1)
    plan = hsim.Plan(lat)
    R, M, S = 20, 12, 4
    T = np.linspace(0.4, 2.4, R)[:, None] * np.ones((1, S))
    Bf = np.linspace(-0.3, 0.3, S)[None, :] * np.ones((R, 1))
    out = {}
    for launch in (hsim.LAUNCH_PLAIN, hsim.LAUNCH_GRAPH):
        b = hsim.Batch([plan] * R, seed=9, precision=hsim.FP32, layout=layout).bind(S, M)
        b.init_spins(hsim.INIT_RANDOM)
        for s in range(S):                      # one call per step: later calls replay
            if s == 2:                          # new outputs drop the cached graph
                b.bind_outputs(snapshots=True)
            b.run(T[:, s:s + 1], Bf[:, s:s + 1], first_step=s, recompute_every=4, launch=launch)
        torch.cuda.synchronize()
        assert b.status() == 0
        out[launch] = (_spins(b), b.history.cpu().numpy(), b.snapshots.cpu().numpy())
    for a, c in zip(out[hsim.LAUNCH_PLAIN], out[hsim.LAUNCH_GRAPH]):
        assert np.array_equal(a, c)


@pytest.mark.parametrize("launch", [hsim.LAUNCH_AUTO, hsim.LAUNCH_PERSISTENT])
def test_caller_records_a_run_into_its_own_graph(launch):
    lat = synth.sc_periodic(12)
    lat.k = np.full(lat.n, 0.05)
    plan = hsim.Plan(lat)
    R, M, S = 24, 10, 2
    T = np.linspace(0.5, 2.0, R)[:, None] * np.ones((1, S))
    Bf = np.full((R, S), 0.2)
    # eager references: the same launch mode (bit for bit) and, for the
    # persistent launch, plain launches (the same spins and accept counts;
    # energies and magnetisations within rounding)
    eager = [hsim.LAUNCH_PLAIN] if launch == hsim.LAUNCH_AUTO else [launch, hsim.LAUNCH_PLAIN]
    rec = hsim.Batch([plan] * R, seed=4, precision=hsim.FP32).bind(S, M)
    refs = [hsim.Batch([plan] * R, seed=4, precision=hsim.FP32).bind(S, M) for _ in eager]
    assert rec.layout == "replica"
    for b in [rec] + refs:
        b.init_spins(hsim.INIT_RANDOM)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="thread_local"):
        rec.run(T, Bf, recompute_every=5, launch=launch)
    # nothing ran during the recording
    assert np.all(rec.history.cpu().numpy() == 0.0)
    for k in range(3):
        # a replay repeats the recorded steps (same random words) from the
        # current spins; the eager references do the same
        g.replay()
        for ref, mode in zip(refs, eager):
            ref.run(T, Bf, recompute_every=5, launch=mode)
        torch.cuda.synchronize()
        assert rec.status() == 0 and all(ref.status() == 0 for ref in refs)
        # eager work between replays
        h = rec.history.cpu().numpy()
        assert np.array_equal(_spins(rec), _spins(refs[0])), k
        assert np.array_equal(h, refs[0].history.cpu().numpy()), k
        if len(refs) > 1:
            hp = refs[1].history.cpu().numpy()
            assert np.array_equal(_spins(rec), _spins(refs[1])), k
            assert np.array_equal(h[..., 4], hp[..., 4]), k
            assert np.allclose(h, hp, rtol=0, atol=1e-9 * lat.n), (k, float(np.abs(h - hp).max()))
        # a run with another schedule between replays must not leak into them
        other = hsim.Batch([plan] * R, seed=5, precision=hsim.FP32).bind(S, M)
        other.init_spins(hsim.INIT_COLD_Z)
        other.run(T * 2.0, -Bf, launch=hsim.LAUNCH_GRAPH)
        torch.cuda.synchronize()
