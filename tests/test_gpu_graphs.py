"""Graph launches through the C-ABI.

  * GRAPH mode keeps its instantiated graph across calls: a run split into
    several GRAPH calls (the graph captured by the first and replayed by the
    later ones), with a rebind and new optional outputs in between, gives the
    spins and history of plain launches bit for bit.
  * A caller may record hsim_batch_run itself into a graph of its own (here a
    torch CUDA graph, run made in AUTO mode): the schedule travels inside the
    recorded work, and every replay, with eager work and synchronisation
    between replays, equals the same run made eagerly.
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


def test_caller_records_an_auto_run_into_its_own_graph():
    lat = synth.sc_periodic(12)
    lat.k = np.full(lat.n, 0.05)
    plan = hsim.Plan(lat)
    R, M, S = 24, 10, 2
    T = np.linspace(0.5, 2.0, R)[:, None] * np.ones((1, S))
    Bf = np.full((R, S), 0.2)
    rec = hsim.Batch([plan] * R, seed=4, precision=hsim.FP32).bind(S, M)
    ref = hsim.Batch([plan] * R, seed=4, precision=hsim.FP32).bind(S, M)
    assert rec.layout == "replica"
    for b in (rec, ref):
        b.init_spins(hsim.INIT_RANDOM)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="thread_local"):
        rec.run(T, Bf, recompute_every=5, launch=hsim.LAUNCH_AUTO)
    # nothing ran during the recording
    assert np.all(rec.history.cpu().numpy() == 0.0)
    for k in range(3):
        # a replay repeats the recorded steps (same random words) from the
        # current spins; the eager reference does the same
        g.replay()
        ref.run(T, Bf, recompute_every=5, launch=hsim.LAUNCH_PLAIN)
        torch.cuda.synchronize()
        assert rec.status() == 0 and ref.status() == 0
        # eager work between replays
        assert np.array_equal(_spins(rec), _spins(ref)), k
        assert np.array_equal(rec.history.cpu().numpy(), ref.history.cpu().numpy()), k
        # a run with another schedule between replays must not leak into them
        other = hsim.Batch([plan] * R, seed=5, precision=hsim.FP32).bind(S, M)
        other.init_spins(hsim.INIT_COLD_Z)
        other.run(T * 2.0, -Bf, launch=hsim.LAUNCH_GRAPH)
        torch.cuda.synchronize()
