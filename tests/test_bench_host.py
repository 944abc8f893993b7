"""Host-side checks of the benchmark's bookkeeping and of lattices without
sites (no GPU needed): the algorithmic-byte models, the source hash that
keys the committed byte counters, the single-GPU guard, and plan and batch
sizes of an empty lattice."""
import json
import os
import subprocess
import sys

import pytest

import bench
import synth
from paper_1803_07030_amd import hsim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_models():
    # replica-lane: own spin + neighbour spins once per MCS + write on accept
    # + the row (offset and z (column, J) pairs) shared by the lanes
    assert bench.b_alg_replica_lane(6.0, 0.5, 64) == pytest.approx(24 + 6 + 52 / 64)
    assert bench.b_alg_replica_lane(6.0, 0.0, 32) == pytest.approx(24 + 52 / 32)
    # site-lane: user index + row + own and neighbour spins + write on accept
    assert bench.b_alg_site_lane(5.0, 0.25) == pytest.approx(4 + 40 + 24 + 3)


def test_kernel_hash_ignores_comments_only():
    code = "int f(int a) { return a + 1; }"
    assert bench._code_only(code) == bench._code_only(
        "// lead\nint f(int a) /* args */ {\n  return a + 1;  // one\n}\n")
    assert bench._code_only(code) != bench._code_only(code.replace("+ 1", "+ 2"))


def test_committed_traffic_matches_the_kernel_sources():
    """The byte counters in profiles/ were taken on the kernel as it is now;
    their algorithmic bytes follow the replica-lane model."""
    t = bench.measured_traffic()
    if t is None:
        pytest.skip("the committed byte counters predate the current kernel sources "
                    "(bench.py then reports roofline.traffic as null)")
    assert t["kernel_hash"] == bench.kernel_hash()
    assert t["updates_per_launch"] == 131072 * 64
    assert 1.0 < t["bytes_per_launch"] / t["algorithmic_bytes_per_launch"] < 2.0
    with open(os.path.join(ROOT, "profiles", "rep_phase_traffic.json")) as fh:
        assert json.load(fh)["fetch_scale"] == pytest.approx(2.0, rel=1e-3)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_empty_lattice_plan_and_batch_sizes():
    plan = hsim.Plan(synth.isolated(0))
    assert plan.info.n_sites == 0 and plan.info.n_colours == 0 and plan.info.n_bonds == 0
    for layout in (hsim.LAYOUT_SITE, hsim.LAYOUT_BLOCK, hsim.LAYOUT_REPLICA):
        prec = hsim.FP32 if layout == hsim.LAYOUT_REPLICA else hsim.FP64_EXACT
        b = hsim.hsim_batch_create([plan.handle] * 20, 1, None, prec, layout)
        try:
            ws, sp, hist = hsim.hsim_batch_sizes(b, 2, 3)
            assert hist == 20 * 2 * 3 * 5 * 8
            assert ws > 0 and sp > 0
        finally:
            hsim.hsim_batch_destroy(b)
