"""Benchmark of the batched Heisenberg Metropolis sweep on one MI355X.

Workload (one "step" = one whole run of the hot path): periodic simple-cubic
64^3 lattice (262144 unit spins), J = 1 to the 6 nearest neighbours, uniaxial
K = 0.1 along z, B = 0; 64 replicas at temperatures 0.1 -> 3.0 (one per
replica), cold start, seed 1, 10^4 MCS per replica, single-precision spins and
fields with a double-precision history of (E, M, accepted) after every MCS;
all replicas in one batch (replica-lane layout), one launch per colour phase.

Printed: one JSON line with the throughput (attempted spin updates per second,
inputs resident in HBM), the per-replica plain-launch rate on a bounded sample,
the roofline of the dominant kernel (one colour phase of all replicas: HBM,
algorithmic bytes per update over its average launch duration, timed with HIP
events on the stream it runs on, every n-th MCS of the timed region) and the
CPU oracle's rate on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin updates/sec (batched replicas) vs plain launch; % HBM roofline; obs err"
HBM_PEAK_GBS = 8000.0
L, R, MCS, K_ANI, SEED = 64, 64, 10000, 0.1, 1


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mcs", type=int, default=MCS, help="MCS per replica per step")
    ap.add_argument("--size", type=int, default=L,
                    help="edge of the simple-cubic lattice of the sc64 workload (64: the headline)")
    ap.add_argument("--launch", default="plain", choices=["persistent", "graph", "plain", "auto"])
    ap.add_argument("--shape", default=None,
                    help="replica tiles: 'SPW,MASKED' (sites per wave 4/8/32, store policy 0/1)")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the tile shape and store policy before timing (untimed)")
    ap.add_argument("--time-every", type=int, default=None,
                    help="plain launch: time every n-th MCS's colour-phase launches with HIP events "
                         "(default 10; films 0: their roofline is taken over the whole step)")
    ap.add_argument("--plain-mcs", type=int, default=8, help="MCS per replica of the plain-launch sample")
    ap.add_argument("--cpu-mcs", type=int, default=400, help="MCS per thread of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--policy", default="random",
                    choices=["random", "flip", "small_step", "gaussian", "hn", "adaptive"],
                    help="update policy of every site (sc64 workload): random (the headline), "
                         "flip, small step (30 degrees), Gaussian (sigma 0.5), Hinzke-Nowak "
                         "(30 degrees), adaptive (sigma from 1.0)")
    ap.add_argument("--workload", default="sc64",
                    choices=["sc64", "films", "policies", "ball", "validation", "energy"],
                    help="sc64: the headline workload; films: 256 diluted films, one replica "
                         "each (site-lane layout), for the site-lane kernel's numbers; policies: "
                         "equilibrium correlation times of every update policy; ball: the "
                         "core/shell hysteresis run (32 seeds, 401 field steps); validation: the "
                         "double-precision SC 8^3 run against the oracle's time; energy: the "
                         "energy forward and backward over 1024 configurations of SC 32^3")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB (HBM byte-counter calibration)")
    return ap.parse_args()


def copy_calibration():
    """A plain device-to-device copy of a known size: the reference for
    scaling the HBM byte counters (FETCH_SIZE / WRITE_SIZE) of the sweep."""
    import torch
    n = 1 << 28                                    # 2^28 floats = 1 GiB
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 3}))


def copy_bandwidth(stream, resident_bytes):
    """Device-copy bandwidth on this GPU, the practical ceilings the sweep is
    compared with: a 1 GiB copy (2 GiB moved, far beyond the 256 MB
    last-level cache: HBM-bound) and a copy whose source plus destination
    equal the spin set (cache-resident like the sweep's data).  GB/s counts
    bytes read plus bytes written."""
    import torch
    out = {}
    for name, nbytes in (("hbm_copy", 1 << 30), ("resident_copy", resident_bytes // 2)):
        n = nbytes // 4
        with torch.cuda.stream(stream):
            a = torch.ones(n, dtype=torch.float32, device="cuda")
            b = torch.empty_like(a)
            for _ in range(3):
                b.copy_(a)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            reps = 20
            e0.record(stream)
            for _ in range(reps):
                b.copy_(a)
            e1.record(stream)
        stream.synchronize()
        out[name + "_GBps"] = 2 * 4 * n * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
        out[name + "_bytes"] = 2 * 4 * n
        del a, b
    torch.cuda.empty_cache()
    return out


# Sources of the dominant kernel; the committed byte counts in
# profiles/rep_phase_traffic.json are used only while these hash the same.
KERNEL_SOURCES = ["paper_1803_07030_amd/csrc/rep_kernels.hip", "paper_1803_07030_amd/csrc/update.h",
                  "paper_1803_07030_amd/csrc/hsim_dev.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rep_phase_traffic.json")


def _code_only(text):
    """C++ source without comments and with whitespace runs collapsed, so that
    an edit of comments alone keeps the hash."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per colour-phase launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, calibrated on a plain copy), or None if the
    kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t


def workload(size=L):
    import synth
    lat = synth.sc_periodic(size)
    lat.k = np.full(lat.n, K_ANI)
    T = synth.replica_temperatures(R, 0.1, 3.0)
    return lat, T


def b_alg_replica_lane(zbar, a, lanes):
    """Algorithmic bytes per attempted update, replica-lane layout: own spin
    (12) + neighbour spins counted once per MCS (12) + write on accept (12 a)
    + the lattice row (4 B offset + 8 B per neighbour: column and J) shared by
    the lanes."""
    return 24.0 + 12.0 * a + (4.0 + 8.0 * zbar) / lanes


def main():
    args = parse()
    if args.time_every is None and args.workload != "films":
        args.time_every = 10
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(replicas shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1803_07030_amd import hsim
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    stream = torch.cuda.Stream()
    if args.workload == "films":
        films_bench(args, stream)
        return
    if args.workload == "policies":
        policies_bench(args, stream)
        return
    if args.workload == "ball":
        ball_bench(args, stream)
        return
    if args.workload == "validation":
        validation_bench(args, stream)
        return
    if args.workload == "energy":
        energy_bench(args, stream)
        return
    lat, T = workload(args.size)
    launch = dict(persistent=hsim.LAUNCH_PERSISTENT, graph=hsim.LAUNCH_GRAPH,
                  plain=hsim.LAUNCH_PLAIN, auto=hsim.LAUNCH_AUTO)[args.launch]
    with torch.cuda.stream(stream):
        plan = hsim.Plan(lat)
        batch = hsim.Batch([plan] * R, seed=SEED, precision=hsim.FP32,
                           layout=hsim.LAYOUT_REPLICA).bind(1, args.mcs)
        if args.policy != "random":
            pol = {"flip": (hsim.POLICY_FLIP, 0.0), "small_step": (hsim.POLICY_SMALL_STEP, np.pi / 6),
                   "gaussian": (hsim.POLICY_GAUSSIAN, 0.5), "hn": (hsim.POLICY_HN, np.pi / 6),
                   "adaptive": (hsim.POLICY_ADAPTIVE, 1.0)}[args.policy]
            batch.set_policies([pol])
        Tm = T[:, None]
        timed_phases = args.launch == "plain" and args.time_every > 0
        if args.shape:
            spw, masked = (int(x) for x in args.shape.split(","))
            batch.set_shape(spw, masked)
        if args.launch == "auto" or args.tune:
            batch.init_spins(hsim.INIT_COLD_Z)
            batch.run(Tm, 0.0, recompute_every=100, launch=hsim.LAUNCH_PLAIN)   # stage T for the trials
            batch.autotune(trial_mcs=20)         # untimed: picks the shape and the launch AUTO uses

        def one_step():
            batch.init_spins(hsim.INIT_COLD_Z)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            batch.run(Tm, 0.0, recompute_every=100, launch=launch)
            e1.record(stream)
            return e0, e1

        for _ in range(args.warmup):
            one_step()
        stream.synchronize()
        assert batch.status() == 0
        torch.cuda.synchronize()
        if timed_phases:
            batch.phase_times()                  # drop anything recorded before
            batch.time_phases(args.time_every)
        t0 = time.perf_counter()
        evs = [one_step() for _ in range(args.steps)]
        stream.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        assert batch.status() == 0
        step_ms = [a.elapsed_time(b) for a, b in evs]
        if timed_phases:
            ph_ms, ph_n, ph_upd = batch.phase_times()
            batch.time_phases(0)
        hist = batch.history.cpu().numpy()
    n_upd_step = R * lat.n * args.mcs
    value = n_upd_step * args.steps / wall
    acc = float(hist[..., 4].mean() / lat.n)
    zbar = lat.mean_degree
    balg = b_alg_replica_lane(zbar, acc, 64)
    if timed_phases:
        # dominant kernel: one colour phase of all replicas (k_rep_phase)
        kernel = "k_rep_phase"
        launch_ms = ph_ms / ph_n
        upd_per_launch = ph_upd / ph_n
    else:
        # persistent: one launch per step; graph: the step's launches together
        kernel = "k_rep_persistent" if args.launch == "persistent" else "step"
        launch_ms = float(np.mean(step_ms))
        upd_per_launch = n_upd_step
    achieved = balg * upd_per_launch / (launch_ms / 1e3) / 1e9
    # the committed byte counters are for the 64^3 headline lattice only
    tr = measured_traffic() if kernel == "k_rep_phase" and args.size == L else None
    out = {
        "metric": METRIC, "value": value, "unit": "spin updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"sc{args.size}^3 periodic J=1 K={K_ANI} z, {R} replicas T=0.1..3.0, "
                               f"{args.mcs} MCS, cold start, f32 spins, f64 history, "
                               f"{args.launch} launch, replica-lane layout"
                               + ("" if args.policy == "random" else f", {args.policy} move"),
                   "sites": lat.n, "replicas": R, "mcs": args.mcs,
                   "updates_per_step": n_upd_step, "launch": args.launch, "policy": args.policy,
                   "sites_per_wave": int(batch.info.sites_per_wave),
                   "masked_store": int(batch.info.masked_store),
                   "tuned": bool(args.launch == "auto" or args.tune)},
        "acceptance": acc,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if tr is None else tr["bytes_per_launch"],
                     "kernel": kernel, "launch_ms": launch_ms,
                     "updates_per_launch": upd_per_launch, "bytes_per_update": balg,
                     "timed_launches": ph_n if timed_phases else args.steps},
    }
    if tr is not None:
        out["roofline"]["traffic_vs_algorithmic"] = tr["bytes_per_launch"] / (balg * upd_per_launch)
    cb = copy_bandwidth(stream, 3 * 4 * lat.n * 64)
    cb["frac_achieved_vs_hbm_copy"] = achieved / cb["hbm_copy_GBps"]
    if tr is not None:
        cb["traffic_GBps"] = tr["bytes_per_launch"] / (launch_ms / 1e3) / 1e9
        cb["frac_traffic_vs_resident_copy"] = cb["traffic_GBps"] / cb["resident_copy_GBps"]
    out["copy_roofline"] = cb
    if not args.no_plain:
        out["plain_launch"] = plain_launch(lat, T, args.plain_mcs, stream)
        out["vs_plain_launch"] = value / out["plain_launch"]["value"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(lat, T, args.cpu_mcs, hist)
    print(json.dumps(out))


def b_alg_site_lane(zbar, a):
    """Algorithmic bytes per attempted update, site-lane layout, per-bond J:
    user index (4) + row of zbar (column, J) pairs (8 zbar) + own spin (12) +
    neighbour spins counted once per MCS (12) + write on accept (12 a)."""
    return 4.0 + 8.0 * zbar + 24.0 + 12.0 * a


def films_bench(args, stream):
    """256 diluted films (L in 16..128, d in 2..10, 10% vacancies, per-bond J
    in [0.5, 1.5], K = 0.05 z), each film one replica at its own temperature
    in [0.2, 2.0], single precision, site-lane layout.  The roofline is taken
    over the whole step; with --time-every n, plain launches also time the
    colour-phase launches of every n-th MCS."""
    import torch
    import synth
    from paper_1803_07030_amd import hsim
    mcs = args.mcs if args.mcs != MCS else 1000
    films, Ts = synth.film_batch()
    nsites = sum(f.n for f in films)
    zbar = sum(f.nnz for f in films) / nsites
    launch = dict(persistent=hsim.LAUNCH_PERSISTENT, graph=hsim.LAUNCH_GRAPH,
                  plain=hsim.LAUNCH_PLAIN, auto=hsim.LAUNCH_AUTO)[args.launch]
    if launch == hsim.LAUNCH_PERSISTENT:
        sys.exit("the persistent launch needs the replica layout; films use the site layout")
    every = 0 if args.time_every is None else args.time_every
    timed_phases = launch == hsim.LAUNCH_PLAIN and every > 0
    with torch.cuda.stream(stream):
        plans = [hsim.Plan(f) for f in films]
        batch = hsim.Batch(plans, seed=3, precision=hsim.FP32, layout=hsim.LAYOUT_SITE).bind(1, mcs)
        Tm = np.asarray(Ts)[:, None]
        if launch == hsim.LAUNCH_AUTO:
            batch.autotune(trial_mcs=20)
        for _ in range(args.warmup):
            batch.init_spins(hsim.INIT_COLD_Z)
            batch.run(Tm, 0.0, launch=launch)
        stream.synchronize()
        if timed_phases:
            batch.phase_times()
            batch.time_phases(every)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            batch.init_spins(hsim.INIT_COLD_Z)
            batch.run(Tm, 0.0, launch=launch)
        stream.synchronize()
        wall = time.perf_counter() - t0
        assert batch.status() == 0
        if timed_phases:
            ph_ms, ph_n, ph_upd = batch.phase_times()
            batch.time_phases(0)
        hist = batch.history.cpu().numpy()
    acc = float(hist[..., 4].sum() / (nsites * mcs))
    balg = b_alg_site_lane(zbar, acc)
    # the films with trailing colour classes and the others run as two groups
    # on two streams, so single phase launches overlap the other group's
    # work: the roofline is taken over the whole step, and the sampled
    # phase-launch times are reported beside it
    kernel, launch_ms, upd, n_timed = "step", wall / args.steps * 1e3, nsites * mcs, args.steps
    achieved = balg * upd / (launch_ms / 1e3) / 1e9
    phases = None
    if timed_phases:
        phases = {"kernel": "k_site_phase", "launch_ms": ph_ms / ph_n, "updates_per_launch": ph_upd / ph_n,
                  "timed_launches": ph_n,
                  "achieved_GBps": balg * (ph_upd / ph_n) / (ph_ms / ph_n / 1e3) / 1e9}
    print(json.dumps({
        "metric": "spin updates/sec, site-lane films batch", "value": nsites * mcs * args.steps / wall,
        "unit": "spin updates/s", "steps": args.steps, "warmup": args.warmup,
        "config": {"workload": f"256 diluted films, {nsites} sites, {mcs} MCS, f32, site-lane, "
                               f"{args.launch} launch",
                   "sites": nsites, "mean_degree": zbar, "launch": args.launch,
                   "tuned_launch": {-1: None, 0: "plain", 1: "persistent", 2: "graph"}.get(
                       int(batch.info.tuned_launch))},
        "acceptance": acc,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "kernel": kernel,
                     "launch_ms": launch_ms, "updates_per_launch": upd,
                     "bytes_per_update": balg, "timed_launches": n_timed},
        "phase_launches": phases}))


def ball_bench(args, stream):
    """Core/shell sphere cut from SC (R = 20, 33,401 sites; core J = 1, shell
    0.3, interface -0.5; core K = 0.01 z, radial K = 1 on surface sites), 32
    seeds at T = 0.1, the field swept +2 -> -2 -> +2 in 401 steps of `mcs`
    MCS (default 200), single precision, replica-lane layout with 32-lane
    rows.  The spins (12.8 MB) stay in the caches: no HBM roofline."""
    import torch
    import synth
    from paper_1803_07030_amd import hsim
    R, S = 32, 401
    M = args.mcs if args.mcs != MCS else 200
    lat = synth.core_shell_ball()
    Bs = synth.hysteresis_fields(S)
    launch = dict(persistent=hsim.LAUNCH_PERSISTENT, graph=hsim.LAUNCH_GRAPH,
                  plain=hsim.LAUNCH_PLAIN, auto=hsim.LAUNCH_AUTO)[args.launch]
    timed = launch == hsim.LAUNCH_PLAIN and args.time_every > 0
    with torch.cuda.stream(stream):
        plan = hsim.Plan(lat)
        b = hsim.Batch([plan] * R, seed=2, precision=hsim.FP32, layout=hsim.LAYOUT_REPLICA).bind(S, M)
        if launch == hsim.LAUNCH_AUTO:
            b.autotune(trial_mcs=20)
        for _ in range(args.warmup):
            b.init_spins(hsim.INIT_COLD_Z)
            b.run(np.full((R, 2), 0.1), np.repeat(Bs[None, :2], R, 0), launch=launch)
        stream.synchronize()
        if timed:
            b.phase_times()
            b.time_phases(args.time_every)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.init_spins(hsim.INIT_COLD_Z)
            b.run(np.full((R, S), 0.1), np.repeat(Bs[None, :], R, 0), launch=launch)
        stream.synchronize()
        wall = time.perf_counter() - t0
        assert b.status() == 0
        ph = b.phase_times() if timed else None
        b.time_phases(0)
        mz = b.history.cpu().numpy()[..., -1, 3].mean(axis=0) / lat.n   # <M_z>/N at each step end
    upd = R * S * M * lat.n * args.steps
    print(json.dumps({
        "metric": "spin updates/sec, core/shell hysteresis batch", "value": upd / wall,
        "unit": "spin updates/s", "steps": args.steps, "warmup": args.warmup,
        "config": {"workload": f"core/shell ball R=20, {lat.n} sites, 32 seeds, T=0.1, {S} field "
                               f"steps x {M} MCS, f32, replica-lane, {args.launch} launch",
                   "sites": lat.n, "launch": args.launch},
        "phase_us": None if ph is None else ph[0] / ph[1] * 1e3,
        "updates_per_phase": None if ph is None else ph[2] / ph[1],
        "mz_at_B": {"+2": float(mz[0]), "0 (down)": float(mz[S // 4]), "-2": float(mz[S // 2]),
                    "0 (up)": float(mz[3 * S // 4])}}))


def validation_bench(args, stream):
    """The double-precision validation run: SC 8^3, J = 1, random start
    (seed 0), 20 temperatures 3.0 -> 0.1 of 1000 MCS, one replica in the
    block layout (spins in LDS); its CPU baseline is the oracle on one host
    thread over the same run, whose accept counts must equal the GPU's."""
    import torch
    import oracle
    import synth
    from paper_1803_07030_amd import hsim
    lat = synth.sc_periodic(8)
    T = synth.cooling_schedule(20)
    M = 1000
    with torch.cuda.stream(stream):
        plan = hsim.Plan(lat)
        b = hsim.Batch([plan], seed=0, precision=hsim.FP64_EXACT, layout=hsim.LAYOUT_BLOCK).bind(20, M)
        for _ in range(max(args.warmup, 1)):
            b.init_spins(hsim.INIT_RANDOM)
            b.run(T, 0.0, launch=hsim.LAUNCH_PLAIN)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.init_spins(hsim.INIT_RANDOM)
            b.run(T, 0.0, launch=hsim.LAUNCH_PLAIN)
        stream.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        assert b.status() == 0
        h = b.history.cpu().numpy()[0]
    t0 = time.perf_counter()
    ref = oracle.run(lat, T, 0.0, M, seed=0, init="random")
    t_or = time.perf_counter() - t0
    upd = lat.n * 20 * M
    print(json.dumps({
        "metric": "spin updates/sec, FP64 validation run", "value": upd / wall,
        "unit": "spin updates/s", "steps": args.steps,
        "config": {"workload": "sc8^3 J=1, random start seed 0, 20 temperatures 3.0..0.1 x 1000 MCS, "
                               "f64, block layout, one replica"},
        "ms_per_run": wall * 1e3,
        "cpu_baseline": {"value": upd / t_or, "unit": "spin updates/s", "cores": 1, "kind": "oracle",
                         "sample": "the whole run", "ms_per_run": t_or * 1e3,
                         "accept_counts_equal": bool(np.array_equal(h[..., 4], ref["history"][..., 4]))}}))


def energy_bench(args, stream):
    """Energy forward and backward (dE/dS, dE/dJ, dE/dk, dE/dB) of 1024
    configurations of SC 32^3 with per-bond J ~ N(1, 0.1), per-site K and
    axes, B = 0.5 z, single precision.  Algorithmic bytes per
    site-configuration: 12 read (forward), 12 read + 12 written (backward);
    the lattice tables are shared by the batch and not counted."""
    import torch
    import synth
    from paper_1803_07030_amd import hsim
    lat = synth.gradient_lattice(L=32, seed=4)
    nb = 1024
    reps = max(args.steps, 1) * 10
    with torch.cuda.stream(stream):
        plan = hsim.Plan(lat)
        _, _, Jb = lat.bonds()
        S = torch.tensor(synth.random_spins(44, lat.n, batch=nb).astype(np.float32).transpose(0, 2, 1).copy(),
                         device="cuda")
        J = torch.tensor(Jb, dtype=torch.float32, device="cuda")
        k = torch.tensor(lat.k, dtype=torch.float32, device="cuda")
        ax = torch.tensor(lat.axis.T.copy(), dtype=torch.float32, device="cuda")
        E = torch.empty(nb, dtype=torch.float64, device="cuda")
        gE = torch.ones(nb, dtype=torch.float64, device="cuda")
        gS, gJ, gk = torch.empty_like(S), torch.empty_like(J), torch.empty_like(k)
        gB = torch.empty(1, dtype=torch.float64, device="cuda")

        def fwd():
            hsim.hsim_energy_forward(plan.handle, nb, hsim.FP32, S, J, k, ax, 0.5, None, E)

        def bwd():
            hsim.hsim_energy_backward(plan.handle, nb, hsim.FP32, S, J, k, ax, 0.5, None, gE,
                                      gS, gJ, gk, gB)

        res = {}
        for name, fn, bytes_per in (("forward", fwd, 12.0), ("backward", bwd, 24.0)):
            for _ in range(max(args.warmup, 1)):
                fn()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            stream.synchronize()
            ms = e0.elapsed_time(e1) / reps
            gbs = bytes_per * nb * lat.n / (ms / 1e3) / 1e9
            res[name] = {"ms_per_call": ms, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "bytes_per_site_config": bytes_per}
    print(json.dumps({
        "metric": "energy forward/backward bandwidth", "unit": "GB/s",
        "config": {"workload": f"sc32^3, per-bond J ~ N(1, 0.1), per-site K and axes, B=0.5 z, "
                               f"{nb} configurations, f32", "sites": lat.n, "batch": nb},
        "calls_timed": reps, **res}))


def policies_bench(args, stream):
    """Equilibrium correlation times per update policy: SC 32^3 periodic,
    J = 1, K = 0.1 z, 64 replicas at T = 0.4 .. 1.4 (below the ordering
    temperature, about 1.44), cold start, one step of `mcs` MCS to
    equilibrate, then `mcs` MCS measured; integrated autocorrelation times of
    E and |M| by the library's analysis (Sokal window, c = 6), and the sweep
    rate."""
    import torch
    import synth
    from paper_1803_07030_amd import hsim
    L, R = 32, 64
    mcs = args.mcs if args.mcs != MCS else 4000
    lat = synth.sc_periodic(L)
    lat.k = np.full(lat.n, K_ANI)
    T = np.linspace(0.4, 1.4, R)
    pols = {"random": None, "small_step_15deg": (hsim.POLICY_SMALL_STEP, np.pi / 12),
            "small_step_30deg": (hsim.POLICY_SMALL_STEP, np.pi / 6),
            "gaussian_0.2": (hsim.POLICY_GAUSSIAN, 0.2),
            "hinzke_nowak_15deg": (hsim.POLICY_HN, np.pi / 12),
            "hinzke_nowak_30deg": (hsim.POLICY_HN, np.pi / 6),
            "adaptive": (hsim.POLICY_ADAPTIVE, 1.0)}
    res = {}
    with torch.cuda.stream(stream):
        plan = hsim.Plan(lat)
        for name, pol in pols.items():
            b = hsim.Batch([plan] * R, seed=SEED, precision=hsim.FP32,
                           layout=hsim.LAYOUT_REPLICA).bind(2, mcs)
            if pol is not None:
                b.set_policies([pol])
            b.init_spins(hsim.INIT_COLD_Z)
            Tm = np.stack([T, T], axis=1)
            stream.synchronize()
            t0 = time.perf_counter()
            b.run(Tm[:, :1], 0.0, first_step=0, launch=hsim.LAUNCH_GRAPH)
            b.run(Tm[:, 1:], 0.0, first_step=1, launch=hsim.LAUNCH_GRAPH)
            stream.synchronize()
            dt = time.perf_counter() - t0
            assert b.status() == 0
            h = b.history[:, 1:2].contiguous()
            tE, _ = hsim.hsim_analysis_tau(h, 0, 0)
            tM, _ = hsim.hsim_analysis_tau(h, 0, 1)
            acc = b.history[:, 1, :, 4].mean(dim=1) / lat.n
            res[name] = {"tau_E": tE[:, 0].cpu().numpy().round(2).tolist(),
                         "tau_M": tM[:, 0].cpu().numpy().round(2).tolist(),
                         "acceptance": acc.cpu().numpy().round(3).tolist(),
                         "updates_per_s": R * lat.n * mcs * 2 / dt}
    print(json.dumps({"workload": f"sc{L}^3 K={K_ANI} z, {R} replicas T=0.4..1.4, {mcs} MCS "
                                  f"equilibration, {mcs} MCS measured, f32, replica-lane, graph",
                      "T": T.round(4).tolist(), "policies": res}))


def plain_launch(lat, T, mcs, stream):
    """Per-replica plain launches: each replica its own single-replica batch
    (site-lane kernel), one launch per (replica, MCS, colour) plus the per-MCS
    history reduction, no graph; bounded sample of mcs MCS per replica."""
    import torch
    from paper_1803_07030_amd import hsim
    with torch.cuda.stream(stream):
        plan = hsim.Plan(lat)
        batches = []
        for r in range(R):
            b = hsim.Batch([plan], seed=SEED, replica_ids=[r], precision=hsim.FP32,
                           layout=hsim.LAYOUT_SITE).bind(1, mcs)
            b.init_spins(hsim.INIT_COLD_Z)
            batches.append(b)
        batches[0].run([[T[0]]], 0.0, launch=hsim.LAUNCH_PLAIN)   # warm-up
        stream.synchronize()
        for b in batches:
            b.init_spins(hsim.INIT_COLD_Z)
        stream.synchronize()
        t0 = time.perf_counter()
        for r, b in enumerate(batches):
            b.run([[T[r]]], 0.0, launch=hsim.LAUNCH_PLAIN)
        stream.synchronize()
        dt = time.perf_counter() - t0
    upd = R * lat.n * mcs
    return {"value": upd / dt, "unit": "spin updates/s", "sample": f"{R} replicas x {mcs} MCS",
            "launches": R * mcs * (lat_colours(plan) + 1)}


def lat_colours(plan):
    return int(plan.info.n_colours)


def block_se(x, nblocks=20):
    """Mean and standard error of a correlated series from nblocks
    consecutive block means (Flyvbjerg and Petersen 1989)."""
    n = len(x) // nblocks * nblocks
    b = np.asarray(x[:n]).reshape(nblocks, -1).mean(axis=1)
    return float(b.mean()), float(b.std(ddof=1) / np.sqrt(nblocks))


def cpu_baseline(lat, T, mcs, gpu_hist):
    """The CPU oracle (double precision, exact proposal map) on a bounded
    sample: one replica per thread at the workload's temperatures, cold
    start, mcs MCS each.  Observable error of the single-precision GPU chains
    against these double-precision chains, which draw other random words
    (oracle replica ids 1000 + r): per-site energy, |M| and M_z over MCS
    mcs/5 .. mcs-1 of both (the same cold start, so the same expected
    values at every MCS), standard errors from 20 block means per chain,
    combined in quadrature.  Temperatures in [1.3, 1.6] (near the ordering
    temperature, where the correlation time is comparable to a block) are
    reported but left out of the maximum."""
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    reps = [int(r) for r in np.linspace(0, R - 1, threads).round()]
    jobs = [dict(lat=lat, T=[T[r]], B=[0.0], mcs_per_step=mcs, seed=SEED, replica=1000 + r,
                 init="cold") for r in reps]
    t0 = time.perf_counter()
    res, used = oracle.run_replicas(jobs, threads=threads)
    dt = time.perf_counter() - t0
    upd = len(jobs) * lat.n * mcs
    m0 = mcs // 5

    def series(h, name):
        if name == "M_abs_per_site":
            return np.sqrt((h[:, 1:4] ** 2).sum(axis=1)) / lat.n
        return h[:, {"E_per_site": 0, "Mz_per_site": 3}[name]] / lat.n

    obs = {}
    for name in ("E_per_site", "M_abs_per_site", "Mz_per_site"):
        dmax, zmax, per = 0.0, 0.0, []
        for r, x in zip(reps, res):
            mg, sg = block_se(series(gpu_hist[r, 0, m0:mcs], name))
            mo, so = block_se(series(x["history"][0, m0:], name))
            d = abs(mg - mo)
            se = np.hypot(sg, so)
            z = d / se if se > 0 else (0.0 if d == 0 else float("inf"))
            per.append(round(float(z), 3))
            if not 1.3 <= T[r] <= 1.6:
                dmax = max(dmax, d)
                zmax = max(zmax, z)
        obs[name] = {"max_abs_diff": dmax, "max_diff_in_se": zmax, "diff_in_se": per}
    return {"value": upd / dt, "unit": "spin updates/s", "cores": used, "kind": "oracle",
            "sample": f"{len(jobs)} replicas x {lat.n} sites x {mcs} MCS, one replica per thread",
            "seconds": dt,
            "obs_err": dict(obs, window=f"MCS {m0}..{mcs - 1}, 20 block means per chain, "
                                        "independent oracle chains (replica ids 1000 + r)",
                            replicas=reps, graded="T outside [1.3, 1.6]")}


if __name__ == "__main__":
    main()
