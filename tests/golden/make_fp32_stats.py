"""Writes tests/golden/fp32_stats.json: reference statistics of the benchmark
workloads from chains of the double-precision CPU oracle (exact proposal
map), for the single-precision GPU statistics tests.  Calls only oracle/ (and
synth/ for the inputs); the oracle's chains use replica ids the GPU runs do
not use, so the two sides are independent samples of the same ensemble
(Eq. 4's stationary distribution; section "Thermal averages").

  C1  SC 64^3, J = 1, K = 0.1 z, cold start, seed 1: eight of the 64 replica
      temperatures outside [1.3, 1.6] (near the ordering temperature the
      correlation time is comparable to a block), 2000 MCS each, oracle
      replica ids 1000 + r.
  C2  core/shell sphere R = 20 at T = 0.1, field +2 -> -2 -> +2 in 401 steps
      of 200 MCS, cold start, seed 2, 16 oracle seeds (replica ids 100..115):
      <M_z>/N of every step (its last 80% of MCS) and the coercive fields of
      both branches, mean and spread over seeds.
  C3  the 16 smallest films of the 256-film batch (generator seed 3) at their
      own temperatures, 1000 MCS, cold start, seed 3, 32 chains per film
      (oracle replica ids 1000000 + 64 f + k); mean and spread over chains.
Statistics per chain (tests/_stats.py chain_stats): 20% burn-in, 20 blocks.

Run from the repository root:  python tests/golden/make_fp32_stats.py [c1 c2 c3]
(naming parts regenerates only those and keeps the others).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import oracle  # noqa: E402
import synth  # noqa: E402
from _stats import OBSERVABLES, chain_means, chain_stats  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fp32_stats.json")
C1_REPS = [0, 8, 16, 24, 40, 48, 56, 63]
C1_MCS = 2000
C2_SEEDS = list(range(100, 116))
C3_FILMS = 16
C3_CHAINS = 32
C3_ORACLE_ID0 = 1000000


def coercive(B, mz_step):
    """Fields where the step means cross zero: first sign change on the
    descending half (steps 0..200), first on the ascending half; linear
    interpolation between the two steps."""
    half = (len(B) - 1) // 2
    out = []
    for lo, hi, sgn in ((0, half, -1), (half, len(B) - 1, 1)):
        x = np.nan
        for s in range(lo + 1, hi + 1):
            if np.sign(mz_step[s]) == sgn and np.sign(mz_step[s - 1]) != sgn:
                a, b = mz_step[s - 1], mz_step[s]
                x = B[s - 1] + (B[s] - B[s - 1]) * a / (a - b)
                break
        out.append(float(x))
    return out


def c1():
    lat = synth.sc_periodic(64)
    lat.k = np.full(lat.n, 0.1)
    T = synth.replica_temperatures(64, 0.1, 3.0)
    jobs = [dict(lat=lat, T=[T[r]], B=[0.0], mcs_per_step=C1_MCS, seed=1, replica=1000 + r,
                 init="cold") for r in C1_REPS]
    res, used = oracle.run_replicas(jobs)
    stats = {k: {"mean": [], "se": []} for k in OBSERVABLES}
    for r, x in zip(C1_REPS, res):
        st = chain_stats(x["history"][0], lat.n, T[r])
        for k in OBSERVABLES:
            stats[k]["mean"].append(st[k][0])
            stats[k]["se"].append(st[k][1])
    return dict(replicas=C1_REPS, T=[float(T[r]) for r in C1_REPS], mcs=C1_MCS, seed=1,
                oracle_replica_ids=[1000 + r for r in C1_REPS], stats=stats, threads=used)


def c2():
    lat = synth.core_shell_ball()
    B = synth.hysteresis_fields(401)
    M = 200
    jobs = [dict(lat=lat, T=np.full(B.size, 0.1), B=B, mcs_per_step=M, seed=2, replica=rid,
                 init="cold") for rid in C2_SEEDS]
    res, used = oracle.run_replicas(jobs)
    m0 = M // 5
    mz = np.array([x["history"][:, m0:, 3].mean(axis=1) / lat.n for x in res])   # [seed][step]
    hc = np.array([coercive(B, row) for row in mz])
    R = len(C2_SEEDS)
    return dict(seed=2, oracle_replica_ids=C2_SEEDS, T=0.1, mcs_per_step=M, burn_per_step=m0,
                mz_mean=mz.mean(axis=0).tolist(), mz_se=(mz.std(axis=0, ddof=1) / np.sqrt(R)).tolist(),
                coercive_mean=hc.mean(axis=0).tolist(),
                coercive_se=(hc.std(axis=0, ddof=1) / np.sqrt(R)).tolist(), threads=used)


def c3():
    """The small films are thin, with an easy axis: below their ordering
    temperature a film's magnetisation can reverse on time scales longer than
    the run, so one chain's block errors do not measure the spread.  Each
    film therefore gets C3_CHAINS independent chains, and the statistics are
    the mean and spread over chains of each chain's averages (after 20%
    burn-in) and of its fluctuations (chi, C_v)."""
    films, Ts = synth.film_batch()
    order = np.argsort([f.n for f in films], kind="stable")[:C3_FILMS]
    jobs = []
    for f in order:
        for k in range(C3_CHAINS):
            jobs.append(dict(lat=films[f], T=[Ts[f]], B=[0.0], mcs_per_step=1000, seed=3,
                             replica=C3_ORACLE_ID0 + int(f) * 64 + k, init="cold"))
    res, used = oracle.run_replicas(jobs)
    stats = {k: {"mean": [], "se": []} for k in OBSERVABLES}
    for a, f in enumerate(order):
        per = chain_means([x["history"][0] for x in res[a * C3_CHAINS:(a + 1) * C3_CHAINS]],
                          films[f].n, Ts[f])
        for k in OBSERVABLES:
            stats[k]["mean"].append(float(per[k].mean()))
            stats[k]["se"].append(float(per[k].std(ddof=1) / np.sqrt(C3_CHAINS)))
    return dict(films=[int(f) for f in order], T=[float(Ts[f]) for f in order], mcs=1000, seed=3,
                chains=C3_CHAINS, gpu_replica_ids="64 f + k", oracle_replica_ids=f"{C3_ORACLE_ID0} + 64 f + k",
                stats=stats, threads=used)


def main():
    only = sys.argv[1:]            # e.g. "c3": regenerate those parts only
    out = {"about": __doc__.split("\n\n")[0], "command": "python tests/golden/make_fp32_stats.py"}
    if only and os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f)
    for name, fn in (("c3", c3), ("c1", c1), ("c2", c2)):
        if only and name not in only:
            continue
        t0 = time.perf_counter()
        out[name] = fn()
        out[name]["seconds"] = time.perf_counter() - t0
        print(name, f"{out[name]['seconds']:.1f} s", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
