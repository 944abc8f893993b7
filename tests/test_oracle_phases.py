"""Pins of the oracle's per-phase magnetisation (the statistics of each
magnetic phase, i.e. site type) and per-step final states (section "VEGAS
software package" feature list): per-type Langevin laws of isolated spins of
two lengths, the exact two-state values of flip-only sites, the per-type sums
adding up to the total, and snapshots equal to the spins of runs stopped at
each step."""
import numpy as np

import oracle
import synth
from _stats import block_mean_se, langevin, after_burn_in


def test_per_type_langevin_of_two_spin_lengths():
    """Isolated spins, type 0 of length 1 and type 1 of length 2, field B
    along z at T = 1: <M_z> per type is N_t mu_t L(B mu_t)."""
    N, M, B = 4096, 240, 0.8
    lat = synth.isolated(N)
    types = (np.arange(N) % 2).astype(np.int32)
    lat.norm = np.where(types == 1, 2.0, 1.0)
    r = oracle.run(lat, [1.0], [B], M, seed=41, init="random", type_mag=True,
                   policies=[(oracle.POLICY_RANDOM, 0.0)] * 2, site_type=types)
    tm = after_burn_in(r["type_mag"][0], 1 / 4)
    for t, mu in ((0, 1.0), (1, 2.0)):
        m, se = block_mean_se(tm[:, t, 2] / (N / 2))
        assert abs(m - mu * float(langevin(B * mu))) <= 4 * se + 1e-12


def test_flip_type_is_exact_and_types_add_up():
    """A lattice with a flip-move type: that type's M stays on the z axis
    with an integer z component; the types' sums equal the total M."""
    lat = synth.sc_periodic(6)
    types = (np.arange(lat.n) % 3 == 0).astype(np.int32)
    r = oracle.run(lat, [2.0, 1.0], [0.1, 0.0], 7, seed=4, init="cold", type_mag=True,
                   policies=[(oracle.POLICY_RANDOM, 0.0), (oracle.POLICY_FLIP, 0.0)], site_type=types)
    tm = r["type_mag"]
    assert np.all(tm[..., 1, 0] == 0.0) and np.all(tm[..., 1, 1] == 0.0)
    assert np.all(tm[..., 1, 2] == np.round(tm[..., 1, 2]))
    assert np.allclose(tm.sum(axis=2), r["history"][..., 1:4], rtol=0, atol=1e-12 * lat.n)
    # without types: one type, the total
    r1 = oracle.run(lat, [2.0], [0.1], 4, seed=4, init="cold", type_mag=True)
    assert np.allclose(r1["type_mag"][..., 0, :], r1["history"][..., 1:4], rtol=0, atol=1e-12 * lat.n)


def test_snapshots_are_the_spins_at_each_step_end():
    lat = synth.sc_periodic(5)
    T = [2.0, 1.0, 0.5]
    r = oracle.run(lat, T, [0.0] * 3, 4, seed=9, init="random", snapshots=True)
    assert np.array_equal(r["snapshots"][-1], r["spins"])
    for s in range(2):
        part = oracle.run(lat, T[: s + 1], [0.0] * (s + 1), 4, seed=9, init="random")
        assert np.array_equal(r["snapshots"][s], part["spins"])
