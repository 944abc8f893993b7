"""Pins of the oracle's update policies (random, spin-flip, small step,
Gaussian, Hinzke-Nowak combination, adaptive; named in the paper's
"Monte Carlo Metropolis algorithm" section and feature list, the moves as
defined by Hinzke and Nowak 1999).

Every check is against something other than the oracle itself: the library
logarithm, geometric facts of the moves, an independent numpy sampler of the
Gaussian move, closed forms of isolated spins (the stationary distribution of
every symmetric proposal is the Boltzmann one), the two-state closed form of a
spin that can only flip, and the fixed point of the adaptive width.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from _stats import block_mean_se, langevin, after_burn_in

EXACT, F32MAP = oracle.PROPOSAL_EXACT, oracle.PROPOSAL_F32MAP
P = oracle


def test_own_log_matches_library_log():
    """or_log (exponent split + atanh series) is within 2 ulp of libm's log,
    over 600 decades and on (0, 1) where the Gaussian move uses it."""
    rng = np.random.default_rng(5)
    xs = np.concatenate([np.logspace(-300, 300, 1501), rng.uniform(0, 1, 2000),
                         [np.nextafter(1.0, 0.0), 1.0, np.nextafter(1.0, 2.0), 2.0 ** -1074 * 3,
                          0.5, 2.0, math.sqrt(0.5), math.sqrt(2.0)]])
    for x in xs:
        ref = math.log(x)
        got = oracle.log(x)
        assert abs(got - ref) <= 2 * math.ulp(ref) + 1e-300, x


def _rand_unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]


def _trials(proposal, policy, param, n=4000, seed=11):
    rng = np.random.default_rng(seed)
    S = _rand_unit(rng, n)
    out = np.empty((n, 3))
    u = np.empty(n)
    for t in range(n):
        out[t], u[t] = oracle.trial(proposal, policy, 77, t, 3, 1, S[t], param)
    return S, out, u


@pytest.mark.parametrize("proposal", [EXACT, F32MAP])
def test_flip_is_exact_negation(proposal):
    S, out, u = _trials(proposal, P.POLICY_FLIP, 0.0, n=200)
    assert np.array_equal(out, -S)
    assert np.all((u > 0) & (u < 1))


@pytest.mark.parametrize("proposal", [EXACT, F32MAP])
@pytest.mark.parametrize("theta", [0.2, 0.6, 1.5, math.pi])
def test_small_step_uniform_in_cap(proposal, theta):
    """Trials are unit vectors inside the cap of half-angle theta around S;
    the cosine of the angle to S is uniform on [cos theta, 1] and the azimuth
    around S (measured in an independent frame) is uniform."""
    S, out, _ = _trials(proposal, P.POLICY_SMALL_STEP, theta)
    assert np.allclose(np.linalg.norm(out, axis=1), 1.0, atol=1e-12)
    c = np.sum(S * out, axis=1)
    ct = math.cos(theta)
    assert np.all(c >= ct - 1e-12)
    assert stats.kstest((c - ct) / (1 - ct), "uniform").pvalue > 1e-3
    # azimuth in a frame built from a fixed reference vector
    ref = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    e1 = ref - np.sum(S * ref, axis=1)[:, None] * S
    e1 /= np.linalg.norm(e1, axis=1)[:, None]
    e2 = np.cross(S, e1)
    perp = out - c[:, None] * S
    phi = np.arctan2(np.sum(perp * e2, axis=1), np.sum(perp * e1, axis=1))
    assert stats.kstest((phi + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3


@pytest.mark.parametrize("proposal", [EXACT, F32MAP])
@pytest.mark.parametrize("sigma", [0.1, 0.5, 2.0])
def test_gaussian_move_matches_independent_sampler(proposal, sigma):
    """The angle between S and the Gaussian trial has the distribution of
    normalise(S + sigma g) drawn with numpy's own normal generator."""
    S, out, _ = _trials(proposal, P.POLICY_GAUSSIAN, sigma)
    assert np.allclose(np.linalg.norm(out, axis=1), 1.0, atol=1e-12)
    c = np.sum(S * out, axis=1)
    rng = np.random.default_rng(99)
    ref = S + sigma * rng.normal(size=S.shape)
    ref /= np.linalg.norm(ref, axis=1)[:, None]
    cr = np.sum(S * ref, axis=1)
    assert stats.ks_2samp(c, cr).pvalue > 1e-3


@pytest.mark.parametrize("proposal", [EXACT, F32MAP])
def test_hinzke_nowak_mixes_three_moves(proposal):
    """Each trial is a flip, a small step (inside the cap) or a random point,
    about one third each, in the proportions of the fourth random word."""
    theta = 0.3
    S, out, _ = _trials(proposal, P.POLICY_HN, theta, n=3000)
    flip = np.all(out == -S, axis=1)
    c = np.sum(S * out, axis=1)
    small = ~flip & (c >= math.cos(theta) - 1e-12)
    rest = ~flip & ~small
    n = len(S)
    # a uniform point falls in the cap with probability (1 - cos theta)/2
    p_cap = (1 - math.cos(theta)) / 2
    for frac, p in ((flip.mean(), 1 / 3), (small.mean(), 1 / 3 + p_cap / 3),
                    (rest.mean(), (1 - p_cap) / 3)):
        assert abs(frac - p) <= 4 * math.sqrt(p * (1 - p) / n)


def _isolated_sz(policy, param, x, proposal, N=4096, M=240, init="random"):
    lat = synth.isolated(N)
    r = oracle.run(lat, [1.0], [x], M, seed=202, init=init, proposal=proposal,
                   policies=[(policy, param)])
    h = after_burn_in(r["history"][0], 1 / 4)
    return block_mean_se(h[:, 3] / N)


@pytest.mark.parametrize("proposal", [EXACT, F32MAP])
@pytest.mark.parametrize("policy,param", [(P.POLICY_SMALL_STEP, 0.5), (P.POLICY_SMALL_STEP, math.pi),
                                          (P.POLICY_GAUSSIAN, 0.4), (P.POLICY_HN, 0.3),
                                          (P.POLICY_ADAPTIVE, 1.0)])
@pytest.mark.parametrize("x", [0.5, 2.0])
def test_symmetric_moves_sample_langevin(policy, param, x, proposal):
    """Every symmetric proposal leaves the Boltzmann distribution invariant:
    isolated spins in a field reach <S_z> = L(beta B)."""
    m, se = _isolated_sz(policy, param, x, proposal)
    assert abs(m - langevin(x)) <= 4 * se + 1e-12


@pytest.mark.parametrize("proposal", [EXACT, F32MAP])
@pytest.mark.parametrize("x", [0.3, 1.0])
def test_flip_only_spins_are_two_state(x, proposal):
    """A spin that can only flip, started along +z in a field along z, is a
    two-state chain: it stays exactly at +-z and <S_z> = tanh(beta B)."""
    N, M = 4096, 300
    lat = synth.isolated(N)
    r = oracle.run(lat, [1.0], [x], M, seed=9, init="cold", proposal=proposal,
                   policies=[(P.POLICY_FLIP, 0.0)])
    assert set(np.unique(r["spins"][:, 2])) <= {-1.0, 1.0}
    assert np.all(r["spins"][:, :2] == 0.0)
    h = after_burn_in(r["history"][0], 1 / 5)
    m, se = block_mean_se(h[:, 3] / N)
    assert abs(m - math.tanh(x)) <= 4 * se + 1e-12


def test_policy_per_site_type():
    """Two site types with different moves in one lattice (exact mode): the
    flip-type sites of a cold start stay exactly at +-z while the random-type
    sites leave the axis; every decision is counted in the history."""
    lat = synth.sc_periodic(8)
    types = (np.arange(lat.n) % 3 == 0).astype(np.int32)       # type 1: flip
    r = oracle.run(lat, [2.0], [0.0], 20, seed=4, init="cold",
                   policies=[(P.POLICY_RANDOM, 0.0), (P.POLICY_FLIP, 0.0)], site_type=types)
    s = r["spins"]
    assert np.all(np.abs(s[types == 1, 2]) == 1.0)
    assert np.all(s[types == 1, :2] == 0.0)
    assert np.mean(np.abs(s[types == 0, 2]) < 1.0) > 0.99
    # with all types random the run is the plain random-move run
    r0 = oracle.run(lat, [2.0], [0.0], 5, seed=4, init="cold")
    r1 = oracle.run(lat, [2.0], [0.0], 5, seed=4, init="cold",
                    policies=[(P.POLICY_RANDOM, 0.0), (P.POLICY_RANDOM, 0.0)], site_type=types)
    assert np.array_equal(r0["spins"], r1["spins"])
    assert np.array_equal(r0["history"], r1["history"])


@pytest.mark.parametrize("proposal", [EXACT, F32MAP])
@pytest.mark.parametrize("T,sigma0", [(0.5, 5.0), (1.0, 0.01), (1.4, 1.0), (2.0, 1.0)])
def test_adaptive_width_settles_at_half_acceptance(T, sigma0, proposal):
    """The adaptive move drives the acceptance of a ferromagnet toward 50%
    from widths far too large or too small.  Where even the random move
    (the limit of an infinite width) accepts more than half the trials (here
    above T ~ 1.6), the width runs to its upper bound and the acceptance is
    the random move's."""
    lat = synth.sc_periodic(10)
    M = 120
    r = oracle.run(lat, [T], [0.0], M, seed=8, init="cold", proposal=proposal,
                   policies=[(P.POLICY_ADAPTIVE, sigma0)], trace_sigma=True)
    acc = r["history"][0, M // 2:, 4] / lat.n
    tr = r["sigma_trace"]
    assert tr[0] == sigma0
    assert np.all((tr >= P.SIGMA_MIN) & (tr <= P.SIGMA_MAX))
    rnd = oracle.run(lat, [T], [0.0], M, seed=8, init="cold", proposal=proposal)
    acc_rnd = rnd["history"][0, M // 2:, 4].mean() / lat.n
    if acc_rnd < 0.45:
        assert abs(acc.mean() - 0.5) < 0.03
        assert r["sigma"] < P.SIGMA_MAX
    else:
        assert r["sigma"] == P.SIGMA_MAX
        assert abs(acc.mean() - acc_rnd) < 0.03


def test_policy_validation():
    lat = synth.sc_periodic(4)
    with pytest.raises(ValueError):
        oracle.run(lat, [1.0], [0.0], 1, seed=0, policies=[(P.POLICY_SMALL_STEP, 0.0)])
    with pytest.raises(ValueError):
        oracle.run(lat, [1.0], [0.0], 1, seed=0, policies=[(P.POLICY_GAUSSIAN, -1.0)])
    with pytest.raises(ValueError):
        oracle.run(lat, [1.0], [0.0], 1, seed=0, policies=[(9, 1.0)])
    with pytest.raises(ValueError):
        oracle.run(lat, [1.0], [0.0], 1, seed=0, policies=[(P.POLICY_RANDOM, 0.0)],
                   site_type=np.ones(lat.n, dtype=np.int32))
