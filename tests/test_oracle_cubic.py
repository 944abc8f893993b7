"""Pins of the oracle's cubic anisotropy (paper, Eq. 3) and per-site spin
norms (the spin norm of the material file, section "Material building"):
isolated spins against sphere quadratures and the scaled Langevin law, the
zero-temperature energy of a cold start, the incremental energy against the
full recompute, gradients against central differences, and neutrality of
the default values."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from _stats import block_mean_se, langevin, after_burn_in

EXACT, F32MAP = oracle.PROPOSAL_EXACT, oracle.PROPOSAL_F32MAP


def _cubic(x, y, z):
    return x * x * y * y + y * y * z * z + x * x * z * z


def _sphere_avg(fn, weight):
    """<fn> over the unit sphere with Boltzmann weight exp(weight(s))."""
    def integrand(th, ph, g):
        s = (math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th))
        return g(*s) * math.exp(weight(*s)) * math.sin(th)
    Z = integrate.dblquad(lambda th, ph: integrand(th, ph, lambda *a: 1.0), 0, 2 * math.pi, 0, math.pi)[0]
    N = integrate.dblquad(lambda th, ph: integrand(th, ph, fn), 0, 2 * math.pi, 0, math.pi)[0]
    return N / Z


@pytest.mark.parametrize("proposal", [EXACT, F32MAP])
@pytest.mark.parametrize("kc", [2.0, -3.0])
def test_isolated_cubic_spins(kc, proposal):
    """Isolated spins with cubic constant kc at T = 1: <E>/N = -kc <f> and
    <S_z^4>, both against quadratures of exp(kc f) on the sphere."""
    N, M = 4096, 240
    lat = synth.isolated(N)
    lat.kc = np.full(N, kc)
    r = oracle.run(lat, [1.0], [0.0], M, seed=31, init="random", proposal=proposal)
    h = after_burn_in(r["history"][0], 1 / 4)
    e, se = block_mean_se(h[:, 0] / N)
    f_avg = _sphere_avg(_cubic, lambda x, y, z: kc * _cubic(x, y, z))
    assert abs(e + kc * f_avg) <= 4 * se + 1e-12
    z4 = np.mean(r["spins"][:, 2] ** 4)
    z4_ref = _sphere_avg(lambda x, y, z: z ** 4, lambda x, y, z: kc * _cubic(x, y, z))
    sd = np.std(r["spins"][:, 2] ** 4) / math.sqrt(N)
    assert abs(z4 - z4_ref) <= 4 * sd


@pytest.mark.parametrize("proposal", [EXACT, F32MAP])
@pytest.mark.parametrize("mu,x", [(0.5, 1.0), (2.0, 0.5), (1.5, 3.0)])
def test_isolated_spins_with_norm(mu, x, proposal):
    """Spins of length mu in a field B along z at T = 1: S_z/mu follows the
    Langevin law of x = beta B mu, and every spin keeps its length."""
    N, M = 4096, 240
    lat = synth.isolated(N)
    lat.norm = np.full(N, mu)
    B = x / mu
    r = oracle.run(lat, [1.0], [B], M, seed=32, init="random", proposal=proposal)
    assert np.allclose(np.linalg.norm(r["spins"], axis=1), mu, rtol=1e-12)
    h = after_burn_in(r["history"][0], 1 / 4)
    m, se = block_mean_se(h[:, 3] / N)
    assert abs(m - mu * float(langevin(x))) <= 4 * se + 1e-12
    e, se_e = block_mean_se(h[:, 0] / N)
    assert abs(e + B * mu * float(langevin(x))) <= 4 * se_e + 1e-12


def test_policies_keep_the_norm():
    """Every policy moves the direction only: after a run each spin has its
    own length (two lengths mixed)."""
    lat = synth.sc_periodic(6)
    lat.norm = np.where(np.arange(lat.n) % 2 == 0, 0.5, 2.0)
    for pol in ([(oracle.POLICY_SMALL_STEP, 0.5)], [(oracle.POLICY_GAUSSIAN, 0.4)],
                [(oracle.POLICY_HN, 0.3)], [(oracle.POLICY_ADAPTIVE, 1.0)], [(oracle.POLICY_FLIP, 0.0)]):
        for proposal in (EXACT, F32MAP):
            r = oracle.run(lat, [1.5], [0.2], 10, seed=5, init="random", proposal=proposal, policies=pol)
            assert np.allclose(np.linalg.norm(r["spins"], axis=1), lat.norm, rtol=1e-12)


def test_zero_temperature_cold_start_with_norm_and_cubic():
    """SC 6^3, norms mu, J = 1, k = 0.3 along z, kc = -0.5 (z is a minimum of
    the cubic term when kc < 0), B = 0.2 along z, T = 0, cold start: nothing
    is accepted and E = -N (3 J mu^2 + B mu + k mu^2)."""
    lat = synth.sc_periodic(6)
    mu = 1.7
    lat.norm = np.full(lat.n, mu)
    lat.k = np.full(lat.n, 0.3)
    lat.kc = np.full(lat.n, -0.5)
    r = oracle.run(lat, [0.0], [0.2], 5, seed=1, init="cold")
    assert np.all(r["history"][0, :, 4] == 0)
    E = -lat.n * (3 * mu * mu + 0.2 * mu + 0.3 * mu * mu)
    assert abs(r["history"][0, -1, 0] - E) <= 1e-12 * abs(E)


def test_incremental_energy_with_cubic_and_norms():
    """Every accepted move's energy change equals the difference of full
    energies, and the carried energy equals the full sum after every MCS."""
    lat = synth.diluted_film(9, 3, seed=4)
    lat.kc = 0.8 * synth.uniform01(7, lat.n, tag=1) - 0.4
    lat.norm = 0.5 + synth.uniform01(7, lat.n, tag=2)
    lat.k = 0.2 * synth.uniform01(7, lat.n, tag=3)
    lat.axis = synth.unit_vectors(7, lat.n, tag=4)
    r = oracle.run(lat, [0.8, 2.0], [0.3, -0.2], 6, seed=2, full_energy=True,
                   check_every_update=True)
    assert r["max_update_err"] <= 1e-13
    assert r["max_incr_err"] <= 1e-12


def test_gradient_with_cubic_and_norms():
    """dE/dS with the cubic term against central differences of the energy
    (quartic in S: the difference is accurate to O(h^2))."""
    lat = synth.sc_periodic(4)
    lat.kc = 1.3 * synth.uniform01(9, lat.n, tag=1) - 0.6
    lat.k = 0.2 * synth.uniform01(9, lat.n, tag=2)
    lat.axis = synth.unit_vectors(9, lat.n, tag=3)
    rng = np.random.default_rng(3)
    S = rng.normal(size=(lat.n, 3)) * 1.3
    gS, _, _, _ = oracle.energy_grad(lat, 0.4, S)
    h = 1e-5
    for idx in rng.choice(3 * lat.n, 40, replace=False):
        i, c = divmod(int(idx), 3)
        Sp, Sm = S.copy(), S.copy()
        Sp[i, c] += h
        Sm[i, c] -= h
        fd = (oracle.energy(lat, 0.4, Sp)["E"] - oracle.energy(lat, 0.4, Sm)["E"]) / (2 * h)
        assert abs(gS[i, c] - fd) <= 1e-7 * max(1.0, abs(fd))


def test_default_values_are_neutral():
    """Explicit unit norms and zero cubic constants give the trajectory of
    the plain model bit for bit."""
    lat = synth.sc_periodic(6)
    r0 = oracle.run(lat, [1.2], [0.1], 6, seed=3, init="random")
    lat.norm = np.ones(lat.n)
    lat.kc = np.zeros(lat.n)
    r1 = oracle.run(lat, [1.2], [0.1], 6, seed=3, init="random")
    assert np.array_equal(r0["spins"], r1["spins"])
    assert np.array_equal(r0["history"], r1["history"])


def test_validation_of_new_terms():
    lat = synth.sc_periodic(4)
    lat.norm = np.zeros(lat.n)
    assert oracle.validate(lat) == -3
    lat.norm = None
    lat.kc = np.full(lat.n, np.nan)
    assert oracle.validate(lat) == -3
