"""Pins of the oracle's history analysis (oracle/analysis.py) against closed
forms: isolated spins in a field sampled exactly from the Boltzmann
distribution (Langevin moments, specific heat 1 - x^2/sinh^2 x, the
cumulants d ln<|M|^j>/d beta), the Binder cumulant of a paramagnet (sum of
independent unit vectors) and of a rigid moment, the integrated
autocorrelation time of an AR(1) series, and reweighting and multiple
histograms of isolated spins, whose partition function is known."""
import math

import numpy as np
import pytest

from oracle import analysis as A
from _stats import langevin, langevin_var


def exact_isolated(rng, n_samples, N, x):
    """n_samples configurations of N independent unit spins in a field along z
    at x = beta B, drawn exactly (cos theta by inverting its distribution
    exp(x c) on [-1, 1]).  Returns the summed magnetisation (n, 3)."""
    u = rng.uniform(size=(n_samples, N))
    if x == 0.0:
        c = 2 * u - 1
    else:
        c = np.log(np.exp(-x) + u * (np.exp(x) - np.exp(-x))) / x
    phi = rng.uniform(0, 2 * np.pi, size=(n_samples, N))
    s = np.sqrt(np.clip(1 - c * c, 0, None))
    return np.stack([(s * np.cos(phi)).sum(1), (s * np.sin(phi)).sum(1), c.sum(1)], axis=1)


@pytest.mark.parametrize("x", [0.7, 2.0, 5.0])
def test_thermal_of_isolated_spins(x):
    """N = 256 spins, B = 1, beta = x: e = -L(x), cv = 1 - x^2/sinh^2 x;
    <|M|^2> = N + N(N-1) L^2 exactly (independent spins), so
    v2 = d ln<|M|^2>/d beta = 2 B (N-1) L L' / (1 + (N-1) L^2) with
    L' = Var(S_z); chi -> beta Var(S_z) and v1 -> B Var(S_z)/<S_z>
    (|M| ~ M_z up to O(1/N))."""
    rng = np.random.default_rng(1)
    N, n, B = 256, 20000, 1.0
    beta = x / B
    M = exact_isolated(rng, n, N, x)
    E = -B * M[:, 2]
    t = A.thermal(E, M, N, beta)
    L, V = float(langevin(x)), float(langevin_var(x))
    assert abs(t["e"] + B * L) < 4 * math.sqrt(V / N / n)
    assert abs(t["cv"] - (1 - x * x / math.sinh(x) ** 2)) < 0.05 * t["cv"]
    assert abs(t["chi"] - beta * V) < 0.06 * beta * V
    assert abs(t["v1"] - B * V / L) < 0.06 * B * V / L
    v2 = 2 * B * (N - 1) * L * V / (1 + (N - 1) * L * L)
    assert abs(t["v2"] - v2) < 0.04 * v2
    assert abs(t["m2"] * N * N - (N + N * (N - 1) * L * L)) < 0.01 * N * N * t["m2"]
    assert abs(t["m_abs"] - L) < 0.01


def test_binder_cumulant_limits():
    """A sum of N independent uniform unit vectors: <|M|^2> = N,
    <|M|^4> = N^2 + 2N(N-1)/3, so u4 = 2/3 - 2(N-1)/(9N) (4/9 for large N);
    a rigid moment of fixed length: u4 = 2/3."""
    rng = np.random.default_rng(2)
    N, n = 32, 40000
    M = exact_isolated(rng, n, N, 0.0)
    t = A.thermal(np.zeros(n), M, N, 1.0)
    assert abs(t["m2"] * N - 1.0) < 0.02
    assert abs(t["u4"] - (2 / 3 - 2 * (N - 1) / (9 * N))) < 0.01
    v = rng.normal(size=(1000, 3))
    v *= 7.0 / np.linalg.norm(v, axis=1)[:, None]
    assert abs(A.thermal(np.zeros(1000), v, 7, 1.0)["u4"] - 2 / 3) < 1e-12


@pytest.mark.parametrize("phi", [0.5, 0.9])
def test_tau_of_ar1_series(phi):
    """x_m = phi x_{m-1} + noise has rho(t) = phi^t, so
    tau = 1/2 + phi/(1 - phi) = (1 + phi) / (2 (1 - phi))."""
    rng = np.random.default_rng(3)
    n = 200000
    e = rng.normal(size=n)
    x = np.empty(n)
    x[0] = e[0]
    for m in range(1, n):
        x[m] = phi * x[m - 1] + e[m]
    tau, W = A.tau_int(x)
    exact = (1 + phi) / (2 * (1 - phi))
    assert abs(tau - exact) < 0.05 * exact
    assert W >= 6 * tau - 1


def test_tau_of_independent_samples_and_constant():
    rng = np.random.default_rng(4)
    tau, _ = A.tau_int(rng.normal(size=50000))
    assert abs(tau - 0.5) < 0.05
    assert A.tau_int(np.ones(100))[0] == 0.5


def test_reweighting():
    """Reweighting to the sampling beta is the plain average; samples of
    N = 4 isolated spins at beta0 = 1 (B = 1) reweighted to beta = 0.7 and
    1.4 give <S_z> = L(beta B) and the specific heat 1 - x^2/sinh^2 x."""
    rng = np.random.default_rng(5)
    N, n, B, b0 = 4, 400000, 1.0, 1.0
    M = exact_isolated(rng, n, N, b0 * B)
    E = -B * M[:, 2]
    same = A.reweight(E, M, N, b0, b0)
    plain = A.thermal(E, M, N, b0)
    for k in A.THERMAL_FIELDS:
        assert abs(same[k] - plain[k]) <= 1e-12 * max(1.0, abs(plain[k]))
    for b in (0.7, 1.4):
        t = A.reweight(E, M, N, b0, b)
        x = b * B
        assert abs(-t["e"] / B - float(langevin(x))) < 0.01
        assert abs(t["cv"] - (1 - x * x / math.sinh(x) ** 2)) < 0.03


def test_multiple_histograms():
    """Four sample sets of N = 8 isolated spins at beta = 0.6 .. 1.5 (B = 1):
    the free energies equal -ln Z(beta_k) + ln Z(beta_0) with
    Z = (4 pi sinh(beta B)/(beta B))^N, and the interpolated energy at
    beta = 1.05 is -N B L(beta B)."""
    rng = np.random.default_rng(6)
    N, n, B = 8, 40000, 1.0
    betas = np.array([0.6, 0.9, 1.2, 1.5])
    Ms = [exact_isolated(rng, n, N, b * B) for b in betas]
    Es = [-B * m[:, 2] for m in Ms]
    f, logD, it = A.multihist(Es, betas)
    lnZ = N * np.log(np.sinh(betas * B) / (betas * B))
    exact = -(lnZ - lnZ[0])
    assert np.max(np.abs(f - exact)) < 0.02
    assert it < 5000
    t = A.multihist_thermal(Es, Ms, betas, f, logD, N, 1.05)
    assert abs(-t["e"] / B - float(langevin(1.05 * B))) < 0.005
