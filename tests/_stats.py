"""Estimators used by the tests: block means (Flyvbjerg and Petersen 1989)
and closed forms of isolated classical spins."""
import numpy as np


def block_mean_se(x, n_blocks=20):
    """Mean and standard error from n_blocks consecutive block means."""
    x = np.asarray(x, dtype=np.float64)
    L = x.size // n_blocks
    xb = x[: n_blocks * L].reshape(n_blocks, L).mean(axis=1)
    return xb.mean(), xb.std(ddof=1) / np.sqrt(n_blocks)


def langevin(x):
    """L(x) = coth x - 1/x, series near 0."""
    x = np.asarray(x, dtype=np.float64)
    small = np.abs(x) < 1e-3
    xs = np.where(small, 1.0, x)
    return np.where(small, x / 3.0 - x ** 3 / 45.0, 1.0 / np.tanh(xs) - 1.0 / xs)


def langevin_var(x):
    """Var(S_z) of an isolated unit spin in a field, x = beta B: 1/x^2 - 1/sinh^2 x."""
    x = np.asarray(x, dtype=np.float64)
    return 1.0 / x ** 2 - 1.0 / np.sinh(x) ** 2


def within(a, b, se, n_se=4.0, abs_floor=0.0):
    return abs(a - b) <= n_se * se + abs_floor


def after_burn_in(h, frac=0.2):
    """Drop the first frac of the MCS axis of a history (S, M, 5) or (M, 5)."""
    M = h.shape[-2]
    return h[..., int(frac * M):, :]
