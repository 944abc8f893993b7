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


def _jackknife(blocks, fn):
    """Jackknife mean and standard error of fn over leave-one-block-out
    samples (blocks: list of arrays)."""
    nb = len(blocks)
    full = fn(np.concatenate(blocks))
    loo = np.array([fn(np.concatenate(blocks[:k] + blocks[k + 1:])) for k in range(nb)])
    se = np.sqrt((nb - 1) / nb * np.sum((loo - loo.mean()) ** 2))
    return float(full), float(se)


OBSERVABLES = ("e", "m_abs", "mz", "chi", "cv", "acc")


def chain_stats(h, n_sites, T, n_blocks=20, burn=0.2):
    """Per-site thermal averages of one chain's history h (M, 5) at
    temperature T after dropping the first `burn` of its MCS, each with a
    standard error from n_blocks consecutive blocks (Flyvbjerg and Petersen
    1989; jackknife over blocks for the fluctuations): <E>/N, <|M|>/N,
    <M_z>/N, chi = beta (<|M|^2> - <|M|>^2)/N, C_v = beta^2 Var(E)/N and the
    acceptance <n_acc>/N."""
    h = np.asarray(h, dtype=np.float64)[int(burn * h.shape[0]):]
    L = h.shape[0] // n_blocks
    h = h[: n_blocks * L]
    N = float(n_sites)
    beta = 1.0 / T
    E = h[:, 0]
    Mabs = np.sqrt((h[:, 1:4] ** 2).sum(axis=1))
    out = {}
    for name, x in (("e", E / N), ("m_abs", Mabs / N), ("mz", h[:, 3] / N), ("acc", h[:, 4] / N)):
        out[name] = block_mean_se(x, n_blocks)
    bM = [Mabs[k * L:(k + 1) * L] for k in range(n_blocks)]
    bE = [E[k * L:(k + 1) * L] for k in range(n_blocks)]
    out["chi"] = _jackknife(bM, lambda m: beta * np.var(m) / N)
    out["cv"] = _jackknife(bE, lambda e: beta ** 2 * np.var(e) / N)
    return {k: (float(v[0]), float(v[1])) for k, v in out.items()}


def grade(pairs, n_se=3.0, hard=5.0, p=0.0027):
    """pairs: list of (mean_a, se_a, mean_b, se_b).  Returns the deviations in
    combined SE, the number above n_se and the 99% binomial bound on that
    number for a two-sided normal tail p; a set passes when the count is
    within the bound and no deviation exceeds `hard`."""
    from scipy import stats
    z = np.array([abs(a - b) / np.hypot(sa, sb) if np.hypot(sa, sb) > 0 else
                  (0.0 if a == b else np.inf) for a, sa, b, sb in pairs])
    bound = int(stats.binom.ppf(0.99, len(z), p))
    return z, int((z > n_se).sum()), bound


def chain_means(hists, n_sites, T, burn=0.2):
    """Per-chain averages of independent chains (histories (M, 5)) after
    dropping the first `burn` of their MCS: arrays over chains of <E>/N,
    <|M|>/N, <M_z>/N, chi, C_v and the acceptance (the chain's own
    fluctuations for chi and C_v)."""
    out = {k: [] for k in OBSERVABLES}
    beta, N = 1.0 / T, float(n_sites)
    for h in hists:
        h = np.asarray(h, dtype=np.float64)[int(burn * len(h)):]
        Mabs = np.sqrt((h[:, 1:4] ** 2).sum(axis=1))
        out["e"].append(h[:, 0].mean() / N)
        out["m_abs"].append(Mabs.mean() / N)
        out["mz"].append(h[:, 3].mean() / N)
        out["chi"].append(beta * Mabs.var() / N)
        out["cv"].append(beta ** 2 * h[:, 0].var() / N)
        out["acc"].append(h[:, 4].mean() / N)
    return {k: np.array(v) for k, v in out.items()}
