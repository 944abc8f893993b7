"""Analysis of the per-MCS history, written out from the definitions (numpy,
double precision).

TEST INFRASTRUCTURE ONLY (see the package docstring): the tests use it to
check the library's analysis kernels.

Paper: thermal averages of M, chi and the specific heat ("Thermal
averages"); cumulants of the magnetisation for finite-size scaling ("Critical
exponents"); equilibrium correlation times ("Dynamic behavior"); single and
multiple histogram reweighting ("Histogram and multiple histogram methods").
A series is the history of one replica at one temperature/field step:
E_m (total energy), M_m (magnetisation vector) for MCS m = m0 .. M-1.
"""
import numpy as np

# fields of a thermal summary
THERMAL_FIELDS = ("e", "m_abs", "m2", "m4", "cv", "chi", "u4", "v1", "v2")


def thermal(E, Mvec, n_sites, beta, logw=None):
    """Thermal averages of samples (E_m, M_m) with weights w_m = exp(logw_m)
    (None: equal weights), per site, k_B = 1.  With <.> the weighted mean
    and |M| the length of the magnetisation vector:
      e = <E>/N, m_abs = <|M|>/N, m2 = <|M|^2>/N^2, m4 = <|M|^4>/N^4,
      cv  = beta^2 <(E - <E>)^2> / N,
      chi = beta <(|M| - <|M|>)^2> / N,
      u4  = 1 - m4 / (3 m2^2)                                (Binder cumulant),
      v_j = -<(|M|^j - <|M|^j>)(E - <E>)> / <|M|^j>, j = 1, 2
            (= d ln<|M|^j> / d beta, the cumulants of finite-size scaling).
    Means are taken first and the central moments in a second pass; the
    weights are shifted by their largest exponent."""
    E = np.asarray(E, dtype=np.float64)
    Mvec = np.asarray(Mvec, dtype=np.float64)
    A = np.sqrt(np.sum(Mvec * Mvec, axis=1))
    if logw is None:
        w = np.ones_like(E)
    else:
        logw = np.asarray(logw, dtype=np.float64)
        w = np.exp(logw - logw.max())
    W = w.sum()
    mean = lambda x: float((w * x).sum() / W)
    mE, mA, mA2, mA4 = mean(E), mean(A), mean(A * A), mean(A ** 4)
    dE, dA, dA2 = E - mE, A - mA, A * A - mA2
    varE, varA = mean(dE * dE), mean(dA * dA)
    c1, c2 = mean(dA * dE), mean(dA2 * dE)
    N = float(n_sites)
    m2, m4 = mA2 / N ** 2, mA4 / N ** 4
    return dict(e=mE / N, m_abs=mA / N, m2=m2, m4=m4,
                cv=beta * beta * varE / N, chi=beta * varA / N,
                u4=1.0 - m4 / (3.0 * m2 * m2) if m2 > 0 else 0.0,
                v1=-c1 / mA if mA > 0 else 0.0,
                v2=-c2 / mA2 if mA2 > 0 else 0.0)


def thermal_array(d):
    return np.array([d[k] for k in THERMAL_FIELDS])


def reweight(E, Mvec, n_sites, beta0, beta):
    """Single-histogram reweighting (Ferrenberg and Swendsen 1988): the
    thermal summary at beta of samples drawn at beta0, weights
    exp(-(beta - beta0) E_m)."""
    E = np.asarray(E, dtype=np.float64)
    return thermal(E, Mvec, n_sites, beta, logw=-(beta - beta0) * E)


def autocorr(x, t):
    """Normalised autocorrelation at lag t: C(t)/C(0) with
    C(t) = sum_{m < n-t} (x_m - xbar)(x_{m+t} - xbar) / (n - t)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    d = x - x.mean()
    c0 = (d * d).sum() / n
    if c0 == 0.0:
        return 0.0
    return float((d[: n - t] * d[t:]).sum() / (n - t) / c0)


def tau_int(x, c=6.0):
    """Integrated autocorrelation time with Sokal's automatic window:
    tau(W) = 1/2 + sum_{t=1..W} rho(t), W the first lag with W >= c tau(W)
    (at most n/2).  Returns (tau, W)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    tau = 0.5
    for t in range(1, n // 2 + 1):
        tau += autocorr(x, t)
        if t >= c * tau:
            return tau, t
    return tau, n // 2


def _logsumexp(a):
    m = a.max()
    return m + np.log(np.exp(a - m).sum())


def multihist(Es, betas_k, iters=5000, tol=1e-11):
    """Multiple-histogram free energies (Ferrenberg and Swendsen 1989) of K
    series Es[k] sampled at betas_k[k]: iterate
      f_k = -ln sum_{i,m} exp(-beta_k E_im - ln D_im),
      ln D_im = ln sum_j n_j exp(f_j - beta_j E_im),
    every sum in log space (shifted by its largest exponent), f_0 held at 0,
    until max_k |f_new - f| < tol.  Returns (f, log D per sample, iterations)."""
    betas_k = np.asarray(betas_k, dtype=np.float64)
    nk = np.array([len(e) for e in Es], dtype=np.float64)
    allE = np.concatenate([np.asarray(e, dtype=np.float64) for e in Es])
    f = np.zeros(len(Es))
    it = 0
    while it < iters:
        it += 1
        logD = np.array([_logsumexp(np.log(nk) + f - betas_k * e) for e in allE])
        fn = np.array([-_logsumexp(-b * allE - logD) for b in betas_k])
        fn = fn - fn[0]
        done = np.max(np.abs(fn - f)) < tol
        f = fn
        if done:
            break
    logD = np.array([_logsumexp(np.log(nk) + f - betas_k * e) for e in allE])
    return f, logD, it


def multihist_thermal(Es, Ms, betas_k, f, logD, n_sites, beta):
    """Thermal summary at beta from the K series and their free energies:
    samples of all series, weights exp(-beta E_im - ln D_im)."""
    allE = np.concatenate([np.asarray(e, dtype=np.float64) for e in Es])
    allM = np.concatenate([np.asarray(m, dtype=np.float64) for m in Ms])
    return thermal(allE, allM, n_sites, beta, logw=-beta * allE - logD)
