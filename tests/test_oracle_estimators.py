"""Pins of the oracle's fluctuation estimator (oracle.fluct_gradients) on
chains the oracle samples itself, against closed forms of models whose
canonical averages are known exactly.

The estimator differentiates a Boltzmann average (section "Thermal averages":
responses as fluctuations of the sampled chain):
    d<O>/dtheta = <dO/dtheta> - beta Cov(O, dE/dtheta).
Closed forms used:
  * a tree (Fisher 1964) with B = k = 0: the bond variables c_b = S_i.S_j are
    independent, each with density proportional to exp(beta J_b c) on
    [-1, 1], so <c_b> = L(x_b) and Var(c_b) = L'(x_b), x_b = beta J_b, and
    d<E>/dJ_b = -[L(x_b) + x_b L'(x_b)];  the energy does not depend on the
    absolute orientation, so d<E>/dk_i = -<(S_i.e_i)^2> = -1/3 and
    d<E>/dB = 0 at B = 0;
  * isolated spins in a field (Langevin): d<M_z>/dB = beta N L'(x) and
    d<E>/dB = -N [L(x) + x L'(x)], x = beta B.
A sign error in the covariance term, a dropped <dO/dtheta> term or a wrong
bond index moves the estimate by O(1) of these values.
Standard errors come from the spread of independent replicas; exceedances of
3 SE are counted against the 99% binomial bound for the two-sided tail of
Student's t with R - 1 degrees of freedom, and none may exceed 5 SE.
"""
import numpy as np
from scipy import stats

import oracle
import synth
from _stats import langevin


def langevin_prime(x):
    """L'(x) = 1/x^2 - 1/sinh^2 x (series near 0)."""
    x = np.asarray(x, dtype=np.float64)
    small = np.abs(x) < 1e-3
    xs = np.where(small, 1.0, x)
    return np.where(small, 1.0 / 3.0 - x ** 2 / 15.0, 1.0 / xs ** 2 - 1.0 / np.sinh(xs) ** 2)


def _grade(est, exact, R, n_se=3.0, hard=5.0):
    """est: (R, m) per-replica estimates; exact: (m,).  Returns the number of
    3-SE exceedances, the bound it must stay within and the largest
    deviation in SE."""
    mean = est.mean(axis=0)
    se = est.std(axis=0, ddof=1) / np.sqrt(R)
    z = np.abs(mean - exact) / se
    p = 2 * stats.t.sf(n_se, R - 1)
    bound = stats.binom.ppf(0.99, z.size, p)
    return int((z > n_se).sum()), bound, float(z.max()), hard


def _snapshots(lat, T, B, steps, mcs, seed, reps, init="random", burn=0.2):
    jobs = [dict(lat=lat, T=np.full(steps, T), B=np.full(steps, B), mcs_per_step=mcs, seed=seed,
                 replica=r, init=init, snapshots=True) for r in range(reps)]
    res, _ = oracle.run_replicas(jobs)
    s0 = int(burn * steps)
    return [r["snapshots"][s0:] for r in res], [r["history"][s0:, -1] for r in res]


def test_tree_exchange_response_is_fishers():
    lat = synth.random_tree(80, seed=21)
    _, _, Jb = lat.bonds()
    T, R = 1.0, 32
    snaps, _ = _snapshots(lat, T, 0.0, steps=150, mcs=4, seed=611, reps=R)
    gJ, gk, gB = [], [], []
    for s in snaps:
        g = oracle.fluct_gradients(lat, 0.0, s, 1.0 / T)
        gJ.append(g["gJ"])
        gk.append(g["gk"])
        gB.append(g["gB"])
    gJ, gk, gB = np.array(gJ), np.array(gk), np.array(gB)[:, None]
    x = Jb / T
    exact = -(langevin(x) + x * langevin_prime(x))
    for est, ex in ((gJ, exact), (gk, np.full(lat.n, -1.0 / 3.0)), (gB, np.zeros(1))):
        n_out, bound, zmax, hard = _grade(est, ex, R)
        assert n_out <= bound and zmax <= hard, (n_out, bound, zmax)
    # global scale J -> lambda J: d<E>/dlambda = sum_b J_b d<E>/dJ_b
    lam = gJ @ Jb
    n_out, bound, zmax, hard = _grade(lam[:, None], np.array([exact @ Jb]), R)
    assert zmax <= 3.0, zmax
    # the plausible slip: a plus sign on the covariance term
    wrong = -langevin(x) + x * langevin_prime(x)
    assert np.abs(gJ.mean(axis=0) - wrong).max() > 0.1


def test_isolated_spin_field_response_is_langevin():
    N, Bf, T, R = 1024, 1.0, 1.0, 16
    lat = synth.isolated(N)
    snaps, hist_last = _snapshots(lat, T, Bf, steps=120, mcs=2, seed=612, reps=R)
    x = Bf / T
    exact_m = 1.0 / T * N * float(langevin_prime(x))
    exact_e = -N * float(langevin(x) + x * langevin_prime(x))
    em, ee = [], []
    for s, h in zip(snaps, hist_last):
        mz = s[:, :, 2].sum(axis=1)
        # the history's magnetisation at each step end is the snapshot's
        assert np.allclose(mz, h[:, 3], rtol=0, atol=1e-9 * N)
        em.append(oracle.fluct_gradients(lat, Bf, s, 1.0 / T, O=mz)["gB"])
        ee.append(oracle.fluct_gradients(lat, Bf, s, 1.0 / T)["gB"])
    for est, ex in ((em, exact_m), (ee, exact_e)):
        n_out, bound, zmax, hard = _grade(np.array(est)[:, None], np.array([ex]), R)
        assert zmax <= 3.0, (zmax, np.mean(est), ex)
