"""The rule every single-precision site-by-site test asserts.

The FP32 kernels and the oracle draw the same random words and the oracle
evaluates the same proposal map in double precision.  Eq. 4's test accepts a
move iff dE < t with the threshold t = -ln(u)/beta (t = 0 at T = 0; every
move at T = inf), so a decision can come out differently only when the
oracle's dE lies within the single-precision error of the kernel's dE and
threshold from t ("a near tie").  A site whose decision differed changes the
field of its neighbours, so a neighbour in a LATER colour class of the same
MCS may then decide differently too.  Everything else must agree: decisions
exactly, and accepted spins to single-precision accuracy.

Error bound of the kernel's dE at site i (fused multiply-add chains in CSR
order, unit-roundoff u32 = 2^-24): the field sums deg_i + 1 terms, the
energy change adds a 3-term dot product with |S' - S| <= 2 mu_i and the
anisotropy differences, and the trial point carries the error of the
hardware sine/cosine/square root (a few ulp, bounded here by 2^-19 of each
term's size):
    delta_i = u32 (8 (deg_i + 3) s_i + 8 (|dE_i| + |t_i|)) + 2^-19 s_i + 2^-22 / beta
with s_i = sum_j |J_ij| mu_i mu_j + |B| mu_i + 2 (k_i + |kc_i|) mu_i^2.  The
last term is the float exponential's rounding, moved to the dE axis.  A near
tie is a margin |dE_i - t_i| <= 4 delta_i.
"""
import numpy as np

import oracle

U32 = 2.0 ** -24


def site_scale(lat, Bf):
    n = lat.n
    mu = np.ones(n) if getattr(lat, "norm", None) is None else np.asarray(lat.norm, dtype=np.float64)
    rows = np.repeat(np.arange(n), np.diff(lat.row_ptr))
    sJ = np.zeros(n)
    np.add.at(sJ, rows, np.abs(lat.J) * mu[rows] * mu[lat.col])
    k = np.zeros(n) if lat.k is None else np.abs(lat.k)
    kc = np.zeros(n) if getattr(lat, "kc", None) is None else np.abs(lat.kc)
    return sJ + abs(Bf) * mu + 2.0 * (k + kc) * mu ** 2


def check_one_mcs(lat, colour, start, T, Bf, seed, rep, got, policies=None, spin_tol=4e-6):
    """One MCS of replica rep from `start` (both sides): returns the number of
    differing decisions; asserts that each is a near tie or follows a
    differing neighbour of an earlier colour, and that the other sites agree."""
    ref = oracle.run(lat, [T], [Bf], 1, seed=seed, replica=rep, init="given", spins=start,
                     proposal=oracle.PROPOSAL_F32MAP, trace_accepts=True, decision_trace=True,
                     policies=policies)
    acc = ref["accept"][0].astype(bool)
    moved = np.any(got != start, axis=1)
    dec = moved != acc
    same = ~dec
    if same.any():
        err = np.max(np.abs(got[same] - ref["spins"][same]))
        assert err <= spin_tol, (rep, err)
    if not dec.any():
        return 0
    dE, u = ref["dE_trace"][0], ref["u_trace"][0]
    if T == 0.0:
        t, inv_beta = np.zeros_like(u), 0.0
    elif np.isinf(T):
        raise AssertionError("a decision differs at T = inf, where every move is accepted")
    else:
        beta = 1.0 / T
        t, inv_beta = -np.log(u) / beta, T
    deg = np.diff(lat.row_ptr)
    s = site_scale(lat, Bf)
    delta = U32 * (8 * (deg + 3) * s + 8 * (np.abs(dE) + np.abs(t))) + 2.0 ** -19 * s + \
        2.0 ** -22 * inv_beta
    tie = np.abs(dE - t) <= 4.0 * delta
    for i in np.flatnonzero(dec):
        if tie[i]:
            continue
        nb = lat.col[lat.row_ptr[i]:lat.row_ptr[i + 1]]
        earlier = nb[colour[nb] < colour[i]]
        assert dec[earlier].any(), (
            f"replica {rep}, site {i}: decision differs {abs(dE[i] - t[i]):.3g} from its "
            f"tie (bound {4 * delta[i]:.3g}) with no differing earlier neighbour")
    return int(dec.sum())
