"""History analysis on the GPU (through the C-ABI) against the oracle's
definitions (oracle/analysis.py): thermal summaries with single-histogram
reweighting, integrated autocorrelation times with the automatic window, and
multiple-histogram free energies and interpolation, on synthetic histories
(independent spins sampled exactly) and on the history of a real run.  The
two sides sum in different orders: agreement to 1e-9 relative."""
import numpy as np
import pytest
import torch

import synth
from oracle import analysis as A
from paper_1803_07030_amd import hsim

from test_oracle_analysis import exact_isolated

pytestmark = pytest.mark.gpu


def _close(got, ref, rel=1e-9, floor=1e-12):
    got, ref = np.asarray(got), np.asarray(ref)
    assert np.all(np.abs(got - ref) <= rel * np.abs(ref) + floor), (got, ref)


def _synthetic_history(R, S, M, N, betas, seed=11):
    """history [R][S][M][5] of N isolated spins in B = 1 sampled exactly at
    betas[r][s]; column 4 (accepted) is 0."""
    rng = np.random.default_rng(seed)
    h = np.zeros((R, S, M, 5))
    for r in range(R):
        for s in range(S):
            Mv = exact_isolated(rng, M, N, betas[r][s])
            h[r, s, :, 0] = -Mv[:, 2]
            h[r, s, :, 1:4] = Mv
    return h


def test_thermal_and_reweighting_match_oracle():
    R, S, M, N, m0 = 2, 3, 3000, 16, 100
    betas = np.array([[0.5, 1.0, 1.5], [0.8, 1.2, 2.0]])
    h = _synthetic_history(R, S, M, N, betas)
    d = torch.tensor(h, device="cuda")
    ev = np.stack([betas * f for f in (0.9, 1.0, 1.1)], axis=-1)      # [R][S][3]
    out = hsim.hsim_analysis_thermal(d, m0, N, betas, ev).cpu().numpy()
    plain = hsim.hsim_analysis_thermal(d, m0, N, betas).cpu().numpy()
    for r in range(R):
        for s in range(S):
            E, Mv = h[r, s, m0:, 0], h[r, s, m0:, 1:4]
            _close(plain[r, s, 0], A.thermal_array(A.thermal(E, Mv, N, betas[r, s])))
            for j in range(3):
                ref = A.thermal_array(A.reweight(E, Mv, N, betas[r, s], ev[r, s, j]))
                _close(out[r, s, j], ref)
            _close(out[r, s, 1], plain[r, s, 0], rel=1e-12)


def test_tau_matches_oracle():
    """AR(1) series of several correlations in the E and |M| columns."""
    R, S, M, m0 = 1, 4, 6000, 200
    rng = np.random.default_rng(3)
    h = np.zeros((R, S, M, 5))
    for s, phi in enumerate([0.0, 0.5, 0.8, 0.95]):
        for col in (0, 3):
            e = rng.normal(size=M)
            x = np.empty(M)
            x[0] = e[0]
            for m in range(1, M):
                x[m] = phi * x[m - 1] + e[m]
            h[0, s, :, col] = x + (50.0 if col == 3 else 0.0)       # |M| = M_z > 0
    d = torch.tensor(h, device="cuda")
    for obs, col in ((0, 0), (1, 3)):
        tau, win = hsim.hsim_analysis_tau(d, m0, obs)
        tau, win = tau.cpu().numpy(), win.cpu().numpy()
        for s in range(S):
            t_ref, w_ref = A.tau_int(np.abs(h[0, s, m0:, col]) if obs else h[0, s, m0:, col])
            assert win[0, s] == w_ref
            _close(tau[0, s], t_ref)


def test_multihist_matches_oracle():
    R, S, M, N, m0 = 2, 2, 4000, 6, 0
    betas = np.array([[0.6, 0.9], [1.2, 1.5]])
    h = _synthetic_history(R, S, M, N, betas, seed=5)
    d = torch.tensor(h, device="cuda")
    series = [(0, 0), (0, 1), (1, 0), (1, 1)]
    bk = np.array([betas[r, s] for r, s in series])
    ev = np.array([0.7, 1.05, 1.4])
    f, it, out = hsim.hsim_analysis_multihist(d, m0, N, series, bk, ev, tol=1e-11)
    Es = [h[r, s, m0:, 0] for r, s in series]
    Ms = [h[r, s, m0:, 1:4] for r, s in series]
    f_ref, logD, it_ref = A.multihist(Es, bk, tol=1e-11)
    _close(f, f_ref, rel=1e-9, floor=1e-9)
    assert abs(it - it_ref) <= 1
    out = out.cpu().numpy()
    for j, b in enumerate(ev):
        _close(out[j], A.thermal_array(A.multihist_thermal(Es, Ms, bk, f_ref, logD, N, b)),
               rel=1e-8, floor=1e-10)


def test_analysis_of_a_run():
    """The history of a real run (SC 8^3, 4 replicas, FP32): GPU analysis
    equals the oracle's on the same tensor."""
    lat = synth.sc_periodic(8)
    plan = hsim.Plan(lat)
    R, M = 4, 600
    T = np.array([0.8, 1.2, 1.6, 2.4])
    b = hsim.Batch([plan] * R, seed=2, precision=hsim.FP32, layout=hsim.LAYOUT_SITE).bind(1, M)
    b.init_spins(hsim.INIT_COLD_Z)
    b.run(T[:, None], 0.0, launch=hsim.LAUNCH_GRAPH)
    torch.cuda.synchronize()
    assert b.status() == 0
    beta = (1.0 / T)[:, None]
    th = hsim.hsim_analysis_thermal(b.history, 100, lat.n, beta).cpu().numpy()
    tau, win = hsim.hsim_analysis_tau(b.history, 100, 0)
    h = b.history.cpu().numpy()
    for r in range(R):
        _close(th[r, 0, 0], A.thermal_array(A.thermal(h[r, 0, 100:, 0], h[r, 0, 100:, 1:4], lat.n,
                                                      beta[r, 0])), rel=1e-9, floor=1e-12)
        t_ref, w_ref = A.tau_int(h[r, 0, 100:, 0])
        assert int(win[r, 0]) == w_ref
        _close(float(tau[r, 0]), t_ref)


def test_analysis_argument_errors():
    d = torch.zeros((1, 1, 10, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(hsim.HsimError):
        hsim.hsim_analysis_thermal(d, 9, 8, [[1.0]])          # one sample left
    with pytest.raises(hsim.HsimError):
        hsim.hsim_analysis_tau(d, 0, 2)
    with pytest.raises(hsim.HsimError):
        hsim.hsim_analysis_multihist(d, 0, 8, [(1, 0)], [1.0], [1.0])
