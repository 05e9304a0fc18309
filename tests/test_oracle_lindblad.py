"""P6: the oracle's trajectory averages against a brute-force density-matrix
solution of the Lindblad equation on a tiny grid.

This is the pin of the stochastic part of the method (Secs. "The
Monte-Carlo Wave-Function method" and "The waiting time approach"): the
average over trajectories of the block indicator 1{c,l} must reproduce
Tr rho_{c,l}(t), and the average of 1{s,0} |<1S|u>|^2/<u|u> (the oracle's
reported 1S overlap) must reproduce <1S|rho_{s,0}|1S>, which also pins the
reading that overlaps are taken on the normalised state.
"""
import numpy as np
import pytest

import oracle
from paper_2107_06147_amd import workloads as W
from tests import lindblad_bruteforce as LB

N, L, M = 32, 10.0, W.MASS_B
T, KH, GH = 0.5, 4.0, -2.0
DT, STEPS, LMAX = 0.002, 1000, 6
NTRAJ = 100000
# Bias allowance: jumps fall on the step grid, about dt/2 after the
# continuous-time waiting time.  At 2e5 trajectories (seed 99) every block
# population agreed with the density matrix within 2.2 sigma (largest
# difference 1.7e-3 at sigma 1.1e-3) at this dt, so the time-step bias is
# below the sampling noise; 5e-4 covers it.
BIAS = 5e-4


@pytest.mark.slow
def test_trajectory_averages_match_bruteforce_lindblad(oracle_lib):
    alpha = 4.0 / 3.0 * W.ALPHA_S
    dr = L / N
    r = np.arange(N) * dr
    u0 = r * np.exp(-r * r / 2.0)
    u0 /= np.sqrt(dr * np.sum(u0**2))
    rho = LB.solve(N, L, M, alpha, KH * T**3, GH * T**3, LMAX,
                   {(0, 0): dr * np.outer(u0[1:], u0[1:])}, DT, STEPS)
    traces = {k: float(np.trace(v).real) for k, v in rho.items()}
    assert sum(traces.values()) > 1.0 - 1e-3          # truncation at l_max is small

    cfg = W.base(N=N, L=L, dt=DT, kappa_hat=KH, gamma_hat=GH, init_kind=W.INIT_ARRAY,
                 n_traj=NTRAJ, seed=21, **W.constant_T(T, STEPS))
    cfg["u0"] = u0.astype(complex)
    res = oracle.run(cfg)
    assert np.all(res["status"] == oracle.STATUS_OK)
    # the blocks beyond l_max hold what the truncated density matrix drops
    assert np.mean(res["l"] > LMAX) < 1e-3
    for (c, l), p in traces.items():
        frac = np.mean((res["color"] == c) & (res["l"] == l))
        sigma = np.sqrt(max(p * (1 - p), 1.0 / NTRAJ) / NTRAJ)
        assert abs(frac - p) < 3 * sigma + BIAS, ((c, l), frac, p, sigma)

    phi = oracle.basis_state(N, L, M, W.ALPHA_S, 1, 0)
    exact = dr * float(phi[1:] @ rho[(0, 0)].real @ phi[1:])   # rho = dr |u><u|
    est = res["overlap"][:, 0]
    sigma = est.std() / np.sqrt(NTRAJ)
    assert abs(est.mean() - exact) < 3 * sigma + BIAS, (est.mean(), exact, sigma)
