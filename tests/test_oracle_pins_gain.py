"""Pins for the oracle's explicit-gain CGD-EnKF (Figure 2, Section 3.1:
one CG per column of K^T) against routes other than its own formula.

* Converged, it is the EnKF: K^T against the brute-force gain of Section 2.2
  (np.linalg.inv of H P H^T + R), X^a against the brute-force analysis.
* Proposition 1 holds for every column's iterates in the energy norm.
* CG's energy-norm errors never increase, and with R = r I (Example 1b's
  R = I) every column ends within N steps: Psi has at most N distinct
  eigenvalues (the bulk at r, N - 1 above it).
* Example 1b's spectrum: with H = I and R = I, m - (N - 1) eigenvalues of
  Psi equal 1 and the rest exceed 1.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.mark.parametrize("seed,n,m,N,k,stochastic", [(0, 30, 12, 7, 2, True),
                                                     (1, 20, 25, 6, 1, False),
                                                     (2, 15, 9, 12, 3, True)])
def test_gain_form_converges_to_bruteforce(seed, n, m, N, k, stochastic):
    p = W.random_problem(n, m, N, k, seed=seed, stochastic=stochastic)
    out = O.enkf_gain_cg(p.Xf, p.idx, p.w, p.y, p.r, p.eps, tol=1e-13, maxit=1000)
    H = O.dense_H(p.idx, p.w, n)
    K = O.kalman_gain_bruteforce(p.Xf, H, np.diag(p.r))
    assert O.rel_frob(out["KT"], K.T) < 1e-10
    assert O.rel_frob(out["Xa"], O.enkf_bruteforce(p.Xf, p.idx, p.w, p.y, p.r, p.eps)) < 1e-10


def test_gain_form_prop1_and_monotone():
    p = W.random_problem(25, 30, 8, 1, seed=4)
    out = O.enkf_gain_cg(p.Xf, p.idx, p.w, p.y, p.r, p.eps, tol=0.0, maxit=12, record=True)
    Psi, B = out["Psi"], out["B"]
    ev = np.linalg.eigvalsh(Psi)
    kappa = ev[-1] / ev[0]
    rate = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    for i in range(B.shape[1]):
        e = O.energy_errors(Psi, B[:, i], out["iterates"][i])
        assert np.all(np.diff(e) <= 1e-12 * e[0] + 1e-15)
        for r, er in enumerate(e):
            assert er <= 2 * rate ** r * e[0] * (1 + 1e-9) + 1e-14


@pytest.mark.parametrize("m,N", [(40, 5), (60, 12)])
def test_example1b_termination_and_spectrum(m, N):
    p = W.example1b(m=m, N=N, rep=0)
    out = O.enkf_gain_cg(p.Xf, p.idx, p.w, p.y, p.r, p.eps, tol=1e-12, maxit=1000)
    assert out["iters"].max() <= N
    ev = np.sort(np.linalg.eigvalsh(out["Psi"]))
    assert np.allclose(ev[:m - (N - 1)], 1.0, atol=1e-12)
    assert np.all(ev[m - (N - 1):] > 1.0 + 1e-9)
