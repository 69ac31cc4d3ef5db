"""Pins for the oracle's non-diagonal R (Section 5.1: R = L L^T with a sparse
L; Section 5.3 and Example 2: tridiagonal Toeplitz R, sigma^2 on the
diagonal, sigma^2 rho beside it), each against an independent route: a
hand-built matrix, the brute-force Kalman gain, the Woodbury identity of
Algorithm 2, SciPy's preconditioned CG, Lemma 1's step bound and the
convergence of CGD-EnKF-Reduced to EnKF-Reduced (the trend of Table 5)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W


def _tri_problem(n=40, m=30, N=8, k=1, seed=0, sigma=0.3, rho=0.2, stochastic=True):
    p = W.random_problem(n, m, N, k, seed=seed, stochastic=stochastic)
    rd, ro = O.tridiag_toeplitz_R(m, sigma, rho)
    R = O.tridiag_R(rd, ro)
    if stochastic:   # perturbations drawn with the correlated R
        p = __import__("dataclasses").replace(
            p, eps=np.linalg.cholesky(R) @ np.random.default_rng(seed + 1).standard_normal((m, N)))
    return p, R


def test_tridiag_R_hand_example():
    R = O.tridiag_R([1.0, 2.0, 3.0], [0.5, -0.25])
    assert np.array_equal(R, np.array([[1.0, 0.5, 0.0], [0.5, 2.0, -0.25], [0.0, -0.25, 3.0]]))
    rd, ro = O.tridiag_toeplitz_R(4, 0.3, 0.2)
    assert np.allclose(rd, 0.09) and np.allclose(ro, 0.018) and ro.size == 3


def test_cholesky_factor_of_tridiagonal_R_is_bidiagonal():
    # Section 5.3: the factor of a tridiagonal R is bidiagonal (no fill-in)
    rd, ro = O.tridiag_toeplitz_R(50, 0.3, 0.45)
    L = np.linalg.cholesky(O.tridiag_R(rd, ro))
    assert np.count_nonzero(np.tril(L, -2)) == 0
    assert np.allclose(L @ L.T, O.tridiag_R(rd, ro), rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed,n,m,N,k", [(0, 40, 30, 8, 1), (1, 60, 60, 12, 2), (2, 25, 10, 20, 3)])
@pytest.mark.parametrize("stochastic", [False, True])
def test_bruteforce_gain_with_tridiagonal_R(seed, n, m, N, k, stochastic):
    p, R = _tri_problem(n, m, N, k, seed, stochastic=stochastic)
    H = O.dense_H(p.idx, p.w, n)
    K = O.kalman_gain_bruteforce(p.Xf, H, R)
    Y = np.outer(p.y, np.ones(N)) + (0 if p.eps is None else p.eps)
    ref = p.Xf + K @ (Y - H @ p.Xf)
    got = O.enkf_analysis_R(p.Xf, p.idx, p.w, p.y, R, p.eps)["Xa"]
    assert O.rel_frob(got, ref) < 1e-12


@pytest.mark.parametrize("stochastic", [False, True])
def test_reduced_equals_full_with_tridiagonal_R(stochastic):
    # Algorithm 2 with R_N = (N-1) R = L L^T against Algorithm 1 (Woodbury)
    p, R = _tri_problem(50, 40, 9, 2, seed=3, rho=0.4, stochastic=stochastic)
    full = O.enkf_analysis_R(p.Xf, p.idx, p.w, p.y, R, p.eps)["Xa"]
    red = O.enkf_reduced_R(p.Xf, p.idx, p.w, p.y, R, p.eps)["Xa"]
    assert O.rel_frob(red, full) < 1e-12
    redcg = O.enkf_reduced_R(p.Xf, p.idx, p.w, p.y, R, p.eps, solver="cg", tol=1e-14, maxit=200)
    # N steps in exact arithmetic; with sigma^2 = 0.09 the N x N system is
    # ill-conditioned, so FP64 needs a few steps more to reach 1e-14
    assert O.rel_frob(redcg["Xa"], full) < 1e-11 and redcg["iters"].max() <= p.N + 3


def test_pcg_with_M_equal_R_matches_scipy():
    p, R = _tri_problem(60, 45, 10, 1, seed=4, rho=0.45)
    S = O.obs_anomalies(p.idx, p.w, p.Xf)
    D = O.innovations(p.idx, p.w, p.Xf, p.y, p.eps)
    Psi = O.innovation_matrix_R(S, R)
    cf = sla.cho_factor(R, lower=True)
    Mop = spla.LinearOperator(R.shape, matvec=lambda v: sla.cho_solve(cf, v))
    seen = []
    spla.cg(Psi, D[:, 1], M=Mop, rtol=1e-300, atol=0.0, maxiter=6,
            callback=lambda xk: seen.append(xk.copy()))
    ours = O.textbook_pcg_op(O.matvec_free_R(S, R), lambda v: sla.cho_solve(cf, v), D[:, 1], 0.0,
                             6, record=True).iterates[1:]
    for a, b in zip(ours, seen):
        assert np.linalg.norm(a - b) <= 1e-11 * np.linalg.norm(b)


def test_pcg_with_M_equal_R_terminates_in_N_steps_and_reaches_cholesky():
    # whitened by R's factor, Psi becomes I + P P^T with rank(P) <= N-1 (Lemma 1)
    p, R = _tri_problem(400, 300, 8, 1, seed=5, rho=0.45)
    pcg = O.enkf_analysis_R(p.Xf, p.idx, p.w, p.y, R, p.eps, solver="pcg", tol=1e-11)
    cg = O.enkf_analysis_R(p.Xf, p.idx, p.w, p.y, R, p.eps, solver="cg", tol=1e-11)
    chol = O.enkf_analysis_R(p.Xf, p.idx, p.w, p.y, R, p.eps)
    assert pcg["iters"].max() <= p.N
    assert cg["iters"].max() > p.N
    assert O.rel_frob(pcg["Xa"], chol["Xa"]) < 1e-10
    assert O.rel_frob(cg["Xa"], chol["Xa"]) < 1e-9


def test_diagonal_R_reduces_to_the_diagonal_oracle():
    p = W.random_problem(40, 25, 7, 2, seed=6)
    a = O.enkf_analysis_R(p.Xf, p.idx, p.w, p.y, np.diag(p.r), p.eps, solver="pcg", tol=1e-12)
    b = O.enkf_analysis(p.Xf, p.idx, p.w, p.y, p.r, p.eps, solver="pcg_free", tol=1e-12)
    assert O.rel_frob(a["Xa"], b["Xa"]) < 1e-13 and np.array_equal(a["iters"], b["iters"])
    r1 = O.enkf_reduced_R(p.Xf, p.idx, p.w, p.y, np.diag(p.r), p.eps)["Xa"]
    r2 = O.enkf_reduced(p.Xf, p.idx, p.w, p.y, p.r, p.eps)["Xa"]
    assert O.rel_frob(r1, r2) < 1e-13


def test_table5_trend_error_falls_with_r():
    """Example 2b: CGD-EnKF-Reduced with a fixed number r of CG steps against
    EnKF-Reduced, Lorenz-96 with H = I and the tridiagonal R (sigma 0.3,
    rho 0.2).  The error falls as r grows and vanishes by r = N (exact
    termination), the trend Table 5 reports."""
    rng = np.random.default_rng(7)
    n, N = 200, 20
    xt = W.l96_truth(n, rng, steps=200, dt=0.05)
    Xf = xt[:, None] + rng.standard_normal((n, N))
    idx, w = W.identity_obs(n)
    rd, ro = O.tridiag_toeplitz_R(n, 0.3, 0.2)
    R = O.tridiag_R(rd, ro)
    y = xt + np.linalg.cholesky(R) @ rng.standard_normal(n)
    ref = O.enkf_reduced_R(Xf, idx, w, y, R)["Xa"]
    errs = [O.rel_frob(O.enkf_reduced_R(Xf, idx, w, y, R, solver="cg", tol=0.0, maxit=r)["Xa"],
                       ref) for r in (1, 2, 3, 5, 8, 12, N)]
    assert all(a > b for a, b in zip(errs, errs[1:-1])), errs
    assert errs[0] > 1e-2 and errs[-1] < 1e-10
