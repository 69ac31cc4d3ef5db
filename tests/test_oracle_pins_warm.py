"""Pins for the parts of the oracle that a warm start or a preconditioner
reaches: the stall-window restart of textbook CG, textbook PCG with
M = diag(r), and the warm-start network's features and Jacobi start.

Each compares the oracle with an independent route: a closed form of the CG
residual history, SciPy's preconditioned CG, Cholesky, Lemma 1's step bound,
hand-computed feature values and the formed innovation matrix.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
import oracle.enkf as E
from oracle import wsnet as NET
import workloads as W


# --------------------------------------------------------------------------
# Stall window (no paper source: the warm-start restart rule).  Closed form:
# for T = tridiag(-1, 2, -1) of order M with T[0, 0] = 1 + u and a residual
# r_0 = c e_1, the Krylov space K_k(T, e_1) is span(e_1..e_k), so the CG
# iterate solves the leading k x k block and r_k = c x_k[k-1] e_{k+1} with
# x_k[k-1] = 1/det(T_k) = 1/(1 + k u) (the determinants obey
# D_k = 2 D_{k-1} - D_{k-2}, D_0 = 1, D_1 = 1 + u).  Hence
# ||r_k|| / ||r_{k-w}|| = (1 + (k-w) u)/(1 + k u), and the first k >= w at
# which it exceeds f is the first integer above 10 w - 1/u for f = 0.9.
# --------------------------------------------------------------------------
U_STALL = Fraction(2, 81)          # 1/u = 40.5: the rule (5, 0.9) fires at k = 10


def stall_matrix(M: int, u: Fraction = U_STALL) -> np.ndarray:
    T = 2.0 * np.eye(M) - np.eye(M, k=1) - np.eye(M, k=-1)
    T[0, 0] = 1.0 + float(u)
    return T


def closed_form_restart(window: int, factor: Fraction, u: Fraction = U_STALL) -> int:
    """First k >= window with (1 + (k-window) u)/(1 + k u) > factor, exactly."""
    k = window
    while not (1 + (k - window) * u) > factor * (1 + k * u):
        k += 1
    return k


def stall_problem(M=30, seed=0, c=0.7):
    """A system T z = d and a warm start z0 whose residual is c e_1."""
    rng = np.random.default_rng(seed)
    T = stall_matrix(M)
    z0 = rng.standard_normal(M) * 3.0
    e1 = np.zeros(M)
    e1[0] = c
    d = e1 + T @ z0
    return T, d, z0


def test_stall_closed_form_residual_history():
    # the closed form itself, checked against the oracle's recursive residuals
    T, d, z0 = stall_problem()
    res = O.textbook_cg(O.matvec_dense(T), d, 0.0, 12, z0=z0)
    c = np.linalg.norm(d - T @ z0)
    for k in range(12):
        assert abs(res.resnorms[k] - c / (1.0 + k * float(U_STALL))) <= 1e-11 * c, k


def test_stall_window_restart_point():
    T, d, z0 = stall_problem()
    assert np.linalg.norm(d - T @ z0) <= np.linalg.norm(d)   # the window branch, not ||r0|| > ||d||
    mv = O.matvec_dense(T)
    zero = O.textbook_cg(mv, d, 1e-10, 500)
    warm = O.textbook_cg(mv, d, 1e-10, 500, z0=z0, fallback_on_stall=True)
    assert warm.fallback
    # after the restart the column repeats the zero-start run step for step
    assert warm.it - zero.it == closed_form_restart(5, Fraction(9, 10)) == 10
    assert np.array_equal(warm.z, zero.z)
    assert np.linalg.norm(T @ warm.z - d) <= 1e-9 * np.linalg.norm(d)


def test_stall_closed_form_separates_the_constants():
    # the pin above fails for a wrong window or factor (planted in the mutation tests)
    assert closed_form_restart(4, Fraction(9, 10)) == 4
    assert closed_form_restart(5, Fraction(8, 10)) == 5
    assert closed_form_restart(6, Fraction(9, 10)) == 20


def test_stall_rule_inactive_without_warm_start_and_after_restart():
    T, d, _ = stall_problem()
    mv = O.matvec_dense(T)
    a = O.textbook_cg(mv, d, 1e-10, 500)
    b = O.textbook_cg(mv, d, 1e-10, 500, fallback_on_stall=True)
    assert not b.fallback and a.it == b.it and np.array_equal(a.z, b.z)


def test_pcg_stall_window_with_scalar_preconditioner():
    # M = c I: PCG takes CG's steps and measures r in a norm scaled by
    # 1/sqrt(c), so the restart point is the same closed-form k
    T, d, z0 = stall_problem(seed=1)
    mv = O.matvec_dense(T)
    minv = np.full(T.shape[0], 1.0 / 3.0)
    zero = O.textbook_pcg(mv, minv, d, 1e-10, 500)
    warm = O.textbook_pcg(mv, minv, d, 1e-10, 500, z0=z0, fallback_on_stall=True)
    assert warm.fallback and warm.it - zero.it == 10


# --------------------------------------------------------------------------
# Textbook PCG with M = diag(r) (diag(R) preconditioning: the L^{-1} scaling
# of Algorithm 2 applied to the full system; Section 5.2, Lemma 1)
# --------------------------------------------------------------------------
def _enkf(p):
    S = O.obs_anomalies(p.idx, p.w, p.Xf)
    D = O.innovations(p.idx, p.w, p.Xf, p.y, p.eps)
    return S, D


def test_pcg_iterates_match_scipy_preconditioned_cg():
    p = W.random_problem(60, 40, 9, 2, seed=31, r_lo=0.1, r_hi=5.0)
    S, D = _enkf(p)
    Psi = O.innovation_matrix(S, p.r)
    d = D[:, 2]
    minv = 1.0 / p.r
    Mop = spla.LinearOperator(Psi.shape, matvec=lambda v: minv * v)
    seen = []
    spla.cg(Psi, d, M=Mop, rtol=1e-300, atol=0.0, maxiter=7,
            callback=lambda xk: seen.append(xk.copy()))
    ours = O.textbook_pcg(O.matvec_dense(Psi), minv, d, 0.0, 7, record=True).iterates[1:]
    assert len(seen) >= 7
    for a, b in zip(ours, seen):
        assert np.linalg.norm(a - b) <= 1e-11 * np.linalg.norm(b)


def test_pcg_terminates_in_at_most_N_steps_for_diagonal_R():
    # Lemma 1: the scaled matrix is I + P P^T with rank(P) <= N - 1, so PCG
    # with M = R needs at most N steps for any diagonal R, where plain CG
    # needs many more
    p = W.random_problem(600, 300, 8, 1, seed=32, r_lo=0.05, r_hi=20.0)
    pcg = O.enkf_analysis(*(p.Xf, p.idx, p.w, p.y, p.r, p.eps), solver="pcg_free", tol=1e-11)
    cg = O.enkf_analysis(*(p.Xf, p.idx, p.w, p.y, p.r, p.eps), solver="cg_free", tol=1e-11)
    chol = O.enkf_analysis(*(p.Xf, p.idx, p.w, p.y, p.r, p.eps))
    assert pcg["iters"].max() <= p.N
    assert cg["iters"].max() > 2 * p.N
    assert O.rel_frob(pcg["Xa"], chol["Xa"]) < 1e-10
    assert O.rel_frob(pcg["Z"], chol["Z"]) < 1e-9


def test_pcg_converges_to_cholesky():
    p = W.config1()
    chol = O.enkf_analysis(p.Xf, p.idx, p.w, p.y, p.r, p.eps)
    errs = [O.rel_frob(O.enkf_analysis(p.Xf, p.idx, p.w, p.y, p.r, p.eps, solver="pcg_free",
                                       tol=t)["Xa"], chol["Xa"]) for t in (1e-2, 1e-5, 1e-10)]
    assert errs[-1] < 1e-10 and errs[0] > errs[-1]


def test_pcg_stop_rule_is_the_rinv_norm_of_the_true_residual():
    p = W.random_problem(80, 50, 10, 2, seed=33, r_lo=0.01, r_hi=10.0)
    S, D = _enkf(p)
    mv = O.matvec_free(S, p.r)
    minv = 1.0 / p.r
    tol = 1e-4
    for j in range(3):
        d = D[:, j]
        rec = O.textbook_pcg(mv, minv, d, tol, 500, record=True)
        # first k at which the true residual meets the rule in the R^{-1} norm
        nrm = lambda v: np.sqrt(v @ (minv * v))
        first = next(k for k, z in enumerate(rec.iterates) if nrm(d - mv(z)) <= tol * nrm(d))
        assert rec.it == first


def test_pcg_with_scalar_preconditioner_is_cg():
    p = W.random_problem(50, 30, 8, 1, seed=34, r_lo=1.5, r_hi=1.5)
    S, D = _enkf(p)
    mv = O.matvec_free(S, p.r)
    a = O.textbook_cg(mv, D[:, 0], 1e-9, 200, record=True)
    b = O.textbook_pcg(mv, 1.0 / p.r, D[:, 0], 1e-9, 200, record=True)
    assert a.it == b.it
    for x, y in zip(a.iterates, b.iterates):
        assert np.linalg.norm(x - y) <= 1e-12 * max(1.0, np.linalg.norm(y))


def test_pcg_warm_start_fallback_uses_rinv_norm():
    p = W.random_problem(40, 25, 10, 1, seed=35, r_lo=0.2, r_hi=5.0)
    S, D = _enkf(p)
    mv = O.matvec_free(S, p.r)
    zs = O.solve_cholesky(O.innovation_matrix(S, p.r), D)
    minv = 1.0 / p.r
    Zw, its, cols = O.solve_pcg_columns(mv, minv, D, 1e-10, 500, Z0=-10 * zs,
                                        fallback_on_stall=True)
    assert all(c.fallback for c in cols)
    Zg, itg, colg = O.solve_pcg_columns(mv, minv, D, 1e-10, 500, Z0=zs * (1 + 1e-7),
                                        fallback_on_stall=True)
    assert not any(c.fallback for c in colg)
    assert np.max(np.abs(Zg - zs)) <= 1e-8 * np.abs(zs).max()


# --------------------------------------------------------------------------
# Warm-start network features (no paper source): hand-computed example
# --------------------------------------------------------------------------
def test_features_hand_example():
    # m = 4 observations, N = 3 members.
    # d_1 = (3, 4, 0, 0): RMS = sqrt(25/4) = 2.5;  d_2 = (1, 1, 1, 1): RMS = 1;
    # d_3 = (0, 0, 0, 6): RMS = sqrt(36/4) = 3.
    D = np.array([[3.0, 1.0, 0.0], [4.0, 1.0, 0.0], [0.0, 1.0, 0.0], [0.0, 1.0, 6.0]])
    # rows of S sum to zero; sum_j S_ij^2 = (2, 8, 0, 18), so divided by N - 1 = 2:
    S = np.array([[1.0, -1.0, 0.0], [2.0, 0.0, -2.0], [0.0, 0.0, 0.0], [3.0, -3.0, 0.0]])
    r = np.array([0.5, 1.0, 2.0, 4.0])
    x, s = NET.features(D, S, r)
    assert np.allclose(s, [2.5, 1.0, 3.0], rtol=0, atol=1e-15)
    assert np.allclose(x[0, 0], [1.2, 1.6, 0.0, 0.0], atol=1e-15)
    assert np.allclose(x[1, 0], [1.0, 1.0, 1.0, 1.0], atol=1e-15)
    assert np.allclose(x[2, 0], [0.0, 0.0, 0.0, 2.0], atol=1e-15)
    for j in range(3):
        assert np.allclose(x[j, 1], [1.0, 4.0, 0.0, 9.0], atol=1e-15)
        assert np.allclose(x[j, 2], r, atol=0)


def test_features_zero_innovation_keeps_scale_one():
    D = np.zeros((5, 2))
    S = np.ones((5, 2)) * np.array([1.0, -1.0])
    x, s = NET.features(D, S, np.ones(5))
    assert np.all(s == 1.0) and not x[:, 0].any()


# --------------------------------------------------------------------------
# Jacobi start: z0 = D / diag(Psi), against the formed innovation matrix
# --------------------------------------------------------------------------
def test_jacobi_z0_matches_formed_psi_diagonal():
    p = W.random_problem(40, 30, 7, 3, seed=36)
    S, D = _enkf(p)
    dg = np.diag(O.innovation_matrix(S, p.r))
    z0 = NET.jacobi_z0(D, S, p.r)
    assert np.allclose(z0, D / dg[:, None], rtol=1e-14, atol=0)
    # one Jacobi sweep from zero: the diagonal part of Psi z0 reproduces D exactly
    assert np.allclose(dg[:, None] * z0, D, rtol=1e-14, atol=1e-15)
