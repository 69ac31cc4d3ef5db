"""FP64 oracle: the EnKF analysis by its definitions (test infrastructure only).

Notation (build <- paper): n <- m (state dim), m <- p (obs dim), S <- Z-hat
(centred predicted observations), D <- Y - Z (innovations, one column per
member), Z_sol <- the CG unknowns Psi^{-1} D.

Nothing here is blocked, fused or reordered beyond what the cited definition
states; library primitives (matmul, Cholesky) serve as single steps.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np
import scipy.linalg as sla

__all__ = [
    "observe", "ensemble_mean", "state_anomalies", "obs_anomalies", "innovations",
    "innovation_matrix", "cross_covariance", "dense_H", "matvec_dense", "matvec_free",
    "CGResult", "textbook_cg", "solve_cg_columns", "textbook_pcg", "solve_pcg_columns",
    "solve_cholesky", "analysis_update",
    "enkf_analysis", "alg1_exact", "kalman_gain_bruteforce", "enkf_bruteforce",
    "enkf_reduced", "senkf", "true_relres", "true_relres_rinv", "rel_frob", "STALL_WINDOW",
    "STALL_FACTOR", "tridiag_R", "tridiag_toeplitz_R", "innovation_matrix_R", "matvec_free_R",
    "textbook_pcg_op", "enkf_analysis_R", "enkf_reduced_R", "enkf_gain_cg", "energy_errors",
]


# ---------------------------------------------------------------------------
# Section 2.3: ensemble statistics and predicted observations
# ---------------------------------------------------------------------------
def observe(idx: np.ndarray, w: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Z = H X^f for an observation operator given as rows of (index, weight)
    pairs: (H X)_{ij} = sum_t w_{it} X_{idx_{it}, j}  (Section 2.3)."""
    idx = np.asarray(idx)
    w = np.asarray(w, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    out = np.zeros((idx.shape[0], X.shape[1]))
    for i in range(idx.shape[0]):
        for t in range(idx.shape[1]):
            out[i] += w[i, t] * X[idx[i, t]]
    return out


def ensemble_mean(X: np.ndarray) -> np.ndarray:
    """x-bar = (1/N) sum_i x_i  (Section 2.3)."""
    return np.asarray(X, dtype=np.float64).mean(axis=1)


def state_anomalies(X: np.ndarray) -> np.ndarray:
    """A = X^f - x-bar 1^T, i.e. X^f (I - Q_1) with Q_1 = 11^T/N  (Section 5)."""
    X = np.asarray(X, dtype=np.float64)
    return X - ensemble_mean(X)[:, None]


def obs_anomalies(idx, w, X) -> np.ndarray:
    """S = H A.  Equal to Z - z-bar 1^T (eq. Zhat_def) since H is linear."""
    return observe(idx, w, state_anomalies(X))


def innovations(idx, w, X, y, eps=None) -> np.ndarray:
    """D = Y - Z with Y = y 1^T (deterministic form, Section 2.3) plus the
    member perturbations eps for the stochastic form (Remark in Section 2.3)."""
    HX = observe(idx, w, X)
    D = np.asarray(y, dtype=np.float64)[:, None] - HX
    if eps is not None:
        D = D + np.asarray(eps, dtype=np.float64)
    return D


def innovation_matrix(S: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Psi_z = S S^T/(N-1) + R with R = diag(r)  (eq. Psi_zz), symmetrised."""
    N = S.shape[1]
    Psi = S @ S.T / (N - 1) + np.diag(np.asarray(r, dtype=np.float64))
    return 0.5 * (Psi + Psi.T)


def cross_covariance(A: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Psi_x = A S^T/(N-1)  (Section 2.3)."""
    return A @ S.T / (S.shape[1] - 1)


def dense_H(idx, w, n: int) -> np.ndarray:
    H = np.zeros((idx.shape[0], n))
    for i in range(idx.shape[0]):
        for t in range(idx.shape[1]):
            H[i, idx[i, t]] += w[i, t]
    return H


def matvec_dense(Psi: np.ndarray) -> Callable[[np.ndarray], np.ndarray]:
    return lambda v: Psi @ v


def matvec_free(S: np.ndarray, r: np.ndarray) -> Callable[[np.ndarray], np.ndarray]:
    """Psi v = S (S^T v)/(N-1) + R v, the three-stage product of Section 3.3
    (eq. matvec_decomp), without forming Psi."""
    N = S.shape[1]
    r = np.asarray(r, dtype=np.float64)

    def mv(v):
        return S @ (S.T @ v) / (N - 1) + (r * v.T).T if v.ndim > 1 else S @ (S.T @ v) / (N - 1) + r * v
    return mv


# ---------------------------------------------------------------------------
# Section 3.1: classical CG (Hestenes-Stiefel) on the SPD system Psi z = d
# ---------------------------------------------------------------------------
STALL_WINDOW = 5     # iterations over which a warm-started column must make progress
STALL_FACTOR = 0.9   # ... by at least this factor, or it restarts from zero


@dataclasses.dataclass
class CGResult:
    z: np.ndarray
    it: int
    resnorms: list
    iterates: list
    fallback: bool = False


def textbook_cg(matvec, d: np.ndarray, tol: float, maxit: int, z0: Optional[np.ndarray] = None,
                fallback_on_stall: bool = False, record: bool = False) -> CGResult:
    """Classical conjugate gradients for one right-hand side (Section 3.1).

    Iteration: q = Psi p, alpha = rho / p^T q, z += alpha p, r -= alpha q,
    rho' = r^T r, beta = rho'/rho, p = r + beta p.  Stop when
    ||r|| <= tol * ||d|| (recursive residual, relative to the data even with
    a warm start) or after maxit iterations.  tol = 0 runs exactly maxit
    iterations unless the residual vanishes.

    Warm-start fallback (no paper source; the rule the library implements):
    if the initial residual of a warm start exceeds ||d||, or while still on
    the warm start ||r_k|| > STALL_FACTOR * ||r_{k-STALL_WINDOW}||, the column
    restarts once from z = 0; iterations spent before the restart still count.
    """
    d = np.asarray(d, dtype=np.float64)
    dnorm = np.linalg.norm(d)
    fallback = False
    warm = z0 is not None
    if warm:
        z = np.array(z0, dtype=np.float64)
        r = d - matvec(z)
        if fallback_on_stall and np.linalg.norm(r) > dnorm:
            z = np.zeros_like(d)
            r = d.copy()
            fallback, warm = True, False
    else:
        z = np.zeros_like(d)
        r = d.copy()
    p = r.copy()
    rho = float(r @ r)
    hist = [np.sqrt(rho)]
    iterates = [z.copy()] if record else []
    it = 0
    while np.sqrt(rho) > tol * dnorm and it < maxit and rho > 0.0:
        # the stall test runs only after the convergence and cap tests above
        if (fallback_on_stall and warm and len(hist) > STALL_WINDOW
                and hist[-1] > STALL_FACTOR * hist[-1 - STALL_WINDOW]):
            z = np.zeros_like(d)
            r = d.copy()
            p = r.copy()
            rho = float(r @ r)
            fallback, warm = True, False
            continue
        q = matvec(p)
        alpha = rho / float(p @ q)
        z = z + alpha * p
        r = r - alpha * q
        rho_new = float(r @ r)
        it += 1
        hist.append(np.sqrt(rho_new))
        if record:
            iterates.append(z.copy())
        p = r + (rho_new / rho) * p
        rho = rho_new
    return CGResult(z, it, hist, iterates, fallback)


def solve_cg_columns(matvec, D: np.ndarray, tol: float, maxit: int, Z0=None,
                     fallback_on_stall: bool = False):
    """One independent textbook CG per column of D: the N right-hand sides
    share Psi but nothing else (the multi-RHS reading of the paper's block CG)."""
    cols = [textbook_cg(matvec, D[:, j], tol, maxit, None if Z0 is None else Z0[:, j],
                        fallback_on_stall) for j in range(D.shape[1])]
    Z = np.stack([c.z for c in cols], axis=1) if cols else np.zeros_like(D)
    return Z, np.array([c.it for c in cols], dtype=np.int64), cols


def textbook_pcg(matvec, minv: np.ndarray, d: np.ndarray, tol: float, maxit: int,
                 z0: Optional[np.ndarray] = None, fallback_on_stall: bool = False,
                 record: bool = False) -> CGResult:
    """Preconditioned conjugate gradients with a diagonal preconditioner M
    (minv = diag(M^{-1})), in the form of Shewchuk's preconditioned CG (the
    reference the paper cites for CG): s = M^{-1} r, delta = r^T s,
    q = Psi p, alpha = delta / p^T q, z += alpha p, r -= alpha q,
    s = M^{-1} r, delta' = r^T s, p = s + (delta'/delta) p.

    For M = R = diag(r) this is CG on the system scaled by L^{-1} as in
    Algorithm 2 (Section 5.2, whose Lemma 1 bounds the steps by the number of
    distinct eigenvalues of I + P P^T, at most N).  Its natural norm is the
    M^{-1}-norm ||v||_{M^{-1}} = sqrt(v^T M^{-1} v): stop when
    ||r||_{M^{-1}} <= tol * ||d||_{M^{-1}} (relative to the data even with a
    warm start) or after maxit iterations.  The warm-start fallback of
    textbook_cg applies with the same norm (resnorms records it)."""
    d = np.asarray(d, dtype=np.float64)
    minv = np.asarray(minv, dtype=np.float64)
    dnorm = np.sqrt(float(d @ (minv * d)))
    fallback = False
    warm = z0 is not None
    if warm:
        z = np.array(z0, dtype=np.float64)
        r = d - matvec(z)
        if fallback_on_stall and np.sqrt(float(r @ (minv * r))) > dnorm:
            z = np.zeros_like(d)
            r = d.copy()
            fallback, warm = True, False
    else:
        z = np.zeros_like(d)
        r = d.copy()
    s = minv * r
    p = s.copy()
    delta = float(r @ s)
    hist = [np.sqrt(delta)]
    iterates = [z.copy()] if record else []
    it = 0
    while np.sqrt(delta) > tol * dnorm and it < maxit and delta > 0.0:
        if (fallback_on_stall and warm and len(hist) > STALL_WINDOW
                and hist[-1] > STALL_FACTOR * hist[-1 - STALL_WINDOW]):
            z = np.zeros_like(d)
            r = d.copy()
            s = minv * r
            p = s.copy()
            delta = float(r @ s)
            fallback, warm = True, False
            continue
        q = matvec(p)
        alpha = delta / float(p @ q)
        z = z + alpha * p
        r = r - alpha * q
        s = minv * r
        delta_new = float(r @ s)
        it += 1
        hist.append(np.sqrt(delta_new))
        if record:
            iterates.append(z.copy())
        p = s + (delta_new / delta) * p
        delta = delta_new
    return CGResult(z, it, hist, iterates, fallback)


def solve_pcg_columns(matvec, minv: np.ndarray, D: np.ndarray, tol: float, maxit: int, Z0=None,
                      fallback_on_stall: bool = False):
    """textbook_pcg independently per column of D (one preconditioner)."""
    cols = [textbook_pcg(matvec, minv, D[:, j], tol, maxit, None if Z0 is None else Z0[:, j],
                         fallback_on_stall) for j in range(D.shape[1])]
    Z = np.stack([c.z for c in cols], axis=1) if cols else np.zeros_like(D)
    return Z, np.array([c.it for c in cols], dtype=np.int64), cols


def solve_cholesky(Psi: np.ndarray, D: np.ndarray) -> np.ndarray:
    """Z = Psi^{-1} D by Cholesky: the classical EnKF solve (eq. K_EnKF)."""
    return sla.cho_solve(sla.cho_factor(Psi, lower=True), D)


# ---------------------------------------------------------------------------
# Algorithm 1 and the update used by the CG form
# ---------------------------------------------------------------------------
def analysis_update(Xf: np.ndarray, S: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """X^a = X^f + Psi_x Z = X^f + A (S^T Z)/(N-1): the EnKF update
    X^a = X^f + K (Y - Z) with K (Y - Z) = Psi_x Psi_z^{-1} D (Section 2.3)."""
    A = state_anomalies(Xf)
    return np.asarray(Xf, dtype=np.float64) + A @ (S.T @ Z) / (S.shape[1] - 1)


def enkf_analysis(Xf, idx, w, y, r, eps=None, solver: str = "cholesky", tol: float = 1e-10,
                  maxit: int = 10000, Z0=None, fallback_on_stall: bool = False) -> dict:
    """One EnKF analysis.  solver: 'cholesky' (formed Psi, direct),
    'cg' (textbook CG on the formed Psi, per column), 'cg_free' (textbook CG
    with the three-stage product of Section 3.3, Psi never formed),
    'pcg_free' (textbook_pcg with M = diag(r) and the three-stage product)."""
    S = obs_anomalies(idx, w, Xf)
    D = innovations(idx, w, Xf, y, eps)
    out = {"S": S, "D": D}
    if solver == "cholesky":
        Z = solve_cholesky(innovation_matrix(S, r), D)
        its = np.zeros(D.shape[1], dtype=np.int64)
    elif solver in ("cg", "cg_free"):
        mv = matvec_dense(innovation_matrix(S, r)) if solver == "cg" else matvec_free(S, r)
        Z, its, cols = solve_cg_columns(mv, D, tol, maxit, Z0, fallback_on_stall)
        out["fallbacks"] = np.array([c.fallback for c in cols])
    elif solver == "pcg_free":
        minv = 1.0 / np.asarray(r, dtype=np.float64)
        Z, its, cols = solve_pcg_columns(matvec_free(S, r), minv, D, tol, maxit, Z0,
                                         fallback_on_stall)
        out["fallbacks"] = np.array([c.fallback for c in cols])
    else:
        raise ValueError(solver)
    out["Z"] = Z
    out["iters"] = its
    out["Xa"] = analysis_update(Xf, S, Z)
    return out


def alg1_exact(Xf, idx, w, y, r, eps=None) -> np.ndarray:
    """Algorithm 1 literally: X^a = X^f + X^f Zhat^T (Zhat Zhat^T + R_N)^{-1}
    ((y - z-bar) 1^T - Zhat) with R_N = (N-1) R, Zhat = Z (I - Q_1); the
    stochastic form adds eps to the bracket."""
    Xf = np.asarray(Xf, dtype=np.float64)
    N = Xf.shape[1]
    Zp = observe(idx, w, Xf)
    Q1 = np.full((N, N), 1.0 / N)
    Zhat = Zp @ (np.eye(N) - Q1)
    zbar = Zp @ np.ones(N) / N
    RN = (N - 1) * np.diag(np.asarray(r, dtype=np.float64))
    rhs = np.outer(np.asarray(y) - zbar, np.ones(N)) - Zhat
    if eps is not None:
        rhs = rhs + eps
    return Xf + Xf @ Zhat.T @ np.linalg.solve(Zhat @ Zhat.T + RN, rhs)


def kalman_gain_bruteforce(Xf, H: np.ndarray, R: np.ndarray) -> np.ndarray:
    """K = P^f H^T (H P^f H^T + R)^{-1}  (Section 2.2) with the ensemble
    covariance P^f = A A^T/(N-1) of Section 2.3; inverse by np.linalg.inv."""
    A = state_anomalies(Xf)
    Pf = A @ A.T / (Xf.shape[1] - 1)
    return Pf @ H.T @ np.linalg.inv(H @ Pf @ H.T + R)


def enkf_bruteforce(Xf, idx, w, y, r, eps=None) -> np.ndarray:
    """X^a = X^f + K (y 1^T + E - H X^f) with the brute-force gain."""
    Xf = np.asarray(Xf, dtype=np.float64)
    H = dense_H(idx, w, Xf.shape[0])
    K = kalman_gain_bruteforce(Xf, H, np.diag(np.asarray(r, dtype=np.float64)))
    Y = np.outer(y, np.ones(Xf.shape[1]))
    if eps is not None:
        Y = Y + eps
    return Xf + K @ (Y - H @ Xf)


# ---------------------------------------------------------------------------
# Figure 2 / Section 3.1: the explicit-gain form, one CG per column of K^T
# ---------------------------------------------------------------------------
def enkf_gain_cg(Xf, idx, w, y, r, eps=None, tol: float = 1e-10, maxit: int = 10000,
                 record: bool = False) -> dict:
    """CGD-EnKF as Figure 2 draws it: Psi_z and Psi_x formed (Section 2.3),
    then for every column i of K^T the system Psi_z (K^T e_i) = Psi_x^T e_i
    (eqs. K_KF_T, K_KF_T_rewrite) by textbook CG from zero with the
    analysis's stop rule (||r|| <= tol ||b||, or maxit), K = (K^T)^T and
    X^a = X^f + K (Y - Z).  Returns Xa, KT (m x n), iters (n), and with
    `record` the CG iterates of every column."""
    Xf = np.asarray(Xf, dtype=np.float64)
    n = Xf.shape[0]
    S = obs_anomalies(idx, w, Xf)
    Psi = innovation_matrix(S, r)
    B = cross_covariance(state_anomalies(Xf), S).T
    KT = np.zeros((S.shape[0], n))
    its = np.zeros(n, dtype=np.int64)
    iterates = []
    for i in range(n):
        res = textbook_cg(matvec_dense(Psi), B[:, i], tol, maxit, record=record)
        KT[:, i] = res.z
        its[i] = res.it
        if record:
            iterates.append(res.iterates)
    D = innovations(idx, w, Xf, y, eps)
    out = {"Xa": Xf + KT.T @ D, "KT": KT, "iters": its, "Psi": Psi, "B": B}
    if record:
        out["iterates"] = iterates
    return out


def energy_errors(Psi: np.ndarray, b: np.ndarray, iterates) -> np.ndarray:
    """||x* - x_k||_Psi for each iterate x_k, x* = Psi^{-1} b by Cholesky: the
    CG error of Section 4 (eq. e_r_def) in the energy norm, one column."""
    xs = sla.cho_solve(sla.cho_factor(Psi), b)
    return np.array([np.sqrt(max(float((xs - x) @ Psi @ (xs - x)), 0.0)) for x in iterates])


# ---------------------------------------------------------------------------
# Algorithm 2 (EnKF-Reduced) and CGD-EnKF-Reduced (Section 5.2)
# ---------------------------------------------------------------------------
def enkf_reduced(Xf, idx, w, y, r, eps=None, solver: str = "direct", tol: float = 0.0,
                 maxit: int = 10000) -> dict:
    """X^a = X^f (I + P^T P)^{-1} [I + P^T L^{-1} Yhat] with R_N = (N-1) R = L L^T,
    P = L^{-1} Zhat, Yhat = (y - z-bar) 1^T (+ eps)  (Algorithm 2, eqs. LL-0..LL-2).
    For diagonal R, L = diag(sqrt((N-1) r)).  solver 'direct' solves the
    N x N system by Cholesky; 'cg' runs textbook CG per column of the
    right-hand side starting from W = 0 (CGD-EnKF-Reduced)."""
    Xf = np.asarray(Xf, dtype=np.float64)
    N = Xf.shape[1]
    Zp = observe(idx, w, Xf)
    zbar = Zp.mean(axis=1)
    Zhat = Zp - zbar[:, None]
    Ldiag = np.sqrt((N - 1) * np.asarray(r, dtype=np.float64))
    P = Zhat / Ldiag[:, None]
    Yhat = np.outer(np.asarray(y) - zbar, np.ones(N))
    if eps is not None:
        Yhat = Yhat + eps
    G = np.eye(N) + P.T @ P
    G = 0.5 * (G + G.T)
    B = np.eye(N) + P.T @ (Yhat / Ldiag[:, None])
    if solver == "direct":
        W = sla.cho_solve(sla.cho_factor(G, lower=True), B)
        its = np.zeros(N, dtype=np.int64)
    elif solver == "cg":
        W, its, _ = solve_cg_columns(matvec_dense(G), B, tol, maxit)
    else:
        raise ValueError(solver)
    return {"Xa": Xf @ W, "W": W, "G": G, "B": B, "P": P, "iters": its}


def senkf(Xf, idx, w, y, r, eps=None) -> np.ndarray:
    """Simultaneous serial-EnKF form (Appendix A, Algorithm 3): the inverse of
    Algorithm 1 replaced by the inverse of its diagonal."""
    Xf = np.asarray(Xf, dtype=np.float64)
    N = Xf.shape[1]
    Zp = observe(idx, w, Xf)
    zbar = Zp.mean(axis=1)
    Zhat = Zp - zbar[:, None]
    diag = (Zhat ** 2).sum(axis=1) + (N - 1) * np.asarray(r, dtype=np.float64)
    Y = np.outer(y, np.ones(N))
    if eps is not None:
        Y = Y + eps
    return Xf + Xf @ Zhat.T @ ((Y - Zp) / diag[:, None])


# ---------------------------------------------------------------------------
# Diagnostics
# ---------------------------------------------------------------------------
def true_relres(S, r, Z, D) -> np.ndarray:
    """Per column ||d_j - Psi z_j|| / ||d_j|| with Psi applied matrix-free in FP64."""
    S = np.asarray(S, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    res = D - matvec_free(S, r)(Z)
    dn = np.linalg.norm(D, axis=0)
    return np.linalg.norm(res, axis=0) / np.where(dn > 0, dn, 1.0)


# ---------------------------------------------------------------------------
# Non-diagonal R (Section 5.1: R = L L^T with a sparse lower-triangular L;
# Section 5.3 and Example 2: symmetric tridiagonal Toeplitz R, bidiagonal L)
# ---------------------------------------------------------------------------
def tridiag_R(r_diag, r_off) -> np.ndarray:
    """Dense symmetric tridiagonal R: R_ii = r_diag[i], R_{i,i+1} = R_{i+1,i} = r_off[i]."""
    r_diag = np.asarray(r_diag, dtype=np.float64)
    r_off = np.asarray(r_off, dtype=np.float64)
    return np.diag(r_diag) + np.diag(r_off, 1) + np.diag(r_off, -1)


def tridiag_toeplitz_R(m: int, sigma: float, rho: float):
    """Example 2's observation covariance: sigma^2 on the diagonal, sigma^2 rho
    next to it; returns (r_diag, r_off)."""
    return np.full(m, sigma * sigma), np.full(m - 1, sigma * sigma * rho)


def innovation_matrix_R(S: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Psi_z = S S^T/(N-1) + R for a dense (symmetric) R (eq. Psi_zz)."""
    N = S.shape[1]
    Psi = S @ S.T / (N - 1) + np.asarray(R, dtype=np.float64)
    return 0.5 * (Psi + Psi.T)


def matvec_free_R(S: np.ndarray, R: np.ndarray) -> Callable[[np.ndarray], np.ndarray]:
    """Psi v = S (S^T v)/(N-1) + R v (Section 3.3's three stages; stage 3 with
    the given R)."""
    N = S.shape[1]
    R = np.asarray(R, dtype=np.float64)
    return lambda v: S @ (S.T @ v) / (N - 1) + R @ v


def textbook_pcg_op(matvec, prec_solve, d: np.ndarray, tol: float, maxit: int,
                    z0: Optional[np.ndarray] = None, fallback_on_stall: bool = False,
                    record: bool = False) -> CGResult:
    """textbook_pcg with the preconditioner given as an operator s = M^{-1} r
    (prec_solve), for a non-diagonal M = R: the same steps, norms and rules."""
    d = np.asarray(d, dtype=np.float64)
    nrm = lambda v: np.sqrt(float(v @ prec_solve(v)))
    dnorm = nrm(d)
    fallback = False
    warm = z0 is not None
    if warm:
        z = np.array(z0, dtype=np.float64)
        r = d - matvec(z)
        if fallback_on_stall and nrm(r) > dnorm:
            z = np.zeros_like(d)
            r = d.copy()
            fallback, warm = True, False
    else:
        z = np.zeros_like(d)
        r = d.copy()
    s = prec_solve(r)
    p = s.copy()
    delta = float(r @ s)
    hist = [np.sqrt(delta)]
    iterates = [z.copy()] if record else []
    it = 0
    while np.sqrt(delta) > tol * dnorm and it < maxit and delta > 0.0:
        if (fallback_on_stall and warm and len(hist) > STALL_WINDOW
                and hist[-1] > STALL_FACTOR * hist[-1 - STALL_WINDOW]):
            z = np.zeros_like(d)
            r = d.copy()
            s = prec_solve(r)
            p = s.copy()
            delta = float(r @ s)
            fallback, warm = True, False
            continue
        q = matvec(p)
        alpha = delta / float(p @ q)
        z = z + alpha * p
        r = r - alpha * q
        s = prec_solve(r)
        delta_new = float(r @ s)
        it += 1
        hist.append(np.sqrt(delta_new))
        if record:
            iterates.append(z.copy())
        p = s + (delta_new / delta) * p
        delta = delta_new
    return CGResult(z, it, hist, iterates, fallback)


def enkf_analysis_R(Xf, idx, w, y, R, eps=None, solver: str = "cholesky", tol: float = 1e-10,
                    maxit: int = 10000, Z0=None, fallback_on_stall: bool = False) -> dict:
    """One EnKF analysis with a dense observation covariance R.  solver:
    'cholesky' (formed Psi), 'cg' (textbook CG, the product with R applied
    as a matrix), 'pcg' (textbook PCG with M = R, M^{-1} by a Cholesky
    factorisation of R: the stop rule in the R^{-1}-norm)."""
    S = obs_anomalies(idx, w, Xf)
    D = innovations(idx, w, Xf, y, eps)
    R = np.asarray(R, dtype=np.float64)
    out = {"S": S, "D": D}
    if solver == "cholesky":
        Z = solve_cholesky(innovation_matrix_R(S, R), D)
        its = np.zeros(D.shape[1], dtype=np.int64)
    elif solver in ("cg", "pcg"):
        mv = matvec_free_R(S, R)
        if solver == "cg":
            cols = [textbook_cg(mv, D[:, j], tol, maxit, None if Z0 is None else Z0[:, j],
                                fallback_on_stall) for j in range(D.shape[1])]
        else:
            cf = sla.cho_factor(R, lower=True)
            pre = lambda v: sla.cho_solve(cf, v)
            cols = [textbook_pcg_op(mv, pre, D[:, j], tol, maxit,
                                    None if Z0 is None else Z0[:, j], fallback_on_stall)
                    for j in range(D.shape[1])]
        Z = np.stack([c.z for c in cols], axis=1)
        its = np.array([c.it for c in cols], dtype=np.int64)
        out["fallbacks"] = np.array([c.fallback for c in cols])
    else:
        raise ValueError(solver)
    out["Z"] = Z
    out["iters"] = its
    out["Xa"] = analysis_update(Xf, S, Z)
    return out


def enkf_reduced_R(Xf, idx, w, y, R, eps=None, solver: str = "direct", tol: float = 0.0,
                   maxit: int = 10000) -> dict:
    """Algorithm 2 with a dense R: R_N = (N-1) R = L L^T (Cholesky), P = L^{-1} Zhat,
    Yhat = (y - z-bar) 1^T (+ eps), X^a = X^f (I + P^T P)^{-1} [I + P^T L^{-1} Yhat];
    'direct' solves the N x N system by Cholesky, 'cg' by textbook CG per column
    from W = 0 (CGD-EnKF-Reduced)."""
    Xf = np.asarray(Xf, dtype=np.float64)
    N = Xf.shape[1]
    Zp = observe(idx, w, Xf)
    zbar = Zp.mean(axis=1)
    Zhat = Zp - zbar[:, None]
    L = np.linalg.cholesky((N - 1) * np.asarray(R, dtype=np.float64))
    P = sla.solve_triangular(L, Zhat, lower=True)
    Yhat = np.outer(np.asarray(y) - zbar, np.ones(N))
    if eps is not None:
        Yhat = Yhat + eps
    G = np.eye(N) + P.T @ P
    G = 0.5 * (G + G.T)
    B = np.eye(N) + P.T @ sla.solve_triangular(L, Yhat, lower=True)
    if solver == "direct":
        W = sla.cho_solve(sla.cho_factor(G, lower=True), B)
        its = np.zeros(N, dtype=np.int64)
    elif solver == "cg":
        W, its, _ = solve_cg_columns(matvec_dense(G), B, tol, maxit)
    else:
        raise ValueError(solver)
    return {"Xa": Xf @ W, "W": W, "G": G, "B": B, "P": P, "iters": its}


def true_relres_rinv(S, r, Z, D) -> np.ndarray:
    """Per column ||d_j - Psi z_j||_{R^{-1}} / ||d_j||_{R^{-1}}, the norm of the
    diag(R)-preconditioned stop rule (||v||_{R^{-1}} = sqrt(v^T R^{-1} v))."""
    S = np.asarray(S, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    w = 1.0 / np.sqrt(np.asarray(r, dtype=np.float64))
    res = (D - matvec_free(S, r)(Z)) * w[:, None]
    dn = np.linalg.norm(D * w[:, None], axis=0)
    return np.linalg.norm(res, axis=0) / np.where(dn > 0, dn, 1.0)


def rel_frob(X, Xref) -> float:
    """Relative Frobenius error (eq. rel_frob)."""
    Xref = np.asarray(Xref, dtype=np.float64)
    den = np.linalg.norm(Xref)
    return float(np.linalg.norm(np.asarray(X, dtype=np.float64) - Xref) / (den if den > 0 else 1.0))
