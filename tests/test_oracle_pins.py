"""Pins for the FP64 oracle against facts the paper and the mathematics fix.

None of these re-types the oracle's formula: each compares it with an
independent route (brute-force gain, exact rational arithmetic, Krylov
optimality, SciPy's CG, closed forms, invariants, the paper's theorems).
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W


def _problem(n=30, m=12, N=7, k=2, seed=0, stochastic=True, r_lo=0.5, r_hi=2.0):
    return W.random_problem(n, m, N, k, seed=seed, stochastic=stochastic, r_lo=r_lo, r_hi=r_hi)


def _args(p):
    return p.Xf, p.idx, p.w, p.y, p.r, p.eps


# --------------------------------------------------------------------------
# P1: brute-force Kalman gain (Section 2.2 with the ensemble covariance) vs
# the innovation-system form (Section 2.3 / Algorithm 1)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed,n,m,N,k", [(0, 30, 12, 7, 2), (1, 50, 60, 9, 1), (2, 40, 20, 20, 4),
                                          (3, 12, 3, 2, 1)])
@pytest.mark.parametrize("stochastic", [False, True])
def test_bruteforce_gain_matches_innovation_form(seed, n, m, N, k, stochastic):
    p = _problem(n, m, N, k, seed, stochastic)
    ref = O.enkf_bruteforce(*_args(p))
    got = O.enkf_analysis(*_args(p), solver="cholesky")["Xa"]
    assert O.rel_frob(got, ref) < 1e-12


def test_bruteforce_config1():
    p = W.config1()
    ref = O.enkf_bruteforce(*_args(p))
    assert O.rel_frob(O.enkf_analysis(*_args(p))["Xa"], ref) < 1e-12
    assert O.rel_frob(O.alg1_exact(*_args(p)), ref) < 1e-12


# --------------------------------------------------------------------------
# Exact rational arithmetic on a tiny hand-sized problem: an independent
# re-derivation of X^a = X^f + P H^T (H P H^T + R)^{-1} (Y - H X^f) with
# Fractions and Gauss-Jordan inversion.
# --------------------------------------------------------------------------
def _frac_inv(M):
    n = len(M)
    a = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(M)]
    for c in range(n):
        piv = next(r for r in range(c, n) if a[r][c] != 0)
        a[c], a[piv] = a[piv], a[c]
        f = a[c][c]
        a[c] = [v / f for v in a[c]]
        for r in range(n):
            if r != c and a[r][c] != 0:
                g = a[r][c]
                a[r] = [vr - g * vc for vr, vc in zip(a[r], a[c])]
    return [row[n:] for row in a]


def _mm(A, B):
    return [[sum(A[i][t] * B[t][j] for t in range(len(B))) for j in range(len(B[0]))] for i in range(len(A))]


def _tr(A):
    return [list(c) for c in zip(*A)]


def test_exact_rational_tiny():
    # n = 3 states, N = 3 members, m = 2 observations (one of them a weighted pair)
    X = [[Fraction(v) for v in row] for row in ([1, 3, -2], [0, 2, 5], [4, -1, 1])]
    idx = np.array([[0, 2], [1, 1]], dtype=np.int32)
    w = [[Fraction(1, 2), Fraction(3, 2)], [Fraction(1), Fraction(0)]]
    r = [Fraction(1, 4), Fraction(2)]
    y = [Fraction(3), Fraction(-1)]
    E = [[Fraction(1, 8), Fraction(-1, 3), Fraction(0)], [Fraction(1, 2), Fraction(0), Fraction(-1)]]
    n, N, m = 3, 3, 2
    H = [[Fraction(0)] * n for _ in range(m)]
    for i in range(m):
        for t in range(2):
            H[i][int(idx[i, t])] += w[i][t]
    mean = [sum(row) / N for row in X]
    A = [[X[i][j] - mean[i] for j in range(N)] for i in range(n)]
    P = [[v / (N - 1) for v in row] for row in _mm(A, _tr(A))]
    Sinn = _mm(_mm(H, P), _tr(H))
    for i in range(m):
        Sinn[i][i] += r[i]
    K = _mm(_mm(P, _tr(H)), _frac_inv(Sinn))
    HX = _mm(H, X)
    Dm = [[y[i] + E[i][j] - HX[i][j] for j in range(N)] for i in range(m)]
    Xa = [[X[i][j] + v for j, v in enumerate(row)] for i, row in enumerate(_mm(K, Dm))]
    exact = np.array([[float(v) for v in row] for row in Xa])

    Xf = np.array([[float(v) for v in row] for row in X])
    wf = np.array([[float(v) for v in row] for row in w])
    got = O.enkf_analysis(Xf, idx, wf, np.array([3.0, -1.0]), np.array([0.25, 2.0]),
                          np.array([[float(v) for v in row] for row in E]))["Xa"]
    assert np.max(np.abs(got - exact)) < 1e-13
    red = O.enkf_reduced(Xf, idx, wf, np.array([3.0, -1.0]), np.array([0.25, 2.0]),
                         np.array([[float(v) for v in row] for row in E]))["Xa"]
    assert np.max(np.abs(red - exact)) < 1e-13


# --------------------------------------------------------------------------
# P2: Algorithm 2 (Reduced, via the Woodbury identity) equals Algorithm 1
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed,n,m,N,k", [(4, 40, 30, 6, 1), (5, 60, 10, 16, 2), (6, 40, 20, 20, 1)])
@pytest.mark.parametrize("stochastic", [False, True])
def test_reduced_equals_full(seed, n, m, N, k, stochastic):
    p = _problem(n, m, N, k, seed, stochastic)
    full = O.alg1_exact(*_args(p))
    red = O.enkf_reduced(*_args(p))
    assert O.rel_frob(red["Xa"], full) < 1e-12
    # CGD-EnKF-Reduced converges to the direct reduced result
    redcg = O.enkf_reduced(*_args(p), solver="cg", tol=1e-14, maxit=200)
    assert O.rel_frob(redcg["Xa"], full) < 1e-11
    assert np.all(redcg["iters"] <= N)


# --------------------------------------------------------------------------
# P3 / Prop. 2: CG -> Cholesky as the tolerance goes to zero
# --------------------------------------------------------------------------
def test_cg_converges_to_cholesky_config1():
    p = W.config1()
    chol = O.enkf_analysis(*_args(p), solver="cholesky")
    errs = []
    for tol in (1e-2, 1e-4, 1e-6, 1e-10):
        cg = O.enkf_analysis(*_args(p), solver="cg", tol=tol)
        errs.append(O.rel_frob(cg["Xa"], chol["Xa"]))
    assert errs[-1] < 1e-10
    assert all(a >= b for a, b in zip(errs, errs[1:]))
    free = O.enkf_analysis(*_args(p), solver="cg_free", tol=1e-10)
    assert O.rel_frob(free["Xa"], chol["Xa"]) < 1e-10
    assert 5 <= free["iters"].max() <= 20


# --------------------------------------------------------------------------
# Textbook CG vs independent routes: Krylov optimality and SciPy's CG
# --------------------------------------------------------------------------
def test_cg_iterates_are_krylov_minimisers():
    p = _problem(40, 25, 10, 1, seed=7)
    S = O.obs_anomalies(p.idx, p.w, p.Xf)
    Psi = O.innovation_matrix(S, p.r)
    d = O.innovations(p.idx, p.w, p.Xf, p.y, p.eps)[:, 3]
    res = O.textbook_cg(O.matvec_dense(Psi), d, 0.0, 6, record=True)
    for k in range(1, 7):
        V = np.stack([np.linalg.matrix_power(Psi, t) @ d for t in range(k)], 1)
        V, _ = np.linalg.qr(V)
        zk = V @ np.linalg.solve(V.T @ Psi @ V, V.T @ d)
        assert np.linalg.norm(res.iterates[k] - zk) <= 1e-9 * np.linalg.norm(zk)


def test_cg_iterates_match_scipy():
    p = _problem(40, 25, 10, 2, seed=8)
    S = O.obs_anomalies(p.idx, p.w, p.Xf)
    Psi = O.innovation_matrix(S, p.r)
    d = O.innovations(p.idx, p.w, p.Xf, p.y, p.eps)[:, 0]
    seen = []
    spla.cg(Psi, d, rtol=1e-300, atol=0.0, maxiter=8, callback=lambda xk: seen.append(xk.copy()))
    ours = O.textbook_cg(O.matvec_dense(Psi), d, 0.0, 8, record=True).iterates[1:]
    assert len(seen) >= 8
    for a, b in zip(ours, seen):
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


# --------------------------------------------------------------------------
# P4: exact termination (<= m always; <= N for scalar R, Lemma 1 sharpened)
# --------------------------------------------------------------------------
def test_exact_termination_scalar_R():
    p = W.random_problem(800, 400, 8, 1, seed=9, r_lo=1.0, r_hi=1.0)
    out = O.enkf_analysis(*_args(p), solver="cg_free", tol=1e-10)
    assert out["iters"].max() <= p.N
    chol = O.enkf_analysis(*_args(p))
    assert O.rel_frob(out["Xa"], chol["Xa"]) < 1e-10


def test_exact_termination_general_R():
    p = _problem(40, 10, 30, 1, seed=10)
    out = O.enkf_analysis(*_args(p), solver="cg", tol=1e-12)
    assert out["iters"].max() <= p.m + 1


def test_lemma1_full_space_identity_plus_low_rank():
    # (I + P P^T) v = g on the m x m space needs at most N CG steps (Lemma 1)
    rng = np.random.default_rng(11)
    m, N = 200, 10
    P = rng.standard_normal((m, N))
    P -= P.mean(axis=1, keepdims=True)
    M = np.eye(m) + P @ P.T
    g = rng.standard_normal(m)
    res = O.textbook_cg(O.matvec_dense(M), g, 1e-11, 1000)
    assert res.it <= N
    assert np.linalg.norm(M @ res.z - g) <= 1e-10 * np.linalg.norm(g)


# --------------------------------------------------------------------------
# P5 / P8: structure of Psi
# --------------------------------------------------------------------------
def test_psi_spd_and_spectrum():
    p = _problem(50, 30, 8, 2, seed=12)
    S = O.obs_anomalies(p.idx, p.w, p.Xf)
    Psi = O.innovation_matrix(S, p.r)
    assert np.array_equal(Psi, Psi.T)
    ev = np.linalg.eigvalsh(Psi)
    assert ev.min() >= p.r.min() * (1 - 1e-12)
    # R = I: eigenvalue 1 with multiplicity m - (N - 1), N - 1 outliers above it
    q = W.random_problem(50, 30, 8, 2, seed=12, r_lo=1.0, r_hi=1.0)
    ev = np.linalg.eigvalsh(O.innovation_matrix(O.obs_anomalies(q.idx, q.w, q.Xf), q.r))
    ones = np.abs(ev - 1.0) < 1e-12
    assert ones.sum() == 30 - (8 - 1)
    assert np.all(ev[~ones] > 1.0)


# --------------------------------------------------------------------------
# P6: centring identities: S 1 = 0, 1^T W = 0, X^f W = A W
# --------------------------------------------------------------------------
def test_centring_identities():
    p = W.config1()
    out = O.enkf_analysis(*_args(p))
    S, Z = out["S"], out["Z"]
    assert np.abs(S.sum(axis=1)).max() < 1e-12 * np.abs(S).max() * p.N
    Wm = S.T @ Z / (p.N - 1)
    assert np.abs(Wm.sum(axis=0)).max() < 1e-12 * np.abs(Wm).max() * p.N
    A = O.state_anomalies(p.Xf)
    assert O.rel_frob(p.Xf @ Wm, A @ Wm) < 1e-12


# --------------------------------------------------------------------------
# P7: Proposition 1 (classical CG bound, per column, Psi-norm)
# P8: Proposition 3 (outlier form), read per column (Section 4)
# --------------------------------------------------------------------------
def _psi_norm(Psi, e):
    return float(np.sqrt(e @ Psi @ e))


def test_prop1_bound():
    p = _problem(60, 40, 12, 1, seed=13)
    S = O.obs_anomalies(p.idx, p.w, p.Xf)
    Psi = O.innovation_matrix(S, p.r)
    D = O.innovations(p.idx, p.w, p.Xf, p.y, p.eps)
    ev = np.linalg.eigvalsh(Psi)
    kappa = ev[-1] / ev[0]
    rho = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    for j in range(D.shape[1]):
        zs = np.linalg.solve(Psi, D[:, j])
        res = O.textbook_cg(O.matvec_dense(Psi), D[:, j], 0.0, 15, record=True)
        e0 = _psi_norm(Psi, zs)
        for k, zk in enumerate(res.iterates):
            assert _psi_norm(Psi, zs - zk) <= 2 * rho ** k * e0 * (1 + 1e-9) + 1e-13


def test_prop3_outlier_bound():
    # diag R in [0.9, 1.1]: the bulk cluster sits near 1, the N-1 ensemble
    # directions are outliers; bound 2 C rho_eff^(r-l) for r >= l
    p = W.random_problem(300, 120, 6, 1, seed=14, r_lo=0.9, r_hi=1.1, spread=2.0)
    S = O.obs_anomalies(p.idx, p.w, p.Xf)
    Psi = O.innovation_matrix(S, p.r)
    ev = np.linalg.eigvalsh(Psi)
    lam_a, lam_b = ev[0], p.r.max() + 1e-12
    bulk = ev[ev <= lam_b]
    lam_b = bulk.max()
    outl = ev[ev > lam_b]
    l = outl.size
    C = max(np.prod(np.abs(1 - lam / outl)) for lam in bulk)
    keff = lam_b / lam_a
    rho_eff = (np.sqrt(keff) - 1) / (np.sqrt(keff) + 1)
    d = O.innovations(p.idx, p.w, p.Xf, p.y, p.eps)[:, 0]
    zs = np.linalg.solve(Psi, d)
    res = O.textbook_cg(O.matvec_dense(Psi), d, 0.0, l + 6, record=True)
    e0 = _psi_norm(Psi, zs)
    for r in range(l, len(res.iterates)):
        assert _psi_norm(Psi, zs - res.iterates[r]) <= 2 * C * rho_eff ** (r - l) * e0 * (1 + 1e-6) + 1e-12


# --------------------------------------------------------------------------
# P9: deterministic form updates the mean by the Kalman formula and the
# anomalies by (I - K H)
# --------------------------------------------------------------------------
def test_mean_and_anomaly_update():
    p = _problem(30, 12, 9, 2, seed=15, stochastic=False)
    Xa = O.enkf_analysis(*_args(p))["Xa"]
    H = O.dense_H(p.idx, p.w, p.n)
    K = O.kalman_gain_bruteforce(p.Xf, H, np.diag(p.r))
    xf = p.Xf.mean(1)
    assert np.allclose(Xa.mean(1), xf + K @ (p.y - H @ xf), atol=1e-12, rtol=0)
    Af = O.state_anomalies(p.Xf)
    assert np.allclose(O.state_anomalies(Xa), (np.eye(p.n) - K @ H) @ Af, atol=1e-12, rtol=0)


# --------------------------------------------------------------------------
# P10: special cases
# --------------------------------------------------------------------------
def test_scalar_observation_one_cg_step_and_senkf():
    p = _problem(20, 1, 6, 3, seed=16)
    out = O.enkf_analysis(*_args(p), solver="cg", tol=1e-14)
    assert out["iters"].max() == 1
    chol = O.enkf_analysis(*_args(p))
    assert O.rel_frob(out["Xa"], chol["Xa"]) < 1e-14
    # with one observation the diagonal of Psi is Psi: sEnKF is exact (Appendix A)
    assert O.rel_frob(O.senkf(*_args(p)), chol["Xa"]) < 1e-13


def test_identity_H_scalar_R_closed_form():
    rng = np.random.default_rng(17)
    n, N, s2 = 25, 7, 0.3
    Xf = rng.standard_normal((n, N))
    idx, w = W.identity_obs(n)
    y = rng.standard_normal(n)
    r = np.full(n, s2)
    out = O.enkf_analysis(Xf, idx, w, y, r)
    A = Xf - Xf.mean(1, keepdims=True)
    U, sv, _ = np.linalg.svd(A, full_matrices=False)
    D = y[:, None] - Xf
    Z = U @ ((U.T @ D) / (sv[:, None] ** 2 / (N - 1) + s2)) + (D - U @ (U.T @ D)) / s2
    assert np.max(np.abs(out["Z"] - Z)) < 1e-10 * np.abs(Z).max()


# --------------------------------------------------------------------------
# P11: invariances
# --------------------------------------------------------------------------
def test_member_and_observation_permutation_and_linearity():
    p = _problem(30, 15, 8, 2, seed=18)
    base = O.enkf_analysis(*_args(p))
    perm = np.random.default_rng(0).permutation(p.N)
    out = O.enkf_analysis(p.Xf[:, perm], p.idx, p.w, p.y, p.r, p.eps[:, perm])
    assert O.rel_frob(out["Xa"], base["Xa"][:, perm]) < 1e-13
    op = np.random.default_rng(1).permutation(p.m)
    out = O.enkf_analysis(p.Xf, p.idx[op], p.w[op], p.y[op], p.r[op], p.eps[op])
    assert O.rel_frob(out["Xa"], base["Xa"]) < 1e-12
    S = O.obs_anomalies(p.idx, p.w, p.Xf)
    mv = O.matvec_free(S, p.r)
    d = base["D"][:, 2]
    z1 = O.textbook_cg(mv, d, 1e-12, 500).z
    z2 = O.textbook_cg(mv, 3.5 * d, 1e-12, 500).z
    assert np.linalg.norm(z2 - 3.5 * z1) <= 1e-10 * np.linalg.norm(z2)


def test_degenerate_zero_innovation_column():
    p = _problem(20, 8, 5, 1, seed=19, stochastic=False)
    S = O.obs_anomalies(p.idx, p.w, p.Xf)
    res = O.textbook_cg(O.matvec_free(S, p.r), np.zeros(p.m), 1e-10, 100)
    assert res.it == 0 and not res.z.any()


# --------------------------------------------------------------------------
# Warm start and the stall fallback
# --------------------------------------------------------------------------
def test_fallback_restarts_bad_warm_start():
    p = _problem(40, 25, 10, 1, seed=20)
    S = O.obs_anomalies(p.idx, p.w, p.Xf)
    mv = O.matvec_free(S, p.r)
    D = O.innovations(p.idx, p.w, p.Xf, p.y, p.eps)
    zs = O.solve_cholesky(O.innovation_matrix(S, p.r), D)
    cold = O.solve_cg_columns(mv, D, 1e-10, 500)[0]
    Zw, its, cols = O.solve_cg_columns(mv, D, 1e-10, 500, Z0=-10 * zs, fallback_on_stall=True)
    assert all(c.fallback for c in cols)
    assert np.max(np.abs(Zw - cold)) <= 1e-12 * np.abs(cold).max()
    # a good warm start converges in fewer iterations and never falls back
    Zg, itg, colg = O.solve_cg_columns(mv, D, 1e-10, 500, Z0=zs + 1e-6 * cold, fallback_on_stall=True)
    assert not any(c.fallback for c in colg)
    assert np.max(np.abs(Zg - zs)) <= 1e-8 * np.abs(zs).max()
