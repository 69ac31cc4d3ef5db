"""Pins for the oracle's sEnKF (Section 2.4, Figure 1, Appendix A
Algorithm 3) against routes other than its own matrix formula.

* The per-observation form of Section 2.4: gain vectors psi_{j,x} / psi_{j,z},
  each from the same X^f, added one observation at a time, in plain loops.
* Where Zhat Zhat^T is diagonal (orthogonal observed anomalies) the
  diagonal of Psi is Psi, so the sEnKF is the exact EnKF (brute-force gain).
* One observation: the same, trivially (test_oracle_pins.py covers it too).
* Large R: the gains vanish and X^a tends to X^f at the rate 1/r.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _serial_gain_loops(Xf, idx, w, y, r, eps):
    """Section 2.4 written out: for every observation component j the gain
    vector K e_j = psi_{j,x} / psi_{j,z} with
        psi_{j,x} = 1/(N-1) sum_i (x_i - xbar)(z_{j,i} - zbar_j),
        psi_{j,z} = 1/(N-1) sum_i (z_{j,i} - zbar_j)^2 + R_jj,
    all from the same X^f, and X^a = X^f + sum_j (K e_j)(Y - Z)_{j,:}."""
    n, N = len(Xf), len(Xf[0])
    m, k = len(idx), len(idx[0])
    Z = [[sum(w[j][t] * Xf[idx[j][t]][i] for t in range(k)) for i in range(N)] for j in range(m)]
    xbar = [sum(Xf[a][i] for i in range(N)) / N for a in range(n)]
    Xa = [[Xf[a][i] for i in range(N)] for a in range(n)]
    for j in range(m):
        zbar = sum(Z[j]) / N
        psi_z = sum((Z[j][i] - zbar) ** 2 for i in range(N)) / (N - 1) + r[j]
        psi_x = [sum((Xf[a][i] - xbar[a]) * (Z[j][i] - zbar) for i in range(N)) / (N - 1)
                 for a in range(n)]
        innov = [y[j] + (eps[j][i] if eps is not None else 0.0) - Z[j][i] for i in range(N)]
        for a in range(n):
            g = psi_x[a] / psi_z
            for i in range(N):
                Xa[a][i] += g * innov[i]
    return np.array(Xa)


@pytest.mark.parametrize("seed,n,m,N,k,stochastic", [(0, 9, 6, 5, 2, True), (1, 7, 11, 4, 1, False),
                                                     (2, 12, 3, 8, 3, True)])
def test_senkf_matches_per_observation_gains(seed, n, m, N, k, stochastic):
    p = W.random_problem(n, m, N, k, seed=seed, stochastic=stochastic, duplicate_idx=True)
    ref = _serial_gain_loops(p.Xf.tolist(), p.idx.tolist(), p.w.tolist(), p.y.tolist(),
                             p.r.tolist(), None if p.eps is None else p.eps.tolist())
    assert O.rel_frob(O.senkf(p.Xf, p.idx, p.w, p.y, p.r, p.eps), ref) < 1e-13


def _orthogonal_anomaly_problem(n, m, N, seed):
    """H picks state rows 0..m-1 (k = 1, weight 1), whose anomalies are
    mutually orthogonal (m <= N - 1): Zhat Zhat^T is diagonal."""
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((N, m))
    U -= U.mean(axis=0)                      # orthogonal to the ones vector
    Q, _ = np.linalg.qr(U)                   # orthonormal columns, still centred
    Xf = rng.standard_normal((n, N))
    Xf[:m] = rng.standard_normal(m)[:, None] + rng.uniform(0.5, 3.0, m)[:, None] * Q.T
    idx = np.arange(m, dtype=np.int32)[:, None]
    w = np.ones((m, 1))
    r = rng.uniform(0.2, 2.0, m)
    y = rng.standard_normal(m)
    eps = np.sqrt(r)[:, None] * rng.standard_normal((m, N))
    return Xf, idx, w, y, r, eps


@pytest.mark.parametrize("n,m,N,seed", [(20, 5, 8, 3), (40, 15, 16, 4), (10, 1, 2, 5)])
def test_senkf_is_exact_when_observed_anomalies_are_orthogonal(n, m, N, seed):
    args = _orthogonal_anomaly_problem(n, m, N, seed)
    Xf, idx, w, y, r, eps = args
    S = O.obs_anomalies(idx, w, Xf)
    off = S @ S.T - np.diag(np.diag(S @ S.T))
    assert np.abs(off).max() < 1e-12          # the construction holds
    assert O.rel_frob(O.senkf(*args), O.enkf_bruteforce(*args)) < 1e-12


def test_senkf_differs_from_enkf_with_correlated_anomalies():
    """Not the exact EnKF in general (the diagonal approximation is real)."""
    p = W.random_problem(30, 12, 7, 2, seed=9)
    a = O.senkf(p.Xf, p.idx, p.w, p.y, p.r, p.eps)
    b = O.enkf_bruteforce(p.Xf, p.idx, p.w, p.y, p.r, p.eps)
    assert O.rel_frob(a, b) > 1e-3


def test_senkf_large_r_limit():
    """Gains ~ 1/r: X^a - X^f shrinks in proportion to 1/r."""
    p = W.random_problem(25, 10, 6, 2, seed=11, stochastic=False)
    d = []
    for scale in (1e6, 1e7):
        Xa = O.senkf(p.Xf, p.idx, p.w, p.y, p.r * scale, None)
        d.append(np.linalg.norm(Xa - p.Xf))
    assert d[1] < d[0]
    assert abs(d[0] / d[1] - 10.0) < 1e-3
