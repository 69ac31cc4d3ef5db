"""The explicit-gain form of Figure 2 on the GPU (cgd_enkf_gain_analysis:
one CG per column of K^T) against the oracle's enkf_gain_cg, and the CG
error study of Example 1b (Section 6.1) from the GPU's own records.

Bars: FP64 X_a and K^T to 1e-10 of the oracle's at tol 1e-12 (iteration
counts within max(2, 5%)); FP32 X_a to 1e-4 of the oracle's EnKF at tol 1e-6
on the same FP32-rounded inputs.  The per-step records alpha_t ||r_t||^2 are
checked against the oracle's energy-norm errors of its own iterates
(Hestenes-Stiefel: their tail sums are ||e_t||^2_Psi).  Shapes: every padded
width (16, 32, 64, 128), n and m not multiples of 16 or of the 128-row
padding, m < N, N = 2.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import assert_iters_close, dev_problem, rel, rounded, say

pytestmark = pytest.mark.gpu

SHAPES = [
    # n, m, N, k
    (37, 50, 10, 2),
    (130, 257, 20, 3),
    (200, 91, 50, 1),
    (64, 300, 100, 2),
    (50, 5, 8, 1),
    (30, 40, 2, 1),
    (40, 70, 128, 2),
]


def _run(lib, p, prec, tol, maxit, **kw):
    out = lib.gain_analysis(**dev_problem(p, prec), tol=tol, maxit=maxit, prec=prec, **kw)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("n,m,N,k", SHAPES)
def test_gain_fp64_against_oracle(lib, n, m, N, k):
    p = W.random_problem(n, m, N, k, seed=3 * n + m + N)
    say(f"case: gain fp64 n={n} m={m} N={N} k={k}")
    out = _run(lib, p, "fp64", 1e-12, 2000, want_kt=True, want_iters=True)
    ref = O.enkf_gain_cg(p.Xf, p.idx, p.w, p.y, p.r, p.eps, tol=1e-12, maxit=2000)
    assert out["status"] == 0 and out["stats"]["n_converged"] == n
    assert rel(out["Xa"].cpu().numpy(), ref["Xa"]) <= 1e-10
    assert rel(out["KT"].cpu().numpy(), ref["KT"]) <= 1e-10
    assert_iters_close(out["iters"].cpu().numpy(), ref["iters"])


@pytest.mark.parametrize("n,m,N,k", SHAPES[:4])
def test_gain_fp32(lib, n, m, N, k):
    p = W.random_problem(n, m, N, k, seed=3 * n + m + N + 1)
    say(f"case: gain fp32 n={n} m={m} N={N} k={k}")
    out = _run(lib, p, "fp32", 1e-6, 2000)
    q = rounded(p)
    ref = O.enkf_analysis(q.Xf, q.idx, q.w, q.y, q.r, q.eps)["Xa"]
    assert out["status"] == 0
    assert rel(out["Xa"].double().cpu().numpy(), ref) <= 1e-4


def test_gain_matches_member_form_at_convergence(lib):
    """Proposition 2: converged, the explicit-gain form and Algorithm 1's
    N-column form give the same X_a (the Lorenz-96 twin analysis, n = 4096,
    m = 2048, N = 64, FP64)."""
    p = W.L96Cycler().step(lambda q: q.Xf)
    a = dev_problem(p, "fp64")
    say("case: gain vs member form, config 2 fp64")
    g = lib.gain_analysis(**a, tol=1e-11, maxit=2000, prec="fp64")
    f = lib.analysis(**a, tol=1e-11, maxit=2000, prec="fp64")
    torch.cuda.synchronize()
    assert g["status"] == 0 and f["status"] == 0
    assert rel(g["Xa"].cpu().numpy(), f["Xa"].cpu().numpy()) <= 1e-9


def test_energy_records_match_oracle_errors(lib):
    """The records' tail sums are the squared energy-norm errors of the
    iterates, which the oracle computes from its own CG iterates and a
    Cholesky solve."""
    p = W.random_problem(24, 60, 8, 1, seed=12)
    say("case: gain energy records")
    maxit = 200
    out = _run(lib, p, "fp64", 1e-13, maxit, want_hist=True, want_iters=True)
    ref = O.enkf_gain_cg(p.Xf, p.idx, p.w, p.y, p.r, p.eps, tol=1e-13, maxit=maxit, record=True)
    hist = out["hist"].cpu().numpy()
    its = out["iters"].cpu().numpy()
    for i in range(24):
        e = O.energy_errors(ref["Psi"], ref["B"][:, i], ref["iterates"][i]) ** 2
        t = its[i]
        tail = np.cumsum(hist[:t, i][::-1])[::-1]       # sum_{s >= k} alpha_s |r_s|^2
        kk = min(t, len(e) - 1)
        # early iterates, where the error is well above the final rounding level
        for k_ in range(kk):
            if e[k_] < 1e-16 * e[0] * 1e6:
                break
            assert abs(tail[k_] - e[k_]) <= 1e-8 * e[0], (i, k_)
        assert np.all(hist[t:, i] == 0.0)


@pytest.mark.parametrize("m", [10, 20, 200])
def test_example1b_bound_and_termination(lib, m):
    """Example 1b (H = I, R = I, Q = 0.1 I, N = 50, tol 1e-12) at its first
    analysis: every column of K^T meets Proposition 1's bound at every step,
    ends within N + 2 steps (R = I leaves at most N distinct eigenvalues), and
    the converged gain is the oracle's."""
    p = W.example1b(m=m, N=50, rep=0)
    say(f"case: example 1b m={m}")
    maxit = 400
    out = _run(lib, p, "fp64", 1e-12, maxit, want_hist=True, want_iters=True, want_kt=True)
    ref = O.enkf_gain_cg(p.Xf, p.idx, p.w, p.y, p.r, p.eps, tol=1e-12, maxit=maxit)
    assert out["status"] == 0
    assert rel(out["KT"].cpu().numpy(), ref["KT"]) <= 1e-10
    its = out["iters"].cpu().numpy()
    assert its.max() <= 50 + 2
    ev = np.linalg.eigvalsh(ref["Psi"])
    kappa = ev[-1] / ev[0]
    rate = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    hist = out["hist"].cpu().numpy()
    for i in range(m):
        tail = np.cumsum(hist[:its[i], i][::-1])[::-1]
        e0 = np.sqrt(tail[0]) if its[i] else 0.0
        for k_ in range(its[i]):
            assert np.sqrt(max(tail[k_], 0.0)) <= 2 * rate ** k_ * e0 * (1 + 1e-6) + 1e-12


def test_gain_in_place_and_errors(lib):
    p = W.random_problem(100, 80, 12, 2, seed=31)
    a = dev_problem(p, "fp64")
    say("case: gain in place and errors")
    first = lib.gain_analysis(**a, tol=1e-10, maxit=500, prec="fp64")["Xa"].clone()
    Xf = a["Xf"].clone()
    lib.gain_analysis(**dict(a, Xf=Xf), tol=1e-10, maxit=500, prec="fp64", out=Xf)
    torch.cuda.synchronize()
    assert torch.equal(Xf, first)
    bad = dict(a, idx=a["idx"].clone())
    bad["idx"][3, 0] = -1
    out = lib.gain_analysis(**bad, tol=1e-10, maxit=500, prec="fp64", raise_on_error=False)
    assert out["status"] == -2                      # CGD_ERR_INDEX
    ok = lib.gain_analysis(**a, tol=1e-10, maxit=500, prec="fp64", workspace=out["workspace"])
    assert ok["status"] == 0
    # maxit reached: CGD_NOT_CONVERGED, iterations = maxit
    out = lib.gain_analysis(**a, tol=1e-14, maxit=3, prec="fp64", want_iters=True)
    assert out["status"] == 1 and int(out["iters"].max()) == 3
    # N past the MFMA widths, and the BF16 modes: not supported
    q = W.random_problem(40, 30, 130, 1, seed=2)
    out = lib.gain_analysis(**dev_problem(q, "fp64"), prec="fp64", raise_on_error=False)
    assert out["status"] == -7                      # CGD_ERR_UNSUPPORTED
    out = lib.gain_analysis(**dev_problem(p, "fp32"), prec="mixed", raise_on_error=False,
                            stats=False)
    assert out["status"] == -7


@pytest.mark.parametrize("n,m,N", [(5, 1, 2), (1, 40, 12), (16, 3, 33)])
def test_gain_small_edges(lib, n, m, N):
    """n below one 16-column block (and exactly one), one observation, N = 2."""
    p = W.random_problem(n, m, N, 1, seed=n + 7 * m + N, duplicate_idx=True)
    say(f"case: gain edges n={n} m={m} N={N}")
    out = _run(lib, p, "fp64", 1e-12, 500, want_kt=True, want_iters=True)
    ref = O.enkf_gain_cg(p.Xf, p.idx, p.w, p.y, p.r, p.eps, tol=1e-12, maxit=500)
    assert out["status"] == 0
    assert rel(out["Xa"].cpu().numpy(), ref["Xa"]) <= 1e-10
    assert rel(out["KT"].cpu().numpy(), ref["KT"]) <= 1e-10
    # one observation: Psi is a scalar, every column ends in one step
    if m == 1:
        assert int(out["iters"].max()) <= 1


def test_gain_validate(lib):
    """validate = 1: r <= 0 gives CGD_ERR_NONPOS_R, a non-finite X_f
    CGD_ERR_NONFINITE, before any launch of the analysis."""
    p = W.random_problem(60, 50, 10, 2, seed=6)
    a = dev_problem(p, "fp64")
    say("case: gain validate")
    bad = dict(a, r=a["r"].clone())
    bad["r"][0] = -1.0
    assert lib.gain_analysis(**bad, prec="fp64", validate=True,
                             raise_on_error=False)["status"] == -3
    bad = dict(a, Xf=a["Xf"].clone())
    bad["Xf"][3, 2] = float("inf")
    assert lib.gain_analysis(**bad, prec="fp64", validate=True,
                             raise_on_error=False)["status"] == -4
    assert lib.gain_analysis(**a, prec="fp64", validate=True, tol=1e-10)["status"] == 0


def test_example1b_prop3_outlier_bound(lib):
    """Proposition 3 on the GPU's energy-error curves (tail sums of the
    records) for Example 1b at m = 200: with the l = 8 largest eigenvalues of
    Psi as the outliers mu_i and the rest as the bulk [lambda_a, lambda_b],
    ||e_r|| <= 2 C rho_eff^(r - l) ||e_0|| for r >= l, where
    C = max over the bulk of prod_i |1 - lambda/mu_i| and rho_eff is the
    Chebyshev rate of lambda_b / lambda_a."""
    p = W.example1b(m=200, N=50, rep=1)
    say("case: example 1b proposition 3")
    maxit = 400
    out = _run(lib, p, "fp64", 1e-12, maxit, want_hist=True, want_iters=True)
    ref = O.enkf_gain_cg(p.Xf, p.idx, p.w, p.y, p.r, p.eps, tol=1e-12, maxit=1)
    ev = np.sort(np.linalg.eigvalsh(ref["Psi"]))
    l = 8
    mu, bulk = ev[-l:], ev[:-l]
    C = max(np.prod(np.abs(1.0 - lam / mu)) for lam in bulk)
    keff = bulk[-1] / bulk[0]
    rate = (np.sqrt(keff) - 1) / (np.sqrt(keff) + 1)
    its = out["iters"].cpu().numpy()
    hist = out["hist"].cpu().numpy()
    checked = 0
    for i in range(200):
        if its[i] == 0:
            continue
        tail = np.cumsum(hist[:its[i], i][::-1])[::-1]
        e0 = np.sqrt(tail[0])
        for r in range(l, its[i]):
            assert np.sqrt(max(tail[r], 0.0)) <= 2 * C * rate ** (r - l) * e0 * (1 + 1e-6) + 1e-12
            checked += 1
    assert checked > 0
