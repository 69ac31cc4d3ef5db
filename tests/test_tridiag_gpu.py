"""Non-diagonal observation covariance on the GPU (cgd_options.r_factor:
R = L L^T with L lower bidiagonal, Section 5.1; the tridiagonal Toeplitz R
of Example 2).  The library whitens by L and runs the solvers on the
whitened system; the oracle solves with the dense R directly (textbook PCG
with M = R, Cholesky, Algorithm 2 with R_N = (N-1) R = L L^T).

Tolerances as elsewhere: FP64 1e-10 against the oracle's PCG with the same
stop rule (the R^{-1}-norm), FP32 and mixed 1e-4 against Cholesky."""
import dataclasses

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import assert_iters_close, dev_problem, rel, rounded, say

pytestmark = pytest.mark.gpu


def _tri(n, m, N, k, seed, rho=0.35, sigma=0.6, tol=1e-12):
    p = W.random_problem(n, m, N, k, seed=seed, tol=tol)
    rd, ro = O.tridiag_toeplitz_R(m, sigma, rho)
    rng = np.random.default_rng(seed + 7)
    rd = rd * rng.uniform(0.8, 1.25, m)          # a non-Toeplitz SPD tridiagonal R
    eps = W.ma1_tridiag_noise(rng, m, N, sigma, rho)
    return dataclasses.replace(p, r=rd, eps=eps), ro


def _factor(lib, p, ro, prec):
    import torch
    dt = torch.float64 if prec == "fp64" else torch.float32
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0")
    return lib.tridiag_cholesky(t(p.r), t(ro), prec=prec)


def _run(lib, p, ro, **kw):
    import torch
    vprec = "fp64" if kw["prec"] == "fp64" else "fp32"   # value type of the arrays
    d = dev_problem(p, vprec)
    out = lib.analysis(**d, r_factor=_factor(lib, p, ro, vprec), **kw)
    torch.cuda.synchronize()
    res = {"Xa": out["Xa"].double().cpu().numpy(), "status": out["status"], "stats": out["stats"]}
    for key in ("Z", "iters", "relres"):
        if out[key] is not None:
            res[key] = out[key].double().cpu().numpy() if key != "iters" else out[key].cpu().numpy()
    return res


def test_factor_matches_dense_cholesky(lib):
    import torch
    rng = np.random.default_rng(1)
    m = 300
    rd = rng.uniform(1.0, 2.0, m)
    ro = rng.uniform(-0.45, 0.45, m - 1)
    f = lib.tridiag_cholesky(torch.as_tensor(rd, device="cuda:0"),
                             torch.as_tensor(ro, device="cuda:0")).cpu().numpy()
    L = np.linalg.cholesky(O.tridiag_R(rd, ro))
    assert np.allclose(f[:m], np.diag(L), rtol=1e-14, atol=0)
    assert np.allclose(f[m:], np.diag(L, -1), rtol=1e-13, atol=1e-15)
    # not positive definite: refused
    bad = np.array([1.0, 1.0, 1.0])
    with pytest.raises(lib.CGDError) as ei:
        lib.tridiag_cholesky(torch.as_tensor(bad, device="cuda:0"),
                             torch.as_tensor(np.array([0.9, 0.9]), device="cuda:0"))
    assert ei.value.status == -3


CASES = [(500, 300, 33, 3), (300, 257, 16, 2), (200, 150, 5, 1), (600, 513, 64, 1)]
SOLVER_CASES = [(s, c) for s in (1, 2, 3, 4) for c in CASES if not (s == 4 and c[2] == 64)]


@pytest.mark.parametrize("solver,case", SOLVER_CASES)
def test_fp64_parity(lib, solver, case):
    n, m, N, k = case
    p, ro = _tri(n, m, N, k, seed=5100 + m + N)
    R = O.tridiag_R(p.r, ro)
    say(f"case: tridiagonal R fp64 solver={solver} n={n} m={m} N={N} k={k}")
    got = _run(lib, p, ro, tol=p.tol, maxit=p.maxit, prec="fp64", solver=solver,
               want_z=True, want_iters=True, want_relres=True)
    assert got["status"] == 0
    ref = O.enkf_analysis_R(p.Xf, p.idx, p.w, p.y, R, p.eps, solver="pcg", tol=p.tol,
                            maxit=p.maxit)
    assert rel(got["Xa"], ref["Xa"]) <= 1e-10
    assert rel(got["Z"], ref["Z"]) <= 1e-10
    assert_iters_close(got["iters"], ref["iters"])
    assert got["iters"].max() <= N + 4          # Lemma 1 on the whitened system
    assert got["relres"].max() <= 1.5e-12
    chol = O.enkf_analysis_R(p.Xf, p.idx, p.w, p.y, R, p.eps)
    assert rel(got["Xa"], chol["Xa"]) <= 1e-9


@pytest.mark.parametrize("maxit", [1, 4])
def test_fp64_fixed_iterations_and_residual_norm(lib, maxit):
    p, ro = _tri(400, 300, 20, 2, seed=5150)
    R = O.tridiag_R(p.r, ro)
    got = _run(lib, p, ro, tol=0.0, maxit=maxit, prec="fp64", want_z=True,
               want_iters=True, want_relres=True)
    ref = O.enkf_analysis_R(p.Xf, p.idx, p.w, p.y, R, p.eps, solver="pcg", tol=0.0, maxit=maxit)
    assert np.all(got["iters"] == maxit)
    assert rel(got["Z"], ref["Z"]) <= 1e-12
    # relres_out: ||L^{-1}(d - Psi z)|| / ||L^{-1} d|| with Psi's dense R
    S, D = ref["S"], ref["D"]
    L = np.linalg.cholesky(R)
    res = np.linalg.solve(L, D - O.innovation_matrix_R(S, R) @ ref["Z"])
    want = np.linalg.norm(res, axis=0) / np.linalg.norm(np.linalg.solve(L, D), axis=0)
    assert np.allclose(got["relres"], want, rtol=1e-9)


def test_fp64_warm_start(lib):
    import torch
    p, ro = _tri(400, 300, 20, 2, seed=5160)
    R = O.tridiag_R(p.r, ro)
    chol = O.enkf_analysis_R(p.Xf, p.idx, p.w, p.y, R, p.eps)
    Z0 = np.ascontiguousarray(chol["Z"] * (1 + 1e-3 * np.random.default_rng(2).standard_normal(
        chol["Z"].shape)))
    z0 = torch.as_tensor(Z0, device="cuda:0")
    got = _run(lib, p, ro, tol=p.tol, maxit=p.maxit, prec="fp64", z0=z0,
               fallback_on_stall=True, want_z=True, want_iters=True)
    ref = O.enkf_analysis_R(p.Xf, p.idx, p.w, p.y, R, p.eps, solver="pcg", tol=p.tol,
                            maxit=p.maxit, Z0=Z0, fallback_on_stall=True)
    assert got["stats"]["n_fallbacks"] == int(ref["fallbacks"].sum())
    assert rel(got["Z"], ref["Z"]) <= 1e-10
    assert_iters_close(got["iters"], ref["iters"])


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_fp32_and_mixed(lib, prec):
    p, ro = _tri(3000, 2000, 64, 2, seed=5170, tol=1e-6)
    q = rounded(p)
    R = O.tridiag_R(q.r, np.asarray(ro, dtype=np.float32).astype(np.float64))
    say(f"case: tridiagonal R {prec}")
    got = _run(lib, p, ro, tol=1e-6, maxit=2000, prec=prec, want_relres=True,
               want_iters=True)
    assert got["status"] == 0
    chol = O.enkf_analysis_R(q.Xf, q.idx, q.w, q.y, R, q.eps)
    assert rel(got["Xa"], chol["Xa"]) <= 1e-4
    say(f"  iterations {got['iters'].max()}, true residual (R^-1 norm) {got['relres'].max():.2e}")


@pytest.mark.parametrize("N", [20, 64, 100, 160])
def test_reduced_parity(lib, N):
    p, ro = _tri(500, 300, N, 2, seed=5180 + N)
    R = O.tridiag_R(p.r, ro)
    say(f"case: tridiagonal R reduced N={N}")
    got = _run(lib, p, ro, tol=1e-13, maxit=1000, prec="fp64", reduced=True,
               want_iters=True)
    assert got["status"] == 0
    ref = O.enkf_reduced_R(p.Xf, p.idx, p.w, p.y, R, p.eps)
    assert rel(got["Xa"], ref["Xa"]) <= 1e-10
    f32 = _run(lib, p, ro, tol=1e-6, maxit=1000, prec="fp32", reduced=True)
    assert rel(f32["Xa"], ref["Xa"]) <= 1e-4


def test_example2_workload(lib):
    """Example 2's setting at one analysis: Lorenz-96 n = m = 4096 (H = I),
    N = 100, tridiagonal Toeplitz R (sigma 0.3, rho 0.2), FP32 to 1e-6, full
    and reduced mode against the FP64 oracle's direct solutions."""
    p, ro = W.example2(n=4096, N=100)
    q = rounded(p)
    R = O.tridiag_R(q.r, np.asarray(ro, dtype=np.float32).astype(np.float64))
    say("case: example 2, n = m = 4096, N = 100")
    full = _run(lib, p, ro, tol=1e-6, maxit=2000, prec="fp32", want_iters=True,
                want_relres=True)
    red = _run(lib, p, ro, tol=1e-6, maxit=2000, prec="fp32", reduced=True)
    ref = O.enkf_reduced_R(q.Xf, q.idx, q.w, q.y, R, q.eps)["Xa"]   # = Algorithm 1's X_a
    e1, e2 = rel(full["Xa"], ref), rel(red["Xa"], ref)
    say(f"  full: iterations {full['iters'].max()}, rel err {e1:.2e}; reduced rel err {e2:.2e}")
    assert full["status"] == 0 and e1 <= 1e-4 and e2 <= 1e-4


def test_fp32_tile_solver(lib):
    """The row-block x member-group solver on the whitened problem (N = 100,
    so the last member group is part empty)."""
    p, ro = _tri(5000, 4100, 100, 2, seed=5190, tol=1e-6)
    q = rounded(p)
    R = O.tridiag_R(q.r, np.asarray(ro, dtype=np.float32).astype(np.float64))
    say("case: tridiagonal R fp32 tile solver")
    got = _run(lib, p, ro, tol=1e-6, maxit=2000, prec="fp32", solver=5, want_relres=True,
               want_iters=True)
    assert got["status"] == 0
    chol = O.enkf_analysis_R(q.Xf, q.idx, q.w, q.y, R, q.eps)
    err = rel(got["Xa"], chol["Xa"])
    say(f"  iterations {got['iters'].max()}, X_a vs Cholesky {err:.2e}, "
        f"true residual {got['relres'].max():.2e}")
    assert err <= 1e-4
    assert got["relres"].max() <= 2e-5
