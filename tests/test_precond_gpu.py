"""diag(R)-preconditioned CG (CGD_PRECOND_DIAG_R) on every solver against the
oracle's textbook PCG with M = diag(r) (the L^{-1} scaling of Algorithm 2
applied to the full system; Section 5.2, Lemma 1).

Tolerances as for plain CG: 1e-10 relative in FP64 against the oracle's PCG
with the same stop rule (the R^{-1}-norm of the residual), 1e-4 in FP32 and
the mixed mode against the oracle's Cholesky solution."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import assert_iters_close, dev_problem, rel, run, say

pytestmark = pytest.mark.gpu


def _pcg(p, tol=None, maxit=None, Z0=None, fallback=False):
    return O.enkf_analysis(p.Xf, p.idx, p.w, p.y, p.r, p.eps, solver="pcg_free",
                           tol=p.tol if tol is None else tol,
                           maxit=p.maxit if maxit is None else maxit, Z0=Z0,
                           fallback_on_stall=fallback)


def _chol(p):
    return O.enkf_analysis(p.Xf, p.idx, p.w, p.y, p.r, p.eps, solver="cholesky")


CASES = [(500, 300, 33, 3), (600, 513, 64, 1), (300, 257, 16, 2), (200, 150, 5, 1)]
# the forced split solver needs a member's row slices co-resident: at N = 64
# in FP64 that takes fewer rows than 513
SOLVER_CASES = [(s, c) for s in (1, 2, 3, 4) for c in CASES if not (s == 4 and c[2] == 64)]


@pytest.mark.parametrize("solver,case", SOLVER_CASES)
def test_fp64_parity(lib, solver, case):
    n, m, N, k = case
    # a wide spread of diag(R), where plain CG needs many more than N steps
    p = W.random_problem(n, m, N, k, seed=2100 + m + N, r_lo=0.05, r_hi=20.0, tol=1e-12)
    say(f"case: precond fp64 solver={solver} n={n} m={m} N={N} k={k}")
    got = run(lib, p, "fp64", solver=solver, precond="diag_r", want_z=True, want_iters=True,
              want_relres=True)
    assert got["status"] == 0
    ref = _pcg(p)
    assert rel(got["Xa"], ref["Xa"]) <= 1e-10
    assert rel(got["Z"], ref["Z"]) <= 1e-10
    assert_iters_close(got["iters"], ref["iters"])
    # Lemma 1: at most N steps in exact arithmetic (a few more for FP64 rounding at 1e-12)
    assert got["iters"].max() <= N + 4
    # the reported true residual is in the R^{-1}-norm of the stop rule; at
    # convergence both it and the oracle's value are at the rounding floor
    S = O.obs_anomalies(p.idx, p.w, p.Xf)
    D = O.innovations(p.idx, p.w, p.Xf, p.y, p.eps)
    assert got["relres"].max() <= 1e-12 * 1.5
    assert O.true_relres_rinv(S, p.r, got["Z"], D).max() <= 1e-12 * 1.5


@pytest.mark.parametrize("maxit", [0, 1, 5])
@pytest.mark.parametrize("solver", [2, 4])
def test_fp64_fixed_iterations(lib, solver, maxit):
    p = W.random_problem(500, 333, 24, 2, seed=2117, r_lo=0.1, r_hi=10.0, tol=1e-12)
    say(f"case: precond fp64 fixed maxit={maxit} solver={solver}")
    got = run(lib, p, "fp64", solver=solver, precond="diag_r", tol=0.0, maxit=maxit,
              want_z=True, want_iters=True, want_relres=True)
    ref = _pcg(p, tol=0.0, maxit=maxit)
    assert np.all(got["iters"] == maxit)
    assert rel(got["Z"], ref["Z"]) <= 1e-12
    assert rel(got["Xa"], ref["Xa"]) <= 1e-12
    # away from convergence the reported residual is the R^{-1}-norm of d - Psi z
    S = O.obs_anomalies(p.idx, p.w, p.Xf)
    D = O.innovations(p.idx, p.w, p.Xf, p.y, p.eps)
    assert np.allclose(got["relres"], O.true_relres_rinv(S, p.r, ref["Z"], D), rtol=1e-9)


@pytest.mark.parametrize("solver", [2, 3, 4])
def test_fp64_warm_start(lib, solver):
    import torch
    p = W.random_problem(400, 300, 20, 2, seed=2119, r_lo=0.1, r_hi=10.0, tol=1e-12)
    chol = _chol(p)
    rng = np.random.default_rng(5)
    Z0 = np.ascontiguousarray(chol["Z"] * (1.0 + 1e-3 * rng.standard_normal(chol["Z"].shape)))
    say(f"case: precond fp64 warm start solver={solver}")
    z0 = torch.as_tensor(Z0, dtype=torch.float64, device="cuda:0")
    got = run(lib, p, "fp64", solver=solver, precond="diag_r", z0=z0, fallback_on_stall=True,
              want_z=True, want_iters=True)
    ref = _pcg(p, Z0=Z0, fallback=True)
    assert got["stats"]["n_fallbacks"] == int(ref["fallbacks"].sum()) == 0
    assert rel(got["Z"], ref["Z"]) <= 1e-10
    assert_iters_close(got["iters"], ref["iters"])
    # a warm start that overshoots falls back from the R^{-1}-norm test
    bad = torch.as_tensor(np.ascontiguousarray(-20.0 * chol["Z"]), dtype=torch.float64,
                          device="cuda:0")
    got = run(lib, p, "fp64", solver=solver, precond="diag_r", z0=bad, fallback_on_stall=True,
              want_z=True)
    ref = _pcg(p, Z0=-20.0 * chol["Z"], fallback=True)
    assert got["stats"]["n_fallbacks"] == int(ref["fallbacks"].sum()) == p.N
    assert rel(got["Z"], ref["Z"]) <= 1e-10


@pytest.mark.parametrize("solver", [0, 5])
@pytest.mark.parametrize("n,m,N,k", [(4096, 2048, 64, 1), (3000, 2500, 48, 2), (900, 700, 128, 4)])
def test_fp32_parity(lib, n, m, N, k, solver):
    p = W.random_problem(n, m, N, k, seed=2150 + N, r_lo=0.05, r_hi=20.0, tol=1e-6)
    say(f"case: precond fp32 solver={solver} n={n} m={m} N={N} k={k}")
    got = run(lib, p, "fp32", solver=solver, precond="diag_r", want_relres=True, want_iters=True)
    plain = run(lib, p, "fp32", solver=solver, want_iters=True)
    assert got["status"] == 0
    assert rel(got["Xa"], _chol(p)["Xa"]) <= 1e-4
    assert got["relres"].max() <= 2e-5
    say(f"  iterations preconditioned {got['iters'].max()}, plain {plain['iters'].max()}")
    assert got["iters"].max() < plain["iters"].max()


def test_mixed_parity(lib):
    p = W.random_problem(3000, 2000, 64, 4, seed=2160, r_lo=0.5, r_hi=2.0, tol=1e-6)
    say("case: precond mixed")
    got = run(lib, p, "mixed", precond="diag_r", want_relres=True, want_iters=True)
    assert got["status"] == 0
    assert rel(got["Xa"], _chol(p)["Xa"]) <= 1e-4
    # the outer stop test is on the true residual in the R^{-1}-norm
    assert got["relres"].max() <= 1e-6


def test_batched_parity(lib):
    probs = [W.random_problem(n, m, N, k, seed=2170 + i, r_lo=0.05, r_hi=20.0, tol=1e-12)
             for i, (n, m, N, k) in enumerate([(300, 257, 33, 2), (100, 40, 16, 1),
                                               (700, 640, 64, 3)])]
    say("case: precond batched fp64")
    b = lib.Batch([{k: v for k, v in dev_problem(p, "fp64").items()} for p in probs],
                  prec="fp64", precond="diag_r")
    status, stats = b.run(tol=1e-12, maxit=1000, stats=True)
    assert status == 0
    import torch
    torch.cuda.synchronize()
    for p, out, it in zip(probs, b.outs, b.iters):
        ref = _pcg(p, tol=1e-12, maxit=1000)
        assert rel(out.cpu().numpy(), ref["Xa"]) <= 1e-10
        assert_iters_close(it.cpu().numpy(), ref["iters"])


def test_config3_fp32_and_mixed(lib):
    """The 2-D advection-diffusion workload at full size: the preconditioned
    solve reaches the FP32 accuracy of plain CG in a fraction of the steps."""
    p = W.config3()
    say("case: config3 precond fp32 and mixed")
    chol_free = _pcg(p, tol=1e-10, maxit=500)
    got = run(lib, p, "fp32", precond="diag_r", want_relres=True, want_iters=True)
    assert got["status"] == 0
    err = rel(got["Xa"], chol_free["Xa"])
    say(f"  fp32: iterations {got['iters'].min()}..{got['iters'].max()}, X_a vs FP64 PCG at 1e-10 "
        f"{err:.2e}, R^-1 true residual {got['relres'].max():.2e}")
    assert err <= 1e-4
    assert got["iters"].max() <= 60
    mix = run(lib, p, "mixed", precond="diag_r", want_relres=True, want_iters=True)
    assert mix["status"] == 0
    err = rel(mix["Xa"], chol_free["Xa"])
    say(f"  mixed: inner iterations {mix['iters'].max()}, X_a vs FP64 PCG {err:.2e}, "
        f"true residual {mix['relres'].max():.2e}")
    assert err <= 1e-4
    assert mix["relres"].max() <= 1e-6
