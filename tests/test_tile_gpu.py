"""The row-block x member-group solver (solver=5) against the oracle, in
FP32, in the mixed mode (BF16 inner CG, FP64-accumulated outer residual) and
in the split-BF16 mode (each S-product as five BF16 products of S's two-part
and the vector's three-part BF16 splits): member counts that leave part of the last group of 32 empty,
ragged row blocks, one to 256 workgroups, both paddings of N (64, 128) and
both row blocks (128, 256), fixed iteration counts, preconditioning,
statistics, statuses and bitwise repeatability."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import dev_problem, rel, rounded, run, say

pytestmark = pytest.mark.gpu


def _chol(p):
    return O.enkf_analysis(p.Xf, p.idx, p.w, p.y, p.r, p.eps, solver="cholesky")


# (n, m, N, k): groups of 32 members x blocks of 128 or 256 rows
CASES = [
    (60, 20, 20, 1),        # one workgroup: its owner step sums the whole exchange
    (600, 513, 64, 1),      # N = 64 (NP 64), 2 groups x 5 ragged blocks
    (900, 700, 128, 4),     # 4 groups x 6 blocks
    (5000, 4100, 100, 1),   # last group has 4 members
    (3000, 2048, 16, 2),    # 16 blocks, one group half empty
    (20000, 16384, 40, 1),  # 2 groups x 128 blocks = 256 workgroups
    (70000, 16384, 128, 4),  # 256-row blocks: 4 groups x 64 blocks (the 2-D workload's shape)
]


@pytest.mark.parametrize("n,m,N,k", CASES)
def test_fp32_against_cholesky(lib, n, m, N, k):
    p = W.random_problem(n, m, N, k, seed=500 + N + m, tol=1e-6)
    say(f"case: tile fp32 n={n} m={m} N={N} k={k}")
    got = run(lib, p, "fp32", solver=5, want_relres=True, want_iters=True, want_z=True)
    assert got["status"] == 0, got["status"]
    ref = _chol(p)
    err = rel(got["Xa"], ref["Xa"])
    say(f"  X_a vs Cholesky {err:.2e}, iterations {got['iters'].min()}..{got['iters'].max()}, "
        f"true rel. residual {got['relres'].max():.2e}")
    assert err <= 1e-4
    assert got["relres"].max() <= 2e-5
    assert rel(got["Z"], ref["Z"]) <= 1e-3


@pytest.mark.parametrize("n,m,N,k", [(900, 700, 128, 4), (600, 513, 64, 1), (60, 20, 20, 1)])
def test_fixed_iterations_follow_the_oracle(lib, n, m, N, k):
    """Seven steps from zero: the iterates of the FP64 textbook CG on the
    same (FP32-rounded) inputs, to FP32 rounding."""
    p = W.random_problem(n, m, N, k, seed=600 + N, tol=1e-6)
    got = run(lib, p, "fp32", solver=5, tol=0.0, maxit=7, want_z=True, want_iters=True,
              raise_on_error=False)
    assert got["status"] == 1  # CGD_NOT_CONVERGED: every member stopped at maxit
    assert np.all(got["iters"] == 7)
    q = rounded(p)
    ref = O.enkf_analysis(q.Xf, q.idx, q.w, q.y, q.r, q.eps, solver="cg_free", tol=0.0, maxit=7)
    assert rel(got["Z"], ref["Z"]) <= 2e-5
    assert rel(got["Xa"], ref["Xa"]) <= 2e-6


def test_iterations_match_the_oracle(lib):
    p = W.random_problem(5000, 4100, 100, 1, seed=610, tol=1e-6)
    got = run(lib, p, "fp32", solver=5, want_iters=True)
    q = rounded(p)
    ref = O.enkf_analysis(q.Xf, q.idx, q.w, q.y, q.r, q.eps, solver="cg_free", tol=1e-6,
                          maxit=p.maxit)
    # FP32 recurrences lose a little conjugacy: a few more steps, never fewer
    d = got["iters"].astype(int) - ref["iters"].astype(int)
    say(f"  iterations minus oracle: {d.min()}..{d.max()}")
    assert d.min() >= -2 and d.max() <= max(3, int(0.15 * ref["iters"].max()))


def test_preconditioned(lib):
    p = W.random_problem(5000, 4100, 100, 1, seed=620, tol=1e-6)
    p.r[:] = np.random.default_rng(620).uniform(0.5, 2.0, size=p.r.shape)
    got = run(lib, p, "fp32", solver=5, precond="diag_r", want_iters=True, want_z=True,
              want_relres=True)
    assert got["status"] == 0
    ref = _chol(p)
    assert rel(got["Xa"], ref["Xa"]) <= 1e-4
    # z_out is in the original variables
    assert rel(got["Z"], ref["Z"]) <= 1e-3
    plain = run(lib, p, "fp32", solver=5, want_iters=True)
    say(f"  iterations plain {plain['iters'].max()}, preconditioned {got['iters'].max()}")


def test_repeatable_and_same_as_auto(lib):
    import torch
    p = W.random_problem(900, 700, 128, 4, seed=630, tol=1e-6)
    d = dev_problem(p, "fp32")
    a = lib.analysis(**d, tol=1e-6, maxit=1000, prec="fp32", solver=5)["Xa"].clone()
    b = lib.analysis(**d, tol=1e-6, maxit=1000, prec="fp32", solver=5)["Xa"].clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    info = lib.Plan(900, 700, 128, 4, prec="fp32").solver_info()
    say(f"  automatic choice: {info}")


def test_nonfinite_and_immediate_stop(lib):
    import dataclasses
    p = W.random_problem(900, 700, 128, 4, seed=640, tol=1e-6)
    y = p.y.copy()
    y[5] = np.nan
    bad = run(lib, dataclasses.replace(p, y=y), "fp32", solver=5, raise_on_error=False)
    assert bad["status"] == -4  # CGD_ERR_NONFINITE (no validation: the CG coefficient)
    # tol 1: every member meets the stop rule at step 0, W = 0 and X_a = X_f exactly
    got = run(lib, p, "fp32", solver=5, tol=1.0, want_iters=True)
    assert got["status"] == 0
    assert np.all(got["iters"] == 0)
    assert np.array_equal(got["Xa"], p.Xf.astype(np.float32).astype(np.float64))


def test_out_of_range_shape_is_unsupported(lib):
    """4 groups x 129 blocks of 256 rows cannot all be resident."""
    p = W.random_problem(40000, 33000, 128, 1, seed=650, tol=1e-6)
    got = run(lib, p, "fp32", solver=5, raise_on_error=False)
    assert got["status"] == -7


# --- the mixed mode: restarted refinement, BF16 inner CG on the MFMA ---------
@pytest.mark.parametrize("n,m,N,k", CASES)
def test_mixed_against_cholesky(lib, n, m, N, k):
    """The FP32 bar against the FP64 direct solve, and the reported true
    residual (the outer stop test, FP64-accumulated products of the FP32 S)
    within the tolerance."""
    p = W.random_problem(n, m, N, k, seed=700 + N + m, tol=1e-6)
    say(f"case: tile mixed n={n} m={m} N={N} k={k}")
    got = run(lib, p, "mixed", solver=5, want_relres=True, want_iters=True, want_z=True)
    assert got["status"] == 0, got["status"]
    ref = _chol(p)
    err = rel(got["Xa"], ref["Xa"])
    f32 = run(lib, p, "fp32", solver=5, want_iters=True)
    say(f"  X_a vs Cholesky {err:.2e}, inner iterations {got['iters'].min()}..{got['iters'].max()} "
        f"(FP32 CG {f32['iters'].max()}), true rel. residual {got['relres'].max():.2e}")
    assert err <= 1e-4
    assert got["relres"].max() <= 1e-6
    assert rel(got["Z"], ref["Z"]) <= 1e-3


def test_mixed_true_residual_matches_the_oracle(lib):
    """The reported relres is the true residual of the returned z on the
    FP32-rounded problem: recomputed by the oracle from z_out (as FP64)."""
    p = W.random_problem(900, 700, 128, 4, seed=710, tol=1e-6)
    got = run(lib, p, "mixed", solver=5, want_relres=True, want_z=True)
    q = rounded(p)
    # the solver sees S and D rounded to FP32 after their FP64 formation
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    S = f32(O.obs_anomalies(q.idx, q.w, q.Xf))
    D = f32(O.innovations(q.idx, q.w, q.Xf, q.y, q.eps))
    want = O.true_relres(S, q.r, got["Z"], D)
    say(f"  reported {got['relres'].max():.3e}, recomputed {want.max():.3e}")
    np.testing.assert_allclose(got["relres"], want, rtol=1e-2, atol=1e-9)


def test_mixed_fixed_budget_and_immediate_stop(lib):
    p = W.random_problem(900, 700, 128, 4, seed=720, tol=1e-6)
    # a budget of 5 inner steps: not converged, every member used it
    got = run(lib, p, "mixed", solver=5, tol=1e-12, maxit=5, want_iters=True,
              raise_on_error=False)
    assert got["status"] == 1
    assert np.all(got["iters"] == 5)
    # tol 1: every member meets the stop rule before any step, W = 0 and X_a = X_f
    got = run(lib, p, "mixed", solver=5, tol=1.0, want_iters=True)
    assert got["status"] == 0
    assert np.all(got["iters"] == 0)
    assert np.array_equal(got["Xa"], p.Xf.astype(np.float32).astype(np.float64))
    # after a call that wrote W, maxit 0 must still give W = 0
    run(lib, p, "mixed", solver=5, want_iters=True)
    got = run(lib, p, "mixed", solver=5, maxit=0, want_iters=True, raise_on_error=False)
    assert got["status"] == 1
    assert np.array_equal(got["Xa"], p.Xf.astype(np.float32).astype(np.float64))


def test_mixed_preconditioned(lib):
    p = W.random_problem(5000, 4100, 100, 1, seed=730, tol=1e-6)
    p.r[:] = np.random.default_rng(730).uniform(0.5, 2.0, size=p.r.shape)
    got = run(lib, p, "mixed", solver=5, precond="diag_r", want_iters=True, want_z=True,
              want_relres=True)
    assert got["status"] == 0
    ref = _chol(p)
    assert rel(got["Xa"], ref["Xa"]) <= 1e-4
    assert rel(got["Z"], ref["Z"]) <= 1e-3
    # the outer stop test is on the true residual in the R^{-1}-norm
    assert got["relres"].max() <= 1e-6


def test_mixed_repeatable_nonfinite_and_automatic(lib):
    import dataclasses
    import torch
    p = W.random_problem(900, 700, 128, 4, seed=740, tol=1e-6)
    d = dev_problem(p, "fp32")
    a = lib.analysis(**d, tol=1e-6, maxit=1000, prec="mixed", solver=5)["Xa"].clone()
    b = lib.analysis(**d, tol=1e-6, maxit=1000, prec="mixed", solver=5)["Xa"].clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    y = p.y.copy()
    y[3] = np.inf
    bad = run(lib, dataclasses.replace(p, y=y), "mixed", solver=5, raise_on_error=False)
    assert bad["status"] == -4
    # vectors beyond the column solver's LDS room: the automatic choice is this solver
    info = lib.Plan(70000, 16384, 128, 4, prec="mixed").solver_info()
    say(f"  automatic choice at m = 16384: {info}")
    assert info["solver"] == "k_cg_tilemx"


# --- the split-BF16 mode: five BF16 products per S-product --------------------
@pytest.mark.parametrize("n,m,N,k", CASES)
def test_bf16split_against_cholesky(lib, n, m, N, k):
    """The FP32 bar against the FP64 direct solve; the reported residual is
    the true one (FP64-accumulated products of the FP32 S)."""
    p = W.random_problem(n, m, N, k, seed=800 + N + m, tol=1e-6)
    say(f"case: tile bf16split n={n} m={m} N={N} k={k}")
    got = run(lib, p, "bf16split", solver=5, want_relres=True, want_iters=True, want_z=True)
    assert got["status"] == 0, got["status"]
    ref = _chol(p)
    err = rel(got["Xa"], ref["Xa"])
    f32 = run(lib, p, "fp32", solver=5, want_iters=True, want_relres=True)
    say(f"  X_a vs Cholesky {err:.2e}, iterations {got['iters'].min()}..{got['iters'].max()} "
        f"(FP32 {f32['iters'].max()}), true rel. residual {got['relres'].max():.2e} "
        f"(FP32 {f32['relres'].max():.2e})")
    assert err <= 1e-4
    # S's two BF16 parts carry about 16 bits (2^-18 relative), which sets the
    # true residual's floor near 1e-5 (FP32: ~1e-6)
    assert got["relres"].max() <= 1e-4
    assert rel(got["Z"], ref["Z"]) <= 1e-3
    # a few more steps than FP32 at most
    assert got["iters"].max() <= f32["iters"].max() + max(3, f32["iters"].max() // 10)


@pytest.mark.parametrize("n,m,N,k", [(900, 700, 128, 4), (600, 513, 64, 1)])
def test_bf16split_fixed_iterations_follow_the_oracle(lib, n, m, N, k):
    """Seven steps from zero: the FP64 textbook CG's iterates on the same
    (FP32-rounded) inputs, to the split products' rounding."""
    p = W.random_problem(n, m, N, k, seed=810 + N, tol=1e-6)
    got = run(lib, p, "bf16split", solver=5, tol=0.0, maxit=7, want_z=True, want_iters=True,
              raise_on_error=False)
    assert got["status"] == 1
    assert np.all(got["iters"] == 7)
    q = rounded(p)
    ref = O.enkf_analysis(q.Xf, q.idx, q.w, q.y, q.r, q.eps, solver="cg_free", tol=0.0, maxit=7)
    ez, ex = rel(got["Z"], ref["Z"]), rel(got["Xa"], ref["Xa"])
    say(f"  Z {ez:.2e}, X_a {ex:.2e} against the FP64 iterates")
    assert ez <= 2e-4
    assert ex <= 2e-5


def test_bf16split_statuses(lib):
    import dataclasses
    p = W.random_problem(900, 700, 128, 4, seed=820, tol=1e-6)
    got = run(lib, p, "bf16split", solver=5, tol=1.0, want_iters=True)
    assert got["status"] == 0
    assert np.all(got["iters"] == 0)
    assert np.array_equal(got["Xa"], p.Xf.astype(np.float32).astype(np.float64))
    y = p.y.copy()
    y[7] = np.nan
    bad = run(lib, dataclasses.replace(p, y=y), "bf16split", solver=5, raise_on_error=False)
    assert bad["status"] == -4
    # only on this solver and in the full mode
    d = dev_problem(p, "fp32")
    assert lib.analysis(**d, prec="bf16split", solver=3, raise_on_error=False)["status"] == -7
    assert lib.analysis(**d, prec="bf16split", reduced=True, raise_on_error=False)["status"] == -7
    info = lib.Plan(900, 700, 128, 4, prec="bf16split").solver_info()
    assert info["solver"] == "k_cg_tilesplit"


def test_bf16split_preconditioned_and_repeatable(lib):
    import torch
    p = W.random_problem(5000, 4100, 100, 1, seed=830, tol=1e-6)
    got = run(lib, p, "bf16split", solver=5, precond="diag_r", want_iters=True, want_relres=True)
    assert got["status"] == 0
    assert rel(got["Xa"], _chol(p)["Xa"]) <= 1e-4
    d = dev_problem(p, "fp32")
    a = lib.analysis(**d, tol=1e-6, maxit=1000, prec="bf16split")["Xa"].clone()
    b = lib.analysis(**d, tol=1e-6, maxit=1000, prec="bf16split")["Xa"].clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
