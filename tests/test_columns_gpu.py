"""The column-parallel solver (solver=3: one workgroup per member, S streamed
through L2, update applied in the same launch) against the oracle."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import assert_iters_close, dev_problem, rel, run, say

pytestmark = pytest.mark.gpu


def _cg(p, tol=None, maxit=None):
    return O.enkf_analysis(p.Xf, p.idx, p.w, p.y, p.r, p.eps, solver="cg_free",
                           tol=p.tol if tol is None else tol,
                           maxit=p.maxit if maxit is None else maxit)


def _chol(p):
    return O.enkf_analysis(p.Xf, p.idx, p.w, p.y, p.r, p.eps, solver="cholesky")


# (n, m, N, k): ragged row steps, every padded width (16/32/64), m below one row step,
# N = 2, and the largest FP64 m
CASES64 = [(40, 20, 20, 1), (50, 37, 3, 2), (40, 3, 17, 1), (30, 12, 2, 1), (300, 257, 33, 4),
           (600, 513, 64, 1), (700, 1000, 48, 2), (2500, 2048, 64, 1), (100, 65, 16, 3)]


@pytest.mark.parametrize("n,m,N,k", CASES64)
def test_fp64_parity(lib, n, m, N, k):
    p = W.random_problem(n, m, N, k, seed=900 + m + N, tol=1e-12)
    say(f"case: columns fp64 n={n} m={m} N={N} k={k}")
    got = run(lib, p, "fp64", solver=3, want_z=True, want_iters=True, want_relres=True)
    assert got["status"] in (0, 1)
    ref = _cg(p)
    assert rel(got["Xa"], ref["Xa"]) <= 1e-10
    assert rel(got["Z"], ref["Z"]) <= 1e-10
    assert_iters_close(got["iters"], ref["iters"])
    assert got["relres"].max() <= 1e-11


@pytest.mark.parametrize("maxit", [0, 1, 7])
def test_fp64_fixed_iterations(lib, maxit):
    p = W.random_problem(500, 333, 20, 2, seed=7, tol=1e-12)
    say(f"case: columns fp64 fixed maxit={maxit}")
    got = run(lib, p, "fp64", solver=3, tol=0.0, maxit=maxit, want_z=True, want_iters=True)
    ref = _cg(p, tol=0.0, maxit=maxit)
    assert np.all(got["iters"] == maxit)
    assert rel(got["Z"], ref["Z"]) <= 1e-12
    assert rel(got["Xa"], ref["Xa"]) <= 1e-12
    if maxit == 0:
        assert np.array_equal(got["Xa"], p.Xf)


@pytest.mark.parametrize("n,m,N,k", [(4096, 2048, 64, 1), (5000, 4096, 64, 1), (5000, 4096, 16, 2),
                                     (60, 20, 20, 1), (700, 513, 33, 1)])
def test_fp32_parity(lib, n, m, N, k):
    p = W.random_problem(n, m, N, k, seed=950 + N, tol=1e-6)
    say(f"case: columns fp32 n={n} m={m} N={N} k={k}")
    got = run(lib, p, "fp32", solver=3, want_relres=True, want_iters=True)
    assert got["status"] == 0
    assert rel(got["Xa"], _chol(p)["Xa"]) <= 1e-4
    assert got["relres"].max() <= 2e-5


def test_config2_cycle_fp32_and_auto_choice(lib):
    """One Lorenz-96 twin-experiment analysis at its real size; the automatic
    choice runs the column solver there."""
    import ctypes
    cyc = W.L96Cycler(tol=1e-6, maxit=1000)
    p = cyc.problem()
    plan = lib.Plan(p.n, p.m, p.N, p.k, prec="fp32")
    assert plan.solver_info()["solver"] in ("k_cg_columns", "k_cg_split")
    got = run(lib, p, "fp32", want_relres=True)
    assert got["status"] == 0
    assert rel(got["Xa"], _chol(p)["Xa"]) <= 1e-4
    assert got["relres"].max() <= 2e-5
    b = run(lib, p, "fp32")
    assert np.array_equal(got["Xa"], b["Xa"])


def test_warm_start_and_fallback(lib):
    import torch
    p = W.random_problem(300, 150, 12, 2, seed=12, tol=1e-10)
    S = O.obs_anomalies(p.idx, p.w, p.Xf)
    D = O.innovations(p.idx, p.w, p.Xf, p.y, p.eps)
    zs = np.ascontiguousarray(O.solve_cholesky(O.innovation_matrix(S, p.r), D))
    a = dev_problem(p, "fp64")
    for z0, expect_fb in ((-10 * zs, True), (zs * (1 + 1e-6), False)):
        say(f"case: columns warm start, fallback expected={expect_fb}")
        out = lib.analysis(**a, tol=p.tol, maxit=p.maxit, prec="fp64", solver=3,
                           z0=torch.as_tensor(np.ascontiguousarray(z0), device="cuda:0"),
                           fallback_on_stall=True, want_z=True, want_iters=True)
        torch.cuda.synchronize()
        ref = O.solve_cg_columns(O.matvec_free(S, p.r), D, p.tol, p.maxit, Z0=z0,
                                 fallback_on_stall=True)
        assert (out["stats"]["n_fallbacks"] == p.N) == expect_fb
        assert rel(out["Z"].cpu().numpy(), ref[0]) <= 1e-10
        assert np.max(np.abs(out["iters"].cpu().numpy() - ref[1])) <= 2
        # the update uses W accumulated from the CG's own products: it must
        # equal X_f + A S^T Z/(N-1) for the Z the solver returned
        Zg = out["Z"].cpu().numpy()
        Xa_own = p.Xf + (p.Xf - p.Xf.mean(1, keepdims=True)) @ (S.T @ Zg) / (p.N - 1)
        assert rel(out["Xa"].cpu().numpy(), Xa_own) <= 1e-12


def test_in_place_update(lib):
    import torch
    p = W.random_problem(400, 300, 24, 2, seed=21, tol=1e-10)
    a = dev_problem(p, "fp64")
    Xf_dev = a["Xf"].clone()
    a["Xf"] = Xf_dev
    out = lib.analysis(**a, tol=p.tol, maxit=p.maxit, prec="fp64", solver=3, out=Xf_dev)
    torch.cuda.synchronize()
    assert out["Xa"].data_ptr() == Xf_dev.data_ptr()
    assert rel(Xf_dev.cpu().numpy(), _cg(p)["Xa"]) <= 1e-10


def test_bad_index_reported(lib):
    p = W.random_problem(100, 40, 8, 2, seed=15)
    a = dev_problem(p, "fp64")
    a["idx"] = a["idx"].clone()
    a["idx"][5, 1] = 100
    a["idx"][7, 0] = -3
    out = lib.analysis(**a, solver=3, raise_on_error=False)
    assert out["status"] == -2


def test_outside_its_range_is_unsupported(lib):
    for (n, m, N, prec) in ((200, 100, 129, "fp32"), (200, 100, 65, "fp64")):
        p = W.random_problem(n, m, N, 1, seed=3)
        out = lib.analysis(**dev_problem(p, prec), prec=prec, solver=3, raise_on_error=False)
        assert out["status"] == -7, (n, m, N, prec)


def test_matches_resident_solver(lib):
    p = W.random_problem(1500, 1024, 40, 2, seed=31, tol=1e-12)
    a = run(lib, p, "fp64", solver=3)
    b = run(lib, p, "fp64", solver=2)
    assert rel(a["Xa"], b["Xa"]) <= 1e-11


# --- mixed precision: restarted iterative refinement on a BF16 copy of S -------
@pytest.mark.parametrize("n,m,N,k", [(4096, 2048, 64, 1), (700, 513, 33, 1), (60, 20, 20, 1),
                                     (3000, 1000, 16, 2)])
def test_mixed_precision_parity(lib, n, m, N, k):
    """FP32 data, BF16 inner products, FP64-accumulated outer residual: the
    same 1e-4 bar as FP32 against the FP64 direct solve, and the reported
    true residual (the outer stop test) within the tolerance."""
    p = W.random_problem(n, m, N, k, seed=970 + N, tol=1e-6)
    say(f"case: columns mixed n={n} m={m} N={N} k={k}")
    got = run(lib, p, "mixed", want_relres=True, want_iters=True)
    f32 = run(lib, p, "fp32", solver=3, want_iters=True)
    ref = _chol(p)
    err = rel(got["Xa"], ref["Xa"])
    say(f"  X_a vs FP64 {err:.2e}, true residual {got['relres'].max():.2e}, inner iterations "
        f"{got['iters'].max()} (FP32 CG {f32['iters'].max()})")
    assert got["status"] == 0
    assert err <= 1e-4
    assert got["relres"].max() <= 1e-6


def test_mixed_precision_config2_cycle(lib):
    cyc = W.L96Cycler(tol=1e-6, maxit=1000)
    p = cyc.problem()
    got = run(lib, p, "mixed", want_relres=True, want_iters=True)
    assert got["status"] == 0
    assert rel(got["Xa"], _chol(p)["Xa"]) <= 1e-4
    assert got["relres"].max() <= 1e-6


def test_mixed_precision_only_on_the_column_and_tile_solvers(lib):
    p = W.random_problem(200, 100, 129, 1, seed=3)
    out = lib.analysis(**dev_problem(p, "fp32"), prec="mixed", raise_on_error=False)
    assert out["status"] == -7
    q = W.random_problem(200, 100, 16, 1, seed=3)
    out = lib.analysis(**dev_problem(q, "fp32"), prec="mixed", solver=2, raise_on_error=False)
    assert out["status"] == -7


# --- N up to 128 (FP32 and mixed), and the CG vectors in global memory when
# they do not fit in LDS (any m) ---------------------------------------------
@pytest.mark.parametrize("n,m,N,k", [(700, 513, 100, 1), (3000, 2500, 128, 2), (6000, 5000, 96, 1)])
def test_fp32_parity_wide(lib, n, m, N, k):
    p = W.random_problem(n, m, N, k, seed=1400 + N, tol=1e-6)
    say(f"case: columns fp32 wide n={n} m={m} N={N} k={k}")
    got = run(lib, p, "fp32", solver=3, want_relres=True, want_iters=True)
    assert got["status"] == 0
    assert rel(got["Xa"], _chol(p)["Xa"]) <= 1e-4
    assert got["relres"].max() <= 2e-5


@pytest.mark.parametrize("n,m,N,k", [(3000, 2600, 48, 2), (5000, 4500, 20, 1)])
def test_fp64_parity_global_vectors(lib, n, m, N, k):
    """m beyond the LDS room for the CG vectors (FP64: m > ~2000 at N = 48)."""
    p = W.random_problem(n, m, N, k, seed=1450 + N, tol=1e-12)
    say(f"case: columns fp64 global vectors n={n} m={m} N={N} k={k}")
    got = run(lib, p, "fp64", solver=3, want_z=True, want_iters=True, want_relres=True)
    ref = _cg(p)
    assert rel(got["Xa"], ref["Xa"]) <= 1e-10
    assert rel(got["Z"], ref["Z"]) <= 1e-10
    assert_iters_close(got["iters"], ref["iters"])


@pytest.mark.parametrize("n,m,N,k", [(9000, 8192, 64, 1), (6000, 5000, 100, 2)])
def test_mixed_parity_global_vectors(lib, n, m, N, k):
    p = W.random_problem(n, m, N, k, seed=1500 + N, tol=1e-6)
    say(f"case: columns mixed global vectors n={n} m={m} N={N} k={k}")
    got = run(lib, p, "mixed", solver=3, want_relres=True, want_iters=True)
    assert got["status"] == 0
    assert rel(got["Xa"], _chol(p)["Xa"]) <= 1e-4
    assert got["relres"].max() <= 1e-6


def test_global_vectors_in_place_and_repeatable(lib):
    import torch
    p = W.random_problem(9000, 8192, 64, 1, seed=1550, tol=1e-6)
    a = dev_problem(p, "fp32")
    ref = lib.analysis(**a, tol=p.tol, maxit=p.maxit, prec="fp32", solver=3)["Xa"].clone()
    again = lib.analysis(**a, tol=p.tol, maxit=p.maxit, prec="fp32", solver=3)["Xa"]
    torch.cuda.synchronize()
    assert torch.equal(ref, again)
    Xf_dev = a["Xf"].clone()
    a["Xf"] = Xf_dev
    lib.analysis(**a, tol=p.tol, maxit=p.maxit, prec="fp32", solver=3, out=Xf_dev)
    torch.cuda.synchronize()
    assert torch.equal(Xf_dev, ref)
