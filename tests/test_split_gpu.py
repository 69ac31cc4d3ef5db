"""The split per-member solver (solver=4: P workgroups per member, each with
a slice of S in LDS, partial sums exchanged through flag-in-word slots once
per pass, the update applied per member column) against the oracle."""
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


def _info(lib, p, prec, solver=0):
    return lib.Plan(p.n, p.m, p.N, p.k, prec=prec, solver=solver).solver_info()


# (n, m, N, k): N a multiple of 8 (parts of a member kept on one XCD) and not,
# every padded width, ragged slices (m not a multiple of P or of the row step)
CASES64 = [(600, 600, 40, 1), (500, 300, 33, 3), (300, 257, 16, 2), (200, 150, 5, 1),
           (900, 1000, 32, 2)]


@pytest.mark.parametrize("n,m,N,k", CASES64)
def test_fp64_parity(lib, n, m, N, k):
    p = W.random_problem(n, m, N, k, seed=1300 + m + N, tol=1e-12)
    info = _info(lib, p, "fp64", solver=4)
    say(f"case: split fp64 n={n} m={m} N={N} k={k}: {info}")
    got = run(lib, p, "fp64", solver=4, want_z=True, want_iters=True, want_relres=True)
    assert got["status"] in (0, 1)
    ref = _cg(p)
    assert rel(got["Xa"], ref["Xa"]) <= 1e-10
    assert rel(got["Z"], ref["Z"]) <= 1e-10
    assert_iters_close(got["iters"], ref["iters"])
    assert got["relres"].max() <= 1e-11


@pytest.mark.parametrize("maxit", [0, 1, 6])
def test_fp64_fixed_iterations(lib, maxit):
    p = W.random_problem(500, 333, 24, 2, seed=17, tol=1e-12)
    say(f"case: split fp64 fixed maxit={maxit}")
    got = run(lib, p, "fp64", solver=4, tol=0.0, maxit=maxit, want_z=True, want_iters=True)
    ref = _cg(p, tol=0.0, maxit=maxit)
    assert np.all(got["iters"] == maxit)
    assert rel(got["Z"], ref["Z"]) <= 1e-12
    assert rel(got["Xa"], ref["Xa"]) <= 1e-12
    if maxit == 0:
        assert np.array_equal(got["Xa"], p.Xf)


@pytest.mark.parametrize("n,m,N,k", [(4096, 2048, 64, 1), (3000, 2500, 48, 2), (700, 513, 33, 1),
                                     (5000, 4096, 16, 2)])
def test_fp32_parity(lib, n, m, N, k):
    p = W.random_problem(n, m, N, k, seed=1350 + N, tol=1e-6)
    info = _info(lib, p, "fp32", solver=4)
    say(f"case: split fp32 n={n} m={m} N={N} k={k}: {info}")
    got = run(lib, p, "fp32", solver=4, want_relres=True, want_iters=True)
    assert got["status"] == 0
    assert rel(got["Xa"], _chol(p)["Xa"]) <= 1e-4
    assert got["relres"].max() <= 2e-5
    # the same recurrence as the single-workgroup column solver, summed in
    # another order.  In FP32 (u = 2^-24) the two recursive residuals differ
    # by rounding from the first step on and flatten out near a 1e-6 stop
    # threshold, so a member's first crossing moves by a few iterations:
    # allow max(4, 10%) per member and under one iteration on average.
    col = run(lib, p, "fp32", solver=3, want_iters=True)
    d = got["iters"].astype(np.int64) - col["iters"].astype(np.int64)
    say(f"  iterations split {got['iters'].max()} / columns {col['iters'].max()}, "
        f"largest member difference {np.abs(d).max()}")
    assert np.abs(d).max() <= max(4, int(np.ceil(0.1 * col["iters"].max())))
    assert abs(d.mean()) <= 1.0


def test_config2_cycle_auto_choice_and_repeatability(lib):
    """One Lorenz-96 twin-experiment analysis at its real size: the automatic
    choice runs the split solver there, bitwise repeatably."""
    cyc = W.L96Cycler(tol=1e-6, maxit=1000)
    p = cyc.problem()
    info = _info(lib, p, "fp32")
    say(f"case: split config2 auto choice {info}")
    assert info["solver"] == "k_cg_split"
    got = run(lib, p, "fp32", want_relres=True)
    assert got["status"] == 0
    assert rel(got["Xa"], _chol(p)["Xa"]) <= 1e-4
    assert got["relres"].max() <= 2e-5
    b = run(lib, p, "fp32")
    assert np.array_equal(got["Xa"], b["Xa"])
    # smaller m: the column solver streams little of S, and stays the choice
    q = W.random_problem(2048, 1024, 64, 1, seed=3)
    assert _info(lib, q, "fp32")["solver"] == "k_cg_columns"


def test_warm_start_and_fallback(lib):
    import torch
    p = W.random_problem(300, 300, 16, 2, seed=12, tol=1e-10)
    S = O.obs_anomalies(p.idx, p.w, p.Xf)
    D = O.innovations(p.idx, p.w, p.Xf, p.y, p.eps)
    zs = np.ascontiguousarray(O.solve_cholesky(O.innovation_matrix(S, p.r), D))
    a = dev_problem(p, "fp64")
    for z0, expect_fb in ((-10 * zs, True), (zs * (1 + 1e-6), False)):
        say(f"case: split warm start, fallback expected={expect_fb}")
        out = lib.analysis(**a, tol=p.tol, maxit=p.maxit, prec="fp64", solver=4,
                           z0=torch.as_tensor(np.ascontiguousarray(z0), device="cuda:0"),
                           fallback_on_stall=True, want_z=True, want_iters=True)
        torch.cuda.synchronize()
        ref = O.solve_cg_columns(O.matvec_free(S, p.r), D, p.tol, p.maxit, Z0=z0,
                                 fallback_on_stall=True)
        assert (out["stats"]["n_fallbacks"] == p.N) == expect_fb
        assert rel(out["Z"].cpu().numpy(), ref[0]) <= 1e-10
        assert np.max(np.abs(out["iters"].cpu().numpy() - ref[1])) <= 2
        Zg = out["Z"].cpu().numpy()
        Xa_own = p.Xf + (p.Xf - p.Xf.mean(1, keepdims=True)) @ (S.T @ Zg) / (p.N - 1)
        assert rel(out["Xa"].cpu().numpy(), Xa_own) <= 1e-12


def test_in_place(lib):
    """X_a aliasing X_f: the gather runs in a launch of its own and each
    update tile reads its rows of X_f just before writing them, so the
    split solver runs in place and gives the out-of-place result."""
    import torch
    p = W.random_problem(4096, 2048, 64, 1, seed=23, tol=1e-6)
    a = dev_problem(p, "fp32")
    ref = lib.analysis(**a, tol=p.tol, maxit=p.maxit, prec="fp32", solver=4)["Xa"].clone()
    Xf_dev = a["Xf"].clone()
    a["Xf"] = Xf_dev
    out = lib.analysis(**a, tol=p.tol, maxit=p.maxit, prec="fp32", solver=4, out=Xf_dev)
    torch.cuda.synchronize()
    assert out["Xa"].data_ptr() == Xf_dev.data_ptr()
    assert torch.equal(Xf_dev, ref)
    assert rel(Xf_dev.double().cpu().numpy(), _chol(p)["Xa"]) <= 1e-4


def test_bad_index_reported(lib):
    p = W.random_problem(300, 200, 16, 2, seed=15)
    a = dev_problem(p, "fp64")
    a["idx"] = a["idx"].clone()
    a["idx"][5, 1] = 300
    a["idx"][190, 0] = -3
    out = lib.analysis(**a, solver=4, raise_on_error=False)
    assert out["status"] == -2


@pytest.mark.parametrize("solver", [3, 4])
def test_error_word_cleared_for_the_next_call(lib, solver):
    """The gather launch clears the error word each call: a bad call, then a
    good one on the same workspace, reports the good one clean."""
    import torch
    p = W.random_problem(300, 200, 16, 2, seed=16, tol=1e-10)
    good = dev_problem(p, "fp64")
    bad = dict(good)
    bad["idx"] = good["idx"].clone()
    bad["idx"][7, 0] = 10 ** 6
    first = lib.analysis(**bad, solver=solver, raise_on_error=False)
    assert first["status"] == -2
    out = lib.analysis(**good, solver=solver, tol=1e-10, workspace=first["workspace"],
                       raise_on_error=False)
    torch.cuda.synchronize()
    assert out["status"] == 0
    ref = O.enkf_analysis(p.Xf, p.idx, p.w, p.y, p.r, p.eps, solver="cg_free", tol=1e-10,
                          maxit=p.maxit)
    assert rel(out["Xa"].cpu().numpy(), ref["Xa"]) <= 1e-10


def test_unsupported_shapes(lib):
    # N above 64; FP64 with N = 64 and m = 4096 (no slice fits with N * P <= 256)
    for (n, m, N, prec) in ((200, 100, 65, "fp32"), (5000, 4096, 64, "fp64")):
        p = W.random_problem(n, m, N, 1, seed=3)
        out = lib.analysis(**dev_problem(p, prec), prec=prec, solver=4, raise_on_error=False)
        assert out["status"] == -7, (n, m, N, prec)
