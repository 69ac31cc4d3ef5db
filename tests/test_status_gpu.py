"""Status reporting and option handling through the C ABI: the reduced
mode's per-column status (a non-finite coefficient, convergence on the last
allowed step), the mixed mode's refinement period and its unsupported
warm-start fallback, and the per-member solvers beside a kernel on another
stream (cooperative launch: the result is right or the call fails)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import dev_problem, rel, run, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [20, 64, 200])
def test_reduced_nonfinite_is_an_error_without_validation(lib, prec, N):
    p = W.random_problem(300, 120, N, 2, seed=3000 + N, tol=1e-10)
    p.y[7] = np.nan
    say(f"case: reduced nonfinite y prec={prec} N={N}")
    out = lib.analysis(**dev_problem(p, prec), tol=1e-10, maxit=1000, prec=prec, reduced=True,
                       raise_on_error=False)
    assert out["status"] == -4


@pytest.mark.parametrize("N", [20, 64, 200])
def test_reduced_converged_on_the_last_allowed_step(lib, N):
    p = W.random_problem(300, 200, N, 2, seed=3100 + N, tol=1e-10)
    d = dev_problem(p, "fp64")
    say(f"case: reduced maxit = exact count N={N}")
    first = lib.analysis(**d, tol=1e-10, maxit=1000, prec="fp64", reduced=True, want_iters=True)
    its = first["iters"].cpu().numpy()
    assert first["status"] == 0
    exact = int(its.max())
    again = lib.analysis(**d, tol=1e-10, maxit=exact, prec="fp64", reduced=True, want_iters=True)
    assert again["status"] == 0, "a column converging on its maxit-th step is converged"
    assert again["stats"]["n_converged"] == N
    assert np.array_equal(again["iters"].cpu().numpy(), its)
    short = lib.analysis(**d, tol=1e-10, maxit=exact - 1, prec="fp64", reduced=True)
    assert short["status"] == 1


def test_mixed_refinement_period(lib):
    p = W.random_problem(3000, 2000, 64, 2, seed=3200, tol=1e-6)
    chol = O.enkf_analysis(p.Xf, p.idx, p.w, p.y, p.r, p.eps)
    d = dev_problem(p, "fp32")
    say("case: mixed rr_period")
    a = run(lib, p, "mixed", want_iters=True, want_relres=True)
    b = run(lib, p, "mixed", want_iters=True, want_relres=True, rr_period=3)
    for got in (a, b):
        assert got["status"] == 0
        assert rel(got["Xa"], chol["Xa"]) <= 1e-4
        assert got["relres"].max() <= 1e-6
    # at most three inner steps per refinement step: more outer steps, and a
    # different (not fewer-constrained) inner count
    assert not np.array_equal(a["iters"], b["iters"])


def test_mixed_warm_start_fallback_is_unsupported(lib):
    import torch
    p = W.random_problem(300, 200, 16, 1, seed=3300, tol=1e-6)
    d = dev_problem(p, "fp32")
    z0 = torch.zeros((p.m, p.N), dtype=torch.float32, device="cuda:0")
    say("case: mixed + z0 + fallback")
    out = lib.analysis(**d, tol=1e-6, maxit=100, prec="mixed", z0=z0, fallback_on_stall=True,
                       raise_on_error=False)
    assert out["status"] == -7
    ok = lib.analysis(**d, tol=1e-6, maxit=1000, prec="mixed", z0=z0, raise_on_error=False)
    assert ok["status"] == 0


@pytest.mark.parametrize("cooperative", [False, True])
@pytest.mark.parametrize("solver", [2, 3, 4, 5])
def test_per_member_solver_beside_another_stream(lib, solver, cooperative):
    """A matrix product runs on a second stream while the resident or a
    per-member solver (whose workgroups wait for each other) runs on the
    first.  A cooperative
    launch runs all workgroups together or is refused; a plain launch's
    start-up census fails fast (CGD_ERR_BUSY) when the grid is not resident.
    So the call returns the right X_a or an error, promptly, never a wait
    that runs out."""
    import time
    import torch
    p = W.random_problem(4096, 2048, 64, 1, seed=3400, tol=1e-6)
    d = dev_problem(p, "fp32")
    ref = lib.analysis(**d, tol=1e-6, maxit=1000, prec="fp32", solver=solver)["Xa"].clone()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    a = torch.randn(4096, 4096, device="cuda:0")
    say(f"case: solver {solver} beside a second stream")
    t0 = time.time()
    for _ in range(3):
        with torch.cuda.stream(side):
            for _ in range(8):
                a = torch.tanh(a @ a * 1e-3)
        out = lib.analysis(**d, tol=1e-6, maxit=1000, prec="fp32", solver=solver,
                           cooperative=cooperative, raise_on_error=False)
        torch.cuda.synchronize()
        assert out["status"] in (0, -6, -8), out["status"]
        if out["status"] == 0:
            assert torch.equal(out["Xa"], ref)
    assert time.time() - t0 < 20.0


@pytest.mark.parametrize("solver", [2, 3, 4, 5])
def test_census_timeout_fails_fast_and_leaves_the_workspace_usable(lib, solver):
    """A census wait of one tick (10 ns) makes the start-up check give up
    before the grid has checked in: every workgroup returns, the call reports
    CGD_ERR_BUSY with X_a untouched (or, if all arrived within the tick, the
    right result), and the next call on the same workspace is correct."""
    import torch
    p = W.random_problem(4096, 2048, 64, 1, seed=3500, tol=1e-6)
    d = dev_problem(p, "fp32")
    ref = lib.analysis(**d, tol=1e-6, maxit=1000, prec="fp32", solver=solver)
    torch.cuda.synchronize()
    say(f"case: census timeout solver {solver}")
    ws = ref["workspace"]
    seen = set()
    for _ in range(3):
        sentinel = torch.full_like(ref["Xa"], 7.0)
        out = lib.analysis(**d, tol=1e-6, maxit=1000, prec="fp32", solver=solver, census_ticks=1,
                           workspace=ws, raise_on_error=False, out=sentinel.clone())
        torch.cuda.synchronize()
        seen.add(out["status"])
        assert out["status"] in (0, -8), out["status"]
        if out["status"] == 0:
            assert torch.equal(out["Xa"], ref["Xa"])
        else:
            assert torch.equal(out["Xa"], sentinel)
        again = lib.analysis(**d, tol=1e-6, maxit=1000, prec="fp32", solver=solver, workspace=ws)
        torch.cuda.synchronize()
        assert again["status"] == 0 and torch.equal(again["Xa"], ref["Xa"])
    say(f"  statuses with a one-tick census: {sorted(seen)}")
