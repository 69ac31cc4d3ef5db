"""The 2-D advection-diffusion workload at its full size (n = 65536,
m = 16384 bilinear observations, N = 128, diag R ~ U[0.5, 2]) against the
FP64 oracle's textbook CG at the same stop rule."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import rel, run, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfg3():
    p = W.config3()
    ref = O.enkf_analysis(p.Xf, p.idx, p.w, p.y, p.r, p.eps, solver="cg_free", tol=p.tol,
                          maxit=p.maxit)
    return p, ref


@pytest.mark.parametrize("solver", [0, 1, 3])
def test_config3_fp32(lib, cfg3, solver):
    p, ref = cfg3
    say(f"case: config3 fp32 solver={solver}")
    got = run(lib, p, "fp32", solver=solver, want_relres=True, want_iters=True)
    assert got["status"] == 0
    err = rel(got["Xa"], ref["Xa"])
    say(f"  iters {got['iters'].min()}..{got['iters'].max()} (oracle {ref['iters'].min()}.."
        f"{ref['iters'].max()}), X_a vs FP64 CG {err:.2e}, true rel. residual "
        f"{got['relres'].max():.2e}")
    assert err <= 1e-4
    # FP32 floor of the true residual (recursive residual stops at 1e-6)
    assert got["relres"].max() <= 2e-5
    # FP32 rounding costs some conjugacy: a few more iterations than FP64, never fewer
    # than FP64 less rounding slack
    it, it64 = int(got["iters"].max()), int(ref["iters"].max())
    assert it64 - 2 <= it <= 1.15 * it64 + 2


@pytest.mark.parametrize("solver", [5, 3])
def test_config3_mixed(lib, cfg3, solver):
    """The mixed mode on the workload it is specified for: BF16 copy of S in
    the inner CG, FP32 accumulation, FP64-accumulated outer residual (the
    row-block x member-group solver, the automatic choice, and the column
    solver with its vectors in global memory, N = 128)."""
    p, ref = cfg3
    say(f"case: config3 mixed solver={solver}")
    got = run(lib, p, "mixed", solver=solver, want_relres=True, want_iters=True)
    assert got["status"] == 0
    err = rel(got["Xa"], ref["Xa"])
    say(f"  inner iterations {got['iters'].min()}..{got['iters'].max()}, X_a vs FP64 CG {err:.2e}, "
        f"true rel. residual {got['relres'].max():.2e}")
    assert err <= 1e-4
    # the outer stop test is on the FP64-accumulated true residual
    assert got["relres"].max() <= 1e-6


def test_config3_bf16split(lib, cfg3):
    """Split-BF16 products (five BF16 MFMA products per S-product) on the
    2-D workload: the FP32 bar, with iteration counts close to FP32's."""
    p, ref = cfg3
    say("case: config3 bf16split")
    got = run(lib, p, "bf16split", want_relres=True, want_iters=True)
    assert got["status"] == 0
    err = rel(got["Xa"], ref["Xa"])
    say(f"  iters {got['iters'].min()}..{got['iters'].max()} (oracle {ref['iters'].max()}), "
        f"X_a vs FP64 CG {err:.2e}, true rel. residual {got['relres'].max():.2e}")
    assert err <= 1e-4
    it, it64 = int(got["iters"].max()), int(ref["iters"].max())
    assert it64 - 2 <= it <= 1.2 * it64 + 2
