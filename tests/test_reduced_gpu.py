"""CGD-EnKF-Reduced (Algorithm 2) on the GPU: the MFMA path for N <= 128
(the N x 2N product over the observations, the N x N CG one wavefront per
column, the X_f W update) and the scalar path above it, against the FP64
oracle's direct (Cholesky) and CG solutions of the reduced system.

Bars: FP64 relative Frobenius 1e-10; FP32 1e-4 against the oracle run on the
same inputs rounded to FP32.  Shapes cover each padded width (32, 64, 128),
ragged m (not a multiple of the 32-row blocks or of the chunk), m < N, and
N past the MFMA range.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import dev_problem, rel, rounded, run, say

pytestmark = pytest.mark.gpu

SHAPES = [
    # n, m, N, k
    (300, 257, 20, 2),
    (700, 1001, 33, 3),
    (2000, 3001, 100, 3),
    (4096, 2048, 64, 1),
    (500, 40, 128, 1),
    (64, 5, 2, 1),
]


def _direct(p):
    return O.enkf_reduced(p.Xf, p.idx, p.w, p.y, p.r, p.eps)


@pytest.mark.parametrize("n,m,N,k", SHAPES)
def test_reduced_fp64_shapes(lib, n, m, N, k):
    p = W.random_problem(n, m, N, k, seed=7 * n + m, tol=1e-12)
    say(f"case: reduced fp64 n={n} m={m} N={N} k={k}")
    got = run(lib, p, "fp64", reduced=True, want_iters=True)
    ref = O.enkf_reduced(p.Xf, p.idx, p.w, p.y, p.r, p.eps, solver="cg", tol=1e-12, maxit=1000)
    assert got["status"] == 0
    assert rel(got["Xa"], ref["Xa"]) <= 1e-10
    assert rel(got["Xa"], _direct(p)["Xa"]) <= 1e-10
    # Lemma 1: at most N steps in exact arithmetic (N + 1 allows one for rounding)
    assert got["iters"].max() <= N + 1


@pytest.mark.parametrize("n,m,N,k", SHAPES)
@pytest.mark.parametrize("prec", ["fp32", "mixed"])
@pytest.mark.parametrize("tol", [1e-6, 1e-7])
def test_reduced_fp32_shapes(lib, n, m, N, k, prec, tol):
    """At the benches' tolerance (1e-6) and a tighter one."""
    p = W.random_problem(n, m, N, k, seed=7 * n + m + 1, tol=tol)
    say(f"case: reduced {prec} n={n} m={m} N={N} k={k} tol={tol}")
    got = run(lib, p, prec, reduced=True, tol=tol)
    assert got["status"] == 0
    assert rel(got["Xa"], _direct(rounded(p))["Xa"]) <= 1e-4


@pytest.mark.parametrize("prec,N", [("fp64", 129), ("fp32", 130)])
def test_reduced_past_mfma_range(lib, prec, N):
    """N > 128 runs the scalar path; same bars."""
    p = W.random_problem(400, 300, N, 2, seed=N, tol=1e-12)
    say(f"case: reduced {prec} N={N}")
    got = run(lib, p, prec, reduced=True, tol=1e-12 if prec == "fp64" else 1e-7)
    bar = 1e-10 if prec == "fp64" else 1e-4
    assert rel(got["Xa"], _direct(p if prec == "fp64" else rounded(p))["Xa"]) <= bar


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_reduced_in_place_and_repeatable(lib, prec):
    import torch
    p = W.random_problem(1500, 1200, 64, 2, seed=21, tol=1e-10)
    say(f"case: reduced in place {prec}")
    a = dev_problem(p, prec)
    first = lib.analysis(**a, reduced=True, tol=1e-10, prec=prec)["Xa"].clone()
    again = lib.analysis(**a, reduced=True, tol=1e-10, prec=prec)["Xa"]
    assert torch.equal(first, again)
    Xf = a["Xf"].clone()
    lib.analysis(**dict(a, Xf=Xf), reduced=True, tol=1e-10, prec=prec, out=Xf)
    torch.cuda.synchronize()
    assert torch.equal(Xf, first)


def test_reduced_workspace_reuse_smaller_then_larger(lib):
    """One workspace serves shapes of decreasing size without stale data."""
    import torch
    big = W.random_problem(900, 1031, 128, 4, seed=31, tol=1e-12)
    small = W.random_problem(300, 257, 20, 2, seed=32, tol=1e-12)
    need = lib.workspace_bytes(900, 1031, 128, 4, "fp64", reduced=True)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    for p in (big, small, big):
        out = lib.analysis(**dev_problem(p, "fp64"), reduced=True, tol=1e-12, prec="fp64",
                           workspace=ws)
        torch.cuda.synchronize()
        assert rel(out["Xa"].cpu().numpy(), _direct(p)["Xa"]) <= 1e-10


def test_reduced_bad_index_reported(lib):
    p = W.random_problem(200, 100, 32, 2, seed=33)
    for prec in ("fp64", "fp32"):
        a = dev_problem(p, prec)
        a["idx"] = a["idx"].clone()
        a["idx"][17, 1] = 200
        assert lib.analysis(**a, reduced=True, prec=prec, raise_on_error=False)["status"] == -2


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("fp32", 1e-7), ("fp64", 1e-12)])
def test_reduced_config3(lib, prec, tol):
    """The 2-D advection-diffusion workload (n = 65536, m = 16384, N = 128,
    k = 4): every tile of the N x 2N product, 74 row chunks; FP32 at the
    bench's tolerance (1e-6) and a tighter one."""
    p = W.config3()
    say(f"case: reduced config3 {prec} tol={tol}")
    got = run(lib, p, prec, reduced=True, tol=tol, maxit=1000, want_iters=True)
    assert got["status"] == 0
    ref = _direct(p if prec == "fp64" else rounded(p))
    assert rel(got["Xa"], ref["Xa"]) <= (1e-10 if prec == "fp64" else 1e-4)
    assert got["iters"].max() <= p.N + 1
