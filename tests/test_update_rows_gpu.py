"""The ensemble update that reads X_f straight into the MFMA's registers
(large n: at least 32768 state rows, N a multiple of the 16-byte vector),
through the analyses that end in it: the reduced mode and the sEnKF
(X_f + X_f (W - I)), and the row-block x member-group solver's analysis
(X_f + A W, rows centred by the kernel).  Against the oracle; n = 40003 leaves
a ragged last 16-row block, the shapes cover every padded width, and an N
that is not a multiple of 4 takes the LDS-tiled update instead.

Bars: FP64 relative Frobenius 1e-10 (1e-12 for the sEnKF), FP32 1e-4
(1e-5 for the sEnKF), against the oracle on the same rounded inputs.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import dev_problem, rel, rounded, run, say

pytestmark = pytest.mark.gpu

N_ROWS = 40003


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [16, 32, 64, 100, 128, 30])
def test_reduced_large_n(lib, prec, N):
    p = W.random_problem(N_ROWS, 300, N, 2, seed=N + 3)
    say(f"case: update rows, reduced {prec} n={N_ROWS} N={N}")
    got = run(lib, p, prec, reduced=True, tol=1e-12 if prec == "fp64" else 1e-7)
    q = p if prec == "fp64" else rounded(p)
    ref = O.enkf_reduced(q.Xf, q.idx, q.w, q.y, q.r, q.eps)["Xa"]
    assert got["status"] == 0
    assert rel(got["Xa"], ref) <= (1e-10 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [32, 128, 30])
def test_senkf_large_n(lib, prec, N):
    p = W.random_problem(N_ROWS, 500, N, 3, seed=N + 5)
    say(f"case: update rows, sEnKF {prec} n={N_ROWS} N={N}")
    a = dev_problem(p, prec)
    got = lib.senkf_analysis(**a, prec=prec)["Xa"].double().cpu().numpy()
    q = p if prec == "fp64" else rounded(p)
    ref = O.senkf(q.Xf, q.idx, q.w, q.y, q.r, q.eps)
    assert rel(got, ref) <= (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("N", [64, 100, 128])
def test_tile_solver_update_large_n(lib, N):
    """FP32 row-block x member-group solver (its update is a launch of its
    own, mode 0) at n = 40003."""
    p = W.random_problem(N_ROWS, 2100, N, 2, seed=N + 9, tol=1e-6)
    say(f"case: update rows, tile solver fp32 n={N_ROWS} N={N}")
    got = run(lib, p, "fp32", solver=5, tol=1e-6)
    q = rounded(p)
    ref = O.enkf_analysis(q.Xf, q.idx, q.w, q.y, q.r, q.eps)["Xa"]
    assert got["status"] == 0
    assert rel(got["Xa"], ref) <= 1e-4


def test_in_place_large_n(lib):
    """X_a aliasing X_f: the same result as a separate output."""
    p = W.random_problem(N_ROWS, 300, 64, 2, seed=77)
    say("case: update rows in place")
    a = dev_problem(p, "fp32")
    sep = lib.analysis(**a, reduced=True, tol=1e-7, prec="fp32")["Xa"].clone()
    Xf = a["Xf"].clone()
    lib.analysis(**dict(a, Xf=Xf), reduced=True, tol=1e-7, prec="fp32", out=Xf)
    torch.cuda.synchronize()
    assert torch.equal(Xf, sep)
