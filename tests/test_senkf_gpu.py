"""sEnKF (Section 2.4, Appendix A Algorithm 3) on the GPU through
cgd_senkf_analysis, against the oracle's sEnKF.

Bars: FP64 relative Frobenius 1e-12 (no iteration: only the rounding of the
row sums and the N x N products); FP32 1e-5 against the oracle run on the
same inputs rounded to FP32.  Shapes cover each padded width of the MFMA
path (32, 64, 128), ragged m (not a multiple of the 32-row chunks), m < N,
N = 2, and N past the MFMA range (the scalar FP64-sum path).
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import dev_problem, rel, rounded, say

pytestmark = pytest.mark.gpu

SHAPES = [
    # n, m, N, k
    (300, 257, 20, 2),
    (700, 1001, 33, 3),
    (2000, 3001, 100, 3),
    (4096, 2048, 64, 1),
    (500, 40, 128, 1),
    (64, 5, 2, 1),
    (400, 300, 129, 2),
    (350, 77, 160, 3),
]


def _senkf(p):
    return O.senkf(p.Xf, p.idx, p.w, p.y, p.r, p.eps)


def _run(lib, p, prec, **kw):
    out = lib.senkf_analysis(**dev_problem(p, prec), prec=prec, **kw)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("n,m,N,k", SHAPES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("stochastic", [True, False])
def test_senkf_shapes(lib, n, m, N, k, prec, stochastic):
    p = W.random_problem(n, m, N, k, seed=5 * n + m + N, stochastic=stochastic)
    say(f"case: senkf {prec} n={n} m={m} N={N} k={k} stochastic={stochastic}")
    out = _run(lib, p, prec, want_iters=True)
    assert out["status"] == 0
    assert out["stats"]["n_converged"] == N and out["stats"]["iters_max"] == 0
    assert int(out["iters"].abs().max()) == 0
    got = out["Xa"].double().cpu().numpy()
    if prec == "fp64":
        assert rel(got, _senkf(p)) <= 1e-12
    else:
        assert rel(got, _senkf(rounded(p))) <= 1e-5


def test_senkf_config2_full_size(lib):
    """The Lorenz-96 twin analysis at its full size (n = 4096, m = 2048,
    N = 64), FP32 and FP64."""
    p = W.L96Cycler().step(lambda q: q.Xf)
    for prec, bar in (("fp64", 1e-12), ("fp32", 1e-5)):
        say(f"case: senkf config2 {prec}")
        got = _run(lib, p, prec)["Xa"].double().cpu().numpy()
        assert rel(got, _senkf(p if prec == "fp64" else rounded(p))) <= bar


def test_senkf_config3_full_size(lib):
    """The 2-D advection-diffusion workload at its full size (n = 65536,
    m = 16384, N = 128, k = 4) in FP32, as the bench runs it: every tile of the
    N x N product and 74 row chunks."""
    p = W.config3()
    say("case: senkf config3 fp32")
    got = _run(lib, p, "fp32")["Xa"].double().cpu().numpy()
    assert rel(got, _senkf(rounded(p))) <= 1e-5


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_senkf_in_place_and_repeatable(lib, prec):
    p = W.random_problem(1500, 1200, 64, 2, seed=23)
    say(f"case: senkf in place {prec}")
    a = dev_problem(p, prec)
    first = lib.senkf_analysis(**a, prec=prec)["Xa"].clone()
    again = lib.senkf_analysis(**a, prec=prec)["Xa"]
    assert torch.equal(first, again)
    Xf = a["Xf"].clone()
    lib.senkf_analysis(**dict(a, Xf=Xf), prec=prec, out=Xf)
    torch.cuda.synchronize()
    assert torch.equal(Xf, first)


def test_senkf_exact_for_orthogonal_anomalies(lib):
    """Where Zhat Zhat^T is diagonal the sEnKF is the EnKF: the GPU sEnKF
    then meets the full CGD-EnKF analysis (and the oracle's Cholesky EnKF)."""
    import tests.test_oracle_pins_senkf as SP
    Xf, idx, w, y, r, eps = SP._orthogonal_anomaly_problem(3000, 40, 64, seed=7)
    p = W.Problem(Xf, idx.astype(np.int32), w, y, r, eps, 1e-12, 1000)
    say("case: senkf orthogonal anomalies")
    got = _run(lib, p, "fp64")["Xa"].double().cpu().numpy()
    ref = O.enkf_analysis(Xf, idx, w, y, r, eps)["Xa"]
    assert rel(got, ref) <= 1e-12


def test_senkf_errors(lib):
    p = W.random_problem(200, 100, 16, 2, seed=3)
    a = dev_problem(p, "fp32")
    say("case: senkf errors")
    bad = dict(a, idx=a["idx"].clone())
    bad["idx"][7, 1] = 200
    out = lib.senkf_analysis(**bad, prec="fp32", raise_on_error=False)
    assert out["status"] == -2                      # CGD_ERR_INDEX
    # the error does not leak into the next call on the same workspace
    ok = lib.senkf_analysis(**a, prec="fp32", workspace=out["workspace"])
    assert ok["status"] == 0
    for prec in ("mixed", "bf16split"):
        a2 = dev_problem(p, "fp32")
        out = lib.senkf_analysis(**a2, prec=prec, raise_on_error=False, stats=False)
        assert out["status"] == -7                  # CGD_ERR_UNSUPPORTED
    # a workspace below cgd_enkf_workspace_bytes(..., 1), through the C-ABI (the
    # binding would allocate a larger one)
    import ctypes
    n, N = a["Xf"].shape
    m, k = a["idx"].shape
    small = torch.empty(64, dtype=torch.uint8, device="cuda:0")
    opt = lib.Options()
    lib.load().cgd_options_default(ctypes.byref(opt))
    opt.prec = lib.PREC["fp32"]
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    st = lib.load().cgd_senkf_analysis(n, m, N, k, ptr(a["Xf"]), ptr(torch.empty_like(a["Xf"])),
                                       ptr(a["idx"]), ptr(a["w"]), ptr(a["y"]), ptr(a["r"]),
                                       ptr(a["eps"]), ctypes.byref(opt), ptr(small), 64, None,
                                       None)
    assert st == -5                                 # CGD_ERR_WORKSPACE


def test_senkf_neglects_observation_correlations(lib):
    """Example 2's setting (H = I, m = n = 2048, N = 64, tridiagonal R): the
    GPU sEnKF, which takes diag(R) only and every gain from the same X^f,
    meets the oracle's sEnKF and stays far from the oracle's EnKF with the
    full R (relative difference about 6.9 here; Sections 2.4 and 3.3)."""
    P, r_off = W.example2(n=2048, N=64, rep=0)
    say("case: senkf example2 tridiagonal R")
    a = dev_problem(P, "fp64")
    got_s = lib.senkf_analysis(**a, prec="fp64")["Xa"].double().cpu().numpy()
    ref_s = O.senkf(P.Xf, P.idx, P.w, P.y, P.r, P.eps)
    ref_e = O.enkf_analysis_R(P.Xf, P.idx, P.w, P.y, O.tridiag_R(P.r, r_off), P.eps)["Xa"]
    assert rel(got_s, ref_s) <= 1e-12
    assert rel(got_s, ref_e) > 1e-3


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_senkf_single_observation_is_the_enkf(lib, prec):
    """With one observation the diagonal of Psi is Psi (Appendix A): the GPU
    sEnKF meets the oracle's Cholesky EnKF."""
    p = W.random_problem(300, 1, 24, 3, seed=41)
    say(f"case: senkf m=1 {prec}")
    got = _run(lib, p, prec)["Xa"].double().cpu().numpy()
    q = p if prec == "fp64" else rounded(p)
    ref = O.enkf_analysis(q.Xf, q.idx, q.w, q.y, q.r, q.eps)["Xa"]
    assert rel(got, ref) <= (1e-12 if prec == "fp64" else 1e-5)


def test_senkf_validate(lib):
    """validate = 1 checks the inputs on the device before any launch of the
    analysis: r <= 0 gives CGD_ERR_NONPOS_R, a non-finite y CGD_ERR_NONFINITE."""
    p = W.random_problem(200, 100, 16, 2, seed=4)
    a = dev_problem(p, "fp64")
    say("case: senkf validate")
    bad = dict(a, r=a["r"].clone())
    bad["r"][5] = 0.0
    assert lib.senkf_analysis(**bad, prec="fp64", validate=True,
                              raise_on_error=False)["status"] == -3
    bad = dict(a, y=a["y"].clone())
    bad["y"][9] = float("nan")
    assert lib.senkf_analysis(**bad, prec="fp64", validate=True,
                              raise_on_error=False)["status"] == -4
    assert lib.senkf_analysis(**a, prec="fp64", validate=True)["status"] == 0
