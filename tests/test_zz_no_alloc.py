"""cgd_enkf_analysis_static (static scratch, no allocation) against
cgd_enkf_analysis (caller workspace) through the C ABI: two calls in a row,
the second on a smaller problem, each bitwise equal to the workspace call
(same kernels, deterministic order), and the FP64 result within 1e-10 of the
oracle; sizes beyond the scratch are refused before any launch."""
import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import dev_problem, rel, say

pytestmark = pytest.mark.gpu


def _static_sig(lib):
    L = lib.load()
    vp, ci, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.cgd_enkf_analysis_static.argtypes = [ci, ci, ci, ci, vp, vp, vp, vp, vp, vp, vp, cd, ci,
                                           ctypes.POINTER(lib.Options), ctypes.POINTER(lib.Stats),
                                           vp]
    L.cgd_enkf_analysis_static.restype = ci
    L.cgd_enkf_static_scratch_bytes.restype = ctypes.c_size_t
    return L


def _call_static(lib, L, d, prec, tol, maxit):
    import torch
    n, N = d["Xf"].shape
    m, k = d["idx"].shape
    Xa = torch.empty_like(d["Xf"])
    iters = torch.empty(N, dtype=torch.int32, device=d["Xf"].device)
    opt = lib.Options()
    L.cgd_options_default(ctypes.byref(opt))
    opt.prec = lib.PREC[prec]
    opt.iters_out = iters.data_ptr()
    st = lib.Stats()
    p = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
    status = L.cgd_enkf_analysis_static(n, m, N, k, p(d["Xf"]), p(Xa), p(d["idx"]), p(d["w"]),
                                        p(d["y"]), p(d["r"]), p(d["eps"]), tol, maxit,
                                        ctypes.byref(opt), ctypes.byref(st),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return status, Xa, iters, st


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_static_scratch_matches_workspace_call(lib, prec):
    import torch
    L = _static_sig(lib)
    big = W.random_problem(4096, 2048, 64, 1, seed=4100, tol=1e-10 if prec == "fp64" else 1e-6)
    small = W.config1()
    for p in (big, small):   # the second call is on a smaller problem
        tol = 1e-10 if prec == "fp64" else 1e-6
        d = dev_problem(p, prec)
        say(f"case: static scratch prec={prec} n={p.Xf.shape[0]} m={p.m} N={p.N}")
        status, Xa, iters, st = _call_static(lib, L, d, prec, tol, 1000)
        torch.cuda.synchronize()
        assert status == 0, status
        ref = lib.analysis(**d, tol=tol, maxit=1000, prec=prec, want_iters=True)
        torch.cuda.synchronize()
        assert torch.equal(Xa, ref["Xa"])
        assert torch.equal(iters, ref["iters"])
        assert st.iters_max == ref["stats"]["iters_max"]
        if prec == "fp64":
            orc = O.enkf_analysis(p.Xf, p.idx, p.w, p.y, p.r, p.eps, solver="cg_free", tol=tol,
                                  maxit=1000)
            assert rel(Xa.cpu().numpy(), orc["Xa"]) <= 1e-10


def test_static_scratch_refuses_sizes_beyond_it(lib):
    L = _static_sig(lib)
    cap = int(L.cgd_enkf_static_scratch_bytes())
    assert cap == 32 << 20
    # n = 65536, m = 16384, N = 128 in FP32 needs ~335 MiB: refused before any launch
    need = lib.workspace_bytes(65536, 16384, 128, 4, "fp32")
    assert need > cap
    opt = lib.Options()
    L.cgd_options_default(ctypes.byref(opt))
    opt.prec = lib.PREC["fp32"]
    dummy = ctypes.c_void_p(256)   # never dereferenced: the size check comes first
    status = L.cgd_enkf_analysis_static(65536, 16384, 128, 4, dummy, dummy, dummy, dummy, dummy,
                                        dummy, None, 1e-6, 100, ctypes.byref(opt), None, None)
    assert status == -5
