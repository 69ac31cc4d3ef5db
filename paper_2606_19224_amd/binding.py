"""Thin ctypes binding of libcgd_enkf.so (argument marshalling only).

Every step of the analysis runs in the library's HIP kernels; PyTorch only
provides device memory (tensors, the workspace) and the current stream.
Importing this module on a machine without the built library raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os
from typing import Optional

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcgd_enkf.so")

CGD_FP64, CGD_FP32, CGD_MIXED_BF16, CGD_BF16_SPLIT = 0, 1, 2, 3
PREC = {"fp64": CGD_FP64, "fp32": CGD_FP32, "mixed": CGD_MIXED_BF16, "bf16": CGD_MIXED_BF16,
        "bf16split": CGD_BF16_SPLIT}
STATUS = {0: "CGD_OK", 1: "CGD_NOT_CONVERGED", -1: "CGD_ERR_ARG", -2: "CGD_ERR_INDEX",
          -3: "CGD_ERR_NONPOS_R", -4: "CGD_ERR_NONFINITE", -5: "CGD_ERR_WORKSPACE",
          -6: "CGD_ERR_HIP", -7: "CGD_ERR_UNSUPPORTED", -8: "CGD_ERR_BUSY"}


PRECOND = {None: 0, "none": 0, "diag_r": 1}


class Tuning(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int), ("solver", ctypes.c_int),
                ("rows_per_block", ctypes.c_int), ("prof_events", ctypes.c_void_p),
                ("trace", ctypes.c_void_p), ("cooperative", ctypes.c_int),
                ("census_ticks", ctypes.c_uint)]


class Options(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("precond", ctypes.c_int), ("rr_period", ctypes.c_int),
                ("z0", ctypes.c_void_p), ("fallback_on_stall", ctypes.c_int),
                ("z_out", ctypes.c_void_p), ("iters_out", ctypes.c_void_p),
                ("relres_out", ctypes.c_void_p), ("validate", ctypes.c_int),
                ("r_factor", ctypes.c_void_p), ("tuning", ctypes.POINTER(Tuning))]


class Stats(ctypes.Structure):
    _fields_ = [("iters_max", ctypes.c_int), ("iters_min", ctypes.c_int),
                ("n_converged", ctypes.c_int), ("n_fallbacks", ctypes.c_int),
                ("relres_max", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_19224_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ci, cd, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    sig = [ci, ci, ci, ci, vp, vp, vp, vp, vp, vp, vp, cd, ci, ctypes.POINTER(Options), vp, sz,
           ctypes.POINTER(Stats), vp]
    for name in ("cgd_enkf_analysis", "cgd_enkf_reduced_analysis"):
        f = getattr(lib, name)
        f.argtypes = sig
        f.restype = ci
    lib.cgd_senkf_analysis.argtypes = sig[:11] + sig[13:]
    lib.cgd_senkf_analysis.restype = ci
    lib.cgd_enkf_workspace_bytes.argtypes = [ci, ci, ci, ci, ci, ci]
    lib.cgd_enkf_workspace_bytes.restype = sz
    lib.cgd_status_string.argtypes = [ci]
    lib.cgd_status_string.restype = ctypes.c_char_p
    lib.cgd_version.restype = ctypes.c_char_p
    lib.cgd_options_default.argtypes = [ctypes.POINTER(Options)]
    ip = ctypes.POINTER(ci)
    lib.cgd_enkf_solver_info.argtypes = [ci, ci, ci, ci, ctypes.POINTER(Options), ip, ip, ip]
    lib.cgd_enkf_solver_info.restype = ci
    _lib = lib
    return lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(t: torch.Tensor, name: str, dtype, shape, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def workspace_bytes(n, m, N, k, prec="fp64", reduced=False, tridiag=False) -> int:
    mode = (1 if reduced else 0) | (2 if tridiag else 0)
    return int(load().cgd_enkf_workspace_bytes(n, m, N, k, PREC[prec], mode))


def tridiag_cholesky(r_diag: torch.Tensor, r_off: torch.Tensor, prec: str = "fp64",
                     stream=None) -> torch.Tensor:
    """Cholesky factor of the symmetric tridiagonal R (cgd_tridiag_cholesky):
    a device tensor of 2m-1 values (diag(L), then L[i+1][i]) for r_factor."""
    lib = load()
    lib.cgd_tridiag_cholesky.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    lib.cgd_tridiag_cholesky.restype = ctypes.c_int
    m = r_diag.shape[0]
    dt = torch.float64 if prec == "fp64" else torch.float32
    _check(r_diag, "r_diag", dt, (m,), r_diag.device)
    _check(r_off, "r_off", dt, (max(m - 1, 0),), r_diag.device)
    out = torch.empty(2 * m - 1, dtype=dt, device=r_diag.device)
    if stream is None:
        stream = torch.cuda.current_stream(r_diag.device)
    st = lib.cgd_tridiag_cholesky(m, _ptr(r_diag), _ptr(r_off), _ptr(out), PREC[prec],
                                  ctypes.c_void_p(stream.cuda_stream))
    if st < 0:
        raise CGDError(st, "cgd_tridiag_cholesky")
    return out


class CGDError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where} returned {STATUS.get(status, status)}")
        self.status = status


def analysis(Xf: torch.Tensor, idx: torch.Tensor, w: torch.Tensor, y: torch.Tensor,
             r: torch.Tensor, eps: Optional[torch.Tensor] = None, tol: float = 1e-6,
             maxit: int = 1000, prec: str = "fp64", reduced: bool = False,
             z0: Optional[torch.Tensor] = None, fallback_on_stall: bool = False,
             want_z: bool = False, want_iters: bool = False, want_relres: bool = False,
             stats: bool = True, grid: int = 0, validate: bool = False, rr_period: int = 0,
             out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
             stream=None, raise_on_error: bool = True, prof_events=None, solver: int = 0,
             rows_per_block: int = 0, trace: Optional[torch.Tensor] = None,
             precond: Optional[str] = None, cooperative: bool = False,
             census_ticks: int = 0, r_factor: Optional[torch.Tensor] = None) -> dict:
    """One CGD-EnKF (or CGD-EnKF-Reduced) analysis on the GPU.

    Xf n x N, idx/w m x k, y/r m, eps m x N (or None), all on one CUDA device,
    contiguous; values float64 for prec='fp64', float32 otherwise; idx int32.
    Returns {'Xa', 'Z', 'iters', 'relres', 'stats', 'status'}.
    """
    lib = load()
    n, N = Xf.shape
    m, k = idx.shape
    dev = Xf.device
    vdt = torch.float64 if prec == "fp64" else torch.float32
    _check(Xf, "Xf", vdt, (n, N), dev)
    _check(idx, "idx", torch.int32, (m, k), dev)
    _check(w, "w", vdt, (m, k), dev)
    _check(y, "y", vdt, (m,), dev)
    _check(r, "r", vdt, (m,), dev)
    if eps is not None:
        _check(eps, "eps", vdt, (m, N), dev)
    if z0 is not None:
        _check(z0, "z0", vdt, (m, N), dev)
    Xa = out if out is not None else torch.empty_like(Xf)
    _check(Xa, "out", vdt, (n, N), dev)
    if r_factor is not None:
        _check(r_factor, "r_factor", vdt, (2 * m - 1,), dev)
    need = workspace_bytes(n, m, N, k, prec, reduced, r_factor is not None)
    if need == 0:
        raise CGDError(-1, "cgd_enkf_workspace_bytes")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    Z = torch.empty((m, N), dtype=vdt, device=dev) if want_z else None
    iters = torch.empty(N, dtype=torch.int32, device=dev) if want_iters else None
    relres = torch.empty(N, dtype=torch.float64, device=dev) if want_relres else None
    tuning = Tuning(grid, solver, rows_per_block,
                    None if prof_events is None else prof_events.address(), _ptr(trace),
                    1 if cooperative else 0, census_ticks)
    opt = Options(PREC[prec], PRECOND[precond], rr_period, _ptr(z0),
                  1 if fallback_on_stall else 0, _ptr(Z), _ptr(iters), _ptr(relres),
                  1 if validate else 0, _ptr(r_factor), ctypes.pointer(tuning))
    st = Stats()
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    fn = lib.cgd_enkf_reduced_analysis if reduced else lib.cgd_enkf_analysis
    status = fn(n, m, N, k, _ptr(Xf), _ptr(Xa), _ptr(idx), _ptr(w), _ptr(y), _ptr(r), _ptr(eps),
                float(tol), int(maxit), ctypes.byref(opt), _ptr(workspace), workspace.numel(),
                ctypes.byref(st) if stats else None, ctypes.c_void_p(stream.cuda_stream))
    if raise_on_error and status < 0:
        raise CGDError(status, fn.__name__)
    return {"Xa": Xa, "Z": Z, "iters": iters, "relres": relres,
            "stats": st.as_dict() if stats else None, "status": status, "workspace": workspace}


def senkf_analysis(Xf: torch.Tensor, idx: torch.Tensor, w: torch.Tensor, y: torch.Tensor,
                   r: torch.Tensor, eps: Optional[torch.Tensor] = None, prec: str = "fp64",
                   want_iters: bool = False, stats: bool = True, validate: bool = False,
                   out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                   stream=None, raise_on_error: bool = True, prof_events=None) -> dict:
    """One sEnKF analysis on the GPU (cgd_senkf_analysis: Appendix A,
    Algorithm 3, diag(R) = r only).  Arguments as for analysis(); prec 'fp64'
    or 'fp32'.  Returns {'Xa', 'iters', 'stats', 'status', 'workspace'}."""
    lib = load()
    n, N = Xf.shape
    m, k = idx.shape
    dev = Xf.device
    vdt = torch.float64 if prec == "fp64" else torch.float32
    _check(Xf, "Xf", vdt, (n, N), dev)
    _check(idx, "idx", torch.int32, (m, k), dev)
    _check(w, "w", vdt, (m, k), dev)
    _check(y, "y", vdt, (m,), dev)
    _check(r, "r", vdt, (m,), dev)
    if eps is not None:
        _check(eps, "eps", vdt, (m, N), dev)
    Xa = out if out is not None else torch.empty_like(Xf)
    _check(Xa, "out", vdt, (n, N), dev)
    need = workspace_bytes(n, m, N, k, prec, reduced=True)
    if need == 0:
        raise CGDError(-1, "cgd_enkf_workspace_bytes")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    iters = torch.full((N,), -1, dtype=torch.int32, device=dev) if want_iters else None
    tuning = Tuning(0, 0, 0, None if prof_events is None else prof_events.address(), None, 0, 0)
    opt = Options(PREC[prec], 0, 0, None, 0, None, _ptr(iters), None, 1 if validate else 0, None,
                  ctypes.pointer(tuning))
    st = Stats()
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    status = lib.cgd_senkf_analysis(n, m, N, k, _ptr(Xf), _ptr(Xa), _ptr(idx), _ptr(w), _ptr(y),
                                    _ptr(r), _ptr(eps), ctypes.byref(opt), _ptr(workspace),
                                    workspace.numel(), ctypes.byref(st) if stats else None,
                                    ctypes.c_void_p(stream.cuda_stream))
    if raise_on_error and status < 0:
        raise CGDError(status, "cgd_senkf_analysis")
    return {"Xa": Xa, "iters": iters, "stats": st.as_dict() if stats else None, "status": status,
            "workspace": workspace}


def gain_analysis(Xf: torch.Tensor, idx: torch.Tensor, w: torch.Tensor, y: torch.Tensor,
                  r: torch.Tensor, eps: Optional[torch.Tensor] = None, tol: float = 1e-6,
                  maxit: int = 1000, prec: str = "fp64", want_kt: bool = False,
                  want_hist: bool = False, want_iters: bool = False, stats: bool = True,
                  validate: bool = False, out: Optional[torch.Tensor] = None,
                  workspace: Optional[torch.Tensor] = None, stream=None,
                  raise_on_error: bool = True, prof_events=None) -> dict:
    """The explicit-gain form of Figure 2 on the GPU (cgd_enkf_gain_analysis):
    one CG per column of K^T.  Arguments as for analysis(); prec 'fp64' or
    'fp32', N <= 128.  Returns {'Xa', 'KT' (m x n), 'hist' (maxit x n:
    alpha_t ||r_t||^2 per column and step), 'iters' (n), 'stats', 'status',
    'workspace'}."""
    lib = load()
    f = lib.cgd_enkf_gain_analysis
    vp, ci, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    f.argtypes = [ci, ci, ci, ci, vp, vp, vp, vp, vp, vp, vp, cd, ci, ctypes.POINTER(Options), vp,
                  vp, vp, ctypes.c_size_t, ctypes.POINTER(Stats), vp]
    f.restype = ci
    lib.cgd_enkf_gain_workspace_bytes.argtypes = [ci, ci, ci, ci, ci]
    lib.cgd_enkf_gain_workspace_bytes.restype = ctypes.c_size_t
    n, N = Xf.shape
    m, k = idx.shape
    dev = Xf.device
    vdt = torch.float64 if prec == "fp64" else torch.float32
    _check(Xf, "Xf", vdt, (n, N), dev)
    _check(idx, "idx", torch.int32, (m, k), dev)
    _check(w, "w", vdt, (m, k), dev)
    _check(y, "y", vdt, (m,), dev)
    _check(r, "r", vdt, (m,), dev)
    if eps is not None:
        _check(eps, "eps", vdt, (m, N), dev)
    Xa = out if out is not None else torch.empty_like(Xf)
    _check(Xa, "out", vdt, (n, N), dev)
    need = int(lib.cgd_enkf_gain_workspace_bytes(n, m, N, k, PREC[prec]))
    if need == 0 and raise_on_error:
        raise CGDError(-7, "cgd_enkf_gain_workspace_bytes")
    if need and (workspace is None or workspace.numel() < need):
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    KT = torch.empty((m, n), dtype=vdt, device=dev) if want_kt else None
    hist = torch.zeros((max(maxit, 1), n), dtype=torch.float64, device=dev) if want_hist else None
    iters = torch.full((n,), -1, dtype=torch.int32, device=dev) if want_iters else None
    tuning = Tuning(0, 0, 0, None if prof_events is None else prof_events.address(), None, 0, 0)
    opt = Options(PREC[prec], 0, 0, None, 0, None, _ptr(iters), None, 1 if validate else 0, None,
                  ctypes.pointer(tuning))
    st = Stats()
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    status = f(n, m, N, k, _ptr(Xf), _ptr(Xa), _ptr(idx), _ptr(w), _ptr(y), _ptr(r), _ptr(eps),
               float(tol), int(maxit), ctypes.byref(opt), _ptr(KT), _ptr(hist), _ptr(workspace),
               0 if workspace is None else workspace.numel(), ctypes.byref(st) if stats else None,
               ctypes.c_void_p(stream.cuda_stream))
    if raise_on_error and status < 0:
        raise CGDError(status, "cgd_enkf_gain_analysis")
    return {"Xa": Xa, "KT": KT, "hist": hist, "iters": iters,
            "stats": st.as_dict() if stats else None, "status": status, "workspace": workspace}


class Plan:
    """A pre-validated analysis of one shape for repeated calls (benchmarks,
    filter cycles): the workspace and small outputs are allocated once and a
    call is a single C-ABI call on the given device pointers."""

    def __init__(self, n, m, N, k, prec="fp32", reduced=False, tol=1e-6, maxit=1000,
                 device="cuda:0", grid=0, want_iters=True, fallback_on_stall=False, solver=0,
                 rows_per_block=0, precond=None, cooperative=False, solver_table=None,
                 senkf=False, gain=False):
        """solver: 0 automatic, 1-5 a given solver, or "tuned": the fastest
        solver of the autotuned table (autotune.tune_solvers; `solver_table` a
        path, default tuning/solver_<arch>.json) for this shape class, the
        automatic choice where the table has none.  senkf=True plans the sEnKF
        analysis (cgd_senkf_analysis) instead; tol, maxit and the solver
        choices are then unused.  gain=True plans the explicit-gain form
        (cgd_enkf_gain_analysis; iters then has n entries)."""
        self.lib = load()
        self.shape = (n, m, N, k)
        self.senkf, self.gain = bool(senkf), bool(gain)
        reduced = reduced or self.senkf  # the sEnKF takes the reduced mode's workspace
        if solver == "tuned":
            from . import autotune
            pick = autotune.solver_for(autotune.load_table(solver_table or
                                                           autotune.solver_table_path()),
                                       prec, m, N) if not reduced else None
            solver, rows_per_block, grid = ((pick["solver"], pick["rows_per_block"], pick["grid"])
                                            if pick else (0, rows_per_block, grid))
        self.prec, self.reduced, self.tol, self.maxit = prec, reduced, float(tol), int(maxit)
        self.dtype = torch.float64 if prec == "fp64" else torch.float32
        self.device = torch.device(device)
        if self.gain:
            self.lib.cgd_enkf_gain_workspace_bytes.argtypes = [ctypes.c_int] * 5
            self.lib.cgd_enkf_gain_workspace_bytes.restype = ctypes.c_size_t
            need = int(self.lib.cgd_enkf_gain_workspace_bytes(n, m, N, k, PREC[prec]))
        else:
            need = workspace_bytes(n, m, N, k, prec, reduced)
        if need == 0:
            raise CGDError(-1, "cgd_enkf_workspace_bytes")
        self.workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        self.iters = (torch.zeros(n if self.gain else N, dtype=torch.int32, device=self.device)
                      if want_iters else None)
        self.tuning = Tuning(grid, solver, rows_per_block, None, None, 1 if cooperative else 0)
        self.opt = Options(PREC[prec], PRECOND[precond], 0, None, 1 if fallback_on_stall else 0,
                           None, _ptr(self.iters), None, 0, None, ctypes.pointer(self.tuning))
        self.fn = (self.lib.cgd_senkf_analysis if self.senkf else
                   self.lib.cgd_enkf_gain_analysis if self.gain else
                   self.lib.cgd_enkf_reduced_analysis if reduced else self.lib.cgd_enkf_analysis)
        if self.gain:
            vp, ci = ctypes.c_void_p, ctypes.c_int
            self.fn.argtypes = [ci, ci, ci, ci, vp, vp, vp, vp, vp, vp, vp, ctypes.c_double, ci,
                                ctypes.POINTER(Options), vp, vp, vp, ctypes.c_size_t,
                                ctypes.POINTER(Stats), vp]
            self.fn.restype = ci

    def solver_info(self) -> dict:
        """The solver variant a call of this plan runs (full mode only)."""
        n, m, N, k = self.shape
        sv, rb, wg = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        st = self.lib.cgd_enkf_solver_info(n, m, N, k, ctypes.byref(self.opt), ctypes.byref(sv),
                                           ctypes.byref(rb), ctypes.byref(wg))
        if st < 0:
            raise CGDError(st, "cgd_enkf_solver_info")
        name = {1: "k_cg_solve (streaming)", 2: "k_cg_resident", 3: "k_cg_columns",
                4: "k_cg_split", 5: "k_cg_tile"}[sv.value]
        if sv.value == 5 and self.prec in ("mixed", "bf16"):
            name = "k_cg_tilemx"  # the mixed-precision kernel of the same solver
        elif sv.value == 5 and self.prec == "bf16split":
            name = "k_cg_tilesplit"  # k_cg_tilemx in its split-BF16 variant
        return {"solver": name, "rows_per_block": rb.value, "workgroups": wg.value}

    def check(self, Xf, idx, w, y, r, eps, out):
        n, m, N, k = self.shape
        dev, dt = self.device, self.dtype
        _check(Xf, "Xf", dt, (n, N), dev)
        _check(idx, "idx", torch.int32, (m, k), dev)
        _check(w, "w", dt, (m, k), dev)
        _check(y, "y", dt, (m,), dev)
        _check(r, "r", dt, (m,), dev)
        _check(out, "out", dt, (n, N), dev)
        if eps is not None:
            _check(eps, "eps", dt, (m, N), dev)

    def __call__(self, Xf, idx, w, y, r, eps, out, events=None, stream=None, z0=None):
        n, m, N, k = self.shape
        self.tuning.prof_events = None if events is None else events.address()
        self.opt.z0 = None if z0 is None else z0.data_ptr()
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        head = (n, m, N, k, Xf.data_ptr(), out.data_ptr(), idx.data_ptr(), w.data_ptr(),
                y.data_ptr(), r.data_ptr(), None if eps is None else eps.data_ptr())
        solve = () if self.senkf else (self.tol, self.maxit)
        extra = (None, None) if self.gain else ()   # no K^T or step records
        status = self.fn(*head, *solve, ctypes.byref(self.opt), *extra,
                         self.workspace.data_ptr(), self.workspace.numel(), None, st.cuda_stream)
        if status < 0:
            raise CGDError(status, self.fn.__name__)
        return status


class CProblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("m", ctypes.c_int), ("N", ctypes.c_int), ("k", ctypes.c_int),
                ("X_f", ctypes.c_void_p), ("X_a", ctypes.c_void_p), ("idx", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("y", ctypes.c_void_p), ("r_diag", ctypes.c_void_p),
                ("eps", ctypes.c_void_p), ("iters_out", ctypes.c_void_p),
                ("gather_rows", ctypes.c_int), ("update_rows", ctypes.c_int)]


class BatchPlan(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int), ("prec", ctypes.c_int), ("n_gather", ctypes.c_int),
                ("n_solve", ctypes.c_int), ("n_update", ctypes.c_int),
                ("off_desc", ctypes.c_size_t), ("off_gtab", ctypes.c_size_t),
                ("off_stab", ctypes.c_size_t), ("off_utab", ctypes.c_size_t),
                ("off_prefix", ctypes.c_size_t), ("off_coli", ctypes.c_size_t),
                ("ws_bytes", ctypes.c_size_t)]


class Batch:
    """Many independent analyses in one call (gather, per-member CG and
    update launches over work tables).

    problems: list of dicts with device tensors Xf, idx, w, y, r and optional
    eps (shapes as for analysis()).  Outputs go to new tensors (or in place
    with inplace=True).  prepare() runs once here; run() only launches.

    tiles: rows per gather and per update work-table entry of each problem:
    None (the library's defaults), "auto" (the autotuned table for this GPU,
    defaults where it has no entry), or a list of (gather_rows, update_rows)
    pairs, one per problem (0 for a default).  Results do not depend on it.
    """

    def __init__(self, problems, prec="fp32", want_iters=True, inplace=False, tiles=None,
                 precond=None):
        lib = load()
        if tiles == "auto":
            from . import autotune
            table = autotune.load_table()
            tiles = [autotune.tiles_for(table, q["idx"].shape[0], q["Xf"].shape[1])
                     for q in problems]
        elif tiles is None:
            tiles = [(0, 0)] * len(problems)
        if len(tiles) != len(problems):
            raise ValueError("tiles: one (gather_rows, update_rows) pair per problem")
        self.tiles = [(int(g), int(u)) for g, u in tiles]
        self.lib = lib
        self.prec = prec
        dt = torch.float64 if prec == "fp64" else torch.float32
        self.problems = problems
        self.outs, self.iters = [], []
        arr = (CProblem * len(problems))()
        for b, q in enumerate(problems):
            n, N = q["Xf"].shape
            m, k = q["idx"].shape
            dev = q["Xf"].device
            _check(q["Xf"], "Xf", dt, (n, N), dev)
            _check(q["idx"], "idx", torch.int32, (m, k), dev)
            _check(q["w"], "w", dt, (m, k), dev)
            _check(q["y"], "y", dt, (m,), dev)
            _check(q["r"], "r", dt, (m,), dev)
            if q.get("eps") is not None:
                _check(q["eps"], "eps", dt, (m, N), dev)
            out = q["Xf"] if inplace else torch.empty_like(q["Xf"])
            it = torch.zeros(N, dtype=torch.int32, device=dev) if want_iters else None
            self.outs.append(out)
            self.iters.append(it)
            arr[b] = CProblem(n, m, N, k, q["Xf"].data_ptr(), out.data_ptr(), q["idx"].data_ptr(),
                              q["w"].data_ptr(), q["y"].data_ptr(), q["r"].data_ptr(),
                              None if q.get("eps") is None else q["eps"].data_ptr(),
                              None if it is None else it.data_ptr(), *self.tiles[b])
        self._arr = arr
        lib.cgd_enkf_batched_workspace_bytes.argtypes = [ctypes.c_int, ctypes.POINTER(CProblem),
                                                         ctypes.c_int]
        lib.cgd_enkf_batched_workspace_bytes.restype = ctypes.c_size_t
        lib.cgd_enkf_batched_prepare.argtypes = [ctypes.c_int, ctypes.POINTER(CProblem), ctypes.c_int,
                                                 ctypes.c_void_p, ctypes.c_size_t,
                                                 ctypes.POINTER(BatchPlan), ctypes.c_void_p]
        lib.cgd_enkf_batched_prepare.restype = ctypes.c_int
        lib.cgd_enkf_batched_run.argtypes = [ctypes.POINTER(BatchPlan), ctypes.c_void_p,
                                             ctypes.c_double, ctypes.c_int, ctypes.POINTER(Options),
                                             ctypes.c_void_p, ctypes.c_void_p]
        lib.cgd_enkf_batched_run.restype = ctypes.c_int
        need = lib.cgd_enkf_batched_workspace_bytes(len(problems), arr, PREC[prec])
        if need == 0:
            raise CGDError(-1, "cgd_enkf_batched_workspace_bytes")
        dev = problems[0]["Xf"].device
        self.workspace = torch.empty(need, dtype=torch.uint8, device=dev)
        self.plan = BatchPlan()
        st = lib.cgd_enkf_batched_prepare(len(problems), arr, PREC[prec], self.workspace.data_ptr(),
                                          need, ctypes.byref(self.plan),
                                          torch.cuda.current_stream(dev).cuda_stream)
        if st < 0:
            raise CGDError(st, "cgd_enkf_batched_prepare")
        self.opt = Options()
        lib.cgd_options_default(ctypes.byref(self.opt))
        self.opt.prec = PREC[prec]
        self.opt.precond = PRECOND[precond]
        self.tuning = Tuning()
        self.opt.tuning = ctypes.pointer(self.tuning)
        self.device = dev

    def run(self, tol=1e-6, maxit=1000, stats=False, events=None, stream=None):
        st_arr = (Stats * len(self.problems))() if stats else None
        self.tuning.prof_events = None if events is None else events.address()
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        status = self.lib.cgd_enkf_batched_run(ctypes.byref(self.plan), self.workspace.data_ptr(),
                                               float(tol), int(maxit), ctypes.byref(self.opt),
                                               st_arr, s.cuda_stream)
        if status < 0:
            raise CGDError(status, "cgd_enkf_batched_run")
        return status, ([x.as_dict() for x in st_arr] if stats else None)


_hip = None
# hipEvent_t handles still alive: destroyed by an exit hook while the HIP
# runtime is still loaded, not by __del__ during interpreter teardown, whose
# order relative to the runtime's own shutdown is not defined
_live_events: dict = {}


def _destroy_event(handle) -> None:
    if handle and _live_events.pop(handle, None) is not None:
        try:
            hip_runtime().hipEventDestroy(handle)
        except Exception:
            pass


@atexit.register
def _destroy_live_events() -> None:
    for handle in list(_live_events):
        _destroy_event(handle)


def hip_runtime() -> ctypes.CDLL:
    """The HIP runtime (already loaded by torch), for events only."""
    global _hip
    if _hip is None:
        h = ctypes.CDLL("libamdhip64.so")
        h.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        h.hipEventCreate.restype = ctypes.c_int
        h.hipEventDestroy.argtypes = [ctypes.c_void_p]
        h.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        h.hipEventSynchronize.restype = ctypes.c_int
        h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                          ctypes.c_void_p]
        h.hipEventElapsedTime.restype = ctypes.c_int
        _hip = h
    return _hip


class EventPair:
    """Two hipEvent_t handed to the library (cgd_tuning.prof_events); it records
    them on its stream right before and after the solve kernel."""

    def __init__(self):
        self._arr = (ctypes.c_void_p * 2)()
        h = hip_runtime()
        for i in range(2):
            ev = ctypes.c_void_p()
            if h.hipEventCreate(ctypes.byref(ev)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self._arr[i] = ev.value
            _live_events[ev.value] = True

    def address(self) -> int:
        return ctypes.addressof(self._arr)

    def elapsed_ms(self) -> float:
        h = hip_runtime()
        if h.hipEventSynchronize(self._arr[1]) != 0:
            raise RuntimeError("hipEventSynchronize failed")
        ms = ctypes.c_float()
        if h.hipEventElapsedTime(ctypes.byref(ms), self._arr[0], self._arr[1]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)

    def handle(self, i: int) -> int:
        return self._arr[i]

    def __del__(self):
        for i in range(2):
            _destroy_event(self._arr[i])


class HipEvent:
    """One hipEvent_t recorded by the caller on a stream (brackets around a
    library call, read against the library's own events)."""

    def __init__(self):
        h = hip_runtime()
        ev = ctypes.c_void_p()
        if h.hipEventCreate(ctypes.byref(ev)) != 0:
            raise RuntimeError("hipEventCreate failed")
        self.ev = ev.value
        _live_events[ev.value] = True

    def record(self, stream=None, device=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(device)
        h = hip_runtime()
        h.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        h.hipEventRecord.restype = ctypes.c_int
        if h.hipEventRecord(self.ev, ctypes.c_void_p(s.cuda_stream)) != 0:
            raise RuntimeError("hipEventRecord failed")

    @staticmethod
    def elapsed_ms(a: int, b: int) -> float:
        """Milliseconds from raw event a to raw event b (b must be complete)."""
        h = hip_runtime()
        if h.hipEventSynchronize(b) != 0:
            raise RuntimeError("hipEventSynchronize failed")
        ms = ctypes.c_float()
        if h.hipEventElapsedTime(ctypes.byref(ms), a, b) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)

    def __del__(self):
        _destroy_event(self.ev)


def declared_functions(header: Optional[str] = None) -> list[str]:
    """Names of the functions declared in include/cgd_enkf.h."""
    import re
    header = header or os.path.join(os.path.dirname(_PKG), "include", "cgd_enkf.h")
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cgd_[a-z0-9_]+)\s*\(", text)))


# ---------------------------------------------------------------------------
# learned warm start (include/cgd_wsnet.h)
# ---------------------------------------------------------------------------
_WS_LAYERS = ((3, 64), (64, 64), (64, 64), (64, 1))


def _wsnet_sigs(lib):
    vp, ci, sz, cf = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_float
    lib.cgd_wsnet_param_count.restype = sz
    lib.cgd_wsnet_workspace_bytes.argtypes = [ci, ci, ci]
    lib.cgd_wsnet_workspace_bytes.restype = sz
    lib.cgd_wsnet_features.argtypes = [ci, ci, ci, ci, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.cgd_wsnet_forward.argtypes = [ci, ci, vp, vp, vp, vp, sz, vp]
    lib.cgd_wsnet_infer.argtypes = [ci, ci, ci, ci, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.cgd_wsnet_target.argtypes = [ci, ci, vp, vp, vp, vp]
    lib.cgd_wsnet_jacobi_z0.argtypes = [ci, ci, vp, vp, vp, vp]
    lib.cgd_wsnet_loss_grad.argtypes = [ci, ci, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.cgd_wsnet_train_step.argtypes = [ci, ci, vp, vp, vp, ci, cf, vp, vp, vp, vp, sz, vp]
    for f in ("cgd_wsnet_features", "cgd_wsnet_forward", "cgd_wsnet_infer",
              "cgd_wsnet_loss_grad", "cgd_wsnet_train_step", "cgd_wsnet_target",
              "cgd_wsnet_jacobi_z0"):
        getattr(lib, f).restype = ci


def wsnet_init_params(seed: int = 0) -> np.ndarray:
    """He-initialised FP32 parameter vector in the library's order (per layer
    W[o][c][t], then b[o]); the biases start at zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for cin, cout in _WS_LAYERS:
        std = np.sqrt(2.0 / (cin * 5))
        parts.append((rng.standard_normal((cout, cin, 5)) * std).ravel())
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32)


def wsnet_unpack(vec) -> list:
    """Parameter vector -> [(W [cout, cin, 5], b [cout]), ...] (NumPy, float64)."""
    v = np.asarray(vec, dtype=np.float64)
    out, o = [], 0
    for cin, cout in _WS_LAYERS:
        nw = cout * cin * 5
        out.append((v[o:o + nw].reshape(cout, cin, 5), v[o + nw:o + nw + cout]))
        o += nw + cout
    return out


class WarmStartNet:
    """The warm-start network on the device: FP32 parameters and Adam moments
    as torch tensors, calls marshalled to the C ABI."""

    def __init__(self, params=None, seed: int = 0, device="cuda:0"):
        self.lib = load()
        _wsnet_sigs(self.lib)
        self.device = torch.device(device)
        n = int(self.lib.cgd_wsnet_param_count())
        p = wsnet_init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        if p.size != n:
            raise ValueError(f"expected {n} parameters, got {p.size}")
        self.params = torch.as_tensor(p, device=self.device).clone()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self._ws = {}
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)

    def save(self, path: str, **extra) -> None:
        """Write the training state (parameters, Adam moments, step count and
        any extra arrays or scalars, e.g. the epoch) to an .npz file of plain
        arrays (no pickled objects)."""
        arrays = {"params": self.params.cpu().numpy(), "adam_m": self.m.cpu().numpy(),
                  "adam_v": self.v.cpu().numpy(), "step": np.array(self.step, dtype=np.int64)}
        for k, v in extra.items():
            arrays["extra_" + k] = np.asarray(v)
        np.savez(path, **arrays)

    @classmethod
    def load_state(cls, path: str, device="cuda:0"):
        """The network of a file written by save(); returns (net, extra)."""
        with np.load(path, allow_pickle=False) as f:
            net = cls(params=f["params"], device=device)
            net.m.copy_(torch.as_tensor(f["adam_m"]))
            net.v.copy_(torch.as_tensor(f["adam_v"]))
            net.step = int(f["step"])
            extra = {k[len("extra_"):]: f[k] for k in f.files if k.startswith("extra_")}
        return net, extra

    def _workspace(self, batch, m, training):
        key = (batch, m, training)
        if key not in self._ws:
            need = self.lib.cgd_wsnet_workspace_bytes(batch, m, training)
            if need == 0:
                raise CGDError(-1, "cgd_wsnet_workspace_bytes")
            self._ws[key] = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws[key]

    def _stream(self, stream):
        return (stream if stream is not None else torch.cuda.current_stream(self.device)).cuda_stream

    def features(self, Xf, idx, w, y, r, eps=None, stream=None):
        """(feat [N, m, 4], scale [N]) of one analysis (FP32 inputs)."""
        n, N = Xf.shape
        m, k = idx.shape
        feat = torch.empty((N, m, 4), dtype=torch.float32, device=self.device)
        scale = torch.empty(N, dtype=torch.float32, device=self.device)
        ws = self._workspace(N, m, 0)
        st = self.lib.cgd_wsnet_features(n, m, N, k, Xf.data_ptr(), idx.data_ptr(), w.data_ptr(),
                                         y.data_ptr(), r.data_ptr(), _ptr(eps), feat.data_ptr(),
                                         scale.data_ptr(), ws.data_ptr(), ws.numel(),
                                         self._stream(stream))
        if st < 0:
            raise CGDError(st, "cgd_wsnet_features")
        return feat, scale

    def forward(self, feat, stream=None):
        B, m, _ = feat.shape
        out = torch.empty((B, m), dtype=torch.float32, device=self.device)
        ws = self._workspace(B, m, 0)
        st = self.lib.cgd_wsnet_forward(B, m, self.params.data_ptr(), feat.data_ptr(),
                                        out.data_ptr(), ws.data_ptr(), ws.numel(),
                                        self._stream(stream))
        if st < 0:
            raise CGDError(st, "cgd_wsnet_forward")
        return out

    def predict_z0(self, Xf, idx, w, y, r, eps=None, out=None, stream=None):
        """z0 [m, N] for cgd_options.z0."""
        n, N = Xf.shape
        m, k = idx.shape
        z0 = out if out is not None else torch.empty((m, N), dtype=torch.float32,
                                                     device=self.device)
        ws = self._workspace(N, m, 0)
        st = self.lib.cgd_wsnet_infer(n, m, N, k, Xf.data_ptr(), idx.data_ptr(), w.data_ptr(),
                                      y.data_ptr(), r.data_ptr(), _ptr(eps),
                                      self.params.data_ptr(), z0.data_ptr(), ws.data_ptr(),
                                      ws.numel(), self._stream(stream))
        if st < 0:
            raise CGDError(st, "cgd_wsnet_infer")
        return z0

    def target(self, Z, scale, stream=None):
        """Training target [N, m] = Z[i, j] / s_j (cgd_wsnet_target)."""
        m, N = Z.shape
        _check(Z, "Z", torch.float32, (m, N), self.device)
        _check(scale, "scale", torch.float32, (N,), self.device)
        out = torch.empty((N, m), dtype=torch.float32, device=self.device)
        st = self.lib.cgd_wsnet_target(m, N, Z.data_ptr(), scale.data_ptr(), out.data_ptr(),
                                       self._stream(stream))
        if st < 0:
            raise CGDError(st, "cgd_wsnet_target")
        return out

    def jacobi_z0(self, feat, scale, out=None, stream=None):
        """Jacobi start z0 [m, N] = d_ij / Psi_ii from the features (cgd_wsnet_jacobi_z0)."""
        N, m, _ = feat.shape
        _check(feat, "feat", torch.float32, (N, m, 4), self.device)
        _check(scale, "scale", torch.float32, (N,), self.device)
        z0 = out if out is not None else torch.empty((m, N), dtype=torch.float32,
                                                     device=self.device)
        st = self.lib.cgd_wsnet_jacobi_z0(m, N, feat.data_ptr(), scale.data_ptr(), z0.data_ptr(),
                                          self._stream(stream))
        if st < 0:
            raise CGDError(st, "cgd_wsnet_jacobi_z0")
        return z0

    def loss_grad(self, feat, target, stream=None):
        B, m, _ = feat.shape
        grad = torch.empty_like(self.params)
        ws = self._workspace(B, m, 1)
        st = self.lib.cgd_wsnet_loss_grad(B, m, self.params.data_ptr(), feat.data_ptr(),
                                          target.data_ptr(), self.loss.data_ptr(),
                                          grad.data_ptr(), ws.data_ptr(), ws.numel(),
                                          self._stream(stream))
        if st < 0:
            raise CGDError(st, "cgd_wsnet_loss_grad")
        return self.loss, grad

    def train_step(self, feat, target, lr=1e-3, stream=None):
        """One Adam step; returns the (device) loss before the update."""
        B, m, _ = feat.shape
        ws = self._workspace(B, m, 1)
        self.step += 1
        st = self.lib.cgd_wsnet_train_step(B, m, self.params.data_ptr(), self.m.data_ptr(),
                                           self.v.data_ptr(), self.step, float(lr),
                                           feat.data_ptr(), target.data_ptr(),
                                           self.loss.data_ptr(), ws.data_ptr(), ws.numel(),
                                           self._stream(stream))
        if st < 0:
            raise CGDError(st, "cgd_wsnet_train_step")
        return self.loss
