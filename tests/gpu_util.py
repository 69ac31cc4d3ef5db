"""Helpers for the GPU tests: move a workloads.Problem to the device and run
the library through its binding."""
import sys

import numpy as np
import torch


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev_problem(p, prec="fp64", device="cuda:0"):
    dt = torch.float64 if prec == "fp64" else torch.float32
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
    return dict(Xf=t(p.Xf), idx=torch.as_tensor(np.ascontiguousarray(p.idx), dtype=torch.int32,
                                                 device=device),
                w=t(p.w), y=t(p.y), r=t(p.r), eps=None if p.eps is None else t(p.eps))


def run(lib, p, prec="fp64", tol=None, maxit=None, **kw):
    args = dev_problem(p, prec)
    out = lib.analysis(**args, tol=p.tol if tol is None else tol,
                       maxit=p.maxit if maxit is None else maxit, prec=prec, **kw)
    torch.cuda.synchronize()
    res = {"Xa": out["Xa"].double().cpu().numpy(), "status": out["status"], "stats": out["stats"]}
    if out["Z"] is not None:
        res["Z"] = out["Z"].double().cpu().numpy()
    if out["iters"] is not None:
        res["iters"] = out["iters"].cpu().numpy()
    if out["relres"] is not None:
        res["relres"] = out["relres"].cpu().numpy()
    return res


def rel(a, b):
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / (d if d > 0 else 1.0))


def rounded(p, dtype=np.float32):
    """The same problem with every value array rounded through `dtype`: the
    inputs an FP32 run actually sees, for an oracle run on identical data."""
    import dataclasses
    r = lambda a: None if a is None else np.asarray(a, dtype=dtype).astype(np.float64)
    return dataclasses.replace(p, Xf=r(p.Xf), w=r(p.w), y=r(p.y), r=r(p.r), eps=r(p.eps))



def assert_iters_close(got, ref):
    """Per-column iteration counts of two valid FP64 CG implementations with
    the same stop rule.  Near the threshold the recursive residuals round
    differently, and over tens of iterations the two Krylov trajectories
    drift apart by more than rounding (CG is not forward stable in its
    iterates, only in the final accuracy), so the first crossing can move by
    a few iterations: allow max(2, 5%).  The solution itself is checked
    separately, to the parity tolerance."""
    got, ref = np.asarray(got), np.asarray(ref)
    allow = np.maximum(2, np.ceil(0.05 * ref))
    assert np.all(np.abs(got - ref) <= allow), (got - ref, allow)
