"""Autotuners: the batched mode's work tables, and the single analysis's
solver choice.

The batched analysis runs three launches over work tables.  How many rows a
gather entry and an update entry cover is a free choice: it changes how the
work is cut into workgroups, never the arithmetic.  This module measures, for
each class of problem shapes, the gather and update launch times of every
candidate row count on the GPU at hand, and keeps the fastest in a JSON table
that Batch(tiles="auto") reads.

A class is (N padded to 16, 32 or 64; m rounded up to a power of two).  The
tuner times a batch made of one class's problems alone (the class's problems
repeated until the batch has at least `min_batch` of them), with events around
the gather and the update.

    python -m paper_2606_19224_amd.autotune            # tune on 256 filters of the
                                                      # uneven Lorenz-96 workload, write
                                                      # tuning/batched_<arch>.json

The single analysis has more than one solver that can run a shape: the
per-member column and split solvers (VALU products), the row-block x
member-group and the resident solvers (MFMA products; the resident solver in
16-, 32- or 64-row blocks) and the streaming solver (any grid).  Which is
fastest depends on the shape in ways the library's built-in rule only
approximates.  `tune_solvers` times every candidate the library accepts for
each (precision, N class, m bucket) on a synthetic problem of that class and
keeps the fastest in tuning/solver_<arch>.json, which Plan(solver="tuned")
reads.  The candidates differ in summation order, not in the method: each is
held to the same parity tests.

    python -m paper_2606_19224_amd.autotune --solvers  # tune the default shape set,
                                                      # write tuning/solver_<arch>.json
"""
import argparse
import json
import math
import os
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_DIR = os.path.join(_HERE, "tuning")
GATHER_CANDIDATES = (64, 128, 256, 512, 1024)
UPDATE_CANDIDATES = (64, 128, 256, 512, 1024)


def shape_class(m: int, N: int) -> tuple:
    """(padded N, m bucket): N -> 16, 32 or 64; m -> the next power of two."""
    npad = 16 if N <= 16 else 32 if N <= 32 else 64
    return npad, 1 << max(0, math.ceil(math.log2(max(1, m))))


def table_path(arch: str = "gfx950") -> str:
    return os.path.join(TABLE_DIR, f"batched_{arch}.json")


def load_table(path: str = None):
    """The tuned table (dict), or None when there is none for this GPU."""
    path = path or table_path()
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def tiles_for(table, m: int, N: int) -> tuple:
    """(gather_rows, update_rows) for a problem; (0, 0), the library's
    defaults, when the table has no entry for its class."""
    if not table:
        return (0, 0)
    npad, mb = shape_class(m, N)
    for e in table.get("entries", []):
        if e["N"] == npad and e["m_bucket"] == mb:
            return (int(e["gather_rows"]), int(e["update_rows"]))
    return (0, 0)


# (solver, rows_per_block, grid): the launch shapes the single analysis can
# take; the library answers CGD_ERR_UNSUPPORTED for those a shape cannot run.
SOLVER_CANDIDATES = ((3, 0, 0), (4, 0, 0), (5, 0, 0), (2, 16, 0), (2, 32, 0), (2, 64, 0),
                     (1, 0, 128), (1, 0, 256), (1, 0, 512))
# (m, N) shapes tuned by default: the benches' configurations and their
# neighbours
SOLVER_SHAPES = ((20, 20), (512, 32), (2048, 64), (4096, 64), (8192, 128), (16384, 128),
                 (2048, 128), (16384, 40))


def solver_class(prec: str, m: int, N: int) -> tuple:
    """(precision, N padded to 16, 32, 64 or 128, m rounded up to a power of
    two); N > 128 has no class (the streaming solver alone runs it)."""
    npad = 16 if N <= 16 else 32 if N <= 32 else 64 if N <= 64 else 128 if N <= 128 else 0
    return prec, npad, 1 << max(0, math.ceil(math.log2(max(1, m))))


def solver_table_path(arch: str = "gfx950") -> str:
    return os.path.join(TABLE_DIR, f"solver_{arch}.json")


def solver_for(table, prec: str, m: int, N: int):
    """{"solver", "rows_per_block", "grid"} of the table's pick for this
    shape, or None (the automatic choice) when the table has no entry."""
    if not table:
        return None
    p, npad, mb = solver_class(prec, m, N)
    for e in table.get("entries", []):
        if e["prec"] == p and e["N"] == npad and e["m_bucket"] == mb:
            return {"solver": int(e["solver"]), "rows_per_block": int(e["rows_per_block"]),
                    "grid": int(e["grid"])}
    return None


def _time_solvers(p, prec, reps):
    """{candidate: median us per analysis} for one synthetic problem (the
    candidates the library accepts for its shape)."""
    import numpy as np
    import torch

    from . import binding as B

    dev = torch.device("cuda:0")
    dt = torch.float64 if prec == "fp64" else torch.float32
    t = lambda a, d=dt: torch.as_tensor(np.ascontiguousarray(a), dtype=d, device=dev)
    Xf, idx, w, y, r = t(p.Xf), t(p.idx, torch.int32), t(p.w), t(p.y), t(p.r)
    eps = None if p.eps is None else t(p.eps)
    n, m, N, k = p.Xf.shape[0], p.m, p.N, p.idx.shape[1]
    out = torch.empty((n, N), dtype=dt, device=dev)
    res = {}
    for cand in SOLVER_CANDIDATES:
        solver, rb, grid = cand
        try:
            plan = B.Plan(n, m, N, k, prec=prec, tol=p.tol, maxit=p.maxit, solver=solver,
                          rows_per_block=rb, grid=grid, want_iters=False)
            plan.solver_info()  # raises for a launch shape this problem cannot take
        except B.CGDError:
            continue
        st = []
        for rep in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plan(Xf, idx, w, y, r, eps, out)
            e1.record()
            torch.cuda.synchronize()
            if rep:
                st.append(e0.elapsed_time(e1) * 1e3)
        res[cand] = float(np.median(st))
        del plan
    return res


def tune_solvers(shapes=SOLVER_SHAPES, precs=("fp32", "fp64"), reps=7, seed=0, log=print):
    """Time every accepted candidate for each (precision, shape) and return
    the table (one entry per class: the fastest candidate and every time)."""
    sys.path.insert(0, os.path.dirname(_HERE))
    import workloads as W

    entries, seen = [], set()
    for prec in precs:
        for m, N in shapes:
            cls = solver_class(prec, m, N)
            if cls in seen or cls[1] == 0:
                continue
            seen.add(cls)
            p = W.random_problem(2 * m, m, N, 1, seed=seed + m + N, tol=1e-6 if prec != "fp64"
                                 else 1e-10, maxit=1000)
            times = _time_solvers(p, prec, reps)
            if not times:
                continue
            best = min(times, key=times.get)
            e = {"prec": prec, "N": cls[1], "m_bucket": cls[2], "shape": [m, N],
                 "solver": best[0], "rows_per_block": best[1], "grid": best[2],
                 "us": {f"{c[0]}/{c[1]}/{c[2]}": round(v, 2) for c, v in times.items()}}
            log(json.dumps(e))
            entries.append(e)
    return {"arch": "gfx950", "kind": "solver", "candidates": [list(c) for c in
                                                                SOLVER_CANDIDATES],
            "entries": entries}


def _time_class(problems, prec, reps):
    """{(g, u): (gather_us, update_us)} medians for one class's batch."""
    import numpy as np
    import torch

    from . import binding as B

    res = {}
    for g in GATHER_CANDIDATES:
        u = UPDATE_CANDIDATES[GATHER_CANDIDATES.index(g)]
        batch = B.Batch(problems, prec=prec, want_iters=False, tiles=[(g, u)] * len(problems))
        ev, s0, s1 = B.EventPair(), B.HipEvent(), B.HipEvent()
        ga, up = [], []
        for r in range(reps + 1):
            s0.record()
            batch.run(tol=1e-6, maxit=1000, events=ev)  # events after the gather and the CG
            s1.record()
            torch.cuda.synchronize()
            if r == 0:
                continue  # warm-up
            ga.append(B.HipEvent.elapsed_ms(s0.ev, ev.handle(0)))
            up.append(B.HipEvent.elapsed_ms(ev.handle(1), s1.ev))
        res[(g, u)] = (float(np.median(ga)) * 1e3, float(np.median(up)) * 1e3)
        del batch
    return res


def tune(problems, prec="fp32", reps=5, min_batch=64, log=print):
    """Tune every shape class present in `problems` (dicts as for Batch);
    returns the table."""
    classes = {}
    for q in problems:
        classes.setdefault(shape_class(q["idx"].shape[0], q["Xf"].shape[1]), []).append(q)
    entries = []
    for (npad, mb), qs in sorted(classes.items()):
        batch = (qs * ((min_batch + len(qs) - 1) // len(qs)))[:max(min_batch, len(qs))]
        times = _time_class(batch, prec, reps)
        g_best = min(GATHER_CANDIDATES, key=lambda g: times[(g, UPDATE_CANDIDATES[
            GATHER_CANDIDATES.index(g)])][0])
        u_best = min(UPDATE_CANDIDATES, key=lambda u: times[(GATHER_CANDIDATES[
            UPDATE_CANDIDATES.index(u)], u)][1])
        e = {"N": npad, "m_bucket": mb, "gather_rows": g_best, "update_rows": u_best,
             "problems": len(qs), "batch": len(batch),
             "gather_us": {str(g): round(times[(g, u)][0], 2) for g, u in times},
             "update_us": {str(u): round(times[(g, u)][1], 2) for g, u in times}}
        log(json.dumps(e))
        entries.append(e)
    return {"arch": "gfx950", "prec": prec, "candidates": {"gather_rows": GATHER_CANDIDATES,
                                                            "update_rows": UPDATE_CANDIDATES},
            "entries": entries}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--count", type=int, default=256, help="filters of the uneven workload")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=None, help="table path (default tuning/batched_<arch>.json)")
    ap.add_argument("--solvers", action="store_true",
                    help="tune the single analysis's solver choice instead")
    args = ap.parse_args(argv)
    import numpy as np
    import torch

    if args.solvers:
        table = tune_solvers(reps=args.reps, log=lambda s: print(s, file=sys.stderr, flush=True))
        out = args.out or solver_table_path()
        os.makedirs(os.path.dirname(out), exist_ok=True)
        with open(out, "w") as f:
            json.dump(table, f, indent=1)
        print(f"wrote {out}", file=sys.stderr)
        return

    sys.path.insert(0, os.path.dirname(_HERE))
    import workloads as W

    dev = torch.device("cuda:0")
    t = lambda a, d=torch.float32: torch.as_tensor(np.ascontiguousarray(a), dtype=d, device=dev)
    problems = [dict(Xf=t(p.Xf), idx=t(p.idx, torch.int32), w=t(p.w), y=t(p.y), r=t(p.r),
                     eps=None if p.eps is None else t(p.eps)) for p in W.config4(count=args.count)]
    table = tune(problems, reps=args.reps, log=lambda s: print(s, file=sys.stderr, flush=True))
    out = args.out or table_path()
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"wrote {out}", file=sys.stderr)


if __name__ == "__main__":
    main()
