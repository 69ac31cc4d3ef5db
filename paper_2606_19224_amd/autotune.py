"""Autotuner for the batched mode's work tables.

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
    args = ap.parse_args(argv)
    import numpy as np
    import torch

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
