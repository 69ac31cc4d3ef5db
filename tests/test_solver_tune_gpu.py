"""The solver autotuner on the GPU: a tuned plan runs the table's pick
(bitwise the same X_a as forcing that solver) and meets the parity bar."""
import json

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import dev_problem, rel, say

pytestmark = pytest.mark.gpu


def test_tuned_plan_runs_the_pick(lib, tmp_path):
    import torch

    from paper_2606_19224_amd import autotune as A

    table = A.tune_solvers(shapes=((512, 32),), precs=("fp32",), reps=2, log=say)
    assert len(table["entries"]) == 1
    e = table["entries"][0]
    say(f"  pick {e['solver']}/{e['rows_per_block']}/{e['grid']} of {e['us']}")
    assert len(e["us"]) >= 3  # columns, split, tile at least
    path = tmp_path / "solver.json"
    path.write_text(json.dumps(table))
    p = W.random_problem(1000, 500, 30, 1, seed=77, tol=1e-6)
    d = dev_problem(p, "fp32")
    n, m, N, k = p.Xf.shape[0], p.m, p.N, 1
    outs = []
    for kw in ({"solver": "tuned", "solver_table": str(path)},
               {"solver": e["solver"], "rows_per_block": e["rows_per_block"], "grid": e["grid"]}):
        plan = lib.Plan(n, m, N, k, prec="fp32", tol=1e-6, maxit=1000, **kw)
        out = torch.empty((n, N), dtype=torch.float32, device="cuda:0")
        plan(d["Xf"], d["idx"], d["w"], d["y"], d["r"], d["eps"], out)
        torch.cuda.synchronize()
        outs.append(out.clone())
    assert torch.equal(outs[0], outs[1])
    ref = O.enkf_analysis(p.Xf, p.idx, p.w, p.y, p.r, p.eps, solver="cholesky")
    assert rel(outs[0].double().cpu().numpy(), ref["Xa"]) <= 1e-4
