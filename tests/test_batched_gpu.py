"""Batched analyses (one call: gather, one CG workgroup per member of every
problem, update) against the oracle, problem by problem."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import dev_problem, rel, rounded, say

pytestmark = pytest.mark.gpu


def _dev(p, prec):
    d = dev_problem(p, prec)
    return {"Xf": d["Xf"], "idx": d["idx"], "w": d["w"], "y": d["y"], "r": d["r"], "eps": d["eps"]}


MIXED = [  # n, m, N, k, deterministic
    (40, 20, 20, 1, False), (300, 257, 33, 4, False), (100, 3, 17, 1, True), (30, 12, 2, 1, False),
    (700, 640, 64, 2, False), (500, 65, 16, 1, False), (2000, 1000, 32, 3, True), (64, 64, 5, 1, False),
]


def test_batched_fp64_mixed(lib):
    import torch
    probs = [W.random_problem(n, m, N, k, seed=400 + i, tol=1e-12, stochastic=not det)
             for i, (n, m, N, k, det) in enumerate(MIXED)]
    say("case: batched fp64 mixed")
    b = lib.Batch([_dev(p, "fp64") for p in probs], prec="fp64")
    status, stats = b.run(tol=1e-12, maxit=1000, stats=True)
    torch.cuda.synchronize()
    assert status == 0
    for p, out, it, st in zip(probs, b.outs, b.iters, stats):
        ref = O.enkf_analysis(p.Xf, p.idx, p.w, p.y, p.r, p.eps, solver="cg_free", tol=1e-12,
                              maxit=1000)
        assert rel(out.cpu().numpy(), ref["Xa"]) <= 1e-10, p.name
        # near the threshold the stopping iteration is not unique (see test_parity_gpu)
        assert np.max(np.abs(it.cpu().numpy() - ref["iters"])) <= 2, p.name
        assert st["n_converged"] == p.N and st["iters_max"] == it.max().item()
    # repeated runs on the same plan are bitwise identical
    first = [o.clone() for o in b.outs]
    b.run(tol=1e-12, maxit=1000)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(first, b.outs))


def test_batched_fixed_iterations_match_single(lib):
    import torch
    probs = [W.random_problem(n, m, N, k, seed=500 + i) for i, (n, m, N, k, _) in enumerate(MIXED)]
    b = lib.Batch([_dev(p, "fp64") for p in probs], prec="fp64")
    b.run(tol=0.0, maxit=4)
    torch.cuda.synchronize()
    for p, out, it in zip(probs, b.outs, b.iters):
        ref = O.enkf_analysis(p.Xf, p.idx, p.w, p.y, p.r, p.eps, solver="cg_free", tol=0.0, maxit=4)
        assert np.all(it.cpu().numpy() == 4)
        assert rel(out.cpu().numpy(), ref["Xa"]) <= 1e-10


def test_batched_fp32_config4_sizes(lib):
    """A few problems of the batched Lorenz-96 recipe at their real sizes
    (n up to 32768, m = n/4, N in {16, 32, 64}, R = I), FP32 at tol 1e-6."""
    import torch
    probs = W.config4(count=6, heal_steps=5)
    say("case: batched config4 sizes " + str([(p.n, p.N) for p in probs]))
    b = lib.Batch([_dev(p, "fp32") for p in probs], prec="fp32")
    status, stats = b.run(tol=1e-6, maxit=1000, stats=True)
    torch.cuda.synchronize()
    assert status == 0
    for p, out, st in zip(probs, b.outs, stats):
        # same algorithm, stop rule and (FP32-rounded) inputs in FP64: the
        # difference is the FP32 arithmetic; kappa(Psi) ~ m/(N-1) up to ~500 here
        q = rounded(p)
        ref = O.enkf_analysis(q.Xf, q.idx, q.w, q.y, q.r, q.eps, solver="cg_free", tol=1e-6,
                              maxit=2000)
        err = rel(out.cpu().numpy(), ref["Xa"])
        say(f"  n={p.n} N={p.N} iters={st['iters_max']} rel err vs FP64 CG {err:.2e}")
        assert err <= 1e-4
        # R = I: at most N distinct eigenvalues (Lemma 1, sharpened)
        assert st["iters_max"] <= p.N + 2


def test_batched_graph_replay(lib):
    """The run call captured into a HIP graph: every replay equals the eager
    result, with eager work and synchronisation between replays."""
    import torch
    probs = [W.random_problem(n, m, N, k, seed=600 + i, tol=1e-6)
             for i, (n, m, N, k, _) in enumerate(MIXED)]
    b = lib.Batch([_dev(p, "fp32") for p in probs], prec="fp32")
    b.run(tol=1e-6, maxit=500)
    torch.cuda.synchronize()
    eager = [o.clone() for o in b.outs]
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        b.run(tol=1e-6, maxit=500, stream=torch.cuda.current_stream())
    for rep in range(3):
        for o in b.outs:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert all(torch.equal(x, y) for x, y in zip(eager, b.outs)), rep


def test_batched_bad_index_reported(lib):
    import torch
    probs = [W.random_problem(100, 40, 8, 2, seed=700 + i) for i in range(3)]
    ds = [_dev(p, "fp64") for p in probs]
    ds[1]["idx"] = ds[1]["idx"].clone()
    ds[1]["idx"][3, 0] = 100
    b = lib.Batch(ds, prec="fp64")
    with pytest.raises(lib.CGDError) as ei:
        b.run(tol=1e-8, maxit=100, stats=True)
    assert ei.value.status == -2


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_tiles_do_not_change_results(lib, prec):
    """The rows per gather / update entry only cut the work differently: every
    choice (including a different one per problem, and the tuned table) gives
    bitwise the same X_a and iteration counts."""
    import torch
    probs = [W.random_problem(n, m, N, k, seed=700 + i, tol=1e-10)
             for i, (n, m, N, k, _) in enumerate(MIXED)]
    dev = [_dev(p, prec) for p in probs]
    say(f"case: batched tiles {prec}")
    base = lib.Batch(dev, prec=prec)
    base.run(tol=1e-10, maxit=1000)
    torch.cuda.synchronize()
    choices = [[(32, 64)] * len(probs), [(128, 128)] * len(probs), [(1024, 4096)] * len(probs),
               [((i % 4 + 1) * 64, (i % 3 + 1) * 64) for i in range(len(probs))], "auto"]
    for tiles in choices:
        b = lib.Batch(dev, prec=prec, tiles=tiles)
        b.run(tol=1e-10, maxit=1000)
        torch.cuda.synchronize()
        for x, y in zip(base.outs, b.outs):
            assert torch.equal(x, y), tiles
        for x, y in zip(base.iters, b.iters):
            assert torch.equal(x, y), tiles


def test_batched_full_256_filter_workload(lib):
    """The benchmark's batch itself: all 256 filters of the batched Lorenz-96
    workload (20 healing steps, the autotuned tiles, graph replay as timed),
    each against the FP64 oracle's CG on its FP32-rounded inputs at 1e-4."""
    import torch
    probs = W.config4()
    say(f"case: batched full workload, {len(probs)} filters")
    b = lib.Batch([_dev(p, "fp32") for p in probs], prec="fp32", tiles="auto")
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    b.run(tol=1e-6, maxit=1000)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=stream):
        b.run(tol=1e-6, maxit=1000, stream=torch.cuda.current_stream())
    for o in b.outs:
        o.zero_()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    worst = 0.0
    for p, out in zip(probs, b.outs):
        q = rounded(p)
        ref = O.enkf_analysis(q.Xf, q.idx, q.w, q.y, q.r, q.eps, solver="cg_free", tol=1e-6,
                              maxit=2000)
        err = rel(out.cpu().numpy(), ref["Xa"])
        worst = max(worst, err)
        assert err <= 1e-4, (p.n, p.N, err)
    say(f"  worst rel err vs FP64 CG over {len(probs)} filters: {worst:.2e}")
