"""The warm-start stall window on the GPU solvers against the oracle.

The problem embeds the tridiagonal system of the oracle's stall-window pin
in an EnKF analysis: S = [F | -F] (centred rows) with F F^T = (N-1)(T - rho I)/2,
so Psi = S S^T/(N-1) + rho I = T, and each member's warm start leaves the
residual c_j e_1 with c_j < ||d_j||.  The CG residual history is then the
closed form 1/(1 + k u) of the pin, every member passes the initial-residual
test (||r_0|| <= ||d||) and restarts from the 5-step window at k = 10."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_util import assert_iters_close, rel, say
from tests.test_oracle_pins_warm import stall_matrix

pytestmark = pytest.mark.gpu


def stall_problem(M=30, N=64, rho=1e-3, seed=5):
    rng = np.random.default_rng(seed)
    T = stall_matrix(M)
    q = N // 2
    lam, V = np.linalg.eigh((N - 1) * (T - rho * np.eye(M)) / 2)
    F = np.zeros((M, q))
    F[:, :M] = V * np.sqrt(lam)
    S = np.concatenate([F, -F], axis=1)
    mu = rng.standard_normal(M) * 2
    Xf = S + mu[:, None]
    idx = np.arange(M, dtype=np.int32)[:, None]
    w = np.ones((M, 1))
    y = rng.standard_normal(M) + mu
    r = np.full(M, rho)
    D = O.innovations(idx, w, Xf, y)
    Psi = O.innovation_matrix(O.obs_anomalies(idx, w, Xf), r)
    c = rng.uniform(0.3, 0.9, N) * np.linalg.norm(D, axis=0)
    E1 = np.zeros((M, N))
    E1[0] = c
    Z0 = np.linalg.solve(Psi, D - E1)
    return Xf, idx, w, y, r, Z0


@pytest.mark.parametrize("solver", [1, 2, 3, 4])
def test_stall_window_fp64(lib, solver):
    import torch
    Xf, idx, w, y, r, Z0 = stall_problem()
    tol = 1e-10
    ref = O.enkf_analysis(Xf, idx, w, y, r, None, solver="cg_free", tol=tol, maxit=500, Z0=Z0,
                          fallback_on_stall=True)
    zero = O.enkf_analysis(Xf, idx, w, y, r, None, solver="cg_free", tol=tol, maxit=500)
    assert ref["fallbacks"].all() and np.all(ref["iters"] - zero["iters"] == 10)
    t = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt,
                                                    device="cuda:0")
    say(f"case: stall window fp64 solver={solver}")
    out = lib.analysis(t(Xf), t(idx, torch.int32), t(w), t(y), t(r), None, tol=tol, maxit=500,
                       prec="fp64", solver=solver, z0=t(Z0), fallback_on_stall=True, want_z=True,
                       want_iters=True)
    torch.cuda.synchronize()
    assert out["status"] == 0
    assert out["stats"]["n_fallbacks"] == int(ref["fallbacks"].sum()) == 64
    assert rel(out["Z"].cpu().numpy(), ref["Z"]) <= 1e-10
    assert rel(out["Xa"].cpu().numpy(), ref["Xa"]) <= 1e-10
    assert_iters_close(out["iters"].cpu().numpy(), ref["iters"])
