"""Plant plausible mistakes in the oracle (CPU only) and check that the pins
catch every one of them: a dropped term, a wrong sign or index, a transposed
operand, a wrong CG coefficient."""
import numpy as np
import pytest

import oracle.enkf as E
import tests.test_oracle_pins as PINS


def _pins():
    """A fixed subset of pins; each raises AssertionError on a failure."""
    yield lambda: PINS.test_bruteforce_config1()
    yield lambda: PINS.test_exact_rational_tiny()
    yield lambda: PINS.test_bruteforce_gain_matches_innovation_form(0, 30, 12, 7, 2, True)
    yield lambda: PINS.test_reduced_equals_full(4, 40, 30, 6, 1, True)
    yield lambda: PINS.test_cg_converges_to_cholesky_config1()
    yield lambda: PINS.test_cg_iterates_match_scipy()
    yield lambda: PINS.test_cg_iterates_are_krylov_minimisers()
    yield lambda: PINS.test_identity_H_scalar_R_closed_form()
    yield lambda: PINS.test_mean_and_anomaly_update()


def _caught() -> bool:
    for pin in _pins():
        try:
            with np.errstate(all="ignore"):
                pin()
        except (AssertionError, np.linalg.LinAlgError, ValueError):
            return True
    return False


def _cg_mutant(kind):
    orig = E.textbook_cg

    def cg(matvec, d, tol, maxit, z0=None, fallback_on_stall=False, record=False):
        d = np.asarray(d, dtype=np.float64)
        z = np.zeros_like(d) if z0 is None else np.array(z0, dtype=np.float64)
        r = d - matvec(z)
        p = r.copy()
        rho = float(r @ r)
        its, hist = 0, [z.copy()]
        while np.sqrt(rho) > tol * np.linalg.norm(d) and its < maxit and rho > 0:
            q = matvec(p)
            alpha = rho / float(p @ q)
            if kind == "alpha_from_r":
                alpha = rho / float(r @ matvec(r))
            z = z + alpha * p
            r = r - alpha * q
            rho_new = float(r @ r)
            beta = rho / rho_new if kind == "beta_inverted" else rho_new / rho
            p = (r - beta * p) if kind == "p_sign" else (r + beta * p)
            rho = rho_new
            its += 1
            hist.append(z.copy())
        return E.CGResult(z, its, [], hist if record else [])
    assert orig is not None
    return cg


def _mutants():
    obs = E.observe
    yield "innovation_sign", "innovations", \
        lambda idx, w, X, y, eps=None: -(np.asarray(y)[:, None] - obs(idx, w, X)
                                         + (0 if eps is None else eps))
    yield "eps_dropped", "innovations", \
        lambda idx, w, X, y, eps=None: np.asarray(y)[:, None] - obs(idx, w, X)
    yield "psi_missing_scale", "innovation_matrix", \
        lambda S, r: S @ S.T + np.diag(r)
    yield "psi_missing_R", "innovation_matrix", \
        lambda S, r: S @ S.T / (S.shape[1] - 1) + np.eye(S.shape[0]) * 1e-3
    yield "uncentred_S", "obs_anomalies", lambda idx, w, X: obs(idx, w, X)
    yield "update_transposed", "analysis_update", \
        lambda Xf, S, Z: Xf + E.state_anomalies(Xf) @ (Z.T @ S) / (S.shape[1] - 1)
    yield "update_uses_N", "analysis_update", \
        lambda Xf, S, Z: Xf + E.state_anomalies(Xf) @ (S.T @ Z) / S.shape[1]

    def observe_first_only(idx, w, X):
        return obs(idx[:, :1], w[:, :1], X)
    yield "observe_drops_terms", "observe", observe_first_only

    def observe_wrong_index(idx, w, X):
        return obs(np.minimum(idx + 1, X.shape[0] - 1), w, X)
    yield "observe_wrong_index", "observe", observe_wrong_index
    for kind in ("beta_inverted", "p_sign", "alpha_from_r"):
        yield "cg_" + kind, "textbook_cg", _cg_mutant(kind)


@pytest.mark.parametrize("name,attr,fn", list(_mutants()), ids=[m[0] for m in _mutants()])
def test_pins_catch_planted_mistake(monkeypatch, name, attr, fn):
    monkeypatch.setattr(E, attr, fn)
    assert _caught(), f"no pin caught the planted mistake {name}"


def test_pins_pass_unmutated():
    assert not _caught()


# --- warm-start network oracle -------------------------------------------------
import oracle.wsnet as NET  # noqa: E402
import tests.test_wsnet_oracle as NPINS  # noqa: E402


def _net_caught() -> bool:
    for pin in (NPINS.test_conv_matches_library_wrap_correlation, NPINS.test_adjoint_identity,
                NPINS.test_weight_gradient_is_exact_linearisation,
                NPINS.test_backward_matches_central_differences,
                NPINS.test_adam_first_step_has_size_lr_and_zero_gradient_keeps_parameters):
        try:
            pin()
        except AssertionError:
            return True
    return False


def _adjoint_wrong_shift(g, w):
    B, O, M = g.shape
    dx = np.zeros((B, w.shape[1], M))
    for bb in range(B):
        for t in range(w.shape[2]):
            dx[bb] += np.roll(w[:, :, t].T @ g[bb], -(t - 2), axis=1)  # sign of the shift flipped
    return dx


def _backward_without_relu_mask(params, acts, gout):
    grads = [None] * len(params)
    g = gout
    for l in range(len(params) - 1, -1, -1):
        w, _ = params[l]
        grads[l] = (_weight_grad_orig(acts[l], g), g.sum(axis=(0, 2)))
        if l > 0:
            g = NET.conv1d_circular_adjoint(g, w)  # ReLU derivative dropped
    return grads


def _adam_without_bias_correction(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    return p - lr * m / (np.sqrt(v) + eps), m, v


_weight_grad_orig = NET.conv1d_weight_grad


def _weight_grad_transposed(x, g):
    return _weight_grad_orig(x, g)[:, :, ::-1].copy()  # taps reversed


@pytest.mark.parametrize("name,mutant", [
    ("conv1d_circular_adjoint", _adjoint_wrong_shift),
    ("backward", _backward_without_relu_mask),
    ("adam_step", _adam_without_bias_correction),
    ("conv1d_weight_grad", _weight_grad_transposed),
])
def test_planted_network_mistake_is_caught(monkeypatch, name, mutant):
    monkeypatch.setattr(NET, name, mutant)
    assert _net_caught(), name


# --- warm-start rule, PCG, features and the Jacobi start ------------------------
import tests.test_oracle_pins_warm as WPINS  # noqa: E402


def _warm_caught() -> bool:
    for pin in (WPINS.test_stall_window_restart_point,
                WPINS.test_pcg_stall_window_with_scalar_preconditioner,
                WPINS.test_pcg_iterates_match_scipy_preconditioned_cg,
                WPINS.test_pcg_terminates_in_at_most_N_steps_for_diagonal_R,
                WPINS.test_pcg_stop_rule_is_the_rinv_norm_of_the_true_residual,
                WPINS.test_features_hand_example,
                WPINS.test_jacobi_z0_matches_formed_psi_diagonal):
        try:
            with np.errstate(all="ignore"):
                pin()
        except (AssertionError, np.linalg.LinAlgError, StopIteration):
            return True
    return False


def _features_divisor_N(D, S, r):
    m, N = D.shape
    s = np.sqrt(np.mean(D * D, axis=0))
    s = np.where(s > 0, s, 1.0)
    x = np.empty((N, 3, m))
    x[:, 0, :] = (D / s).T
    x[:, 1, :] = (np.sum(S * S, axis=1) / N)[None, :]
    x[:, 2, :] = r[None, :]
    return x, s


def _features_l2_scale(D, S, r):
    m, N = D.shape
    s = np.linalg.norm(D, axis=0)
    s = np.where(s > 0, s, 1.0)
    x = np.empty((N, 3, m))
    x[:, 0, :] = (D / s).T
    x[:, 1, :] = (np.sum(S * S, axis=1) / (N - 1))[None, :]
    x[:, 2, :] = r[None, :]
    return x, s


def _jacobi_divisor_N(D, S, r):
    return D / (np.sum(S * S, axis=1) / S.shape[1] + r)[:, None]


_pcg_orig = E.textbook_pcg


def _pcg_with_M_not_Minv(matvec, minv, d, tol, maxit, z0=None, fallback_on_stall=False,
                         record=False):
    return _pcg_orig(matvec, 1.0 / np.asarray(minv), d, tol, maxit, z0, fallback_on_stall, record)


def _pcg_two_norm_stop(matvec, minv, d, tol, maxit, z0=None, fallback_on_stall=False,
                       record=False):
    # preconditioned steps, but the stop rule on the 2-norm of r
    d = np.asarray(d, dtype=np.float64)
    z = np.zeros_like(d) if z0 is None else np.array(z0, dtype=np.float64)
    r = d - matvec(z)
    s = minv * r
    p = s.copy()
    delta = float(r @ s)
    its, hist = 0, [z.copy()]
    while np.linalg.norm(r) > tol * np.linalg.norm(d) and its < maxit and delta > 0:
        q = matvec(p)
        alpha = delta / float(p @ q)
        z = z + alpha * p
        r = r - alpha * q
        s = minv * r
        dn = float(r @ s)
        p = s + (dn / delta) * p
        delta = dn
        its += 1
        hist.append(z.copy())
    return E.CGResult(z, its, [], hist if record else [])


@pytest.mark.parametrize("name,target,attr,value", [
    ("stall_window_4", E, "STALL_WINDOW", 4),
    ("stall_factor_0.8", E, "STALL_FACTOR", 0.8),
    ("stall_window_6", E, "STALL_WINDOW", 6),
    ("features_divisor_N", NET, "features", _features_divisor_N),
    ("features_l2_scale", NET, "features", _features_l2_scale),
    ("jacobi_divisor_N", NET, "jacobi_z0", _jacobi_divisor_N),
    ("pcg_M_not_Minv", E, "textbook_pcg", _pcg_with_M_not_Minv),
    ("pcg_two_norm_stop", E, "textbook_pcg", _pcg_two_norm_stop),
])
def test_planted_warm_start_mistake_is_caught(monkeypatch, name, target, attr, value):
    import oracle
    monkeypatch.setattr(target, attr, value)
    if target is E and hasattr(oracle, attr):  # the package re-exports the function too
        monkeypatch.setattr(oracle, attr, value)
    assert _warm_caught(), name


def test_warm_pins_pass_unmutated():
    assert not _warm_caught()


# --- non-diagonal R -----------------------------------------------------------
import tests.test_oracle_pins_tridiag as TPINS  # noqa: E402


def _tri_caught() -> bool:
    for pin in (TPINS.test_tridiag_R_hand_example,
                lambda: TPINS.test_bruteforce_gain_with_tridiagonal_R(0, 40, 30, 8, 1, True),
                lambda: TPINS.test_reduced_equals_full_with_tridiagonal_R(True),
                TPINS.test_pcg_with_M_equal_R_matches_scipy,
                TPINS.test_pcg_with_M_equal_R_terminates_in_N_steps_and_reaches_cholesky):
        try:
            with np.errstate(all="ignore"):
                pin()
        except (AssertionError, np.linalg.LinAlgError):
            return True
    return False


def _tridiag_R_wrong_band(r_diag, r_off):
    r_diag = np.asarray(r_diag, dtype=np.float64)
    r_off = np.asarray(r_off, dtype=np.float64)
    return np.diag(r_diag) + np.diag(r_off[:-1], 2) + np.diag(r_off[:-1], -2)


def _psi_R_missing_scale(S, R):
    return S @ S.T + np.asarray(R)


_reduced_R_orig = E.enkf_reduced_R


def _reduced_R_unscaled_factor(Xf, idx, w, y, R, eps=None, solver="direct", tol=0.0,
                               maxit=10000):
    N = np.asarray(Xf).shape[1]
    return _reduced_R_orig(Xf, idx, w, y, np.asarray(R) / (N - 1), eps, solver, tol, maxit)


_pcg_op_orig = E.textbook_pcg_op


def _pcg_op_drops_preconditioner(matvec, prec_solve, d, tol, maxit, z0=None,
                                 fallback_on_stall=False, record=False):
    return _pcg_op_orig(matvec, lambda v: v, d, tol, maxit, z0, fallback_on_stall, record)


@pytest.mark.parametrize("name,attr,value", [
    ("tridiag_wrong_band", "tridiag_R", _tridiag_R_wrong_band),
    ("psi_R_missing_scale", "innovation_matrix_R", _psi_R_missing_scale),
    ("reduced_R_unscaled_factor", "enkf_reduced_R", _reduced_R_unscaled_factor),
    ("pcg_op_no_preconditioner", "textbook_pcg_op", _pcg_op_drops_preconditioner),
])
def test_planted_tridiag_mistake_is_caught(monkeypatch, name, attr, value):
    import oracle
    monkeypatch.setattr(E, attr, value)
    monkeypatch.setattr(oracle, attr, value)
    assert _tri_caught(), name


def test_tridiag_pins_pass_unmutated():
    assert not _tri_caught()


# --- sEnKF (Appendix A) ---------------------------------------------------------
import tests.test_oracle_pins_senkf as SPINS  # noqa: E402


def _senkf_caught() -> bool:
    for pin in (lambda: SPINS.test_senkf_matches_per_observation_gains(0, 9, 6, 5, 2, True),
                lambda: SPINS.test_senkf_matches_per_observation_gains(1, 7, 11, 4, 1, False),
                lambda: SPINS.test_senkf_is_exact_when_observed_anomalies_are_orthogonal(
                    40, 15, 16, 4),
                SPINS.test_senkf_large_r_limit):
        try:
            with np.errstate(all="ignore"):
                pin()
        except (AssertionError, np.linalg.LinAlgError, ValueError):
            return True
    return False


def _senkf_mutant(kind):
    def senkf(Xf, idx, w, y, r, eps=None):
        Xf = np.asarray(Xf, dtype=np.float64)
        N = Xf.shape[1]
        Zp = E.observe(idx, w, Xf)
        Zhat = Zp - Zp.mean(axis=1)[:, None]
        rr = np.asarray(r, dtype=np.float64)
        scale = {"r_unscaled": 1, "divisor_N": N}.get(kind, N - 1)
        diag = (Zhat ** 2).sum(axis=1) + scale * rr
        if kind == "no_r":
            diag = (Zhat ** 2).sum(axis=1)
        Y = np.outer(y, np.ones(N)) + (0 if eps is None else eps)
        innov = Y - Zp
        if kind == "innovation_from_mean":
            innov = Y - Zp.mean(axis=1)[:, None]
        if kind == "gain_squared_norm":
            diag = diag ** 2 / diag.mean()
        return Xf + Xf @ Zhat.T @ (innov / diag[:, None])
    return senkf


@pytest.mark.parametrize("kind", ["r_unscaled", "divisor_N", "no_r", "innovation_from_mean",
                                  "gain_squared_norm"])
def test_planted_senkf_mistake_is_caught(monkeypatch, kind):
    import oracle
    monkeypatch.setattr(E, "senkf", _senkf_mutant(kind))
    monkeypatch.setattr(oracle, "senkf", _senkf_mutant(kind))
    assert _senkf_caught(), kind


def test_senkf_pins_pass_unmutated():
    assert not _senkf_caught()


# --- explicit-gain form (Figure 2) ---------------------------------------------
import tests.test_oracle_pins_gain as GPINS  # noqa: E402

_gain_orig = E.enkf_gain_cg


def _gain_caught() -> bool:
    for pin in (lambda: GPINS.test_gain_form_converges_to_bruteforce(0, 30, 12, 7, 2, True),
                lambda: GPINS.test_gain_form_converges_to_bruteforce(1, 20, 25, 6, 1, False),
                GPINS.test_gain_form_prop1_and_monotone,
                lambda: GPINS.test_example1b_termination_and_spectrum(40, 5)):
        try:
            with np.errstate(all="ignore"):
                pin()
        except (AssertionError, np.linalg.LinAlgError, ValueError):
            return True
    return False


def _gain_mutant(kind):
    def gain(Xf, idx, w, y, r, eps=None, tol=1e-10, maxit=10000, record=False):
        Xf = np.asarray(Xf, dtype=np.float64)
        n, N = Xf.shape
        S = E.obs_anomalies(idx, w, Xf)
        Psi = E.innovation_matrix(S, r)
        if kind == "psi_without_r":
            Psi = S @ S.T / (N - 1) + 1e-12 * np.eye(S.shape[0])
        B = E.state_anomalies(Xf) @ S.T
        if kind != "psi_x_unscaled":
            B = B / (N - 1)
        B = B.T
        KT = np.zeros((S.shape[0], n))
        its, iterates = np.zeros(n, dtype=np.int64), []
        for i in range(n):
            res = E.textbook_cg(E.matvec_dense(Psi), B[:, i], tol, maxit, record=record)
            KT[:, i], its[i] = res.z, res.it
            iterates.append(res.iterates)
        D = E.innovations(idx, w, Xf, y, eps)
        if kind == "innovation_from_mean":
            D = D + (E.observe(idx, w, Xf) - E.observe(idx, w, Xf).mean(1)[:, None])
        if kind == "no_eps":
            D = E.innovations(idx, w, Xf, y, None)
        return {"Xa": Xf + KT.T @ D, "KT": KT, "iters": its, "Psi": Psi, "B": B,
                "iterates": iterates}
    return gain


@pytest.mark.parametrize("kind", ["psi_x_unscaled", "psi_without_r", "innovation_from_mean",
                                  "no_eps"])
def test_planted_gain_form_mistake_is_caught(monkeypatch, kind):
    import oracle
    monkeypatch.setattr(E, "enkf_gain_cg", _gain_mutant(kind))
    monkeypatch.setattr(oracle, "enkf_gain_cg", _gain_mutant(kind))
    assert _gain_caught(), kind


def test_gain_pins_pass_unmutated():
    assert not _gain_caught()
