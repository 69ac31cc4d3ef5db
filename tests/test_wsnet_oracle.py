"""Pins for the warm-start network oracle (oracle/wsnet.py), each independent
of the code it checks: a library correlation, the adjoint identity, exact
linearity in the weights, central finite differences of the loss, Adam's
known first-step behaviour, and exact scale equivariance."""
import numpy as np
import pytest
from scipy.ndimage import correlate1d

from oracle import wsnet as N


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv_matches_library_wrap_correlation():
    x = _rand((2, 3, 11), 1)
    w = _rand((4, 3, 5), 2)
    b = _rand(4, 3)
    y = N.conv1d_circular(x, w, b)
    ref = np.zeros_like(y)
    for bb in range(2):
        for o in range(4):
            ref[bb, o] = b[o] + sum(correlate1d(x[bb, c], w[o, c], mode="wrap", origin=0)
                                    for c in range(3))
    assert np.max(np.abs(y - ref)) < 1e-12


def test_adjoint_identity():
    x = _rand((3, 5, 17), 4)
    g = _rand((3, 6, 17), 5)
    w = _rand((6, 5, 5), 6)
    lhs = np.sum(N.conv1d_circular(x, w, np.zeros(6)) * g)
    rhs = np.sum(x * N.conv1d_circular_adjoint(g, w))
    assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(lhs))


def test_weight_gradient_is_exact_linearisation():
    x = _rand((2, 4, 13), 7)
    g = _rand((2, 3, 13), 8)
    dw_dir = _rand((3, 4, 5), 9)
    dw = N.conv1d_weight_grad(x, g)
    lhs = np.sum(dw * dw_dir)
    rhs = np.sum(N.conv1d_circular(x, dw_dir, np.zeros(3)) * g)
    assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(rhs))


def _small_params(seed):
    rng = np.random.default_rng(seed)
    ch = (3, 4, 4, 4, 1)
    return [(rng.standard_normal((co, ci, 5)) * 0.5, rng.standard_normal(co) * 0.1)
            for ci, co in zip(ch[:-1], ch[1:])]


def _loss(params, x, t):
    out, _ = N.forward(params, x)
    return N.mse_loss(out, t)[0]


def test_backward_matches_central_differences():
    params = _small_params(10)
    x = _rand((2, 3, 12), 11)
    t = _rand((2, 1, 12), 12)
    out, acts = N.forward(params, x)
    _, gout = N.mse_loss(out, t)
    grads = N.backward(params, acts, gout)
    h = 1e-6
    rng = np.random.default_rng(13)
    for l, (w, b) in enumerate(params):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in w.shape)
            wp = [(ww.copy(), bb.copy()) for ww, bb in params]
            wm = [(ww.copy(), bb.copy()) for ww, bb in params]
            wp[l][0][idx] += h
            wm[l][0][idx] -= h
            fd = (_loss(wp, x, t) - _loss(wm, x, t)) / (2 * h)
            assert abs(fd - grads[l][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx)
        k = int(rng.integers(0, b.shape[0]))
        bp = [(ww.copy(), bb.copy()) for ww, bb in params]
        bm = [(ww.copy(), bb.copy()) for ww, bb in params]
        bp[l][1][k] += h
        bm[l][1][k] -= h
        fd = (_loss(bp, x, t) - _loss(bm, x, t)) / (2 * h)
        assert abs(fd - grads[l][1][k]) <= 1e-6 * max(1.0, abs(fd)), (l, k)


def test_adam_first_step_has_size_lr_and_zero_gradient_keeps_parameters():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([3.0, -0.01, 1e4])
    m = v = np.zeros(3)
    p1, m1, v1 = N.adam_step(p, g, m, v, 1, lr=1e-3)
    # bias-corrected first step: -lr * g / (|g| + eps)
    assert np.allclose(p1 - p, -1e-3 * np.sign(g), rtol=1e-5)
    p2, _, _ = N.adam_step(p, np.zeros(3), np.zeros(3), np.zeros(3), 1)
    assert np.array_equal(p2, p)


def test_prediction_is_equivariant_to_innovation_scale():
    params = N.init_params(3)
    rng = np.random.default_rng(14)
    S = rng.standard_normal((40, 6))
    S -= S.mean(1, keepdims=True)
    D = rng.standard_normal((40, 6))
    r = rng.uniform(0.5, 2.0, 40)
    z1 = N.predict_z0(params, D, S, r)
    z2 = N.predict_z0(params, 3.5 * D, S, r)
    assert np.max(np.abs(z2 - 3.5 * z1)) <= 1e-12 * max(1.0, np.max(np.abs(z2)))


def test_jacobi_start_is_exact_for_diagonal_innovation_matrix():
    # S = 0 (identical members): Psi = diag(r), so D / diag(Psi) solves it
    rng = np.random.default_rng(15)
    D = rng.standard_normal((30, 5))
    r = rng.uniform(0.5, 2.0, 30)
    assert np.allclose(N.jacobi_z0(D, np.zeros((30, 5)), r), D / r[:, None], rtol=0, atol=0)


def test_output_shapes_and_channel_plan():
    params = N.init_params(0)
    assert [w.shape for w, _ in params] == [(64, 3, 5), (64, 64, 5), (64, 64, 5), (1, 64, 5)]
    out, acts = N.forward(params, _rand((2, 3, 16), 16))
    assert out.shape == (2, 1, 16) and len(acts) == 5
