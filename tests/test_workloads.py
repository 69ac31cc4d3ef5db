"""Checks on the synthetic input generators (no analysis arithmetic here)."""
import numpy as np

import workloads as W


def test_l96_nonlinear_term_conserves_energy():
    # sum_i x_i (x_{i+1} - x_{i-2}) x_{i-1} = 0 for cyclic indices (eq. l96)
    x = np.random.default_rng(0).standard_normal(37)
    adv = W.l96_tendency(x, 0.0) + x
    assert abs(float(x @ adv)) < 1e-12 * float(x @ x) * np.abs(x).max()


def test_rk4_is_fourth_order():
    x0 = np.random.default_rng(1).standard_normal(40) + 8
    T = 0.2
    ref = W.l96_integrate(x0, 256, T / 256)
    e1 = np.linalg.norm(W.l96_integrate(x0, 8, T / 8) - ref)
    e2 = np.linalg.norm(W.l96_integrate(x0, 16, T / 16) - ref)
    assert 12.0 < e1 / e2 < 20.0


def test_config1_shapes_and_determinism():
    a, b = W.config1(), W.config1()
    assert a.Xf.shape == (40, 20) and a.idx.shape == (20, 1) and a.m == 20
    assert np.array_equal(a.Xf, b.Xf) and np.array_equal(a.eps, b.eps)
    assert np.array_equal(a.idx[:, 0], np.arange(0, 40, 2))
    assert np.all(a.r == 1.0) and a.tol == 1e-10
    c = W.config1(rep=1)
    assert not np.array_equal(a.Xf, c.Xf)
    # spun-up Lorenz-96 at F = 8: mean ~2.3, std ~3.6
    assert 0.5 < a.truth.mean() < 4.5 and 2.0 < a.truth.std() < 5.0


def test_grf_unit_variance_and_length_scale():
    f = W.gaussian_random_fields((128, 128), 16, 8.0, np.random.default_rng(2))
    assert abs(f.var() - 1.0) < 0.1
    c1 = np.mean(f * np.roll(f, 8, axis=2))  # expected exp(-0.5) ~ 0.61
    assert 0.45 < c1 < 0.75


def test_bilinear_weights():
    idx, w = W.bilinear_obs((64, 64), 500, np.random.default_rng(3))
    assert idx.shape == (500, 4) and idx.min() >= 0 and idx.max() < 64 * 64
    assert np.all(w >= 0) and np.allclose(w.sum(1), 1.0)
    # bilinear interpolation reproduces a linear-in-x field away from the wrap
    xs = np.tile(np.arange(64, dtype=float), (64, 1)).reshape(-1)
    vals = W.apply_obs_operator(idx, w, xs)
    ix0 = idx[:, 0] % 64
    ok = ix0 < 63
    assert np.all((vals[ok] >= ix0[ok] - 1e-12) & (vals[ok] <= ix0[ok] + 1 + 1e-12))


def test_advection_diffusion_conserves_mass():
    u = np.random.default_rng(4).standard_normal((32, 32))
    v = W.advect_diffuse(u, steps=5)
    assert abs(u.sum() - v.sum()) < 1e-9 and v.std() < u.std()


def test_config4_recipe_small():
    probs = W.config4(count=6, n_lo=256, n_hi=512, heal_steps=2)
    for p in probs:
        assert p.n % 4 == 0 and p.m == p.n // 4 and p.N in (16, 32, 64)
        assert np.all(np.diff(p.idx[:, 0]) > 0)


def test_cycler_reproducible():
    a = W.L96Cycler(n=64, N=8, spinup=50)
    b = W.L96Cycler(n=64, N=8, spinup=50)
    pa = a.step(lambda p: p.Xf)
    pb = b.step(lambda p: p.Xf)
    assert np.array_equal(pa.y, pb.y) and np.array_equal(pa.eps, pb.eps)
    assert pa.m == 32 and np.all(pa.r == 0.5)


def test_ma1_noise_has_the_tridiagonal_toeplitz_covariance():
    import numpy as np
    import workloads as W
    v = W.ma1_tridiag_noise(np.random.default_rng(3), 6, 400000, 0.3, 0.2)
    C = np.cov(v)
    want = 0.09 * (np.eye(6) + 0.2 * (np.eye(6, k=1) + np.eye(6, k=-1)))
    assert np.max(np.abs(C - want)) < 1.5e-3
