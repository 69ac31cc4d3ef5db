"""Seeded synthetic inputs for the EnKF analysis step.

This module is shared by the CPU oracle side and the GPU side.  It holds the
forecast models and the observation geometry that produce an analysis
problem, and none of the analysis arithmetic itself: no ensemble means of
observations, no innovation matrix, no solve.  Every random number that an
analysis consumes (observation noise, perturbed observations) is drawn here
and handed to both sides as an input.

Conventions (shared with the C-ABI):
  * ensembles are row-major n x N arrays, member index fastest;
  * the observation operator is an (idx, w) pair of m x k arrays: observation i
    is sum_t w[i, t] * x[idx[i, t]];
  * r is the diagonal of R (length m); eps is m x N (column j perturbs
    member j's observation) or None for the deterministic form.

Model references: Lorenz-96 tendency and its fourth-order Runge-Kutta
integration follow Section 6.2 (eq. l96) of the paper; everything about the
2-D advection-diffusion field and the batched set is a synthetic stand-in
whose recipe is stated in the function docstrings.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np

# Child-stream order for np.random.SeedSequence(1000 * cfg + rep).spawn(...)
_STREAMS = ("truth", "ensemble", "geometry", "obs_noise", "eps", "extra")


def streams(cfg: int, rep: int = 0) -> dict:
    """Independent generators for one configuration / repetition."""
    children = np.random.SeedSequence(1000 * cfg + rep).spawn(len(_STREAMS))
    return {name: np.random.default_rng(c) for name, c in zip(_STREAMS, children)}


# --------------------------------------------------------------------------
# Lorenz-96 (Section 6.2, eq. l96): dx_i/dt = (x_{i+1} - x_{i-2}) x_{i-1} - x_i + F
# State index is axis 0, so the same code advances one state or a whole
# n x N ensemble.
# --------------------------------------------------------------------------
def l96_tendency(x: np.ndarray, forcing: float = 8.0) -> np.ndarray:
    return (np.roll(x, -1, axis=0) - np.roll(x, 2, axis=0)) * np.roll(x, 1, axis=0) - x + forcing


def rk4_step(x: np.ndarray, dt: float, forcing: float = 8.0) -> np.ndarray:
    k1 = l96_tendency(x, forcing)
    k2 = l96_tendency(x + 0.5 * dt * k1, forcing)
    k3 = l96_tendency(x + 0.5 * dt * k2, forcing)
    k4 = l96_tendency(x + dt * k3, forcing)
    return x + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def l96_integrate(x: np.ndarray, steps: int, dt: float, forcing: float = 8.0) -> np.ndarray:
    for _ in range(steps):
        x = rk4_step(x, dt, forcing)
    return x


def l96_truth(n: int, rng: np.random.Generator, steps: int = 1000, dt: float = 0.05,
              forcing: float = 8.0) -> np.ndarray:
    """Truth after `steps` RK4 steps from an N(0, 1) start."""
    return l96_integrate(rng.standard_normal(n), steps, dt, forcing)


def every_kth(n: int, stride: int = 2) -> tuple[np.ndarray, np.ndarray]:
    """H that observes variables 0, stride, 2*stride, ... (k = 1, w = 1)."""
    idx = np.arange(0, n, stride, dtype=np.int32)[:, None]
    return idx, np.ones(idx.shape, dtype=np.float64)


def identity_obs(n: int) -> tuple[np.ndarray, np.ndarray]:
    idx = np.arange(n, dtype=np.int32)[:, None]
    return idx, np.ones(idx.shape, dtype=np.float64)


def apply_obs_operator(idx: np.ndarray, w: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Observe a state (or a state ensemble) with an (idx, w) operator.

    Used to synthesise y = H x_t + v; it is the measurement model of the
    synthetic twin experiment, not part of the analysis.
    """
    out = np.zeros((idx.shape[0],) + x.shape[1:], dtype=np.float64)
    for t in range(idx.shape[1]):
        wt = w[:, t] if x.ndim == 1 else w[:, t:t + 1]
        out += wt * x[idx[:, t]]
    return out


@dataclasses.dataclass
class Problem:
    """One analysis problem, all arrays FP64 (cast by the caller)."""
    Xf: np.ndarray            # n x N
    idx: np.ndarray           # m x k int32
    w: np.ndarray             # m x k
    y: np.ndarray             # m
    r: np.ndarray             # m, diagonal of R
    eps: Optional[np.ndarray]  # m x N or None
    tol: float
    maxit: int
    truth: Optional[np.ndarray] = None
    name: str = ""

    @property
    def n(self) -> int:
        return self.Xf.shape[0]

    @property
    def N(self) -> int:
        return self.Xf.shape[1]

    @property
    def m(self) -> int:
        return self.idx.shape[0]

    @property
    def k(self) -> int:
        return self.idx.shape[1]


def draw_obs(truth, idx, w, r, rng_obs, rng_eps, N, stochastic=True):
    """y = H x_t + N(0, R) and, for the stochastic form, eps ~ N(0, R) (m x N)."""
    sd = np.sqrt(r)
    y = apply_obs_operator(idx, w, truth) + sd * rng_obs.standard_normal(r.shape[0])
    eps = (sd[:, None] * rng_eps.standard_normal((r.shape[0], N))) if stochastic else None
    return y, eps


# --------------------------------------------------------------------------
# Configurations
# --------------------------------------------------------------------------
def config1(rep: int = 0, stochastic: bool = True) -> Problem:
    """Lorenz-96 n=40, F=8, truth after 1000 RK4 steps (dt 0.05) from N(0,1);
    N=20 members = truth + N(0,1); H observes every 2nd variable (m=20); R=I;
    y = Hx + N(0,R); one FP64 analysis at CG tol 1e-10."""
    g = streams(1, rep)
    n, N = 40, 20
    xt = l96_truth(n, g["truth"])
    Xf = xt[:, None] + g["ensemble"].standard_normal((n, N))
    idx, w = every_kth(n, 2)
    r = np.ones(idx.shape[0])
    y, eps = draw_obs(xt, idx, w, r, g["obs_noise"], g["eps"], N, stochastic)
    return Problem(Xf, idx, w, y, r, eps, 1e-10, 1000, truth=xt, name="cfg1")


def random_problem(n: int, m: int, N: int, k: int = 1, seed: int = 0, r_lo: float = 0.5,
                   r_hi: float = 2.0, stochastic: bool = True, duplicate_idx: bool = False,
                   tol: float = 1e-12, maxit: int = 10000, spread: float = 1.0) -> Problem:
    """Unstructured random problem for parity sweeps (Gaussian ensemble,
    random indices and positive weights, r ~ U[r_lo, r_hi])."""
    rng = np.random.default_rng(seed)
    xt = rng.standard_normal(n)
    Xf = xt[:, None] + spread * rng.standard_normal((n, N))
    if duplicate_idx or m * k > n:
        idx = rng.integers(0, n, size=(m, k)).astype(np.int32)
    else:
        idx = rng.choice(n, size=m * k, replace=False).reshape(m, k).astype(np.int32)
    w = rng.uniform(0.1, 1.0, size=(m, k))
    r = rng.uniform(r_lo, r_hi, size=m) if r_hi > r_lo else np.full(m, r_lo)
    y = apply_obs_operator(idx, w, xt) + np.sqrt(r) * rng.standard_normal(m)
    eps = np.sqrt(r)[:, None] * rng.standard_normal((m, N)) if stochastic else None
    return Problem(Xf, idx, w, y, r, eps, tol, maxit, truth=xt, name=f"rand_n{n}_m{m}_N{N}_k{k}")


def ma1_tridiag_noise(rng: np.random.Generator, m: int, cols: int, sigma: float,
                     rho: float) -> np.ndarray:
    """Samples with the tridiagonal Toeplitz covariance sigma^2 (diagonal),
    sigma^2 rho (beside it), 0 <= rho < 0.5, drawn as a moving average
    v_i = sigma (a u_i + b u_{i+1}) of independent N(0, 1) values, with
    a^2 + b^2 = 1 and a b = rho (exact for every i, no factorisation)."""
    a = 0.5 * (np.sqrt(1 + 2 * rho) + np.sqrt(1 - 2 * rho))
    b = 0.5 * (np.sqrt(1 + 2 * rho) - np.sqrt(1 - 2 * rho))
    u = rng.standard_normal((m + 1, cols))
    return sigma * (a * u[:-1] + b * u[1:])


def example2(n: int = 4096, N: int = 100, sigma: float = 0.3, rho: float = 0.2, rep: int = 0,
             tol: float = 1e-6, maxit: int = 2000, spin_steps: int = 200,
             stochastic: bool = True):
    """The paper's Example 2 setting at one analysis: Lorenz-96 (F = 8) with
    every variable observed (H = I, m = n) and the tridiagonal Toeplitz
    observation covariance (sigma^2, sigma^2 rho); truth spun up from N(0,1)
    by `spin_steps` RK4 steps of dt 0.05, members = truth + N(0, 1).
    Returns (Problem, r_off): Problem.r is diag(R), r_off the off-diagonal."""
    g = streams(6, rep)
    xt = l96_truth(n, g["truth"], steps=spin_steps)
    Xf = xt[:, None] + g["ensemble"].standard_normal((n, N))
    idx, w = identity_obs(n)
    r = np.full(n, sigma * sigma)
    r_off = np.full(n - 1, sigma * sigma * rho)
    y = xt + ma1_tridiag_noise(g["obs_noise"], n, 1, sigma, rho)[:, 0]
    eps = ma1_tridiag_noise(g["eps"], n, N, sigma, rho) if stochastic else None
    return Problem(Xf, idx, w, y, r, eps, tol, maxit, truth=xt, name="ex2"), r_off


def example1b(m: int = 200, N: int = 50, rep: int = 0, q: float = 0.1,
              tol: float = 1e-12, maxit: int = 10000) -> Problem:
    """The paper's Example 1b at its first analysis (Section 6.1): a constant
    random truth x^t ~ N(0, I_m), H = F = I (p = m), R = I, Q = q I (0.1).
    The initial ensemble is drawn from the truth's distribution, N(0, I); the
    first forecast adds model noise N(0, Q) to each member; y = x^t + v with
    v ~ N(0, R); stochastic perturbations E ~ N(0, R)."""
    g = streams(7, rep)
    xt = g["truth"].standard_normal(m)
    X0 = g["ensemble"].standard_normal((m, N))
    Xf = X0 + np.sqrt(q) * g["extra"].standard_normal((m, N))
    idx, w = identity_obs(m)
    r = np.ones(m)
    y = xt + g["obs_noise"].standard_normal(m)
    eps = g["eps"].standard_normal((m, N))
    return Problem(Xf, idx, w, y, r, eps, tol, maxit, truth=xt, name=f"ex1b_m{m}_N{N}")


class L96Cycler:
    """Configuration 2's twin experiment: Lorenz-96 n=4096, F=8, every 2nd
    variable observed (m=2048), N=64, R=0.5 I, forecast ensemble spread N(0,1),
    5 RK4 steps of dt=0.05 between analyses, stochastic EnKF.

    The analysis is supplied by the caller (`analysis(problem) -> Xa`), so this
    driver holds no analysis arithmetic.  Cycle c uses generator streams
    derived from (seed, c), which makes every cycle's draws reproducible
    regardless of what drove the trajectory.
    """

    def __init__(self, n: int = 4096, N: int = 64, r_value: float = 0.5, obs_every: int = 5,
                 dt: float = 0.05, seed: int = 0, tol: float = 1e-6, maxit: int = 1000,
                 spinup: int = 1000):
        self.n, self.N, self.dt, self.obs_every = n, N, dt, obs_every
        self.tol, self.maxit, self.seed = tol, maxit, seed
        g = streams(2, seed)
        self.truth = l96_truth(n, g["truth"], steps=spinup, dt=dt)
        self.X = self.truth[:, None] + g["ensemble"].standard_normal((n, N))
        self.idx, self.w = every_kth(n, 2)
        self.r = np.full(self.idx.shape[0], r_value)
        self.cycle = 0

    def _rngs(self):
        ss = np.random.SeedSequence([2, self.seed, self.cycle])
        a, b = ss.spawn(2)
        return np.random.default_rng(a), np.random.default_rng(b)

    def forecast(self):
        self.truth = l96_integrate(self.truth, self.obs_every, self.dt)
        self.X = l96_integrate(self.X, self.obs_every, self.dt)

    def problem(self) -> Problem:
        ro, re = self._rngs()
        y, eps = draw_obs(self.truth, self.idx, self.w, self.r, ro, re, self.N)
        return Problem(self.X.copy(), self.idx, self.w, y, self.r, eps, self.tol, self.maxit,
                       truth=self.truth.copy(), name=f"cfg2_c{self.cycle}")

    def step(self, analysis: Callable[[Problem], np.ndarray]) -> Problem:
        """Forecast, draw observations, analyse; returns the problem analysed."""
        self.forecast()
        prob = self.problem()
        self.X = np.asarray(analysis(prob), dtype=np.float64)
        self.cycle += 1
        return prob


# --------------------------------------------------------------------------
# Configuration 3: 2-D advection-diffusion field.
# --------------------------------------------------------------------------
def gaussian_random_fields(shape: tuple[int, int], count: int, length: float,
                           rng: np.random.Generator) -> np.ndarray:
    """`count` stationary unit-variance Gaussian random fields on a periodic
    grid, covariance exp(-d^2 / (2 length^2)) with minimum-image distance d,
    sampled by circulant embedding: field = ifft2(sqrt(spec) * fft2(white))."""
    ny, nx = shape
    dy = np.minimum(np.arange(ny), ny - np.arange(ny))
    dx = np.minimum(np.arange(nx), nx - np.arange(nx))
    d2 = dy[:, None] ** 2 + dx[None, :] ** 2
    cov = np.exp(-d2 / (2.0 * length ** 2))
    spec = np.clip(np.fft.fft2(cov).real, 0.0, None)
    amp = np.sqrt(spec)
    white = rng.standard_normal((count, ny, nx))
    fields = np.fft.ifft2(amp[None] * np.fft.fft2(white, axes=(1, 2)), axes=(1, 2)).real
    var = spec.sum() / (ny * nx)  # theoretical variance of the sampled field
    return fields / np.sqrt(var)


def advect_diffuse(u: np.ndarray, steps: int = 20, vel=(0.5, 0.25), kappa: float = 0.05) -> np.ndarray:
    """Explicit periodic upwind advection (velocity in cells/step, positive)
    plus diffusion (cells^2/step) on the last two axes."""
    cx, cy = vel
    for _ in range(steps):
        lap = (np.roll(u, 1, -1) + np.roll(u, -1, -1) + np.roll(u, 1, -2) + np.roll(u, -1, -2) - 4 * u)
        u = u - cx * (u - np.roll(u, 1, -1)) - cy * (u - np.roll(u, 1, -2)) + kappa * lap
    return u


def bilinear_obs(shape: tuple[int, int], m: int, rng: np.random.Generator):
    """m positions uniform on the periodic [0, nx) x [0, ny) grid; each
    observation is the bilinear interpolant of its 4 surrounding nodes
    (k = 4, weights >= 0 summing to 1), flattened index iy * nx + ix."""
    ny, nx = shape
    px = rng.uniform(0, nx, m)
    py = rng.uniform(0, ny, m)
    ix0 = np.floor(px).astype(np.int64) % nx
    iy0 = np.floor(py).astype(np.int64) % ny
    fx = px - np.floor(px)
    fy = py - np.floor(py)
    ix1 = (ix0 + 1) % nx
    iy1 = (iy0 + 1) % ny
    idx = np.stack([iy0 * nx + ix0, iy0 * nx + ix1, iy1 * nx + ix0, iy1 * nx + ix1], 1).astype(np.int32)
    w = np.stack([(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy], 1)
    return idx, w


def config3(rep: int = 0, grid: int = 256, m: int = 16384, N: int = 128, length: float = 8.0,
            tol: float = 1e-6, maxit: int = 2000) -> Problem:
    """2-D advection-diffusion 256x256 (n=65536): truth and N=128 members are
    independent unit-variance GRFs (length scale 8 cells) advanced 20 upwind
    advection-diffusion steps; m=16384 random-cell observations with bilinear
    weights; diag R ~ U[0.5, 2]; stochastic EnKF."""
    g = streams(3, rep)
    shape = (grid, grid)
    fields = gaussian_random_fields(shape, N + 1, length, g["truth"])
    fields = advect_diffuse(fields)
    xt = fields[0].reshape(-1)
    Xf = np.ascontiguousarray(fields[1:].reshape(N, -1).T)
    idx, w = bilinear_obs(shape, m, g["geometry"])
    r = g["obs_noise"].uniform(0.5, 2.0, m)
    y, eps = draw_obs(xt, idx, w, r, g["obs_noise"], g["eps"], N)
    return Problem(Xf, idx, w, y, r, eps, tol, maxit, truth=xt, name="cfg3")


# --------------------------------------------------------------------------
# Configuration 4: batched, uneven Lorenz-96 filters.
# --------------------------------------------------------------------------
def config4(count: int = 256, rep: int = 0, n_lo: int = 256, n_hi: int = 8192,
            Ns=(16, 32, 64), tol: float = 1e-6, maxit: int = 1000, heal_steps: int = 20) -> list:
    """`count` independent Lorenz-96 filters, n = 4 * U{n_lo..n_hi} (so n in
    [1024, 32768] and m = n/4 is an integer), m distinct sorted random
    indices, N uniform over `Ns`, R = I, stochastic EnKF.  Truths are windows
    of one spun-up n=32768 state (1000 RK4 steps, dt 0.05) healed by
    `heal_steps` RK4 steps of their own size."""
    g = streams(4, rep)
    base = l96_truth(4 * n_hi, g["truth"])
    probs = []
    for b in range(count):
        n = 4 * int(g["geometry"].integers(n_lo, n_hi + 1))
        m = n // 4
        N = int(Ns[int(g["geometry"].integers(0, len(Ns)))])
        off = int(g["geometry"].integers(0, base.size))
        xt = l96_integrate(np.roll(base, -off)[:n].copy(), heal_steps, 0.05)
        Xf = xt[:, None] + g["ensemble"].standard_normal((n, N))
        idx = np.sort(g["geometry"].choice(n, size=m, replace=False)).astype(np.int32)[:, None]
        w = np.ones(idx.shape)
        r = np.ones(m)
        y, eps = draw_obs(xt, idx, w, r, g["obs_noise"], g["eps"], N)
        probs.append(Problem(Xf, idx, w, y, r, eps, tol, maxit, truth=xt, name=f"cfg4_{b}"))
    return probs
