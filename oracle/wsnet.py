"""Oracle for the learned warm start: a plain FP64 1-D convolutional network
over the observation chain, its hand-derived gradients and one Adam step.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this module; the library never does.

The paper has no learned component; the network is the north-star
extension that predicts the CG starting point z0 for each member from
observation-space features (the per-member innovation d_j, the ensemble
variance diag(S S^T)/(N-1) and diag(R)).  Readings (no paper source):

* features, per member j and observation i:
      f_0 = d_ij / s_j,  f_1 = (S S^T)_ii / (N-1),  f_2 = r_i,
  with s_j the root-mean-square of d_j (z is linear in d, so scaling the
  input by s_j and the output back by s_j makes the prediction exactly
  equivariant to the scale of the innovation);
* 4 layers of conv1d along the observation index, kernel 5, circular
  padding (the observed Lorenz-96 chain is periodic), channels
  3 -> 64 -> 64 -> 64 -> 1, ReLU after every layer but the last;
* output: z0_j = s_j * net(f)_j; loss: mean squared error on z_j / s_j;
* Adam with the usual bias correction.

Layout: activations [B, C, M] (batch of members, channels, observations);
weights [C_out, C_in, K]; bias [C_out].
"""
from __future__ import annotations

import numpy as np

KSIZE = 5
HALF = KSIZE // 2
CHANNELS = (3, 64, 64, 64, 1)


def conv1d_circular(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[b, o, i] = bias[o] + sum_{c, t} w[o, c, t] * x[b, c, (i + t - HALF) mod M]."""
    B, C, M = x.shape
    O, C2, K = w.shape
    assert C2 == C
    y = np.empty((B, O, M))
    for bb in range(B):
        acc = np.zeros((O, M)) + b[:, None]
        for t in range(K):
            shifted = np.roll(x[bb], -(t - (K // 2)), axis=1)  # shifted[:, i] = x[:, i + t - half]
            acc += w[:, :, t] @ shifted
        y[bb] = acc
    return y


def conv1d_circular_adjoint(g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """The adjoint of conv1d_circular in x (bias excluded):
    dx[b, c, j] = sum_{o, t} w[o, c, t] * g[b, o, (j - t + HALF) mod M]."""
    B, O, M = g.shape
    _, C, K = w.shape
    dx = np.zeros((B, C, M))
    for bb in range(B):
        for t in range(K):
            contrib = w[:, :, t].T @ g[bb]           # [C, M], indexed by output position i
            dx[bb] += np.roll(contrib, t - (K // 2), axis=1)  # moves position i to i + t - half
    return dx


def conv1d_weight_grad(x: np.ndarray, g: np.ndarray) -> np.ndarray:
    """dW[o, c, t] = sum_{b, i} g[b, o, i] * x[b, c, (i + t - HALF) mod M]."""
    B, C, M = x.shape
    O = g.shape[1]
    dw = np.zeros((O, C, KSIZE))
    for bb in range(B):
        for t in range(KSIZE):
            shifted = np.roll(x[bb], -(t - HALF), axis=1)
            dw[:, :, t] += g[bb] @ shifted.T
    return dw


def init_params(seed: int = 0):
    """He-style initialisation, seeded: list of (w, b) per layer."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in zip(CHANNELS[:-1], CHANNELS[1:]):
        std = np.sqrt(2.0 / (cin * KSIZE))
        params.append((rng.standard_normal((cout, cin, KSIZE)) * std, np.zeros(cout)))
    return params


def forward(params, x: np.ndarray):
    """Returns (output [B, 1, M], activations list for backward).  acts[0] is
    the input; acts[l+1] the post-ReLU output of layer l (pre-activation for
    the last layer)."""
    acts = [x]
    h = x
    for l, (w, b) in enumerate(params):
        h = conv1d_circular(h, w, b)
        if l < len(params) - 1:
            h = np.maximum(h, 0.0)
        acts.append(h)
    return h, acts


def mse_loss(pred: np.ndarray, target: np.ndarray):
    """Mean over all elements of (pred - target)^2, and its gradient in pred."""
    diff = pred - target
    return float(np.mean(diff * diff)), 2.0 * diff / diff.size


def backward(params, acts, gout: np.ndarray):
    """Gradients (dw, db) per layer for the loss whose gradient in the
    network output is gout.  ReLU'(h) taken as [h > 0] on the stored
    post-activation (the same set as the pre-activation > 0)."""
    grads = [None] * len(params)
    g = gout
    for l in range(len(params) - 1, -1, -1):
        w, _ = params[l]
        x = acts[l]
        grads[l] = (conv1d_weight_grad(x, g), g.sum(axis=(0, 2)))
        if l > 0:
            g = conv1d_circular_adjoint(g, w) * (acts[l] > 0.0)
    return grads


def adam_step(p: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, step: int,
              lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba 2015, with bias correction); returns the
    new (p, m, v).  step counts from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def features(D: np.ndarray, S: np.ndarray, r: np.ndarray):
    """Network input [N, 3, m] and the per-member scales s_j (RMS of d_j)."""
    m, N = D.shape
    s = np.sqrt(np.mean(D * D, axis=0))
    s = np.where(s > 0, s, 1.0)
    var = np.sum(S * S, axis=1) / (N - 1)
    x = np.empty((N, 3, m))
    x[:, 0, :] = (D / s).T
    x[:, 1, :] = var[None, :]
    x[:, 2, :] = r[None, :]
    return x, s


def predict_z0(params, D: np.ndarray, S: np.ndarray, r: np.ndarray) -> np.ndarray:
    """z0 [m, N] = s_j * net(features)_j."""
    x, s = features(D, S, r)
    out, _ = forward(params, x)
    return (out[:, 0, :] * s[:, None]).T


def jacobi_z0(D: np.ndarray, S: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Non-learned baseline start: z0 = D / diag(Psi)."""
    N = S.shape[1]
    return D / (np.sum(S * S, axis=1) / (N - 1) + r)[:, None]
