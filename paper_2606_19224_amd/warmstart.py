"""Training data and training loop for the learned warm start.

Pairs come from the filter itself: for every analysis, the network features
of each member (cgd_wsnet_features) and the converged solution z_j of the
zero-start CG, scaled by the member's innovation RMS s_j (the network's
target).  Training runs the library's own kernels (cgd_wsnet_train_step);
PyTorch only holds the tensors and shuffles minibatch indices.
"""
from __future__ import annotations

import torch

from . import binding


class PairCollector:
    """Collects (features, target) pairs from analyses of one shape."""

    def __init__(self, net: "binding.WarmStartNet"):
        self.net = net
        self.feats, self.targets = [], []

    def add(self, Xf, idx, w, y, r, eps=None, tol=1e-6, maxit=1000, prec="fp32"):
        """Analyse one problem from a zero start and keep its pairs; returns
        the analysis result (X_a, per-member iterations)."""
        feat, scale = self.net.features(Xf, idx, w, y, r, eps)
        out = binding.analysis(Xf, idx, w, y, r, eps, tol=tol, maxit=maxit, prec=prec, want_z=True,
                               want_iters=True, stats=False)
        self.feats.append(feat)
        self.targets.append(self.net.target(out["Z"], scale))
        return out

    def tensors(self, count=None):
        feat = torch.cat(self.feats)
        target = torch.cat(self.targets)
        if count is not None:
            feat, target = feat[:count].contiguous(), target[:count].contiguous()
        return feat, target


def train(net: "binding.WarmStartNet", feat: torch.Tensor, target: torch.Tensor, epochs: int,
          batch: int = 64, lr: float = 1e-3, seed: int = 0, start_epoch: int = 0,
          checkpoint: str = None) -> list:
    """Adam on shuffled minibatches of `batch` pairs; returns the mean
    training loss of every epoch (one host synchronisation per epoch).

    Resuming: epochs start_epoch .. epochs-1 are run, with the shuffles those
    epochs have in an uninterrupted run (the first start_epoch permutations
    are drawn and dropped), so a run stopped after epoch e and resumed from
    its checkpoint with start_epoch = e ends with the same parameters.  With
    `checkpoint`, the state (net.save, plus the epoch) is written after every
    epoch."""
    gen = torch.Generator(device="cpu").manual_seed(seed)
    n = feat.shape[0]
    nb = n // batch
    history = []
    for _ in range(start_epoch):
        torch.randperm(n, generator=gen)
    for epoch in range(start_epoch, epochs):
        perm = torch.randperm(n, generator=gen)[: nb * batch].to(feat.device)
        acc = torch.zeros(1, dtype=torch.float32, device=feat.device)
        for b in range(nb):
            sel = perm[b * batch:(b + 1) * batch]
            fb = feat.index_select(0, sel).contiguous()
            tb = target.index_select(0, sel).contiguous()
            acc += net.train_step(fb, tb, lr=lr)
        history.append(acc.item() / max(nb, 1))
        if checkpoint:
            net.save(checkpoint, epoch=epoch + 1)
    return history


def jacobi_z0(net: "binding.WarmStartNet", feat: torch.Tensor, scale: torch.Tensor,
              out=None) -> torch.Tensor:
    """Non-learned baseline start z0 = D / diag(Psi) [m, N], from the features
    (the library's cgd_wsnet_jacobi_z0)."""
    return net.jacobi_z0(feat, scale, out=out)
