"""The warm-start network's HIP kernels (BF16 MFMA, FP32 accumulation)
against the FP64 oracle: features, forward, loss and gradient, Adam, the z0
pipeline, and that training lowers the loss.

BF16 tolerance: operands are rounded to 8 significant bits (unit roundoff
u = 2^-9 ~ 2e-3) before every product, with FP32 accumulation; through four
layers the relative error of an output or gradient stays within a few times
4 * 2u, so the bar is 3e-2 for outputs and losses and 5e-2 for gradients
(which pass through the same four layers twice), with a cosine similarity
close to 1 as a direction check."""
import numpy as np
import pytest

import oracle.enkf as E
import oracle.wsnet as NET
import workloads as W
from tests.gpu_util import dev_problem, rel, rounded, say

pytestmark = pytest.mark.gpu


def _net(lib, seed=0):
    return lib.WarmStartNet(seed=seed)


def _cos(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


def _problem():
    cyc = W.L96Cycler(n=1024, N=32, tol=1e-6)
    return rounded(cyc.problem())


def test_features_match_oracle(lib):
    import torch
    p = _problem()
    net = _net(lib)
    feat, scale = net.features(**dev_problem(p, "fp32"))
    torch.cuda.synchronize()
    S = E.obs_anomalies(p.idx, p.w, p.Xf)
    D = E.innovations(p.idx, p.w, p.Xf, p.y, p.eps)
    x, s = NET.features(D, S, p.r)
    assert rel(scale.cpu().numpy(), s) <= 1e-6
    assert rel(feat.cpu().numpy()[:, :, :3], np.transpose(x, (0, 2, 1))) <= 1e-5
    assert np.all(feat.cpu().numpy()[:, :, 3] == 0)


@pytest.mark.parametrize("B,m", [(3, 300), (2, 64), (1, 2048)])
def test_forward_matches_oracle(lib, B, m):
    import torch
    net = _net(lib, seed=1)
    rng = np.random.default_rng(2)
    x = np.stack([rng.standard_normal((B, m)), rng.uniform(0.5, 3, (B, m)),
                  rng.uniform(0.5, 2, (B, m))], axis=1)            # [B, 3, m]
    feat = torch.zeros((B, m, 4), dtype=torch.float32, device="cuda:0")
    feat[:, :, :3] = torch.as_tensor(np.transpose(x, (0, 2, 1)), device="cuda:0")
    out = net.forward(feat)
    torch.cuda.synchronize()
    params = lib.wsnet_unpack(net.params.cpu().numpy())
    xb = np.transpose(feat.cpu().numpy()[:, :, :3].astype(np.float64), (0, 2, 1))
    ref, _ = NET.forward(params, xb)
    err = rel(out.cpu().numpy(), ref[:, 0, :])
    say(f"case: wsnet forward B={B} m={m}: rel err {err:.2e}")
    assert err <= 3e-2


def _batch(B, m, seed):
    import torch
    rng = np.random.default_rng(seed)
    x = np.stack([rng.standard_normal((B, m)), rng.uniform(0.5, 3, (B, m)),
                  rng.uniform(0.5, 2, (B, m))], axis=1)
    feat = torch.zeros((B, m, 4), dtype=torch.float32, device="cuda:0")
    feat[:, :, :3] = torch.as_tensor(np.transpose(x, (0, 2, 1)), device="cuda:0")
    t = rng.standard_normal((B, m)) * 0.3
    target = torch.as_tensor(t, dtype=torch.float32, device="cuda:0")
    xb = np.transpose(feat.cpu().numpy()[:, :, :3].astype(np.float64), (0, 2, 1))
    return feat, target, xb, target.cpu().numpy().astype(np.float64)[:, None, :]


@pytest.mark.parametrize("B,m", [(4, 200), (2, 256)])
def test_loss_and_gradient_match_oracle(lib, B, m):
    import torch
    net = _net(lib, seed=3)
    feat, target, xb, tb = _batch(B, m, 4)
    loss, grad = net.loss_grad(feat, target)
    torch.cuda.synchronize()
    params = lib.wsnet_unpack(net.params.cpu().numpy())
    out, acts = NET.forward(params, xb)
    lref, gout = NET.mse_loss(out, tb)
    gref = NET.backward(params, acts, gout)
    assert abs(loss.item() - lref) <= 3e-2 * lref
    g = lib.wsnet_unpack(grad.cpu().numpy())
    for l, ((gw, gb), (rw, rb)) in enumerate(zip(g, gref)):
        ew, cw = rel(gw, rw), _cos(gw, rw)
        say(f"case: wsnet gradient B={B} m={m} layer {l}: W rel {ew:.2e} cos {cw:.5f}, "
            f"b rel {rel(gb, rb):.2e}")
        assert ew <= 5e-2 and cw >= 0.998
        assert rel(gb, rb) <= 5e-2


def test_adam_step_matches_oracle(lib):
    import torch
    net = _net(lib, seed=5)
    feat, target, _, _ = _batch(2, 128, 6)
    p0 = net.params.cpu().numpy().astype(np.float64)
    _, grad = net.loss_grad(feat, target)
    g = grad.cpu().numpy().astype(np.float64)
    net.train_step(feat, target, lr=1e-3)        # recomputes the same gradient (deterministic)
    torch.cuda.synchronize()
    p1, m1, v1 = NET.adam_step(p0, g, np.zeros_like(p0), np.zeros_like(p0), 1, lr=1e-3)
    assert np.max(np.abs(net.params.cpu().numpy() - p1)) <= 1e-6
    assert np.max(np.abs(net.m.cpu().numpy() - m1)) <= 1e-6 * max(1.0, np.abs(m1).max())
    # second step from the stored moments
    _, grad2 = net.loss_grad(feat, target)
    g2 = grad2.cpu().numpy().astype(np.float64)
    q0 = net.params.cpu().numpy().astype(np.float64)
    net.train_step(feat, target, lr=1e-3)
    torch.cuda.synchronize()
    p2, _, _ = NET.adam_step(q0, g2, m1, v1, 2, lr=1e-3)
    assert np.max(np.abs(net.params.cpu().numpy() - p2)) <= 2e-6


def test_predict_z0_is_scaled_forward_of_features(lib):
    import torch
    p = _problem()
    net = _net(lib, seed=7)
    d = dev_problem(p, "fp32")
    z0 = net.predict_z0(**d)
    feat, scale = net.features(**d)
    out = net.forward(feat)
    torch.cuda.synchronize()
    z_ref = (out * scale[:, None]).T.contiguous()
    assert torch.equal(z0, z_ref)
    S = E.obs_anomalies(p.idx, p.w, p.Xf)
    D = E.innovations(p.idx, p.w, p.Xf, p.y, p.eps)
    zo = NET.predict_z0(lib.wsnet_unpack(net.params.cpu().numpy()), D, S, p.r)
    assert rel(z0.cpu().numpy(), zo) <= 3e-2


def test_training_lowers_the_loss(lib):
    import torch
    net = _net(lib, seed=8)
    feat, target, _, _ = _batch(8, 256, 9)
    first = net.loss_grad(feat, target)[0].item()
    for _ in range(200):
        net.train_step(feat, target, lr=2e-3)
    torch.cuda.synchronize()
    last = net.loss_grad(feat, target)[0].item()
    say(f"case: wsnet training loss {first:.4f} -> {last:.4f}")
    assert last < 0.5 * first


def test_training_resumes_from_a_checkpoint(lib, tmp_path):
    """Four epochs in one run, against two epochs, a checkpoint, a fresh
    network loaded from it and two more epochs (warmstart.train with
    start_epoch = 2): the same parameters and Adam moments, bit for bit."""
    import torch
    from paper_2606_19224_amd import warmstart
    feat, target, _, _ = _batch(96, 256, 21)
    say("case: wsnet checkpoint and resume")
    full = _net(lib, seed=5)
    h_full = warmstart.train(full, feat, target, epochs=4, batch=16, lr=1e-3, seed=3)
    part = _net(lib, seed=5)
    path = str(tmp_path / "ws.npz")
    h1 = warmstart.train(part, feat, target, epochs=2, batch=16, lr=1e-3, seed=3,
                         checkpoint=path)
    resumed, extra = lib.WarmStartNet.load_state(path)
    assert int(extra["epoch"]) == 2
    h2 = warmstart.train(resumed, feat, target, epochs=4, batch=16, lr=1e-3, seed=3,
                         start_epoch=2)
    torch.cuda.synchronize()
    assert torch.equal(resumed.params, full.params)
    assert torch.equal(resumed.m, full.m) and torch.equal(resumed.v, full.v)
    assert resumed.step == full.step
    assert h1 + h2 == h_full
