"""Checkpoint files of the warm-start trainer: a save/load round trip of the
training state (host only; the GPU resume test is in test_wsnet_gpu.py)."""
import os

import numpy as np
import pytest

from paper_2606_19224_amd import binding as B


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("library not built")
    return B.load()


def test_state_round_trip(lib, tmp_path):
    net = B.WarmStartNet(seed=3, device="cpu")
    net.m += 0.25
    net.v += 0.5
    net.step = 17
    path = str(tmp_path / "ws.npz")
    net.save(path, epoch=4)
    back, extra = B.WarmStartNet.load_state(path, device="cpu")
    assert np.array_equal(back.params.numpy(), net.params.numpy())
    assert np.array_equal(back.m.numpy(), net.m.numpy())
    assert np.array_equal(back.v.numpy(), net.v.numpy())
    assert back.step == 17 and int(extra["epoch"]) == 4
    # plain arrays only: loads without pickle
    with np.load(path, allow_pickle=False) as f:
        assert set(f.files) == {"params", "adam_m", "adam_v", "step", "extra_epoch"}
