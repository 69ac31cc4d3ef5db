"""Host-side pieces of bench.py: the measured-traffic records, the streaming
byte and flop models of a CG solve, and the one-GPU guard.  No GPU needed."""
import copy
import subprocess
import sys
from pathlib import Path

import pytest

import bench

ROOT = Path(__file__).resolve().parent.parent


def test_measured_traffic_scales_the_raw_counters():
    for name, rec in bench.MEASURED_TRAFFIC.items():
        got = bench.measured_traffic(name)
        want = 1024.0 * (rec["fetch_kib_raw"] * rec["fetch_scale"]
                         + rec["write_kib_raw"] * rec["write_scale"])
        # a record either matches the sources it was taken on, or reports nothing
        assert got is None or got == pytest.approx(want, rel=1e-12)


def test_measured_traffic_is_null_once_the_sources_change(monkeypatch):
    recs = copy.deepcopy(bench.MEASURED_TRAFFIC)
    for rec in recs.values():
        rec["sha256_16"] = "0" * 16
    monkeypatch.setattr(bench, "MEASURED_TRAFFIC", recs)
    for name in recs:
        assert bench.measured_traffic(name) is None
    assert bench.measured_traffic("no_such_kernel") is None


def test_streaming_model_counts_each_term():
    m, N, k = 2048, 64, 1
    base = bench.cg_bytes(m, N, k, 0)
    # gather: X_f values, idx and w, eps, S and D; finish: S and Z
    assert base == k * m * N * 4 + 8 * m * k + m * N * 4 + 2 * m * N * 4 + 2 * m * N * 4
    # each iteration: S twice and eight m x N vectors
    assert bench.cg_bytes(m, N, k, 5) - base == 5 * (2 * m * N * 4 + 8 * m * N * 4)
    # FP64 doubles every term but the 8-byte index and weight pair
    b64 = bench.cg_bytes(m, N, k, 3, b_x=8, b_s=8, b_v=8)
    assert b64 == 2 * bench.cg_bytes(m, N, k, 3) - 8 * m * k
    # flops: the gather's H X_f, 4 m N^2 + 12 m N per iteration, S^T Z
    f0 = bench.cg_flops(m, N, k, 0)
    assert bench.cg_flops(m, N, k, 2) - f0 == 2 * (4 * m * N * N + 12 * m * N)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr
