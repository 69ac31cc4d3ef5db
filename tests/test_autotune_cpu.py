"""The batched mode's autotuner table and its use, without a GPU: the class
of a problem shape, the table lookup with its defaults, that the committed
table is well formed, and that the library refuses row counts outside the
documented ranges (the workspace size is 0)."""
import ctypes
import json
import os

import pytest

from paper_2606_19224_amd import autotune as A


def test_shape_class():
    assert A.shape_class(256, 16) == (16, 256)
    assert A.shape_class(257, 16) == (16, 512)
    assert A.shape_class(2048, 33) == (64, 2048)
    assert A.shape_class(1, 2) == (16, 1)
    assert A.shape_class(3000, 32) == (32, 4096)


def test_lookup_and_defaults():
    table = {"entries": [{"N": 32, "m_bucket": 1024, "gather_rows": 128, "update_rows": 512}]}
    assert A.tiles_for(table, 1000, 20) == (128, 512)
    assert A.tiles_for(table, 1025, 20) == (0, 0)
    assert A.tiles_for(None, 1000, 20) == (0, 0)


def test_committed_table_is_well_formed():
    path = A.table_path()
    if not os.path.exists(path):
        pytest.skip("no tuned table for this GPU in the tree")
    t = json.load(open(path))
    assert t["arch"] == "gfx950" and t["entries"]
    seen = set()
    for e in t["entries"]:
        assert e["N"] in (16, 32, 64) and e["m_bucket"] & (e["m_bucket"] - 1) == 0
        assert e["gather_rows"] in A.GATHER_CANDIDATES and e["update_rows"] in A.UPDATE_CANDIDATES
        assert e["gather_rows"] % 32 == 0 and e["update_rows"] % 64 == 0
        assert (e["N"], e["m_bucket"]) not in seen
        seen.add((e["N"], e["m_bucket"]))
        # the chosen candidates are the fastest measured
        g = e["gather_us"]
        assert g[str(e["gather_rows"])] == min(g.values())
        u = e["update_us"]
        assert u[str(e["update_rows"])] == min(u.values())


@pytest.mark.parametrize("g,u,ok", [(0, 0, True), (32, 64, True), (4096, 4096, True),
                                    (48, 64, False), (64, 96, False), (8192, 64, False),
                                    (64, 8192, False), (-32, 0, False)])
def test_library_checks_row_counts(g, u, ok):
    from paper_2606_19224_amd import binding as B
    lib = B.load()
    lib.cgd_enkf_batched_workspace_bytes.argtypes = [ctypes.c_int, ctypes.POINTER(B.CProblem),
                                                     ctypes.c_int]
    lib.cgd_enkf_batched_workspace_bytes.restype = ctypes.c_size_t
    arr = (B.CProblem * 1)()
    arr[0] = B.CProblem(400, 300, 32, 2, None, None, None, None, None, None, None, None, g, u)
    need = lib.cgd_enkf_batched_workspace_bytes(1, arr, B.PREC["fp32"])
    assert (need > 0) == ok


# --- the single analysis's solver table -------------------------------------
def test_solver_class():
    assert A.solver_class("fp32", 2048, 64) == ("fp32", 64, 2048)
    assert A.solver_class("fp64", 2049, 65) == ("fp64", 128, 4096)
    assert A.solver_class("fp32", 20, 20) == ("fp32", 32, 32)
    assert A.solver_class("mixed", 16384, 128) == ("mixed", 128, 16384)
    assert A.solver_class("fp32", 100, 129)[1] == 0  # no class past N = 128


def test_solver_lookup_and_defaults():
    table = {"entries": [{"prec": "fp32", "N": 64, "m_bucket": 2048, "solver": 4,
                          "rows_per_block": 0, "grid": 0}]}
    assert A.solver_for(table, "fp32", 2000, 64) == {"solver": 4, "rows_per_block": 0, "grid": 0}
    assert A.solver_for(table, "fp64", 2000, 64) is None
    assert A.solver_for(table, "fp32", 2049, 64) is None
    assert A.solver_for(None, "fp32", 2000, 64) is None


def test_committed_solver_table_is_well_formed():
    path = A.solver_table_path()
    if not os.path.exists(path):
        pytest.skip("no tuned solver table for this GPU in the tree")
    t = json.load(open(path))
    assert t["arch"] == "gfx950" and t["kind"] == "solver" and t["entries"]
    cands = {tuple(c) for c in A.SOLVER_CANDIDATES}
    seen = set()
    for e in t["entries"]:
        assert e["N"] in (16, 32, 64, 128) and e["m_bucket"] & (e["m_bucket"] - 1) == 0
        assert (e["solver"], e["rows_per_block"], e["grid"]) in cands
        # the pick is the fastest of the times recorded with it
        best = min(e["us"], key=e["us"].get)
        assert best == f"{e['solver']}/{e['rows_per_block']}/{e['grid']}"
        assert (e["prec"], e["N"], e["m_bucket"]) not in seen
        seen.add((e["prec"], e["N"], e["m_bucket"]))
