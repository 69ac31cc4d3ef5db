"""Host-side checks of the C ABI (no GPU needed, no compute calls)."""
import ctypes
import os

import pytest

from paper_2606_19224_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("library not built")
    return B.load()


def test_exports_every_declared_symbol(lib):
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            names |= set(B.declared_functions(os.path.join(ROOT, "include", f)))
    assert {"cgd_enkf_analysis", "cgd_enkf_reduced_analysis", "cgd_enkf_workspace_bytes"} <= names
    for name in sorted(names):
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code, name in B.STATUS.items():
        assert lib.cgd_status_string(code).decode() == name
    assert lib.cgd_version().decode().count(".") == 2


def test_workspace_bytes_rejects_bad_sizes(lib):
    assert B.workspace_bytes(40, 20, 20, 1) > 0
    assert B.workspace_bytes(40, 20, 20, 1, reduced=True) > 0
    for bad in [(0, 20, 20, 1), (40, 0, 20, 1), (40, 20, 1, 1), (40, 20, 20, 0)]:
        assert lib.cgd_enkf_workspace_bytes(*bad, 0, 0) == 0
    assert lib.cgd_enkf_workspace_bytes(40, 20, 20, 1, 7, 0) == 0
    assert lib.cgd_enkf_workspace_bytes(40, 20, 20, 1, 0, 4) == 0
    # mode bit 2: the whitening buffers of a non-diagonal R
    assert lib.cgd_enkf_workspace_bytes(40, 20, 20, 1, 0, 2) > lib.cgd_enkf_workspace_bytes(40, 20, 20, 1, 0, 0)
    # grows with the problem, 256-byte granularity
    a = B.workspace_bytes(4096, 2048, 64, 1, "fp32")
    b = B.workspace_bytes(4096, 4096, 64, 1, "fp32")
    assert b > a and a % 256 == 0


def test_host_argument_checks_return_before_any_launch(lib):
    opt = B.Options()
    lib.cgd_options_default(ctypes.byref(opt))
    assert opt.prec == 0 and opt.z0 is None and opt.precond == 0 and not opt.tuning
    dummy = ctypes.c_void_p(256)  # never dereferenced: every call below fails its host checks
    calls = [
        (40, 20, 1, 1, 1e-6, 10),     # N = 1
        (40, 0, 20, 1, 1e-6, 10),     # m = 0
        (40, 20, 20, 1, -1.0, 10),    # tol < 0
        (40, 20, 20, 1, 1e-6, -1),    # maxit < 0
    ]
    for n, m, N, k, tol, maxit in calls:
        for fn in (lib.cgd_enkf_analysis, lib.cgd_enkf_reduced_analysis):
            st = fn(n, m, N, k, dummy, dummy, dummy, dummy, dummy, dummy, None, tol, maxit,
                    ctypes.byref(opt), dummy, 1 << 30, None, None)
            assert st == -1, (n, m, N, tol, maxit)
    # NULL pointers and a short workspace
    st = lib.cgd_enkf_analysis(40, 20, 20, 1, None, dummy, dummy, dummy, dummy, dummy, None, 1e-6,
                               10, ctypes.byref(opt), dummy, 1 << 30, None, None)
    assert st == -1
    st = lib.cgd_enkf_analysis(40, 20, 20, 1, dummy, dummy, dummy, dummy, dummy, dummy, None, 1e-6,
                               10, ctypes.byref(opt), dummy, 16, None, None)
    assert st == -5
    bad = B.Options()
    lib.cgd_options_default(ctypes.byref(bad))
    bad.prec = 9
    st = lib.cgd_enkf_analysis(40, 20, 20, 1, dummy, dummy, dummy, dummy, dummy, dummy, None, 1e-6,
                               10, ctypes.byref(bad), dummy, 1 << 30, None, None)
    assert st == -1


def test_workspace_layout_fits_every_solver_variant(lib):
    """Regression: the resident solver once indexed its partial buffers with
    stride 64 while the workspace was sized with N rounded to 16 (48 for
    N = 33).  The library's self-check recomputes every kernel's largest
    index per region on the host."""
    lib.cgd_layout_selfcheck.restype = ctypes.c_int
    lib.cgd_layout_selfcheck.argtypes = [ctypes.c_int] * 5
    for prec in (0, 1, 2):
        for N in list(range(2, 140)) + [200, 256, 513]:
            for m in (1, 15, 16, 17, 257, 2048, 16384, 70000):
                assert lib.cgd_layout_selfcheck(1000, m, N, 2, prec) == 0, (prec, N, m)
    assert lib.cgd_layout_selfcheck(1000, 10, 1, 1, 0) == -1


def test_comparison_forms_host_checks(lib):
    """cgd_senkf_analysis and cgd_enkf_gain_analysis refuse bad sizes,
    unsupported precisions and short workspaces before any launch."""
    opt = B.Options()
    lib.cgd_options_default(ctypes.byref(opt))
    dummy = ctypes.c_void_p(256)  # never dereferenced
    sen, gain = lib.cgd_senkf_analysis, lib.cgd_enkf_gain_analysis
    gain.argtypes = [ctypes.c_int] * 4 + [ctypes.c_void_p] * 7 + [ctypes.c_double, ctypes.c_int,
                     ctypes.POINTER(B.Options), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                     ctypes.c_size_t, ctypes.POINTER(B.Stats), ctypes.c_void_p]
    gain.restype = ctypes.c_int

    def s_call(n, m, N, k, o=opt, ws=1 << 30):
        return sen(n, m, N, k, dummy, dummy, dummy, dummy, dummy, dummy, None, ctypes.byref(o),
                   dummy, ws, None, None)

    def g_call(n, m, N, k, tol=1e-6, maxit=10, o=opt, ws=1 << 30):
        return gain(n, m, N, k, dummy, dummy, dummy, dummy, dummy, dummy, None, tol, maxit,
                    ctypes.byref(o), None, None, dummy, ws, None, None)

    for n, m, N, k in [(40, 20, 1, 1), (40, 0, 20, 1), (0, 20, 20, 1), (40, 20, 20, 0)]:
        assert s_call(n, m, N, k) == -1 and g_call(n, m, N, k) == -1
    assert g_call(40, 20, 20, 1, tol=-1.0) == -1
    assert g_call(40, 20, 20, 1, maxit=-1) == -1
    assert s_call(40, 20, 20, 1, ws=16) == -5
    assert g_call(40, 20, 20, 1, ws=16) == -5
    assert g_call(40, 20, 130, 1) == -7          # N past the MFMA widths
    assert lib.cgd_enkf_gain_workspace_bytes(40, 20, 130, 1, 0) == 0
    assert lib.cgd_enkf_gain_workspace_bytes(40, 20, 20, 1, 1) > 0
    for prec in (B.PREC["mixed"], B.PREC["bf16split"]):
        o = B.Options()
        lib.cgd_options_default(ctypes.byref(o))
        o.prec = prec
        assert s_call(40, 20, 20, 1, o=o) == -7 and g_call(40, 20, 20, 1, o=o) == -7
    o = B.Options()
    lib.cgd_options_default(ctypes.byref(o))
    o.r_factor = dummy
    assert g_call(40, 20, 20, 1, o=o) == -7       # non-diagonal R
