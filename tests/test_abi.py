"""The C-ABI library loads on a machine without a GPU and exports every
function that include/h2.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "h2.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(h2_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("h2_build", "h2_factor", "h2_solve", "h2_matvec", "h2_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2502_02395_amd import h2
    if not os.path.exists(h2.LIB_PATH):
        pytest.skip("libh2.so not built")
    lib = ctypes.CDLL(h2.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(h2.SYMBOLS) == _declared()


def test_status_strings_and_argument_errors_without_gpu():
    from paper_2502_02395_amd import h2
    if not os.path.exists(h2.LIB_PATH):
        pytest.skip("libh2.so not built")
    L = h2.load()
    assert L.h2_status_str(0).decode() == "ok"
    assert "positive definite" in L.h2_status_str(4).decode()
    # argument validation happens before any device call
    out = ctypes.c_void_p()
    prm = h2.make_params(3, 1, 1.0, 1e-6)  # leaf < 2
    k = h2.Kernel(0, 1e-3, 1.0, 1.0, 0.0)
    import numpy as np
    pts = np.zeros((4, 3))
    assert L.h2_build(pts.ctypes.data, 4, ctypes.byref(k), ctypes.byref(prm), None, None,
                      ctypes.byref(out)) == h2.ERR_ARG
    prm = h2.make_params(4, 8, 1.0, 1e-6)  # dim 4
    assert L.h2_build(pts.ctypes.data, 4, ctypes.byref(k), ctypes.byref(prm), None, None,
                      ctypes.byref(out)) == h2.ERR_ARG
    # Gauss-Seidel sweeps outside 0..64, unknown precisions
    for kw in ({"gs_sweeps": -1}, {"gs_sweeps": 65}, {"gemm_prec": 7}, {"solve_prec": 3},
               {"matvec_prec": 2}):
        prm = h2.make_params(3, 8, 1.0, 1e-6, **kw)
        assert L.h2_build(pts.ctypes.data, 4, ctypes.byref(k), ctypes.byref(prm), None, None,
                          ctypes.byref(out)) == h2.ERR_ARG, kw
    # the LU variant (a non-symmetric drift kernel, or factor_lu) takes FP64
    # or FP32 substitution copies, the FP64 matvec and stationary
    # refinement; factor_lu is 0 or 1; beta must be finite
    kd = h2.Kernel(4, 1e-3, 1.0, 1.0, 0.0, 0.5)
    for kw in ({"solve_prec": h2.PREC_BF16}, {"gemm_prec": h2.PREC_BF16X3, "solve_prec": h2.PREC_BF16},
               {"matvec_prec": h2.PREC_FP32}, {"use_pcg": True}):
        prm = h2.make_params(3, 8, 1.0, 1e-6, **kw)
        assert L.h2_build(pts.ctypes.data, 4, ctypes.byref(kd), ctypes.byref(prm), None, None,
                          ctypes.byref(out)) == h2.ERR_ARG, kw
        prm = h2.make_params(3, 8, 1.0, 1e-6, factor_lu=True, **kw)
        assert L.h2_build(pts.ctypes.data, 4, ctypes.byref(k), ctypes.byref(prm), None, None,
                          ctypes.byref(out)) == h2.ERR_ARG, kw
    prm = h2.make_params(3, 8, 1.0, 1e-6)
    prm.factor_lu = 2
    assert L.h2_build(pts.ctypes.data, 4, ctypes.byref(k), ctypes.byref(prm), None, None,
                      ctypes.byref(out)) == h2.ERR_ARG
    prm = h2.make_params(3, 8, 1.0, 1e-6)
    for bad in (h2.Kernel(4, 1e-3, 1.0, 1.0, 0.0, float("inf")), h2.Kernel(4, 0.0, 1.0, 1.0, 0.0, 0.5),
                h2.Kernel(5, 1e-3, 1.0, 1.0, 0.0, 0.0)):
        assert L.h2_build(pts.ctypes.data, 4, ctypes.byref(bad), ctypes.byref(prm), None, None,
                          ctypes.byref(out)) == h2.ERR_ARG
    # non-finite coordinates
    for v in (float("nan"), float("inf")):
        bad_pts = np.zeros((4, 3))
        bad_pts[2, 1] = v
        assert L.h2_build(bad_pts.ctypes.data, 4, ctypes.byref(k), ctypes.byref(prm), None, None,
                          ctypes.byref(out)) == h2.ERR_ARG
    assert L.h2_factor(None, None) == h2.ERR_ARG
    assert L.h2_solve(None, None, None, 1, 1, None) == h2.ERR_ARG
    assert L.h2_solve_noalloc(None, None, None, 1, 1, None) == h2.ERR_ARG


def test_graft_entry_has_build_and_smoke():
    import importlib.util
    spec = importlib.util.spec_from_file_location("ge", os.path.join(ROOT, "__graft_entry__.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    assert callable(m.build) and callable(m.smoke)


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No fallback: without libh2.so every entry of the binding raises."""
    import numpy as np
    from paper_2502_02395_amd import h2
    import workloads as W
    monkeypatch.setattr(h2, "_lib", None)
    monkeypatch.setattr(h2, "LIB_PATH", str(tmp_path / "libh2.so"))
    with pytest.raises(ImportError, match="missing"):
        h2.load()
    with pytest.raises(ImportError, match="missing"):
        h2.build(np.random.default_rng(0).random((64, 3)), W.Kernel(W.LAPLACE), 16, 1.0, 1e-6)
