"""The C-ABI library loads and exports every entry point include/lagp.h
declares; host-side argument checks that need no GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lagp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lagp_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import importlib.util
    import torch  # noqa: F401  (one HIP runtime: torch's, as in the package)
    spec = importlib.util.spec_from_file_location("_lagp_hipbuild",
                                                  os.path.join(ROOT, "paper_1303_0383_amd", "build.py"))
    build = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(build)
    if not os.path.exists(build.LIB):
        build.build()
    return ctypes.CDLL(build.LIB)


def test_header_declares_entry_points():
    names = _declared()
    for n in ("lagp_design_create", "lagp_design_destroy", "lagp_knn", "lagp_predict",
              "lagp_workspace_bytes", "lagp_device_count", "lagp_last_error", "lagp_version"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    import paper_1303_0383_amd as L
    for name in _declared():
        assert callable(getattr(L, name)), name


def test_version_and_error_string(lib):
    lib.lagp_version.restype = ctypes.c_int
    assert lib.lagp_version() == 100
    lib.lagp_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.lagp_last_error(), bytes)


def test_argument_errors_without_device(lib):
    import paper_1303_0383_amd as L
    P = ctypes.c_void_p
    lib.lagp_design_create.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, P,
                                       ctypes.POINTER(P)]
    out = P()
    X = np.zeros((10, 2))
    y = np.zeros(10)
    # NULL output pointer, bad N, bad p and an unknown flag are argument errors.
    assert lib.lagp_design_create(X.ctypes.data, y.ctypes.data, 10, 2, 1, None, None) == L.LAGP_E_INVAL
    assert lib.lagp_design_create(X.ctypes.data, y.ctypes.data, 0, 2, 1, None, ctypes.byref(out)) == L.LAGP_E_INVAL
    assert lib.lagp_design_create(X.ctypes.data, y.ctypes.data, 10, 0, 1, None, ctypes.byref(out)) == L.LAGP_E_INVAL
    assert lib.lagp_design_create(X.ctypes.data, y.ctypes.data, 10, 2, 64, None, ctypes.byref(out)) == L.LAGP_E_INVAL
    lib.lagp_predict.argtypes = [P, P, ctypes.c_int64, P] + [P] * 7 + [ctypes.c_int64, P, P]
    assert lib.lagp_predict(None, None, 0, None, None, None, None, None, None, None, None, 0, None, None) \
        == L.LAGP_E_INVAL


def test_no_device_is_reported():
    import torch
    import paper_1303_0383_amd as L
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    assert L.lagp_device_count() == 0
    with pytest.raises(L.LagpError) as e:
        L.Design(np.zeros((10, 2)), np.zeros(10))
    assert e.value.code == L.LAGP_E_NODEVICE
