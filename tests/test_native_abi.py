"""Host-side checks of the C ABI (no GPU needed): the library builds and
loads, exports every function include/clipverify.h declares, and rejects
invalid arguments before touching the device."""
import ctypes as C

import numpy as np
import os
import re

import pytest

from paper_2512_11087_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "clipverify.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cv_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(N.LIB_PATH):
        from paper_2512_11087_amd import build
        build.build()
    return N.lib()


def test_header_and_binding_list_the_same_functions():
    assert header_functions() == sorted(N.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in header_functions():
        assert hasattr(lib, name), name


def test_status_strings_and_version(lib):
    assert lib.cv_status_string(0) == b"ok"
    assert lib.cv_status_string(-4) == b"workspace too small"
    assert lib.cv_version() >= 10000
    assert lib.cv_last_hip_error() == 0


def test_invalid_arguments_are_rejected_on_the_host(lib):
    out = C.c_void_p()
    assert lib.cv_net_create(None, 2, C.byref(out)) == -1
    d = (N.LayerDesc * 1)()
    assert lib.cv_net_create(d, 1, C.byref(out)) == -3          # needs a hidden layer
    d2 = (N.LayerDesc * 2)()
    d2[0].kind = N.CV_CONV2D
    assert lib.cv_net_create(d2, 2, C.byref(out)) == -1         # conv without W / geometry
    W = np.zeros(16 * 3 * 4 * 4, np.float32)
    b = np.zeros(16, np.float32)
    d2[0].W, d2[0].b = W.ctypes.data, b.ctypes.data
    d2[0].in_c, d2[0].in_h, d2[0].in_w, d2[0].kernel, d2[0].stride, d2[0].pad = 3, 32, 32, 4, 2, 1
    d2[0].out_c, d2[0].out_h, d2[0].out_w = 16, 15, 16                  # 16 x 16 expected
    d2[0].in_features, d2[0].out_features = 3072, 16 * 15 * 16
    assert lib.cv_net_create(d2, 2, C.byref(out)) == -2         # output size inconsistent
    d2[0].out_h = 16
    d2[0].out_features = 4000                                          # not 16*16*16
    assert lib.cv_net_create(d2, 2, C.byref(out)) == -2
    d2[0].kind = 7
    assert lib.cv_net_create(d2, 2, C.byref(out)) == -1
    # a conv as the last (objective) layer is not supported
    d3 = (N.LayerDesc * 2)()
    W0, b0 = np.zeros(48 * 4, np.float32), np.zeros(48, np.float32)
    W1, b1 = np.zeros(2 * 3 * 9, np.float32), np.zeros(2, np.float32)
    d3[0].kind, d3[0].in_features, d3[0].out_features = N.CV_LINEAR, 4, 48
    d3[0].W, d3[0].b = W0.ctypes.data, b0.ctypes.data
    d3[1].kind, d3[1].in_features, d3[1].out_features = N.CV_CONV2D, 48, 32
    d3[1].in_c, d3[1].in_h, d3[1].in_w, d3[1].kernel, d3[1].stride, d3[1].pad = 3, 4, 4, 3, 1, 1
    d3[1].out_c, d3[1].out_h, d3[1].out_w = 2, 4, 4
    d3[1].W, d3[1].b = W1.ctypes.data, b1.ctypes.data
    assert lib.cv_net_create(d3, 2, C.byref(out)) == -3
    assert lib.cv_clip_domains(None, None, -1, 4, None, None, None, None, 0, None) == -2
    assert lib.cv_clip_domains(None, None, 0, 4, None, None, None, None, 0, None) == 0  # B == 0
    assert lib.cv_clip_domains(None, None, 3, 4, None, None, None, None, 0, None) == -1
    assert lib.cv_concretize(None, None, 2, 2, 0, None, 0, None, None, None, None, 1, None, None,
                             None, None, None) == -2
    assert lib.cv_root_create(None, None, None, C.c_float(0.5), None, C.byref(out)) == -1
    assert lib.cv_root_create_ex(None, None, None, C.c_float(0.5), 2, None, C.byref(out)) == -1
    n = C.c_size_t()
    assert lib.cv_bound_propagate_workspace(None, 1, 1, 1, C.byref(n)) == -1
    # property sets: no roots / a null member / P < 1
    assert lib.cv_rootset_create(None, 2, C.byref(out)) == -1
    two = (C.c_void_p * 2)(None, None)
    assert lib.cv_rootset_create(two, 2, C.byref(out)) == -1
    assert lib.cv_rootset_create(two, 0, C.byref(out)) == -1
    assert lib.cv_root_count(None, C.byref(C.c_int())) == -1
    assert lib.cv_net_autotune(None, 4, 4, None) == -1
    assert lib.cv_net_tuning(None, 0, 2, None, None) == -1
    assert lib.cv_net_set_tuning(None, 0, 2, 0) == -1
    assert lib.cv_net_destroy(None) == 0 and lib.cv_root_destroy(None) == 0


def test_debug_build_loads_and_reports_itself(lib):
    # the debug build (input scans, a check after every kernel) exports the
    # same functions and says it is one; the release build says it is not
    if not os.path.exists(N.DEBUG_LIB_PATH):
        from paper_2512_11087_amd import build
        build.build(debug=True)
    dbg = N.load(N.DEBUG_LIB_PATH)
    for name in header_functions():
        assert hasattr(dbg, name), name
    assert dbg.cv_debug_build() == 1 and lib.cv_debug_build() == 0
    assert dbg.cv_status_string(-7) == b"non-finite input (debug build)"
    assert dbg.cv_last_kernel() is None
