"""The debug build on the GPU (libclipverify_debug.so, loaded beside the
release build): finite inputs give the release build's results, the
launched kernel is named, and a NaN or infinity in an input returns
CV_E_NONFINITE with nothing enqueued."""
import ctypes as C
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2512_11087_amd import _native as N  # noqa: E402

pytestmark = pytest.mark.gpu


def ptr(t):
    return C.c_void_p(t.data_ptr())


def concretize(L, A, c, lo, hi, lb):
    B, n = lo.shape
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.cv_concretize(None, None, B, 1, n, ptr(A), 1, ptr(c), ptr(lo), ptr(hi), None, 1,
                           ptr(lb), None, None, None, s)


def test_debug_build_scans_inputs_and_names_kernels():
    if not os.path.exists(N.DEBUG_LIB_PATH):
        pytest.skip("debug build not built")
    dbg, rel = N.load(N.DEBUG_LIB_PATH), N.lib()
    assert dbg.cv_debug_build() == 1
    g = torch.Generator().manual_seed(5)
    B, n = 64, 300
    lo = (torch.rand(B, n, generator=g) - 0.5).cuda()
    hi = lo + torch.rand(B, n, generator=g).cuda()
    A = torch.randn(1, n, generator=g).cuda()
    c = torch.randn(1, generator=g).cuda()
    lb_rel = torch.empty(B, device="cuda")
    lb_dbg = torch.full((B,), 7.0, device="cuda")
    assert concretize(rel, A, c, lo, hi, lb_rel) == 0
    assert concretize(dbg, A, c, lo, hi, lb_dbg) == 0
    torch.cuda.synchronize()
    assert torch.equal(lb_rel, lb_dbg)
    assert dbg.cv_last_kernel() == b"ca_generic"
    for bad in (float("nan"), float("inf"), float("-inf")):
        for arr in (lo, A, c):
            keep = arr.view(-1)[3 % arr.numel()].item()
            arr.view(-1)[3 % arr.numel()] = bad
            lb_dbg.fill_(7.0)
            assert concretize(dbg, A, c, lo, hi, lb_dbg) == -7
            torch.cuda.synchronize()
            assert (lb_dbg == 7.0).all(), "a kernel ran after the scan failed"
            arr.view(-1)[3 % arr.numel()] = keep
    assert concretize(dbg, A, c, lo, hi, lb_dbg) == 0
    torch.cuda.synchronize()
    assert torch.equal(lb_rel, lb_dbg)
