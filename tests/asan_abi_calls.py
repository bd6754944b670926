"""Run by tests/test_native_asan.py in a child process under the
AddressSanitizer runtime: drives the host side of every C-ABI entry point
through its argument checks (null handles and pointers, negative and
inconsistent sizes, out-of-range values) and through net creation on a host
without a usable device (allocation failure and the cleanup of a partly
built net), so that the sanitizer sees the host code's memory accesses.
Prints "asan abi calls: N checked" on success."""
import ctypes as C
import sys

import numpy as np

sys.path.insert(0, sys.argv[2])
from paper_2512_11087_amd import _native as N  # noqa: E402

L = N.load(sys.argv[1])
P = C.c_void_p
n_checked = 0


def expect(got, want, what):
    global n_checked
    assert got == want, f"{what}: status {got}, expected {want}"
    n_checked += 1


INVALID, SHAPE, UNSUPPORTED = -1, -2, -3
assert L.cv_version() > 0
for code in range(-8, 1):
    assert L.cv_status_string(code)
assert L.cv_debug_build() in (0, 1)
L.cv_last_kernel()
L.cv_last_hip_error()

out = P()
need = C.c_size_t()
expect(L.cv_net_create(None, 2, C.byref(out)), INVALID, "net_create null layers")
W = np.ones((3, 4), np.float32)
b = np.zeros(3, np.float32)
W2 = np.ones((2, 5), np.float32)   # in_features 5 != 3 outputs of layer 1
b2 = np.zeros(2, np.float32)
layers = (N.LayerDesc * 2)()
layers[0] = N.LayerDesc(N.CV_LINEAR, 4, 3, 0, 0, 0, 0, 0, 0, 0, 0, 0,
                        W.ctypes.data_as(P), b.ctypes.data_as(P))
layers[1] = N.LayerDesc(N.CV_LINEAR, 5, 2, 0, 0, 0, 0, 0, 0, 0, 0, 0,
                        W2.ctypes.data_as(P), b2.ctypes.data_as(P))
expect(L.cv_net_create(layers, 2, C.byref(out)), SHAPE, "net_create inconsistent sizes")
expect(L.cv_net_create(layers, 1, C.byref(out)), UNSUPPORTED, "net_create one layer")
conv = (N.LayerDesc * 2)()
Kc = np.ones((2, 1, 3, 3), np.float32)
conv[0] = N.LayerDesc(N.CV_CONV2D, 16, 8, 1, 4, 4, 2, 2, 2, 3, 1, 0,
                      Kc.ctypes.data_as(P), np.zeros(2, np.float32).ctypes.data_as(P))
Kc2 = np.ones((2, 2, 2, 2), np.float32)
conv[1] = N.LayerDesc(N.CV_CONV2D, 8, 2, 2, 2, 2, 2, 1, 1, 2, 1, 0,
                      Kc2.ctypes.data_as(P), np.zeros(2, np.float32).ctypes.data_as(P))
expect(L.cv_net_create(conv, 2, C.byref(out)), UNSUPPORTED, "net_create conv objective layer")
# a consistent net: creation allocates device memory, which fails without a
# usable device (or succeeds with one); either way the handle is cleaned up
layers[1] = N.LayerDesc(N.CV_LINEAR, 3, 2, 0, 0, 0, 0, 0, 0, 0, 0, 0,
                        W2[:, :3].copy().ctypes.data_as(P), b2.ctypes.data_as(P))
st = L.cv_net_create(layers, 2, C.byref(out))
if st == 0:
    expect(L.cv_net_destroy(out), 0, "net_destroy")
else:
    assert st in (-5, -6), st
    n_checked += 1
expect(L.cv_net_destroy(None), 0, "net_destroy null")
expect(L.cv_root_destroy(None), 0, "root_destroy null")
expect(L.cv_net_info(None, None, None, None, None), INVALID, "net_info null")
expect(L.cv_net_tuning(None, 0, 1, None, None), INVALID, "net_tuning null")
expect(L.cv_net_set_tuning(None, 0, 1, 0), INVALID, "net_set_tuning null")
expect(L.cv_net_autotune(None, 1, 1, None), INVALID, "net_autotune null")
expect(L.cv_root_create(None, None, None, 0.5, None, C.byref(out)), INVALID, "root_create null")
expect(L.cv_rootset_create(None, 0, C.byref(out)), INVALID, "rootset_create null")
expect(L.cv_root_count(None, None), INVALID, "root_count null")
expect(L.cv_root_bounds(None, None, None, None), INVALID, "root_bounds null")
expect(L.cv_root_unstable_count(None, None), INVALID, "root_unstable_count null")
cons = N.Constraints(2, None, None, None, None, None, None)
expect(L.cv_clip_domains(None, None, -1, 4, C.byref(cons), None, None, None, 0, None), SHAPE,
       "clip negative B")
expect(L.cv_clip_domains(None, None, 4, 4, C.byref(cons), None, None, None, 7, None), INVALID,
       "clip bad mode")
expect(L.cv_clip_domains(None, None, 0, 4, None, None, None, None, 0, None), 0, "clip empty batch")
expect(L.cv_clip_domains(None, None, 4, 4, None, None, None, None, 0, None), INVALID,
       "clip null arrays")
buf = (C.c_float * 64)()
expect(L.cv_clip_domains(None, None, 4, 5000, C.byref(cons), buf, buf, buf, 0, None), UNSUPPORTED,
       "clip n > 4096")
expect(L.cv_concretize(None, None, -1, 1, 4, None, 0, None, None, None, None, 1, None, None, None,
                       None, None), SHAPE, "concretize negative B")
expect(L.cv_concretize(None, None, 2, 1, 4, None, 0, None, None, None, None, 1, None, None, None,
                       None, None), INVALID, "concretize null A")
expect(L.cv_concretize(None, None, 2, 1, 4, buf, 0, buf, buf, buf, C.byref(cons), 0, buf, None,
                       None, None, None), INVALID, "concretize passes 0")
expect(L.cv_concretize_planes(None, None, 4, None, None, None, 0, 1, -1, None, None, None, None,
                              None, None, 0, None), INVALID, "concretize_planes null root")
expect(L.cv_concretize_planes_static(None, None, 4, None, None, None, 0, 1, -1, None, None, None,
                                     None, None, None), INVALID, "concretize_planes_static null")
expect(L.cv_concretize_planes_workspace(None, 4, 1, C.byref(need)), INVALID, "planes workspace")
expect(L.cv_bound_propagate(None, 4, 9, None, None, None, None, None, 0.5, None, None, None, None,
                            None, None, 1, None, None, None, None, 0, None), INVALID,
       "bound_propagate null net")
expect(L.cv_bound_propagate_workspace(None, 1, 4, 9, C.byref(need)), INVALID, "propagate workspace")
expect(L.cv_alpha_step(None, 4, 9, None, None, None, None, None, -1.0, None, None, None, None,
                       None, None, 1, None, None, 2, 0.1, 0.9, 0.999, 1e-8, None, None, None, None,
                       0, None), INVALID, "alpha_step null net")
expect(L.cv_alpha_step_workspace(None, 1, 4, 9, C.byref(need)), INVALID, "alpha workspace")
expect(L.cv_babsr_weights_workspace(None, 9, C.byref(need)), INVALID, "babsr workspace")
expect(L.cv_intermediate_bounds_workspace(None, 4, C.byref(need)), INVALID,
       "intermediate workspace")
expect(L.cv_branch_input(-1, 1, 4, None, None, None, None, None, None, None), SHAPE,
       "branch_input negative B")
expect(L.cv_measure_peaks(None, None, None), INVALID, "measure_peaks null")
expect(L.cv_profile_reset(), 0, "profile_reset")
cnt = C.c_int()
expect(L.cv_profile_collect(C.byref(cnt)), 0, "profile_collect")
print(f"asan abi calls: {n_checked} checked", flush=True)
