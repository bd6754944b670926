"""ctypes view of libclipverify.so (the C ABI declared in include/clipverify.h).

Loading fails loudly: there is no fallback implementation.  Build the
library first with ``python -m paper_2512_11087_amd.build``.  With
CV_DEBUG=1 in the environment the debug build (libclipverify_debug.so:
input scans, a synchronisation and error check after every kernel) is
loaded instead.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libclipverify.so")
DEBUG_LIB_PATH = os.path.join(HERE, "libclipverify_debug.so")

CV_LINEAR, CV_CONV2D = 0, 1
CV_CLIP_PARALLEL, CV_CLIP_SEQUENTIAL = 0, 1
CV_TUNE_RELAX, CV_TUNE_FINAL, CV_TUNE_ADJOINT = 0, 1, 2

STATUS = {0: "CV_OK", -1: "CV_E_INVALID", -2: "CV_E_SHAPE", -3: "CV_E_UNSUPPORTED",
          -4: "CV_E_WORKSPACE", -5: "CV_E_HIP", -6: "CV_E_NOMEM", -7: "CV_E_NONFINITE"}

# every function the header declares (checked by the CPU test suite)
EXPORTS = [
    "cv_status_string", "cv_last_hip_error", "cv_version", "cv_debug_build", "cv_last_kernel",
    "cv_net_create", "cv_net_destroy", "cv_net_info",
    "cv_net_autotune", "cv_net_tuning", "cv_net_set_tuning",
    "cv_root_create", "cv_root_create_ex", "cv_root_destroy", "cv_root_bounds", "cv_root_planes",
    "cv_root_unstable_count", "cv_rootset_create", "cv_root_count",
    "cv_clip_domains", "cv_constraint_order", "cv_concretize_planes", "cv_concretize_planes_static",
    "cv_concretize_planes_workspace", "cv_babsr_weights", "cv_babsr_weights_workspace",
    "cv_concretize", "cv_bound_propagate", "cv_bound_propagate_workspace",
    "cv_branch_relu", "cv_branch_input", "cv_intermediate_bounds",
    "cv_intermediate_bounds_workspace",
    "cv_alpha_step", "cv_alpha_step_workspace",
    "cv_profile_enable", "cv_profile_reset", "cv_profile_collect", "cv_profile_entry",
    "cv_measure_peaks",
]


class LayerDesc(C.Structure):
    _fields_ = [("kind", C.c_int), ("in_features", C.c_int), ("out_features", C.c_int),
                ("in_c", C.c_int), ("in_h", C.c_int), ("in_w", C.c_int),
                ("out_c", C.c_int), ("out_h", C.c_int), ("out_w", C.c_int),
                ("kernel", C.c_int), ("stride", C.c_int), ("pad", C.c_int),
                ("W", C.c_void_p), ("b", C.c_void_p)]


class Constraints(C.Structure):
    _fields_ = [("kmax", C.c_int), ("count", C.c_void_p), ("neuron", C.c_void_p),
                ("sign", C.c_void_p), ("G", C.c_void_p), ("h", C.c_void_p),
                ("order", C.c_void_p)]


class CvError(RuntimeError):
    def __init__(self, fn, status, hip):
        super().__init__(f"{fn} failed: {STATUS.get(status, status)}"
                         + (f" (hip error {hip})" if status == -5 else ""))
        self.status = status


_lib = None


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        _lib = load(DEBUG_LIB_PATH if os.environ.get("CV_DEBUG") == "1" else LIB_PATH)
    return _lib


def load(path):
    """Load a build of the library at `path` with the ABI's signatures."""
    if not os.path.exists(path):
        raise RuntimeError(f"libclipverify is not built ({path} missing); "
                           "run `python -m paper_2512_11087_amd.build`")
    L = C.CDLL(path)
    P, I, F, S, V = C.c_void_p, C.c_int, C.c_float, C.c_size_t, None
    sig = {
        "cv_status_string": (C.c_char_p, [I]),
        "cv_last_hip_error": (I, []),
        "cv_version": (I, []),
        "cv_debug_build": (I, []),
        "cv_last_kernel": (C.c_char_p, []),
        "cv_net_create": (I, [P, I, P]),
        "cv_net_destroy": (I, [P]),
        "cv_net_info": (I, [P, P, P, P, P]),
        "cv_net_autotune": (I, [P, I, I, P]),
        "cv_net_tuning": (I, [P, I, I, P, P]),
        "cv_net_set_tuning": (I, [P, I, I, I]),
        "cv_root_create": (I, [P, P, P, F, P, P]),
        "cv_root_create_ex": (I, [P, P, P, F, I, P, P]),
        "cv_root_destroy": (I, [P]),
        "cv_root_bounds": (I, [P, P, P, P]),
        "cv_root_planes": (I, [P, P, P, P, P, P]),
        "cv_root_unstable_count": (I, [P, P]),
        "cv_rootset_create": (I, [P, I, P]),
        "cv_root_count": (I, [P, P]),
        "cv_clip_domains": (I, [P, P, I, I, P, P, P, P, I, P]),
        "cv_constraint_order": (I, [P, P, I, I, P, P, P, P, P]),
        "cv_concretize_planes": (I, [P, P, I, P, P, P, I, I, I, P, P, P, P, P, P, S, P]),
        "cv_concretize_planes_static": (I, [P, P, I, P, P, P, I, I, I, P, P, P, P, P, P]),
        "cv_babsr_weights": (I, [P, P, I, P, P, P, P, S, P]),
        "cv_babsr_weights_workspace": (I, [P, I, P]),
        "cv_branch_relu": (I, [P, P, I, P, P, P, P, P, P, I, P, P, P, P, P, P, P]),
        "cv_branch_input": (I, [I, I, I, P, P, P, P, P, P, P]),
        "cv_intermediate_bounds": (I, [P, P, I, P, P, P, P, P, P, S, P]),
        "cv_intermediate_bounds_workspace": (I, [P, I, P]),
        "cv_concretize_planes_workspace": (I, [P, I, I, P]),
        "cv_concretize": (I, [P, P, I, I, I, P, I, P, P, P, P, I, P, P, P, P, P]),
        "cv_bound_propagate": (I, [P, I, I, P, P, P, P, P, F, P, P, P, P, P, P, I, P, P, P, P, S,
                                   P]),
        "cv_bound_propagate_workspace": (I, [P, I, I, I, P]),
        "cv_alpha_step": (I, [P, I, I, P, P, P, P, P, F, P, P, P, P, P, P, I, P, P, I, F, F, F,
                              F, P, P, P, P, S, P]),
        "cv_alpha_step_workspace": (I, [P, I, I, I, P]),
        "cv_profile_enable": (I, [I]),
        "cv_measure_peaks": (I, [P, P, P]),
        "cv_profile_reset": (I, []),
        "cv_profile_collect": (I, [P]),
        "cv_profile_entry": (I, [I, P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def check(fn_name, status):
    if status != 0:
        raise CvError(fn_name, status, lib().cv_last_hip_error())


def call(name, *args):
    """Call a cv_* function and raise CvError on a non-zero status."""
    st = getattr(lib(), name)(*args)
    check(name, st)
    return st


def profile_enable(on=True):
    call("cv_profile_enable", int(bool(on)))


def profile_reset():
    call("cv_profile_reset")


def profile_collect():
    """{kernel name: dict(launches, ms, flops, bytes)} of the records so far
    (call after synchronising the streams)."""
    n = C.c_int()
    call("cv_profile_collect", C.byref(n))
    out = {}
    for i in range(n.value):
        name = C.c_char_p()
        cnt = C.c_int()
        ms, fl, by = C.c_double(), C.c_double(), C.c_double()
        call("cv_profile_entry", i, C.byref(name), C.byref(cnt), C.byref(ms), C.byref(fl),
             C.byref(by))
        out[name.value.decode()] = dict(launches=cnt.value, ms=ms.value, flops=fl.value,
                                        bytes=by.value)
    return out


def measure_peaks(stream=None):
    """(HBM GB/s of a streaming copy, FP64 matrix-core TFLOP/s) measured on the
    current device by cv_measure_peaks."""
    gbs, tfl = C.c_double(), C.c_double()
    call("cv_measure_peaks", C.byref(gbs), C.byref(tfl), stream)
    return gbs.value, tfl.value
