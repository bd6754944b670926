"""Build libclipverify.so (HIP for gfx950) in-tree.

    python -m paper_2512_11087_amd.build        # or build() from Python

Every HIP source under csrc/ is compiled with hipcc for gfx950 into an
object under _build/ and linked into paper_2512_11087_amd/libclipverify.so;
build(debug=True) makes paper_2512_11087_amd/libclipverify_debug.so, the
same sources with CV_DEBUG defined (input scans, a synchronisation and error
check after every kernel).  build_asan() makes a copy whose host code is
built with AddressSanitizer (device code unchanged) under _build/asan/, for
host-side checks of the C ABI.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libclipverify.so")
ARCH = "gfx950"

# Packed float32 VALU instructions are disabled for every device compile.
HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC,
            "-Wno-unused-result"]


def hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found: the HIP toolchain is required to build libclipverify")
    return p


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


DEBUG_LIB = os.path.join(HERE, "libclipverify_debug.so")
ASAN_DIR = os.path.join(BUILD, "asan")
ASAN_LIB = os.path.join(ASAN_DIR, "libclipverify_asan.so")
# host code only: each sanitizer flag applies to the host pass
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src, outdir, extra):
    obj = os.path.join(outdir, os.path.basename(src) + ".o")
    cmd = [hipcc()] + HIPFLAGS + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _build(out, outdir, extra, link_extra=(), verbose=False, jobs=None):
    os.makedirs(outdir, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, outdir, extra), srcs))
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}"] + list(link_extra) + ["-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


def build(verbose=False, jobs=None, debug=False):
    if debug:
        return _build(DEBUG_LIB, os.path.join(BUILD, "debug"), ["-DCV_DEBUG=1"], verbose=verbose,
                      jobs=jobs)
    return _build(LIB, BUILD, [], verbose=verbose, jobs=jobs)


def build_asan(verbose=False, jobs=None):
    """The library with AddressSanitizer in its host code (run it under the
    sanitizer's runtime, e.g. LD_PRELOAD of asan_runtime())."""
    return _build(ASAN_LIB, ASAN_DIR, ASAN_FLAGS, ["-shared-libsan"] + ASAN_FLAGS, verbose=verbose,
                  jobs=jobs)


def asan_runtime():
    """Path of the AddressSanitizer runtime the sanitized build links to."""
    r = subprocess.run([hipcc(), "--print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    p = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(p) or not os.path.exists(p):
        raise RuntimeError("AddressSanitizer runtime not found")
    return p


if __name__ == "__main__":
    build(verbose=True)
    build(verbose=True, debug=True)
    sys.exit(0)
