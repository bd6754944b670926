"""Host AddressSanitizer run of the C ABI (no GPU needed): the library is
built with AddressSanitizer in its host code (device code unchanged) and
tests/asan_abi_calls.py drives every entry point's argument checks, and net
creation through its allocation and cleanup, in a child process under the
sanitizer's runtime; any sanitizer report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_abi_host_code_is_clean_under_address_sanitizer():
    from paper_2512_11087_amd import build
    try:
        rt = build.asan_runtime()
    except RuntimeError:
        pytest.skip("no AddressSanitizer runtime in this toolchain")
    lib = build.build_asan()
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               HIP_VISIBLE_DEVICES=os.environ.get("HIP_VISIBLE_DEVICES", ""))
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "asan_abi_calls.py"), lib, ROOT],
                       capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "asan abi calls:" in r.stdout
