"""Host AddressSanitizer build of the library: the ABI tests (the library's host-only logic:
validation, FFT plans, status strings, the no-device path) run against a build whose host code
is instrumented, in a child process with the sanitizer runtime preloaded.  Any invalid host
memory access makes that process report and fail."""

import os
import subprocess
import sys

import pytest

from paper_2601_22793_amd import build as B
from tests.helpers import has_gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(has_gpu(), reason="runs the device-free ABI tests")
def test_abi_tests_pass_under_host_asan():
    lib = B.build_host_asan()
    env = dict(os.environ)
    env.update(LD_PRELOAD=B.asan_runtime(), EPR_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:exitcode=66")
    check = ("import ctypes, paper_2601_22793_amd._lib as L; L.load(); "
             "maps = open('/proc/self/maps').read(); "
             "assert 'libepr_asan.so' in maps and 'libepr.so' not in maps, 'wrong library'; "
             "assert ctypes.CDLL(None).__asan_init, 'no sanitizer runtime'")
    r = subprocess.run([sys.executable, "-c", check], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_abi.py", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "AddressSanitizer" not in r.stderr
