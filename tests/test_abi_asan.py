"""The interface layer under the host AddressSanitizer (no GPU): the ABI
and stencil-builder tests run against the sanitizer build of the library
(`python -m paper_2206_02607_amd.build --asan`, host code instrumented,
device code as usual) with the sanitizer runtime preloaded; any report
fails the test.  Skipped when that build is absent (it is not part of the
default build)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ASAN_LIB = os.path.join(ROOT, "paper_2206_02607_amd", "libcrom_asan.so")


@pytest.mark.skipif(not os.path.exists(ASAN_LIB), reason="sanitizer build not present (build.py --asan)")
def test_abi_under_address_sanitizer():
    from paper_2206_02607_amd import build
    env = dict(os.environ, CROM_LIBRARY=ASAN_LIB, LD_PRELOAD=build.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=99")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py"), os.path.join(ROOT, "tests", "test_fe_stencil.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    print(out[-2000:])
    assert "AddressSanitizer" not in out
    assert r.returncode == 0
