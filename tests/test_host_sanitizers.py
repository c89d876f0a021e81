"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the library is rebuilt with the sanitizers on its host compilation
(paper_1205_6333_amd.build.build_host_sanitized, about a minute), and
tests/test_abi.py (loading, exported symbols, every argument check, plan and
configuration validation, status strings) runs against that build in a child
process with the compiler's ASan runtime preloaded; any memory error or
undefined behaviour aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def test_abi_tests_pass_under_asan_and_ubsan():
    sys.path.insert(0, ROOT)
    from paper_1205_6333_amd import build as B
    rt = B.asan_runtime()
    if not rt:
        pytest.skip("no clang ASan runtime in this ROCm installation")
    out_dir = os.path.join(B.BUILD, "sanitized")
    os.makedirs(out_dir, exist_ok=True)
    lib = B.build_host_sanitized(os.path.join(out_dir, "libsd_san.so"))
    env = dict(os.environ, SD_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True, timeout=600)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-3000:]
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stdout
    assert "runtime error" not in r.stdout      # UBSan's report line
