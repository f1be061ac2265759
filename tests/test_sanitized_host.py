"""The host-only tests (channel factorization, C-ABI checks, the reduced
DMRG-RPA solver) rerun against libdmrg_san.so, the library whose host C++
is built with AddressSanitizer and UndefinedBehaviorSanitizer, in a
subprocess with the sanitizer runtime preloaded; any report aborts the
subprocess."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_LIB = os.path.join(ROOT, "paper_1311_1646_amd", "libdmrg_san.so")
RUNTIME = "/opt/rocm/llvm/lib/clang/22/lib/linux/libclang_rt.asan-x86_64.so"


@pytest.mark.skipif(not os.path.exists(SAN_LIB) or not os.path.exists(RUNTIME),
                    reason="host-sanitizer build not present (python -m paper_1311_1646_amd.build --sanitize)")
def test_host_paths_clean_under_asan_ubsan():
    env = dict(os.environ)
    env.update(LD_PRELOAD=RUNTIME, DMRG_LIBRARY=SAN_LIB,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    probe = ("import paper_1311_1646_amd as l, ctypes; "
             "assert l.LIB_PATH.endswith('libdmrg_san.so'); "
             "assert hasattr(ctypes.CDLL(None), '__asan_init')")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        "tests/test_host_factorization.py", "tests/test_abi.py", "tests/test_host_rpa_reduced.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed" in r.stdout
