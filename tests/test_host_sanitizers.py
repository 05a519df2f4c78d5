"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the library is rebuilt with both sanitizers on its host code
(paper_2401_06861_amd/build.py, build_sanitized) and the device-free tests
-- argument validation of the C ABI, the OpenQASM reader (which reads
untrusted text), the fusion planner -- run against that build in a child
process that preloads the sanitizer runtime.  Any report fails the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_host_code_under_asan_and_ubsan():
    sys.path.insert(0, ROOT)
    from paper_2401_06861_amd import build as b
    lib = b.build_sanitized(verbose=False)
    env = dict(os.environ)
    env["LD_PRELOAD"] = b.sanitizer_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["NWQ_LIB"] = lib
    tests = [os.path.join(ROOT, "tests", t) for t in ("test_qasm.py", "test_fusion_plan.py", "test_abi_load.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
