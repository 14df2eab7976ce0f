"""The host code of the library (runtime and C ABI, adjoint and batch
orchestration, model builder) built with AddressSanitizer and
UndefinedBehaviorSanitizer, driven through every entry point that runs
without a GPU: the ABI and validation tests (create's checks up to the
first device call, the closed form of eq. (23), workspace sizes, PEC
validation) and the model-builder tests (SPRIM, identity basis, the
eq. (27) clip, PEC cells).  Any sanitizer report fails the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.timeout(900)
def test_host_code_under_sanitizers(tmp_path):
    from paper_1609_07114_amd import build
    lib = build.build_sanitized(str(tmp_path))
    env = dict(os.environ, FDTD_ROM_LIB=lib, LD_PRELOAD=build.sanitizer_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    probe = subprocess.run([sys.executable, "-c",
                            "from paper_1609_07114_amd import capi; capi.lib(); "
                            "print([l.split()[-1] for l in open('/proc/self/maps') if 'fdtdrom' in l][0])"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0, probe.stderr[-2000:]
    assert probe.stdout.strip().endswith("libfdtdrom_san.so")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          "tests/test_abi.py", "tests/test_romgen.py"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
