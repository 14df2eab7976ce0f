"""The library and PyTorch share one HIP runtime in the process."""
import subprocess
import sys
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_single_hip_runtime_loaded():
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1609_07114_amd import capi\n"
            "capi.lib()\n"
            "maps = open('/proc/self/maps').read()\n"
            "libs = {l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l}\n"
            "print(len(libs)); print(sorted(libs))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, check=True)
    assert out.stdout.splitlines()[0] == "1", out.stdout
