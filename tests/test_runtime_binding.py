"""The binding loads the library after torch, so that one HIP runtime (torch's)
serves both: the streams and device memory torch hands over are then valid in
the library's calls.  Checked in a fresh process from the runtime libraries
mapped into it (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_one_hip_runtime_after_load():
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2302_13680_amd import binding\n"
            "binding.load()\n"
            "maps = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(maps))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1"
