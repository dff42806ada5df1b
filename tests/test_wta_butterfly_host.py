"""The compile-time pixel-to-lane table of the V-pass WTA butterfly agrees with
a host emulation of the six merge stages, for every segment length the
library compiles (and a few odd counts)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_butterfly_lane_table_matches_emulation(tmp_path):
    exe = tmp_path / "wta_butterfly_emulation"
    src = os.path.join(ROOT, "tests", "wta_butterfly_emulation.hip")
    subprocess.run([HIPCC, "-O1", "-std=c++17", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2212_00476_amd", "csrc"), src, "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "bad 0", r.stdout + r.stderr
