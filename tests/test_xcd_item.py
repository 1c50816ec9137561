"""The persistent column passes walk their items in XCD-blocked order
(xcd_item): every item must be visited exactly once for any grid size, also
grids of fewer than eight workgroups (one per XCD range is then not
available).  Checked on the host: the same header function, compiled for the
host by hipcc, over all grids G <= 64 and item counts <= 300."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1810_12707_amd", "csrc")


def test_every_item_visited_once(tmp_path):
    hipcc = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "xcd_item_check")
    src = os.path.join(ROOT, "tests", "native", "xcd_item_check.hip")
    subprocess.run([hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950", "-I", CSRC, src, "-o", exe],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe, "64", "300"], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
