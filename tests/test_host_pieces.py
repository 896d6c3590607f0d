"""Host-side check of the kernels' piece-bound helpers (no GPU needed).

The tile, count and fix-up kernels compute the pieces of one tile in all k
regions from the two piece offsets the level table holds for it and the two
of the next tile (region lengths take only two values);
tests/host_checks/pieces_check.hip compares that against the direct formula
for random subproblems.  Compiled for the host only with hipcc.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_tile_pieces_match_piece_of(tmp_path):
    exe = tmp_path / "pieces_check"
    subprocess.check_call([
        "hipcc", "--cuda-host-only", "-O2", "-std=c++17",
        "-I", os.path.join(ROOT, "paper_2302_03317_amd", "csrc"),
        "-I", os.path.join(ROOT, "include"),
        os.path.join(ROOT, "tests", "host_checks", "pieces_check.hip"),
        "-o", str(exe),
    ])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok ")
