"""Host-side logic of bench.py, without a GPU: the algorithmic byte counts
behind the roofline figures, and the single-GPU guard."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_of_the_gmres_iteration():
    """200x200x50 cells, 13.88M blocks: the apply reads every off-diagonal
    block and D^-1 once plus four block vectors (7.62 GB); the fused lower
    half of the SpMV adds the lower blocks and four vectors (3.55 GB):
    about 5,586 bytes per cell in all, halved in FP32 storage."""
    b = bench.algorithmic_bytes(2_000_000, 13_880_000)
    assert b["ilu_apply"] == 7_618_560_000
    assert b["ilu_spmv"] == 11_171_840_000
    assert round(b["ilu_spmv"] / 2_000_000) == 5_586
    assert b["ilu_spmv32"] == b["ilu_spmv"] // 2
    assert b["spmv"] == (13_880_000 - 2_000_000) * 512 + 2 * 2_000_000 * 64


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr
