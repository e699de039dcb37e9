"""bench.py's command-line contract that needs no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_of_a_solve():
    sys.path.insert(0, ROOT)
    import bench
    n, nnz = 1000, 6000
    # fp32 iteration 8 nnz + 44 n; fp64 iteration 12 nnz + 88 n
    assert bench.pcg_bytes(n, nnz, 2, 0, True, False) - bench.pcg_bytes(n, nnz, 1, 0, True, False) == 8 * nnz + 44 * n
    assert bench.pcg_bytes(n, nnz, 2, 0, False, False) - bench.pcg_bytes(n, nnz, 1, 0, False, False) == 12 * nnz + 88 * n
    assert bench.pcg_bytes(n, nnz, 1, 0, True, True) - bench.pcg_bytes(n, nnz, 1, 0, True, False) == 24 * n
