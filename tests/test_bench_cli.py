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
    # per iteration: fp32 8 nnz + 52 n, fp64 12 nnz + 100 n; per refinement 12 nnz + 28 n
    assert bench.solve_bytes(n, nnz, 2, 0, True) - bench.solve_bytes(n, nnz, 1, 0, True) == 8 * nnz + 52 * n
    assert bench.solve_bytes(n, nnz, 2, 0, False) - bench.solve_bytes(n, nnz, 1, 0, False) == 12 * nnz + 100 * n
    assert bench.solve_bytes(n, nnz, 1, 1, True) - bench.solve_bytes(n, nnz, 1, 0, True) == 12 * nnz + 28 * n
