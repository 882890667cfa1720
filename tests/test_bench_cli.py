"""bench.py's command-line contract on the CPU: more than one GPU is refused
with a message (this build measures one GPU), and the byte models of the
reported kernels count what their docstrings say."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr


@pytest.mark.parametrize("elem", [8, 4])
def test_byte_models(elem):
    n, nnzb, nnz = 1000, 14000, 60000
    # A-product: 9 values + one 4-byte column per block, x once, y written
    assert bench.spmv_A_bytes(n, nnzb, elem) == nnzb * (9 * elem + 4) + 3 * elem * n * 2
    # CG product: the A-product's blocks, z once, p and q read and written
    assert bench.cg_spmv_bytes(n, nnzb, elem) == nnzb * (9 * elem + 4) + 3 * elem * n * 5
    # S^ product: value + 2-byte offset per entry, the diagonal, x once, y written
    assert bench.shat_bytes(n, nnz, elem, 2) == nnz * (elem + 2) + elem * n * 3
