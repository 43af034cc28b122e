"""Host logic of bench.py: the algorithmic byte counts the roofline divides by, and the one-GPU
contract.  No GPU is touched."""
import importlib.util
import os
import subprocess
import sys

import pytest

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    pytest.importorskip("torch")
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("ib,spmv,step", [(2, 187_760_644, 288_423_940), (4, 216_924_164, 317_587_460)])
def test_algorithmic_bytes_of_the_128_cubed_workload(bench, ib, spmv, step):
    """The fused kernel moves the FP64 values, ib bytes per column index, n + 1 row pointers, and
    reads w_j and writes z (n FP64 each); a step adds the window update (z and k = 4 columns read,
    w_{j+1} written).  The operator's own nonzero count is used, so the quoted figures follow it."""
    A = wl.convdiff_3d(128, 50.0)
    n, nnz = A.n, A.nnz
    assert (n, nnz) == (128 ** 3, 7 * 128 ** 3 - 6 * 128 ** 2)   # 7-point stencil, Dirichlet faces
    got_spmv, got_step = bench.algorithmic_bytes(n, nnz, 4, es=8, ib=ib)
    assert got_spmv == spmv
    assert got_step == step
    assert got_step - got_spmv == 6 * 8 * n


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
