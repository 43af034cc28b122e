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


def test_overlap_summary_counts_only_the_library_kernels_after_the_marker(bench, tmp_path):
    """summarize_overlap takes the library's kernels after the last other kernel (the marker) and
    reports their summed durations, the union of their intervals and the most running at once:
    here two overlapping kernels [0, 10) and [5, 15), then one [20, 30), in ns."""
    import csv
    rows = [("fab::k_before", 0, 100), ("at::native::fill", 200, 210),
            ("fab::k_a", 1000, 1010), ("fab::k_b", 1005, 1015), ("fab::k_c", 1020, 1030)]
    with open(tmp_path / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for r in rows:
            w.writerow(r)
    out = tmp_path / "overlap.md"
    bench.summarize_overlap(str(tmp_path), str(out), "cmd")
    text = out.read_text()
    assert "| kernels of the replayed solve | 3 |" in text
    assert "| sum of kernel durations | 0.00 ms |" in text  # 30 ns
    assert "| sum / union (average kernels running at once) | 1.20 |" in text  # 30 / 25
    assert "| most kernels running at once | 2 |" in text
