#!/usr/bin/env python3
"""Benchmark of the restarted sketched Krylov f(A)b path on one MI355X.

Workload (one "step" = one complete solve, i.e. every cycle of the hot path):
  3-D convection-diffusion, 128^3 interior grid (n = 2,097,152, nnz = 14,581,760), central
  differences, wind (1,1,1), Peclet 50, CSR FP64; x = exp(-1e-4 A) b with b ~ N(0,1) (seed 0);
  sketched restarted Krylov m = 50, window k = 4, sketch d = 200 rows, zeta = 8, seed 1, tol 1e-8.

Prints one JSON line: solves/s, the roofline of the dominant kernel (fused SpMV + sketch, timed
with HIP events that each launch's dispatch records on the kernel's stream, over solves timed
like the headline ones), the step-loop bandwidth, the plain
restarted Arnoldi comparator on the same GPU, and the CPU oracle timed on the host as baseline
(which also gives the relative error of the GPU result against the exact FP64 solution).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extra] [--profile]
    python bench.py --profile-256 {f32,f64} | --profile-batched     # short runs for rocprofv3
    python bench.py --summarize-pmc FETCH_DIR WRITE_DIR    # turn rocprofv3 --pmc output into traffic
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import platform
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = {"workload": "convdiff_3d_N128_Pe50", "operator": "3-D 7-point convection-diffusion, wind (1,1,1)",
            "N": 128, "peclet": 50.0, "f": "exp(-t z)", "t": 1e-4, "m": 50, "k": 4, "d": 200, "zeta": 8,
            "sketch_seed": 1, "b_seed": 0, "tol": 1e-8, "values": "f64"}
HBM_PEAK_GBS = 8000.0
METRIC = "f(A)b solves/s at rel err 1e-8 vs FP64 oracle; loop HBM GB/s (% of peak)"
# the sources the fused SpMV + sketch kernel is compiled from (the kernel and its inlined helpers)
KERNEL_SRC = [os.path.join(ROOT, "paper_2503_22631_amd", "csrc", f) for f in ("step_kernels.hip", "fab_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "spmv_sketch_convdiff128_traffic.json")
COPY_BYTES = 256 << 20


def algorithmic_bytes(n: int, nnz: int, k: int, es: int = 8, ib: int = 4):
    """Bytes the method must move: per launch of the fused SpMV + sketch kernel (values + column
    indices of ib bytes, the operator's stored form + row pointers + read w_j + write z; S is
    generated, not read) and per Arnoldi step (that plus the window update: read z and k basis
    columns, write w_{j+1})."""
    spmv = (es + ib) * nnz + 4 * (n + 1) + 2 * es * n
    step = spmv + (2 + k) * es * n
    return spmv, step


def plain_cycle_bytes(n: int, nnz: int, m: int, nt: int = 1, es: int = 8, ib: int = 4) -> int:
    """Bytes one cycle of the plain restarted Arnoldi comparator moves, by its kernels: the start
    vector's norm (es n) and scaling (2 es n); per step j the product (as above), the two
    classical Gram-Schmidt sweeps (each a Gram pass reading j + 1 basis columns and z, and an
    update reading them and writing z: (2j + 5) es n) and the scaling of the new vector (2 es n);
    the pass over the m + 1 basis columns and nt columns of x (read and written, FP64)."""
    spmv = (es + ib) * nnz + 4 * (n + 1) + 2 * es * n
    steps = sum(spmv + 2 * (2 * j + 5) * es * n + 2 * es * n for j in range(m))
    return 3 * es * n + steps + (m + 1) * es * n + 16 * nt * n


def update_bytes(n: int, m: int, k: int, es: int = 8) -> float:
    """Average bytes per window update of a full cycle: step j reads z and its min(k, j+1) window
    columns and writes w_{j+1}."""
    return sum((2 + min(k, j + 1)) * es * n for j in range(m)) / m


def kernel_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def read_traffic():
    """Measured HBM bytes per launch of the fused kernel, if taken on the current kernel source."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha") != kernel_sha():
        return None
    return rec.get("traffic_bytes_per_launch")


def cpu_info():
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                model = line.split(":", 1)[1].strip()
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model or platform.processor()}


def cpu_plain_leg(A, b):
    """The plain restarted Arnoldi method on the host cores (cpu_baseline/, C++/OpenMP, FP64, CGS2,
    the same quadrature restart and stopping test as the GPU comparator), on the same workload: one
    warm-up solve and up to three timed ones, about 10 s of work at most."""
    import cpu_baseline

    w = WORKLOAD
    run = lambda: cpu_baseline.expv(A.rowptr, A.colind, A.vals, b, w["t"], w["m"], tol=w["tol"], max_cycles=100)
    x, info = run()
    solves, total = 0, 0.0
    while solves < 3 and (solves == 0 or total < 6.0):
        t0 = time.perf_counter()
        x, info = run()
        total += time.perf_counter() - t0
        solves += 1
    dt = total / solves
    return {"solves_per_s": 1.0 / dt, "seconds_per_solve": dt, "threads": cpu_baseline.threads(),
            "cycles": info["cycles"], "matvecs": info["matvecs"], "status": info["status"],
            "sample": f"{solves} timed solve(s) after one warm-up"}, x


def cpu_baseline_leg(A, b, x_gpu, x_plain, checks=(), x_cpu_plain=None):
    """The oracle, as it stands, on the host: complete solves of the same workload by its FP64
    step-by-step twin (same sketch), with BLAS on all the host's threads (its sparse products are
    scipy's, one thread), repeated until about 10 s of CPU work (at most 4 solves).  Also the exact
    solution by the Kronecker-product closed form, for the relative errors of the GPU results."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import exact, krylov, sketch

    w = WORKLOAD
    As = A.to_scipy()
    blas_threads = max([int(p.get("num_threads", 1)) for p in threadpool_info()] or [1])
    solves, total = 0, 0.0
    while solves < 4 and (solves == 0 or total < 10.0):
        t0 = time.perf_counter()
        S = sketch.sketch_matrix(A.n, w["d"], w["zeta"], seed=w["sketch_seed"])
        xo, info = krylov.restart_solve(As, b, "exp", w["t"], m=w["m"], k=w["k"], S=S, tol=w["tol"])
        total += time.perf_counter() - t0
        solves += 1
    dt = total / solves
    for rec, key, fn in checks:  # errors of the extra legs' GPU results against the exact FP64 results
        rec[key] = fn(exact)
    factors, _ = exact.problem_factors("convdiff_3d", w["N"], peclet=w["peclet"])
    ref = exact.kron_exp_fab(b, factors, w["t"])
    rel = lambda v: float(np.linalg.norm(v - ref) / np.linalg.norm(ref))
    return ({"value": 1.0 / dt, "unit": "solves/s", "cores": blas_threads, "kind": "oracle",
             "sample": f"{solves} full solve(s) of the same workload by the FP64 oracle twin ({info.cycles} cycles, "
                       f"{info.matvecs} matvecs each, sketch generation included; scipy CSR products on one "
                       f"thread, BLAS on {blas_threads}); {total:.1f} s in total",
             "seconds_per_solve": dt, "oracle_rel_err": rel(xo)},
            {"gpu_rel_err": rel(x_gpu), "plain_rel_err": rel(x_plain) if x_plain is not None else None,
             "cpu_plain_rel_err": rel(x_cpu_plain) if x_cpu_plain is not None else None})


def summarize_pmc(fetch_dir: str, write_dir: str, out_json: str = TRAFFIC_FILE, workload: str = None,
                  kernel_label: str = "k_spmv_sketch<double, SpMV+sketch, zeta<=8>",
                  kernel_re: str = r"k_spmv_sketch<\w+, 0,"):
    """Average FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the fused kernel, scaled by what the
    same counters read for a device copy of known size; writes the traffic record under profiles/."""
    def load(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows += [r for r in csv.DictReader(open(f)) if r.get("Counter_Name") == counter]
        return rows

    def avg(rows, pred):
        vals = [float(r["Counter_Value"]) for r in rows if pred(r["Kernel_Name"])]
        return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)

    def calib(rows):
        """The counter value of the largest device copy (the calibration copy of COPY_BYTES)."""
        cps = [r for r in rows if "copyBuffer" in r["Kernel_Name"]]
        if not cps:
            return None
        return float(max(cps, key=lambda r: int(r["Grid_Size"]))["Counter_Value"])

    is_spmv = lambda k: re.search(kernel_re, k) is not None   # mode 0 = SpMV + sketch
    fetch = load(fetch_dir, "FETCH_SIZE")
    write = load(write_dir, "WRITE_SIZE")
    f_k, nf = avg(fetch, is_spmv)
    w_k, nw = avg(write, is_spmv)
    f_c, w_c = calib(fetch), calib(write)
    kib = 1024.0
    f_scale = (COPY_BYTES / kib) / f_c if f_c else 1.0
    w_scale = (COPY_BYTES / kib) / w_c if w_c else 1.0
    traffic = (f_k * f_scale + w_k * w_scale) * kib if (f_k is not None and w_k is not None) else None
    rec = {"kernel": kernel_label, "workload": workload or WORKLOAD["workload"],
           "kernel_source_sha": kernel_sha(), "dispatches": [nf, nw],
           "fetch_kib_per_dispatch": f_k, "write_kib_per_dispatch": w_k,
           "copy_fetch_kib": f_c, "copy_write_kib": w_c, "copy_bytes": COPY_BYTES,
           "fetch_scale": f_scale, "write_scale": w_scale, "traffic_bytes_per_launch": traffic,
           "unscaled_bytes_per_launch": (f_k + w_k) * kib if (f_k is not None and w_k is not None) else None}
    os.makedirs(os.path.dirname(out_json), exist_ok=True)
    json.dump(rec, open(out_json, "w"), indent=1)
    print(json.dumps(rec))


def profile_ragged():
    """A short run for rocprofv3 --kernel-trace: the ragged workload (32 FP32 Laplacians, 64^2 ..
    512^2, exp t = 1e-3, m = 20, k = 2, d = 80), a first call (capture and replay), a one-element
    fill as a marker, then one replay of the branch graphs into the first call's outputs."""
    import numpy as np
    import torch

    import paper_2503_22631_amd as fab
    import workloads as wl

    ctx = fab.Context()
    Ns = [int(round(64 * 8 ** (i / 31))) for i in range(32)]
    ops, bs = [], []
    for i, Ng in enumerate(Ns):
        Ag = wl.laplacian_2d(Ng)
        ops.append(fab.CSROperator.from_arrays(ctx, Ag.rowptr, Ag.colind, Ag.vals, dtype=torch.float32))
        bs.append(torch.as_tensor(wl.gaussian_vector(Ag.n, 1000 + i).astype(np.float32), device="cuda"))
    kw = dict(m=20, k=2, d=80, zeta=8, seed=1, tol=1e-6, max_cycles=300)
    xs = fab.solve_ragged(ops, bs, "exp", t=1e-3, **kw)[0]
    torch.cuda.synchronize()
    torch.zeros(1, device="cuda")  # marker between the two calls in the trace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, infos = fab.solve_ragged(ops, bs, "exp", t=1e-3, xs=xs, **kw)
    torch.cuda.synchronize()
    print(json.dumps({"profile_ragged": True, "operators": len(ops), "replay_seconds": time.perf_counter() - t0,
                      "cycles": max(i["cycles"] for i in infos)}))
    return 0


def summarize_overlap(trace_dir: str, out_md: str, command: str):
    """How much the library's kernels after the last non-library kernel (the marker of
    --profile-ragged) overlap in time: span, sum of durations, union of intervals, most at once."""
    f = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)[0]
    rows = sorted(csv.DictReader(open(f)), key=lambda r: int(r["Start_Timestamp"]))
    last = max(i for i, r in enumerate(rows) if "fab::" not in r["Kernel_Name"])
    iv = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows[last + 1:] if "fab::" in r["Kernel_Name"]]
    total = sum(e - s for s, e in iv)
    union, cs, ce = 0, None, None
    for s, e in iv:
        if cs is None or s > ce:
            union += (ce - cs) if cs is not None else 0
            cs, ce = s, e
        else:
            ce = max(ce, e)
    union += ce - cs
    ev = sorted([(s, 1) for s, _ in iv] + [(e, -1) for _, e in iv])
    cur = most = 0
    for _, dlt in ev:
        cur += dlt
        most = max(most, cur)
    span = max(e for _, e in iv) - iv[0][0]
    lines = ["# Kernel overlap of one ragged solve (32 FP32 Laplacians, 64^2 .. 512^2)", "",
             "Command (from the repository root, on the MI355X machine):", "", "```", command, "```", "",
             "| quantity | value |", "|---|---|",
             f"| kernels of the replayed solve | {len(iv)} |",
             f"| span, first start to last end | {span / 1e6:.2f} ms |",
             f"| sum of kernel durations | {total / 1e6:.2f} ms |",
             f"| union of kernel intervals | {union / 1e6:.2f} ms |",
             f"| sum / union (average kernels running at once) | {total / union:.2f} |",
             f"| most kernels running at once | {most} |", ""]
    open(out_md, "w").write("\n".join(lines))
    print("\n".join(lines))


def summarize_trace(trace_dir: str, out_md: str, command: str, workload: str = None):
    """Markdown table of a rocprofv3 --kernel-trace --stats run (kernel_stats.csv)."""
    f = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)[0]
    rows = list(csv.DictReader(open(f)))
    lines = [f"# rocprofv3 kernel statistics: {workload or WORKLOAD['workload']}", "",
             "Command (from the repository root, on the MI355X machine):",
             "", "```", command, "```", "",
             "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"].split("(")[0].replace("|", "/")
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    print(out_md)


def _timed(fn, reps=1):
    """(seconds per call, last result) of fn after one warm-up call, bracketed by device syncs."""
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, r


def profile_256(dtype_name: str):
    """A short run for rocprofv3: z^(-1/2) of the shifted 3-D Laplacian at 256^3 (n = 16.8M), m = 30,
    k = 2, d = 120, zeta = 8, FP32 or FP64 values and basis, two solves of three cycles each (90
    launches of the fused product + sketch), then a device copy of COPY_BYTES for counter
    calibration."""
    import numpy as np
    import torch

    import paper_2503_22631_amd as fab
    import workloads as wl

    N = 256
    dt = torch.float32 if dtype_name == "f32" else torch.float64
    A = wl.shifted_laplacian_3d(N, 1.0)
    b = wl.gaussian_vector(A.n, 0)
    lo = 3 * 4 * (N + 1) ** 2 * np.sin(np.pi / (2 * (N + 1))) ** 2 + 1.0
    ctx = fab.Context()
    op = fab.CSROperator.from_arrays(ctx, A.rowptr, A.colind, A.vals, dtype=dt)
    bt = torch.as_tensor(b, dtype=dt, device="cuda")
    for _ in range(2):
        fab.solve(op, bt, "invsqrt", m=30, k=2, d=120, zeta=8, seed=1, tol=1e-6, spec=(lo, 12 * (N + 1) ** 2 + 1.0),
                  max_cycles=3, check=False)
    torch.cuda.synchronize()
    src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile_256": dtype_name, "n": A.n, "nnz": A.nnz,
                      "spmv_bytes_per_launch": algorithmic_bytes(A.n, A.nnz, 2, es=4 if dtype_name == "f32" else 8,
                                                                 ib=op.index_bytes())[0]}))
    return 0


def profile_batched():
    """A short run for rocprofv3: the batched workload (anisotropic 1024^2 operator, FP32, 64
    right-hand sides x 8 time points, m = 20, k = 2, d = 80, zeta = 8), groups of 16 members per
    block, two solves of two cycles each (80 launches of the grouped product + sketch), then a
    device copy of COPY_BYTES for counter calibration."""
    import numpy as np
    import torch

    import paper_2503_22631_amd as fab
    import workloads as wl

    N, nb = 1024, 64
    T = [10.0 ** (-5 + 2 * i / 7) for i in range(8)]
    A = wl.anisotropic_2d(N, 0.01)
    Bm = np.stack([wl.gaussian_vector(A.n, 300 + r) for r in range(nb)], axis=1).astype(np.float32)
    ctx = fab.Context()
    fab.batch_group(ctx, 16)
    op = fab.CSROperator.from_arrays(ctx, A.rowptr, A.colind, A.vals, dtype=torch.float32)
    Bt = torch.as_tensor(Bm, device="cuda")
    for _ in range(2):
        fab.solve_batched(op, Bt, "exp", t=T, m=20, k=2, d=80, zeta=8, seed=1, tol=1e-4, max_cycles=2, check=False)
    torch.cuda.synchronize()
    src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    floor = 4 * (A.nnz * 6 + 4 * (A.n + 1)) + nb * A.n * 8  # A once per group of 16, x read, z written
    print(json.dumps({"profile_batched": True, "n": A.n, "nnz": A.nnz, "members": nb, "group": 16,
                      "floor_bytes_per_launch": floor}))
    return 0


def extra_legs(fab, ctx):
    """The other workloads of the method on the same GPU: the paper's restart-rand (k = m, growing
    restart) on the headline workload; z^(-1/2) with FP32 against FP64 values
    and basis; 64 right-hand sides x 8 time points in one batched FP32 solve against single FP64
    solves; 32 Laplacians of uneven size in one ragged solve; the gradient of <c, exp(-tA) b>
    (forward solve + adjoint solve on A^T).  Returns (results, checks): each check is
    (record, key, fn) with fn(exact) the error of a kept GPU result against the exact FP64 result,
    evaluated in the CPU leg (the oracle's closed forms run only there)."""
    import numpy as np
    import torch

    import workloads as wl

    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out, checks = {}, []
    # --- the small workload: 2-D Laplacian 64^2 (n = 4096), exp(-1e-3 A) b, m=20, k=2, d=80, tol 1e-10;
    # the whole working set (~0.7 MB) stays in the caches, so this is the latency of a solve
    Nl = 64
    A = wl.laplacian_2d(Nl)
    b = wl.gaussian_vector(A.n, 0)
    op = fab.CSROperator.from_arrays(ctx, A.rowptr, A.colind, A.vals)
    bt = torch.as_tensor(b, device="cuda")
    sec, (x, info) = _timed(lambda: fab.solve(op, bt, "exp", t=1e-3, m=20, k=2, d=80, zeta=8, seed=1, tol=1e-10),
                            reps=50)
    leg = {"workload": "laplacian_2d_N64, exp(-1e-3 A) b, m=20, k=2, d=80, zeta=8, tol 1e-10, f64",
           "solves_per_s": 1.0 / sec, "ms_per_solve": 1e3 * sec, "cycles": info["cycles"], "status": info["status"]}
    xh = x[:, 0].cpu().numpy()
    checks.append((leg, "rel_err", lambda ex, xh=xh, b=b: rel(xh, ex.sine_fab("exp", b, 64, [1, 1], 0.0, t=1e-3))))
    out["laplacian_64"] = leg
    del op, bt, x, A
    # --- the paper's restart-rand on the headline workload: full sketched Gram-Schmidt (k = m) and the
    # restart as Algorithm 2 states it (exp of the growing block matrix), against the default (k = 4,
    # quadrature restart) timed above
    w = WORKLOAD
    A = wl.convdiff_3d(w["N"], w["peclet"])
    b = wl.gaussian_vector(A.n, w["b_seed"])
    op = fab.CSROperator.from_arrays(ctx, A.rowptr, A.colind, A.vals)
    bt = torch.as_tensor(b, device="cuda")
    kw = dict(m=w["m"], k=w["m"], d=w["d"], zeta=w["zeta"], seed=w["sketch_seed"], tol=w["tol"], max_cycles=20,
              method="growing")
    sec, (x, info) = _timed(lambda: fab.solve(op, bt, "exp", t=w["t"], **kw), reps=3)
    leg = {"workload": "convdiff_3d_N128_Pe50, k = m = 50, restart by exp of the growing block matrix",
           "solves_per_s": 1.0 / sec, "cycles": info["cycles"], "matvecs": info["matvecs"], "status": info["status"],
           "kappa_T": info["kappa_T"]}
    xh = x[:, 0].cpu().numpy()
    checks.append((leg, "rel_err", lambda ex, xh=xh, b=b, w=w: rel(
        xh, ex.kron_exp_fab(b, ex.problem_factors("convdiff_3d", w["N"], peclet=w["peclet"])[0], w["t"]))))
    out["restart_rand_128"] = leg
    # --- the paper's unrestarted randomized Arnoldi at its sketch sizes: one cycle, k = m = 60 (the
    # whole basis in the Gram-Schmidt and the update), d = 1200 and 3600, on the same operator; the
    # update reads up to 61 basis columns per step (the tall-skinny product of Section 2.2)
    for d_un in (1200, 3600):
        kw = dict(m=60, k=60, d=d_un, zeta=w["zeta"], seed=w["sketch_seed"], tol=1e-12, max_cycles=1)
        sec, (x, info) = _timed(lambda kw=kw: fab.solve(op, bt, "exp", t=w["t"], check=False, **kw), reps=3)
        fab.timing_enable(ctx, True)
        fab.solve(op, bt, "exp", t=w["t"], check=False, **kw)
        tm = fab.timing_read(ctx)
        fab.timing_enable(ctx, False)
        ub = update_bytes(A.n, 60, 60)
        us = tm["update_ms"] / max(tm["update_launches"], 1) / 1e3
        sb, _ = algorithmic_bytes(A.n, A.nnz, 60, ib=op.index_bytes())
        ss = tm["spmv_ms"] / max(tm["spmv_launches"], 1) / 1e3
        leg = {"workload": f"convdiff_3d_N128_Pe50, one cycle (no restart), m = k = 60, d = {d_un}",
               "solves_per_s": 1.0 / sec, "ms_per_solve": 1e3 * sec, "status": info["status"],
               "update": {"kernel": "k_update_wide<double> (k = m window update)", "avg_us": us * 1e6, "bytes_per_launch_avg": ub,
                          "GB/s": ub / us / 1e9, "frac": ub / us / 1e9 / HBM_PEAK_GBS},
               "spmv_sketch": {"avg_us": ss * 1e6, "GB/s": sb / ss / 1e9, "frac": sb / ss / 1e9 / HBM_PEAK_GBS}}
        xh = x[:, 0].cpu().numpy()
        checks.append((leg, "rel_err", lambda ex, xh=xh, b=b, w=w: rel(
            xh, ex.kron_exp_fab(b, ex.problem_factors("convdiff_3d", w["N"], peclet=w["peclet"])[0], w["t"]))))
        out[f"unrestarted_rand_128_d{d_un}"] = leg
    del op, bt, x, A
    torch.cuda.empty_cache()
    # --- z^(-1/2) of the shifted 3-D Laplacian, 256^3 (n = 16.8M), FP32 vs FP64
    N = 256
    A = wl.shifted_laplacian_3d(N, 1.0)
    b = wl.gaussian_vector(A.n, 0)
    lo = 3 * 4 * (N + 1) ** 2 * np.sin(np.pi / (2 * (N + 1))) ** 2 + 1.0
    spec = (lo, 12 * (N + 1) ** 2 + 1.0)
    leg = {"workload": "shifted_laplacian_3d_N256 z^(-1/2)", "n": A.n, "nnz": A.nnz, "m": 30, "k": 2, "d": 120,
           "zeta": 8, "tol": 1e-6}
    for dt, name in ((torch.float32, "f32"), (torch.float64, "f64")):
        op = fab.CSROperator.from_arrays(ctx, A.rowptr, A.colind, A.vals, dtype=dt)
        bt = torch.as_tensor(b, dtype=dt, device="cuda")
        sec, (x, info) = _timed(lambda: fab.solve(op, bt, "invsqrt", m=30, k=2, d=120, zeta=8, seed=1, tol=1e-6,
                                                  spec=spec, max_cycles=300))
        leg[name] = {"solves_per_s": 1.0 / sec, "cycles": info["cycles"], "ms_per_cycle": 1e3 * sec / info["cycles"],
                     "status": info["status"], "kappa_T": info["kappa_T"]}
        # HBM roofline of this workload's loop: three cycles again with HIP events recorded by every
        # launch of the fused SpMV + sketch kernel and around every step loop (algorithmic bytes as for
        # the headline)
        fab.timing_enable(ctx, True)
        fab.solve(op, bt, "invsqrt", m=30, k=2, d=120, zeta=8, seed=1, tol=1e-6, spec=spec, max_cycles=3,
                  check=False)
        tm = fab.timing_read(ctx)
        # the step loop again with events only at its ends (events between its kernels add gaps)
        fab.timing_enable(ctx, 2)
        fab.solve(op, bt, "invsqrt", m=30, k=2, d=120, zeta=8, seed=1, tol=1e-6, spec=spec, max_cycles=3,
                  check=False)
        tl = fab.timing_read(ctx)
        fab.timing_enable(ctx, False)
        sb, stb = algorithmic_bytes(A.n, A.nnz, 2, es=4 if dt == torch.float32 else 8, ib=op.index_bytes())
        spmv_gbs = sb / (tm["spmv_ms"] / tm["spmv_launches"] / 1e3) / 1e9
        loop_gbs = stb * tl["loop_steps"] / (tl["loop_ms"] / 1e3) / 1e9
        leg[name]["roofline"] = {"spmv_sketch_GB/s": spmv_gbs, "spmv_sketch_frac": spmv_gbs / HBM_PEAK_GBS,
                                 "spmv_bytes_per_launch": sb, "loop_GB/s": loop_gbs,
                                 "loop_frac": loop_gbs / HBM_PEAK_GBS, "bytes_per_step": stb,
                                 "loop_frac_with_kernel_events":
                                     stb * tm["loop_steps"] / (tm["loop_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS}
        xh = x[:, 0].cpu().numpy()
        bb = b if dt == torch.float64 else b.astype(np.float32).astype(np.float64)
        checks.append((leg[name], "rel_err",
                       lambda ex, xh=xh, bb=bb, N=N: rel(xh, ex.sine_fab("invsqrt", bb, N, [1, 1, 1], 1.0))))
        del op, bt, x
        torch.cuda.empty_cache()
    out["invsqrt_256"] = leg
    del A
    # --- batched: 64 right-hand sides x 8 time points, anisotropic 1024^2, FP32; single FP64 for comparison
    N, nb = 1024, 64
    T = [10.0 ** (-5 + 2 * i / 7) for i in range(8)]
    A = wl.anisotropic_2d(N, 0.01)
    Bm = np.stack([wl.gaussian_vector(A.n, 300 + r) for r in range(nb)], axis=1).astype(np.float32)
    op32 = fab.CSROperator.from_arrays(ctx, A.rowptr, A.colind, A.vals, dtype=torch.float32)
    Bt = torch.as_tensor(Bm, device="cuda")
    kw = dict(m=20, k=2, d=80, zeta=8, seed=1, tol=1e-6, max_cycles=300)
    sec, (X, infos) = _timed(lambda: fab.solve_batched(op32, Bt, "exp", t=T, **kw))
    samples = {(r, i): X[:, r, i].cpu().numpy() for r in (0, nb - 1) for i in range(len(T))}
    op64 = fab.CSROperator.from_arrays(ctx, A.rowptr, A.colind, A.vals, dtype=torch.float64)
    b64 = torch.as_tensor(Bm[:, 0].astype(np.float64), device="cuda")
    sec1, (x1, info1) = _timed(lambda: fab.solve(op64, b64, "exp", t=T, **kw))
    single = [x1[:, i].cpu().numpy() for i in range(len(T))]
    # the same FP64 single solves at looser tolerances, so the batched FP32 rate can be set against
    # the FP64 rate at the accuracy the FP32 batch reaches (its error is in rel_err_sampled_max)
    by_tol = {}
    for tl in (1e-5, 1e-4):
        kwl = dict(kw, tol=tl)
        sec2, (x2, info2) = _timed(lambda kwl=kwl: fab.solve(op64, b64, "exp", t=T, **kwl))
        s2 = [x2[:, i].cpu().numpy() for i in range(len(T))]
        by_tol[f"{tl:.0e}"] = {"results_per_s": len(T) / sec2, "cycles": info2["cycles"]}
        checks.append((by_tol[f"{tl:.0e}"], "rel_err_max", lambda ex, N=N, T=T, Bm=Bm, s2=s2: max(
            rel(s2[i], ex.sine_fab("exp", Bm[:, 0].astype(np.float64), N, [1.0, 0.01], 0.0, t=t))
            for i, t in enumerate(T))))
    # the batch at tol 1e-4, which FP32 reaches on this problem (at 1e-6 its increments stall at the
    # FP32 rounding level and it runs to the cycle limit), against the FP64 single solves at 1e-4
    kw4 = dict(kw, tol=1e-4)
    sec4, (X4, infos4) = _timed(lambda: fab.solve_batched(op32, Bt, "exp", t=T, **kw4))
    samples4 = {(r, i): X4[:, r, i].cpu().numpy() for r in (0, nb - 1) for i in range(len(T))}
    at4 = {"tol": 1e-4, "results_per_s": nb * len(T) / sec4, "seconds": sec4,
           "cycles_max": max(i["cycles"] for i in infos4), "group": infos4[0]["group"],
           "single_f64_results_per_s": by_tol["1e-04"]["results_per_s"],
           "speedup_vs_single_f64_same_tol": (nb * len(T) / sec4) / by_tol["1e-04"]["results_per_s"]}
    checks.append((at4, "rel_err_sampled_max", lambda ex, N=N, T=T, Bm=Bm, samples=samples4: max(
        rel(v, ex.sine_fab("exp", Bm[:, r].astype(np.float64), N, [1.0, 0.01], 0.0, t=T[i]))
        for (r, i), v in samples.items())))
    leg = {"workload": "anisotropic_2d_N1024 (1, 0.01), exp, 64 rhs x 8 t in [1e-5, 1e-3]", "n": A.n,
           "results": nb * len(T), "results_per_s": nb * len(T) / sec, "seconds": sec,
           "cycles_max": max(i["cycles"] for i in infos), "group": infos[0]["group"], "values": "f32",
           "single_f64": {"results_per_s": len(T) / sec1, "cycles": info1["cycles"], "tol": kw["tol"]},
           "single_f64_looser_tol": by_tol,
           "speedup_vs_single_f64": (nb * len(T) / sec) / (len(T) / sec1),
           "at_tol_1e-4": at4}
    checks.append((leg, "rel_err_sampled_max", lambda ex, N=N, T=T, Bm=Bm, samples=samples: max(
        rel(v, ex.sine_fab("exp", Bm[:, r].astype(np.float64), N, [1.0, 0.01], 0.0, t=T[i])) for (r, i), v in samples.items())))
    checks.append((leg["single_f64"], "rel_err_max", lambda ex, N=N, T=T, Bm=Bm, single=single: max(
        rel(single[i], ex.sine_fab("exp", Bm[:, 0].astype(np.float64), N, [1.0, 0.01], 0.0, t=t)) for i, t in enumerate(T))))
    out["batched_1024"] = leg
    del op32, op64, Bt, X, x1
    torch.cuda.empty_cache()
    # --- ragged: 32 Laplacians on grids 64^2 .. 512^2, FP32, one solve
    Ns = [int(round(64 * 8 ** (i / 31))) for i in range(32)]
    ops, bs, b64s = [], [], []
    for i, Ng in enumerate(Ns):
        Ag = wl.laplacian_2d(Ng)
        bg = wl.gaussian_vector(Ag.n, 1000 + i).astype(np.float32)
        ops.append(fab.CSROperator.from_arrays(ctx, Ag.rowptr, Ag.colind, Ag.vals, dtype=torch.float32))
        bs.append(torch.as_tensor(bg, device="cuda"))
        b64s.append(bg.astype(np.float64))
    xs_out = fab.solve_ragged(ops, bs, "exp", t=1e-3, **kw)[0]   # outputs kept: the timed calls replay one graph
    sec, (xs, infos) = _timed(lambda: fab.solve_ragged(ops, bs, "exp", t=1e-3, xs=xs_out, **kw))
    xr = [v[:, 0].cpu().numpy() for v in xs]
    leg = {"workload": "32 laplacian_2d, N = 64 .. 512 (geometric), exp t = 1e-3", "values": "f32",
           "rows_total": sum(Ng * Ng for Ng in Ns), "operators_per_s": 32 / sec, "seconds": sec,
           "cycles_max": max(i["cycles"] for i in infos)}
    checks.append((leg, "rel_err_max", lambda ex, xr=xr, b64s=b64s, Ns=Ns: max(
        rel(xr[i], ex.sine_fab("exp", b64s[i], Ng, [1, 1], 0.0, t=1e-3)) for i, Ng in enumerate(Ns))))
    out["ragged_32"] = leg
    del ops, bs, xs, xs_out
    torch.cuda.empty_cache()
    # --- gradient of <c, exp(-tA) b>: 96^3 convection-diffusion, Pe 20, t = 1e-4
    N, t = 96, 1e-4
    A = wl.convdiff_3d(N, 20.0)
    op = fab.CSROperator.from_arrays(ctx, A.rowptr, A.colind, A.vals)
    op_t = op.transpose()
    bn, cn = wl.gaussian_vector(A.n, 0), wl.gaussian_vector(A.n, 7)
    c = torch.as_tensor(cn, device="cuda")

    def grad_once():
        bb = torch.as_tensor(bn, device="cuda").requires_grad_(True)
        tt = torch.tensor(t, dtype=torch.float64, requires_grad=True)
        L = torch.dot(c, fab.exp_action(op, bb, tt, op_t=op_t, m=40, k=4, d=160, zeta=8, seed=1, tol=1e-10))
        L.backward()
        return bb.grad.cpu().numpy(), float(tt.grad)

    sec, (gb, gt) = _timed(grad_once)
    leg = {"workload": "convdiff_3d_N96_Pe20, d<c, exp(-tA) b>/db and /dt, t = 1e-4", "n": A.n,
           "forward_plus_adjoint_ms": 1e3 * sec}

    def grad_errs(ex):
        factors, _ = ex.problem_factors("convdiff_3d", N, peclet=20.0)
        _, gbo, gto = ex.exp_action_grads(factors, bn, cn, t)
        leg["rel_err_dt"] = abs(gt - gto) / abs(gto)
        return rel(gb, gbo)

    checks.append((leg, "rel_err_db", grad_errs))
    out["adjoint_96"] = leg
    return out, checks


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the plain restarted Arnoldi comparator")
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads (FP32, batched, ragged, adjoint)")
    ap.add_argument("--profile", action="store_true",
                    help="few solves, no CPU leg, plus a device copy of known size for counter calibration")
    ap.add_argument("--profile-batched", action="store_true",
                    help="short batched 1024^2 x 64 run for rocprofv3 (grouped kernel)")
    ap.add_argument("--profile-256", choices=("f32", "f64"),
                    help="a short 256^3 z^(-1/2) run (FP32 or FP64 values and basis) for rocprofv3")
    ap.add_argument("--profile-ragged", action="store_true",
                    help="the ragged 32-operator solve, replayed once after a marker, for rocprofv3 --kernel-trace")
    ap.add_argument("--summarize-overlap", nargs=3, metavar=("TRACE_DIR", "OUT_MD", "COMMAND"))
    ap.add_argument("--summarize-pmc", nargs="+", metavar="ARG",
                    help="FETCH_DIR WRITE_DIR [OUT_JSON WORKLOAD KERNEL_LABEL KERNEL_REGEX]")
    ap.add_argument("--summarize-trace", nargs="+", metavar="ARG", help="TRACE_DIR OUT_MD COMMAND [WORKLOAD]")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return 0
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return 0
    if args.summarize_overlap:
        summarize_overlap(*args.summarize_overlap)
        return 0
    if args.profile_ragged:
        return profile_ragged()
    if args.profile_256:
        return profile_256(args.profile_256)
    if args.profile_batched:
        return profile_batched()
    if args.gpus != 1:
        print(f"bench.py: this build runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is documented, not built).", file=sys.stderr)
        return 2
    if args.profile:
        args.no_cpu_baseline, args.no_extra = True, True
        args.steps, args.warmup = min(args.steps, 3), min(args.warmup, 1)

    import numpy as np
    import torch

    import paper_2503_22631_amd as fab
    import workloads as wl

    w = WORKLOAD
    A = wl.convdiff_3d(w["N"], w["peclet"])
    b = wl.gaussian_vector(A.n, w["b_seed"])
    ctx = fab.Context()
    op = fab.CSROperator.from_arrays(ctx, A.rowptr, A.colind, A.vals)
    bt = torch.as_tensor(b, device="cuda")
    params = fab.Params(m=w["m"], k=w["k"], d=w["d"], zeta=w["zeta"], seed=w["sketch_seed"], tol=w["tol"])
    x = torch.empty((1, A.n), dtype=torch.float64, device="cuda")
    work = torch.empty(fab.workspace_size(op, params, 1), dtype=torch.uint8, device="cuda")
    solve = lambda prm: fab.solve(op, bt, "exp", t=w["t"], x=x, work=work, params=prm)

    for _ in range(args.warmup):
        solve(params)
    # timed region: K complete solves, each cycle replayed from its captured graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        xv, info = solve(params)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x_gpu = xv[:, 0].cpu().numpy().copy()
    elapsed = t1 - t0
    value = args.steps / elapsed
    # instrumented region: the same K solves with HIP events recorded by every launch of the fused
    # SpMV + sketch kernel (start and end of its dispatch) and around each step loop (cycles enqueued
    # directly on the stream)
    fab.timing_enable(ctx, True)
    torch.cuda.synchronize()
    i0 = time.perf_counter()
    for _ in range(args.steps):
        solve(params)
    torch.cuda.synchronize()
    i1 = time.perf_counter()
    tm = fab.timing_read(ctx)
    # the step loops again with events only at their ends: the events between a loop's kernels
    # (above) add gaps of their own, which the solve's graph replay does not have
    fab.timing_enable(ctx, 2)
    for _ in range(args.steps):
        solve(params)
    torch.cuda.synchronize()
    tl = fab.timing_read(ctx)
    fab.timing_enable(ctx, False)

    spmv_bytes, step_bytes = algorithmic_bytes(A.n, A.nnz, w["k"], ib=op.index_bytes())
    spmv_avg_s = tm["spmv_ms"] / max(tm["spmv_launches"], 1) / 1e3
    achieved = spmv_bytes / spmv_avg_s / 1e9
    loop_gbs = step_bytes * tl["loop_steps"] / (tl["loop_ms"] / 1e3) / 1e9 if tl["loop_ms"] > 0 else None
    loop_gbs_ev = step_bytes * tm["loop_steps"] / (tm["loop_ms"] / 1e3) / 1e9 if tm["loop_ms"] > 0 else None
    upd_b = update_bytes(A.n, w["m"], w["k"])
    upd_s = tm["update_ms"] / max(tm["update_launches"], 1) / 1e3

    comparison, x_plain = None, None
    if not args.no_compare:
        pp = fab.Params(m=w["m"], k=w["k"], d=w["d"], zeta=w["zeta"], seed=w["sketch_seed"], tol=w["tol"],
                        method="plain")
        wp = torch.empty(fab.workspace_size(op, pp, 1), dtype=torch.uint8, device="cuda")
        xp = torch.empty((1, A.n), dtype=torch.float64, device="cuda")
        fab.solve(op, bt, "exp", t=w["t"], x=xp, work=wp, params=pp)
        kp = max(2, args.steps // 3)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(kp):
            xpv, pinfo = fab.solve(op, bt, "exp", t=w["t"], x=xp, work=wp, params=pp)
        torch.cuda.synchronize()
        pdt = (time.perf_counter() - p0) / kp
        x_plain = xpv[:, 0].cpu().numpy().copy()
        # The comparator's kernels are less tuned than the sketched path's: its bytes per solve over
        # its time give its HBM fraction, and the time it would take at the sketched loop's
        # fraction gives the speedup at equal bandwidth efficiency (a bound on what tuning it buys).
        pbytes = pinfo["cycles"] * plain_cycle_bytes(A.n, A.nnz, w["m"], 1, ib=op.index_bytes())
        p_gbs = pbytes / pdt / 1e9
        comparison = {"plain_restarted_arnoldi_solves_per_s": 1.0 / pdt, "plain_cycles": pinfo["cycles"],
                      "plain_matvecs": pinfo["matvecs"], "sketched_speedup_time_to_tol": value * pdt,
                      "plain_bytes_per_solve": pbytes, "plain_GB/s": p_gbs, "plain_frac": p_gbs / HBM_PEAK_GBS,
                      "sketched_speedup_at_equal_frac": value * pbytes / (loop_gbs * 1e9) if loop_gbs else None}
        del wp, xp

    if args.profile:
        src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    out = {"metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {**w, "n": A.n, "nnz": A.nnz, "cycles": info["cycles"], "matvecs": info["matvecs"],
                      "status": info["status"], "est_rel_update": info["est_rel_update"]},
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": read_traffic(),
                        "kernel": "k_spmv_sketch (fused CSR SpMV + sparse-sign sketch)",
                        "bytes_per_launch": spmv_bytes, "avg_launch_us": spmv_avg_s * 1e6,
                        "launches_timed": tm["spmv_launches"],
                        "timing": "HIP events recorded by every launch's dispatch on the kernel's stream "
                                  "(hipExtLaunchKernelGGL start/stop events), over the instrumented region "
                                  f"({args.steps} solves, {1e3 * (i1 - i0) / args.steps:.2f} ms/solve)"},
           "loop": {"GB/s": loop_gbs, "frac": (loop_gbs / HBM_PEAK_GBS) if loop_gbs else None,
                    "bytes_per_step": step_bytes, "steps_timed": tl["loop_steps"],
                    "avg_step_us": 1e3 * tl["loop_ms"] / max(tl["loop_steps"], 1),
                    "timing": "HIP events at each cycle's step-loop ends only (no events between its kernels)",
                    "with_kernel_events": {"frac": (loop_gbs_ev / HBM_PEAK_GBS) if loop_gbs_ev else None,
                                           "avg_step_us": 1e3 * tm["loop_ms"] / max(tm["loop_steps"], 1)},
                    "update": {"kernel": "k_orth_update (sketch-space Gram-Schmidt + window update)",
                               "avg_us": upd_s * 1e6, "bytes_per_launch_avg": upd_b,
                               "GB/s": upd_b / upd_s / 1e9 if upd_s > 0 else None,
                               "frac": upd_b / upd_s / 1e9 / HBM_PEAK_GBS if upd_s > 0 else None,
                               "launches_timed": tm["update_launches"]}},
           "comparison": comparison}
    checks = []
    if not args.no_extra:
        del work, x
        torch.cuda.empty_cache()
        out["extra"], checks = extra_legs(fab, ctx)
    if not args.no_cpu_baseline:
        x_cpu_plain = None
        if comparison is not None:  # the plain method on the host cores, beside the GPU comparator
            comparison["cpu_plain_arnoldi"], x_cpu_plain = cpu_plain_leg(A, b)
            comparison["sketched_gpu_vs_plain_cpu"] = value * comparison["cpu_plain_arnoldi"]["seconds_per_solve"]
        cpu, errs = cpu_baseline_leg(A, b, x_gpu, x_plain, checks, x_cpu_plain)
        cpu["host"] = cpu_info()
        out["cpu_baseline"] = cpu
        out["rel_err_vs_oracle"] = errs["gpu_rel_err"]
        if comparison is not None:
            comparison["plain_rel_err_vs_oracle"] = errs["plain_rel_err"]
            comparison["cpu_plain_arnoldi"]["rel_err_vs_oracle"] = errs["cpu_plain_rel_err"]
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
