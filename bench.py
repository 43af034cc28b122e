#!/usr/bin/env python3
"""Benchmark of the restarted sketched Krylov f(A)b path on one MI355X.

Workload (one "step" = one complete solve, i.e. every cycle of the hot path):
  3-D convection-diffusion, 128^3 interior grid (n = 2,097,152, nnz = 14,581,760), central
  differences, wind (1,1,1), Peclet 50, CSR FP64; x = exp(-1e-4 A) b with b ~ N(0,1) (seed 0);
  sketched restarted Krylov m = 50, window k = 4, sketch d = 200 rows, zeta = 8, seed 1, tol 1e-8.

Prints one JSON line: solves/s, the roofline of the dominant kernel (fused SpMV + sketch, timed
with HIP events on its own stream during the timed solves), the step-loop bandwidth, the plain
restarted Arnoldi comparator on the same GPU, and the CPU oracle timed on the host as baseline
(which also gives the relative error of the GPU result against the exact FP64 solution).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--profile]
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
KERNEL_SRC = os.path.join(ROOT, "paper_2503_22631_amd", "csrc", "step_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "spmv_sketch_convdiff128_traffic.json")
COPY_BYTES = 256 << 20


def algorithmic_bytes(n: int, nnz: int, k: int, es: int = 8):
    """Bytes the method must move (int32 indices): per launch of the fused SpMV + sketch kernel
    (values + column indices + row pointers + read w_j + write z; S is generated, not read) and
    per Arnoldi step (that plus the window update: read z and k basis columns, write w_{j+1})."""
    spmv = (es + 4) * nnz + 4 * (n + 1) + 2 * es * n
    step = spmv + (2 + k) * es * n
    return spmv, step


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


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


def cpu_baseline_leg(A, b, x_gpu, x_plain):
    """The oracle, as it stands, on the host: complete solves of the same workload by its FP64
    step-by-step twin (same sketch), with BLAS limited to one thread, repeated until about 10 s of
    CPU work (at most 4 solves).  Also the exact solution by the Kronecker-product closed form, for
    the relative errors of the GPU results."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import exact, krylov, sketch

    w = WORKLOAD
    As = A.to_scipy()
    solves, total = 0, 0.0
    with threadpool_limits(limits=1):
        while solves < 4 and (solves == 0 or total < 10.0):
            t0 = time.perf_counter()
            S = sketch.sketch_matrix(A.n, w["d"], w["zeta"], seed=w["sketch_seed"])
            xo, info = krylov.restart_solve(As, b, "exp", w["t"], m=w["m"], k=w["k"], S=S, tol=w["tol"])
            total += time.perf_counter() - t0
            solves += 1
    dt = total / solves
    factors, _ = exact.problem_factors("convdiff_3d", w["N"], peclet=w["peclet"])
    ref = exact.kron_exp_fab(b, factors, w["t"])
    rel = lambda v: float(np.linalg.norm(v - ref) / np.linalg.norm(ref))
    return ({"value": 1.0 / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
             "sample": f"{solves} full solve(s) of the same workload by the FP64 oracle twin ({info.cycles} cycles, "
                       f"{info.matvecs} matvecs each, sketch generation included; scipy CSR products, 1 BLAS "
                       f"thread); {total:.1f} s in total",
             "seconds_per_solve": dt, "oracle_rel_err": rel(xo)},
            {"gpu_rel_err": rel(x_gpu), "plain_rel_err": rel(x_plain) if x_plain is not None else None})


def summarize_pmc(fetch_dir: str, write_dir: str):
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

    is_spmv = lambda k: re.search(r"k_spmv_sketch<\w+, 0,", k) is not None   # mode 0 = SpMV + sketch
    fetch = load(fetch_dir, "FETCH_SIZE")
    write = load(write_dir, "WRITE_SIZE")
    f_k, nf = avg(fetch, is_spmv)
    w_k, nw = avg(write, is_spmv)
    f_c, w_c = calib(fetch), calib(write)
    kib = 1024.0
    f_scale = (COPY_BYTES / kib) / f_c if f_c else 1.0
    w_scale = (COPY_BYTES / kib) / w_c if w_c else 1.0
    traffic = (f_k * f_scale + w_k * w_scale) * kib if (f_k is not None and w_k is not None) else None
    rec = {"kernel": "k_spmv_sketch<double, SpMV+sketch, zeta<=8>", "workload": WORKLOAD["workload"],
           "kernel_source_sha": kernel_sha(), "dispatches": [nf, nw],
           "fetch_kib_per_dispatch": f_k, "write_kib_per_dispatch": w_k,
           "copy_fetch_kib": f_c, "copy_write_kib": w_c, "copy_bytes": COPY_BYTES,
           "fetch_scale": f_scale, "write_scale": w_scale, "traffic_bytes_per_launch": traffic,
           "unscaled_bytes_per_launch": (f_k + w_k) * kib if (f_k is not None and w_k is not None) else None}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    json.dump(rec, open(TRAFFIC_FILE, "w"), indent=1)
    print(json.dumps(rec))


def summarize_trace(trace_dir: str, out_md: str, command: str):
    """Markdown table of a rocprofv3 --kernel-trace --stats run (kernel_stats.csv)."""
    f = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)[0]
    rows = list(csv.DictReader(open(f)))
    lines = [f"# rocprofv3 kernel statistics: {WORKLOAD['workload']}", "", "Command (from the repository root on the GPU box):",
             "", "```", command, "```", "",
             "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"].split("(")[0].replace("|", "/")
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    print(out_md)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the plain restarted Arnoldi comparator")
    ap.add_argument("--profile", action="store_true",
                    help="few solves, no CPU leg, plus a device copy of known size for counter calibration")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-trace", nargs=3, metavar=("TRACE_DIR", "OUT_MD", "COMMAND"))
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return 0
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return 0
    if args.gpus != 1:
        print(f"bench.py: this build runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is documented, not built).", file=sys.stderr)
        return 2
    if args.profile:
        args.no_cpu_baseline, args.steps, args.warmup = True, min(args.steps, 3), min(args.warmup, 1)

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
    # instrumented region: the same K solves with HIP events around every launch of the fused
    # SpMV + sketch kernel and around each step loop (cycles enqueued directly on the stream)
    fab.timing_enable(ctx, True)
    torch.cuda.synchronize()
    i0 = time.perf_counter()
    for _ in range(args.steps):
        solve(params)
    torch.cuda.synchronize()
    i1 = time.perf_counter()
    tm = fab.timing_read(ctx)
    fab.timing_enable(ctx, False)

    spmv_bytes, step_bytes = algorithmic_bytes(A.n, A.nnz, w["k"])
    spmv_avg_s = tm["spmv_ms"] / max(tm["spmv_launches"], 1) / 1e3
    achieved = spmv_bytes / spmv_avg_s / 1e9
    loop_gbs = step_bytes * tm["loop_steps"] / (tm["loop_ms"] / 1e3) / 1e9 if tm["loop_ms"] > 0 else None

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
        comparison = {"plain_restarted_arnoldi_solves_per_s": 1.0 / pdt, "plain_cycles": pinfo["cycles"],
                      "plain_matvecs": pinfo["matvecs"], "sketched_speedup_time_to_tol": value * pdt}
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
                        "timing": "HIP events on the kernel's stream around every launch, over the instrumented "
                                  f"region ({args.steps} solves, {1e3 * (i1 - i0) / args.steps:.2f} ms/solve)"},
           "loop": {"GB/s": loop_gbs, "frac": (loop_gbs / HBM_PEAK_GBS) if loop_gbs else None,
                    "bytes_per_step": step_bytes, "steps_timed": tm["loop_steps"],
                    "avg_step_us": 1e3 * tm["loop_ms"] / max(tm["loop_steps"], 1)},
           "comparison": comparison}
    if not args.no_cpu_baseline:
        cpu, errs = cpu_baseline_leg(A, b, x_gpu, x_plain)
        cpu["host"] = cpu_info()
        out["cpu_baseline"] = cpu
        out["rel_err_vs_oracle"] = errs["gpu_rel_err"]
        if comparison is not None:
            comparison["plain_rel_err_vs_oracle"] = errs["plain_rel_err"]
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
