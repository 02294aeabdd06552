"""Benchmark: SpMV GB/s of the autotuned format vs fixed CSR on the HPCG
27-point problem at 104^3 (1,124,864 rows, 29,791,000 nnz, FP64), plus CG
solves/s with p50/p99 latency on the same matrix.

A timed step is one SpMV y = A x in the format the selector picked, with A,
x and y resident in HBM.  Around the K timed steps the same run measures the
fixed-CSR SpMV, the selection (conversion + profiling cost), the CG solves
and the CPU oracle; everything is printed as one JSON line on stdout.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 104]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def event_times_us(torch, fn, steps):
    """Runs fn() `steps` times on the current stream, each bracketed by HIP
    events on that stream; returns per-launch durations in microseconds."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return [a.elapsed_time(b) * 1000.0 for a, b in ev]


def cpu_baseline(p, budget_s=12.0):
    """The oracle's CSR SpMV on the host cores, timed on a bounded sample."""
    import numpy as np
    import inputs
    import oracle
    cores = oracle.set_threads(len(os.sched_getaffinity(0)))
    x = inputs.uniform_vector(p.ncols)
    oracle.spmv_csr(p.row_ptr, p.col, p.val, x)  # warm
    reps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s and reps < 200:
        oracle.spmv_csr(p.row_ptr, p.col, p.val, x)
        reps += 1
    dt = (time.perf_counter() - t0) / reps
    bytes_ = p.nnz * 12 + (p.nrows + 1) * 4 + 16 * p.nrows
    # oracle CG on a small sample problem (16^3) for CPU solves/s
    q = inputs.hpcg27(16)
    t1 = time.perf_counter()
    ncg = 0
    while time.perf_counter() - t1 < 3.0:
        oracle.cg(q.row_ptr, q.col, q.val, q.b, tol=1e-10)
        ncg += 1
    return {"value": round(bytes_ / dt / 1e9, 2), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"{reps} oracle CSR SpMVs (FP64, OpenMP rows) on the full {p.name} matrix, "
                      f"{dt * 1e3:.1f} ms each; oracle CG on hpcg27_16: "
                      f"{ncg / (time.perf_counter() - t1):.1f} solves/s single-threaded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=104)
    ap.add_argument("--cg-solves", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only-spmv", action="store_true", help="skip selection/CG (profiling runs)")
    ap.add_argument("--format", default=None, help="force a format instead of selecting")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after the timed steps, run a device copy of this many MiB `steps` times "
                         "(calibration kernel of known size for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import inputs
    import paper_2209_06478_amd as dsm

    dev = torch.device("cuda:0")
    log(f"[bench] generating hpcg27_{args.n}")
    p = inputs.hpcg27(args.n)
    ctx = dsm.Context(0)
    rp = torch.from_numpy(p.row_ptr).to(dev)
    col = torch.from_numpy(p.col).to(dev)
    val = torch.from_numpy(p.val).to(dev)
    A = dsm.Matrix.from_csr(ctx, p.nrows, p.ncols, rp, col, val)
    del rp, col, val
    x = torch.from_numpy(inputs.uniform_vector(p.ncols)).to(dev)
    y = torch.empty(p.nrows, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def spmv():
        A.spmv(x, out=y)

    # fixed CSR (default kernel) for the comparison
    log("[bench] fixed CSR")
    A.variant = 0
    for _ in range(args.warmup):
        spmv()
    csr_us = event_times_us(torch, spmv, args.steps)
    csr_bytes = p.nnz * 12 + (p.nrows + 1) * 4 + 16 * p.nrows
    csr_avg = float(np.mean(csr_us))

    sel = None
    if args.format:
        A.convert(args.format)
    elif not args.only_spmv:
        log("[bench] selecting")
        t0 = time.perf_counter()
        sel = A.select(use_cache=False)
        sel["wall_ms"] = (time.perf_counter() - t0) * 1e3
        log(f"[bench] chose {sel['chosen']} variant {sel['chosen_variant']}")
    info = A.info()
    fmt = info["format_name"]
    vdt_b = 8
    N, nnz = p.nrows, p.nnz
    bytes_by_fmt = {
        "csr": nnz * (vdt_b + 4) + (N + 1) * 4 + 16 * N,
        "coo": nnz * (vdt_b + 8) + 16 * N,
        "dia": info["ndiag"] * N * vdt_b + info["ndiag"] * 4 + 16 * N,
        "ell": info["ell_width"] * N * (vdt_b + 4) + 16 * N,
        "hyb": info["ell_width"] * N * (vdt_b + 4) + info["coo_nnz"] * (vdt_b + 8) + 16 * N,
        "hdc": info["ndiag"] * N * vdt_b + info["ndiag"] * 4 + info["csr_nnz"] * (vdt_b + 4) + (N + 1) * 4 + 16 * N,
    }
    sel_bytes = bytes_by_fmt[fmt]

    # timed region: K SpMV steps in the selected format
    log(f"[bench] timed region: {args.steps} SpMV steps in {fmt}")
    for _ in range(args.warmup):
        spmv()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        spmv()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    ev_us = event_times_us(torch, spmv, args.steps)
    avg_us = float(np.mean(ev_us))
    value = sel_bytes / (ms_per_step * 1e-3) / 1e9
    achieved = sel_bytes / (avg_us * 1e-6) / 1e9

    copy = None
    if args.copy_mb > 0:
        nel = args.copy_mb * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        cus = event_times_us(torch, lambda: dst.copy_(src), args.steps)
        copy = {"mib": args.copy_mb, "avg_us": round(float(np.mean(cus)), 3),
                "gbps": round(2 * nel * 8 / (float(np.mean(cus)) * 1e-6) / 1e9, 1)}
        del src, dst

    # CG solves on the selected format
    cg = None
    if not args.only_spmv and args.cg_solves > 0:
        log("[bench] CG solves")
        b = torch.from_numpy(p.b).to(dev)
        lat = []
        res = None
        for i in range(args.cg_solves + 1):
            xs = torch.zeros(N, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            xs, res = A.cg(b, x=xs, tol=1e-10)
            lat.append((time.perf_counter() - t1) * 1e3)
        lat = np.array(lat[1:])
        cg = {"format": fmt, "tol": 1e-10, "iters": res["iters"], "status": res["status"],
              "relres_true": res["relres_true"], "solves_per_s": round(1e3 / float(lat.mean()), 3),
              "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
              "ms_per_iter": round(float(lat.mean()) / max(res["iters"], 1), 4)}

    cpu = None if args.no_cpu else cpu_baseline(p)
    out = {
        "metric": "SpMV GB/s vs HBM peak (selected vs fixed CSR); CG solves/s + p99 latency",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"hpcg27_{args.n}", "nrows": N, "nnz": nnz, "format": fmt,
                   "variant": A.variant, "value_dtype": "f64", "vector_dtype": "f64"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel_avg_us": round(avg_us, 3), "algorithmic_bytes": int(sel_bytes)},
        "fixed_csr": {"gbps": round(csr_bytes / (csr_avg * 1e-6) / 1e9, 2), "avg_us": round(csr_avg, 3),
                      "bytes": int(csr_bytes)},
        "speedup_vs_fixed_csr": round(csr_avg / avg_us, 3),
        "select": sel,
        "copy_probe": copy,
        "cg": cg,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    A.close()
    ctx.close()


if __name__ == "__main__":
    main()
