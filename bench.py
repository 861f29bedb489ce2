#!/usr/bin/env python3
"""Benchmark of the red-black Gauss-Seidel hot path on one MI355X.

Workload: 8191 x 8191 interior points (h = 1/8192), FP64, zero Dirichlet
ring, f i.i.d. uniform[-1, 1) from seed 0, u0 = 0, 200 full sweeps.  One
step is one rbgs_solve call with a fixed sweep count: pack u and f into the
split colour layout, 200 red+black sweeps, the FP64 residual norm, unpack.
Inputs are resident in HBM before the timed region.

Output: one JSON line with GLUP/s (lattice point updates per second,
N^2 * sweeps / time), the dominant kernel's roofline (algorithmic bytes per
launch over its measured average duration, against 8 TB/s HBM), the STREAM
probe bandwidth, and the CPU oracle timed on a bounded sample as baseline.
Progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GLUP/s + HBM GB/s (% peak) per sweep; time-to-1e-8 residual vs plain FP64"
HBM_PEAK_GBS = 8000.0
BYTES_PER_LUP = {"f64": 24.0, "f32": 12.0}  # split layout: other colour + own f read, own colour written
PROFILE_DIR = os.path.join(ROOT, "profiles")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the sources of the kernels the roofline figure refers to."""
    h = hashlib.sha256()
    for name in ("sweep_plain.hip", "sweep_blocked.hip", "rbgs_internal.h"):
        with open(os.path.join(ROOT, "paper_2607_01735_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_name, n):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    path = os.path.join(PROFILE_DIR, f"traffic_{kernel_name}_n{n}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def stream_probe(torch, rb, gib=2.0):
    n = int(gib * (1 << 30) / 8) // 2 * 2
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    c = torch.empty(n, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b.fill_(2.0)
    c.fill_(3.0)
    out = {}
    for kind, name, words in ((0, "copy", 2), (1, "triad", 3)):
        rb.rbgs_stream_probe(kind, a, b, c)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        reps = 10
        for _ in range(reps):
            rb.rbgs_stream_probe(kind, a, b, c)
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / reps
        out[f"{name}_gbs"] = round(words * n * 8 / (ms * 1e-3) / 1e9, 1)
    del a, b, c
    torch.cuda.empty_cache()
    return out


def cpu_baseline(n, sweeps_cap, budget_s=12.0):
    """The oracle (plain C, OpenMP over rows of one colour) on the host cores:
    whole sweeps of the same 8191^2 FP64 problem until about budget_s
    seconds have passed."""
    import numpy as np

    import oracle
    import workloads as W
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=0)
    u = W.zeros(n)
    oracle.sweep(u, f, h, 1)  # warm-up (page faults, thread start)
    done, t0 = 0, time.perf_counter()
    while done < sweeps_cap:
        oracle.sweep(u, f, h, 1)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(n * n * done / dt / 1e9, 3), "unit": "GLUP/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{done} full sweeps of the {n}x{n} FP64 workload (of {sweeps_cap}), "
                      f"{dt:.1f} s wall, OpenMP threads={cores}"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=8191)
    ap.add_argument("--sweeps", type=int, default=200)
    ap.add_argument("--kernel", default="auto", choices=["auto", "plain", "blocked"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU: every box here has exactly one MI355X, so "
              f"--gpus {args.gpus} is not run (the multi-GPU design is described, not built).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2607_01735_amd as rb
    import workloads as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    n, sweeps = args.n, args.sweeps
    h = W.spacing(n)
    log(f"device {torch.cuda.get_device_name(0)}; building inputs n={n}")
    f = torch.from_numpy(W.uniform_rhs(n, seed=0)).to("cuda")
    u = torch.zeros((n + 2, n + 2), dtype=torch.float64, device="cuda")
    grid = rb.make_grid(u, h)
    ws = torch.empty(rb.rbgs_workspace_size(grid, rb.rbgs.F64), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()

    def step():
        return rb.rbgs_solve(u, f, sweeps, 0.0, check_every=sweeps, h=h, kernel=args.kernel,
                             workspace=ws, timing=True)

    for k in range(args.warmup):
        info = step()
        log(f"warmup {k + 1}/{args.warmup}: rel={info['rel_residual']:.6e} "
            f"sweep_ms={info['timing']['sweep_ms']:.2f}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sweep_ms = 0.0
    launches = 0
    for k in range(args.steps):
        info = step()
        sweep_ms += info["timing"]["sweep_ms"]
        launches += info["timing"]["sweep_launches"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    glups = n * n * sweeps / (ms_per_step * 1e-3) / 1e9
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {glups:.1f} GLUP/s, "
        f"rel={info['rel_residual']:.6e}")

    kernel_used = args.kernel if args.kernel != "auto" else "plain"
    # Dominant kernel: the half-sweep.  One launch updates one colour:
    # ceil(n^2/2) red or floor(n^2/2) black points, 24 B each (FP64).
    avg_launch_ms = sweep_ms / max(launches, 1)
    per_launch_bytes = BYTES_PER_LUP["f64"] * n * n / 2.0
    achieved = per_launch_bytes / (avg_launch_ms * 1e-3) / 1e9
    traffic = read_traffic("half_sweep_f64", n)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": "k_half_sweep<double,2>",
                "avg_launch_us": round(avg_launch_ms * 1e3, 2),
                "bytes_per_launch": per_launch_bytes}
    probe = None if args.no_probe else stream_probe(torch, rb)
    if probe:
        log(f"STREAM probe: {probe}")
    base = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        base = cpu_baseline(n, sweeps)
        log(f"cpu baseline {base}")
    line = {
        "metric": METRIC, "value": round(glups, 2), "unit": "GLUP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{n}x{n} interior FP64, h=1/{n + 1}, zero Dirichlet, "
                               f"f~U[-1,1) seed 0, u0=0, {sweeps} sweeps per step",
                   "n": n, "sweeps": sweeps, "kernel": kernel_used},
        "hbm_gbs_algorithmic": round(glups * BYTES_PER_LUP["f64"], 1),
        "roofline": roofline,
        "stream_probe": probe,
        "cpu_baseline": base,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
