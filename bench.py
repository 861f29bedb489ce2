#!/usr/bin/env python3
"""Benchmark of the red-black Gauss-Seidel hot path on one MI355X.

Workload: 8191 x 8191 interior points (h = 1/8192), FP64, zero Dirichlet
ring, f i.i.d. uniform[-1, 1) from seed 0, u0 = 0, 200 full sweeps.  One
step is one rbgs_solve call with a fixed sweep count: pack u and f into the
split colour layout, 200 red+black sweeps, the FP64 residual norm, unpack.
Inputs are resident in HBM before the timed region.  The timed kernel is
the library's default (the persistent temporally blocked sweep at this
size); the plain one-launch-per-half-sweep kernel is timed beside it.

Output: one JSON line with GLUP/s (lattice point updates per second,
N^2 * sweeps / time), the dominant kernel's roofline (algorithmic bytes per
launch over its measured average duration, against 8 TB/s HBM), the plain
kernel's figures, and the comparisons of time to a relative residual of
1e-8 against the plain FP64 sweep: the 255 x 255 sine problem for the
resident, blocked and mixed-precision solves, 16 small grids solved as one
batch, and 511 x 511 GRF problems with the learned initial guess; beside
them the 16383^2 refinement throughput, the 512-grid batch throughput, the
STREAM probe bandwidth and the CPU oracle timed on a bounded sample as
baseline.  Progress goes to stderr.
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


def kernel_source_hash(names):
    """Hash of the sources of the kernel a roofline figure refers to."""
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2607_01735_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "half_sweep_f64": ("sweep_plain.hip", "rbgs_internal.h"),
    "blocked_f64": ("sweep_blocked.hip", "blocked_pipeline.h", "rbgs_blocked.h", "rbgs_internal.h"),
    "mg_restrict_f64": ("multigrid.hip",),
    "mg_prolong_red_f64": ("multigrid.hip",),
    "residual_f64": ("residual.hip",),
    "mc9_quarter_f64": ("multicolour9.hip",),
    "rb3_half_f64": ("sweep3d.hip", "rbgs_internal.h"),
}


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
    if vals.get("kernel_source_sha256") != kernel_source_hash(KERNEL_SOURCES[kernel_name]):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def read_profile_avg(kernel_name, n):
    """Average launch duration (us) of a kernel in the committed rocprofv3
    kernel-trace summary of this workload, if that summary was taken on the
    current kernel source; else None.  Summary lines read
    `stat: <kernel_name> avg_us=<v> calls=<c> sha=<source hash>`."""
    path = os.path.join(PROFILE_DIR, f"sweep_f64_n{n}_stats.md")
    if not os.path.exists(path):
        return None
    want = kernel_source_hash(KERNEL_SOURCES[kernel_name])
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) >= 3 and parts[0] == "stat:" and parts[1] == kernel_name:
                kv = dict(p.split("=", 1) for p in parts[2:] if "=" in p)
                if kv.get("sha") != want:
                    return None
                try:
                    return {"avg_us": float(kv["avg_us"]), "calls": int(kv["calls"])}
                except (KeyError, ValueError):
                    return None
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


def _timed_solve(torch, rb, u, f, **kw):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = rb.rbgs_solve(u, f, **kw)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, info


def time_to_tolerance(torch, rb, W, n=255, tol=1e-8):
    """Wall time and sweeps to rel <= tol from u = 0 on the n x n problem with
    f = 2 pi^2 sin(pi x) sin(pi y) (124 616 sweeps at n = 255 by the closed
    form), for the plain FP64 judge and the faster forms: the resident band
    kernel and the blocked kernel in FP64, FP64 refinement around FP32 (or
    bfloat16-rhs) inner sweeps on the resident kernel, and red-black SOR at
    the optimal omega (the extension that changes the sweep count)."""
    h = W.spacing(n)
    f = torch.from_numpy(W.sine_rhs(n)).to("cuda")
    out = {"problem": f"{n}x{n} FP64 sine, u0=0, rel<={tol:g}"}
    forms = [("plain_f64", dict(kernel="plain", check_every=1000)),
             ("resident_f64", dict(kernel="resident", check_every=1000)),
             ("blocked_f64", dict(kernel="blocked", fuse=4, tile_rows=8, check_every=1000)),
             ("f32_ir_resident", dict(kernel="resident", precision="f32_ir", inner_sweeps=4000,
                                      check_every=4000)),
             ("bf16rhs_ir_resident", dict(kernel="resident", precision="bf16rhs_ir",
                                          inner_sweeps=1000, check_every=1000)),
             ("sor_f64", dict(kernel="plain", omega=0.0, check_every=10)),
             ("sor_resident_f64", dict(kernel="resident", omega=0.0, check_every=100))]
    for name, kw in forms:
        u = torch.zeros((n + 2, n + 2), dtype=torch.float64, device="cuda")
        warm = {k: v for k, v in kw.items() if k not in ("inner_sweeps", "check_every")}
        rb.rbgs_solve(u, f, 8, 0.0, check_every=8, h=h, **warm)
        u.zero_()
        dt, info = _timed_solve(torch, rb, u, f, max_sweeps=4_000_000, rel_tol=tol, h=h, **kw)
        out[name] = {"seconds": round(dt, 4), "sweeps": info["sweeps"],
                     "rel_residual": info["rel_residual"], "status": info["status"]}
        log(f"time-to-tol {name}: {dt:.3f} s, {info['sweeps']} sweeps, "
            f"rel={info['rel_residual']:.3e}")
    base = out["plain_f64"]["seconds"]
    for name, _ in forms[1:]:
        out[name]["speedup_vs_plain_f64"] = round(base / out[name]["seconds"], 3)
    # precision and relaxation against the same kernel in FP64 Gauss-Seidel
    same = out["resident_f64"]["seconds"]
    for name in ("f32_ir_resident", "bf16rhs_ir_resident", "sor_resident_f64"):
        out[name]["speedup_vs_same_kernel_f64"] = round(same / out[name]["seconds"], 3)
    return out


def time_to_tolerance_fourier(torch, rb, W, n=1023, tol=1e-8):
    """The mixed-precision recipe at a size where the solve finishes: the
    64-mode Fourier right-hand side (seed 0) on n x n from u = 0 to rel <=
    tol (108 000 sweeps at n = 1023 by the closed form), for the plain FP64
    judge, the library's FP64 choice (blocked) and FP64 refinement around
    FP32 / bfloat16-rhs inner sweeps."""
    h = W.spacing(n)
    f = torch.from_numpy(W.fourier_rhs(n, seed=0)).to("cuda")
    out = {"problem": f"{n}x{n} FP64, 64 Fourier modes seed 0, u0=0, rel<={tol:g}"}
    forms = [("plain_f64", dict(kernel="plain", check_every=1000)),
             ("auto_f64", dict(kernel="auto", check_every=1000)),
             ("blocked_f64", dict(kernel="blocked", check_every=4000)),
             ("f32_ir", dict(kernel="auto", precision="f32_ir", inner_sweeps=4000,
                             check_every=4000)),
             ("f32_ir_blocked", dict(kernel="blocked", precision="f32_ir", inner_sweeps=4000,
                                     check_every=4000)),
             ("bf16rhs_ir", dict(kernel="auto", precision="bf16rhs_ir", inner_sweeps=1000,
                                 check_every=1000)),
             ("sor_f64", dict(kernel="plain", omega=0.0, check_every=50))]
    for name, kw in forms:
        u = torch.zeros((n + 2, n + 2), dtype=torch.float64, device="cuda")
        warm = {k: v for k, v in kw.items() if k not in ("inner_sweeps", "check_every")}
        rb.rbgs_solve(u, f, 16, 0.0, check_every=16, h=h, **warm)
        u.zero_()
        dt, info = _timed_solve(torch, rb, u, f, max_sweeps=1_000_000, rel_tol=tol, h=h, **kw)
        out[name] = {"seconds": round(dt, 4), "sweeps": info["sweeps"],
                     "rel_residual": info["rel_residual"], "status": info["status"]}
        log(f"time-to-tol {n} {name}: {dt:.3f} s, {info['sweeps']} sweeps, "
            f"rel={info['rel_residual']:.3e}")
    base = out["plain_f64"]["seconds"]
    for name, _ in forms[1:]:
        out[name]["speedup_vs_plain_f64"] = round(base / out[name]["seconds"], 3)
    # each precision against the same kernel choice in FP64
    for name, ref in (("f32_ir", "auto_f64"), ("bf16rhs_ir", "auto_f64"),
                      ("f32_ir_blocked", "blocked_f64")):
        out[name]["speedup_vs_same_kernel_f64"] = round(out[ref]["seconds"] / out[name]["seconds"], 3)
    return out


MG_RESTRICT_BYTES = 20.0  # per fine point: u and f read, coarse f written, coarse u zeroed
MG_PROLONG_RED_BYTES = 13.0  # black and red f read, red written (interpolant fused into the red half-sweep)


def mg_model_bytes(sizes, nu1, nu2, coarse_sweeps):
    """Algorithmic HBM bytes of one V-cycle plus the finest-level residual
    check, as the library runs it: on each level above the coarsest, nu1 +
    nu2 sweeps at 24 B per point, of which the first post-smoothing red half
    (12 B) is replaced by the fused prolongation (13 B), and the restriction
    (20 B); the coarsest level's sweeps; the residual reads u and f once
    (16 B/point).  Levels of at most 127^2 run in one workgroup from the L2
    and are counted the same way (they are a rounding error here)."""
    total = 0.0
    for n in sizes[:-1]:
        per = (nu1 + nu2) * BYTES_PER_LUP["f64"] + MG_RESTRICT_BYTES
        if nu2 >= 1:
            per += MG_PROLONG_RED_BYTES - BYTES_PER_LUP["f64"] / 2
        else:
            per += 18.0
        total += n * n * per
    total += sizes[-1] ** 2 * coarse_sweeps * BYTES_PER_LUP["f64"]
    return total + 16.0 * sizes[0] ** 2


def multigrid_to_tolerance(torch, rb, W, tol=1e-8, sizes=(1023, 8191, 16383)):
    """Red-black Gauss-Seidel as the smoother of a V-cycle (the multilevel
    extension): wall time and cycles to rel <= tol from u = 0 on the 64-mode
    Fourier right-hand side (seed 0), V(2,2) and V(1,1) on the plain
    smoother, and the time per cycle from 10 fixed cycles with the model
    bytes of a cycle per that time."""
    out = {"problem": f"n x n FP64, 64 Fourier modes seed 0, u0=0, rel<={tol:g}"}
    for n in sizes:
        h = W.spacing(n)
        f = torch.from_numpy(W.fourier_rhs(n, seed=0)).to("cuda")
        grid = rb.make_grid(f, h)
        ws = torch.empty(rb.rbgs_mg_workspace_size(grid, rb.rbgs.F64), dtype=torch.uint8,
                         device="cuda")
        levels = []
        m = n
        while True:
            levels.append(m)
            if m < 3 or m % 2 == 0:
                break
            m = (m - 1) // 2
        for nu in ((2, 2), (1, 1)):
            u = torch.zeros_like(f)
            rb.rbgs_mg_solve(u, f, 1, -1.0, pre_sweeps=nu[0], post_sweeps=nu[1], h=h,
                             kernel="plain", workspace=ws)  # warm-up
            best, info = None, None
            for _ in range(3):
                u.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = rb.rbgs_mg_solve(u, f, 40, tol, pre_sweeps=nu[0], post_sweeps=nu[1], h=h,
                                        kernel="plain", workspace=ws)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            u.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rb.rbgs_mg_solve(u, f, 10, -1.0, pre_sweeps=nu[0], post_sweeps=nu[1], h=h,
                             kernel="plain", workspace=ws)
            torch.cuda.synchronize()
            per_cycle = (time.perf_counter() - t0) / 10
            model = mg_model_bytes(levels, nu[0], nu[1], info["coarse_sweeps"])
            key = f"n{n}_V{nu[0]}{nu[1]}"
            out[key] = {"seconds": round(best, 5), "cycles": info["cycles"],
                        "rel_residual": info["rel_residual"], "status": info["status"],
                        "levels": info["levels"], "graph": info["graph"],
                        "ms_per_cycle": round(per_cycle * 1e3, 3),
                        "model_bytes_per_cycle": model,
                        "model_GBs": round(model / per_cycle / 1e9, 1)}
            log(f"multigrid {key}: {best * 1e3:.2f} ms, {info['cycles']} cycles, "
                f"rel={info['rel_residual']:.3e}, {per_cycle * 1e3:.3f} ms/cycle, "
                f"{model / per_cycle / 1e9:.0f} GB/s model")
        del f, ws, u
        torch.cuda.empty_cache()
    return out


MC9_BYTES_PER_LUP = 40.0  # per sweep: four quarter-sweeps, each 5 words per updated point


def multicolour9_throughput(torch, rb, W, n=8191, sweeps=100, with_solve=True):
    """Four-colour Gauss-Seidel for the 9-point Laplacian (the multi-colour
    extension) on the 8191^2 FP64 grid: time of `sweeps` sweeps as the
    difference of a (sweeps + 1)-sweep call and a 1-sweep call (both pack and
    unpack once), GLUP/s and model bytes (40 B per point per sweep); and the
    time to rel <= 1e-8 at 255^2 from u = 0 (sine right-hand side); each for
    the plain kernel (a launch per colour) and the flag-driven form (one
    launch, a counter per block)."""
    h = W.spacing(n)
    f = torch.from_numpy(W.uniform_rhs(n, seed=0)).to("cuda")
    u = torch.zeros_like(f)
    ws = torch.empty(rb.rbgs_mc9_workspace_size(rb.make_grid(f, h)), dtype=torch.uint8,
                     device="cuda")

    def timed(k, kernel):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rb.rbgs_mc9_sweep(u, f, k, h=h, kernel=kernel, workspace=ws)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    out = {"workload": f"{n}x{n} FP64, f~U[-1,1) seed 0, {sweeps} sweeps"}
    for kernel in ("plain", "resident"):
        timed(3, kernel)
        one = min(timed(1, kernel) for _ in range(3))
        many = min(timed(sweeps + 1, kernel) for _ in range(2))
        per_sweep = (many - one) / sweeps
        glups = n * n / per_sweep / 1e9
        res = {"ms_per_sweep": round(per_sweep * 1e3, 4), "GLUP/s": round(glups, 2),
               "model_bytes_per_lup": MC9_BYTES_PER_LUP,
               "model_GBs": round(glups * MC9_BYTES_PER_LUP, 1),
               "frac_of_8TBs": round(glups * MC9_BYTES_PER_LUP / HBM_PEAK_GBS, 4)}
        out["plain" if kernel == "plain" else "flag_driven"] = res
        log(f"multicolour 9-point {n} {kernel}: {per_sweep * 1e3:.3f} ms/sweep, {glups:.1f} GLUP/s, "
            f"{glups * MC9_BYTES_PER_LUP:.0f} GB/s model")
    del u, f, ws
    torch.cuda.empty_cache()
    if not with_solve:
        return out
    m = 255
    hm = W.spacing(m)
    fm = torch.from_numpy(W.sine_rhs(m)).to("cuda")
    um = torch.zeros_like(fm)
    for kernel in ("plain", "resident"):
        rb.rbgs_mc9_solve(um, fm, 8, -1.0, check_every=8, h=hm, kernel=kernel)
        um.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = rb.rbgs_mc9_solve(um, fm, 4_000_000, 1e-8, check_every=1000, h=hm, kernel=kernel)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        key = "time_to_1e-8_255_sine_" + ("plain" if kernel == "plain" else "flag_driven")
        out[key] = {"seconds": round(dt, 4), "sweeps": info["sweeps"],
                    "rel_residual": info["rel_residual"], "status": info["status"]}
        log(f"multicolour 9-point time-to-tol 255 {kernel}: {dt:.3f} s, {info['sweeps']} sweeps")
        um.zero_()
    return out


UNET_CHANNELS = (16, 32, 64, 128)


def unet_flops(n, factor=4, channels=UNET_CHANNELS):
    """Multiply-add FLOPs (2 per MAC) of the U-Net's 3x3 convolutions for one
    n x n sample: forward, and a training step (forward, input gradients of
    every layer but the first, weight gradients); the first layer counts
    its input as the 16 channels the kernel pads it to."""
    sizes = [n]
    for _ in channels[1:]:
        sizes.append((sizes[-1] + 1) // factor - 1)
    layers = []  # (cin, cout, level)
    cin = 16
    for l, c in enumerate(channels):
        layers += [(cin, c, l), (c, c, l)]
        cin = c
    for l in range(len(channels) - 2, -1, -1):
        layers += [(channels[l + 1] + channels[l], channels[l], l), (channels[l], channels[l], l)]
    fwd = sum(2.0 * 9 * ci * co * sizes[l] ** 2 for ci, co, l in layers)
    first = 2.0 * 9 * layers[0][0] * layers[0][1] * sizes[0] ** 2
    return fwd, 3.0 * fwd - first


def unet_throughput(torch, rb, n=511, batch=8, steps=10):
    """The learned part's network on its workload: the shipped factor-4 U-Net
    on 511 x 511 GRF inputs (held-out seeds), `steps` training steps at batch
    8 (forward, backward, Adam; lr tiny so the weights barely move) and
    `steps` forward passes, with achieved TFLOP/s of the 3x3 convolutions
    against the bfloat16 dense MFMA peak."""
    from paper_2607_01735_amd import learned
    shipped = learned.pretrained_net(rb)
    f = learned.fields_on_device(torch, n, [learned.TEST_SEED0 + 100 + i for i in range(batch)])
    net = rb.UNet(n, batch, factor=4)
    net.set_params(shipped.get_params())
    target = torch.zeros_like(f)
    for _ in range(2):
        net.train_step(f, target, 1e-7)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.train_step(f, target, 1e-7)
    torch.cuda.synchronize()
    train_ms = (time.perf_counter() - t0) * 1e3 / steps
    u0 = torch.zeros_like(f)
    net.forward(f, u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.forward(f, u0)
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t0) * 1e3 / steps
    fwd, train = unet_flops(n)
    out = {"workload": f"factor-4 U-Net on {n}x{n}, batch {batch}, shipped weights",
           "train_step_ms": round(train_ms, 3), "forward_ms": round(fwd_ms, 3),
           "conv_gflop_forward_per_sample": round(fwd / 1e9, 3),
           "conv_gflop_train_per_sample": round(train / 1e9, 3),
           "train_tflops": round(batch * train / (train_ms * 1e-3) / 1e12, 2),
           "forward_tflops": round(batch * fwd / (fwd_ms * 1e-3) / 1e12, 2),
           "peak_tflops_bf16_dense": 2500.0}
    log(f"unet: {out}")
    del f, u0, target
    torch.cuda.empty_cache()
    return out


def pass_overlap(torch, rb, W, n=8191, sweeps=200):
    """The GPU form of the paper's red/black overlap traces (Section 4): the
    headline workload once more through the verification kernel with the
    per-item trace on (not timed with the headline; the trace adds a store
    and two counter reads per item).  From the records (device real-time
    counter, 10 ns): the wall time of each pass (first start to last end),
    how far consecutive passes overlap, and how many passes have items in
    flight at once, sampled over the launch."""
    import numpy as np
    h = W.spacing(n)
    f = torch.from_numpy(W.uniform_rhs(n, seed=0)).to("cuda")
    u = torch.zeros_like(f)
    cap = 1 << 16
    trace = torch.zeros(cap * 4, dtype=torch.int64, device="cuda")
    t = rb.rbgs_sweep(u, f, sweeps, h=h, kernel="blocked", debug_trace=trace, timing=True)
    rec = trace.view(cap, 4).cpu().numpy().view(np.uint64)
    items = int(np.count_nonzero(rec[:, 0]))
    passes = int(t["passes"])
    if items == 0 or items % passes:
        return {"error": f"{items} trace records for {passes} passes"}
    ntiles = items // passes
    rec = rec[:items].astype(np.int64)
    pas = rec[:, 2] >> 32
    t0 = rec[:, 0].min()
    start, end = rec[:, 0] - t0, rec[:, 1] - t0
    first = np.array([start[pas == p].min() for p in range(passes)])
    last = np.array([end[pas == p].max() for p in range(passes)])
    span = last - first
    overlap = [(last[p - 1] - first[p]) / span[p] for p in range(1, passes)]
    grid = np.linspace(0, end.max(), 400, endpoint=False)
    in_flight = [len(np.unique(pas[(start <= x) & (end > x)])) for x in grid]
    ticks_us = 0.01
    return {"workload": f"{n}x{n} FP64, {sweeps} sweeps, fuse {t['fuse']}: the deeper "
                        f"passes' launch, {passes} passes x {ntiles} tiles",
            "launch_us": round(float(end.max()) * ticks_us, 1),
            "pass_wall_us_median": round(float(np.median(span)) * ticks_us, 1),
            "item_us_median": round(float(np.median(end - start)) * ticks_us, 1),
            "consecutive_pass_overlap_median": round(float(np.median(overlap)), 3),
            "passes_in_flight_mean": round(float(np.mean(in_flight)), 2),
            "passes_in_flight_max": int(np.max(in_flight))}


def rb3_throughput(torch, rb, n=767, sweeps=40, tol_sizes=(63, 127), tol=1e-8):
    """Red-black Gauss-Seidel in 3D (the higher-dimension extension): n^3
    FP64 with f ~ U[-1, 1) drawn on the device (seeded), time per sweep from
    the difference of a (sweeps + 1)-sweep and a 1-sweep call, GLUP/s and
    model bytes (24 B per point per sweep, as in 2D), for the plain kernel
    (one launch per half-sweep) and the flag-driven form (one launch, a
    counter per block).  Then, per size in tol_sizes, the solve from u = 0 to
    rel <= tol with each (residual every 500 sweeps; the plain solve's
    rounds are graph-captured)."""
    h = 1.0 / (n + 1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    f = torch.zeros((n + 2,) * 3, dtype=torch.float64, device="cuda")
    f[1:-1, 1:-1, 1:-1] = torch.rand((n, n, n), dtype=torch.float64, device="cuda",
                                     generator=gen) * 2.0 - 1.0
    u = torch.zeros_like(f)
    ws = torch.empty(rb.rbgs_rb3_workspace_size(rb.make_grid3(f, h)), dtype=torch.uint8,
                     device="cuda")

    def per_sweep_of(kernel):
        def timed(k):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rb.rbgs_rb3_sweep(u, f, k, h=h, workspace=ws, kernel=kernel)
            torch.cuda.synchronize()
            return time.perf_counter() - t0

        timed(2)
        one = min(timed(1) for _ in range(3))
        many = min(timed(sweeps + 1) for _ in range(2))
        return (many - one) / sweeps

    def figures(per_sweep):
        glups = n ** 3 / per_sweep / 1e9
        return {"ms_per_sweep": round(per_sweep * 1e3, 4), "GLUP/s": round(glups, 2),
                "model_bytes_per_lup": BYTES_PER_LUP["f64"],
                "model_GBs": round(glups * BYTES_PER_LUP["f64"], 1),
                "frac_of_8TBs": round(glups * BYTES_PER_LUP["f64"] / HBM_PEAK_GBS, 4)}

    plain = per_sweep_of("plain")
    flags = per_sweep_of("resident")
    out = {"workload": f"{n}^3 FP64, f~U[-1,1) (device generator, seed 0), {sweeps} sweeps"}
    out.update(figures(plain))
    out["flag_driven"] = dict(figures(flags), speedup_vs_plain=round(plain / flags, 3))
    log(f"3D red-black {n}^3: plain {plain * 1e3:.3f} ms/sweep ({n ** 3 / plain / 1e9:.1f} GLUP/s), "
        f"flag-driven {flags * 1e3:.3f} ms/sweep ({n ** 3 / flags / 1e9:.1f} GLUP/s)")
    del u, f, ws
    torch.cuda.empty_cache()
    for m in tol_sizes:
        hm = 1.0 / (m + 1)
        gen.manual_seed(1)
        fm = torch.zeros((m + 2,) * 3, dtype=torch.float64, device="cuda")
        fm[1:-1, 1:-1, 1:-1] = torch.rand((m, m, m), dtype=torch.float64, device="cuda",
                                          generator=gen) * 2.0 - 1.0
        row = {"problem": f"{m}^3 FP64, f~U[-1,1) (device generator, seed 1), u0=0, "
                          f"rel<={tol:g}, residual every 500 sweeps"}
        for kernel in ("plain", "resident"):
            um = torch.zeros_like(fm)
            rb.rbgs_rb3_solve(um, fm, 1000, tol, check_every=500, h=hm, kernel=kernel)  # warm-up
            um.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = rb.rbgs_rb3_solve(um, fm, 2_000_000, tol, check_every=500, h=hm, kernel=kernel)
            torch.cuda.synchronize()
            row["plain" if kernel == "plain" else "flag_driven"] = {
                "seconds": round(time.perf_counter() - t0, 4), "sweeps": info["sweeps"],
                "rel_residual": info["rel_residual"], "status": info["status"]}
        row["speedup_flag_driven_vs_plain"] = round(row["plain"]["seconds"] /
                                                    row["flag_driven"]["seconds"], 3)
        out[f"time_to_{tol:g}_{m}"] = row
        log(f"3D time to {tol:g} at {m}^3: {row}")
    return out


def learned_guess(torch, rb, tol=1e-8, seeds=4):
    """The learned-guess workload: 511 x 511 GRF right-hand sides (held-out
    seeds 10^6 + 20 + i), FP64 solve to rel <= tol from u = 0 (the judge)
    against the same solve started from the shipped network's guess, kept
    only if it wins the residual comparison after 500 sweeps of both starts
    (inference and comparison sweeps included in the time); the literal
    comparison of starting residuals is reported beside it."""
    from paper_2607_01735_amd import learned
    n = 511
    net = learned.pretrained_net(rb)
    ids = [learned.TEST_SEED0 + 20 + i for i in range(seeds)]
    fs = learned.fields_on_device(torch, n, ids)
    rows = []
    for i, seed in enumerate(ids):
        f = fs[i]
        u = torch.zeros_like(f)
        rb.rbgs_solve(u, f, 16, 0.0, check_every=16)  # warm-up
        u.zero_()
        dt0, base = _timed_solve(torch, rb, u, f, max_sweeps=2_000_000, rel_tol=tol,
                                 check_every=2000)
        row = {"seed": seed, "zero_start": {"seconds": round(dt0, 4), "sweeps": base["sweeps"]}}
        for k in (500, 0):
            u = torch.zeros_like(f)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            got = net.solve_learned(u, f, 2_000_000, tol, check_every=2000, compare_after=k)
            torch.cuda.synchronize()
            row[f"learned_k{k}"] = {"seconds": round(time.perf_counter() - t0, 4),
                                    "sweeps": got["sweeps"], "used_guess": got["used_guess"],
                                    "rel_residual": got["rel_residual"]}
        log(f"learned seed {seed}: {row}")
        rows.append(row)
    z = sum(r["zero_start"]["seconds"] for r in rows)
    out = {"workload": f"{n}x{n} GRF (length scale U[0.02,0.3]), held-out seeds {ids}, FP64, "
                       f"rel<={tol:g}, network weights/unet_grf511_f4.npy", "per_seed": rows}
    for k in (500, 0):
        out[f"time_ratio_k{k}"] = round(sum(r[f"learned_k{k}"]["seconds"] for r in rows) / z, 4)
        out[f"sweep_ratio_k{k}"] = round(sum(r[f"learned_k{k}"]["sweeps"] for r in rows) /
                                         sum(r["zero_start"]["sweeps"] for r in rows), 4)
    del fs
    torch.cuda.empty_cache()
    return out


def batched_to_tolerance(torch, rb, W, count=16, tol=1e-8, chunk=4000):
    """Many small grids to rel <= tol: `count` grids with sizes uniform on
    {63, 127, 255} (seed 1), f i.i.d. N(0,1) (seed 1000+g), FP64, u0 = 0.
    Batched: one graph-captured persistent launch of `chunk` sweeps for all
    grids, then every grid's residual, until all are below tol; the batched
    refinement solve (FP32 inner sweeps of all grids batched, FP64 residual
    and correction per grid); and the batched FP64 solve (converged grids
    leave the batch).  Judge: each
    grid solved alone with the plain FP64 kernel (residual every 1000
    sweeps)."""
    import numpy as np
    rng = np.random.default_rng(1)
    sizes = [int(x) for x in rng.choice([63, 127, 255], size=count)]
    fs = [torch.from_numpy(W.normal_rhs(n, seed=1000 + g)).to("cuda") for g, n in enumerate(sizes)]
    us = [torch.zeros_like(f) for f in fs]
    plan = rb.BatchPlan(us, fs, chunk)
    plan.launch()
    plan.check()
    for u in us:
        u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while True:
        plan.launch()
        plan.check()
        done += chunk
        rels = [rb.rbgs_residual(u, f)[1] for u, f in zip(us, fs)]
        if max(rels) <= tol or done >= 400_000:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.close()
    out = {"workload": f"{count} grids, N in {{63,127,255}} seed 1, f~N(0,1), FP64, u0=0, "
                       f"rel<={tol:g} for every grid", "sizes": sizes,
           "batched": {"seconds": round(dt, 4), "sweeps": done, "max_rel": max(rels)}}
    # The same grids through the batched solve: FP64 refinement per grid,
    # the FP32 inner sweeps (`chunk` per outer step) of every unconverged
    # grid in one batched persistent launch.
    rb.rbgs_solve_batched(us, fs, 10, tol, 10)  # warm-up
    for u in us:
        u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = rb.rbgs_solve_batched(us, fs, 400_000, tol, chunk)
    torch.cuda.synchronize()
    dt_ir = time.perf_counter() - t0
    out["batched_f32_ir"] = {"seconds": round(dt_ir, 4),
                             "max_sweeps": max(i["sweeps"] for i in infos),
                             "max_outer": max(i["outer_iters"] for i in infos),
                             "max_rel": max(i["rel_residual"] for i in infos),
                             "all_converged": all(i["status"] == 0 for i in infos)}
    # The batched FP64 solve: `chunk` FP64 sweeps of every unconverged grid
    # in one batched persistent launch, then each of those grids' residual;
    # a grid below tol drops out of the next launch.
    rb.rbgs_solve_batched(us, fs, 10, tol, 10, precision="f64")  # warm-up
    for u in us:
        u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = rb.rbgs_solve_batched(us, fs, 400_000, tol, chunk, precision="f64")
    torch.cuda.synchronize()
    dt_f64 = time.perf_counter() - t0
    out["batched_f64_solve"] = {"seconds": round(dt_f64, 4),
                                "max_sweeps": max(i["sweeps"] for i in infos),
                                "max_rel": max(i["rel_residual"] for i in infos),
                                "all_converged": all(i["status"] == 0 for i in infos)}
    # The same batched FP64 solve with red-black SOR at each grid's optimum
    # omega (the F1 extension), residual every 100 sweeps.
    rb.rbgs_solve_batched(us, fs, 10, tol, 10, precision="f64", omega=0.0)  # warm-up
    for u in us:
        u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = rb.rbgs_solve_batched(us, fs, 400_000, tol, 100, precision="f64", omega=0.0)
    torch.cuda.synchronize()
    dt_sor = time.perf_counter() - t0
    out["batched_sor_solve"] = {"seconds": round(dt_sor, 4),
                                "max_sweeps": max(i["sweeps"] for i in infos),
                                "max_rel": max(i["rel_residual"] for i in infos),
                                "all_converged": all(i["status"] == 0 for i in infos)}
    t_plain = 0.0
    sweeps_plain = 0
    for f in fs:
        u = torch.zeros_like(f)
        dt1, info = _timed_solve(torch, rb, u, f, max_sweeps=400_000, rel_tol=tol,
                                 check_every=1000, kernel="plain")
        t_plain += dt1
        sweeps_plain = max(sweeps_plain, info["sweeps"])
    out["plain_f64_one_by_one"] = {"seconds": round(t_plain, 4), "max_sweeps": sweeps_plain}
    out["speedup_vs_plain_f64"] = round(t_plain / dt, 2)
    out["speedup_f32_ir_vs_plain_f64"] = round(t_plain / dt_ir, 2)
    out["speedup_f64_solve_vs_plain_f64"] = round(t_plain / dt_f64, 2)
    out["speedup_sor_solve_vs_plain_f64"] = round(t_plain / dt_sor, 2)
    log(f"batched to tolerance: {out}")
    return out


def refinement_throughput(torch, rb, W, n=16383, inner=100, outer=2):
    """The mixed-precision workload: 16383^2, f = 64 random Fourier modes
    (seed 0), u0 = 0.  Times `outer` refinement steps of `inner` FP32 sweeps
    (FP64 residual and correction around them) and the same number of FP64
    sweeps, both with the persistent kernel.  Reaching rel 1e-10 here needs
    millions of sweeps; the solve to tolerance is measured at smaller N."""
    h = W.spacing(n)
    log(f"refinement workload n={n}: building f")
    f = torch.from_numpy(W.fourier_rhs(n, seed=0)).to("cuda")
    u = torch.zeros((n + 2, n + 2), dtype=torch.float64, device="cuda")
    out = {"workload": f"{n}x{n}, 64 Fourier modes seed 0, u0=0, {outer} outer steps x {inner} "
                       f"FP32 sweeps vs {outer * inner} FP64 sweeps"}
    for name, kw in (("f32_ir", dict(precision="f32_ir", inner_sweeps=inner)),
                     ("bf16rhs_ir", dict(precision="bf16rhs_ir", inner_sweeps=inner)),
                     ("f64", dict(precision="f64"))):
        u.zero_()
        rb.rbgs_solve(u, f, inner, 0.0, check_every=inner, h=h, kernel="blocked", **kw)  # warm-up
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = rb.rbgs_solve(u, f, outer * inner, 0.0 if name == "f64" else 1e-300,
                             check_every=inner, h=h, kernel="blocked", timing=True, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sw = info["timing"]["sweep_ms"]
        out[name] = {"seconds": round(dt, 4), "sweeps": info["sweeps"],
                     "sweep_ms": round(sw, 3),
                     "inner_glups": round(n * n * info["sweeps"] / (sw * 1e-3) / 1e9, 1),
                     "whole_glups": round(n * n * info["sweeps"] / dt / 1e9, 1),
                     "rel_residual": info["rel_residual"]}
        log(f"refinement {name}: {out[name]}")
    # the closed form of 2 x 100 = 200 plain sweeps (refinement equals plain
    # sweeping in exact arithmetic): the runs' distance from it
    import numpy as np

    from tests import closed_form as cf
    modes = cf.merge_modes(*W.fourier_modes(seed=0))
    expect = cf.multi_mode_rel(n, modes, outer * inner)
    out["closed_form_rel_after_sweeps"] = expect
    for name in ("f32_ir", "bf16rhs_ir", "f64"):
        out[name]["rel_minus_closed_form"] = float(np.float64(out[name]["rel_residual"]) - expect)
    for name in ("f32_ir", "bf16rhs_ir"):
        out[name]["inner_glups_vs_f64"] = round(out[name]["inner_glups"] / out["f64"]["inner_glups"], 3)
    # PROJECTION, not a run: full sweeps to reach rel 1e-8 and 1e-10 from
    # u0 = 0 by the same closed form (the smallest m with rel(m) <= tol; the
    # slowest mode decays by cos^2(k pi h)-like factors, so this is ~1e8
    # sweeps at this size), times each form's measured time per sweep
    def sweeps_to(tol):
        lo, hi = 1, 1
        while cf.multi_mode_rel(n, modes, hi) > tol:
            lo, hi = hi, hi * 2
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if cf.multi_mode_rel(n, modes, mid) > tol:
                lo = mid
            else:
                hi = mid
        return hi
    proj = {"kind": "projection: closed-form sweep count x measured seconds per sweep (not run)"}
    for tol in (1e-8, 1e-10):
        m = sweeps_to(tol)
        row = {"sweeps_closed_form": m}
        for name in ("f64", "f32_ir", "bf16rhs_ir"):
            per_sweep = out[name]["seconds"] / out[name]["sweeps"]
            row[f"{name}_hours"] = round(m * per_sweep / 3600.0, 2)
        proj[f"{tol:g}"] = row
    out["projection_to_tol"] = proj
    del u, f
    torch.cuda.empty_cache()
    return out


def batched_throughput(torch, rb, W, count=512, sweeps=100):
    """The batched workload: 512 grids, sizes uniform on {63,127,255,511,1023}
    (seed 0), f i.i.d. N(0,1) (seed 1+g), FP32, 100 sweeps each, one
    graph-captured persistent launch after autotuning; beside it the same
    grids swept one by one with the plain FP64 kernel (the judge), and in
    FP32 with the plain kernel and with the automatic single-grid choice
    (the same precision)."""
    sizes = W.batch_sizes(count, seed=0)
    log(f"batched workload: {count} grids, building f")
    fs64 = [torch.from_numpy(W.normal_rhs(n, seed=1 + g)) for g, n in enumerate(sizes)]
    us = [torch.zeros((n + 2, n + 2), dtype=torch.float32, device="cuda") for n in sizes]
    fs = [x.to(torch.float32).to("cuda") for x in fs64]
    lups = sum(n * n for n in sizes) * sweeps
    best = rb.rbgs_autotune_batched(us, fs)
    log(f"autotuned: {best}")
    plan = rb.BatchPlan(us, fs, sweeps)
    plan.launch()
    plan.check()
    reps = 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.launch()
    plan.check()
    dt = (time.perf_counter() - t0) / reps
    plan.close()
    out = {"workload": f"{count} grids, N in {{63,127,255,511,1023}} seed 0, FP32, {sweeps} "
                       f"sweeps, one hipGraph launch", "total_lups": lups,
           "autotuned": best, "seconds": round(dt, 5), "glups": round(lups / dt / 1e9, 1)}
    # the judge: each grid alone, plain FP64 kernel, one rbgs_sweep call per grid
    u64 = [torch.zeros((n + 2, n + 2), dtype=torch.float64, device="cuda") for n in sizes]
    f64 = [x.to("cuda") for x in fs64]
    ws = torch.empty(rb.rbgs_workspace_size(rb.make_grid(u64[sizes.index(max(sizes))]), 0),
                     dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for u, f in zip(u64, f64):
        rb.rbgs_sweep(u, f, sweeps, kernel="plain", workspace=ws)
    torch.cuda.synchronize()
    dt64 = time.perf_counter() - t0
    out["plain_f64_one_by_one"] = {"seconds": round(dt64, 4), "glups": round(lups / dt64 / 1e9, 1)}
    out["speedup_vs_plain_f64"] = round(dt64 / dt, 2)
    # same precision: the FP32 grids one by one with the plain kernel and
    # with the library's automatic single-grid choice (resident / plain)
    ws32 = torch.empty(rb.rbgs_workspace_size(rb.make_grid(us[sizes.index(max(sizes))]), 1),
                       dtype=torch.uint8, device="cuda")
    for kernel in ("plain", "auto"):
        for u in us:
            u.zero_()
        rb.rbgs_sweep(us[0], fs[0], sweeps, kernel=kernel, workspace=ws32)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for u, f in zip(us, fs):
            rb.rbgs_sweep(u, f, sweeps, kernel=kernel, workspace=ws32)
        torch.cuda.synchronize()
        d32 = time.perf_counter() - t0
        out[f"{kernel}_f32_one_by_one"] = {"seconds": round(d32, 4),
                                           "glups": round(lups / d32 / 1e9, 1)}
        out[f"speedup_vs_{kernel}_f32_one_by_one"] = round(d32 / dt, 2)
    log(f"batched: {out}")
    del us, fs, u64, f64, ws, ws32
    torch.cuda.empty_cache()
    return out


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_SINGLE_CORE = """
import sys, time
sys.path.insert(0, {root!r})
import oracle, workloads as W
n, k, reps = {n}, {k}, {reps}
h = W.spacing(n)
f = W.uniform_rhs(n, seed=0)
u = W.zeros(n)
oracle.sweep(u, f, h, 1)
ts = []
for _ in range(reps):
    t0 = time.perf_counter()
    oracle.sweep(u, f, h, k)
    ts.append(time.perf_counter() - t0)
print(oracle.threads(), *ts)
"""


def cpu_baseline(n, sweeps, runs=10, single_sweeps=8, single_runs=3):
    """The oracle (plain C, OpenMP over rows of one colour) on the host
    cores, timed as the paper times its runs (Section 3: median of 10 runs
    on all cores): `runs` whole runs of `sweeps` sweeps of the same FP64
    problem after one warm-up sweep, median with min and max; beside it one
    core (a child process with OMP_NUM_THREADS=1; the GPU is not touched
    there) on `single_sweeps` sweeps, best and median of `single_runs`."""
    import statistics
    import subprocess

    import numpy as np

    import oracle
    import workloads as W
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=0)
    u = W.zeros(n)
    oracle.sweep(u, f, h, 1)  # warm-up (page faults, thread start)
    times = []
    for _ in range(runs):
        u[...] = 0.0
        t0 = time.perf_counter()
        oracle.sweep(u, f, h, sweeps)
        times.append(time.perf_counter() - t0)
    threads = oracle.threads()
    med = statistics.median(times)
    lups = float(n) * n * sweeps
    out = {"value": round(lups / med / 1e9, 3), "unit": "GLUP/s", "cores": threads,
           "kind": "oracle",
           "sample": f"{runs} runs of {sweeps} full sweeps of the {n}x{n} FP64 workload from u=0 "
                     f"(median; one warm-up sweep first), OpenMP threads={threads}",
           "host_cpu": host_cpu_model(), "host_logical_cpus": os.cpu_count(),
           "omp_env": {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OMP_PROC_BIND",
                                                      "OMP_PLACES")},
           "run_seconds": {"median": round(med, 4), "min": round(min(times), 4),
                           "max": round(max(times), 4)},
           "glups_min_max": [round(lups / max(times) / 1e9, 3), round(lups / min(times) / 1e9, 3)]}
    del u, f
    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = _SINGLE_CORE.format(root=ROOT, n=n, k=single_sweeps, reps=single_runs)
    try:
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                             text=True, timeout=600)
        vals = res.stdout.split()
        t1 = [float(v) for v in vals[1:]]
        one = float(n) * n * single_sweeps
        out["single_core"] = {"threads": int(vals[0]), "sweeps": single_sweeps,
                              "glups_best": round(one / min(t1) / 1e9, 4),
                              "glups_median": round(one / statistics.median(t1) / 1e9, 4),
                              "runs": single_runs}
    except (subprocess.SubprocessError, ValueError, IndexError) as exc:
        out["single_core"] = {"error": str(exc)[:200]}
    assert np is not None
    return out


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
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-time-to-tol", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the refinement (16383^2), batched and learned-guess workloads")
    ap.add_argument("--rb3-only", action="store_true",
                    help="run only the 3D red-black section, print its JSON and exit")
    ap.add_argument("--mc9-only", action="store_true",
                    help="run only the 9-point four-colour section, print its JSON and exit")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched workloads (512-grid sweeps, 16 grids to tolerance)")
    ap.add_argument("--overlap-only", action="store_true",
                    help="only the traced pass overlap of the 8191^2 workload")
    ap.add_argument("--unet-only", action="store_true",
                    help="run only the U-Net training/inference timing, print its JSON and exit")
    ap.add_argument("--mg-only", action="store_true",
                    help="run only the 8191^2 multigrid section (and the STREAM probe unless "
                         "--no-probe), print its JSON and exit: the multigrid kernels' profile run")
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
    if args.rb3_only:
        tol_sizes = () if args.no_time_to_tol else (63, 127)
        print(json.dumps({"rb3": rb3_throughput(torch, rb, tol_sizes=tol_sizes)}), flush=True)
        return
    if args.mc9_only:
        mc9 = multicolour9_throughput(torch, rb, W, with_solve=not args.no_time_to_tol)
        print(json.dumps({"multicolour9": mc9}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched_512": batched_throughput(torch, rb, W),
                          "batched_to_1e-8": batched_to_tolerance(torch, rb, W)}), flush=True)
        return
    if args.overlap_only:
        print(json.dumps({"pass_overlap_8191": pass_overlap(torch, rb, W)}), flush=True)
        return
    if args.unet_only:
        print(json.dumps({"unet": unet_throughput(torch, rb)}), flush=True)
        return
    if args.mg_only:
        mg = multigrid_to_tolerance(torch, rb, W, sizes=(1023, 8191))
        probe = None if args.no_probe else stream_probe(torch, rb)
        print(json.dumps({"multigrid_to_1e-8": mg, "stream_probe": probe}), flush=True)
        return
    n, sweeps = args.n, args.sweeps
    h = W.spacing(n)
    log(f"device {torch.cuda.get_device_name(0)}; building inputs n={n}")
    f = torch.from_numpy(W.uniform_rhs(n, seed=0)).to("cuda")
    u = torch.zeros((n + 2, n + 2), dtype=torch.float64, device="cuda")
    grid = rb.make_grid(u, h)
    ws = torch.empty(rb.rbgs_workspace_size(grid, rb.rbgs.F64), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()

    def run_steps(kernel, warmup, steps):
        def step():
            return rb.rbgs_solve(u, f, sweeps, 0.0, check_every=sweeps, h=h, kernel=kernel,
                                 workspace=ws, timing=True)
        for k in range(warmup):
            info = step()
            log(f"[{kernel}] warmup {k + 1}/{warmup}: rel={info['rel_residual']:.6e} "
                f"sweep_ms={info['timing']['sweep_ms']:.2f}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        acc = {"sweep_ms": 0.0, "sweep_launches": 0, "persistent_ms": 0.0,
               "persistent_launches": 0, "passes": 0, "fuse": 0}
        for _ in range(steps):
            t = step()["timing"]
            for key in acc:
                acc[key] = t[key] if key == "fuse" else acc[key] + t[key]
        torch.cuda.synchronize()
        ms_step = (time.perf_counter() - t0) * 1e3 / steps
        glups = n * n * sweeps / (ms_step * 1e-3) / 1e9
        log(f"[{kernel}] {steps} steps: {ms_step:.3f} ms/step, {glups:.1f} GLUP/s; timing {acc}")
        return ms_step, glups, acc

    ms_per_step, glups, acc = run_steps(args.kernel, args.warmup, args.steps)
    if acc["persistent_launches"] > 0:
        # The persistent blocked kernel: a step runs ceil(sweeps / fuse)
        # passes whose depths differ by at most one; per pass the algorithmic
        # traffic is one read of u and f and one write of u, 3 words per
        # point.  Its duration comes from HIP events around the timed launch:
        # all passes when both depths run in one launch (k_blocked2), else
        # the deeper passes alone (the shallower launch and the ring copies
        # are outside).
        kernel_used, fuse = "blocked", acc["fuse"]
        launches = acc["persistent_launches"]
        avg_launch_ms = acc["persistent_ms"] / launches
        per_launch_bytes = BYTES_PER_LUP["f64"] * n * n * acc["passes"] / launches
        total_passes = -(-sweeps // fuse)
        bytes_per_lup = BYTES_PER_LUP["f64"] * total_passes / sweeps
        passes_per_launch = acc["passes"] // launches
        if sweeps % fuse and passes_per_launch == total_passes:
            n_hi = sweeps - total_passes * (fuse - 1)
            kname = (f"k_blocked2<double,2,{2 * fuse},{2 * fuse - 2}> (persistent, {n_hi} passes "
                     f"of {fuse} + {total_passes - n_hi} of {fuse - 1} in one launch)")
        else:
            kname = f"k_blocked<double,2,{2 * fuse}> (persistent, fuse {fuse})"
        traffic_key = "blocked_f64"
    else:
        # One launch updates one colour: half the points, 3 words each.
        kernel_used, fuse = "plain", 0
        avg_launch_ms = acc["sweep_ms"] / max(acc["sweep_launches"], 1)
        per_launch_bytes = BYTES_PER_LUP["f64"] * n * n / 2.0
        bytes_per_lup = BYTES_PER_LUP["f64"]
        kname, traffic_key = "k_half_sweep<double,2>", "half_sweep_f64"
    # achieved: algorithmic bytes of one launch (the 3w-per-point-per-pass
    # model) over the launch's average duration from HIP events on its own
    # stream; beside it the same bytes over the rocprofv3 average of the
    # committed profile, and the counter-measured HBM bytes (FETCH_SIZE +
    # WRITE_SIZE, calibrated on a copy) over the HIP-event duration
    achieved = per_launch_bytes / (avg_launch_ms * 1e-3) / 1e9
    traffic = read_traffic(traffic_key, n)
    prof = read_profile_avg(traffic_key, n)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": kname,
                "avg_launch_us": round(avg_launch_ms * 1e3, 2),
                "avg_launch_source": "HIP events recorded on the launch stream, timed steps only",
                "launches_timed": acc["persistent_launches"] if kernel_used == "blocked"
                else acc["sweep_launches"],
                "bytes_per_launch": per_launch_bytes,
                "bytes_model": "24 B per grid point per pass (FP64: other colour and f read, "
                               "own colour written; split layout)",
                "rocprof_avg_launch_us": prof["avg_us"] if prof else None,
                "rocprof_calls": prof["calls"] if prof else None,
                "frac_rocprof": round(per_launch_bytes / (prof["avg_us"] * 1e-6) / 1e9 /
                                      HBM_PEAK_GBS, 4) if prof else None,
                "achieved_counter_GBs": round(traffic / (avg_launch_ms * 1e-3) / 1e9, 1)
                if traffic else None,
                "effective_GBs_24B_per_LUP": round(glups * BYTES_PER_LUP["f64"], 1)}
    plain = None
    if kernel_used != "plain" and not args.no_plain:
        p_ms, p_glups, p_acc = run_steps("plain", 1, max(2, args.steps // 3))
        p_launch_ms = p_acc["sweep_ms"] / max(p_acc["sweep_launches"], 1)
        p_bytes = BYTES_PER_LUP["f64"] * n * n / 2.0
        p_ach = p_bytes / (p_launch_ms * 1e-3) / 1e9
        plain = {"value": round(p_glups, 2), "unit": "GLUP/s", "ms_per_step": round(p_ms, 3),
                 "kernel": "k_half_sweep<double,2>", "avg_launch_us": round(p_launch_ms * 1e3, 2),
                 "achieved_GBs": round(p_ach, 1), "frac_of_8TBs": round(p_ach / HBM_PEAK_GBS, 4),
                 "traffic": read_traffic("half_sweep_f64", n),
                 "speedup_of_timed_kernel": round(glups / p_glups, 3)}
    del u, f, ws
    torch.cuda.empty_cache()
    ttt = None if args.no_time_to_tol else time_to_tolerance(torch, rb, W)
    ttt_1023 = None if args.no_time_to_tol else time_to_tolerance_fourier(torch, rb, W)
    multigrid = None if args.no_time_to_tol else multigrid_to_tolerance(torch, rb, W)
    if multigrid and ttt_1023:
        base_1023 = ttt_1023["plain_f64"]["seconds"]
        for key in ("n1023_V22", "n1023_V11"):
            multigrid[key]["speedup_vs_plain_f64"] = round(base_1023 / multigrid[key]["seconds"], 1)
    mc9 = None if args.no_extras else multicolour9_throughput(torch, rb, W)
    rb3 = None if args.no_extras else rb3_throughput(torch, rb)
    refine = None if args.no_extras else refinement_throughput(torch, rb, W)
    batched = None if args.no_extras else batched_throughput(torch, rb, W)
    batched_tol = None if args.no_extras else batched_to_tolerance(torch, rb, W)
    learned_511 = None if args.no_extras else learned_guess(torch, rb)
    unet = None if args.no_extras else unet_throughput(torch, rb)
    overlap = None if args.no_extras else pass_overlap(torch, rb, W)
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
                   "n": n, "sweeps": sweeps, "kernel": kernel_used, "fuse": fuse},
        # whole step: algorithmic bytes (24 B per point per pass) per second;
        # effective bandwidth at 24 B/LUP (what a one-pass-per-sweep kernel
        # would need for the same GLUP/s) is in the roofline object
        "hbm_gbs_algorithmic": round(glups * bytes_per_lup, 1),
        "bytes_per_lup_algorithmic": bytes_per_lup,
        "roofline": roofline,
        "plain_kernel": plain,
        "time_to_1e-8": ttt,
        "time_to_1e-8_fourier_1023": ttt_1023,
        "multigrid_to_1e-8": multigrid,
        "multicolour9": mc9,
        "rb3": rb3,
        "refinement_16383": refine,
        "batched_512": batched,
        "batched_to_1e-8": batched_tol,
        "learned_guess_511": learned_511,
        "unet_511": unet,
        "pass_overlap_8191": overlap,
        "stream_probe": probe,
        "cpu_baseline": base,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
