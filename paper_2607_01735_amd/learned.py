"""Learned initial guess: data generation, training and held-out evaluation.

Every numerical step runs in librbgs.so: the (f, u*) training pairs come
from the library's batched persistent Gauss-Seidel in FP32 by nested
iteration (coarse levels solved first, then interpolated by the library's
grid transfers), the network is trained by the library's U-Net kernels,
and the evaluation compares the library's FP64 solve to a relative residual
from u = 0 (the judge) with the same solve started from the network's guess
(rbgs_solve_learned).  This module only orchestrates and moves tensors.

Inputs are Gaussian random fields (workloads.grf_rhs): squared-exponential
covariance through a sine series, length scale uniform on [0.02, 0.3],
normalised to unit RMS; training seeds 0, 1, ..., test seeds 10^6 + i.

Usage (from the repository root, on a GPU):
  python -m paper_2607_01735_amd.learned --train 2048 --epochs 8 --out unet.npy
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TEST_SEED0 = 10 ** 6

# Parameters trained by this module for 511 x 511 GRF problems (coarsening
# factor 4); weights/unet_grf511_f4.json records how.
PRETRAINED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                          "unet_grf511_f4.npy")


def pretrained_net(rb, batch=1, path=PRETRAINED):
    """The library's U-Net for 511 x 511 grids with the shipped parameters."""
    net = rb.UNet(511, batch, factor=4)
    net.set_params(np.load(path))
    return net

# (name, input channels, output channels) of the library's conv layers, in
# its parameter order; the 1x1 head (16 -> 1) follows them.
LAYERS = (("enc0.0", 1, 16), ("enc0.1", 16, 16), ("enc1.0", 16, 32), ("enc1.1", 32, 32),
          ("enc2.0", 32, 64), ("enc2.1", 64, 64), ("enc3.0", 64, 128), ("enc3.1", 128, 128),
          ("dec2.0", 192, 64), ("dec2.1", 64, 64), ("dec1.0", 96, 32), ("dec1.1", 32, 32),
          ("dec0.0", 48, 16), ("dec0.1", 16, 16))


def initial_params(seed=0):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, FP32 vector in
    the library's parameter order."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, cin, cout in LAYERS:
        parts.append(rng.standard_normal(cout * cin * 9) * math.sqrt(2.0 / (cin * 9)))
        parts.append(np.zeros(cout))
    parts.append(rng.standard_normal(16) * math.sqrt(1.0 / 16))
    parts.append(np.zeros(1))
    return np.concatenate(parts).astype(np.float32)


def log(msg):
    print(f"[learned] {msg}", file=sys.stderr, flush=True)


def fields(n, seeds):
    """Stack of GRF right-hand sides, natural layout (B, n+2, n+2), FP64."""
    import workloads as W
    return np.stack([W.grf_rhs(n, seed=int(s))[0] for s in seeds])


def fields_on_device(torch, n, seeds, chunk=256):
    """The same stack built chunk by chunk straight into device memory."""
    seeds = list(seeds)
    out = torch.empty((len(seeds), n + 2, n + 2), dtype=torch.float64, device="cuda")
    for s in range(0, len(seeds), chunk):
        part = fields(n, seeds[s:s + chunk])
        out[s:s + part.shape[0]].copy_(torch.from_numpy(part))
    return out


# Full sweeps per level of the nested iteration, coarsest level first.  From
# u = 0 on the coarsest grid (N = 63 for N = 511) each finer level starts from
# the bilinear interpolation of the coarser solution; the smooth error that
# plain Gauss-Seidel removes slowly is then already small, and the sweeps on
# each level remove what interpolation adds.  On 511^2 GRF fields this leaves
# a relative error of about 1e-4 against the exact discrete solution, where
# 20000 sweeps from zero on 511^2 alone leave 25-45 %.
LEVEL_SWEEPS = (8000, 3000, 3000, 3000)


def level_sizes(n, levels):
    sizes = [n]
    for _ in range(levels - 1):
        if sizes[-1] % 2 == 0 or sizes[-1] < 3:
            raise ValueError(f"n = {n} cannot be halved {levels - 1} times (needs 2^k - 1)")
        sizes.append((sizes[-1] - 1) // 2)
    return sizes


def nested_targets(rb, torch, f, level_sweeps=LEVEL_SWEEPS, chunk=512, tune=True):
    """u* for every f (device FP64 (B, n+2, n+2)) by nested iteration in FP32:
    restrict f to each coarser level (full weighting), sweep the coarsest
    level from u = 0, then prolong (bilinear) and sweep each finer level, all
    grids of a chunk in one persistent batched launch per level.  Widened to
    FP64 at the end."""
    count, n = f.shape[0], f.shape[1] - 2
    sizes = level_sizes(n, len(level_sweeps))
    out = torch.empty_like(f)
    tuned = set()
    for s in range(0, count, chunk):
        fc = f[s:s + chunk].to(torch.float32).contiguous()
        b = fc.shape[0]
        rhs = [fc]
        for m in sizes[1:]:
            c = torch.zeros((b, m + 2, m + 2), dtype=torch.float32, device=f.device)
            rb.rbgs_restrict(rhs[-1], c)
            rhs.append(c)
        u = None
        for lvl, sweeps in zip(range(len(sizes) - 1, -1, -1), level_sweeps):
            m = sizes[lvl]
            nxt = torch.zeros((b, m + 2, m + 2), dtype=torch.float32, device=f.device)
            if u is not None:
                rb.rbgs_prolong(u, nxt)
            u = nxt
            us = [u[i] for i in range(b)]
            fs = [rhs[lvl][i] for i in range(b)]
            if tune and (m, b) not in tuned:
                # the tuner sweeps its own copies; u and f are only read
                log(f"autotune {b} x {m}^2: {rb.rbgs_autotune_batched(us, fs)}")
                tuned.add((m, b))
            with rb.BatchPlan(us, fs, sweeps) as plan:
                plan.launch()
                plan.check()
        out[s:s + b] = u.to(torch.float64)
        log(f"targets {s + b}/{count}")
    return out


def target_residuals(rb, f, u, count=8):
    rels = []
    for i in range(min(count, f.shape[0])):
        rels.append(rb.rbgs_residual(u[i], f[i])[1])
    return rels


def train(net, torch, f, u, epochs, batch, lr0, seed=0, lr_min_frac=0.05):
    """Adam with cosine-decayed learning rate over shuffled minibatches."""
    rng = np.random.default_rng(seed)
    count = f.shape[0]
    steps_per_epoch = count // batch
    total = epochs * steps_per_epoch
    step = 0
    history = []
    for ep in range(epochs):
        order = rng.permutation(count)
        losses = []
        for k in range(steps_per_epoch):
            idx = torch.as_tensor(order[k * batch:(k + 1) * batch], device=f.device)
            lr = lr0 * (lr_min_frac + (1 - lr_min_frac) * 0.5 * (1 + math.cos(math.pi * step / total)))
            losses.append(net.train_step(f[idx].contiguous(), u[idx].contiguous(), lr))
            step += 1
            if step % 1000 == 0:
                log(f"step {step}/{total}: loss {np.mean(losses[-1000:]):.4e}")
        history.append(float(np.mean(losses)))
        log(f"epoch {ep + 1}/{epochs}: loss {history[-1]:.4e} lr {lr:.2e}")
    return history


def _timed(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def evaluate(rb, torch, net, n, seeds, tol, compare_after=(0,), kernel="auto",
             max_sweeps=2_000_000, check_every=2000):
    """Sweeps and wall time (network inference included) to rel <= tol: the
    FP64 solve from u = 0 (the judge) against the same solve through
    rbgs_solve_learned for each comparison depth in `compare_after`."""
    rows = []
    f_all = fields_on_device(torch, n, seeds)
    for i, s in enumerate(seeds):
        f = f_all[i]
        u = torch.zeros_like(f)
        base, t_base = _timed(torch, lambda: rb.rbgs_solve(u, f, max_sweeps, tol,
                                                           check_every=check_every, kernel=kernel))
        row = {"seed": int(s), "zero_start": {"sweeps": base["sweeps"], "seconds": round(t_base, 4),
                                              "rel": base["rel_residual"]}}
        for ca in compare_after:
            u = torch.zeros_like(f)
            got, t_nn = _timed(torch, lambda: net.solve_learned(
                u, f, max_sweeps, tol, check_every=check_every, kernel=kernel, compare_after=ca))
            row[f"learned_k{ca}"] = {"sweeps": got["sweeps"], "seconds": round(t_nn, 4),
                                     "rel": got["rel_residual"], "used_guess": got["used_guess"],
                                     "rel_start": got["rel_start"]}
        rows.append(row)
        log(f"test seed {s}: {row}")
    return rows


def summarise(rows, compare_after):
    """Totals over the test seeds: sweep and time ratios learned / zero start."""
    out = {}
    zs = sum(r["zero_start"]["sweeps"] for r in rows)
    zt = sum(r["zero_start"]["seconds"] for r in rows)
    for ca in compare_after:
        key = f"learned_k{ca}"
        out[key] = {"sweep_ratio": round(sum(r[key]["sweeps"] for r in rows) / zs, 4),
                    "time_ratio": round(sum(r[key]["seconds"] for r in rows) / zt, 4),
                    "guess_used": sum(bool(r[key]["used_guess"]) for r in rows),
                    "of": len(rows)}
    return out


def guess_quality(rb, torch, net, n, seeds, level_sweeps):
    """Relative error of the network's guess against the solver's u* on
    held-out fields (the same target definition as training)."""
    f = torch.from_numpy(fields(n, seeds)).to("cuda")
    us = nested_targets(rb, torch, f, level_sweeps, chunk=len(seeds))
    g = torch.zeros_like(f)
    net.forward(f, g)
    err = [(torch.linalg.norm(g[i] - us[i]) / torch.linalg.norm(us[i])).item()
           for i in range(len(seeds))]
    return err


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=511)
    ap.add_argument("--train", type=int, default=2048)
    ap.add_argument("--level-sweeps", default=",".join(map(str, LEVEL_SWEEPS)),
                    help="FP32 sweeps per nested-iteration level, coarsest first")
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--factor", type=int, default=4, help="coarsening factor between levels")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--test", type=int, default=4, help="held-out fields for the guess error")
    ap.add_argument("--eval", type=int, default=2, help="held-out fields solved to --tol")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--compare-after", type=int, default=500,
                    help="sweeps given to both starts before the residual comparison")
    ap.add_argument("--params", default=None, help="start from these parameters (.npy)")
    ap.add_argument("--out", default=None, help="write the trained parameters here (.npy)")
    ap.add_argument("--summary", default=None, help="write a JSON summary here")
    ap.add_argument("--skip-eval", action="store_true")
    args = ap.parse_args()

    import torch

    import paper_2607_01735_amd as rb

    n = args.n
    net = rb.UNet(n, args.batch, factor=args.factor)
    if args.params:
        net.set_params(np.load(args.params))
    else:
        vec = initial_params(args.init_seed)
        if vec.size != rb.rbgs_unet_param_count():
            raise RuntimeError("layer table out of step with the library")
        net.set_params(vec)
    level_sweeps = tuple(int(x) for x in args.level_sweeps.split(","))
    summary = {"n": n, "train": args.train, "level_sweeps": level_sweeps, "epochs": args.epochs,
               "batch": args.batch, "lr": args.lr, "factor": args.factor}
    if args.train > 0:
        t0 = time.perf_counter()
        f = fields_on_device(torch, n, range(args.train))
        summary["field_seconds"] = round(time.perf_counter() - t0, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u = nested_targets(rb, torch, f, level_sweeps)
        torch.cuda.synchronize()
        summary["target_seconds"] = round(time.perf_counter() - t0, 2)
        summary["target_rel_residual"] = target_residuals(rb, f, u)
        log(f"targets: {summary['target_seconds']} s, residuals {summary['target_rel_residual'][:4]}")
        t0 = time.perf_counter()
        summary["loss_history"] = train(net, torch, f, u, args.epochs, args.batch, args.lr)
        torch.cuda.synchronize()
        summary["train_seconds"] = round(time.perf_counter() - t0, 2)
        del f, u
        torch.cuda.empty_cache()
        if args.out:
            np.save(args.out, net.get_params())
    test_seeds = [TEST_SEED0 + i for i in range(args.test)]
    summary["guess_rel_error"] = guess_quality(rb, torch, net, n, test_seeds, level_sweeps)
    log(f"held-out guess error vs u*: {summary['guess_rel_error']}")
    if not args.skip_eval:
        depths = sorted({0, args.compare_after})
        rows = evaluate(rb, torch, net, n, test_seeds[:args.eval], args.tol, depths)
        summary["eval"] = rows
        summary["eval_summary"] = summarise(rows, depths)
        log(f"evaluation: {summary['eval_summary']}")
    out = json.dumps(summary)
    if args.summary:
        with open(args.summary, "w") as fh:
            fh.write(out + "\n")
    print(out, flush=True)


if __name__ == "__main__":
    main()
