"""GPU U-Net kernels against the FP64 reference network (oracle/unet_ref.py).

The GPU path keeps conv weights and activations in bfloat16 and accumulates
in FP32 (FP32 masters, biases and head).  The reference runs in FP64 on the
same stored values: conv weights rounded to bfloat16, and every activation
and activation gradient rounded to bfloat16 where the kernels store one
(unet_ref's rnd).  What remains is FP32 against FP64 accumulation; the
tolerances (FWD_TOL, GRAD_TOL, LOSS_TOL below) are the measured errors with
a margin.  Gradients are reproducible bit for bit (fixed-order reductions);
Adam is checked over five steps; the learned solve's choice rule is checked
exactly: the final iterate is the oracle's solve from the chosen start, bit
for bit.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import unet_ref as U

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2607_01735_amd as rb  # noqa: E402

DEV = torch.device("cuda:0")
# Measured on MI355X against the reference that rounds to bfloat16 where the
# kernels store bfloat16 (tests print the measured values); the remaining
# difference is FP32 against FP64 accumulation, which moves an occasional
# stored value across a bfloat16 rounding boundary.
FWD_TOL = {2: 2e-3, 4: 1e-2}   # by coarsening factor
GRAD_TOL = 5e-3
LOSS_TOL = 1e-4
N = 127     # the factor-4 network (levels 127, 31, 7, 1)
FACTOR = 4
CONFIGS = [(2, 63), (4, 127)]  # (coarsening factor, N)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def flatten(p):
    parts = []
    for name in U.param_names():
        parts += [p[name + ".w"].ravel(), p[name + ".b"].ravel()]
    return np.concatenate(parts)


def unflatten(vec, like):
    out, off = {}, 0
    for name in U.param_names():
        for suffix in (".w", ".b"):
            k = name + suffix
            size = like[k].size
            out[k] = vec[off:off + size].reshape(like[k].shape).astype(np.float64)
            off += size
    assert off == vec.size
    return out


def bf16_round(a):
    return torch.from_numpy(np.asarray(a, np.float64)).to(torch.bfloat16).to(torch.float64).numpy()


def make_params(seed=1):
    p = U.init_params(seed=seed)
    rng = np.random.default_rng(seed + 100)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.05
    # the library stores FP32 masters: start from FP32-representable values
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def batch_fields(seeds, n=N):
    fs = [W.grf_rhs(n, seed=s)[0] for s in seeds]
    return np.stack(fs)


def round_weights(p):
    """The kernels' operands: 3x3 conv weights in bfloat16; biases and the
    1x1 head stay in FP32 (their masters)."""
    return {k: (bf16_round(v) if k.endswith(".w") and not k.startswith("head") else v)
            for k, v in p.items()}


def ref_forward(p, f_nat, factor=FACTOR):
    """Reference output u0 (interior), FP64 arithmetic on the kernels'
    stored values: bfloat16 conv weights, the input f/rms (rms in FP32)
    rounded to bfloat16, every stored activation rounded to bfloat16."""
    pr = round_weights(p)
    n = f_nat.shape[0] - 2
    fi = f_nat[1:n + 1, 1:n + 1]
    rms = float(np.float32(np.sqrt(np.mean(fi * fi))))
    x0 = bf16_round((fi / rms).astype(np.float32))
    y, cache = U.forward(pr, x0, factor=factor, rnd=bf16_round)
    return y * rms, y, cache, pr, rms


@pytest.mark.parametrize("factor,n", CONFIGS)
def test_forward_matches_reference(factor, n):
    say(f"unet forward n={n} factor={factor} batch=2")
    p = make_params()
    net = rb.UNet(n, 2, factor=factor)
    net.set_params(flatten(p).astype(np.float32))
    assert np.array_equal(net.get_params(), flatten(p).astype(np.float32))
    f = batch_fields([0, 1], n)
    ft = torch.from_numpy(f).to(DEV)
    u0 = torch.zeros_like(ft)
    net.forward(ft, u0)
    got = u0.cpu().numpy()
    for b in range(2):
        ref, *_ = ref_forward(p, f[b], factor)
        g = got[b, 1:n + 1, 1:n + 1]
        err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
        say(f"forward n={n} F={factor} sample {b}: relative L2 error {err:.3e}")
        assert err < FWD_TOL[factor], f"sample {b}: relative error {err}"
        assert not np.any(got[b, 0]) and not np.any(got[b, :, 0])  # ring untouched


@pytest.mark.parametrize("factor,n", CONFIGS)
def test_gradients_match_reference(factor, n):
    say(f"unet gradients n={n} factor={factor} batch=2")
    p = make_params(seed=2)
    net = rb.UNet(n, 2, factor=factor)
    net.set_params(flatten(p).astype(np.float32))
    f = batch_fields([5, 6], n)
    target = np.zeros_like(f)
    rng = np.random.default_rng(7)
    target[:, 1:n + 1, 1:n + 1] = rng.standard_normal((2, n, n)) * 0.01
    loss = net.train_step(torch.from_numpy(f).to(DEV), torch.from_numpy(target).to(DEV), 0.0,
                          update=False)
    g_gpu = unflatten(net.get_grads().astype(np.float64), p)
    # reference: mean over the batch of per-sample mean squared errors
    g_ref = {k: np.zeros_like(v) for k, v in p.items()}
    loss_ref = 0.0
    for b in range(2):
        _, y, cache, pr, rms = ref_forward(p, f[b], factor)
        t = target[b, 1:n + 1, 1:n + 1] / rms
        lb, dy = U.mse_loss(y, t)
        loss_ref += lb / 2
        gb = U.backward(pr, cache, dy / 2, factor=factor, rnd=bf16_round)
        for k in g_ref:
            g_ref[k] += gb[k]
    say(f"loss {loss!r} reference {loss_ref!r}")
    assert loss == pytest.approx(loss_ref, rel=LOSS_TOL)
    worst = (0.0, "")
    for k in g_ref:
        a, r = g_gpu[k].ravel(), g_ref[k].ravel()
        if np.linalg.norm(r) < 1e-6 * max(1.0, np.abs(loss_ref)):
            continue
        rel = np.linalg.norm(a - r) / np.linalg.norm(r)
        worst = max(worst, (rel, k))
        assert rel < GRAD_TOL, f"{k}: relative L2 error {rel:.3e}"
    say(f"gradients n={n} F={factor}: worst tensor {worst[1]} relative L2 error {worst[0]:.3e}")


def test_gradients_are_reproducible():
    """The gradient reductions add partial sums in a fixed order (no
    floating-point atomics): two backward passes give the same bits."""
    say("unet gradient reproducibility")
    p = make_params(seed=8)
    net = rb.UNet(N, 2)
    net.set_params(flatten(p).astype(np.float32))
    f = torch.from_numpy(batch_fields([3, 4])).to(DEV)
    target = torch.zeros_like(f)
    l1 = net.train_step(f, target, 0.0, update=False)
    g1 = net.get_grads()
    l2 = net.train_step(f, target, 0.0, update=False)
    g2 = net.get_grads()
    assert l1 == l2
    assert np.array_equal(g1.view(np.uint32), g2.view(np.uint32))


def test_adam_matches_reference_over_steps():
    """Five Adam updates on the GPU against the reference Adam (FP64)
    applied to the same FP32 parameters with the GPU's gradients of each
    step: bias correction, both moments and the step count are exercised
    beyond the first step."""
    say("unet adam over 5 steps")
    p = make_params(seed=9)
    vec = flatten(p).astype(np.float32)
    net = rb.UNet(N, 2)
    net.set_params(vec)
    f = torch.from_numpy(batch_fields([13, 14])).to(DEV)
    u = np.zeros(tuple(f.shape))
    for b in range(2):
        u[b, 1:N + 1, 1:N + 1] = -W.grf_rhs(N, seed=13 + b)[0][1:N + 1, 1:N + 1] * 0.02
    ut = torch.from_numpy(u).to(DEV)
    lr = 2e-3
    ref = {"a": vec.astype(np.float64)}
    state = {}
    for t in range(1, 6):
        before = net.get_params()
        net.train_step(f, ut, lr, update=True)
        g = net.get_grads().astype(np.float64)
        after = net.get_params()
        ref = {"a": before.astype(np.float64)}
        U.adam_step(ref, {"a": g}, state, lr=lr)
        tol = 4 * np.spacing(np.abs(after)).astype(np.float64) + 2e-6 * lr
        err = np.abs(after.astype(np.float64) - ref["a"])
        say(f"adam step {t}: max |gpu - ref| {err.max():.3e}")
        assert np.all(err <= tol), f"step {t}: {int(np.sum(err > tol))} parameters off"
        assert not np.array_equal(after, before)


def test_adam_state_resumes_training_bit_for_bit():
    """Save parameters and Adam's state after three steps, restore both into a
    fresh network, and take two more steps on each: the same bits.  Without
    the Adam state (parameters only, a restarted Adam) the run differs."""
    say("unet adam save / resume")
    p = make_params(seed=15)
    vec = flatten(p).astype(np.float32)
    f = torch.from_numpy(batch_fields([21, 22])).to(DEV)
    u = np.zeros(tuple(f.shape))
    for b in range(2):
        u[b, 1:N + 1, 1:N + 1] = -W.grf_rhs(N, seed=21 + b)[0][1:N + 1, 1:N + 1] * 0.02
    ut = torch.from_numpy(u).to(DEV)
    lr = 1e-3
    a = rb.UNet(N, 2)
    a.set_params(vec)
    for _ in range(3):
        a.train_step(f, ut, lr, update=True)
    params = a.get_params()
    m, v, step = a.get_adam()
    assert step == 3 and np.any(m != 0) and np.all(v >= 0)
    b, c = rb.UNet(N, 2), rb.UNet(N, 2)
    b.set_params(params)
    b.set_adam(m, v, step)
    c.set_params(params)  # restarts Adam
    m0, v0, s0 = c.get_adam()
    assert s0 == 0 and not np.any(m0) and not np.any(v0)
    for net in (a, b, c):
        for _ in range(2):
            net.train_step(f, ut, lr, update=True)
    pa, pb, pc = a.get_params(), b.get_params(), c.get_params()
    assert np.array_equal(pa.view(np.uint32), pb.view(np.uint32))
    assert a.get_adam()[2] == b.get_adam()[2] == 5
    assert not np.array_equal(pa, pc)
    with pytest.raises(rb.RbgsError):
        b.set_adam(m, v, -1)


def test_adam_step_and_training_decreases_loss():
    say("unet adam + short training")
    p = make_params(seed=3)
    vec = flatten(p).astype(np.float32)
    net = rb.UNet(N, 2)
    net.set_params(vec)
    f = torch.from_numpy(batch_fields([11, 12])).to(DEV)
    fn = f.cpu().numpy()
    u = np.zeros_like(fn)
    for b in range(2):
        u[b, 1:N + 1, 1:N + 1] = -W.grf_rhs(N, seed=11 + b)[0][1:N + 1, 1:N + 1] * 0.02
    ut = torch.from_numpy(u).to(DEV)
    net.train_step(f, ut, 0.0, update=False)
    g = net.get_grads()
    lr = 1e-3
    net.set_params(vec)
    first = net.train_step(f, ut, lr, update=True)
    new = net.get_params()
    # first bias-corrected Adam step moves each weight by lr * g/(|g| + eps')
    step = vec - new
    big = np.abs(g) > 1e-4
    assert np.allclose(step[big], lr * np.sign(g[big]), rtol=1e-3, atol=1e-7)
    assert np.all(np.abs(step) <= lr * 1.001)
    losses = [first]
    for _ in range(40):
        losses.append(net.train_step(f, ut, lr, update=True))
    assert losses[-1] < 0.5 * losses[0], losses[::10]


def test_learned_solve_choice_rule(oracle):
    """Both branches of the rule: a zero start beats an untrained network's
    guess, and the guess beats a deliberately bad start; either way the
    result is the oracle's solve from the chosen start, bit for bit."""
    say("learned solve choice rule")
    p = make_params(seed=4)
    net = rb.UNet(N, 1)
    net.set_params(flatten(p).astype(np.float32))
    h = W.spacing(N)
    f = W.grf_rhs(N, seed=21)[0]
    ft = torch.from_numpy(f).to(DEV)
    guess = torch.zeros((1, N + 2, N + 2), dtype=torch.float64, device=DEV)
    net.forward(ft[None].contiguous(), guess)
    guess_np = guess[0].cpu().numpy()
    _, rel_guess = oracle.residual(guess_np, f, h)
    for start in (W.zeros(N), W.uniform_rhs(N, seed=3) * 1e3):
        _, rel_start = oracle.residual(start, f, h)
        ut = torch.from_numpy(start.copy()).to(DEV)
        info = net.solve_learned(ut, ft, 300, 1e-12, check_every=100, kernel="plain")
        use = rel_guess < rel_start
        assert info["used_guess"] == use
        ref = (guess_np if use else start).copy()
        oracle.sweep(ref, f, h, 300)
        assert np.array_equal(ut.cpu().numpy(), ref)
        assert info["sweeps"] == 300
    # comparing after 10 sweeps of both starts
    k = 10
    for start in (W.zeros(N), W.uniform_rhs(N, seed=3) * 1e3):
        a, b = start.copy(), guess_np.copy()
        oracle.sweep(a, f, h, k)
        oracle.sweep(b, f, h, k)
        use = oracle.residual(b, f, h)[1] < oracle.residual(a, f, h)[1]
        ut = torch.from_numpy(start.copy()).to(DEV)
        info = net.solve_learned(ut, ft, 300, 1e-12, check_every=100, kernel="plain",
                                 compare_after=k)
        # both starts were swept k times before the choice
        assert info["used_guess"] == use and info["sweeps"] == 300 + k
        ref = (guess_np if use else start).copy()
        oracle.sweep(ref, f, h, 300)
        assert np.array_equal(ut.cpu().numpy(), ref)
