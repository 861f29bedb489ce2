"""GPU parity: the HIP path through the C ABI against the oracle.

FP64 sweeps must equal the oracle bit for bit (same term order, no FMA);
FP32 sweeps must equal the oracle's FP32 emulation bit for bit; residual
norms agree within 1e-13 relative (the GPU reduces in a different, fixed
order).  Sizes span several workgroup tiles and ragged tails, odd and even
N, padded row pitches and nonzero Dirichlet rings.
"""
import sys

import numpy as np
import pytest

import workloads as W
from tests.sampling import sample_after_sweeps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2607_01735_amd as rb  # noqa: E402

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def gpu_sweep(u, f, h, nsweeps, **kw):
    ut, ft = dev(u), dev(f)
    rb.rbgs_sweep(ut, ft, nsweeps, h=h, **kw)
    return host(ut)


CASES = [  # (n, ld_extra, nsweeps, seed)
    (1, 0, 3, 0), (2, 0, 4, 1), (3, 1, 5, 2), (7, 0, 9, 3), (8, 3, 6, 4), (33, 0, 11, 5),
    (64, 5, 7, 6), (255, 0, 25, 7), (256, 0, 13, 8), (257, 9, 13, 9), (513, 0, 8, 10),
    (1000, 24, 6, 11), (1023, 0, 20, 12), (2049, 7, 4, 13),
]


@pytest.mark.parametrize("n,extra,nsweeps,seed", CASES)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_plain_sweep_bitwise(oracle, n, extra, nsweeps, seed, dtype):
    say(f"plain sweep n={n} ld=n+2+{extra} sweeps={nsweeps} seed={seed} {dtype.__name__}")
    h = W.spacing(n)
    ld = n + 2 + extra
    f = W.uniform_rhs(n, seed=seed, ld=ld).astype(dtype)
    u = W.random_ring(n, seed=seed + 100, ld=ld).astype(dtype)
    u[1:n + 1, 1:n + 1] = W.uniform_rhs(n, seed=seed + 200)[1:n + 1, 1:n + 1]
    f[:, n + 2:] = np.nan  # padding beyond the grid must never be read
    u[:, n + 2:] = 7.0
    # the ring of f is never read
    f[0, :] = f[-1, :] = f[:, 0] = f[:, n + 1] = np.nan
    got = gpu_sweep(u, f, h, nsweeps, kernel="plain")
    ref = u.copy()
    fo = np.nan_to_num(f, nan=0.0)
    oracle.sweep(ref, fo, h, nsweeps)
    ref[:, n + 2:] = 7.0
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), \
        f"max diff {np.nanmax(np.abs(got - ref))}"


def test_config0_closed_form_and_oracle(oracle):
    """255 x 255, h = 1/256, f = 2 pi^2 sin sin, 1000 sweeps, FP64."""
    from tests import closed_form as cf
    n, m = 255, 1000
    say(f"small-grid workload n={n} sweeps={m}")
    h = W.spacing(n)
    f = W.sine_rhs(n)
    got = gpu_sweep(W.zeros(n), f, h, m, kernel="plain")
    ref = W.zeros(n)
    oracle.sweep(ref, f, h, m)
    assert np.array_equal(got, ref)
    expect = cf.iterate(n, [(1, 1, 2 * np.pi ** 2)], m)
    assert np.max(np.abs(got - expect)) / np.max(np.abs(expect)) < 1e-12


@pytest.mark.parametrize("n", [1, 5, 64, 255, 1025])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_residual_matches_oracle(oracle, n, dtype):
    say(f"residual n={n} {dtype.__name__}")
    h = W.spacing(n)
    ld = n + 2 + (n % 3)
    f = W.uniform_rhs(n, seed=n, ld=ld).astype(dtype)
    u = W.random_ring(n, seed=n + 1, ld=ld)
    u[1:n + 1, 1:n + 1] = W.uniform_rhs(n, seed=n + 2)[1:n + 1, 1:n + 1] * 1e-3
    u = u.astype(dtype)
    a_ref, r_ref = oracle.residual(u, f, h)
    a, r = rb.rbgs_residual(dev(u), dev(f), h=h)
    assert a == pytest.approx(a_ref, rel=1e-13, abs=0)
    assert r == pytest.approx(r_ref, rel=1e-13, abs=0)
    # repeated calls are bitwise reproducible
    a2, r2 = rb.rbgs_residual(dev(u), dev(f), h=h)
    assert (a2, r2) == (a, r)


@pytest.mark.parametrize("n,tol,check", [(15, 1e-6, 1), (63, 1e-9, 7), (127, 1e-8, 50)])
def test_solve_matches_oracle(oracle, n, tol, check):
    say(f"solve n={n} tol={tol} check_every={check}")
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=3)
    u0 = W.zeros(n)
    ref = u0.copy()
    rc, done, rel = oracle.solve(ref, f, h, 200000, tol, check)
    ut = dev(u0)
    info = rb.rbgs_solve(ut, dev(f), 200000, tol, check_every=check, h=h, kernel="plain")
    assert info["status"] == 0 and rc == 0
    assert info["sweeps"] == done
    assert info["rel_residual"] == pytest.approx(rel, rel=1e-12)
    assert np.array_equal(host(ut), ref)


def test_solve_fixed_sweeps_and_noconv(oracle):
    n = 31
    h = W.spacing(n)
    f = W.sine_rhs(n)
    ut = dev(W.zeros(n))
    info = rb.rbgs_solve(ut, dev(f), 17, 0.0, check_every=5, h=h)
    assert info["status"] == 0 and info["sweeps"] == 17
    ref = W.zeros(n)
    oracle.sweep(ref, f, h, 17)
    assert np.array_equal(host(ut), ref)
    ut = dev(W.zeros(n))
    info = rb.rbgs_solve(ut, dev(f), 10, 1e-12, check_every=3, h=h)
    assert info["status"] == rb.rbgs.ENOCONV and info["sweeps"] == 10


@pytest.mark.parametrize("bf16", [False, True])
def test_ir_solve_matches_oracle(oracle, bf16):
    """FP64 refinement around FP32 inner sweeps: same bits as the oracle's
    refinement (FP32 inner sweeps are bitwise, the FP64 residual per point is
    bitwise, rounding to FP32/bfloat16 is round-to-nearest-even)."""
    n = 63
    say(f"IR solve n={n} bf16={bf16}")
    h = W.spacing(n)
    f = W.fourier_rhs(n, seed=1, count=16, kmax=16)
    ref = W.zeros(n)
    inner = 300
    rc, outer, rel = oracle.ir_solve(ref, f, h, inner, 80, 1e-11, rhs_bf16=bf16)
    assert rc == 0
    ut = dev(W.zeros(n))
    info = rb.rbgs_solve(ut, dev(f), inner * 80, 1e-11, check_every=inner, h=h,
                         precision="bf16rhs_ir" if bf16 else "f32_ir", inner_sweeps=inner,
                         kernel="plain")
    assert info["status"] == 0
    assert info["outer_iters"] == outer
    got = host(ut)
    assert np.array_equal(got, ref)
    assert info["rel_residual"] == pytest.approx(rel, rel=1e-12)


def test_error_paths_on_device():
    n = 15
    u = dev(W.zeros(n))
    f = dev(W.sine_rhs(n))
    # host tensors are rejected before any kernel runs
    ws_ok = torch.empty(rb.rbgs_workspace_size(rb.make_grid(u), rb.rbgs.F64), dtype=torch.uint8,
                        device=DEV)
    with pytest.raises(rb.RbgsError) as e:
        rb.rbgs_sweep(u.cpu(), f.cpu(), 1, workspace=ws_ok)
    assert e.value.status == rb.rbgs.EINVAL
    # a workspace that is too small
    ws = torch.empty(64, dtype=torch.uint8, device=DEV)
    with pytest.raises(rb.RbgsError) as e:
        rb.rbgs_sweep(u, f, 1, workspace=ws)
    assert e.value.status == rb.rbgs.EWORKSPACE
    # SOR (omega != 1) runs in FP64 and without the persistent kernel's
    # verification modes
    with pytest.raises(rb.RbgsError) as e:
        rb.rbgs_solve(u, f, 10, 1e-6, omega=1.5, kernel="blocked", debug_tile_order=1)
    assert e.value.status == rb.rbgs.EUNSUPPORTED
    with pytest.raises(rb.RbgsError) as e:
        rb.rbgs_solve(u.float(), f.float(), 10, 1e-6, omega=1.5)
    assert e.value.status == rb.rbgs.EUNSUPPORTED
    # a NaN right-hand side gives a non-finite residual
    fn = f.clone()
    fn[3, 3] = float("nan")
    info = rb.rbgs_solve(u, fn, 10, 1e-6, check_every=2)
    assert info["status"] == rb.rbgs.ENONFINITE


def test_large_grid_sampled_light_cone(oracle):
    """8191 x 8191 FP64, f ~ U[-1, 1] (seed 0), 200 sweeps, in the launch
    configuration the benchmark times: sampled points (corners, edges,
    interior, tile seams) equal the oracle's values bit for bit."""
    n, m = 8191, 200
    say(f"large grid n={n} sweeps={m}")
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=0)
    ut = torch.zeros((n + 2, n + 2), dtype=torch.float64, device=DEV)
    ft = dev(f)
    rb.rbgs_sweep(ut, ft, m, h=h, kernel="plain")
    got = host(ut)
    pts = [(1, 1), (1, n), (n, 1), (n, n), (2, 2), (n // 2, n // 2), (4096, 4097),
           (4095, 4094), (1234, 5678), (7777, 333), (32, 511), (33, 512), (500, 1), (1, 700)]
    ref = sample_after_sweeps(oracle, W.zeros(n), f, h, m, pts)
    for (p, r) in zip(pts, ref):
        assert got[p] == r, f"point {p}: {got[p]!r} vs {r!r}"
    # the ring is untouched and no NaN appears
    assert not np.any(got[0]) and not np.any(got[-1]) and not np.any(got[:, 0]) and not np.any(got[:, -1])
    assert np.all(np.isfinite(got))
