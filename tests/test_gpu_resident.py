"""GPU parity of the resident band sweep (RBGS_KERNEL_RESIDENT).

The bands exchange their boundary rows every 4 sweeps and run 4 sweeps in
between on a halo of 8 rows; any such schedule computes the values of the
sequential red-black sweep (the dependency argument of Section 2.3), so
the result must equal the oracle bit for bit: every size from one band to
the most lanes the kernel takes, sweep counts that are and are not
multiples of 4, random Dirichlet rings, padded rows, both precisions,
injected delays between epochs, and inside solves and refinement.
"""
import sys

import numpy as np
import pytest

import workloads as W

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


def start(n, seed, ld=None, dtype=np.float64):
    u = W.random_ring(n, seed=seed, ld=ld)
    u[1:n + 1, 1:n + 1] = W.uniform_rhs(n, seed=seed + 1)[1:n + 1, 1:n + 1]
    f = W.uniform_rhs(n, seed=seed + 2, ld=ld)
    return u.astype(dtype), f.astype(dtype)


CASES = [  # n, sweeps
    (1, 5), (2, 3), (5, 7), (17, 4), (18, 9), (19, 13), (36, 8), (37, 1), (63, 40), (64, 6),
    (100, 17), (255, 24), (257, 11), (300, 8), (511, 40), (512, 12),
]
CASES32 = CASES + [(513, 9), (700, 20), (1000, 12), (1023, 16), (1024, 5)]


@pytest.mark.parametrize("n,sweeps", CASES)
def test_resident_sweep_bitwise_f64(oracle, n, sweeps):
    say(f"resident f64 n={n} sweeps={sweeps}")
    h = W.spacing(n)
    ld = n + 2 + (n % 3)
    u0, f = start(n, n, ld=ld)
    ut, ft = dev(u0), dev(f)
    rb.rbgs_sweep(ut, ft, sweeps, h=h, kernel="resident")
    ref = u0.copy()
    oracle.sweep(ref, f, h, sweeps)
    got = host(ut)
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), \
        f"max |diff| {np.max(np.abs(got - ref))}"


@pytest.mark.parametrize("n,sweeps", CASES32)
def test_resident_sweep_bitwise_f32(oracle, n, sweeps):
    say(f"resident f32 n={n} sweeps={sweeps}")
    h = W.spacing(n)
    u0, f = start(n, n + 7, dtype=np.float32)
    ut, ft = dev(u0), dev(f)
    rb.rbgs_sweep(ut, ft, sweeps, h=h, kernel="resident")
    ref = u0.copy()
    oracle.sweep(ref, f, h, sweeps)
    got = host(ut)
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), \
        f"max |diff| {np.max(np.abs(got.astype(np.float64) - ref))}"


@pytest.mark.parametrize("delay", [5, 40])
def test_resident_delay_injection(oracle, delay):
    """Pseudo-random stalls between epochs let bands drift apart; the bits
    must not change."""
    n, sweeps = 255, 33
    say(f"resident delay={delay} n={n}")
    h = W.spacing(n)
    u0, f = start(n, 11)
    ut, ft = dev(u0), dev(f)
    rb.rbgs_sweep(ut, ft, sweeps, h=h, kernel="resident", debug_delay=delay)
    ref = u0.copy()
    oracle.sweep(ref, f, h, sweeps)
    assert np.array_equal(host(ut), ref)


def test_resident_equals_plain_many_sweeps():
    n, sweeps = 511, 2001
    say(f"resident vs plain n={n} sweeps={sweeps}")
    h = W.spacing(n)
    u0, f = start(n, 21)
    a, b, ft = dev(u0), dev(u0), dev(f)
    rb.rbgs_sweep(a, ft, sweeps, h=h, kernel="resident")
    rb.rbgs_sweep(b, ft, sweeps, h=h, kernel="plain")
    assert torch.equal(a, b)


def test_resident_rejects_large_grids():
    for n, dtype in ((513, torch.float64), (1025, torch.float32)):
        u = torch.zeros((n + 2, n + 2), dtype=dtype, device=DEV)
        with pytest.raises(rb.RbgsError) as e:
            rb.rbgs_sweep(u, u.clone(), 2, kernel="resident")
        assert e.value.status == rb.rbgs.EUNSUPPORTED


def test_resident_watchdog_returns_timeout():
    """Band 0 never publishes; its neighbour's bounded wait expires, every
    workgroup leaves and the call reports a timeout."""
    n = 255
    say("resident watchdog (stalled band, bounded waits)")
    u0, f = start(n, 3)
    ut, ft = dev(u0), dev(f)
    with pytest.raises(rb.RbgsError) as e:
        rb.rbgs_sweep(ut, ft, 12, kernel="resident", debug_stall_tile=1, debug_spin_limit=2000)
    assert e.value.status == rb.rbgs.ETIMEOUT
    ut, ft = dev(u0), dev(f)
    rb.rbgs_sweep(ut, ft, 12, kernel="resident")
    torch.cuda.synchronize()


def test_resident_solve_matches_oracle(oracle):
    n, tol, check, cap = 255, 1e-3, 500, 60000
    say(f"resident solve n={n} tol={tol}")
    h = W.spacing(n)
    f = W.sine_rhs(n)
    ref = W.zeros(n)
    rc, done, rel = oracle.solve(ref, f, h, cap, tol, check)
    ut = dev(W.zeros(n))
    info = rb.rbgs_solve(ut, dev(f), cap, tol, check_every=check, h=h, kernel="resident")
    assert info["status"] == rc and info["sweeps"] == done
    assert info["rel_residual"] == pytest.approx(rel, rel=1e-12)
    assert np.array_equal(host(ut), ref)


def test_resident_ir_matches_oracle(oracle):
    n, inner = 255, 64
    say(f"resident IR n={n}")
    h = W.spacing(n)
    f = W.fourier_rhs(n, seed=3, count=16, kmax=16)
    ref = W.zeros(n)
    rc, outer, rel = oracle.ir_solve(ref, f, h, inner, 20, 1e-9)
    ut = dev(W.zeros(n))
    info = rb.rbgs_solve(ut, dev(f), inner * 20, 1e-9, check_every=inner, h=h,
                         precision="f32_ir", inner_sweeps=inner, kernel="resident")
    assert info["outer_iters"] == outer and rc == info["status"]
    assert np.array_equal(host(ut), ref)
