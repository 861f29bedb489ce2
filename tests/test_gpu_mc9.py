"""Four-colour Gauss-Seidel for the 9-point Laplacian on the GPU (the
multi-colour extension): sweeps and solves must equal the oracle bit for
bit, and the residual must agree with the oracle's to rounding.  Kernel
"resident" is the flag-driven form (all quarter-sweeps in one launch, each
block waiting on its eight neighbours' counters)."""
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


def start(n, seed, ld=None):
    u = W.random_ring(n, seed=seed, ld=ld)
    u[1:n + 1, 1:n + 1] = W.uniform_rhs(n, seed=seed + 1)[1:n + 1, 1:n + 1]
    return u, W.uniform_rhs(n, seed=seed + 2, ld=ld)


@pytest.mark.parametrize("n", [1, 2, 3, 8, 33, 100, 255, 1000, 1023])
@pytest.mark.parametrize("kernel", ["plain", "auto", "resident"])
def test_sweeps_bitwise(oracle, n, kernel):
    say(f"mc9 sweeps n={n} kernel={kernel}")
    h = W.spacing(n)
    ld = n + 2 + (n % 3)
    u0, f = start(n, 5 * n, ld=ld)
    ut = dev(u0)
    rb.rbgs_mc9_sweep(ut, dev(f), 3, h=h, kernel=kernel)
    ref = oracle.mc9_sweep(u0.copy(), f, h, 3)
    assert np.array_equal(ut.cpu().numpy(), ref)


@pytest.mark.parametrize("n", [1, 17, 255])
def test_residual_matches_oracle(oracle, n):
    say(f"mc9 residual n={n}")
    h = W.spacing(n)
    u0, f = start(n, 7)
    a, r = rb.rbgs_mc9_residual(dev(u0), dev(f), h=h)
    ra, rr = oracle.mc9_residual(u0, f, h)
    assert a == pytest.approx(ra, rel=1e-12) and r == pytest.approx(rr, rel=1e-12)


@pytest.mark.parametrize("kernel", ["plain", "auto", "resident"])
def test_solve_matches_oracle(oracle, kernel):
    n = 63
    say(f"mc9 solve n={n} kernel={kernel}")
    h = W.spacing(n)
    f = W.fourier_rhs(n, seed=3, count=16, kmax=16)
    ut = dev(W.zeros(n))
    info = rb.rbgs_mc9_solve(ut, dev(f), 100000, 1e-8, check_every=50, h=h, kernel=kernel)
    ref = W.zeros(n)
    rc, done, rel = oracle.mc9_solve(ref, f, h, 100000, 1e-8, 50)
    assert rc == 0 and info["status"] == 0 and info["sweeps"] == done
    assert np.array_equal(ut.cpu().numpy(), ref)
    assert info["rel_residual"] == pytest.approx(rel, rel=1e-9)


@pytest.mark.parametrize("kernel", ["plain", "auto", "resident"])
def test_fixed_sweeps_and_cap(oracle, kernel):
    n = 31
    say(f"mc9 fixed sweeps / cap kernel={kernel}")
    h = W.spacing(n)
    u0, f = start(n, 9)
    ut = dev(u0)
    info = rb.rbgs_mc9_solve(ut, dev(f), 7, -1.0, check_every=3, h=h, kernel=kernel)
    assert info["sweeps"] == 7
    assert np.array_equal(ut.cpu().numpy(), oracle.mc9_sweep(u0.copy(), f, h, 7))
    ut = dev(u0)
    info = rb.rbgs_mc9_solve(ut, dev(f), 10, 1e-15, check_every=4, h=h, kernel=kernel)
    assert info["sweeps"] == 10 and info["status"] == rb.rbgs.ENOCONV
    assert np.array_equal(ut.cpu().numpy(), oracle.mc9_sweep(u0.copy(), f, h, 10))


@pytest.mark.parametrize("kernel", ["plain", "auto", "resident"])
def test_full_size_sweeps_bitwise(oracle, kernel):
    """8191^2, the sweep benchmark's grid: two sweeps equal the oracle's."""
    n = 8191
    say(f"mc9 full size n={n} kernel={kernel}")
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=0)
    ut = dev(W.zeros(n))
    rb.rbgs_mc9_sweep(ut, dev(f), 2, h=h, kernel=kernel)
    got = ut.cpu().numpy()
    del ut
    assert np.array_equal(got, oracle.mc9_sweep(W.zeros(n), f, h, 2))


@pytest.mark.parametrize("kernel", ["blocked"])
def test_persistent_kernels_are_unsupported(kernel):
    """There is no temporally blocked 9-point kernel (the flag-driven form
    is kernel "resident"); it is refused before any device work."""
    u = torch.zeros(9, 9, dtype=torch.float64, device=DEV)
    with pytest.raises(rb.RbgsError) as exc:
        rb.rbgs_mc9_sweep(u, u.clone(), 1, kernel=kernel)
    assert exc.value.status == rb.rbgs.EUNSUPPORTED


def test_f32_is_unsupported():
    u = torch.zeros(9, 9, dtype=torch.float32, device=DEV)
    with pytest.raises(rb.RbgsError):
        rb.rbgs_mc9_sweep(u, u.clone(), 1)
