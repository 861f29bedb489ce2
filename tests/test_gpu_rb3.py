"""Red-black Gauss-Seidel in 3D (7-point Laplacian) on the GPU: sweeps and
solves must equal the oracle bit for bit; the residual agrees to rounding."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2607_01735_amd as rb  # noqa: E402

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def start(n, seed, ld=None, ring=True):
    """A random Dirichlet ring, a random interior start and f ~ U[-1, 1)."""
    ld = n + 2 if ld is None else ld
    rng = np.random.default_rng(seed)
    u = np.zeros((n + 2, n + 2, ld))
    if ring:
        u[:, :, :n + 2] = rng.standard_normal((n + 2, n + 2, n + 2))
    u[1:n + 1, 1:n + 1, 1:n + 1] = rng.uniform(-1.0, 1.0, (n, n, n))
    f = np.zeros_like(u)
    f[1:n + 1, 1:n + 1, 1:n + 1] = rng.uniform(-1.0, 1.0, (n, n, n))
    return u, f


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


# 384 and up: the two-column kernel (odd and even n, padded rows)
@pytest.mark.parametrize("n", [1, 2, 3, 7, 33, 64, 127, 384, 385, 386])
def test_sweeps_bitwise(oracle, n):
    say(f"rb3 sweeps n={n}")
    h = 1.0 / (n + 1)
    u0, f = start(n, n, ld=n + 2 + (n % 3))
    ut = dev(u0)
    rb.rbgs_rb3_sweep(ut, dev(f), 3, h=h)
    ref = oracle.rb3_sweep(u0.copy(), f, h, 3)
    assert np.array_equal(ut.cpu().numpy(), ref)


@pytest.mark.parametrize("n", [1, 9, 64])
def test_residual_matches_oracle(oracle, n):
    say(f"rb3 residual n={n}")
    h = 1.0 / (n + 1)
    u0, f = start(n, 3)
    a, r = rb.rbgs_rb3_residual(dev(u0), dev(f), h=h)
    ra, rr = oracle.rb3_residual(u0, f, h)
    assert a == pytest.approx(ra, rel=1e-12) and r == pytest.approx(rr, rel=1e-12)


def test_solve_matches_oracle(oracle):
    n = 31
    say(f"rb3 solve n={n}")
    h = 1.0 / (n + 1)
    _, f = start(n, 4, ring=False)
    ut = torch.zeros((n + 2,) * 3, dtype=torch.float64, device=DEV)
    info = rb.rbgs_rb3_solve(ut, dev(f), 100000, 1e-8, check_every=20, h=h)
    ref = np.zeros((n + 2,) * 3)
    rc, done, rel = oracle.rb3_solve(ref, f, h, 100000, 1e-8, 20)
    assert rc == 0 and info["status"] == 0 and info["sweeps"] == done
    assert np.array_equal(ut.cpu().numpy(), ref)


def test_fixed_sweeps_and_cap(oracle):
    n = 15
    say("rb3 fixed sweeps / cap")
    h = 1.0 / (n + 1)
    u0, f = start(n, 6)
    ut = dev(u0)
    info = rb.rbgs_rb3_solve(ut, dev(f), 5, -1.0, check_every=2, h=h)
    assert info["sweeps"] == 5
    assert np.array_equal(ut.cpu().numpy(), oracle.rb3_sweep(u0.copy(), f, h, 5))
    ut = dev(u0)
    info = rb.rbgs_rb3_solve(ut, dev(f), 9, 1e-15, check_every=4, h=h)
    assert info["sweeps"] == 9 and info["status"] == rb.rbgs.ENOCONV


def test_large_grid_sweeps_bitwise(oracle):
    """511^3 (1.07 GB per FP64 array): two sweeps equal the oracle's."""
    n = 511
    say(f"rb3 large n={n}")
    h = 1.0 / (n + 1)
    rng = np.random.default_rng(0)
    f = np.zeros((n + 2,) * 3)
    f[1:-1, 1:-1, 1:-1] = rng.uniform(-1.0, 1.0, (n, n, n))
    ut = torch.zeros_like(dev(f))
    rb.rbgs_rb3_sweep(ut, dev(f), 2, h=h)
    got = ut.cpu().numpy()
    del ut
    assert np.array_equal(got, oracle.rb3_sweep(np.zeros_like(f), f, h, 2))


# The flag-driven form (kernel "resident": one launch, (half-sweep, block)
# items from a ticket queue, a counter per block, each block's half-sweep
# waiting only on its six face neighbours)

@pytest.mark.parametrize("n,sweeps", [(1, 3), (2, 4), (7, 5), (20, 3), (33, 4), (64, 3), (127, 5),
                                      (200, 2)])
def test_flags_sweeps_bitwise(oracle, n, sweeps):
    say(f"rb3 flag-driven sweeps n={n} sweeps={sweeps}")
    h = 1.0 / (n + 1)
    u0, f = start(n, 40 + n, ld=n + 2 + (n % 3))
    ut = dev(u0)
    rb.rbgs_rb3_sweep(ut, dev(f), sweeps, h=h, kernel="resident")
    ref = oracle.rb3_sweep(u0.copy(), f, h, sweeps)
    assert np.array_equal(ut.cpu().numpy(), ref)


def test_flags_delay_injection(oracle):
    """Pseudo-random stalls per block and half-sweep change the schedule,
    not the result."""
    n = 33
    say(f"rb3 flag-driven with delays n={n}")
    h = 1.0 / (n + 1)
    u0, f = start(n, 77)
    ut = dev(u0)
    rb.rbgs_rb3_sweep(ut, dev(f), 6, h=h, kernel="resident", debug_delay=4)
    assert np.array_equal(ut.cpu().numpy(), oracle.rb3_sweep(u0.copy(), f, h, 6))


def test_flags_watchdog_then_recovers(oracle):
    """A block that never publishes: the waits on it expire, the call
    returns RBGS_ETIMEOUT, every wave exits, and the next call is correct."""
    n = 33
    say("rb3 flag-driven watchdog")
    h = 1.0 / (n + 1)
    u0, f = start(n, 78)
    ut = dev(u0)
    with pytest.raises(rb.RbgsError) as e:
        rb.rbgs_rb3_sweep(ut, dev(f), 4, h=h, kernel="resident", debug_stall_block=1,
                          debug_spin_limit=20000)
    assert e.value.status == rb.rbgs.ETIMEOUT
    ut = dev(u0)
    rb.rbgs_rb3_sweep(ut, dev(f), 4, h=h, kernel="resident")
    assert np.array_equal(ut.cpu().numpy(), oracle.rb3_sweep(u0.copy(), f, h, 4))


def test_flags_solve_matches_oracle(oracle):
    """Solve to a tolerance with the flag-driven form (one launch per group
    of check_every sweeps): the oracle's sweeps, residual and bits; the
    fixed-count path too."""
    n = 31
    say(f"rb3 flag-driven solve n={n}")
    h = 1.0 / (n + 1)
    _, f = start(n, 4, ring=False)
    ut = torch.zeros((n + 2,) * 3, dtype=torch.float64, device=DEV)
    info = rb.rbgs_rb3_solve(ut, dev(f), 100000, 1e-8, check_every=20, h=h, kernel="resident")
    ref = np.zeros((n + 2,) * 3)
    rc, done, rel = oracle.rb3_solve(ref, f, h, 100000, 1e-8, 20)
    assert rc == 0 and info["status"] == 0 and info["sweeps"] == done
    assert info["rel_residual"] == pytest.approx(rel, rel=1e-12)
    assert np.array_equal(ut.cpu().numpy(), ref)
    u0, f0 = start(15, 6)
    ut = dev(u0)
    info = rb.rbgs_rb3_solve(ut, dev(f0), 7, -1.0, check_every=3, h=1.0 / 16, kernel="resident")
    assert info["sweeps"] == 7
    assert np.array_equal(ut.cpu().numpy(), oracle.rb3_sweep(u0.copy(), f0, 1.0 / 16, 7))


def test_flags_blocked_kernel_rejected():
    n = 7
    u0, f = start(n, 1)
    with pytest.raises(rb.RbgsError) as e:
        rb.rbgs_rb3_sweep(dev(u0), dev(f), 1, kernel="blocked")
    assert e.value.status == rb.rbgs.EUNSUPPORTED


@pytest.mark.parametrize("n", [639, 640, 767])
def test_flags_large_grid_bitwise(oracle, n):
    """767^3, the size the benchmark times (3.6 GB per FP64 array), in the
    launch configuration it times, and the two sides of the switch from the
    deep to the lean plane chunk (639^3, 640^3): two flag-driven sweeps
    equal the oracle's on every point."""
    say(f"rb3 flag-driven large n={n}")
    h = 1.0 / (n + 1)
    rng = np.random.default_rng(0)
    f = np.zeros((n + 2,) * 3)
    f[1:-1, 1:-1, 1:-1] = rng.uniform(-1.0, 1.0, (n, n, n))
    ft = dev(f)
    ut = torch.zeros_like(ft)
    rb.rbgs_rb3_sweep(ut, ft, 2, h=h, kernel="resident")
    got = ut.cpu().numpy()
    del ut, ft
    torch.cuda.empty_cache()
    ref = oracle.rb3_sweep(np.zeros_like(f), f, h, 2)
    assert np.array_equal(got, ref)
