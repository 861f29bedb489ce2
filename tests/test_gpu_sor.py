"""Red-black SOR on the GPU (the over-relaxed extension of the method):
sweeps and solves must equal the oracle's SOR bit for bit, and omega = 0
selects the model problem's optimum."""
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


@pytest.mark.parametrize("n", [1, 2, 7, 63, 100, 255, 1023])
@pytest.mark.parametrize("omega", [0.8, 1.5, 1.9])
def test_sor_sweeps_bitwise(oracle, n, omega):
    say(f"SOR sweeps n={n} omega={omega}")
    h = W.spacing(n)
    ld = n + 2 + (n % 3)
    u0, f = start(n, n, ld=ld)
    ut, ft = dev(u0), dev(f)
    info = rb.rbgs_solve(ut, ft, 5, 0.0, check_every=5, h=h, omega=omega, kernel="plain")
    assert info["sweeps"] == 5
    ref = oracle.sor_sweep(u0.copy(), f, h, omega, 5)
    assert np.array_equal(ut.cpu().numpy(), ref)


@pytest.mark.parametrize("kernel", ["plain", "auto"])
def test_sor_solve_matches_oracle(oracle, kernel):
    n = 127
    say(f"SOR solve n={n} kernel={kernel}")
    h = W.spacing(n)
    f = W.fourier_rhs(n, seed=2, count=16, kmax=16)
    omega = oracle.omega_opt(n)
    ut = dev(W.zeros(n))
    info = rb.rbgs_solve(ut, dev(f), 20000, 1e-9, check_every=10, h=h, omega=omega, kernel=kernel)
    ref = W.zeros(n)
    rc, done, rel = oracle.sor_solve(ref, f, h, omega, 20000, 1e-9, 10)
    assert rc == 0 and info["status"] == 0
    assert info["sweeps"] == done
    assert np.array_equal(ut.cpu().numpy(), ref)
    assert info["rel_residual"] == pytest.approx(rel, rel=1e-12)


def test_sor_omega_zero_is_the_optimum():
    n = 255
    say("SOR omega = 0")
    h = W.spacing(n)
    f = dev(W.sine_rhs(n))
    a, b = dev(W.zeros(n)), dev(W.zeros(n))
    ia = rb.rbgs_solve(a, f, 20000, 1e-8, check_every=10, h=h, omega=0.0)
    ib = rb.rbgs_solve(b, f, 20000, 1e-8, check_every=10, h=h,
                       omega=2.0 / (1.0 + np.sin(np.pi * h)))
    assert ia["status"] == ib["status"] == 0
    assert ia["sweeps"] == ib["sweeps"] < 2000
    assert torch.equal(a, b)


@pytest.mark.parametrize("n", [1, 7, 63, 100, 255, 512])
@pytest.mark.parametrize("omega", [0.7, 1.6])
def test_sor_resident_kernel_bitwise(oracle, n, omega):
    """SOR on the resident band kernel (rows in registers, redundant halo
    epochs): the same bits as the oracle's SOR sweeps."""
    say(f"SOR resident n={n} omega={omega}")
    h = W.spacing(n)
    u0, f = start(n, 7 * n + 3)
    ut = dev(u0)
    info = rb.rbgs_solve(ut, dev(f), 13, 0.0, check_every=13, h=h, omega=omega, kernel="resident")
    assert info["sweeps"] == 13
    ref = oracle.sor_sweep(u0.copy(), f, h, omega, 13)
    assert np.array_equal(ut.cpu().numpy(), ref)


def test_sor_resident_solve_matches_plain():
    n = 255
    say("SOR resident vs plain solve")
    h = W.spacing(n)
    f = dev(W.sine_rhs(n))
    a, b = dev(W.zeros(n)), dev(W.zeros(n))
    ia = rb.rbgs_solve(a, f, 20000, 1e-8, check_every=10, h=h, omega=0.0, kernel="resident")
    ib = rb.rbgs_solve(b, f, 20000, 1e-8, check_every=10, h=h, omega=0.0, kernel="plain")
    assert ia["status"] == ib["status"] == 0 and ia["sweeps"] == ib["sweeps"]
    assert torch.equal(a, b)


BLOCKED_CASES = [  # n, sweeps, fuse, tile_rows (0 = default)
    (1, 5, 4, 0), (7, 11, 5, 8), (63, 9, 1, 8), (100, 16, 4, 16), (255, 24, 4, 0),
    (511, 43, 6, 14), (1023, 40, 7, 0), (1500, 21, 7, 32), (2049, 16, 4, 128), (300, 13, 4, 8),
]


@pytest.mark.parametrize("n,sweeps,fuse,rows", BLOCKED_CASES)
@pytest.mark.parametrize("omega", [0.7, 1.6])
def test_sor_blocked_kernel_bitwise(oracle, n, sweeps, fuse, rows, omega):
    """SOR on the persistent blocked kernel (levels relax from each point's
    previous version; red read and written every pass): the oracle's SOR
    sweeps bit for bit, ragged tiles and passes of two depths included."""
    say(f"SOR blocked n={n} sweeps={sweeps} fuse={fuse} rows={rows} omega={omega}")
    h = W.spacing(n)
    ld = n + 2 + (n % 5)
    u0, f = start(n, 3 * n + 1, ld=ld)
    ut = dev(u0)
    info = rb.rbgs_solve(ut, dev(f), sweeps, 0.0, check_every=sweeps, h=h, omega=omega,
                         kernel="blocked", fuse=fuse, tile_rows=rows)
    assert info["sweeps"] == sweeps
    ref = oracle.sor_sweep(u0.copy(), f, h, omega, sweeps)
    got = ut.cpu().numpy()
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), \
        f"max |diff| {np.max(np.abs(got - ref))}"


def test_sor_blocked_solve_matches_plain():
    n = 1023
    say("SOR blocked vs plain solve")
    h = W.spacing(n)
    f = dev(W.sine_rhs(n))
    a, b = dev(W.zeros(n)), dev(W.zeros(n))
    ia = rb.rbgs_solve(a, f, 40000, 1e-8, check_every=50, h=h, omega=0.0, kernel="blocked")
    ib = rb.rbgs_solve(b, f, 40000, 1e-8, check_every=50, h=h, omega=0.0, kernel="plain")
    assert ia["status"] == ib["status"] == 0 and ia["sweeps"] == ib["sweeps"]
    assert torch.equal(a, b)
