"""Multigrid V-cycles with the red-black Gauss-Seidel smoother on the GPU
(rbgs_mg_solve): the iterate after any number of cycles must equal the
oracle's V-cycle bit for bit, on every smoother kernel, with and without a
Dirichlet ring, on hierarchies that end on one point or on an even size;
to a tolerance the cycle count must match the oracle's."""
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


def start(n, seed, ld=None, ring=True):
    u = W.random_ring(n, seed=seed, ld=ld) if ring else W.zeros(n, ld=ld)
    u[1:n + 1, 1:n + 1] = W.uniform_rhs(n, seed=seed + 1)[1:n + 1, 1:n + 1]
    return u, W.uniform_rhs(n, seed=seed + 2, ld=ld)


@pytest.mark.parametrize("n", [1, 3, 7, 23, 63, 127, 255, 767])
@pytest.mark.parametrize("kernel", ["plain", "blocked", "auto"])
def test_fixed_cycles_bitwise(oracle, n, kernel):
    say(f"mg fixed cycles n={n} kernel={kernel}")
    h = W.spacing(n)
    ld = n + 2 + (n % 5)
    u0, f = start(n, 3 * n + 1, ld=ld)
    ut, ft = dev(u0), dev(f)
    info = rb.rbgs_mg_solve(ut, ft, 3, -1.0, pre_sweeps=2, post_sweeps=1, h=h, kernel=kernel)
    ref = u0.copy()
    rc, cycles, rel = oracle.mg_solve(ref, f, h, 2, 1, 3, -1.0)
    assert info["cycles"] == 3 and info["status"] == 0
    assert info["levels"] == len(oracle.mg_levels(n))
    assert np.array_equal(ut.cpu().numpy(), ref)
    assert info["rel_residual"] == pytest.approx(rel, rel=1e-9, abs=1e-300)


@pytest.mark.parametrize("nu", [(1, 1), (0, 2), (3, 0), (2, 2)])
def test_smoothing_counts_bitwise(oracle, nu):
    n = 127
    say(f"mg smoothing counts {nu}")
    h = W.spacing(n)
    u0, f = start(n, 17)
    ut = dev(u0)
    rb.rbgs_mg_solve(ut, dev(f), 2, -1.0, pre_sweeps=nu[0], post_sweeps=nu[1], h=h)
    ref = u0.copy()
    oracle.mg_solve(ref, f, h, nu[0], nu[1], 2, -1.0)
    assert np.array_equal(ut.cpu().numpy(), ref)


@pytest.mark.parametrize("levels,coarse", [(1, 5), (2, 0), (3, 40)])
def test_level_cap_and_coarse_sweeps(oracle, levels, coarse):
    n = 63
    say(f"mg max_levels={levels} coarse_sweeps={coarse}")
    h = W.spacing(n)
    u0, f = start(n, 5, ring=False)
    ut = dev(u0)
    info = rb.rbgs_mg_solve(ut, dev(f), 2, -1.0, pre_sweeps=1, post_sweeps=1, max_levels=levels,
                            coarse_sweeps=coarse, h=h)
    sizes = oracle.mg_levels(n, levels)
    assert info["levels"] == len(sizes) and info["coarsest_n"] == sizes[-1]
    want = coarse if coarse else oracle.mg_default_coarse_sweeps(sizes[-1])
    assert info["coarse_sweeps"] == want
    ref = u0.copy()
    oracle.mg_solve(ref, f, h, 1, 1, 2, -1.0, max_levels=levels, coarse_sweeps=coarse)
    assert np.array_equal(ut.cpu().numpy(), ref)


@pytest.mark.parametrize("n,kernel", [(255, "auto"), (511, "blocked"), (100, "plain")])
def test_to_tolerance_matches_oracle(oracle, n, kernel):
    say(f"mg to tolerance n={n} kernel={kernel}")
    h = W.spacing(n)
    f = W.fourier_rhs(n, seed=4, count=16, kmax=16)
    ut = dev(W.zeros(n))
    info = rb.rbgs_mg_solve(ut, dev(f), 40, 1e-10, h=h, kernel=kernel)
    ref = W.zeros(n)
    rc, cycles, rel = oracle.mg_solve(ref, f, h, 2, 2, 40, 1e-10)
    assert rc == 0 and info["status"] == 0 and info["graph"] == 1
    assert info["cycles"] == cycles
    assert np.array_equal(ut.cpu().numpy(), ref)
    assert info["rel_residual"] <= 1e-10


def test_resident_smoother_bitwise(oracle):
    n = 255
    say("mg resident smoother")
    h = W.spacing(n)
    u0, f = start(n, 9)
    ut = dev(u0)
    rb.rbgs_mg_solve(ut, dev(f), 2, -1.0, h=h, kernel="resident")
    ref = u0.copy()
    oracle.mg_solve(ref, f, h, 2, 2, 2, -1.0)
    assert np.array_equal(ut.cpu().numpy(), ref)


def test_zero_cycles_and_converged_start(oracle):
    n = 31
    say("mg zero cycles / converged start")
    h = W.spacing(n)
    u0, f = start(n, 2)
    ut = dev(u0)
    info = rb.rbgs_mg_solve(ut, dev(f), 0, -1.0, h=h)
    assert info["cycles"] == 0 and np.array_equal(ut.cpu().numpy(), u0)
    assert info["rel_residual"] == pytest.approx(oracle.residual(u0, f, h)[1], rel=1e-12)
    # a start that already meets the tolerance runs no cycle
    ref = u0.copy()
    oracle.mg_solve(ref, f, h, 2, 2, 30, 1e-12)
    ut = dev(ref)
    info = rb.rbgs_mg_solve(ut, dev(f), 30, 1e-11, h=h)
    assert info["cycles"] == 0 and np.array_equal(ut.cpu().numpy(), ref)


def test_cap_reached_reports_noconv(oracle):
    n = 127
    say("mg cycle cap")
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=8)
    ut = dev(W.zeros(n))
    info = rb.rbgs_mg_solve(ut, dev(f), 2, 1e-14, h=h)
    assert info["cycles"] == 2 and info["status"] == rb.rbgs.ENOCONV
    ref = W.zeros(n)
    rc, cycles, rel = oracle.mg_solve(ref, f, h, 2, 2, 2, 1e-14)
    assert rc == oracle.ENOCONV and np.array_equal(ut.cpu().numpy(), ref)


def test_f32_is_unsupported():
    n = 31
    u = torch.zeros(n + 2, n + 2, dtype=torch.float32, device=DEV)
    with pytest.raises(rb.RbgsError) as exc:
        rb.rbgs_mg_solve(u, u.clone(), 2, 1e-6)
    assert exc.value.status == rb.rbgs.EUNSUPPORTED


def test_full_size_one_cycle_bitwise(oracle):
    """The largest single-GPU grid of the sweep benchmark, 8191^2: one
    V(2,2) cycle on the automatic smoother (blocked on the finest levels)
    equals the oracle's cycle at every point."""
    n = 8191
    say(f"mg full size n={n}")
    h = W.spacing(n)
    f = W.fourier_rhs(n, seed=0)
    ut = dev(W.zeros(n))
    info = rb.rbgs_mg_solve(ut, dev(f), 1, -1.0, h=h)
    assert info["levels"] == 13 and info["coarsest_n"] == 1
    ref = W.zeros(n)
    oracle.mg_solve(ref, f, h, 2, 2, 1, -1.0)
    got = ut.cpu().numpy()
    del ut
    assert np.array_equal(got, ref)


def test_full_size_reaches_tolerance(oracle):
    """8191^2 to a relative residual of 1e-8 in a handful of cycles; the
    residual of the returned iterate, recomputed by the oracle, confirms it."""
    n = 8191
    say(f"mg full size to 1e-8 n={n}")
    h = W.spacing(n)
    f = W.fourier_rhs(n, seed=0)
    ut = dev(W.zeros(n))
    info = rb.rbgs_mg_solve(ut, dev(f), 30, 1e-8, h=h)
    assert info["status"] == 0 and info["cycles"] <= 12
    got = ut.cpu().numpy()
    del ut
    _, rel = oracle.residual(got, f, h)
    assert rel <= 1e-8 * (1 + 1e-6)
    assert rel == pytest.approx(info["rel_residual"], rel=1e-6)


def test_large_rounds_run_uncaptured(oracle):
    """A cycle of more launches than a graph is allowed to hold (here a
    255^2 coarsest level with 40 000 sweeps) runs launch by launch, with the
    same bits."""
    n = 511
    say(f"mg uncaptured cycle n={n}")
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=12)
    ut = dev(W.zeros(n))
    info = rb.rbgs_mg_solve(ut, dev(f), 1, -1.0, pre_sweeps=1, post_sweeps=1, max_levels=2,
                            coarse_sweeps=40000, h=h, kernel="plain")
    assert info["graph"] == 0 and info["cycles"] == 1 and info["coarsest_n"] == 255
    ref = W.zeros(n)
    oracle.mg_solve(ref, f, h, 1, 1, 1, -1.0, max_levels=2, coarse_sweeps=40000)
    assert np.array_equal(ut.cpu().numpy(), ref)
