"""GPU parity of the batched persistent sweep, its graph-captured plan and
the autotuner: every grid of a batch must equal the oracle run on that grid
alone, bit for bit, whatever the mix of sizes, fusion depth and schedule."""
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


def make_batch(sizes, dtype, seed0=1, ring=True):
    us, fs = [], []
    for g, n in enumerate(sizes):
        ld = n + 2 + (g % 3)
        u = W.random_ring(n, seed=seed0 + 1000 + g, ld=ld) if ring else W.zeros(n, ld)
        f = W.normal_rhs(n, seed=seed0 + g, ld=ld)
        us.append(u.astype(dtype))
        fs.append(f.astype(dtype))
    return us, fs


def to_dev(arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in arrs]


SIZES = [1, 2, 7, 31, 63, 64, 100, 127, 255, 300, 511, 63, 127, 1, 255, 65]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("nsweeps,fuse", [(12, 4), (13, 4), (10, 3), (7, 2), (5, 1), (17, 5),
                                          (20, 6), (23, 7), (16, 8), (30, 10)])
def test_batched_bitwise(oracle, dtype, nsweeps, fuse):
    say(f"batched {dtype.__name__} sweeps={nsweeps} fuse={fuse} grids={len(SIZES)}")
    us, fs = make_batch(SIZES, dtype)
    ut, ft = to_dev(us), to_dev(fs)
    rb.rbgs_sweep_batched(ut, ft, nsweeps, fuse=fuse, tile_rows=16)
    torch.cuda.synchronize()
    for g, n in enumerate(SIZES):
        ref = us[g].copy()
        oracle.sweep(ref, fs[g], W.spacing(n), nsweeps)
        got = ut[g].cpu().numpy()
        assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), f"grid {g} (n={n})"


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("lds_max_n", [-1, 31, 63, 127])
def test_batched_lds_resident(oracle, dtype, lds_max_n):
    """Grids up to lds_max_n are swept in one workgroup's LDS (when they fit:
    127 only in FP32), the rest through the tiles; -1 sends every grid
    through the tiles.  Either way each grid is the oracle's, bit for bit."""
    say(f"batched LDS-resident {dtype.__name__} lds_max_n={lds_max_n}")
    us, fs = make_batch(SIZES, dtype, seed0=90)
    ut, ft = to_dev(us), to_dev(fs)
    t = rb.rbgs_sweep_batched(ut, ft, 11, fuse=4, tile_rows=16, lds_max_n=lds_max_n, timing=True)
    assert t["sweep_launches"] >= 1
    for g, n in enumerate(SIZES):
        ref = us[g].copy()
        oracle.sweep(ref, fs[g], W.spacing(n), 11)
        got = ut[g].cpu().numpy()
        assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), f"grid {g} (n={n})"


def test_batched_all_small(oracle):
    """A batch with no grid left for the tiles (no persistent launch at all)."""
    sizes = [63, 5, 127, 31, 1]
    say("batched, every grid LDS-resident")
    us, fs = make_batch(sizes, np.float32, seed0=95)
    ut, ft = to_dev(us), to_dev(fs)
    t = rb.rbgs_sweep_batched(ut, ft, 9, lds_max_n=127, timing=True)
    assert t["sweep_launches"] == 1
    for g, n in enumerate(sizes):
        ref = us[g].copy()
        oracle.sweep(ref, fs[g], W.spacing(n), 9)
        assert np.array_equal(ut[g].cpu().numpy(), ref), f"grid {g} (n={n})"


def test_batched_delay_injection(oracle):
    sizes = [255, 64, 511, 31, 127]
    say("batched with delay injection")
    us, fs = make_batch(sizes, np.float32, seed0=40)
    ut, ft = to_dev(us), to_dev(fs)
    rb.rbgs_sweep_batched(ut, ft, 16, fuse=4, tile_rows=16, debug_delay=20)
    for g, n in enumerate(sizes):
        ref = us[g].copy()
        oracle.sweep(ref, fs[g], W.spacing(n), 16)
        assert np.array_equal(ut[g].cpu().numpy(), ref)


def test_plan_graph_replays(oracle):
    """The captured graph replayed three times, with eager work and host
    synchronisation between replays: replay k gives the oracle after k*m
    sweeps, so flags and tickets are cleared inside the graph."""
    sizes = [127, 255, 63, 300]
    m = 8
    say("batched plan: three graph replays")
    us, fs = make_batch(sizes, np.float32, seed0=7)
    ut, ft = to_dev(us), to_dev(fs)
    refs = [u.copy() for u in us]
    with rb.BatchPlan(ut, ft, m, fuse=4, tile_rows=32) as plan:
        for k in range(3):
            plan.launch()
            scratch = torch.randn(1 << 20, device=DEV)
            _ = (scratch * 2).sum().item()  # eager work between replays
            plan.check()
            for g, n in enumerate(sizes):
                oracle.sweep(refs[g], fs[g], W.spacing(n), m)
                assert np.array_equal(ut[g].cpu().numpy(), refs[g]), f"replay {k} grid {g}"


def test_plan_graph_replays_lds(oracle):
    """As above with the small grids LDS-resident inside the graph."""
    sizes = [127, 255, 63, 31, 300]
    m = 6
    say("batched plan with LDS-resident grids: three graph replays")
    us, fs = make_batch(sizes, np.float32, seed0=8)
    ut, ft = to_dev(us), to_dev(fs)
    refs = [u.copy() for u in us]
    with rb.BatchPlan(ut, ft, m, fuse=4, tile_rows=32, lds_max_n=127) as plan:
        for k in range(3):
            plan.launch()
            plan.check()
            for g, n in enumerate(sizes):
                oracle.sweep(refs[g], fs[g], W.spacing(n), m)
                assert np.array_equal(ut[g].cpu().numpy(), refs[g]), f"replay {k} grid {g}"


def test_autotune_then_sweep(oracle):
    sizes = [255, 511, 127, 63, 255, 1023]
    say("batched autotune")
    us, fs = make_batch(sizes, np.float32, seed0=70, ring=False)
    ut, ft = to_dev(us), to_dev(fs)
    best = rb.rbgs_autotune_batched(ut, ft)
    assert best["fuse"] in (4, 5, 6, 7) and best["tile_rows"] in (64, 128, 256)
    assert best["lds_max_n"] in (-1, 127)
    assert best["ms_per_sweep"] > 0
    # the tuner only read u; a sweep with the tuned choice (picked up from the
    # process-wide table) is still bitwise the oracle
    for g in range(len(sizes)):
        assert np.array_equal(ut[g].cpu().numpy(), us[g])
    nsw = 2 * best["fuse"]
    rb.rbgs_sweep_batched(ut, ft, nsw)
    for g, n in enumerate(sizes):
        ref = us[g].copy()
        oracle.sweep(ref, fs[g], W.spacing(n), nsw)
        assert np.array_equal(ut[g].cpu().numpy(), ref)


def test_batched_watchdog():
    sizes = [255, 127]
    us, fs = make_batch(sizes, np.float32, seed0=3)
    ut, ft = to_dev(us), to_dev(fs)
    say("batched watchdog")
    with pytest.raises(rb.RbgsError) as e:
        rb.rbgs_sweep_batched(ut, ft, 8, fuse=1, tile_rows=8, debug_stall_tile=1,
                              debug_spin_limit=2000)
    assert e.value.status == rb.rbgs.ETIMEOUT


def test_batched_workload_sampled(oracle):
    """512 grids, sizes uniform on {63, 127, 255, 511, 1023} (seed 0), f
    i.i.d. N(0,1) (seed 1+g), FP32, 100 sweeps, one graph-captured launch:
    two grids of every size equal the oracle bit for bit."""
    sizes = W.batch_sizes(512, seed=0)
    say("batched workload: 512 grids, 100 sweeps, FP32")
    ut, ft = [], []
    host_f = {}
    pick = {}
    for g, n in enumerate(sizes):
        f = W.normal_rhs(n, seed=1 + g).astype(np.float32)
        if n not in pick or len(pick[n]) < 2:
            pick.setdefault(n, []).append(g)
            host_f[g] = f
        ut.append(torch.zeros((n + 2, n + 2), dtype=torch.float32, device=DEV))
        ft.append(torch.from_numpy(f).to(DEV))
    with rb.BatchPlan(ut, ft, 100) as plan:
        plan.launch()
        plan.check()
    for n, gs in pick.items():
        for g in gs:
            ref = W.zeros(n).astype(np.float32)
            oracle.sweep(ref, host_f[g], W.spacing(n), 100)
            assert np.array_equal(ut[g].cpu().numpy(), ref), f"grid {g} n={n}"


@pytest.mark.parametrize("bf16", [False, True])
def test_solve_batched_matches_oracle(oracle, bf16):
    """Batched FP64 refinement around batched FP32 inner sweeps: each grid is
    the oracle's refinement of that grid alone, bit for bit, with the same
    number of outer steps; a grid with f = 0 has converged before any step."""
    sizes = [63, 31, 127, 63, 15, 7]
    inner, max_outer, tol = 1000, 40, 1e-9
    say(f"batched IR solve bf16={bf16}")
    fs = [W.fourier_rhs(n, seed=g + 1, count=8, kmax=8) for g, n in enumerate(sizes)]
    fs[5] = np.zeros_like(fs[5])
    ut = to_dev([W.zeros(n) for n in sizes])
    ft = to_dev(fs)
    infos = rb.rbgs_solve_batched(ut, ft, inner * max_outer, tol, inner,
                                  precision="bf16rhs_ir" if bf16 else "f32_ir")
    for g, n in enumerate(sizes):
        ref = W.zeros(n)
        rc, outer, rel = oracle.ir_solve(ref, fs[g], W.spacing(n), inner, max_outer, tol,
                                         rhs_bf16=bf16)
        assert rc == 0 and infos[g]["status"] == 0, (g, infos[g], rc)
        assert infos[g]["outer_iters"] == outer, (g, infos[g], outer)
        assert infos[g]["sweeps"] == inner * outer
        assert np.array_equal(ut[g].cpu().numpy(), ref), f"grid {g} (n={n})"
        assert infos[g]["rel_residual"] == pytest.approx(rel, rel=1e-12, abs=1e-300)
    assert infos[5]["outer_iters"] == 0


@pytest.mark.parametrize("check", [300, 301])
@pytest.mark.parametrize("lds", [0, 63])
def test_solve_batched_f64_matches_oracle(oracle, check, lds):
    """Batched FP64 solve: each grid follows the oracle's solve loop alone,
    bit for bit, with the same sweep count and residual.  check = 300 at the
    default depth (4 for these sizes) gives an odd pass count, so a grid's
    iterate alternates between the ping-pong buffers from round to round;
    lds = 63 sweeps the grids up to 63 in LDS instead of as tiles."""
    sizes = [63, 31, 127, 63, 15, 7, 1]
    tol = 1e-8
    say(f"batched FP64 solve check_every={check} lds_max_n={lds}")
    fs = [W.fourier_rhs(n, seed=g + 1, count=8, kmax=8) for g, n in enumerate(sizes)]
    fs[5] = np.zeros_like(fs[5])
    us = [W.random_ring(n, seed=50 + g) if g != 5 else W.zeros(n) for g, n in enumerate(sizes)]
    ut = to_dev(us)
    ft = to_dev(fs)
    infos = rb.rbgs_solve_batched(ut, ft, 200_000, tol, check, precision="f64", lds_max_n=lds)
    for g, n in enumerate(sizes):
        ref = us[g].copy()
        rc, done, rel = oracle.solve(ref, fs[g], W.spacing(n), 200_000, tol, check)
        assert rc == 0 and infos[g]["status"] == 0, (g, infos[g], rc)
        assert infos[g]["sweeps"] == done, (g, infos[g], done)
        assert infos[g]["outer_iters"] == 0 and infos[g]["precision"] == rb.rbgs.PREC_F64
        assert np.array_equal(ut[g].cpu().numpy(), ref), f"grid {g} (n={n})"
        assert infos[g]["rel_residual"] == pytest.approx(rel, rel=1e-12, abs=1e-300)
    assert infos[5]["sweeps"] == 0  # f = 0 and u = 0: converged before any sweep


def test_solve_batched_f64_sweep_cap(oracle):
    """max_sweeps not a multiple of check_every: the last round takes the
    remainder and every grid ends at max_sweeps with RBGS_ENOCONV, each
    iterate the oracle's."""
    sizes = [127, 63, 255]
    say("batched FP64 solve, sweep cap")
    fs = [W.normal_rhs(n, seed=21 + g) for g, n in enumerate(sizes)]
    ut = to_dev([W.zeros(n) for n in sizes])
    ft = to_dev(fs)
    infos = rb.rbgs_solve_batched(ut, ft, 1000, 1e-14, 300, precision="f64")
    for g, n in enumerate(sizes):
        ref = W.zeros(n)
        rc, done, rel = oracle.solve(ref, fs[g], W.spacing(n), 1000, 1e-14, 300)
        assert done == 1000 == infos[g]["sweeps"]
        assert infos[g]["status"] == rb.rbgs.ENOCONV
        assert np.array_equal(ut[g].cpu().numpy(), ref), f"grid {g} (n={n})"
        assert infos[g]["rel_residual"] == pytest.approx(rel, rel=1e-12)


def test_solve_batched_sweep_cap():
    """max_sweeps not a multiple of inner_sweeps: the last step of a grid takes
    the remaining sweeps (the single-grid solve's rule), and a grid that does
    not reach the tolerance reports RBGS_ENOCONV with sweeps == max_sweeps."""
    sizes = [127, 63]
    say("batched IR solve, sweep cap")
    fs = [W.fourier_rhs(n, seed=11 + g, count=8, kmax=8) for g, n in enumerate(sizes)]
    ut = to_dev([W.zeros(n) for n in sizes])
    ft = to_dev(fs)
    infos = rb.rbgs_solve_batched(ut, ft, 1000, 1e-14, 300)
    single = []
    for g, n in enumerate(sizes):
        u1 = to_dev([W.zeros(n)])[0]
        single.append(rb.rbgs_solve(u1, ft[g], 1000, 1e-14, check_every=300, precision="f32_ir",
                                    inner_sweeps=300, kernel="plain"))
        assert np.array_equal(ut[g].cpu().numpy(), u1.cpu().numpy()), f"grid {g}"
    for g in range(len(sizes)):
        assert infos[g]["sweeps"] == 1000 == single[g]["sweeps"]
        assert infos[g]["outer_iters"] == 4 == single[g]["outer_iters"]
        assert infos[g]["status"] == rb.rbgs.ENOCONV


@pytest.mark.parametrize("omega,check", [(0.0, 50), (0.0, 51), (1.5, 40)])
def test_solve_batched_sor_matches_oracle(oracle, omega, check):
    """Batched red-black SOR (FP64): each grid is the oracle's SOR solve of
    that grid alone, bit for bit, with its own optimum omega (omega = 0) or
    a common one; odd and even pass counts per round."""
    import math
    sizes = [127, 63, 31, 255, 15, 63, 7]
    tol = 1e-9
    say(f"batched SOR solve omega={omega} check_every={check}")
    fs = [W.fourier_rhs(n, seed=30 + g, count=8, kmax=8) for g, n in enumerate(sizes)]
    us = [W.random_ring(n, seed=60 + g) for g, n in enumerate(sizes)]
    ut, ft = to_dev(us), to_dev(fs)
    infos = rb.rbgs_solve_batched(ut, ft, 100_000, tol, check, precision="f64", omega=omega)
    for g, n in enumerate(sizes):
        h = W.spacing(n)
        w = 2.0 / (1.0 + math.sin(math.pi * h)) if omega == 0.0 else omega
        ref = us[g].copy()
        rc, done, rel = oracle.sor_solve(ref, fs[g], h, w, 100_000, tol, check)
        assert rc == 0 and infos[g]["status"] == 0, (g, infos[g], rc)
        assert infos[g]["sweeps"] == done, (g, infos[g], done)
        assert np.array_equal(ut[g].cpu().numpy(), ref), f"grid {g} (n={n})"
        assert infos[g]["rel_residual"] == pytest.approx(rel, rel=1e-12)
    if omega == 0.0:  # SOR at the optimum needs O(n) sweeps, not O(n^2)
        assert infos[3]["sweeps"] < 5000
