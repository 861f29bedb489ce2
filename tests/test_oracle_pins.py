"""Pins of the oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each test checks it against a
closed form of Eq. (1)'s iteration, a textbook solver, a brute-force small
case, an invariant of the red-black method, or the loop bounds of Algorithm 1.
"""
import os

import numpy as np
import pytest

import workloads as W
from tests import closed_form as cf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel_err(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# --------------------------------------------------------------------------
# Colouring and loop bounds (Section 2 colouring rule; Algorithm 1 loops)
# --------------------------------------------------------------------------
def _load_colours():
    sets = {"red": set(), "black": set()}
    with open(os.path.join(GOLDEN, "alg1_colours_n6.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            x = int(parts[1])
            for y in parts[2:]:
                sets[parts[0]].add((x, int(y)))
    return sets


def test_half_sweep_visits_exactly_algorithm1_points(oracle):
    """Each half-sweep changes exactly the points Algorithm 1 visits for its
    colour on the 6 x 6 example grid (N = 4 interior points per side)."""
    expected = _load_colours()
    n = 4
    for colour, name in ((0, "red"), (1, "black")):
        u = np.ones((n + 2, n + 2))
        f = np.ones((n + 2, n + 2))
        oracle.half_sweep(u, f, W.spacing(n), colour)
        changed = {(i, j) for i in range(n + 2) for j in range(n + 2) if u[i, j] != 1.0}
        assert changed == expected[name]
        # every neighbour of a visited point is 1 and f = 1: (4 - h^2)/4
        h2 = W.spacing(n) ** 2
        for (i, j) in changed:
            assert u[i, j] == 0.25 * (4.0 - h2)
    for i in range(6):
        for j in range(6):
            assert oracle.colour(i, j) == (i + j) % 2


def test_n1_single_point(oracle):
    """N = 1: the only interior point is red; Eq. (1) with a zero ring gives
    u_11 = -h^2 f_11 / 4 = -f_11 / 16, and the black half changes nothing."""
    u = np.zeros((3, 3))
    f = np.zeros((3, 3))
    f[1, 1] = 3.0
    oracle.half_sweep(u, f, 0.5, 0)
    assert u[1, 1] == -3.0 / 16.0
    oracle.half_sweep(u, f, 0.5, 1)
    assert u[1, 1] == -3.0 / 16.0
    assert np.count_nonzero(u) == 1


def test_n2_by_hand(oracle):
    """N = 2, h = 1/3, ring g, f = 0: red points (1,1), (2,2) then black
    points (1,2), (2,1), each the mean of its four neighbours."""
    u = np.zeros((4, 4))
    u[0, :] = [0.0, 1.0, 2.0, 0.0]
    u[3, :] = [0.0, 3.0, 4.0, 0.0]
    u[1:3, 0] = [5.0, 6.0]
    u[1:3, 3] = [7.0, 8.0]
    f = np.zeros((4, 4))
    oracle.sweep(u, f, 1.0 / 3.0, 1)
    r11 = (0.0 + 1.0 + 0.0 + 5.0) / 4      # (2,1)=0, (0,1)=1, (1,2)=0, (1,0)=5
    r22 = (4.0 + 0.0 + 8.0 + 0.0) / 4      # (3,2)=4, (1,2)=0, (2,3)=8, (2,1)=0
    b12 = (r22 + 2.0 + 7.0 + r11) / 4      # (2,2), (0,2), (1,3), (1,1)
    b21 = (3.0 + r11 + r22 + 6.0) / 4      # (3,1), (1,1), (2,2), (2,0)
    assert u[1, 1] == r11 and u[2, 2] == r22
    assert u[1, 2] == pytest.approx(b12, abs=0, rel=1e-15)
    assert u[2, 1] == pytest.approx(b21, abs=0, rel=1e-15)


# --------------------------------------------------------------------------
# Closed-form iterates
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,m", [(1, 1), (1, 5), (3, 1), (3, 7), (15, 1), (15, 40),
                                 (15, 400), (63, 10), (63, 200), (255, 1), (255, 200)])
def test_single_mode_iterate(oracle, n, m):
    """f = 2 pi^2 sin(pi x) sin(pi y): red a*(1-c^(2m-1)) s, black a*(1-c^(2m)) s."""
    h = W.spacing(n)
    f = W.sine_rhs(n)
    u = W.zeros(n)
    oracle.sweep(u, f, h, m)
    expect = cf.iterate(n, [(1, 1, 2 * np.pi ** 2)], m)
    assert rel_err(u, expect) < 4e-15 * max(1, m) ** 0.5 * 4


@pytest.mark.parametrize("n,m", [(15, 3), (63, 25)])
def test_single_mode_after_red_half(oracle, n, m):
    """After the red half of sweep m the black points still hold sweep m-1."""
    h = W.spacing(n)
    f = W.sine_rhs(n)
    u = W.zeros(n)
    oracle.sweep(u, f, h, m - 1)
    oracle.half_sweep(u, f, h, 0)
    expect = cf.iterate(n, [(1, 1, 2 * np.pi ** 2)], m, half=True)
    assert rel_err(u, expect) < 1e-13


def test_config0_closed_form(oracle):
    """255 x 255, h = 1/256, 1000 sweeps (the small FP64 workload): every
    point within 1e-12 of the closed-form iterate; the red coefficient is the
    fraction 1 - c^1999 of a*, and a* = -pi^2 h^2 / (4 sin^2(pi h/2))."""
    n, m = 255, 1000
    h = W.spacing(n)
    u = W.zeros(n)
    oracle.sweep(u, W.sine_rhs(n), h, m)
    expect = cf.iterate(n, [(1, 1, 2 * np.pi ** 2)], m)
    assert rel_err(u, expect) < 1e-12
    c = np.cos(np.pi * h)
    astar = -np.pi ** 2 * h ** 2 / (4 * np.sin(np.pi * h / 2) ** 2)
    s = cf.mode(n, 1, 1)
    i, j = 128, 128  # i+j even: red
    assert u[i, j] / (astar * s[i, j]) == pytest.approx(-np.expm1(1999 * np.log(c)), rel=1e-12)
    _, rel = oracle.residual(u, W.sine_rhs(n), h)
    assert rel == pytest.approx(cf.single_mode_rel(n, m), rel=1e-10)


def test_multi_mode_iterate(oracle):
    """Six modes, including ones above the Nyquist half (k > (N+1)/2), at
    N = 63 after 1, 17 and 300 sweeps."""
    n = 63
    h = W.spacing(n)
    modes = [(1, 2, 1.5), (3, 3, -0.7), (5, 1, 0.25), (17, 40, 2.0), (60, 7, -1.0), (33, 31, 0.6)]
    f = cf.rhs(n, modes)
    for m in (1, 17, 300):
        u = W.zeros(n)
        oracle.sweep(u, f, h, m)
        expect = cf.iterate(n, modes, m)
        assert rel_err(u, expect) < 2e-13


def test_fourier_workload_modes(oracle):
    """The 64-mode right-hand side generator at N = 255 (all k, l <= 64 <
    (N+1)/2): oracle iterate equals the closed form, and the residual equals
    the orthogonality formula after merging duplicate modes."""
    n = 255
    h = W.spacing(n)
    k, l, a = W.fourier_modes(seed=0)
    modes = cf.merge_modes(k, l, a)
    f = W.fourier_rhs(n, seed=0)
    assert rel_err(f, cf.rhs(n, modes)) < 1e-12
    m = 30
    u = W.zeros(n)
    oracle.sweep(u, f, h, m)
    assert rel_err(u, cf.iterate(n, modes, m)) < 1e-12
    _, rel = oracle.residual(u, f, h)
    assert rel == pytest.approx(cf.multi_mode_rel(n, modes, m), rel=1e-9)


# --------------------------------------------------------------------------
# Residual
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [3, 15, 255])
def test_single_mode_residual_rate(oracle, n):
    """rel after sweep m = c^(2m-1)(1+c)/sqrt(2): the residual falls by
    cos^2(pi h) per sweep, exactly for this mode."""
    h = W.spacing(n)
    f = W.sine_rhs(n)
    u = W.zeros(n)
    for m in range(1, 41):
        oracle.sweep(u, f, h, 1)
        _, rel = oracle.residual(u, f, h)
        assert rel == pytest.approx(cf.single_mode_rel(n, m), rel=2e-10)


def test_residual_field_closed_form(oracle):
    """The residual field itself: zero on black points, A mu^(2m-1)(1+mu) s on
    red points, after m full sweeps."""
    n = 31
    h = W.spacing(n)
    modes = [(1, 1, 2.0), (2, 5, -1.0), (9, 3, 0.5)]
    f = cf.rhs(n, modes)
    u = W.zeros(n)
    oracle.sweep(u, f, h, 7)
    _, _, r = oracle.residual(u, f, h, want_field=True)
    assert rel_err(r, cf.residual_field(n, modes, 7)) < 1e-9


def test_residual_special_cases(oracle):
    n = 31
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=3)
    # u = 0 with a zero ring: r = b = f, rel = 1
    a, rel = oracle.residual(W.zeros(n), f, h)
    assert rel == 1.0
    assert a == pytest.approx(np.linalg.norm(f), rel=1e-14)
    # f = 0, u = s_kl, zero ring: r = -lambda_kl s_kl, b = 0 so rel = ||r||
    k, l = 2, 3
    u = cf.mode(n, k, l)
    u[0, :] = u[-1, :] = u[:, 0] = u[:, -1] = 0.0
    lam = -(4 / h ** 2) * (np.sin(k * np.pi * h / 2) ** 2 + np.sin(l * np.pi * h / 2) ** 2)
    a, rel = oracle.residual(u, W.zeros(n), h)
    assert a == pytest.approx(abs(lam) * np.linalg.norm(u), rel=1e-10)
    assert rel == a
    # u = ring only: r equals b, rel = 1
    ring = W.random_ring(n, seed=5)
    a, rel = oracle.residual(ring, f, h)
    assert rel == pytest.approx(1.0, abs=1e-15)
    b = cf.ring_rhs(ring, f)
    assert a == pytest.approx(np.linalg.norm(b), rel=1e-13)


def test_residual_f32_is_fp64_residual_of_widened_iterate(oracle):
    """The residual of a binary32 iterate is the FP64 residual (pinned above)
    of the same values widened to FP64.  Widening is exact, so the two agree
    bit for bit, field included.  The data are random binary32 values of
    mixed magnitude, so a sum or product formed in binary32 (a dropped
    widening) rounds differently; a plain NumPy form of the residual in FP64
    agrees to rounding."""
    n = 33
    h = W.spacing(n)
    rng = np.random.default_rng(21)
    u32 = (W.random_ring(n, seed=22) * 3.0).astype(np.float32)
    u32[1:-1, 1:-1] = (rng.standard_normal((n, n)) * np.exp(rng.uniform(-3, 3, (n, n)))).astype(np.float32)
    f32 = W.zeros(n).astype(np.float32)
    f32[1:-1, 1:-1] = rng.standard_normal((n, n)).astype(np.float32)
    a32, r32, fld32 = oracle.residual(u32, f32, h, want_field=True)
    u64, f64 = u32.astype(np.float64), f32.astype(np.float64)
    a64, r64, fld64 = oracle.residual(u64, f64, h, want_field=True)
    assert a32 == a64 and r32 == r64
    assert np.array_equal(fld32, fld64)
    # independent NumPy form, FP64 throughout
    s = ((u64[2:, 1:-1] + u64[:-2, 1:-1]) + u64[1:-1, 2:]) + u64[1:-1, :-2]
    r = f64[1:-1, 1:-1] - (s - 4.0 * u64[1:-1, 1:-1]) / (h * h)
    assert a32 == pytest.approx(np.linalg.norm(r), rel=1e-13)
    # the same arithmetic in binary32 gives a visibly different residual
    s32 = ((u32[2:, 1:-1] + u32[:-2, 1:-1]) + u32[1:-1, 2:]) + u32[1:-1, :-2]
    r_lo = f32[1:-1, 1:-1].astype(np.float64) - (s32.astype(np.float64) - 4.0 * u64[1:-1, 1:-1]) / (h * h)
    assert abs(np.linalg.norm(r_lo) - a32) > 2e-11 * a32


@pytest.mark.parametrize("seed", [0, 1])
def test_updated_colour_has_zero_residual(oracle, seed):
    """After a red half-sweep the residual vanishes at red points (to
    rounding), after a black half-sweep at black points (random f and ring)."""
    n = 47
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=seed)
    u = W.random_ring(n, seed=seed + 10)
    red, black = cf.colour_masks(n)
    eps = np.finfo(np.float64).eps
    for it in range(4):
        for colour, mask in ((0, red), (1, black)):
            oracle.half_sweep(u, f, h, colour)
            nb = u[2:, 1:-1] + u[:-2, 1:-1] + u[1:-1, 2:] + u[1:-1, :-2]
            lhs = nb - 4 * u[1:-1, 1:-1]
            rhs = h * h * f[1:-1, 1:-1]
            bound = 8 * eps * np.maximum(np.abs(nb), np.abs(rhs)) + 1e-300
            m = mask[1:-1, 1:-1]
            assert np.all(np.abs(lhs - rhs)[m] <= bound[m])


def test_asymptotic_rate_random_f(oracle):
    """For random f the residual ratio per sweep tends to cos^2(pi h), the
    spectral radius of red-black Gauss-Seidel (Young: rho(Jacobi)^2)."""
    n = 31
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=7)
    u = W.zeros(n)
    oracle.sweep(u, f, h, 1000)
    _, r0 = oracle.residual(u, f, h)
    oracle.sweep(u, f, h, 1)
    _, r1 = oracle.residual(u, f, h)
    # subdominant modes have decayed by (mu_12/mu_11)^2000 ~ 5e-7 here
    assert r1 / r0 == pytest.approx(np.cos(np.pi * h) ** 2, rel=2e-6)


# --------------------------------------------------------------------------
# Textbook solvers
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [7, 9, 11, 13, 15])
def test_converges_to_dense_solve(oracle, n):
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=n)
    u = W.zeros(n)
    oracle.sweep(u, f, h, 3000)
    assert rel_err(u, cf.dense_solve(f)) < 1e-13


def test_converges_to_dense_solve_with_ring(oracle):
    n = 9
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=1)
    ring = W.random_ring(n, seed=2)
    u = ring.copy()
    oracle.sweep(u, f, h, 3000)
    assert rel_err(u, cf.dense_solve(f, ring)) < 1e-13
    # the ring is never written
    assert np.array_equal(u[0], ring[0]) and np.array_equal(u[-1], ring[-1])
    assert np.array_equal(u[:, 0], ring[:, 0]) and np.array_equal(u[:, -1], ring[:, -1])


def test_dst_matches_dense():
    for n in (7, 12):
        f = W.uniform_rhs(n, seed=4)
        assert rel_err(cf.dst_solve(f), cf.dense_solve(f)) < 1e-13


def test_converges_to_dst_solve(oracle):
    n = 63
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=9)
    u = W.zeros(n)
    rc, done, rel = oracle.solve(u, f, h, 40000, 1e-13, 500)
    assert rc == 0 and rel <= 1e-13
    assert rel_err(u, cf.dst_solve(f)) < 1e-11


# --------------------------------------------------------------------------
# Invariants
# --------------------------------------------------------------------------
def _python_half_sweep_random_order(u, f, h, colour, rng):
    n = u.shape[0] - 2
    pts = [(i, j) for i in range(1, n + 1) for j in range(1, n + 1) if (i + j) % 2 == colour]
    rng.shuffle(pts)
    h2 = h * h
    for i, j in pts:
        s = u[i + 1, j] + u[i - 1, j]
        s = s + u[i, j + 1]
        s = s + u[i, j - 1]
        s = s - h2 * f[i, j]
        u[i, j] = 0.25 * s


def test_within_colour_order_is_irrelevant(oracle):
    """Points of one colour never read each other (Section 2): any visiting
    order inside a colour gives the same bits."""
    n = 9
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=11)
    rng = np.random.default_rng(12)
    a = W.random_ring(n, seed=13)
    b = a.copy()
    for _ in range(5):
        _python_half_sweep_random_order(a, f, h, 0, rng)
        _python_half_sweep_random_order(a, f, h, 1, rng)
    oracle.sweep(b, f, h, 5)
    assert np.array_equal(a, b)


def test_linearity_powers_of_two(oracle):
    n = 33
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=14)
    a = W.zeros(n)
    b = W.zeros(n)
    oracle.sweep(a, f, h, 20)
    oracle.sweep(b, 8.0 * f, h, 20)
    assert np.array_equal(8.0 * a, b)


def _stripe_update(self_colour, u, f, h, rows):
    """Eq. (1) on the points of one colour within a stripe of rows."""
    h2 = h * h
    n = u.shape[0] - 2
    for i in rows:
        j0 = 2 if (i % 2 == 0) == (self_colour == 0) else 1
        j = np.arange(j0, n + 1, 2)
        s = u[i + 1, j] + u[i - 1, j]
        s = s + u[i, j + 1]
        s = s + u[i, j - 1]
        s = s - h2 * f[i, j]
        u[i, j] = 0.25 * s


def test_task_dependency_schedules_match(oracle):
    """Algorithm 2: 2*nb stripe tasks per iteration with inout on the own
    colour's block and in on the opposite colour's blocks b-1, b, b+1.  Any
    execution order that respects those edges (RAW, WAR, WAW serialised)
    gives the bits of the plain sweep (Section 2.3)."""
    n, nb, iters = 24, 4, 6
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=21)
    bs = n // nb
    tasks = []  # (iteration, colour, block)
    for it in range(iters):
        for colour in (0, 1):
            for b in range(nb):
                tasks.append((it, colour, b))
    index = {t: k for k, t in enumerate(tasks)}

    def reads_writes(t):
        it, c, b = t
        w = {(c, b)}
        r = {(1 - c, bb) for bb in (b - 1, b, b + 1) if 0 <= bb < nb} | {(c, b)}
        return r, w

    # edges from the program (creation) order, as the task runtime derives them
    preds = {t: set() for t in tasks}
    for k, t in enumerate(tasks):
        r, w = reads_writes(t)
        for p in tasks[:k]:
            pr, pw = reads_writes(p)
            if (w & pr) or (w & pw) or (r & pw):
                preds[t].add(p)
    ref = W.zeros(n)
    oracle.sweep(ref, f, h, iters)
    for seed in range(6):
        rng = np.random.default_rng(seed)
        done = set()
        ready = [t for t in tasks if not preds[t]]
        u = W.zeros(n)
        while ready:
            t = ready.pop(int(rng.integers(len(ready))))
            it, c, b = t
            _stripe_update(c, u, f, h, range(1 + b * bs, 1 + (b + 1) * bs))
            done.add(t)
            ready = [x for x in tasks if x not in done and x not in ready and preds[x] <= done] + ready
            ready = sorted(set(ready), key=lambda x: index[x])
        assert len(done) == len(tasks)
        assert np.array_equal(u, ref)


# --------------------------------------------------------------------------
# FP32 emulation and bf16 rounding
# --------------------------------------------------------------------------
def test_f32_single_mode_within_f32_error(oracle):
    n = 63
    h = W.spacing(n)
    f = W.sine_rhs(n).astype(np.float32)
    u = np.zeros_like(f)
    oracle.sweep(u, f, h, 100)
    expect = cf.iterate(n, [(1, 1, 2 * np.pi ** 2)], 100)
    assert rel_err(u.astype(np.float64), expect) < 2e-5
    assert rel_err(u.astype(np.float64), expect) > 1e-9  # really binary32


def test_f32_exact_on_exact_data(oracle):
    """Small dyadic values: every operation is exact in binary32, so the FP32
    form equals the FP64 form bit for bit."""
    n = 15
    h = 1.0 / 16
    rng = np.random.default_rng(3)
    f64 = W.zeros(n)
    f64[1:-1, 1:-1] = rng.integers(-64, 64, size=(n, n)).astype(np.float64)
    u64 = W.zeros(n)
    u64[1:-1, 1:-1] = rng.integers(-64, 64, size=(n, n)).astype(np.float64)
    u32 = u64.astype(np.float32)
    oracle.sweep(u64, f64, h, 1)
    oracle.sweep(u32, f64.astype(np.float32), h, 1)
    assert np.array_equal(u32.astype(np.float64), u64)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    import oracle
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(2000).astype(np.float32),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 1.0078125 + 2 ** -8,
                                  3.0e38, -3.0e38, 1e-40, np.inf, -np.inf], np.float32)])
    # exact ties: 1 + 2^-8 (tie, even down) and 1 + 3*2^-8 (tie, even up)
    x = np.concatenate([x, np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8], np.float32)])
    ours = oracle.round_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours.view(np.uint32), ref.view(np.uint32))


# --------------------------------------------------------------------------
# Solve and iterative refinement
# --------------------------------------------------------------------------
def test_solve_sweep_count_matches_closed_form(oracle):
    """With check_every = 1 the solve stops at the first m whose closed-form
    residual c^(2m-1)(1+c)/sqrt(2) is <= tol."""
    n = 15
    h = W.spacing(n)
    tol = 1e-6
    m = 1
    while cf.single_mode_rel(n, m) > tol:
        m += 1
    u = W.zeros(n)
    rc, done, rel = oracle.solve(u, W.sine_rhs(n), h, 10000, tol, 1)
    assert rc == 0 and done == m and rel <= tol
    u = W.zeros(n)
    rc, done, rel = oracle.solve(u, W.sine_rhs(n), h, m - 1, tol, 1)
    assert rc == oracle.ENOCONV and done == m - 1
    # tol <= 0: exactly max_sweeps
    u = W.zeros(n)
    rc, done, rel = oracle.solve(u, W.sine_rhs(n), h, 37, 0.0, 5)
    assert rc == 0 and done == 37
    assert rel == pytest.approx(cf.single_mode_rel(n, 37), rel=1e-9)


def test_config0_time_to_tolerance_count():
    """Sweeps for rel <= 1e-8 on the 255 x 255 sine problem, from the closed
    form: the first m with c^(2m-1)(1+c)/sqrt(2) <= 1e-8."""
    n = 255
    c = np.cos(np.pi * W.spacing(n))
    m = int(np.ceil((np.log(1e-8 * np.sqrt(2) / (1 + c)) / np.log(c) + 1) / 2))
    assert cf.single_mode_rel(n, m) <= 1e-8 < cf.single_mode_rel(n, m - 1)
    assert m == 124616


@pytest.mark.parametrize("bf16", [False, True])
def test_ir_reaches_fp64_solution(oracle, bf16):
    n = 31
    h = W.spacing(n)
    f = W.fourier_rhs(n, seed=2, count=8, kmax=8)
    u = W.zeros(n)
    rc, outer, rel = oracle.ir_solve(u, f, h, inner_sweeps=400, max_outer=60, rel_tol=1e-12,
                                     rhs_bf16=bf16)
    assert rc == 0 and rel <= 1e-12
    assert rel_err(u, cf.dst_solve(f)) < 1e-10
    _, rel_check = oracle.residual(u, f, h)
    assert rel_check == rel


# --------------------------------------------------------------------------
# Red-black SOR (the first extension: over-relaxed Gauss-Seidel)
# --------------------------------------------------------------------------
def sor_sweep_numpy(u, f, h, omega, nsweeps):
    """The same SOR, written independently of the oracle: each colour is
    updated as a whole array (points of one colour never read each other)."""
    n = u.shape[0] - 2
    h2 = h * h
    ii, jj = np.meshgrid(np.arange(1, n + 1), np.arange(1, n + 1), indexing="ij")
    for _ in range(nsweeps):
        for c in (0, 1):
            m = ((ii + jj) & 1) == c
            i, j = ii[m], jj[m]
            s = u[i + 1, j] + u[i - 1, j]
            s = s + u[i, j + 1]
            s = s + u[i, j - 1]
            s = s - h2 * f[i, j]
            g = 0.25 * s
            old = u[i, j]
            u[i, j] = old + omega * (g - old)
    return u


@pytest.mark.parametrize("n,omega", [(15, 0.7), (16, 1.3), (23, 1.9)])
def test_sor_matches_independent_numpy(oracle, n, omega):
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=n)
    u = W.random_ring(n, seed=n + 1)
    u[1:n + 1, 1:n + 1] = W.uniform_rhs(n, seed=n + 2)[1:n + 1, 1:n + 1]
    ref = sor_sweep_numpy(u.copy(), f, h, omega, 7)
    got = oracle.sor_sweep(u.copy(), f, h, omega, 7)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("omega", [0.6, 1.5, 1.95])
def test_sor_fixed_point_is_the_discrete_solution(oracle, omega):
    """A sweep leaves the exact discrete solution in place (to rounding)."""
    n = 13
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=3)
    ring = W.random_ring(n, seed=4)
    u = cf.dense_solve(f, ring)
    before = u.copy()
    oracle.sor_sweep(u, f, h, omega, 3)
    assert rel_err(u, before) < 1e-13


def test_sor_omega_one_is_gauss_seidel(oracle):
    n = 31
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=5)
    a, b = W.zeros(n), W.zeros(n)
    oracle.sor_sweep(a, f, h, 1.0, 50)
    oracle.sweep(b, f, h, 50)
    assert rel_err(a, b) < 1e-13


@pytest.mark.parametrize("omega", [1.3, 1.6])
def test_sor_rate_is_youngs(oracle, omega):
    """Below the optimum, the asymptotic error factor per red-black SOR sweep
    is Young's ((omega mu + sqrt(omega^2 mu^2 - 4(omega - 1))) / 2)^2 with
    mu = cos(pi h), the Jacobi factor of the model problem."""
    n = 31
    h = W.spacing(n)
    mu = np.cos(np.pi * h)
    assert omega < oracle.omega_opt(n)
    rho = ((omega * mu + np.sqrt(omega ** 2 * mu ** 2 - 4 * (omega - 1))) / 2) ** 2
    f = W.uniform_rhs(n, seed=6)
    exact = cf.dst_solve(f)
    u = W.zeros(n)
    oracle.sor_sweep(u, f, h, omega, 150)
    e0 = np.linalg.norm(u - exact)
    oracle.sor_sweep(u, f, h, omega, 40)
    e1 = np.linalg.norm(u - exact)
    assert (e1 / e0) ** (1 / 40) == pytest.approx(rho, rel=2e-3)


def test_sor_optimal_omega_cuts_sweeps(oracle):
    """At omega_opt = 2/(1 + sin(pi h)) the sweeps to 1e-8 fall from O(N^2)
    to O(N): at N = 63, a few hundred instead of about ten thousand."""
    n = 63
    h = W.spacing(n)
    f = W.sine_rhs(n)
    rc, done_sor, rel = oracle.sor_solve(W.zeros(n), f, h, oracle.omega_opt(n), 20000, 1e-8, 10)
    assert rc == 0 and rel <= 1e-8
    rc, done_gs, _ = oracle.solve(W.zeros(n), f, h, 20000, 1e-8, 10)
    assert rc == 0
    assert done_sor < 400 and done_gs > 10 * done_sor


@pytest.mark.parametrize("bf16", [False, True])
def test_ir_trajectory_within_rounding_bound_of_gauss_seidel(oracle, bf16):
    """Refinement with s inner sweeps per outer step equals, in exact
    arithmetic, s plain sweeps per step (closed_form.refinement_rel_bound
    derives it), so after 2 x 100 inner sweeps of the 64-mode workload at
    N = 1023 its relative residual is the multi-mode closed form of 200
    sweeps within the stated first-order rounding bound -- and not exactly
    (the inner sweeps really are binary32 / the rhs really is bfloat16)."""
    n, inner = 1023, 100
    h = W.spacing(n)
    f = W.fourier_rhs(n, seed=0)
    modes = cf.merge_modes(*W.fourier_modes(seed=0))
    u = W.zeros(n)
    rc, outer, rel = oracle.ir_solve(u, f, h, inner, 2, 1e-30, rhs_bf16=bf16)
    assert outer == 2
    expect = cf.multi_mode_rel(n, modes, 2 * inner)
    bound = cf.refinement_rel_bound([1.0, cf.multi_mode_rel(n, modes, inner)], inner,
                                    2.0 ** -8 if bf16 else 2.0 ** -24)
    assert abs(rel - expect) <= bound
    assert abs(rel - expect) > 1e-12 * expect


# --------------------------------------------------------------------------
# Refinement with the precision fallback (the build's rule, not the paper's)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("bf16", [False, True])
def test_fallback_on_overflow_is_fp64_sweeping(oracle, bf16):
    """A Dirichlet ring of 1e36 puts residuals of ~1e36/h^2 next to it, beyond
    binary32 and bfloat16: the solve switches to FP64 sweeps before any
    inner solve, so it equals the (pinned) FP64 sweep bit for bit; without
    the fallback the refinement runs into non-finite values."""
    n, inner, cap = 63, 50, 400
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=1)
    u0 = W.random_ring(n, seed=2) * 1e36
    u = u0.copy()
    rc, outer, done, rel, prec = oracle.ir_solve_fallback(u, f, h, inner, cap, 1e-12, rhs_bf16=bf16)
    assert (outer, done, prec) == (0, cap, 0)
    ref = u0.copy()
    oracle.sweep(ref, f, h, cap)
    assert np.array_equal(u, ref)
    assert rel == oracle.residual(ref, f, h)[1]
    plain = u0.copy()
    oracle.ir_solve(plain, f, h, inner, cap // inner, 1e-12, rhs_bf16=bf16)
    assert not np.all(np.isfinite(plain))


@pytest.mark.parametrize("bf16", [False, True])
def test_fallback_on_stall_reaches_what_refinement_cannot(oracle, bf16):
    """At 63^2 with 2000 inner sweeps per step the refinement stalls near
    1e-15 (the binary32 correction cannot resolve less); with the fallback
    the solve widens to FP64 sweeps and reaches rel <= 1e-15 within the
    budget, while the plain refinement with the same sweep budget does not."""
    n, inner, tol = 63, 2000, 1e-15
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=3)
    u = W.zeros(n)
    rc, outer, done, rel, prec = oracle.ir_solve_fallback(u, f, h, inner, 200 * inner, tol,
                                                          rhs_bf16=bf16)
    assert rc == 0 and rel <= tol and prec == 0 and outer >= 2
    assert done % inner == 0 and done < 200 * inner
    plain = W.zeros(n)
    rc2, _, rel2 = oracle.ir_solve(plain, f, h, inner, done // inner, tol, rhs_bf16=bf16)
    assert rc2 != 0 and rel2 > tol
