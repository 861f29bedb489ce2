"""Pins of the oracle's multigrid cycle (red-black Gauss-Seidel as the
smoother; an extension beyond the paper, whose conclusion in Section 5 names
multilevel odd-even techniques as future work).

Nothing here compares the oracle with itself: the transfers are checked
against exactness on bilinear functions, their adjoint relation and the
separately pinned numpy transfers; the cycle against the dense solve, a
closed-form discrete solution with a nonzero ring, the exact one-point case,
and the textbook convergence factor of the red-black Gauss-Seidel V-cycle
with full weighting and bilinear interpolation (about 0.1 for V(1,1),
independent of h).
"""
import numpy as np
import pytest

import workloads as W
from oracle import transfer_ref as T
from tests import closed_form as cf


def rel_err(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _bilinear(n, a, b, c, d):
    """a + b x + c y + d x y on the (n+2)^2 natural grid (ring included)."""
    x = np.arange(n + 2) / (n + 1)
    X, Y = np.meshgrid(x, x, indexing="ij")
    return a + b * X + c * Y + d * X * Y


# --------------------------------------------------------------------------
# Level sizes
# --------------------------------------------------------------------------
def test_level_sizes(oracle):
    assert oracle.mg_levels(1) == [1]
    assert oracle.mg_levels(2) == [2]
    assert oracle.mg_levels(3) == [3, 1]
    assert oracle.mg_levels(8191) == [2 ** k - 1 for k in range(13, 0, -1)]
    assert oracle.mg_levels(767) == [767, 383, 191, 95, 47, 23, 11, 5, 2]
    assert oracle.mg_levels(64) == [64]
    assert oracle.mg_levels(255, 3) == [255, 127, 63]
    for n in (5, 23, 1023):
        sizes = oracle.mg_levels(n)
        for fine, coarse in zip(sizes, sizes[1:]):
            assert fine == 2 * coarse + 1  # the vertex-centred nesting
        assert sizes[-1] < 3 or sizes[-1] % 2 == 0


# --------------------------------------------------------------------------
# Transfers
# --------------------------------------------------------------------------
@pytest.mark.parametrize("nc", [1, 3, 8])
def test_restrict_constant_and_bilinear(oracle, nc):
    nf = 2 * nc + 1
    r = np.full((nf + 2, nf + 2), 3.25)
    assert np.all(oracle.mg_restrict(r)[1:-1, 1:-1] == 3.25)  # weights sum to one, exactly
    r = _bilinear(nf, 0.5, -1.25, 2.0, 3.0)
    rc = oracle.mg_restrict(r)
    # full weighting reproduces a bilinear function at the coarse points
    expect = r[2:2 * nc + 1:2, 2:2 * nc + 1:2]
    assert rel_err(rc[1:-1, 1:-1], expect) < 1e-14
    assert np.all(rc[0] == 0) and np.all(rc[:, 0] == 0)


@pytest.mark.parametrize("nc", [1, 3, 8])
def test_prolong_bilinear_exact_and_additive(oracle, nc):
    nf = 2 * nc + 1
    e_fine = _bilinear(nf, -0.75, 1.5, 0.25, -2.0)
    ec = e_fine[0:nf + 2:2, 0:nf + 2:2].copy()  # coarse samples, ring included
    base = np.random.default_rng(nc).standard_normal((nf + 2, nf + 2))
    u = base.copy()
    oracle.mg_prolong_add(ec, u)
    inner = (slice(1, nf + 1), slice(1, nf + 1))
    assert rel_err(u[inner] - base[inner], e_fine[inner]) < 1e-14
    # the ring of u is not written
    assert np.array_equal(u[0], base[0]) and np.array_equal(u[-1], base[-1])
    assert np.array_equal(u[:, 0], base[:, 0]) and np.array_equal(u[:, -1], base[:, -1])


def test_restrict_is_quarter_adjoint_of_prolong(oracle):
    """<R r, e>_coarse = 1/4 <r, P e>_fine for interior fields (zero rings)."""
    rng = np.random.default_rng(5)
    nc = 9
    nf = 2 * nc + 1
    r = np.zeros((nf + 2, nf + 2))
    r[1:-1, 1:-1] = rng.standard_normal((nf, nf))
    ec = np.zeros((nc + 2, nc + 2))
    ec[1:-1, 1:-1] = rng.standard_normal((nc, nc))
    pe = np.zeros((nf + 2, nf + 2))
    oracle.mg_prolong_add(ec, pe)
    lhs = np.sum(oracle.mg_restrict(r) * ec)
    rhs = 0.25 * np.sum(r * pe)
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_transfers_match_pinned_numpy_transfers(oracle):
    rng = np.random.default_rng(6)
    nc = 6
    nf = 2 * nc + 1
    r = np.zeros((nf + 2, nf + 2))
    r[1:-1, 1:-1] = rng.standard_normal((nf, nf))
    assert rel_err(oracle.mg_restrict(r), T.restrict(r)) < 1e-14
    ec = np.zeros((nc + 2, nc + 2))
    ec[1:-1, 1:-1] = rng.standard_normal((nc, nc))
    u = np.zeros((nf + 2, nf + 2))
    oracle.mg_prolong_add(ec, u)
    assert rel_err(u, T.prolong(ec)) < 1e-14


# --------------------------------------------------------------------------
# The cycle
# --------------------------------------------------------------------------
def test_one_point_is_exact_in_one_cycle(oracle):
    n = 1
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=3)
    u = W.zeros(n)
    rc, cycles, rel = oracle.mg_solve(u, f, h, 1, 1, 5, 1e-15)
    assert rc == 0 and cycles == 1 and rel <= 1e-15
    assert u[1, 1] == -0.25 * h * h * f[1, 1]


@pytest.mark.parametrize("n,nu", [(15, (1, 1)), (31, (2, 1)), (23, (0, 2))])
def test_converges_to_dense_solve(oracle, n, nu):
    """The cycle's fixed point is the discrete solution (23: a hierarchy
    23 -> 11 -> 5 -> 2 that ends on an even size, solved by sweeps)."""
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=n)
    u = W.zeros(n)
    rc, cycles, rel = oracle.mg_solve(u, f, h, nu[0], nu[1], 60, 1e-14)
    assert rc == 0 and rel <= 1e-14
    assert rel_err(u, cf.dense_solve(f)) < 1e-12


def test_quadratic_with_ring_is_reproduced(oracle):
    """u* = x^2 + y^2 has a discrete Laplacian of exactly 4, so with f = 4
    and u* on the ring the discrete solution is u* itself."""
    n = 63
    h = W.spacing(n)
    x = np.arange(n + 2) * h
    X, Y = np.meshgrid(x, x, indexing="ij")
    exact = X * X + Y * Y
    f = np.full((n + 2, n + 2), 4.0)
    u = exact.copy()
    u[1:-1, 1:-1] = 0.0
    rc, cycles, rel = oracle.mg_solve(u, f, h, 2, 2, 40, 1e-13)
    assert rc == 0 and cycles <= 12
    assert np.max(np.abs(u - exact)) < 1e-11
    assert np.array_equal(u[0], exact[0]) and np.array_equal(u[:, -1], exact[:, -1])


def _asymptotic_factor(oracle, n, nu1, nu2, cycles=10):
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=11)
    f[1:-1, 1:-1] -= 0.5  # zero-mean random right-hand side
    u = W.zeros(n)
    rels = []
    for _ in range(cycles):
        oracle.mg_solve(u, f, h, nu1, nu2, 1, -1.0)
        rels.append(oracle.residual(u, f, h)[0])
    return (rels[-1] / rels[-4]) ** (1.0 / 3.0)


@pytest.mark.parametrize("n", [63, 255])
def test_vcycle_factor_is_textbook_and_h_independent(oracle, n):
    """Red-black Gauss-Seidel V(1,1) with full weighting and bilinear
    interpolation: a factor near 0.1 per cycle (local Fourier analysis of
    the two-grid cycle gives 0.074 for two smoothing steps; the V-cycle is
    slightly weaker), the same on every grid; V(2,2) is faster."""
    f11 = _asymptotic_factor(oracle, n, 1, 1)
    assert 0.07 < f11 < 0.13
    f22 = _asymptotic_factor(oracle, n, 2, 2)
    assert 0.03 < f22 < 0.075 and f22 < f11


def test_default_coarse_sweeps_rule(oracle):
    assert oracle.mg_default_coarse_sweeps(1) == 1
    assert oracle.mg_default_coarse_sweeps(2) == 18
    assert oracle.mg_default_coarse_sweeps(31) == 2048
