"""Pins of the oracle's 4-colour Gauss-Seidel for the 9-point Laplacian (the
multi-colour extension named in the conclusion, Section 5).

Nothing here compares the oracle with itself: the sweep is checked against
the colouring's defining property (no two neighbours share a colour), the
by-hand one-point case, a dense solve of the 9-point matrix built here from
the stencil, a quadratic whose 9-point Laplacian is exactly 4, the zero
residual Gauss-Seidel leaves at the colour it just updated, and the
independence of the order inside a colour.
"""
import numpy as np
import pytest

import workloads as W


def rel_err(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


EDGES = ((1, 0), (-1, 0), (0, 1), (0, -1))
CORNERS = ((1, 1), (1, -1), (-1, 1), (-1, -1))


def dense9(n, f, ring=None):
    """Exact discrete solution of the 9-point system by a dense solve: the
    matrix (4 edges + corners - 20 centre) / (6 h^2) over the interior, the
    ring's contributions moved to the right-hand side."""
    h = 1.0 / (n + 1)
    g = np.zeros((n + 2, n + 2)) if ring is None else ring
    size = n * n
    a = np.zeros((size, size))
    b = f[1:n + 1, 1:n + 1].reshape(-1).copy() * 6.0 * h * h
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            p = (i - 1) * n + (j - 1)
            a[p, p] = -20.0
            for (di, dj), w in [(d, 4.0) for d in EDGES] + [(d, 1.0) for d in CORNERS]:
                ii, jj = i + di, j + dj
                if 1 <= ii <= n and 1 <= jj <= n:
                    a[p, (ii - 1) * n + (jj - 1)] = w
                else:
                    b[p] -= w * g[ii, jj]
    out = g.copy()
    out[1:n + 1, 1:n + 1] = np.linalg.solve(a, b).reshape(n, n)
    return out


def test_colouring_separates_every_neighbour(oracle):
    for i in range(1, 12):
        for j in range(1, 12):
            c = oracle.mc9_colour(i, j)
            assert c == (i % 2) + 2 * (j % 2)
            for di, dj in EDGES + CORNERS:
                assert oracle.mc9_colour(i + di, j + dj) != c


def test_quarter_sweep_touches_exactly_its_colour(oracle):
    n = 6
    h = W.spacing(n)
    for colour in range(4):
        u = np.ones((n + 2, n + 2))
        f = np.ones((n + 2, n + 2))
        oracle.mc9_quarter_sweep(u, f, h, colour)
        changed = {(i, j) for i in range(n + 2) for j in range(n + 2) if u[i, j] != 1.0}
        want = {(i, j) for i in range(1, n + 1) for j in range(1, n + 1)
                if (i % 2) + 2 * (j % 2) == colour}
        assert changed == want
        for (i, j) in changed:  # all neighbours 1, f = 1: (20 - 6 h^2) / 20
            assert u[i, j] == (20.0 - 6.0 * (h * h)) / 20.0


def test_one_point(oracle):
    n = 1
    h = W.spacing(n)
    u = W.random_ring(n, seed=4)
    f = np.full((3, 3), 2.5)
    ring = u.copy()
    oracle.mc9_sweep(u, f, h, 1)
    e = ring[2, 1] + ring[0, 1] + ring[1, 2] + ring[1, 0]
    c = ring[2, 2] + ring[2, 0] + ring[0, 2] + ring[0, 0]
    assert u[1, 1] == pytest.approx((4 * e + c - 6 * h * h * 2.5) / 20, rel=1e-15)
    _, rel = oracle.mc9_residual(u, f, h)
    assert rel < 1e-14


@pytest.mark.parametrize("n", [4, 7, 10])
def test_converges_to_dense_solve(oracle, n):
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=n)
    ring = W.random_ring(n, seed=n + 1)
    u = ring.copy()
    rc, done, rel = oracle.mc9_solve(u, f, h, 5000, 1e-14, 10)
    assert rc == 0
    assert rel_err(u, dense9(n, f, ring)) < 1e-12


def test_quadratic_is_reproduced(oracle):
    """u* = x^2 + y^2 has a 9-point Laplacian of exactly 4 (the stencil is
    exact on quadratics), so with f = 4 and u* on the ring it is the
    discrete solution."""
    n = 31
    h = W.spacing(n)
    x = np.arange(n + 2) * h
    X, Y = np.meshgrid(x, x, indexing="ij")
    exact = X * X + Y * Y
    f = np.full((n + 2, n + 2), 4.0)
    _, rel0 = oracle.mc9_residual(exact, f, h)
    assert rel0 < 1e-12
    u = exact.copy()
    u[1:-1, 1:-1] = 0.0
    rc, done, rel = oracle.mc9_solve(u, f, h, 20000, 1e-13, 50)
    assert rc == 0 and np.max(np.abs(u - exact)) < 1e-11


def test_updated_colour_has_zero_residual(oracle):
    n = 15
    h = W.spacing(n)
    rng = np.random.default_rng(3)
    u = rng.standard_normal((n + 2, n + 2))
    f = rng.standard_normal((n + 2, n + 2))
    for colour in range(4):
        oracle.mc9_quarter_sweep(u, f, h, colour)
        _, _, r = oracle.mc9_residual(u, f, h, want_field=True)
        mask = np.zeros_like(u, bool)
        for i in range(1, n + 1):
            for j in range(1, n + 1):
                mask[i, j] = (i % 2) + 2 * (j % 2) == colour
        scale = np.max(np.abs(f))
        assert np.max(np.abs(r[mask])) < 1e-9 * scale
        assert np.max(np.abs(r[1:-1, 1:-1][~mask[1:-1, 1:-1]])) > 1e-3
    # after a whole sweep the last colour (3) is the one at zero residual
    oracle.mc9_sweep(u, f, h, 1)
    _, _, r = oracle.mc9_residual(u, f, h, want_field=True)
    assert np.max(np.abs(r[1:n + 1:2, 1:n + 1:2])) < 1e-9 * np.max(np.abs(f))
    assert np.max(np.abs(r[2:n + 1:2, 2:n + 1:2])) > 1e-3


def test_order_within_a_colour_is_irrelevant(oracle):
    n = 9
    h = W.spacing(n)
    rng = np.random.default_rng(7)
    u0 = rng.standard_normal((n + 2, n + 2))
    f = rng.standard_normal((n + 2, n + 2))
    ref = oracle.mc9_sweep(u0.copy(), f, h, 1)
    u = u0.copy()
    c6 = 6.0 * (h * h)
    for colour in range(4):
        pts = [(i, j) for i in range(1, n + 1) for j in range(1, n + 1)
               if (i % 2) + 2 * (j % 2) == colour]
        rng.shuffle(pts)
        for i, j in pts:
            e = ((u[i + 1, j] + u[i - 1, j]) + u[i, j + 1]) + u[i, j - 1]
            c = ((u[i + 1, j + 1] + u[i + 1, j - 1]) + u[i - 1, j + 1]) + u[i - 1, j - 1]
            u[i, j] = ((4.0 * e + c) - c6 * f[i, j]) / 20.0
    assert np.array_equal(u, ref)
