"""Pins of the oracle's three-dimensional red-black Gauss-Seidel (7-point
Laplacian; the higher-dimension extension named in the conclusion, Section 5).

Checked against the colouring's loop bounds, the one-point case by hand, a
dense solve of the 7-point matrix built here, a quadratic whose discrete
Laplacian is exactly 6, the zero residual at the colour just updated, and
the asymptotic rate cos^2(pi h) of red-black Gauss-Seidel (the square of the
Jacobi factor (cos + cos + cos)/3 of the lowest mode, the method being
consistently ordered).
"""
import numpy as np
import pytest

NB = ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))


def rel_err(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def cube(n, rng=None, ring=False):
    a = np.zeros((n + 2, n + 2, n + 2))
    if rng is not None:
        if ring:
            a[...] = rng.standard_normal(a.shape)
            a[1:-1, 1:-1, 1:-1] = 0.0
        else:
            a[1:-1, 1:-1, 1:-1] = rng.standard_normal((n, n, n))
    return a


def dense7(n, f, g):
    h = 1.0 / (n + 1)
    idx = lambda i, j, k: ((i - 1) * n + (j - 1)) * n + (k - 1)
    a = np.zeros((n ** 3, n ** 3))
    b = np.zeros(n ** 3)
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            for k in range(1, n + 1):
                p = idx(i, j, k)
                a[p, p] = -6.0
                b[p] = h * h * f[i, j, k]
                for di, dj, dk in NB:
                    ii, jj, kk = i + di, j + dj, k + dk
                    if 1 <= ii <= n and 1 <= jj <= n and 1 <= kk <= n:
                        a[p, idx(ii, jj, kk)] = 1.0
                    else:
                        b[p] -= g[ii, jj, kk]
    out = g.copy()
    out[1:-1, 1:-1, 1:-1] = np.linalg.solve(a, b).reshape(n, n, n)
    return out


def test_half_sweep_touches_exactly_its_colour(oracle):
    n = 4
    h = 1.0 / (n + 1)
    for colour in (0, 1):
        u = np.ones((n + 2, n + 2, n + 2))
        f = np.ones_like(u)
        oracle.rb3_half_sweep(u, f, h, colour)
        changed = set(zip(*np.nonzero(u != 1.0)))
        want = {(i, j, k) for i in range(1, n + 1) for j in range(1, n + 1)
                for k in range(1, n + 1) if (i + j + k) % 2 == colour}
        assert changed == want
        for p in changed:  # six neighbours at 1, f = 1
            assert u[p] == (6.0 - h * h) / 6.0


def test_one_point(oracle):
    n = 1
    h = 0.5
    rng = np.random.default_rng(1)
    u = cube(n, rng, ring=True)
    f = np.full_like(u, 3.0)
    g = u.copy()
    oracle.rb3_sweep(u, f, h, 1)
    s = sum(g[1 + a, 1 + b, 1 + c] for a, b, c in NB)
    assert u[1, 1, 1] == pytest.approx((s - h * h * 3.0) / 6.0, rel=1e-15)


@pytest.mark.parametrize("n", [4, 5])
def test_converges_to_dense_solve(oracle, n):
    rng = np.random.default_rng(n)
    h = 1.0 / (n + 1)
    g = cube(n, rng, ring=True)
    f = cube(n, rng)
    u = g.copy()
    rc, done, rel = oracle.rb3_solve(u, f, h, 5000, 1e-14, 10)
    assert rc == 0
    assert rel_err(u, dense7(n, f, g)) < 1e-12


def test_quadratic_is_reproduced(oracle):
    n = 15
    h = 1.0 / (n + 1)
    x = np.arange(n + 2) * h
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    exact = X * X + Y * Y + Z * Z
    f = np.full_like(exact, 6.0)
    assert oracle.rb3_residual(exact, f, h)[1] < 1e-12
    u = exact.copy()
    u[1:-1, 1:-1, 1:-1] = 0.0
    rc, done, rel = oracle.rb3_solve(u, f, h, 20000, 1e-13, 20)
    assert rc == 0 and np.max(np.abs(u - exact)) < 1e-11


def test_updated_colour_has_zero_residual(oracle):
    n = 7
    h = 1.0 / (n + 1)
    rng = np.random.default_rng(2)
    u = rng.standard_normal((n + 2, n + 2, n + 2))
    f = rng.standard_normal(u.shape)
    I, J, K = np.meshgrid(*(np.arange(n + 2),) * 3, indexing="ij")
    inner = (I >= 1) & (I <= n) & (J >= 1) & (J <= n) & (K >= 1) & (K <= n)
    for colour in (0, 1):
        oracle.rb3_half_sweep(u, f, h, colour)
        _, _, r = oracle.rb3_residual(u, f, h, want_field=True)
        mine = inner & ((I + J + K) % 2 == colour)
        assert np.max(np.abs(r[mine])) < 1e-9
        assert np.max(np.abs(r[inner & ~mine])) > 1e-3


def test_asymptotic_rate_is_cos_squared(oracle):
    n = 15
    h = 1.0 / (n + 1)
    rng = np.random.default_rng(3)
    u = cube(n, rng)
    f = np.zeros_like(u)
    oracle.rb3_sweep(u, f, h, 400)
    r0 = oracle.rb3_residual(u, f, h)[0]
    oracle.rb3_sweep(u, f, h, 1)
    r1 = oracle.rb3_residual(u, f, h)[0]
    assert r1 / r0 == pytest.approx(np.cos(np.pi * h) ** 2, rel=1e-4)
