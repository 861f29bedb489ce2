"""Oracle values at sampled points of a large grid, computed one by one.

After m full sweeps (2m half-sweeps) from a given start, a point's value
depends only on data within grid distance 2m of it: each half-sweep reads
neighbours at distance 1.  So the oracle can run on a square window around
the point whose edges are either the true Dirichlet ring or at least 2m+1
away from it; the window's frozen edge values cannot reach the point.  The
window origin must have even coordinate sum so that local and global
colours agree.  Test helper: it only cuts windows and calls the oracle.
"""
import numpy as np


def _origins(c, n, S, r):
    """Window starts a (window rows a..a+S) keeping point c at least r from
    every edge that is not the true ring (rows 0 and n+1)."""
    out = []
    for a in range(max(0, c - S), min(c, n + 1 - S) + 1):
        top_ok = a == 0 or c - a >= r
        bot_ok = a + S == n + 1 or a + S - c >= r
        if top_ok and bot_ok:
            out.append(a)
    return out


def window_for(i, j, n, m):
    return window_for_radius(i, j, n, 2 * m + 1)


def window_for_radius(i, j, n, r):
    """Window (a, b, S) around (i, j) whose non-ring edges are at least r
    away from it."""
    S = 2 * r + 2
    if S >= n + 1:
        return 0, 0, n + 1
    for a in _origins(i, n, S, r):
        for b in _origins(j, n, S, r):
            if (a + b) % 2 == 0:
                return a, b, S
    raise AssertionError("no window found")


def sample_after_sweeps(oracle, u0, f, h, m, points):
    """Oracle value of u at each point after m sweeps from u0 (natural
    layout, same ld for u0 and f)."""
    n = f.shape[0] - 2
    vals = []
    for (i, j) in points:
        a, b, S = window_for(i, j, n, m)
        wu = np.ascontiguousarray(u0[a:a + S + 1, b:b + S + 1])
        wf = np.ascontiguousarray(f[a:a + S + 1, b:b + S + 1])
        oracle.sweep(wu, wf, h, m)
        vals.append(wu[i - a, j - b])
    return np.array(vals, dtype=u0.dtype)


def sample_after_refinement(oracle, u0, f, h, inner, outer, points, rhs_bf16=False):
    """Oracle value of u at each point after `outer` refinement steps of
    `inner` low-precision sweeps each (oracle.ir_solve).  One step reads u
    at distance 1 (the residual) and then sweeps e from zero with a zero
    ring for 2 * inner half-sweeps, so a wrong value at the window edge (a
    frozen u, a zero e) travels at most 2 * inner + 1 points per step."""
    n = f.shape[0] - 2
    r = outer * (2 * inner + 1) + 1
    vals = []
    for (i, j) in points:
        a, b, S = window_for_radius(i, j, n, r)
        wu = np.ascontiguousarray(u0[a:a + S + 1, b:b + S + 1])
        wf = np.ascontiguousarray(f[a:a + S + 1, b:b + S + 1])
        _, done, _ = oracle.ir_solve(wu, wf, h, inner, outer, 1e-300, rhs_bf16=rhs_bf16)
        assert done == outer
        vals.append(wu[i - a, j - b])
    return np.array(vals, dtype=u0.dtype)
