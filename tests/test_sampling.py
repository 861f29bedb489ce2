"""The light-cone sampler agrees with a full oracle run (CPU)."""
import numpy as np

import workloads as W
from tests.sampling import sample_after_sweeps, window_for


def test_windows_respect_parity_and_bounds():
    n, m = 8191, 200
    for (i, j) in [(1, 1), (1, n), (n, n), (4096, 4097), (401, 402), (402, 402), (7000, 3)]:
        a, b, S = window_for(i, j, n, m)
        assert (a + b) % 2 == 0 and 0 <= a and a + S <= n + 1 and 0 <= b and b + S <= n + 1


def test_sampler_matches_full_run(oracle):
    n, m = 301, 20
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=5)
    u0 = W.random_ring(n, seed=6)
    full = u0.copy()
    oracle.sweep(full, f, h, m)
    pts = [(1, 1), (1, n), (n, 1), (n, n), (150, 150), (151, 150), (2, 299), (83, 84), (84, 200)]
    got = sample_after_sweeps(oracle, u0, f, h, m, pts)
    for p, v in zip(pts, got):
        assert v == full[p]
