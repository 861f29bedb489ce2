"""The light-cone sampler agrees with a full oracle run (CPU)."""
import numpy as np
import pytest

import workloads as W
from tests.sampling import (sample_after_refinement, sample_after_sweeps, window_for,
                            window_for_radius)


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


@pytest.mark.parametrize("bf16", [False, True])
def test_refinement_light_cone_sampling_matches_full_grid(oracle, bf16):
    """Windows cut for refinement (2 outer steps of 20 inner sweeps) give the
    full-grid refinement's values bit for bit, windows smaller than the grid."""
    n = 511
    h = W.spacing(n)
    f = W.fourier_rhs(n, seed=0)
    u = W.zeros(n)
    oracle.ir_solve(u, f, h, 20, 2, 1e-300, rhs_bf16=bf16)
    pts = [(1, 1), (255, 256), (n, n), (100, 400), (300, 3)]
    got = sample_after_refinement(oracle, W.zeros(n), f, h, 20, 2, pts, rhs_bf16=bf16)
    assert np.array_equal(got, np.array([u[p] for p in pts]))
    assert window_for_radius(255, 256, n, 2 * (2 * 20 + 1) + 1)[2] < n
