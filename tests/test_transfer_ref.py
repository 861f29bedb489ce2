"""Pins of the reference grid transfers (oracle/transfer_ref.py)."""
import numpy as np
import pytest

from oracle import transfer_ref as T
from oracle import unet_ref as U


def bilinear(n, a, b, c, d):
    x = np.arange(n + 2) / (n + 1)
    X, Y = np.meshgrid(x, x, indexing="ij")
    return a + b * X + c * Y + d * X * Y


@pytest.mark.parametrize("nc", [1, 3, 7])
def test_restrict_exact_on_bilinear(nc):
    """Full weighting is separable and each 1-D (1,2,1)/4 average reproduces
    linear functions, so bilinear functions restrict to their samples."""
    nf = 2 * nc + 1
    fine = bilinear(nf, 0.3, -1.2, 2.5, 0.7)
    want = bilinear(nc, 0.3, -1.2, 2.5, 0.7)
    got = T.restrict(fine)
    assert np.allclose(got[1:-1, 1:-1], want[1:-1, 1:-1], rtol=0, atol=1e-14)
    assert not np.any(got[0]) and not np.any(got[:, -1])


@pytest.mark.parametrize("nc", [1, 4, 7])
def test_prolong_exact_on_bilinear_with_ring(nc):
    """Bilinear interpolation reproduces bilinear functions, ring included."""
    nf = 2 * nc + 1
    coarse = bilinear(nc, -0.4, 1.1, 0.9, -2.0)
    want = bilinear(nf, -0.4, 1.1, 0.9, -2.0)
    ring = np.full((nf + 2, nf + 2), 7.0)
    got = T.prolong(coarse, ring=ring)
    assert np.allclose(got[1:-1, 1:-1], want[1:-1, 1:-1], rtol=0, atol=1e-14)
    assert np.all(got[0] == 7.0) and np.all(got[:, 0] == 7.0)


def test_prolong_is_four_times_restrict_transpose():
    """With a zero coarse ring, <P c, x>_fine = 4 <c, R x>_coarse."""
    rng = np.random.default_rng(0)
    nc = 6
    nf = 2 * nc + 1
    for _ in range(5):
        c = np.zeros((nc + 2, nc + 2))
        c[1:-1, 1:-1] = rng.standard_normal((nc, nc))
        x = np.zeros((nf + 2, nf + 2))
        x[1:-1, 1:-1] = rng.standard_normal((nf, nf))
        lhs = np.sum(T.prolong(c) * x)
        rhs = 4.0 * np.sum(c * T.restrict(x))
        assert lhs == pytest.approx(rhs, rel=1e-12)


def test_agrees_with_unet_channel_transfers():
    """The U-Net reference implements the same two operators on interior
    channel arrays (written separately, with slicing instead of loops)."""
    rng = np.random.default_rng(1)
    nc = 7
    nf = 2 * nc + 1
    fine = np.zeros((nf + 2, nf + 2))
    fine[1:-1, 1:-1] = rng.standard_normal((nf, nf))
    assert np.allclose(T.restrict(fine)[1:-1, 1:-1], U.restrict(fine[None, 1:-1, 1:-1])[0],
                       rtol=0, atol=1e-14)
    c = np.zeros((nc + 2, nc + 2))
    c[1:-1, 1:-1] = rng.standard_normal((nc, nc))
    assert np.allclose(T.prolong(c)[1:-1, 1:-1], U.prolong(c[None, 1:-1, 1:-1], nf)[0],
                       rtol=0, atol=1e-14)


def test_transfers_of_constants():
    """R keeps constants (weights sum to 1); P of a constant coarse grid
    with the same constant on its ring is that constant."""
    nc = 5
    nf = 2 * nc + 1
    fine = np.full((nf + 2, nf + 2), 3.25)
    assert np.all(T.restrict(fine)[1:-1, 1:-1] == 3.25)
    coarse = np.full((nc + 2, nc + 2), -1.5)
    assert np.all(T.prolong(coarse)[1:-1, 1:-1] == -1.5)
