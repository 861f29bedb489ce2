"""GPU grid transfers (rbgs_restrict, rbgs_prolong) against oracle/transfer_ref.py.

Each output point is a sum of at most nine products by exact weights, in a
different order on the two sides, so the tolerance is a few units in the
last place of the largest input: 8 eps * max|x|.  The rings the kernels
must not write are filled with a sentinel and checked bit for bit.
"""
import numpy as np
import pytest

from oracle import transfer_ref as T

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2607_01735_amd as rb  # noqa: E402

DEV = torch.device("cuda:0")
SENTINEL = -123.5


def batch_array(b, n, pad, dtype, rng):
    """(b, n+2, n+2+pad) random array, plus the tensor view with that ld."""
    a = rng.standard_normal((b, n + 2, n + 2 + pad))
    t = torch.from_numpy(a).to(dtype=dtype, device=DEV)
    return t


def tol(x, dtype):
    eps = torch.finfo(dtype).eps
    return 8 * eps * float(np.max(np.abs(x)))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nc,batch,pad", [(1, 1, 0), (3, 2, 5), (31, 3, 1), (63, 2, 0), (255, 1, 3)])
def test_restrict_matches_reference(dtype, nc, batch, pad):
    print(f"restrict nc={nc} batch={batch} pad={pad} {dtype}", flush=True)
    rng = np.random.default_rng(nc + batch)
    nf = 2 * nc + 1
    fine = batch_array(batch, nf, pad, dtype, rng)
    coarse = torch.full((batch, nc + 2, nc + 2 + pad), SENTINEL, dtype=dtype, device=DEV)
    rb.rbgs_restrict(fine, coarse)
    got = coarse.cpu().numpy().astype(np.float64)
    fin = fine.cpu().numpy().astype(np.float64)
    for b in range(batch):
        want = T.restrict(fin[b, :, :nf + 2])
        assert np.max(np.abs(got[b, 1:-1, 1:nc + 1] - want[1:-1, 1:-1])) <= tol(fin[b], dtype)
        ring = np.ones_like(got[b], dtype=bool)
        ring[1:nc + 1, 1:nc + 1] = False
        assert np.all(got[b][ring] == SENTINEL)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nc,batch,pad", [(1, 1, 0), (3, 2, 5), (31, 3, 1), (63, 2, 0), (255, 1, 3)])
def test_prolong_matches_reference(dtype, nc, batch, pad):
    print(f"prolong nc={nc} batch={batch} pad={pad} {dtype}", flush=True)
    rng = np.random.default_rng(100 + nc + batch)
    nf = 2 * nc + 1
    coarse = batch_array(batch, nc, pad, dtype, rng)  # nonzero coarse ring
    fine = torch.full((batch, nf + 2, nf + 2 + pad), SENTINEL, dtype=dtype, device=DEV)
    rb.rbgs_prolong(coarse, fine)
    got = fine.cpu().numpy().astype(np.float64)
    co = coarse.cpu().numpy().astype(np.float64)
    for b in range(batch):
        want = T.prolong(co[b, :, :nc + 2])
        assert np.max(np.abs(got[b, 1:nf + 1, 1:nf + 1] - want[1:-1, 1:-1])) <= tol(co[b], dtype)
        ring = np.ones_like(got[b], dtype=bool)
        ring[1:nf + 1, 1:nf + 1] = False
        assert np.all(got[b][ring] == SENTINEL)


def test_transfer_rejects_bad_sizes():
    a = torch.zeros((9, 9), dtype=torch.float64, device=DEV)
    b = torch.zeros((6, 6), dtype=torch.float64, device=DEV)  # n_c = 4 needs n_f = 9
    with pytest.raises(rb.RbgsError):
        rb.rbgs_restrict(a, b)
    with pytest.raises(rb.RbgsError):
        rb.rbgs_prolong(b, a)
