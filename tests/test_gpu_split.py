"""The split colour layout at the boundary: rbgs_pack / rbgs_unpack and
rbgs_sweep_split must give the bits of rbgs_sweep (and so of the oracle) on
every kernel, without the per-call pack and unpack."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def start(n, seed):
    u = W.random_ring(n, seed=seed)
    u[1:n + 1, 1:n + 1] = W.uniform_rhs(n, seed=seed + 1)[1:n + 1, 1:n + 1]
    return u, W.uniform_rhs(n, seed=seed + 2)


@pytest.mark.parametrize("n", [1, 2, 63, 255, 1000])
def test_pack_unpack_round_trip(n):
    say(f"split pack/unpack n={n}")
    u0, _ = start(n, n)
    ut = dev(u0)
    red, black = rb.rbgs_pack(ut)
    assert red.shape[1] == rb.rbgs_split_pitch(rb.make_grid(ut), rb.rbgs.F64)
    # colour (i + j) & 1 at (i, j >> 1)
    r, b = red.cpu().numpy(), black.cpu().numpy()
    for i in (0, 1, n // 2, n + 1):
        for j in (0, 1, n, n + 1):
            got = (b if (i + j) & 1 else r)[i, j >> 1]
            assert got == u0[i, j]
    out = torch.zeros_like(ut)
    rb.rbgs_unpack(out, red, black)
    o = out.cpu().numpy()
    assert np.array_equal(o[1:n + 1, 1:n + 1], u0[1:n + 1, 1:n + 1])
    assert np.all(o[0] == 0) and np.all(o[:, 0] == 0)  # the ring is not written


@pytest.mark.parametrize("n", [1, 63, 255, 1000])
@pytest.mark.parametrize("kernel", ["plain", "blocked", "resident", "auto"])
def test_sweep_split_bitwise(oracle, n, kernel):
    if kernel == "resident" and n > 512:
        pytest.skip("the resident kernel takes n <= 512 in FP64")
    say(f"split sweep n={n} kernel={kernel}")
    h = W.spacing(n)
    u0, f = start(n, 3 * n + 5)
    ut, ft = dev(u0), dev(f)
    ur, ub = rb.rbgs_pack(ut)
    fr, fb = rb.rbgs_pack(ft)
    rb.rbgs_sweep_split(n, ur, ub, fr, fb, 9, h=h, kernel=kernel)
    rb.rbgs_sweep_split(n, ur, ub, fr, fb, 4, h=h, kernel=kernel)  # state carries over
    rb.rbgs_unpack(ut, ur, ub)
    assert np.array_equal(ut.cpu().numpy(), oracle.sweep(u0.copy(), f, h, 13))
