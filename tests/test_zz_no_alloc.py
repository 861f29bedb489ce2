"""The residual entry point that allocates nothing (rbgs_residual_noalloc)
against rbgs_residual, through the C ABI.

Both run the same kernels on the same data; the no-allocation form keeps
its partial sums in the library's static per-GPU scratch instead of a
caller workspace, so the norms must agree bit for bit.  Two calls in a row,
the second on a smaller grid (the scratch keeps the first call's contents),
in FP64 and FP32, and at the largest grid the static scratch holds.
"""
import ctypes
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2607_01735_amd as rb  # noqa: E402
from paper_2607_01735_amd import rbgs as abi  # noqa: E402

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def field(n, seed, dtype):
    u = W.random_ring(n, seed=seed)
    u[1:-1, 1:-1] = W.uniform_rhs(n, seed=seed + 1)[1:-1, 1:-1]
    f = W.uniform_rhs(n, seed=seed + 2)
    return (torch.from_numpy(u.astype(dtype)).to(DEV), torch.from_numpy(f.astype(dtype)).to(DEV))


def noalloc_raw(u, f, h):
    """The entry point called through ctypes directly (no binding code)."""
    grid = abi.rbgs_grid(u.shape[0] - 2, u.shape[1], h)
    a, r = ctypes.c_double(), ctypes.c_double()
    code = abi.F64 if u.dtype == torch.float64 else abi.F32
    rc = abi._lib.rbgs_residual_noalloc(ctypes.byref(grid), code, ctypes.c_void_p(u.data_ptr()),
                                        ctypes.c_void_p(f.data_ptr()), ctypes.byref(a),
                                        ctypes.byref(r), None)
    return rc, a.value, r.value


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_noalloc_matches_workspace_residual_twice(dtype):
    for n, seed in ((2047, 1), (301, 7)):  # second call smaller: stale partials stay behind
        say(f"noalloc residual n={n} dtype={np.dtype(dtype).name}")
        u, f = field(n, seed, dtype)
        h = W.spacing(n)
        ref = rb.rbgs_residual(u, f, h=h)
        rc, a, r = noalloc_raw(u, f, h)
        assert rc == 0, abi.rbgs_last_error()
        assert (a, r) == ref, (a, r, ref)
        assert rb.rbgs_residual_noalloc(u, f, h=h) == ref


def test_noalloc_largest_grid_and_rejection():
    n = 16383  # partial sums 2 MiB of the 4 MiB scratch
    say(f"noalloc residual n={n}")
    h = W.spacing(n)
    f = torch.from_numpy(W.fourier_rhs(n, seed=0)).to(DEV)
    u = torch.zeros_like(f)
    ref = rb.rbgs_residual(u, f, h=h)
    assert noalloc_raw(u, f, h)[1:] == ref
    del u, f
    torch.cuda.empty_cache()
    # too large for the static scratch: refused before any device work
    n = 32767
    grid = abi.rbgs_grid(n, n + 2, W.spacing(n))
    rc = abi._lib.rbgs_residual_noalloc(ctypes.byref(grid), abi.F64, ctypes.c_void_p(256),
                                        ctypes.c_void_p(256), None, None, None)
    assert rc == abi.EINVAL and "static scratch" in abi.rbgs_last_error()
