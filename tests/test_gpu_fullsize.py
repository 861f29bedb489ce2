"""Parity at the full workload sizes, through the C ABI.

* 8191 x 8191 FP64, f ~ U[-1, 1) (seed 0), u0 = 0, 200 sweeps -- the
  benchmark's step, launched as the benchmark launches it (rbgs_solve with
  a fixed sweep count): every element of the iterate equals the oracle's
  200 sweeps bit for bit, for the plain kernel (one launch per half-sweep,
  Algorithm 1) and for the default persistent blocked kernel (Algorithm 2's
  dependency rule, 26 passes of 7 fused sweeps and 3 of 6).
* 16383 x 16383, 64 Fourier modes (seed 0), u0 = 0: 200 FP64 sweeps, and FP64
  refinement around 2 x 100 FP32 inner sweeps (and the bfloat16-rhs form).
  The relative residual is checked against the multi-mode closed form of
  Eq. (1)'s iteration: FP64 within 1e-12 relative; the refinement within
  the first-order rounding bound of closed_form.refinement_rel_bound (it
  equals plain sweeping in exact arithmetic).  Sampled points equal the
  oracle bit for bit (light cones, sampling.py), and the FP64 iterate equals
  the closed form at the same points.
"""
import sys

import numpy as np
import pytest

import workloads as W
from tests import closed_form as cf
from tests.sampling import sample_after_refinement, sample_after_sweeps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2607_01735_amd as rb  # noqa: E402

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def headline(oracle):
    """The 8191^2 workload and the oracle's 200 sweeps of it (every point)."""
    n, m = 8191, 200
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=0)
    say(f"oracle: {m} sweeps at n={n}")
    ref = W.zeros(n)
    oracle.sweep(ref, f, h, m)
    return n, m, h, f, ref


@pytest.mark.parametrize("kernel", ["plain", "auto"])
def test_headline_every_element_bitwise(headline, kernel):
    n, m, h, f, ref = headline
    say(f"full-grid parity n={n} sweeps={m} kernel={kernel}")
    ft = torch.from_numpy(f).to(DEV)
    ut = torch.zeros((n + 2, n + 2), dtype=torch.float64, device=DEV)
    info = rb.rbgs_solve(ut, ft, m, 0.0, check_every=m, h=h, kernel=kernel, timing=True)
    assert info["status"] == 0 and info["sweeps"] == m
    if kernel == "auto":  # the benchmark's launch: the persistent blocked kernel at depth 7
        assert info["timing"]["fuse"] == 7, info["timing"]
    got = ut.cpu().numpy()
    del ut, ft
    torch.cuda.empty_cache()
    diff = got.view(np.uint64) != ref.view(np.uint64)
    assert not diff.any(), f"{int(diff.sum())} elements differ, first at " \
                           f"{np.argwhere(diff)[0].tolist()}"
    _, rel = rb_free_residual(ref, f, h)
    assert info["rel_residual"] == pytest.approx(rel, rel=1e-13)


def rb_free_residual(u, f, h):
    """Relative residual in FP64 with NumPy (a check of the reported norm
    that needs no device)."""
    s = ((u[2:, 1:-1] + u[:-2, 1:-1]) + u[1:-1, 2:]) + u[1:-1, :-2]
    r = f[1:-1, 1:-1] - (s - 4.0 * u[1:-1, 1:-1]) / (h * h)
    return np.linalg.norm(r), np.linalg.norm(r) / np.linalg.norm(f[1:-1, 1:-1])


N2 = 16383
PTS2 = [(1, 1), (1, N2), (N2, 1), (N2, N2), (1024, 1025), (1025, 7), (8192, 8192),
        (16000, 333), (511, 16383), (12345, 6789)]


@pytest.fixture(scope="module")
def fourier16k():
    h = W.spacing(N2)
    say(f"fourier workload n={N2}")
    f = W.fourier_rhs(N2, seed=0)
    modes = cf.merge_modes(*W.fourier_modes(seed=0))
    return h, f, modes


def closed_form_at(n, modes, m, pts):
    """Closed-form iterate after m full sweeps at the given points."""
    h = W.spacing(n)
    out = []
    for (i, j) in pts:
        p = 2 * m - 1 if (i + j) % 2 == 0 else 2 * m
        v = 0.0
        for k, l, a in modes:
            s = np.sin(k * np.pi * i * h) * np.sin(l * np.pi * j * h)
            v += cf.fixed_point(n, k, l, a) * cf.one_minus_pow(n, k, l, p) * s
        out.append(v)
    return np.array(out)


def test_16383_fp64_closed_form_and_samples(oracle, fourier16k):
    h, f, modes = fourier16k
    m = 200
    say(f"n={N2} FP64 {m} sweeps")
    ft = torch.from_numpy(f).to(DEV)
    ut = torch.zeros_like(ft)
    info = rb.rbgs_solve(ut, ft, m, 0.0, check_every=m, h=h)
    assert info["status"] == 0 and info["sweeps"] == m
    expect = cf.multi_mode_rel(N2, modes, m)
    assert info["rel_residual"] == pytest.approx(expect, rel=1e-12)
    got = np.array([ut[p].item() for p in PTS2])
    del ut, ft
    torch.cuda.empty_cache()
    ref = sample_after_sweeps(oracle, W.zeros(N2), f, h, m, PTS2)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), (got, ref)
    cfv = closed_form_at(N2, modes, m, PTS2)
    scale = np.max(np.abs(cfv))
    assert np.max(np.abs(got - cfv)) <= 1e-11 * scale


@pytest.mark.parametrize("precision,unit", [("f32_ir", 2.0 ** -24), ("bf16rhs_ir", 2.0 ** -8)])
def test_16383_refinement_closed_form_and_samples(oracle, fourier16k, precision, unit):
    h, f, modes = fourier16k
    inner, outer = 100, 2
    say(f"n={N2} refinement {precision} {outer} x {inner}")
    ft = torch.from_numpy(f).to(DEV)
    ut = torch.zeros_like(ft)
    info = rb.rbgs_solve(ut, ft, inner * outer, 1e-300, check_every=inner, h=h,
                         precision=precision, inner_sweeps=inner)
    assert info["status"] == rb.rbgs.ENOCONV and info["outer_iters"] == outer
    assert info["sweeps"] == inner * outer
    expect = cf.multi_mode_rel(N2, modes, inner * outer)
    bound = cf.refinement_rel_bound([1.0, cf.multi_mode_rel(N2, modes, inner)], inner, unit)
    say(f"rel {info['rel_residual']!r} closed form {expect!r} bound {bound:.3e}")
    assert abs(info["rel_residual"] - expect) <= bound
    got = np.array([ut[p].item() for p in PTS2])
    del ut, ft
    torch.cuda.empty_cache()
    ref = sample_after_refinement(oracle, W.zeros(N2), f, h, inner, outer, PTS2,
                                  rhs_bf16=precision == "bf16rhs_ir")
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), (got, ref)
