"""The refinement's precision fallback on the GPU against the oracle's.

rbgs_solve with fallback=True widens the inner precision when it stops
helping (a residual value its right-hand-side format cannot hold: FP64
sweeps at once; an outer step after the first that leaves rel no lower:
bfloat16 rhs -> FP32 -> FP64 sweeps).  The oracle's
rbgs_ref_ir_solve_fallback applies the same rule; the iterate must agree
bit for bit, and the sweep count, outer steps and final precision exactly,
both through the graph-captured rounds and the host loop (timing on).
"""
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
PREC = {"f32_ir": 1, "bf16rhs_ir": 2}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check(oracle, u0, f, h, inner, cap, tol, precision, timing):
    ref = u0.copy()
    rc, outer, done, rel, prec = oracle.ir_solve_fallback(ref, f, h, inner, cap, tol,
                                                          rhs_bf16=precision == "bf16rhs_ir")
    ut = torch.from_numpy(u0.copy()).to(DEV)
    info = rb.rbgs_solve(ut, torch.from_numpy(f).to(DEV), cap, tol, check_every=inner, h=h,
                         precision=precision, inner_sweeps=inner, fallback=True, timing=timing)
    say(f"  oracle outer={outer} sweeps={done} prec={prec} rel={rel:.3e}; gpu {info}")
    assert (info["outer_iters"], info["sweeps"], info["precision"]) == (outer, done, prec)
    assert np.array_equal(ut.cpu().numpy(), ref)
    assert info["rel_residual"] == pytest.approx(rel, rel=1e-12)
    return info, prec


@pytest.mark.parametrize("precision", ["f32_ir", "bf16rhs_ir"])
@pytest.mark.parametrize("timing", [False, True])
def test_overflow_switches_to_fp64(oracle, precision, timing):
    n, inner, cap = 63, 50, 400
    say(f"fallback overflow {precision} timing={timing}")
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=1)
    u0 = W.random_ring(n, seed=2) * 1e36
    info, prec = check(oracle, u0, f, h, inner, cap, 1e-12, precision, timing)
    assert prec == 0 and info["outer_iters"] == 0


@pytest.mark.parametrize("precision", ["f32_ir", "bf16rhs_ir"])
@pytest.mark.parametrize("timing", [False, True])
def test_stall_widens_precision(oracle, precision, timing):
    n, inner, tol = 63, 2000, 1e-15
    say(f"fallback stall {precision} timing={timing}")
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=3)
    info, prec = check(oracle, W.zeros(n), f, h, inner, 200 * inner, tol, precision, timing)
    assert prec == 0 and info["status"] == 0 and info["rel_residual"] <= tol


def test_no_fallback_when_refinement_converges(oracle):
    """When every outer step helps, the fallback changes nothing: the same
    bits, steps and precision as without it."""
    n, inner, tol = 255, 4000, 1e-8
    say("fallback idle")
    h = W.spacing(n)
    f = W.sine_rhs(n)
    a = torch.zeros((n + 2, n + 2), dtype=torch.float64, device=DEV)
    b = torch.zeros_like(a)
    ft = torch.from_numpy(f).to(DEV)
    ia = rb.rbgs_solve(a, ft, 200000, tol, check_every=inner, h=h, precision="f32_ir",
                       inner_sweeps=inner, fallback=True)
    ib = rb.rbgs_solve(b, ft, 200000, tol, check_every=inner, h=h, precision="f32_ir",
                       inner_sweeps=inner)
    assert torch.equal(a, b) and ia == ib and ia["precision"] == 1 and ia["status"] == 0
