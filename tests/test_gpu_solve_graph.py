"""The solve driver's rounds (check_every sweeps, the FP64 residual, a
device-side convergence test) run as a captured HIP graph with a converged
flag that stops later rounds' sweeps.  Its result must be the host loop's:
the same sweep count, the same residual and the same bits (the host loop is
what a solve with timing runs), and the oracle's solve for FP64."""
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


@pytest.mark.parametrize("kernel", ["plain", "blocked", "resident", "auto"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_graph_rounds_equal_host_loop(oracle, kernel, dtype):
    # FP32 iterates stall near a relative residual of 1e-5 at this size
    n, tol, check, cap = 63, (1e-6 if dtype == np.float64 else 1e-4), 100, 20000
    say(f"graph solve {kernel} {dtype.__name__}")
    h = W.spacing(n)
    f = W.sine_rhs(n).astype(dtype)
    u_graph, u_host = dev(W.zeros(n).astype(dtype)), dev(W.zeros(n).astype(dtype))
    a = rb.rbgs_solve(u_graph, dev(f), cap, tol, check_every=check, h=h, kernel=kernel)
    b = rb.rbgs_solve(u_host, dev(f), cap, tol, check_every=check, h=h, kernel=kernel,
                      timing=True)
    assert a["status"] == b["status"] == 0
    assert a["sweeps"] == b["sweeps"] and a["rel_residual"] == b["rel_residual"]
    assert np.array_equal(u_graph.cpu().numpy(), u_host.cpu().numpy())
    if dtype == np.float64:
        ref = W.zeros(n)
        rc, done, rel = oracle.solve(ref, f, h, cap, tol, check)
        assert rc == 0 and done == a["sweeps"]
        assert np.array_equal(u_graph.cpu().numpy(), ref)


@pytest.mark.parametrize("kernel", ["plain", "blocked"])
def test_graph_rounds_sweep_cap(kernel):
    """max_sweeps not a multiple of check_every: whole rounds in the graph,
    the rest in the host loop, as without the graph."""
    n = 63
    say(f"graph solve cap {kernel}")
    h = W.spacing(n)
    f = dev(W.sine_rhs(n))
    u_graph, u_host = dev(W.zeros(n)), dev(W.zeros(n))
    a = rb.rbgs_solve(u_graph, f, 2550, 1e-14, check_every=100, h=h, kernel=kernel)
    b = rb.rbgs_solve(u_host, f, 2550, 1e-14, check_every=100, h=h, kernel=kernel, timing=True)
    assert a["sweeps"] == b["sweeps"] == 2550
    assert a["status"] == b["status"] == rb.rbgs.ENOCONV
    assert a["rel_residual"] == b["rel_residual"]
    assert np.array_equal(u_graph.cpu().numpy(), u_host.cpu().numpy())


def test_graph_rounds_timeout_is_reported():
    """A tile that never publishes its progress inside a captured round: the
    bounded waits expire, every wave leaves, and the solve returns
    RBGS_ETIMEOUT instead of running on."""
    n = 255
    say("graph solve with a stalled tile")
    h = W.spacing(n)
    f = dev(W.sine_rhs(n))
    u = dev(W.zeros(n))
    with pytest.raises(rb.RbgsError) as e:
        rb.rbgs_solve(u, f, 400, 1e-12, check_every=20, h=h, kernel="blocked", fuse=2,
                      tile_rows=16, debug_stall_tile=3, debug_spin_limit=2000)
    assert e.value.status == rb.rbgs.ETIMEOUT
    # the library is usable afterwards
    u.zero_()
    # (from u = 0 the relative residual of this problem rises to 1.41, then falls
    # slowly: below 1.4 within 100 sweeps)
    info = rb.rbgs_solve(u, f, 400, 1.4, check_every=20, h=h, kernel="blocked")
    assert info["status"] == 0


@pytest.mark.parametrize("kernel,precision", [("plain", "f32_ir"), ("blocked", "f32_ir"),
                                              ("plain", "bf16rhs_ir"), ("resident", "f32_ir")])
def test_graph_refinement_equals_host_loop(oracle, kernel, precision):
    """Refinement steps (zero e, inner FP32 sweeps, correction, residual with
    r for the next step) captured as graph rounds: same outer steps, sweeps,
    residual and bits as the host loop and the oracle's refinement."""
    n, inner, tol = 63, 500, 1e-10
    say(f"graph refinement {kernel} {precision}")
    h = W.spacing(n)
    f = W.fourier_rhs(n, seed=4, count=8, kmax=8)
    a_u, b_u = dev(W.zeros(n)), dev(W.zeros(n))
    kw = dict(check_every=inner, h=h, precision=precision, inner_sweeps=inner, kernel=kernel)
    a = rb.rbgs_solve(a_u, dev(f), 40 * inner + 123, tol, **kw)
    b = rb.rbgs_solve(b_u, dev(f), 40 * inner + 123, tol, timing=True, **kw)
    assert a["status"] == b["status"] == 0
    assert a["outer_iters"] == b["outer_iters"] and a["sweeps"] == b["sweeps"]
    assert a["rel_residual"] == b["rel_residual"]
    assert np.array_equal(a_u.cpu().numpy(), b_u.cpu().numpy())
    ref = W.zeros(n)
    rc, outer, rel = oracle.ir_solve(ref, f, h, inner, 40, tol, rhs_bf16=precision == "bf16rhs_ir")
    assert rc == 0 and outer == a["outer_iters"]
    assert np.array_equal(a_u.cpu().numpy(), ref)


def test_oversized_round_runs_uncaptured(oracle):
    """check_every = 40 000 plain sweeps is more launches than one captured
    round may hold: the solve runs them launch by launch, same bits."""
    import workloads as W
    n = 31
    h = W.spacing(n)
    f = W.uniform_rhs(n, seed=4)
    ut = torch.from_numpy(W.zeros(n)).to("cuda")
    info = rb.rbgs_solve(ut, torch.from_numpy(f).to("cuda"), 40000, 1e-30, check_every=40000,
                         h=h, kernel="plain")
    assert info["sweeps"] == 40000
    ref = W.zeros(n)
    oracle.solve(ref, f, h, 40000, 1e-30, 40000)
    assert np.array_equal(ut.cpu().numpy(), ref)
