"""Pins of the reference U-Net (CPU): library correlation for the conv,
adjoint identities for restriction/prolongation, and finite differences for
the hand-written backward pass."""
import numpy as np
import pytest

from oracle import unet_ref as U

scipy_signal = pytest.importorskip("scipy.signal")


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 9, 7))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = U.conv3x3(x, w, b)
    for co in range(4):
        ref = sum(scipy_signal.correlate2d(x[ci], w[co, ci], mode="same", boundary="fill")
                  for ci in range(3)) + b[co]
        assert np.allclose(y[co], ref, rtol=1e-13, atol=1e-13)


def test_restrict_and_prolong_identities():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 15, 15))
    y = rng.standard_normal((2, 7, 7))
    # adjoint: <R x, y> = <x, R^T y>
    assert np.isclose(np.sum(U.restrict(x) * y), np.sum(x * U.restrict_transpose(y, 15)), rtol=1e-13)
    # weights sum to one: a constant restricts to itself
    assert np.allclose(U.restrict(np.full((1, 15, 15), 2.5)), 2.5)
    # prolongation injects coarse values at coinciding points and averages between
    p = U.prolong(y, 15)
    assert np.allclose(p[:, 1::2, 1::2], y)
    assert np.allclose(p[:, 1::2, 2:-1:2], 0.5 * (y[:, :, :-1] + y[:, :, 1:]))
    assert np.allclose(p[:, 2:-1:2, 2:-1:2],
                       0.25 * (y[:, :-1, :-1] + y[:, 1:, :-1] + y[:, :-1, 1:] + y[:, 1:, 1:]))


def test_factor_four_transfers():
    """F = 4: 1-D weights (1,2,3,4,3,2,1)/16, P = 16 R^T; both exact on
    linear functions (R at every coarse point, P between coarse points)."""
    rng = np.random.default_rng(5)
    nc, nf = 7, 31
    x = rng.standard_normal((2, nf, nf))
    y = rng.standard_normal((2, nc, nc))
    assert np.isclose(np.sum(U.restrict(x, 4) * y), np.sum(x * U.restrict_transpose(y, nf, 4)),
                      rtol=1e-13)
    assert np.allclose(U.restrict(np.full((1, nf, nf), -1.25), 4), -1.25)
    i = np.arange(nf, dtype=np.float64)
    lin = (0.3 + 0.7 * i[:, None] - 1.1 * i[None, :])[None]
    centres = 4 * np.arange(nc) + 3
    assert np.allclose(U.restrict(lin, 4)[0], lin[0][np.ix_(centres, centres)], rtol=0, atol=1e-12)
    coarse = lin[0][np.ix_(centres, centres)][None]
    p = U.prolong(coarse, nf, 4)
    inner = slice(3, 4 * (nc - 1) + 4)
    assert np.allclose(p[0, inner, inner], lin[0, inner, inner], rtol=0, atol=1e-12)
    # one coarse point: a pyramid of height 1 and base 7 x 7
    e = np.zeros((1, nc, nc))
    e[0, 2, 3] = 1.0
    p = U.prolong(e, nf, 4)
    tri = np.array([1, 2, 3, 4, 3, 2, 1]) / 4.0
    assert np.allclose(p[0, 8:15, 12:19], np.outer(tri, tri))
    assert np.isclose(p.sum(), 16.0)


def test_conv_backward_by_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 5, 6))
    w = rng.standard_normal((3, 2, 3, 3))
    b = rng.standard_normal(3)
    dy = rng.standard_normal((3, 5, 6))
    dx, dw, db = U.conv3x3_backward(x, w, dy)
    loss = lambda x_, w_, b_: float(np.sum(U.conv3x3(x_, w_, b_) * dy))
    eps = 1e-6
    for _ in range(10):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        assert np.isclose((loss(xp, w, b) - loss(xm, w, b)) / (2 * eps), dx[idx], rtol=1e-6, atol=1e-8)
        idx = tuple(rng.integers(0, s) for s in w.shape)
        wp, wm = w.copy(), w.copy()
        wp[idx] += eps
        wm[idx] -= eps
        assert np.isclose((loss(x, wp, b) - loss(x, wm, b)) / (2 * eps), dw[idx], rtol=1e-6, atol=1e-8)
    bp = b.copy()
    bp[1] += eps
    bm = b.copy()
    bm[1] -= eps
    assert np.isclose((loss(x, w, bp) - loss(x, w, bm)) / (2 * eps), db[1], rtol=1e-6)


@pytest.mark.parametrize("factor,n", [(2, 15), (4, 127)])
def test_network_gradient_by_finite_differences(factor, n):
    channels = (2, 3, 4, 5)
    p = U.init_params(channels, seed=3)
    rng = np.random.default_rng(4)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.1
    x0 = rng.standard_normal((n, n))
    target = rng.standard_normal((n, n))

    def loss_of(params):
        y, _ = U.forward(params, x0, channels, factor)
        return U.mse_loss(y, target)[0]

    y, cache = U.forward(p, x0, channels, factor)
    _, dy = U.mse_loss(y, target)
    g = U.backward(p, cache, dy, channels, factor)
    assert set(g) == set(p)
    eps = 1e-6
    checked = 0
    for k in sorted(p):
        flat = p[k].reshape(-1)
        for j in rng.choice(flat.size, size=min(3, flat.size), replace=False):
            pp = {kk: vv.copy() for kk, vv in p.items()}
            pm = {kk: vv.copy() for kk, vv in p.items()}
            pp[k].reshape(-1)[j] += eps
            pm[k].reshape(-1)[j] -= eps
            fd = (loss_of(pp) - loss_of(pm)) / (2 * eps)
            an = g[k].reshape(-1)[j]
            assert np.isclose(fd, an, rtol=1e-4, atol=1e-8), (k, j, fd, an)
            checked += 1
    assert checked > 40


def check_adam_first_step(mod):
    p = {"a": np.array([1.0, -2.0])}
    g = {"a": np.array([0.5, -0.25])}
    state = {}
    mod.adam_step(p, g, state, lr=0.1)
    # first bias-corrected Adam step is lr * sign(g)
    assert np.allclose(p["a"], [0.9, -1.9], atol=1e-7)


def check_adam_constant_gradient(mod):
    """With the same gradient g at every step, m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2, so the bias-corrected moments are exactly g and
    g^2 and every step moves the parameter by lr g / (|g| + eps), at every
    t, not only the first.  A wrong bias-correction exponent, a missing
    correction or swapped betas break this from t = 2 on."""
    lr, eps = 1e-2, 1e-8
    g0 = np.array([0.5, -0.25, 3e-3, -7.0, 1e-6])
    p = {"a": np.array([1.0, -2.0, 0.0, 4.0, -1.0])}
    state = {}
    for t in range(1, 9):
        before = p["a"].copy()
        mod.adam_step(p, {"a": g0.copy()}, state, lr=lr, eps=eps)
        step = before - p["a"]
        assert np.allclose(step, lr * g0 / (np.abs(g0) + eps), rtol=1e-9, atol=1e-15), t
    assert state["t"] == 8


def check_adam_sum_form(mod):
    """Varying gradients: the moments are the exponentially weighted sums
    m_t = (1 - b1) sum_s b1^(t-s) g_s and v_t = (1 - b2) sum_s b2^(t-s) g_s^2,
    each divided by its bias correction 1 - b^t; the update is
    lr m^ / (sqrt(v^) + eps) (Kingma and Ba, Algorithm 1)."""
    b1, b2, eps, lr = 0.9, 0.999, 1e-8, 3e-3
    rng = np.random.default_rng(5)
    gs = [rng.standard_normal(6) * 10.0 ** rng.uniform(-3, 1, 6) for _ in range(7)]
    p = {"a": rng.standard_normal(6)}
    expect = p["a"].copy()
    state = {}
    for t in range(1, len(gs) + 1):
        mod.adam_step(p, {"a": gs[t - 1].copy()}, state, lr=lr)
        m = (1 - b1) * sum(b1 ** (t - s) * gs[s - 1] for s in range(1, t + 1))
        v = (1 - b2) * sum(b2 ** (t - s) * gs[s - 1] ** 2 for s in range(1, t + 1))
        expect = expect - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        assert np.allclose(p["a"], expect, rtol=1e-12, atol=1e-15), t


def test_adam_step_moves_against_gradient():
    check_adam_first_step(U)


def test_adam_constant_gradient_every_step():
    check_adam_constant_gradient(U)


def test_adam_matches_weighted_sum_form():
    check_adam_sum_form(U)
