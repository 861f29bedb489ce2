"""Reference U-Net for the learned initial guess (test infrastructure only).

Plain FP64 numpy: the forward pass, the hand-derived backward pass and an
Adam step of the network whose GPU kernels live in the library.  It is the
oracle for those kernels (per layer and end to end) and is itself pinned by
finite differences (tests/test_unet_ref.py).  Nothing here is imported by
the library.

Network (the build's reading of the learned-guess configuration; the paper
has no learned part):
  input   x0 = f / rms(f) on the N x N interior, 1 channel
  level l = 0..3 on grids of N_l = (N_{l-1} + 1)/F - 1 points, coarsening
          factor F = 2 (default) or 4
  encoder e_l = relu(conv(relu(conv(in_l))))   channels C = (16, 32, 64, 128)
          in_0 = x0, in_{l+1} = R(e_l)          R: averaging restriction,
          1-D weights (F - |d|)/F^2 for |d| < F (full weighting for F = 2)
  decoder d_3 = e_3; d_l = relu(conv(relu(conv([P(d_{l+1}), e_l]))))
          P: bilinear prolongation (= F^2 R^T), [., .] channel concatenation
  head    y = conv1x1(d_0) (no activation);  u0 = y * rms(f)
  convs are 3x3, stride 1, zero padding 1, with bias.
Loss: mean squared error against u*/rms(f) over the interior.

Layouts: activations are (channels, H, W) per sample; a conv weight is
(C_out, C_in, 3, 3) and its bias (C_out,).  Batches are loops over samples.
"""
import numpy as np

CHANNELS = (16, 32, 64, 128)


def conv3x3(x, w, b):
    """y[co,i,j] = b[co] + sum_{ci,a,c} w[co,ci,a,c] x[ci,i+a-1,j+c-1] (zero pad)."""
    cin, h, wd = x.shape
    xp = np.zeros((cin, h + 2, wd + 2))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((w.shape[0], h, wd))
    for a in range(3):
        for c in range(3):
            patch = xp[:, a:a + h, c:c + wd].reshape(cin, -1)
            y += (w[:, :, a, c] @ patch).reshape(-1, h, wd)
    return y + b[:, None, None]


def conv3x3_backward(x, w, dy):
    """Gradients of conv3x3 with respect to x, w and b, given dL/dy."""
    cin, h, wd = x.shape
    xp = np.zeros((cin, h + 2, wd + 2))
    xp[:, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    dyf = dy.reshape(dy.shape[0], -1)
    for a in range(3):
        for c in range(3):
            patch = xp[:, a:a + h, c:c + wd].reshape(cin, -1)
            dw[:, :, a, c] = dyf @ patch.T
            dxp[:, a:a + h, c:c + wd] += (w[:, :, a, c].T @ dyf).reshape(cin, h, wd)
    db = dyf.sum(axis=1)
    return dxp[:, 1:-1, 1:-1], dw, db


def _weights_1d(factor):
    """Offsets d = 1-F .. F-1 and their restriction weights (F - |d|)/F^2."""
    d = np.arange(1 - factor, factor)
    return d, (factor - np.abs(d)) / float(factor * factor)


def restrict(x, factor=2):
    """Restriction from (C, F n + F - 1, same) to (C, n, n): coarse point
    (I, J) sits on fine point (F I + F - 1, F J + F - 1) (0-based interior
    indices); separable weights (F - |d|)/F^2 per axis ((1,2,1)/4 for F = 2)."""
    c, nf, _ = x.shape
    if (nf + 1) % factor:
        raise ValueError("fine size must be F n + F - 1")
    nc = (nf + 1) // factor - 1
    d, w = _weights_1d(factor)
    out = np.zeros((c, nc, nc))
    for a, wa in zip(d, w):
        for bb, wb in zip(d, w):
            r0, c0 = factor - 1 + a, factor - 1 + bb
            out += wa * wb * x[:, r0:r0 + factor * nc:factor, c0:c0 + factor * nc:factor]
    return out


def restrict_transpose(y, nf, factor=2):
    """The adjoint of restrict: (C, n, n) -> (C, nf, nf)."""
    c, nc, _ = y.shape
    d, w = _weights_1d(factor)
    out = np.zeros((c, nf, nf))
    for a, wa in zip(d, w):
        for bb, wb in zip(d, w):
            r0, c0 = factor - 1 + a, factor - 1 + bb
            out[:, r0:r0 + factor * nc:factor, c0:c0 + factor * nc:factor] += wa * wb * y
    return out


def prolong(y, nf, factor=2):
    """Bilinear prolongation P = F^2 R^T from (C, n, n) to (C, nf, nf)."""
    return float(factor * factor) * restrict_transpose(y, nf, factor)


def init_params(channels=CHANNELS, seed=0):
    """He-normal weights, zero biases.  Returns a dict of FP64 arrays."""
    rng = np.random.default_rng(seed)
    p = {}

    def conv(name, cin, cout, k=3):
        std = np.sqrt(2.0 / (cin * k * k))
        p[name + ".w"] = rng.standard_normal((cout, cin, k, k)) * std
        p[name + ".b"] = np.zeros(cout)

    cin = 1
    for l, c in enumerate(channels):
        conv(f"enc{l}.0", cin, c)
        conv(f"enc{l}.1", c, c)
        cin = c
    for l in range(len(channels) - 2, -1, -1):
        conv(f"dec{l}.0", channels[l + 1] + channels[l], channels[l])
        conv(f"dec{l}.1", channels[l], channels[l])
    p["head.w"] = rng.standard_normal((1, channels[0], 1, 1)) * np.sqrt(1.0 / channels[0])
    p["head.b"] = np.zeros(1)
    return p


def param_names(channels=CHANNELS):
    names = []
    for l in range(len(channels)):
        names += [f"enc{l}.0", f"enc{l}.1"]
    for l in range(len(channels) - 2, -1, -1):
        names += [f"dec{l}.0", f"dec{l}.1"]
    names.append("head")
    return names


def _keep(x):
    return x


def forward(p, x0, channels=CHANNELS, factor=2, rnd=None):
    """Normalised network output y (N x N) for normalised input x0 (N x N);
    returns (y, cache) where cache holds what the backward pass needs.

    rnd (optional): a rounding applied to every stored activation (each
    layer's ReLU output, each restriction and prolongation), for comparing
    with an implementation that stores activations in a narrower format;
    the arithmetic itself stays FP64.  None keeps every value."""
    rnd = rnd or _keep
    L = len(channels)
    cache = {"x0": x0}
    inp = x0[None]
    enc = []
    for l in range(L):
        z0 = conv3x3(inp, p[f"enc{l}.0.w"], p[f"enc{l}.0.b"])
        a0 = rnd(np.maximum(z0, 0.0))
        z1 = conv3x3(a0, p[f"enc{l}.1.w"], p[f"enc{l}.1.b"])
        a1 = rnd(np.maximum(z1, 0.0))
        cache[f"enc{l}"] = (inp, z0, a0, z1)
        enc.append(a1)
        if l + 1 < L:
            inp = rnd(restrict(a1, factor))
    d = enc[-1]
    for l in range(L - 2, -1, -1):
        up = rnd(prolong(d, enc[l].shape[1], factor))
        cat = np.concatenate([up, enc[l]], axis=0)
        z0 = conv3x3(cat, p[f"dec{l}.0.w"], p[f"dec{l}.0.b"])
        a0 = rnd(np.maximum(z0, 0.0))
        z1 = conv3x3(a0, p[f"dec{l}.1.w"], p[f"dec{l}.1.b"])
        d = rnd(np.maximum(z1, 0.0))
        cache[f"dec{l}"] = (cat, z0, a0, z1, up.shape[0])
    y = np.tensordot(p["head.w"][0, :, 0, 0], d, axes=(0, 0)) + p["head.b"][0]
    cache["d0"] = d
    return y, cache


def backward(p, cache, dy, channels=CHANNELS, factor=2, rnd=None):
    """Gradients of a loss with dL/dy = dy with respect to every parameter.

    rnd (optional): a rounding applied to every stored activation gradient
    (the gradients reaching each layer's input, each restriction's output,
    and a skip connection's gradient once the path from the level below is
    added to it), matching forward's rnd; the arithmetic stays FP64."""
    rnd = rnd or _keep
    L = len(channels)
    g = {}
    d0 = cache["d0"]
    g["head.w"] = np.tensordot(dy, d0, axes=([0, 1], [1, 2]))[None, :, None, None]
    g["head.b"] = np.array([dy.sum()])
    grad_d = rnd(p["head.w"][0, :, 0, 0][:, None, None] * dy[None])
    denc = [0.0] * L  # gradients reaching e_l through the skip connections
    # the decoder ran from level L-2 down to 0: walk it back from level 0 up
    for l in range(0, L - 1):
        cat, z0, a0, z1, cup = cache[f"dec{l}"]
        dz1 = grad_d * (z1 > 0)
        da0, g[f"dec{l}.1.w"], g[f"dec{l}.1.b"] = conv3x3_backward(a0, p[f"dec{l}.1.w"], dz1)
        dz0 = rnd(da0) * (z0 > 0)
        dcat, g[f"dec{l}.0.w"], g[f"dec{l}.0.b"] = conv3x3_backward(cat, p[f"dec{l}.0.w"], dz0)
        dcat = rnd(dcat)
        dup, denc_l = dcat[:cup], dcat[cup:]
        denc[l] = denc[l] + denc_l
        # up = P(d_{l+1}) with P = F^2 R^T, so dL/dd_{l+1} = F^2 R(dup)
        grad_d = rnd(float(factor * factor) * restrict(dup, factor))
    denc[L - 1] = grad_d
    # encoder, from the bottom level up
    carry = None
    for l in range(L - 1, -1, -1):
        inp, z0, a0, z1 = cache[f"enc{l}"]
        da1 = denc[l] if carry is None else rnd(denc[l] + carry)
        dz1 = da1 * (z1 > 0)
        da0, g[f"enc{l}.1.w"], g[f"enc{l}.1.b"] = conv3x3_backward(a0, p[f"enc{l}.1.w"], dz1)
        dz0 = rnd(da0) * (z0 > 0)
        dinp, g[f"enc{l}.0.w"], g[f"enc{l}.0.b"] = conv3x3_backward(inp, p[f"enc{l}.0.w"], dz0)
        if l > 0:
            # inp = R(e_{l-1})
            carry = restrict_transpose(rnd(dinp), cache[f"enc{l - 1}"][1].shape[1], factor)
    return g


def mse_loss(y, target):
    diff = y - target
    return float(np.mean(diff * diff)), 2.0 * diff / diff.size


def normalise(f_interior):
    rms = float(np.sqrt(np.mean(f_interior * f_interior)))
    return f_interior / rms, rms


def adam_step(p, g, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of every parameter (bias-corrected)."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m." + k, np.zeros_like(p[k]))
        v = state.setdefault("v." + k, np.zeros_like(p[k]))
        m[...] = beta1 * m + (1 - beta1) * g[k]
        v[...] = beta2 * v + (1 - beta2) * g[k] * g[k]
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p
