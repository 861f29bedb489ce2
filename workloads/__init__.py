"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

This module holds input generation only: right-hand sides f, Dirichlet
rings and batch size draws, all on the host in FP64 from numpy's
default_rng.  It contains none of the solver's arithmetic.  Every array is
in the natural layout: (n+2) x ld, row-major, ring included; the interior is
rows/columns 1..n and the grid spacing is h = 1/(n+1) (Section 2).
Lower-precision forms are obtained by the caller with a round-to-nearest cast.
"""
import numpy as np


def spacing(n):
    """h = 1/(N+1) for N interior points per side (Section 2)."""
    return 1.0 / (n + 1)


def coords(n):
    """Interior coordinates x_i = i*h, i = 0..n+1 (ring included)."""
    return np.arange(n + 2, dtype=np.float64) * spacing(n)


def _embed(interior, ld=None):
    n = interior.shape[0]
    ld = n + 2 if ld is None else ld
    a = np.zeros((n + 2, ld), np.float64)
    a[1:n + 1, 1:n + 1] = interior
    return a


def zeros(n, ld=None, dtype=np.float64):
    ld = n + 2 if ld is None else ld
    return np.zeros((n + 2, ld), dtype)


def sine_rhs(n, ld=None):
    """f = 2 pi^2 sin(pi x) sin(pi y) on the interior; ring zero."""
    x = coords(n)
    s = np.sin(np.pi * x)
    f = 2.0 * np.pi ** 2 * np.outer(s, s)
    out = zeros(n, ld)
    out[1:n + 1, 1:n + 1] = f[1:n + 1, 1:n + 1]
    return out


def uniform_rhs(n, seed=0, ld=None, lo=-1.0, hi=1.0):
    """f_ij i.i.d. uniform on [lo, hi) from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return _embed(rng.uniform(lo, hi, size=(n, n)), ld)


def normal_rhs(n, seed=0, ld=None):
    """f_ij i.i.d. standard normal from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return _embed(rng.standard_normal(size=(n, n)), ld)


def fourier_modes(seed=0, count=64, kmax=64):
    """count random modes: (k, l) uniform on {1..kmax}^2 and amplitudes
    N(0,1)/(k^2+l^2).  Returned as (k, l, A) arrays, in draw order."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, kmax + 1, size=count)
    l = rng.integers(1, kmax + 1, size=count)
    a = rng.standard_normal(size=count) / (k.astype(np.float64) ** 2 + l.astype(np.float64) ** 2)
    return k, l, a


def fourier_rhs(n, seed=0, count=64, kmax=64, ld=None):
    """f = sum_m A_m sin(k_m pi x) sin(l_m pi y) over fourier_modes(seed)."""
    k, l, a = fourier_modes(seed, count, kmax)
    x = coords(n)[1:n + 1]
    sk = np.sin(np.pi * np.outer(k, x))  # (count, n)
    sl = np.sin(np.pi * np.outer(l, x))
    f = (sk * a[:, None]).T @ sl          # sum_m A_m sk_m(x_i) sl_m(y_j)
    return _embed(f, ld)


def grf_rhs(n, seed=0, ld=None, length_scale=None):
    """Gaussian random field on the interior, normalised to unit RMS.

    Squared-exponential field through its sine-series spectral density:
    f = sum_{k,l<=n} xi_kl exp(-pi^2 ls^2 (k^2+l^2)/4) sin(k pi x) sin(l pi y),
    xi ~ N(0,1); the length scale ls ~ U[0.02, 0.3] is drawn first from the
    same generator unless given.  Returns (f, ls)."""
    rng = np.random.default_rng(seed)
    ls = rng.uniform(0.02, 0.3) if length_scale is None else float(length_scale)
    k = np.arange(1, n + 1, dtype=np.float64)
    amp = np.exp(-np.pi ** 2 * ls ** 2 * k ** 2 / 4.0)
    keep = amp > 1e-12 * amp[0]
    kk = k[keep]
    xi = rng.standard_normal(size=(kk.size, kk.size))
    coef = xi * np.outer(amp[keep], amp[keep])
    x = coords(n)[1:n + 1]
    s = np.sin(np.pi * np.outer(kk, x))     # (K, n)
    f = s.T @ coef @ s
    f = f / np.sqrt(np.mean(f * f))
    return _embed(f, ld), ls


def random_ring(n, seed=0, ld=None, scale=1.0):
    """A grid whose ring holds i.i.d. uniform Dirichlet data and whose
    interior is zero: a starting u with nonzero g."""
    rng = np.random.default_rng(seed)
    a = zeros(n, ld)
    a[0, :n + 2] = rng.uniform(-scale, scale, n + 2)
    a[n + 1, :n + 2] = rng.uniform(-scale, scale, n + 2)
    a[1:n + 1, 0] = rng.uniform(-scale, scale, n)
    a[1:n + 1, n + 1] = rng.uniform(-scale, scale, n)
    return a


def random_start(n, seed=0, ld=None):
    """A random starting iterate: interior i.i.d. uniform[-1, 1), ring zero."""
    return uniform_rhs(n, seed, ld)


BATCH_SIZES = (63, 127, 255, 511, 1023)


def batch_sizes(count=512, seed=0, choices=BATCH_SIZES):
    """Interior sizes drawn uniformly from choices with default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return [int(choices[i]) for i in rng.integers(0, len(choices), size=count)]


def batch_rhs(sizes, first_seed=1):
    """f for grid g is normal_rhs(sizes[g], seed=first_seed + g)."""
    return [normal_rhs(n, first_seed + g) for g, n in enumerate(sizes)]
