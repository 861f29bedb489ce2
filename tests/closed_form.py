"""Closed forms and textbook solvers that pin the oracle (test helpers).

Everything here is derived from the mathematics of Eq. (1) (Section 2), not
from the oracle's code, so a dropped term, a wrong sign or a swapped colour
in the oracle makes one of these disagree.

Notation: N interior points per side, h = 1/(N+1), s_kl(i, j) =
sin(k pi i h) sin(l pi j h).  Neighbour sum identity: the four neighbours of
s_kl at any interior point sum to 4 mu_kl s_kl with
mu_kl = (cos(k pi h) + cos(l pi h)) / 2, and s_kl vanishes on the ring.

Gauss-Seidel with red-black ordering on f = A s_kl from u = 0 keeps the
ansatz "alpha s on red points, beta s on black points":
  red:   alpha' = mu beta  - h^2 A / 4
  black: beta'  = mu alpha' - h^2 A / 4
Fixed point a* = -(h^2 A / 4) / (1 - mu) = A / lambda_kl with
lambda_kl = -(4/h^2)(sin^2(k pi h/2) + sin^2(l pi h/2)); the error of each
colour is multiplied by mu per half-sweep, so after m full sweeps
  red   alpha_m = a* (1 - mu^(2m-1)),   black beta_m = a* (1 - mu^(2m)).
After full sweep m the residual vanishes on black points and equals
A mu^(2m-1) (1 + mu) s_kl on red points.
"""
import numpy as np


def spacing(n):
    return 1.0 / (n + 1)


def mode(n, k, l):
    """s_kl on the natural (n+2) x (n+2) grid (ring included, where it is 0)."""
    x = np.arange(n + 2, dtype=np.float64) * spacing(n)
    return np.outer(np.sin(k * np.pi * x), np.sin(l * np.pi * x))


def colour_masks(n):
    i, j = np.meshgrid(np.arange(n + 2), np.arange(n + 2), indexing="ij")
    interior = (i >= 1) & (i <= n) & (j >= 1) & (j <= n)
    red = interior & ((i + j) % 2 == 0)
    black = interior & ((i + j) % 2 == 1)
    return red, black


def one_minus_mu(n, k, l):
    """1 - mu_kl = sin^2(k pi h/2) + sin^2(l pi h/2), free of cancellation."""
    h = spacing(n)
    return np.sin(k * np.pi * h / 2) ** 2 + np.sin(l * np.pi * h / 2) ** 2


def one_minus_pow(n, k, l, p):
    """1 - mu_kl^p without cancellation when mu_kl is close to 1."""
    d = one_minus_mu(n, k, l)
    if d < 1.0:
        return -np.expm1(p * np.log1p(-d))
    return 1.0 - (1.0 - d) ** p


def mu_of(n, k, l):
    return 1.0 - one_minus_mu(n, k, l) if one_minus_mu(n, k, l) < 0.5 else \
        0.5 * (np.cos(k * np.pi * spacing(n)) + np.cos(l * np.pi * spacing(n)))


def fixed_point(n, k, l, amp):
    """a*_kl = -(h^2 A / 4) / (1 - mu_kl), written via sin^2 to avoid the
    cancellation in 1 - mu: 1 - mu = sin^2(k pi h/2) + sin^2(l pi h/2)."""
    h = spacing(n)
    return -(h * h * amp / 4.0) / one_minus_mu(n, k, l)


def iterate(n, modes, m, half=False):
    """Closed-form iterate after m full sweeps (half=True: after the red half
    of sweep m, i.e. red done m times and black m-1 times), from u = 0 with a
    zero ring, for f = sum A s_kl.  modes: iterable of (k, l, A)."""
    red, black = colour_masks(n)
    u = np.zeros((n + 2, n + 2))
    for k, l, a in modes:
        astar = fixed_point(n, k, l, a)
        alpha = astar * one_minus_pow(n, k, l, 2 * m - 1)
        beta = astar * one_minus_pow(n, k, l, 2 * m - 2 if half else 2 * m)
        s = mode(n, k, l)
        u = u + np.where(red, alpha * s, 0.0) + np.where(black, beta * s, 0.0)
    return u


def residual_field(n, modes, m):
    """Closed-form residual after m full sweeps: A mu^(2m-1)(1+mu) s on red
    points, zero on black points."""
    red, _ = colour_masks(n)
    r = np.zeros((n + 2, n + 2))
    for k, l, a in modes:
        mu = mu_of(n, k, l)
        r = r + np.where(red, a * mu ** (2 * m - 1) * (1.0 + mu) * mode(n, k, l), 0.0)
    return r


def rhs(n, modes):
    f = np.zeros((n + 2, n + 2))
    for k, l, a in modes:
        f = f + a * mode(n, k, l)
    f[0, :] = f[-1, :] = f[:, 0] = f[:, -1] = 0.0
    return f


def single_mode_rel(n, m):
    """rel residual after m >= 1 full sweeps for f = 2 pi^2 s_11 and odd n >= 3:
    c^(2m-1)(1+c)/sqrt(2) with c = cos(pi h) (each colour carries half of
    ||s_11||^2 when n is odd)."""
    c = np.cos(np.pi * spacing(n))
    return c ** (2 * m - 1) * (1.0 + c) / np.sqrt(2.0)


def multi_mode_rel(n, modes, m):
    """rel residual after m full sweeps using orthogonality of distinct modes
    with k, l < (n+1)/2 on each colour: each colour carries half of every
    ||s_kl||^2 and all ||s_kl||^2 are equal.  Duplicate (k, l) must be merged
    first (merge_modes)."""
    num = 0.0
    den = 0.0
    for k, l, a in modes:
        mu = mu_of(n, k, l)
        num += a * a * mu ** (2 * (2 * m - 1)) * (1.0 + mu) ** 2 / 2.0
        den += a * a
    return np.sqrt(num) / np.sqrt(den)


def merge_modes(k, l, a):
    acc = {}
    for kk, ll, aa in zip(k, l, a):
        acc[(int(kk), int(ll))] = acc.get((int(kk), int(ll)), 0.0) + float(aa)
    return [(kk, ll, aa) for (kk, ll), aa in sorted(acc.items())]


def dense_matrix(n):
    """A_h as an explicit (n^2 x n^2) matrix over the interior, row-major."""
    h2 = spacing(n) ** 2
    size = n * n
    a = np.zeros((size, size))
    for i in range(n):
        for j in range(n):
            p = i * n + j
            a[p, p] = -4.0 / h2
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < n and 0 <= jj < n:
                    a[p, ii * n + jj] = 1.0 / h2
    return a


def ring_rhs(u_ring, f):
    """Right-hand side of the interior system A u_int = b: b = f minus the
    ring neighbours' contribution divided by h^2."""
    n = f.shape[0] - 2
    h2 = spacing(n) ** 2
    g = np.zeros((n, n))
    g[0, :] += u_ring[0, 1:n + 1]
    g[-1, :] += u_ring[n + 1, 1:n + 1]
    g[:, 0] += u_ring[1:n + 1, 0]
    g[:, -1] += u_ring[1:n + 1, n + 1]
    return f[1:n + 1, 1:n + 1] - g / h2


def dense_solve(f, u_ring=None):
    """Exact discrete solution by a dense LU solve (textbook), natural layout."""
    n = f.shape[0] - 2
    b = ring_rhs(u_ring, f) if u_ring is not None else f[1:n + 1, 1:n + 1]
    x = np.linalg.solve(dense_matrix(n), b.reshape(-1)).reshape(n, n)
    out = np.zeros((n + 2, n + 2)) if u_ring is None else u_ring[:, :n + 2].copy()
    out[1:n + 1, 1:n + 1] = x
    return out


def dst_solve(f):
    """Exact discrete solution for a zero ring through the DST-I, which
    diagonalises A_h with eigenvalues lambda_kl."""
    from scipy.fft import dstn, idstn
    n = f.shape[0] - 2
    h = spacing(n)
    k = np.arange(1, n + 1)
    lam1 = -(4.0 / h ** 2) * np.sin(k * np.pi * h / 2) ** 2
    lam = lam1[:, None] + lam1[None, :]
    fh = dstn(f[1:n + 1, 1:n + 1], type=1)
    x = idstn(fh / lam, type=1)
    out = np.zeros((n + 2, n + 2))
    out[1:n + 1, 1:n + 1] = x
    return out


def refinement_rel_bound(rels, inner, rhs_unit, unit=2.0 ** -24, ops=5):
    """First-order bound on how far the relative residual of FP64
    refinement around low-precision inner sweeps may drift from plain FP64
    Gauss-Seidel after the same total number of sweeps.

    In exact arithmetic an outer step (r = f - A u; e = s sweeps from 0 on
    A e = r; u += e) equals s more sweeps on u: with the sweep operator
    M = I - N A, sum_{j<s} M^j N A = I - M^s, so u + sum M^j N (f - A u) =
    M^s u + sum M^j N f.  Rounding enters twice per step: r is stored with
    unit roundoff rhs_unit (an error of at most rhs_unit ||r|| that the
    step passes on to the new residual through I - M^s, counted twice), and
    the inner sweeps round every update with unit roundoff `unit` (e after
    s sweeps is about s h^2 |r| / 2 for the smooth modes, A amplifies by at
    most 8/h^2, and each update has `ops` rounded operations: 4 ops s unit
    ||r||).  rels: relative residual before each outer step."""
    return sum((2.0 * rhs_unit + 4.0 * ops * inner * unit) * r for r in rels)
