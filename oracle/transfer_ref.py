"""Reference grid transfers for nested iteration (test infrastructure only).

Plain numpy definitions of the two vertex-centred transfers the library
uses to converge training targets for the learned initial guess (not a
part of the paper's method): a fine grid of N_f = 2 N_c + 1 interior points
per side and a coarse grid of N_c share the unit square, coarse point
(I, J) lying on fine point (2I, 2J) in natural indexing (ring at 0 and N+1).

  restrict: coarse[I, J] = sum_{a,b in -1..1} w_a w_b fine[2I+a, 2J+b] / 16,
            w = (1, 2, 1), for 1 <= I, J <= N_c; the coarse ring is zero.
  prolong:  fine[i, j] = bilinear interpolation of the coarse grid, ring
            included, at fine point (i, j), for 1 <= i, j <= N_f; the fine
            ring is copied from the argument `ring` (zero if None).

Pinned in tests/test_transfer_ref.py by exactness on bilinear functions,
the adjoint relation P = 4 R^T and agreement with the U-Net reference's
channel transfers.
"""
import numpy as np


def restrict(fine):
    """Full weighting of a natural-layout (N_f+2)^2 array to (N_c+2)^2."""
    nf = fine.shape[0] - 2
    if (nf - 1) % 2:
        raise ValueError("fine size must be 2 N_c + 1")
    nc = (nf - 1) // 2
    out = np.zeros((nc + 2, nc + 2))
    w = (1.0, 2.0, 1.0)
    for I in range(1, nc + 1):
        for J in range(1, nc + 1):
            s = 0.0
            for a in (-1, 0, 1):
                for b in (-1, 0, 1):
                    s += w[a + 1] * w[b + 1] * fine[2 * I + a, 2 * J + b]
            out[I, J] = s / 16.0
    return out


def prolong(coarse, ring=None):
    """Bilinear interpolation of a natural-layout (N_c+2)^2 array onto the
    interior of a (N_f+2)^2 array (N_f = 2 N_c + 1)."""
    nc = coarse.shape[0] - 2
    nf = 2 * nc + 1
    out = np.zeros((nf + 2, nf + 2)) if ring is None else np.array(ring, dtype=np.float64)
    for i in range(1, nf + 1):
        for j in range(1, nf + 1):
            # fine point (i, j) sits at coarse coordinates (i/2, j/2)
            I0, J0 = i // 2, j // 2
            ti, tj = (i % 2) * 0.5, (j % 2) * 0.5
            I1, J1 = min(I0 + 1, nc + 1), min(J0 + 1, nc + 1)
            out[i, j] = ((1 - ti) * (1 - tj) * coarse[I0, J0] + ti * (1 - tj) * coarse[I1, J0]
                         + (1 - ti) * tj * coarse[I0, J1] + ti * tj * coarse[I1, J1])
    return out
