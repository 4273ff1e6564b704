"""Two-level deflation of a subdomain system (oracle; test infrastructure only).

Sec. 2, eq. 4: the deflated subdomain system is P A x = P f with
    P = I - A Q,   Q = Z E^{-1} Z^T,   E = Z^T A Z,
where the columns of the deflation matrix Z span a coarse space.

1D deflation matrices (n fine nodes, m = floor(n/2) coarse nodes, coarse node c sits on
fine node 2c+1, 0-based; stencil entries falling outside the tile are dropped):
* ``linear``: linear interpolation from a grid of spacing H = 2h, column c holds
  1/2, 1, 1/2 on fine rows 2c, 2c+1, 2c+2;
* ``bezier``: the quadratic rational Bezier stencil of Sec. 2, 1/8 [1 4 6 4 1] on fine
  rows 2c-1 .. 2c+3.  The paper prints the map from fine values to coarse values,
  which is Z^T; it states Z is n x n/2, so the printed formula is read as the
  restriction and Z is its transpose.

2D (eq. 5): Z = Z^y kron Z^x with x running fastest.
E is factored with a dense LU (scipy.linalg.lu_factor, partial pivoting).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

LINEAR = "linear"
BEZIER = "bezier"


def z1d(n: int, kind: str = LINEAR) -> sp.csr_matrix:
    m = n // 2
    if m < 1:
        raise ValueError("a deflation direction needs at least two fine nodes")
    if kind == LINEAR:
        offs, w = (-1, 0, 1), (0.5, 1.0, 0.5)
    elif kind == BEZIER:
        offs, w = (-2, -1, 0, 1, 2), (1 / 8, 4 / 8, 6 / 8, 4 / 8, 1 / 8)
    else:
        raise ValueError(kind)
    rows, cols, vals = [], [], []
    for c in range(m):
        centre = 2 * c + 1
        for o, v in zip(offs, w):
            r = centre + o
            if 0 <= r < n:
                rows.append(r)
                cols.append(c)
                vals.append(v)
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, m)).tocsr()


def z2d(nx: int, ny: int, kind: str = LINEAR) -> sp.csr_matrix:
    """Z = Z^y kron Z^x (eq. 5), lexicographic with x fastest."""
    return sp.kron(z1d(ny, kind), z1d(nx, kind)).tocsr()


class Deflation:
    """P, Q and E of eq. 4 for one subdomain matrix B and deflation matrix Z."""

    def __init__(self, B: sp.spmatrix, Z: sp.spmatrix):
        self.B = B.tocsr()
        self.Z = Z.tocsr().astype(np.complex128)
        self.Zt = self.Z.T.tocsr()
        self.E = (self.Zt @ (self.B @ self.Z)).toarray()
        self.lu = sla.lu_factor(self.E)

    @property
    def ncoarse(self) -> int:
        return self.E.shape[0]

    def coarse_solve(self, t: np.ndarray) -> np.ndarray:
        return sla.lu_solve(self.lu, t)

    def Q(self, v: np.ndarray) -> np.ndarray:
        """Q v = Z E^{-1} Z^T v."""
        return self.Z @ self.coarse_solve(self.Zt @ v)

    def P(self, v: np.ndarray) -> np.ndarray:
        """P v = v - B Q v."""
        return v - self.B @ self.Q(v)

    def PB(self, v: np.ndarray) -> np.ndarray:
        """The deflated operator P B v."""
        return self.P(self.B @ v)

    def recover(self, f: np.ndarray, x: np.ndarray) -> np.ndarray:
        """Subdomain solution from a solution x of the deflated system.

        u = Q f + x - Q B x, which satisfies f - B u = P (f - B x), so the deflated
        residual is the true residual of u.  The paper does not print this step.
        """
        return self.Q(f) + x - self.Q(self.B @ x)
