"""Two-level Schwarz with a global coarse space (oracle; test infrastructure only).

Sec. 4 names the step after the one-level method: add a coarse space on the global
level and combine it with the inexact subdomain solves of eq. 3, so that the outer
iteration count no longer grows with the number of subdomains.  The paper fixes
neither the coarse space nor how it is combined with the one-level preconditioner.
The readings taken here:

* Coarse grid: M coarse intervals per edge whose nodes are fine-grid nodes.  Coarse
  node c (c = 0..M) sits at fine index p_c = floor(c N / M + 1/2), so p_0 = 0,
  p_M = N, and consecutive spacings differ by at most one fine interval.  The interior
  coarse nodes c = 1..M-1 carry the unknowns (u = 0 on the boundary, as for A).
* Coarse space: Z_0 = Z^y kron Z^x (x fastest, as eq. 5), where column c of the 1D
  factor is the piecewise-linear hat of coarse node c sampled at the fine interior
  nodes: 1 at p_c, falling linearly to 0 at p_{c-1} and p_{c+1}.  With M = N/2 this is
  the linear interpolation of Sec. 2 (H = 2h) on the whole grid; with M = N it is the
  identity.
* Coarse operator: E_0 = Z_0^T A Z_0 (the Galerkin product of eq. 4, now of the global
  matrix), factored with a sparse LU; Q_0 = Z_0 E_0^{-1} Z_0^T.
* Combination: M^{-1} r = M_1^{-1} (r - A Q_0 r) + Q_0 r, with M_1^{-1} the one-level
  restricted Schwarz preconditioner of eq. 3 (inexact or direct local solves).  This is
  the deflation-type two-level form: the coarse correction is applied first and the
  subdomain solves act on the coarse-orthogonal residual, Z_0^T (r - A Q_0 r) = 0.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import krylov
from .schwarz import Schwarz, SolveStats


def coarse_nodes(n: int, m: int) -> np.ndarray:
    """Fine indices p_0..p_M of the coarse grid lines: p_c = floor(c N / M + 1/2)."""
    if m < 2 or m > n:
        raise ValueError(f"coarse intervals must lie in [2, N]; got M={m}, N={n}")
    c = np.arange(m + 1, dtype=np.int64)
    return (2 * c * n + m) // (2 * m)


def z1d(n: int, m: int) -> sp.csr_matrix:
    """(N-1) x (M-1) matrix of the coarse hats at the fine interior nodes 1..N-1."""
    p = coarse_nodes(n, m)
    rows, cols, vals = [], [], []
    for c in range(1, m):
        lo, mid, hi = int(p[c - 1]), int(p[c]), int(p[c + 1])
        for i in range(lo + 1, hi):
            w = (i - lo) / (mid - lo) if i <= mid else (hi - i) / (hi - mid)
            rows.append(i - 1)
            cols.append(c - 1)
            vals.append(w)
    return sp.coo_matrix((vals, (rows, cols)), shape=(n - 1, m - 1)).tocsr()


def z2d(n: int, m: int) -> sp.csr_matrix:
    """Z_0 = Z^y kron Z^x on the (N-1)^2 interior nodes, x fastest."""
    z = z1d(n, m)
    return sp.kron(z, z).tocsr()


class CoarseSpace:
    """Z_0, E_0 and Q_0 of the global coarse problem."""

    def __init__(self, A: sp.spmatrix, n: int, m: int):
        self.n, self.m = n, m
        self.A = A.tocsr()
        self.Z = z2d(n, m).astype(np.complex128)
        self.Zt = self.Z.T.tocsr()
        self.E = (self.Zt @ (self.A @ self.Z)).tocsc()
        self.lu = spla.splu(self.E)

    @property
    def ncoarse(self) -> int:
        return self.E.shape[0]

    def restrict(self, r: np.ndarray) -> np.ndarray:
        return self.Zt @ r

    def coarse_solve(self, t: np.ndarray) -> np.ndarray:
        return self.lu.solve(t)

    def Q(self, r: np.ndarray) -> np.ndarray:
        """Q_0 r = Z_0 E_0^{-1} Z_0^T r."""
        return self.Z @ self.coarse_solve(self.restrict(r))


class TwoLevel:
    """M^{-1} r = M_1^{-1} (r - A Q_0 r) + Q_0 r around a one-level ``Schwarz``."""

    def __init__(self, S: Schwarz, m: int):
        self.S = S
        self.coarse = CoarseSpace(S.A, S.prob.n, m)

    def correct(self, r: np.ndarray):
        """(q, w) with q = Q_0 r and w = r - A q, the residual the subdomain solves see."""
        q = self.coarse.Q(r)
        return q, r - self.S.A @ q

    def apply(self, r, mode="deflated", tol=1e-2, maxit=200, stats: SolveStats | None = None):
        q, w = self.correct(r)
        return self.S.apply(w, mode, tol, maxit, stats) + q

    def solve(self, f, mode="deflated", inner_tol=1e-2, inner_maxit=200,
              outer_tol=1e-6, outer_maxit=2000, restart=None):
        """Outer FGMRES (Sec. 3) preconditioned by the two-level ``apply``."""
        stats = SolveStats()
        A = self.S.A
        res = krylov.fgmres(lambda v: A @ v,
                            lambda v: self.apply(v, mode, inner_tol, inner_maxit, stats),
                            f, rtol=outer_tol, maxit=outer_maxit, restart=restart)
        stats.outer_iters = res.iters
        stats.converged = res.converged
        stats.history = res.history
        stats.true_relres = float(np.linalg.norm(f - A @ res.x) / np.linalg.norm(f))
        return res.x, stats
