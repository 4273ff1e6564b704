"""ILU(0)-preconditioned GMRES subdomain solves (oracle; test infrastructure only).

Sec. 3, Table 5: for perspective the paper repeats its 10-points-per-wavelength runs with
every subdomain system solved by GMRES preconditioned with the zero-fill incomplete LU
factorisation, ILU(0), to the same relative tolerance, and reports far higher inner
counts than with two-level deflation.

ILU(0) (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Sec. 10.3.2): L unit
lower triangular and U upper triangular, with the sparsity of the strictly lower and the
upper part of B, such that (L U)_{ij} = B_{ij} for every (i, j) in the pattern of B.  It
is computed row by row: entries of row i left of the diagonal are eliminated in column
order with the already finished rows, and every update that would fall outside the
pattern of row i is dropped.

Readings (the paper states only "GMRES preconditioned by ILU(0)" and the tolerance):
right preconditioning, so that the stopping test ||f - B x|| <= tol ||f|| is on the true
local residual as for the other local solvers; zero initial guess; no restart.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import krylov


def ilu0(B: sp.spmatrix):
    """(L, U) of ILU(0): L unit lower (diagonal stored), U upper, both CSR."""
    B = sp.csr_matrix(B, dtype=np.complex128)
    B.sort_indices()
    n = B.shape[0]
    rows = []          # finished rows: dict column -> value (L part below the diagonal, U part from it)
    for i in range(n):
        lo, hi = B.indptr[i], B.indptr[i + 1]
        row = dict(zip(B.indices[lo:hi].tolist(), B.data[lo:hi].tolist()))
        for k in sorted(c for c in row if c < i):
            piv = rows[k][k]
            if piv == 0:
                raise ZeroDivisionError(f"zero pivot in row {k}")
            row[k] = row[k] / piv
            lik = row[k]
            for j, ukj in rows[k].items():
                if j > k and j in row:
                    row[j] = row[j] - lik * ukj
        if row.get(i, 0) == 0:
            raise ZeroDivisionError(f"zero pivot in row {i}")
        rows.append(row)
    lr, lc, lv, ur, uc, uv = [], [], [], [], [], []
    for i, row in enumerate(rows):
        for j, v in row.items():
            if j < i:
                lr.append(i); lc.append(j); lv.append(v)
            else:
                ur.append(i); uc.append(j); uv.append(v)
        lr.append(i); lc.append(i); lv.append(1.0)
    L = sp.csr_matrix((lv, (lr, lc)), shape=(n, n), dtype=np.complex128)
    U = sp.csr_matrix((uv, (ur, uc)), shape=(n, n), dtype=np.complex128)
    return L, U


class Ilu0Solver:
    """GMRES on B x = f right-preconditioned by ILU(0) of B."""

    def __init__(self, B: sp.spmatrix):
        self.B = sp.csr_matrix(B)
        self.L, self.U = ilu0(self.B)

    def precondition(self, r: np.ndarray) -> np.ndarray:
        """(L U)^{-1} r by forward and backward substitution."""
        y = spla.spsolve_triangular(self.L, r, lower=True, unit_diagonal=True)
        return spla.spsolve_triangular(self.U, y, lower=False)

    def solve(self, f: np.ndarray, tol: float, maxit: int):
        """(x, iterations) with ||f - B x|| <= tol ||f|| (estimate), or maxit reached."""
        if np.linalg.norm(f) == 0.0:
            return np.zeros_like(f), 0
        res = krylov.fgmres(lambda v: self.B @ v, self.precondition, f, rtol=tol, maxit=maxit)
        return res.x, res.iters
