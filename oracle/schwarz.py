"""Restricted additive Schwarz with inexact deflated-GMRES subdomain solves (oracle).

Test infrastructure only.  Follows the paper step by step:

* Sec. 2, eq. 3: M^{-1} r = sum_j R_j^T D_j u_j where u_j solves the local system with
  right-hand side f_j = R_j r.  The local matrix is either the paper's Dirichlet
  restriction A_j = R_j A R_j^T or the impedance-interface matrix
  B_j = K_j - k^2 M_j - i k M_Gamma_j (the optimised, "ORAS", variant).
* Sec. 2, eq. 4 and Sec. 3: each local system is solved by GMRES on the deflated system
  P_j B_j x = P_j f_j to a relative tolerance, from a zero guess unless one is given;
  the local solution is recovered as u_j = Q_j f_j + x - Q_j B_j x.  The stopping test
  is ||P_j (f_j - B_j x)|| <= tol * ||P_j f_j||, relative to the zero-guess residual
  even when a guess is supplied (the paper only says "relative residual").
  A direct mode replaces the subdomain GMRES by a sparse LU solve (Sec. 3, Table 1), an
  "ilu" mode by GMRES preconditioned with ILU(0) (Sec. 3, Table 5; oracle/ilu.py).
* Sec. 3: the outer solver is FGMRES with relative tolerance 1e-6 from a zero guess.
  The outer count is the number of preconditioner applications; the average inner
  count is the total inner iterations over all subdomain solves of the run.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse.linalg as spla

from . import deflation as dfl
from . import fem
from . import krylov
from . import partition as part


@dataclass
class Problem:
    k: float
    n: int
    cuts_x: np.ndarray
    cuts_y: np.ndarray
    overlap: int = 1
    local_bc: str = part.ROBIN
    deflation: str = dfl.LINEAR


class Subdomain:
    def __init__(self, prob: Problem, geom: part.SubdomainGeometry, A=None):
        self.geom = geom
        if prob.local_bc == part.ROBIN:
            B, _ = fem.impedance_matrix(prob.k, prob.n, geom.ax, geom.bx, geom.ay, geom.by)
        else:
            B = A[geom.idx][:, geom.idx]
        self.B = B.tocsr()
        self.defl = dfl.Deflation(self.B, dfl.z2d(geom.nx, geom.ny, prob.deflation))
        self._lu = None
        self._ilu = None

    def direct(self, f: np.ndarray) -> np.ndarray:
        if self._lu is None:
            self._lu = spla.splu(self.B.tocsc())
        return self._lu.solve(f)

    def ilu_gmres(self, f: np.ndarray, tol: float, maxit: int):
        """ILU(0)-preconditioned GMRES local solve (Sec. 3, Table 5): (u, iterations)."""
        if self._ilu is None:
            from .ilu import Ilu0Solver
            self._ilu = Ilu0Solver(self.B)
        return self._ilu.solve(f, tol, maxit)

    def deflated_gmres(self, f: np.ndarray, tol: float, maxit: int, guess=None):
        """Inexact local solve; returns (u, iterations, accepted_guess)."""
        d = self.defl
        Pf = d.P(f)
        ref = np.linalg.norm(Pf)
        if ref == 0.0:
            return d.recover(f, np.zeros_like(f)), 0, False
        x0 = None
        accepted = False
        if guess is not None:
            # accept the guess only if it lowers the deflated residual
            if np.linalg.norm(Pf - d.PB(guess)) < ref:
                x0, accepted = guess, True
        res = krylov.gmres(d.PB, Pf, x0=x0, rtol=tol, maxit=maxit, ref_norm=ref)
        return d.recover(f, res.x), res.iters, accepted


@dataclass
class SolveStats:
    outer_iters: int = 0
    inner_iters: int = 0
    subdomain_solves: int = 0
    converged: bool = False
    history: list = field(default_factory=list)
    true_relres: float = float("nan")

    @property
    def avg_inner(self) -> float:
        return self.inner_iters / max(self.subdomain_solves, 1)


class Schwarz:
    """One-level restricted additive Schwarz preconditioner and the outer solver."""

    def __init__(self, prob: Problem):
        self.prob = prob
        self.A = fem.helmholtz_matrix(prob.k, prob.n)
        self.geoms = part.subdomains(prob.n, prob.cuts_x, prob.cuts_y, prob.overlap, prob.local_bc)
        self.subs = [Subdomain(prob, g, self.A) for g in self.geoms]

    @property
    def ndof(self) -> int:
        return self.A.shape[0]

    def local_rhs(self, r: np.ndarray):
        return [r[s.geom.idx] for s in self.subs]

    def scatter(self, us) -> np.ndarray:
        """z = sum_j R_j^T D_j u_j."""
        z = np.zeros(self.ndof, dtype=np.complex128)
        for s, u in zip(self.subs, us):
            g = s.geom
            z[g.idx[g.owned]] += u[g.owned]
        return z

    def local_solves(self, r, mode="deflated", tol=1e-2, maxit=200, guesses=None):
        us, its = [], []
        for j, (s, f) in enumerate(zip(self.subs, self.local_rhs(r))):
            if mode == "direct":
                us.append(s.direct(f))
                its.append(0)
            elif mode == "ilu":
                u, it = s.ilu_gmres(f, tol, maxit)
                us.append(u)
                its.append(it)
            else:
                g = None if guesses is None else guesses[j]
                u, it, _ = s.deflated_gmres(f, tol, maxit, g)
                us.append(u)
                its.append(it)
        return us, its

    def apply(self, r, mode="deflated", tol=1e-2, maxit=200, stats: SolveStats | None = None):
        """z = M^{-1} r (eq. 3) with direct or deflated-GMRES local solves."""
        us, its = self.local_solves(r, mode, tol, maxit)
        if stats is not None:
            stats.inner_iters += int(np.sum(its))
            stats.subdomain_solves += len(its)
        return self.scatter(us)

    def solve(self, f, mode="deflated", inner_tol=1e-2, inner_maxit=200,
              outer_tol=1e-6, outer_maxit=2000, restart=None):
        """Outer FGMRES (Sec. 3) preconditioned by ``apply``.  Returns (u, stats)."""
        stats = SolveStats()
        res = krylov.fgmres(lambda v: self.A @ v,
                            lambda v: self.apply(v, mode, inner_tol, inner_maxit, stats),
                            f, rtol=outer_tol, maxit=outer_maxit, restart=restart)
        stats.outer_iters = res.iters
        stats.converged = res.converged
        stats.history = res.history
        stats.true_relres = float(np.linalg.norm(f - self.A @ res.x) / np.linalg.norm(f))
        return res.x, stats


def problem_from_workload(w, local_bc=part.ROBIN, deflation=dfl.LINEAR) -> Problem:
    return Problem(w.k, w.n, np.asarray(w.cuts_x), np.asarray(w.cuts_y), w.overlap,
                   local_bc, deflation)
