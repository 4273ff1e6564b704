"""Krylov subspace recycling for the subdomain solves across outer iterations (oracle;
test infrastructure only).

The paper's conclusions (Sec. 4) name recycling as a way to cut the inner iteration
counts further: every outer FGMRES iteration solves each deflated subdomain system
P_j B_j x = P_j f_j again, with the same matrix and a new right-hand side.  This module
carries a recycle space from one such solve to the next with GCRO-DR (Parks, de Sturler,
Mackey, Johnson and Maiti, "Recycling Krylov subspaces for sequences of linear systems",
SIAM J. Sci. Comput. 28, 2006), restated here for one matrix A and a sequence of b:

Recycle space: U (n x k) and C = A U with orthonormal columns (C^H C = I).
One solve of A x = b, stopping test ||b - A x|| <= tol * ref:
  1. x0 = U C^H b and r0 = b - C C^H b (the minimal-residual approximation from span U);
  2. Arnoldi on the projected operator (I - C C^H) A from v_1 = r0 / ||r0||, modified
     Gram-Schmidt: (I - C C^H) A V_m = V_{m+1} Hbar_m, with B_m = C^H A V_m;
  3. y minimises ||beta e_1 - Hbar_m y|| (Givens rotations, as in krylov.py); then
     x = x0 + V_m y - U B_m y, whose residual is V_{m+1}(beta e_1 - Hbar_m y): the
     minimal residual over x0 + span(U) + K_m((I - C C^H) A, r0).
New recycle space (after the solve): harmonic Ritz vectors of A over S = [U V_m].  With
A S = W G, W = [C V_{m+1}] (orthonormal columns), G = [[I, B_m], [0, Hbar_m]], the
harmonic Ritz pairs (theta, S p) satisfy (A S)^H (A S p - theta S p) = 0, i.e.
  G^H G p = theta G^H W^H S p;
the k pairs of smallest |theta| give P_k, U' = S P_k, and W G P_k = Q R (thin QR) gives
C = Q, U = U' R^{-1}.  Without a recycle space (the first solve) S = V_m, W = V_{m+1},
G = Hbar_m.  With `update=False` the space built after the first solve is kept.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .krylov import givens


@dataclass
class RecycleResult:
    x: np.ndarray
    iters: int
    converged: bool
    residual_estimate: float


class Recycler:
    """GCRO-DR solves of A x = b for one fixed operator A and a sequence of b."""

    def __init__(self, apply_op, k: int, update: bool = True):
        self.apply_op = apply_op
        self.k = k
        self.update = update
        self.U = None           # n x k
        self.C = None           # n x k, C = A U, orthonormal columns

    def solve(self, b: np.ndarray, tol: float, maxit: int, ref: float | None = None) -> RecycleResult:
        ref = np.linalg.norm(b) if ref is None else ref
        atol = tol * ref
        n = b.shape[0]
        have_u = self.U is not None
        if have_u:
            cb = self.C.conj().T @ b
            x0 = self.U @ cb
            r0 = b - self.C @ cb
        else:
            x0 = np.zeros(n, dtype=np.complex128)
            r0 = b.astype(np.complex128)
        beta = np.linalg.norm(r0)
        if beta <= atol:
            return RecycleResult(x0, 0, True, beta)
        kc = self.C.shape[1] if have_u else 0
        V = [r0 / beta]
        Hbar = np.zeros((maxit + 1, maxit), dtype=np.complex128)   # unrotated, kept for the update
        Bm = np.zeros((kc, maxit), dtype=np.complex128)
        R = np.zeros((maxit + 1, maxit), dtype=np.complex128)      # rotated copy
        cs = np.zeros(maxit)
        sn = np.zeros(maxit, dtype=np.complex128)
        g = np.zeros(maxit + 1, dtype=np.complex128)
        g[0] = beta
        m = 0
        converged = False
        breakdown = False
        while m < maxit:
            w = self.apply_op(V[m])
            if have_u:
                Bm[:, m] = self.C.conj().T @ w
                w = w - self.C @ Bm[:, m]
            for i in range(m + 1):
                Hbar[i, m] = np.vdot(V[i], w)
                w = w - Hbar[i, m] * V[i]
            hnext = np.linalg.norm(w)
            Hbar[m + 1, m] = hnext
            R[:m + 2, m] = Hbar[:m + 2, m]
            for i in range(m):
                a, bb = R[i, m], R[i + 1, m]
                R[i, m] = cs[i] * a + sn[i] * bb
                R[i + 1, m] = -np.conj(sn[i]) * a + cs[i] * bb
            c, s, r = givens(R[m, m], R[m + 1, m])
            cs[m], sn[m] = c, s
            R[m, m], R[m + 1, m] = r, 0.0
            g[m + 1] = -np.conj(s) * g[m]
            g[m] = c * g[m]
            m += 1
            if hnext == 0.0:
                converged = breakdown = True
                break
            V.append(w / hnext)   # v_{m+1}: also needed by the recycle-space update
            if abs(g[m]) <= atol:
                converged = True
                break
        y = np.zeros(m, dtype=np.complex128)
        for i in range(m - 1, -1, -1):
            y[i] = (g[i] - R[i, i + 1:m] @ y[i + 1:m]) / R[i, i]
        Vm = np.column_stack(V[:m])
        x = x0 + Vm @ y
        if have_u:
            x = x - self.U @ (Bm[:, :m] @ y)
        if (self.update or not have_u) and self.k > 0 and not breakdown:
            self._new_space(Vm, V[m], Hbar[:m + 1, :m], Bm[:, :m], have_u)
        return RecycleResult(x, m, converged, float(abs(g[m])))

    def _new_space(self, Vm, vnext, Hbar, Bm, have_u):
        """Harmonic Ritz vectors of A over [U V_m] for the k values of smallest modulus."""
        m = Vm.shape[1]
        Vm1 = np.column_stack([Vm, vnext])
        if have_u:
            kc = self.U.shape[1]
            S = np.column_stack([self.U, Vm])
            W = np.column_stack([self.C, Vm1])
            G = np.zeros((kc + m + 1, kc + m), dtype=np.complex128)
            G[:kc, :kc] = np.eye(kc)
            G[:kc, kc:] = Bm
            G[kc:, kc:] = Hbar
        else:
            S, W, G = Vm, Vm1, Hbar
        k = min(self.k, S.shape[1])
        lhs = G.conj().T @ G
        rhs = G.conj().T @ (W.conj().T @ S)
        theta, P = sla.eig(lhs, rhs)
        order = np.argsort(np.abs(theta))
        Pk = P[:, order[:k]]
        Unew = S @ Pk
        Q, Rq = np.linalg.qr(W @ (G @ Pk))
        self.C = Q
        self.U = sla.solve_triangular(Rq, Unew.T, trans="T", lower=False).T


class RecyclingSchwarz:
    """The one-level preconditioner of eq. 3 whose deflated subdomain GMRES solves (eq. 4)
    recycle: subdomain j keeps its own recycle space for P_j B_j across applications."""

    def __init__(self, S, k: int, update: bool = True):
        self.S = S
        self.rec = [Recycler(s.defl.PB, k, update) for s in S.subs]
        self.max_per_apply = []   # largest subdomain iteration count of each application

    def apply(self, r, tol=1e-2, maxit=200, stats=None):
        us, its = [], []
        for s, rec, f in zip(self.S.subs, self.rec, self.S.local_rhs(r)):
            d = s.defl
            Pf = d.P(f)
            ref = np.linalg.norm(Pf)
            if ref == 0.0:
                us.append(d.recover(f, np.zeros_like(f)))
                its.append(0)
                continue
            res = rec.solve(Pf, tol, maxit, ref)
            us.append(d.recover(f, res.x))
            its.append(res.iters)
        if stats is not None:
            stats.inner_iters += int(np.sum(its))
            stats.subdomain_solves += len(its)
        self.max_per_apply.append(int(np.max(its)))
        return self.S.scatter(us)

    def solve(self, f, inner_tol=1e-2, inner_maxit=200, outer_tol=1e-6, outer_maxit=2000):
        """Outer FGMRES (Sec. 3) preconditioned by ``apply``.  Returns (u, stats)."""
        from . import krylov
        from .schwarz import SolveStats
        stats = SolveStats()
        res = krylov.fgmres(lambda v: self.S.A @ v,
                            lambda v: self.apply(v, inner_tol, inner_maxit, stats),
                            f, rtol=outer_tol, maxit=outer_maxit)
        stats.outer_iters = res.iters
        stats.converged = res.converged
        stats.history = res.history
        stats.true_relres = float(np.linalg.norm(f - self.S.A @ res.x) / np.linalg.norm(f))
        return res.x, stats
