"""GMRES and flexible GMRES (oracle; test infrastructure only).

Both use the Arnoldi process with modified Gram-Schmidt under the Hermitian inner
product, and complex Givens rotations to keep the least-squares residual estimate
|g_{k+1}|.  The paper (Sec. 3) runs preconditioned GMRES on every subdomain system and
an outer flexible GMRES, which is required because the inexact subdomain solves make
the preconditioner change from one outer iteration to the next; it does not state
restart lengths or the orthogonalisation scheme.

Givens rotation zeroing b in (a, b)^T with b real:
    c = |a| / t,  s = (a/|a|) conj(b) / t,  t = sqrt(|a|^2 + |b|^2),
    G = [[c, s], [-conj(s), c]].
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def givens(a: complex, b: complex):
    """(c, s, r) with [[c, s], [-conj(s), c]] @ [a, b] = [r, 0]."""
    if b == 0:
        return 1.0, 0.0 + 0.0j, a
    if a == 0:
        return 0.0, np.conj(b) / abs(b), abs(b)
    t = np.hypot(abs(a), abs(b))
    ph = a / abs(a)
    return abs(a) / t, ph * np.conj(b) / t, ph * t


@dataclass
class KrylovResult:
    x: np.ndarray
    iters: int
    history: list = field(default_factory=list)   # residual estimates |g_k|, k = 0..iters
    converged: bool = False


def _arnoldi_solve(apply_op, precond, b, x0, atol, maxit, flexible):
    n = b.shape[0]
    r0 = b.copy() if x0 is None else b - apply_op(x0)
    x0 = np.zeros(n, dtype=np.complex128) if x0 is None else x0.astype(np.complex128)
    beta = np.linalg.norm(r0)
    hist = [beta]
    if beta <= atol:
        return KrylovResult(x0, 0, hist, True)
    V = [r0 / beta]
    Zs = []
    H = np.zeros((maxit + 1, maxit), dtype=np.complex128)
    cs = np.zeros(maxit)
    sn = np.zeros(maxit, dtype=np.complex128)
    g = np.zeros(maxit + 1, dtype=np.complex128)
    g[0] = beta
    k = 0
    converged = False
    while k < maxit:
        z = precond(V[k]) if flexible else V[k]
        if flexible:
            Zs.append(z)
        w = apply_op(z)
        for i in range(k + 1):                 # modified Gram-Schmidt
            H[i, k] = np.vdot(V[i], w)
            w = w - H[i, k] * V[i]
        hnext = np.linalg.norm(w)
        H[k + 1, k] = hnext
        for i in range(k):                     # previous rotations
            a, bb = H[i, k], H[i + 1, k]
            H[i, k] = cs[i] * a + sn[i] * bb
            H[i + 1, k] = -np.conj(sn[i]) * a + cs[i] * bb
        c, s, r = givens(H[k, k], H[k + 1, k])
        cs[k], sn[k] = c, s
        H[k, k], H[k + 1, k] = r, 0.0
        g[k + 1] = -np.conj(s) * g[k]
        g[k] = c * g[k]
        k += 1
        hist.append(abs(g[k]))
        if abs(g[k]) <= atol:
            converged = True
            break
        if hnext == 0.0:                       # lucky breakdown: exact in the Krylov space
            converged = True
            break
        V.append(w / hnext)
    y = np.zeros(k, dtype=np.complex128)
    for i in range(k - 1, -1, -1):             # back substitution with R = H[:k, :k]
        y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    basis = Zs if flexible else V
    x = x0.copy()
    for i in range(k):
        x = x + y[i] * basis[i]
    return KrylovResult(x, k, hist, converged)


def gmres(apply_op, b, x0=None, rtol=1e-6, maxit=200, ref_norm=None):
    """GMRES (no restart) for apply_op(x) = b.

    Stops when the residual estimate is <= rtol * ref_norm (default: ||b||).
    """
    ref = np.linalg.norm(b) if ref_norm is None else ref_norm
    return _arnoldi_solve(apply_op, None, b, x0, rtol * ref, maxit, flexible=False)


def fgmres(apply_op, precond, b, rtol=1e-6, maxit=1000, restart=None):
    """Right-preconditioned flexible GMRES from a zero initial guess.

    Stops when the residual estimate is <= rtol * ||b||.  ``iters`` counts the
    preconditioner applications over all restart cycles.
    """
    ref = np.linalg.norm(b)
    restart = maxit if restart is None else restart
    x = np.zeros(b.shape[0], dtype=np.complex128)
    total, hist = 0, []
    first = True
    while total < maxit:
        res = _arnoldi_solve(apply_op, precond, b, None if first else x, rtol * ref,
                             min(restart, maxit - total), flexible=True)
        x = res.x
        total += res.iters
        hist.extend(res.history if first else res.history[1:])
        first = False
        if res.converged:
            return KrylovResult(x, total, hist, True)
    return KrylovResult(x, total, hist, False)
