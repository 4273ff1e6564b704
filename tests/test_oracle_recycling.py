"""Pins of the oracle's Krylov recycling (oracle/recycling.py, GCRO-DR for the subdomain
solves across outer iterations, the recycling the paper's conclusions suggest).

What fixes it independently of its own code:
* with no recycle space it is GMRES: same iteration count and iterate as krylov.gmres;
* its iterate is the minimal-residual point of x0 + span(U) + K_m((I - C C^H) A, r0),
  checked against a dense least-squares solve over that space built explicitly (Krylov
  matrix of the projected operator, QR-orthonormalised) on a tiny system;
* a right-hand side inside span(C) = A span(U) is solved with no iteration;
* the harmonic Ritz vectors it keeps converge to the eigenvectors of the eigenvalues of
  smallest modulus (a normal matrix with three isolated tiny eigenvalues);
* inside the Schwarz preconditioner every recycled subdomain solve meets the deflated
  tolerance of eq. 4 and the outer FGMRES converges.
"""

import numpy as np
import pytest

from oracle import krylov, recycling, schwarz
from paper_2103_17081_amd import inputs


def _rand(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def _matrix(rng, n, tiny=(1e-3, 2e-3, -3e-3), scale=0.01):
    lam = np.concatenate([np.asarray(tiny, dtype=complex), 1.0 + rng.random(n - len(tiny))])
    return np.diag(lam) + scale * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))


def test_without_recycle_space_is_gmres():
    rng = np.random.default_rng(1)
    A = _matrix(rng, 50)
    op = lambda v: A @ v
    rec = recycling.Recycler(op, k=0)
    for _ in range(3):
        b = _rand(rng, 50)
        r = rec.solve(b, 1e-8, 80)
        g = krylov.gmres(op, b, rtol=1e-8, maxit=80)
        assert r.iters == g.iters
        assert np.linalg.norm(r.x - g.x) <= 1e-10 * np.linalg.norm(g.x)
        assert rec.U is None


@pytest.mark.parametrize("m", [1, 3, 6])
def test_minimal_residual_over_augmented_space(m):
    rng = np.random.default_rng(2)
    n, k = 24, 4
    A = _matrix(rng, n, scale=0.2)
    op = lambda v: A @ v
    rec = recycling.Recycler(op, k=k)
    rec.solve(_rand(rng, n), 1e-12, 40)            # builds U, C
    U, C = rec.U.copy(), rec.C.copy()
    assert np.linalg.norm(C.conj().T @ C - np.eye(k)) < 1e-10
    assert np.linalg.norm(A @ U - C) < 1e-8 * np.linalg.norm(C)
    b = _rand(rng, n)
    r = rec.solve(b, 0.0, m)                       # exactly m Arnoldi steps
    assert r.iters == m
    # explicit space: span(U) + K_m((I - C C^H) A, r0)
    r0 = b - C @ (C.conj().T @ b)
    proj = lambda v: A @ v - C @ (C.conj().T @ (A @ v))
    K = [r0]
    for _ in range(m - 1):
        K.append(proj(K[-1]))
    Kq, _ = np.linalg.qr(np.column_stack(K))
    S = np.column_stack([U, Kq])
    c, *_ = np.linalg.lstsq(A @ S, b, rcond=None)
    best = np.linalg.norm(b - A @ (S @ c))
    got = np.linalg.norm(b - A @ r.x)
    assert abs(got - best) <= 1e-8 * np.linalg.norm(b)
    assert abs(r.residual_estimate - got) <= 1e-8 * np.linalg.norm(b)


def test_rhs_in_recycle_space_needs_no_iteration():
    rng = np.random.default_rng(3)
    A = _matrix(rng, 40)
    rec = recycling.Recycler(lambda v: A @ v, k=5)
    rec.solve(_rand(rng, 40), 1e-10, 60)
    b = rec.C @ _rand(rng, 5)
    r = rec.solve(b, 1e-10, 60)
    assert r.iters == 0
    assert np.linalg.norm(b - A @ r.x) <= 1e-12 * np.linalg.norm(b)


def test_harmonic_ritz_vectors_find_small_eigenvectors():
    rng = np.random.default_rng(4)
    n = 60
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.concatenate([[1e-3, 2e-3, -3e-3], 1.0 + rng.random(n - 3)])
    A = (Q * lam) @ Q.conj().T                     # normal, eigenvectors Q
    op = lambda v: A @ v
    rec = recycling.Recycler(op, k=3)
    rec.solve(_rand(rng, n), 1e-12, 80)
    Uq, _ = np.linalg.qr(rec.U)
    s = np.linalg.svd(Q[:, :3].conj().T @ Uq, compute_uv=False)
    assert s.min() > 1 - 1e-6                      # all principal angles near 0
    # the next systems converge faster than plain GMRES
    b = _rand(rng, n)
    assert rec.solve(b, 1e-8, 80).iters < krylov.gmres(op, b, rtol=1e-8, maxit=80).iters - 3


def test_recycled_subdomain_solves_in_schwarz():
    w = inputs.workload("small")
    S = schwarz.Schwarz(schwarz.problem_from_workload(w))
    R = recycling.RecyclingSchwarz(S, k=5)
    rng = np.random.default_rng(5)
    tol = w.inner_tol
    plain = S.apply(w.rhs[0], tol=tol)
    first = R.apply(w.rhs[0], tol=tol)             # no recycle space yet: the plain solves
    assert np.linalg.norm(first - plain) <= 1e-12 * np.linalg.norm(plain)
    for _ in range(3):
        r = _rand(rng, S.ndof)
        R.apply(r, tol=tol)
        # every recycled local solve meets ||P f - P B x|| <= tol ||P f||
        for s, rec, f in zip(S.subs, R.rec, S.local_rhs(r)):
            d = s.defl
            Pf = d.P(f)
            x = rec.solve(Pf, tol, 200, np.linalg.norm(Pf)).x
            assert np.linalg.norm(Pf - d.PB(x)) <= tol * np.linalg.norm(Pf) * (1 + 1e-10)
    u, st = recycling.RecyclingSchwarz(S, k=5).solve(w.rhs[0], inner_tol=tol)
    assert st.converged and st.true_relres <= 1e-6
