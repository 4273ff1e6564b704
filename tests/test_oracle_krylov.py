"""Pins of the oracle's GMRES and FGMRES (Sec. 3) against textbook facts."""

import numpy as np
import pytest

from oracle import krylov


def _rand(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def test_givens_zeroes_second_entry():
    for a, b in [(1 + 2j, 0.5), (0.0, 2.0), (3 - 1j, 0.0), (-2j, 1e-3)]:
        c, s, r = krylov.givens(a, b)
        G = np.array([[c, s], [-np.conj(s), c]])
        out = G @ np.array([a, b])
        assert abs(out[1]) < 1e-15 and abs(out[0] - r) < 1e-14
        assert abs(abs(c) ** 2 + abs(s) ** 2 - 1) < 1e-14


def test_distinct_eigenvalues_bound_iterations():
    n, d = 40, 6
    rng = np.random.default_rng(4)
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    lam = np.repeat(np.array([1, 2 + 1j, -3, 0.5j, 4 - 2j, -1 - 1j]), [7, 7, 7, 7, 6, 6])
    A = X @ np.diag(lam) @ np.linalg.inv(X)
    b = _rand(n, 5)
    res = krylov.gmres(lambda v: A @ v, b, rtol=1e-10, maxit=n)
    assert res.iters <= d
    np.testing.assert_allclose(A @ res.x, b, atol=1e-7 * np.linalg.norm(b))


def test_estimate_equals_true_residual_and_monotone():
    n = 60
    rng = np.random.default_rng(6)
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) / np.sqrt(n) + 1j * rng.standard_normal((n, n)) / np.sqrt(n)
    b = _rand(n, 7)
    for m in [3, 9, 17]:
        res = krylov.gmres(lambda v: A @ v, b, rtol=1e-30, maxit=m)
        assert res.iters == m
        true = np.linalg.norm(b - A @ res.x)
        assert abs(true - res.history[-1]) < 1e-12 * np.linalg.norm(b)
        assert np.all(np.diff(res.history) <= 1e-14)


def test_fgmres_with_fixed_preconditioner_equals_right_preconditioned_gmres():
    n = 50
    rng = np.random.default_rng(8)
    A = np.eye(n) * 2 + rng.standard_normal((n, n)) / 3
    Minv = np.linalg.inv(A + rng.standard_normal((n, n)) / 5)
    b = _rand(n, 9)
    f = krylov.fgmres(lambda v: A @ v, lambda v: Minv @ v, b, rtol=1e-10, maxit=n)
    g = krylov.gmres(lambda v: A @ (Minv @ v), b, rtol=1e-10, maxit=n)
    assert f.iters == g.iters
    np.testing.assert_allclose(f.x, Minv @ g.x, atol=1e-9)
    exact = krylov.fgmres(lambda v: A @ v, lambda v: np.linalg.solve(A, v), b, rtol=1e-10)
    assert exact.iters == 1


def test_fgmres_restart_still_converges():
    n = 80
    rng = np.random.default_rng(10)
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = _rand(n, 11)
    res = krylov.fgmres(lambda v: A @ v, lambda v: v, b, rtol=1e-8, maxit=400, restart=10)
    assert res.converged
    assert np.linalg.norm(b - A @ res.x) <= 1.01e-8 * np.linalg.norm(b)
