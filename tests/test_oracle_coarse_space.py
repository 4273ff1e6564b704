"""Pins of the oracle's two-level method (global coarse space, Sec. 4's next step).

* the coarse grid lines: p_0 = 0, p_M = N, p_c within half an interval of c N / M,
  spacings differing by at most one;
* the 1D coarse hats reproduce the piecewise-linear interpolant that numpy.interp
  computes from the coarse values (zero on the boundary);
* with M = N/2 the 1D factor is the linear deflation stencil of Sec. 2 (oracle's
  already pinned deflation.z1d) on the whole grid;
* with M = N the coarse space is everything: Q_0 = A^{-1}, the two-level
  preconditioner is the exact inverse and FGMRES stops after one iteration;
* coarse orthogonality of the corrected residual, Z_0^T (r - A Q_0 r) = 0, and
  Q_0 A Q_0 = Q_0;
* with k = 0 (A = K), E_0 annihilates the constant coarse vector on coarse rows whose
  hats and stencil neighbours stay away from the boundary (Z_0 1 = 1 there, K 1 = 0);
* the coarse space lowers the outer count of the one-level method.
"""

import numpy as np
import pytest

from oracle import coarse_space as cs
from oracle import deflation as dfl
from oracle import fem, schwarz
from paper_2103_17081_amd import inputs


@pytest.mark.parametrize("n,m", [(32, 16), (637, 212), (637, 159), (160, 53), (7, 7), (9, 2)])
def test_coarse_nodes(n, m):
    p = cs.coarse_nodes(n, m)
    assert p[0] == 0 and p[-1] == n and len(p) == m + 1
    assert np.all(np.diff(p) >= 1)
    assert np.all(np.abs(p - np.arange(m + 1) * n / m) <= 0.5)
    d = np.diff(p)
    assert d.max() - d.min() <= 1


def test_coarse_nodes_reject():
    with pytest.raises(ValueError):
        cs.coarse_nodes(10, 1)
    with pytest.raises(ValueError):
        cs.coarse_nodes(10, 11)


@pytest.mark.parametrize("n,m", [(32, 16), (45, 13), (50, 17), (21, 20)])
def test_hats_are_piecewise_linear_interpolation(n, m):
    rng = np.random.default_rng(n * 100 + m)
    y = rng.standard_normal(m - 1)
    p = cs.coarse_nodes(n, m)
    ref = np.interp(np.arange(1, n), p, np.concatenate([[0.0], y, [0.0]]))
    np.testing.assert_allclose(cs.z1d(n, m) @ y, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [8, 32, 40])
def test_half_ratio_is_linear_deflation(n):
    a = cs.z1d(n, n // 2).toarray()
    b = dfl.z1d(n - 1, dfl.LINEAR).toarray()
    np.testing.assert_array_equal(a, b)


def test_full_coarse_space_is_exact():
    n, k = 16, 11.0
    prob = schwarz.Problem(k, n, inputs.uniform_cuts(n, 2), inputs.uniform_cuts(n, 2))
    S = schwarz.Schwarz(prob)
    T = cs.TwoLevel(S, n)
    np.testing.assert_array_equal(T.coarse.Z.toarray(), np.eye(S.ndof))
    rng = np.random.default_rng(5)
    r = rng.standard_normal(S.ndof) + 1j * rng.standard_normal(S.ndof)
    x = np.linalg.solve(S.A.toarray(), r)
    np.testing.assert_allclose(T.apply(r, tol=1e-2), x, rtol=0, atol=1e-10 * np.abs(x).max())
    _, st = T.solve(inputs.point_source(n), inner_tol=1e-2)
    assert st.outer_iters == 1 and st.true_relres <= 1e-10


@pytest.mark.parametrize("m", [5, 8, 13])
def test_coarse_orthogonality_and_projection(m):
    n, k = 26, 14.0
    prob = schwarz.Problem(k, n, inputs.uniform_cuts(n, 3), inputs.uniform_cuts(n, 2))
    T = cs.TwoLevel(schwarz.Schwarz(prob), m)
    rng = np.random.default_rng(m)
    r = rng.standard_normal(T.S.ndof) + 1j * rng.standard_normal(T.S.ndof)
    q, w = T.correct(r)
    assert np.linalg.norm(T.coarse.Zt @ w) <= 1e-12 * np.linalg.norm(T.coarse.Zt @ r)
    qq = T.coarse.Q(T.S.A @ q)
    np.testing.assert_allclose(qq, q, rtol=0, atol=1e-11 * np.abs(q).max())
    E = T.coarse.E.toarray()
    np.testing.assert_allclose(E, E.T, rtol=0, atol=1e-14 * np.abs(E).max())


@pytest.mark.parametrize("n,m", [(40, 10), (45, 13)])
def test_laplace_coarse_operator_kills_constants(n, m):
    C = cs.CoarseSpace(fem.helmholtz_matrix(0.0, n), n, m)
    e = C.E @ np.ones(C.ncoarse)
    mc = m - 1
    inner = [(cy - 1) * mc + (cx - 1) for cy in range(2, m - 1) for cx in range(2, m - 1)]
    assert len(inner) > 0
    assert np.abs(e[inner]).max() <= 1e-12
    # rows next to the boundary feel the Dirichlet condition
    assert np.abs(e[0]) > 1e-3


def test_coarse_space_lowers_outer_count():
    n, k = 48, 30.0
    prob = schwarz.Problem(k, n, inputs.uniform_cuts(n, 4), inputs.uniform_cuts(n, 4))
    S = schwarz.Schwarz(prob)
    f = inputs.point_source(n)
    _, one = S.solve(f, inner_tol=1e-2)
    _, two = cs.TwoLevel(S, 24).solve(f, inner_tol=1e-2)
    assert two.true_relres <= 1e-6 and one.true_relres <= 1e-6
    assert two.outer_iters < one.outer_iters
