"""Pins of the oracle's Schwarz preconditioner and outer solver (Sec. 2 eq. 3, Sec. 3).

* the partition of unity sums to the identity (eq. 3's condition);
* with direct subdomain solves, the preconditioner equals the dense matrix
  sum_j R_j^T D_j B_j^{-1} R_j built with numpy.linalg.inv, and FGMRES gives the same
  count as GMRES right-preconditioned with that matrix;
* a single subdomain covering the domain makes the preconditioner the exact inverse;
* exact inner solves (tol 1e-12) reproduce the direct-solve outer count;
* the Dirichlet local matrices are the restrictions R_j A R_j^T.
"""

import json
import os

import numpy as np
import pytest

from oracle import fem, krylov
from oracle import partition as part
from oracle import schwarz
from paper_2103_17081_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("bc", [part.ROBIN, part.DIRICHLET])
def test_partition_of_unity(bc):
    rng = np.random.default_rng(3)
    n = 57
    cx = inputs.perturbed_cuts(n, 5, 0.25, rng)
    cy = inputs.uniform_cuts(n, 3)
    subs = part.subdomains(n, cx, cy, 1, bc)
    np.testing.assert_array_equal(part.partition_of_unity_sum(n, subs), 1.0)


def test_direct_preconditioner_is_dense_sum():
    n, k = 14, 9.0
    prob = schwarz.Problem(k, n, inputs.uniform_cuts(n, 3), inputs.uniform_cuts(n, 2))
    S = schwarz.Schwarz(prob)
    nd = S.ndof
    Minv = np.zeros((nd, nd), dtype=np.complex128)
    for s in S.subs:
        g = s.geom
        R = np.zeros((g.ndof, nd))
        R[np.arange(g.ndof), g.idx] = 1.0
        D = np.diag(g.owned.astype(float))
        Minv += R.T @ D @ np.linalg.inv(s.B.toarray()) @ R
    rng = np.random.default_rng(0)
    r = rng.standard_normal(nd) + 1j * rng.standard_normal(nd)
    np.testing.assert_allclose(S.apply(r, mode="direct"), Minv @ r, atol=1e-10)
    f = inputs.point_source(n)
    u, st = S.solve(f, mode="direct")
    A = S.A.toarray()
    g = krylov.gmres(lambda v: A @ (Minv @ v), f, rtol=1e-6, maxit=nd)
    assert st.outer_iters == g.iters
    assert st.true_relres <= 1e-6


def test_single_subdomain_is_exact():
    n, k = 12, 7.0
    prob = schwarz.Problem(k, n, inputs.uniform_cuts(n, 1), inputs.uniform_cuts(n, 1))
    S = schwarz.Schwarz(prob)
    u, st = S.solve(inputs.point_source(n), mode="direct")
    assert st.outer_iters == 1 and st.true_relres < 1e-12


def test_dirichlet_local_is_restriction():
    n, k = 16, 8.0
    prob = schwarz.Problem(k, n, inputs.uniform_cuts(n, 2), inputs.uniform_cuts(n, 2),
                           local_bc=part.DIRICHLET)
    S = schwarz.Schwarz(prob)
    A = fem.helmholtz_matrix(k, n).toarray()
    for s in S.subs:
        np.testing.assert_array_equal(s.B.toarray(), A[np.ix_(s.geom.idx, s.geom.idx)])


def test_exact_inner_reproduces_direct_counts():
    w = inputs.workload("small")
    S = schwarz.Schwarz(schwarz.problem_from_workload(w))
    _, d = S.solve(w.rhs[0], mode="direct")
    _, e = S.solve(w.rhs[0], mode="deflated", inner_tol=1e-12)
    assert abs(d.outer_iters - e.outer_iters) <= 1
    assert e.true_relres <= 1e-6 and d.true_relres <= 1e-6


def test_small_workload_golden():
    """Outer/inner counts of the small workload, written by tests/golden/make_golden.py."""
    with open(os.path.join(GOLDEN, "oracle_counts.json")) as fh:
        gold = json.load(fh)["small"]
    w = inputs.workload("small")
    S = schwarz.Schwarz(schwarz.problem_from_workload(w))
    _, st = S.solve(w.rhs[0], mode="deflated", inner_tol=w.inner_tol)
    assert st.outer_iters == gold["outer_iters"]
    assert st.inner_iters == gold["inner_iters"]
    assert st.true_relres <= 1e-6


def test_inner_guess_acceptance_and_tolerance_reference():
    """A guess is used only if it lowers the deflated residual; the tolerance stays ||P f||."""
    w = inputs.workload("small")
    S = schwarz.Schwarz(schwarz.problem_from_workload(w))
    s = S.subs[0]
    rng = np.random.default_rng(4)
    f = rng.standard_normal(s.geom.ndof) + 1j * rng.standard_normal(s.geom.ndof)
    exact = s.direct(f)
    u0, it0, _ = s.deflated_gmres(f, 1e-6, 200)
    u1, it1, acc1 = s.deflated_gmres(f, 1e-6, 200, guess=exact * (1 + 1e-3))
    u2, it2, acc2 = s.deflated_gmres(f, 1e-6, 200, guess=1e6 * f)
    assert acc1 and not acc2
    assert it1 < it0 and it2 == it0
    for u in (u0, u1, u2):
        assert np.linalg.norm(f - s.B @ u) <= 1e-6 * np.linalg.norm(s.defl.P(f)) * 1.0001


def test_zero_local_rhs_takes_no_iterations():
    w = inputs.workload("small")
    S = schwarz.Schwarz(schwarz.problem_from_workload(w))
    s = S.subs[1]
    u, it, _ = s.deflated_gmres(np.zeros(s.geom.ndof, dtype=np.complex128), 1e-2, 50)
    assert it == 0 and not np.any(u)
