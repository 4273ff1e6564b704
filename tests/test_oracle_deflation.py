"""Pins of the oracle's two-level deflation (Sec. 2, eqs. 4-5).

* linear interpolation reproduces (bi)linear functions away from the tile ends;
* the Bezier restriction acts on constants and linear functions as its printed
  stencil 1/8 [1 4 6 4 1] dictates;
* the Kronecker form equals the separable 2D interpolation evaluated pointwise;
* projection identities: P^2 = P, P B Z = 0, Z^T P = 0, Q invariant under Z -> Z S;
* recovery identity f - B u = P (f - B x);
* deflated GMRES terminates at the direct solution in at most n - n_c steps.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import deflation as dfl
from oracle import fem, krylov


@pytest.mark.parametrize("n", [7, 8, 13])
def test_linear_interpolation_reproduces_linears(n):
    Z = dfl.z1d(n, dfl.LINEAR).toarray()
    m = n // 2
    assert Z.shape == (n, m)
    a, b = 0.3, -1.7
    coarse = a + b * (2 * np.arange(m) + 1)          # samples on fine nodes 2c+1
    fine = Z @ coarse
    inner = np.arange(1, 2 * m)                       # fully covered fine nodes
    np.testing.assert_allclose(fine[inner], a + b * inner, atol=1e-14)


def test_bezier_restriction_on_polynomials():
    n = 21
    Zt = dfl.z1d(n, dfl.BEZIER).toarray().T
    u1 = np.ones(n)
    ul = np.arange(n, dtype=float)
    for c in range(1, n // 2 - 1):                     # stencil fully inside the tile
        assert abs(Zt[c] @ u1 - 2.0) < 1e-14           # (1+4+6+4+1)/8
        assert abs(Zt[c] @ ul - 2.0 * (2 * c + 1)) < 1e-13


def test_kron_is_separable_interpolation():
    nx, ny = 9, 6
    Z = dfl.z2d(nx, ny, dfl.LINEAR).toarray()
    mx, my = nx // 2, ny // 2
    hat = lambda fine, c: max(0.0, 1.0 - abs(fine - (2 * c + 1)) / 2.0)
    for cy in range(my):
        for cx in range(mx):
            col = Z[:, cy * mx + cx]
            for j in range(ny):
                for i in range(nx):
                    assert col[j * nx + i] == hat(i, cx) * hat(j, cy)


def _tile(k=13.0, n=24, rect=(5, 15, 3, 12), kind=dfl.LINEAR):
    B, _ = fem.impedance_matrix(k, n, *rect)
    ax, bx, ay, by = rect
    nx, ny = bx - ax + 1, by - ay + 1
    return dfl.Deflation(B, dfl.z2d(nx, ny, kind)), nx * ny


@pytest.mark.parametrize("kind", [dfl.LINEAR, dfl.BEZIER])
def test_projection_identities(kind):
    d, nloc = _tile(kind=kind)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(nloc) + 1j * rng.standard_normal(nloc)
    np.testing.assert_allclose(d.P(d.P(v)), d.P(v), atol=1e-10)
    BZ = (d.B @ d.Z).toarray()
    PBZ = np.stack([d.P(BZ[:, c]) for c in range(BZ.shape[1])], axis=1)
    assert np.abs(PBZ).max() < 1e-11
    assert np.abs(d.Zt @ d.P(v)).max() < 1e-11
    # Q does not depend on the basis of the coarse space
    S = rng.standard_normal((d.ncoarse, d.ncoarse)) + np.eye(d.ncoarse) * 4
    d2 = dfl.Deflation(d.B, sp.csr_matrix(d.Z @ S))
    np.testing.assert_allclose(d2.Q(v), d.Q(v), atol=1e-9)


def test_recovery_identity():
    d, nloc = _tile()
    rng = np.random.default_rng(2)
    f = rng.standard_normal(nloc) + 1j * rng.standard_normal(nloc)
    x = rng.standard_normal(nloc) + 1j * rng.standard_normal(nloc)
    u = d.recover(f, x)
    np.testing.assert_allclose(f - d.B @ u, d.P(f - d.B @ x), atol=1e-10)


def test_deflated_gmres_finite_termination():
    d, nloc = _tile(k=5.0, n=12, rect=(2, 7, 3, 8))   # a 6x6 tile
    rng = np.random.default_rng(3)
    f = rng.standard_normal(nloc) + 1j * rng.standard_normal(nloc)
    Pf = d.P(f)
    res = krylov.gmres(d.PB, Pf, rtol=1e-13, maxit=nloc)
    assert res.iters <= nloc - d.ncoarse
    u = d.recover(f, res.x)
    u_direct = spla.spsolve(d.B.tocsc(), f)
    np.testing.assert_allclose(u, u_direct, rtol=1e-9, atol=1e-9 * np.abs(u_direct).max())
