"""Pins of the oracle's P1 assembly (Sec. 2, eqs. 1-2) against independent facts.

* a brute-force element-by-element assembly written another way (basis coefficients
  from the 3x3 vertex system, mass by the edge-midpoint rule, exact for quadratics);
* the closed-form interior stencil of P1 on a uniform right-triangle mesh;
* closed-form impedance rows on an interface edge and at an interface corner;
* row sums and total mass;
* the manufactured solution u = sin(pi x) sin(pi y) converging at second order.
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem


def brute_force_A(k, n):
    """Dense A from loops over cells and triangles (pure Python, tiny grids only)."""
    h = 1.0 / n
    nn = (n - 1) ** 2
    A = np.zeros((nn, nn), dtype=np.complex128)

    def gidx(i, j):
        if 0 < i < n and 0 < j < n:
            return (j - 1) * (n - 1) + (i - 1)
        return None

    for cy in range(n):
        for cx in range(n):
            sw, se, ne, nw = (cx, cy), (cx + 1, cy), (cx + 1, cy + 1), (cx, cy + 1)
            for tri in ((sw, se, ne), (sw, ne, nw)):
                P = np.array([[1.0, a * h, b * h] for a, b in tri])
                coef = np.linalg.inv(P)          # column a: (c0, cx, cy) of basis a
                area = 0.5 * abs(np.linalg.det(P))
                mids = [((tri[0][0] + tri[1][0]) * h / 2, (tri[0][1] + tri[1][1]) * h / 2),
                        ((tri[1][0] + tri[2][0]) * h / 2, (tri[1][1] + tri[2][1]) * h / 2),
                        ((tri[2][0] + tri[0][0]) * h / 2, (tri[2][1] + tri[0][1]) * h / 2)]
                phi = np.array([[coef[0, a] + coef[1, a] * x + coef[2, a] * y for a in range(3)]
                                for x, y in mids])
                for a in range(3):
                    for b in range(3):
                        ga, gb = gidx(*tri[a]), gidx(*tri[b])
                        if ga is None or gb is None:
                            continue
                        kab = area * (coef[1, a] * coef[1, b] + coef[2, a] * coef[2, b])
                        mab = area / 3.0 * np.sum(phi[:, a] * phi[:, b])
                        A[ga, gb] += kab - k * k * mab
    return A


@pytest.mark.parametrize("n,k", [(4, 3.0), (5, 7.5), (8, 11.0)])
def test_assembly_matches_brute_force(n, k):
    A = fem.helmholtz_matrix(k, n).toarray()
    np.testing.assert_allclose(A, brute_force_A(k, n), rtol=0, atol=1e-13)


def test_interior_stencil_closed_form():
    n, k = 12, 17.0
    h = 1.0 / n
    A = fem.helmholtz_matrix(k, n).tocsr()
    i, j = 5, 6
    g = lambda a, b: (b - 1) * (n - 1) + (a - 1)
    row = A[g(i, j)].toarray().ravel()
    kh2 = (k * h) ** 2
    expect = {
        (0, 0): 4 - kh2 / 2,
        (1, 0): -1 - kh2 / 12, (-1, 0): -1 - kh2 / 12,
        (0, 1): -1 - kh2 / 12, (0, -1): -1 - kh2 / 12,
        (1, 1): -kh2 / 12, (-1, -1): -kh2 / 12,     # along the SW-NE cell diagonals
        (1, -1): 0.0, (-1, 1): 0.0,
    }
    for (di, dj), v in expect.items():
        assert abs(row[g(i + di, j + dj)] - v) < 1e-14
    assert np.count_nonzero(np.abs(row) > 0) == 7


def test_row_sums_and_total_mass():
    n = 9
    K, M = fem.assemble_rect(n, 0, n, 0, n)
    assert abs(M.sum() - 1.0) < 1e-14                 # integral of 1 over the unit square
    np.testing.assert_allclose(K @ np.ones(K.shape[0]), 0.0, atol=1e-13)   # constants in the kernel
    Kd, Md = fem.global_matrices(n)
    assert (Kd - Kd.T).count_nonzero() == 0 and (Md - Md.T).count_nonzero() == 0


def test_impedance_rows_closed_form():
    """Rows of B = K - k^2 M - i k M_Gamma on a left interface edge and at a corner."""
    n, k = 20, 9.0
    h = 1.0 / n
    kh2 = (k * h) ** 2
    ax, bx, ay, by = 6, 14, 4, 12          # strictly interior rectangle: all four sides are Robin
    B, keep = fem.impedance_matrix(k, n, ax, bx, ay, by)
    B = B.toarray()
    w = bx - ax + 1
    loc = {int(r): q for q, r in enumerate(keep)}
    L = lambda i, j: loc[(j - ay) * w + (i - ax)]
    # left edge node, not a corner
    i, j = ax, 8
    r = B[L(i, j)]
    assert abs(r[L(i, j)] - (2 - kh2 / 4 - 1j * k * 2 * h / 3)) < 1e-14
    assert abs(r[L(i + 1, j)] - (-1 - kh2 / 12)) < 1e-14
    assert abs(r[L(i, j + 1)] - (-0.5 - kh2 / 24 - 1j * k * h / 6)) < 1e-14
    assert abs(r[L(i, j - 1)] - (-0.5 - kh2 / 24 - 1j * k * h / 6)) < 1e-14
    assert abs(r[L(i + 1, j + 1)] - (-kh2 / 12)) < 1e-14
    assert np.count_nonzero(r) == 5
    # south-west corner: only the NE cell, both adjacent sides are Robin edges
    i, j = ax, ay
    r = B[L(i, j)]
    assert abs(r[L(i, j)] - (1 - kh2 / 6 - 1j * k * 2 * h / 3)) < 1e-14
    assert abs(r[L(i + 1, j)] - (-0.5 - kh2 / 24 - 1j * k * h / 6)) < 1e-14
    assert abs(r[L(i, j + 1)] - (-0.5 - kh2 / 24 - 1j * k * h / 6)) < 1e-14
    assert abs(r[L(i + 1, j + 1)] - (-kh2 / 12)) < 1e-14
    # north-west corner: only the SE cell, whose corner there has no diagonal partner
    i, j = ax, by
    r = B[L(i, j)]
    assert abs(r[L(i, j)] - (1 - kh2 / 12 - 1j * k * 2 * h / 3)) < 1e-14
    assert abs(r[L(i + 1, j - 1)]) == 0.0
    assert np.allclose(B, B.T, atol=0)


def test_whole_domain_impedance_equals_global():
    n, k = 10, 6.0
    B, _ = fem.impedance_matrix(k, n, 0, n, 0, n)
    A = fem.helmholtz_matrix(k, n)
    assert abs(B - A).max() < 1e-15


def test_robin_mass_length():
    n = 16
    G = fem.robin_edge_mass(n, 3, 9, 0, 5)    # left, right and top sides interior
    assert abs(G.sum() - (5 + 5 + 6) / n) < 1e-14


@pytest.mark.parametrize("k", [5.0, 12.0])
def test_manufactured_solution_second_order(k):
    errs = []
    sizes = [16, 32, 64]
    for n in sizes:
        K, M = fem.global_matrices(n)
        A = (K - k * k * M).tocsc()
        h = 1.0 / n
        x = np.arange(1, n) * h
        X, Y = np.meshgrid(x, x, indexing="xy")
        u = (np.sin(np.pi * X) * np.sin(np.pi * Y)).ravel()
        F = M @ ((2 * np.pi ** 2 - k * k) * u)
        uh = spla.spsolve(A, F)
        errs.append(np.max(np.abs(uh - u)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), rates
