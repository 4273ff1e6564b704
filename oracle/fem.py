"""P1 finite-element assembly (oracle; test infrastructure only).

Model problem (Sec. 2, eq. 1): -Delta u - k^2 u = f on (0,1)^2, u = 0 on the boundary.
Discretisation (Sec. 2, eq. 2): piecewise-linear elements on a uniform grid, bilinear
form a(u,v) = int grad u . grad v - k^2 u v (no complex conjugation, so every matrix
here is complex symmetric), giving A u = f.

Mesh: N intervals per edge, h = 1/N, nodes (i, j) at (i h, j h).  Each square cell is
split along its SW->NE diagonal into the triangles (SW, SE, NE) and (SW, NE, NW); the
paper does not say which diagonal its mesh uses, this is the reading taken here.

Element matrices use the generic P1 formulas from the vertex coordinates (not a
precomputed stencil): with b_a = (y_b - y_c, x_c - x_b) for each cyclic vertex triple,
K_ab = b_a . b_b / (4|T|) and M_ab = |T| (1 + delta_ab) / 12.

Local impedance matrices (the interface condition d_n u - i k u = 0 on the part of a
subdomain boundary that is interior to the domain) integrate only over the cells of
the subdomain and add -i k times the 1D edge mass (h/6)[2 1; 1 2] on each such edge.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def p1_element_matrices(xy: np.ndarray):
    """Stiffness and mass matrices of P1 triangles.

    xy: (T, 3, 2) vertex coordinates.  Returns K, M of shape (T, 3, 3).
    """
    x, y = xy[..., 0], xy[..., 1]
    # b_a = (y_b - y_c, x_c - x_b) with (a, b, c) cyclic
    bx = np.stack([y[:, 1] - y[:, 2], y[:, 2] - y[:, 0], y[:, 0] - y[:, 1]], axis=1)
    by = np.stack([x[:, 2] - x[:, 1], x[:, 0] - x[:, 2], x[:, 1] - x[:, 0]], axis=1)
    area = 0.5 * np.abs((x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0])
                        - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0]))
    K = (bx[:, :, None] * bx[:, None, :] + by[:, :, None] * by[:, None, :]) / (4.0 * area[:, None, None])
    M = area[:, None, None] * (np.ones((3, 3)) + np.eye(3)) / 12.0
    return K, M


def rect_triangles(ax: int, bx: int, ay: int, by: int):
    """Triangles of the cells [ax, bx) x [ay, by), as global node pairs (i, j).

    Returns an int array (T, 3, 2) of node coordinates in grid units.
    """
    cx, cy = np.meshgrid(np.arange(ax, bx), np.arange(ay, by), indexing="xy")
    cx, cy = cx.ravel(), cy.ravel()
    sw = np.stack([cx, cy], axis=1)
    se = np.stack([cx + 1, cy], axis=1)
    ne = np.stack([cx + 1, cy + 1], axis=1)
    nw = np.stack([cx, cy + 1], axis=1)
    t1 = np.stack([sw, se, ne], axis=1)
    t2 = np.stack([sw, ne, nw], axis=1)
    return np.concatenate([t1, t2], axis=0)


def assemble_rect(n: int, ax: int, bx: int, ay: int, by: int):
    """Assemble K and M over the cells of [ax,bx] x [ay,by] (node coordinates).

    Nodes of the rectangle are numbered locally as (j - ay) * (bx - ax + 1) + (i - ax).
    Returns (K, M) as CSR matrices on those nodes, before any boundary elimination.
    """
    h = 1.0 / n
    tri = rect_triangles(ax, bx, ay, by)
    K_e, M_e = p1_element_matrices(tri.astype(np.float64) * h)
    w = bx - ax + 1
    loc = (tri[..., 1] - ay) * w + (tri[..., 0] - ax)
    rows = np.repeat(loc[:, :, None], 3, axis=2).ravel()
    cols = np.repeat(loc[:, None, :], 3, axis=1).ravel()
    nn = w * (by - ay + 1)
    K = sp.coo_matrix((K_e.ravel(), (rows, cols)), shape=(nn, nn)).tocsr()
    M = sp.coo_matrix((M_e.ravel(), (rows, cols)), shape=(nn, nn)).tocsr()
    return K, M


def interior_mask_rect(n: int, ax: int, bx: int, ay: int, by: int) -> np.ndarray:
    """True for nodes of the rectangle that are not on the boundary of (0,1)^2."""
    i, j = np.meshgrid(np.arange(ax, bx + 1), np.arange(ay, by + 1), indexing="xy")
    return ((i > 0) & (i < n) & (j > 0) & (j < n)).ravel()


def global_matrices(n: int):
    """K and M of the whole domain restricted to interior nodes (Dirichlet eliminated)."""
    K, M = assemble_rect(n, 0, n, 0, n)
    keep = np.flatnonzero(interior_mask_rect(n, 0, n, 0, n))
    return K[keep][:, keep].tocsr(), M[keep][:, keep].tocsr()


def helmholtz_matrix(k: float, n: int) -> sp.csr_matrix:
    """A = K - k^2 M on the interior nodes, complex128 (Sec. 2, eq. 2)."""
    K, M = global_matrices(n)
    return (K - (k * k) * M).astype(np.complex128).tocsr()


def robin_edge_mass(n: int, ax: int, bx: int, ay: int, by: int) -> sp.csr_matrix:
    """1D mass matrix of the edges of the rectangle's boundary that are interior to (0,1)^2.

    Local numbering as in ``assemble_rect``.
    """
    h = 1.0 / n
    w = bx - ax + 1
    nn = w * (by - ay + 1)
    segs = []
    if ax > 0:   # left side x = ax
        segs += [((ax, s), (ax, s + 1)) for s in range(ay, by)]
    if bx < n:   # right side x = bx
        segs += [((bx, s), (bx, s + 1)) for s in range(ay, by)]
    if ay > 0:   # bottom side y = ay
        segs += [((s, ay), (s + 1, ay)) for s in range(ax, bx)]
    if by < n:   # top side y = by
        segs += [((s, by), (s + 1, by)) for s in range(ax, bx)]
    rows, cols, vals = [], [], []
    for (i0, j0), (i1, j1) in segs:
        length = h * np.hypot(i1 - i0, j1 - j0)
        a = (j0 - ay) * w + (i0 - ax)
        b = (j1 - ay) * w + (i1 - ax)
        for r, c, v in ((a, a, 2.0), (b, b, 2.0), (a, b, 1.0), (b, a, 1.0)):
            rows.append(r)
            cols.append(c)
            vals.append(v * length / 6.0)
    return sp.coo_matrix((vals, (rows, cols)), shape=(nn, nn)).tocsr()


def impedance_matrix(k: float, n: int, ax: int, bx: int, ay: int, by: int):
    """Local matrix B = K_j - k^2 M_j - i k M_Gamma on the subdomain [ax,bx] x [ay,by].

    Returns (B, keep) where keep are the rectangle-local indices of the retained
    (non-Dirichlet) nodes, in x-fastest order; B is indexed by them.
    """
    K, M = assemble_rect(n, ax, bx, ay, by)
    G = robin_edge_mass(n, ax, bx, ay, by)
    B = (K - (k * k) * M).astype(np.complex128) - 1j * k * G
    keep = np.flatnonzero(interior_mask_rect(n, ax, bx, ay, by))
    return B[keep][:, keep].tocsc(), keep
