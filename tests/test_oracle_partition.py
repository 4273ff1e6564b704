"""Pins of the oracle's subdomain extents (Sec. 2, eq. 3; Sec. 3).

Sec. 3 builds the overlapping subdomains from a Cartesian split of the mesh cells by
appending one layer of mesh elements on every side that faces another subdomain, so a
subdomain touching the boundary of the unit square stays a rectangle.  These tests
characterise that by brute force over cells, nodes and edges -- without the interval
arithmetic `oracle.partition.subdomains` uses -- and compare:

* cells: a subdomain holds exactly the cells of the square within one layer (Chebyshev
  distance <= 1 in cell units) of its block's cells; neighbouring subdomains then share
  two cell layers (overlap width 2h);
* nodes: the impedance (Robin) local unknowns are the vertices of those cells that are
  not on the boundary of the square; the Dirichlet ones (the paper's A_j = R_j A R_j^T)
  are the nodes whose four surrounding cells all belong to the subdomain;
* impedance edges: the mesh edges with exactly one adjacent cell in the subdomain that
  do not lie on the boundary of the square carry the 1D edge mass h/6 [2 1; 1 2].

Self-tests check that the brute-force comparison catches the plausible mistakes: one
layer too many, shifted cuts, Dirichlet node ranges taken for impedance ones, and an
impedance edge on the square's boundary.
"""

import itertools

import numpy as np
import pytest

from oracle import fem
from oracle import partition as part
from paper_2103_17081_amd import inputs


def block_cells(cuts_x, cuts_y, px, py):
    return {(cx, cy) for cx in range(cuts_x[px], cuts_x[px + 1]) for cy in range(cuts_y[py], cuts_y[py + 1])}


def grown_cells(n, cells, layers):
    """Cells of [0, n)^2 within Chebyshev distance `layers` of `cells`."""
    out = set()
    for (cx, cy) in cells:
        for dx, dy in itertools.product(range(-layers, layers + 1), repeat=2):
            x, y = cx + dx, cy + dy
            if 0 <= x < n and 0 <= y < n:
                out.add((x, y))
    return out


def robin_nodes(n, cells):
    """Vertices of the cells that are interior nodes of the square, x fastest."""
    nodes = {(cx + a, cy + b) for (cx, cy) in cells for a in (0, 1) for b in (0, 1)}
    nodes = [(i, j) for (i, j) in nodes if 0 < i < n and 0 < j < n]
    return sorted(nodes, key=lambda t: (t[1], t[0]))


def dirichlet_nodes(n, cells):
    """Nodes whose four surrounding cells all belong to the subdomain, x fastest."""
    nodes = []
    for i in range(1, n):
        for j in range(1, n):
            if all((i - a, j - b) in cells for a in (0, 1) for b in (0, 1)):
                nodes.append((i, j))
    return sorted(nodes, key=lambda t: (t[1], t[0]))


def impedance_edges(n, cells):
    """Mesh edges with exactly one adjacent subdomain cell, not on the square's boundary."""
    edges = []
    for i in range(0, n + 1):
        for j in range(0, n):       # vertical edge (i, j)-(i, j+1): cells (i-1, j) and (i, j)
            if i in (0, n):
                continue
            if ((i - 1, j) in cells) != ((i, j) in cells):
                edges.append(((i, j), (i, j + 1)))
    for j in range(0, n + 1):
        for i in range(0, n):       # horizontal edge (i, j)-(i+1, j): cells (i, j-1) and (i, j)
            if j in (0, n):
                continue
            if ((i, j - 1) in cells) != ((i, j) in cells):
                edges.append(((i, j), (i + 1, j)))
    return edges


def global_index(n, nodes):
    return np.array([(j - 1) * (n - 1) + (i - 1) for (i, j) in nodes], dtype=np.int64)


def extent_mismatches(n, cuts_x, cuts_y, subs, bc, layers=1):
    """Descriptions of every way `subs` differs from the brute-force characterisation."""
    bad = []
    P, Q = len(cuts_x) - 1, len(cuts_y) - 1
    if len(subs) != P * Q:
        return [f"{len(subs)} subdomains for a {P} x {Q} split"]
    for g in subs:
        cells = grown_cells(n, block_cells(cuts_x, cuts_y, g.px, g.py), layers)
        have = {(cx, cy) for cx in range(g.ax, g.bx) for cy in range(g.ay, g.by)}
        if have != cells:
            bad.append(f"subdomain ({g.px},{g.py}): cells differ")
        nodes = robin_nodes(n, cells) if bc == part.ROBIN else dirichlet_nodes(n, cells)
        if not np.array_equal(g.idx, global_index(n, nodes)):
            bad.append(f"subdomain ({g.px},{g.py}): local unknowns differ")
    return bad


def perturbed(n, P, seed):
    return inputs.perturbed_cuts(n, P, 0.25, np.random.default_rng(seed))


SPLITS = [
    ("uniform 3x2", 23, lambda n: inputs.uniform_cuts(n, 3), lambda n: inputs.uniform_cuts(n, 2)),
    ("uniform 4x4", 32, lambda n: inputs.uniform_cuts(n, 4), lambda n: inputs.uniform_cuts(n, 4)),
    ("perturbed 5x3", 41, lambda n: perturbed(n, 5, 11), lambda n: perturbed(n, 3, 12)),
    ("single block", 9, lambda n: inputs.uniform_cuts(n, 1), lambda n: inputs.uniform_cuts(n, 1)),
]


@pytest.mark.parametrize("bc", [part.ROBIN, part.DIRICHLET])
@pytest.mark.parametrize("name,n,fx,fy", SPLITS, ids=[s[0] for s in SPLITS])
def test_extents_match_one_appended_layer(name, n, fx, fy, bc):
    cx, cy = fx(n), fy(n)
    subs = part.subdomains(n, cx, cy, 1, bc)
    assert extent_mismatches(n, cx, cy, subs, bc) == []


@pytest.mark.parametrize("name,n,fx,fy", SPLITS[:3], ids=[s[0] for s in SPLITS[:3]])
def test_neighbours_overlap_by_two_layers(name, n, fx, fy):
    """Adjacent subdomains share exactly two cell layers across each interior cut."""
    cx, cy = fx(n), fy(n)
    subs = {(g.px, g.py): g for g in part.subdomains(n, cx, cy, 1)}
    P, Q = len(cx) - 1, len(cy) - 1
    for (px, py), g in subs.items():
        if px + 1 < P:
            h = subs[(px + 1, py)]
            assert g.bx - h.ax == 2 and h.ax < cx[px + 1] < g.bx
        if py + 1 < Q:
            h = subs[(px, py + 1)]
            assert g.by - h.ay == 2 and h.ay < cy[py + 1] < g.by


@pytest.mark.parametrize("name,n,fx,fy", SPLITS, ids=[s[0] for s in SPLITS])
def test_impedance_edges(name, n, fx, fy):
    """The 1D edge mass of the impedance matrices sits exactly on the subdomain boundary
    edges interior to the square (brute-force edge enumeration, assembled here)."""
    cx, cy = fx(n), fy(n)
    h = 1.0 / n
    for g in part.subdomains(n, cx, cy, 1):
        cells = grown_cells(n, block_cells(cx, cy, g.px, g.py), 1)
        w = g.bx - g.ax + 1
        nn = w * (g.by - g.ay + 1)
        ref = np.zeros((nn, nn))
        for (i0, j0), (i1, j1) in impedance_edges(n, cells):
            a = (j0 - g.ay) * w + (i0 - g.ax)
            b = (j1 - g.ay) * w + (i1 - g.ax)
            ref[a, a] += 2 * h / 6
            ref[b, b] += 2 * h / 6
            ref[a, b] += h / 6
            ref[b, a] += h / 6
        G = fem.robin_edge_mass(n, g.ax, g.bx, g.ay, g.by).toarray()
        np.testing.assert_allclose(G, ref, rtol=0, atol=1e-15)


def test_mismatches_are_detected():
    """Plausible mistakes in the extents fail the brute-force comparison."""
    n = 32
    cx, cy = perturbed(n, 4, 21), inputs.uniform_cuts(n, 3)
    good = part.subdomains(n, cx, cy, 1, part.ROBIN)
    assert extent_mismatches(n, cx, cy, good, part.ROBIN) == []
    # one layer too many (an off-by-one overlap)
    assert extent_mismatches(n, cx, cy, part.subdomains(n, cx, cy, 2, part.ROBIN), part.ROBIN)
    # cuts shifted by one cell
    shifted = cx.copy()
    shifted[1:-1] += 1
    assert extent_mismatches(n, cx, cy, part.subdomains(n, shifted, cy, 1, part.ROBIN), part.ROBIN)
    # Dirichlet node ranges taken for impedance ones, and the reverse
    dirich = part.subdomains(n, cx, cy, 1, part.DIRICHLET)
    assert extent_mismatches(n, cx, cy, dirich, part.ROBIN)
    assert extent_mismatches(n, cx, cy, good, part.DIRICHLET)
    # a subdomain whose right side is shifted by one cell
    g = good[1]
    wrong = part.SubdomainGeometry(g.px, g.py, g.ax, g.bx + 1, g.ay, g.by, g.i0, g.i1 + 1, g.j0, g.j1,
                                   g.idx, g.owned)
    assert extent_mismatches(n, cx, cy, [*good[:1], wrong, *good[2:]], part.ROBIN)


def test_edge_enumeration_detects_boundary_edges():
    """An impedance edge on the square's boundary (a wrong clamp) changes the edge set."""
    n = 12
    cells = grown_cells(n, block_cells(inputs.uniform_cuts(n, 2), inputs.uniform_cuts(n, 2), 0, 0), 1)
    edges = impedance_edges(n, cells)
    assert not any(e[0][0] == e[1][0] == 0 or e[0][1] == e[1][1] == 0 for e in edges)
    # the block (0, 0) grown by one layer covers cells [0, 7) x [0, 7): impedance sides x = 7, y = 7
    assert sorted({e[0][0] for e in edges if e[0][0] == e[1][0]}) == [7]
    assert sorted({e[0][1] for e in edges if e[0][1] == e[1][1]}) == [7]
    assert len(edges) == 14
