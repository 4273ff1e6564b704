"""Overlapping Cartesian partition and partition of unity (oracle; test infrastructure only).

Sec. 2 (eq. 3) defines an overlapping partition {Omega_j} with restrictions R_j and
diagonal partition-of-unity matrices D_j satisfying sum_j R_j^T D_j R_j = I; Sec. 3 uses
Cartesian subdomains whose overlap is one layer of mesh elements appended on each
side facing another subdomain.

Given cut points 0 = c_0 < ... < c_P = N per direction, block p covers the cells
[c_p, c_{p+1}); its subdomain extends that by ``overlap`` cell layers on interior sides:
a_p = max(0, c_p - overlap), b_p = min(N, c_{p+1} + overlap) (node coordinates).

Local unknowns:
* impedance (Robin) subdomains: nodes a_p <= i <= b_p that are interior to (0,1)^2;
* Dirichlet subdomains (the paper's A_j = R_j A R_j^T): nodes a_p < i < b_p.

Partition of unity: the paper fixes only sum_j R_j^T D_j R_j = I.  The reading taken
here is Boolean: node i belongs to the block p with c_p <= i < c_{p+1} and D_j is 1 on
the nodes block j owns, 0 elsewhere.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

ROBIN = "robin"
DIRICHLET = "dirichlet"


@dataclass
class SubdomainGeometry:
    px: int
    py: int
    ax: int   # rectangle of the overlapping subdomain, node coordinates
    bx: int
    ay: int
    by: int
    i0: int   # first/last local node, inclusive
    i1: int
    j0: int
    j1: int
    idx: np.ndarray    # global dof index of each local node, x fastest
    owned: np.ndarray  # bool, D_j diagonal

    @property
    def nx(self) -> int:
        return self.i1 - self.i0 + 1

    @property
    def ny(self) -> int:
        return self.j1 - self.j0 + 1

    @property
    def ndof(self) -> int:
        return self.nx * self.ny


def owner_block(cuts: np.ndarray, i: np.ndarray) -> np.ndarray:
    """Block p with cuts[p] <= i < cuts[p+1]."""
    return np.searchsorted(cuts, i, side="right") - 1


def subdomains(n: int, cuts_x, cuts_y, overlap: int = 1, local_bc: str = ROBIN):
    """Geometry of every subdomain, ordered with the x block index fastest."""
    if overlap < 1:
        raise ValueError("overlap must be at least one element layer")
    cuts_x = np.asarray(cuts_x, dtype=np.int64)
    cuts_y = np.asarray(cuts_y, dtype=np.int64)
    out = []
    for py in range(len(cuts_y) - 1):
        for px in range(len(cuts_x) - 1):
            ax = max(0, int(cuts_x[px]) - overlap)
            bx = min(n, int(cuts_x[px + 1]) + overlap)
            ay = max(0, int(cuts_y[py]) - overlap)
            by = min(n, int(cuts_y[py + 1]) + overlap)
            if local_bc == ROBIN:
                i0, i1 = max(ax, 1), min(bx, n - 1)
                j0, j1 = max(ay, 1), min(by, n - 1)
            elif local_bc == DIRICHLET:
                i0, i1, j0, j1 = ax + 1, bx - 1, ay + 1, by - 1
            else:
                raise ValueError(local_bc)
            ii, jj = np.meshgrid(np.arange(i0, i1 + 1), np.arange(j0, j1 + 1), indexing="xy")
            ii, jj = ii.ravel(), jj.ravel()
            idx = (jj - 1) * (n - 1) + (ii - 1)
            owned = (owner_block(cuts_x, ii) == px) & (owner_block(cuts_y, jj) == py)
            out.append(SubdomainGeometry(px, py, ax, bx, ay, by, i0, i1, j0, j1, idx, owned))
    return out


def partition_of_unity_sum(n: int, subs) -> np.ndarray:
    """Diagonal of sum_j R_j^T D_j R_j (must be all ones)."""
    s = np.zeros((n - 1) ** 2)
    for g in subs:
        np.add.at(s, g.idx, g.owned.astype(np.float64))
    return s
