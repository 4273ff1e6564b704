"""Seeded synthetic inputs shared by the solver, its tests and the benchmark.

This module holds no arithmetic of the solution method.  It only fixes the
workloads: mesh size from wave number and points per wavelength (Sec. 2 of the
paper gives h = 2*pi/(k*ppwl)), cut points of the Cartesian partition (uniform,
Sec. 3, or width-perturbed for the uneven-batching workloads), and the discrete
right-hand sides (the point source at the centre of Sec. 3, plus seeded
Gaussian sources).

Vectors are complex128, one entry per interior grid node, ordered
lexicographically with x running fastest (the ordering Sec. 2 assumes for the
Kronecker deflation matrix): interior node (i, j), 1 <= i, j <= N-1, has index
(j-1)*(N-1) + (i-1).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 17081


def n_intervals(k: float, ppwl: float) -> int:
    """Number of mesh intervals per edge: N = ceil(k*ppwl/(2*pi)), so h = 1/N <= 2*pi/(k*ppwl)."""
    return int(math.ceil(k * ppwl / (2.0 * math.pi) - 1e-9))


def uniform_cuts(n: int, parts: int) -> np.ndarray:
    """Cut points c_p = floor(p*N/P), p = 0..P, of a uniform split of N cells into P blocks."""
    if parts < 1 or parts > n:
        raise ValueError(f"cannot split {n} cells into {parts} blocks")
    return np.array([(p * n) // parts for p in range(parts + 1)], dtype=np.int64)


def perturbed_cuts(n: int, parts: int, perturb: float, rng: np.random.Generator,
                   min_width: int = 4) -> np.ndarray:
    """Cut points of P blocks whose widths are (N/P)(1 + U[-perturb, perturb]).

    The widths are rescaled to sum to N and the cumulative sums rounded to the
    nearest integer.  Raises if a block ends up narrower than ``min_width`` cells.
    """
    w = (n / parts) * (1.0 + rng.uniform(-perturb, perturb, size=parts))
    w *= n / w.sum()
    cuts = np.concatenate([[0], np.rint(np.cumsum(w)).astype(np.int64)])
    cuts[-1] = n
    if np.any(np.diff(cuts) < min_width):
        raise ValueError(f"perturbed partition has a block narrower than {min_width} cells")
    return cuts


def node_coords(n: int):
    """Coordinates (x, y) of the interior nodes in global order, each an array of (N-1)^2."""
    h = 1.0 / n
    i = np.arange(1, n)
    x, y = np.meshgrid(i * h, i * h, indexing="xy")
    return x.ravel(), y.ravel()


def point_source(n: int, at=(0.5, 0.5)) -> np.ndarray:
    """Unit nodal load at the interior node nearest to ``at`` (ties go to the lower index)."""
    def nearest(c):
        t = c * n
        lo = int(math.floor(t))
        i = lo if (t - lo) <= 0.5 else lo + 1
        return min(max(i, 1), n - 1)
    i, j = nearest(at[0]), nearest(at[1])
    f = np.zeros((n - 1) ** 2, dtype=np.complex128)
    f[(j - 1) * (n - 1) + (i - 1)] = 1.0
    return f


@dataclass
class Gaussian:
    cx: float
    cy: float
    sigma: float
    phase: float


def gaussian_params(rng: np.random.Generator, count: int = 3):
    """Seeded Gaussian sources: centres U[0.1,0.9]^2, widths U[0.02,0.1], phases U[0,2*pi)."""
    out = []
    for _ in range(count):
        cx, cy = rng.uniform(0.1, 0.9, size=2)
        out.append(Gaussian(float(cx), float(cy), float(rng.uniform(0.02, 0.1)),
                            float(rng.uniform(0.0, 2.0 * math.pi))))
    return out


def gaussian_load(n: int, params) -> np.ndarray:
    """Nodal load F_i = h^2 * sum_g exp(-|x_i - c_g|^2 / (2 sigma_g^2)) * exp(i phi_g)."""
    x, y = node_coords(n)
    h = 1.0 / n
    f = np.zeros(x.size, dtype=np.complex128)
    for g in params:
        r2 = (x - g.cx) ** 2 + (y - g.cy) ** 2
        f += np.exp(-r2 / (2.0 * g.sigma ** 2)) * np.exp(1j * g.phase)
    return h * h * f


@dataclass
class Workload:
    """One named problem: grid, partition, tolerances and right-hand sides."""
    name: str
    k: float
    n: int
    cuts_x: np.ndarray
    cuts_y: np.ndarray
    overlap: int = 1
    inner_tol: float = 1e-2
    outer_tol: float = 1e-6
    rhs: list = field(default_factory=list)

    @property
    def ndof(self) -> int:
        return (self.n - 1) ** 2

    @property
    def nsub(self) -> int:
        return (len(self.cuts_x) - 1) * (len(self.cuts_y) - 1)


def training_problem(seed: int, block: int = 40) -> Workload:
    """Seeded problem of the initial-guess training set: k ~ U[50, 250], ppwl drawn from
    {10, 20}, N = n_intervals(k, ppwl), P x P blocks with P = max(2, round(N / block)) and
    widths perturbed by +-25%, three seeded Gaussian sources; inner tol 1e-2."""
    rng = np.random.default_rng(seed)
    k = float(rng.uniform(50.0, 250.0))
    ppwl = float(rng.choice([10.0, 20.0]))
    n = n_intervals(k, ppwl)
    parts = max(2, int(round(n / block)))
    cx = perturbed_cuts(n, parts, 0.25, rng)
    cy = perturbed_cuts(n, parts, 0.25, rng)
    return Workload(f"train-{seed}", k, n, cx, cy, rhs=[gaussian_load(n, gaussian_params(rng))])


def workload(name: str, nrhs: int = 1) -> Workload:
    """Preset problems.

    * ``small``   k=20, ppwl=10 (N=32), 2x2 uniform blocks, unit point source at (0.5,0.5),
                  inner tol 1e-2.
    * ``medium``  k=100, ppwl=10 (N=160), 8x8 uniform blocks, point source plus three
                  seeded Gaussians (seed 17081 + rhs index), inner tol 1e-2.
    * ``large``   k=200, ppwl=20 (N=637), 16x16 blocks with widths perturbed by +-25%
                  (seed 17081, x then y), three seeded Gaussians, inner tol 1e-2.
    * ``xlarge``  k=400, ppwl=20 (N=1274), 32x32 blocks perturbed by +-25%, ``nrhs``
                  right-hand sides (default 8), each three Gaussians plus a point source at
                  a seeded interior node.
    """
    if name == "small":
        n = n_intervals(20, 10)
        return Workload(name, 20.0, n, uniform_cuts(n, 2), uniform_cuts(n, 2),
                        rhs=[point_source(n)])
    if name == "medium":
        n = n_intervals(100, 10)
        rhs = []
        for r in range(nrhs):
            rng = np.random.default_rng(SEED_BASE + r)
            rhs.append(point_source(n) + gaussian_load(n, gaussian_params(rng)))
        return Workload(name, 100.0, n, uniform_cuts(n, 8), uniform_cuts(n, 8), rhs=rhs)
    if name == "large":
        n = n_intervals(200, 20)
        rng = np.random.default_rng(SEED_BASE)
        cx = perturbed_cuts(n, 16, 0.25, rng)
        cy = perturbed_cuts(n, 16, 0.25, rng)
        rhs = []
        for r in range(nrhs):
            grng = np.random.default_rng(SEED_BASE + r)
            rhs.append(gaussian_load(n, gaussian_params(grng)))
        return Workload(name, 200.0, n, cx, cy, rhs=rhs)
    if name == "xlarge":
        nrhs = nrhs if nrhs > 1 else 8
        n = n_intervals(400, 20)
        rng = np.random.default_rng(SEED_BASE)
        cx = perturbed_cuts(n, 32, 0.25, rng)
        cy = perturbed_cuts(n, 32, 0.25, rng)
        rhs = []
        for r in range(nrhs):
            grng = np.random.default_rng(SEED_BASE + r)
            g = gaussian_load(n, gaussian_params(grng))
            px, py = grng.uniform(0.1, 0.9, size=2)
            rhs.append(g + point_source(n, (px, py)))
        return Workload(name, 400.0, n, cx, cy, rhs=rhs)
    raise ValueError(f"unknown workload {name!r}")
