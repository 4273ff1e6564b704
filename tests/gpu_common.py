"""Shared helpers of the GPU parity tests: oracle <-> packed-layout conversions."""

import functools

import numpy as np

from oracle import schwarz
from paper_2103_17081_amd import inputs


@functools.lru_cache(maxsize=None)
def oracle_for(name: str, local_bc: str = "robin", deflation: str = "linear"):
    w = inputs.workload(name)
    return w, schwarz.Schwarz(schwarz.problem_from_workload(w, local_bc=local_bc, deflation=deflation))


def solver_for(name: str, precision: int = 64, local_bc: str = "impedance", **kw):
    from paper_2103_17081_amd.binding import Solver
    w = inputs.workload(name)
    kw.setdefault("outer_maxit", {"small": 200, "medium": 2000}.get(name, 4000))
    kw.setdefault("inner_tol", w.inner_tol)
    return Solver(w.k, n_intervals=w.n, cuts_x=w.cuts_x, cuts_y=w.cuts_y, overlap=w.overlap,
                  local_bc=local_bc, inner_precision=precision, **kw)


def check_layout(S, gpu):
    for j, s in enumerate(S.subs):
        g = s.geom
        i0, j0, nx, ny, ax, bx, ay, by, mx, my = gpu.layout[j, :10]
        assert (i0, j0, nx, ny) == (g.i0, g.j0, g.nx, g.ny)
        assert (ax, bx, ay, by) == (g.ax, g.bx, g.ay, g.by)
        assert mx * my == s.defl.ncoarse


def pack(S, gpu, per_sub):
    out = np.zeros(gpu.nfine, dtype=np.complex128)
    for j, v in enumerate(per_sub):
        off = int(gpu.layout[j, 10])
        out[off:off + v.size] = v
    return out


def unpack(S, gpu, packed):
    res = []
    for j, s in enumerate(S.subs):
        off = int(gpu.layout[j, 10])
        res.append(packed[off:off + s.geom.ndof])
    return res


def pack_coarse(S, gpu, per_sub):
    out = np.zeros(gpu.ncoarse, dtype=np.complex128)
    for j, v in enumerate(per_sub):
        off = int(gpu.layout[j, 11])
        out[off:off + v.size] = v
    return out


def unpack_coarse(S, gpu, packed):
    res = []
    for j, s in enumerate(S.subs):
        off = int(gpu.layout[j, 11])
        res.append(packed[off:off + s.defl.ncoarse])
    return res


def crandn(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def to_gpu(torch, x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    return t if dtype is None else t.to(dtype)


def to_np(t):
    return t.detach().cpu().numpy()
