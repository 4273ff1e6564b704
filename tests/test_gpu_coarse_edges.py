"""Edge cases of the subdomain coarse solve (twisted block factorisation of E_j).

The preset workloads give coarse blocks of 8 to 26 unknowns per row and 8 to 23 block
rows.  These cases cover what they do not reach, against the oracle:

* ``wide``: N = 130, 2 x 5 blocks, so tiles 66 nodes wide and coarse blocks of 33
  unknowns, beyond the register-ring path (at most 32): the solve takes the general path
  in both the kernel-level operation (256 threads) and the batched subdomain-solve kernel
  (512 threads);
* ``tiny8`` / ``tiny12``: N = 8 and 12 with 4 x 4 blocks, so 1 to 3 coarse rows: the
  middle row alone (one row), the bottom sweep alone (two rows), and one step each way
  (three rows).

Checks: the coarse solve (1e-9 relative, cond(E) eps), the recovered inner solves (same
iteration counts, solutions within 1e-8), the preconditioner (1e-8 in FP64, 2e-3 in FP32),
and the FP64 solve (outer count within +-1 of the oracle's, true residual <= 1e-6).
"""

import functools

import numpy as np
import pytest

from oracle import schwarz
from tests.gpu_common import crandn, pack, pack_coarse, to_gpu, to_np, unpack, unpack_coarse

pytestmark = pytest.mark.gpu

CASES = {
    "wide": (40.0, 130, [0, 65, 130], [0, 26, 52, 78, 104, 130]),
    "tiny8": (5.0, 8, [0, 2, 4, 6, 8], [0, 2, 4, 6, 8]),
    "tiny12": (8.0, 12, [0, 3, 6, 9, 12], [0, 3, 6, 9, 12]),
}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@functools.lru_cache(maxsize=None)
def _oracle(name):
    k, n, cx, cy = CASES[name]
    return schwarz.Schwarz(schwarz.Problem(k, n, np.asarray(cx), np.asarray(cy)))


def _solver(name, precision=64, **kw):
    from paper_2103_17081_amd.binding import Solver
    k, n, cx, cy = CASES[name]
    kw.setdefault("outer_maxit", 400)
    return Solver(k, n_intervals=n, cuts_x=cx, cuts_y=cy, overlap=1, inner_precision=precision, inner_tol=1e-2,
                  **kw)


def _case(*a):
    print("case:", *a, flush=True)


@pytest.mark.parametrize("name", list(CASES))
def test_block_shapes(torch, name):
    """The case reaches the shapes it is meant to cover."""
    with _solver(name) as gpu:
        mx, my = gpu.layout[:, 8], gpu.layout[:, 9]
        if name == "wide":
            assert mx.max() > 32
        else:
            assert my.min() <= (1 if name == "tiny8" else 2) and my.max() >= 2


@pytest.mark.parametrize("name", list(CASES))
def test_coarse_solve_edges(torch, name):
    _case("coarse solve", name)
    S = _oracle(name)
    with _solver(name) as gpu:
        rng = np.random.default_rng(31)
        ys = [crandn(rng, s.defl.ncoarse) for s in S.subs]
        sol = unpack_coarse(S, gpu, to_np(gpu.op_coarse_solve(to_gpu(torch, pack_coarse(S, gpu, ys)))))
        for j, (s, y, x) in enumerate(zip(S.subs, ys, sol)):
            ref = s.defl.coarse_solve(y)
            assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref), j


@pytest.mark.parametrize("name", list(CASES))
def test_inner_solves_edges(torch, name):
    _case("inner solves", name)
    S = _oracle(name)
    with _solver(name) as gpu:
        rng = np.random.default_rng(32)
        fs = [crandn(rng, s.geom.ndof) for s in S.subs]
        u, iters, flags = gpu.op_inner_solve(to_gpu(torch, pack(S, gpu, fs)))
        us = unpack(S, gpu, to_np(u))
        mism = 0
        for s, f, ug, it in zip(S.subs, fs, us, iters):
            ur, itr, _ = s.deflated_gmres(f, 1e-2, 100)
            if it != itr:
                assert abs(int(it) - itr) <= 1
                mism += 1
                continue
            assert np.linalg.norm(ug - ur) <= 1e-8 * np.linalg.norm(ur)
        assert mism <= max(1, len(S.subs) // 50)
        assert not np.any(flags & 2)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", [64, 32])
def test_preconditioner_edges(torch, name, prec):
    _case("apply", name, prec)
    S = _oracle(name)
    with _solver(name, precision=prec) as gpu:
        rng = np.random.default_rng(33)
        r = crandn(rng, S.ndof)
        z = to_np(gpu.apply_preconditioner(to_gpu(torch, r)))
        zr = S.apply(r, "deflated", 1e-2, 100)
        tol = 1e-8 if prec == 64 else 2e-3
        assert np.linalg.norm(z - zr) <= tol * np.linalg.norm(zr)


@pytest.mark.parametrize("name", list(CASES))
def test_solve_edges(torch, name):
    _case("solve", name)
    S = _oracle(name)
    k, n, _, _ = CASES[name]
    rng = np.random.default_rng(34)
    f = crandn(rng, S.ndof)
    _, ost = S.solve(f, "deflated", 1e-2, 100, 1e-6, 400)
    with _solver(name) as gpu:
        u, st = gpu.solve(to_gpu(torch, f))
        rel = np.linalg.norm(f - S.A @ to_np(u)) / np.linalg.norm(f)
        print(name, "gpu", st["outer_iters"], "oracle", ost.outer_iters, "relres", rel, flush=True)
        assert st["status"] == "DD_OK" and rel <= 1e-6
        assert abs(st["outer_iters"] - ost.outer_iters) <= 1
