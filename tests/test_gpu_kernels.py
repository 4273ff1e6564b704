"""Kernel-level parity of the HIP library against the oracle, element by element.

Tolerances follow from the arithmetic:
* FP64 stencil / restriction / prolongation / gather / scatter: a handful of
  products per output (coefficients summed in a different order than the oracle's
  element assembly), so agreement to 1e-13 relative to the vector norm (gather and
  scatter move values and are bit-exact).
* FP64 coarse solves: bounded by cond(E) * eps; the test asserts 1e-9 relative.
* FP32 stencil: 7 products, rounding ~1e-7 relative; asserted at 2e-6 of max |w|.
* FP32 deflated operator: the FP32 input and output roundings are amplified by the
  coarse solve; asserted at 1e-4 relative to ||P B v||.
"""

import numpy as np
import pytest

from tests.gpu_common import (check_layout, crandn, oracle_for, pack, pack_coarse, solver_for, to_gpu, to_np,
                              unpack, unpack_coarse)

pytestmark = pytest.mark.gpu

WORKLOADS = ["small", "medium", "large"]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _print_case(*a):
    print("case:", *a, flush=True)


@pytest.mark.parametrize("name", WORKLOADS)
def test_layout_and_global_apply(torch, name):
    _print_case("global_apply", name)
    w, S = oracle_for(name)
    with solver_for(name, outer_maxit=10) as gpu:
        check_layout(S, gpu)
        rng = np.random.default_rng(1)
        v = crandn(rng, S.ndof)
        got = to_np(gpu.op_global_apply(to_gpu(torch, v)))
        ref = S.A @ v
        assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", WORKLOADS)
@pytest.mark.parametrize("prec", [64, 32])
def test_local_apply(torch, name, prec):
    _print_case("local_apply", name, prec)
    w, S = oracle_for(name)
    with solver_for(name, precision=prec, outer_maxit=10) as gpu:
        rng = np.random.default_rng(2)
        vs = [crandn(rng, s.geom.ndof) for s in S.subs]
        dt = torch.complex64 if prec == 32 else torch.complex128
        vin = pack(S, gpu, vs).astype(np.complex64 if prec == 32 else np.complex128)
        got = unpack(S, gpu, to_np(gpu.op_local_apply(to_gpu(torch, vin), precision=prec)).astype(np.complex128))
        for s, v, g in zip(S.subs, vs, got):
            ref = s.B @ v.astype(vin.dtype).astype(np.complex128)
            if prec == 64:
                assert np.linalg.norm(g - ref) <= 1e-13 * np.linalg.norm(ref)
            else:
                assert np.abs(g - ref).max() <= 2e-6 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["small", "medium"])
def test_coarse_matrix(torch, name):
    _print_case("coarse_matrix", name)
    w, S = oracle_for(name)
    with solver_for(name, outer_maxit=10) as gpu:
        for j, s in enumerate(S.subs):
            coef, piv = gpu.coarse_matrix(j)
            mx, my = int(gpu.layout[j, 8]), int(gpu.layout[j, 9])
            nc = mx * my
            E = np.zeros((nc, nc), dtype=np.complex128)
            for c in range(nc):
                cx, cy = c % mx, c // mx
                for o in range(9):
                    qx, qy = cx + o % 3 - 1, cy + o // 3 - 1
                    if 0 <= qx < mx and 0 <= qy < my:
                        E[c, qy * mx + qx] = coef[c, o]
            ref = s.defl.E
            assert np.abs(E - ref).max() <= 1e-14 * np.abs(ref).max()
            assert piv > 0


@pytest.mark.parametrize("name", WORKLOADS)
def test_restrict_prolong_coarse_solve(torch, name):
    _print_case("restrict/prolong/coarse_solve", name)
    w, S = oracle_for(name)
    with solver_for(name, outer_maxit=10) as gpu:
        rng = np.random.default_rng(3)
        vs = [crandn(rng, s.geom.ndof) for s in S.subs]
        ts = unpack_coarse(S, gpu, to_np(gpu.op_restrict(to_gpu(torch, pack(S, gpu, vs)))))
        for s, v, t in zip(S.subs, vs, ts):
            ref = s.defl.Zt @ v
            assert np.linalg.norm(t - ref) <= 1e-15 * np.linalg.norm(ref) * 10
        ys = [crandn(rng, s.defl.ncoarse) for s in S.subs]
        ps = unpack(S, gpu, to_np(gpu.op_prolong(to_gpu(torch, pack_coarse(S, gpu, ys)))))
        for s, y, p in zip(S.subs, ys, ps):
            ref = s.defl.Z @ y
            assert np.linalg.norm(p - ref) <= 1e-15 * np.linalg.norm(ref) * 10
        sol = unpack_coarse(S, gpu, to_np(gpu.op_coarse_solve(to_gpu(torch, pack_coarse(S, gpu, ys)))))
        for s, y, x in zip(S.subs, ys, sol):
            ref = s.defl.coarse_solve(y)
            assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", WORKLOADS)
@pytest.mark.parametrize("prec", [64, 32])
def test_deflated_apply(torch, name, prec):
    _print_case("deflated_apply", name, prec)
    w, S = oracle_for(name)
    with solver_for(name, precision=prec, outer_maxit=10) as gpu:
        rng = np.random.default_rng(4)
        vs = [crandn(rng, s.geom.ndof) for s in S.subs]
        npdt = np.complex64 if prec == 32 else np.complex128
        vin = pack(S, gpu, vs).astype(npdt)
        got = unpack(S, gpu, to_np(gpu.op_deflated_apply(to_gpu(torch, vin), precision=prec)).astype(np.complex128))
        for s, v, g in zip(S.subs, vs, got):
            ref = s.defl.PB(v.astype(npdt).astype(np.complex128))
            tol = 1e-10 if prec == 64 else 1e-4
            assert np.linalg.norm(g - ref) <= tol * np.linalg.norm(ref)


@pytest.mark.parametrize("name", WORKLOADS)
def test_gather_scatter_exact(torch, name):
    _print_case("gather/scatter", name)
    w, S = oracle_for(name)
    with solver_for(name, outer_maxit=10) as gpu:
        rng = np.random.default_rng(5)
        r = crandn(rng, S.ndof)
        f = unpack(S, gpu, to_np(gpu.op_gather(to_gpu(torch, r))))
        for s, fj in zip(S.subs, f):
            assert np.array_equal(fj, r[s.geom.idx])
        us = [crandn(rng, s.geom.ndof) for s in S.subs]
        z = to_np(gpu.op_scatter(to_gpu(torch, pack(S, gpu, us))))
        assert np.array_equal(z, S.scatter(us))
