"""Exact subdomain solves on the GPU (FP64 block LU of each local matrix, the direct-solve
baseline of Sec. 3, Table 1) against the oracle's sparse LU solves.

Tolerances: both sides solve the same local systems exactly up to rounding, so the
solutions agree to cond(B_j) times eps (asserted 1e-10 relative); preconditioner
applications likewise; full solves reach the outer tolerance with outer counts within
one of the oracle's direct-solve counts (tests/golden/oracle_counts.json, written by
tests/golden/make_golden.py --direct from the oracle alone).
"""

import json
import os

import numpy as np
import pytest

from tests.gpu_common import crandn, oracle_for, pack, solver_for, to_gpu, to_np, unpack

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _case(*a):
    print("case:", *a, flush=True)


def _oracle(name, bc):
    return oracle_for(name, "robin" if bc == "impedance" else bc)


@pytest.mark.parametrize("name,bc", [("small", "impedance"), ("medium", "impedance"), ("small", "dirichlet"),
                                     ("medium", "dirichlet"), ("large", "impedance")])
def test_direct_local_solves(torch, name, bc):
    _case("direct local solves", name, bc)
    w, S = _oracle(name, bc)
    with solver_for(name, precision=64, local_bc=bc, local_solver="direct", outer_maxit=10) as gpu:
        rng = np.random.default_rng(41)
        fs = [crandn(rng, s.geom.ndof) for s in S.subs]
        u, iters, flags = gpu.op_inner_solve(to_gpu(torch, pack(S, gpu, fs)))
        us = unpack(S, gpu, to_np(u))
        assert not iters.any() and not flags.any()
        check = range(len(S.subs)) if len(S.subs) <= 64 else rng.choice(len(S.subs), 8, replace=False)
        for j in check:
            ref = S.subs[j].direct(fs[j])
            assert np.linalg.norm(us[j] - ref) <= 1e-10 * np.linalg.norm(ref), j


@pytest.mark.parametrize("name", ["small", "medium"])
def test_direct_preconditioner(torch, name):
    _case("direct preconditioner", name)
    w, S = _oracle(name, "impedance")
    with solver_for(name, precision=64, local_solver="direct", outer_maxit=10) as gpu:
        rng = np.random.default_rng(43)
        r = crandn(rng, S.ndof)
        z = to_np(gpu.apply_preconditioner(to_gpu(torch, r)))
        zr = S.apply(r, "direct")
        assert np.linalg.norm(z - zr) <= 1e-10 * np.linalg.norm(zr)


@pytest.mark.parametrize("name", ["small", "medium"])
def test_direct_solve_counts(torch, name):
    _case("direct solve", name)
    with open(os.path.join(HERE, "golden", "oracle_counts.json")) as fh:
        gold = json.load(fh)[name]["direct"]
    w, S = _oracle(name, "impedance")
    f = w.rhs[0]
    for graph in (True, False):
        with solver_for(name, precision=64, local_solver="direct", use_graph=graph) as gpu:
            u, st = gpu.solve(to_gpu(torch, f))
            rel = np.linalg.norm(f - S.A @ to_np(u)) / np.linalg.norm(f)
            print(name, "graph" if graph else "eager", st["outer_iters"], "oracle", gold["outer_iters"], rel,
                  flush=True)
            assert st["status"] == "DD_OK" and rel <= 1e-6
            assert abs(st["outer_iters"] - gold["outer_iters"]) <= 1
            assert st["inner_iters_total"] == 0 and st["subdomain_solves"] == st["precond_applies"] * len(S.subs)


def test_direct_on_tiles_too_wide_for_the_subdomain_gmres(torch):
    """The large grid cut 12 x 12 (tiles up to 56 x 56 nodes): the complex128 subdomain GMRES
    needs more LDS than a workgroup has (189 KB), so a handle with it is refused at set-up
    (DD_EINVAL, not a HIP error), while a handle with exact local solves, which never runs
    that kernel, sets up and solves sampled subdomains like the oracle's sparse LU."""
    import dataclasses

    from oracle import schwarz
    from paper_2103_17081_amd import inputs
    from paper_2103_17081_amd.binding import DD_EINVAL, DDError, Solver

    _case("direct local solves, large grid 12x12")
    w = inputs.workload("large")
    cuts = inputs.uniform_cuts(w.n, 12)
    w = dataclasses.replace(w, cuts_x=cuts, cuts_y=cuts)
    kw = dict(n_intervals=w.n, cuts_x=cuts, cuts_y=cuts, overlap=w.overlap, inner_precision=64, outer_maxit=10)
    with pytest.raises(DDError) as err:
        Solver(w.k, **kw)
    assert err.value.status == DD_EINVAL and "LDS" in str(err.value)
    S = schwarz.Schwarz(schwarz.problem_from_workload(w))
    with Solver(w.k, local_solver="direct", **kw) as gpu:
        rng = np.random.default_rng(43)
        fs = [crandn(rng, s.geom.ndof) for s in S.subs]
        u, iters, flags = gpu.op_inner_solve(to_gpu(torch, pack(S, gpu, fs)))
        us = unpack(S, gpu, to_np(u))
        assert not iters.any() and not flags.any()
        for j in rng.choice(len(S.subs), 6, replace=False):
            ref = S.subs[j].direct(fs[j])
            assert np.linalg.norm(us[j] - ref) <= 1e-10 * np.linalg.norm(ref), j
