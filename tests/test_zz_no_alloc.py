"""dd_op_inner_solve_static (the subdomain solves with their scratch in the library's static
device array, allocating nothing) against dd_op_inner_solve (scratch in the handle's
workspaces): the same kernel on the same inputs, so solutions, iteration counts and flags
must agree bit for bit -- on two calls in a row, the second on a smaller problem (the
shared array keeps the first call's contents), with and without the host copies of the
counts, and a handle whose solves need more scratch than the array holds is refused."""

import numpy as np
import pytest

from paper_2103_17081_amd import binding
from tests.gpu_common import crandn, solver_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _packed_rhs(torch, gpu, seed, precision):
    rng = np.random.default_rng(seed)
    f = torch.from_numpy(crandn(rng, gpu.nfine * gpu.nrhs)).to("cuda")
    return f.to(torch.complex64) if precision == 32 else f


def test_static_scratch_matches_handle_scratch(torch):
    # first call: medium (8 x 8 subdomains, about 29 MB of scratch); second: small (2 x 2)
    for name, prec, maxit, seed in (("medium", 64, 40, 1), ("small", 32, 100, 2)):
        print("case: static scratch", name, prec, flush=True)
        with solver_for(name, precision=prec, inner_maxit=maxit) as gpu:
            f = _packed_rhs(torch, gpu, seed, prec)
            u1, it1, fl1 = gpu.op_inner_solve(f)
            u2, it2, fl2 = gpu.op_inner_solve_static(f)
            torch.cuda.synchronize()
            print(f"{name}: iterations {it1.sum()} / {it2.sum()}", flush=True)
            assert torch.equal(u1, u2)
            assert np.array_equal(it1, it2) and np.array_equal(fl1, fl2)
            assert it1.sum() > 0 and not np.any(fl1 & 2)
            u3, it3, fl3 = gpu.op_inner_solve_static(f, counts=False)
            torch.cuda.synchronize()
            assert it3 is None and fl3 is None
            assert torch.equal(u1, u3)


def test_static_scratch_refuses_oversized_handles(torch):
    print("case: static scratch oversized", flush=True)
    with solver_for("medium", precision=64, inner_maxit=100) as gpu:
        f = _packed_rhs(torch, gpu, 3, 64)
        with pytest.raises(binding.DDError) as e:
            gpu.op_inner_solve_static(f)
        assert e.value.status == binding.DD_EINVAL and "static scratch holds" in str(e.value)
    with solver_for("small", precision=64, local_solver="direct") as gpu:
        f = _packed_rhs(torch, gpu, 4, 64)
        with pytest.raises(binding.DDError) as e:
            gpu.op_inner_solve_static(f)
        assert e.value.status == binding.DD_EINVAL
