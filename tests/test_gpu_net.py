"""GPU parity tests of the learned initial guess: the bf16 MFMA network kernels against
the float64 oracle (oracle/cnn.py), the tile builders against the oracle's tiles, and the
subdomain solver with an attached network against the oracle's guessed solves.

Tolerances.  Weights and network inputs are bfloat16 values on both sides, so the
first layer sees identical operands; the GPU then rounds every activation (and, in the
backward pass, every activation gradient) to bfloat16, relative error u = 2^-9 per
rounding, over 7 layers plus pooling/upsampling re-roundings.  Outputs are compared in
relative 2-norm per tile at 3e-2 (about 10 u times the depth), gradients per parameter
tensor at 5e-2 and as a whole by cosine >= 0.999; the loss at 2e-2.
"""

import os

import numpy as np
import pytest

from oracle import cnn
from tests.gpu_common import crandn, oracle_for, pack, solver_for, to_gpu, to_np, unpack

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
WIDTHS = (16, 32, 64, 64)


def bf16_round(a):
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _case(*what):
    print("case:", *what, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def oracle_params(seed, widths):
    rng = np.random.default_rng(seed)
    p = cnn.init_params(rng, widths)
    for k in p:
        if k.startswith("b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    v = cnn.flatten(p)
    # weights bfloat16-exact (the GPU multiplies bf16 weights); biases stay fp32
    out = v.astype(np.float32).astype(np.float64)
    q = cnn.unflatten(out.copy(), widths)
    for k in q:
        if k.startswith("W"):
            q[k] = bf16_round(q[k])
    return cnn.flatten(q)


def oracle_descs(S):
    n = S.prob.n
    out = []
    for sd in S.subs:
        g = sd.geom
        edges = (g.i0 == g.ax) | (g.i1 == g.bx) << 1 | (g.j0 == g.ay) << 2 | (g.j1 == g.by) << 3
        robin = (g.ax > 0) | (g.bx < n) << 1 | (g.ay > 0) << 2 | (g.by < n) << 3
        out.append((g.nx, g.ny, int(edges), int(robin) if edges else 0))
    return out


def desc_array(S, kh, reps=1):
    from paper_2103_17081_amd.binding import TileDesc
    ds = oracle_descs(S) * reps
    arr = (TileDesc * len(ds))()
    for i, (nx, ny, e, r) in enumerate(ds):
        arr[i].nx, arr[i].ny, arr[i].edges, arr[i].robin, arr[i].kh = nx, ny, e, r, kh
    return arr


def small_batch(S, w, T, rng):
    """Inputs and targets of the 4 small-workload subdomains for the workload's source and
    one white-noise vector (8 tiles), from the oracle's tiles and direct local solves."""
    kh = w.k / S.prob.n
    xs, ts = [], []
    for r in (w.rhs[0], crandn(rng, S.ndof)):
        x, s = cnn.tile_inputs(S, r, T, kh)
        us = [sd.direct(r[sd.geom.idx]) for sd in S.subs]
        xs.append(x)
        ts.append(cnn.tile_targets(S, us, s, T))
    return bf16_round(np.concatenate(xs)), np.concatenate(ts).astype(np.float32).astype(np.float64)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_net_forward_matches_oracle(torch):
    _case("net forward")
    from paper_2103_17081_amd.binding import GuessNet
    w, S = oracle_for("small")
    rng = np.random.default_rng(5)
    x, _ = small_batch(S, w, 32, rng)
    x = np.concatenate([x, bf16_round(rng.standard_normal((2, 32, 32, 4)))])
    v = oracle_params(7, WIDTHS)
    net = GuessNet(WIDTHS, tile=32, max_batch=16)
    net.set_params(v.astype(np.float32))
    y = to_np(net.forward(to_gpu(torch, x.astype(np.float32))))
    yo, _ = cnn.forward(cnn.unflatten(v, WIDTHS), x)
    for b in range(x.shape[0]):
        e = rel(y[b], yo[b])
        print("tile", b, "rel err", e)
        assert e <= 3e-2
    assert np.abs(net.get_params() - v.astype(np.float32)).max() == 0.0
    net.close()


def test_net_forward_tile64_matches_oracle(torch):
    _case("net forward tile 64")
    from paper_2103_17081_amd.binding import GuessNet
    rng = np.random.default_rng(6)
    x = bf16_round(rng.standard_normal((3, 64, 64, 4)))
    x[:, 50:, :, :] = 0.0
    v = oracle_params(8, WIDTHS)
    net = GuessNet(WIDTHS, tile=64, max_batch=4)
    net.set_params(v.astype(np.float32))
    y = to_np(net.forward(to_gpu(torch, x.astype(np.float32))))
    yo, _ = cnn.forward(cnn.unflatten(v, WIDTHS), x)
    for b in range(3):
        assert rel(y[b], yo[b]) <= 3e-2
    net.close()


def test_net_gradient_matches_oracle(torch):
    _case("net gradient")
    from paper_2103_17081_amd.binding import GuessNet
    w, S = oracle_for("small")
    rng = np.random.default_rng(9)
    x, t = small_batch(S, w, 32, rng)
    v = oracle_params(11, WIDTHS)
    kh = w.k / S.prob.n
    net = GuessNet(WIDTHS, tile=32, max_batch=8, train=True)
    net.set_params(v.astype(np.float32))
    loss, g = net.gradient(to_gpu(torch, x.astype(np.float32)), to_gpu(torch, t.astype(np.float32)),
                           desc_array(S, kh, 2), w_res=1.0, w_err=0.1, want_grad=True)
    g = to_np(g).astype(np.float64)
    p = cnn.unflatten(v, WIDTHS)
    y, c = cnn.forward(p, x)
    lo, dy = cnn.loss(y, t, cnn.tile_operators(S) * 2, 1.0, 0.1)
    go = cnn.flatten(cnn.backward(p, c, dy))
    print("loss gpu", loss, "oracle", lo)
    assert abs(loss - lo) <= 2e-2 * lo
    gp, gop = cnn.unflatten(g, WIDTHS), cnn.unflatten(go, WIDTHS)
    for k in gop:
        e = rel(gp[k], gop[k])
        print(k, "rel err", e)
        assert e <= 5e-2, k
    cos = np.dot(g, go) / (np.linalg.norm(g) * np.linalg.norm(go))
    assert cos >= 0.999
    net.close()


def test_net_adam_first_step(torch):
    """First Adam step from zero state moves each parameter by -lr g / (|g| + eps); on the
    components whose oracle gradient is not tiny, GPU and oracle agree."""
    _case("net adam")
    from paper_2103_17081_amd.binding import GuessNet
    w, S = oracle_for("small")
    rng = np.random.default_rng(12)
    x, t = small_batch(S, w, 32, rng)
    v = oracle_params(13, WIDTHS)
    net = GuessNet(WIDTHS, tile=32, max_batch=8, train=True)
    net.set_params(v.astype(np.float32))
    net.gradient(to_gpu(torch, x.astype(np.float32)), to_gpu(torch, t.astype(np.float32)),
                 desc_array(S, w.k / S.prob.n, 2), w_res=1.0, w_err=0.1)
    lr = 1e-3
    net.adam(lr)
    after = net.get_params().astype(np.float64)
    p = cnn.unflatten(v, WIDTHS)
    y, c = cnn.forward(p, x)
    _, dy = cnn.loss(y, t, cnn.tile_operators(S) * 2, 1.0, 0.1)
    go = cnn.backward(p, c, dy)
    q = {k: p[k].copy() for k in p}
    cnn.adam(q, go, {}, lr=lr)
    gflat, qflat = cnn.flatten(go), cnn.flatten(q)
    big = np.abs(gflat) > 0.1 * np.abs(gflat).max()
    assert big.sum() > 10
    assert np.abs(after[big] - qflat[big]).max() <= 1e-6
    net.close()


@pytest.mark.parametrize("name,T", [("small", 32), ("large", 64)])
def test_tiles_match_oracle(torch, name, T):
    _case("tiles", name)
    w, S = oracle_for(name)
    kh = w.k / S.prob.n
    with solver_for(name, precision=64) as gpu:
        rng = np.random.default_rng(21)
        r = crandn(rng, S.ndof)
        x, s = gpu.tiles(to_gpu(torch, r), T)
        xo, so = cnn.tile_inputs(S, r, T, kh)
        assert np.abs(to_np(s) - so).max() <= 1e-12 * so.max()
        assert np.abs(to_np(x) - xo).max() <= 2e-6 * np.abs(xo).max()
        us = [crandn(rng, sd.geom.ndof) for sd in S.subs]
        t = gpu.packed_to_tiles(to_gpu(torch, pack(S, gpu, us)), s, T)
        to = cnn.tile_targets(S, us, so, T)
        assert np.abs(to_np(t) - to).max() <= 2e-6 * np.abs(to).max()
        descs = gpu.tile_descs()
        for j, (nx, ny, e, rb) in enumerate(oracle_descs(S)):
            d = descs[j]
            assert (d.nx, d.ny, d.edges) == (nx, ny, e)
            assert d.edges == 0 or (d.robin & d.edges) == rb
            assert abs(d.kh - kh) <= 1e-15


def _fixture_net(torch):
    from paper_2103_17081_amd.binding import GuessNet
    v = np.load(os.path.join(HERE, "golden", "guess_small_params.npy"))
    net = GuessNet((16, 16, 16, 16), tile=32, max_batch=8)
    net.set_params(v)
    return net, v.astype(np.float64)


def test_guess_path_matches_oracle(torch):
    """Preconditioner apply with the attached (oracle-trained) network: per subdomain the
    accept / reject decision equals the oracle's wherever the oracle's deflated-residual
    ratio is not within 5% of 1, rejected guesses give the zero-guess iteration count,
    accepted ones are within one iteration of the oracle's guessed solve.  The local
    solutions are then checked one by one: the batched subdomain solves are run on the
    same right-hand sides with the GPU network's guesses passed as packed initial guesses,
    every local solution u_j must satisfy ||f_j - B_j u_j|| <= tol ||P_j f_j|| recomputed
    with the oracle's matrices, and the apply's output must equal those solutions on the
    owned nodes; with the oracle network's guesses the iteration counts and solutions must
    equal the oracle's guessed solves."""
    _case("guess path")
    w, S = oracle_for("small")
    net, v = _fixture_net(torch)
    kh = w.k / S.prob.n
    tol = w.inner_tol
    with solver_for("small", precision=64) as gpu:
        gpu.set_guess(net)
        rng = np.random.default_rng(31)
        for r in (w.rhs[0], crandn(rng, S.ndof), crandn(rng, S.ndof)):
            z = to_np(gpu.apply_preconditioner(to_gpu(torch, r)))
            iters, flags = gpu.last_inner()
            x, s = cnn.tile_inputs(S, r, 32, kh)
            y, _ = cnn.forward(cnn.unflatten(v, (16, 16, 16, 16)), bf16_round(x))
            gs = cnn.guesses(S, y, s)
            fs = [r[sd.geom.idx] for sd in S.subs]
            zo = np.zeros_like(r)
            oracle_solves = []
            for j, sd in enumerate(S.subs):
                f = fs[j]
                Pf = sd.defl.P(f)
                ratio = np.linalg.norm(Pf - sd.defl.PB(gs[j])) / np.linalg.norm(Pf)
                u, k, acc = sd.deflated_gmres(f, tol, 100, guess=gs[j])
                _, k0, _ = sd.deflated_gmres(f, tol, 100)
                oracle_solves.append((u, k, acc, ratio))
                zo[sd.geom.idx[sd.geom.owned]] = u[sd.geom.owned]
                print(f"sub {j}: ratio {ratio:.3f} oracle acc {acc} its {k} (zero guess {k0}); "
                      f"gpu acc {bool(flags[j] & 1)} its {iters[j]}", flush=True)
                if abs(ratio - 1.0) > 0.05:
                    assert bool(flags[j] & 1) == acc
                if not flags[j] & 1:
                    assert iters[j] == k0
                elif acc:
                    assert abs(int(iters[j]) - k) <= 1
            F = to_gpu(torch, pack(S, gpu, fs))
            # the GPU network's guesses as packed initial guesses: the same solves as the apply
            xg, sg = gpu.tiles(to_gpu(torch, r), 32)
            yg = to_np(net.forward(xg))
            gg = cnn.guesses(S, yg.astype(np.float64), to_np(sg))
            ug, itg, flg = gpu.op_inner_solve(F, guess=to_gpu(torch, pack(S, gpu, gg)))
            assert np.array_equal(flg & 1, flags & 1)
            assert np.array_equal(itg, iters)
            for j, (sd, uj) in enumerate(zip(S.subs, unpack(S, gpu, to_np(ug)))):
                g = sd.geom
                res = np.linalg.norm(fs[j] - sd.B @ uj)
                assert res <= tol * np.linalg.norm(sd.defl.P(fs[j])) * (1 + 1e-6), (j, res)
                np.testing.assert_allclose(z[g.idx[g.owned]], uj[g.owned], rtol=0,
                                           atol=1e-9 * np.abs(uj).max())
            # the oracle network's guesses: counts and solutions equal the oracle's guessed solves
            uo, ito, flo = gpu.op_inner_solve(F, guess=to_gpu(torch, pack(S, gpu, gs)))
            for j, (uj, (u, k, acc, ratio)) in enumerate(zip(unpack(S, gpu, to_np(uo)), oracle_solves)):
                if abs(ratio - 1.0) > 1e-8:
                    assert bool(flo[j] & 1) == acc, j
                # FP64 on both sides: equal counts unless an estimate lands within rounding of
                # the tolerance, then one iteration apart and the solutions tolerance-close
                assert abs(int(ito[j]) - k) <= 1, (j, ito[j], k)
                assert rel(uj, u) <= (1e-8 if ito[j] == k else 10 * tol), j
            assert rel(z, zo) <= 0.1
    net.close()


def test_guess_solve_converges_and_graph_matches_eager(torch):
    """Full solves with the attached network: converged to the outer tolerance (true
    residual), graph replay bitwise equal to eager steps, and the acceptance counter set."""
    _case("guess solve graph")
    w, S = oracle_for("small")
    net, _ = _fixture_net(torch)
    with solver_for("small", precision=32) as gpu:
        gpu.set_guess(net)
        f = to_gpu(torch, w.rhs[0])
        u1, st1 = gpu.solve(f)
        gpu.set_graph(False)
        u2, st2 = gpu.solve(f)
        u1, u2 = to_np(u1), to_np(u2)
        relres = np.linalg.norm(w.rhs[0] - S.A @ u1) / np.linalg.norm(w.rhs[0])
        print("with guess:", st1, "relres", relres, flush=True)
        assert st1["status"] == "DD_OK" and relres <= 1e-6
        assert st1["guesses_accepted"] > 0
        assert np.array_equal(u1, u2)
        assert st2["ms_guess"] > 0.0
        gpu.set_guess(None)
        _, st3 = gpu.solve(f)
        assert st3["guesses_accepted"] == 0
    net.close()
