"""Learned initial guess: training-data generation, training loop, evaluation and the
weights file (a host driver around the dd_net C ABI; every numerical step runs in the
library's kernels).

Training pairs come from the method itself: a complex64-inner solve of a training
problem provides its outer FGMRES basis vectors v_j; for each, the network inputs are
the tiles of R_j v_j and the targets the tiles of complex128 deflated-GMRES subdomain
solves of the same right-hand sides at inner tolerance 1e-8, both scaled by
s_j = sqrt(n_j) / ||R_j v_j||.

    python -m paper_2103_17081_amd.guess train --out weights.ddnet   (on a GPU)

Weights file: 8 bytes b"DDHNET01", a little-endian uint32 header length, a JSON header
(widths, tile, nparams and training metadata), then nparams little-endian float32 in the
flat order of include/ddhelm.h (W1, b1, ..., W8, b8).
"""

from __future__ import annotations

import argparse
import json
import struct
import sys
import time

import numpy as np

from . import inputs
from .binding import DDError, GuessNet, Solver, TileDesc

MAGIC = b"DDHNET01"


# ---- weights file ---------------------------------------------------------------------

def save_weights(net: GuessNet, path: str, meta: dict | None = None):
    params = net.get_params()
    head = dict(meta or {})
    head.update(widths=list(net.widths), tile=net.tile, nparams=int(params.size))
    hb = json.dumps(head, sort_keys=True).encode()
    with open(path, "wb") as fh:
        fh.write(MAGIC)
        fh.write(struct.pack("<I", len(hb)))
        fh.write(hb)
        fh.write(params.astype("<f4").tobytes())


def read_weights(path: str):
    """(header dict, float32 parameters); raises ValueError on a malformed file."""
    with open(path, "rb") as fh:
        data = fh.read()
    if data[:8] != MAGIC:
        raise ValueError(f"{path}: not a guess-network weights file")
    (hl,) = struct.unpack("<I", data[8:12])
    head = json.loads(data[12:12 + hl].decode())
    params = np.frombuffer(data[12 + hl:], dtype="<f4").astype(np.float32)
    if params.size != head["nparams"]:
        raise ValueError(f"{path}: {params.size} parameters, header says {head['nparams']}")
    return head, params


def load_net(path: str, max_batch: int, tile: int | None = None) -> GuessNet:
    """The library reads and validates the file (dd_net_load; DD_EWEIGHTS if it is bad)."""
    return GuessNet.load(path, max_batch=max_batch, tile=tile or 0)


# ---- data ---------------------------------------------------------------------------

def make_solver(w, precision: int, **kw) -> Solver:
    kw.setdefault("inner_tol", w.inner_tol)
    kw.setdefault("outer_maxit", 4000)
    return Solver(w.k, n_intervals=w.n, cuts_x=w.cuts_x, cuts_y=w.cuts_y, overlap=w.overlap,
                  inner_precision=precision, **kw)


def collect(w, tile: int, vectors: int = 16, target_tol: float = 1e-8, target_maxit: int = 60):
    """Training pairs of one problem: (x [n, T, T, 4], t [n, T, T, 2], descs list, info)."""
    import torch
    f = torch.from_numpy(w.rhs[0]).to("cuda")
    with make_solver(w, 32) as s32:
        _, st = s32.solve(f)
        m = st["outer_iters"]
        js = sorted(set(np.linspace(0, max(m - 1, 0), vectors).round().astype(int).tolist()))
        basis = [s32.outer_basis(j).clone() for j in js]
    xs, ts, keep = [], [], []
    try:
        s64 = make_solver(w, 64, inner_tol=target_tol, inner_maxit=target_maxit, use_graph=False)
    except DDError as e:
        # the largest tiles of a problem may not fit the complex128 kernel's LDS at this
        # iteration cap: fewer kept iterations (targets that do not converge are dropped)
        if "LDS" not in str(e):
            raise
        s64 = make_solver(w, 64, inner_tol=target_tol, inner_maxit=target_maxit * 2 // 3, use_graph=False)
    with s64:
        descs = list(s64.tile_descs())
        for v in basis:
            x, s = s64.tiles(v, tile)
            F = s64.op_gather(v, 64)
            U, _, flags = s64.op_inner_solve(F)
            t = s64.packed_to_tiles(U, s, tile)
            ok = torch.from_numpy(((flags & 2) == 0)).to("cuda") & (s > 0)
            xs.append(x[ok])
            ts.append(t[ok])
            keep.extend([descs[j] for j in np.nonzero(ok.cpu().numpy())[0]])
    info = dict(name=w.name, k=w.k, n=w.n, nsub=len(descs), outer_iters=m, vectors=len(basis),
                pairs=len(keep))
    return torch.cat(xs), torch.cat(ts), keep, info


# Training problems: blocks of about 40 cells (widths perturbed by +-25%), the size of the
# large evaluation workload's subdomains, for the 64 tile; every tile stays below the network
# tile, and the complex128 target solves (inner_maxit 60) within the kernel's LDS budget.
BLOCK = {32: 20, 64: 40}


def build_dataset(seeds, tile: int, vectors: int = 16, log=print, block: int | None = None):
    import torch
    X, T, D, infos = [], [], [], []
    for sd in seeds:
        w = inputs.training_problem(sd, block=block or BLOCK.get(tile, 32))
        t0 = time.perf_counter()
        x, t, d, info = collect(w, tile, vectors)
        info["seconds"] = round(time.perf_counter() - t0, 2)
        log(f"data {info}")
        X.append(x)
        T.append(t)
        D.extend(d)
        infos.append(info)
    return torch.cat(X), torch.cat(T), D, infos


def desc_batch(descs, idx):
    arr = (TileDesc * len(idx))()
    for i, j in enumerate(idx):
        d = descs[j]
        arr[i].nx, arr[i].ny, arr[i].edges, arr[i].robin, arr[i].kh = d.nx, d.ny, d.edges, d.robin, d.kh
    return arr


# ---- training -------------------------------------------------------------------------

def train(net: GuessNet, X, T, descs, steps: int, batch: int = 64, lr: float = 1e-3, w_res: float = 0.1,
          w_err: float = 1.0, seed: int = 0, log=print, every: int = 200):
    """Adam on minibatches drawn uniformly (seeded); cosine learning-rate decay to lr/20.
    Returns the list of (step, loss)."""
    import torch
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    hist = []
    for it in range(steps):
        idx = np.sort(rng.choice(n, size=min(batch, n), replace=False))
        ti = torch.from_numpy(idx).to("cuda")
        x = X.index_select(0, ti).contiguous()
        t = T.index_select(0, ti).contiguous()
        loss, _ = net.gradient(x, t, desc_batch(descs, idx), w_res=w_res, w_err=w_err)
        cur = lr * (0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * it / max(steps - 1, 1))))
        net.adam(cur)
        hist.append((it, loss))
        if it % every == 0 or it == steps - 1:
            log(f"step {it}: loss {loss:.4f} lr {cur:.2e}")
    return hist


def validation_loss(net: GuessNet, X, T, descs, w_res: float, w_err: float, batch: int = 64):
    tot, cnt = 0.0, 0
    for a in range(0, X.shape[0], batch):
        idx = np.arange(a, min(a + batch, X.shape[0]))
        loss, _ = net.gradient(X[a:a + len(idx)].contiguous(), T[a:a + len(idx)].contiguous(),
                               desc_batch(descs, idx), w_res=w_res, w_err=w_err)
        tot += loss * len(idx)
        cnt += len(idx)
    return tot / max(cnt, 1)


# ---- evaluation (ablation) ------------------------------------------------------------------

def ablation(w, net: GuessNet, precision: int = 32, vectors: int = 8):
    """Subdomain solves of held-out right-hand sides (outer basis vectors of a zero-guess
    solve of w) with and without the guess: mean inner iterations, acceptance rate and
    time per preconditioner application; then full solves with and without the guess."""
    import torch
    f = torch.from_numpy(w.rhs[0]).to("cuda")
    out = {}
    with make_solver(w, precision) as s:
        u0, st0 = s.solve(f)
        m = st0["outer_iters"]
        js = sorted(set(np.linspace(0, max(m - 1, 0), vectors).round().astype(int).tolist()))
        basis = [s.outer_basis(j).clone() for j in js]
        rows = []
        for mode in ("zero", "guess"):
            s.set_guess(net if mode == "guess" else None)
            its, acc, ms = [], [], []
            for v in basis:
                s.apply_preconditioner(v)          # warm
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                s.apply_preconditioner(v)
                e1.record()
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
                it, fl = s.last_inner()
                its.append(it.mean())
                acc.append((fl & 1).mean())
            rows.append(dict(mode=mode, mean_inner=float(np.mean(its)), accepted=float(np.mean(acc)),
                             ms_apply=float(np.median(ms))))
        out["applies"] = rows
        solves = []
        for mode in ("zero", "guess"):
            s.set_guess(net if mode == "guess" else None)
            s.solve(f)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, st = s.solve(f)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            r = f - s.op_global_apply(u)
            solves.append(dict(mode=mode, seconds=dt, outer_iters=st["outer_iters"],
                               avg_inner=st["inner_iters_total"] / max(st["subdomain_solves"], 1),
                               accepted=st["guesses_accepted"], status=st["status"],
                               true_relres=float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(f))))
        s.set_guess(None)
        out["solves"] = solves
    return out


def applies(w, net: GuessNet, repeat: int = 20, precision: int = 32):
    """`repeat` preconditioner applications of the normalised right-hand side with the
    network attached, then `repeat` without (for kernel traces); returns the mean
    inner iterations of the last application of each."""
    import torch
    f = torch.from_numpy(w.rhs[0]).to("cuda")
    r = f / torch.linalg.vector_norm(f)
    out = {}
    with make_solver(w, precision) as s:
        for mode in ("guess", "zero"):
            s.set_guess(net if mode == "guess" else None)
            for _ in range(repeat):
                s.apply_preconditioner(r)
            torch.cuda.synchronize()
            it, fl = s.last_inner()
            out[mode] = dict(mean_inner=float(it.mean()), accepted=float((fl & 1).mean()))
        s.set_guess(None)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    for name in ("ablation", "applies"):
        sp = sub.add_parser(name)
        sp.add_argument("--weights", required=True)
        sp.add_argument("--workload", default="large")
        sp.add_argument("--repeat", type=int, default=20)
    tr = sub.add_parser("train")
    tr.add_argument("--out", required=True)
    tr.add_argument("--tile", type=int, default=64)
    tr.add_argument("--problems", type=int, default=8)
    tr.add_argument("--vectors", type=int, default=16)
    tr.add_argument("--steps", type=int, default=4000)
    tr.add_argument("--batch", type=int, default=64)
    tr.add_argument("--lr", type=float, default=1e-3)
    tr.add_argument("--w-res", type=float, default=0.1)
    tr.add_argument("--w-err", type=float, default=1.0)
    tr.add_argument("--eval", default="large", help="workload of the ablation after training ('' for none)")
    tr.add_argument("--heldout-problems", type=int, default=1)
    tr.add_argument("--block", type=int, default=0, help="cells per training block (0: by tile)")
    tr.add_argument("--widths", type=int, nargs=4, default=[16, 32, 64, 64])
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)  # noqa: E731
    if a.cmd in ("ablation", "applies"):
        w = inputs.workload(a.workload)
        head, _ = read_weights(a.weights)
        net = load_net(a.weights, max_batch=len(w.cuts_x) ** 2, tile=head["tile"])
        res = ablation(w, net) if a.cmd == "ablation" else applies(w, net, a.repeat)
        log(json.dumps(res))
        net.close()
        return 0
    X, T, D, infos = build_dataset(range(1000, 1000 + a.problems), a.tile, a.vectors, log, a.block)
    Xv, Tv, Dv, _ = build_dataset(range(2000, 2000 + a.heldout_problems), a.tile, a.vectors, log, a.block)
    net = GuessNet(tuple(a.widths), tile=a.tile, max_batch=max(a.batch, 256), train=True)
    log(f"training pairs {X.shape[0]}, held-out {Xv.shape[0]}, parameters {net.nparams}")
    t0 = time.perf_counter()
    hist = train(net, X, T, D, a.steps, a.batch, a.lr, a.w_res, a.w_err, log=log)
    secs = time.perf_counter() - t0
    vl = validation_loss(net, Xv, Tv, Dv, a.w_res, a.w_err)
    tl = validation_loss(net, X[:Xv.shape[0]], T[:Xv.shape[0]], D[:Xv.shape[0]], a.w_res, a.w_err)
    log(f"trained {a.steps} steps in {secs:.1f} s; training-set loss {tl:.4f}, held-out loss {vl:.4f}")
    meta = dict(problems=infos, steps=a.steps, batch=a.batch, lr=a.lr, w_res=a.w_res, w_err=a.w_err,
                final_loss=hist[-1][1], heldout_loss=vl, train_loss=tl, train_pairs=int(X.shape[0]),
                heldout_pairs=int(Xv.shape[0]), train_seconds=round(secs, 1))
    save_weights(net, a.out, meta)
    log(f"wrote {a.out}")
    if a.eval:
        infer = load_net(a.out, max_batch=1024, tile=a.tile)
        log(json.dumps(ablation(inputs.workload(a.eval), infer)))
        infer.close()
    net.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
