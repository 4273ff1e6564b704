"""Write tests/golden/guess_small_params.npy: guess-network parameters trained by the
float64 oracle (numpy forward/backward and Adam, oracle/cnn.py) on the 2 x 2 small
workload, so that the GPU integration test runs a network whose guesses the subdomain
solver actually accepts.  Calls only oracle/ and the seeded input generators.

    python tests/golden/make_guess_fixture.py        (about two minutes on one core)

Training data: complex white-noise global vectors r (seeded), network inputs built from
R_j r, targets s_j B_j^{-1} R_j r from direct local solves; loss weights w_res = 1,
w_err = 0.1; 400 Adam steps of 8 tiles, learning rate 3e-3; widths (16, 16, 16, 16),
32 x 32 tiles.  Parameters are rounded to bfloat16 values (stored as float32) so both
sides of a parity test use identical weights.
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import cnn, schwarz  # noqa: E402
from paper_2103_17081_amd import inputs  # noqa: E402

WIDTHS = (16, 16, 16, 16)
TILE = 32
OUT = os.path.join(HERE, "guess_small_params.npy")


def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def main():
    w = inputs.workload("small")
    S = schwarz.Schwarz(schwarz.problem_from_workload(w))
    kh = w.k / S.prob.n
    ops = cnn.tile_operators(S)
    rng = np.random.default_rng(2103)
    p = cnn.init_params(rng, WIDTHS)
    state = {}
    n = S.A.shape[0]
    for it in range(400):
        xs, ts = [], []
        for _ in range(2):
            r = rng.standard_normal(n) + 1j * rng.standard_normal(n)
            x, s = cnn.tile_inputs(S, r, TILE, kh)
            us = [sd.direct(r[sd.geom.idx]) for sd in S.subs]
            xs.append(x)
            ts.append(cnn.tile_targets(S, us, s, TILE))
        X, T = np.concatenate(xs), np.concatenate(ts)
        y, c = cnn.forward(p, X)
        loss, dy = cnn.loss(y, T, ops * 2, 1.0, 0.1)
        cnn.adam(p, cnn.backward(p, c, dy), state, lr=3e-3)
        if it % 50 == 0:
            print(f"step {it}: loss {loss:.4f}", flush=True)
    v = cnn.flatten(p)
    np.save(OUT, bf16_round(v))
    print("wrote", OUT, v.size, "parameters")


if __name__ == "__main__":
    main()
