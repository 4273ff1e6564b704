"""float64 reference of the learned initial-guess network (oracle; test infrastructure only).

The paper has no learned component; the subdomain solver it describes starts GMRES
from a zero guess (Sec. 3).  This library adds an optional initial guess produced by a
small convolutional encoder-decoder from the subdomain right-hand side; the guess is
used only if it lowers the deflated residual, so the method itself is unchanged.

Tensors are NHWC.  Input channels: (Re f, Im f) of the local right-hand side
normalised by its norm, the constant k h, and a boundary-type mask; output channels:
(Re g, Im g) of the guess in the same normalised units.

Layers (widths c1..c4; "conv" = 3x3 correlation with zero padding, stride 1):
    a1 = relu(conv(x,  W1) + b1)                      c1 channels, H x W
    a2 = relu(conv(pool(a1), W2) + b2)                c2, H/2
    a3 = relu(conv(pool(a2), W3) + b3)                c3, H/4
    a4 = relu(conv(pool(a3), W4) + b4)                c4, H/8
    a5 = relu(conv(cat(up(a4), a3), W5) + b5)         c2, H/4
    a6 = relu(conv(cat(up(a5), a2), W6) + b6)         c1, H/2
    a7 = relu(conv(cat(up(a6), a1), W7) + b7)         c1, H
    y  = a7 W8 + b8                                   2,  H     (1x1)
pool: 2x2 average; up: 2x nearest; cat: channel concatenation (first operand first).
Weights of a 3x3 layer are indexed [ky][kx][cin][cout] and act as
out[y, x, co] = b[co] + sum_{ky, kx, ci} W[ky, kx, ci, co] in[y + ky - 1, x + kx - 1, ci].

Loss (per batch, see `loss`): a residual term ||B (y - t)||^2 / ||B t||^2 with B the
subdomain operator, and an error term ||y - t||^2 / ||t||^2, both over the subdomain's
nodes, with t the normalised target solution.  A guess u_j = y_j / s_j is kept by the
subdomain solver only if it lowers the deflated residual (Sec. 2, eq. 4), which is why
the residual term is the one the training weights most.
"""

from __future__ import annotations

import numpy as np

LAYERS = ["W1", "W2", "W3", "W4", "W5", "W6", "W7", "W8"]


def layer_shapes(widths=(16, 32, 64, 64), cin=4, cout=2):
    c1, c2, c3, c4 = widths
    return {
        "W1": (3, 3, cin, c1), "W2": (3, 3, c1, c2), "W3": (3, 3, c2, c3), "W4": (3, 3, c3, c4),
        "W5": (3, 3, c4 + c3, c2), "W6": (3, 3, c2 + c2, c1), "W7": (3, 3, c1 + c1, c1),
        "W8": (1, 1, c1, cout),
    }


def init_params(rng: np.random.Generator, widths=(16, 32, 64, 64)):
    """He-normal weights, zero biases."""
    p = {}
    for name, shp in layer_shapes(widths).items():
        fan_in = shp[0] * shp[1] * shp[2]
        p[name] = rng.standard_normal(shp) * np.sqrt(2.0 / fan_in)
        p["b" + name[1:]] = np.zeros(shp[3])
    return p


def flatten(p) -> np.ndarray:
    """Parameters in the order W1, b1, W2, b2, ..., W8, b8 (each array C-ordered)."""
    return np.concatenate([np.concatenate([p[w].ravel(), p["b" + w[1:]].ravel()]) for w in LAYERS])


def unflatten(v: np.ndarray, widths=(16, 32, 64, 64)):
    p, o = {}, 0
    for name, shp in layer_shapes(widths).items():
        n = int(np.prod(shp))
        p[name] = v[o:o + n].reshape(shp)
        o += n
        p["b" + name[1:]] = v[o:o + shp[3]].copy()
        o += shp[3]
    return p


def conv(x, W, b):
    """Zero-padded stride-1 correlation with a kh x kw kernel, NHWC."""
    kh, kw = W.shape[0], W.shape[1]
    ph, pw = kh // 2, kw // 2
    B, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (ph, ph), (pw, pw), (0, 0)))
    out = np.broadcast_to(b, (B, H, Wd, W.shape[3])).copy()
    for ky in range(kh):
        for kx in range(kw):
            out += np.einsum("bhwc,cd->bhwd", xp[:, ky:ky + H, kx:kx + Wd, :], W[ky, kx])
    return out


def conv_backward(x, W, dout):
    """Gradients of conv(x, W, b) with respect to x, W and b."""
    kh, kw = W.shape[0], W.shape[1]
    ph, pw = kh // 2, kw // 2
    B, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (ph, ph), (pw, pw), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ky in range(kh):
        for kx in range(kw):
            dW[ky, kx] = np.einsum("bhwc,bhwd->cd", xp[:, ky:ky + H, kx:kx + Wd, :], dout)
            dxp[:, ky:ky + H, kx:kx + Wd, :] += np.einsum("bhwd,cd->bhwc", dout, W[ky, kx])
    dx = dxp[:, ph:ph + H, pw:pw + Wd, :]
    return dx, dW, dout.sum(axis=(0, 1, 2))


def pool(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool_backward(dout):
    return 0.25 * np.repeat(np.repeat(dout, 2, axis=1), 2, axis=2)


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_backward(dout):
    B, H, W, C = dout.shape
    return dout.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def relu(x):
    return np.maximum(x, 0.0)


def forward(p, x):
    """Returns the output and the activations needed by backward."""
    c = {"x": x}
    c["a1"] = relu(conv(x, p["W1"], p["b1"]))
    c["p1"] = pool(c["a1"])
    c["a2"] = relu(conv(c["p1"], p["W2"], p["b2"]))
    c["p2"] = pool(c["a2"])
    c["a3"] = relu(conv(c["p2"], p["W3"], p["b3"]))
    c["p3"] = pool(c["a3"])
    c["a4"] = relu(conv(c["p3"], p["W4"], p["b4"]))
    c["c5"] = np.concatenate([up(c["a4"]), c["a3"]], axis=3)
    c["a5"] = relu(conv(c["c5"], p["W5"], p["b5"]))
    c["c6"] = np.concatenate([up(c["a5"]), c["a2"]], axis=3)
    c["a6"] = relu(conv(c["c6"], p["W6"], p["b6"]))
    c["c7"] = np.concatenate([up(c["a6"]), c["a1"]], axis=3)
    c["a7"] = relu(conv(c["c7"], p["W7"], p["b7"]))
    y = conv(c["a7"], p["W8"], p["b8"])
    return y, c


def backward(p, c, dy):
    """Gradients of all parameters given dL/dy."""
    g = {}

    def layer(dout_pre, inp, name):
        dx, dW, db = conv_backward(inp, p[name], dout_pre)
        g[name], g["b" + name[1:]] = dW, db
        return dx

    def relu_b(dout, a):
        return dout * (a > 0)

    da7 = layer(dy, c["a7"], "W8")
    dc7 = layer(relu_b(da7, c["a7"]), c["c7"], "W7")
    n6 = c["a6"].shape[3]
    da6 = up_backward(dc7[..., :n6])
    da1 = dc7[..., n6:].copy()
    dc6 = layer(relu_b(da6, c["a6"]), c["c6"], "W6")
    n5 = c["a5"].shape[3]
    da5 = up_backward(dc6[..., :n5])
    da2 = dc6[..., n5:].copy()
    dc5 = layer(relu_b(da5, c["a5"]), c["c5"], "W5")
    n4 = c["a4"].shape[3]
    da4 = up_backward(dc5[..., :n4])
    da3 = dc5[..., n4:].copy()
    dp3 = layer(relu_b(da4, c["a4"]), c["p3"], "W4")
    da3 += pool_backward(dp3)
    dp2 = layer(relu_b(da3, c["a3"]), c["p2"], "W3")
    da2 += pool_backward(dp2)
    dp1 = layer(relu_b(da2, c["a2"]), c["p1"], "W2")
    da1 += pool_backward(dp1)
    layer(relu_b(da1, c["a1"]), c["x"], "W1")
    return g


def loss(y, t, tiles, w_res=1.0, w_err=0.0):
    """Training loss and its gradient with respect to y.

    Sample b covers the nodes (x < nx_b, y < ny_b) of its tile; on them e = y - t is read
    as the complex local vector (x fastest) and B_b is the subdomain operator:
        L = mean_b ( w_res ||B_b e||^2 / ||B_b t||^2 + w_err ||e||^2 / ||t||^2 ),
    d L / d(Re y, Im y) = (Re, Im) of (2 w_res B^H B e / ||B t||^2 + 2 w_err e / ||t||^2) / n_b.
    `tiles` is a list of dicts with keys nx, ny and B (matrix, may be None when w_res = 0).
    """
    nb = y.shape[0]
    dy = np.zeros_like(y)
    total = 0.0
    for b, tl in enumerate(tiles):
        nx, ny = tl["nx"], tl["ny"]
        ys = y[b, :ny, :nx, 0] + 1j * y[b, :ny, :nx, 1]
        ts = t[b, :ny, :nx, 0] + 1j * t[b, :ny, :nx, 1]
        e = (ys - ts).reshape(-1)
        tv = ts.reshape(-1)
        g = np.zeros_like(e)
        if w_err:
            den = np.vdot(tv, tv).real
            den = den if den > 0 else 1.0
            total += w_err * np.vdot(e, e).real / den
            g += 2.0 * w_err * e / den
        if w_res:
            B = tl["B"]
            r = B @ e
            bt = B @ tv
            den = np.vdot(bt, bt).real
            den = den if den > 0 else 1.0
            total += w_res * np.vdot(r, r).real / den
            g += 2.0 * w_res * (B.conj().T @ r) / den
        g = g.reshape(ny, nx) / nb
        dy[b, :ny, :nx, 0] = g.real
        dy[b, :ny, :nx, 1] = g.imag
    return total / nb, dy


# ---- tiles of a Schwarz problem (local right-hand sides and solutions) -------------------

def impedance_node_mask(g, n: int) -> np.ndarray:
    """[ny, nx] bool: local node lies on an impedance side of its subdomain (a side of the
    overlapping rectangle that is interior to the domain and carries local nodes)."""
    m = np.zeros((g.ny, g.nx), dtype=bool)
    if g.i0 == g.ax and g.ax > 0:
        m[:, 0] = True
    if g.i1 == g.bx and g.bx < n:
        m[:, -1] = True
    if g.j0 == g.ay and g.ay > 0:
        m[0, :] = True
    if g.j1 == g.by and g.by < n:
        m[-1, :] = True
    return m


def tile_inputs(S, r: np.ndarray, T: int, kh: float):
    """Network inputs [nsub, T, T, 4] of the local right-hand sides R_j r and the scales
    s_j = sqrt(n_j) / ||R_j r|| (0 for a zero right-hand side)."""
    n = S.prob.n
    x = np.zeros((len(S.subs), T, T, 4))
    scale = np.zeros(len(S.subs))
    for j, sd in enumerate(S.subs):
        g = sd.geom
        f = r[g.idx]
        nrm = np.linalg.norm(f)
        s = np.sqrt(g.ndof) / nrm if nrm > 0 else 0.0
        scale[j] = s
        fs = (s * f).reshape(g.ny, g.nx)
        x[j, :g.ny, :g.nx, 0] = fs.real
        x[j, :g.ny, :g.nx, 1] = fs.imag
        x[j, :g.ny, :g.nx, 2] = kh
        x[j, :g.ny, :g.nx, 3] = np.where(impedance_node_mask(g, n), -1.0, 1.0)
    return x, scale


def tile_targets(S, us, scale, T: int):
    """Targets [nsub, T, T, 2] = s_j u_j placed like the inputs."""
    t = np.zeros((len(S.subs), T, T, 2))
    for j, sd in enumerate(S.subs):
        g = sd.geom
        u = (scale[j] * us[j]).reshape(g.ny, g.nx)
        t[j, :g.ny, :g.nx, 0] = u.real
        t[j, :g.ny, :g.nx, 1] = u.imag
    return t


def tile_operators(S):
    return [{"nx": sd.geom.nx, "ny": sd.geom.ny, "B": sd.B} for sd in S.subs]


def guesses(S, y, scale):
    """Local initial guesses u_j = y_j / s_j from network outputs (zero where s_j = 0)."""
    out = []
    for j, sd in enumerate(S.subs):
        g = sd.geom
        v = y[j, :g.ny, :g.nx, 0] + 1j * y[j, :g.ny, :g.nx, 1]
        out.append(v.reshape(-1) / scale[j] if scale[j] > 0 else np.zeros(g.ndof, dtype=complex))
    return out


def adam(p, g, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015) on every parameter array, in place."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m" + k, np.zeros_like(p[k]))
        v = state.setdefault("v" + k, np.zeros_like(p[k]))
        m[...] = beta1 * m + (1 - beta1) * g[k]
        v[...] = beta2 * v + (1 - beta2) * g[k] ** 2
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        p[k] -= lr * mh / (np.sqrt(vh) + eps)
