"""Reference network of the learned initial guess, in FP64 numpy.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the library and its binding never
do.  It shares no code with the HIP kernels.

The network is not part of the paper's method.  It predicts the initial
guess of the pressure Poisson solve of the projection step (Section 3,
Eq. 9, L = M G) from the right-hand side and the previous pressure.  What it
computes, written out plainly:

* ``pad(a)`` adds one cell on each side of the (z, y, x) axes: periodic in
  z and x, a copy of the edge cell in y.
* ``conv(a, W, b)[n, o, z, y, x] = b[o] + sum_{c, dz, dy, dx}
  W[o, c, dz, dy, dx] * pad(a)[n, c, z + dz, y + dy, x + dx]``.
* Four layers 2 -> 32 -> 32 -> 32 -> 1, ReLU after the first three; the
  output adds the input's channel 1 (the scaled previous pressure), so the
  layers learn a correction to the previous pressure.
* Loss = mean of (out - target)^2; gradients by the chain rule, with the
  adjoint of ``pad`` folding each halo cell back onto the cell it copies.
* Adam (Kingma and Ba, 2015) with bias correction.
* Input of a right-hand side b (plane-major, cell c of plane l at
  ``l * n_b + c``) and previous pressure p: f = (b - mean b) / (area * dz)
  (mean removed only for a singular operator), s = rms(f) (1 if zero),
  channels (f / s, p / s).  Guess x0 = s * (out - mean out) (mean removed
  only for a singular operator).

Parameters are one flat vector: per layer W[o][c][tap] with
tap = (dz*3 + dy)*3 + dx, then b[o].
"""
from __future__ import annotations

import numpy as np

C = 32
LAYERS = ((2, C, True), (C, C, True), (C, C, True), (C, 1, False))  # (c_in, c_out, relu)


def n_params() -> int:
    return sum(co * ci * 27 + co for ci, co, _ in LAYERS)


def unpack(params):
    """Flat parameters -> [(W[o, c, 3, 3, 3], b[o]), ...] in float64."""
    p = np.asarray(params, dtype=np.float64)
    assert p.size == n_params()
    out, o = [], 0
    for ci, co, _ in LAYERS:
        W = p[o:o + co * ci * 27].reshape(co, ci, 3, 3, 3)
        o += co * ci * 27
        out.append((W, p[o:o + co]))
        o += co
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def pad(a: np.ndarray) -> np.ndarray:
    """One halo cell per side of the last three axes (z, y, x)."""
    a = np.concatenate([a[..., -1:, :, :], a, a[..., :1, :, :]], axis=-3)  # z periodic
    a = np.concatenate([a[..., :, :1, :], a, a[..., :, -1:, :]], axis=-2)  # y edge copy
    a = np.concatenate([a[..., :, :, -1:], a, a[..., :, :, :1]], axis=-1)  # x periodic
    return a


def pad_adjoint(g: np.ndarray) -> np.ndarray:
    """Adjoint of ``pad``: each halo value is added to the cell it copied."""
    g = np.array(g, dtype=np.float64)
    x = g[..., :, :, 1:-1].copy()
    x[..., :, :, -1] += g[..., :, :, 0]
    x[..., :, :, 0] += g[..., :, :, -1]
    y = x[..., :, 1:-1, :].copy()
    y[..., :, 0, :] += x[..., :, 0, :]
    y[..., :, -1, :] += x[..., :, -1, :]
    z = y[..., 1:-1, :, :].copy()
    z[..., -1, :, :] += y[..., 0, :, :]
    z[..., 0, :, :] += y[..., -1, :, :]
    return z


def _window(ap, dz, dy, dx, shape):
    Z, Y, X = shape
    return ap[:, :, dz:dz + Z, dy:dy + Y, dx:dx + X]


def conv(a: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """a [n, c, Z, Y, X] -> [n, o, Z, Y, X]."""
    n, _, Z, Y, X = a.shape
    ap = pad(a)
    out = np.empty((n, W.shape[0], Z, Y, X))
    out[:] = b[None, :, None, None, None]
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                out += np.einsum("oc,nczyx->nozyx", W[:, :, dz, dy, dx], _window(ap, dz, dy, dx, (Z, Y, X)))
    return out


def forward(params, inp: np.ndarray):
    """Activations [input, h1, h2, h3, out] (hidden ones after the ReLU)."""
    acts = [np.asarray(inp, dtype=np.float64)]
    for (W, b), (_, _, relu) in zip(unpack(params), LAYERS):
        h = conv(acts[-1], W, b)
        acts.append(np.maximum(h, 0.0) if relu else h)
    acts[-1] = acts[-1] + acts[0][:, 1:2]
    return acts


def forward_at(params, inp: np.ndarray, n: int, z: int, y: int, x: int) -> float:
    """Output of the network at one cell of sample n, evaluated from that
    cell's receptive field alone, cell by cell: the value read at tap offset
    (dz, dy, dx) of cell (z, y, x) is the cell ((z + dz - 1) mod Z,
    clamp(y + dy - 1), (x + dx - 1) mod X).  For sampled checks of large
    grids."""
    layers = unpack(params)
    a = np.asarray(inp, dtype=np.float64)
    Z, Y, X = a.shape[2:]

    def src(c, dz, dy, dx):
        return ((c[0] + dz - 1) % Z, min(max(c[1] + dy - 1, 0), Y - 1), (c[2] + dx - 1) % X)

    taps = [(dz, dy, dx) for dz in range(3) for dy in range(3) for dx in range(3)]
    need = [{(z, y, x)}]
    for _ in range(len(layers)):
        need.append({src(c, *t) for c in need[-1] for t in taps})
    vals = {c: a[n, :, c[0], c[1], c[2]] for c in need[-1]}
    for li, ((W, b), (_, _, relu)) in enumerate(zip(layers, LAYERS)):
        new = {}
        for c in need[len(layers) - 1 - li]:
            acc = b.copy()
            for t in taps:
                acc = acc + W[:, :, t[0], t[1], t[2]] @ vals[src(c, *t)]
            new[c] = np.maximum(acc, 0.0) if relu else acc
        vals = new
    return float(vals[(z, y, x)][0] + a[n, 1, z, y, x])


def loss_and_grads(params, inp: np.ndarray, target: np.ndarray):
    """(loss, flat gradient) of mean((out - target)^2)."""
    layers = unpack(params)
    acts = forward(params, inp)
    out = acts[-1]
    t = np.asarray(target, dtype=np.float64).reshape(out.shape)
    loss = float(np.mean((out - t) ** 2))
    d = 2.0 * (out - t) / out.size
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        a = acts[l]
        shape = a.shape[2:]
        ap = pad(a)
        gW = np.empty_like(W)
        for dz in range(3):
            for dy in range(3):
                for dx in range(3):
                    gW[:, :, dz, dy, dx] = np.einsum("nozyx,nczyx->oc", d, _window(ap, dz, dy, dx, shape))
        grads[l] = (gW, d.sum(axis=(0, 2, 3, 4)))
        if l > 0:
            gpad = np.zeros_like(ap)
            for dz in range(3):
                for dy in range(3):
                    for dx in range(3):
                        _window(gpad, dz, dy, dx, shape)[...] += np.einsum("oc,nozyx->nczyx", W[:, :, dz, dy, dx], d)
            d = pad_adjoint(gpad) * (a > 0.0)
    return loss, pack(grads)


def adam(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (t >= 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def prepare(b, p_prev, area, dz: float, nx: int, ny: int, k: int, singular: bool):
    """Network input [1, 2, k, ny, nx] and the scale s of a right-hand side."""
    B = np.asarray(b, dtype=np.float64).reshape(k, ny, nx)
    mean = B.mean() if singular else 0.0
    f = (B - mean) / (np.asarray(area, dtype=np.float64).reshape(1, ny, nx) * dz)
    s = float(np.sqrt(np.mean(f * f)))
    s = s if s > 0.0 else 1.0
    P = np.zeros_like(B) if p_prev is None else np.asarray(p_prev, dtype=np.float64).reshape(k, ny, nx)
    return np.stack([f / s, P / s])[None], s


def guess(params, b, p_prev, area, dz: float, nx: int, ny: int, k: int, singular: bool) -> np.ndarray:
    """Initial guess x0, plane-major [k * nx * ny]."""
    inp, s = prepare(b, p_prev, area, dz, nx, ny, k, singular)
    out = forward(params, inp)[-1][0, 0]
    if singular:
        out = out - out.mean()
    return (s * out).ravel()
