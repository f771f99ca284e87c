"""FP64 oracle of the learned crosstalk filter -- TEST INFRASTRUCTURE.

Only tests/ and the smoke check import this module; the product library
never calls it.  It is plain numpy in float64, written from the textbook
definitions of the operations, and shares no code with the HIP kernels.

The filter is a 3-D U-Net that maps an RTM image made with one random-
boundary realisation (the image condition of Eq. (3), with the boundary of
the section on wavefield reconstruction) to the image averaged over many
realisations, whose uncorrelated boundary crosstalk has cancelled.  It is a
project extension of the method, not part of the paper.

Conventions (single sample): activations are arrays of shape (C, D, H, W),
weights (Cout, Cin, 3, 3, 3), biases (Cout,).  Convolutions are cross-
correlations with one cell of zero padding ("same" size):

    y[o, p] = b[o] + sum_{i, k} w[o, i, k] x[i, p + k - 1],   k in {0,1,2}^3.

Network (levels of 16, 32, 64, 128 channels, one convolution per level,
additive skips, residual output):

    e1 = relu(conv(x, w1) + b1)                       full size, 16
    e2 = relu(conv(pool(e1), w2) + b2)                 1/2, 32
    e3 = relu(conv(pool(e2), w3) + b3)                 1/4, 64
    e4 = relu(conv(pool(e3), w4) + b4)                 1/8, 128
    d3 = relu(conv(up(e4), w5) + b5) + e3              1/4, 64
    d2 = relu(conv(up(d3), w6) + b6) + e2              1/2, 32
    d1 = relu(conv(up(d2), w7) + b7) + e1              full, 16
    out = x + conv(d1, w8) + b8                        full, 1
    loss = mean((out - target)^2)

pool is the mean over 2x2x2 blocks and up the nearest-neighbour copy to
2x2x2 blocks.  With quant=True the oracle rounds to bfloat16 (round to
nearest even of the float32 value) exactly where the GPU path stores
bfloat16: every convolution input, every weight, the stored activations and
the gradients that feed a convolution; everything else is float64.  With
quant=False it is the exact float64 network (used for finite differences).
"""
from __future__ import annotations

import numpy as np

LEVELS = (16, 32, 64, 128)
# (name, cin, cout) of the eight convolutions
LAYERS = (("c1", 1, 16), ("c2", 16, 32), ("c3", 32, 64), ("c4", 64, 128),
          ("c5", 128, 64), ("c6", 64, 32), ("c7", 32, 16), ("c8", 16, 1))


def bf16(x):
    """Round to bfloat16: the float32 value rounded to nearest even at 8
    significand bits (float32 with the low 16 bits cleared), as float64."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)


def _taps():
    return [(kz, ky, kx) for kz in range(3) for ky in range(3) for kx in range(3)]


def conv3d(x, w, b=None):
    """Forward convolution, one tensordot over the channels per tap."""
    C, D, H, W = x.shape
    xp = np.pad(np.asarray(x, np.float64), ((0, 0), (1, 1), (1, 1), (1, 1)))
    y = np.zeros((w.shape[0], D, H, W))
    for kz, ky, kx in _taps():
        y += np.tensordot(w[:, :, kz, ky, kx], xp[:, kz:kz + D, ky:ky + H, kx:kx + W], axes=([1], [0]))
    if b is not None:
        y += np.asarray(b, np.float64)[:, None, None, None]
    return y


def conv3d_dgrad(dy, w):
    """Gradient with respect to the input: dx[i, q] = sum_{o,k} w[o,i,k] dy[o, q - k + 1]."""
    O, D, H, W = dy.shape
    dyp = np.pad(np.asarray(dy, np.float64), ((0, 0), (1, 1), (1, 1), (1, 1)))
    dx = np.zeros((w.shape[1], D, H, W))
    for kz, ky, kx in _taps():
        # dy[o, q - k + 1] = dyp[o, q - k + 2]
        sl = dyp[:, 2 - kz:2 - kz + D, 2 - ky:2 - ky + H, 2 - kx:2 - kx + W]
        dx += np.tensordot(w[:, :, kz, ky, kx], sl, axes=([0], [0]))
    return dx


def conv3d_wgrad(x, dy):
    """Gradients of the weights and bias: dw[o,i,k] = sum_p dy[o,p] x[i,p+k-1], db[o] = sum_p dy[o,p]."""
    C, D, H, W = x.shape
    xp = np.pad(np.asarray(x, np.float64), ((0, 0), (1, 1), (1, 1), (1, 1)))
    dw = np.zeros((dy.shape[0], C, 3, 3, 3))
    for kz, ky, kx in _taps():
        dw[:, :, kz, ky, kx] = np.tensordot(dy, xp[:, kz:kz + D, ky:ky + H, kx:kx + W], axes=([1, 2, 3], [1, 2, 3]))
    return dw, dy.sum(axis=(1, 2, 3))


def conv3d_at(x, w, b, points):
    """Forward convolution at chosen voxels only, from the definition:
    y[o, p] = b[o] + sum_{i, k} w[o, i, k] x[i, p + k - 1], with x = 0 outside.
    points: (n, 3) integer (z, y, x); returns (n, Cout)."""
    C, D, H, W = x.shape
    x = np.asarray(x, np.float64)
    out = np.zeros((len(points), w.shape[0]))
    for j, (z, y, xx) in enumerate(np.asarray(points, np.int64)):
        acc = np.zeros(w.shape[0]) if b is None else np.asarray(b, np.float64).copy()
        for kz, ky, kx in _taps():
            q = (z + kz - 1, y + ky - 1, xx + kx - 1)
            if 0 <= q[0] < D and 0 <= q[1] < H and 0 <= q[2] < W:
                acc += w[:, :, kz, ky, kx] @ x[:, q[0], q[1], q[2]]
        out[j] = acc
    return out


def conv3d_dgrad_at(dy, w, points):
    """Input gradient at chosen voxels only, from the definition:
    dx[i, q] = sum_{o, k} w[o, i, k] dy[o, q - k + 1], dy = 0 outside.
    points: (n, 3) integer (z, y, x); returns (n, Cin)."""
    O, D, H, W = dy.shape
    dy = np.asarray(dy, np.float64)
    out = np.zeros((len(points), w.shape[1]))
    for j, (z, y, xx) in enumerate(np.asarray(points, np.int64)):
        acc = np.zeros(w.shape[1])
        for kz, ky, kx in _taps():
            q = (z - kz + 1, y - ky + 1, xx - kx + 1)
            if 0 <= q[0] < D and 0 <= q[1] < H and 0 <= q[2] < W:
                acc += w[:, :, kz, ky, kx].T @ dy[:, q[0], q[1], q[2]]
        out[j] = acc
    return out


def pool2(x):
    """Mean over 2x2x2 blocks."""
    C, D, H, W = x.shape
    return x.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).mean(axis=(2, 4, 6))


def pool2_bwd(g):
    """Adjoint of pool2: each fine cell receives 1/8 of its block's gradient."""
    return up2(g) / 8.0


def up2(x):
    """Nearest-neighbour upsampling by 2 along each axis."""
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def up2_bwd(g):
    """Adjoint of up2: sum over each 2x2x2 block."""
    C, D, H, W = g.shape
    return g.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).sum(axis=(2, 4, 6))


def relu(x):
    return np.maximum(x, 0.0)


def mse(out, target):
    """Mean squared error and its gradient with respect to out."""
    d = np.asarray(out, np.float64) - np.asarray(target, np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1), returning new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """He-normal weights and zero biases; the output convolution starts at
    zero so that the untrained network is the identity."""
    rng = np.random.default_rng(seed)
    P = {}
    for name, ci, co in LAYERS:
        std = np.sqrt(2.0 / (ci * 27))
        P[name + ".w"] = rng.standard_normal((co, ci, 3, 3, 3)) * std if name != "c8" else np.zeros((co, ci, 3, 3, 3))
        P[name + ".b"] = np.zeros(co)
    return P


def forward(P, img, quant=True):
    """Network output for one image (D, H, W) and the values the backward
    pass needs."""
    q = bf16 if quant else (lambda a: np.asarray(a, np.float64))
    W = {n: q(P[n + ".w"]) for n, _, _ in LAYERS}
    B = {n: np.asarray(P[n + ".b"], np.float64) for n, _, _ in LAYERS}
    S = {}
    S["x0"] = q(img)[None]
    S["e1"] = q(relu(conv3d(S["x0"], W["c1"], B["c1"])))
    S["p1"] = q(pool2(S["e1"]))
    S["e2"] = q(relu(conv3d(S["p1"], W["c2"], B["c2"])))
    S["p2"] = q(pool2(S["e2"]))
    S["e3"] = q(relu(conv3d(S["p2"], W["c3"], B["c3"])))
    S["p3"] = q(pool2(S["e3"]))
    S["e4"] = q(relu(conv3d(S["p3"], W["c4"], B["c4"])))
    S["u4"] = up2(S["e4"])
    r5 = relu(conv3d(S["u4"], W["c5"], B["c5"]))
    S["r5"], S["d3"] = q(r5), q(r5 + S["e3"])
    S["u3"] = up2(S["d3"])
    r6 = relu(conv3d(S["u3"], W["c6"], B["c6"]))
    S["r6"], S["d2"] = q(r6), q(r6 + S["e2"])
    S["u2"] = up2(S["d2"])
    r7 = relu(conv3d(S["u2"], W["c7"], B["c7"]))
    S["r7"], S["d1"] = q(r7), q(r7 + S["e1"])
    y = conv3d(S["d1"], W["c8"], B["c8"])[0]
    out = np.asarray(img, np.float64) + y
    return out, S, W


def backward(P, img, target, quant=True):
    """Loss and its gradient with respect to every parameter."""
    q = bf16 if quant else (lambda a: np.asarray(a, np.float64))
    out, S, W = forward(P, img, quant)
    loss, g_out = mse(out, target)
    G = {}

    def layer(name, x_in, gpre):
        dw, db = conv3d_wgrad(x_in, gpre)
        G[name + ".w"], G[name + ".b"] = dw, db
        return conv3d_dgrad(gpre, W[name])

    g8 = q(g_out)[None]
    g_d1 = layer("c8", S["d1"], g8)
    g_u2 = layer("c7", S["u2"], q(g_d1 * (S["r7"] > 0)))
    g_d2 = up2_bwd(g_u2)
    g_u3 = layer("c6", S["u3"], q(g_d2 * (S["r6"] > 0)))
    g_d3 = up2_bwd(g_u3)
    g_u4 = layer("c5", S["u4"], q(g_d3 * (S["r5"] > 0)))
    g_e4 = up2_bwd(g_u4)
    g_p3 = layer("c4", S["p3"], q(g_e4 * (S["e4"] > 0)))
    g_p2 = layer("c3", S["p2"], q((g_d3 + pool2_bwd(g_p3)) * (S["e3"] > 0)))
    g_p1 = layer("c2", S["p1"], q((g_d2 + pool2_bwd(g_p2)) * (S["e2"] > 0)))
    dw, db = conv3d_wgrad(S["x0"], q((g_d1 + pool2_bwd(g_p1)) * (S["e1"] > 0)))
    G["c1.w"], G["c1.b"] = dw, db
    return loss, G, out
