"""Oracle of the learned initial guess for the pressure projection.

TEST INFRASTRUCTURE ONLY: a plain numpy FP64 forward and hand-written
backward of the network, used by the tests to check the GPU kernels.  It
shares no code with the GPU library.

The network (a small 3-level convolutional encoder-decoder, 16/32/64
channels, 3x3x3 kernels with zero "same" padding, ReLU, average pooling and
nearest upsampling, skip connections by channel concatenation) maps four
feature channels built from the projection's right-hand side, the density
and the previous pressure to a correction delta, and the initial guess is
p0 = p_prev + P0 delta with P0 = rho_w g d.

Arrays are channel-first (C, Z, Y, X) here.  With bf16=True every value the
GPU stores in bfloat16 is rounded to bfloat16 (round to nearest even) at the
same point: the features, the weights of the 3x3x3 convolutions, every
activation, and in the backward pass every activation gradient (after its
ReLU mask, after the input-gradient convolution, after the upsampling's
adjoint, after a skip connection's sum).  The 1x1x1 head keeps its weights
and its output in FP32 on the GPU, so they are not rounded.  Products and
sums stay in FP64 here (the GPU sums in FP32).
"""
from __future__ import annotations

import numpy as np

# (name, cin, cout, kernel size)
LAYERS = [("c1", 4, 16, 3), ("c2", 16, 32, 3), ("c3", 32, 64, 3),
          ("c4", 96, 32, 3), ("c5", 48, 16, 3), ("head", 16, 1, 1)]


def param_shapes():
    out = []
    for name, ci, co, k in LAYERS:
        out.append((name + ".w", (co, ci, k, k, k)))
        out.append((name + ".b", (co,)))
    return out


def param_count():
    return sum(int(np.prod(s)) for _, s in param_shapes())


def unflatten(flat):
    """Split a flat parameter vector (layer order, weights (co, ci, kz, ky, kx)
    then bias) into a dict."""
    flat = np.asarray(flat, dtype=np.float64)
    P, o = {}, 0
    for name, shp in param_shapes():
        n = int(np.prod(shp))
        P[name] = flat[o:o + n].reshape(shp)
        o += n
    assert o == flat.size
    return P


def flatten(P):
    return np.concatenate([np.asarray(P[name], dtype=np.float64).ravel() for name, _ in param_shapes()])


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((u >> 16) & 1)
    u = ((u + bias) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- primitives
def conv(x, w, b):
    """Cross-correlation with zero same padding: y[o] = b[o] + sum_c,t w[o,c,t] x[c, . + t]."""
    co, ci, k = w.shape[0], w.shape[1], w.shape[2]
    r = k // 2
    C, Z, Y, X = x.shape
    assert C == ci
    xp = np.zeros((C, Z + 2 * r, Y + 2 * r, X + 2 * r))
    xp[:, r:r + Z, r:r + Y, r:r + X] = x
    y = np.zeros((co, Z, Y, X))
    for dz in range(k):
        for dy in range(k):
            for dx in range(k):
                y += np.einsum("oc,czyx->ozyx", w[:, :, dz, dy, dx],
                               xp[:, dz:dz + Z, dy:dy + Y, dx:dx + X])
    return y + b[:, None, None, None]


def conv_backward(x, w, dy):
    """Gradients of conv: (dx, dw, db)."""
    co, ci, k = w.shape[0], w.shape[1], w.shape[2]
    r = k // 2
    C, Z, Y, X = x.shape
    xp = np.zeros((C, Z + 2 * r, Y + 2 * r, X + 2 * r))
    xp[:, r:r + Z, r:r + Y, r:r + X] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for dz in range(k):
        for dy_ in range(k):
            for dx_ in range(k):
                sl = (slice(None), slice(dz, dz + Z), slice(dy_, dy_ + Y), slice(dx_, dx_ + X))
                dw[:, :, dz, dy_, dx_] = np.einsum("ozyx,czyx->oc", dy, xp[sl])
                dxp[sl] += np.einsum("oc,ozyx->czyx", w[:, :, dz, dy_, dx_], dy)
    return dxp[:, r:r + Z, r:r + Y, r:r + X], dw, dy.sum(axis=(1, 2, 3))


def pool(x):
    """2x2x2 average."""
    C, Z, Y, X = x.shape
    return x.reshape(C, Z // 2, 2, Y // 2, 2, X // 2, 2).mean(axis=(2, 4, 6))


def pool_backward(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up(x):
    """Nearest-neighbour x2 upsampling."""
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up_backward(dy):
    C, Z, Y, X = dy.shape
    return dy.reshape(C, Z // 2, 2, Y // 2, 2, X // 2, 2).sum(axis=(2, 4, 6))


# ---------------------------------------------------------------- network
def forward(P, feat, bf16=False):
    """delta and the cache for backward.  feat: (4, Z, Y, X)."""
    q = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W = {k: (q(v) if k.endswith(".w") and k != "head.w" else np.asarray(v, dtype=np.float64))
         for k, v in P.items()}
    x0 = q(feat)
    a1 = q(np.maximum(conv(x0, W["c1.w"], W["c1.b"]), 0.0))
    p1 = q(pool(a1))
    a2 = q(np.maximum(conv(p1, W["c2.w"], W["c2.b"]), 0.0))
    p2 = q(pool(a2))
    a3 = q(np.maximum(conv(p2, W["c3.w"], W["c3.b"]), 0.0))
    c2 = np.concatenate([a2, up(a3)], axis=0)
    a4 = q(np.maximum(conv(c2, W["c4.w"], W["c4.b"]), 0.0))
    c1 = np.concatenate([a1, up(a4)], axis=0)
    a5 = q(np.maximum(conv(c1, W["c5.w"], W["c5.b"]), 0.0))
    out = conv(a5, W["head.w"], W["head.b"])[0]
    cache = dict(W=W, x0=x0, a1=a1, p1=p1, a2=a2, p2=p2, a3=a3, c2=c2, a4=a4, c1=c1, a5=a5, bf16=bf16)
    return out, cache


def backward(cache, dout):
    """Parameter gradients (dict) for d(loss)/d(out) = dout (Z, Y, X)."""
    W = cache["W"]
    q = bf16_round if cache.get("bf16") else (lambda a: a)
    g = {}
    d5, g["head.w"], g["head.b"] = conv_backward(cache["a5"], W["head.w"], dout[None])
    d5 = q(d5 * (cache["a5"] > 0))
    dc1, g["c5.w"], g["c5.b"] = conv_backward(cache["c1"], W["c5.w"], d5)
    dc1 = q(dc1)
    da1 = dc1[:16].copy()
    d4 = q(up_backward(dc1[16:]) * (cache["a4"] > 0))
    dc2, g["c4.w"], g["c4.b"] = conv_backward(cache["c2"], W["c4.w"], d4)
    dc2 = q(dc2)
    da2 = dc2[:32].copy()
    d3 = q(up_backward(dc2[32:]) * (cache["a3"] > 0))
    dp2, g["c3.w"], g["c3.b"] = conv_backward(cache["p2"], W["c3.w"], d3)
    dp2 = q(dp2)
    da2 += pool_backward(dp2)
    d2 = q(da2 * (cache["a2"] > 0))
    dp1, g["c2.w"], g["c2.b"] = conv_backward(cache["p1"], W["c2.w"], d2)
    dp1 = q(dp1)
    da1 += pool_backward(dp1)
    d1 = q(da1 * (cache["a1"] > 0))
    _, g["c1.w"], g["c1.b"] = conv_backward(cache["x0"], W["c1.w"], d1)
    return g


def loss_and_grad(delta, target):
    """Relative squared error sum (delta - target)^2 / sum target^2 and its
    gradient: with p0 = p_prev + P0 delta and p* = p_prev + P0 target this is
    ||p0 - p*||^2 / ||p_prev - p*||^2, below 1 when the guess beats p_prev."""
    den = float(np.sum(target * target))
    e = delta - target
    return float(np.sum(e * e)) / den, 2.0 * e / den


def energy_loss_and_grad(delta, target, apply_A):
    """Energy-norm ratio ||e||_A^2 / ||target||_A^2 with e = target - delta:
    with p0 = p_prev + P0 delta and p* = p_prev + P0 target this is
    ||p* - p0||_A^2 / ||p* - p_prev||_A^2, the norm CG minimises, so values
    below 1 mean the guess beats p_prev.  Returns (loss, d loss / d delta)
    for a symmetric operator apply_A."""
    e = target - delta
    Ae = apply_A(e)
    den = float(np.sum(target * apply_A(target)))
    return float(np.sum(e * Ae)) / den, -2.0 * Ae / den


def features(b, rho, p_prev, r0, h, rho_w, rho_a, P0):
    """The four input channels: scaled rhs, log-density fraction, scaled
    previous pressure, scaled residual of the previous pressure."""
    s = h * h * rho_w / P0
    return np.stack([b * s, np.log(rho / rho_w) / np.log(rho_a / rho_w), p_prev / P0, r0 * s])


def he_init(seed: int, zero_head: bool = False):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, as a flat
    vector; with zero_head the output layer starts at zero (delta = 0)."""
    rng = np.random.default_rng(seed)
    P = {}
    for name, ci, co, k in LAYERS:
        fan_in = ci * k ** 3
        P[name + ".w"] = rng.standard_normal((co, ci, k, k, k)) * np.sqrt(2.0 / fan_in)
        if zero_head and name == "head":
            P[name + ".w"][:] = 0.0
        P[name + ".b"] = np.zeros(co)
    return flatten(P)


def adam_step(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), returning new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
