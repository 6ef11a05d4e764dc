"""Oracle of the closure MLP (36 -> 64 -> 64 -> 3, GELU), FP64 with the GPU's BF16 rounding points.

Test infrastructure only (see the package docstring).  Not in the paper.

Parameters are one flat FP32 vector in the order
    W1 (64 x 36, row-major out x in), b1 (64), W2 (64 x 64), b2 (64), W3 (3 x 64), b3 (3)
(6723 values).  Forward, with rnd = round to BF16 (nearest-even, through FP32):
    x' = rnd(x),  z1 = x' rnd(W1)^T + b1,  h1 = gelu(z1)
    z2 = rnd(h1) rnd(W2)^T + b2,           h2 = gelu(z2)
    y  = rnd(h2) rnd(W3)^T + b3
GELU is the exact erf form 0.5 z (1 + erf(z / sqrt 2)).  Loss: mean of (y - t)^2
over the batch and the 3 outputs.  Backward, same rounding points:
    dy  = 2 (y - t) / (3 B);   dW3 = rnd(dy)^T rnd(h2);  db3 = sum dy
    dz2 = (rnd(dy) rnd(W3)) * gelu'(z2);  dW2 = rnd(dz2)^T rnd(h1);  db2 = sum dz2
    dz1 = (rnd(dz2) rnd(W2)) * gelu'(z1); dW1 = rnd(dz1)^T x';       db1 = sum dz1
``rounding=False`` gives the exact FP64 network (for finite-difference checks).
Adam: the standard bias-corrected update with FP32 master weights.
"""
from __future__ import annotations

import math

import numpy as np

NIN, NH, NOUT = 36, 64, 3
SHAPES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NOUT, NH)), ("b3", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def bf16(a):
    """Round to the nearest BF16 value (ties to even), via the FP32 representation."""
    f = np.asarray(a, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


_erf = np.vectorize(math.erf)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(p, x, rounding=True):
    """x (B, 36) normalised features -> y (B, 3) and the cache for backward."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    P = unpack(p)
    xr = r(x)
    z1 = xr @ r(P["W1"]).T + P["b1"]
    h1 = gelu(z1)
    h1r = r(h1)
    z2 = h1r @ r(P["W2"]).T + P["b2"]
    h2 = gelu(z2)
    h2r = r(h2)
    y = h2r @ r(P["W3"]).T + P["b3"]
    return y, dict(xr=xr, z1=z1, h1r=h1r, z2=z2, h2r=h2r, P=P, r=r)


def loss(y, t):
    return float(np.mean((y - t) ** 2))


def backward(p, x, t, rounding=True):
    """(loss, flat gradient) of the mean squared error."""
    y, c = forward(p, x, rounding)
    r, P = c["r"], c["P"]
    B = x.shape[0]
    dy = 2.0 * (y - t) / (NOUT * B)
    dyr = r(dy)
    g = {}
    g["W3"] = dyr.T @ c["h2r"]
    g["b3"] = dy.sum(axis=0)
    dz2 = (dyr @ r(P["W3"])) * gelu_grad(c["z2"])
    dz2r = r(dz2)
    g["W2"] = dz2r.T @ c["h1r"]
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2r @ r(P["W2"])) * gelu_grad(c["z1"])
    dz1r = r(dz1)
    g["W1"] = dz1r.T @ c["xr"]
    g["b1"] = dz1.sum(axis=0)
    return loss(y, t), pack(g)


def adam(p, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update (step counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1**step)
    vh = v / (1 - b2**step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed):
    """Xavier-uniform weights, zero biases (the random numbers the training draws, passed to the GPU)."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            lim = math.sqrt(6.0 / (shape[0] + shape[1]))
            d[name] = rng.uniform(-lim, lim, size=shape)
        else:
            d[name] = np.zeros(shape)
    return pack(d).astype(np.float32)
