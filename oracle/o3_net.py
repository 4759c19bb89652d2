"""Oracle tier O3: FP64 reference of the learned coarse-to-fine corrector.

TEST INFRASTRUCTURE ONLY -- see the package docstring.  Plain numpy, FP64,
channels-last tensors ``[D, H, W, C]`` (one sample).

Operations (each the plain definition):

* 3x3x3 convolution with zero padding, stride 1 (cross-correlation, as in
  every deep-learning framework): y[v, co] = b[co] + sum_{tap, ci}
  w[co, tap, ci] x[v + off(tap), ci], tap = 9 (dz + 1) + 3 (dy + 1) + (dx + 1);
* its gradients with respect to the input and the weights;
* 2x2x2 average pooling and nearest 2x upsampling (and their adjoints);
* the fixed coarse-to-fine trilinear upsampling of the coarse velocity: fine
  node 2i coincides with coarse node i, odd fine nodes take the mean of their
  two (four, eight) coarse neighbours, the last coarse node is repeated past
  the upper boundary;
* the masked mean squared error and the Adam update.

The network composes them (see :data:`LAYERS`): a two-level U-net on the
coarse grid, a nearest 2x upsampling to the fine grid, two fine convolutions
and a residual added to the trilinear upsampling of the coarse velocity.
"""

from __future__ import annotations

import numpy as np

OFFS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shift(x, dz, dy, dx):
    """x[v + (dz, dy, dx)] with zeros outside (x: [D, H, W, C])."""
    D, H, W = x.shape[:3]
    out = np.zeros_like(x)
    zs, zd = (slice(dz, D), slice(0, D - dz)) if dz >= 0 else (slice(0, D + dz), slice(-dz, D))
    ys, yd = (slice(dy, H), slice(0, H - dy)) if dy >= 0 else (slice(0, H + dy), slice(-dy, H))
    xs, xd = (slice(dx, W), slice(0, W - dx)) if dx >= 0 else (slice(0, W + dx), slice(-dx, W))
    out[zd, yd, xd] = x[zs, ys, xs]
    return out


def conv3d(x, w, b):
    """x [D,H,W,Ci], w [Co,27,Ci], b [Co] -> [D,H,W,Co]."""
    y = np.zeros(x.shape[:3] + (w.shape[0],))
    for t, (dz, dy, dx) in enumerate(OFFS):
        y += _shift(x, dz, dy, dx) @ w[:, t, :].T
    return y + b


def conv3d_backward(x, w, dy):
    """Gradients (dx, dw, db) of conv3d for output gradient dy."""
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for t, (dz, dyo, dxo) in enumerate(OFFS):
        xs = _shift(x, dz, dyo, dxo)
        dw[:, t, :] = np.einsum("zyxo,zyxi->oi", dy, xs)
        dx += _shift(dy @ w[:, t, :], -dz, -dyo, -dxo)
    db = dy.sum(axis=(0, 1, 2))
    return dx, dw, db


def avgpool2(x):
    D, H, W, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(1, 3, 5))


def avgpool2_backward(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, 0), 2, 1), 2, 2) / 8.0


def upsample2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def upsample2_backward(dy):
    D, H, W, C = dy.shape
    return dy.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


def trilinear2(x):
    """Coarse [d,h,w,C] -> fine [2d,2h,2w,C] (fine node 2i on coarse node i)."""
    out = x
    for ax in range(3):
        n = out.shape[ax]
        nxt = np.concatenate([np.take(out, np.arange(1, n), axis=ax),
                              np.take(out, [n - 1], axis=ax)], axis=ax)
        mid = 0.5 * (out + nxt)
        stacked = np.stack([out, mid], axis=ax + 1)
        shape = list(out.shape)
        shape[ax] = 2 * n
        out = stacked.reshape(shape)
    return out


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even) and return FP64: the value
    is first rounded to FP32, then the low 16 bits of the FP32 pattern are
    rounded away (finite inputs)."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def masked_mse(pred, target, mask):
    """Mean over masked voxels and the 3 components; returns (loss, dloss/dpred)."""
    m = mask.astype(np.float64)[..., None]
    n = max(1.0, float(m.sum()) * pred.shape[-1])
    d = (pred - target) * m
    return float((d * d).sum() / n), 2.0 * d / n


def adam(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) on FP64 arrays; returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ---- the network ------------------------------------------------------------------
# (name, c_in, c_out, relu, level) ; level c = coarse, h = half, f = fine
LAYERS = [
    ("e1a", 4, 16, True, "c"), ("e1b", 16, 16, True, "c"),
    ("e2a", 16, 32, True, "h"), ("e2b", 32, 32, True, "h"), ("e2c", 32, 32, True, "h"),
    ("u1", 32, 16, True, "c"),
    ("d1a", 32, 16, True, "c"), ("d1b", 16, 16, True, "c"),
    ("f1", 16, 16, True, "f"), ("f2", 16, 16, True, "f"),
    ("head", 16, 3, False, "f"),
]


def init_params(seed=0):
    """He-style random initial weights [Co, 27, Ci] and zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co, relu, _ in LAYERS:
        scale = np.sqrt(2.0 / (27 * ci)) * (1.0 if relu else 0.1)
        p[name] = (rng.normal(0.0, scale, (co, 27, ci)), np.zeros(co))
    return p


def _ident(a):
    return a


def forward(params, x, q=None):
    """x: coarse input [d,h,w,4] = (u_c (3), mask_c) -> (fine velocity, cache).

    q (optional) is a rounding applied where a reduced-precision implementation
    stores values: the weights, the network input, every stored activation
    (convolution outputs but the head's, the pooled tensor).  q = None is the
    exact network."""
    q = q or _ident
    cache = {"q": q}

    def conv(name, inp, relu):
        w, b = params[name]
        y = conv3d(inp, q(w), b)
        out = q(np.maximum(y, 0.0)) if relu else y
        cache[name] = (inp, out)
        return out

    e1 = conv("e1b", conv("e1a", q(x), True), True)
    p = q(avgpool2(e1))
    e2 = conv("e2c", conv("e2b", conv("e2a", p, True), True), True)
    u1 = conv("u1", upsample2(e2), True)
    cat = np.concatenate([e1, u1], axis=-1)
    d1 = conv("d1b", conv("d1a", cat, True), True)
    f = conv("f2", conv("f1", upsample2(d1), True), True)
    r = conv("head", f, False)
    return trilinear2(x[..., :3]) + r, cache


def backward(params, cache, dout):
    """Parameter gradients {name: (dw, db)} for output gradient dout.  With the
    rounding q of the forward pass, each layer's output gradient (after the
    ReLU mask) is rounded before it meets the weights and the inputs; the bias
    gradient sums the unrounded one."""
    grads = {}
    q = cache["q"]

    def conv_b(name, dy, relu):
        inp, out = cache[name]
        if relu:
            dy = dy * (out > 0)
        dx, dw, _ = conv3d_backward(inp, q(params[name][0]), q(dy))
        grads[name] = (dw, dy.sum(axis=(0, 1, 2)))
        return dx

    d = conv_b("head", dout, False)
    d = conv_b("f1", conv_b("f2", d, True), True)
    d = upsample2_backward(d)
    dcat = conv_b("d1a", conv_b("d1b", d, True), True)
    de1 = dcat[..., :16]
    d = conv_b("u1", dcat[..., 16:], True)
    d = upsample2_backward(d)
    d = conv_b("e2a", conv_b("e2b", conv_b("e2c", d, True), True), True)
    de1 = de1 + avgpool2_backward(d)
    conv_b("e1a", conv_b("e1b", de1, True), True)
    return grads
