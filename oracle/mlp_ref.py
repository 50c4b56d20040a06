"""FP64 reference of the surrogate network (TEST INFRASTRUCTURE ONLY).

Same architecture and parameter layout as the library's network: `depth` linear layers
nin -> width -> ... -> width -> 2, SiLU between layers; parameters one flat array, per layer
W [out][in] then b [out].  Loss: mean over samples of 0.5 (y - mu)^2 exp(-2 s) + s with
(mu, s) the two outputs.  Backward pass by the chain rule, written out layer by layer.
"""
from __future__ import annotations

import numpy as np


def layout(nin, width, depth):
    dims, off = [], 0
    for l in range(depth):
        i = nin if l == 0 else width
        o = 2 if l + 1 == depth else width
        dims.append((i, o, off, off + i * o))
        off += i * o + o
    return dims, off


def _unpack(p, dims):
    out = []
    for (i, o, wo, bo) in dims:
        out.append((p[wo:wo + i * o].reshape(o, i), p[bo:bo + o]))
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s + z * s * (1.0 - s)


def forward(p, X, nin, width, depth):
    dims, _ = layout(nin, width, depth)
    h = np.asarray(X, dtype=np.float64)
    for l, (W, b) in enumerate(_unpack(np.asarray(p, dtype=np.float64), dims)):
        z = h @ W.T + b
        h = silu(z) if l + 1 < depth else z
    return h


def loss(p, X, y, nin, width, depth):
    out = forward(p, X, nin, width, depth)
    mu, s = out[:, 0], out[:, 1]
    r = np.asarray(y, dtype=np.float64) - mu
    return float(np.mean(0.5 * r * r * np.exp(-2.0 * s) + s))


def loss_grad(p, X, y, nin, width, depth):
    dims, n = layout(nin, width, depth)
    p = np.asarray(p, dtype=np.float64)
    params = _unpack(p, dims)
    hs, zs = [np.asarray(X, dtype=np.float64)], []
    for l, (W, b) in enumerate(params):
        z = hs[-1] @ W.T + b
        zs.append(z)
        hs.append(silu(z) if l + 1 < depth else z)
    out = hs[-1]
    M = out.shape[0]
    mu, s = out[:, 0], out[:, 1]
    r = np.asarray(y, dtype=np.float64) - mu
    e = np.exp(-2.0 * s)
    L = float(np.mean(0.5 * r * r * e + s))
    d = np.stack([-r * e, 1.0 - r * r * e], axis=1) / M
    g = np.zeros(n)
    for l in range(depth - 1, -1, -1):
        i, o, wo, bo = dims[l]
        if l + 1 < depth:
            d = d * silu_grad(zs[l])
        g[wo:wo + i * o] = (d.T @ hs[l]).reshape(-1)
        g[bo:bo + o] = d.sum(axis=0)
        d = d @ params[l][0]
    return L, g
