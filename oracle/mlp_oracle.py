"""FP64 CPU oracle of the surrogate's per-element MLP, its gradients and Adam.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library never does.

The network is not from the paper (which only motivates learning-oriented
workflows); it is the library's learned coarse step: 4 linear layers
F_in -> 256 -> 256 -> 256 -> 12, SiLU x*sigmoid(x) after the first three,
BF16 weights and BF16 activations between layers (round to nearest even at
each layer input), sums of products in FP64 here (FP32 accumulation on the
GPU), FP32 bias, FP32 output.  Adam (Kingma & Ba 2015): m = b1 m + (1-b1) g,
v = b2 v + (1-b2) g^2, w -= lr * m_hat / (sqrt(v_hat) + eps) with
m_hat = m / (1 - b1^t), v_hat = v / (1 - b2^t).
"""
from __future__ import annotations

import numpy as np

LAYERS = (96, 256, 256, 256, 12)


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), returned as FP64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    # NaN/Inf pass through unchanged
    bad = ~np.isfinite(f)
    if bad.any():
        out[bad] = f[bad]
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(seed, layers=LAYERS):
    """He-style uniform initialisation: W ~ U(-a, a), a = sqrt(6 / fan_in); b = 0.
    Returns a list of (W [K, N], b [N]) in FP64."""
    rng = np.random.default_rng(seed)
    out = []
    for k, n in zip(layers[:-1], layers[1:]):
        a = np.sqrt(6.0 / k)
        out.append((rng.uniform(-a, a, size=(k, n)), np.zeros(n)))
    return out


def forward(params, x, bf16=True):
    """Forward pass.  Returns (y, cache) with cache holding each layer's input
    (as rounded) and pre-activation, for backward()."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    a = r(x)
    cache = []
    L = len(params)
    for li, (W, b) in enumerate(params):
        Wr = r(W)
        bb = np.asarray(b, np.float32).astype(np.float64) if bf16 else np.asarray(b, np.float64)
        z = a @ Wr + bb
        cache.append((a, Wr, z))
        if li < L - 1:
            a = r(silu(z))
        else:
            a = z
    return a, cache


def backward(params, cache, dy, bf16=True):
    """Gradients of sum(dy * y) with respect to every W and b (FP64), through
    the same rounding points as forward() (rounding treated as identity, i.e.
    straight-through, as the GPU does).  Returns (grads, dx)."""
    grads = [None] * len(params)
    g = np.asarray(dy, np.float64)
    L = len(params)
    for li in range(L - 1, -1, -1):
        a, Wr, z = cache[li]
        if li < L - 1:
            g = g * dsilu(z)
        grads[li] = (a.T @ g, g.sum(axis=0))
        g = g @ Wr.T
    return grads, g


def mse_loss(y, t, mask=None):
    """sum(mask * (y - t)^2) / (number of entries), and its gradient; masked
    entries contribute nothing but still count in the mean."""
    d = y - t
    if mask is None:
        mask = np.ones_like(d)
    cnt = d.size
    return float((mask * d * d).sum() / cnt), 2.0 * mask * d / cnt


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]

    def step(self, params, grads, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        out = []
        for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for j, (p, g) in enumerate(((W, gW), (b, gb))):
                m = self.b1 * self.m[i][j] + (1 - self.b1) * g
                v = self.b2 * self.v[i][j] + (1 - self.b2) * g * g
                self.m[i] = tuple(m if jj == j else self.m[i][jj] for jj in range(2))
                self.v[i] = tuple(v if jj == j else self.v[i][jj] for jj in range(2))
                mh = m / (1 - self.b1 ** self.t)
                vh = v / (1 - self.b2 ** self.t)
                new.append(p - lr * mh / (np.sqrt(vh) + self.eps))
            out.append(tuple(new))
        return out


def flatten(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unflatten(vec, layers=LAYERS):
    out, o = [], 0
    for k, n in zip(layers[:-1], layers[1:]):
        W = vec[o:o + k * n].reshape(k, n)
        o += k * n
        b = vec[o:o + n]
        o += n
        out.append((W.copy(), b.copy()))
    return out
