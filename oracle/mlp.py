"""FP64 reference of the learned LRX surrogate (features, network, gradient, Adam, selection).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The surrogate is not part of the
paper.  It predicts log1p of the LRX score (eq. 1) of a pixel from features of its
annulus (outer minus inner window, Sec. 2.2), so that the exact detector only runs near
the eq. (12) threshold and on a seeded audit sample.

Everything here follows the plain definitions in double precision:
  features   z_i = (x_i - mu_i) / sqrt(v_i + 1e-12), log(v_i + 1e-12), mu_i for every band
             i, where mu and v are the annulus mean and 1/n variance (from the oracle's
             window statistics),
  network    h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), y = h2 . w3 + b3 (hidden 128),
  loss       (1/B) sum over the batch of (y - t)^2, rows with NaN targets contributing 0,
  gradient   back-propagation written out layer by layer,
  Adam       Kingma and Ba (ICLR 2015), Algorithm 1 with beta1 0.9, beta2 0.999, eps 1e-8,
  SplitMix64 Steele, Lea and Flood (OOPSLA 2014): output i of the stream seeded with s is
             the finaliser applied to s + (i + 1) * 0x9E3779B97F4A7C15.
Parameter vector layout: W1 [Dp][128] | b1 | W2 [128][128] | b2 | w3 | b3 | 3 padding.
"""
from __future__ import annotations

import numpy as np

HID = 128
GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def dims(Lp: int):
    """(D, Dp, nparams) for L' reduced bands."""
    D = 3 * int(Lp)
    Dp = (D + 31) // 32 * 32
    return D, Dp, Dp * HID + HID + HID * HID + HID + HID + 4


def unpack(params, Dp: int):
    p = np.asarray(params, dtype=np.float64)
    o = 0
    W1 = p[o:o + Dp * HID].reshape(Dp, HID); o += Dp * HID
    b1 = p[o:o + HID]; o += HID
    W2 = p[o:o + HID * HID].reshape(HID, HID); o += HID * HID
    b2 = p[o:o + HID]; o += HID
    w3 = p[o:o + HID]; o += HID
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3, 0.0, 0.0, 0.0]])


def forward(X, params, Dp: int):
    """Network output for the rows of X (n x Dp)."""
    W1, b1, W2, b2, w3, b3 = unpack(params, Dp)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.maximum(X @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h2 @ w3 + b3


def loss_and_grad(X, tgt, params, Dp: int):
    """(loss, gradient vector) of the mean squared error over the rows of X.  The ReLU
    decisions a > 0 are taken on the FP64 pre-activations."""
    W1, b1, W2, b2, w3, b3 = unpack(params, Dp)
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(tgt, dtype=np.float64)
    B = X.shape[0]
    a1 = X @ W1 + b1
    m1 = a1 > 0
    h1 = np.where(m1, a1, 0.0)
    a2 = h1 @ W2 + b2
    m2 = a2 > 0
    h2 = np.where(m2, a2, 0.0)
    y = h2 @ w3 + b3
    ok = ~np.isnan(t)
    r = np.where(ok, y - np.where(ok, t, 0.0), 0.0)
    loss = float(np.sum(r * r) / B)
    dy = 2.0 * r / B                                 # dL/dy
    g_w3 = h2.T @ dy
    g_b3 = dy.sum()
    d2 = np.outer(dy, w3) * m2                       # dL/da2
    g_W2 = h1.T @ d2
    g_b2 = d2.sum(0)
    d1 = (d2 @ W2.T) * m1                            # dL/da1
    g_W1 = X.T @ d1
    g_b1 = d1.sum(0)
    return loss, pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3)


def adam_step(params, grad, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update; returns (params, m, v) as new arrays."""
    g = np.asarray(grad, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return np.asarray(params, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def features(x, inner: int, outer: int, idx=None):
    """Feature rows [z | log-variance | mean] (n x 3 L') of the reduced cube x at idx."""
    from . import window_stats
    x = np.asarray(x, dtype=np.float64)
    H, W, Lp = x.shape
    idx = np.arange(H * W) if idx is None else np.asarray(idx).ravel()
    out = np.empty((idx.size, 3 * Lp))
    for j, p in enumerate(idx):
        py, px = divmod(int(p), W)
        _, mu, C, _, _, _ = window_stats(x, inner, outer, py, px)
        ve = np.diag(C) + 1e-12
        out[j] = np.concatenate([(x[py, px] - mu) / np.sqrt(ve), np.log(ve), mu])
    return out


def splitmix64(seed: int, i):
    """SplitMix64 outputs i (array of non-negative integers) of the stream seeded with seed."""
    i = np.asarray(i, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _M64) + (i + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def splitmix64_sequential(seed: int, n: int):
    """The same stream generated the textbook way, one state increment per call."""
    out, s = [], seed & _M64
    for _ in range(n):
        s = (s + GAMMA) & _M64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        out.append(z ^ (z >> 31))
    return np.array(out, dtype=np.uint64)


def select(yhat, tau: float, band: float, seed: int, audit_frac: float):
    """Selection flags: 1 for |yhat - log1p(tau)| <= band (NaN included), 2 for the audit
    (top 32 bits of SplitMix64 output i below audit_frac * 2^32)."""
    y = np.asarray(yhat, dtype=np.float64)
    in_band = ~(np.abs(y - np.log1p(tau)) > band)
    cut = min(int(np.ldexp(audit_frac, 32)), 0xFFFFFFFF)
    top = splitmix64(seed, np.arange(y.size)) >> np.uint64(32)
    audit = top < np.uint64(cut)
    return in_band.astype(np.uint8) | (audit.astype(np.uint8) << 1)
