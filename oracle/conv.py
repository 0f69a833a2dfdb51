"""FP64 numpy reference of the surrogate's layers (TEST INFRASTRUCTURE ONLY).

Channels-last arrays x[n, d, h, w, c].  A 3-D convolution with kernel size k
(3: zero padding 1, 1: no padding) and stride s computes

    y[n, o, co] = b[co] + sum_{t, ci} x[n, s*o + t - pad, ci] * w[co, t, ci],

t running over the k^3 taps (t = (kd*k + kh)*k + kw).  The backward functions
are the adjoints of that sum written out directly (scatter of the same
products), not derived from any GPU code.
"""
import numpy as np


def _taps(k):
    return [(kd, kh, kw) for kd in range(k) for kh in range(k) for kw in range(k)]


def _out(n, s):
    return (n + s - 1) // s


def conv3d(x, w, b=None, k=3, s=1, relu=False):
    """x [N,D,H,W,Ci], w [Co, k^3, Ci] -> y [N,Do,Ho,Wo,Co] (FP64)."""
    pad = 1 if k == 3 else 0
    N, D, H, W, _ = x.shape
    Do, Ho, Wo = _out(D, s), _out(H, s), _out(W, s)
    xp = np.pad(x.astype(np.float64), ((0, 0), (pad, pad + s), (pad, pad + s), (pad, pad + s), (0, 0)))
    y = np.zeros((N, Do, Ho, Wo, w.shape[0]))
    for t, (kd, kh, kw) in enumerate(_taps(k)):
        sl = xp[:, kd:kd + s * Do:s, kh:kh + s * Ho:s, kw:kw + s * Wo:s, :]
        y += np.einsum("ndhwc,oc->ndhwo", sl, w[:, t, :].astype(np.float64))
    if b is not None:
        y += b
    if relu:
        y = np.maximum(y, 0.0)
    return y


def conv3d_bwd_data(dy, w, xshape, k=3, s=1):
    """Adjoint of conv3d with respect to x: dx [N,D,H,W,Ci]."""
    pad = 1 if k == 3 else 0
    N, D, H, W, Ci = xshape
    _, Do, Ho, Wo, _ = dy.shape
    dxp = np.zeros((N, D + 2 * pad + s, H + 2 * pad + s, W + 2 * pad + s, Ci))
    for t, (kd, kh, kw) in enumerate(_taps(k)):
        dxp[:, kd:kd + s * Do:s, kh:kh + s * Ho:s, kw:kw + s * Wo:s, :] += np.einsum(
            "ndhwo,oc->ndhwc", dy.astype(np.float64), w[:, t, :].astype(np.float64))
    return dxp[:, pad:pad + D, pad:pad + H, pad:pad + W, :]


def conv3d_bwd_weight(x, dy, k=3, s=1):
    """Adjoint of conv3d with respect to w and b: (dw [Co,k^3,Ci], db [Co])."""
    pad = 1 if k == 3 else 0
    _, Do, Ho, Wo, Co = dy.shape
    xp = np.pad(x.astype(np.float64), ((0, 0), (pad, pad + s), (pad, pad + s), (pad, pad + s), (0, 0)))
    dw = np.zeros((Co, k ** 3, x.shape[-1]))
    for t, (kd, kh, kw) in enumerate(_taps(k)):
        sl = xp[:, kd:kd + s * Do:s, kh:kh + s * Ho:s, kw:kw + s * Wo:s, :]
        dw[:, t, :] = np.einsum("ndhwc,ndhwo->oc", sl, dy.astype(np.float64))
    return dw, dy.astype(np.float64).sum(axis=(0, 1, 2, 3))


def upsample2(x):
    """Nearest-neighbour 2x upsampling of [N,D,H,W,C]."""
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def upsample2_bwd(dy):
    """Adjoint of upsample2: the sum over each 2x2x2 group."""
    N, D, H, W, C = dy.shape
    return dy.reshape(N, D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4, 6))


def bf16_round(a):
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
