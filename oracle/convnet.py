"""FP64 reference for the learned right preconditioner's network
(TEST INFRASTRUCTURE ONLY: see oracle/__init__.py).

The paper has no learned component; this is the plain definition of the network the GPU trains
and runs: a stack of 3x3 convolutions with zero "same" padding, a bias per output channel and a
ReLU after every layer but the last.  Activations are [B, C, H, W]; weights [Cout, Cin, 3, 3].

  conv:  y[b,o,i,j] = bias[o] + sum_{c,p,q} W[o,c,p,q] x[b,c,i+p-1,j+q-1]   (x = 0 outside)

Backward is the chain rule written out: the data gradient is the correlation of the output
gradient with the spatially flipped, channel-transposed weights; the weight gradient correlates
the output gradient with the input; the bias gradient sums the output gradient.
"""
from __future__ import annotations

import numpy as np


def conv3x3(x: np.ndarray, W: np.ndarray, bias: np.ndarray) -> np.ndarray:
    B, C, H, Wd = x.shape
    O = W.shape[0]
    xp = np.zeros((B, C, H + 2, Wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((B, O, H, Wd)) + bias[None, :, None, None]
    for p in range(3):
        for q in range(3):
            patch = xp[:, :, p:p + H, q:q + Wd]                  # [B, C, H, W]
            y += np.einsum("oc,bchw->bohw", W[:, :, p, q], patch)
    return y


def conv3x3_backward(x: np.ndarray, W: np.ndarray, gy: np.ndarray):
    """Returns (gx, gW, gbias) for y = conv3x3(x, W, bias)."""
    B, C, H, Wd = x.shape
    xp = np.zeros((B, C, H + 2, Wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    gxp = np.zeros_like(xp)
    gW = np.zeros_like(W)
    for p in range(3):
        for q in range(3):
            patch = xp[:, :, p:p + H, q:q + Wd]
            gW[:, :, p, q] = np.einsum("bohw,bchw->oc", gy, patch)
            gxp[:, :, p:p + H, q:q + Wd] += np.einsum("oc,bohw->bchw", W[:, :, p, q], gy)
    gb = gy.sum(axis=(0, 2, 3))
    return gxp[:, :, 1:-1, 1:-1], gW, gb


def net_forward(x: np.ndarray, params):
    """params = [(W0, b0), ..., (W_{L-1}, b_{L-1})]; ReLU after every layer except the last.
    Returns (output, cache) with cache = the input of every layer and its pre-activation."""
    cache = []
    a = x
    for li, (W, b) in enumerate(params):
        z = conv3x3(a, W, b)
        cache.append((a, z))
        a = np.maximum(z, 0.0) if li < len(params) - 1 else z
    return a, cache


def net_backward(gout: np.ndarray, params, cache):
    """Gradients [(gW, gb), ...] and the input gradient, given dLoss/dOutput."""
    grads = [None] * len(params)
    g = gout
    for li in range(len(params) - 1, -1, -1):
        a, z = cache[li]
        if li < len(params) - 1:
            g = g * (z > 0.0)
        gx, gW, gb = conv3x3_backward(a, params[li][0], g)
        grads[li] = (gW, gb)
        g = gx
    return grads, g


def pc_loss(r: np.ndarray, e: np.ndarray, params):
    """Relative squared error of the corrected residual over the batch:
    sum_b ||r_b + N(r_b) - e_b||^2 / ||e_b||^2 / B, and its gradient w.r.t. the parameters."""
    out, cache = net_forward(r, params)
    diff = r + out - e
    B = r.shape[0]
    en = np.array([np.sum(e[b] ** 2) for b in range(B)])
    loss = float(np.sum([np.sum(diff[b] ** 2) / en[b] for b in range(B)]) / B)
    gout = 2.0 * diff / en[:, None, None, None] / B
    grads, _ = net_backward(gout, params, cache)
    return loss, grads


def coarse_loss(x: np.ndarray, t: np.ndarray, w: np.ndarray, params):
    """Mean over the batch of w_b ||N(x_b) - t_b||^2 and its parameter gradients.

    This is the training objective of the coarse-grid correction z = v + s P N(R v / s) (R: F x F
    block average, P: piecewise-constant prolongation, s: RMS of v): with x = R r / s and
    t = R(e - r) / s, ||r + s P N(x) - e||^2 = ||(I - P R)(r - e)||^2 + F^2 s^2 ||N(x) - t||^2
    because P R is the orthogonal projector onto block-constant fields, so the fine-grid relative
    loss ||r + s P N(x) - e||^2 / ||e||^2 differs from w ||N(x) - t||^2 (w = F^2 s^2 / ||e||^2)
    only by a term independent of the network."""
    out, cache = net_forward(x, params)
    diff = out - t
    B = x.shape[0]
    per = np.array([np.sum(diff[b] ** 2) for b in range(B)])
    loss = float(np.sum(w * per) / B)
    gout = 2.0 * diff * (w / B)[:, None, None, None]
    grads, _ = net_backward(gout, params, cache)
    return loss, grads


def restrict(v: np.ndarray, F: int) -> np.ndarray:
    """F x F block average of [..., H, W] (H, W multiples of F)."""
    *lead, H, W = v.shape
    return v.reshape(*lead, H // F, F, W // F, F).mean(axis=(-3, -1))


def prolong(vc: np.ndarray, F: int) -> np.ndarray:
    """Piecewise-constant prolongation: each coarse value fills its F x F block."""
    return np.repeat(np.repeat(vc, F, axis=-2), F, axis=-1)


def prolong_bilinear(vc: np.ndarray, F: int) -> np.ndarray:
    """Bilinear interpolation from coarse cell centres to fine cell centres (cell-centred grids,
    coarse cell I covers fine cells I*F .. I*F+F-1).  A fine centre at coarse coordinate
    xi = (i + 1/2)/F - 1/2 takes (1 - a) v[I0] + a v[I0+1], I0 = floor(xi), a = xi - I0, with the
    indices clamped to the coarse grid (constant extension beyond the outer coarse centres)."""
    *lead, Hc, Wc = vc.shape
    def weights(nc):
        n = nc * F
        xi = (np.arange(n) + 0.5) / F - 0.5
        i0 = np.floor(xi).astype(int)
        a = xi - i0
        lo = np.clip(i0, 0, nc - 1)
        hi = np.clip(i0 + 1, 0, nc - 1)
        W = np.zeros((n, nc))
        W[np.arange(n), lo] += 1 - a
        W[np.arange(n), hi] += a
        return W
    Wy, Wx = weights(Hc), weights(Wc)
    return np.einsum("yI,...IJ,xJ->...yx", Wy, vc, Wx)


def precondition(v: np.ndarray, params, F: int) -> np.ndarray:
    """The learned right preconditioner on one channel vector v [C, ny, nx]:
    z = v + s P N(R v / s), R = F x F block average, P = bilinear prolongation,
    s = root-mean-square of v."""
    s = np.sqrt(np.mean(v ** 2))
    if s == 0.0:
        return v.copy()
    y, _ = net_forward(restrict(v, F)[None] / s, params)
    return v + s * prolong_bilinear(y[0], F)


def adam_step(param, grad, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), bias-corrected; returns new (param, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return param - lr * mh / (np.sqrt(vh) + eps), m, v
