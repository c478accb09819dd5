"""Pins of the FP64 network oracle: convolution vs scipy's correlate2d, gradients vs central
finite differences, Adam vs its first-step closed form."""
import numpy as np
from scipy import signal

from oracle import convnet as cn


def test_conv3x3_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    B, C, O, H, W = 2, 3, 4, 7, 9
    x = rng.standard_normal((B, C, H, W))
    Wt = rng.standard_normal((O, C, 3, 3))
    b = rng.standard_normal(O)
    y = cn.conv3x3(x, Wt, b)
    for bb in range(B):
        for o in range(O):
            ref = b[o] + sum(signal.correlate2d(x[bb, c], Wt[o, c], mode="same", boundary="fill")
                             for c in range(C))
            assert np.abs(y[bb, o] - ref).max() < 1e-13


def test_net_gradients_finite_differences():
    rng = np.random.default_rng(1)
    B, C, Hd, H, W = 2, 2, 3, 6, 5
    params = [(0.4 * rng.standard_normal((Hd, C, 3, 3)), 0.1 * rng.standard_normal(Hd)),
              (0.4 * rng.standard_normal((Hd, Hd, 3, 3)), 0.1 * rng.standard_normal(Hd)),
              (0.4 * rng.standard_normal((C, Hd, 3, 3)), 0.1 * rng.standard_normal(C))]
    r = rng.standard_normal((B, C, H, W))
    e = rng.standard_normal((B, C, H, W))
    loss, grads = cn.pc_loss(r, e, params)
    eps = 1e-6
    for li in range(3):
        for which in (0, 1):
            arr = params[li][which]
            flat = arr.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + eps
                lp, _ = cn.pc_loss(r, e, params)
                flat[idx] = old - eps
                lm, _ = cn.pc_loss(r, e, params)
                flat[idx] = old
                fd = (lp - lm) / (2 * eps)
                an = grads[li][which].reshape(-1)[idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd))
    # input gradient
    out, cache = cn.net_forward(r, params)
    g = rng.standard_normal(out.shape)
    _, gx = cn.net_backward(g, params, cache)
    for _ in range(5):
        idx = tuple(rng.integers(0, s) for s in r.shape)
        rp = r.copy(); rp[idx] += eps
        rm = r.copy(); rm[idx] -= eps
        fd = (np.sum(g * cn.net_forward(rp, params)[0]) - np.sum(g * cn.net_forward(rm, params)[0])) / (2 * eps)
        assert abs(fd - gx[idx]) <= 1e-6 * max(1.0, abs(fd))


def test_adam_first_step_is_signed_lr():
    """After one bias-corrected step, Adam moves each weight by lr * g/(|g| + eps)."""
    rng = np.random.default_rng(2)
    p = rng.standard_normal(10)
    g = rng.standard_normal(10)
    p1, m, v = cn.adam_step(p, g, np.zeros(10), np.zeros(10), 1, lr=1e-2)
    assert np.abs((p - p1) - 1e-2 * g / (np.abs(g) + 1e-8)).max() < 1e-12


def test_coarse_loss_gradient_and_decomposition():
    """Finite-difference check of the coarse loss, and the identity
    ||r + s P y - e||^2 = ||(I - P R)(r - e)||^2 + F^2 s^2 ||y - R(e - r)/s||^2."""
    rng = np.random.default_rng(3)
    C, Hd, F, B = 3, 4, 4, 2
    params = [(0.3 * rng.standard_normal((Hd, C, 3, 3)), 0.1 * rng.standard_normal(Hd)),
              (0.3 * rng.standard_normal((C, Hd, 3, 3)), 0.1 * rng.standard_normal(C))]
    x = rng.standard_normal((B, C, 5, 6))
    t = rng.standard_normal((B, C, 5, 6))
    w = rng.random(B) + 0.5
    loss, grads = cn.coarse_loss(x, t, w, params)
    eps = 1e-6
    for li in range(2):
        arr = params[li][0].reshape(-1)
        for idx in rng.choice(arr.size, 5, replace=False):
            old = arr[idx]
            arr[idx] = old + eps
            lp, _ = cn.coarse_loss(x, t, w, params)
            arr[idx] = old - eps
            lm, _ = cn.coarse_loss(x, t, w, params)
            arr[idx] = old
            assert abs((lp - lm) / (2 * eps) - grads[li][0].reshape(-1)[idx]) <= 1e-6 * max(1, abs(lp))
    r = rng.standard_normal((C, 8, 12))
    e = rng.standard_normal((C, 8, 12))
    y = rng.standard_normal((C, 2, 3))
    s = 0.7
    lhs = np.sum((r + s * cn.prolong(y, F) - e) ** 2)
    rhs = np.sum(((r - e) - cn.prolong(cn.restrict(r - e, F), F)) ** 2) + \
        F * F * s * s * np.sum((y - cn.restrict(e - r, F) / s) ** 2)
    assert abs(lhs - rhs) <= 1e-12 * lhs


def test_bilinear_prolongation_reproduces_linear_fields():
    """Bilinear interpolation is exact for fields linear in the coordinates (away from the outer
    half coarse cell, where the clamp extends the outer values), and keeps constants everywhere."""
    F, Hc, Wc = 4, 5, 6
    yc = (np.arange(Hc) + 0.5) * F
    xc = (np.arange(Wc) + 0.5) * F
    vc = 2.0 + 0.3 * yc[:, None] - 0.7 * xc[None, :]
    v = cn.prolong_bilinear(vc, F)
    yf = np.arange(Hc * F) + 0.5
    xf = np.arange(Wc * F) + 0.5
    exact = 2.0 + 0.3 * yf[:, None] - 0.7 * xf[None, :]
    inner = slice(F // 2, -(F // 2))
    assert np.abs(v[inner, inner] - exact[inner, inner]).max() < 1e-12
    c = cn.prolong_bilinear(np.full((2, Hc, Wc), 3.25), F)
    assert np.abs(c - 3.25).max() < 1e-15
    # block average of the prolongation of a linear field returns it (interior blocks)
    assert np.abs(cn.restrict(v, F)[1:-1, 1:-1] - vc[1:-1, 1:-1]).max() < 1e-12


def test_precondition_is_homogeneous_without_biases():
    rng = np.random.default_rng(4)
    C, Hd, F = 3, 8, 4
    params = [(0.3 * rng.standard_normal((Hd, C, 3, 3)), np.zeros(Hd)),
              (0.3 * rng.standard_normal((C, Hd, 3, 3)), np.zeros(C))]
    v = rng.standard_normal((C, 16, 12))
    z = cn.precondition(v, params, F)
    assert np.abs(cn.precondition(3.7 * v, params, F) - 3.7 * z).max() < 1e-12 * np.abs(z).max()
