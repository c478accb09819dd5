"""Kernel entries of the Nystrom matrix (TEST INFRASTRUCTURE ONLY: see oracle/__init__.py).

Isotropic kernel (eq. iso_operator2 with constant mu_t, Sec. 2.3.1):
    kappa(r) = exp(-mu_t r) / (|S^{d-1}| r^{d-1}),  |S^1| = 2 pi, |S^2| = 4 pi.
Mode-coupled kernel (eq. ani_2d_operator, Sec. 3.1.1 and 3.3.1): the entry coupling output mode
k at x_i to input mode k' at x_j is
    h^2 kappa(|x_i - x_j|) exp(i (k' - k) theta_ij),  theta_ij = polar angle of x_i - x_j.
Reading of the angle: the paper writes theta as an arccos of the vector (x - y)/|x - y|; the
characteristics of T^{-1} run from y = x - s v to x, so theta is the direction angle of x - y,
i.e. atan2(y_i - y_j, x_i - x_j).  The exponent is (k' - k), acting on input mode k'.

Self cell (Sec. 2.3, the diagonal entry of the Nystrom matrix): the diagonal entry is the exact
integral of the kernel over the square (cube) cell centred at the node.  The paper evaluates it
as an analytic mean plus Gauss-Legendre on the smooth remainder; here it is the exact integral
reduced to one (2D) or two (3D) smooth dimensions and integrated by Gauss-Legendre.
"""
from __future__ import annotations

import numpy as np


def gauss_legendre(npts: int, a: float, b: float):
    x, w = np.polynomial.legendre.leggauss(npts)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def _one_minus_exp_over_mu(mu: float, R):
    """(1 - exp(-mu R)) / mu, with its mu -> 0 limit R."""
    R = np.asarray(R, dtype=np.float64)
    if mu == 0.0:
        return R
    return -np.expm1(-mu * R) / mu


def self_cell_2d(m: int, h: float, mu_t: float, npts: int = 64) -> float:
    """Integral over [-h/2,h/2]^2 of exp(-mu_t r)/(2 pi r) * exp(i m theta).

    In polar coordinates about the centre the radial integral is exact:
        (1/2pi) int_0^{2pi} e^{i m theta} (1 - exp(-mu_t R(theta)))/mu_t dtheta,
    R(theta) = (h/2)/max(|cos|,|sin|).  R has the symmetry of the square, so the integral is
    8 int_0^{pi/4} cos(m theta) (...) dtheta / (2 pi) when 4 | m and 0 otherwise.  The result is
    real."""
    if m % 4 != 0:
        return 0.0
    th, w = gauss_legendre(npts, 0.0, np.pi / 4.0)
    R = 0.5 * h / np.cos(th)
    return float((4.0 / np.pi) * np.sum(w * np.cos(m * th) * _one_minus_exp_over_mu(mu_t, R)))


def self_cell_3d(h: float, mu_t: float, npts: int = 48) -> float:
    """Integral over the cube [-h/2,h/2]^3 of exp(-mu_t r)/(4 pi r^2).

    Polar about the centre: (1/4pi) int_{S^2} (1 - exp(-mu_t R(w)))/mu_t dw.  Split the sphere by
    the six faces; for the face z = a (a = h/2) a direction through the face point (x, y, a) has
    R = rho = sqrt(x^2+y^2+a^2) and solid angle a/rho^3 dx dy.  So the integral is
        (6/(4 pi)) int_{[-a,a]^2} (1 - exp(-mu_t rho))/mu_t * a/rho^3 dx dy,
    and the integrand is smooth (rho >= a).  By symmetry use 4x the quarter [0,a]^2."""
    a = 0.5 * h
    x, w = gauss_legendre(npts, 0.0, a)
    X, Y = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w)
    rho = np.sqrt(X * X + Y * Y + a * a)
    integrand = _one_minus_exp_over_mu(mu_t, rho) * a / rho ** 3
    return float((6.0 / (4.0 * np.pi)) * 4.0 * np.sum(W * integrand))


def kernel_entry_2d(ox, oy, m: int, h: float, mu_t: float):
    """Nystrom entry for the integer cell offset (ox, oy) = (i - j) and mode difference
    m = k' - k: h^2 exp(-mu_t r)/(2 pi r) exp(i m theta), r = h |o|, theta = atan2(oy, ox);
    the exact self-cell integral at o = 0."""
    ox = np.asarray(ox, dtype=np.float64)
    oy = np.asarray(oy, dtype=np.float64)
    r = h * np.hypot(ox, oy)
    zero = r == 0.0
    rs = np.where(zero, 1.0, r)
    theta = np.arctan2(oy, ox)
    val = h * h * np.exp(-mu_t * rs) / (2.0 * np.pi * rs) * np.exp(1j * m * theta)
    val = np.where(zero, self_cell_2d(m, h, mu_t), val)
    return val


def kernel_entry_3d(ox, oy, oz, h: float, mu_t: float):
    """Isotropic 3D entry: h^3 exp(-mu_t r)/(4 pi r^2), exact cell integral at o = 0."""
    ox = np.asarray(ox, dtype=np.float64)
    oy = np.asarray(oy, dtype=np.float64)
    oz = np.asarray(oz, dtype=np.float64)
    r = h * np.sqrt(ox * ox + oy * oy + oz * oz)
    zero = r == 0.0
    rs = np.where(zero, 1.0, r)
    val = h ** 3 * np.exp(-mu_t * rs) / (4.0 * np.pi * rs * rs)
    return np.where(zero, self_cell_3d(h, mu_t), val)


def kernel_table_2d(n: int, m: int, h: float, mu_t: float) -> np.ndarray:
    """K_m[oy + n - 1, ox + n - 1] for all offsets o in (-n, n)^2 (shape (2n-1, 2n-1))."""
    o = np.arange(-(n - 1), n)
    OY, OX = np.meshgrid(o, o, indexing="ij")
    return kernel_entry_2d(OX, OY, m, h, mu_t)


def kernel_table_3d(n: int, h: float, mu_t: float) -> np.ndarray:
    """K[oz + n - 1, oy + n - 1, ox + n - 1] for all offsets in (-n, n)^3."""
    o = np.arange(-(n - 1), n)
    OZ, OY, OX = np.meshgrid(o, o, o, indexing="ij")
    return kernel_entry_3d(OX, OY, OZ, h, mu_t)
