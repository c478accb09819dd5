"""Real spherical harmonics of the 3D anisotropic modes (TEST INFRASTRUCTURE ONLY: see
oracle/__init__.py).

The angular modes of the 3D flux are coefficients in a real orthonormal spherical-harmonic basis
(Sec. 3.1.2 expands in spherical harmonics; its printed formulas are garbled, so the basis is fixed
here).  For l = 0..L and m = -l..l, with the mode index a = l^2 + l + m,

    Y~_{l,0}  = sqrt(4 pi) Y_l^0,
    Y~_{l,m}  = sqrt(2) sqrt(4 pi) (-1)^m Re Y_l^m      (m > 0),
    Y~_{l,-m} = sqrt(2) sqrt(4 pi) (-1)^m Im Y_l^m      (m > 0),

where Y_l^m are the complex orthonormal harmonics with the Condon-Shortley phase (scipy's
sph_harm_y), so the phase cancels.  The basis is orthonormal for the mean over the sphere,
mean_S2 Y~_a Y~_b = delta_ab, Y~_{0,0} = 1, and on the unit sphere
Y~_{1,-1} = sqrt(3) y, Y~_{1,0} = sqrt(3) z, Y~_{1,1} = sqrt(3) x.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def nmodes(L: int) -> int:
    return (L + 1) ** 2


def degree(a: int) -> int:
    """l of the mode index a = l^2 + l + m."""
    return int(np.floor(np.sqrt(a) + 1e-12))


def lm(a: int):
    l = degree(a)
    return l, a - l * l - l


def real_sh(L: int, w) -> np.ndarray:
    """Y~_a(w) for all a < (L+1)^2 at unit vectors w (shape (..., 3)); returns (..., (L+1)^2)."""
    w = np.asarray(w, dtype=np.float64)
    x, y, z = w[..., 0], w[..., 1], w[..., 2]
    theta = np.arccos(np.clip(z, -1.0, 1.0))
    phi = np.arctan2(y, x)
    out = np.empty(w.shape[:-1] + (nmodes(L),))
    s4 = np.sqrt(4.0 * np.pi)
    for l in range(L + 1):
        out[..., l * l + l] = s4 * special.sph_harm_y(l, 0, theta, phi).real
        for m in range(1, l + 1):
            Y = special.sph_harm_y(l, m, theta, phi)
            c = np.sqrt(2.0) * s4 * (-1.0) ** m
            out[..., l * l + l + m] = c * Y.real
            out[..., l * l + l - m] = c * Y.imag
    return out
