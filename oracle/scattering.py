"""The scattering term at discrete angles, written out plainly (TEST INFRASTRUCTURE ONLY: see
oracle/__init__.py).

With the angular Fourier modes u[k + L] of the flux (k = -L..L) and the truncated phase function
sigma(theta) ~ sum_k sigma_hat_|k| e^{i k theta}, the scattering term of Sec. 3.1 is

  S(x, theta) = mu_s sum_{k=-L..L} sigma_hat_|k| u_k(x) e^{i k theta}      (eq. ani_2d_scattering)

(the operator A~ applied to the flux, times mu_s).  It is real for the image of a real flux
(u_{-k} = conj u_k); for any other input the real part is taken.  The angles are
theta_q = 2 pi q / ntheta, q = 0..ntheta-1.
"""
from __future__ import annotations

import numpy as np


def scattering_term(u: np.ndarray, L: int, mu_s: float, sigma_hat, ntheta: int) -> np.ndarray:
    """S[q, ...] = Re( mu_s sum_k sigma_hat_|k| u[k + L, ...] exp(i k theta_q) ), as defined above."""
    sh = np.asarray(sigma_hat, dtype=np.float64)
    theta = 2.0 * np.pi * np.arange(ntheta) / ntheta
    out = np.zeros((ntheta,) + u.shape[1:], dtype=np.float64)
    for k in range(-L, L + 1):
        phase = np.exp(1j * k * theta).reshape((ntheta,) + (1,) * (u.ndim - 1))
        out += (mu_s * sh[abs(k)] * u[k + L][None] * phase).real
    return out
