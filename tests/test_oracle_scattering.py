"""Pins of the oracle's scattering term S(x, theta) = mu_s sum_k sigma_hat_|k| u_k e^{i k theta}
(eq. ani_2d_scattering) against facts that do not reuse its sum: the isotropic closed form, the
angular mean, and a library DFT over the angles that gives back each mode."""
import numpy as np
import pytest

from oracle.scattering import scattering_term
from paper_1802_03061_amd import inputs


def _conj_modes(rng, L, shape):
    u = np.zeros((2 * L + 1,) + shape, complex)
    u[L] = rng.standard_normal(shape)
    for k in range(1, L + 1):
        z = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        u[L + k], u[L - k] = z, np.conj(z)
    return u


def test_isotropic_is_mu_s_times_density():
    rng = np.random.default_rng(0)
    u = rng.standard_normal((1, 5, 7)) + 0j
    S = scattering_term(u, 0, 2.5, [1.0], 9)
    assert np.allclose(S, 2.5 * u[0].real[None], rtol=0, atol=1e-15)


@pytest.mark.parametrize("ntheta", [5, 12, 64])
def test_angular_mean_is_mode_zero(ntheta):
    # sum_q e^{i k theta_q} = 0 for 0 < |k| < ntheta, so the mean over the angles keeps mode 0 only
    L = 4
    rng = np.random.default_rng(ntheta)
    u = _conj_modes(rng, L, (6, 3))
    sh = inputs.hg_sigma_hat(0.6, L)
    S = scattering_term(u, L, 3.0, sh, ntheta)
    assert np.allclose(S.mean(axis=0), 3.0 * sh[0] * u[L].real, rtol=0, atol=1e-13)


@pytest.mark.parametrize("L,ntheta", [(1, 3), (4, 9), (8, 40)])
def test_dft_over_angles_recovers_the_modes(L, ntheta):
    # with ntheta > 2L there is no aliasing: the DFT of S over q at index k (mod ntheta) is
    # ntheta mu_s sigma_hat_|k| u_k for the image of a real flux, and for a general complex input
    # ntheta (mu_s/2)(sigma_hat_|k| u_k + conj(sigma_hat_|k| u_{-k}))
    rng = np.random.default_rng(L)
    sh = inputs.hg_sigma_hat(0.5, L)
    for general in (False, True):
        u = _conj_modes(rng, L, (4, 5))
        if general:
            u = u + 1j * rng.standard_normal(u.shape) + rng.standard_normal(u.shape)
        S = scattering_term(u, L, 1.7, sh, ntheta)
        F = np.fft.fft(S, axis=0) / ntheta
        for k in range(-L, L + 1):
            want = 1.7 * sh[abs(k)] * (u[k + L] + np.conj(u[-k + L])) / 2
            assert np.allclose(F[k % ntheta], want, rtol=0, atol=1e-12)
        for q in range(L + 1, ntheta - L):   # frequencies past L are empty
            assert np.abs(F[q]).max() <= 1e-12


def test_single_mode_is_a_cosine():
    # u_1 = u_{-1} = 1/2 (a flux cos(theta)) gives S = mu_s sigma_hat_1 cos(theta)
    L, ntheta = 1, 16
    u = np.zeros((3, 1, 1), complex)
    u[2] = u[0] = 0.5
    S = scattering_term(u, L, 2.0, [1.0, 0.4], ntheta)[:, 0, 0]
    theta = 2 * np.pi * np.arange(ntheta) / ntheta
    assert np.allclose(S, 2.0 * 0.4 * np.cos(theta), rtol=0, atol=1e-15)
