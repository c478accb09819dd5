"""Pins of the 3D anisotropic oracle (real spherical harmonics) against what the mathematics fixes
(no GPU needed): the basis's orthonormality and low-order closed forms, brute-force quadrature of
the self-cell integrals, the isotropic limit, the transpose identity of K~, agreement of LU, GMRES
and the Neumann series, the outward current of a centred source, exact rotation and reflection
equivariance on the grid, the mu_s = 0 closed form per mode, positivity, and which side of K~ the
scattering diagonal acts on.  A dropped Jacobian, a wrong sign of the flight direction, a missing
Y~ factor, a wrong normalisation of the harmonics or of sigma_hat_l fails at least one of them."""
import json
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import closed_form as cf
from oracle import kernels as K
from oracle import krylov as kr
from oracle import operator3d as op3
from oracle import operator3d_sh as o3s
from oracle import sh3d
from paper_1802_03061_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sphere_rule(nt=40, nphi=80):
    x, w = np.polynomial.legendre.leggauss(nt)
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    T, P = np.meshgrid(np.arccos(x), phi, indexing="ij")
    W = np.outer(w, np.full(nphi, 2 * np.pi / nphi)) / (4 * np.pi)        # mean over the sphere
    pts = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1)
    return pts, W


def test_real_harmonics_orthonormal_and_low_order_forms():
    pts, W = _sphere_rule()
    Y = sh3d.real_sh(4, pts)
    G = np.einsum("ij,ija,ijb->ab", W, Y, Y)
    assert np.abs(G - np.eye(25)).max() < 1e-13
    rng = np.random.default_rng(0)
    v = rng.standard_normal((20, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    x, y, z = v.T
    Yv = sh3d.real_sh(2, v)
    assert np.allclose(Yv[:, 0], 1.0, atol=1e-15)
    assert np.allclose(Yv[:, 1:4], np.sqrt(3) * np.stack([y, z, x], -1), atol=1e-14)
    assert np.allclose(Yv[:, 6], np.sqrt(5) * (3 * z * z - 1) / 2, atol=1e-14)
    assert np.allclose(Yv[:, 8], np.sqrt(15) / 2 * (x * x - y * y), atol=1e-14)
    assert np.allclose(Yv[:, 4], np.sqrt(15) * x * y, atol=1e-14)
    # addition theorem: sum over m of Y~_lm(v)^2 = 2l+1
    for l in range(3):
        assert np.allclose((Yv[:, l * l:(l + 1) ** 2] ** 2).sum(1), 2 * l + 1, atol=1e-13)


@pytest.mark.parametrize("mu_t", [1.05, 20.0])
@pytest.mark.parametrize("a,b", [(0, 0), (2, 2), (1, 3), (6, 6), (4, 4), (0, 6), (6, 8), (3, 5)])
def test_self_cell_pairs_vs_spherical_brute_force(mu_t, a, b):
    """c_ab against adaptive quadrature over the sphere of directions in spherical coordinates
    (radial part exact, R(w) = (h/2)/max|w_i|), split where the exit face changes."""
    L, h = 2, 1.0 / 16
    got = o3s.self_cell_pairs(L, h, mu_t)[a, b]
    half = 0.5 * h

    def g(t, p):
        w = np.array([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)])
        R = half / np.abs(w).max()
        Y = sh3d.real_sh(L, w)
        return np.sin(t) * Y[a] * Y[b] * (-np.expm1(-mu_t * R)) / mu_t / (4 * np.pi)

    tot = 0.0
    for q in range(8):
        p0, p1 = q * np.pi / 4, (q + 1) * np.pi / 4
        pm = 0.5 * (p0 + p1)
        # polar angle at which the exit face changes from the top to a side, for azimuth p
        tc = lambda p: np.arctan(1.0 / max(abs(np.cos(p)), abs(np.sin(p))))
        tl = lambda p: np.pi - tc(p)
        for lo, hi in ((lambda p: 0.0, tc), (tc, tl), (tl, lambda p: np.pi)):
            tot += integrate.dblquad(g, p0, p1, lo, hi, epsabs=1e-15, epsrel=1e-11)[0]
        del pm
    ref = K.self_cell_3d(h, mu_t)
    assert abs(got - tot) <= 1e-10 * ref
    if (sh3d.degree(a) + sh3d.degree(b)) % 2 == 1:
        assert abs(got) < 1e-16


def test_isotropic_limit_is_the_3d_isotropic_oracle():
    """L = 0 keeps the single mode Y~_00 = 1: K~ and the FFT apply equal oracle.operator3d exactly."""
    nz, ny, nx, h, mu_t, mu_s = 3, 4, 5, 0.25, 1.5, 1.2
    K0 = o3s.dense_Ktilde(nz, ny, nx, 0, h, mu_t)
    Ki = op3.dense_Ktilde(nz, ny, nx, h, mu_t)
    assert np.abs(K0 - Ki).max() <= 1e-14 * np.abs(Ki).max()      # quadrature rounding of the self cell
    u = np.random.default_rng(1).standard_normal((1, nz, ny, nx))
    y0 = o3s.apply_fft(u, 0, h, mu_t, mu_s, [1.0])
    yi = op3.apply_fft(u[0], h, mu_t, mu_s)
    assert np.abs(y0[0] - yi).max() <= 1e-14 * np.abs(yi).max()


def test_fft_apply_equals_direct_sum_and_sampled():
    """Circulant embedding reproduces the dense matrix, ragged grid, L = 2; so do sampled rows."""
    rng = np.random.default_rng(2)
    nz, ny, nx, L = 3, 4, 5, 2
    h, mu_t, mu_s = 0.2, 2.3, 1.9
    sh = [1.0, 0.6, 0.36]
    u = rng.standard_normal((9, nz, ny, nx))
    for op in ("A", "KT"):
        y1 = o3s.apply_direct(u, L, h, mu_t, mu_s, sh, op)
        y2 = o3s.apply_fft(u, L, h, mu_t, mu_s, sh, op)
        assert np.linalg.norm(y1 - y2) <= 1e-14 * np.linalg.norm(y1)
        cells = [(0, 0, 0), (2, 3, 4), (1, 2, 1)]
        ys = o3s.apply_sampled(u, cells, L, h, mu_t, mu_s, sh, op)
        for q, (iz, iy, ix) in enumerate(cells):
            assert np.abs(ys[q] - y1[:, iz, iy, ix]).max() <= 1e-14 * np.abs(y1).max()


def test_transpose_identity():
    """K~ is real and K~^T = J K~ J, J = diag((-1)^l): the flight direction reverses under the
    transpose and Y~_lm(-w) = (-1)^l Y~_lm(w).  K~ itself is not symmetric for L >= 1."""
    L = 2
    Kd = o3s.dense_Ktilde(3, 3, 4, L, 0.25, 1.7)
    N = 36
    J = np.repeat([(-1.0) ** sh3d.degree(a) for a in range(9)], N)
    assert np.abs(Kd.T - J[:, None] * Kd * J[None, :]).max() <= 1e-16 * np.abs(Kd).max() * 10
    assert np.abs(Kd.T - Kd).max() > 1e-3 * np.abs(Kd).max()


def _solve(f, L, n, mu_a, mu_s, sh):
    h = 1.0 / n
    mu_t = mu_a + mu_s
    A = o3s.dense_A(n, n, n, L, h, mu_t, mu_s, sh)
    b = o3s.rhs(f, L, h, mu_t, method="direct")
    return kr.solve_dense(A, b.reshape(-1)).reshape(b.shape)


def test_solvers_agree_and_gmres_bound():
    rng = np.random.default_rng(3)
    n, L = 4, 2
    h, mu_a, mu_s = 0.25, 0.3, 3.0
    mu_t = mu_a + mu_s
    sh = inputs.hg_sigma_hat(0.5, L)
    f = rng.random((n, n, n))
    A = o3s.dense_A(n, n, n, L, h, mu_t, mu_s, sh)
    b = o3s.rhs(f, L, h, mu_t, method="direct")
    x_lu = kr.solve_dense(A, b.reshape(-1)).reshape(b.shape)
    x_gm, hist = kr.gmres(lambda u: o3s.apply_fft(u, L, h, mu_t, mu_s, sh), b, 1e-14)
    x_ne = kr.neumann(lambda u: u - o3s.apply_fft(u, L, h, mu_t, mu_s, sh), b, 1e-15)
    nrm = np.linalg.norm(x_lu)
    assert np.linalg.norm(x_gm - x_lu) <= 1e-12 * nrm
    assert np.linalg.norm(x_ne - x_lu) <= 1e-12 * nrm
    c = np.linalg.norm(np.eye(A.shape[0]) - A, 2)
    assert c < 1
    for k, r in enumerate(hist):
        assert r <= c ** k * (1 + 1e-9) + 1e-15


def test_outward_current():
    """The current J = mean_v v Phi = (u_{1,1}, u_{1,-1}, u_{1,0}) / sqrt(3) points away from a
    centred source along every axis; with the flight direction reversed it would point inward."""
    n, L = 8, 1
    f = inputs.centred_gaussian_source(n, 0.08, d=3)
    u = _solve(f, L, n, 0.1, 1.0, inputs.hg_sigma_hat(0.5, L))
    Jx, Jy, Jz = u[3] / np.sqrt(3), u[1] / np.sqrt(3), u[2] / np.sqrt(3)
    c, lo, hi = n // 2, 1, n - 2
    assert Jx[c, c, hi] > 0 and Jx[c, c, lo] < 0
    assert Jy[c, hi, c] > 0 and Jy[c, lo, c] < 0
    assert Jz[hi, c, c] > 0 and Jz[lo, c, c] < 0


def _sh_transform(L, R):
    """Matrix D with Y~_a(R w) = sum_b D_ab Y~_b(w), fitted on random directions."""
    rng = np.random.default_rng(9)
    w = rng.standard_normal((400, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    Y = sh3d.real_sh(L, w)
    YR = sh3d.real_sh(L, w @ R.T)
    D = np.linalg.lstsq(Y, YR, rcond=None)[0].T
    assert np.abs(Y @ D.T - YR).max() < 1e-12
    return D


def test_rotation_and_reflection_equivariance():
    """A quarter turn about the z axis through the centre, x -> (-y, x) relative to the centre, with
    the rotated source f'(x) = f(R^{-1} x), gives u'_a(x) = sum_b D_ab u_b(R^{-1} x) with D the
    harmonics' transform, Y~_a(R w) = sum_b D_ab Y~_b(w); the reflection x1 -> 1 - x1 likewise.  Both
    are exact on the cell-centred grid."""
    n, L = 5, 2
    sh = inputs.hg_sigma_hat(0.5, L)
    f = np.random.default_rng(4).random((n, n, n))
    u = _solve(f, L, n, 0.1, 2.0, sh)
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    D = _sh_transform(L, Rz)
    # R^{-1}(x, y, z) = (y, -x, z) about the centre; in indices f'[iz, iy, ix] = f[iz, n-1-ix, iy]
    fr = np.empty_like(f)
    for iy in range(n):
        for ix in range(n):
            fr[:, iy, ix] = f[:, n - 1 - ix, iy]
    ur = _solve(fr, L, n, 0.1, 2.0, sh)
    want = np.empty_like(u)
    for iy in range(n):
        for ix in range(n):
            want[:, :, iy, ix] = np.einsum("ab,bz->az", D, u[:, :, n - 1 - ix, iy])
    assert np.abs(ur - want).max() <= 1e-12 * np.abs(u).max()
    P = np.diag([-1.0, 1.0, 1.0])
    Dp = _sh_transform(L, P)
    up = _solve(f[:, :, ::-1].copy(), L, n, 0.1, 2.0, sh)
    want = np.einsum("ab,bzyx->azyx", Dp, u[:, :, :, ::-1])
    assert np.abs(up - want).max() <= 1e-12 * np.abs(u).max()


@pytest.mark.slow
def test_mus0_closed_form_moments_first_order():
    """mu_s = 0, f = 1: the Nystrom u = K~ g converges at first order to the attenuated-source
    moments mean_w Y~_a(w) (1 - exp(-mu_t tau))/mu_t, for modes of degree 0, 1 and 2."""
    mu_t, L = 1.0, 2
    pts = ((0.5, 0.5, 0.5), (0.3, 0.6, 0.15), (0.8, 0.2, 0.7))
    modes = (0, 2, 3, 6, 4)
    exact = {}
    errs = []
    for n in (8, 16, 32):
        h = 1.0 / n
        b = o3s.rhs(np.ones((n, n, n)), L, h, mu_t, workers=os.cpu_count())
        e = 0.0
        for p in pts:
            iz, iy, ix = int(p[2] * n), int(p[1] * n), int(p[0] * n)
            x = ((ix + 0.5) * h, (iy + 0.5) * h, (iz + 0.5) * h)
            for a in modes:
                key = (n, p, a)
                exact[key] = cf.mus0_moment_3d(x, a, L, mu_t)
                scale = cf.mus0_moment_3d(x, 0, L, mu_t)
                e = max(e, abs(b[a, iz, iy, ix] - exact[key]) / scale)
        errs.append(e)
    assert errs[-1] < 3e-2
    for a, b_ in zip(errs[:-1], errs[1:]):
        assert 1.5 < a / b_ < 2.8


def test_positivity_and_moment_bounds():
    """f >= 0 and a non-negative truncated phase function (HG g = 0.5 to l = 2:
    sigma(t) = 0.375 + 1.5 t + 1.875 t^2 > 0) keep Phi >= 0, so u_0 > 0 and
    |u_lm| <= sqrt(2l+1) u_0 (Cauchy-Schwarz with the addition theorem)."""
    n, L = 6, 2
    f = inputs.centred_gaussian_source(n, 0.1, d=3)
    u = _solve(f, L, n, 0.1, 3.0, inputs.hg_sigma_hat(0.5, L))
    assert u[0].min() > 0
    for a in range(1, 9):
        l = sh3d.degree(a)
        assert (np.abs(u[a]) <= np.sqrt(2 * l + 1) * u[0] * (1 + 1e-12)).all()


def test_scattering_diagonal_acts_on_the_input_modes():
    """With sigma_hat = (1, 0, 0) only mode 0 scatters: mode 0 obeys the 3D isotropic equation
    (oracle.operator3d) and every mode is the transported isotropic source
    u_a = (K~ (mu_s u_0 + f) e_0)_a; the output-side reading A = I - D K~ fails the first."""
    n, L = 5, 2
    h, mu_a, mu_s = 1.0 / n, 0.1, 2.0
    mu_t = mu_a + mu_s
    f = inputs.centred_gaussian_source(n, 0.12, d=3)
    sh = np.array([1.0, 0.0, 0.0])
    u = _solve(f, L, n, mu_a, mu_s, sh)
    Ai = op3.dense_A(n, n, n, h, mu_t, mu_s)
    ui = np.linalg.solve(Ai, op3.dense_Ktilde(n, n, n, h, mu_t) @ f.reshape(-1)).reshape(f.shape)
    assert np.abs(u[0] - ui).max() <= 1e-13 * np.abs(ui).max()
    want = o3s.apply_direct(o3s.source_vector(mu_s * u[0] + f, L), L, h, mu_t, 0.0, np.ones(L + 1), op="KT")
    assert np.abs(u - want).max() <= 1e-13 * np.abs(u).max()
    assert np.abs(u[2:4]).max() > 1e-3 * np.abs(u[0]).max() or np.abs(u[1]).max() > 1e-3 * np.abs(u[0]).max()
    Kd = o3s.dense_Ktilde(n, n, n, L, h, mu_t)
    d = np.repeat(o3s.mode_scaling(L, mu_s, sh), n ** 3)
    b = o3s.rhs(f, L, h, mu_t, method="direct").reshape(-1)
    u_out = np.linalg.solve(np.eye(Kd.shape[0]) - d[:, None] * Kd, b).reshape(u.shape)
    assert np.abs(u_out[0] - ui).max() > 1e-4 * np.abs(ui).max()


def test_iso3d_golden_density_at_L0_matches():
    """Golden cross-check with the 3D isotropic oracle's stored constant: the mu_t -> 0 self-cell
    limit (3 I / pi) h of the mode-0 pair."""
    with open(os.path.join(GOLDEN, "self_cell_limits.json")) as fh:
        gold = json.load(fh)
    h = 1.0 / 64
    c = o3s.self_cell_pairs(1, h, 0.0)
    assert abs(c[0, 0] / h - gold["c3d_over_h"]) < 1e-13
    # degree-1 diagonal entries equal the mode-0 one by the cube's symmetry (sum_m Y~_1m^2 = 3)
    assert np.allclose(np.diag(c)[1:4], c[0, 0], rtol=1e-13)
