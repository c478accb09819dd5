"""The discrete 3D anisotropic operator in real spherical harmonics (TEST INFRASTRUCTURE ONLY: see
oracle/__init__.py).

Sec. 3.1.2 expands the flux and the phase function in spherical harmonics and arrives at the
Fredholm equation eq. ani_3d_Fredholm; its printed kernel is garbled (a missing Jacobian and
conjugate, an integral over the wrong variable, two names for one operator), so the equation is
re-derived here from the characteristic solution, the way Sec. 3.1.1 derives the 2D one.

Reading.  The phase function sigma(v . v') has unit mean over the sphere and Legendre coefficients
sigma_hat_l = (1/2) int_{-1}^{1} sigma(t) P_l(t) dt (sigma_hat_0 = 1; Henyey-Greenstein:
sigma_hat_l = g^l).  By the Funk-Hecke theorem the scattering operator acts on the real harmonics
Y~_a of oracle.sh3d by mean_{v'} sigma(v . v') Y~_a(v') = sigma_hat_{l(a)} Y~_a(v).  With
Phi(x, v) = sum_a u_a(x) Y~_a(v), u_a(x) = mean_v Phi(x, v) Y~_a(v), the characteristic solution
Phi(x, v) = int_0^tau exp(-mu_t s) S(x - s v, v) ds of eq. ani_solution, with the scattering source
S(y, v) = sum_b (mu_s sigma_hat_{l(b)} u_b(y) + f(y) delta_{b0}) Y~_b(v), becomes after the change of
variables y = x - s v (dy = s^2 ds dv, v = (x - y)/|x - y|)

    u_a(x) = sum_b int_Omega kappa(|x - y|) Y~_a(w) Y~_b(w) (mu_s sigma_hat_{l(b)} u_b(y) + f(y) delta_{b0}) dy,
    kappa(r) = exp(-mu_t r) / (4 pi r^2),   w = (x - y)/|x - y|.

So, as in 2D, (I - K~ D) u = K~ g with D = diag(mu_s sigma_hat_{l(a)}) acting on the input modes and
g = f in mode 0.  K~ is real; its (a, b) block is the Nystrom matrix of kappa(r) Y~_a(w) Y~_b(w):
point values times h^3 off the diagonal and the exact cell integral on it.  Keeping l <= L gives
(L+1)^2 modes; L = 0 is the isotropic u-form of oracle.operator3d.  Unknowns are u[a, iz, iy, ix].
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.fft as sfft

from .kernels import gauss_legendre
from .sh3d import degree, nmodes, real_sh


def mode_scaling(L: int, mu_s: float, sigma_hat) -> np.ndarray:
    """Diagonal of D per mode a: mu_s sigma_hat_{l(a)}."""
    s = np.asarray(sigma_hat, dtype=np.float64)
    return np.array([mu_s * s[degree(a)] for a in range(nmodes(L))])


def self_cell_pairs(L: int, h: float, mu_t: float, npts: int = 48) -> np.ndarray:
    """c[a, b] = integral over the cube [-h/2, h/2]^3 of kappa(|z|) Y~_a(z/|z|) Y~_b(z/|z|).

    In polar coordinates about the centre the radial integral is exact:
        (1/4pi) int_{S^2} Y~_a Y~_b (1 - exp(-mu_t R(w)))/mu_t dw,
    R(w) the distance to the cube's surface.  The sphere is split by the six faces: the directions
    through the face point p (|p_axis| = a = h/2) have R = |p| and solid angle a/|p|^3 dA, and each
    face is integrated by Gauss-Legendre on its four quarters (the integrand is smooth there)."""
    a = 0.5 * h
    t, wt = gauss_legendre(npts, 0.0, a)
    s = np.concatenate([-t[::-1], t])
    ws = np.concatenate([wt[::-1], wt])
    U, V = np.meshgrid(s, s, indexing="ij")
    W = np.outer(ws, ws)
    M = nmodes(L)
    c = np.zeros((M, M))
    for axis in range(3):
        others = [q for q in range(3) if q != axis]
        for sign in (-1.0, 1.0):
            p = np.empty(U.shape + (3,))
            p[..., axis] = sign * a
            p[..., others[0]] = U
            p[..., others[1]] = V
            rho = np.linalg.norm(p, axis=-1)
            radial = (rho if mu_t == 0.0 else -np.expm1(-mu_t * rho) / mu_t) * a / rho ** 3
            Y = real_sh(L, p / rho[..., None])
            c += np.einsum("ij,ija,ijb->ab", W * radial, Y, Y)
    return c / (4.0 * np.pi)


def _offsets_sh(ox, oy, oz, L):
    o = np.stack([np.asarray(ox, float), np.asarray(oy, float), np.asarray(oz, float)], axis=-1)
    r = np.linalg.norm(o, axis=-1)
    rs = np.where(r == 0.0, 1.0, r)
    Y = real_sh(L, o / rs[..., None])
    return r, Y


def kernel_table_pair(nz, ny, nx, a, b, L, h, mu_t, cself=None) -> np.ndarray:
    """K_ab on all offsets o in (-n, n)^3: h^3 kappa(h|o|) Y~_a(o/|o|) Y~_b(o/|o|), the exact cell
    integral at o = 0.  Indexed [oz + nz - 1, oy + ny - 1, ox + nx - 1]."""
    OZ, OY, OX = np.meshgrid(np.arange(-(nz - 1), nz), np.arange(-(ny - 1), ny), np.arange(-(nx - 1), nx),
                             indexing="ij")
    r, Y = _offsets_sh(OX, OY, OZ, L)
    rr = h * np.where(r == 0.0, 1.0, r)
    val = h ** 3 * np.exp(-mu_t * rr) / (4.0 * np.pi * rr * rr) * Y[..., a] * Y[..., b]
    if cself is None:
        cself = self_cell_pairs(L, h, mu_t)
    return np.where(r == 0.0, cself[a, b], val)


def dense_Ktilde(nz, ny, nx, L, h, mu_t) -> np.ndarray:
    """The full real (M N) x (M N) matrix K~, row/column index a N + (iz ny + iy) nx + ix."""
    N = nz * ny * nx
    M = nmodes(L)
    iz, rem = np.divmod(np.arange(N), ny * nx)
    iy, ix = np.divmod(rem, nx)
    r, Y = _offsets_sh(ix[:, None] - ix[None, :], iy[:, None] - iy[None, :], iz[:, None] - iz[None, :], L)
    rr = h * np.where(r == 0.0, 1.0, r)
    kap = np.where(r == 0.0, 0.0, h ** 3 * np.exp(-mu_t * rr) / (4.0 * np.pi * rr * rr))
    c = self_cell_pairs(L, h, mu_t)
    K = np.zeros((M * N, M * N))
    eye = np.eye(N)
    for a in range(M):
        for b in range(M):
            K[a * N:(a + 1) * N, b * N:(b + 1) * N] = kap * Y[..., a] * Y[..., b] + c[a, b] * eye
    return K


def dense_A(nz, ny, nx, L, h, mu_t, mu_s, sigma_hat) -> np.ndarray:
    """A = I - K~ D as a dense matrix."""
    K = dense_Ktilde(nz, ny, nx, L, h, mu_t)
    d = np.repeat(mode_scaling(L, mu_s, sigma_hat), nz * ny * nx)
    return np.eye(K.shape[0]) - K * d[None, :]


def source_vector(f: np.ndarray, L: int) -> np.ndarray:
    """g[a] = f delta_{a0}, shape ((L+1)^2, nz, ny, nx)."""
    g = np.zeros((nmodes(L),) + f.shape)
    g[0] = f
    return g


def apply_sampled(u: np.ndarray, cells, L: int, h: float, mu_t: float, mu_s: float, sigma_hat,
                  op: str = "A") -> np.ndarray:
    """Rows of A u (or K~ u) at the output cells (iz, iy, ix) only, by the direct sum over every
    cell and mode: y_a = sum_j kappa_ij Y~_a(w_ij) sum_b Y~_b(w_ij) w_b(j) + sum_b c_ab w_b(i),
    w = D u (u for K~).  Returns shape (len(cells), (L+1)^2)."""
    M, nz, ny, nx = u.shape
    d = mode_scaling(L, mu_s, sigma_hat) if op == "A" else np.ones(M)
    w = (u * d[:, None, None, None]).reshape(M, -1)
    Z, Yg, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    Z, Yg, X = Z.reshape(-1), Yg.reshape(-1), X.reshape(-1)
    c = self_cell_pairs(L, h, mu_t)
    out = np.zeros((len(cells), M))
    for q, (iz, iy, ix) in enumerate(cells):
        r, Ysh = _offsets_sh(ix - X, iy - Yg, iz - Z, L)
        rr = h * np.where(r == 0.0, 1.0, r)
        kap = np.where(r == 0.0, 0.0, h ** 3 * np.exp(-mu_t * rr) / (4.0 * np.pi * rr * rr))
        s = np.einsum("jb,bj->j", Ysh, w)                     # sum_b Y~_b(w_ij) w_b(j)
        j0 = (iz * ny + iy) * nx + ix
        v = Ysh.T @ (kap * s) + c @ w[:, j0]
        out[q] = (u[:, iz, iy, ix] - v) if op == "A" else v
    return out


def apply_direct(u: np.ndarray, L: int, h: float, mu_t: float, mu_s: float, sigma_hat, op: str = "A"):
    """y = A u or K~ u with the dense matrix (small grids)."""
    M, nz, ny, nx = u.shape
    K = dense_Ktilde(nz, ny, nx, L, h, mu_t)
    d = mode_scaling(L, mu_s, sigma_hat) if op == "A" else np.ones(M)
    v = (K @ (u * d[:, None, None, None]).reshape(-1)).reshape(u.shape)
    return u - v if op == "A" else v


def kernel_spectra(nz, ny, nx, L, h, mu_t, workers: int | None = None) -> dict:
    """Real-input FFTs of the wrapped tables K_ab on the (2nz, 2ny, 2nx) grid (circulant embedding;
    offsets +-n stay zero), for a <= b; K_ba = K_ab.  The tables are kernel_table_pair's entries,
    with kappa and the harmonics of every offset evaluated once for all pairs."""
    P = (2 * nz, 2 * ny, 2 * nx)
    OZ, OY, OX = np.meshgrid(np.arange(-(nz - 1), nz), np.arange(-(ny - 1), ny), np.arange(-(nx - 1), nx),
                             indexing="ij")
    r, Y = _offsets_sh(OX, OY, OZ, L)
    rr = h * np.where(r == 0.0, 1.0, r)
    kap = h ** 3 * np.exp(-mu_t * rr) / (4.0 * np.pi * rr * rr)
    zero = r == 0.0
    c = self_cell_pairs(L, h, mu_t)
    M = nmodes(L)
    spectra = {}
    for a in range(M):
        for b in range(a, M):
            tab = np.zeros(P)
            tab[OZ % P[0], OY % P[1], OX % P[2]] = np.where(zero, c[a, b], kap * Y[..., a] * Y[..., b])
            spectra[(a, b)] = sfft.rfftn(tab, workers=workers)
    return spectra


def apply_fft(u: np.ndarray, L: int, h: float, mu_t: float, mu_s: float, sigma_hat, op: str = "A",
              spectra=None, workers: int | None = None) -> np.ndarray:
    """The same operator by circulant embedding: zero-pad each mode to (2nz, 2ny, 2nx), transform,
    output mode a gets sum_b FFT(K_ab) FFT(w_b), inverse transform, keep the first nz x ny x nx."""
    M, nz, ny, nx = u.shape
    P = (2 * nz, 2 * ny, 2 * nx)
    if spectra is None:
        spectra = kernel_spectra(nz, ny, nx, L, h, mu_t, workers)
    d = mode_scaling(L, mu_s, sigma_hat) if op == "A" else np.ones(M)
    W = []
    for b in range(M):
        pad = np.zeros(P)
        pad[:nz, :ny, :nx] = d[b] * np.asarray(u[b]).real
        W.append(sfft.rfftn(pad, workers=workers))
    v = np.zeros(u.shape)
    nthreads = min(M, workers or 1)
    inner = 1 if nthreads > 1 else workers

    def output_mode(a):
        acc = np.zeros_like(W[0])
        tmp = np.empty_like(acc)
        for b in range(M):
            np.multiply(spectra[(min(a, b), max(a, b))], W[b], out=tmp)
            acc += tmp
        v[a] = sfft.irfftn(acc, s=P, workers=inner)[:nz, :ny, :nx]

    if nthreads > 1:
        with ThreadPoolExecutor(nthreads) as ex:
            list(ex.map(output_mode, range(M)))
    else:
        for a in range(M):
            output_mode(a)
    return u - v if op == "A" else v


def rhs(f: np.ndarray, L: int, h: float, mu_t: float, method: str = "fft", spectra=None,
        workers: int | None = None) -> np.ndarray:
    """b = K~ g with g = f in mode 0."""
    g = source_vector(np.asarray(f, dtype=np.float64), L)
    ones = np.ones(L + 1)
    if method == "direct":
        return apply_direct(g, L, h, mu_t, 0.0, ones, op="KT")
    return apply_fft(g, L, h, mu_t, 0.0, ones, op="KT", spectra=spectra, workers=workers)
