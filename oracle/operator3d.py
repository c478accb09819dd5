"""The discrete 3D isotropic operator (TEST INFRASTRUCTURE ONLY: see oracle/__init__.py).

With only the mode 0 kept (the isotropic case M = {0}, end of Sec. 3.1.2) the 3D equation is the
u-form of eq. iso_Fredholm: u = mu_s K~ u + K~ f, K~ the Nystrom matrix of
kappa(r) = exp(-mu_t r)/(4 pi r^2) on an nz x ny x nx grid of cubic cells of side h.
Arrays are indexed [iz, iy, ix].
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .kernels import kernel_entry_3d


def dense_Ktilde(nz: int, ny: int, nx: int, h: float, mu_t: float) -> np.ndarray:
    N = nz * ny * nx
    iz, rem = np.divmod(np.arange(N), ny * nx)
    iy, ix = np.divmod(rem, nx)
    return kernel_entry_3d(ix[:, None] - ix[None, :], iy[:, None] - iy[None, :],
                           iz[:, None] - iz[None, :], h, mu_t)


def dense_A(nz, ny, nx, h, mu_t, mu_s) -> np.ndarray:
    K = dense_Ktilde(nz, ny, nx, h, mu_t)
    return np.eye(K.shape[0]) - mu_s * K


def apply_sampled(u: np.ndarray, cells, h: float, mu_t: float, mu_s: float, op: str = "A"):
    """(A u)_i or (K~ u)_i at output cells (iz, iy, ix) by the direct sum over all cells."""
    nz, ny, nx = u.shape
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros(len(cells))
    for c, (iz, iy, ix) in enumerate(cells):
        K = kernel_entry_3d(ix - X, iy - Y, iz - Z, h, mu_t)
        s = float(np.sum(K * u))
        out[c] = (u[iz, iy, ix] - mu_s * s) if op == "A" else s
    return out


def kernel_spectrum(nz: int, ny: int, nx: int, h: float, mu_t: float,
                    workers: int | None = None) -> np.ndarray:
    """FFT of the wrapped kernel table on the (2nz, 2ny, 2nx) padded grid (circulant embedding).
    The table is real, so its real-input transform (last axis halved) is kept."""
    P = (2 * nz, 2 * ny, 2 * nx)
    oz = np.arange(-(nz - 1), nz)
    oy = np.arange(-(ny - 1), ny)
    ox = np.arange(-(nx - 1), nx)
    OZ, OY, OX = np.meshgrid(oz, oy, ox, indexing="ij")
    tab = np.zeros(P)
    tab[OZ % P[0], OY % P[1], OX % P[2]] = kernel_entry_3d(OX, OY, OZ, h, mu_t)
    return sfft.rfftn(tab, workers=workers)


def apply_fft(u: np.ndarray, h: float, mu_t: float, mu_s: float, op: str = "A",
              spectrum=None, workers: int | None = None) -> np.ndarray:
    """y = u - mu_s K~ u (op "A") or y = K~ u (op "KT") for a real density u by circulant
    embedding: zero-pad to (2nz, 2ny, 2nx), transform, multiply by the kernel spectrum, inverse
    transform, keep the first nz x ny x nx."""
    nz, ny, nx = u.shape
    P = (2 * nz, 2 * ny, 2 * nx)
    if spectrum is None:
        spectrum = kernel_spectrum(nz, ny, nx, h, mu_t, workers)
    scale = mu_s if op == "A" else 1.0
    pad = np.zeros(P)
    pad[:nz, :ny, :nx] = scale * np.asarray(u).real
    v = sfft.irfftn(spectrum * sfft.rfftn(pad, workers=workers), s=P, workers=workers)[:nz, :ny, :nx]
    return u - v if op == "A" else v
