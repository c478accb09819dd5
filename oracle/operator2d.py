"""The discrete 2D operator, written out plainly (TEST INFRASTRUCTURE ONLY: see oracle/__init__.py).

Unknowns u[k + L, iy, ix] approximate the angular Fourier mode k of the flux at the cell centre
(ix + 1/2, iy + 1/2) h (eq. ani_discretization, Sec. 3.3).  For an ny x nx grid of cells of side h
and modes k = -L..L:

  (K~ w)[k, i] = sum_j sum_{k'} K_{k'-k}[i - j] w[k', j]               (K_m from oracle.kernels)
  D = diag(mu_s sigma_hat_|k|)          (sigma_hat_{-k} = sigma_hat_k for a real even phase function)
  A u = u - K~ D u                       (eq. ani_AU: A = I - K)
  b   = K~ g,  g[k, j] = f_j delta_{k0}  (step T.1; the mu_s in K and the 1/mu_s in f cancel)

L = 0 is the isotropic u-form u = K u + K~ f (eq. iso_Fredholm, discretised per Sec. 2.3).
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.fft as sfft

from .kernels import kernel_table_2d, kernel_entry_2d


def mode_scaling(L: int, mu_s: float, sigma_hat) -> np.ndarray:
    """Diagonal of D per mode index k + L: mu_s * sigma_hat_|k|."""
    s = np.asarray(sigma_hat, dtype=np.float64)
    return np.array([mu_s * s[abs(k)] for k in range(-L, L + 1)])


def dense_Ktilde(ny: int, nx: int, L: int, h: float, mu_t: float) -> np.ndarray:
    """The full NM x NM matrix K~, row/column index (k + L) * N + iy * nx + ix."""
    N = ny * nx
    M = 2 * L + 1
    iy, ix = np.divmod(np.arange(N), nx)
    OX = ix[:, None] - ix[None, :]
    OY = iy[:, None] - iy[None, :]
    K = np.zeros((M * N, M * N), dtype=np.complex128)
    for a, k in enumerate(range(-L, L + 1)):
        for b, kp in enumerate(range(-L, L + 1)):
            K[a * N:(a + 1) * N, b * N:(b + 1) * N] = kernel_entry_2d(OX, OY, kp - k, h, mu_t)
    return K


def dense_A(ny, nx, L, h, mu_t, mu_s, sigma_hat) -> np.ndarray:
    """A = I - K~ D as a dense matrix."""
    K = dense_Ktilde(ny, nx, L, h, mu_t)
    d = np.repeat(mode_scaling(L, mu_s, sigma_hat), ny * nx)
    return np.eye(K.shape[0]) - K * d[None, :]


def source_vector(f: np.ndarray, L: int) -> np.ndarray:
    """g[k, j] = f_j delta_{k0}, shape (2L+1, ny, nx)."""
    g = np.zeros((2 * L + 1,) + f.shape, dtype=np.complex128)
    g[L] = f
    return g


def apply_direct(u: np.ndarray, L: int, h: float, mu_t: float, mu_s: float, sigma_hat,
                 op: str = "A") -> np.ndarray:
    """y = A u (op "A") or y = K~ u (op "KT") by the direct double sum over cells and modes.
    u has shape (2L+1, ny, nx).  Cost (N M)^2; meant for small grids."""
    M, ny, nx = u.shape
    assert M == 2 * L + 1
    N = ny * nx
    iy, ix = np.divmod(np.arange(N), nx)
    OX = ix[:, None] - ix[None, :]
    OY = iy[:, None] - iy[None, :]
    d = mode_scaling(L, mu_s, sigma_hat) if op == "A" else np.ones(M)
    w = (u * d[:, None, None]).reshape(M, N)
    blocks = {m: kernel_entry_2d(OX, OY, m, h, mu_t) for m in range(-2 * L, 2 * L + 1)}
    v = np.zeros((M, N), dtype=np.complex128)
    for a, k in enumerate(range(-L, L + 1)):
        for b, kp in enumerate(range(-L, L + 1)):
            v[a] += blocks[kp - k] @ w[b]
    v = v.reshape(M, ny, nx)
    return u - v if op == "A" else v


def apply_sampled(u: np.ndarray, cells, L: int, h: float, mu_t: float, mu_s: float, sigma_hat,
                  op: str = "A") -> np.ndarray:
    """Rows of A u (or K~ u) at the given output cells only: cells is a list of (iy, ix).
    Returns shape (len(cells), 2L+1).  Cost per cell N M^2."""
    M, ny, nx = u.shape
    N = ny * nx
    jy, jx = np.divmod(np.arange(N), nx)
    d = mode_scaling(L, mu_s, sigma_hat) if op == "A" else np.ones(M)
    w = (u * d[:, None, None]).reshape(M, N)          # w[k', j]
    ms = list(range(-2 * L, 2 * L + 1))
    out = np.zeros((len(cells), M), dtype=np.complex128)
    for c, (iy, ix) in enumerate(cells):
        Km = np.stack([kernel_entry_2d(ix - jx, iy - jy, m, h, mu_t) for m in ms])  # (4L+1, N)
        T = Km @ w.T                                    # T[m, k'] = sum_j K_m[i-j] w[k', j]
        for a, k in enumerate(range(-L, L + 1)):
            s = 0.0
            for b, kp in enumerate(range(-L, L + 1)):
                s = s + T[kp - k + 2 * L, b]
            out[c, a] = (u[a, iy, ix] - s) if op == "A" else s
    return out


def kernel_spectra(ny: int, nx: int, L: int, h: float, mu_t: float, workers: int | None = None):
    """FFTs of the zero-padded, periodically wrapped kernel tables on a (2ny, 2nx) grid, for
    every mode difference m = -2L..2L (circulant embedding, Sec. 2.3.1 and 3.3.1).  Offset o is
    stored at index o mod P; the offsets +-n are never used and stay zero."""
    Py, Px = 2 * ny, 2 * nx
    spectra = {}
    oy = np.arange(-(ny - 1), ny)
    ox = np.arange(-(nx - 1), nx)
    OY, OX = np.meshgrid(oy, ox, indexing="ij")
    for m in range(-2 * L, 2 * L + 1):
        tab = np.zeros((Py, Px), dtype=np.complex128)
        tab[OY % Py, OX % Px] = kernel_entry_2d(OX, OY, m, h, mu_t)
        spectra[m] = sfft.fft2(tab, workers=workers)
    return spectra


def apply_fft(u: np.ndarray, L: int, h: float, mu_t: float, mu_s: float, sigma_hat,
              op: str = "A", spectra=None, workers: int | None = None) -> np.ndarray:
    """The same operator by circulant embedding: zero-pad each mode to (2ny, 2nx), FFT, multiply
    output mode k by sum_{k'} FFT(K_{k'-k}) FFT(w_{k'}), inverse FFT, keep the first ny x nx."""
    M, ny, nx = u.shape
    if spectra is None:
        spectra = kernel_spectra(ny, nx, L, h, mu_t)
    d = mode_scaling(L, mu_s, sigma_hat) if op == "A" else np.ones(M)
    W = []
    for b in range(M):
        pad = np.zeros((2 * ny, 2 * nx), dtype=np.complex128)
        pad[:ny, :nx] = d[b] * u[b]
        W.append(sfft.fft2(pad, workers=workers))
    v = np.zeros_like(u, dtype=np.complex128)

    def output_mode(a):
        # sum over input modes k' in increasing order, as written above
        k = a - L
        acc = np.zeros((2 * ny, 2 * nx), dtype=np.complex128)
        tmp = np.empty_like(acc)
        for b, kp in enumerate(range(-L, L + 1)):
            np.multiply(spectra[kp - k], W[b], out=tmp)
            acc += tmp
        v[a] = sfft.ifft2(acc, workers=inner)[:ny, :nx]

    nthreads = min(M, workers or 1)
    inner = 1 if nthreads > 1 else workers
    if nthreads > 1:
        # the output modes are independent sums: evaluate them on a thread pool
        with ThreadPoolExecutor(nthreads) as ex:
            list(ex.map(output_mode, range(M)))
    else:
        for a in range(M):
            output_mode(a)
    return u - v if op == "A" else v


def rhs(f: np.ndarray, L: int, h: float, mu_t: float, method: str = "fft", spectra=None,
        workers: int | None = None):
    """b = K~ g with g = f delta_{k0} (step T.1)."""
    g = source_vector(f, L)
    if method == "direct":
        return apply_direct(g, L, h, mu_t, 0.0, np.ones(L + 1), op="KT")
    return apply_fft(g, L, h, mu_t, 0.0, np.ones(L + 1), op="KT", spectra=spectra, workers=workers)
