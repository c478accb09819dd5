"""Seeded synthetic inputs shared by the HIP path's tests/bench and the CPU oracle.

This module only *describes workloads*: grids of cell centres, source terms f sampled at the cell
centres, the scattering coefficients of the phase functions, random test vectors and the batched
problem list.  It holds none of the method's arithmetic (no kernel, no operator, no solver), so
both sides can take their inputs from here without sharing any of the computation under test.

Conventions
-----------
* Domain [0,1]^d split into n^d square cells of side h = 1/n; unknowns and sources live at the
  cell centres x_i = (i + 1/2) h (Nystrom points of Sec. 2.3, "Fast algorithms").
* 2D arrays are indexed [iy][ix] (x fastest); 3D arrays [iz][iy][ix].
* Angular modes k = -L..L are stored at index k + L.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "cell_centres", "gaussian", "centred_gaussian_source", "paper_sources",
    "gaussian_mixture_params", "gaussian_mixture_source", "hg_sigma_hat", "paper_sigma_hat",
    "random_modes", "random_conj_symmetric_modes", "batched_problems", "workload",
]


def cell_centres(n: int, d: int = 2):
    """Coordinates of the n^d cell centres of [0,1]^d, as d arrays of shape (n,)*d.

    2D returns (X, Y) with X[iy, ix] = (ix + 1/2)/n; 3D returns (X, Y, Z) indexed [iz, iy, ix]."""
    c = (np.arange(n, dtype=np.float64) + 0.5) / n
    if d == 2:
        Y, X = np.meshgrid(c, c, indexing="ij")
        return X, Y
    if d == 3:
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        return X, Y, Z
    raise ValueError("d must be 2 or 3")


def gaussian(n: int, centre, width: float, d: int = 2) -> np.ndarray:
    """exp(-|x - centre|^2 / (2 width^2)) at the cell centres."""
    P = cell_centres(n, d)
    r2 = sum((P[a] - centre[a]) ** 2 for a in range(d))
    return np.exp(-r2 / (2.0 * width * width))


def centred_gaussian_source(n: int, width: float = 0.1, d: int = 2) -> np.ndarray:
    """The single centred Gaussian exp(-|x-(1/2,..)|^2/(2*0.1^2)) of the small isotropic case."""
    return gaussian(n, [0.5] * d, width, d)


def paper_sources(n: int) -> dict:
    """The three 2D test sources of the numerical section (eq. source): two normalised Gaussians
    with T = 4e-3 at (0.3,0.7) and (0.7,0.3); an annulus |x-(0.6,0.4)| in [3/20,1/4]; and the
    indicator of the square [1/2,3/4]^2."""
    X, Y = cell_centres(n, 2)
    T = 4e-3
    norm = 1.0 / np.sqrt(2.0 * np.pi * T)
    f1 = norm * (np.exp(-((X - 0.3) ** 2 + (Y - 0.7) ** 2) / (2 * T))
                 + np.exp(-((X - 0.7) ** 2 + (Y - 0.3) ** 2) / (2 * T)))
    r = np.sqrt((X - 0.6) ** 2 + (Y - 0.4) ** 2)
    f2 = ((r >= 3.0 / 20.0) & (r <= 0.25)).astype(np.float64)
    f3 = ((X >= 0.5) & (X <= 0.75) & (Y >= 0.5) & (Y <= 0.75)).astype(np.float64)
    return {"f1": f1, "f2": f2, "f3": f3}


def gaussian_mixture_params(rng: np.random.Generator, d: int = 2):
    """Draw K ~ U{1..4} Gaussians, each with centre ~ U[0.2,0.8]^d then width ~ U[0.03,0.15]
    (drawn in that order), amplitude 1."""
    K = int(rng.integers(1, 5))
    out = []
    for _ in range(K):
        c = rng.uniform(0.2, 0.8, d)
        w = float(rng.uniform(0.03, 0.15))
        out.append((c, w))
    return out


def gaussian_mixture_source(n: int, params, d: int = 2) -> np.ndarray:
    """Sum of the Gaussians described by ``params`` at the cell centres."""
    f = np.zeros((n,) * d)
    for c, w in params:
        f += gaussian(n, c, w, d)
    return f


def hg_sigma_hat(g: float, L: int) -> np.ndarray:
    """Fourier coefficients sigma_hat_k, k = 0..L, of the 2D Henyey-Greenstein phase function
    (1-g^2)/(1+g^2-2g cos t) under the average-integral normalisation: g^k."""
    return np.array([g ** k for k in range(L + 1)], dtype=np.float64)


def paper_sigma_hat() -> np.ndarray:
    """sigma(t) = 1 + (1/5)e^{it} + (1/5)e^{-it} of the anisotropic experiments (eq. sigma)."""
    return np.array([1.0, 0.2], dtype=np.float64)


def random_modes(rng: np.random.Generator, L: int, n: int) -> np.ndarray:
    """A general complex vector of 2L+1 modes, shape (2L+1, n, n)."""
    M = 2 * L + 1
    return rng.standard_normal((M, n, n)) + 1j * rng.standard_normal((M, n, n))


def random_conj_symmetric_modes(rng: np.random.Generator, L: int, n: int) -> np.ndarray:
    """Modes of a real angular function: u_{-k} = conj(u_k), u_0 real."""
    M = 2 * L + 1
    u = np.zeros((M, n, n), dtype=np.complex128)
    u[L] = rng.standard_normal((n, n))
    for k in range(1, L + 1):
        z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        u[L + k] = z
        u[L - k] = np.conj(z)
    return u


def batched_problems(count: int = 128, seed: int = 3, sizes=(64, 128, 256, 512)):
    """The heterogeneous batch: for each problem draw n ~ choice(sizes), mu_s ~ U[0.5,20],
    mu_a ~ U[0.01,0.5], then a Gaussian-mixture source, all from one generator."""
    rng = np.random.default_rng(seed)
    probs = []
    for _ in range(count):
        n = int(rng.choice(np.asarray(sizes)))
        mu_s = float(rng.uniform(0.5, 20.0))
        mu_a = float(rng.uniform(0.01, 0.5))
        params = gaussian_mixture_params(rng, 2)
        probs.append({"n": n, "mu_s": mu_s, "mu_a": mu_a, "params": params})
    return probs


def workload(name: str, seed: int = 0, mu_s: float | None = None, n: int | None = None):
    """Named workloads (grid, coefficients, source).  Returns a dict with keys
    dim, n, L, mu_a, mu_s, sigma_hat, f (float64 array at cell centres)."""
    rng = np.random.default_rng(seed)
    if name == "iso32":            # 2D isotropic, 32^2, single centred Gaussian
        nn = n or 32
        return dict(dim=2, n=nn, L=0, mu_a=0.1, mu_s=1.0 if mu_s is None else mu_s,
                    sigma_hat=np.array([1.0]), f=centred_gaussian_source(nn))
    if name == "hg512":            # 2D HG g=0.5, L=8, 512^2
        nn = n or 512
        p = gaussian_mixture_params(rng, 2)
        return dict(dim=2, n=nn, L=8, mu_a=0.1, mu_s=1.0 if mu_s is None else mu_s,
                    sigma_hat=hg_sigma_hat(0.5, 8), f=gaussian_mixture_source(nn, p))
    if name == "iso3d":            # 3D isotropic, 128^3
        nn = n or 128
        p = gaussian_mixture_params(rng, 3)
        return dict(dim=3, n=nn, L=0, mu_a=0.05, mu_s=1.0 if mu_s is None else mu_s,
                    sigma_hat=np.array([1.0]), f=gaussian_mixture_source(nn, p, 3))
    if name == "diff256":          # diffusion regime, HG g=0.3, L=4, 256^2
        nn = n or 256
        p = gaussian_mixture_params(rng, 2)
        return dict(dim=2, n=nn, L=4, mu_a=0.01, mu_s=50.0 if mu_s is None else mu_s,
                    sigma_hat=hg_sigma_hat(0.3, 4), f=gaussian_mixture_source(nn, p))
    if name == "sh3d":             # 3D anisotropic, HG g=0.5, spherical harmonics to degree 2, 64^3
        nn = n or 64
        p = gaussian_mixture_params(rng, 3)
        return dict(dim=3, n=nn, L=2, mu_a=0.05, mu_s=10.0 if mu_s is None else mu_s,
                    sigma_hat=hg_sigma_hat(0.5, 2), f=gaussian_mixture_source(nn, p, 3))
    if name == "modes":            # 2D, strongly forward-peaked HG g=0.9, L=16 (33 modes), 256^2
        nn = n or 256
        p = gaussian_mixture_params(rng, 2)
        return dict(dim=2, n=nn, L=16, mu_a=0.05, mu_s=10.0 if mu_s is None else mu_s,
                    sigma_hat=hg_sigma_hat(0.9, 16), f=gaussian_mixture_source(nn, p))
    if name == "multi":            # one 256^2 medium (HG g=0.5, L=4) for many sources
        nn = n or 256
        p = gaussian_mixture_params(rng, 2)
        return dict(dim=2, n=nn, L=4, mu_a=0.1, mu_s=10.0 if mu_s is None else mu_s,
                    sigma_hat=hg_sigma_hat(0.5, 4), f=gaussian_mixture_source(nn, p))
    raise KeyError(name)
