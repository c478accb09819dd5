"""Linear solvers for the oracle (TEST INFRASTRUCTURE ONLY: see oracle/__init__.py).

The paper solves step T.2 / S.2 with GMRES (and MINRES for the symmetric isotropic form) to a
relative-residual tolerance eps (Sec. 2.4, 3.4).  Reading of the unstated details: start from
x0 = 0, no restart, residual measured as ||b - A x||_2 / ||b||_2 over all entries.  The oracle's
GMRES orthogonalises by classical Gram-Schmidt repeated twice and solves the small least-squares
problem by Givens rotations.  For grids beyond a dense matrix it is the full-size reference, as
the paper's own references for large n are FFT-method solves at a very small tolerance
(Sec. 2.4.1, Sec. 3.4.1).  Dense LU and the Neumann series are independent cross-checks.
"""
from __future__ import annotations

import numpy as np


def solve_dense(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Direct method (Sec. 2.3): LU factorisation of the dense matrix."""
    return np.linalg.solve(A, b)


def gmres(matvec, b: np.ndarray, tol: float = 1e-13, maxiter: int = 200):
    """Unrestarted GMRES from x0 = 0.  Returns (x, history of estimated relative residuals).

    b may have any shape; matvec maps arrays of that shape to that shape.  Real b gives real
    arithmetic throughout, complex b complex arithmetic.  Each new Arnoldi vector is
    orthogonalised against the basis by classical Gram-Schmidt applied twice (the projection
    coefficients h = V^H w are formed as matrix-vector products with the stored basis, then
    w <- w - V h; the two passes' coefficients add up to the Hessenberg column), which is as
    orthogonal as modified Gram-Schmidt twice and lets the basis products run as library
    matrix-vector products on large vectors."""
    shape = b.shape
    dtype = np.complex128 if np.iscomplexobj(b) else np.float64
    bf = np.ascontiguousarray(b.reshape(-1), dtype=dtype)
    beta = np.linalg.norm(bf)
    if beta == 0.0:
        return np.zeros(shape, dtype=dtype), [0.0]
    # the basis is stored in blocks of rows, allocated as the iteration reaches them
    BLK = 16
    blocks = []

    def row(i):
        if i // BLK == len(blocks):
            blocks.append(np.empty((BLK, bf.size), dtype=dtype))
        return blocks[i // BLK][i % BLK]

    def rows(n):     # the first n basis vectors, block by block
        for q in range((n + BLK - 1) // BLK):
            yield blocks[q][:min(BLK, n - q * BLK)]

    row(0)[:] = bf / beta
    H = np.zeros((maxiter + 1, maxiter), dtype=dtype)
    cs = np.zeros(maxiter, dtype=dtype)
    sn = np.zeros(maxiter, dtype=dtype)
    g = np.zeros(maxiter + 1, dtype=dtype)
    g[0] = beta
    hist = [1.0]
    j_end = 0
    for j in range(maxiter):
        w = np.array(matvec(row(j).reshape(shape)), dtype=dtype).reshape(-1)
        for _ in range(2):                      # classical Gram-Schmidt, twice
            wc = np.conj(w)
            hc = np.concatenate([np.conj(Vb @ wc) for Vb in rows(j + 1)])   # h_i = <V_i, w>
            H[:j + 1, j] += hc
            for q, Vb in enumerate(rows(j + 1)):
                w -= hc[q * BLK:q * BLK + Vb.shape[0]] @ Vb
        H[j + 1, j] = np.linalg.norm(w)
        # previous rotations
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
            H[i, j] = t
        # new rotation zeroing H[j+1, j]
        a, c = H[j, j], H[j + 1, j]
        den = np.sqrt(abs(a) ** 2 + abs(c) ** 2)
        if den == 0.0:
            cs[j], sn[j] = 1.0, 0.0
        else:
            cs[j] = np.conj(a) / den if a != 0 else 0.0
            sn[j] = np.conj(c) / den
            if a == 0:
                cs[j], sn[j] = 0.0, 1.0
        H[j, j] = cs[j] * a + sn[j] * c
        H[j + 1, j] = 0.0
        g[j + 1] = -np.conj(sn[j]) * g[j]
        g[j] = cs[j] * g[j]
        rel = abs(g[j + 1]) / beta
        hist.append(float(rel))
        j_end = j + 1
        hnext = np.linalg.norm(w)
        if rel <= tol or hnext == 0.0 or j + 1 == maxiter:
            break
        row(j + 1)[:] = w / hnext
    y = np.linalg.solve(np.triu(H[:j_end, :j_end]), g[:j_end])
    x = np.zeros(bf.size, dtype=dtype)
    for q, Vb in enumerate(rows(j_end)):
        x += y[q * BLK:q * BLK + Vb.shape[0]] @ Vb
    return x.reshape(shape), hist


def neumann(apply_KD, b: np.ndarray, tol: float = 1e-13, maxiter: int = 10000):
    """u = sum_j (K~ D)^j b: the fixed-point iteration u <- b + K~ D u behind the contraction
    argument of Lemma 1 / Lemma 3.  Converges geometrically at rate ||K~ D|| < 1."""
    u = b.copy()
    term = b.copy()
    nb = np.linalg.norm(b)
    for _ in range(maxiter):
        term = apply_KD(term)
        u = u + term
        if np.linalg.norm(term) <= tol * nb:
            break
    return u
