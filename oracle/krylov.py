"""Linear solvers for the oracle (TEST INFRASTRUCTURE ONLY: see oracle/__init__.py).

The paper solves step T.2 / S.2 with GMRES (and MINRES for the symmetric isotropic form) to a
relative-residual tolerance eps (Sec. 2.4, 3.4).  Reading of the unstated details: start from
x0 = 0, no restart, residual measured as ||b - A x||_2 / ||b||_2 over all entries.  The oracle's
GMRES orthogonalises by modified Gram-Schmidt repeated twice and solves the small least-squares
problem by Givens rotations.  Dense LU and the Neumann series are independent cross-checks.
"""
from __future__ import annotations

import numpy as np


def solve_dense(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Direct method (Sec. 2.3): LU factorisation of the dense matrix."""
    return np.linalg.solve(A, b)


def gmres(matvec, b: np.ndarray, tol: float = 1e-13, maxiter: int = 200):
    """Unrestarted GMRES from x0 = 0.  Returns (x, history of estimated relative residuals).

    b may have any shape; matvec maps arrays of that shape to that shape."""
    shape = b.shape
    bf = b.reshape(-1).astype(np.complex128)
    beta = np.linalg.norm(bf)
    if beta == 0.0:
        return np.zeros_like(b, dtype=np.complex128), [0.0]
    V = [bf / beta]
    H = np.zeros((maxiter + 1, maxiter), dtype=np.complex128)
    cs = np.zeros(maxiter, dtype=np.complex128)
    sn = np.zeros(maxiter, dtype=np.complex128)
    g = np.zeros(maxiter + 1, dtype=np.complex128)
    g[0] = beta
    hist = [1.0]
    j_end = 0
    for j in range(maxiter):
        w = matvec(V[j].reshape(shape)).reshape(-1).astype(np.complex128)
        for _ in range(2):                      # MGS, twice
            for i in range(j + 1):
                hij = np.vdot(V[i], w)
                H[i, j] += hij
                w = w - hij * V[i]
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
        if rel <= tol or hnext == 0.0:
            break
        V.append(w / hnext)
    y = np.linalg.solve(np.triu(H[:j_end, :j_end]), g[:j_end])
    x = sum(y[i] * V[i] for i in range(j_end))
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
