"""The mu_s = 0 solution for the source f = 1 on the unit square / cube
(TEST INFRASTRUCTURE ONLY: see oracle/__init__.py).

With no scattering the Fredholm equation reduces to u = K~ g (eq. ani_2d_Fredholm with K = 0),
and K~ g is the angular average of the characteristic solution T^{-1} J f (eq. def_cTinv):
    Phi(x, v) = int_0^{tau(x,v)} exp(-mu_t s) f(x - s v) ds = (1 - exp(-mu_t tau))/mu_t  (f = 1),
with tau(x, v) the distance from x to the boundary travelling along -v (eq. def_tau).  Hence
    2D: u_k(x) = (1/2pi) int_0^{2pi} exp(-i k theta) (1 - exp(-mu_t tau(x,theta)))/mu_t dtheta
        (the Fourier convention of eq. ani_Fouriermode),
    3D: u(x)   = (1/4pi) int_{S^2} (1 - exp(-mu_t tau(x,w)))/mu_t dw.
The Nystrom solution converges to these at the cell centres as h -> 0.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate


def _phi(mu_t: float, tau: float) -> float:
    return tau if mu_t == 0.0 else -np.expm1(-mu_t * tau) / mu_t


def tau_2d(x: float, y: float, theta: float) -> float:
    """Distance from (x, y) in [0,1]^2 to the boundary along -(cos theta, sin theta)."""
    c, s = np.cos(theta), np.sin(theta)
    t = np.inf
    if c > 0:
        t = min(t, x / c)
    elif c < 0:
        t = min(t, (1.0 - x) / (-c))
    if s > 0:
        t = min(t, y / s)
    elif s < 0:
        t = min(t, (1.0 - y) / (-s))
    return t


def mus0_mode_2d(x: float, y: float, k: int, mu_t: float) -> complex:
    """u_k(x, y) for mu_s = 0 and f = 1 on [0,1]^2."""
    corners = [(0.0, 0.0), (1.0, 0.0), (1.0, 1.0), (0.0, 1.0)]
    pts = sorted(np.mod(np.arctan2(y - cy, x - cx), 2 * np.pi) for cx, cy in corners)
    re = integrate.quad(lambda t: np.cos(k * t) * _phi(mu_t, tau_2d(x, y, t)), 0.0, 2 * np.pi,
                        points=pts, limit=400, epsabs=1e-13, epsrel=1e-12)[0]
    im = integrate.quad(lambda t: -np.sin(k * t) * _phi(mu_t, tau_2d(x, y, t)), 0.0, 2 * np.pi,
                        points=pts, limit=400, epsabs=1e-13, epsrel=1e-12)[0]
    return (re + 1j * im) / (2 * np.pi)


def mus0_density_3d(p, mu_t: float) -> float:
    """u(x) for mu_s = 0 and f = 1 on [0,1]^3.

    The sphere of directions is split by the six faces of the cube; the directions through a face
    at perpendicular distance d have tau = rho = |y - x| and solid angle d/rho^3 dA(y), so
        u = (1/4pi) sum_faces int_face (1 - exp(-mu_t rho))/mu_t * d / rho^3 dA.
    Each face is split at the foot of the perpendicular so the adaptive rule sees a smooth peak
    in a corner."""
    p = np.asarray(p, dtype=np.float64)
    total = 0.0
    for axis in range(3):
        others = [a for a in range(3) if a != axis]
        for wall in (0.0, 1.0):
            d = abs(p[axis] - wall)
            u0, v0 = p[others[0]], p[others[1]]

            def f(v, u, d=d, u0=u0, v0=v0):
                rho = np.sqrt((u - u0) ** 2 + (v - v0) ** 2 + d * d)
                return _phi(mu_t, rho) * d / rho ** 3

            for (ua, ub) in ((0.0, u0), (u0, 1.0)):
                for (va, vb) in ((0.0, v0), (v0, 1.0)):
                    if ub > ua and vb > va:
                        total += integrate.dblquad(f, ua, ub, va, vb,
                                                   epsabs=1e-12, epsrel=1e-11)[0]
    return total / (4 * np.pi)


def mus0_moment_3d(p, a: int, L: int, mu_t: float) -> float:
    """Mode a of the real spherical-harmonic expansion (oracle.sh3d) of the mu_s = 0, f = 1 flux on
    [0,1]^3: u_a(x) = (1/4pi) int_{S^2} Y~_a(w) (1 - exp(-mu_t tau(x,w)))/mu_t dw.  The flux at x
    travelling along w comes from the boundary point y = x - tau w, so w = (x - y)/|x - y|; the same
    face decomposition as mus0_density_3d, with Y~_a(w) in the integrand."""
    from .sh3d import real_sh
    p = np.asarray(p, dtype=np.float64)
    total = 0.0
    for axis in range(3):
        others = [q for q in range(3) if q != axis]
        for wall in (0.0, 1.0):
            d = abs(p[axis] - wall)
            u0, v0 = p[others[0]], p[others[1]]

            def f(v, u, d=d, u0=u0, v0=v0, axis=axis, wall=wall, others=others):
                y = np.empty(3)
                y[axis] = wall
                y[others[0]] = u
                y[others[1]] = v
                dv = p - y
                rho = np.sqrt(dv @ dv)
                return real_sh(L, dv / rho)[a] * _phi(mu_t, rho) * d / rho ** 3

            for (ua, ub) in ((0.0, u0), (u0, 1.0)):
                for (va, vb) in ((0.0, v0), (v0, 1.0)):
                    if ub > ua and vb > va:
                        total += integrate.dblquad(f, ua, ub, va, vb, epsabs=1e-12, epsrel=1e-10)[0]
    return total / (4 * np.pi)


def mus0_mode_2d_source(x: float, y: float, k: int, mu_t: float, g: dict) -> complex:
    """u_k(x, y) for mu_s = 0 and the spatially uniform anisotropic source
    f(theta) = sum_{k'} g[k'] exp(i k' theta) on [0,1]^2: the characteristic solution is
    f(theta) (1 - exp(-mu_t tau))/mu_t, so u_k = (1/2pi) int exp(-i k theta) f(theta) (...) dtheta."""
    corners = [(0.0, 0.0), (1.0, 0.0), (1.0, 1.0), (0.0, 1.0)]
    pts = sorted(np.mod(np.arctan2(y - cy, x - cx), 2 * np.pi) for cx, cy in corners)

    def integrand(t):
        ft = sum(gk * np.exp(1j * kp * t) for kp, gk in g.items())
        return np.exp(-1j * k * t) * ft * _phi(mu_t, tau_2d(x, y, t))

    re = integrate.quad(lambda t: integrand(t).real, 0.0, 2 * np.pi, points=pts, limit=400,
                        epsabs=1e-13, epsrel=1e-12)[0]
    im = integrate.quad(lambda t: integrand(t).imag, 0.0, 2 * np.pi, points=pts, limit=400,
                        epsabs=1e-13, epsrel=1e-12)[0]
    return (re + 1j * im) / (2 * np.pi)
