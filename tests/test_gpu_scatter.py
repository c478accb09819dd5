"""GPU parity of the scattering term at discrete angles (rte_scattering_term) against the
oracle's sum S(x, theta_q) = Re(mu_s sum_k sigma_hat_|k| u_k e^{i k theta_q}) (eq.
ani_2d_scattering), through the C ABI.  Both sides are FP64; the bar is 1e-13 relative (the only
differences are the summation order and the angle evaluation)."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_util import dev, host, relerr, say
from oracle.scattering import scattering_term
from paper_1802_03061_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-13


@pytest.fixture(scope="module")
def rte():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1802_03061_amd import rte as r
    r.load()
    return r


def _to_ch(u, L):
    out = [u[L].real]
    for k in range(1, L + 1):
        out += [np.sqrt(2) * u[L + k].real, np.sqrt(2) * u[L + k].imag]
    return np.stack(out)


@pytest.mark.parametrize("L,ny,nx,ntheta", [(0, 9, 7, 5), (2, 12, 10, 1), (3, 16, 16, 64), (8, 11, 13, 100),
                                            (4, 5, 21, 130), (1, 3, 300, 7), (5, 4, 6, 9), (6, 2, 2, 3),
                                            (7, 7, 3, 64), (12, 6, 5, 17), (32, 4, 3, 65)])
def test_scattering_term_small_vs_oracle(rte, L, ny, nx, ntheta):
    say("scattering", L, ny, nx, ntheta)
    rng = np.random.default_rng(L * 31 + ny)
    sh = inputs.hg_sigma_hat(0.6, L)
    mu_s = 4.0
    ctx = rte.Context((nx, ny), h=1.0 / max(nx, ny), mu_a=0.2, mu_s=mu_s, sigma_hat=sh, L=L, prec=rte.PREC_FP64)
    # modes layout: any complex vector (the real part of the sum is written)
    u = rng.standard_normal((2 * L + 1, ny, nx)) + 1j * rng.standard_normal((2 * L + 1, ny, nx))
    got = host(ctx.scattering_term(dev(u), ntheta))
    ref = scattering_term(u, L, mu_s, sh, ntheta)
    e = relerr(got, ref)
    say("  modes relerr", e)
    assert got.shape == (ntheta, ny, nx) and e <= TOL
    # channel layout: the image of a real flux
    uc = inputs.random_conj_symmetric_modes(rng, L, max(nx, ny))[:, :ny, :nx].copy()
    got = host(ctx.scattering_term(dev(_to_ch(uc, L)), ntheta, layout=rte.LAYOUT_CHANNELS))
    ref = scattering_term(uc, L, mu_s, sh, ntheta)
    e = relerr(got, ref)
    say("  channels relerr", e)
    assert e <= TOL
    ctx.close()


def test_scattering_term_of_a_solution_full_size(rte):
    """512^2, L = 8, 64 angles, of the solved flux of the 512^2 HG workload: sampled cells against
    the oracle's sum, and the angular mean equals mu_s times the mean local density."""
    w = inputs.workload("hg512", seed=1, mu_s=10.0)
    n, L = w["n"], w["L"]
    ctx = rte.Context(n, mu_a=w["mu_a"], mu_s=w["mu_s"], sigma_hat=w["sigma_hat"], L=L, prec=rte.PREC_FP32)
    u, info = ctx.solve(dev(w["f"]), tol=1e-8)
    say("  solve", info)
    S = ctx.scattering_term(u, 64)
    uh, Sh = host(u), host(S)
    rng = np.random.default_rng(2)
    cells = [(0, 0), (511, 511), (256, 3)] + [tuple(rng.integers(0, n, 2)) for _ in range(20)]
    iy = np.array([c[0] for c in cells]); ix = np.array([c[1] for c in cells])
    ref = scattering_term(uh[:, iy, ix], L, w["mu_s"], w["sigma_hat"], 64)
    e = relerr(Sh[:, iy, ix], ref)
    say("  sampled relerr", e)
    assert e <= TOL
    mean = Sh.mean(axis=0)
    assert relerr(mean, w["mu_s"] * uh[L].real) <= 1e-12
    ctx.close()


def test_scattering_term_errors(rte):
    lib = rte.load()
    ctx = rte.Context(8, mu_a=0.1, mu_s=1.0, L=1, sigma_hat=[1.0, 0.5], prec=rte.PREC_FP64)
    u = torch.zeros(ctx.mode_shape, dtype=torch.complex128, device="cuda")
    S = torch.zeros((4,) + tuple(ctx.channel_shape[1:]), dtype=torch.float64, device="cuda")
    up, sp = C.c_void_p(u.data_ptr()), C.c_void_p(S.data_ptr())
    assert lib.rte_scattering_term(ctx._h, 0, up, 0, sp) == rte.RTE_EINVAL
    assert lib.rte_scattering_term(ctx._h, 7, up, 4, sp) == rte.RTE_EINVAL
    assert lib.rte_scattering_term(ctx._h, 0, None, 4, sp) == rte.RTE_EINVAL
    ctx.close()
    c3 = rte.Context(8, dim=3, mu_a=0.1, mu_s=1.0, L=0, prec=rte.PREC_FP64)
    assert lib.rte_scattering_term(c3._h, 0, up, 4, sp) == rte.RTE_EUNSUPPORTED
    c3.close()
