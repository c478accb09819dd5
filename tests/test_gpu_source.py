"""Anisotropic sources (rte_rhs_source / rte_solve_source) against the CPU oracle through the C ABI,
and the paper's own anisotropic workload (sigma(t) = 1 + (1/5) e^{it} + (1/5) e^{-it}, mu_a = 0.2,
mu_s = 1, the two-Gaussian source of its numerical section) on a small grid against dense LU."""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, relerr, say
from oracle import krylov as kr
from oracle import operator2d as op2
from oracle import operator3d_sh as o3s
from paper_1802_03061_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rte():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1802_03061_amd import rte as r
    r.load()
    return r


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("L,ny,nx", [(2, 12, 10), (4, 9, 16), (0, 8, 8)])
def test_rhs_source_2d_vs_oracle(rte, prec, L, ny, nx):
    """b = K~ g for conjugate-symmetric source modes, FP64 apply (prec selects only the context)."""
    say("rhs source 2d", L, ny, nx, "prec", prec)
    rng = np.random.default_rng(L + ny)
    h = 1.0 / max(nx, ny)
    ctx = rte.Context((nx, ny), h=h, mu_a=0.1, mu_s=2.0, sigma_hat=inputs.hg_sigma_hat(0.5, L), L=L, prec=prec)
    g = inputs.random_conj_symmetric_modes(rng, L, max(nx, ny))[:, :ny, :nx].copy()
    b = host(ctx.rhs_source(dev(g)))
    ref = op2.apply_direct(g, L, h, 2.1, 0.0, np.ones(L + 1), op="KT")
    e = relerr(b, ref)
    say("  relerr", e)
    assert e <= 1e-12
    gc = host(ctx.modes_to_channels(dev(g)))
    bc = host(ctx.rhs_source(dev(gc), layout=rte.LAYOUT_CHANNELS))
    assert relerr(host(ctx.channels_to_modes(dev(bc))), ref) <= 1e-12
    ctx.close()


@pytest.mark.parametrize("prec,bar", [(1, 1e-10), (0, 1e-6)])
@pytest.mark.parametrize("L,n", [(1, 16), (3, 10)])
def test_solve_source_2d_vs_lu(rte, prec, bar, L, n):
    """A u = K~ g for a smooth anisotropic source (a Gaussian beam with a preferred direction)."""
    say("solve source 2d", L, n, "prec", prec)
    h, mu_a, mu_s = 1.0 / n, 0.1, 4.0
    sh = inputs.hg_sigma_hat(0.5, L)
    g = np.zeros((2 * L + 1, n, n), dtype=complex)
    blob = inputs.gaussian(n, (0.4, 0.55), 0.15)
    g[L] = blob
    for k in range(1, L + 1):                       # f(x, theta) = blob(x) (1 + sum_k 0.6^k 2 cos k(theta - 0.7))
        g[L + k] = blob * 0.6 ** k * np.exp(-1j * k * 0.7)
        g[L - k] = np.conj(g[L + k])
    ctx = rte.Context(n, mu_a=mu_a, mu_s=mu_s, sigma_hat=sh, L=L, prec=prec)
    u, info = ctx.solve_source(dev(g), tol=1e-11)
    say("  info", info)
    A = op2.dense_A(n, n, L, h, mu_a + mu_s, mu_s, sh)
    b = op2.apply_direct(g, L, h, mu_a + mu_s, 0.0, np.ones(L + 1), op="KT")
    ref = kr.solve_dense(A, b.reshape(-1)).reshape(b.shape)
    e = relerr(host(u), ref)
    say("  relerr vs LU", e)
    assert e <= bar
    ctx.close()


@pytest.mark.parametrize("prec,bar", [(1, 1e-10), (0, 1e-6)])
def test_solve_source_3d_vs_lu(rte, prec, bar):
    """3D, L = 1: a source with a first moment along x (channels layout)."""
    n, L = 5, 1
    h, mu_a, mu_s = 1.0 / n, 0.1, 3.0
    sh = inputs.hg_sigma_hat(0.5, L)
    blob = inputs.centred_gaussian_source(n, 0.15, d=3)
    g = np.zeros((4, n, n, n))
    g[0] = blob
    g[3] = 0.5 * blob
    ctx = rte.Context((n, n, n), h=h, mu_a=mu_a, mu_s=mu_s, sigma_hat=sh, L=L, prec=prec)
    u, info = ctx.solve_source(dev(g), tol=1e-11, layout=rte.LAYOUT_CHANNELS)
    say("solve source 3d prec", prec, info)
    A = o3s.dense_A(n, n, n, L, h, mu_a + mu_s, mu_s, sh)
    b = o3s.apply_direct(g, L, h, mu_a + mu_s, 0.0, np.ones(L + 1), op="KT")
    ref = kr.solve_dense(A, b.reshape(-1)).reshape(b.shape)
    e = relerr(host(u), ref)
    say("  relerr vs LU", e)
    assert e <= bar
    ctx.close()


@pytest.mark.parametrize("prec,bar", [(1, 1e-10), (0, 1e-6)])
def test_paper_anisotropic_workload_vs_lu(rte, prec, bar):
    """The paper's homogeneous anisotropic experiment (Sec. 3.4.1): three modes,
    sigma_hat = (1, 1/5), mu_a = 0.2, mu_s = 1, source f1, here on a 32^2 grid, GMRES to 1e-10."""
    n = 32
    f = inputs.paper_sources(n)["f1"]
    sh = inputs.paper_sigma_hat()
    L = len(sh) - 1
    h, mu_a, mu_s = 1.0 / n, 0.2, 1.0
    ctx = rte.Context(n, mu_a=mu_a, mu_s=mu_s, sigma_hat=sh, L=L, prec=prec)
    u, info = ctx.solve(dev(f), tol=1e-10)
    say("paper workload prec", prec, info)
    A = op2.dense_A(n, n, L, h, mu_a + mu_s, mu_s, sh)
    b = op2.rhs(f, L, h, mu_a + mu_s, method="direct")
    ref = kr.solve_dense(A, b.reshape(-1)).reshape(b.shape)
    e = relerr(host(u), ref)
    say("  relerr vs LU", e)
    assert e <= bar
    ctx.close()


def test_source_bad_arguments(rte):
    ctx = rte.Context(8, mu_a=0.1, mu_s=1.0, L=1, sigma_hat=[1, 0.5], prec=1)
    g = torch.zeros((3, 8, 8), dtype=torch.complex128, device="cuda")
    lib = rte.load()
    import ctypes
    p = ctypes.c_void_p(g.data_ptr())
    assert lib.rte_rhs_source(ctx._h, p, 0, p) == rte.RTE_EINVAL          # aliasing
    assert lib.rte_rhs_source(ctx._h, p, 7, ctypes.c_void_p(g.data_ptr() + 16)) == rte.RTE_EINVAL
    with pytest.raises(rte.RteError) as ei:
        ctx.solve_source(g, tol=0.0)
    assert ei.value.code == rte.RTE_EINVAL
    u, info = ctx.solve_source(g, tol=1e-8)                              # zero source: zero solution
    assert info["status"] == rte.RTE_OK and float(u.abs().max()) == 0.0
    ctx.close()
