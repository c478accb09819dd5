"""GPU parity of the 3D anisotropic path (real spherical harmonics to degree L = 1..3) against the
CPU oracle, through the C ABI: the apply on ragged small grids against the dense matrix, sampled
rows of the apply at 128^3 against the direct sum, the right-hand side, solves against dense LU,
mid-size solves against the oracle's FP64 reference solve, a 128^3 solve checked by the oracle's
FFT apply, and the size limits.  Bars: FP64 path 1e-12 (apply) / 1e-10 (solve), FP32 path 1e-6."""
import numpy as np
import pytest
import torch

import oracle_ref
from gpu_util import dev, host, relerr, say
from oracle import krylov as kr
from oracle import operator3d_sh as o3s
from paper_1802_03061_amd import inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-6


@pytest.fixture(scope="module")
def rte():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1802_03061_amd import rte as r
    r.load()
    return r


def _ctx(rte, shape_xyz, L, h, mu_a, mu_s, g, prec):
    sh = inputs.hg_sigma_hat(g, L)
    if isinstance(shape_xyz, int):
        shape_xyz = (shape_xyz,) * 3
    return rte.Context(shape_xyz, h=h, mu_a=mu_a, mu_s=mu_s, sigma_hat=sh, L=L, prec=prec), sh


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("L,nz,ny,nx", [(1, 3, 4, 5), (2, 5, 3, 4), (3, 4, 4, 4), (2, 2, 2, 2), (1, 7, 6, 9),
                                         (3, 2, 3, 2)])
def test_apply_small_vs_dense(rte, prec, L, nz, ny, nx):
    """Random complex modes (the real operator acts on both parts) and random channels, operators
    A and K~, against the oracle's dense matrix."""
    say("sh3d apply small", L, nz, ny, nx, "prec", prec)
    rng = np.random.default_rng(10 * L + nz + ny)
    h, mu_a, mu_s = 1.0 / max(nx, ny, nz), 0.1, 2.0
    ctx, sh = _ctx(rte, (nx, ny, nz), L, h, mu_a, mu_s, 0.6, prec)
    M = (L + 1) ** 2
    assert ctx.modes == M and ctx.channels == M
    u = rng.standard_normal((M, nz, ny, nx)) + 1j * rng.standard_normal((M, nz, ny, nx))
    for op, name in ((rte.OP_A, "A"), (rte.OP_KT, "KT")):
        y = host(ctx.apply(dev(u), op=op))
        ref = (o3s.apply_direct(u.real, L, h, mu_a + mu_s, mu_s, sh, name)
               + 1j * o3s.apply_direct(u.imag, L, h, mu_a + mu_s, mu_s, sh, name))
        e = relerr(y, ref)
        say("  op", name, "modes relerr", e)
        assert e <= (TOL64 if prec == 1 else TOL32)
        yc = host(ctx.apply(dev(u.real), op=op, layout=rte.LAYOUT_CHANNELS))
        e = relerr(yc, ref.real)
        say("  op", name, "channels relerr", e)
        assert e <= (TOL64 if prec == 1 else TOL32)
    ctx.close()


@pytest.mark.parametrize("L", [1, 2, 3])
def test_rhs_vs_oracle(rte, L):
    n = 6
    h, mu_a, mu_s = 1.0 / n, 0.2, 1.5
    ctx, sh = _ctx(rte, (n, n, n), L, h, mu_a, mu_s, 0.5, 1)
    f = inputs.gaussian_mixture_source(n, inputs.gaussian_mixture_params(np.random.default_rng(L), 3), 3)
    b = host(ctx.rhs(dev(f)))
    ref = o3s.rhs(f, L, h, mu_a + mu_s, method="direct")
    e = relerr(b, ref)
    say("sh3d rhs L", L, "relerr", e)
    assert e <= TOL64
    ctx.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("L,prec", [(2, 0), (2, 1), (3, 0)])
def test_apply_128_sampled_vs_direct_sum(rte, L, prec):
    """128^3 (256^3 padded), sampled output cells (corners, faces, interior) against the oracle's
    direct sum over every cell and mode."""
    say("sh3d apply 128 sampled L", L, "prec", prec)
    n = 128
    h, mu_a, mu_s = 1.0 / n, 0.05, 5.0
    ctx, sh = _ctx(rte, n, L, h, mu_a, mu_s, 0.5, prec)
    M = (L + 1) ** 2
    rng = np.random.default_rng(5 + L)
    u = rng.standard_normal((M, n, n, n))
    y = host(ctx.apply(dev(u), layout=rte.LAYOUT_CHANNELS))
    cells = [(0, 0, 0), (127, 127, 127), (0, 64, 127), (64, 64, 64), (31, 100, 7), (127, 0, 55)]
    ref = o3s.apply_sampled(u, cells, L, h, mu_a + mu_s, mu_s, sh)
    got = np.array([y[:, iz, iy, ix] for iz, iy, ix in cells])
    # relative to the size of the sampled outputs
    e = float(np.abs(got - ref).max() / np.abs(ref).max())
    say("  sampled max relerr", e)
    assert e <= (1e-11 if prec == 1 else 2e-6)
    ctx.close()


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("L,n,mu_s", [(1, 6, 3.0), (2, 5, 8.0), (3, 4, 2.0)])
def test_solve_small_vs_lu(rte, prec, L, n, mu_s):
    say("sh3d solve small", L, n, mu_s, "prec", prec)
    h, mu_a = 1.0 / n, 0.1
    ctx, sh = _ctx(rte, n, L, h, mu_a, mu_s, 0.5, prec)
    f = np.random.default_rng(n + L).random((n, n, n))
    u, info = ctx.solve(dev(f), tol=1e-11)
    say("  info", info)
    A = o3s.dense_A(n, n, n, L, h, mu_a + mu_s, mu_s, sh)
    b = o3s.rhs(f, L, h, mu_a + mu_s, method="direct")
    ref = kr.solve_dense(A, b.reshape(-1)).reshape(b.shape)
    uu = host(u)
    assert np.abs(uu.imag).max() == 0.0
    e = relerr(uu.real, ref)
    say("  relerr vs LU", e)
    assert e <= (1e-10 if prec == 1 else 1e-6)
    ctx.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,tol,bar", [(0, 1e-8, 1e-6), (1, 1e-12, 1e-10)])
@pytest.mark.parametrize("L,n", [(2, 48), (3, 32)])
def test_solve_mid_vs_oracle_reference(rte, L, n, prec, tol, bar):
    """HG g = 0.5, mu_a = 0.05, mu_s = 10, Gaussian-mixture source: the GPU solution against the
    oracle's FP64 GMRES over its FFT apply (1e-13), element by element over all modes."""
    say("sh3d solve mid L", L, "n", n, "prec", prec)
    h, mu_a, mu_s = 1.0 / n, 0.05, 10.0
    ctx, sh = _ctx(rte, n, L, h, mu_a, mu_s, 0.5, prec)
    f = inputs.gaussian_mixture_source(n, inputs.gaussian_mixture_params(np.random.default_rng(0), 3), 3)
    u, info = ctx.solve(dev(f), tol=tol)
    say("  info", info)
    ref = _ref_mid(L, n)
    say(f"  oracle reference {ref['iterations']} iterations, {ref['seconds']:.1f} s")
    e = relerr(host(u).real, ref["u"])
    say("  relerr vs oracle", e)
    assert e <= bar
    ctx.close()


_REFS = {}


def _ref_mid(L, n):
    if (L, n) not in _REFS:
        import time
        h, mu_a, mu_s = 1.0 / n, 0.05, 10.0
        sh = inputs.hg_sigma_hat(0.5, L)
        f = inputs.gaussian_mixture_source(n, inputs.gaussian_mixture_params(np.random.default_rng(0), 3), 3)
        t0 = time.perf_counter()
        sp = o3s.kernel_spectra(n, n, n, L, h, mu_a + mu_s, workers=oracle_ref.WORKERS)
        b = o3s.rhs(f, L, h, mu_a + mu_s, spectra=sp, workers=oracle_ref.WORKERS)
        x, hist = kr.gmres(lambda v: o3s.apply_fft(v, L, h, mu_a + mu_s, mu_s, sh, spectra=sp,
                                                   workers=oracle_ref.WORKERS), b, 1e-13, 400)
        _REFS.clear()
        _REFS[(L, n)] = {"u": x, "iterations": len(hist) - 1, "seconds": time.perf_counter() - t0}
    return _REFS[(L, n)]


@pytest.mark.timeout(900)
def test_solve_128_full_size_residual(rte):
    """128^3, L = 2 (9 modes), HG g = 0.5, mu_a = 0.05, mu_s = 10: FP32 apply with FP64 Krylov to
    1e-8; the oracle's FP64 FFT apply confirms the true residual of the GPU solution, and the
    density is positive."""
    say("sh3d solve 128 L2")
    n, L = 128, 2
    h, mu_a, mu_s = 1.0 / n, 0.05, 10.0
    ctx, sh = _ctx(rte, n, L, h, mu_a, mu_s, 0.5, 0)
    f = inputs.gaussian_mixture_source(n, inputs.gaussian_mixture_params(np.random.default_rng(0), 3), 3)
    u, info = ctx.solve(dev(f), tol=1e-8)
    say("  info", info)
    uu = host(u).real
    ctx.close()
    sp = o3s.kernel_spectra(n, n, n, L, h, mu_a + mu_s, workers=oracle_ref.WORKERS)
    b = o3s.rhs(f, L, h, mu_a + mu_s, spectra=sp, workers=oracle_ref.WORKERS)
    r = b - o3s.apply_fft(uu, L, h, mu_a + mu_s, mu_s, sh, spectra=sp, workers=oracle_ref.WORKERS)
    rr = float(np.linalg.norm(r) / np.linalg.norm(b))
    say("  oracle true residual", rr)
    assert rr <= 1.5e-8
    assert uu[0].min() >= -1e-7 * np.abs(uu[0]).max()


def test_limits(rte):
    """3D keeps degrees up to 3, and grids up to 128 per side when L > 0."""
    with pytest.raises(rte.RteError) as ei:
        rte.Context(8, dim=3, mu_a=0.1, mu_s=1.0, L=4, sigma_hat=[1, .5, .25, .125, .0625])
    assert ei.value.code == rte.RTE_EUNSUPPORTED
    with pytest.raises(rte.RteError) as ei:
        rte.Context(129, dim=3, mu_a=0.1, mu_s=1.0, L=1, sigma_hat=[1, .5])
    assert ei.value.code == rte.RTE_EUNSUPPORTED
    c = rte.Context(8, dim=3, mu_a=0.1, mu_s=1.0, L=3, sigma_hat=[1, .5, .25, .125])
    assert c.modes == 16 and c.channels == 16
    c.close()
