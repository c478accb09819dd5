"""GPU parity of the FFT apply and the right-hand side against the CPU oracle (through the C ABI).

Bars: FP64 path relative L2 error <= 1e-12 against the oracle; FP32 path <= 1e-6, the FP32 path's
parity target (an FP32 FFT of length P carries a relative error of order eps32 * log2(P); the
measured worst case over these cases is about 1.5e-7)."""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, relerr, say
from oracle import operator2d as op2
from oracle import operator3d as op3
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


def _ctx(rte, n, L, g=0.5, mu_a=0.1, mu_s=2.0, prec=1, h=None):
    sh = inputs.hg_sigma_hat(g, L)
    return rte.Context(n, h=h, mu_a=mu_a, mu_s=mu_s, sigma_hat=sh, L=L, prec=prec), sh


# the last five: every L the library compiles a pass B for is covered, down to the smallest grid
SMALL = [(0, 8, 8), (1, 12, 10), (2, 9, 13), (3, 16, 16), (8, 12, 16), (4, 5, 21),
         (0, 2, 2), (5, 3, 2), (6, 7, 9), (7, 2, 2), (7, 11, 6)]


@pytest.mark.parametrize("L,ny,nx", SMALL)
@pytest.mark.parametrize("prec", [1, 0])
def test_apply_modes_small_vs_direct_sum(rte, L, ny, nx, prec):
    say("apply small", L, ny, nx, "prec", prec)
    rng = np.random.default_rng(100 + L * 7 + ny)
    h = 1.0 / max(nx, ny)
    mu_a, mu_s = 0.1, 2.0
    ctx, sh = _ctx(rte, (nx, ny), L, mu_a=mu_a, mu_s=mu_s, prec=prec, h=h)
    u = rng.standard_normal((2 * L + 1, ny, nx)) + 1j * rng.standard_normal((2 * L + 1, ny, nx))
    for op, opname in ((rte.OP_A, "A"), (rte.OP_KT, "KT")):
        y = host(ctx.apply(dev(u), op=op))
        ref = op2.apply_direct(u, L, h, mu_a + mu_s, mu_s, sh, opname)
        e = relerr(y, ref)
        say("  op", opname, "relerr", e)
        assert e <= (TOL64 if prec == 1 else TOL32)
    ctx.close()


@pytest.mark.parametrize("L,ny,nx", [(3, 96, 200), (1, 150, 40)])
@pytest.mark.parametrize("prec", [1, 0])
def test_apply_nonsquare_vs_oracle_fft(rte, L, ny, nx, prec):
    """Non-square grids (different padded sizes in x and y, ragged row tiles and column groups)
    against the oracle's FP64 FFT apply."""
    say("apply nonsquare", L, ny, nx, "prec", prec)
    rng = np.random.default_rng(ny + nx + L)
    h = 1.0 / max(nx, ny)
    mu_a, mu_s = 0.1, 3.0
    ctx, sh = _ctx(rte, (nx, ny), L, mu_a=mu_a, mu_s=mu_s, prec=prec, h=h)
    u = inputs.random_conj_symmetric_modes(rng, L, max(nx, ny))[:, :ny, :nx].copy()
    y = host(ctx.apply(dev(u), op=rte.OP_A))
    ref = op2.apply_fft(u, L, h, mu_a + mu_s, mu_s, sh, "A")
    e = relerr(y, ref)
    say("  relerr", e)
    assert e <= (TOL64 if prec == 1 else TOL32)
    ctx.close()


@pytest.mark.parametrize("L,n", [(8, 64), (4, 100), (0, 128), (2, 33)])
@pytest.mark.parametrize("prec", [1, 0])
def test_apply_mid_vs_oracle_fft(rte, L, n, prec):
    say("apply mid", L, n, "prec", prec)
    rng = np.random.default_rng(7 + n + L)
    h = 1.0 / n
    mu_a, mu_s = 0.1, 10.0
    ctx, sh = _ctx(rte, n, L, mu_a=mu_a, mu_s=mu_s, prec=prec)
    u = inputs.random_conj_symmetric_modes(rng, L, n)
    y = host(ctx.apply(dev(u)))
    ref = op2.apply_fft(u, L, h, mu_a + mu_s, mu_s, sh, "A")
    e = relerr(y, ref)
    say("  relerr", e)
    assert e <= (TOL64 if prec == 1 else TOL32)
    # the channel layout gives the same operator on a conjugate-symmetric vector
    ch = ctx.modes_to_channels(dev(u))
    yc = ctx.channels_to_modes(ctx.apply(ch, layout=rte.LAYOUT_CHANNELS))
    assert relerr(host(yc), ref) <= (TOL64 if prec == 1 else TOL32)
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_apply_full_size_sampled(rte, prec):
    """512^2, L = 8 (17 modes): the apply at sampled output cells against the oracle's direct sum
    over all cells (each sampled row costs N M^2)."""
    n, L = 512, 8
    say("apply full 512 L8 prec", prec)
    rng = np.random.default_rng(11)
    mu_a, mu_s = 0.1, 10.0
    ctx, sh = _ctx(rte, n, L, mu_a=mu_a, mu_s=mu_s, prec=prec)
    u = inputs.random_conj_symmetric_modes(rng, L, n)
    y = host(ctx.apply(dev(u)))
    cells = [(0, 0), (511, 511), (0, 511), (255, 256)] + [tuple(rng.integers(0, n, 2)) for _ in range(12)]
    ref = op2.apply_sampled(u, cells, L, 1.0 / n, mu_a + mu_s, mu_s, sh, "A")
    got = np.stack([y[:, iy, ix] for iy, ix in cells])
    e = relerr(got, ref)
    say("  sampled relerr", e)
    assert e <= (TOL64 if prec == 1 else TOL32)
    ctx.close()


@pytest.mark.parametrize("L,n", [(0, 32), (3, 24), (8, 32), (6, 40), (8, 200), (5, 77)])
def test_rhs_vs_oracle(rte, L, n):
    say("rhs", L, n)
    w = inputs.workload("hg512", seed=3, n=n)
    ctx, sh = _ctx(rte, n, L, mu_a=0.1, mu_s=1.0, prec=0)
    b = host(ctx.rhs(dev(w["f"])))
    ref = op2.rhs(w["f"], L, 1.0 / n, 1.1)
    e = relerr(b, ref)
    say("  relerr", e)
    assert e <= TOL64
    ctx.close()


@pytest.mark.parametrize("shape", [(8, 8, 8), (9, 10, 7), (2, 3, 2)])
@pytest.mark.parametrize("prec", [1, 0])
def test_apply_3d_small_vs_dense(rte, shape, prec):
    nx, ny, nz = shape
    say("apply 3d", shape, "prec", prec)
    rng = np.random.default_rng(5)
    h, mu_a, mu_s = 1.0 / 10, 0.05, 3.0
    ctx = rte.Context((nx, ny, nz), h=h, mu_a=mu_a, mu_s=mu_s, L=0, prec=prec)
    u = rng.standard_normal((1, nz, ny, nx)) + 1j * rng.standard_normal((1, nz, ny, nx))
    A = op3.dense_A(nz, ny, nx, h, mu_a + mu_s, mu_s)
    ref = (A @ u.reshape(-1)).reshape(u.shape)
    y = host(ctx.apply(dev(u)))
    e = relerr(y, ref)
    say("  relerr", e)
    assert e <= (TOL64 if prec == 1 else TOL32)
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_apply_3d_max_size_sampled(rte, prec):
    """The largest 3D grid the library accepts (256^3, a 512^3 padded FFT): sampled outputs,
    corners included, against the oracle's direct sum."""
    n = 256
    say("apply 3d 256 prec", prec)
    rng = np.random.default_rng(8)
    h, mu_a, mu_s = 1.0 / n, 0.05, 10.0
    ctx = rte.Context(n, dim=3, h=h, mu_a=mu_a, mu_s=mu_s, L=0, prec=prec)
    u = rng.standard_normal((n, n, n))
    y = host(ctx.apply(dev(u[None]), layout=rte.LAYOUT_CHANNELS))[0]
    cells = [(0, 0, 0), (255, 255, 255), (0, 255, 128)] + [tuple(rng.integers(0, n, 3)) for _ in range(3)]
    ref = op3.apply_sampled(u, cells, h, mu_a + mu_s, mu_s)
    got = np.array([y[c] for c in cells])
    e = relerr(got, ref)
    say("  sampled relerr", e)
    assert e <= (TOL64 if prec == 1 else TOL32)
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_apply_3d_full_size_sampled(rte, prec):
    n = 128
    say("apply 3d 128 prec", prec)
    rng = np.random.default_rng(6)
    h, mu_a, mu_s = 1.0 / n, 0.05, 10.0
    ctx = rte.Context(n, dim=3, h=h, mu_a=mu_a, mu_s=mu_s, L=0, prec=prec)
    u = rng.standard_normal((n, n, n))
    y = host(ctx.apply(dev(u[None]), layout=rte.LAYOUT_CHANNELS))[0]
    cells = [(0, 0, 0), (127, 127, 127), (64, 3, 100)] + [tuple(rng.integers(0, n, 3)) for _ in range(5)]
    ref = op3.apply_sampled(u, cells, h, mu_a + mu_s, mu_s)
    got = np.array([y[c] for c in cells])
    e = relerr(got, ref)
    say("  sampled relerr", e)
    assert e <= (TOL64 if prec == 1 else TOL32)
    ctx.close()
