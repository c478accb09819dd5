"""Several sources sharing one operator (rte_solve_multi, global GMRES on the stacked system)
against the CPU oracle through the C ABI: every source's solution matches its own dense-LU
solution (small grids, 2D and 3D, both precisions, a zero source among them), a full-size batch
matches the single-source solver and the oracle's FP64 reference solve, and bad arguments are
refused."""
import ctypes

import numpy as np
import pytest
import torch

import oracle_ref
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


@pytest.mark.parametrize("prec,bar", [(1, 1e-10), (0, 1e-6)])
def test_multi_small_2d_vs_lu(rte, prec, bar):
    n, L, B = 12, 2, 5
    h, mu_a, mu_s = 1.0 / n, 0.1, 6.0
    sh = inputs.hg_sigma_hat(0.5, L)
    rng = np.random.default_rng(31)
    fs = [rng.random((n, n)) * (s + 1) for s in range(B)]
    fs[2] = np.zeros((n, n))                         # a zero source gives u = 0
    ctx = rte.Context(n, mu_a=mu_a, mu_s=mu_s, sigma_hat=sh, L=L, prec=prec)
    us, infos, rc = ctx.solve_multi([dev(f) for f in fs], tol=1e-11)
    say("multi 2d prec", prec, "iterations", infos[0]["iterations"], [round(i["relres_true"], 14) for i in infos])
    assert rc == rte.RTE_OK
    A = op2.dense_A(n, n, L, h, mu_a + mu_s, mu_s, sh)
    for s, (f, u, info) in enumerate(zip(fs, us, infos)):
        b = op2.rhs(f, L, h, mu_a + mu_s, method="direct")
        uu = host(u)
        if not f.any():
            assert float(np.abs(uu).max()) == 0.0
            continue
        ref = kr.solve_dense(A, b.reshape(-1)).reshape(b.shape)
        e = relerr(uu, ref)
        say(f"  source {s}: relres {info['relres_true']:.2e} relerr vs LU {e:.2e}")
        assert info["relres_true"] <= 1e-11 and info["status"] == rte.RTE_OK
        assert e <= bar
    ctx.close()


@pytest.mark.parametrize("prec,bar", [(1, 1e-10), (0, 1e-6)])
def test_multi_small_3d_vs_lu(rte, prec, bar):
    n, L, B = 5, 1, 3
    h, mu_a, mu_s = 1.0 / n, 0.1, 3.0
    sh = inputs.hg_sigma_hat(0.5, L)
    rng = np.random.default_rng(7)
    fs = [rng.random((n, n, n)) for _ in range(B)]
    ctx = rte.Context((n, n, n), h=h, mu_a=mu_a, mu_s=mu_s, sigma_hat=sh, L=L, prec=prec)
    us, infos, rc = ctx.solve_multi([dev(f) for f in fs], tol=1e-11)
    assert rc == rte.RTE_OK
    A = o3s.dense_A(n, n, n, L, h, mu_a + mu_s, mu_s, sh)
    for f, u in zip(fs, us):
        b = o3s.rhs(f, L, h, mu_a + mu_s, method="direct")
        ref = kr.solve_dense(A, b.reshape(-1)).reshape(b.shape)
        e = relerr(host(u).real, ref)
        say("multi 3d prec", prec, "relerr vs LU", e)
        assert e <= bar
    ctx.close()


@pytest.mark.timeout(900)
def test_multi_full_size_vs_single_and_oracle(rte):
    """16 Gaussian-mixture sources on one 256^2, L = 4 medium (HG g = 0.5, mu_a = 0.1, mu_s = 10),
    FP32 apply, tol 1e-8: every source meets the tolerance, matches the single-source solver, and
    two of them match the oracle's FP64 reference solve."""
    n, L, B = 256, 4, 16
    mu_a, mu_s = 0.1, 10.0
    sh = inputs.hg_sigma_hat(0.5, L)
    fs = [inputs.gaussian_mixture_source(n, inputs.gaussian_mixture_params(np.random.default_rng(s), 2))
          for s in range(B)]
    ctx = rte.Context(n, mu_a=mu_a, mu_s=mu_s, sigma_hat=sh, L=L, prec=rte.PREC_FP32)
    fd = [dev(f) for f in fs]
    us, infos, rc = ctx.solve_multi(fd, tol=1e-8)
    assert rc == rte.RTE_OK
    say(f"multi 256 L4 x{B}: {infos[0]['iterations']} stacked iterations, {infos[0]['t_solve_ms']:.2f} ms, "
        f"worst relres {max(i['relres_true'] for i in infos):.2e}")
    t_single = 0.0
    for s in range(B):
        assert infos[s]["relres_true"] <= 1e-8
        u1, i1 = ctx.solve(fd[s], tol=1e-8)
        t_single += i1["t_solve_ms"]
        e1 = relerr(host(us[s]), host(u1))
        assert e1 <= 1e-6
    say(f"  {B} single solves: {t_single:.2f} ms in all")
    for s in (0, 5):
        ref = oracle_ref.Ref2D(fs[s], n, L, mu_a, mu_s, sh)
        e = relerr(host(us[s]), ref.u)
        say(f"  source {s}: relerr vs oracle {e:.2e} (reference {ref.iterations} it, {ref.seconds:.1f} s)")
        assert e <= 1e-6
    ctx.close()


def test_multi_bad_arguments(rte):
    ctx = rte.Context(8, mu_a=0.1, mu_s=1.0, L=1, sigma_hat=[1, 0.5], prec=1)
    lib = rte.load()
    f = torch.ones((8, 8), dtype=torch.float64, device="cuda")
    u = torch.empty((3, 8, 8), dtype=torch.complex128, device="cuda")
    P = ctypes.c_void_p
    fp = (P * 1)(P(f.data_ptr()))
    up = (P * 1)(P(u.data_ptr()))
    assert lib.rte_solve_multi(ctx._h, 0, fp, 1e-8, 10, up, None) == rte.RTE_EINVAL
    assert lib.rte_solve_multi(ctx._h, rte.MAX_RHS + 1, fp, 1e-8, 10, up, None) == rte.RTE_EINVAL
    assert lib.rte_solve_multi(ctx._h, 1, fp, 0.0, 10, up, None) == rte.RTE_EINVAL
    nul = (P * 1)(None)
    assert lib.rte_solve_multi(ctx._h, 1, nul, 1e-8, 10, up, None) == rte.RTE_EINVAL
    ctx.close()


def test_time_apply_multi(rte):
    """The batched apply timing over stacked right-hand sides: every pass timed, more sources take
    longer, and out-of-range counts are refused."""
    ctx = rte.Context(256, mu_a=0.1, mu_s=2.0, L=2, sigma_hat=[1, .5, .25], prec=rte.PREC_FP32)
    t1, p1 = ctx.time_apply_multi(1, reps=5)
    t16, p16 = ctx.time_apply_multi(16, reps=5)
    say("time_apply_multi 1:", t1, p1[:3], "16:", t16, p16[:3])
    assert all(x > 0 for x in p1[:3]) and all(x > 0 for x in p16[:3])
    assert t16 > 2 * t1          # sixteen times the vector traffic at a size well past launch latency
    with pytest.raises(rte.RteError) as ei:
        ctx.time_apply_multi(rte.MAX_RHS + 1, reps=1)
    assert ei.value.code == rte.RTE_EINVAL
    ctx.close()
