"""The batched solver (rte_solve_batched): many isotropic problems of uneven size solved together
in lockstep, one graph-captured inner iteration replayed, against individual solves and the CPU
oracle (through the C ABI)."""
import numpy as np
import pytest
import torch

import oracle_ref
from gpu_util import dev, host, relerr, say
from oracle import krylov as kr
from oracle import operator2d as op2
from paper_1802_03061_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rte():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1802_03061_amd import rte as r
    r.load()
    return r


def _small_batch(seed=5):
    rng = np.random.default_rng(seed)
    probs = []
    for n in (16, 24, 33, 40, 16, 64, 24):
        probs.append(dict(n=n, mu_s=float(rng.uniform(0.5, 8.0)), mu_a=float(rng.uniform(0.05, 0.5)),
                          params=inputs.gaussian_mixture_params(rng, 2)))
    return probs


@pytest.mark.parametrize("prec", [1, 0])
def test_batched_small_vs_lu_and_single(rte, prec):
    """Seven problems of sizes 16..64 (three padded sizes, ragged tiles): every batched solution
    matches the dense LU solution of its own system and the single-problem solver."""
    say("batched small prec", prec)
    probs = _small_batch()
    ctxs = [rte.Context(p["n"], mu_a=p["mu_a"], mu_s=p["mu_s"], L=0, prec=prec) for p in probs]
    fs = [dev(inputs.gaussian_mixture_source(p["n"], p["params"])) for p in probs]
    tol = 1e-11
    us, infos, rc = rte.solve_batched(ctxs, fs, [tol] * len(ctxs))
    assert rc == rte.RTE_OK
    for i, (p, c, f, u, info) in enumerate(zip(probs, ctxs, fs, us, infos)):
        n = p["n"]
        h, mu_t = 1.0 / n, p["mu_a"] + p["mu_s"]
        A = op2.dense_A(n, n, 0, h, mu_t, p["mu_s"], np.ones(1))
        b = op2.rhs(host(f), 0, h, mu_t, method="direct")
        x = kr.solve_dense(A, b.reshape(-1)).reshape(b.shape)
        e_lu = relerr(host(u), x)
        u1, i1 = c.solve(f, tol=tol)
        e_single = relerr(host(u), host(u1))
        say(f"  {i} n={n} iters={info['iterations']} (single {i1['iterations']}) cycles={info['cycles']} "
            f"res={info['relres_true']:.2e} vs LU {e_lu:.2e} vs single {e_single:.2e}")
        assert info["status"] == rte.RTE_OK and info["relres_true"] <= tol
        assert e_lu <= 1e-9
        assert e_single <= 1e-9
        assert abs(info["iterations"] - i1["iterations"]) <= 2 * max(1, info["cycles"])
    for c in ctxs:
        c.close()


def test_batched_zero_source_and_repeat(rte):
    """A zero source inside a batch gives u = 0 with no iterations; a second call on the same
    contexts (fewer problems) reproduces the first call's solutions."""
    say("batched zero source")
    probs = _small_batch(seed=9)[:4]
    ctxs = [rte.Context(p["n"], mu_a=p["mu_a"], mu_s=p["mu_s"], L=0, prec=0) for p in probs]
    fs = [dev(inputs.gaussian_mixture_source(p["n"], p["params"])) for p in probs]
    fs[1] = torch.zeros_like(fs[1])
    us, infos, rc = rte.solve_batched(ctxs, fs, [1e-8] * 4)
    assert rc == rte.RTE_OK
    assert infos[1]["iterations"] == 0 and float(host(us[1]).__abs__().max()) == 0.0
    us2, infos2, rc2 = rte.solve_batched(ctxs[2:], fs[2:], [1e-8] * 2)
    assert rc2 == rte.RTE_OK
    for a, b in zip(us[2:], us2):
        assert relerr(host(b), host(a)) <= 1e-14
    for c in ctxs:
        c.close()


def test_batched_iteration_cap(rte):
    say("batched iteration cap")
    p = _small_batch()[5]
    ctx = rte.Context(p["n"], mu_a=p["mu_a"], mu_s=p["mu_s"], L=0, prec=0)
    f = dev(inputs.gaussian_mixture_source(p["n"], p["params"]))
    us, infos, rc = rte.solve_batched([ctx], [f], [1e-12], max_iter=2, allow_not_converged=True)
    assert rc == rte.RTE_NOT_CONVERGED and infos[0]["status"] == rte.RTE_NOT_CONVERGED
    assert infos[0]["iterations"] <= 2
    ctx.close()


@pytest.mark.timeout(900)
def test_batched_128_heterogeneous(rte):
    """128 isotropic problems, n drawn from {64, 128, 256, 512}, mu_s ~ U[0.5, 20],
    mu_a ~ U[0.01, 0.5], Gaussian-mixture sources, FP32 apply and FP64 refinement, tol 1e-8: all
    converge; the oracle's FP64 FFT apply confirms the true residual of every problem; for the
    first and the hardest problem (largest mu_s / mu_t) of every size the solution matches the
    oracle's FP64 reference solve element by element (relative L2 error <= 1e-6) and the
    single-problem solver."""
    say("batched 128 heterogeneous")
    probs = inputs.batched_problems(count=128, seed=3)
    ctxs = [rte.Context(p["n"], mu_a=p["mu_a"], mu_s=p["mu_s"], L=0, prec=rte.PREC_FP32) for p in probs]
    fs = [dev(inputs.gaussian_mixture_source(p["n"], p["params"])) for p in probs]
    us, infos, rc = rte.solve_batched(ctxs, fs, [1e-8] * 128)
    assert rc == rte.RTE_OK
    its = [i["iterations"] for i in infos]
    say(f"  iterations min {min(its)} max {max(its)} mean {np.mean(its):.1f}; batch time "
        f"{infos[0]['t_solve_ms']:.1f} ms")
    assert max(i["relres_true"] for i in infos) <= 1e-8
    sample = set()
    for n in (64, 128, 256, 512):
        idx = [i for i, p in enumerate(probs) if p["n"] == n]
        if idx:
            sample.add(max(idx, key=lambda i: probs[i]["mu_s"] / (probs[i]["mu_s"] + probs[i]["mu_a"])))
            sample.add(idx[0])
    worst = 0.0
    for i, p in enumerate(probs):
        n = p["n"]
        h, mu_t = 1.0 / n, p["mu_a"] + p["mu_s"]
        f = host(fs[i])
        uu = host(us[i])
        if i in sample:
            ref = oracle_ref.Ref2D(f, n, 0, p["mu_a"], p["mu_s"], np.ones(1))
            rr = ref.residual(uu)
            e = relerr(uu, ref.u)
            u1, _ = ctxs[i].solve(fs[i], tol=1e-8)
            e1 = relerr(uu, host(u1))
            say(f"  problem {i}: n={n} mu_s={p['mu_s']:.2f} mu_a={p['mu_a']:.3f} iters={infos[i]['iterations']} "
                f"vs oracle {e:.2e} (reference {ref.iterations} it, {ref.seconds:.1f} s), oracle residual "
                f"{rr:.2e}, vs single {e1:.2e}")
            assert e <= 1e-6
            assert e1 <= 1e-6
        else:
            spectra = op2.kernel_spectra(n, n, 0, h, mu_t, workers=oracle_ref.WORKERS)
            b = op2.rhs(f, 0, h, mu_t, spectra=spectra, workers=oracle_ref.WORKERS)
            r = b - op2.apply_fft(uu, 0, h, mu_t, p["mu_s"], np.ones(1), "A", spectra=spectra,
                                  workers=oracle_ref.WORKERS)
            rr = float(np.linalg.norm(r) / np.linalg.norm(b))
        worst = max(worst, rr)
        assert rr <= 1.5e-8
    say(f"  largest oracle true residual over the 128 problems {worst:.2e}")
    for c in ctxs:
        c.close()


def test_batched_nonsquare_fp64(rte):
    """Non-square problems (x and y padded to different sizes) in one FP64 batch against dense LU."""
    say("batched nonsquare fp64")
    rng = np.random.default_rng(21)
    shapes = [(12, 20), (24, 9), (17, 17), (30, 14)]
    ctxs, fs, refs = [], [], []
    for nx, ny in shapes:
        mu_a, mu_s = float(rng.uniform(0.05, 0.3)), float(rng.uniform(1.0, 6.0))
        h = 1.0 / max(nx, ny)
        f = rng.random((ny, nx))
        ctxs.append(rte.Context((nx, ny), h=h, mu_a=mu_a, mu_s=mu_s, L=0, prec=rte.PREC_FP64))
        fs.append(dev(f))
        A = op2.dense_A(ny, nx, 0, h, mu_a + mu_s, mu_s, np.ones(1))
        b = op2.rhs(f, 0, h, mu_a + mu_s, method="direct")
        refs.append(kr.solve_dense(A, b.reshape(-1)).reshape(b.shape))
    us, infos, rc = rte.solve_batched(ctxs, fs, [1e-11] * len(ctxs))
    assert rc == rte.RTE_OK
    for (nx, ny), u, ref, info in zip(shapes, us, refs, infos):
        e = relerr(host(u), ref)
        say(f"  {nx}x{ny}: iters {info['iterations']} vs LU {e:.2e}")
        assert e <= 1e-9
    for c in ctxs:
        c.close()
