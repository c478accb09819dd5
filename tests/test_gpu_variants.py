"""Kernel variants of the 2D apply (row tiles, thread counts, FFT grouping, the register-resident
pass B with its unpacked work buffer) and the autotuner: every variant of every pass, alone and
combined with the others, matches the oracle's FP64 FFT apply to the path's bar (FP32 1e-6,
FP64 1e-12), and the tuner's choice is valid."""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, relerr, say
from oracle import operator2d as op2
from paper_1802_03061_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rte():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1802_03061_amd import rte as r
    r.load()
    return r


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n,L,prec", [(200, 2, 0), (256, 8, 0), (150, 1, 1), (512, 8, 0), (96, 4, 0), (128, 6, 1),
                                      (72, 7, 0), (40, 5, 1)])
def test_variants_match_oracle(rte, n, L, prec):
    say("variants", n, L, prec)
    mu_a, mu_s = 0.1, 2.0
    sh = inputs.hg_sigma_hat(0.5, L)
    ctx = rte.Context(n, mu_a=mu_a, mu_s=mu_s, sigma_hat=sh, L=L, prec=prec)
    rng = np.random.default_rng(n + L)
    u = inputs.random_conj_symmetric_modes(rng, L, n)
    x = dev(u)
    ref = op2.apply_fft(u, L, 1.0 / n, mu_a + mu_s, mu_s, sh, "A", workers=16)
    precs = [prec] if prec == rte.PREC_FP64 else [rte.PREC_FP32, rte.PREC_FP64]
    for p in precs:
        bar = 1e-6 if p == rte.PREC_FP32 else 1e-12
        counts = [ctx.get_variant(p, q)[1] for q in range(3)]
        combos = set()
        for q in range(3):
            for v in range(counts[q]):
                combo = [0, 0, 0]
                combo[q] = v
                combos.add(tuple(combo))
        for vb in range(counts[1]):          # every pass-B variant with the last A and C variants
            combos.add((counts[0] - 1, vb, counts[2] - 1))
        for combo in sorted(combos):
            for q in range(3):
                ctx.set_variant(p, q, combo[q])
            y = host(ctx.apply(x, op=rte.OP_A, prec=p))
            e = relerr(y, ref)
            say(f"  prec {p} variants {combo} of {counts}: relerr vs oracle {e:.2e}")
            assert e <= bar
        with pytest.raises(rte.RteError):
            ctx.set_variant(p, 1, 99)
        for q in range(3):
            ctx.set_variant(p, q, 0)
    ctx.autotune(reps=3)
    for p in precs:
        for pass_ in range(3):
            v, nv = ctx.get_variant(p, pass_)
            assert 0 <= v < nv
    y = host(ctx.apply(x, op=rte.OP_A))
    assert relerr(y, ref) <= (1e-6 if prec == rte.PREC_FP32 else 1e-12)
    ctx.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n,L,prec", [(40, 0, 0), (33, 0, 1), (20, 2, 0), (12, 3, 1)])
def test_variants_3d_match_oracle(rte, n, L, prec):
    """3D: every variant of each of the five passes (x-pass row tiles, y-pass z-rows, z-pass
    columns), the others at variant 0, against the oracle's FP64 FFT apply; then the tuner."""
    from oracle import operator3d as op3
    from oracle import operator3d_sh as o3s
    say("variants 3d", n, L, prec)
    mu_a, mu_s, h = 0.1, 2.0, 1.0 / n
    sh = inputs.hg_sigma_hat(0.5, L)
    ctx = rte.Context((n, n, n), h=h, mu_a=mu_a, mu_s=mu_s, sigma_hat=sh, L=L, prec=prec)
    M = (L + 1) ** 2
    rng = np.random.default_rng(n + 7 * L)
    u = rng.standard_normal((M, n, n, n))
    if L == 0:
        ref = op3.apply_fft(u[0], h, mu_a + mu_s, mu_s, "A", workers=16)[None]
    else:
        ref = o3s.apply_fft(u, L, h, mu_a + mu_s, mu_s, sh, "A", workers=16)
    x = dev(u)
    precs = [prec] if prec == rte.PREC_FP64 else [rte.PREC_FP32, rte.PREC_FP64]
    for p in precs:
        bar = 1e-6 if p == rte.PREC_FP32 else 1e-12
        counts = [ctx.get_variant(p, q)[1] for q in range(5)]
        assert counts[1] == 3 and counts[3] == 3 and counts[2] == (3 if L == 0 else 1)
        for q in range(5):
            for v in range(counts[q]):
                for qq in range(5):
                    ctx.set_variant(p, qq, v if qq == q else 0)
                y = host(ctx.apply(x, op=rte.OP_A, prec=p, layout=rte.LAYOUT_CHANNELS))
                e = relerr(y.reshape(ref.shape), ref)
                say(f"  prec {p} pass {q} variant {v} of {counts[q]}: relerr vs oracle {e:.2e}")
                assert e <= bar
        with pytest.raises(rte.RteError):
            ctx.set_variant(p, 5, 0)
        for qq in range(5):
            ctx.set_variant(p, qq, 0)
    ctx.autotune(reps=2)
    for p in precs:
        for q in range(5):
            v, nv = ctx.get_variant(p, q)
            assert 0 <= v < nv
    y = host(ctx.apply(x, op=rte.OP_A, layout=rte.LAYOUT_CHANNELS))
    assert relerr(y.reshape(ref.shape), ref) <= (1e-6 if prec == rte.PREC_FP32 else 1e-12)
    ctx.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [1, 0])
def test_batched_variants_match_oracle(rte, prec):
    """The batched solver under every forced row-tile variant (passes A and C) and every column-group
    variant (pass B): problems of five padded sizes (64 .. 1024, ragged tiles), each batched
    solution against the oracle's FP64 reference solve of its own problem; then the tuned plan,
    whose reported variants must be in range."""
    import oracle_ref
    say("batched variants prec", prec)
    rng = np.random.default_rng(31 + prec)
    sizes = (20, 64, 100, 150, 300, 64)
    probs = [dict(n=n, mu_s=float(rng.uniform(0.5, 8.0)), mu_a=float(rng.uniform(0.05, 0.5)),
                  params=inputs.gaussian_mixture_params(rng, 2)) for n in sizes]
    srcs = [inputs.gaussian_mixture_source(p["n"], p["params"]) for p in probs]
    refs = [oracle_ref.Ref2D(f, p["n"], 0, p["mu_a"], p["mu_s"], np.ones(1)) for p, f in zip(probs, srcs)]
    tol, bar = (1e-8, 1e-6) if prec == rte.PREC_FP32 else (1e-11, 1e-9)
    ctxs = [rte.Context(p["n"], mu_a=p["mu_a"], mu_s=p["mu_s"], L=0, prec=prec) for p in probs]
    fs = [dev(f) for f in srcs]
    combos = [(v, 0) for v in range(4)] + [(3, v) for v in range(4)] + [(-1, -1)]
    try:
        for vr, vb in combos:
            rte.set_batched_variant(0, vr)
            rte.set_batched_variant(1, vb)
            us, infos, rc = rte.solve_batched(ctxs, fs, [tol] * len(ctxs))
            assert rc == rte.RTE_OK
            _, launches = rte.time_batched_apply(ctxs, reps=2)
            used = {(ps, px): var for ps, px, py, ms, var in launches}
            for (ps, px), var in used.items():
                if px < 128:
                    assert var == 0
                elif vr >= 0:
                    assert var == (vb if ps == 1 else vr)
                else:
                    assert 0 <= var < 4
            worst = max(relerr(host(u), r.u) for u, r in zip(us, refs))
            say(f"  forced ({vr}, {vb}): launches {sorted(used.items())} worst relerr vs oracle {worst:.2e}")
            assert worst <= bar
            assert max(i["relres_true"] for i in infos) <= tol
    finally:
        rte.set_batched_variant(0, -1)
        rte.set_batched_variant(1, -1)
        for c in ctxs:
            c.close()
