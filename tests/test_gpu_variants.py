"""Kernel variants of the 2D apply (row tiles, thread counts, FFT grouping) and the autotuner:
every variant of every pass gives the same result up to rounding (the arithmetic is the same; the
compiler may contract multiply-adds differently per instantiation), and the tuner's choice is
valid."""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, say
from paper_1802_03061_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rte():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1802_03061_amd import rte as r
    r.load()
    return r


@pytest.mark.parametrize("n,L,prec", [(200, 2, 0), (256, 8, 0), (150, 1, 1), (512, 8, 0)])
def test_variants_agree(rte, n, L, prec):
    say("variants", n, L, prec)
    ctx = rte.Context(n, mu_a=0.1, mu_s=2.0, sigma_hat=inputs.hg_sigma_hat(0.5, L), L=L, prec=prec)
    rng = np.random.default_rng(n + L)
    x = dev(inputs.random_conj_symmetric_modes(rng, L, n))
    precs = [prec] if prec == rte.PREC_FP64 else [rte.PREC_FP32, rte.PREC_FP64]
    for p in precs:
        for pass_ in range(3):
            for q in range(3):
                ctx.set_variant(p, q, 0)
        ref = host(ctx.apply(x, op=rte.OP_A, prec=p))
        for pass_ in range(3):
            v0, nv = ctx.get_variant(p, pass_)
            for v in range(1, nv):
                ctx.set_variant(p, pass_, v)
                y = host(ctx.apply(x, op=rte.OP_A, prec=p))
                d = float(np.abs(y - ref).max()) / float(np.abs(ref).max())
                say(f"  prec {p} pass {pass_} variant {v}/{nv}: max |diff| / max |y| = {d:.2e}")
                assert d <= (1e-6 if p == rte.PREC_FP32 else 1e-13)
            ctx.set_variant(p, pass_, 0)
        with pytest.raises(rte.RteError):
            ctx.set_variant(p, 1, 99)
    ctx.autotune(reps=3)
    for p in precs:
        for pass_ in range(3):
            v, nv = ctx.get_variant(p, pass_)
            assert 0 <= v < nv
    ctx.close()
