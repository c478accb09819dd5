"""The allocation-free network forward (rte_nn_forward_noalloc) against rte_nn_forward, through
the C ABI: same kernels on the same operands, so the outputs agree bit for bit; two calls in a
row (the second smaller) and the size limit."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rte():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1802_03061_amd import rte as r
    r.load()
    return r


@pytest.mark.parametrize("C,hidden,layers", [(17, 32, 5), (9, 16, 2), (5, 32, 3)])
def test_forward_noalloc_matches_forward(rte, C, hidden, layers):
    say("nn forward noalloc", C, hidden, layers)
    rng = np.random.default_rng(C * 10 + layers)
    net = rte.Net(C, hidden, layers, seed=C + layers, use_bias=True)
    # non-zero biases, so every bias read matters
    p = host(net.params())
    p = p + 0.05 * rng.standard_normal(p.shape).astype(np.float32)
    net.set_params(dev(p.astype(np.float32)))
    lib = rte.load()
    for B, H, W in ((3, 24, 40), (1, 9, 13)):          # the second call is smaller
        x = dev(rng.standard_normal((B, C, H, W)).astype(np.float32))
        y_ref = net.forward(x)
        y = torch.full((B, C, H, W), float("nan"), dtype=torch.float32, device="cuda")
        rc = lib.rte_nn_forward_noalloc(net._h, ctypes.c_void_p(x.data_ptr()), B, H, W, ctypes.c_void_p(y.data_ptr()))
        assert rc == rte.RTE_OK, rte.last_error()
        a, b = host(y), host(y_ref)
        say(f"  B={B} H={H} W={W}: max |diff| {np.abs(a - b).max():.3e}")
        assert np.isfinite(a).all()
        assert np.array_equal(a, b)
    net.close()


def test_forward_noalloc_rejects_oversize(rte):
    """Inputs beyond the fixed array's limit are refused with RTE_EINVAL before any work."""
    net = rte.Net(17, 32, 5, seed=1)
    lib = rte.load()
    limit = rte.NN_SCRATCH_BYTES // 4 // 2          # floats per activation for a 5-layer network
    H = W = 512
    B = limit // (32 * H * W) + 1
    x = torch.zeros(1, dtype=torch.float32, device="cuda")     # never read: the size check comes first
    y = torch.zeros(1, dtype=torch.float32, device="cuda")
    rc = lib.rte_nn_forward_noalloc(net._h, ctypes.c_void_p(x.data_ptr()), B, H, W, ctypes.c_void_p(y.data_ptr()))
    assert rc == rte.RTE_EINVAL
    assert "exceeds" in rte.last_error()
    net.close()
