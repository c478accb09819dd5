"""GPU tests of the learned preconditioner: the MFMA convolution network against the FP64 oracle
(forward, parameter gradient, Adam), the training-pair builder against the oracle's definition, the
gain of the trained network in FGMRES over plain GMRES, and the fallback when the network is broken.

BF16 operands with FP32 accumulation through 5 layers give relative errors of a few 1e-3 per
layer; the bars below (3e-2 forward, 5e-2 gradients) leave room for that and catch any layout or
indexing error, which shows up as O(1)."""
import numpy as np
import pytest
import torch

import oracle_ref
from gpu_util import dev, host, relerr, say
from oracle import convnet as cn
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


def unpack(p, C, hidden, layers):
    """Packed parameters -> [(W, b)] in FP64 (layout of rte_nn.h)."""
    out, off = [], 0
    for l in range(layers):
        ci = C if l == 0 else hidden
        co = C if l == layers - 1 else hidden
        W = p[off:off + co * ci * 9].reshape(co, ci, 3, 3).astype(np.float64); off += co * ci * 9
        b = p[off:off + co].astype(np.float64); off += co
        out.append((W, b))
    return out


def pack(params):
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in params]).astype(np.float32)


@pytest.mark.parametrize("C,hidden,H,W", [(17, 32, 9, 37), (9, 32, 32, 32), (1, 16, 5, 7), (5, 32, 16, 40)])
def test_forward_matches_oracle(rte, C, hidden, H, W):
    say("nn forward", C, hidden, H, W)
    rng = np.random.default_rng(C + H)
    net = rte.Net(C, hidden, 5, seed=C)
    params = unpack(host(net.params()), C, hidden, 5)
    # non-zero biases to exercise the bias path
    params = [(Wt, 0.1 * rng.standard_normal(b.shape)) for Wt, b in params]
    net.set_params(dev(pack(params)))
    x = rng.standard_normal((3, C, H, W)).astype(np.float32)
    y = host(net.forward(dev(x)))
    ref, _ = cn.net_forward(x.astype(np.float64), params)
    e = relerr(y, ref)
    say("  relerr", e)
    assert e <= 3e-2
    net.close()


def bf16(a):
    """Round to the nearest BF16 (ties to even), returned as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def emulated_grads(x, t, w, params):
    """The oracle's convolutions applied to the operands the GPU kernels use: BF16-rounded layer
    inputs and weights in the forward and data-gradient convolutions, and BF16-rounded layer inputs
    and output gradients in the weight and bias gradients (all three are BF16 GEMMs with FP32
    accumulation on the GPU)."""
    acts, pre = [x], []
    a = x
    for l, (W, b) in enumerate(params):
        z = cn.conv3x3(bf16(a), bf16(W), b)
        pre.append(z)
        a = np.maximum(z, 0.0) if l < len(params) - 1 else z
        acts.append(a)
    B = x.shape[0]
    g = 2.0 * (acts[-1] - t) * (w / B)[:, None, None, None]
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        _, gW, gb = cn.conv3x3_backward(bf16(acts[l]), params[l][0], bf16(g))
        grads[l] = (gW, gb)
        if l > 0:
            gx, _, _ = cn.conv3x3_backward(acts[l], bf16(params[l][0]), bf16(g))
            g = gx * (pre[l - 1] > 0)
    return grads


def test_gradient_matches_oracle(rte):
    C, hidden, H, W, B = 9, 32, 12, 20, 4
    rng = np.random.default_rng(7)
    net = rte.Net(C, hidden, 5, seed=3)
    params = unpack(host(net.params()), C, hidden, 5)
    params = [(Wt, 0.05 * rng.standard_normal(b.shape)) for Wt, b in params]
    net.set_params(dev(pack(params)))
    x = rng.standard_normal((B, C, H, W)).astype(np.float32)
    t = rng.standard_normal((B, C, H, W)).astype(np.float32)
    w = (rng.random(B) + 0.5).astype(np.float32)
    loss, g = net.loss_grad(dev(x), dev(t), dev(w), want_grad=True)
    gg = host(g)
    x64, t64, w64 = x.astype(np.float64), t.astype(np.float64), w.astype(np.float64)
    ref_loss, ref_grads = cn.coarse_loss(x64, t64, w64, params)
    gref = np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in ref_grads])
    say("loss", loss, ref_loss, "grad relerr vs FP64 oracle", relerr(gg, gref))
    assert abs(loss - ref_loss) <= 2e-2 * abs(ref_loss)
    assert relerr(gg, gref) <= 5e-2
    # per layer against the same definition on BF16-rounded operands: tight
    emu = emulated_grads(x64, t64, w64, params)
    off = 0
    for l, ((gW, gb), (rW, rb)) in enumerate(zip(emu, ref_grads)):
        k = gW.size
        e1 = relerr(gg[off:off + k], gW.reshape(-1))
        e2 = relerr(gg[off + k:off + k + gb.size], gb)
        say("  layer", l, "W relerr (bf16-emulated)", e1, "b", e2, "W vs FP64", relerr(gg[off:off + k], rW.reshape(-1)))
        assert e1 <= 2e-3 and e2 <= 2e-3
        assert relerr(gg[off:off + k], rW.reshape(-1)) <= 0.2
        off += k + gb.size
    # one Adam step from zero moments: p - lr * g / (|g| + eps)
    p0 = pack(params)
    net.adam_step(1e-3)
    p1 = host(net.params())
    want, _, _ = cn.adam_step(p0.astype(np.float64), gg.astype(np.float64), 0.0, 0.0, 1, lr=1e-3)
    assert np.abs(p1 - want).max() <= 1e-6
    net.close()


def _to_ch(u, L):
    out = [u[L].real]
    for k in range(1, L + 1):
        out += [np.sqrt(2) * u[L + k].real, np.sqrt(2) * u[L + k].imag]
    return np.stack(out)


def _to_modes(c, L):
    n = c.shape[-1]
    u = np.zeros((2 * L + 1,) + c.shape[1:], complex)
    u[L] = c[0]
    for k in range(1, L + 1):
        z = (c[2 * k - 1] + 1j * c[2 * k]) / np.sqrt(2)
        u[L + k] = z
        u[L - k] = np.conj(z)
    return u


def test_make_pairs_matches_definition(rte):
    n, L, F = 16, 2, 4
    mu_a, mu_s = 0.05, 8.0
    sh = inputs.hg_sigma_hat(0.4, L)
    rng = np.random.default_rng(9)
    ctx = rte.Context(n, mu_a=mu_a, mu_s=mu_s, sigma_hat=sh, L=L, prec=rte.PREC_FP64)
    f = rng.random((n, n))
    h, mu_t = 1.0 / n, mu_a + mu_s
    b = op2.rhs(f, L, h, mu_t, method="direct")
    xstar = kr.solve_dense(op2.dense_A(n, n, L, h, mu_t, mu_s, sh), b.reshape(-1)).reshape(b.shape)
    xs = [inputs.random_conj_symmetric_modes(rng, L, n) * 0.01 for _ in range(3)]
    bc, xsc = _to_ch(b, L), _to_ch(xstar, L)
    it = np.stack([_to_ch(x, L) for x in xs])
    xo, to, wo = ctx.make_pairs(dev(bc), dev(xsc), dev(it), F)
    for j, x in enumerate(xs):
        r = _to_ch(b - op2.apply_direct(x, L, h, mu_t, mu_s, sh), L)
        e = xsc - it[j]
        Rr = cn.restrict(r, F)
        s = np.sqrt(np.mean(r ** 2))
        assert relerr(host(xo)[j], Rr / s) <= 1e-5
        assert relerr(host(to)[j], cn.restrict(e - r, F) / s) <= 1e-5
        assert abs(host(wo)[j] - F * F * s * s / np.sum(e ** 2)) <= 1e-5 * abs(host(wo)[j])
    ctx.close()


def test_learned_pc_reduces_iterations(rte):
    """Diffusion regime, 64^2, L = 2 (HG g = 0.3), mu_s = 50, mu_a = 0.01, 16^2 coarse grid: a
    network trained on pairs from 12 training sources (seeds 10000+) plus noise and multiscale
    pairs cuts FGMRES iterations on held-out sources (seeds 0-2) against plain GMRES and against
    FGMRES with the same network untrained, with the same true-residual tolerance met."""
    from paper_1802_03061_amd import pc_train
    n, L, F = 64, 2, 4
    ctx = rte.Context(n, mu_a=0.01, mu_s=50.0, sigma_hat=inputs.hg_sigma_hat(0.3, L), L=L, prec=rte.PREC_FP32)
    srcs = [inputs.workload("diff256", seed=10000 + s, n=n)["f"] for s in range(12)]
    x, t, w = pc_train.generate_pairs(ctx, srcs, F)
    say("pairs", x.shape)
    net, hist = pc_train.train(x, t, w, ctx.channels, steps=1500, batch=32, lr=1e-3, log_every=500)
    say("loss history", hist)
    untrained = rte.Net(ctx.channels, 32, 5, seed=1, use_bias=False)   # same shape, initial weights
    plain, pcd, raw = [], [], []
    for s in range(3):
        f = dev(inputs.workload("diff256", seed=s, n=n)["f"])
        ctx.attach_pc(None)
        _, i0 = ctx.solve(f, tol=1e-8)
        ctx.attach_pc(untrained.params(), factor=F)
        _, i2 = ctx.solve(f, tol=1e-8)
        ctx.attach_pc(net.params(), factor=F)
        _, i1 = ctx.solve(f, tol=1e-8)
        say("seed", s, "plain", i0["iterations"], "pc", i1["iterations"], "fallback", i1["pc_fallback"],
            "relres", i1["relres_true"], "untrained", i2["iterations"], "fallback", i2["pc_fallback"])
        assert i1["relres_true"] <= 1e-8 and i1["pc_fallback"] == 0
        assert i2["relres_true"] <= 1e-8
        plain.append(i0["iterations"]); pcd.append(i1["iterations"]); raw.append(i2["iterations"])
    assert np.mean(pcd) <= 0.8 * np.mean(plain)
    assert np.mean(pcd) < np.mean(raw)      # the gain is the training's, not the flexible method's
    ctx.close()
    net.close()
    untrained.close()


def test_broken_network_falls_back_to_plain_gmres(rte):
    n, L = 32, 1
    ctx = rte.Context(n, mu_a=0.1, mu_s=5.0, sigma_hat=inputs.hg_sigma_hat(0.5, L), L=L, prec=rte.PREC_FP32)
    net = rte.Net(ctx.channels, 32, 5, seed=1)
    bad = torch.full((net.nparam,), float("nan"), dtype=torch.float32, device="cuda")
    ctx.attach_pc(bad, factor=4)
    f = dev(inputs.centred_gaussian_source(n))
    u, info = ctx.solve(f, tol=1e-8)
    say("nan net:", info)
    assert info["pc_fallback"] == 1 and info["relres_true"] <= 1e-8
    huge = torch.full((net.nparam,), 50.0, dtype=torch.float32, device="cuda")
    ctx.attach_pc(huge, factor=4)
    u, info = ctx.solve(f, tol=1e-8)
    say("huge net:", info)
    assert info["relres_true"] <= 1e-8
    ctx.close()
    net.close()


def test_broken_network_in_the_last_step_of_a_cycle(rte):
    """Restart length 1: the network's non-finite output shows up in the last (only) step of the
    cycle, whose flags the host reads after the cycle end is already queued.  The queued update
    must leave x unchanged, and the solve falls back to plain GMRES and matches it."""
    n, L = 32, 1
    ctx = rte.Context(n, mu_a=1.0, mu_s=0.5, sigma_hat=inputs.hg_sigma_hat(0.5, L), L=L, prec=rte.PREC_FP32)
    ctx.set_opts(restart=1, max_cycles=200)
    f = dev(inputs.centred_gaussian_source(n))
    u_ref, info_ref = ctx.solve(f, tol=1e-8)
    net = rte.Net(ctx.channels, 32, 5, seed=1)
    bad = torch.full((net.nparam,), float("nan"), dtype=torch.float32, device="cuda")
    ctx.attach_pc(bad, factor=4)
    ctx.set_opts(restart=1, max_cycles=200)
    u, info = ctx.solve(f, tol=1e-8)
    say("nan net, restart 1:", info, "plain:", info_ref)
    assert info["pc_fallback"] == 1 and info["relres_true"] <= 1e-8
    assert np.isfinite(host(u)).all()
    assert relerr(host(u), host(u_ref)) <= 1e-7
    ctx.close()
    net.close()


@pytest.mark.parametrize("L,n,F", [(2, 32, 4), (4, 64, 8), (0, 48, 16), (1, 256, 4), (2, 128, 8), (1, 80, 4), (0, 60, 4)])
def test_pc_apply_matches_oracle(rte, L, n, F):
    """The attached preconditioner z = v + s P N(R v / s) (bilinear P) against the oracle."""
    say("pc apply", L, n, F)
    rng = np.random.default_rng(L + n)
    ctx = rte.Context(n, mu_a=0.1, mu_s=3.0, sigma_hat=inputs.hg_sigma_hat(0.5, L), L=L, prec=rte.PREC_FP32)
    net = rte.Net(ctx.channels, 32, 5, seed=L, use_bias=False)
    params = unpack(host(net.params()), ctx.channels, 32, 5)
    ctx.attach_pc(net.params(), factor=F)
    # a smooth field plus noise
    X, Y = inputs.cell_centres(n)
    v = np.stack([np.sin(np.pi * (c + 1) * X) * np.cos(np.pi * Y) for c in range(ctx.channels)])
    v = v + 0.1 * rng.standard_normal(v.shape)
    z = host(ctx.pc_apply(dev(v)))
    ref = cn.precondition(v, params, F)
    e = relerr(z - v, ref - v)
    say("  correction relerr", e)
    assert e <= 3e-2
    ctx.close()
    net.close()


@pytest.mark.parametrize("prec", [1, 0])
def test_fgmres_with_network_matches_lu(rte, prec):
    """Flexible GMRES with an attached (untrained, bias-free) network forms z_j = v_j + s P N(R v_j/s)
    inside the apply and updates x with V y plus one prolongation of the combined coarse outputs;
    whatever the network, the solution is the discrete system's: it matches the oracle's dense LU
    solution (32^2, L = 2, F = 4)."""
    say("fgmres vs LU prec", prec)
    from oracle import krylov as kr
    from oracle import operator2d as op2
    n, L, F = 32, 2, 4
    mu_a, mu_s = 0.1, 4.0
    sh = inputs.hg_sigma_hat(0.5, L)
    f = inputs.gaussian_mixture_source(n, inputs.gaussian_mixture_params(np.random.default_rng(7), 2))
    ctx = rte.Context(n, mu_a=mu_a, mu_s=mu_s, sigma_hat=sh, L=L, prec=prec)
    net = rte.Net(ctx.channels, 32, 5, seed=3, use_bias=False)
    scaled = net.params() * 0.05
    ctx.attach_pc(scaled, factor=F)
    u, info = ctx.solve(dev(f), tol=1e-11)
    say("  info", info)
    h, mu_t = 1.0 / n, mu_a + mu_s
    A = op2.dense_A(n, n, L, h, mu_t, mu_s, sh)
    b = op2.rhs(f, L, h, mu_t, method="direct")
    x = kr.solve_dense(A, b.reshape(-1)).reshape(b.shape)
    e = relerr(host(u), x)
    say("  vs LU", e)
    assert info["pc_used"] == 1 and info["pc_fallback"] == 0
    assert e <= 1e-9
    ctx.close()
    net.close()


@pytest.mark.timeout(900)
def test_learned_pc_diffusion_full_size(rte):
    """The diffusion-regime workload at full size (256^2, HG g = 0.3, L = 4, mu_s = 50,
    mu_a = 0.01): a network trained by the library (16^2 coarse grid, 12 training sources, noise and
    multiscale pairs) at least halves the iterations on held-out sources; the oracle's FP64 FFT
    apply confirms the true residual of preconditioned solutions, which are compared element by
    element with the oracle's FP64 reference solve."""
    from paper_1802_03061_amd import pc_train
    say("learned pc diff256")
    w = inputs.workload("diff256", seed=0)
    n, L = w["n"], w["L"]
    ctx = rte.Context(n, mu_a=w["mu_a"], mu_s=w["mu_s"], sigma_hat=w["sigma_hat"], L=L, prec=rte.PREC_FP32)
    F = pc_train.coarse_factor(n)
    net, meta = pc_train.train_for(ctx, range(10000, 10012), "diff256", F, steps=1500)
    say("  training", {k: meta[k] for k in ("pairs", "factor", "t_data_s", "t_train_s")}, meta["loss_history"])
    plain, pcd = [], []
    for s_ in range(3):
        f = dev(inputs.workload("diff256", seed=s_)["f"])
        ctx.attach_pc(None)
        _, i0 = ctx.solve(f, tol=1e-8)
        ctx.attach_pc(net.params(), factor=F)
        u, i1 = ctx.solve(f, tol=1e-8)
        say(f"  seed {s_}: plain {i0['iterations']} it {i0['t_solve_ms']:.2f} ms, pc {i1['iterations']} it "
            f"{i1['t_solve_ms']:.2f} ms, fallback {i1['pc_fallback']}")
        assert i1["pc_fallback"] == 0 and i1["relres_true"] <= 1e-8
        plain.append(i0["iterations"]); pcd.append(i1["iterations"])
    assert np.mean(pcd) <= 0.5 * np.mean(plain)
    ref = oracle_ref.workload_2d("diff256", 0)
    say(f"  oracle reference: {ref.iterations} iterations, residual {ref.relres:.2e}, {ref.seconds:.1f} s")
    for tol in (1e-8, 1e-10):
        u, info = ctx.solve(dev(w["f"]), tol=tol)
        uu = host(u)
        rr = ref.residual(uu)
        e = relerr(uu, ref.u)
        say(f"  preconditioned solve to {tol:.0e}: {info['iterations']} it, relerr vs oracle {e:.3e}, "
            f"oracle true residual {rr:.3e}")
        assert info["pc_used"] == 1 and info["pc_fallback"] == 0
        assert rr <= 1.5 * tol
        assert e <= 1e-6
    ctx.close()
    net.close()


def _oracle_fgmres_iterates(matvec, precond, b, k):
    """The first k iterates of flexible GMRES from x0 = 0 (right preconditioning z_j = precond(v_j),
    modified Gram-Schmidt, x_i = Z_i y_i with y_i the least-squares solution of the Hessenberg
    system), written out from the definition."""
    beta = np.linalg.norm(b)
    V, Z = [b / beta], []
    H = np.zeros((k + 1, k))
    xs = []
    for j in range(k):
        z = precond(V[j])
        Z.append(z)
        w = matvec(z)
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w).real
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j])
        e1 = np.zeros(j + 2)
        e1[0] = beta
        y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
        xs.append(sum(y[i] * Z[i] for i in range(j + 1)))
    return xs


@pytest.mark.parametrize("prec,n,basis32", [(1, 32, 0), (0, 32, 0), (0, 32, 1), (1, 160, 0)])
def test_fgmres_iterates_match_oracle(rte, prec, n, basis32):
    """The first flexible-GMRES iterates with the attached network, from the single Gram-Schmidt
    pass whose update also normalises and restricts v_{j+1} for the network (reorth 0), and from
    the separate passes (reorth 2): the two agree closely, and both follow the oracle's flexible
    GMRES with z_j = v_j + s P N(R v_j / s), within the BF16 network's accuracy (L = 2, F = 4:
    an 8^2 coarse grid takes the single-workgroup network kernel, 40^2 the per-layer kernels).
    basis32: the FP32 apply's basis stored in FP32."""
    L, F, k = 2, 4, 4
    mu_a, mu_s = 0.1, 4.0
    h, mu_t = 1.0 / n, mu_a + mu_s
    sh = inputs.hg_sigma_hat(0.5, L)
    f = inputs.gaussian_mixture_source(n, inputs.gaussian_mixture_params(np.random.default_rng(11), 2))
    ctx = rte.Context(n, mu_a=mu_a, mu_s=mu_s, sigma_hat=sh, L=L, prec=prec)
    net = rte.Net(ctx.channels, 32, 5, seed=5, use_bias=False)
    w = net.params() * 0.3
    params = unpack(host(w), ctx.channels, 32, 5)
    ctx.attach_pc(w, factor=F)
    # the direct sum costs N^2 (minutes at 160^2); the FFT form is pinned to it by the oracle tests
    b = op2.rhs(f, L, h, mu_t, method="direct" if n <= 32 else "fft")
    bc = _to_ch(b, L)
    recs = {}
    for reorth in (0, 2):
        ctx.set_opts(reorth=reorth, basis_fp32=basis32)
        _, info, rec = ctx.solve_rhs(dev(bc), tol=1e-11, record=k)
        say("  reorth", reorth, info)
        assert info["pc_used"] == 1 and info["pc_fallback"] == 0 and rec.shape[0] == k
        recs[reorth] = host(rec)
    spectra = op2.kernel_spectra(n, n, L, h, mu_t)
    matvec = lambda v: _to_ch(op2.apply_fft(_to_modes(v, L), L, h, mu_t, mu_s, sh, spectra=spectra), L)
    xs = _oracle_fgmres_iterates(matvec, lambda v: cn.precondition(v, params, F), bc, k)
    for i in range(k):
        d_paths = relerr(recs[0][i], recs[2][i])
        d_oracle = max(relerr(recs[0][i], xs[i]), relerr(recs[2][i], xs[i]))
        say("  iterate", i + 1, "fused vs separate", d_paths, "vs oracle", d_oracle)
        assert d_paths <= 1e-4
        assert d_oracle <= 3e-2
    ctx.close()
    net.close()


@pytest.mark.parametrize("n,L,F,basis32,rescale", [(64, 2, 4, 0, 0), (64, 2, 4, 1, 0), (64, 8, 8, 0, 0),
                                                   (160, 2, 8, 0, 0), (512, 8, 32, 0, 0), (64, 2, 4, 0, 1),
                                                   (512, 8, 32, 0, 1)])
def test_early_pass_a_matches_oracle(rte, monkeypatch, n, L, F, basis32, rescale):
    """FP32 apply: the stage-1 launch of each preconditioned Arnoldi step also runs the next apply's
    pass A on v_{j+1} alone, and pass B adds the x-spectrum of the coarse correction (the x-FFT is
    linear, and the bilinear prolongation separates into x and y parts), so the apply still takes
    z_j = v_j + s P N(R v_j / s).  The first iterates agree with the path that adds the correction
    before pass A (RTE_PC_EARLY_A=0) to FP32 rounding and follow the oracle's flexible GMRES within
    the BF16 network's accuracy; full solves of both paths agree with each other.  Padded x 128,
    512 (n = 160, 20^2 coarse grid) and 1024 (n = 512, where each wave of pass B forms the
    correction of its own transforms); L = 8 takes 17 channels.  rescale: RTE_RENORM_TOL=-1 makes
    every step rescale its new vector, so the stage-1 launch folds the factor into pass A and
    rescales each tile after transforming it."""
    k = 4
    mu_a, mu_s = 0.1, 4.0
    h, mu_t = 1.0 / n, mu_a + mu_s
    sh = inputs.hg_sigma_hat(0.5, L)
    f = inputs.gaussian_mixture_source(n, inputs.gaussian_mixture_params(np.random.default_rng(13), 2))
    ctx = rte.Context(n, mu_a=mu_a, mu_s=mu_s, sigma_hat=sh, L=L, prec=0)
    net = rte.Net(ctx.channels, 32, 5, seed=9, use_bias=False)
    w = net.params() * 0.3
    params = unpack(host(w), ctx.channels, 32, 5)
    ctx.attach_pc(w, factor=F)
    ctx.set_opts(basis_fp32=basis32)
    b = op2.rhs(f, L, h, mu_t, method="fft")
    bc = _to_ch(b, L)
    if rescale:
        monkeypatch.setenv("RTE_RENORM_TOL", "-1")
    recs, sols = {}, {}
    for early in ("1", "0"):
        monkeypatch.setenv("RTE_PC_EARLY_A", early)
        say("early pass A", early, "n", n, "L", L, "F", F, "basis32", basis32)
        _, info, rec = ctx.solve_rhs(dev(bc), tol=1e-11, record=k)
        assert info["pc_used"] == 1 and info["pc_fallback"] == 0 and rec.shape[0] == k
        recs[early] = host(rec)
        u, info = ctx.solve_rhs(dev(bc), tol=1e-10)[:2]
        say("  solve", info["iterations"], info["relres_true"])
        assert info["pc_fallback"] == 0 and info["relres_true"] <= 1e-10
        sols[early] = host(u)
    spectra = op2.kernel_spectra(n, n, L, h, mu_t)
    matvec = lambda v: _to_ch(op2.apply_fft(_to_modes(v, L), L, h, mu_t, mu_s, sh, spectra=spectra), L)
    xs = _oracle_fgmres_iterates(matvec, lambda v: cn.precondition(v, params, F), bc, k)
    for i in range(k):
        d_paths = relerr(recs["1"][i], recs["0"][i])
        d_oracle = relerr(recs["1"][i], xs[i])
        say("  iterate", i + 1, "early vs late", d_paths, "vs oracle", d_oracle)
        assert d_paths <= 1e-4
        assert d_oracle <= 3e-2
    d = relerr(sols["1"], sols["0"])
    say("  solutions early vs late", d)
    assert d <= 1e-8
    ctx.close()
    net.close()


def test_gather_rows_and_upsample_match_torch_cpu(rte):
    """The two training-data kernels against PyTorch CPU references: the minibatch gather against
    indexing, and the bilinear upsampling at cell centres against F.interpolate (bilinear,
    align_corners=False), including non-integer ratios and a 1-cell source."""
    rng = np.random.default_rng(5)
    src = rng.standard_normal((10, 3, 4, 5)).astype(np.float32)
    idx = np.array([3, 0, 9, 3, 7], dtype=np.int32)
    got = host(rte.gather_rows(dev(src), dev(idx)))
    assert np.array_equal(got, src[idx])
    lib = rte.load()
    import ctypes
    s = dev(src)
    i = dev(idx)
    p = ctypes.c_void_p(s.data_ptr())
    assert lib.rte_nn_gather_rows(p, 10, 60, ctypes.c_void_p(i.data_ptr()), 5, ctypes.c_void_p(s.data_ptr() + 64),
                                  None) == rte.RTE_EINVAL      # dst overlaps src
    import torch.nn.functional as Fn
    for (hc, wc, ny, nx) in [(4, 6, 16, 24), (4, 6, 9, 13), (1, 1, 5, 7), (8, 8, 8, 8), (3, 5, 64, 32)]:
        c = rng.standard_normal((2, 3, hc, wc))
        ref = Fn.interpolate(torch.from_numpy(c), size=(ny, nx), mode="bilinear", align_corners=False).numpy()
        got = host(rte.upsample_bilinear(dev(c), ny, nx))
        e = float(np.abs(got - ref).max())
        say("upsample", hc, wc, ny, nx, "max abs err", e)
        assert e <= 1e-14
