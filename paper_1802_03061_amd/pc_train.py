"""Training of the learned coarse-grid preconditioner (orchestration only).

Every numerical step runs in librte.so: the solves that produce GMRES iterates, the FP64
residual applies, restriction and normalisation of the training pairs (rte_pc_make_pairs), the
network's forward and backward passes and Adam (rte_nn_*).  This module only sequences the calls:

  1. for each training source f_s: b = K~ g(f_s); x* = GMRES to 1e-12; the iterates x_j of a
     plain GMRES cycle to `rec_tol` are recorded; pairs (R r_j/s, R(e_j - r_j)/s, F^2 s^2/|e_j|^2);
     plus pairs (A u, u) for white-noise u and for random fields u at every scale, which need no
     solve and cover the inputs flexible GMRES feeds the network (Arnoldi vectors, not residuals)
  2. minibatch Adam on mean_b w_b |N(x_b) - t_b|^2 over the pairs (bias-free network by default,
     so the preconditioner is positively homogeneous)
  3. the packed FP32 parameters are returned (and can be saved with their metadata).
"""
from __future__ import annotations

import json
import time

import numpy as np
import torch

from . import inputs, rte


def multiscale_fields(shape, count, gen, scales=(2, 4, 8, 16, 32, 64)):
    """Seeded random fields at every scale: coarse Gaussian noise on an m x m grid (the random
    numbers drawn by torch), bilinearly upsampled to the fine grid by the library, for m cycling
    through `scales`."""
    C, ny, nx = shape
    out = torch.empty((count, C, ny, nx), dtype=torch.float64, device="cuda")
    for i in range(count):
        m = scales[i % len(scales)]
        c = torch.randn((1, C, min(m, ny), min(m, nx)), dtype=torch.float64, device="cuda", generator=gen)
        out[i] = rte.upsample_bilinear(c, ny, nx)[0]
    return out


def generate_pairs(ctx: "rte.Context", sources, factor: int, rec_tol: float = 1e-8, max_record: int = 80,
                   tol_star: float = 1e-12, noise_ratio: float = 1.0, multiscale_ratio: float = 3.0,
                   seed: int = 0):
    """Pairs from plain GMRES iterates of the given sources, plus pairs (r, e) = (A u, u) that need
    no solve: noise_ratio times as many for white-noise u (rough inputs need little correction)
    and multiscale_ratio times as many for random fields at every scale.  The synthetic pairs pass
    the drawn field itself as the "iterate" (so e = -u, r = -A u): the draws are symmetric, so
    this is the same distribution of pairs."""
    xs, ts, ws = [], [], []
    gen = torch.Generator(device="cuda").manual_seed(seed)
    zero = torch.zeros(ctx.channel_shape, dtype=torch.float64, device="cuda")
    for f in sources:
        fd = torch.as_tensor(f, dtype=torch.float64).cuda().contiguous()
        b = ctx.rhs(fd, layout=rte.LAYOUT_CHANNELS)
        x_star, _ = ctx.solve_rhs(b, tol=tol_star, max_iter=4000)
        _, _, rec = ctx.solve_rhs(b, tol=rec_tol, max_iter=4000, record=max_record)
        if rec.shape[0] == 0:
            continue
        x, t, w = ctx.make_pairs(b, x_star, rec, factor)
        xs.append(x); ts.append(t); ws.append(w)
        k = int(round(noise_ratio * rec.shape[0]))
        if k > 0:
            u = torch.randn((k,) + tuple(ctx.channel_shape), dtype=torch.float64, device="cuda", generator=gen)
            x, t, w = ctx.make_pairs(zero, zero, u, factor)
            xs.append(x); ts.append(t); ws.append(w)
        k = int(round(multiscale_ratio * rec.shape[0]))
        if k > 0:
            u = multiscale_fields(tuple(ctx.channel_shape), k, gen)
            x, t, w = ctx.make_pairs(zero, zero, u, factor)
            xs.append(x); ts.append(t); ws.append(w)
    return torch.cat(xs), torch.cat(ts), torch.cat(ws)


def train(x, t, w, channels, hidden=32, layers=5, steps=2000, batch=32, lr=1e-3, seed=0, log_every=0,
          use_bias=False):
    torch.manual_seed(seed)
    net = rte.Net(channels, hidden, layers, seed=seed, use_bias=use_bias)
    n = x.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    for step in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), generator=g, dtype=torch.int32).cuda()
        xb, tb, wb = rte.gather_rows(x, idx), rte.gather_rows(t, idx), rte.gather_rows(w, idx)
        loss = net.loss_grad(xb, tb, wb)
        net.adam_step(lr)
        if log_every and step % log_every == 0:
            hist.append((step, loss))
    return net, hist


def coarse_factor(n: int, coarse: int = 16) -> int:
    """Coarsening factor giving a coarse grid of about `coarse` cells per side (a power of two
    dividing n)."""
    F = 1
    while n // (2 * F) >= coarse and n % (2 * F) == 0:
        F *= 2
    return F


def train_for(ctx: "rte.Context", train_seeds, workload: str, factor: int, n=None, hidden=32, layers=5,
              steps=1500, batch=32, lr=1e-3, seed=0, noise_ratio=1.0, multiscale_ratio=3.0, use_bias=False,
              mu_s=None):
    """Generate pairs on ctx's problem from the workload's training sources and train a network.
    Returns (net, meta)."""
    t0 = time.perf_counter()
    srcs = [inputs.workload(workload, seed=s, n=n, mu_s=mu_s)["f"] for s in train_seeds]
    x, t, w = generate_pairs(ctx, srcs, factor, noise_ratio=noise_ratio, multiscale_ratio=multiscale_ratio,
                             seed=seed)
    t1 = time.perf_counter()
    net, hist = train(x, t, w, ctx.channels, hidden, layers, steps, batch, lr, seed, use_bias=use_bias,
                      log_every=max(1, steps // 4))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    meta = {"pairs": int(x.shape[0]), "factor": factor, "hidden": hidden, "layers": layers, "steps": steps,
            "batch": batch, "lr": lr, "t_data_s": t1 - t0, "t_train_s": t2 - t1, "workload": workload,
            "train_seeds": [int(s) for s in train_seeds], "L": ctx.L, "noise_ratio": noise_ratio,
            "multiscale_ratio": multiscale_ratio, "use_bias": use_bias,
            "loss_history": [(int(a), float(b)) for a, b in hist]}
    return net, meta


def save(path: str, net: "rte.Net", meta: dict):
    np.savez(path, params=net.params().cpu().numpy(), meta=json.dumps(meta))


def load_params(path: str):
    d = np.load(path, allow_pickle=False)
    return torch.from_numpy(d["params"]).cuda(), json.loads(str(d["meta"]))
