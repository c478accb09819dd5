"""Training of the learned coarse-grid preconditioner (orchestration only).

Every numerical step runs in librte.so: the solves that produce GMRES iterates, the FP64
residual applies, restriction and normalisation of the training pairs (rte_pc_make_pairs), the
network's forward and backward passes and Adam (rte_nn_*).  This module only sequences the calls:

  1. for each training source f_s: b = K~ g(f_s); x* = GMRES to 1e-12; the iterates x_j of a
     plain GMRES cycle to `rec_tol` are recorded; pairs (R r_j/s, R(e_j - r_j)/s, F^2 s^2/|e_j|^2)
  2. minibatch Adam on mean_b w_b |N(x_b) - t_b|^2 over the pairs
  3. the packed FP32 parameters are returned (and can be saved with their metadata).
"""
from __future__ import annotations

import json
import time

import numpy as np
import torch

from . import inputs, rte


def generate_pairs(ctx: "rte.Context", sources, factor: int, rec_tol: float = 1e-8, max_record: int = 80,
                   tol_star: float = 1e-12):
    xs, ts, ws = [], [], []
    for f in sources:
        fd = torch.as_tensor(f, dtype=torch.float64).cuda().contiguous()
        b = ctx.rhs(fd, layout=rte.LAYOUT_CHANNELS)
        x_star, _ = ctx.solve_rhs(b, tol=tol_star, max_iter=4000)
        _, _, rec = ctx.solve_rhs(b, tol=rec_tol, max_iter=4000, record=max_record)
        if rec.shape[0] == 0:
            continue
        x, t, w = ctx.make_pairs(b, x_star, rec, factor)
        xs.append(x); ts.append(t); ws.append(w)
    return torch.cat(xs), torch.cat(ts), torch.cat(ws)


def train(x, t, w, channels, hidden=32, layers=5, steps=2000, batch=32, lr=1e-3, seed=0, log_every=0):
    torch.manual_seed(seed)
    net = rte.Net(channels, hidden, layers, seed=seed)
    n = x.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    for step in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), generator=g).cuda()
        xb, tb, wb = x[idx].contiguous(), t[idx].contiguous(), w[idx].contiguous()
        loss = net.loss_grad(xb, tb, wb)
        net.adam_step(lr)
        if log_every and step % log_every == 0:
            hist.append((step, loss))
    return net, hist


def workload_sources(name: str, seeds, n=None):
    return [inputs.workload(name, seed=s, n=n)["f"] for s in seeds]


def train_for(ctx: "rte.Context", train_seeds, workload: str, factor: int, n=None, hidden=32, layers=5,
              steps=2000, batch=32, lr=1e-3, seed=0):
    """Generate pairs on ctx's problem from the workload's training sources and train a network.
    Returns (net, meta)."""
    t0 = time.perf_counter()
    x, t, w = generate_pairs(ctx, workload_sources(workload, train_seeds, n), factor)
    t1 = time.perf_counter()
    net, hist = train(x, t, w, ctx.channels, hidden, layers, steps, batch, lr, seed)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    meta = {"pairs": int(x.shape[0]), "factor": factor, "hidden": hidden, "layers": layers, "steps": steps,
            "batch": batch, "lr": lr, "t_data_s": t1 - t0, "t_train_s": t2 - t1, "workload": workload,
            "train_seeds": [int(s) for s in train_seeds], "L": ctx.L}
    return net, meta


def save(path: str, net: "rte.Net", meta: dict):
    np.savez(path, params=net.params().cpu().numpy(), meta=json.dumps(meta))


def load_params(path: str):
    d = np.load(path, allow_pickle=False)
    return torch.from_numpy(d["params"]).cuda(), json.loads(str(d["meta"]))
