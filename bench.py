"""Benchmark: solve time to relative residual 1e-8 on the 512^2, L = 8 Henyey-Greenstein problem.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--mu-s 10] [--no-cpu-baseline]

One step = one full solve (right-hand side b = K~ g by an FP64 apply, then flexible GMRES with the
learned coarse-grid preconditioner, FP32 FFT applies, FP64 Krylov and FP64 true-residual
refinement) of a seeded Gaussian-mixture source (2D, 512^2 cells, HG g = 0.5 truncated to
|k| <= 8: 17 coupled modes, mu_a = 0.1).  The same solves without the preconditioner (plain GMRES)
are timed beside it.  The network is trained before timing by the library's own kernels on pairs
from training sources (seeds 10000+), disjoint from the timed sources (seeds 0..K-1).  Inputs are
resident in HBM before the timed region; each timed region is K solves bracketed by device
synchronisation.  Prints one JSON line.

Also reported: operator applies/s, per-pass apply times from HIP events on the context stream
with the HBM roofline of the dominant kernel, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "solve time to rel-res 1e-8 (512^2, L=8 HG), learned-PC vs plain; applies/s"


def apply_pass_bytes(n: int, L: int) -> dict:
    """Algorithmic HBM bytes of one FP32 apply on FP64 channel vectors (C = 2L+1 channels, n^2
    cells, x-spectrum of n+1 columns): pass A reads x (8 B/value) and writes the complex64
    x-spectrum; pass B reads and writes that spectrum and reads the quarter kernel spectra;
    pass C reads the spectrum and x and writes y."""
    C = 2 * L + 1
    N = n * n
    spec = C * (n + 1) * n * 8
    kern = (2 * L + 1) * (n + 1) * (n + 1) * 8
    return {"A": 8 * C * N + spec, "B": 2 * spec + kern, "C": spec + 16 * C * N}


def cpu_baseline(w, gpu_applies_per_solve: float) -> dict:
    """The oracle's FP64 FFT apply (scipy.fft, as written) timed on the host on a bounded sample:
    two applies of the same 512^2, L = 8 operator after its spectra are built; solves/s is scaled
    by the applies one GPU solve used."""
    from oracle import operator2d as op2
    n, L = w["n"], w["L"]
    h, mu_t = 1.0 / n, w["mu_a"] + w["mu_s"]
    t0 = time.perf_counter()
    spectra = op2.kernel_spectra(n, n, L, h, mu_t)
    t_pre = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    from paper_1802_03061_amd import inputs
    u = inputs.random_conj_symmetric_modes(rng, L, n)
    reps = 2
    t0 = time.perf_counter()
    for _ in range(reps):
        op2.apply_fft(u, L, h, mu_t, w["mu_s"], w["sigma_hat"], "A", spectra=spectra)
    t_apply = (time.perf_counter() - t0) / reps
    return {
        "value": 1.0 / (t_apply * gpu_applies_per_solve),
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{reps} FP64 FFT applies of the 512^2 L=8 operator (oracle.operator2d.apply_fft, "
                   f"numpy/scipy single thread) at {t_apply:.2f} s each, scaled by the "
                   f"{gpu_applies_per_solve:.1f} applies per GPU solve; spectra precompute "
                   f"{t_pre:.1f} s excluded"),
        "applies_per_s": 1.0 / t_apply,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mu-s", type=float, default=10.0)
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pc", action="store_true", help="time plain GMRES only")
    ap.add_argument("--train-steps", type=int, default=1500)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver has no multi-GPU "
              f"path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1802_03061_amd import inputs, rte

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    rank = int(os.environ.get("RANK", "0"))

    base = inputs.workload("hg512", seed=0, mu_s=args.mu_s)
    n, L = base["n"], base["L"]
    ctx = rte.Context(n, mu_a=base["mu_a"], mu_s=base["mu_s"], sigma_hat=base["sigma_hat"], L=L,
                      prec=rte.PREC_FP32)
    # seeded sources, resident on the device before timing
    nsrc = max(args.steps, 1)
    fs = [torch.from_numpy(inputs.workload("hg512", seed=s, mu_s=args.mu_s)["f"]).cuda()
          for s in range(nsrc)]
    torch.cuda.synchronize()

    def timed(label):
        for i in range(args.warmup):
            ctx.solve(fs[i % nsrc], tol=1e-8)
        torch.cuda.synchronize()
        infos = []
        t0 = time.perf_counter()
        for i in range(args.steps):
            _, info = ctx.solve(fs[i % nsrc], tol=1e-8)
            infos.append(info)
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t0) / args.steps
        return ms, {"label": label, "ms_per_solve": ms, "solves_per_s": 1000.0 / ms,
                    "iterations": float(np.mean([i["iterations"] for i in infos])),
                    "applies": float(np.mean([i["applies"] for i in infos])),
                    "cycles": float(np.mean([i["cycles"] for i in infos])),
                    "pc_fallback": int(max(i["pc_fallback"] for i in infos)),
                    "max_relres_true": float(max(i["relres_true"] for i in infos))}

    ms_plain, plain = timed("plain GMRES")
    t_setup_ms = ctx.solve(fs[0], tol=1e-8)[1]["t_setup_ms"]
    pc = None
    if not args.no_pc:
        from paper_1802_03061_amd import pc_train
        F = pc_train.coarse_factor(n)
        net, meta = pc_train.train_for(ctx, range(10000, 10012), "hg512", F, steps=args.train_steps,
                                       mu_s=args.mu_s)
        ctx.attach_pc(net.params(), hidden=meta["hidden"], layers=meta["layers"], factor=F)
        ms_pc, pc = timed("learned-PC FGMRES")
        pc["training"] = {k: meta[k] for k in ("pairs", "factor", "hidden", "layers", "steps", "t_data_s",
                                                "t_train_s", "noise_ratio", "multiscale_ratio", "use_bias")}
        pc["training"]["final_loss"] = meta["loss_history"][-1][1] if meta["loss_history"] else None
        ctx.attach_pc(None)
        net.close()
    head = pc if pc is not None else plain
    ms_per_step = head["ms_per_solve"]
    iters = head["iterations"]
    applies = plain["applies"]
    relres = head["max_relres_true"]

    # apply throughput and per-pass times (HIP events on the context stream)
    ms_apply, ms_pass = ctx.time_apply(rte.OP_A, rte.PREC_FP32, reps=args.apply_reps)
    ms_apply64, ms_pass64 = ctx.time_apply(rte.OP_A, rte.PREC_FP64, reps=max(5, args.apply_reps // 5))
    pb = apply_pass_bytes(n, L)
    names = ["A", "B", "C"]
    dom = int(np.argmax(ms_pass[:3]))
    dom_name = names[dom]
    achieved = pb[dom_name] / (ms_pass[dom] * 1e-3) / 1e9
    tot_bytes = sum(pb.values())

    out = {
        "metric": METRIC,
        "value": 1000.0 / ms_per_step,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 apply + f64 krylov",
        "data": "synthetic",
        "config": {"workload": f"2D HG g=0.5, L=8 (17 modes), 512^2 cells, mu_a=0.1, mu_s={args.mu_s:g}, "
                               f"seeded Gaussian-mixture sources, tol 1e-8 (true FP64 residual)",
                   "n": n, "L": L, "mu_s": args.mu_s, "tol": 1e-8,
                   "preconditioner": "learned coarse-grid CNN (FGMRES)" if pc else "none"},
        "solve": {"iterations": iters, "max_relres_true": relres, "t_setup_ms": t_setup_ms},
        "plain": plain,
        "learned_pc": pc,
        "pc_speedup_vs_plain": (plain["ms_per_solve"] / pc["ms_per_solve"]) if pc else None,
        "applies_per_s": 1000.0 / ms_apply,
        "apply_ms": {"fp32_total": ms_apply, "fp32_passes": dict(zip(names, ms_pass[:3])),
                     "fp64_total": ms_apply64, "fp64_passes": dict(zip(names, ms_pass64[:3]))},
        "apply_hbm_fraction": tot_bytes / (ms_apply * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "roofline": {"bound": "hbm", "kernel": f"apply pass {dom_name}", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None},
    }
    if rank == 0 and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(base, applies)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
