"""Benchmark of the RTE solver on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload hg512|batched|iso3d|diff256|iso32|sh3d|modes|multi]

Default workload (hg512): solve time to relative residual 1e-8 on the 512^2, L = 8
Henyey-Greenstein problem.  One step = one full solve (right-hand side b = K~ g by an FP64 apply,
then flexible GMRES with the learned coarse-grid preconditioner, FP32 FFT applies, FP64 Krylov and
FP64 true-residual refinement) of a seeded Gaussian-mixture source (2D, 512^2 cells, HG g = 0.5
truncated to |k| <= 8: 17 coupled modes, mu_a = 0.1, mu_s = 10).  The same solves without the
preconditioner (plain GMRES) are timed beside it.  The network is trained before timing by the
library's own kernels on pairs from training sources (seeds 10000+), disjoint from the timed
sources (seeds 0..K-1).  Inputs are resident in HBM before the timed region; each timed region is
K solves bracketed by device synchronisation.  Prints one JSON line.

Other workloads (same JSON shape):
  batched  one step = one rte_solve_batched call over 128 isotropic problems (n drawn from
           {64, 128, 256, 512}, mu_s ~ U[0.5, 20], mu_a ~ U[0.01, 0.5]), FP32 apply, tol 1e-8
  iso3d    one step = one solve of the 128^3 isotropic problem (mu_a = 0.05, mu_s = 10), FP32
           FFT on the 256^3 padded grid, FP64 GMRES, tol 1e-8
  diff256  like hg512 on the diffusion-regime problem (256^2, HG g = 0.3, L = 4, mu_s = 50,
           mu_a = 0.01)
  iso32    the small isotropic problem (32^2, mu_a = 0.1, mu_s = 1, centred Gaussian), FP64
           throughout, tol 1e-10 (latency-bound)
  sh3d     one step = one solve of the 3D anisotropic problem in real spherical harmonics to
           degree 2 (9 modes), 64^3, HG g = 0.5, mu_a = 0.05, mu_s = 10, tol 1e-8
  modes    one step = one solve of a 2D problem with many modes (L = 16, 33 modes; the split
           pass B with the mode-axis FFT or the direct coupling, as tuned), 256^2, HG g = 0.9,
           mu_a = 0.05, mu_s = 10, tol 1e-8
  multi    one step = one rte_solve_multi call for 16 sources sharing one 256^2, L = 4 medium
           (HG g = 0.5, mu_a = 0.1, mu_s = 10), tol 1e-8 per source; value counts sources solved

Also reported: operator applies/s, per-pass apply times from HIP events on the context stream with
the HBM roofline of the dominant kernel, the measured copy bandwidth, the error of the GPU solution
against an FP64 reference solve of the CPU oracle, and the oracle itself timed on the host as the
CPU baseline (a solve of the same problem to the same tolerance, on a bounded sample for the batch).
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
FP32_VECTOR_PEAK_TFLOPS = 157.3
# without packed FP32 instructions (not used by this build): 256 CUs x 4 SIMDs x 16 lanes x
# 2 flops per FMA x 2.4 GHz
FP32_VECTOR_NONPACKED_TFLOPS = 78.6
METRIC = "solve time to rel-res 1e-8 (512^2, L=8 HG), learned-PC vs plain; applies/s"
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "hbm_traffic_hg512_L8.json")
# sources of the 2D apply kernels: counter readings are only reported while these are unchanged
APPLY_SOURCES = ["paper_1802_03061_amd/csrc/" + f for f in
                 ("apply2d.hip", "apply2d_b.hip", "apply2d.h", "apply2d_b.h", "apply2d_tile.h", "passb_split.h", "fft.h",
                  "common.h")]


def sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in APPLY_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pmc_summary(fetch_csv: str, write_csv: str, variants) -> dict:
    """Per-launch HBM traffic of the FP32 apply passes from two rocprofv3 --pmc runs (FETCH_SIZE and
    WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads for the 1 GiB device
    copy that copy_peak_gbs() performs (1 GiB read and 1 GiB written)."""
    import csv
    import collections

    def load(path):
        agg = collections.defaultdict(list)
        with open(path) as fh:
            for r in csv.DictReader(fh):
                agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return agg
    fe, wr = load(fetch_csv), load(write_csv)
    copy = "__amd_rocclr_copyBuffer"
    true_kib = float(2 ** 20)
    ff, fw = true_kib / max(fe[copy]), true_kib / max(wr[copy])
    out = {"fetch_factor": ff, "write_factor": fw, "passes": {}}
    # A, B, C: the apply on FP64 channel vectors that the apply timing runs; A_f32, C_f32: the same
    # passes on the FP32 basis vectors of the solver's inner iterations
    def targs(name):   # template arguments of a kernel name
        return name.split("(")[0].split("<", 1)[1].rstrip(">").split(", ")

    # passes A and C: template arguments T, PX, TR, threads, vector type (and, for A, whether the
    # coarse correction is staged); the apply timing runs the unstaged form
    for label, key, tv in (("A", "k_pass_a<float, 1024,", "double"), ("B", "k_pass_b_lds<float, 1024, 8,", None),
                           ("C", "k_pass_c<float, 1024,", "double"), ("A_f32", "k_pass_a<float, 1024,", "float"),
                           ("C_f32", "k_pass_c<float, 1024,", "float")):
        names = [k for k in fe if key in k and (tv is None or (targs(k)[4] == tv and targs(k)[5:] in ([], ["false"])))]
        if variants and label[0] in "AC":
            # row tile of the pinned variant (FP32: 16, 8, 32 or 4 rows for variants 0..3)
            tr = (16, 8, 32, 4)[variants["ABC".index(label[0])][0]]
            names = [k for k in names if f"<float, 1024, {tr}, 256," in k] or names
        if not names:
            continue
        name = max(names, key=lambda k: len(fe[k]))       # the variant the applies used most
        f_kib = sum(fe[name]) / len(fe[name])
        w_kib = sum(wr[name]) / len(wr[name])
        out["passes"][label] = {"kernel": name.split("(")[0], "dispatches": len(fe[name]), "fetch_kib": f_kib,
                                "write_kib": w_kib, "traffic_bytes": (f_kib * ff + w_kib * fw) * 1024}
    out["sources_sha256"] = sources_digest()
    out["kernel_variants_fp32"] = variants
    return out


def traffic_for(dom: str, variants):
    """Counter-measured bytes per launch of pass `dom`, or None when no summary exists for the
    current kernel sources and that pass's variant."""
    try:
        with open(TRAFFIC_JSON) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    q = "ABC".index(dom)
    stored = t.get("kernel_variants_fp32")
    if t.get("sources_sha256") != sources_digest() or not stored or stored[q][0] != variants[q][0]:
        return None
    p = t.get("passes", {}).get(dom)
    return p["traffic_bytes"] if p else None


def log(*a):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def padded(n: int) -> int:
    P = 16
    while P < 2 * n - 1:
        P *= 2
    return P


def apply_pass_bytes(n: int, L: int, vbytes: int = 8, cbytes: int = 8) -> dict:
    """Algorithmic HBM bytes of one 2D apply on channel vectors of vbytes per value (8: the FP64
    vectors of the API; 4: the solver's FP32 basis) with spectra of cbytes per complex value (8 for
    the FP32 apply, 16 for the FP64 apply) (C = 2L+1 channels, n^2 cells, padded size P, x-spectrum
    of P/2 packed columns): pass A reads x and writes the x-spectrum; pass B reads and writes that
    spectrum and reads the quarter kernel spectra [2L+1][P/2+1][P/2+1]; pass C reads the spectrum
    and x and writes y."""
    C = 2 * L + 1
    N = n * n
    H = padded(n) // 2
    spec = cbytes * C * H * n
    kern = cbytes * (2 * L + 1) * (H + 1) * (H + 1)
    return {"A": vbytes * C * N + spec, "B": 2 * spec + kern, "C": spec + 2 * vbytes * C * N}


def apply3d_pass_bytes(n: int) -> dict:
    """Algorithmic HBM bytes of one FP32 3D isotropic apply (n^3 cells, padded P): x-FFT pass
    (read x, write T1 [n][P/2+1][n] complex64), y-FFT pass (T1 -> T2 [P/2+1][P][n]), z pass (read
    and write T2, read the real octant spectrum), inverse y pass (T2 -> T1), inverse x pass (read
    T1 and x, write y)."""
    N = n ** 3
    P = padded(n)
    H = P // 2 + 1
    t1 = 8 * n * H * n
    t2 = 8 * H * P * n
    q = 4 * H * (P // 2 + 1) * (P // 2 + 1)
    return {"A": 8 * N + t1, "B": t1 + t2, "C": 2 * t2 + q, "D": t2 + t1, "E": t1 + 16 * N}


def apply_split_bytes(n: int, L: int, vbytes: int = 8, cbytes: int = 8) -> dict:
    """As apply_pass_bytes for the split pass B of many modes (L > 8): the x-spectrum has P/2+1
    unpacked columns, and pass B is three kernels over the full-length buffer [C][P/2+1][P]: the
    forward y-FFTs (read the spectrum, write the buffer), the mode coupling (read and write the
    buffer, read the quarter kernel spectra), the inverse y-FFTs (read the buffer, write the
    spectrum)."""
    C = 2 * L + 1
    N = n * n
    P = padded(n)
    NK = P // 2 + 1
    spec = cbytes * C * NK * n
    full = cbytes * C * NK * P
    kern = cbytes * C * NK * (P // 2 + 1)
    return {"A": vbytes * C * N + spec, "B": (spec + full) + (2 * full + kern) + (full + spec),
            "C": spec + 2 * vbytes * C * N}


def apply3d_sh_pass_bytes(n: int, L: int) -> dict:
    """Algorithmic HBM bytes of one FP32 3D apply with spherical harmonics to degree L: the
    isotropic passes for each of the M = (L+1)^2 channels, and in the z pass the real octant
    spectra of the M(M+1)/2 mode pairs."""
    M = (L + 1) ** 2
    iso = apply3d_pass_bytes(n)
    P = padded(n)
    H = P // 2 + 1
    q = 4 * H * (P // 2 + 1) * (P // 2 + 1)
    out = {k: M * v for k, v in iso.items()}
    out["C"] = M * (iso["C"] - q) + (M * (M + 1) // 2) * q
    return out


def copy_peak_gbs(torch, mib: int = 1024, reps: int = 10) -> float:
    """Measured device-to-device copy bandwidth (read + write bytes / time) of a plain copy of
    `mib` MiB, timed with events on torch's stream."""
    a = torch.empty(mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    e.synchronize()
    ms = s.elapsed_time(e) / reps
    del a, b
    return 2 * mib * 2 ** 20 / (ms * 1e-3) / 1e9


def roofline(ctx, rte, pb: dict, reps: int, names, prec=None) -> dict:
    """Per-pass apply times (HIP events on the context stream) and the dominant pass against
    8 TB/s; apply_hbm_fraction is the whole apply's algorithmic bytes over its time."""
    prec = rte.PREC_FP32 if prec is None else prec
    ms_apply, ms_pass = ctx.time_apply(rte.OP_A, prec, reps=reps)
    ms_pass = ms_pass[:len(names)]
    dom = int(np.argmax(ms_pass))
    achieved = pb[names[dom]] / (ms_pass[dom] * 1e-3) / 1e9
    return {"ms_apply": ms_apply, "passes": dict(zip(names, ms_pass)),
            "roofline": {"bound": "hbm", "kernel": f"apply pass {names[dom]}", "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "bytes_per_launch": pb[names[dom]], "ms_per_launch": ms_pass[dom]},
            "apply_hbm_fraction": sum(pb.values()) / (ms_apply * 1e-3) / 1e9 / HBM_PEAK_GBS}


# ------------------------------------------------------------------ the CPU oracle beside it ---

def oracle_threads() -> int:
    """Host threads given to the oracle's FFTs and mode sums: the host's cores, at most 16 (one
    GPU's share of the box)."""
    return max(1, min(16, os.cpu_count() or 1))


def host_cpu() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def relerr(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def oracle_2d(w, tol: float, gpu_u: dict) -> tuple:
    """The oracle's FP64 solve of the workload's seed-0 problem (oracle.operator2d FFT apply by
    circulant embedding inside oracle.krylov.gmres, on the host's threads): timed to the GPU
    solve's tolerance as the CPU baseline, then continued from scratch to 1e-13 as the reference
    that every GPU solution in gpu_u is compared with (relative L2 error over all modes).  Also
    one apply on a single thread."""
    from oracle import krylov as kr
    from oracle import operator2d as op2
    n, L = w["n"], w["L"]
    h, mu_t = 1.0 / n, w["mu_a"] + w["mu_s"]
    nt = oracle_threads()
    log("oracle: CPU baseline solve and reference solve", f"n={n} L={L}")
    t0 = time.perf_counter()
    spectra = op2.kernel_spectra(n, n, L, h, mu_t, workers=nt)
    t_pre = time.perf_counter() - t0
    apply = lambda u, k=nt: op2.apply_fft(u, L, h, mu_t, w["mu_s"], w["sigma_hat"], "A", spectra=spectra, workers=k)
    t0 = time.perf_counter()
    b = op2.rhs(w["f"], L, h, mu_t, spectra=spectra, workers=nt)
    x, hist = kr.gmres(apply, b, tol, 1000)
    t_sol = time.perf_counter() - t0
    log(f"oracle: baseline solve {t_sol:.1f} s, {len(hist) - 1} iterations; reference solve to 1e-13")
    t0 = time.perf_counter()
    apply(x, 1)
    t_apply1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    ref, rhist = kr.gmres(apply, b, 1e-13, 1000)
    t_ref = time.perf_counter() - t0
    nb = np.linalg.norm(b)
    cpu = {"value": 1.0 / t_sol, "unit": "solves/s", "cores": nt, "kind": "oracle",
           "sample": (f"one FP64 solve of the seed-0 source to relative residual {tol:g} "
                      f"(oracle.krylov.gmres over oracle.operator2d.apply_fft, {nt} threads): "
                      f"{len(hist) - 1} iterations, {t_sol:.2f} s; kernel spectra {t_pre:.2f} s excluded"),
           "t_pre_s": t_pre, "t_sol_s": t_sol, "iterations": len(hist) - 1,
           "relres_true": float(np.linalg.norm(b - apply(x)) / nb),
           "single_thread_apply_s": t_apply1, "host": host_cpu()}
    err = {"reference": {"what": "oracle FP64 GMRES over the FFT apply to 1e-13", "iterations": len(rhist) - 1,
                         "relres_true": float(np.linalg.norm(b - apply(ref)) / nb), "seconds": t_ref},
           "seed0_cpu_solve": relerr(x, ref)}
    for k, u in gpu_u.items():
        err[k] = relerr(u, ref)
        err[k + "_mode0"] = relerr(u[L], ref[L])
    return cpu, err


def oracle_3d(w, tol: float, gpu_u: dict) -> tuple:
    """As oracle_2d for the 3D isotropic problem (oracle.operator3d)."""
    from oracle import krylov as kr
    from oracle import operator3d as op3
    n = w["n"]
    h, mu_t = 1.0 / n, w["mu_a"] + w["mu_s"]
    nt = oracle_threads()
    log("oracle: CPU baseline solve and reference solve", f"n={n}")
    t0 = time.perf_counter()
    spec = op3.kernel_spectrum(n, n, n, h, mu_t, workers=nt)
    t_pre = time.perf_counter() - t0
    apply = lambda u, k=nt: op3.apply_fft(u, h, mu_t, w["mu_s"], "A", spectrum=spec, workers=k)
    t0 = time.perf_counter()
    b = op3.apply_fft(w["f"], h, mu_t, 0.0, "KT", spectrum=spec, workers=nt)
    x, hist = kr.gmres(apply, b, tol, 1000)
    t_sol = time.perf_counter() - t0
    log(f"oracle: baseline solve {t_sol:.1f} s, {len(hist) - 1} iterations; reference solve to 1e-13")
    t0 = time.perf_counter()
    apply(x, 1)
    t_apply1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    ref, rhist = kr.gmres(apply, b, 1e-13, 1000)
    t_ref = time.perf_counter() - t0
    nb = np.linalg.norm(b)
    cpu = {"value": 1.0 / t_sol, "unit": "solves/s", "cores": nt, "kind": "oracle",
           "sample": (f"one FP64 solve of the seed-0 source to relative residual {tol:g} "
                      f"(oracle.krylov.gmres over oracle.operator3d.apply_fft, {nt} threads): "
                      f"{len(hist) - 1} iterations, {t_sol:.2f} s; kernel spectrum {t_pre:.2f} s excluded"),
           "t_pre_s": t_pre, "t_sol_s": t_sol, "iterations": len(hist) - 1,
           "relres_true": float(np.linalg.norm(b - apply(x)) / nb),
           "single_thread_apply_s": t_apply1, "host": host_cpu()}
    err = {"reference": {"what": "oracle FP64 GMRES over the FFT apply to 1e-13", "iterations": len(rhist) - 1,
                         "relres_true": float(np.linalg.norm(b - apply(ref)) / nb), "seconds": t_ref},
           "seed0_cpu_solve": relerr(x, ref)}
    for k, u in gpu_u.items():
        err[k] = relerr(u, ref)
    return cpu, err


def oracle_3d_sh(w, tol: float, gpu_u: dict) -> tuple:
    """As oracle_2d for the 3D problem in spherical harmonics (oracle.operator3d_sh)."""
    from oracle import krylov as kr
    from oracle import operator3d_sh as o3s
    n, L = w["n"], w["L"]
    h, mu_t = 1.0 / n, w["mu_a"] + w["mu_s"]
    nt = oracle_threads()
    log("oracle: CPU baseline solve and reference solve", f"n={n} L={L}")
    t0 = time.perf_counter()
    sp = o3s.kernel_spectra(n, n, n, L, h, mu_t, workers=nt)
    t_pre = time.perf_counter() - t0
    apply = lambda u, k=nt: o3s.apply_fft(u, L, h, mu_t, w["mu_s"], w["sigma_hat"], "A", spectra=sp, workers=k)
    t0 = time.perf_counter()
    b = o3s.rhs(w["f"], L, h, mu_t, spectra=sp, workers=nt)
    x, hist = kr.gmres(apply, b, tol, 1000)
    t_sol = time.perf_counter() - t0
    log(f"oracle: baseline solve {t_sol:.1f} s, {len(hist) - 1} iterations; reference solve to 1e-13")
    t0 = time.perf_counter()
    ref, rhist = kr.gmres(apply, b, 1e-13, 1000)
    t_ref = time.perf_counter() - t0
    nb = np.linalg.norm(b)
    cpu = {"value": 1.0 / t_sol, "unit": "solves/s", "cores": nt, "kind": "oracle",
           "sample": (f"one FP64 solve of the seed-0 source to relative residual {tol:g} "
                      f"(oracle.krylov.gmres over oracle.operator3d_sh.apply_fft, {nt} threads): "
                      f"{len(hist) - 1} iterations, {t_sol:.2f} s; kernel spectra {t_pre:.2f} s excluded"),
           "t_pre_s": t_pre, "t_sol_s": t_sol, "iterations": len(hist) - 1,
           "relres_true": float(np.linalg.norm(b - apply(x)) / nb), "host": host_cpu()}
    err = {"reference": {"what": "oracle FP64 GMRES over the FFT apply to 1e-13", "iterations": len(rhist) - 1,
                         "relres_true": float(np.linalg.norm(b - apply(ref)) / nb), "seconds": t_ref},
           "seed0_cpu_solve": relerr(x, ref)}
    for k, u in gpu_u.items():
        err[k] = relerr(u, ref)
    return cpu, err


def timed_solves(ctx, fs, steps, warmup, torch, tol=1e-8):
    nsrc = len(fs)
    for i in range(warmup):
        ctx.solve(fs[i % nsrc], tol=tol)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(steps):
        _, info = ctx.solve(fs[i % nsrc], tol=tol)
        infos.append(info)
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / steps
    return {"ms_per_solve": ms, "solves_per_s": 1000.0 / ms,
            "iterations": float(np.mean([i["iterations"] for i in infos])),
            "applies": float(np.mean([i["applies"] for i in infos])),
            "cycles": float(np.mean([i["cycles"] for i in infos])),
            "pc_fallback": int(max(i["pc_fallback"] for i in infos)),
            "max_relres_true": float(max(i["relres_true"] for i in infos))}


def seed0_solution(ctx, f, tol=1e-8):
    """The GPU solution of the seed-0 source, as complex modes on the host (untimed)."""
    u, _ = ctx.solve(f, tol=tol)
    return u.cpu().numpy()


def scattering_timing(ctx, f, torch, ntheta: int = 64, reps: int = 20) -> dict:
    """The scattering term of a solved flux at ntheta angles (rte_scattering_term): wall time per
    call over `reps` back-to-back calls, against its algorithmic bytes (read the complex128 modes,
    write ntheta float64 values per cell)."""
    u, _ = ctx.solve(f, tol=1e-8)
    S = ctx.scattering_term(u, ntheta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.scattering_term(u, ntheta, out=S)
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / reps
    nbytes = u.numel() * 16 + S.numel() * 8
    return {"ntheta": ntheta, "ms": ms, "bytes": nbytes, "hbm_fraction": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def bench_pc_workload(args, torch, rte, name, mu_s):
    """hg512 / diff256: plain GMRES, then FGMRES with a freshly trained learned preconditioner."""
    from paper_1802_03061_amd import inputs, pc_train
    base = inputs.workload(name, seed=0, mu_s=mu_s)
    n, L = base["n"], base["L"]
    ctx = rte.Context(n, mu_a=base["mu_a"], mu_s=base["mu_s"], sigma_hat=base["sigma_hat"], L=L,
                      prec=rte.PREC_FP32)
    if args.force_variants:
        for q, v in enumerate(json.loads(args.force_variants)):
            ctx.set_variant(rte.PREC_FP32, q, int(v))
    fs = [torch.from_numpy(inputs.workload(name, seed=s, mu_s=mu_s)["f"]).cuda() for s in range(max(args.steps, 1))]
    torch.cuda.synchronize()
    plain = timed_solves(ctx, fs, args.steps, args.warmup, torch)
    plain["label"] = "plain GMRES"
    sols = {"plain": seed0_solution(ctx, fs[0])}
    t_setup_ms = ctx.solve(fs[0], tol=1e-8)[1]["t_setup_ms"]
    pc = None
    if not args.no_pc:
        F = pc_train.coarse_factor(n)
        net, meta = pc_train.train_for(ctx, range(10000, 10012), name, F, steps=args.train_steps, mu_s=mu_s)
        ctx.attach_pc(net.params(), hidden=meta["hidden"], layers=meta["layers"], factor=F)
        pc = timed_solves(ctx, fs, args.steps, args.warmup, torch)
        pc["label"] = "learned-PC FGMRES"
        sols["learned_pc"] = seed0_solution(ctx, fs[0])
        # the same solves with the inner basis stored in FP32 (FP64 sums; an option, not the default)
        ctx.set_opts(basis_fp32=1)
        pc32 = timed_solves(ctx, fs, args.steps, args.warmup, torch)
        sols["learned_pc_basis_fp32"] = seed0_solution(ctx, fs[0])
        ctx.set_opts()
        pc["basis_fp32_option"] = {k: pc32[k] for k in ("ms_per_solve", "solves_per_s", "iterations",
                                                          "max_relres_true")}
        pc["training"] = {k: meta[k] for k in ("pairs", "factor", "hidden", "layers", "steps", "t_data_s",
                                                "t_train_s", "noise_ratio", "multiscale_ratio", "use_bias")}
        pc["training"]["final_loss"] = meta["loss_history"][-1][1] if meta["loss_history"] else None
        ctx.attach_pc(None)
        net.close()
    head = pc if pc is not None else plain
    post = scattering_timing(ctx, fs[0], torch)
    rf = roofline(ctx, rte, apply_pass_bytes(n, L), args.apply_reps, ["A", "B", "C"])
    ms64, pass64 = ctx.time_apply(rte.OP_A, rte.PREC_FP64, reps=max(5, args.apply_reps // 5))
    variants = {name_: [list(ctx.get_variant(p, q)) for q in range(3)]
                for name_, p in (("fp32", rte.PREC_FP32), ("fp64", rte.PREC_FP64))}
    dom = rf["roofline"]["kernel"].split()[-1]
    if name == "hg512":
        rf["roofline"]["traffic"] = traffic_for(dom, variants["fp32"])
    # pass B is also arithmetic-heavy: FLOPs of its FFTs (5 N log2 N per complex transform, forward
    # and inverse, C channels per column) and of the mode coupling ((2L+1)^2 complex MACs per
    # frequency) against the FP32 vector peak
    P = padded(n)
    C = 2 * L + 1
    flops_b = 2 * C * (P // 2) * 5 * P * int(np.log2(P)) + (P // 2) * P * C * C * 8
    ach = flops_b / (rf["passes"]["B"] * 1e-3) / 1e12
    out = {
        "value": head["solves_per_s"], "unit": "solves/s", "ms_per_step": head["ms_per_solve"],
        "dtype": "f32 apply + f64 krylov",
        "config": {"workload": (f"2D HG g={'0.5' if name == 'hg512' else '0.3'}, L={L} ({2 * L + 1} modes), "
                                f"{n}^2 cells, mu_a={base['mu_a']:g}, mu_s={mu_s:g}, seeded Gaussian-mixture "
                                f"sources, tol 1e-8 (true FP64 residual)"),
                   "n": n, "L": L, "mu_s": mu_s, "tol": 1e-8,
                   "preconditioner": "learned coarse-grid CNN (FGMRES)" if pc else "none"},
        "solve": {"iterations": head["iterations"], "max_relres_true": head["max_relres_true"],
                  "t_setup_ms": t_setup_ms},
        "plain": plain, "learned_pc": pc,
        "pc_speedup_vs_plain": (plain["ms_per_solve"] / pc["ms_per_solve"]) if pc else None,
        "applies_per_s": 1000.0 / rf["ms_apply"],
        "apply_ms": {"fp32_total": rf["ms_apply"], "fp32_passes": rf["passes"], "fp64_total": ms64,
                     "fp64_passes": dict(zip("ABC", pass64[:3]))},
        "apply_hbm_fraction": rf["apply_hbm_fraction"], "apply_bytes": apply_pass_bytes(n, L),
        "kernel_variants": variants,
        "scattering_term": post,
        "roofline": rf["roofline"],
        "roofline_alu_pass_B": {"bound": "alu", "achieved": ach, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                "frac": ach / FP32_VECTOR_PEAK_TFLOPS, "flops": flops_b,
                                "peak_nonpacked": FP32_VECTOR_NONPACKED_TFLOPS,
                                "frac_nonpacked": ach / FP32_VECTOR_NONPACKED_TFLOPS},
    }
    return out, ctx, base, sols


def bench_batched(args, torch, rte, with_oracle: bool):
    from paper_1802_03061_amd import inputs
    probs = inputs.batched_problems(count=128, seed=3)
    ctxs = [rte.Context(p["n"], mu_a=p["mu_a"], mu_s=p["mu_s"], L=0, prec=rte.PREC_FP32) for p in probs]
    srcs = [inputs.gaussian_mixture_source(p["n"], p["params"]) for p in probs]
    fs = [torch.from_numpy(f).cuda() for f in srcs]
    torch.cuda.synchronize()
    tols = [1e-8] * len(ctxs)
    for _ in range(args.warmup):
        rte.solve_batched(ctxs, fs, tols)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        us, infos, _ = rte.solve_batched(ctxs, fs, tols)
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / args.steps
    its = [i["iterations"] for i in infos]
    cells = sum(p["n"] ** 2 for p in probs)
    # the batched apply of one inner iteration, launch by launch, against the aggregate algorithmic
    # bytes of the problems each launch covers (FP32 apply, FP64 basis vectors)
    ms_tot, launches = rte.time_batched_apply(ctxs, reps=args.apply_reps)
    lrows = []
    for ps, px, py, lms, var in launches:
        members = [p for p in probs if padded(p["n"]) == px]
        nbytes = sum(apply_pass_bytes(p["n"], 0)["ABC"[ps]] for p in members)
        lrows.append({"pass": "ABC"[ps], "padded": px, "problems": len(members), "variant": var, "ms": lms,
                      "bytes": nbytes, "GBs": nbytes / (lms * 1e-3) / 1e9})
    dom = max(lrows, key=lambda r: r["ms"])
    total_bytes = sum(r["bytes"] for r in lrows)
    out = {
        "value": len(ctxs) * 1000.0 / ms, "unit": "solves/s", "ms_per_step": ms, "dtype": "f32 apply + f64 krylov",
        "config": {"workload": ("128 batched 2D isotropic solves, n from {64,128,256,512}, mu_s~U[0.5,20], "
                                "mu_a~U[0.01,0.5], Gaussian-mixture sources, tol 1e-8"),
                   "problems": len(ctxs), "cells": cells, "tol": 1e-8},
        "solve": {"iterations_min": min(its), "iterations_max": max(its), "iterations_mean": float(np.mean(its)),
                  "max_relres_true": max(i["relres_true"] for i in infos),
                  "max_cycles": max(i["cycles"] for i in infos)},
        "applies_per_s": 1000.0 / ms_tot,
        "batched_apply": {"ms_total": ms_tot, "launches": lrows, "bytes": total_bytes,
                          "hbm_fraction": total_bytes / (ms_tot * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "roofline": {"bound": "hbm", "kernel": f"batched apply pass {dom['pass']} (padded {dom['padded']}, "
                                               f"{dom['problems']} problems)",
                     "achieved": dom["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom["GBs"] / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_launch": dom["bytes"], "ms_per_launch": dom["ms"]},
    }
    cpu = None
    if with_oracle:
        cpu, err = oracle_batched(probs, srcs, [u.cpu().numpy() for u in us])
        out["error_vs_oracle"] = err
    for c in ctxs:
        c.close()
    return out, cpu


def oracle_batched(probs, srcs, gpu_u) -> tuple:
    """CPU baseline on a bounded sample (the first 8 problems of the batch, each solved by the
    oracle to 1e-8 on the host's threads, scaled to solves/s), and the errors against FP64
    reference solves (1e-13) of the first and the hardest (largest mu_s / mu_t) problem of every
    grid size."""
    from oracle import krylov as kr
    from oracle import operator2d as op2
    nt = oracle_threads()
    one = np.ones(1)

    def setup(i):
        p = probs[i]
        n = p["n"]
        h, mu_t = 1.0 / n, p["mu_a"] + p["mu_s"]
        sp = op2.kernel_spectra(n, n, 0, h, mu_t, workers=nt)
        apply = lambda u: op2.apply_fft(u, 0, h, mu_t, p["mu_s"], one, "A", spectra=sp, workers=nt)
        return apply, lambda: op2.rhs(srcs[i], 0, h, mu_t, spectra=sp, workers=nt)
    sample = list(range(8))
    t_sol = 0.0
    its = []
    for i in sample:
        apply, rhs = setup(i)
        t0 = time.perf_counter()
        x, hist = kr.gmres(apply, rhs(), 1e-8, 1000)
        t_sol += time.perf_counter() - t0
        its.append(len(hist) - 1)
    cpu = {"value": len(sample) / t_sol, "unit": "solves/s", "cores": nt, "kind": "oracle",
           "sample": (f"the first {len(sample)} problems of the batch (n = "
                      f"{','.join(str(probs[i]['n']) for i in sample)}), each an FP64 oracle solve to 1e-8 "
                      f"(oracle.krylov.gmres over oracle.operator2d.apply_fft, {nt} threads): {t_sol:.2f} s in all, "
                      f"{sum(its)} iterations; kernel spectra excluded"),
           "t_sol_s": t_sol, "host": host_cpu()}
    check = set()
    for n in sorted({p["n"] for p in probs}):
        idx = [i for i, p in enumerate(probs) if p["n"] == n]
        if idx:
            check.add(idx[0])
            check.add(max(idx, key=lambda i: probs[i]["mu_s"] / (probs[i]["mu_s"] + probs[i]["mu_a"])))
    errs = {}
    for i in sorted(check):
        apply, rhs = setup(i)
        ref, _ = kr.gmres(apply, rhs(), 1e-13, 1000)
        errs[str(i)] = relerr(gpu_u[i], ref)
    err = {"reference": "oracle FP64 GMRES over the FFT apply to 1e-13, per problem",
           "problems": errs, "max": max(errs.values())}
    return cpu, err


def bench_iso3d(args, torch, rte, mu_s):
    from paper_1802_03061_amd import inputs
    w = inputs.workload("iso3d", seed=0, mu_s=mu_s)
    n = w["n"]
    ctx = rte.Context(n, dim=3, mu_a=w["mu_a"], mu_s=w["mu_s"], L=0, prec=rte.PREC_FP32)
    fs = [torch.from_numpy(inputs.workload("iso3d", seed=s, mu_s=mu_s)["f"]).cuda() for s in range(max(args.steps, 1))]
    torch.cuda.synchronize()
    r = timed_solves(ctx, fs, args.steps, args.warmup, torch)
    sols = {"gpu": seed0_solution(ctx, fs[0]).reshape(n, n, n).real}
    pb = apply3d_pass_bytes(n)
    rf = roofline(ctx, rte, pb, args.apply_reps, ["A", "B", "C", "D", "E"])
    out = {
        "value": r["solves_per_s"], "unit": "solves/s", "ms_per_step": r["ms_per_solve"],
        "dtype": "f32 apply + f64 krylov",
        "config": {"workload": f"3D isotropic {n}^3, mu_a={w['mu_a']:g}, mu_s={mu_s:g}, Gaussian-mixture sources, "
                               f"FP32 FFT on the {padded(n)}^3 padded grid, tol 1e-8", "n": n, "mu_s": mu_s},
        "solve": r, "applies_per_s": 1000.0 / rf["ms_apply"],
        "apply_ms": {"fp32_total": rf["ms_apply"], "fp32_passes": rf["passes"]},
        "apply_hbm_fraction": rf["apply_hbm_fraction"], "apply_bytes": pb, "roofline": rf["roofline"],
    }
    return out, ctx, w, sols


def bench_sh3d(args, torch, rte, mu_s):
    """3D anisotropic scattering in real spherical harmonics (degree 2, 9 modes), 64^3."""
    from paper_1802_03061_amd import inputs
    w = inputs.workload("sh3d", seed=0, mu_s=mu_s)
    n, L = w["n"], w["L"]
    ctx = rte.Context(n, dim=3, mu_a=w["mu_a"], mu_s=w["mu_s"], sigma_hat=w["sigma_hat"], L=L, prec=rte.PREC_FP32)
    fs = [torch.from_numpy(inputs.workload("sh3d", seed=s, mu_s=mu_s)["f"]).cuda() for s in range(max(args.steps, 1))]
    torch.cuda.synchronize()
    r = timed_solves(ctx, fs, args.steps, args.warmup, torch)
    sols = {"gpu": seed0_solution(ctx, fs[0]).real}
    pb = apply3d_sh_pass_bytes(n, L)
    rf = roofline(ctx, rte, pb, args.apply_reps, ["A", "B", "C", "D", "E"])
    out = {
        "value": r["solves_per_s"], "unit": "solves/s", "ms_per_step": r["ms_per_solve"],
        "dtype": "f32 apply + f64 krylov",
        "config": {"workload": (f"3D anisotropic {n}^3, HG g=0.5, real spherical harmonics to degree {L} "
                                f"({(L + 1) ** 2} modes), mu_a={w['mu_a']:g}, mu_s={mu_s:g}, Gaussian-mixture "
                                f"sources, FP32 FFT on the {padded(n)}^3 padded grid, tol 1e-8"),
                   "n": n, "L": L, "mu_s": mu_s},
        "solve": r, "applies_per_s": 1000.0 / rf["ms_apply"],
        "apply_ms": {"fp32_total": rf["ms_apply"], "fp32_passes": rf["passes"]},
        "apply_hbm_fraction": rf["apply_hbm_fraction"], "apply_bytes": pb, "roofline": rf["roofline"],
    }
    return out, ctx, w, sols


def bench_modes(args, torch, rte, mu_s):
    """2D with many modes (L = 16, 33 modes; the split pass B with the autotuner's choice of the
    mode-axis FFT or the direct coupling), 256^2."""
    from paper_1802_03061_amd import inputs
    w = inputs.workload("modes", seed=0, mu_s=mu_s)
    n, L = w["n"], w["L"]
    ctx = rte.Context(n, mu_a=w["mu_a"], mu_s=w["mu_s"], sigma_hat=w["sigma_hat"], L=L, prec=rte.PREC_FP32)
    fs = [torch.from_numpy(inputs.workload("modes", seed=s, mu_s=mu_s)["f"]).cuda() for s in range(max(args.steps, 1))]
    torch.cuda.synchronize()
    r = timed_solves(ctx, fs, args.steps, args.warmup, torch)
    sols = {"gpu": seed0_solution(ctx, fs[0])}
    pb = apply_split_bytes(n, L)
    rf = roofline(ctx, rte, pb, args.apply_reps, ["A", "B", "C"])
    coupling = {}
    vb, nvb = ctx.get_variant(rte.PREC_FP32, 1)
    for v in range(nvb):
        ctx.set_variant(rte.PREC_FP32, 1, v)
        coupling[("mode-axis FFT", "direct")[v]] = ctx.time_apply(rte.OP_A, rte.PREC_FP32, reps=args.apply_reps)[1][1]
    ctx.set_variant(rte.PREC_FP32, 1, vb)
    out = {
        "value": r["solves_per_s"], "unit": "solves/s", "ms_per_step": r["ms_per_solve"],
        "dtype": "f32 apply + f64 krylov",
        "config": {"workload": (f"2D HG g=0.9, L={L} ({2 * L + 1} modes), {n}^2 cells, mu_a={w['mu_a']:g}, "
                                f"mu_s={mu_s:g}, seeded Gaussian-mixture sources, tol 1e-8"),
                   "n": n, "L": L, "mu_s": mu_s},
        "solve": r, "applies_per_s": 1000.0 / rf["ms_apply"],
        "apply_ms": {"fp32_total": rf["ms_apply"], "fp32_passes": rf["passes"]},
        "pass_b_ms_by_coupling": coupling, "pass_b_coupling_chosen": ("mode-axis FFT", "direct")[vb],
        "apply_hbm_fraction": rf["apply_hbm_fraction"], "apply_bytes": pb, "roofline": rf["roofline"],
    }
    return out, ctx, w, sols


def bench_multi(args, torch, rte, with_oracle: bool, mu_s, nrhs: int = 16):
    """Several sources sharing one medium (rte_solve_multi: global GMRES on the stacked system, one
    batched apply per iteration), 16 sources on 256^2, L = 4; the single-source solver beside it."""
    from paper_1802_03061_amd import inputs
    w = inputs.workload("multi", seed=0, mu_s=mu_s)
    n, L = w["n"], w["L"]
    ctx = rte.Context(n, mu_a=w["mu_a"], mu_s=w["mu_s"], sigma_hat=w["sigma_hat"], L=L, prec=rte.PREC_FP32)
    srcs = [inputs.workload("multi", seed=s, mu_s=mu_s)["f"] for s in range(nrhs)]
    fs = [torch.from_numpy(f).cuda() for f in srcs]
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        ctx.solve_multi(fs, tol=1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        us, infos, _ = ctx.solve_multi(fs, tol=1e-8)
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / args.steps
    single = timed_solves(ctx, fs, nrhs, 1, torch)
    per = apply_pass_bytes(n, L)
    C = 2 * L + 1
    H = padded(n) // 2
    kern = 8 * C * (H + 1) * (H + 1)
    pb = {"A": nrhs * per["A"], "B": nrhs * (per["B"] - kern) + kern, "C": nrhs * per["C"]}
    ms_apply, ms_pass = ctx.time_apply_multi(nrhs, rte.OP_A, rte.PREC_FP32, reps=max(5, args.apply_reps // 5))
    dom = int(np.argmax(ms_pass[:3]))
    ach = pb["ABC"[dom]] / (ms_pass[dom] * 1e-3) / 1e9
    out = {
        "value": nrhs * 1000.0 / ms, "unit": "solves/s", "ms_per_step": ms, "dtype": "f32 apply + f64 krylov",
        "config": {"workload": (f"{nrhs} Gaussian-mixture sources sharing one 2D medium: {n}^2 cells, HG g=0.5, "
                                f"L={L} ({C} modes), mu_a={w['mu_a']:g}, mu_s={mu_s:g}, tol 1e-8 per source"),
                   "n": n, "L": L, "sources": nrhs, "mu_s": mu_s},
        "solve": {"stacked_iterations": infos[0]["iterations"],
                  "max_relres_true": max(i["relres_true"] for i in infos)},
        "single_source_solver": {"ms_for_all": single["ms_per_solve"] * nrhs,
                                 "solves_per_s": single["solves_per_s"], "iterations": single["iterations"]},
        "batched_apply_ms": {"total": ms_apply, "passes": dict(zip("ABC", ms_pass[:3]))},
        "roofline": {"bound": "hbm", "kernel": f"batched apply pass {'ABC'[dom]} ({nrhs} sources)", "achieved": ach,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": pb["ABC"[dom]], "ms_per_launch": ms_pass[dom]},
        "apply_hbm_fraction": sum(pb.values()) / (ms_apply * 1e-3) / 1e9 / HBM_PEAK_GBS,
    }
    cpu = None
    if with_oracle:
        from oracle import krylov as kr
        from oracle import operator2d as op2
        h, mu_t = 1.0 / n, w["mu_a"] + w["mu_s"]
        nt = oracle_threads()
        sp = op2.kernel_spectra(n, n, L, h, mu_t, workers=nt)
        apply = lambda u: op2.apply_fft(u, L, h, mu_t, w["mu_s"], w["sigma_hat"], "A", spectra=sp, workers=nt)
        sample = [0, 1]
        t_sol, its, errs = 0.0, [], {}
        for s in sample:
            b = op2.rhs(srcs[s], L, h, mu_t, spectra=sp, workers=nt)
            t0 = time.perf_counter()
            x, hist = kr.gmres(apply, b, 1e-8, 1000)
            t_sol += time.perf_counter() - t0
            its.append(len(hist) - 1)
            ref, _ = kr.gmres(apply, b, 1e-13, 1000)
            errs[str(s)] = relerr(us[s].cpu().numpy(), ref)
        cpu = {"value": len(sample) / t_sol, "unit": "solves/s", "cores": nt, "kind": "oracle",
               "sample": (f"sources {sample} of the {nrhs}, each an FP64 oracle solve to 1e-8 (oracle.krylov.gmres "
                          f"over oracle.operator2d.apply_fft, {nt} threads): {t_sol:.2f} s, {sum(its)} iterations; "
                          f"kernel spectra excluded"), "t_sol_s": t_sol, "host": host_cpu()}
        out["error_vs_oracle"] = {"reference": "oracle FP64 GMRES over the FFT apply to 1e-13, per source",
                                  "sources": errs, "max": max(errs.values())}
    ctx.close()
    return out, cpu


def bench_iso32(args, torch, rte, with_oracle: bool):
    """The small isotropic problem in FP64 to 1e-10: every step solves the same deterministic
    source; the reference is the oracle's dense LU solution."""
    from paper_1802_03061_amd import inputs
    w = inputs.workload("iso32")
    n = w["n"]
    ctx = rte.Context(n, mu_a=w["mu_a"], mu_s=w["mu_s"], L=0, prec=rte.PREC_FP64)
    fs = [torch.from_numpy(w["f"]).cuda()]
    torch.cuda.synchronize()
    r = timed_solves(ctx, fs, args.steps, args.warmup, torch, tol=1e-10)
    u = seed0_solution(ctx, fs[0], tol=1e-10)
    rf = roofline(ctx, rte, apply_pass_bytes(n, 0, 8, 16), args.apply_reps, ["A", "B", "C"], prec=rte.PREC_FP64)
    out = {
        "value": r["solves_per_s"], "unit": "solves/s", "ms_per_step": r["ms_per_solve"], "dtype": "f64",
        "config": {"workload": "2D isotropic 32^2, mu_a=0.1, mu_s=1, centred Gaussian source (width 0.1), FP64, "
                               "tol 1e-10 (latency-bound)", "n": n, "tol": 1e-10},
        "solve": r, "applies_per_s": 1000.0 / rf["ms_apply"],
        "apply_ms": {"fp64_total": rf["ms_apply"], "fp64_passes": rf["passes"]},
        "apply_hbm_fraction": rf["apply_hbm_fraction"], "roofline": rf["roofline"],
    }
    ctx.close()
    cpu = None
    if with_oracle:
        from oracle import krylov as kr
        from oracle import operator2d as op2
        h, mu_t = 1.0 / n, w["mu_a"] + w["mu_s"]
        A = op2.dense_A(n, n, 0, h, mu_t, w["mu_s"], w["sigma_hat"])
        b = op2.rhs(w["f"], 0, h, mu_t, method="direct")
        ref = kr.solve_dense(A, b.reshape(-1)).reshape(b.shape)
        out["error_vs_oracle"] = {"reference": "oracle dense LU", "gpu": relerr(u, ref)}
        sp = op2.kernel_spectra(n, n, 0, h, mu_t)
        apply = lambda x: op2.apply_fft(x, 0, h, mu_t, w["mu_s"], w["sigma_hat"], "A", spectra=sp, workers=1)
        reps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 5.0:
            x, hist = kr.gmres(apply, op2.rhs(w["f"], 0, h, mu_t, spectra=sp), 1e-10, 1000)
            reps += 1
        t = (time.perf_counter() - t0) / reps
        cpu = {"value": 1.0 / t, "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": (f"{reps} FP64 oracle solves to 1e-10 (oracle.krylov.gmres over oracle.operator2d.apply_fft, "
                          f"one thread), {len(hist) - 1} iterations each; kernel spectra excluded"),
               "t_sol_s": t, "host": host_cpu()}
    return out, cpu


def solves_only(args, torch, rte):
    """Preconditioned solves alone, after a pause that separates them from the setup in a trace."""
    from paper_1802_03061_amd import inputs, pc_train
    if args.workload not in ("hg512", "diff256"):
        raise SystemExit("--solves-only takes --workload hg512 or diff256")
    mu_s = args.mu_s if args.mu_s is not None else (10.0 if args.workload == "hg512" else 50.0)
    w = inputs.workload(args.workload, seed=0, mu_s=mu_s)
    n, L = w["n"], w["L"]
    ctx = rte.Context(n, mu_a=w["mu_a"], mu_s=w["mu_s"], sigma_hat=w["sigma_hat"], L=L, prec=rte.PREC_FP32)
    fs = [torch.from_numpy(inputs.workload(args.workload, seed=s, mu_s=mu_s)["f"]).cuda()
          for s in range(max(args.steps, 2))]
    F = pc_train.coarse_factor(n)
    net, meta = pc_train.train_for(ctx, range(10000, 10012), args.workload, F, steps=args.train_steps, mu_s=mu_s)
    ctx.attach_pc(net.params(), hidden=meta["hidden"], layers=meta["layers"], factor=F)
    for i in range(2):
        ctx.solve(fs[i])
    torch.cuda.synchronize()
    time.sleep(0.3)
    r = timed_solves(ctx, fs, args.steps, 0, torch)
    ctx.close()
    net.close()
    return {"workload": args.workload, "solves": args.steps, **r}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="hg512",
                    choices=["hg512", "batched", "iso3d", "diff256", "iso32", "sh3d", "modes", "multi"])
    ap.add_argument("--mu-s", type=float, default=None)
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle (its timed solve and the reference solve for the error)")
    ap.add_argument("--no-pc", action="store_true", help="time plain GMRES only")
    ap.add_argument("--train-steps", type=int, default=1500)
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the per-launch HBM traffic summary of the hg512 apply passes from two "
                         "rocprofv3 --pmc counter_collection.csv files (FETCH_SIZE, WRITE_SIZE) and exit; "
                         "--variants gives the FP32 kernel variants of those runs")
    ap.add_argument("--variants", default=None, help="JSON list of [variant, count] for passes A, B, C")
    ap.add_argument("--force-variants", default=None,
                    help="JSON list of the FP32 kernel variants of passes A, B, C to use instead of the tuned ones")
    ap.add_argument("--solves-only", action="store_true",
                    help="hg512 / diff256 for a kernel trace of the solves alone: train the preconditioner, "
                         "run 2 untimed solves, pause 0.3 s (a gap that marks the timed region in the trace), "
                         "then --steps timed preconditioned solves; prints their time and exits")
    args = ap.parse_args()
    if args.pmc_summary:
        t = pmc_summary(args.pmc_summary[0], args.pmc_summary[1], json.loads(args.variants) if args.variants else None)
        with open(TRAFFIC_JSON, "w") as fh:
            json.dump(t, fh, indent=1)
        print(json.dumps(t))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver has no multi-GPU "
              f"path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1802_03061_amd import rte

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    rank = int(os.environ.get("RANK", "0"))
    oracle_on = rank == 0 and not args.no_cpu_baseline
    cpu = None
    if args.solves_only:
        print(json.dumps(solves_only(args, torch, rte)), flush=True)
        return
    if args.workload in ("hg512", "diff256"):
        mu_s = args.mu_s if args.mu_s is not None else (10.0 if args.workload == "hg512" else 50.0)
        out, ctx, base, sols = bench_pc_workload(args, torch, rte, args.workload, mu_s)
        ctx.close()
        if oracle_on:
            cpu, out["error_vs_oracle"] = oracle_2d(base, 1e-8, sols)
    elif args.workload == "batched":
        out, cpu = bench_batched(args, torch, rte, oracle_on)
    elif args.workload == "iso32":
        out, cpu = bench_iso32(args, torch, rte, oracle_on)
    elif args.workload == "multi":
        out, cpu = bench_multi(args, torch, rte, oracle_on, args.mu_s if args.mu_s is not None else 10.0)
    elif args.workload == "sh3d":
        out, ctx, w, sols = bench_sh3d(args, torch, rte, args.mu_s if args.mu_s is not None else 10.0)
        ctx.close()
        if oracle_on:
            cpu, out["error_vs_oracle"] = oracle_3d_sh(w, 1e-8, sols)
    elif args.workload == "modes":
        out, ctx, w, sols = bench_modes(args, torch, rte, args.mu_s if args.mu_s is not None else 10.0)
        ctx.close()
        if oracle_on:
            cpu, out["error_vs_oracle"] = oracle_2d(w, 1e-8, sols)
    else:
        out, ctx, w, sols = bench_iso3d(args, torch, rte, args.mu_s if args.mu_s is not None else 10.0)
        ctx.close()
        if oracle_on:
            cpu, out["error_vs_oracle"] = oracle_3d(w, 1e-8, sols)
    line = {"metric": METRIC if args.workload == "hg512" else f"solves/s ({args.workload})"}
    line.update({"value": out.pop("value"), "unit": out.pop("unit"), "n_gpus": 1, "steps": args.steps,
                 "warmup": args.warmup, "ms_per_step": out.pop("ms_per_step"), "higher_is_better": True,
                 "scaling": "weak", "vs_baseline": None, "dtype": out.pop("dtype"), "data": "synthetic"})
    line.update(out)
    line["copy_peak_gbs"] = copy_peak_gbs(torch)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
