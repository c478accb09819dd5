"""ctypes binding of the C ABI in include/rte.h (argument marshalling only).

Every computation runs in librte.so (HIP, gfx950).  PyTorch supplies device memory and the
stream: tensors are passed by data pointer and the context enqueues on torch's current stream
at creation time.  There is no fallback: if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librte.so")

RTE_OK, RTE_NOT_CONVERGED = 0, 1
RTE_EINVAL, RTE_ENOMEM, RTE_EDEVICE, RTE_ENUMERIC, RTE_EUNSUPPORTED = -1, -2, -3, -4, -5
PREC_FP32, PREC_FP64 = 0, 1
OP_A, OP_KT = 0, 1
LAYOUT_MODES, LAYOUT_CHANNELS = 0, 1
MAX_L = 32
MAX_L3 = 3          # RTE_MAX_L3: largest spherical-harmonic degree of a 3D context
MAX_RHS = 64        # RTE_MAX_RHS: right-hand sides of one rte_solve_multi call
NN_SCRATCH_BYTES = 32 << 20      # RTE_NN_SCRATCH_BYTES of rte_nn.h


class RteError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rte error {code}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("applies", C.c_int), ("cycles", C.c_int),
                ("pc_used", C.c_int), ("pc_fallback", C.c_int),
                ("relres_est", C.c_double), ("relres_true", C.c_double),
                ("t_setup_ms", C.c_double), ("t_solve_ms", C.c_double), ("status", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("max_cycles", C.c_int), ("inner_tol", C.c_double),
                ("reorth", C.c_int), ("use_pc", C.c_int), ("basis_fp32", C.c_int)]


_lib = None


def load():
    """Load librte.so (built in-tree by paper_1802_03061_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_1802_03061_amd.build")
    lib = C.CDLL(LIB_PATH)
    P, I, D = C.c_void_p, C.c_int, C.c_double
    sig = {
        "rte_setup": (I, [C.POINTER(P), C.POINTER(Grid), D, D, C.POINTER(D), I, I, P]),
        "rte_apply": (I, [P, I, I, I, P, P]),
        "rte_rhs": (I, [P, P, I, P]),
        "rte_scattering_term": (I, [P, I, P, I, P]),
        "rte_set_solve_opts": (I, [P, C.POINTER(SolveOpts)]),
        "rte_solve": (I, [P, P, D, I, P, C.POINTER(SolveInfo)]),
        "rte_solve_rhs": (I, [P, P, D, I, P, C.POINTER(SolveInfo), P, I, C.POINTER(I)]),
        "rte_rhs_source": (I, [P, P, I, P]),
        "rte_solve_source": (I, [P, P, I, D, I, P, C.POINTER(SolveInfo)]),
        "rte_solve_multi": (I, [P, I, C.POINTER(P), D, I, C.POINTER(P), C.POINTER(SolveInfo)]),
        "rte_solve_batched": (I, [I, C.POINTER(P), C.POINTER(P), C.POINTER(D), I, C.POINTER(P),
                                  C.POINTER(SolveInfo)]),
        "rte_pc_attach": (I, [P, P, I, I, I]),
        "rte_nn_create": (I, [C.POINTER(P), I, I, I, C.c_ulonglong, I, P]),
        "rte_nn_destroy": (None, [P]),
        "rte_nn_param_count": (I, [P, C.POINTER(C.c_longlong)]),
        "rte_nn_get_params": (I, [P, P]),
        "rte_nn_set_params": (I, [P, P]),
        "rte_nn_forward": (I, [P, P, I, I, I, P]),
        "rte_nn_forward_noalloc": (I, [P, P, I, I, I, P]),
        "rte_nn_loss_grad": (I, [P, P, P, P, I, I, I, C.POINTER(D), P]),
        "rte_nn_adam_step": (I, [P, C.c_float]),
        "rte_nn_gather_rows": (I, [P, C.c_longlong, C.c_longlong, P, I, P, P]),
        "rte_nn_upsample_bilinear": (I, [P, I, I, I, I, I, I, P, P]),
        "rte_pc_make_pairs": (I, [P, P, P, P, I, I, P, P, P]),
        "rte_pc_apply": (I, [P, P, P]),
        "rte_time_apply": (I, [P, I, I, I, C.POINTER(D), C.POINTER(D)]),
        "rte_time_apply_multi": (I, [P, I, I, I, I, C.POINTER(D), C.POINTER(D)]),
        "rte_time_batched_apply": (I, [I, C.POINTER(P), I, C.POINTER(D), I, C.POINTER(I), C.POINTER(D),
                                       C.POINTER(I), C.POINTER(I), C.POINTER(I), C.POINTER(I)]),
        "rte_set_batched_variant": (I, [I, I]),
        "rte_query": (I, [P, C.POINTER(I), C.POINTER(I), C.POINTER(C.c_longlong)]),
        "rte_autotune": (I, [P, I]),
        "rte_set_variant": (I, [P, I, I, I]),
        "rte_get_variant": (I, [P, I, I, C.POINTER(I), C.POINTER(I)]),
        "rte_modes_to_channels": (I, [P, P, P]),
        "rte_channels_to_modes": (I, [P, P, P]),
        "rte_destroy": (None, [P]),
        "rte_last_error": (C.c_char_p, []),
        "rte_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().rte_last_error().decode()


def _check(rc, allow=(RTE_OK,)):
    if rc not in allow:
        raise RteError(rc, last_error())
    return rc


def _ptr(t: torch.Tensor, dtype, numel=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


class Context:
    """One problem: grid, coefficients, precision; owns its device state."""

    def __init__(self, n, h=None, mu_a=0.1, mu_s=1.0, sigma_hat=None, L=0, prec=PREC_FP64, dim=None,
                 device=None):
        lib = load()
        if isinstance(n, int):
            n = (n, n) if (dim or 2) == 2 else (n, n, n)
        n = tuple(int(v) for v in n)
        dim = len(n)
        self.dim, self.shape_xyz, self.L, self.prec = dim, n, int(L), int(prec)
        self.h = float(h if h is not None else 1.0 / n[0])
        self.mu_a, self.mu_s = float(mu_a), float(mu_s)
        g = Grid()
        g.dim = dim
        for a in range(3):
            g.n[a] = n[a] if a < dim else 1
        g.h = self.h
        sh = None
        if sigma_hat is not None:
            arr = (C.c_double * len(sigma_hat))(*[float(s) for s in sigma_hat])
            sh = C.cast(arr, C.POINTER(C.c_double))
            self._sigma = arr
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = C.c_void_p()
        _check(lib.rte_setup(C.byref(h), C.byref(g), self.mu_a, self.mu_s, sh, self.L, self.prec,
                             C.c_void_p(stream.cuda_stream)))
        self._h = h
        ch, md, cells = C.c_int(), C.c_int(), C.c_longlong()
        _check(lib.rte_query(h, C.byref(ch), C.byref(md), C.byref(cells)))
        self.channels, self.modes, self.cells = ch.value, md.value, cells.value
        # array shapes: 2D [..][ny][nx], 3D [nz][ny][nx]
        self.grid_shape = tuple(reversed(n))

    # ---- shapes
    @property
    def mode_shape(self):
        return (self.modes,) + self.grid_shape

    @property
    def channel_shape(self):
        return (self.channels,) + self.grid_shape

    def close(self):
        if getattr(self, "_h", None):
            load().rte_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- operations
    def apply(self, x, op=OP_A, layout=LAYOUT_MODES, prec=None, out=None):
        prec = self.prec if prec is None else prec
        if layout == LAYOUT_MODES:
            xp = _ptr(x, torch.complex128, self.modes * self.cells)
            out = torch.empty_like(x) if out is None else out
            yp = _ptr(out, torch.complex128, self.modes * self.cells)
        else:
            xp = _ptr(x, torch.float64, self.channels * self.cells)
            out = torch.empty_like(x) if out is None else out
            yp = _ptr(out, torch.float64, self.channels * self.cells)
        _check(load().rte_apply(self._h, op, layout, prec, xp, yp))
        return out

    def rhs(self, f, layout=LAYOUT_MODES):
        fp = _ptr(f, torch.float64, self.cells)
        if layout == LAYOUT_MODES:
            out = torch.empty(self.mode_shape, dtype=torch.complex128, device=f.device)
        else:
            out = torch.empty(self.channel_shape, dtype=torch.float64, device=f.device)
        _check(load().rte_rhs(self._h, fp, layout, C.c_void_p(out.data_ptr())))
        return out

    def scattering_term(self, u, ntheta, layout=LAYOUT_MODES, out=None):
        """S[q] = Re(mu_s sum_k sigma_hat_|k| u_k e^{i k theta_q}), theta_q = 2 pi q / ntheta
        (rte_scattering_term); float64 [ntheta, ny, nx]."""
        if layout == LAYOUT_MODES:
            up = _ptr(u, torch.complex128, self.modes * self.cells)
        else:
            up = _ptr(u, torch.float64, self.channels * self.cells)
        if out is None:
            out = torch.empty((int(ntheta),) + tuple(self.channel_shape[1:]), dtype=torch.float64, device=u.device)
        sp = _ptr(out, torch.float64, int(ntheta) * self.cells)
        _check(load().rte_scattering_term(self._h, layout, up, int(ntheta), sp))
        return out

    def set_opts(self, restart=64, max_cycles=8, inner_tol=3e-4, reorth=0, use_pc=1, basis_fp32=0):
        o = SolveOpts(restart, max_cycles, inner_tol, reorth, use_pc, basis_fp32)
        _check(load().rte_set_solve_opts(self._h, C.byref(o)))

    def solve(self, f, tol=1e-8, max_iter=1000, allow_not_converged=False):
        fp = _ptr(f, torch.float64, self.cells)
        u = torch.empty(self.mode_shape, dtype=torch.complex128, device=f.device)
        info = SolveInfo()
        allow = (RTE_OK, RTE_NOT_CONVERGED) if allow_not_converged else (RTE_OK,)
        rc = _check(load().rte_solve(self._h, fp, float(tol), int(max_iter), C.c_void_p(u.data_ptr()),
                                     C.byref(info)), allow)
        d = info.as_dict()
        d["status"] = rc
        return u, d

    def _src_ptr(self, g, layout):
        if layout == LAYOUT_MODES:
            return _ptr(g, torch.complex128, self.modes * self.cells)
        return _ptr(g, torch.float64, self.channels * self.cells)

    def rhs_source(self, g, layout=LAYOUT_MODES):
        """b = K~ g for an anisotropic source given by its angular modes (rte_rhs_source)."""
        out = torch.empty_like(g)
        _check(load().rte_rhs_source(self._h, self._src_ptr(g, layout), layout, C.c_void_p(out.data_ptr())))
        return out

    def solve_source(self, g, tol=1e-8, max_iter=1000, layout=LAYOUT_MODES, allow_not_converged=False):
        """Solve A u = K~ g for an anisotropic source (rte_solve_source); u in g's layout."""
        gp = self._src_ptr(g, layout)
        u = torch.empty_like(g)
        info = SolveInfo()
        allow = (RTE_OK, RTE_NOT_CONVERGED) if allow_not_converged else (RTE_OK,)
        rc = _check(load().rte_solve_source(self._h, gp, layout, float(tol), int(max_iter),
                                            C.c_void_p(u.data_ptr()), C.byref(info)), allow)
        d = info.as_dict()
        d["status"] = rc
        return u, d

    def solve_multi(self, fs, tol=1e-8, max_iter=1000, allow_not_converged=False):
        """Several sources sharing this context's operator (rte_solve_multi): returns the list of
        complex mode tensors, the per-source infos and the status."""
        n = len(fs)
        fp = (C.c_void_p * n)(*[_ptr(f, torch.float64, self.cells) for f in fs])
        us = [torch.empty(self.mode_shape, dtype=torch.complex128, device=f.device) for f in fs]
        up = (C.c_void_p * n)(*[C.c_void_p(u.data_ptr()) for u in us])
        infos = (SolveInfo * n)()
        allow = (RTE_OK, RTE_NOT_CONVERGED) if allow_not_converged else (RTE_OK,)
        rc = _check(load().rte_solve_multi(self._h, n, fp, float(tol), int(max_iter), up, infos), allow)
        return us, [i.as_dict() for i in infos], rc

    def solve_rhs(self, b, tol=1e-8, max_iter=1000, record=0, allow_not_converged=False):
        bp = _ptr(b, torch.float64, self.channels * self.cells)
        x = torch.empty_like(b)
        info = SolveInfo()
        rec = None
        nrec = C.c_int(0)
        if record:
            rec = torch.zeros((record,) + tuple(b.shape), dtype=torch.float64, device=b.device)
        allow = (RTE_OK, RTE_NOT_CONVERGED) if allow_not_converged else (RTE_OK,)
        rc = _check(load().rte_solve_rhs(self._h, bp, float(tol), int(max_iter), C.c_void_p(x.data_ptr()),
                                         C.byref(info),
                                         C.c_void_p(rec.data_ptr()) if rec is not None else None,
                                         int(record), C.byref(nrec)), allow)
        d = info.as_dict()
        d["status"] = rc
        if rec is not None:
            return x, d, rec[:nrec.value]
        return x, d

    def time_apply(self, op=OP_A, prec=None, reps=20):
        prec = self.prec if prec is None else prec
        tot = C.c_double()
        passes = (C.c_double * 5)()
        _check(load().rte_time_apply(self._h, op, prec, reps, C.byref(tot), passes))
        return tot.value, list(passes)

    def time_apply_multi(self, nrhs, op=OP_A, prec=None, reps=20):
        """Per-pass timing of the batched apply over nrhs stacked right-hand sides."""
        prec = self.prec if prec is None else prec
        tot = C.c_double()
        passes = (C.c_double * 5)()
        _check(load().rte_time_apply_multi(self._h, int(nrhs), op, prec, reps, C.byref(tot), passes))
        return tot.value, list(passes)

    def autotune(self, reps=5):
        _check(load().rte_autotune(self._h, int(reps)))

    def set_variant(self, prec, pass_, variant):
        _check(load().rte_set_variant(self._h, int(prec), int(pass_), int(variant)))

    def get_variant(self, prec, pass_):
        v, n = C.c_int(), C.c_int()
        _check(load().rte_get_variant(self._h, int(prec), int(pass_), C.byref(v), C.byref(n)))
        return v.value, n.value

    def attach_pc(self, weights, hidden=32, layers=5, factor=8):
        """Attach the coarse-grid network (packed float32 parameters) as the FGMRES right
        preconditioner; None detaches."""
        if weights is None:
            _check(load().rte_pc_attach(self._h, None, 0, 0, 1))
            return
        wp = _ptr(weights, torch.float32)
        _check(load().rte_pc_attach(self._h, wp, int(hidden), int(layers), int(factor)))

    def pc_apply(self, v):
        """z = M v with the attached preconditioner (channel layout, FP64)."""
        z = torch.empty_like(v)
        _check(load().rte_pc_apply(self._h, _ptr(v, torch.float64, self.channels * self.cells),
                                   C.c_void_p(z.data_ptr())))
        return z

    def make_pairs(self, b, x_star, x_iters, factor):
        """Coarse training pairs (inputs, targets, weights) from iterates of a solve of A x = b."""
        cnt = int(x_iters.shape[0])
        Hc, Wc = self.grid_shape[0] // factor, self.grid_shape[1] // factor
        xo = torch.empty((cnt, self.channels, Hc, Wc), dtype=torch.float32, device=b.device)
        to = torch.empty_like(xo)
        wo = torch.empty((cnt,), dtype=torch.float32, device=b.device)
        n = self.channels * self.cells
        _check(load().rte_pc_make_pairs(self._h, _ptr(b, torch.float64, n), _ptr(x_star, torch.float64, n),
                                        _ptr(x_iters, torch.float64, cnt * n), cnt, int(factor),
                                        C.c_void_p(xo.data_ptr()), C.c_void_p(to.data_ptr()),
                                        C.c_void_p(wo.data_ptr())))
        return xo, to, wo

    def modes_to_channels(self, x):
        out = torch.empty(self.channel_shape, dtype=torch.float64, device=x.device)
        _check(load().rte_modes_to_channels(self._h, _ptr(x, torch.complex128, self.modes * self.cells),
                                            C.c_void_p(out.data_ptr())))
        return out

    def channels_to_modes(self, ch):
        out = torch.empty(self.mode_shape, dtype=torch.complex128, device=ch.device)
        _check(load().rte_channels_to_modes(self._h, _ptr(ch, torch.float64, self.channels * self.cells),
                                            C.c_void_p(out.data_ptr())))
        return out


def solve_batched(ctxs, fs, tols, max_iter=1000, allow_not_converged=False):
    """Solve several isotropic 2D problems together (rte_solve_batched).  The library runs the batch
    on a stream of its own, so pending work on torch's stream is completed first."""
    lib = load()
    torch.cuda.synchronize()
    n = len(ctxs)
    hs = (C.c_void_p * n)(*[c._h for c in ctxs])
    fp = (C.c_void_p * n)(*[_ptr(f, torch.float64, c.cells) for f, c in zip(fs, ctxs)])
    us = [torch.empty(c.mode_shape, dtype=torch.complex128, device=f.device) for c, f in zip(ctxs, fs)]
    up = (C.c_void_p * n)(*[C.c_void_p(u.data_ptr()) for u in us])
    tl = (C.c_double * n)(*[float(t) for t in tols])
    infos = (SolveInfo * n)()
    allow = (RTE_OK, RTE_NOT_CONVERGED) if allow_not_converged else (RTE_OK,)
    rc = _check(lib.rte_solve_batched(n, hs, fp, tl, int(max_iter), up, infos), allow)
    return us, [i.as_dict() for i in infos], rc


def time_batched_apply(ctxs, reps=20):
    """Per-launch times of the batched apply (rte_time_batched_apply); needs a prior solve_batched
    on the same contexts.  Returns (ms_total, [(pass, PX, PY, ms, variant), ...])."""
    n = len(ctxs)
    hs = (C.c_void_p * n)(*[c._h for c in ctxs])
    cap = 64
    tot = C.c_double()
    nl = C.c_int()
    ms = (C.c_double * cap)()
    ps, px, py, pv = (C.c_int * cap)(), (C.c_int * cap)(), (C.c_int * cap)(), (C.c_int * cap)()
    _check(load().rte_time_batched_apply(n, hs, int(reps), C.byref(tot), cap, C.byref(nl), ms, ps, px, py, pv))
    return tot.value, [(ps[i], px[i], py[i], ms[i], pv[i]) for i in range(min(nl.value, cap))]


def set_batched_variant(pass_, variant):
    """Force a kernel variant of the batched apply for plans built afterwards (rte_set_batched_variant):
    pass 0 = row tiles of passes A and C, 1 = column groups of pass B; -1 restores tuning."""
    _check(load().rte_set_batched_variant(int(pass_), int(variant)))


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def gather_rows(src, idx):
    """dst[i] = src[idx[i]] over the first axis (float32 device tensor, int32 device indices)."""
    src = src.contiguous()
    idx = idx.to(torch.int32).contiguous()
    dst = torch.empty((idx.shape[0],) + tuple(src.shape[1:]), dtype=torch.float32, device=src.device)
    row = 1
    for d in src.shape[1:]:
        row *= int(d)
    _check(load().rte_nn_gather_rows(_ptr(src, torch.float32), src.shape[0], row, C.c_void_p(idx.data_ptr()),
                                     int(idx.shape[0]), C.c_void_p(dst.data_ptr()), _stream()))
    return dst


def upsample_bilinear(coarse, ny, nx):
    """Bilinear upsampling at cell centres of FP64 fields [count][C][hc][wc] to [count][C][ny][nx]."""
    coarse = coarse.contiguous()
    n, Cc, hc, wc = coarse.shape
    fine = torch.empty((n, Cc, ny, nx), dtype=torch.float64, device=coarse.device)
    _check(load().rte_nn_upsample_bilinear(_ptr(coarse, torch.float64), n, Cc, hc, wc, ny, nx,
                                           C.c_void_p(fine.data_ptr()), _stream()))
    return fine


class Net:
    """The preconditioner network's parameters, forward, gradient and Adam (rte_nn.h)."""

    def __init__(self, channels, hidden=32, layers=5, seed=0, use_bias=True):
        lib = load()
        h = C.c_void_p()
        _check(lib.rte_nn_create(C.byref(h), int(channels), int(hidden), int(layers), int(seed),
                                 1 if use_bias else 0, C.c_void_p(torch.cuda.current_stream().cuda_stream)))
        self._h = h
        self.channels, self.hidden, self.layers = int(channels), int(hidden), int(layers)
        cnt = C.c_longlong()
        _check(lib.rte_nn_param_count(h, C.byref(cnt)))
        self.nparam = cnt.value

    def close(self):
        if getattr(self, "_h", None):
            load().rte_nn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        out = torch.empty(self.nparam, dtype=torch.float32, device="cuda")
        _check(load().rte_nn_get_params(self._h, C.c_void_p(out.data_ptr())))
        return out

    def set_params(self, p):
        _check(load().rte_nn_set_params(self._h, _ptr(p, torch.float32, self.nparam)))

    def forward(self, x):
        B, Cc, H, W = x.shape
        y = torch.empty((B, self.channels, H, W), dtype=torch.float32, device=x.device)
        _check(load().rte_nn_forward(self._h, _ptr(x, torch.float32), B, H, W, C.c_void_p(y.data_ptr())))
        return y

    def forward_noalloc(self, x, out):
        """y = N(x) into the caller's `out`, with the library's fixed per-GPU activation array."""
        B, Cc, H, W = x.shape
        _check(load().rte_nn_forward_noalloc(self._h, _ptr(x, torch.float32), B, H, W,
                                             _ptr(out, torch.float32, B * self.channels * H * W)))
        return out

    def loss_grad(self, x, t, w, want_grad=False):
        B, Cc, H, W = x.shape
        loss = C.c_double()
        g = torch.empty(self.nparam, dtype=torch.float32, device=x.device) if want_grad else None
        _check(load().rte_nn_loss_grad(self._h, _ptr(x, torch.float32), _ptr(t, torch.float32),
                                       _ptr(w, torch.float32, B), B, H, W, C.byref(loss),
                                       C.c_void_p(g.data_ptr()) if g is not None else None))
        return (loss.value, g) if want_grad else loss.value

    def adam_step(self, lr=1e-3):
        _check(load().rte_nn_adam_step(self._h, float(lr)))
