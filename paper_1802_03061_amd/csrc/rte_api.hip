// C ABI of the RTE library: context set-up, operator apply, right-hand side, GMRES solve.
//
// The solve follows steps T.1/T.2 of Sec. 3.3 (S.1/S.2 of Sec. 2.3 for the isotropic case):
// b = K~ g by one FFT apply, then GMRES on (I - K~ D) u = b from u = 0.  Unknowns are held as real
// channel vectors (see apply2d.hip); for a real angular flux their Euclidean inner product equals
// the complex inner product of the full mode vector, so GMRES runs in real FP64 arithmetic.
// With RTE_PREC_FP32 the inner applies use FP32 FFTs and each restart cycle ends with an FP64
// true-residual apply (iterative refinement); orthogonalisation, the Hessenberg least squares and
// the residual check are FP64 throughout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/rte.h"
#include "apply2d.h"
#include "apply2d_b.h"
#include "apply3d.h"
#include "sh3d.h"
#include "ctx.h"
#include "krylov.h"
#include "nn.h"
#include "spectra.h"

namespace rte {

static thread_local char g_err[512] = "";

int set_error(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int set_hip_error(hipError_t e, const char* what, const char* file, int line) {
    const int code = (e == hipErrorOutOfMemory) ? RTE_ENOMEM : RTE_EDEVICE;
    return set_error(code, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
}

static double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

template <typename P>
static int dalloc(P** p, size_t count) {
    *p = nullptr;
    if (count == 0) return RTE_OK;
    hipError_t e = hipMalloc((void**)p, count * sizeof(P));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_error(e == hipErrorOutOfMemory ? RTE_ENOMEM : RTE_EDEVICE, "hipMalloc of %zu bytes failed: %s",
                         count * sizeof(P), hipGetErrorString(e));
    }
    return RTE_OK;
}

template <typename P>
static void dfree(P*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

// ------------------------------------------------------------------ context lifetime ----------

static void free_krylov(rte_ctx* c) {
    dfree(c->V);
    dfree(c->Z);
    dfree(c->partial);
    dfree(c->dsmall);
    dfree(c->arn);
    dfree(c->arn_flags);
    if (c->hpipe) (void)hipHostFree(c->hpipe);
    c->hpipe = nullptr;
    if (c->hpipe_flags) (void)hipHostFree(c->hpipe_flags);
    c->hpipe_flags = nullptr;
    c->krylov_m = 0;
    c->krylov_n = 0;
    c->krylov_z = false;
    c->krylov_vbytes = 0;
}

static void free_ctx(rte_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    batched_forget(c->id);
    free_krylov(c);
    dfree(c->Qf);
    dfree(c->Qd);
    dfree(c->Q3f);
    dfree(c->Q3d);
    for (int a = 0; a < 3; ++a) {
        dfree(c->twf[a]);
        dfree(c->twd[a]);
    }
    dfree(c->twmf);
    dfree(c->twmd);
    dfree(c->twy1f);
    dfree(c->twy1d);
    dfree(c->twyhf);
    dfree(c->twyhd);
    dfree(c->wf);
    dfree(c->wf2);
    dfree(c->wd);
    dfree(c->wd2);
    dfree(c->xv);
    dfree(c->rv);
    dfree(c->bv);
    dfree(c->xm);
    dfree(c->rm);
    dfree(c->bm);
    dfree(c->t0);
    dfree(c->t1);
    dfree(c->dflag);
    pc_free(c);
    delete c;
}

int ensure_krylov(rte_ctx* c, int m, bool need_z, size_t vbytes, size_t nlen) {
    const size_t n = std::max(nlen ? nlen : c->nvec, c->krylov_n);
    if (c->krylov_m >= m && c->krylov_vbytes >= vbytes && (!need_z || c->krylov_z) && c->krylov_n >= n) return RTE_OK;
    free_krylov(c);
    int rc;
    if ((rc = dalloc(&c->V, (size_t)(m + 1) * n * vbytes))) return rc;
    if (need_z && (rc = dalloc(&c->Z, (size_t)m * n))) return rc;
    if ((rc = dalloc(&c->partial, (size_t)(m + 3) * RTE_KRYLOV_NBLK))) return rc;
    if ((rc = dalloc(&c->dsmall, (size_t)(2 * m + 16)))) return rc;
    // device Arnoldi state: H [(m+1) x m] | cs [m] | sn [m] | g [m+1] | est [m] | inv [m+1]
    if ((rc = dalloc(&c->arn, (size_t)(m + 1) * m + 4 * (size_t)m + 2))) return rc;
    if ((rc = dalloc(&c->arn_flags, 4))) return rc;
    hipError_t e = hipSuccess;
    // per-iteration pinned slots: estimate; (breakdown, non-finite) flags
    // per-iteration slots written by the Arnoldi kernel itself (mapped, coherent host memory)
    // [0, m): per-iteration estimates; [m]: the result of a host-side dot product
    e = hipHostMalloc((void**)&c->hpipe, (size_t)(m + 1) * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) return set_hip_error(e, "hipHostMalloc", __FILE__, __LINE__);
    e = hipHostMalloc((void**)&c->hpipe_flags, (size_t)2 * m * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) return set_hip_error(e, "hipHostMalloc", __FILE__, __LINE__);
    e = hipHostGetDevicePointer((void**)&c->hpipe_dev, c->hpipe, 0);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&c->hpipe_flags_dev, c->hpipe_flags, 0);
    if (e != hipSuccess) return set_hip_error(e, "hipHostMalloc", __FILE__, __LINE__);
    c->krylov_m = m;
    c->krylov_n = n;
    c->krylov_z = need_z;
    c->krylov_vbytes = vbytes;
    return RTE_OK;
}

// FFT work buffers for nb batch entries (right-hand sides); grown on demand, never shrunk.
static int ensure_work(rte_ctx* c, int nb) {
    if (nb <= c->work_nb) return RTE_OK;
    const bool f32 = c->prec == RTE_PREC_FP32;
    const int NK = c->PX / 2 + 1;
    dfree(c->wf);
    dfree(c->wf2);
    dfree(c->wd);
    dfree(c->wd2);
    c->work_nb = 0;
    int rc;
    if (c->dim == 2) {
        const size_t nt = (size_t)nb * c->C * NK * c->ny;
        const size_t nt2 = (size_t)nb * c->C * NK * c->PY;
        if ((rc = dalloc(&c->wd, nt))) return rc;
        if (apply2d_needs_work2<double>(c->L, c->PY) && (rc = dalloc(&c->wd2, nt2))) return rc;
        if (f32) {
            if ((rc = dalloc(&c->wf, nt))) return rc;
            if (apply2d_needs_work2<float>(c->L, c->PY) && (rc = dalloc(&c->wf2, nt2))) return rc;
        }
    } else {
        const size_t n1 = (size_t)nb * c->C * c->nz * NK * c->ny;
        const size_t n2 = (size_t)c->C * NK * c->PY * c->nz;   // shared by the batch entries
        if ((rc = dalloc(&c->wd, n1)) || (rc = dalloc(&c->wd2, n2))) return rc;
        if (f32 && ((rc = dalloc(&c->wf, n1)) || (rc = dalloc(&c->wf2, n2)))) return rc;
    }
    c->work_nb = nb;
    return RTE_OK;
}

// ------------------------------------------------------------------ apply ---------------------

static ChanScale channel_scale(const rte_ctx* c, int mode) {
    ChanScale s;
    for (int i = 0; i < 2 * RTE_MAX_L + 1; ++i) s.s[i] = 1.0;
    if (mode != APPLY_KT) {
        s.s[0] = c->mu_s * c->sigma[0];
        for (int k = 1; k <= c->L; ++k) s.s[2 * k - 1] = s.s[2 * k] = c->mu_s * c->sigma[k];
    }
    return s;
}

// 3D: channel a (the real harmonic of degree l(a)) is scaled by mu_s sigma_hat_l(a) (Funk-Hecke).
static ChanScale3 channel_scale3(const rte_ctx* c, int mode) {
    ChanScale3 s;
    for (int i = 0; i < 16; ++i) s.s[i] = 1.0;
    if (mode != APPLY_KT)
        for (int a = 0; a < c->C; ++a) s.s[a] = c->mu_s * c->sigma[sh_degree(a)];
    return s;
}

// Column 0 of the 2D work buffer packs the x-frequencies 0 and PX/2 (two real sequences) except
// with the register-resident pass B, which takes them as columns of their own.
template <typename T>
static int pack_for(const Apply2DArgs<T>& a) { return apply2d_unpacked<T>(a.L, a.PY, a.var[1]) ? 0 : 1; }

template <typename T>
static Apply2DArgs<T> args2d(const rte_ctx* c);
template <>
Apply2DArgs<float> args2d<float>(const rte_ctx* c) {
    Apply2DArgs<float> a{c->nx, c->ny, c->PX, c->PY, c->L, c->C, c->wf, c->wf2, c->Qf, c->twf[0], c->twf[1], c->stream};
    a.twm = c->twmf;
    a.twy1 = c->twy1f;
    a.twyh = c->twyhf;
    for (int p = 0; p < 3; ++p) a.var[p] = c->varf[p];
    return a;
}
template <>
Apply2DArgs<double> args2d<double>(const rte_ctx* c) {
    Apply2DArgs<double> a{c->nx, c->ny, c->PX, c->PY, c->L, c->C, c->wd, c->wd2, c->Qd, c->twd[0], c->twd[1], c->stream};
    a.twm = c->twmd;
    a.twy1 = c->twy1d;
    a.twyh = c->twyhd;
    for (int p = 0; p < 3; ++p) a.var[p] = c->vard[p];
    return a;
}

template <typename T, typename TV>
static int apply_t(rte_ctx* c, int mode, const TV* x, const double* b, TV* y, int nbatch, hipEvent_t* ev) {
    const ChanScale sc = channel_scale(c, mode);
    if (c->dim == 2) {
        Apply2DArgs<T> a = args2d<T>(c);
        a.pack = pack_for(a);
        if (ev) (void)hipEventRecord(ev[0], c->stream);
        if (apply2d_pass_a<T>(a, x, sc, nbatch)) return set_error(RTE_EUNSUPPORTED, "pass A: unsupported size");
        if (ev) (void)hipEventRecord(ev[1], c->stream);
        if (apply2d_pass_b<T>(a, nbatch)) return set_error(RTE_EUNSUPPORTED, "pass B: unsupported size");
        if (ev) (void)hipEventRecord(ev[2], c->stream);
        if (apply2d_pass_c<T>(a, x, b, y, mode, nbatch)) return set_error(RTE_EUNSUPPORTED, "pass C: unsupported size");
        if (ev) (void)hipEventRecord(ev[3], c->stream);
    } else {
        // x-passes treat every z-slab of every channel of every batch entry as one channel of a 2D
        // apply; the factor of D is applied per channel when pass B loads it
        Apply2DArgs<T> a = args2d<T>(c);
        a.C = 1;
        a.L = 0;
        a.pack = 0;
        const int* v3 = sizeof(T) == 4 ? c->var3f : c->var3d;
        a.var[0] = v3[0];
        a.var[1] = 0;
        a.var[2] = v3[4];
        ChanScale ones;
        for (int i = 0; i < 2 * RTE_MAX_L + 1; ++i) ones.s[i] = 1.0;
        Apply3DArgs<T> a3;
        a3.nx = c->nx; a3.ny = c->ny; a3.nz = c->nz; a3.PX = c->PX; a3.PY = c->PY; a3.PZ = c->PZ;
        a3.C = c->C;
        a3.L = c->L;
        a3.sc = channel_scale3(c, mode);
        a3.stream = c->stream;
        for (int p = 0; p < 3; ++p) a3.var[p] = v3[p + 1];
        const size_t t1sz = (size_t)c->C * c->nz * (c->PX / 2 + 1) * c->ny;   // one batch entry
        if constexpr (sizeof(T) == 4) {
            a3.T1 = c->wf; a3.T2 = c->wf2; a3.Q3 = c->Q3f; a3.twy = c->twf[1]; a3.twz = c->twf[2];
        } else {
            a3.T1 = c->wd; a3.T2 = c->wd2; a3.Q3 = c->Q3d; a3.twy = c->twd[1]; a3.twz = c->twd[2];
        }
        const int slabs = nbatch * c->C * c->nz;
        if (ev) (void)hipEventRecord(ev[0], c->stream);
        if (apply2d_pass_a<T>(a, x, ones, slabs)) return set_error(RTE_EUNSUPPORTED, "3D pass A: unsupported size");
        if (ev) (void)hipEventRecord(ev[1], c->stream);
        cx<T>* T1base = a3.T1;
        for (int bi = 0; bi < nbatch; ++bi) {
            a3.T1 = T1base + (size_t)bi * t1sz;
            if (apply3d_pass<T>(a3, 1)) return set_error(RTE_EUNSUPPORTED, "3D pass B: unsupported size");
            if (ev && bi == nbatch - 1) (void)hipEventRecord(ev[2], c->stream);
            if (apply3d_pass<T>(a3, 2)) return set_error(RTE_EUNSUPPORTED, "3D pass C: unsupported size");
            if (ev && bi == nbatch - 1) (void)hipEventRecord(ev[3], c->stream);
            if (apply3d_pass<T>(a3, 3)) return set_error(RTE_EUNSUPPORTED, "3D pass D: unsupported size");
        }
        if (ev) (void)hipEventRecord(ev[4], c->stream);
        if (apply2d_pass_c<T>(a, x, b, y, mode, slabs)) return set_error(RTE_EUNSUPPORTED, "3D pass E: unsupported size");
        if (ev) (void)hipEventRecord(ev[5], c->stream);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(e, "apply launch", __FILE__, __LINE__);
    return RTE_OK;
}

int apply_channels(rte_ctx* c, int mode, int prec, const double* x, const double* b, double* y, int nbatch) {
    if (prec == RTE_PREC_FP32) return apply_t<float>(c, mode, x, b, y, nbatch, nullptr);
    return apply_t<double>(c, mode, x, b, y, nbatch, nullptr);
}

// y = A x on basis vectors (stored as TV) in the context precision: float vectors only with the
// FP32 apply.
template <typename TV>
static int apply_basis(rte_ctx* c, const TV* x, TV* y, int nb = 1) {
    if constexpr (sizeof(TV) == sizeof(float)) return apply_t<float>(c, APPLY_A, x, nullptr, y, nb, nullptr);
    else return c->prec == RTE_PREC_FP32 ? apply_t<float>(c, APPLY_A, x, nullptr, y, nb, nullptr)
                                         : apply_t<double>(c, APPLY_A, x, nullptr, y, nb, nullptr);
}

// y = A (v + s P Y) in the context precision, the coarse correction added inside passes A and C.
template <typename T, typename TV>
static int apply_pc_t(rte_ctx* c, const TV* v, TV* y, const float* Y) {
    const ChanScale sc = channel_scale(c, APPLY_A);
    Apply2DArgs<T> a = args2d<T>(c);
    a.pack = pack_for(a);
    a.corr = Y;
    a.cF = c->pc_factor;
    a.cs = 1.0 / std::sqrt((double)c->nvec);
    if (apply2d<T>(a, v, nullptr, y, APPLY_A, sc, 1)) return set_error(RTE_EUNSUPPORTED, "apply: unsupported size");
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "apply launch", __FILE__, __LINE__);
}
template <typename TV>
static int apply_basis_pc(rte_ctx* c, const TV* v, TV* y, const float* Y) {
    if constexpr (sizeof(TV) == sizeof(float)) return apply_pc_t<float>(c, v, y, Y);
    else return c->prec == RTE_PREC_FP32 ? apply_pc_t<float>(c, v, y, Y) : apply_pc_t<double>(c, v, y, Y);
}

// The x-spectra of the bilinear prolongation's weight rows (CorrB): phi[X][kx] = sum over fine
// columns x < nx of w_X(x) exp(-2 pi i kx x / PX), w_X(x) the weight of coarse column X at x as
// lerp_at computes it; with the packed work buffer, column 0 holds (phi(0), phi(PX/2)).  Built on
// the host in FP64 once per context and packing.
static int pc_phi_prepare(rte_ctx* c, int pack) {
    if (c->pc_phi && c->pc_phi_pack == pack) return RTE_OK;
    const int F = c->pc_factor, Wc = c->nx / F, PX = c->PX, H = PX / 2;
    const int nkx = pack ? H : H + 1;
    std::vector<std::complex<double>> tw(PX), ph((size_t)Wc * nkx);
    std::vector<double> alt(Wc, 0.0);
    const double pi = 3.14159265358979323846;
    for (int q = 0; q < PX; ++q) tw[q] = std::polar(1.0, -2.0 * pi * q / PX);
    for (int x = 0; x < c->nx; ++x) {
        const float xi = ((float)x + 0.5f) / (float)F - 0.5f;
        const float f0 = std::floor(xi);
        const float a = xi - f0;
        const int i0 = (int)f0;
        const int lo = std::min(std::max(i0, 0), Wc - 1), hi = std::min(std::max(i0 + 1, 0), Wc - 1);
        const double wl = (double)(1.f - a), wh = (double)a;
        for (int k = 0; k < nkx; ++k) {
            const std::complex<double> e = tw[(size_t)k * x % PX];
            ph[(size_t)lo * nkx + k] += wl * e;
            ph[(size_t)hi * nkx + k] += wh * e;
        }
        const double sg = (x & 1) ? -1.0 : 1.0;
        alt[lo] += wl * sg;
        alt[hi] += wh * sg;
    }
    std::vector<cx<float>> hst((size_t)Wc * nkx);
    for (int X = 0; X < Wc; ++X)
        for (int k = 0; k < nkx; ++k) {
            std::complex<double> v = ph[(size_t)X * nkx + k];
            if (pack && k == 0) v = std::complex<double>(v.real(), alt[X]);
            hst[(size_t)X * nkx + k] = cx<float>{(float)v.real(), (float)v.imag()};
        }
    if (c->pc_phi) (void)hipFree(c->pc_phi);
    c->pc_phi = nullptr;
    c->pc_phi_pack = -1;
    int rc = dalloc(&c->pc_phi, hst.size());
    if (rc) return rc;
    RTE_HIP_TRY(hipMemcpy(c->pc_phi, hst.data(), hst.size() * sizeof(cx<float>), hipMemcpyHostToDevice));
    c->pc_phi_pack = pack;
    return RTE_OK;
}

// Whether a preconditioned solve runs the next apply's pass A inside the stage-1 launch, beside
// the network (FP32 2D apply with a pass B that can add the correction); RTE_PC_EARLY_A=0 turns
// it off.  Prepares the correction's x-spectra.
static bool early_a_ok(rte_ctx* c) {
    if (c->dim != 2 || c->prec != RTE_PREC_FP32 || c->L > 8 || c->C > 17) return false;
    if ((c->nx / c->pc_factor) % 4) return false;   // pass B reads the coarse rows as float4s
    const char* env = std::getenv("RTE_PC_EARLY_A");
    if (env && env[0] == '0') return false;
    if (!pc_rescale_net_pa_ok(c)) return false;
    const Apply2DArgs<float> a = args2d<float>(c);
    if (!apply2d_b_corr_ok<float>(c->L, c->PY, a.var[1])) return false;
    if (pc_phi_prepare(c, pack_for(a)) != RTE_OK) return false;
    // the per-channel factors, uploaded again only when the medium changed
    const ChanScale sc = channel_scale(c, APPLY_A);
    const double cs = 1.0 / std::sqrt((double)c->nvec);
    float k[17] = {};
    for (int ch = 0; ch < c->C; ++ch) k[ch] = (float)(sc.s[ch] * cs);
    if (c->pc_coef && std::memcmp(k, c->pc_coef_host, sizeof(k)) == 0) return true;
    if (!c->pc_coef && dalloc(&c->pc_coef, 17) != RTE_OK) return false;
    if (hipMemcpy(c->pc_coef, k, sizeof(k), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    std::memcpy(c->pc_coef_host, k, sizeof(k));
    return true;
}

// y = A (v + s P Y) after the stage-1 launch has run pass A on v alone (early_a_ok): passes B,
// adding the correction's x-spectrum, and C.
template <typename TV>
static int apply_basis_pc_from_b(rte_ctx* c, const TV* v, TV* y, const float* Y) {
    Apply2DArgs<float> a = args2d<float>(c);
    a.pack = pack_for(a);
    a.corr = Y;
    a.cF = c->pc_factor;
    a.cs = 1.0 / std::sqrt((double)c->nvec);
    a.bcorr.y = Y;
    a.bcorr.phi = c->pc_phi;
    a.bcorr.F = c->pc_factor;
    a.bcorr.Hc = c->ny / c->pc_factor;
    a.bcorr.Wc = c->nx / c->pc_factor;
    a.bcorr.coef = c->pc_coef;
    if (apply2d_from_b<float>(a, v, y)) return set_error(RTE_EUNSUPPORTED, "apply: unsupported size");
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "apply launch", __FILE__, __LINE__);
}

// ------------------------------------------------------------------ autotuning -----------------
// Every pass of the 2D apply has a few kernel variants with the same arithmetic (different row
// tiles, thread counts, FFT grouping).  The tuner times each variant of each pass on the
// context's own buffers (`reps` launches between events, the other passes at their current
// choice) and keeps the fastest.  Choices are cached per (precision, L, nx, ny) for the process.

static std::mutex g_tune_mu;
static std::map<std::vector<int>, std::vector<int>> g_tune_cache;

template <typename T>
static int tune_t(rte_ctx* c, int* var, int reps, bool use_cache) {
    const std::vector<int> key = {(int)sizeof(T), c->L, c->nx, c->ny};
    if (use_cache) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            for (int p = 0; p < 3; ++p) var[p] = it->second[p];
            return RTE_OK;
        }
    }
    const ChanScale sc = channel_scale(c, APPLY_A);
    vec_fill(c->t0, 1.0, c->nvec, c->stream);
    hipEvent_t e0, e1;
    RTE_HIP_TRY(hipEventCreate(&e0));
    RTE_HIP_TRY(hipEventCreate(&e1));
    int rc = RTE_OK;
    for (int pass = 0; pass < 3 && !rc; ++pass) {
        const int nv = apply2d_variant_count<T>(pass, c->L, c->PX, c->PY);
        int best = 0;
        float best_ms = 1e30f;
        for (int v = 0; v < nv && !rc; ++v) {
            Apply2DArgs<T> a = args2d<T>(c);
            for (int p = 0; p < 3; ++p) a.var[p] = var[p];
            a.var[pass] = v;
            a.pack = pack_for(a);
            // one full apply first: the work buffer then holds a valid spectrum for passes B and C
            if (apply2d<T>(a, c->t0, nullptr, c->t1, APPLY_A, sc, 1)) { rc = set_error(RTE_EUNSUPPORTED, "tune"); break; }
            (void)hipEventRecord(e0, c->stream);
            for (int r = 0; r < reps; ++r) {
                int lr = pass == 0 ? apply2d_pass_a<T>(a, c->t0, sc, 1)
                                   : pass == 1 ? apply2d_pass_b<T>(a, 1) : apply2d_pass_c<T>(a, c->t0, nullptr, c->t1, APPLY_A, 1);
                if (lr) { rc = set_error(RTE_EUNSUPPORTED, "tune"); break; }
            }
            (void)hipEventRecord(e1, c->stream);
            hipError_t e = hipEventSynchronize(e1);
            if (e != hipSuccess) { rc = set_hip_error(e, "tune", __FILE__, __LINE__); break; }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best_ms) { best_ms = ms; best = v; }
        }
        var[pass] = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = std::vector<int>(var, var + 3);
    return RTE_OK;
}

int autotune_2d(rte_ctx* c, int reps, bool use_cache) {
    if (c->dim != 2) return RTE_OK;
    int rc = tune_t<double>(c, c->vard, reps, use_cache);
    if (!rc && c->prec == RTE_PREC_FP32) rc = tune_t<float>(c, c->varf, reps, use_cache);
    return rc;
}

// ------------------------------------------------------------------ small host helpers ---------

// Slots of device-visible host memory that the device writes once per use: the host sets them to
// kPending before the work that writes them is enqueued and polls them, which wakes it sooner than
// a blocking synchronisation.  The device values (an estimate |g|, a sum of squares) are never
// negative, so the sentinel cannot be confused with one (NaN included).
constexpr double kPending = -1.0;

static int wait_slot(rte_ctx* c, const double* slot) {
    const volatile double* p = slot;
    const double t0 = now_ms();
    while (*p == kPending) {
        if (now_ms() - t0 > 20.0) {   // a long step: block on the stream instead
            RTE_HIP_TRY(hipStreamSynchronize(c->stream));
            if (*p == kPending) return set_error(RTE_EDEVICE, "device result missing after synchronisation");
            break;
        }
    }
    return RTE_OK;
}

// <a, b> into device-visible host memory (slot m of hpipe): enqueue, then wait for the slot.
static void dot_enqueue(rte_ctx* c, const double* a, const double* b, size_t n = 0) {
    const int m = c->krylov_m;
    if (!n) n = c->nvec;
    c->hpipe[m] = kPending;
    krylov_dots(a, n, 1, b, n, c->partial, c->hpipe_dev + m, false, c->stream);
}
static int dot_wait(rte_ctx* c, double* out) {
    const int m = c->krylov_m;
    int rc = wait_slot(c, c->hpipe + m);
    if (rc) return rc;
    *out = c->hpipe[m];
    return RTE_OK;
}

// ------------------------------------------------------------------ GMRES ---------------------

// TV: element type of the basis (double; float with the FP32 apply when opts.basis_fp32 is set);
// the Hessenberg matrix, rotations, dot products, x and the true residual are FP64 in both.
template <typename TV>
static int solve_core_t(rte_ctx* c, const double* b, double tol, int max_iter, double* x, rte_solve_info* info,
                        double* rec, int max_rec, int* nrec, const SolveFinish* finish, int nb) {
    const double t_start = now_ms();
    hipStream_t st = c->stream;
    const size_t n = (size_t)nb * c->nvec;
    const int m = c->opts.restart;
    // several stacked right-hand sides: no preconditioner, no recorded iterates
    const bool use_pc = c->pc_attached && c->opts.use_pc && nb == 1;
    if (nb > 1) rec = nullptr;
    double* const rv = nb > 1 ? c->rm : c->rv;
    const bool mixed = c->prec == RTE_PREC_FP32;
    int rc = ensure_krylov(c, m, false, sizeof(TV), n);
    if (rc) return rc;
    TV* const V = basis<TV>(c);
    if (use_pc && (rc = pc_begin_solve(c, m))) return rc;
    if (nrec) *nrec = 0;
    rte_solve_info inf;
    memset(&inf, 0, sizeof(inf));
    inf.t_setup_ms = c->t_setup_ms;
    inf.pc_used = use_pc ? 1 : 0;

    double bn2;
    // x = 0 and r = b do not depend on |b|: queued while the host waits for it
    dot_enqueue(c, b, b, n);
    vec_fill(x, 0.0, n, st);
    RTE_HIP_TRY(hipMemcpyAsync(rv, b, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    if ((rc = dot_wait(c, &bn2))) return rc;
    if (!std::isfinite(bn2)) {
        inf.status = RTE_ENUMERIC;
        if (info) *info = inf;
        return set_error(RTE_ENUMERIC, "non-finite right-hand side");
    }
    if (bn2 == 0.0) {
        if (finish && finish->fn) finish->fn(c, finish->arg);
        RTE_HIP_TRY(hipStreamSynchronize(st));
        inf.t_solve_ms = now_ms() - t_start;
        if (info) *info = inf;
        return RTE_OK;
    }
    const double bn = std::sqrt(bn2);
    double rn = bn;
    int it = 0, cycles = 0, status = RTE_NOT_CONVERGED;
    double est = bn;
    // the output step ran after the last change of x: it is enqueued with a cycle's true residual
    // only when that cycle can end the solve (its target within 100x of the tolerance), else once
    // after the last cycle
    bool finish_fresh = false;
    bool pc_live = use_pc;
    // single-pass Gram-Schmidt with the normalisation (and the network's restriction) fused into the
    // update; the preconditioned form needs one partial sum per pooling block in c->partial
    const bool fused = c->opts.reorth == 0 &&
                       (!use_pc || (size_t)pc_update_pool_blocks(c) <= (size_t)(m + 3) * RTE_KRYLOV_NBLK);
    const bool rescale_net = fused && use_pc && pc_rescale_net_ok(c);
    const bool early_a = rescale_net && early_a_ok(c);
    // tolerance on |v_{j+1}|^2 - 1 beyond which the stored vector is rescaled; RTE_RENORM_TOL
    // overrides it (a negative value rescales at every step, which tests use)
    const char* renorm_env = std::getenv("RTE_RENORM_TOL");
    const double renorm_tol = renorm_env ? std::atof(renorm_env) : (mixed ? 1e-8 : 1e-10);

    double* dH = c->arn;
    double* dcs = dH + (size_t)(m + 1) * m;
    double* dsn = dcs + m;
    double* dg = dsn + m;
    double* dest = dg + m + 1;
    double* dinv = dest + m;
    int* dfl = c->arn_flags;
    double* hp = c->hpipe;          // per-iteration residual estimates
    int* hfl = c->hpipe_flags;      // per-iteration (breakdown, non-finite)
    while (true) {
        if (rn <= tol * bn) { status = RTE_OK; break; }
        if (cycles >= c->opts.max_cycles || it >= max_iter) { status = RTE_NOT_CONVERGED; break; }
        ++cycles;
        double target = 0.5 * tol * bn;
        if (mixed) target = std::max(target, c->opts.inner_tol * rn);
        const bool may_end = target <= 100.0 * tol * bn;
        // v_0 = r / rn (with the pooled coarse input of the network when preconditioning)
        if (pc_live) {   // with g = (rn, 0, ...) and the flags cleared in the same launch
            pc_scale_pool(c, (const double*)rv, V, nullptr, 1.0 / rn, dg, m + 1, rn, dfl, 4);
        } else {
            vec_scale(V, rv, 1.0 / rn, n, st);
            init_g(dg, m + 1, rn, dfl, 4, st);
        }
        est = rn;
        const double cycle_start_rn = rn;
        // Iterations are enqueued one ahead of the convergence check: when iteration j is queued the
        // host reads the estimate of iteration j-1, so the device never waits for the host.
        int jd = 0;           // columns of this cycle that are valid
        int launched = 0;
        bool net_ready = false;   // the network output of the next step is already being computed
        bool a_ready = false;     // and pass A of its apply (early_a)
        bool stop = false, bad = false;
        for (int j = 0; j < m && it + launched < max_iter && !stop; ++j) {
            TV* vj = V + (size_t)j * n;
            TV* w = V + (size_t)(j + 1) * n;
            // flexible GMRES: w = A z_j with z_j = v_j + s P Y_j formed inside the apply
            if (pc_live) {
                if (!net_ready && early_a && j == 0) {   // v_0's network beside its pass A
                    const Apply2DArgs<float> a = args2d<float>(c);
                    if ((rc = pc_rescale_net_pa<TV>(c, nullptr, vj, c->partial, 0, channel_scale(c, APPLY_A), pack_for(a))))
                        return rc;
                    a_ready = true;
                } else if (!net_ready && (rc = pc_net_slot(c, j))) {   // else the last launch ran it
                    return rc;
                }
                net_ready = false;
                rc = a_ready ? apply_basis_pc_from_b(c, vj, w, pc_slot(c, j)) : apply_basis_pc(c, vj, w, pc_slot(c, j));
                a_ready = false;
                if (rc) return rc;
            } else if ((rc = apply_basis(c, vj, w, nb))) {
                return rc;
            }
            ++inf.applies;
            hp[j] = kPending;   // written by this step's Arnoldi stage 1
            double* sd = c->dsmall;
            // Arnoldi column j on the device (stage 0 after the dots, stage 1 after the update)
            ArnoldiArgs at;
            at.j = j;
            at.m = m;
            at.reorth = c->opts.reorth;
            at.fused = fused ? 1 : 0;
            at.renorm_tol = renorm_tol;
            at.st = sd;
            at.H = dH;
            at.cs = dcs;
            at.sn = dsn;
            at.g = dg;
            at.est = dest;
            at.inv = dinv;
            at.flags = dfl;
            if (fused) {
                // one pass: the update computes the normalising factor from |w|^2 - |h|^2 and writes
                // the normalised vector (and, when preconditioning, the network's pooled input),
                // with stage 0 of the column in its block 0; the rescale kernel runs stage 1 in its
                // block 0 and rescales only when the device finds the norm off
                krylov_dots(V, n, j + 1, w, n, c->partial, sd, true, st);
                at.stage = 0;
                // the update leaves its per-block partial sums of the new norm in c->partial; the
                // rescale kernel adds them up itself
                if (pc_live) pc_update_pool(c, w, V, j + 1, c->partial, nullptr, at);
                else krylov_update(w, V, n, j + 1, sd, n, c->partial, nullptr, st, nullptr, &at);
                at.stage = 1;
                at.est_out = c->hpipe_dev + j;
                at.flags_out = c->hpipe_flags_dev + 2 * j;
                if (pc_live && j + 1 < m && rescale_net) {
                    // stage 1 and the next step's network in one launch (with the next apply's
                    // pass A on the other blocks when early_a)
                    if (early_a) {
                        const Apply2DArgs<float> a = args2d<float>(c);
                        if ((rc = pc_rescale_net_pa(c, &at, w, c->partial, j + 1, channel_scale(c, APPLY_A), pack_for(a))))
                            return rc;
                        a_ready = true;
                    } else if ((rc = pc_rescale_net(c, at, w, c->partial, j + 1))) {
                        return rc;
                    }
                    net_ready = true;
                } else if (pc_live) {
                    pc_rescale_pool_arn1(c, at, w, c->partial);
                } else {
                    rescale_arn1(at, w, n, c->partial, (int)krylov_nblk(n), st);
                }
            } else {
                krylov_dots(V, n, j + 1, w, n, c->partial, sd, true, st);
                krylov_update(w, V, n, j + 1, sd, n, c->partial, sd + j + 2, st);
                at.stage = 0;
                arnoldi_run(at, st);
                if (c->opts.reorth > 0) {   // second pass, skipped on the device unless flagged
                    krylov_dots(V, n, j + 1, w, n, c->partial, sd + m + 4, false, st, dfl);
                    krylov_update(w, V, n, j + 1, sd + m + 4, n, c->partial, sd + j + 2, st, dfl);
                }
                at.stage = 1;
                at.est_out = c->hpipe_dev + j;
                at.flags_out = c->hpipe_flags_dev + 2 * j;
                arnoldi_run(at, st);
                if (pc_live) pc_scale_pool(c, w, w, dinv + j + 1, 0.0);
                else vec_scale_dev(w, w, dinv + j + 1, n, st);
            }
            // no event per step: an event record releases the caches at system scope, an idle
            // gap of about 6 us before the next launch; the host polls the slot instead
            ++launched;
            // check the previous iteration
            if (j >= 1) {
                if ((rc = wait_slot(c, hp + (j - 1)))) return rc;
                const double e1 = hp[j - 1];
                if (hfl[2 * (j - 1) + 1] != 0 || !std::isfinite(e1)) { bad = true; stop = true; break; }
                if (hfl[2 * (j - 1)] != 0) { est = e1; jd = j; stop = true; break; }   // breakdown: drop column j
                est = e1;
                jd = j;
                if (e1 <= target) stop = true;                                  // column j is kept too
            }
        }
        // The cycle end (least squares, solution update, true residual and its norm) is enqueued
        // before the last iteration's flags are read, so the device has it queued when that
        // iteration ends.  The column count assumes that iteration is sound; if it produced a
        // non-finite value, the back-substitution and the update see the device's flag and leave
        // x unchanged (the network outputs may then be non-finite too, so the update is skipped,
        // not multiplied by zero), and the host, reading the same flags below, handles the cycle
        // as before.  Recording solves keep the ordered path.
        const bool spec = launched > 0 && !bad && !(rec && cycles == 1);
        if (spec) {
            const int jl = launched - 1;
            const bool prev_brk = jl >= 1 && hfl[2 * (jl - 1)] != 0;
            const bool last_kept = !prev_brk && jd == jl;   // the host's condition for column jl
            const int jd_end = last_kept ? jl + 1 : jd;
            if (jd_end > 0) {
                const int* guard = last_kept ? dfl : nullptr;
                back_solve_dev(dH, m + 1, dg, jd_end, c->dsmall, st, guard);
                if (pc_live) pc_combine(c, x, (const TV*)V, jd_end, c->dsmall, guard);
                else krylov_combine(x, V, n, jd_end, c->dsmall, n, st, guard);
            }
            if ((rc = apply_channels(c, APPLY_RESID, RTE_PREC_FP64, x, b, rv, nb))) return rc;
            ++inf.applies;
            dot_enqueue(c, rv, rv, n);
            finish_fresh = false;
            if (finish && finish->fn && may_end) {   // runs while the host waits
                finish->fn(c, finish->arg);
                finish_fresh = true;
            }
        }
        // settle the last enqueued iteration
        if (launched > 0 && (rc = wait_slot(c, hp + (launched - 1)))) return rc;
        if (!bad && launched > 0) {
            const int jl = launched - 1;
            const bool prev_brk = jl >= 1 && hfl[2 * (jl - 1)] != 0;
            if (!prev_brk && jd == jl) {
                if (hfl[2 * jl + 1] != 0 || !std::isfinite(hp[jl])) bad = true;
                else { est = hp[jl]; jd = jl + 1; }
            }
        }
        it += launched;
        if (bad) {
            if (spec) {   // the enqueued cycle end left x unchanged; take its norm out of the slot
                double unused;
                if ((rc = dot_wait(c, &unused))) return rc;
            }
            if (pc_live) {   // a broken preconditioner: restart this cycle without it
                pc_live = false;
                inf.pc_fallback = 1;
                continue;
            }
            if (finish && finish->fn && !finish_fresh) finish->fn(c, finish->arg);
            inf.iterations = it;
            inf.cycles = cycles;
            inf.status = RTE_ENUMERIC;
            if (info) *info = inf;
            return set_error(RTE_ENUMERIC, "non-finite value in the Arnoldi process");
        }
        if (!spec) {
            if (jd > 0) {
                // least squares on the device: the rotated H and g never leave it
                if (rec && cycles == 1) {
                    const int nr = std::min(jd, max_rec);
                    for (int k = 1; k <= nr; ++k) {
                        back_solve_dev(dH, m + 1, dg, k, c->dsmall, st);
                        double* xr = rec + (size_t)(k - 1) * n;
                        vec_fill(xr, 0.0, n, st);
                        if (pc_live) pc_combine(c, xr, (const TV*)V, k, c->dsmall);
                        else krylov_combine(xr, V, n, k, c->dsmall, n, st);
                    }
                    if (nrec) *nrec = nr;
                }
                back_solve_dev(dH, m + 1, dg, jd, c->dsmall, st);
                if (pc_live) pc_combine(c, x, (const TV*)V, jd, c->dsmall);
                else krylov_combine(x, V, n, jd, c->dsmall, n, st);
            }
            // true residual with the FP64 apply
            if ((rc = apply_channels(c, APPLY_RESID, RTE_PREC_FP64, x, b, rv, nb))) return rc;
            ++inf.applies;
            dot_enqueue(c, rv, rv, n);
            finish_fresh = false;
            if (finish && finish->fn && may_end) {   // runs while the host waits
                finish->fn(c, finish->arg);
                finish_fresh = true;
            }
        }
        double rn2;
        if ((rc = dot_wait(c, &rn2))) return rc;
        if (!std::isfinite(rn2)) {
            if (finish && finish->fn && !finish_fresh) finish->fn(c, finish->arg);
            inf.iterations = it;
            inf.cycles = cycles;
            inf.status = RTE_ENUMERIC;
            if (info) *info = inf;
            return set_error(RTE_ENUMERIC, "non-finite true residual");
        }
        rn = std::sqrt(rn2);
        // the preconditioned cycle must cut the residual at least 10x (or reach twice its own
        // target, when that asks for less), else the solve continues without it; a cycle that
        // ends the solve is not judged
        if (pc_live && rn > tol * bn && rn > std::max(0.1 * cycle_start_rn, 2.0 * target)) {
            pc_live = false;
            inf.pc_fallback = 1;
        }
    }
    if (finish && finish->fn && !finish_fresh) finish->fn(c, finish->arg);
    RTE_HIP_TRY(hipStreamSynchronize(st));
    inf.iterations = it;
    inf.cycles = cycles;
    inf.relres_est = est / bn;
    inf.relres_true = rn / bn;
    inf.t_solve_ms = now_ms() - t_start;
    inf.status = status;
    if (info) *info = inf;
    if (status == RTE_NOT_CONVERGED)
        set_error(RTE_NOT_CONVERGED, "not converged: relative residual %.3e after %d iterations", rn / bn, it);
    return status;
}

int solve_core(rte_ctx* c, const double* b, double tol, int max_iter, double* x, rte_solve_info* info,
               double* rec, int max_rec, int* nrec, const SolveFinish* finish, int nb) {
    if (c->prec == RTE_PREC_FP32 && c->opts.basis_fp32)
        return solve_core_t<float>(c, b, tol, max_iter, x, info, rec, max_rec, nrec, finish, nb);
    return solve_core_t<double>(c, b, tol, max_iter, x, info, rec, max_rec, nrec, finish, nb);
}

}  // namespace rte

using namespace rte;

// Per-pass event timing of `reps` applies of nb stacked channel vectors x -> y.
static int time_apply_impl(rte_ctx* c, int op, int prec, int reps, int nb, const double* x, double* y,
                           double* ms_total, double* ms_pass) {
    if (prec == RTE_PREC_FP32 && c->prec != RTE_PREC_FP32) return set_error(RTE_EINVAL, "FP32 apply needs an FP32 context");
    const int mode = op == RTE_OP_A ? APPLY_A : APPLY_KT;
    const int nev = c->dim == 2 ? 4 : 6;
    hipEvent_t ev[6];
    for (int i = 0; i < nev; ++i) RTE_HIP_TRY(hipEventCreate(&ev[i]));
    std::vector<double> acc(nev, 0.0);
    int rc = RTE_OK;
    for (int r = 0; r < reps && !rc; ++r) {
        rc = prec == RTE_PREC_FP32 ? apply_t<float>(c, mode, x, nullptr, y, nb, ev)
                                   : apply_t<double>(c, mode, x, nullptr, y, nb, ev);
        if (rc) break;
        RTE_HIP_TRY(hipEventSynchronize(ev[nev - 1]));
        for (int i = 1; i < nev; ++i) {
            float ms = 0.f;
            RTE_HIP_TRY(hipEventElapsedTime(&ms, ev[i - 1], ev[i]));
            acc[i] += ms;
        }
    }
    for (int i = 0; i < nev; ++i) (void)hipEventDestroy(ev[i]);
    if (rc) return rc;
    double tot = 0.0;
    for (int i = 1; i < nev; ++i) tot += acc[i];
    if (ms_total) *ms_total = tot / reps;
    if (ms_pass) {
        for (int i = 0; i < 5; ++i) ms_pass[i] = 0.0;
        for (int i = 1; i < nev; ++i) ms_pass[i - 1] = acc[i] / reps;
    }
    return RTE_OK;
}


// 3D: passes 0 and 4 are the 2D x-passes (row-tile variants), 1..3 the y-, z- and inverse y-passes.
template <typename T>
static int variant_count3(const rte_ctx* c, int pass) {
    if (pass == 0 || pass == 4) return apply2d_variant_count<T>(pass == 0 ? 0 : 2, 0, c->PX, c->PY);
    return apply3d_variant_count<T>(pass, c->C, c->PZ);
}

// The 3D tuner: each pass's variants timed in turn (the others at their current choice) from the
// per-pass events of `reps` applies, the fastest kept; cached per (precision, L, n) for the process.
template <typename T>
static int tune3_t(rte_ctx* c, int* var, int reps, bool use_cache) {
    const std::vector<int> key = {3, (int)sizeof(T), c->L, c->nx, c->ny, c->nz};
    if (use_cache) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            for (int p = 0; p < 5; ++p) var[p] = it->second[p];
            return RTE_OK;
        }
    }
    const int prec = sizeof(T) == 4 ? RTE_PREC_FP32 : RTE_PREC_FP64;
    vec_fill(c->t0, 1.0, c->nvec, c->stream);
    for (int pass = 0; pass < 5; ++pass) {
        const int nv = variant_count3<T>(c, pass);
        int best = var[pass];
        double best_ms = 1e30;
        for (int v = 0; v < nv; ++v) {
            var[pass] = v;
            double tot = 0.0, ms[5] = {0, 0, 0, 0, 0};
            int rc = time_apply_impl(c, RTE_OP_A, prec, reps, 1, c->t0, c->t1, &tot, ms);
            if (rc) return rc;
            if (ms[pass] < best_ms) { best_ms = ms[pass]; best = v; }
        }
        var[pass] = best;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = std::vector<int>(var, var + 5);
    return RTE_OK;
}

static int autotune_3d(rte_ctx* c, int reps, bool use_cache) {
    int rc = tune3_t<double>(c, c->var3d, reps, use_cache);
    if (!rc && c->prec == RTE_PREC_FP32) rc = tune3_t<float>(c, c->var3f, reps, use_cache);
    return rc;
}

// ------------------------------------------------------------------ C ABI --------------------

extern "C" {

const char* rte_last_error(void) { return g_err; }
const char* rte_version(void) { return "rte-mi355x 0.1 (gfx950)"; }

static int validate_setup(const rte_grid* g, double mu_a, double mu_s, const double* sigma_hat, int L, int prec) {
    if (!g) return set_error(RTE_EINVAL, "grid is NULL");
    if (g->dim != 2 && g->dim != 3) return set_error(RTE_EINVAL, "dim must be 2 or 3 (got %d)", g->dim);
    for (int a = 0; a < g->dim; ++a)
        if (g->n[a] < 2) return set_error(RTE_EINVAL, "n[%d] = %d must be >= 2", a, g->n[a]);
    if (!(g->h > 0.0) || !std::isfinite(g->h)) return set_error(RTE_EINVAL, "h must be finite and > 0");
    if (!(mu_a >= 0.0) || !std::isfinite(mu_a)) return set_error(RTE_EINVAL, "mu_a must be finite and >= 0");
    if (!(mu_s >= 0.0) || !std::isfinite(mu_s)) return set_error(RTE_EINVAL, "mu_s must be finite and >= 0");
    if (!(mu_a + mu_s > 0.0)) return set_error(RTE_EINVAL, "mu_t = mu_a + mu_s must be > 0");
    if (L < 0 || L > RTE_MAX_L) return set_error(RTE_EINVAL, "L = %d outside 0..%d", L, RTE_MAX_L);
    if (prec != RTE_PREC_FP32 && prec != RTE_PREC_FP64) return set_error(RTE_EINVAL, "prec must be FP32 or FP64");
    if (L > 0 && !sigma_hat) return set_error(RTE_EINVAL, "sigma_hat is NULL with L > 0");
    if (sigma_hat) {
        if (std::fabs(sigma_hat[0] - 1.0) > 1e-12) return set_error(RTE_EINVAL, "sigma_hat[0] must be 1 (normalised phase function)");
        for (int k = 1; k <= L; ++k)
            if (!(std::fabs(sigma_hat[k]) <= 1.0)) return set_error(RTE_EINVAL, "|sigma_hat[%d]| must be <= 1", k);
    }
    if (g->dim == 3 && L > RTE_MAX_L3)
        return set_error(RTE_EUNSUPPORTED, "3D keeps spherical harmonics up to degree %d (L = %d)", RTE_MAX_L3, L);
    const int nmax = g->dim == 2 ? 512 : (L > 0 ? 128 : 256);
    for (int a = 0; a < g->dim; ++a)
        if (g->n[a] > nmax) return set_error(RTE_EUNSUPPORTED, "n[%d] = %d exceeds %d", a, g->n[a], nmax);
    return RTE_OK;
}

int rte_setup(rte_ctx** out, const rte_grid* g, double mu_a, double mu_s, const double* sigma_hat, int L, int prec,
              void* hip_stream) {
    if (!out) return set_error(RTE_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_setup(g, mu_a, mu_s, sigma_hat, L, prec);
    if (rc) return rc;
    const double t0 = now_ms();
    rte_ctx* c = new (std::nothrow) rte_ctx();
    static std::atomic<unsigned long long> next_id{1};
    if (c) c->id = next_id.fetch_add(1);
    if (!c) return set_error(RTE_ENOMEM, "host allocation failed");
    c->dim = g->dim;
    c->nx = g->n[0];
    c->ny = g->n[1];
    c->nz = g->dim == 3 ? g->n[2] : 1;
    c->h = g->h;
    c->L = L;
    c->C = g->dim == 3 ? sh_modes(L) : 2 * L + 1;   // 3D: real spherical harmonics to degree L
    c->M = c->C;
    c->prec = prec;
    c->mu_a = mu_a;
    c->mu_s = mu_s;
    c->mu_t = mu_a + mu_s;
    c->sigma.assign(L + 1, 1.0);
    for (int k = 0; k <= L && sigma_hat; ++k) c->sigma[k] = sigma_hat[k];
    c->stream = (hipStream_t)hip_stream;
    c->PX = next_pow2(std::max(2 * c->nx - 1, 16));
    c->PY = next_pow2(std::max(2 * c->ny - 1, 16));
    c->PZ = c->dim == 3 ? next_pow2(std::max(2 * c->nz - 1, 16)) : 1;
    c->ncell = (size_t)c->nx * c->ny * c->nz;
    c->nvec = (size_t)c->C * c->ncell;
    c->opts.restart = 64;
    c->opts.max_cycles = 8;
    c->opts.inner_tol = 3e-4;
    c->opts.reorth = 0;
    c->opts.use_pc = 1;
    c->opts.basis_fp32 = 0;
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) { free_ctx(c); return set_hip_error(e, "hipGetDevice", __FILE__, __LINE__); }

    // twiddles of the grid axes, and of the mode axis when pass B couples the modes by an FFT
    const bool mode_fft = c->dim == 2 && c->L > PASSB_FUSED_MAX_L;
    // (index 4: the y axis in the radix-32 schedule, for the pass-B variant that uses it; index 5:
    // length PY/2, for pass B split in halves)
    const int Ps[6] = {c->PX, c->PY, c->PZ, mode_fft ? mode_fft_len(c->L) : 0, c->PY, c->PY / 2};
    for (int a = 0; a < 6; ++a) {
        if (a >= c->dim && !(a == 3 && mode_fft) && !(a >= 4 && c->dim == 2)) continue;
        std::vector<double> re, im;
        twiddles(Ps[a], re, im, a == 4 ? 1 : 0);
        std::vector<cx<double>> td(Ps[a]);
        std::vector<cx<float>> tf(Ps[a]);
        for (int q = 0; q < Ps[a]; ++q) {
            td[q] = mk(re[q], im[q]);
            tf[q] = mk((float)re[q], (float)im[q]);
        }
        cx<double>*& dd = a < 3 ? c->twd[a] : (a == 3 ? c->twmd : (a == 4 ? c->twy1d : c->twyhd));
        cx<float>*& ff = a < 3 ? c->twf[a] : (a == 3 ? c->twmf : (a == 4 ? c->twy1f : c->twyhf));
        if ((rc = dalloc(&dd, Ps[a])) || (rc = dalloc(&ff, Ps[a]))) { free_ctx(c); return rc; }
        e = hipMemcpy(dd, td.data(), Ps[a] * sizeof(cx<double>), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(ff, tf.data(), Ps[a] * sizeof(cx<float>), hipMemcpyHostToDevice);
        if (e != hipSuccess) { free_ctx(c); return set_hip_error(e, "twiddle upload", __FILE__, __LINE__); }
    }
    const bool f32 = prec == RTE_PREC_FP32;
    const int NK = c->PX / 2 + 1;
    // spectra (FP64 on the device)
    {
        const size_t np = (size_t)c->PX * c->PY * c->PZ;
        cx<double>*b0 = nullptr, *b1 = nullptr;
        if ((rc = dalloc(&b0, np)) || (rc = dalloc(&b1, np))) { dfree(b0); dfree(b1); free_ctx(c); return rc; }
        if (c->dim == 2) {
            const size_t nq = (size_t)c->C * NK * (c->PY / 2 + 1);
            if ((rc = dalloc(&c->Qd, nq)) || (f32 && (rc = dalloc(&c->Qf, nq)))) { dfree(b0); dfree(b1); free_ctx(c); return rc; }
            SpectraArgs2D a{c->nx, c->ny, c->PX, c->PY, c->L, c->h, c->mu_t, b0, b1, c->twd[0], c->twd[1],
                            c->Qf, c->Qd, c->stream};
            rc = build_spectra_2d(a);
        } else {
            const size_t no = (size_t)NK * (c->PY / 2 + 1) * (c->PZ / 2 + 1);
            const size_t npair = (size_t)c->C * (c->C + 1) / 2;   // one octant per mode pair a <= b
            if ((rc = dalloc(&c->Q3d, no * npair)) || (f32 && (rc = dalloc(&c->Q3f, no * npair)))) { dfree(b0); dfree(b1); free_ctx(c); return rc; }
            SpectraArgs3D a{c->nx, c->ny, c->nz, c->PX, c->PY, c->PZ, c->h, c->mu_t, b0, b1,
                            c->twd[0], c->twd[1], c->twd[2], c->Q3f, c->Q3d, c->stream};
            rc = c->L == 0 ? build_spectrum_3d(a) : build_spectra_3d_sh(a, c->L);
        }
        e = hipStreamSynchronize(c->stream);
        dfree(b0);
        dfree(b1);
        if (rc || e != hipSuccess) { free_ctx(c); return rc ? set_error(RTE_EDEVICE, "spectrum build failed") : set_hip_error(e, "spectra", __FILE__, __LINE__); }
    }
    // work buffers, sized for two right-hand sides (the general complex apply)
    const int nb = 2;
    if (c->dim == 2) {
        const size_t nt = (size_t)nb * c->C * NK * c->ny;
        const size_t nt2 = (size_t)nb * c->C * NK * c->PY;
        if ((rc = dalloc(&c->wd, nt))) { free_ctx(c); return rc; }
        if (apply2d_needs_work2<double>(c->L, c->PY) && (rc = dalloc(&c->wd2, nt2))) { free_ctx(c); return rc; }
        if (f32) {
            if ((rc = dalloc(&c->wf, nt))) { free_ctx(c); return rc; }
            if (apply2d_needs_work2<float>(c->L, c->PY) && (rc = dalloc(&c->wf2, nt2))) { free_ctx(c); return rc; }
        }
    } else {
        const size_t n1 = (size_t)nb * c->C * c->nz * NK * c->ny;
        const size_t n2 = (size_t)c->C * NK * c->PY * c->nz;
        if ((rc = dalloc(&c->wd, n1)) || (rc = dalloc(&c->wd2, n2))) { free_ctx(c); return rc; }
        if (f32 && ((rc = dalloc(&c->wf, n1)) || (rc = dalloc(&c->wf2, n2)))) { free_ctx(c); return rc; }
    }
    const size_t n = c->nvec;
    if ((rc = dalloc(&c->xv, n)) || (rc = dalloc(&c->rv, n)) || (rc = dalloc(&c->bv, n)) ||
        (rc = dalloc(&c->t0, 2 * n)) || (rc = dalloc(&c->t1, 2 * n)) || (rc = dalloc(&c->dflag, 4))) {
        free_ctx(c);
        return rc;
    }
    if ((rc = ensure_krylov(c, c->opts.restart, false, sizeof(double)))) {
        free_ctx(c);
        return rc;
    }
    // kernel variants: tuned once per shape and process (RTE_AUTOTUNE=0 keeps the defaults)
    const char* at = std::getenv("RTE_AUTOTUNE");
    if (c->dim == 2 && std::max(c->nx, c->ny) >= 128 && !(at && at[0] == '0')) {
        if ((rc = autotune_2d(c, 5, true))) { free_ctx(c); return rc; }
    }
    if (c->dim == 3 && std::max(c->nx, std::max(c->ny, c->nz)) >= 64 && !(at && at[0] == '0')) {
        if ((rc = autotune_3d(c, 3, true))) { free_ctx(c); return rc; }
    }
    c->t_setup_ms = now_ms() - t0;
    *out = c;
    return RTE_OK;
}

int rte_autotune(rte_ctx* c, int reps) {
    if (!c || reps < 1) return set_error(RTE_EINVAL, "bad argument");
    return c->dim == 2 ? autotune_2d(c, reps, false) : autotune_3d(c, reps, false);
}

static int variant_count(const rte_ctx* c, int prec, int pass) {
    const bool f = prec == RTE_PREC_FP32;
    if (c->dim == 3) return f ? variant_count3<float>(c, pass) : variant_count3<double>(c, pass);
    return f ? apply2d_variant_count<float>(pass, c->L, c->PX, c->PY)
             : apply2d_variant_count<double>(pass, c->L, c->PX, c->PY);
}

int rte_set_variant(rte_ctx* c, int prec, int pass, int variant) {
    if (!c || (prec != RTE_PREC_FP32 && prec != RTE_PREC_FP64)) return set_error(RTE_EINVAL, "bad argument");
    const int npass = c->dim == 2 ? 3 : 5;
    if (pass < 0 || pass >= npass) return set_error(RTE_EINVAL, "pass %d out of range (%d passes)", pass, npass);
    const int nv = variant_count(c, prec, pass);
    if (variant < 0 || variant >= nv) return set_error(RTE_EINVAL, "variant %d out of range (%d variants)", variant, nv);
    if (c->dim == 2) (prec == RTE_PREC_FP32 ? c->varf : c->vard)[pass] = variant;
    else (prec == RTE_PREC_FP32 ? c->var3f : c->var3d)[pass] = variant;
    return RTE_OK;
}

int rte_get_variant(const rte_ctx* c, int prec, int pass, int* variant, int* count) {
    if (!c || (prec != RTE_PREC_FP32 && prec != RTE_PREC_FP64)) return set_error(RTE_EINVAL, "bad argument");
    const int npass = c->dim == 2 ? 3 : 5;
    if (pass < 0 || pass >= npass) return set_error(RTE_EINVAL, "pass %d out of range (%d passes)", pass, npass);
    if (variant)
        *variant = c->dim == 2 ? (prec == RTE_PREC_FP32 ? c->varf : c->vard)[pass]
                               : (prec == RTE_PREC_FP32 ? c->var3f : c->var3d)[pass];
    if (count) *count = variant_count(c, prec, pass);
    return RTE_OK;
}

void rte_destroy(rte_ctx* ctx) { free_ctx(ctx); }

int rte_query(const rte_ctx* c, int* channels, int* modes, long long* cells) {
    if (!c) return set_error(RTE_EINVAL, "ctx is NULL");
    if (channels) *channels = c->C;
    if (modes) *modes = c->M;
    if (cells) *cells = (long long)c->ncell;
    return RTE_OK;
}

int rte_set_solve_opts(rte_ctx* c, const rte_solve_opts* o) {
    if (!c) return set_error(RTE_EINVAL, "ctx is NULL");
    rte_solve_opts d;
    d.restart = 64;
    d.max_cycles = 8;
    d.inner_tol = 3e-4;
    d.reorth = 0;
    d.use_pc = 1;
    d.basis_fp32 = 0;
    if (o) {
        if (o->restart < 1 || o->restart > RTE_MAX_RESTART) return set_error(RTE_EINVAL, "restart must be in 1..%d", RTE_MAX_RESTART);
        if (o->max_cycles < 1) return set_error(RTE_EINVAL, "max_cycles must be >= 1");
        if (!(o->inner_tol > 0.0 && o->inner_tol < 1.0)) return set_error(RTE_EINVAL, "inner_tol must be in (0, 1)");
        if (o->reorth < 0 || o->reorth > 2) return set_error(RTE_EINVAL, "reorth must be 0, 1 or 2");
        if (o->basis_fp32 != 0 && o->basis_fp32 != 1) return set_error(RTE_EINVAL, "basis_fp32 must be 0 or 1");
        d = *o;
    }
    c->opts = d;
    return RTE_OK;
}

}  // extern "C"

// Complex modes <-> real channels: 2D pairs modes k and -k (rte.h), 3D modes are real already.
static void to_channels(const rte_ctx* c, const void* x, double* ch, bool one_part) {
    if (c->dim == 3) modes_to_channels_real(x, ch, c->nvec, one_part, c->stream);
    else modes_to_channels(x, ch, c->L, c->ncell, one_part, c->stream);
}
static void to_modes(const rte_ctx* c, const double* ch, void* y, bool one_part) {
    if (c->dim == 3) channels_to_modes_real(ch, y, c->nvec, one_part, c->stream);
    else channels_to_modes(ch, y, c->L, c->ncell, one_part, c->stream);
}

extern "C" {

int rte_apply(rte_ctx* c, int op, int layout, int prec, const void* x, void* y) {
    if (!c) return set_error(RTE_EINVAL, "ctx is NULL");
    if (op != RTE_OP_A && op != RTE_OP_KT) return set_error(RTE_EINVAL, "op must be RTE_OP_A or RTE_OP_KT");
    if (layout != RTE_LAYOUT_MODES && layout != RTE_LAYOUT_CHANNELS) return set_error(RTE_EINVAL, "bad layout");
    if (prec != RTE_PREC_FP32 && prec != RTE_PREC_FP64) return set_error(RTE_EINVAL, "bad prec");
    if (prec == RTE_PREC_FP32 && c->prec != RTE_PREC_FP32) return set_error(RTE_EINVAL, "FP32 apply needs an FP32 context");
    if (!x || !y) return set_error(RTE_EINVAL, "x or y is NULL");
    if (x == y) return set_error(RTE_EINVAL, "x and y may not alias");
    const int mode = op == RTE_OP_A ? APPLY_A : APPLY_KT;
    if (layout == RTE_LAYOUT_CHANNELS) return apply_channels(c, mode, prec, (const double*)x, nullptr, (double*)y, 1);
    to_channels(c, x, c->t0, false);
    int rc = apply_channels(c, mode, prec, c->t0, nullptr, c->t1, 2);
    if (rc) return rc;
    to_modes(c, c->t1, y, false);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "rte_apply", __FILE__, __LINE__);
}

int rte_modes_to_channels(rte_ctx* c, const void* modes, double* ch) {
    if (!c || !modes || !ch) return set_error(RTE_EINVAL, "NULL argument");
    to_channels(c, modes, ch, true);
    return RTE_OK;
}

int rte_channels_to_modes(rte_ctx* c, const double* ch, void* modes) {
    if (!c || !modes || !ch) return set_error(RTE_EINVAL, "NULL argument");
    to_modes(c, ch, modes, true);
    return RTE_OK;
}

// b = K~ g with g = f delta_{k0}: channel 0 carries f, the others are zero.
static int rhs_channels(rte_ctx* c, const double* f, double* b) {
    if (c->dim == 2 && c->C > 1) {
        // b = K~ (f, 0, ..., 0): pass A for channel 0 only, pass B reading channel 0 only (its
        // coupling writes every channel); inverse y-FFTs and pass C as usual
        Apply2DArgs<double> a = args2d<double>(c);
        a.pack = pack_for(a);
        const ChanScale sc = channel_scale(c, APPLY_KT);
        Apply2DArgs<double> a1 = a;
        a1.C = 1;
        if (apply2d_pass_a<double>(a1, f, sc, 1)) return set_error(RTE_EUNSUPPORTED, "rhs pass A: unsupported size");
        a.single_in = 1;
        if (apply2d_pass_b<double>(a, 1)) return set_error(RTE_EUNSUPPORTED, "rhs pass B: unsupported size");
        a.single_in = 0;
        if (apply2d_pass_c<double>(a, (const double*)nullptr, nullptr, b, APPLY_KT, 1))
            return set_error(RTE_EUNSUPPORTED, "rhs pass C: unsupported size");
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? RTE_OK : set_hip_error(e, "rhs launch", __FILE__, __LINE__);
    }
    vec_fill(c->t0, 0.0, c->nvec, c->stream);
    hipError_t e = hipMemcpyAsync(c->t0, f, c->ncell * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return set_hip_error(e, "rhs copy", __FILE__, __LINE__);
    return apply_channels(c, APPLY_KT, RTE_PREC_FP64, c->t0, nullptr, b, 1);
}

int rte_rhs(rte_ctx* c, const double* f, int layout, void* b) {
    if (!c || !f || !b) return set_error(RTE_EINVAL, "NULL argument");
    if (layout != RTE_LAYOUT_MODES && layout != RTE_LAYOUT_CHANNELS) return set_error(RTE_EINVAL, "bad layout");
    if (layout == RTE_LAYOUT_CHANNELS) return rhs_channels(c, f, (double*)b);
    int rc = rhs_channels(c, f, c->bv);
    if (rc) return rc;
    to_modes(c, c->bv, b, true);
    return RTE_OK;
}

int rte_solve(rte_ctx* c, const double* f, double tol, int max_iter, void* u, rte_solve_info* info) {
    if (!c || !f || !u) return set_error(RTE_EINVAL, "NULL argument");
    if (!(tol > 0.0) || !(tol < 1.0)) return set_error(RTE_EINVAL, "tol must be in (0, 1)");
    if (max_iter < 1) return set_error(RTE_EINVAL, "max_iter must be >= 1");
    int rc = rhs_channels(c, f, c->bv);
    if (rc) return rc;
    // the modes of x are written after every true residual, while the host waits for its norm
    SolveFinish fin;
    fin.fn = [](rte_ctx* cc, void* uu) { to_modes(cc, cc->xv, uu, true); };
    fin.arg = u;
    rc = solve_core(c, c->bv, tol, max_iter, c->xv, info, nullptr, 0, nullptr, &fin);
    if (rc < 0) return rc;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return set_hip_error(e, "rte_solve", __FILE__, __LINE__);
    if (rc == RTE_NOT_CONVERGED)
        set_error(RTE_NOT_CONVERGED, "not converged: relative residual %.3e", info ? info->relres_true : -1.0);
    return rc;
}

// b = K~ g for a source given by its angular modes g (all modes, not only mode 0): the FP64 apply
// of K~ to g in channel form.
static int rhs_source_channels(rte_ctx* c, const void* g, int layout, double* b) {
    const double* gc = (const double*)g;
    if (layout == RTE_LAYOUT_MODES) {
        to_channels(c, g, c->t0, true);
        gc = c->t0;
    }
    return apply_channels(c, APPLY_KT, RTE_PREC_FP64, gc, nullptr, b, 1);
}

int rte_rhs_source(rte_ctx* c, const void* g, int layout, void* b) {
    if (!c || !g || !b) return set_error(RTE_EINVAL, "NULL argument");
    if (layout != RTE_LAYOUT_MODES && layout != RTE_LAYOUT_CHANNELS) return set_error(RTE_EINVAL, "bad layout");
    if (g == b) return set_error(RTE_EINVAL, "g and b may not alias");
    if (layout == RTE_LAYOUT_CHANNELS) return rhs_source_channels(c, g, layout, (double*)b);
    int rc = rhs_source_channels(c, g, layout, c->bv);
    if (rc) return rc;
    to_modes(c, c->bv, b, true);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "rte_rhs_source", __FILE__, __LINE__);
}

int rte_solve_source(rte_ctx* c, const void* g, int layout, double tol, int max_iter, void* u, rte_solve_info* info) {
    if (!c || !g || !u) return set_error(RTE_EINVAL, "NULL argument");
    if (layout != RTE_LAYOUT_MODES && layout != RTE_LAYOUT_CHANNELS) return set_error(RTE_EINVAL, "bad layout");
    if (!(tol > 0.0) || !(tol < 1.0)) return set_error(RTE_EINVAL, "tol must be in (0, 1)");
    if (max_iter < 1) return set_error(RTE_EINVAL, "max_iter must be >= 1");
    int rc = rhs_source_channels(c, g, layout, c->bv);
    if (rc) return rc;
    SolveFinish fin;
    fin.arg = u;
    fin.fn = layout == RTE_LAYOUT_MODES
                 ? (void (*)(rte_ctx*, void*))[](rte_ctx* cc, void* uu) { to_modes(cc, cc->xv, uu, true); }
                 : (void (*)(rte_ctx*, void*))[](rte_ctx* cc, void* uu) {
                       (void)hipMemcpyAsync(uu, cc->xv, cc->nvec * sizeof(double), hipMemcpyDeviceToDevice, cc->stream);
                   };
    rc = solve_core(c, c->bv, tol, max_iter, c->xv, info, nullptr, 0, nullptr, &fin);
    if (rc < 0) return rc;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return set_hip_error(e, "rte_solve_source", __FILE__, __LINE__);
    if (rc == RTE_NOT_CONVERGED)
        set_error(RTE_NOT_CONVERGED, "not converged: relative residual %.3e", info ? info->relres_true : -1.0);
    return rc;
}

// Work buffers for nrhs right-hand sides and the stacked solution, residual and right-hand side.
static int ensure_multi(rte_ctx* c, int nrhs) {
    int rc = ensure_work(c, nrhs);
    if (rc) return rc;
    if (c->multi_nb < nrhs) {
        dfree(c->xm);
        dfree(c->rm);
        dfree(c->bm);
        c->multi_nb = 0;
        const size_t n = (size_t)nrhs * c->nvec;
        if ((rc = dalloc(&c->xm, n)) || (rc = dalloc(&c->rm, n)) || (rc = dalloc(&c->bm, n))) return rc;
        c->multi_nb = nrhs;
    }
    return RTE_OK;
}

// Several right-hand sides sharing the context's operator, solved as one GMRES on the stacked
// block-diagonal system diag(A, ..., A) [x_1; ...; x_B] = [b_1; ...; b_B] with each b_s scaled to
// unit norm (global GMRES): every iteration is one batched apply over all B vectors and one
// Gram-Schmidt step over the stacked vector.  With unit-norm blocks, a stacked relative residual
// of tol / sqrt(B') (B' the non-zero sources) bounds every block's relative residual by tol.
int rte_solve_multi(rte_ctx* c, int nrhs, const double* const* f, double tol, int max_iter, void* const* u,
                    rte_solve_info* infos) {
    if (!c || nrhs < 1 || !f || !u) return set_error(RTE_EINVAL, "bad argument");
    if (nrhs > RTE_MAX_RHS) return set_error(RTE_EINVAL, "nrhs = %d exceeds %d", nrhs, RTE_MAX_RHS);
    if (!(tol > 0.0) || !(tol < 1.0)) return set_error(RTE_EINVAL, "tol must be in (0, 1)");
    if (max_iter < 1) return set_error(RTE_EINVAL, "max_iter must be >= 1");
    for (int s = 0; s < nrhs; ++s)
        if (!f[s] || !u[s]) return set_error(RTE_EINVAL, "source or output %d is NULL", s);
    const double t0 = now_ms();
    const size_t nv = c->nvec;
    int rc = ensure_multi(c, nrhs);
    if (rc) return rc;
    hipStream_t st = c->stream;
    // right-hand sides and their norms
    std::vector<double> bn(nrhs);
    for (int s = 0; s < nrhs; ++s) {
        if ((rc = rhs_channels(c, f[s], c->bm + s * nv))) return rc;
        dot_enqueue(c, c->bm + s * nv, c->bm + s * nv);
        double b2;
        if ((rc = dot_wait(c, &b2))) return rc;
        if (!std::isfinite(b2)) return set_error(RTE_ENUMERIC, "non-finite right-hand side %d", s);
        bn[s] = std::sqrt(b2);
    }
    int nz = 0;
    for (int s = 0; s < nrhs; ++s) {
        vec_scale(c->bm + s * nv, c->bm + s * nv, bn[s] > 0.0 ? 1.0 / bn[s] : 0.0, nv, st);
        nz += bn[s] > 0.0;
    }
    rte_solve_info inf;
    memset(&inf, 0, sizeof(inf));
    int status = RTE_OK;
    if (nz > 0) {
        rc = solve_core(c, c->bm, tol / std::sqrt((double)nz), max_iter, c->xm, &inf, nullptr, 0, nullptr, nullptr,
                        nrhs);
        if (rc < 0) return rc;
        status = rc;
    } else {
        vec_fill(c->xm, 0.0, (size_t)nrhs * nv, st);
    }
    // undo the scaling, then every block's own true residual (FP64, one batched apply)
    for (int s = 0; s < nrhs; ++s) {
        vec_scale(c->xm + s * nv, c->xm + s * nv, bn[s], nv, st);
        vec_scale(c->bm + s * nv, c->bm + s * nv, bn[s], nv, st);
    }
    if ((rc = apply_channels(c, APPLY_RESID, RTE_PREC_FP64, c->xm, c->bm, c->rm, nrhs))) return rc;
    for (int s = 0; s < nrhs; ++s) to_modes(c, c->xm + s * nv, u[s], true);
    int worst = RTE_OK;
    for (int s = 0; s < nrhs; ++s) {
        double r2 = 0.0;
        dot_enqueue(c, c->rm + s * nv, c->rm + s * nv);
        if ((rc = dot_wait(c, &r2))) return rc;
        const double rel = bn[s] > 0.0 ? std::sqrt(r2) / bn[s] : 0.0;
        const int ss = !std::isfinite(rel) ? RTE_ENUMERIC : (rel <= tol ? RTE_OK : RTE_NOT_CONVERGED);
        if (ss == RTE_ENUMERIC) worst = RTE_ENUMERIC;
        else if (ss == RTE_NOT_CONVERGED && worst == RTE_OK) worst = RTE_NOT_CONVERGED;
        if (infos) {
            infos[s] = inf;
            infos[s].relres_true = rel;
            infos[s].status = bn[s] > 0.0 ? ss : RTE_OK;
        }
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return set_hip_error(e, "rte_solve_multi", __FILE__, __LINE__);
    const double t = now_ms() - t0;
    if (infos)
        for (int s = 0; s < nrhs; ++s) infos[s].t_solve_ms = t;
    if (worst == RTE_ENUMERIC) return set_error(RTE_ENUMERIC, "non-finite value in the stacked solve");
    if (worst == RTE_NOT_CONVERGED || status == RTE_NOT_CONVERGED) {
        set_error(RTE_NOT_CONVERGED, "some right-hand sides did not converge");
        return RTE_NOT_CONVERGED;
    }
    return RTE_OK;
}

int rte_solve_rhs(rte_ctx* c, const double* b, double tol, int max_iter, double* x, rte_solve_info* info,
                  double* x_iterates, int max_record, int* n_recorded) {
    if (!c || !b || !x) return set_error(RTE_EINVAL, "NULL argument");
    if (!(tol > 0.0) || !(tol < 1.0)) return set_error(RTE_EINVAL, "tol must be in (0, 1)");
    if (max_iter < 1) return set_error(RTE_EINVAL, "max_iter must be >= 1");
    if (x_iterates && max_record < 0) return set_error(RTE_EINVAL, "max_record must be >= 0");
    // x is cleared before b is read, so the two must be distinct storage; so must the iterates
    auto overlap = [](const void* p, size_t np, const void* q, size_t nq) {
        const char* a = (const char*)p;
        const char* b2 = (const char*)q;
        return a < b2 + nq && b2 < a + np;
    };
    const size_t vb = c->nvec * sizeof(double);
    if (overlap(x, vb, b, vb)) return set_error(RTE_EINVAL, "x and b overlap");
    if (x_iterates && max_record > 0) {
        const size_t ib = (size_t)max_record * vb;
        if (overlap(x_iterates, ib, x, vb) || overlap(x_iterates, ib, b, vb))
            return set_error(RTE_EINVAL, "x_iterates overlaps x or b");
    }
    return solve_core(c, b, tol, max_iter, x, info, x_iterates, max_record, n_recorded);
}

int rte_time_apply(rte_ctx* c, int op, int prec, int reps, double* ms_total, double* ms_pass) {
    if (!c || reps < 1) return set_error(RTE_EINVAL, "bad argument");
    vec_fill(c->t0, 1.0, c->nvec, c->stream);
    return time_apply_impl(c, op, prec, reps, 1, c->t0, c->t1, ms_total, ms_pass);
}

int rte_time_apply_multi(rte_ctx* c, int nrhs, int op, int prec, int reps, double* ms_total, double* ms_pass) {
    if (!c || reps < 1 || nrhs < 1) return set_error(RTE_EINVAL, "bad argument");
    if (nrhs > RTE_MAX_RHS) return set_error(RTE_EINVAL, "nrhs = %d exceeds %d", nrhs, RTE_MAX_RHS);
    int rc = ensure_multi(c, nrhs);
    if (rc) return rc;
    vec_fill(c->xm, 1.0, (size_t)nrhs * c->nvec, c->stream);
    return time_apply_impl(c, op, prec, reps, nrhs, c->xm, c->rm, ms_total, ms_pass);
}

}  // extern "C"

extern "C" int rte_solve_batched(int count, rte_ctx* const* ctxs, const double* const* f, const double* tol,
                                 int max_iter, void* const* u, rte_solve_info* infos) {
    return rte::solve_batched_impl(count, ctxs, f, tol, max_iter, u, infos);
}

extern "C" int rte_time_batched_apply(int count, rte_ctx* const* ctxs, int reps, double* ms_total, int max_launch,
                                      int* n_launch, double* ms_launch, int* launch_pass, int* launch_px,
                                      int* launch_py, int* launch_var) {
    return rte::time_batched_impl(count, ctxs, reps, ms_total, max_launch, n_launch, ms_launch, launch_pass,
                                  launch_px, launch_py, launch_var);
}

extern "C" int rte_set_batched_variant(int pass, int variant) { return rte::batched_set_variant(pass, variant); }
