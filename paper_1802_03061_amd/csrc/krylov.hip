// FP64 vector kernels of the (flexible) GMRES iteration: multi-vector dot products against the
// Krylov basis, the classical Gram-Schmidt update with its norm, linear combinations, and the
// packing between complex mode vectors and real channel vectors.
//
// Reductions are deterministic: a fixed grid of blocks writes one partial per (vector, block) and
// a second kernel adds the partials in a fixed order, so repeated runs give bitwise equal sums.
#include "krylov.h"

namespace rte {

constexpr int KT = 256;           // threads per block
constexpr int VB = 8;             // basis vectors per dot block

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum of `v` over the block (KT threads); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < KT / 64; ++i) r += sh[i];
    }
    __syncthreads();
    return r;
}

// partial[v * nblk + blk] = sum over the block's slice of V[v][i] * w[i], v < nvec; an extra row
// v = nvec holds sum w[i]^2 when with_norm.
__global__ __launch_bounds__(KT) void k_dot_partial(const double* __restrict__ V, size_t ld, int nvec,
                                                    const double* __restrict__ w, size_t n,
                                                    double* __restrict__ partial, int with_norm,
                                                    const int* __restrict__ active) {
    __shared__ double sh[KT / 64];
    if (active && *active == 0) return;
    const int nblk = gridDim.x;
    const int v0 = blockIdx.y * VB;
    const int nv = min(VB, nvec - v0);
    const bool do_norm = with_norm && blockIdx.y == 0;
    double acc[VB];
#pragma unroll
    for (int v = 0; v < VB; ++v) acc[v] = 0.0;
    double nrm = 0.0;
    const size_t stride = (size_t)nblk * KT;
    for (size_t i = (size_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride) {
        const double wi = w[i];
        if (do_norm) nrm += wi * wi;
#pragma unroll
        for (int v = 0; v < VB; ++v)
            if (v < nv) acc[v] += V[(size_t)(v0 + v) * ld + i] * wi;
    }
    for (int v = 0; v < nv; ++v) {
        const double s = block_sum(acc[v], sh);
        if (threadIdx.x == 0) partial[(size_t)(v0 + v) * nblk + blockIdx.x] = s;
    }
    if (do_norm) {
        const double s = block_sum(nrm, sh);
        if (threadIdx.x == 0) partial[(size_t)nvec * nblk + blockIdx.x] = s;
    }
}

// out[v] = sum_b partial[v * nblk + b] in a fixed order.
__global__ __launch_bounds__(KT) void k_reduce_partials(const double* __restrict__ partial, int nblk,
                                                        double* __restrict__ out, const int* __restrict__ active) {
    __shared__ double sh[KT / 64];
    if (active && *active == 0) return;
    const int v = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += KT) s += partial[(size_t)v * nblk + b];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[v] = s;
}

// w[i] -= sum_v V[v][i] h[v]; partial_norm[blk] = sum over the slice of w_new[i]^2.
__global__ __launch_bounds__(KT) void k_cgs_update(double* __restrict__ w, const double* __restrict__ V, size_t ld,
                                                   int nvec, const double* __restrict__ h, size_t n,
                                                   double* __restrict__ partial_norm, const int* __restrict__ active) {
    __shared__ double sh[KT / 64];
    __shared__ double hs[RTE_KRYLOV_MAXVEC];
    if (active && *active == 0) return;
    for (int v = threadIdx.x; v < nvec; v += KT) hs[v] = h[v];
    __syncthreads();
    double nrm = 0.0;
    const size_t stride = (size_t)gridDim.x * KT;
    for (size_t i = (size_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride) {
        double s = w[i];
        // unrolled so that eight basis loads are in flight; subtraction order unchanged
#pragma unroll 8
        for (int v = 0; v < nvec; ++v) s -= V[(size_t)v * ld + i] * hs[v];
        w[i] = s;
        nrm += s * s;
    }
    const double t = block_sum(nrm, sh);
    if (threadIdx.x == 0) partial_norm[blockIdx.x] = t;
}

// x[i] += sum_v Z[v][i] y[v]
__global__ __launch_bounds__(KT) void k_combine(double* __restrict__ x, const double* __restrict__ Z, size_t ld,
                                                int nvec, const double* __restrict__ y, size_t n) {
    __shared__ double ys[RTE_KRYLOV_MAXVEC];
    for (int v = threadIdx.x; v < nvec; v += KT) ys[v] = y[v];
    __syncthreads();
    const size_t stride = (size_t)gridDim.x * KT;
    for (size_t i = (size_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride) {
        double s = x[i];
#pragma unroll 8
        for (int v = 0; v < nvec; ++v) s += Z[(size_t)v * ld + i] * ys[v];
        x[i] = s;
    }
}

// dst[i] = (*a) * src[i] with the factor read from device memory
__global__ __launch_bounds__(KT) void k_scale_dev(double* __restrict__ dst, const double* __restrict__ src,
                                                  const double* __restrict__ a, size_t n) {
    const double s = *a;
    const size_t stride = (size_t)gridDim.x * KT;
    for (size_t i = (size_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride) dst[i] = s * src[i];
}

// One Arnoldi column on the device.  stage 0: after the first Gram-Schmidt pass, decide whether
// a second pass runs (reorth 2: always; 1: when the norm fell below 1/sqrt2 of its value; 0: never)
// and store h into H[:, j].
// stage 1: add the second pass, form H[j+1, j], apply the previous Givens rotations and a new
// one, update the residual vector g, and write the estimate |g[j+1]| and 1/H[j+1, j].
// st layout: [0..m] h pass 1 | [m+1] |w|^2 | [m+2] |w1|^2 | [m+4..2m+4] h pass 2
__global__ void k_arnoldi(int stage, int j, int m, double* __restrict__ st, double* __restrict__ H,
                          double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g,
                          double* __restrict__ est, double* __restrict__ inv, int* __restrict__ flags, int reorth,
                          double* __restrict__ est_out, int* __restrict__ flags_out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double* Hj = H + (size_t)j * (m + 1);
    const double* h1 = st;
    const double* h2 = st + m + 4;
    if (stage == 0) {
        for (int i = 0; i <= j; ++i) Hj[i] = h1[i];
        flags[0] = (reorth == 2 || (reorth == 1 && st[j + 2] < 0.5 * st[j + 1])) ? 1 : 0;
        st[m + 3] = st[j + 1];   // |w|^2 before orthogonalisation
        return;
    }
    if (flags[0])
        for (int i = 0; i <= j; ++i) Hj[i] += h2[i];
    const double w0 = st[m + 3];
    const double w1 = st[j + 2] > 0.0 ? st[j + 2] : 0.0;
    const double hn = sqrt(w1);
    Hj[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double t = cs[i] * Hj[i] + sn[i] * Hj[i + 1];
        Hj[i + 1] = -sn[i] * Hj[i] + cs[i] * Hj[i + 1];
        Hj[i] = t;
    }
    const double den = hypot(Hj[j], Hj[j + 1]);
    if (den == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
    else { cs[j] = Hj[j] / den; sn[j] = Hj[j + 1] / den; }
    Hj[j] = den;
    Hj[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    est[j] = fabs(g[j + 1]);
    const bool breakdown = !(hn > 1e-14 * sqrt(w0 > 0.0 ? w0 : 0.0));
    inv[j + 1] = breakdown ? 0.0 : 1.0 / hn;
    flags[1] = breakdown ? 1 : 0;
    if (!isfinite(den) || !isfinite(est[j])) flags[2] = 1;
    if (est_out) *est_out = est[j];
    if (flags_out) {
        flags_out[0] = flags[1];
        flags_out[1] = flags[2];
    }
}

// dst[i] = a * src[i]
__global__ __launch_bounds__(KT) void k_scale(double* __restrict__ dst, const double* __restrict__ src, double a,
                                              size_t n) {
    const size_t stride = (size_t)gridDim.x * KT;
    for (size_t i = (size_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride) dst[i] = a * src[i];
}

__global__ __launch_bounds__(KT) void k_fill(double* __restrict__ dst, double a, size_t n) {
    const size_t stride = (size_t)gridDim.x * KT;
    for (size_t i = (size_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride) dst[i] = a;
}

// Real channels of the conjugate-symmetric parts of a general complex mode vector x[M][N]:
//   p_k = (x_k + conj x_{-k})/2,  q_k = (x_k - conj x_{-k})/(2i),  x = p + i q,
// each stored as channels ch0 = Re(.)_0, ch_{2k-1} = sqrt2 Re(.)_k, ch_{2k} = sqrt2 Im(.)_k.
// Output [2][C][N] (p first); with one_part only p (the input is taken as conjugate-symmetric).
__global__ __launch_bounds__(KT) void k_modes_to_channels(const cx<double>* __restrict__ x, double* __restrict__ ch,
                                                          int L, size_t N, int one_part) {
    const int C = 2 * L + 1;
    const size_t i = (size_t)blockIdx.x * KT + threadIdx.x;
    if (i >= N) return;
    const double r2 = 1.4142135623730951;
    const cx<double> x0 = x[(size_t)L * N + i];
    ch[i] = x0.re;
    if (!one_part) ch[(size_t)C * N + i] = x0.im;
    for (int k = 1; k <= L; ++k) {
        const cx<double> xp = x[(size_t)(L + k) * N + i];
        if (one_part) {
            ch[(size_t)(2 * k - 1) * N + i] = r2 * xp.re;
            ch[(size_t)(2 * k) * N + i] = r2 * xp.im;
        } else {
            const cx<double> xm = x[(size_t)(L - k) * N + i];
            ch[(size_t)(2 * k - 1) * N + i] = r2 * 0.5 * (xp.re + xm.re);
            ch[(size_t)(2 * k) * N + i] = r2 * 0.5 * (xp.im - xm.im);
            ch[(size_t)(C + 2 * k - 1) * N + i] = r2 * 0.5 * (xp.im + xm.im);
            ch[(size_t)(C + 2 * k) * N + i] = r2 * 0.5 * (xm.re - xp.re);
        }
    }
}

// Inverse: y_k = P_k + i Q_k with P_k = (ch_{2k-1} + i ch_{2k})/sqrt2, P_{-k} = conj P_k, P_0 = ch0,
// and Q likewise from the second part (absent when one_part).
__global__ __launch_bounds__(KT) void k_channels_to_modes(const double* __restrict__ ch, cx<double>* __restrict__ y,
                                                          int L, size_t N, int one_part) {
    const int C = 2 * L + 1;
    const size_t i = (size_t)blockIdx.x * KT + threadIdx.x;
    if (i >= N) return;
    const double r2 = 0.70710678118654752440;
    const double q0 = one_part ? 0.0 : ch[(size_t)C * N + i];
    y[(size_t)L * N + i] = mk(ch[i], q0);
    for (int k = 1; k <= L; ++k) {
        const cx<double> P = mk(r2 * ch[(size_t)(2 * k - 1) * N + i], r2 * ch[(size_t)(2 * k) * N + i]);
        cx<double> Q = mk(0.0, 0.0);
        if (!one_part) Q = mk(r2 * ch[(size_t)(C + 2 * k - 1) * N + i], r2 * ch[(size_t)(C + 2 * k) * N + i]);
        y[(size_t)(L + k) * N + i] = P + mul_i(Q);
        y[(size_t)(L - k) * N + i] = conj(P) + mul_i(conj(Q));
    }
}

// NaN/Inf scan helper: flag[0] = 1 if any entry is not finite.
__global__ __launch_bounds__(KT) void k_nonfinite(const double* __restrict__ x, size_t n, int* __restrict__ flag) {
    const size_t stride = (size_t)gridDim.x * KT;
    for (size_t i = (size_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride)
        if (!isfinite(x[i])) flag[0] = 1;
}

// ------------------------------------------------------------------ host wrappers --------------
static inline unsigned grid_for(size_t n, unsigned cap) {
    size_t g = (n + KT - 1) / KT;
    return (unsigned)(g < cap ? (g ? g : 1) : cap);
}

void krylov_dots(const double* V, size_t ld, int nvec, const double* w, size_t n, double* partial,
                 double* out, bool with_norm, hipStream_t st, const int* active) {
    const unsigned nblk = grid_for(n, RTE_KRYLOV_NBLK);
    dim3 grid(nblk, (nvec + VB - 1) / VB);
    if (nvec == 0) grid.y = 1;
    hipLaunchKernelGGL(k_dot_partial, grid, dim3(KT), 0, st, V, ld, nvec, w, n, partial, with_norm ? 1 : 0, active);
    const int nout = nvec + (with_norm ? 1 : 0);
    if (nout > 0) hipLaunchKernelGGL(k_reduce_partials, dim3(nout), dim3(KT), 0, st, partial, (int)nblk, out, active);
}

void krylov_update(double* w, const double* V, size_t ld, int nvec, const double* h, size_t n, double* partial,
                   double* norm_out, hipStream_t st, const int* active) {
    const unsigned nblk = grid_for(n, RTE_KRYLOV_NBLK);
    hipLaunchKernelGGL(k_cgs_update, dim3(nblk), dim3(KT), 0, st, w, V, ld, nvec, h, n, partial, active);
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(KT), 0, st, partial, (int)nblk, norm_out, active);
}

void vec_scale_dev(double* dst, const double* src, const double* a, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_dev, dim3(grid_for(n, 4096)), dim3(KT), 0, st, dst, src, a, n);
}

void arnoldi_step(int stage, int j, int m, double* st, double* H, double* cs, double* sn, double* g, double* est,
                  double* inv, int* flags, int reorth, hipStream_t s, double* est_out, int* flags_out) {
    hipLaunchKernelGGL(k_arnoldi, dim3(1), dim3(64), 0, s, stage, j, m, st, H, cs, sn, g, est, inv, flags, reorth,
                       est_out, flags_out);
}

void krylov_combine(double* x, const double* Z, size_t ld, int nvec, const double* y, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_combine, dim3(grid_for(n, 4096)), dim3(KT), 0, st, x, Z, ld, nvec, y, n);
}

void vec_scale(double* dst, const double* src, double a, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_scale, dim3(grid_for(n, 4096)), dim3(KT), 0, st, dst, src, a, n);
}

void vec_fill(double* dst, double a, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 4096)), dim3(KT), 0, st, dst, a, n);
}

void modes_to_channels(const void* x, double* ch, int L, size_t N, bool one_part, hipStream_t st) {
    hipLaunchKernelGGL(k_modes_to_channels, dim3((unsigned)((N + KT - 1) / KT)), dim3(KT), 0, st,
                       (const cx<double>*)x, ch, L, N, one_part ? 1 : 0);
}

void channels_to_modes(const double* ch, void* y, int L, size_t N, bool one_part, hipStream_t st) {
    hipLaunchKernelGGL(k_channels_to_modes, dim3((unsigned)((N + KT - 1) / KT)), dim3(KT), 0, st, ch,
                       (cx<double>*)y, L, N, one_part ? 1 : 0);
}

void nonfinite_scan(const double* x, size_t n, int* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_nonfinite, dim3(grid_for(n, 1024)), dim3(KT), 0, st, x, n, flag);
}

}  // namespace rte
