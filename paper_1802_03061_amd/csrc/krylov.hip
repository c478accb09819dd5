// Vector kernels of the (flexible) GMRES iteration: multi-vector dot products against the Krylov
// basis, the classical Gram-Schmidt update with its norm, linear combinations, and the packing
// between complex mode vectors and real channel vectors.  Basis vectors are stored as TV (double,
// or float for the inner solve of the FP32 apply); every sum and product is taken in FP64.
//
// Reductions are deterministic: a fixed grid of blocks writes one partial per (vector, block) and
// a second kernel adds the partials in a fixed order, so repeated runs give bitwise equal sums.
#include <algorithm>

#include "arnoldi_dev.h"
#include "krylov.h"

namespace rte {

constexpr int KT = 256;           // threads per block
constexpr int VB = 16;            // basis vectors per dot block

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

// partial[v * nblk + blk] = sum over the block's slice of V[v][i] * w[i] for the NV vectors V[v]
// (v < NV, row stride ld), and norm_partial[blk] = sum of w[i]^2 over the slice when norm_partial
// is given.  The vector count is a template parameter so that every load of a step is issued before
// the first multiply.  With even n and ld (and 16-byte aligned V and w) each thread reads element
// pairs as 16-byte loads.  The slice a block covers and the order of its sums do not depend on the data.
template <int NV, bool PAIRS, typename TV>
__global__ __launch_bounds__(KT) void k_dot_partial(const TV* __restrict__ V, size_t ld,
                                                    const TV* __restrict__ w, size_t n,
                                                    double* __restrict__ partial,
                                                    double* __restrict__ norm_partial,
                                                    const int* __restrict__ active) {
    __shared__ double sh[KT / 64];
    if (active && *active == 0) return;
    const int nblk = gridDim.x;
    const bool do_norm = norm_partial != nullptr;
    double acc[NV > 0 ? NV : 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    double nrm = 0.0;
    const size_t stride = (size_t)nblk * KT;
    if constexpr (PAIRS) {
        using P2 = typename pair_of<TV>::type;
        const size_t np = n / 2, ldp = ld / 2;
        const P2* w2 = reinterpret_cast<const P2*>(w);
        const P2* V2 = reinterpret_cast<const P2*>(V);
        for (size_t i = (size_t)blockIdx.x * KT + threadIdx.x; i < np; i += stride) {
            const P2 wl = w2[i];
            P2 al[NV > 0 ? NV : 1];
#pragma unroll
            for (int v = 0; v < NV; ++v) al[v] = V2[(size_t)v * ldp + i];
            const double wx = (double)wl.x, wy = (double)wl.y;
            if (do_norm) nrm += wx * wx + wy * wy;
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += (double)al[v].x * wx + (double)al[v].y * wy;
        }
    } else {
        for (size_t i = (size_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride) {
            const double wi = (double)w[i];
            double a[NV > 0 ? NV : 1];
#pragma unroll
            for (int v = 0; v < NV; ++v) a[v] = (double)V[(size_t)v * ld + i];
            if (do_norm) nrm += wi * wi;
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += a[v] * wi;
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double s = block_sum(acc[v], sh);
        if (threadIdx.x == 0) partial[(size_t)v * nblk + blockIdx.x] = s;
    }
    if (do_norm) {
        const double s = block_sum(nrm, sh);
        if (threadIdx.x == 0) norm_partial[blockIdx.x] = s;
    }
}

template <bool PAIRS, typename TV>
static void launch_dots(int nv, unsigned nblk, hipStream_t st, const TV* V, size_t ld, const TV* w, size_t n,
                        double* partial, double* norm_partial, const int* active) {
    switch (nv) {
#define RTE_DOTS_CASE(K)                                                                                     \
    case K:                                                                                                  \
        hipLaunchKernelGGL((k_dot_partial<K, PAIRS, TV>), dim3(nblk), dim3(KT), 0, st, V, ld, w, n, partial,     \
                           norm_partial, active);                                                            \
        break;
        RTE_DOTS_CASE(0) RTE_DOTS_CASE(1) RTE_DOTS_CASE(2) RTE_DOTS_CASE(3) RTE_DOTS_CASE(4) RTE_DOTS_CASE(5)
        RTE_DOTS_CASE(6) RTE_DOTS_CASE(7) RTE_DOTS_CASE(8) RTE_DOTS_CASE(9) RTE_DOTS_CASE(10) RTE_DOTS_CASE(11)
        RTE_DOTS_CASE(12) RTE_DOTS_CASE(13) RTE_DOTS_CASE(14) RTE_DOTS_CASE(15) RTE_DOTS_CASE(16)
#undef RTE_DOTS_CASE
        default: break;
    }
}

// out[v] = sum_b partial[v * nblk + b] in a fixed order.
__global__ __launch_bounds__(KT) void k_reduce_partials(const double* __restrict__ partial, int nblk,
                                                        double* __restrict__ out, const int* __restrict__ active) {
    __shared__ double sh[KT / 64];
    if (active && *active == 0) return;
    const int v = blockIdx.x;
    const double* __restrict__ p = partial + (size_t)v * nblk;
    double s = 0.0;
    int b = threadIdx.x;
    for (; b + 3 * KT < nblk; b += 4 * KT) {   // four loads in flight per step
        const double a0 = p[b], a1 = p[b + KT], a2 = p[b + 2 * KT], a3 = p[b + 3 * KT];
        s += (a0 + a1) + (a2 + a3);
    }
    for (; b < nblk; b += KT) s += p[b];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[v] = s;
}

// w[i] = a (w[i] - sum_v V[v][i] h[v]) (FP64 arithmetic, stored as TV); partial_norm[blk] = sum over
// the slice of the stored new w[i]^2.
// a = 1, or with s0.st set (the fused single pass, h = s0.st) the normalising factor computed here
// (arnoldi_stage0_in_update), block 0 also doing stage 0 of the Arnoldi column.  PAIRS: as in
// k_dot_partial, element pairs as 16-byte loads.
template <bool PAIRS, typename TV>
__global__ __launch_bounds__(KT) void k_cgs_update(TV* __restrict__ w, const TV* __restrict__ V, size_t ld,
                                                   int nvec, const double* __restrict__ h, size_t n,
                                                   double* __restrict__ partial_norm, const int* __restrict__ active,
                                                   ArnoldiArgs s0) {
    __shared__ double sh[KT / 64];
    __shared__ double hs[RTE_KRYLOV_MAXVEC];
    __shared__ double a_sh;
    if (active && *active == 0) return;
    for (int v = threadIdx.x; v < nvec; v += KT) hs[v] = h[v];
    if (s0.st) {
        __syncthreads();
        arnoldi_stage0_in_update(s0, hs, &a_sh);
    } else if (threadIdx.x == 0) {
        a_sh = 1.0;
    }
    __syncthreads();
    const double a = a_sh;
    double nrm = 0.0;
    const size_t stride = (size_t)gridDim.x * KT;
    if constexpr (PAIRS) {
        using P2 = typename pair_of<TV>::type;
        const size_t np = n / 2, ldp = ld / 2;
        P2* w2 = reinterpret_cast<P2*>(w);
        const P2* V2 = reinterpret_cast<const P2*>(V);
        for (size_t i = (size_t)blockIdx.x * KT + threadIdx.x; i < np; i += stride) {
            const P2 wl = w2[i];
            double sx = (double)wl.x, sy = (double)wl.y;
#pragma unroll 8
            for (int v = 0; v < nvec; ++v) {
                const P2 b = V2[(size_t)v * ldp + i];
                sx -= (double)b.x * hs[v];
                sy -= (double)b.y * hs[v];
            }
            P2 q;
            q.x = (TV)(sx * a);
            q.y = (TV)(sy * a);
            w2[i] = q;
            nrm += (double)q.x * (double)q.x + (double)q.y * (double)q.y;
        }
    } else {
        for (size_t i = (size_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride) {
            double s = (double)w[i];
            // unrolled so that eight basis loads are in flight; subtraction order unchanged
#pragma unroll 8
            for (int v = 0; v < nvec; ++v) s -= (double)V[(size_t)v * ld + i] * hs[v];
            const TV q = (TV)(s * a);
            w[i] = q;
            nrm += (double)q * (double)q;
        }
    }
    const double t = block_sum(nrm, sh);
    if (threadIdx.x == 0) partial_norm[blockIdx.x] = t;
}

// x[i] += sum_v Z[v][i] y[v]; nothing when skip is given and skip[2] (the device's non-finite
// flag) is set.
template <typename TV>
__global__ __launch_bounds__(KT) void k_combine(double* __restrict__ x, const TV* __restrict__ Z, size_t ld,
                                                int nvec, const double* __restrict__ y, size_t n,
                                                const int* __restrict__ skip) {
    __shared__ double ys[RTE_KRYLOV_MAXVEC];
    if (skip && skip[2] != 0) return;
    for (int v = threadIdx.x; v < nvec; v += KT) ys[v] = y[v];
    __syncthreads();
    const size_t stride = (size_t)gridDim.x * KT;
    for (size_t i = (size_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride) {
        double s = x[i];
#pragma unroll 8
        for (int v = 0; v < nvec; ++v) s += (double)Z[(size_t)v * ld + i] * ys[v];
        x[i] = s;
    }
}

// Stage 1 of the fused single pass (block 0: the Arnoldi column's bookkeeping; every block adds
// up the update's partial sums of nu2 itself) and, when the stored vector needs it,
// w *= 1/sqrt(nu2) over the grid.
template <typename TV>
__global__ __launch_bounds__(KT) void k_rescale_arn1(ArnoldiArgs t, TV* __restrict__ w, size_t n,
                                                    const double* __restrict__ partial, int nblk) {
    const double inv = arnoldi_stage1_in_rescale(t, partial, nblk);
    if (inv < 0.0) return;
    const size_t stride = (size_t)gridDim.x * KT;
    for (size_t i = (size_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride) w[i] = (TV)((double)w[i] * inv);
}

// dst[i] = (*a) * src[i] with the factor read from device memory
template <typename TV>
__global__ __launch_bounds__(KT) void k_scale_dev(TV* __restrict__ dst, const TV* __restrict__ src,
                                                  const double* __restrict__ a, size_t n) {
    const double s = *a;
    const size_t stride = (size_t)gridDim.x * KT;
    for (size_t i = (size_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride) dst[i] = (TV)(s * (double)src[i]);
}

constexpr int ARN_THREADS = 256;

__global__ __launch_bounds__(ARN_THREADS) void k_arnoldi(ArnoldiArgs t) { arnoldi_block(t); }

// y = R^{-1} g for the leading k x k block of the rotated Hessenberg matrix (upper triangular,
// column-major with leading dimension ld) and the first k entries of the rotated residual vector:
// the least-squares solution of k Arnoldi columns (later rotations do not touch these entries).
// The block is staged in LDS; one wave then runs the back substitution, lane l holding y_l and
// y_{l+64} (k <= 128), each row's sum taken by a butterfly reduction that gives every lane the
// same bits.
__global__ __launch_bounds__(256) void k_back_solve(const double* __restrict__ H, int ld, const double* __restrict__ g,
                                                    int k, double* __restrict__ y, const int* __restrict__ flags) {
    extern __shared__ double Rs[];   // [k][k] column-major, then g[k]
    if (flags && flags[2] != 0) {   // a non-finite value in the cycle: y = 0 leaves x unchanged
        for (int i = threadIdx.x; i < k; i += blockDim.x) y[i] = 0.0;
        return;
    }
    double* gs = Rs + (size_t)k * k;
    for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
        const int i = idx % k, j = idx / k;
        Rs[idx] = i <= j ? H[(size_t)j * ld + i] : 0.0;
    }
    for (int i = threadIdx.x; i < k; i += blockDim.x) gs[i] = g[i];
    __syncthreads();
    if (threadIdx.x >= 64) return;
    const int l = threadIdx.x;
    double y0 = 0.0, y1 = 0.0;   // y[l], y[l + 64]
    for (int i = k - 1; i >= 0; --i) {
        double s = 0.0;
        if (l > i && l < k) s += Rs[(size_t)l * k + i] * y0;
        if (l + 64 > i && l + 64 < k) s += Rs[(size_t)(l + 64) * k + i] * y1;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        const double yi = (gs[i] - s) / Rs[(size_t)i * k + i];
        if (l == i) y0 = yi;
        if (l + 64 == i) y1 = yi;
    }
    if (l < k) y[l] = y0;
    if (l + 64 < k) y[l + 64] = y1;
}

// g = (g0, 0, ..., 0), n entries, and flags[0..nflags) = 0
__global__ void k_init_g(double* __restrict__ g, int n, double g0, int* __restrict__ flags, int nflags) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) g[i] = i == 0 ? g0 : 0.0;
    for (int i = threadIdx.x; i < nflags; i += blockDim.x) flags[i] = 0;
}

// dst[i] = a * src[i]
template <typename TD>
__global__ __launch_bounds__(KT) void k_scale(TD* __restrict__ dst, const double* __restrict__ src, double a,
                                              size_t n) {
    const size_t stride = (size_t)gridDim.x * KT;
    for (size_t i = (size_t)blockIdx.x * KT + threadIdx.x; i < n; i += stride) dst[i] = (TD)(a * src[i]);
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

// Real-basis modes (3D spherical harmonics): channel a is Re u_a (and, for a general complex
// vector, channel C + a is Im u_a); no mixing between modes.
__global__ __launch_bounds__(KT) void k_modes_to_channels_real(const cx<double>* __restrict__ x,
                                                               double* __restrict__ ch, size_t n, int one_part) {
    const size_t i = (size_t)blockIdx.x * KT + threadIdx.x;
    if (i >= n) return;
    const cx<double> v = x[i];
    ch[i] = v.re;
    if (!one_part) ch[n + i] = v.im;
}
__global__ __launch_bounds__(KT) void k_channels_to_modes_real(const double* __restrict__ ch,
                                                               cx<double>* __restrict__ y, size_t n, int one_part) {
    const size_t i = (size_t)blockIdx.x * KT + threadIdx.x;
    if (i >= n) return;
    y[i] = mk(ch[i], one_part ? 0.0 : ch[n + i]);
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

unsigned krylov_nblk(size_t n) { return grid_for(n, RTE_KRYLOV_NBLK); }

template <typename TV>
void krylov_dots(const TV* V, size_t ld, int nvec, const TV* w, size_t n, double* partial,
                 double* out, bool with_norm, hipStream_t st, const int* active) {
    const unsigned nblk = grid_for(n, RTE_KRYLOV_NBLK);
    const bool pairs = n % 2 == 0 && ld % 2 == 0 && ((uintptr_t)V % 16) == 0 && ((uintptr_t)w % 16) == 0;
    // groups of up to VB basis vectors; the first group also sums w^2 (into row nvec of partial)
    for (int v0 = 0; v0 < nvec || (v0 == 0 && with_norm); v0 += VB) {
        const int nv = std::min(VB, nvec - v0);
        double* np = (with_norm && v0 == 0) ? partial + (size_t)nvec * nblk : nullptr;
        if (pairs) launch_dots<true>(nv, nblk, st, V + (size_t)v0 * ld, ld, w, n, partial + (size_t)v0 * nblk, np, active);
        else launch_dots<false>(nv, nblk, st, V + (size_t)v0 * ld, ld, w, n, partial + (size_t)v0 * nblk, np, active);
    }
    const int nout = nvec + (with_norm ? 1 : 0);
    if (out && nout > 0)
        hipLaunchKernelGGL(k_reduce_partials, dim3(nout), dim3(KT), 0, st, partial, (int)nblk, out, active);
}

template <typename TV>
void krylov_update(TV* w, const TV* V, size_t ld, int nvec, const double* h, size_t n, double* partial,
                   double* norm_out, hipStream_t st, const int* active, const ArnoldiArgs* stage0) {
    const ArnoldiArgs none;
    const ArnoldiArgs& s0 = stage0 ? *stage0 : none;
    const unsigned nblk = grid_for(n, RTE_KRYLOV_NBLK);
    const bool pairs = n % 2 == 0 && ld % 2 == 0 && ((uintptr_t)V % 16) == 0 && ((uintptr_t)w % 16) == 0;
    if (pairs)
        hipLaunchKernelGGL((k_cgs_update<true, TV>), dim3(nblk), dim3(KT), 0, st, w, V, ld, nvec, h, n, partial, active,
                           s0);
    else
        hipLaunchKernelGGL((k_cgs_update<false, TV>), dim3(nblk), dim3(KT), 0, st, w, V, ld, nvec, h, n, partial, active,
                           s0);
    if (norm_out) hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(KT), 0, st, partial, (int)nblk, norm_out, active);
}

template <typename TV>
void vec_scale_dev(TV* dst, const TV* src, const double* a, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_dev<TV>, dim3(grid_for(n, 4096)), dim3(KT), 0, st, dst, src, a, n);
}

void back_solve_dev(const double* H, int ld, const double* g, int k, double* y, hipStream_t st, const int* flags) {
    const size_t lds = ((size_t)k * k + k) * sizeof(double);
    hipLaunchKernelGGL(k_back_solve, dim3(1), dim3(256), lds, st, H, ld, g, k, y, flags);
}

void init_g(double* g, int n, double g0, int* flags, int nflags, hipStream_t st) {
    hipLaunchKernelGGL(k_init_g, dim3(1), dim3(256), 0, st, g, n, g0, flags, nflags);
}

template <typename TV>
void rescale_arn1(const ArnoldiArgs& t, TV* w, size_t n, const double* partial, int nblk, hipStream_t st) {
    // usually nothing to rescale, so a small grid
    hipLaunchKernelGGL(k_rescale_arn1<TV>, dim3(grid_for(n, 512)), dim3(KT), 0, st, t, w, n, partial, nblk);
}

void reduce_partials(const double* partial, int nblk, double* out, int nout, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(nout), dim3(KT), 0, st, partial, nblk, out, nullptr);
}

void arnoldi_run(const ArnoldiArgs& t, hipStream_t s) {
    hipLaunchKernelGGL(k_arnoldi, dim3(1), dim3(ARN_THREADS), 0, s, t);
}

template <typename TV>
void krylov_combine(double* x, const TV* Z, size_t ld, int nvec, const double* y, size_t n, hipStream_t st,
                    const int* skip) {
    hipLaunchKernelGGL(k_combine<TV>, dim3(grid_for(n, 4096)), dim3(KT), 0, st, x, Z, ld, nvec, y, n, skip);
}

template <typename TD>
void vec_scale(TD* dst, const double* src, double a, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_scale<TD>, dim3(grid_for(n, 4096)), dim3(KT), 0, st, dst, src, a, n);
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

void modes_to_channels_real(const void* x, double* ch, size_t n, bool one_part, hipStream_t st) {
    hipLaunchKernelGGL(k_modes_to_channels_real, dim3((unsigned)((n + KT - 1) / KT)), dim3(KT), 0, st,
                       (const cx<double>*)x, ch, n, one_part ? 1 : 0);
}

void channels_to_modes_real(const double* ch, void* y, size_t n, bool one_part, hipStream_t st) {
    hipLaunchKernelGGL(k_channels_to_modes_real, dim3((unsigned)((n + KT - 1) / KT)), dim3(KT), 0, st, ch,
                       (cx<double>*)y, n, one_part ? 1 : 0);
}

void nonfinite_scan(const double* x, size_t n, int* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_nonfinite, dim3(grid_for(n, 1024)), dim3(KT), 0, st, x, n, flag);
}

#define RTE_KRYLOV_INST(TV)                                                                                     \
    template void krylov_dots<TV>(const TV*, size_t, int, const TV*, size_t, double*, double*, bool, hipStream_t, \
                                  const int*);                                                                  \
    template void krylov_update<TV>(TV*, const TV*, size_t, int, const double*, size_t, double*, double*,       \
                                    hipStream_t, const int*, const ArnoldiArgs*);                               \
    template void vec_scale_dev<TV>(TV*, const TV*, const double*, size_t, hipStream_t);                        \
    template void rescale_arn1<TV>(const ArnoldiArgs&, TV*, size_t, const double*, int, hipStream_t);          \
    template void krylov_combine<TV>(double*, const TV*, size_t, int, const double*, size_t, hipStream_t,      \
                                     const int*);                                                              \
    template void vec_scale<TV>(TV*, const double*, double, size_t, hipStream_t);
RTE_KRYLOV_INST(double)
RTE_KRYLOV_INST(float)
#undef RTE_KRYLOV_INST

}  // namespace rte
