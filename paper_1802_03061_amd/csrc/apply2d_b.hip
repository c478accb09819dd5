// Pass B of the 2D apply for one value of L (this file is compiled once per L = 0..8 with
// -DRTE_PASSB_L=<L>): FFT along y of every channel, per-frequency mode coupling with the kernel
// spectra, inverse FFT along y (Sec. 3.3.1: the kernel depends on x - y and on k' - k only, so
// the convolution over y and the sum over k' meet at each frequency).
//
// Fused form: the NCOL x C column spectra of a block live in LDS (C = 2L+1 channels, NCOL
// adjacent columns), transformed by one batched FFT; each thread then couples the modes at its
// frequencies and writes them back in place; one batched inverse FFT; store the first ny rows.
// Split form (FP64 when C x PY does not fit in LDS): forward y-FFTs to a full-length buffer,
// a pointwise coupling kernel, inverse y-FFTs.
//
// Coupling at frequency (kx, ky), for channels a_0 = u_0, (a_k, b_k) = sqrt2 (Re u_k, Im u_k):
//   W_{+-k} = (A_k +- i B_k)/sqrt2 (W_0 = A_0)   -- the complex modes
//   V_k = sum_{k'} Khat_{k'-k} W_{k'},  k = -L..L  -- Toeplitz in the mode index
//   out: A_0 = V_0, A_k = (V_k + V_{-k})/sqrt2, B_k = -i (V_k - V_{-k})/sqrt2
// with Khat read from the quarter table (see apply2d.hip for the symmetries).
#include "apply2d.h"
#include "apply2d_b.h"
#include "fft.h"

#ifndef RTE_PASSB_L
#error "compile with -DRTE_PASSB_L=<L>"
#endif

namespace rte {

template <typename T, int L>
__device__ __forceinline__ void couple_modes(cx<T>* v /* C values, in/out */, const cx<T>* __restrict__ Q,
                                             size_t qstride_m, size_t qoff, bool flip) {
    constexpr int C = 2 * L + 1;
    const T r2 = (T)0.70710678118654752440084436210485;
    cx<T> W[C];   // complex modes k' = -L..L at index k' + L
    W[L] = v[0];
#pragma unroll
    for (int k = 1; k <= L; ++k) {
        const cx<T> a = v[2 * k - 1], bb = v[2 * k];
        W[L + k] = scale(a + mul_i(bb), r2);
        W[L - k] = scale(a - mul_i(bb), r2);
    }
    cx<T> V[C];
#pragma unroll
    for (int k = 0; k < C; ++k) V[k] = mk((T)0, (T)0);
    // V_k += Khat_m W_{k+m} and V_k += Khat_{-m} W_{k-m}, one kernel spectrum at a time
#pragma unroll
    for (int m = 0; m <= 2 * L; ++m) {
        cx<T> K = Q[m * qstride_m + qoff];
        if (flip) { K.im = -K.im; if (m & 1) { K.re = -K.re; K.im = -K.im; } }
#pragma unroll
        for (int k = -L; k + m <= L; ++k) cmac(V[k + L], K, W[k + m + L]);
        if (m > 0) {
            cx<T> Kn = conj(K);                     // Khat_{-m} = (-1)^m conj Khat_m
            if (m & 1) { Kn.re = -Kn.re; Kn.im = -Kn.im; }
#pragma unroll
            for (int k = -L + m; k <= L; ++k) cmac(V[k + L], Kn, W[k - m + L]);
        }
    }
    v[0] = V[L];
#pragma unroll
    for (int k = 1; k <= L; ++k) {
        v[2 * k - 1] = scale(V[L + k] + V[L - k], r2);
        v[2 * k] = scale(mul_mi(V[L + k] - V[L - k]), r2);
    }
}

// Fused pass B: NCOL columns x C channels per block, spectra resident in LDS.
template <typename T, int PY, int L, int NCOL, int NTHR>
__global__ __launch_bounds__(NTHR) void k_pass_b_lds(cx<T>* __restrict__ Tb, const cx<T>* __restrict__ Q,
                                                     const cx<T>* __restrict__ tw, int ny, int nkx) {
    constexpr int C = 2 * L + 1;
    constexpr int NF = NCOL * C;
    constexpr int LD = PY;
    constexpr int KH = PY / 2 + 1;
    __shared__ cx<T> spec[NF * LD];
    const int tid = threadIdx.x;
    const int kx0 = blockIdx.x * NCOL;
    const int b = blockIdx.y;
    const size_t cstride = (size_t)nkx * ny;
    cx<T>* base = Tb + (size_t)b * C * cstride;
    // spec[(col * C + c) * LD + y]
    for (int idx = tid; idx < NF * PY; idx += NTHR) {
        const int y = idx % PY, fc = idx / PY;
        const int col = fc / C, c = fc % C;
        const int kx = kx0 + col;
        cx<T> v = mk((T)0, (T)0);
        if (y < ny && kx < nkx) v = base[c * cstride + (size_t)kx * ny + y];
        spec[fc * LD + y] = v;
    }
    __syncthreads();
    block_fft<T, PY, NF, LD, NTHR, false>(spec, tw, tid);
    for (int idx = tid; idx < NCOL * PY; idx += NTHR) {
        const int f = idx % PY, col = idx / PY;
        const int kx = kx0 + col;
        if (kx < nkx) {
            const bool flip = f > PY / 2;
            const int fy = flip ? PY - f : f;
            cx<T> v[C];
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] = spec[(col * C + c) * LD + f];
            couple_modes<T, L>(v, Q, (size_t)nkx * KH, (size_t)kx * KH + fy, flip);
#pragma unroll
            for (int c = 0; c < C; ++c) spec[(col * C + c) * LD + f] = v[c];
        }
    }
    __syncthreads();
    block_fft<T, PY, NF, LD, NTHR, true>(spec, tw, tid);
    for (int idx = tid; idx < NF * ny; idx += NTHR) {
        const int y = idx % ny, fc = idx / ny;
        const int col = fc / C, c = fc % C;
        const int kx = kx0 + col;
        if (kx < nkx) base[c * cstride + (size_t)kx * ny + y] = spec[fc * LD + y];
    }
}

// Split form, step 1/3: forward y-FFT of one (channel, column) into a full-length buffer.
template <typename T, int PY, int NTHR>
__global__ __launch_bounds__(NTHR) void k_pass_b_fwd(const cx<T>* __restrict__ Tb, cx<T>* __restrict__ T2,
                                                     const cx<T>* __restrict__ tw, int ny, int nkx, int C) {
    __shared__ cx<T> buf[PY];
    const int tid = threadIdx.x;
    const int kx = blockIdx.x, bc = blockIdx.y;
    const cx<T>* src = Tb + ((size_t)bc * nkx + kx) * ny;
    for (int y = tid; y < PY; y += NTHR) buf[y] = y < ny ? src[y] : mk((T)0, (T)0);
    __syncthreads();
    block_fft<T, PY, 1, PY, NTHR, false>(buf, tw, tid);
    cx<T>* dst = T2 + ((size_t)bc * nkx + kx) * PY;
    for (int y = tid; y < PY; y += NTHR) dst[y] = buf[y];
}

// Split form, step 2/3: pointwise coupling over all (kx, ky).
template <typename T, int PY, int L>
__global__ __launch_bounds__(256) void k_pass_b_couple(cx<T>* __restrict__ T2, const cx<T>* __restrict__ Q,
                                                       int nkx) {
    constexpr int C = 2 * L + 1;
    constexpr int KH = PY / 2 + 1;
    const int b = blockIdx.y;
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)nkx * PY) return;
    const int kx = (int)(idx / PY), f = (int)(idx % PY);
    const size_t cstride = (size_t)nkx * PY;
    cx<T>* p = T2 + (size_t)b * C * cstride + idx;
    const bool flip = f > PY / 2;
    const int fy = flip ? PY - f : f;
    cx<T> v[C];
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = p[c * cstride];
    couple_modes<T, L>(v, Q, (size_t)nkx * KH, (size_t)kx * KH + fy, flip);
#pragma unroll
    for (int c = 0; c < C; ++c) p[c * cstride] = v[c];
}

// Split form, step 3/3: inverse y-FFT and crop back into the work buffer.
template <typename T, int PY, int NTHR>
__global__ __launch_bounds__(NTHR) void k_pass_b_inv(cx<T>* __restrict__ Tb, const cx<T>* __restrict__ T2,
                                                     const cx<T>* __restrict__ tw, int ny, int nkx) {
    __shared__ cx<T> buf[PY];
    const int tid = threadIdx.x;
    const int kx = blockIdx.x, bc = blockIdx.y;
    const cx<T>* src = T2 + ((size_t)bc * nkx + kx) * PY;
    for (int y = tid; y < PY; y += NTHR) buf[y] = src[y];
    __syncthreads();
    block_fft<T, PY, 1, PY, NTHR, true>(buf, tw, tid);
    cx<T>* dst = Tb + ((size_t)bc * nkx + kx) * ny;
    for (int y = tid; y < ny; y += NTHR) dst[y] = buf[y];
}

constexpr int lds_budget() { return 150 * 1024; }

template <typename T, int PY, int L>
constexpr int ncol_for() {
    return (2 * L + 1) >= 4 ? 1 : ((2 * L + 1) == 3 ? 2 : 4);
}
template <typename T, int PY, int L>
constexpr bool fused_fits() {
    // FP64 with L > 4 holds too many complex values per thread for the fused coupling
    return (long)ncol_for<T, PY, L>() * (2 * L + 1) * PY * (long)sizeof(cx<T>) <= lds_budget() &&
           (sizeof(T) == 4 || L <= 4);
}
template <typename T, int NFPY>
constexpr int nthr_for() {
    // about 8 elements per thread, at most 512 threads (256 VGPRs per lane)
    return NFPY / 8 >= 512 ? 512 : (NFPY / 8 >= 256 ? 256 : (NFPY / 8 >= 128 ? 128 : 64));
}

template <typename T, int PY>
static int launch_py(const Apply2DArgs<T>& a, int nbatch) {
    constexpr int L = RTE_PASSB_L;
    constexpr int C = 2 * L + 1;
    const int nkx = a.PX / 2 + 1;
    if constexpr (fused_fits<T, PY, L>()) {
        constexpr int NCOL = ncol_for<T, PY, L>();
        constexpr int NT = nthr_for<T, NCOL * C * PY>();
        dim3 grid((nkx + NCOL - 1) / NCOL, nbatch);
        hipLaunchKernelGGL((k_pass_b_lds<T, PY, L, NCOL, NT>), grid, dim3(NT), 0, a.stream, a.work, a.Q,
                           a.twy, a.ny, nkx);
        return 0;
    } else {
        if (!a.work2) return -2;
        constexpr int NT = PY >= 256 ? 256 : (PY < 64 ? 64 : PY);
        dim3 g1(nkx, nbatch * C);
        hipLaunchKernelGGL((k_pass_b_fwd<T, PY, NT>), g1, dim3(NT), 0, a.stream, a.work, a.work2, a.twy, a.ny,
                           nkx, C);
        dim3 g2((unsigned)(((size_t)nkx * PY + 255) / 256), nbatch);
        hipLaunchKernelGGL((k_pass_b_couple<T, PY, L>), g2, dim3(256), 0, a.stream, a.work2, a.Q, nkx);
        hipLaunchKernelGGL((k_pass_b_inv<T, PY, NT>), g1, dim3(NT), 0, a.stream, a.work, a.work2, a.twy, a.ny,
                           nkx);
        return 0;
    }
}

template <typename T>
static int launch_pass_b_impl(const Apply2DArgs<T>& a, int nbatch) {
    switch (a.PY) {
        case 16: return launch_py<T, 16>(a, nbatch);
        case 32: return launch_py<T, 32>(a, nbatch);
        case 64: return launch_py<T, 64>(a, nbatch);
        case 128: return launch_py<T, 128>(a, nbatch);
        case 256: return launch_py<T, 256>(a, nbatch);
        case 512: return launch_py<T, 512>(a, nbatch);
        case 1024: return launch_py<T, 1024>(a, nbatch);
    }
    return -1;
}

#define RTE_CAT2(a, b) a##b
#define RTE_CAT(a, b) RTE_CAT2(a, b)
#define RTE_PASSB_FN RTE_CAT(pass_b_L, RTE_PASSB_L)

template <>
int RTE_PASSB_FN<float>(const Apply2DArgs<float>& a, int nbatch) { return launch_pass_b_impl<float>(a, nbatch); }
template <>
int RTE_PASSB_FN<double>(const Apply2DArgs<double>& a, int nbatch) { return launch_pass_b_impl<double>(a, nbatch); }

// Whether the split (3-kernel) form is used for this (precision, PY): the caller then provides
// work2 of nbatch * C * (PX/2+1) * PY elements.
template <>
bool RTE_CAT(pass_b_split_L, RTE_PASSB_L)<float>(int PY) {
    switch (PY) {
        case 16: return !fused_fits<float, 16, RTE_PASSB_L>();
        case 32: return !fused_fits<float, 32, RTE_PASSB_L>();
        case 64: return !fused_fits<float, 64, RTE_PASSB_L>();
        case 128: return !fused_fits<float, 128, RTE_PASSB_L>();
        case 256: return !fused_fits<float, 256, RTE_PASSB_L>();
        case 512: return !fused_fits<float, 512, RTE_PASSB_L>();
        default: return !fused_fits<float, 1024, RTE_PASSB_L>();
    }
}
template <>
bool RTE_CAT(pass_b_split_L, RTE_PASSB_L)<double>(int PY) {
    switch (PY) {
        case 16: return !fused_fits<double, 16, RTE_PASSB_L>();
        case 32: return !fused_fits<double, 32, RTE_PASSB_L>();
        case 64: return !fused_fits<double, 64, RTE_PASSB_L>();
        case 128: return !fused_fits<double, 128, RTE_PASSB_L>();
        case 256: return !fused_fits<double, 256, RTE_PASSB_L>();
        case 512: return !fused_fits<double, 512, RTE_PASSB_L>();
        default: return !fused_fits<double, 1024, RTE_PASSB_L>();
    }
}

}  // namespace rte
