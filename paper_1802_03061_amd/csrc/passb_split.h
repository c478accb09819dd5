// The forward and inverse y-FFT kernels of the split pass B, shared by the per-L pass B and the
// large-L pass B.  The work buffer holds the (batch, channel, column) sequences of ny entries one
// after another, the full-length buffer the same sequences with PY entries; a block transforms
// NSEQ consecutive sequences (NSEQ PY about 2-4K entries, so that every thread has butterflies in
// each stage and the twiddle staging is shared), reading or writing them as one contiguous run.
#pragma once
#include "fft.h"

namespace rte {

// Sequences per block of the split y-FFTs.
template <typename T, int PY>
constexpr int split_nseq() {
    return (sizeof(T) == 4 ? 4096 : 2048) / PY > 1 ? (sizeof(T) == 4 ? 4096 : 2048) / PY : 1;
}

// Split form, step 1/3: forward y-FFT of sequences seq0 .. seq0 + NSEQ - 1 (zero-padded from ny
// to PY) into the full-length buffer.
template <typename T, int PY, int NSEQ, int NTHR>
__global__ __launch_bounds__(NTHR) void k_pass_b_fwd(const cx<T>* __restrict__ Tb, cx<T>* __restrict__ T2,
                                                     const cx<T>* __restrict__ tw, int ny, int nseq) {
    constexpr int LD = padded(PY);
    __shared__ cx<T> buf[NSEQ * LD];
    __shared__ cx<T> tws[PY];
    const int tid = threadIdx.x;
    const size_t s0 = (size_t)blockIdx.x * NSEQ;
    const int live = (int)min((size_t)NSEQ, (size_t)nseq - s0);
    stage_twiddles<T, PY, NTHR>(tws, tw, tid);
    const cx<T>* src = Tb + s0 * ny;
    // entries y >= ny (and whole sequences past the last) are the zero padding
    fft_forward_padded<T, PY, NSEQ, LD, NTHR>(buf, tws, tid, [&](int f, int y) {
        return (f < live && y < ny) ? src[(size_t)f * ny + y] : mk((T)0, (T)0);
    });
    cx<T>* dst = T2 + s0 * PY;
    for (int idx = tid; idx < live * PY; idx += NTHR) dst[idx] = buf[(idx / PY) * LD + sw(idx % PY)];
}

// Split form, step 3/3: inverse y-FFT of NSEQ sequences and crop back to ny entries.
template <typename T, int PY, int NSEQ, int NTHR>
__global__ __launch_bounds__(NTHR) void k_pass_b_inv(cx<T>* __restrict__ Tb, const cx<T>* __restrict__ T2,
                                                     const cx<T>* __restrict__ tw, int ny, int nseq) {
    constexpr int LD = padded(PY);
    __shared__ cx<T> buf[NSEQ * LD];
    __shared__ cx<T> tws[PY];
    const int tid = threadIdx.x;
    const size_t s0 = (size_t)blockIdx.x * NSEQ;
    const int live = (int)min((size_t)NSEQ, (size_t)nseq - s0);
    stage_twiddles<T, PY, NTHR>(tws, tw, tid);
    const cx<T>* src = T2 + s0 * PY;
    // every load of the block's sequences is issued before the first LDS store
    constexpr int PER = (NSEQ * PY + NTHR - 1) / NTHR;
    cx<T> v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = tid + u * NTHR;
        v[u] = ((NSEQ * PY) % NTHR == 0 || idx < NSEQ * PY) && idx < live * PY ? src[idx] : mk((T)0, (T)0);
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = tid + u * NTHR;
        if ((NSEQ * PY) % NTHR == 0 || idx < NSEQ * PY) buf[(idx / PY) * LD + sw(idx % PY)] = v[u];
    }
    __syncthreads();
    cx<T>* dst = Tb + s0 * ny;
    fft_inverse_cropped<T, PY, NSEQ, LD, NTHR>(buf, tws, tid, [&](int f, int y, cx<T> v) {
        if (f < live && y < ny) dst[(size_t)f * ny + y] = v;
    });
}

// Launch the forward (INV = false) or inverse y-FFTs over nseq sequences.
template <typename T, int PY, bool INV>
inline void split_fft(cx<T>* Tb, cx<T>* T2, const cx<T>* tw, int ny, size_t nseq, hipStream_t st) {
    constexpr int NSEQ = split_nseq<T, PY>();
    constexpr int NT = 256;
    const unsigned nblk = (unsigned)((nseq + NSEQ - 1) / NSEQ);
    if (nblk == 0) return;
    if constexpr (INV)
        hipLaunchKernelGGL((k_pass_b_inv<T, PY, NSEQ, NT>), dim3(nblk), dim3(NT), 0, st, Tb, T2, tw, ny, (int)nseq);
    else
        hipLaunchKernelGGL((k_pass_b_fwd<T, PY, NSEQ, NT>), dim3(nblk), dim3(NT), 0, st, Tb, T2, tw, ny, (int)nseq);
}

}  // namespace rte
