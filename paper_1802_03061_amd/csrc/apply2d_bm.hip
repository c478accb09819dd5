// Pass B of the 2D apply for many modes (L > 8, up to 2L+1 = 65 channels): the split form
// (forward y-FFT of every (channel, column) sequence to a full-length buffer, the mode coupling per
// frequency, inverse y-FFT) with the coupling done by an FFT along the mode axis.
//
// The kernel of the anisotropic operator depends on the modes only through k' - k (Sec. 3.3.1,
// closing remark), so at every frequency the Toeplitz product V_k = sum_{k'} Khat_{k'-k} W_{k'}
// (k, k' = -L..L) is a convolution V = g * a of a[p] = W_{p-L} (p = 0..2L) with g[d] = Khat_{-d}
// (d = -2L..2L).  With a transform length PM >= 4L+1 along the mode axis the circular convolution
// is exact at the outputs p = k + L (the differences d = k - k' are distinct modulo PM):
//     V_k = IFFT_PM( FFT_PM(g) . FFT_PM(a) )[k + L],
// three length-PM transforms per frequency, O(M log M) against the direct O(M^2).  A direct
// coupling over the same staging (variant 1) is kept beside it; the autotuner times both.
//
// Channels are the real-field pairs of rte.h (ch0 = W_0, (ch_{2k-1} + i ch_{2k})/sqrt2 = W_k,
// (ch_{2k-1} - i ch_{2k})/sqrt2 = W_-k) in the y-spectrum; the work buffer is unpacked (columns
// kx = 0..PX/2 each hold one complex sequence).  Kernel spectra come from the quarter table with
// Khat_{-m} = (-1)^m conj Khat_m and Khat_m(kx, -ky) = (-1)^m conj Khat_m(kx, ky).
#include "apply2d_b.h"
#include "fft.h"
#include "passb_split.h"

#include <algorithm>

namespace rte {

// Khat_m at column kx and y-frequency ky from the quarter table (flip for ky > PY/2).
template <typename T>
__device__ __forceinline__ cx<T> khat(const cx<T>* __restrict__ Q, size_t qs, int KH, int kx, int fy, bool flip,
                                      int m) {
    cx<T> K = Q[(size_t)m * qs + (size_t)kx * KH + fy];
    if (flip) {
        K.im = -K.im;
        if (m & 1) { K.re = -K.re; K.im = -K.im; }
    }
    return K;
}

// Load the F frequencies' C channels of one column into a[f][p], p = k' + L (complex modes W_k'),
// zero past 2L.  Channel 2k-1 is parked at p = L+k and channel 2k at p = L-k, then combined in place.
template <typename T, int F, int LD, int NTHR>
__device__ __forceinline__ void load_modes(cx<T>* a, const cx<T>* __restrict__ T2c, size_t cstride, int ky0, int PY,
                                           int C, int L, int PMlen, int single, int tid) {
    for (int idx = tid; idx < F * PMlen; idx += NTHR) {
        const int f = idx % F, p = idx / F;
        a[f * LD + sw(p)] = mk((T)0, (T)0);
    }
    __syncthreads();
    constexpr int U = 4;   // U entries per thread at a time, loads first
    for (int base = tid; base < F * C; base += U * NTHR) {
        cx<T> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * NTHR;
            const int f = idx % F, c = idx / F;
            const bool ok = idx < F * C && ky0 + f < PY && !(single && c > 0);
            v[u] = ok ? T2c[(size_t)c * cstride + ky0 + f] : mk((T)0, (T)0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * NTHR;
            const int f = idx % F, c = idx / F;
            if (idx >= F * C || ky0 + f >= PY || (single && c > 0)) continue;
            const int p = c == 0 ? L : ((c & 1) ? L + (c + 1) / 2 : L - c / 2);
            a[f * LD + sw(p)] = v[u];
        }
    }
    __syncthreads();
    const T r2 = (T)0.70710678118654752440084436210485;
    for (int idx = tid; idx < F * L; idx += NTHR) {
        const int f = idx % F, k = idx / F + 1;
        const cx<T> A = a[f * LD + sw(L + k)], B = a[f * LD + sw(L - k)];
        a[f * LD + sw(L + k)] = scale(A + mul_i(B), r2);
        a[f * LD + sw(L - k)] = scale(A - mul_i(B), r2);
    }
    __syncthreads();
}

// Store V_k = v[f][k + L] (times s) back as channels: ch0 = V_0, ch_{2k-1} = (V_k + V_-k)/sqrt2,
// ch_{2k} = -i (V_k - V_-k)/sqrt2.
template <typename T, int F, int LD, int NTHR>
__device__ __forceinline__ void store_channels(const cx<T>* v, cx<T>* __restrict__ T2c, size_t cstride, int ky0, int PY,
                                               int L, T s, int tid) {
    const T r2 = (T)0.70710678118654752440084436210485 * s;
    for (int idx = tid; idx < F * (L + 1); idx += NTHR) {
        const int f = idx % F, k = idx / F;
        const int ky = ky0 + f;
        if (ky >= PY) continue;
        if (k == 0) {
            T2c[ky] = scale(v[f * LD + sw(L)], s);
        } else {
            const cx<T> Vp = v[f * LD + sw(L + k)], Vm = v[f * LD + sw(L - k)];
            T2c[(size_t)(2 * k - 1) * cstride + ky] = scale(Vp + Vm, r2);
            T2c[(size_t)(2 * k) * cstride + ky] = scale(mul_mi(Vp - Vm), r2);
        }
    }
}

// Mode-axis FFT coupling: block (frequency group, column kx, batch entry); buf holds the F mode
// sequences a_f followed by the F kernel sequences g_f, each of length PM.
template <typename T, int PM, int F, int NTHR>
__global__ __launch_bounds__(NTHR) void k_couple_modefft(cx<T>* __restrict__ T2, const cx<T>* __restrict__ Q,
                                                         const cx<T>* __restrict__ twm, int nkx, int nkq, int PY,
                                                         int L, int single) {
    constexpr int LD = padded(PM) + 1;
    __shared__ cx<T> buf[2 * F * LD];
    __shared__ cx<T> tws[PM];
    const int tid = threadIdx.x;
    const int ky0 = blockIdx.x * F, kx = blockIdx.y, b = blockIdx.z;
    const int C = 2 * L + 1, KH = PY / 2 + 1;
    const size_t cstride = (size_t)nkx * PY;
    const size_t qs = (size_t)nkq * KH;
    cx<T>* T2c = T2 + (size_t)b * C * cstride + (size_t)kx * PY;
    stage_twiddles<T, PM, NTHR>(tws, twm, tid);
    cx<T>* a = buf;
    cx<T>* g = buf + F * LD;
    // g_f[d mod PM] = Khat_{-d}: d = -m <= 0 takes Khat_m, d = m > 0 takes (-1)^m conj Khat_m
    for (int idx = tid; idx < F * PM; idx += NTHR) {
        const int f = idx % F, p = idx / F;
        g[f * LD + sw(p)] = mk((T)0, (T)0);
    }
    load_modes<T, F, LD, NTHR>(a, T2c, cstride, ky0, PY, C, L, PM, single, tid);   // ends with a barrier
    constexpr int UK = 4;   // UK spectrum entries per thread at a time, loads first
    for (int base = tid; base < F * (2 * L + 1); base += UK * NTHR) {
        cx<T> Kv[UK];
#pragma unroll
        for (int u = 0; u < UK; ++u) {
            const int idx = base + u * NTHR;
            const int f = idx % F, m = idx / F;
            const int ky = ky0 + f;
            const bool flip = ky > PY / 2;
            Kv[u] = (idx < F * (2 * L + 1) && ky < PY) ? khat(Q, qs, KH, kx, flip ? PY - ky : ky, flip, m)
                                                         : mk((T)0, (T)0);
        }
#pragma unroll
        for (int u = 0; u < UK; ++u) {
            const int idx = base + u * NTHR;
            const int f = idx % F, m = idx / F;
            if (idx >= F * (2 * L + 1) || ky0 + f >= PY) continue;
            g[f * LD + sw((PM - m) & (PM - 1))] = Kv[u];
            if (m > 0) {
                cx<T> Kn = conj(Kv[u]);
                if (m & 1) { Kn.re = -Kn.re; Kn.im = -Kn.im; }
                g[f * LD + sw(m)] = Kn;
            }
        }
    }
    __syncthreads();
    block_fft<T, PM, 2 * F, LD, NTHR, false>(buf, tws, tid);
    for (int idx = tid; idx < F * PM; idx += NTHR) {
        const int f = idx % F, p = idx / F;
        a[f * LD + sw(p)] = a[f * LD + sw(p)] * g[f * LD + sw(p)];
    }
    __syncthreads();
    block_fft<T, PM, F, LD, NTHR, true>(a, tws, tid);
    store_channels<T, F, LD, NTHR>(a, T2c, cstride, ky0, PY, L, (T)1 / (T)PM, tid);
}

// Direct coupling, register-blocked.  Each frequency's record in LDS holds the kernel spectra
// Khat_m for m = -2L..2L (KB-1 zeros on each side) and the modes W_k' (KB-1 zeros past k' = L);
// a thread computes KB consecutive outputs V_k, k = k0..k0+KB-1, of one frequency, sweeping k' in
// chunks of KB: per chunk it reads KB modes and 2KB-1 spectra and does KB^2 multiply-adds, so the
// LDS traffic per multiply-add falls by about KB/3 against one read pair per product.  The results
// overwrite the record's modes after a barrier.  F (frequencies per block) and the block size are
// set at launch from the LDS budget.
template <int KB>
__host__ __device__ constexpr int direct_rec(int L) {   // record length in complex entries (odd)
    return (6 * L + 3 * KB - 1) | 1;
}

template <typename T, int KB, int NTHR>
__global__ __launch_bounds__(NTHR) void k_couple_direct(cx<T>* __restrict__ T2, const cx<T>* __restrict__ Q, int nkx,
                                                        int nkq, int PY, int L, int F, int single) {
    extern __shared__ __align__(16) double smem_d[];
    cx<T>* sm = reinterpret_cast<cx<T>*>(smem_d);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int ky0 = blockIdx.x * F, kx = blockIdx.y, b = blockIdx.z;
    const int C = 2 * L + 1, KH = PY / 2 + 1;
    const int S = direct_rec<KB>(L);
    const int KOFF = 2 * L + KB - 1;              // Khat_m at record index KOFF + m
    const int AOFF = 4 * L + 2 * KB - 1;          // W_k' at AOFF + k' + L
    const size_t cstride = (size_t)nkx * PY;
    const size_t qs = (size_t)nkq * KH;
    cx<T>* T2c = T2 + (size_t)b * C * cstride + (size_t)kx * PY;
    for (int idx = tid; idx < F * S; idx += nthr) sm[idx] = mk((T)0, (T)0);
    __syncthreads();
    // U entries per thread at a time, their loads all issued before the LDS stores
    constexpr int U = 4;
    for (int base = tid; base < F * C; base += U * nthr) {
        cx<T> Kv[U], Wv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * nthr;
            const int f = idx % F, m = idx / F;   // m = 0..2L; idx also walks the channels c = m
            const int ky = ky0 + f;
            const bool ok = idx < F * C && ky < PY;
            const bool flip = ky > PY / 2;
            Kv[u] = ok ? khat(Q, qs, KH, kx, flip ? PY - ky : ky, flip, m) : mk((T)0, (T)0);
            Wv[u] = ok && !(single && m > 0) ? T2c[(size_t)m * cstride + ky] : mk((T)0, (T)0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * nthr;
            const int f = idx % F, m = idx / F;
            if (idx >= F * C || ky0 + f >= PY) continue;
            cx<T>* rec = sm + f * S;
            rec[KOFF + m] = Kv[u];
            if (m > 0) {                          // Khat_{-m} = (-1)^m conj Khat_m
                cx<T> Kn = conj(Kv[u]);
                if (m & 1) { Kn.re = -Kn.re; Kn.im = -Kn.im; }
                rec[KOFF - m] = Kn;
            }
            const int c = m;
            if (single && c > 0) continue;
            const int p = c == 0 ? L : ((c & 1) ? L + (c + 1) / 2 : L - c / 2);   // parked as in the mode FFT
            rec[AOFF + p] = Wv[u];
        }
    }
    __syncthreads();
    const T r2 = (T)0.70710678118654752440084436210485;
    for (int idx = tid; idx < F * L; idx += nthr) {
        const int f = idx % F, k = idx / F + 1;
        cx<T>* a = sm + f * S + AOFF;
        const cx<T> A = a[L + k], B = a[L - k];
        a[L + k] = scale(A + mul_i(B), r2);
        a[L - k] = scale(A - mul_i(B), r2);
    }
    __syncthreads();
    const int nkb = (C + KB - 1) / KB;
    cx<T> acc[KB];
    const bool have = tid < F * nkb;
    const int f = tid % F, kb = tid / F;
    const int k0 = kb * KB - L;
    if (have) {
        const cx<T>* rec = sm + f * S;
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] = mk((T)0, (T)0);
        for (int kp0 = -L; kp0 <= L; kp0 += KB) {
            cx<T> W[KB], Kb[2 * KB - 1];
#pragma unroll
            for (int i = 0; i < KB; ++i) W[i] = rec[AOFF + kp0 + i + L];
            const int t0 = KOFF + kp0 - k0 - (KB - 1);   // Khat_{kp - k}, kp - k = kp0 - k0 + i - j
#pragma unroll
            for (int t = 0; t < 2 * KB - 1; ++t) Kb[t] = rec[t0 + t];
#pragma unroll
            for (int i = 0; i < KB; ++i)
#pragma unroll
                for (int j = 0; j < KB; ++j) cmac(acc[j], Kb[i - j + KB - 1], W[i]);
        }
    }
    __syncthreads();                              // every read of the modes is done
    if (have) {
        cx<T>* v = sm + f * S + AOFF;
#pragma unroll
        for (int j = 0; j < KB; ++j)
            if (k0 + j <= L) v[k0 + j + L] = acc[j];
    }
    __syncthreads();
    for (int idx = tid; idx < F * (L + 1); idx += nthr) {
        const int ff = idx % F, k = idx / F;
        const int ky = ky0 + ff;
        if (ky >= PY) continue;
        const cx<T>* v = sm + ff * S + AOFF;
        if (k == 0) {
            T2c[ky] = v[L];
        } else {
            const cx<T> Vp = v[L + k], Vm = v[L - k];
            T2c[(size_t)(2 * k - 1) * cstride + ky] = scale(Vp + Vm, r2);
            T2c[(size_t)(2 * k) * cstride + ky] = scale(mul_mi(Vp - Vm), r2);
        }
    }
}

// Launch shape of the direct coupling: F frequencies per block within the LDS budget, one thread
// per (frequency, block of KB outputs), rounded up to whole waves.
template <typename T, int KB>
static void launch_direct(const Apply2DArgs<T>& a, int nbatch, int PY, int nkx, int nkq) {
    constexpr int NT = 256;
    constexpr size_t BUDGET = 64 * 1024;
    const int C = 2 * a.L + 1, nkb = (C + KB - 1) / KB;
    const size_t rec = (size_t)direct_rec<KB>(a.L) * sizeof(cx<T>);
    int F = std::min<int>(NT / nkb, (int)(BUDGET / rec));
    F = std::max(1, std::min(F, PY));
    const int nthr = std::min(NT, (F * nkb + 63) / 64 * 64);
    dim3 g((PY + F - 1) / F, nkx, nbatch);
    hipLaunchKernelGGL((k_couple_direct<T, KB, NT>), g, dim3(nthr), F * rec, a.stream, a.work2, a.Q, nkx, nkq, PY,
                       a.L, F, a.single_in);
}

template <typename T, int PM, int F>
static void launch_modefft(const Apply2DArgs<T>& a, int nbatch, int PY, int nkx, int nkq) {
    dim3 g2((PY + F - 1) / F, nkx, nbatch);
    hipLaunchKernelGGL((k_couple_modefft<T, PM, F, 256>), g2, dim3(256), 0, a.stream, a.work2, a.Q, a.twm, nkx, nkq,
                       PY, a.L, a.single_in);
}

template <typename T, int PY>
static int launch_large(const Apply2DArgs<T>& a, int nbatch) {
    const int nkq = a.PX / 2 + 1;
    const int nkx = nkq;                      // unpacked
    if (a.single_in && nbatch != 1) return -3;
    const size_t nseq = (size_t)nbatch * a.C * nkx;
    split_fft<T, PY, false>(a.work, a.work2, a.twy, a.ny, a.single_in ? (size_t)nkx : nseq, a.stream);
    const int PM = mode_fft_len(a.L);
    if (a.var[1] == 1) {
        launch_direct<T, 8>(a, nbatch, PY, nkx, nkq);
    } else if (PM == 64) {
        launch_modefft<T, 64, 16>(a, nbatch, PY, nkx, nkq);
    } else if (PM == 128) {
        launch_modefft<T, 128, 16>(a, nbatch, PY, nkx, nkq);
    } else {
        launch_modefft<T, 256, 8>(a, nbatch, PY, nkx, nkq);
    }
    split_fft<T, PY, true>(a.work, a.work2, a.twy, a.ny, nseq, a.stream);
    return 0;
}

template <typename T>
int pass_b_large(const Apply2DArgs<T>& a, int nbatch) {
    if (a.pack || !a.work2 || !a.twm || a.L <= PASSB_FUSED_MAX_L || a.L > RTE_MAX_L) return -1;
    switch (a.PY) {
        case 16: return launch_large<T, 16>(a, nbatch);
        case 32: return launch_large<T, 32>(a, nbatch);
        case 64: return launch_large<T, 64>(a, nbatch);
        case 128: return launch_large<T, 128>(a, nbatch);
        case 256: return launch_large<T, 256>(a, nbatch);
        case 512: return launch_large<T, 512>(a, nbatch);
        case 1024: return launch_large<T, 1024>(a, nbatch);
    }
    return -1;
}
template int pass_b_large<float>(const Apply2DArgs<float>&, int);
template int pass_b_large<double>(const Apply2DArgs<double>&, int);

}  // namespace rte
