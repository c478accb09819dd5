// Workgroup-cooperative FFTs staged through LDS (gfx950, 64-wide waves).
//
// A transform of length P (a power of two) is computed by the Stockham autosort scheme: stage s
// combines R sub-transforms of length Ns into transforms of length Ns*R, reading R values spaced
// P/R apart, applying the twiddles exp(-+2 pi i r (j mod Ns)/(Ns R)), an R-point DFT in
// registers, and writing the R results spaced Ns apart.  The result comes out in natural order.
// Stages run in place in LDS: every thread first reads and transforms all its butterflies into
// registers, a barrier, then writes.  Radices are 8 (with one leading 2 or 4 stage when
// log2 P is not a multiple of 3).  Twiddles come from a table computed in FP64 on the host,
// rounded to the working precision and staged into LDS, laid out per stage: the R-1 factors of
// butterfly k of the stage with sub-length Ns are contiguous at stage_tw_offset(P, Ns) +
// k (R-1), so the lanes of a wave read consecutive 56-byte runs (no bank conflicts).
//
// LDS layout: element i of a transform lives at sw(i) = i + i/16, i.e. one pad slot per 16
// elements.  The strided writes of the early stages (stride R or Ns elements) then fall on
// different banks instead of repeating the same few.
#pragma once
#include "common.h"

namespace rte {

__device__ __forceinline__ int sw(int i) { return i + (i >> 4); }
constexpr int padded(int P) { return P + P / 16; }

// Radix schedules: S = 0 (default) and S = 1 (radix 32: two stages at length 1024, fewer LDS
// round trips per transform at the price of more registers per butterfly).
constexpr int fft_radix(int P, int Ns, int S = 0) {
    // r = log2 of what remains to be combined.
    // S = 0: radix 8 stages, led by one radix-16 stage when r = 1 (mod 3) and r >= 4 (2 when
    // r = 1), or one radix-4 stage when r = 2 (mod 3).
    // S = 1: radix 32 stages, led by one stage of radix 2^(r mod 5) when r is not a multiple of 5.
    return S == 1 ? ((ilog2(P) - ilog2(Ns)) % 5 == 0 ? 32 : (1 << ((ilog2(P) - ilog2(Ns)) % 5)))
                  : ((ilog2(P) - ilog2(Ns)) % 3 == 1 ? ((ilog2(P) - ilog2(Ns)) >= 4 ? 16 : 2)
                                                     : ((ilog2(P) - ilog2(Ns)) % 3 == 2 ? 4 : 8));
}

// Offset of the twiddles of the stage with sub-transform length NS (> 1) in the per-stage table;
// the table holds sum over those stages of NS (R - 1) = P - (first radix) entries.
constexpr int stage_tw_offset(int P, int NS, int S = 0) {
    int off = 0, ns = 1;
    while (ns < NS) {
        const int R = fft_radix(P, ns, S);
        if (ns > 1) off += ns * (R - 1);
        ns *= R;
    }
    return off;
}

template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot_mi(cx<T> a) {  // multiply by -i (forward) or +i (inverse)
    return INV ? mul_i(a) : mul_mi(a);
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_small(cx<T>* v) {
    if constexpr (R == 2) {
        cx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    } else if constexpr (R == 4) {
        cx<T> t0 = v[0] + v[2], t1 = v[0] - v[2];
        cx<T> t2 = v[1] + v[3], t3 = rot_mi<T, INV>(v[1] - v[3]);
        v[0] = t0 + t2;
        v[2] = t0 - t2;
        v[1] = t1 + t3;
        v[3] = t1 - t3;
    } else if constexpr (R == 16) {
        // 16 = 4 x 4: v[4 n1 + n2] -> A[n2][k1] = DFT4 over n1, times W16^(n2 k1), then
        // X[k1 + 4 k2] = DFT4 over n2.  W16^q = exp(-+2 pi i q / 16) for q = n2 k1 <= 9.
        const T c1 = (T)0.92387953251128675612818318939679, s1 = (T)0.38268343236508977172845998403040;
        const T c2 = (T)0.70710678118654752440084436210485;
        const T wr[10] = {(T)1, c1, c2, s1, (T)0, -s1, -c2, -c1, (T)-1, -c1};
        const T wi[10] = {(T)0, s1, c2, c1, (T)1, c1, c2, s1, (T)0, -s1};   // sin(2 pi q / 16)
        cx<T> a[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[4 * n1 + n2];
            dft_small<T, 4, INV>(a[n2]);
#pragma unroll
            for (int k1 = 1; k1 < 4; ++k1) {
                if (n2 == 0) continue;
                const int q = n2 * k1;
                const cx<T> w = mk(wr[q], INV ? wi[q] : -wi[q]);
                a[n2][k1] = a[n2][k1] * w;
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            cx<T> b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
            dft_small<T, 4, INV>(b);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
        }
    } else if constexpr (R == 32) {
        // 32 = 8 x 4: v[8 n1 + n2] -> A[n2][k1] = DFT4 over n1, times W32^(n2 k1), then
        // X[k1 + 4 k2] = DFT8 over n2.  W32^q = cos(pi q/16) -+ i sin(pi q/16), q = n2 k1 <= 21.
        const T c1 = (T)0.98078528040323044912618223613424, s1 = (T)0.19509032201612826784828486847702;
        const T c2 = (T)0.92387953251128675612818318939679, s2 = (T)0.38268343236508977172845998403040;
        const T c3 = (T)0.83146961230254523707878837761791, s3 = (T)0.55557023301960222474283081394853;
        const T rh = (T)0.70710678118654752440084436210485;
        const T wr[22] = {(T)1, c1, c2, c3, rh, s3, s2, s1, (T)0, -s1, -s2, -s3, -rh, -c3, -c2, -c1,
                          (T)-1, -c1, -c2, -c3, -rh, -s3};
        const T wi[22] = {(T)0, s1, s2, s3, rh, c3, c2, c1, (T)1, c1, c2, c3, rh, s3, s2, s1,
                          (T)0, -s1, -s2, -s3, -rh, -c3};   // sin(pi q / 16)
        cx<T> a[8][4];
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[8 * n1 + n2];
            dft_small<T, 4, INV>(a[n2]);
#pragma unroll
            for (int k1 = 1; k1 < 4; ++k1) {
                if (n2 == 0) continue;
                const int q = n2 * k1;
                const cx<T> w = mk(wr[q], INV ? wi[q] : -wi[q]);
                a[n2][k1] = a[n2][k1] * w;
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            cx<T> b[8] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1], a[4][k1], a[5][k1], a[6][k1], a[7][k1]};
            dft_small<T, 8, INV>(b);
#pragma unroll
            for (int k2 = 0; k2 < 8; ++k2) v[k1 + 4 * k2] = b[k2];
        }
    } else {  // R == 8: two 4-point DFTs on the even and odd samples, then W8^q
        cx<T> e[4] = {v[0], v[2], v[4], v[6]};
        cx<T> o[4] = {v[1], v[3], v[5], v[7]};
        dft_small<T, 4, INV>(e);
        dft_small<T, 4, INV>(o);
        const T s = (T)0.70710678118654752440084436210485;
        // W8^1 = (1 -+ i)/sqrt2, W8^2 = -+i, W8^3 = (-1 -+ i)/sqrt2  (upper sign forward)
        cx<T> o1 = INV ? mk(s * (o[1].re - o[1].im), s * (o[1].re + o[1].im))
                       : mk(s * (o[1].re + o[1].im), s * (o[1].im - o[1].re));
        cx<T> o2 = rot_mi<T, INV>(o[2]);
        cx<T> o3 = INV ? mk(-s * (o[3].re + o[3].im), s * (o[3].re - o[3].im))
                       : mk(s * (o[3].im - o[3].re), -s * (o[3].re + o[3].im));
        v[0] = e[0] + o[0];
        v[4] = e[0] - o[0];
        v[1] = e[1] + o1;
        v[5] = e[1] - o1;
        v[2] = e[2] + o2;
        v[6] = e[2] - o2;
        v[3] = e[3] + o3;
        v[7] = e[3] - o3;
    }
}

// One in-place Stockham stage over NFFT transforms of length P at buf + f*LD (swizzled).
template <typename T, int P, int NFFT, int LD, int NTHR, int R, int NS, bool INV, int SCH = 0>
__device__ __forceinline__ void fft_stage(cx<T>* buf, const cx<T>* tw, int tid) {
    constexpr int NB = P / R;
    constexpr int TOTAL = NB * NFFT;
    constexpr int ITEMS = (TOTAL + NTHR - 1) / NTHR;
    constexpr int S = NS * R;
    constexpr int TWOFF = stage_tw_offset(P, NS, SCH);
    cx<T> v[ITEMS][R];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int idx = tid + it * NTHR;
        if ((TOTAL % NTHR == 0) || idx < TOTAL) {
            const int f = idx / NB, j = idx % NB;
            const cx<T>* src = buf + f * LD;
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = src[sw(j + r * NB)];
            if constexpr (NS > 1) {
                const int k = j % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cx<T> w = tw[TWOFF + k * (R - 1) + (r - 1)];
                    if (INV) w.im = -w.im;
                    v[it][r] = v[it][r] * w;
                }
            }
            dft_small<T, R, INV>(v[it]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int idx = tid + it * NTHR;
        if ((TOTAL % NTHR == 0) || idx < TOTAL) {
            const int f = idx / NB, j = idx % NB;
            const int k = j % NS;
            cx<T>* dst = buf + f * LD;
            const int base = (j / NS) * S + k;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[sw(base + r * NS)] = v[it][r];
        }
    }
    __syncthreads();
}

template <typename T, int P, int NFFT, int LD, int NTHR, bool INV, int NS, int SCH = 0>
__device__ __forceinline__ void fft_stages(cx<T>* buf, const cx<T>* tw, int tid) {
    if constexpr (NS < P) {
        constexpr int R = fft_radix(P, NS, SCH);
        fft_stage<T, P, NFFT, LD, NTHR, R, NS, INV, SCH>(buf, tw, tid);
        fft_stages<T, P, NFFT, LD, NTHR, INV, NS * R, SCH>(buf, tw, tid);
    }
}

// Unnormalised DFT (INV=false: exp(-2 pi i jk/P); INV=true: exp(+2 pi i jk/P)) of NFFT
// transforms held in LDS at buf + f*LD, element i at sw(i); LD >= padded(P).  tw is the
// twiddle table (LDS or global).  Must be called by all NTHR threads; ends with a barrier.
template <typename T, int P, int NFFT, int LD, int NTHR, bool INV, int SCH = 0>
__device__ __forceinline__ void block_fft(cx<T>* buf, const cx<T>* tw, int tid) {
    static_assert(is_pow2(P) && P >= 2, "FFT length must be a power of two");
    static_assert(LD >= P + P / 16, "LD must hold the padded transform");
    fft_stages<T, P, NFFT, LD, NTHR, INV, 1, SCH>(buf, tw, tid);
}

// The same over NFFT transforms processed in groups of at most G (fewer butterflies held in
// registers per stage, at the price of more barriers).
template <typename T, int P, int NFFT, int G, int LD, int NTHR, bool INV, int SCH = 0>
__device__ __forceinline__ void block_fft_grouped(cx<T>* buf, const cx<T>* tw, int tid) {
    if constexpr (NFFT <= G) {
        block_fft<T, P, NFFT, LD, NTHR, INV, SCH>(buf, tw, tid);
    } else {
        block_fft<T, P, G, LD, NTHR, INV, SCH>(buf, tw, tid);
        block_fft_grouped<T, P, NFFT - G, G, LD, NTHR, INV, SCH>(buf + G * LD, tw, tid);
    }
}

// The stages with sub-transform length in [NS, NSEND) only (for transforms whose first stage is
// fused into the load or whose last stage is fused into the store by the caller).
template <typename T, int P, int NFFT, int LD, int NTHR, bool INV, int NS, int NSEND, int SCH = 0>
__device__ __forceinline__ void fft_stages_range(cx<T>* buf, const cx<T>* tw, int tid) {
    if constexpr (NS < NSEND) {
        constexpr int R = fft_radix(P, NS, SCH);
        fft_stage<T, P, NFFT, LD, NTHR, R, NS, INV, SCH>(buf, tw, tid);
        fft_stages_range<T, P, NFFT, LD, NTHR, INV, NS * R, NSEND, SCH>(buf, tw, tid);
    }
}
template <typename T, int P, int NFFT, int G, int LD, int NTHR, bool INV, int NS, int NSEND, int SCH = 0>
__device__ __forceinline__ void block_fft_grouped_range(cx<T>* buf, const cx<T>* tw, int tid) {
    if constexpr (NFFT <= G) {
        fft_stages_range<T, P, NFFT, LD, NTHR, INV, NS, NSEND, SCH>(buf, tw, tid);
    } else {
        fft_stages_range<T, P, G, LD, NTHR, INV, NS, NSEND, SCH>(buf, tw, tid);
        block_fft_grouped_range<T, P, NFFT - G, G, LD, NTHR, INV, NS, NSEND, SCH>(buf + G * LD, tw, tid);
    }
}
// Sub-transform length of the last stage of a length-P transform.
constexpr int fft_last_ns(int P, int S = 0) {
    int ns = 1;
    while (ns * fft_radix(P, ns, S) < P) ns *= fft_radix(P, ns, S);
    return ns;
}

// Forward transforms of NFFT sequences whose entries y >= P/2 are zero (zero padding): the first
// stage (radix R0, no twiddles) is computed in registers from ld(f, y), y < P/2 (the functor returns
// zero past the data), and written to buf; the remaining stages run in LDS.  Ends with a barrier.
// Split in two so that a caller can issue the loads of its next group early:
// fft_padded_load fills the registers (PaddedIn), fft_padded_from_regs does the rest.
template <typename T, int P, int NFFT, int NTHR, int SCH = 0>
struct PaddedIn {
    static constexpr int R0 = fft_radix(P, 1, SCH);
    static constexpr int NB0 = P / R0;
    static constexpr int NBT = NFFT * NB0;
    static constexpr int IT = (NBT + NTHR - 1) / NTHR;
    cx<T> v[IT][R0 / 2];
};

template <typename T, int P, int NFFT, int NTHR, int SCH = 0, typename Ld>
__device__ __forceinline__ void fft_padded_load(PaddedIn<T, P, NFFT, NTHR, SCH>& in, int tid, Ld ld) {
    using PI = PaddedIn<T, P, NFFT, NTHR, SCH>;
#pragma unroll
    for (int it = 0; it < PI::IT; ++it) {
        const int idx = tid + it * NTHR;
        const int f = idx / PI::NB0, j = idx % PI::NB0;
#pragma unroll
        for (int r = 0; r < PI::R0 / 2; ++r)
            in.v[it][r] = (PI::NBT % NTHR == 0 || idx < PI::NBT) ? ld(f, j + r * PI::NB0) : mk((T)0, (T)0);
    }
}

template <typename T, int P, int NFFT, int LD, int NTHR, int SCH = 0>
__device__ __forceinline__ void fft_padded_from_regs(cx<T>* buf, const cx<T>* tws, int tid,
                                                     const PaddedIn<T, P, NFFT, NTHR, SCH>& in) {
    using PI = PaddedIn<T, P, NFFT, NTHR, SCH>;
    constexpr int R0 = PI::R0;
#pragma unroll
    for (int it = 0; it < PI::IT; ++it) {
        const int idx = tid + it * NTHR;
        if (PI::NBT % NTHR == 0 || idx < PI::NBT) {
            const int f = idx / PI::NB0, j = idx % PI::NB0;
            cx<T> v[R0];
#pragma unroll
            for (int r = 0; r < R0; ++r) v[r] = r < R0 / 2 ? in.v[it][r] : mk((T)0, (T)0);
            dft_small<T, R0, false>(v);
#pragma unroll
            for (int r = 0; r < R0; ++r) buf[f * LD + sw(j * R0 + r)] = v[r];
        }
    }
    __syncthreads();
    fft_stages_range<T, P, NFFT, LD, NTHR, false, R0, P, SCH>(buf, tws, tid);
}

template <typename T, int P, int NFFT, int LD, int NTHR, int SCH = 0, typename Ld>
__device__ __forceinline__ void fft_forward_padded(cx<T>* buf, const cx<T>* tws, int tid, Ld ld) {
    PaddedIn<T, P, NFFT, NTHR, SCH> in;
    fft_padded_load<T, P, NFFT, NTHR, SCH>(in, tid, ld);
    fft_padded_from_regs<T, P, NFFT, LD, NTHR, SCH>(buf, tws, tid, in);
}

// Inverse transforms of the NFFT sequences in buf of which only outputs y < P/2 are wanted: every
// stage but the last in LDS, the last in registers, handing y = j + r NSL (r < RL/2) to
// st(f, y, value) (the functor skips y past the data).  No barrier at the end.
template <typename T, int P, int NFFT, int LD, int NTHR, int SCH = 0, typename St>
__device__ __forceinline__ void fft_inverse_cropped(cx<T>* buf, const cx<T>* tws, int tid, St st) {
    constexpr int NSL = fft_last_ns(P, SCH);
    constexpr int RL = P / NSL;
    fft_stages_range<T, P, NFFT, LD, NTHR, true, 1, NSL, SCH>(buf, tws, tid);
    constexpr int TWL = stage_tw_offset(P, NSL, SCH);
    for (int idx = tid; idx < NFFT * NSL; idx += NTHR) {
        const int j = idx % NSL, f = idx / NSL;
        cx<T> v[RL];
#pragma unroll
        for (int r = 0; r < RL; ++r) v[r] = buf[f * LD + sw(j + r * NSL)];
        if constexpr (NSL > 1) {
#pragma unroll
            for (int r = 1; r < RL; ++r) {
                cx<T> w = tws[TWL + j * (RL - 1) + (r - 1)];
                w.im = -w.im;
                v[r] = v[r] * w;
            }
        }
        dft_small<T, RL, true>(v);
#pragma unroll
        for (int r = 0; r < RL / 2; ++r) st(f, j + r * NSL, v[r]);
    }
}

// Copy the P-entry twiddle table into LDS (all threads; followed by the caller's barrier).  Every
// load is issued before the first LDS store, so the copy costs one load latency, not P / NTHR.
template <typename T, int P, int NTHR>
__device__ __forceinline__ void stage_twiddles(cx<T>* tws, const cx<T>* __restrict__ tw, int tid) {
    constexpr int K = (P + NTHR - 1) / NTHR;
    cx<T> v[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int q = tid + u * NTHR;
        v[u] = (P % NTHR == 0 || q < P) ? tw[q] : mk((T)0, (T)0);
    }
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int q = tid + u * NTHR;
        if (P % NTHR == 0 || q < P) tws[q] = v[u];
    }
}

}  // namespace rte
