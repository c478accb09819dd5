// 2D FFT apply of the angularly reduced operator (Sec. 3.3.1, "Homogeneous media and FFT-based
// algorithm"; isotropic: Sec. 2.3.1).
//
// The kernel of K~ depends only on x_i - x_j and on k' - k, so K~ w is, per output mode k, a sum
// over input modes k' of 2D convolutions with K_{k'-k}.  Zero-padding each field to a
// PY x PX periodic grid (P >= 2n - 1) makes every convolution circulant and
//     FFT(K~ w)_k(xi) = sum_{k'} Khat_{k'-k}(xi) FFT(w_{k'})(xi),
// a (2L+1)x(2L+1) Toeplitz-in-mode product per frequency.
//
// Data are kept as real channels of a real angular flux (u_{-k} = conj u_k): channel 0 = u_0,
// channel 2k-1 = sqrt2 Re u_k, channel 2k = sqrt2 Im u_k.  Real fields let the x-transform be a
// real-to-complex FFT (frequencies 0..PX/2 only), which halves the work and traffic of the complex
// mode form; the complex modes are recombined per frequency inside pass B.
//
//   pass A  per (channel, tile of TR rows): scale by the channel's D entry, zero-pad to PX, FFT
//           along x (two real rows per complex FFT), store transposed T[c][kx][y]
//   pass B  per column kx: FFT along y for every channel (zero-padded to PY), couple the modes at
//           every frequency with the kernel spectra, inverse FFT along y, store back in place
//   pass C  per (channel, tile of rows): inverse FFT along x (complex-to-real), crop to nx, and
//           finalise y = x - v (operator A), y = v (K~), or y = b - x + v (residual)
//
// In 2D the x-frequencies 0 and PX/2 (real for real rows) share one complex column, so T has
// exactly PX/2 columns and pass B an even number of blocks.
//
// The kernel spectra are read from a quarter table Q[m][kx][ky], m = 0..2L, kx <= PX/2,
// ky <= PY/2, using Khat_m(kx, -ky) = (-1)^m conj Khat_m(kx, ky) (mirror symmetry of the square
// grid) and Khat_{-m} = (-1)^m conj Khat_m; the 1/(PX PY) of the inverse FFT is folded into Q.
#include "apply2d.h"
#include "apply2d_b.h"
#include "apply2d_tile.h"
#include "fft.h"

namespace rte {

// ---------------------------------------------------------------------------- pass A --------
// (the row tile itself, pass_a_tile, is in apply2d_tile.h)
template <typename T, int PX, int TR, int NTHR, typename TV, bool STAGED>
__global__ __launch_bounds__(NTHR) void k_pass_a(const TV* __restrict__ x, cx<T>* __restrict__ Tb,
                                                 const cx<T>* __restrict__ tw, int nx, int ny, int C,
                                                 ChanScale sc, int pack, const float* __restrict__ corr, int cF,
                                                 double cs) {
    constexpr int LD = padded(PX) + 1;
    __shared__ cx<T> buf[TR / 2 * LD];
    __shared__ cx<T> tws[PX];
    const int tid = threadIdx.x;
    const int bc = blockIdx.y;
    stage_twiddles<T, PX, NTHR>(tws, tw, tid);
    const int NKS = pack ? PX / 2 : PX / 2 + 1;
    const float* cc = corr ? corr + (size_t)(bc % C) * (ny / cF) * (nx / cF) : nullptr;
    __shared__ float crow[STAGED ? TR * CORR_WMAX : 1];
    pass_a_tile<T, PX, TR, NTHR, TV, STAGED>(x + (size_t)bc * ny * nx, Tb + (size_t)bc * NKS * ny, nx, ny,
                                             sc.s[bc % C], pack, xcd_tile(blockIdx.x, gridDim.x) * TR, buf, tws,
                                             tid, cc, cF, cs, crow);
}

// Batched form (isotropic problems of one padded size): one block per (problem, row tile).
template <typename T, int PX, int TR, int NTHR>
__global__ __launch_bounds__(NTHR) void k_pass_a_batch(const BatchProb<T>* __restrict__ probs,
                                                       const int2* __restrict__ items, const int* __restrict__ act,
                                                       const int* __restrict__ dj) {
    constexpr int LD = padded(PX) + 1;
    __shared__ cx<T> buf[TR / 2 * LD];
    __shared__ cx<T> tws[PX];
    const int2 item = items[blockIdx.x];
    const BatchProb<T>& d = probs[item.x];
    if (act && !act[item.x]) return;
    const int tid = threadIdx.x;
    const size_t j = dj ? (size_t)*dj : 0;
    stage_twiddles<T, PX, NTHR>(tws, d.twx, tid);
    pass_a_tile<T, PX, TR, NTHR>(d.in + (d.jin ? j * d.stride : 0), d.work, d.nx, d.ny, d.s, 1, item.y * TR, buf, tws,
                                 tid);
}

// ---------------------------------------------------------------------------- pass C --------
// One tile of TR rows of one channel: src is the channel's [NKS][ny] spectrum; xin, bin, yout its
// [ny][nx] input, right-hand side and output.
template <typename T, int PX, int TR, int NTHR, typename TV>
__device__ __forceinline__ void pass_c_tile(const cx<T>* __restrict__ src, const TV* __restrict__ xin,
                                            const double* __restrict__ bin, TV* __restrict__ yout, int nx, int ny,
                                            int mode, int pack, int y0, cx<T>* buf, const cx<T>* tws, int tid,
                                            const float* __restrict__ corr_c = nullptr, int cF = 1, double cs = 0.0,
                                            float* crow = nullptr) {
    constexpr int NP = TR / 2;
    constexpr int LD = padded(PX) + 1;   // odd row pitch: the NP transforms start on different banks
    constexpr int H = PX / 2;
    const int NKS = pack ? H : H + 1;
    constexpr int NL = (H + 1) * NP;
    constexpr int IT = (NL + NTHR - 1) / NTHR;
    cx<T> xa[IT], xb[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int idx = tid + it * NTHR;
        const int p = idx % NP, k = idx / NP;
        const int ya = y0 + 2 * p, yb = ya + 1;
        const bool ok = k < NKS;
        xa[it] = (ok && ya < ny) ? src[(size_t)k * ny + ya] : mk((T)0, (T)0);
        xb[it] = (ok && yb < ny) ? src[(size_t)k * ny + yb] : mk((T)0, (T)0);
    }
    // the staged correction rows are ordered before their use by the barrier after the buf fill
    int Hc = 1, Wc = 1;
    bool staged = false;
    if (corr_c) {
        Hc = ny / cF;
        Wc = nx / cF;
        staged = crow && Wc <= CORR_WMAX;
        if (staged) stage_corr_rows<TR, NTHR>(corr_c, Hc, Wc, cF, y0, ny, crow, tid);
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int idx = tid + it * NTHR;
        const int p = idx % NP, k = idx / NP;
        if (k < NKS) {
            cx<T> Xa = xa[it], Xb = xb[it];
            if (pack && k == 0) {   // (X[0], X[PX/2]) of rows a and b
                buf[p * LD + sw(0)] = mk(Xa.re, Xb.re);
                buf[p * LD + sw(H)] = mk(Xa.im, Xb.im);
            } else {
                if (k == 0 || k == H) { Xa.im = 0; Xb.im = 0; }
                buf[p * LD + sw(k)] = Xa + mul_i(Xb);
                if (k > 0 && k < H) buf[p * LD + sw(PX - k)] = conj(Xa) + mul_i(conj(Xb));
            }
        }
    }
    __syncthreads();
    // Inverse x-FFT: every stage but the last in LDS; the last stage (sub-length NSL, radix RL) is
    // done per butterfly in registers and finalised at once.  Its outputs m = j + r NSL with
    // r < RL/2 are the columns m < PX/2 (only m < nx are kept); the real part is row y0 + 2p, the
    // imaginary part row y0 + 2p + 1.
    constexpr int NSL = fft_last_ns(PX);
    constexpr int RL = PX / NSL;
    fft_stages_range<T, PX, NP, LD, NTHR, true, 1, NSL>(buf, tws, tid);
    constexpr int TWL = stage_tw_offset(PX, NSL);
    constexpr int NBT = NP * NSL;
    for (int idx = tid; idx < NBT; idx += NTHR) {
        const int p = idx / NSL, j = idx % NSL;
        const int ya = y0 + 2 * p, yb = ya + 1;
        double xa_[RL / 2], xb_[RL / 2], ba_[RL / 2], bb_[RL / 2];
        // x loads with a clamped index (no branch), all issued before the widening (as in pass A)
        TV la[RL / 2], lb[RL / 2];
        if (mode != APPLY_KT) {
#pragma unroll
            for (int r = 0; r < RL / 2; ++r) {
                const int m = j + r * NSL;
                la[r] = xin[(m < nx && ya < ny) ? (size_t)ya * nx + m : 0];
                lb[r] = xin[(m < nx && yb < ny) ? (size_t)yb * nx + m : 0];
            }
        }
#pragma unroll
        for (int r = 0; r < RL / 2; ++r) {
            const int m = j + r * NSL;
            const bool oka = m < nx && ya < ny, okb = m < nx && yb < ny;
            xa_[r] = (oka && mode != APPLY_KT) ? (double)la[r] : 0.0;
            xb_[r] = (okb && mode != APPLY_KT) ? (double)lb[r] : 0.0;
            ba_[r] = (oka && mode == APPLY_RESID) ? bin[(size_t)ya * nx + m] : 0.0;
            bb_[r] = (okb && mode == APPLY_RESID) ? bin[(size_t)yb * nx + m] : 0.0;
            if (staged) {
                int x0, x1;
                float ax;
                lerp_at(min(m, nx - 1), cF, Wc, x0, x1, ax);
                if (oka) xa_[r] += cs * (double)corr_row_at(crow, 2 * p, x0, x1, ax);
                if (okb) xb_[r] += cs * (double)corr_row_at(crow, 2 * p + 1, x0, x1, ax);
            } else if (corr_c) {
                if (oka) xa_[r] += cs * (double)coarse_bilerp(corr_c, Hc, Wc, cF, ya, m);
                if (okb) xb_[r] += cs * (double)coarse_bilerp(corr_c, Hc, Wc, cF, yb, m);
            }
        }
        cx<T> v[RL];
#pragma unroll
        for (int r = 0; r < RL; ++r) v[r] = buf[p * LD + sw(j + r * NSL)];
        if constexpr (NSL > 1) {   // a single-stage transform has no twiddles
#pragma unroll
            for (int r = 1; r < RL; ++r) {
                cx<T> w = tws[TWL + j * (RL - 1) + (r - 1)];
                w.im = -w.im;
                v[r] = v[r] * w;
            }
        }
        dft_small<T, RL, true>(v);
#pragma unroll
        for (int r = 0; r < RL / 2; ++r) {
            const int m = j + r * NSL;
            if (m >= nx) continue;
            const double va = (double)v[r].re, vb = (double)v[r].im;
            if (ya < ny)
                yout[(size_t)ya * nx + m] =
                    (TV)(mode == APPLY_A ? xa_[r] - va : mode == APPLY_KT ? va : ba_[r] - xa_[r] + va);
            if (yb < ny)
                yout[(size_t)yb * nx + m] =
                    (TV)(mode == APPLY_A ? xb_[r] - vb : mode == APPLY_KT ? vb : bb_[r] - xb_[r] + vb);
        }
    }
}

template <typename T, int PX, int TR, int NTHR, typename TV>
__global__ __launch_bounds__(NTHR) void k_pass_c(const cx<T>* __restrict__ Tb, const TV* __restrict__ xin,
                                                 const double* __restrict__ bin, TV* __restrict__ yout,
                                                 const cx<T>* __restrict__ tw, int nx, int ny, int mode, int pack,
                                                 int C, const float* __restrict__ corr, int cF, double cs) {
    constexpr int LD = padded(PX) + 1;
    __shared__ cx<T> buf[TR / 2 * LD];
    __shared__ cx<T> tws[PX];
    __shared__ float crow[TR * CORR_WMAX];
    const int tid = threadIdx.x;
    const int bc = blockIdx.y;
    const int NKS = pack ? PX / 2 : PX / 2 + 1;
    stage_twiddles<T, PX, NTHR>(tws, tw, tid);
    const size_t base = (size_t)bc * ny * nx;
    const float* cc = corr ? corr + (size_t)(bc % C) * (ny / cF) * (nx / cF) : nullptr;
    pass_c_tile<T, PX, TR, NTHR>(Tb + (size_t)bc * NKS * ny, xin ? xin + base : nullptr, bin ? bin + base : nullptr,
                                 yout + base, nx, ny, mode, pack, xcd_tile(blockIdx.x, gridDim.x) * TR, buf, tws, tid,
                                 cc, cF, cs, crow);
}

// Batched form: one block per (problem, row tile); the output is written to out + (j + 1) stride
// when jout is set (the next Krylov vector).
template <typename T, int PX, int TR, int NTHR>
__global__ __launch_bounds__(NTHR) void k_pass_c_batch(const BatchProb<T>* __restrict__ probs,
                                                       const int2* __restrict__ items, const int* __restrict__ act,
                                                       const int* __restrict__ dj, int mode) {
    constexpr int LD = padded(PX) + 1;
    __shared__ cx<T> buf[TR / 2 * LD];
    __shared__ cx<T> tws[PX];
    const int2 item = items[blockIdx.x];
    const BatchProb<T>& d = probs[item.x];
    if (act && !act[item.x]) return;
    const int tid = threadIdx.x;
    const size_t j = dj ? (size_t)*dj : 0;
    stage_twiddles<T, PX, NTHR>(tws, d.twx, tid);
    pass_c_tile<T, PX, TR, NTHR>(d.work, d.in + (d.jin ? j * d.stride : 0), d.bvec,
                                 d.out + (d.jout ? (j + 1) * d.stride : 0), d.nx, d.ny, mode, 1, item.y * TR, buf, tws,
                                 tid);
}

// ---------------------------------------------------------------------------- dispatch -------
template <typename T> constexpr int tile_rows() { return sizeof(T) == 4 ? 16 : 8; }
template <typename T, int PX, int TR, typename TV>
static void launch_a_tr(const Apply2DArgs<T>& a, const TV* x, const ChanScale& sc, int nchan_total) {
    dim3 grid((a.ny + TR - 1) / TR, nchan_total);
    if (a.corr && a.nx / a.cF <= CORR_WMAX)
        hipLaunchKernelGGL((k_pass_a<T, PX, TR, 256, TV, true>), grid, dim3(256), 0, a.stream, x, a.work, a.twx,
                           a.nx, a.ny, a.C, sc, a.pack, a.corr, a.cF, a.cs);
    else
        hipLaunchKernelGGL((k_pass_a<T, PX, TR, 256, TV, false>), grid, dim3(256), 0, a.stream, x, a.work, a.twx,
                           a.nx, a.ny, a.C, sc, a.pack, a.corr, a.cF, a.cs);
}
template <typename T, int PX, typename TV>
static void launch_a(const Apply2DArgs<T>& a, const TV* x, const ChanScale& sc, int nchan_total) {
    constexpr int TR = tile_rows<T>();
    if constexpr (PX >= 128) {
        if (a.var[0] == 1) return launch_a_tr<T, PX, TR / 2>(a, x, sc, nchan_total);
        if (a.var[0] == 2) return launch_a_tr<T, PX, TR * 2>(a, x, sc, nchan_total);
        if (a.var[0] == 3) return launch_a_tr<T, PX, TR / 4>(a, x, sc, nchan_total);
    }
    launch_a_tr<T, PX, TR>(a, x, sc, nchan_total);
}

template <typename T, int PX, int TR, typename TV>
static void launch_c_tr(const Apply2DArgs<T>& a, const TV* x, const double* b, TV* y, int mode,
                        int nchan_total) {
    dim3 grid((a.ny + TR - 1) / TR, nchan_total);
    hipLaunchKernelGGL((k_pass_c<T, PX, TR, 256, TV>), grid, dim3(256), 0, a.stream, a.work, x, b, y, a.twx,
                       a.nx, a.ny, mode, a.pack, a.C, mode == APPLY_A ? a.corr : nullptr, a.cF, a.cs);
}
template <typename T, int PX, typename TV>
static void launch_c(const Apply2DArgs<T>& a, const TV* x, const double* b, TV* y, int mode,
                     int nchan_total) {
    constexpr int TR = tile_rows<T>();
    if constexpr (PX >= 128) {
        if (a.var[2] == 1) return launch_c_tr<T, PX, TR / 2>(a, x, b, y, mode, nchan_total);
        if (a.var[2] == 2) return launch_c_tr<T, PX, TR * 2>(a, x, b, y, mode, nchan_total);
        if (a.var[2] == 3) return launch_c_tr<T, PX, TR / 4>(a, x, b, y, mode, nchan_total);
    }
    launch_c_tr<T, PX, TR>(a, x, b, y, mode, nchan_total);
}

#define RTE_P_SWITCH(P, FN, ...)                  \
    switch (P) {                                  \
        case 16: FN<T, 16>(__VA_ARGS__); break;   \
        case 32: FN<T, 32>(__VA_ARGS__); break;   \
        case 64: FN<T, 64>(__VA_ARGS__); break;   \
        case 128: FN<T, 128>(__VA_ARGS__); break; \
        case 256: FN<T, 256>(__VA_ARGS__); break; \
        case 512: FN<T, 512>(__VA_ARGS__); break; \
        case 1024: FN<T, 1024>(__VA_ARGS__); break; \
        default: return -1;                       \
    }

template <typename T>
int apply2d_variant_count(int pass, int L, int PX, int PY) {
    if (pass == 0 || pass == 2) return PX >= 128 ? 4 : 1;
    if (pass != 1) return 0;
    switch (L) {
        case 0: return pass_b_variants_L0<T>(PY);
        case 1: return pass_b_variants_L1<T>(PY);
        case 2: return pass_b_variants_L2<T>(PY);
        case 3: return pass_b_variants_L3<T>(PY);
        case 4: return pass_b_variants_L4<T>(PY);
        case 5: return pass_b_variants_L5<T>(PY);
        case 6: return pass_b_variants_L6<T>(PY);
        case 7: return pass_b_variants_L7<T>(PY);
        case 8: return pass_b_variants_L8<T>(PY);
    }
    return L <= RTE_MAX_L ? 2 : 0;   // mode-axis FFT or direct coupling
}
template int apply2d_variant_count<float>(int, int, int, int);
template int apply2d_variant_count<double>(int, int, int, int);

template <typename T, typename TV>
int apply2d_pass_a(const Apply2DArgs<T>& a, const TV* x, const ChanScale& sc, int nbatch) {
    RTE_P_SWITCH(a.PX, launch_a, a, x, sc, nbatch * a.C);
    return 0;
}
template <typename T>
int apply2d_pass_b(const Apply2DArgs<T>& a, int nbatch) {
    switch (a.L) {
        case 0: return pass_b_L0<T>(a, nbatch);
        case 1: return pass_b_L1<T>(a, nbatch);
        case 2: return pass_b_L2<T>(a, nbatch);
        case 3: return pass_b_L3<T>(a, nbatch);
        case 4: return pass_b_L4<T>(a, nbatch);
        case 5: return pass_b_L5<T>(a, nbatch);
        case 6: return pass_b_L6<T>(a, nbatch);
        case 7: return pass_b_L7<T>(a, nbatch);
        case 8: return pass_b_L8<T>(a, nbatch);
    }
    return pass_b_large<T>(a, nbatch);
}
template <typename T>
bool apply2d_needs_work2(int L, int PY) {
    switch (L) {
        case 0: return pass_b_split_L0<T>(PY);
        case 1: return pass_b_split_L1<T>(PY);
        case 2: return pass_b_split_L2<T>(PY);
        case 3: return pass_b_split_L3<T>(PY);
        case 4: return pass_b_split_L4<T>(PY);
        case 5: return pass_b_split_L5<T>(PY);
        case 6: return pass_b_split_L6<T>(PY);
        case 7: return pass_b_split_L7<T>(PY);
        case 8: return pass_b_split_L8<T>(PY);
    }
    return true;   // L > 8: split form
}
template bool apply2d_needs_work2<float>(int, int);
template bool apply2d_needs_work2<double>(int, int);
template <typename T>
bool apply2d_unpacked(int L, int PY, int var_b) {
    switch (L) {
        case 0: return pass_b_unpacked_L0<T>(PY, var_b);
        case 1: return pass_b_unpacked_L1<T>(PY, var_b);
        case 2: return pass_b_unpacked_L2<T>(PY, var_b);
        case 3: return pass_b_unpacked_L3<T>(PY, var_b);
        case 4: return pass_b_unpacked_L4<T>(PY, var_b);
        case 5: return pass_b_unpacked_L5<T>(PY, var_b);
        case 6: return pass_b_unpacked_L6<T>(PY, var_b);
        case 7: return pass_b_unpacked_L7<T>(PY, var_b);
        case 8: return pass_b_unpacked_L8<T>(PY, var_b);
    }
    return true;   // L > 8: split form over unpacked columns
}
template bool apply2d_unpacked<float>(int, int, int);
template bool apply2d_unpacked<double>(int, int, int);
template <typename T>
bool apply2d_b_corr_ok(int L, int PY, int var_b) {
    switch (L) {
        case 0: return pass_b_corr_ok_L0<T>(PY, var_b);
        case 1: return pass_b_corr_ok_L1<T>(PY, var_b);
        case 2: return pass_b_corr_ok_L2<T>(PY, var_b);
        case 3: return pass_b_corr_ok_L3<T>(PY, var_b);
        case 4: return pass_b_corr_ok_L4<T>(PY, var_b);
        case 5: return pass_b_corr_ok_L5<T>(PY, var_b);
        case 6: return pass_b_corr_ok_L6<T>(PY, var_b);
        case 7: return pass_b_corr_ok_L7<T>(PY, var_b);
        case 8: return pass_b_corr_ok_L8<T>(PY, var_b);
    }
    return false;
}
template bool apply2d_b_corr_ok<float>(int, int, int);
template bool apply2d_b_corr_ok<double>(int, int, int);
template <typename T, typename TV>
int apply2d_pass_c(const Apply2DArgs<T>& a, const TV* x, const double* b, TV* y, int mode,
                   int nbatch) {
    RTE_P_SWITCH(a.PX, launch_c, a, x, b, y, mode, nbatch * a.C);
    return 0;
}

// Row tile of batched variant v (shared by passes A and C): the default, half, twice or a quarter
// of it, as the single-problem variants; padded x >= 128 only.
template <typename T>
int apply2d_batch_row_variants(int PX) { return PX >= 128 ? 4 : 1; }
template <typename T>
int apply2d_batch_rows(int var) {
    constexpr int TR = tile_rows<T>();
    return var == 1 ? TR / 2 : var == 2 ? TR * 2 : var == 3 ? TR / 4 : TR;
}
template <typename T, int PX, int TR>
static void launch_a_batch_tr(const BatchProb<T>* probs, const int2* items, int nitems, const int* act, const int* dj,
                              hipStream_t st) {
    hipLaunchKernelGGL((k_pass_a_batch<T, PX, TR, 256>), dim3(nitems), dim3(256), 0, st, probs, items, act, dj);
}
template <typename T, int PX>
static void launch_a_batch(const BatchProb<T>* probs, const int2* items, int nitems, const int* act, const int* dj,
                           int var, hipStream_t st) {
    constexpr int TR = tile_rows<T>();
    if constexpr (PX >= 128) {
        if (var == 1) return launch_a_batch_tr<T, PX, TR / 2>(probs, items, nitems, act, dj, st);
        if (var == 2) return launch_a_batch_tr<T, PX, TR * 2>(probs, items, nitems, act, dj, st);
        if (var == 3) return launch_a_batch_tr<T, PX, TR / 4>(probs, items, nitems, act, dj, st);
    }
    launch_a_batch_tr<T, PX, TR>(probs, items, nitems, act, dj, st);
}
template <typename T, int PX, int TR>
static void launch_c_batch_tr(const BatchProb<T>* probs, const int2* items, int nitems, const int* act, const int* dj,
                              int mode, hipStream_t st) {
    hipLaunchKernelGGL((k_pass_c_batch<T, PX, TR, 256>), dim3(nitems), dim3(256), 0, st, probs, items, act, dj, mode);
}
template <typename T, int PX>
static void launch_c_batch(const BatchProb<T>* probs, const int2* items, int nitems, const int* act, const int* dj,
                           int mode, int var, hipStream_t st) {
    constexpr int TR = tile_rows<T>();
    if constexpr (PX >= 128) {
        if (var == 1) return launch_c_batch_tr<T, PX, TR / 2>(probs, items, nitems, act, dj, mode, st);
        if (var == 2) return launch_c_batch_tr<T, PX, TR * 2>(probs, items, nitems, act, dj, mode, st);
        if (var == 3) return launch_c_batch_tr<T, PX, TR / 4>(probs, items, nitems, act, dj, mode, st);
    }
    launch_c_batch_tr<T, PX, TR>(probs, items, nitems, act, dj, mode, st);
}
template <typename T>
int apply2d_batch_pass_a(int PX, const BatchProb<T>* probs, const int2* items, int nitems, const int* act,
                         const int* dj, int var, hipStream_t st) {
    if (nitems <= 0) return 0;
    if (var < 0 || var >= apply2d_batch_row_variants<T>(PX)) return -1;
    RTE_P_SWITCH(PX, launch_a_batch, probs, items, nitems, act, dj, var, st);
    return 0;
}
template <typename T>
int apply2d_batch_pass_c(int PX, const BatchProb<T>* probs, const int2* items, int nitems, const int* act,
                         const int* dj, int mode, int var, hipStream_t st) {
    if (nitems <= 0) return 0;
    if (var < 0 || var >= apply2d_batch_row_variants<T>(PX)) return -1;
    RTE_P_SWITCH(PX, launch_c_batch, probs, items, nitems, act, dj, mode, var, st);
    return 0;
}
template int apply2d_batch_row_variants<float>(int);
template int apply2d_batch_row_variants<double>(int);
template int apply2d_batch_rows<float>(int);
template int apply2d_batch_rows<double>(int);
template int apply2d_batch_pass_a<float>(int, const BatchProb<float>*, const int2*, int, const int*, const int*, int,
                                         hipStream_t);
template int apply2d_batch_pass_a<double>(int, const BatchProb<double>*, const int2*, int, const int*, const int*, int,
                                          hipStream_t);
template int apply2d_batch_pass_c<float>(int, const BatchProb<float>*, const int2*, int, const int*, const int*, int,
                                         int, hipStream_t);
template int apply2d_batch_pass_c<double>(int, const BatchProb<double>*, const int2*, int, const int*, const int*, int,
                                          int, hipStream_t);

template <typename T, typename TV>
int apply2d(const Apply2DArgs<T>& a, const TV* x, const double* b, TV* y, int mode,
            const ChanScale& sc, int nbatch) {
    if (apply2d_pass_a<T>(a, x, sc, nbatch)) return -1;
    if (apply2d_pass_b<T>(a, nbatch)) return -1;
    return apply2d_pass_c<T>(a, x, b, y, mode, nbatch);
}

template <typename T, typename TV>
int apply2d_from_b(const Apply2DArgs<T>& a, const TV* x, TV* y) {
    if (!a.bcorr.y || !a.corr) return -1;
    if (apply2d_pass_b<T>(a, 1)) return -1;
    return apply2d_pass_c<T>(a, x, nullptr, y, APPLY_A, 1);
}

// (compute precision, vector storage): FP64 vectors for both precisions, FP32 vectors for the
// FP32 apply (the inner solve's basis)
#define RTE_APPLY2D_INST(T, TV)                                                                             \
    template int apply2d<T, TV>(const Apply2DArgs<T>&, const TV*, const double*, TV*, int, const ChanScale&, \
                                int);                                                                       \
    template int apply2d_pass_a<T, TV>(const Apply2DArgs<T>&, const TV*, const ChanScale&, int);            \
    template int apply2d_pass_c<T, TV>(const Apply2DArgs<T>&, const TV*, const double*, TV*, int, int);     \
    template int apply2d_from_b<T, TV>(const Apply2DArgs<T>&, const TV*, TV*);
RTE_APPLY2D_INST(float, double)
RTE_APPLY2D_INST(double, double)
RTE_APPLY2D_INST(float, float)
#undef RTE_APPLY2D_INST
template int apply2d_pass_b<float>(const Apply2DArgs<float>&, int);
template int apply2d_pass_b<double>(const Apply2DArgs<double>&, int);

}  // namespace rte
