// Device-side pieces of the 2D apply shared by its kernels and by the preconditioned Arnoldi
// step, which runs the next vector's pass A inside its stage-1 launch: the coarse correction's
// bilinear interpolation, the XCD-aware tile order and one row tile of pass A.
#pragma once
#include "apply2d.h"
#include "fft.h"

namespace rte {

// Bilinear interpolation of a coarse field yc[Hc][Wc] (cell-centred, coarse cell I covering fine
// cells I*F .. I*F+F-1, clamped to the outer coarse centres) at fine cell (y, x).
__device__ __forceinline__ void lerp_at(int i, int F, int nc, int& lo, int& hi, float& a) {
    const float xi = ((float)i + 0.5f) / (float)F - 0.5f;
    const float f0 = floorf(xi);
    a = xi - f0;
    const int i0 = (int)f0;
    lo = min(max(i0, 0), nc - 1);
    hi = min(max(i0 + 1, 0), nc - 1);
}
__device__ __forceinline__ float coarse_bilerp(const float* __restrict__ yc, int Hc, int Wc, int F, int y, int x) {
    int y0, y1, x0, x1;
    float ay, ax;
    lerp_at(y, F, Hc, y0, y1, ay);
    lerp_at(x, F, Wc, x0, x1, ax);
    const float top = (1.f - ax) * yc[y0 * Wc + x0] + ax * yc[y0 * Wc + x1];
    const float bot = (1.f - ax) * yc[y1 * Wc + x0] + ax * yc[y1 * Wc + x1];
    return (1.f - ay) * top + ay * bot;
}

// The coarse correction of a tile of TR fine rows, interpolated in y and staged in LDS:
// crow[yl * CORR_WMAX + X] for fine row y0 + yl and coarse column X < Wc (Wc <= CORR_WMAX).  Pass C
// then interpolates in x from two LDS values per cell instead of four loads of the coarse field.
// It is the same bilinear prolongation as coarse_bilerp (pass A), with the two interpolations in
// the other order, so the two passes agree to FP32 rounding.
constexpr int CORR_WMAX = 32;   // keeps two 16-row FP32 tiles per CU (2 x 79.9 KB)
template <int TR, int NTHR>
__device__ __forceinline__ void stage_corr_rows(const float* __restrict__ yc, int Hc, int Wc, int F, int y0, int ny,
                                                float* crow, int tid) {
    for (int idx = tid; idx < TR * Wc; idx += NTHR) {
        const int yl = idx / Wc, X = idx % Wc;
        int r0, r1;
        float ay;
        lerp_at(min(y0 + yl, ny - 1), F, Hc, r0, r1, ay);
        crow[yl * CORR_WMAX + X] = (1.f - ay) * yc[r0 * Wc + X] + ay * yc[r1 * Wc + X];
    }
}
__device__ __forceinline__ float corr_row_at(const float* crow, int yl, int x0, int x1, float ax) {
    const float* r = crow + yl * CORR_WMAX;
    return (1.f - ax) * r[x0] + ax * r[x1];
}

// Row tile of a block: workgroups are dispatched round-robin over the 8 XCDs (linear id mod 8), and
// neighbouring tiles share 128-byte lines of the transposed spectrum (a tile reads or writes TR
// consecutive rows of every column).  When the x-grid is a multiple of 8, XCD k is given the
// contiguous tiles k G/8 .. (k+1) G/8 - 1 so that those lines meet in one L2.
__device__ __forceinline__ int xcd_tile(int b, int G) { return (G & 7) ? b : (b & 7) * (G >> 3) + (b >> 3); }

// ---------------------------------------------------------------------------- pass A --------
// With pack != 0 the x-frequencies 0 and PX/2, whose values are real for real rows, share
// column 0 of T as (X[0], X[PX/2]); T then has PX/2 columns.
// One tile of TR rows of one channel: xin is the channel's [ny][nx] input, out its [NKS][ny]
// transposed x-spectrum; tws holds the staged twiddles.
template <typename T, int PX, int TR, int NTHR, typename TV, bool STAGED = false>
__device__ __forceinline__ void pass_a_tile(const TV* __restrict__ xin, cx<T>* __restrict__ out, int nx, int ny,
                                            double s, int pack, int y0, cx<T>* buf, const cx<T>* tws, int tid,
                                            const float* __restrict__ corr_c = nullptr, int cF = 1, double cs = 0.0,
                                            float* crow = nullptr) {
    constexpr int NP = TR / 2;        // complex FFTs per block (two real rows each)
    constexpr int LD = padded(PX) + 1;   // odd row pitch: the NP transforms start on different banks
    constexpr int H = PX / 2;
    // Rows y0+2p (real part) and y0+2p+1 (imaginary part); only m < nx <= PX/2 is non-zero, so the
    // first Stockham stage (radix R0, no twiddles) runs in registers on the loads: butterfly j takes
    // m = j + r PX/R0 (non-zero only for r < R0/2) and writes its R0 outputs at j R0 + r.
    constexpr int R0 = fft_radix(PX, 1);
    constexpr int NB0 = PX / R0;
    constexpr int NBT = NP * NB0;
    constexpr int IT = (NBT + NTHR - 1) / NTHR;
    // Every load of the tile is issued before the first use: the loads take a clamped index (the
    // channel's first entry when out of range) instead of a branch, and the widening to FP64
    // follows all of them (a conversion next to each load made the FP32 loads wait one by one).
    TV la[IT][R0 / 2], lb[IT][R0 / 2];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int idx = tid + it * NTHR;
        const int p = idx / NB0, j = idx % NB0;
        const int ya = y0 + 2 * p, yb = ya + 1;
#pragma unroll
        for (int r = 0; r < R0 / 2; ++r) {
            const int m = j + r * NB0;
            const bool ok = (NBT % NTHR == 0 || idx < NBT) && m < nx;
            la[it][r] = xin[(ok && ya < ny) ? (size_t)ya * nx + m : 0];
            lb[it][r] = xin[(ok && yb < ny) ? (size_t)yb * nx + m : 0];
        }
    }
    double ra[IT][R0 / 2], rb[IT][R0 / 2];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int idx = tid + it * NTHR;
        const int p = idx / NB0, j = idx % NB0;
        const int ya = y0 + 2 * p, yb = ya + 1;
#pragma unroll
        for (int r = 0; r < R0 / 2; ++r) {
            const int m = j + r * NB0;
            const bool ok = (NBT % NTHR == 0 || idx < NBT) && m < nx;
            ra[it][r] = (ok && ya < ny) ? (double)la[it][r] : 0.0;
            rb[it][r] = (ok && yb < ny) ? (double)lb[it][r] : 0.0;
        }
    }
    if (STAGED) {
        // y-interpolated coarse rows in LDS (nx / cF <= CORR_WMAX), as in pass C; a separate
        // instantiation, since one kernel holding both forms needed 102 registers instead of 66
        const int Hc = ny / cF, Wc = nx / cF;
        stage_corr_rows<TR, NTHR>(corr_c, Hc, Wc, cF, y0, ny, crow, tid);
        __syncthreads();
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int idx = tid + it * NTHR;
            const int p = idx / NB0, j = idx % NB0;
#pragma unroll
            for (int r = 0; r < R0 / 2; ++r) {
                const int m = j + r * NB0;
                const bool ok = (NBT % NTHR == 0 || idx < NBT) && m < nx;   // p < NP when ok
                int x0, x1;
                float ax;
                lerp_at(min(m, nx - 1), cF, Wc, x0, x1, ax);
                if (ok && y0 + 2 * p < ny) ra[it][r] += cs * (double)corr_row_at(crow, 2 * p, x0, x1, ax);
                if (ok && y0 + 2 * p + 1 < ny) rb[it][r] += cs * (double)corr_row_at(crow, 2 * p + 1, x0, x1, ax);
            }
        }
    } else if (corr_c) {
        // direct reads of the coarse field
        const int Hc = ny / cF, Wc = nx / cF;
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int idx = tid + it * NTHR;
            const int p = idx / NB0, j = idx % NB0;
            const int ya = y0 + 2 * p, yb = ya + 1;
#pragma unroll
            for (int r = 0; r < R0 / 2; ++r) {
                const int m = j + r * NB0;
                const bool ok = (NBT % NTHR == 0 || idx < NBT) && m < nx;
                if (ok && ya < ny) ra[it][r] += cs * (double)coarse_bilerp(corr_c, Hc, Wc, cF, ya, m);
                if (ok && yb < ny) rb[it][r] += cs * (double)coarse_bilerp(corr_c, Hc, Wc, cF, yb, m);
            }
        }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int idx = tid + it * NTHR;
        if (NBT % NTHR == 0 || idx < NBT) {
            const int p = idx / NB0, j = idx % NB0;
            cx<T> v[R0];
#pragma unroll
            for (int r = 0; r < R0; ++r)
                v[r] = r < R0 / 2 ? mk((T)(s * ra[it][r]), (T)(s * rb[it][r])) : mk((T)0, (T)0);
            dft_small<T, R0, false>(v);
#pragma unroll
            for (int r = 0; r < R0; ++r) buf[p * LD + sw(j * R0 + r)] = v[r];
        }
    }
    __syncthreads();
    fft_stages_range<T, PX, NP, LD, NTHR, false, R0, PX>(buf, tws, tid);
    const int NKS = pack ? H : H + 1;
    for (int idx = tid; idx < NKS * TR; idx += NTHR) {
        const int yl = idx % TR, k = idx / TR;
        const int y = y0 + yl;
        if (y < ny) {
            const int p = yl >> 1;
            cx<T> X;
            if (pack && k == 0) {
                const cx<T> z0 = buf[p * LD + sw(0)], zh = buf[p * LD + sw(H)];
                X = (yl & 1) ? mk(z0.im, zh.im) : mk(z0.re, zh.re);
            } else {
                const cx<T> z = buf[p * LD + sw(k)];
                const cx<T> zc = conj(buf[p * LD + sw((PX - k) & (PX - 1))]);
                // X_a = (Z + conj Z(-k))/2,  X_b = (Z - conj Z(-k))/(2i)
                X = (yl & 1) ? scale(mul_mi(z - zc), (T)0.5) : scale(z + zc, (T)0.5);
            }
            out[(size_t)k * ny + y] = X;
        }
    }
}

}  // namespace rte
