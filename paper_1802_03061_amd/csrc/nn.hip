// Learned right preconditioner: a coarse-grid 3x3 convolution network (see include/rte_nn.h).
// The correction is computed on an F x F block-averaged grid and interpolated back bilinearly:
// the predicted error is tens of times larger than the residual, so it must come back smooth --
// jumps at block edges would reappear almost unchanged in A z (A is close to the identity on
// rough fields) and swamp the residual.
//
// Convolution as an implicit GEMM on MFMA: out[o][p] = sum_k W[o][k] X[k][p] with k = c*9 + tap
// (tap = 3*(dy+1) + (dx+1)) and X[k][p] the input at p + (dy, dx).  Each 64-lane wave computes a
// 32 (output channels) x 32 (pixels of one row) tile with v_mfma_f32_32x32x8_bf16, K in steps of
// 8; BF16 operands, FP32 accumulation.  The input tile with its one-cell halo is staged in LDS as
// BF16.  The data gradient is the same convolution with the weights flipped in space and
// transposed in channels, masked by the ReLU derivative of the previous layer.  Weight and bias
// gradients are one more GEMM on MFMA (BF16 operands, FP32 accumulation) over the batch's pixels,
// reduced across blocks in a fixed order.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <random>
#include <vector>

#include "../../include/rte_nn.h"
#include "apply2d.h"
#include "apply2d_tile.h"
#include "ctx.h"
#include "arnoldi_dev.h"
#include "krylov.h"
#include "nn.h"

namespace rte {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ unsigned short f2bf(float f) {   // round to nearest even
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

constexpr int kpad(int cin) { return (cin * 9 + 7) / 8 * 8; }

// ------------------------------------------------------------------ convolution (MFMA) --------
// in [B][CIN][H][W] (times *in_scale if given); Wp [32][KP] bf16; out/preact [B][Cout][H][W].
// mask (optional, same shape as out): the output is zeroed where mask <= 0.
template <int CIN>
__global__ __launch_bounds__(256) void k_conv3x3(const float* __restrict__ in, const unsigned short* __restrict__ Wp,
                                                 const float* __restrict__ bias, int Cout, float* __restrict__ out,
                                                 float* __restrict__ preact, const float* __restrict__ mask, int relu,
                                                 const float* __restrict__ in_scale, int B, int H, int W) {
    constexpr int K = CIN * 9;
    constexpr int KP = kpad(CIN);
    constexpr int ROWS = 4, TW = 32;
    __shared__ unsigned short patch[CIN][ROWS + 2][TW + 2];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + ROWS - 1) / ROWS;
    int bid = blockIdx.x;
    const int tx = bid % tiles_x;
    bid /= tiles_x;
    const int ty = bid % tiles_y;
    const int b = bid / tiles_y;
    const int x0 = tx * TW, y0 = ty * ROWS;
    const float sc = in_scale ? *in_scale : 1.0f;
    constexpr int NP = CIN * (ROWS + 2) * (TW + 2);
    unsigned short* pf = &patch[0][0][0];
    // loads in batches of 8 so that their latencies overlap, then the conversions
    for (int base = 0; base < NP; base += 8 * 256) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * 256 + threadIdx.x;
            const int c = idx / ((ROWS + 2) * (TW + 2));
            const int rem = idx % ((ROWS + 2) * (TW + 2));
            const int y = y0 + rem / (TW + 2) - 1, x = x0 + rem % (TW + 2) - 1;
            const bool in_img = idx < NP && y >= 0 && y < H && x >= 0 && x < W;
            v[u] = in_img ? in[((size_t)(b * CIN + c) * H + y) * W + x] * sc : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * 256 + threadIdx.x;
            if (idx < NP) pf[idx] = f2bf(v[u]);
        }
    }
    __syncthreads();
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    const int ai = lane & 31;          // A row (output channel) held by this lane
    const int kq = (lane >> 5) * 4;    // K offset of this lane within a step of 8
    const int j = lane & 31;           // pixel column within the tile
#pragma unroll 4
    for (int kb = 0; kb < KP / 8; ++kb) {
        const bf16x4 a = *reinterpret_cast<const bf16x4*>(Wp + (size_t)ai * KP + kb * 8 + kq);
        bf16x4 bv;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = kb * 8 + kq + r;
            unsigned short val = 0;
            if (k < K) {
                const int c = k / 9, t = k % 9;
                val = patch[c][wave + t / 3][j + t % 3];
            }
            bv[r] = (short)val;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bv, acc, 0, 0, 0);
    }
    const int x = x0 + j, y = y0 + wave;
    if (x < W && y < H) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);   // output channel of acc[r]
            if (i < Cout) {
                const size_t o = ((size_t)(b * Cout + i) * H + y) * W + x;
                float v = acc[r] + (bias ? bias[i] : 0.f);
                if (preact) preact[o] = v;
                if (mask && !(mask[o] > 0.f)) v = 0.f;
                if (relu) v = fmaxf(v, 0.f);
                out[o] = v;
            }
        }
    }
}

// Weight and bias gradients as one GEMM on MFMA: G[o][k] = sum_p gy[o][p] X[p][k] over every pixel
// p of the batch, with X[p][k] = x[c][p + off_t] for k = c*9 + t < Cin*9 and X[p][Cin*9] = 1 (so
// G[o][Cin*9] is the bias gradient); BF16 operands, FP32 accumulation, as in the forward.  Block
// (tile, group) takes one tile of 256 pixels of one sample (WG_ROWS x WG_TW, or 16 x 16 when W <= 16),
// stages the tile's input with its halo and the output gradient in LDS as BF16, and its wave w
// accumulates the 32-column tile kt = 4 group + w of G over the tile's pixels, 8 at a time.  Each
// block writes its 32 x 32 sums to part[tile][32][NKT*32]; k_wgrad_reduce adds the tiles in order.
// The staging loads are issued in batches of 8 so that their latencies overlap.
constexpr int WG_ROWS = 8, WG_TW = 32, WG_MAXCIN = 32;

__host__ __device__ constexpr int wgrad_ktiles(int cin) { return (cin * 9 + 1 + 31) / 32; }
__host__ __device__ constexpr int wgrad_tw(int W) { return W <= 16 ? 16 : WG_TW; }
__host__ __device__ inline int wgrad_tiles(int B, int H, int W) {
    const int tw = wgrad_tw(W), rows = 256 / tw;
    return B * ((H + rows - 1) / rows) * ((W + tw - 1) / tw);
}

__global__ __launch_bounds__(256) void k_conv3x3_wgrad(const float* __restrict__ x, const float* __restrict__ gy,
                                                       float* __restrict__ part, int B, int Cin, int Cout, int H,
                                                       int W) {
    __shared__ unsigned short xs[WG_MAXCIN * (WG_ROWS + 2) * (WG_TW + 2)];
    __shared__ __align__(16) unsigned short gs[32 * 256];
    const int TW = wgrad_tw(W), ROWS = 256 / TW, PW = TW + 2, PH = ROWS + 2;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int NKT = wgrad_ktiles(Cin), K = Cin * 9;
    const int kt = blockIdx.y * 4 + wave;
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + ROWS - 1) / ROWS;
    const int tile = blockIdx.x;
    const int tx = tile % tiles_x, ty = (tile / tiles_x) % tiles_y, b = tile / (tiles_x * tiles_y);
    const int x0 = tx * TW, y0 = ty * ROWS;
    const int NX = Cin * PH * PW, NG = 32 * 256;
    for (int base = 0; base < NX; base += 8 * 256) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * 256 + threadIdx.x;
            const int c = idx / (PH * PW), rem = idx % (PH * PW);
            const int yy = y0 + rem / PW - 1, xx = x0 + rem % PW - 1;
            const bool in = idx < NX && yy >= 0 && yy < H && xx >= 0 && xx < W;
            v[u] = in ? x[((size_t)(b * Cin + c) * H + yy) * W + xx] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * 256 + threadIdx.x;
            if (idx < NX) xs[idx] = f2bf(v[u]);
        }
    }
#pragma unroll
    for (int base = 0; base < NG; base += 8 * 256) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * 256 + threadIdx.x;
            const int o = idx / 256, pr = idx % 256;
            const int yy = y0 + pr / TW, xx = x0 + pr % TW;
            v[u] = (o < Cout && yy < H && xx < W) ? gy[((size_t)(b * Cout + o) * H + yy) * W + xx] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) gs[base + u * 256 + threadIdx.x] = f2bf(v[u]);
    }
    __syncthreads();
    if (kt >= NKT) return;
    const int h = lane >> 5, li = lane & 31;
    // this lane's column of X: an input tap (read from xs), the bias's ones, or zero padding
    const int kcol = kt * 32 + li;
    const int kind = kcol < K ? 0 : (kcol == K ? 1 : 2);
    const int xoff = kcol < K ? (kcol / 9) * PH * PW + ((kcol % 9) / 3) * PW + (kcol % 9) % 3 : 0;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    const int spr = TW / 8;   // pixel steps per row
#pragma unroll 4
    for (int step = 0; step < 32; ++step) {
        const int row = step / spr, cg = (step % spr) * 8 + 4 * h;
        const bf16x4 a = *reinterpret_cast<const bf16x4*>(gs + li * 256 + row * TW + cg);
        bf16x4 bv;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            bv[r] = kind == 0 ? (short)xs[xoff + row * PW + cg + r] : (kind == 1 ? (short)0x3f80 : (short)0);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bv, acc, 0, 0, 0);
    }
    const int KT32 = NKT * 32;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = 8 * (r >> 2) + 4 * h + (r & 3);
        part[((size_t)tile * 32 + i) * KT32 + kt * 32 + li] = acc[r];
    }
}

// gW[o][k] = sum over tiles of part[tile][o][k] (k < Cin*9, the layout of W[o][c][t]); gb[o] from
// the ones column k = Cin*9.  Eight independent loads per step, added in tile order.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ part, int ntiles, int Cin, int Cout,
                                                      float* __restrict__ gW, float* __restrict__ gb) {
    const int K = Cin * 9, KT32 = wgrad_ktiles(Cin) * 32;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= Cout * (K + 1)) return;
    const int o = idx / (K + 1), k = idx % (K + 1);
    const float* p = part + (size_t)o * KT32 + k;
    const size_t st = (size_t)32 * KT32;
    float s = 0.f;
    int g = 0;
    for (; g + 8 <= ntiles; g += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(size_t)(g + u) * st];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; g < ntiles; ++g) s += p[(size_t)g * st];
    if (k < K) gW[(size_t)o * K + k] = s;
    else if (gb) gb[o] = s;
}

// diff = y - t; gout = 2 w_b diff / B; lossb[b] = w_b ||diff||^2 / B.  One block per sample.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, const float* __restrict__ t,
                                              const float* __restrict__ w, float* __restrict__ gout,
                                              double* __restrict__ lossb, int per, int B) {
    __shared__ double sh[4];
    const int b = blockIdx.x;
    const float wb = w[b];
    double s = 0.0;
    for (int i = threadIdx.x; i < per; i += 256) {
        const size_t o = (size_t)b * per + i;
        const float d = y[o] - t[o];
        s += (double)d * d;
        gout[o] = 2.f * wb * d / (float)B;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) lossb[b] = (double)wb * (sh[0] + sh[1] + sh[2] + sh[3]) / B;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       size_t n, float lr, float b1, float b2, float c1, float c2, float eps) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Forward pack: Wf[i][k] = W[i][c][t] (k = c*9 + t) for i < Cout, zero elsewhere (32 x KP(Cin)).
// Backward pack: Wb[c][k'] = W[o][c][8 - t] (k' = o*9 + t) for c < Cin (32 x KP(Cout)).
__global__ void k_pack(const float* __restrict__ W, int Cin, int Cout, unsigned short* __restrict__ Wf,
                       unsigned short* __restrict__ Wb) {
    const int KPf = kpad(Cin), KPb = kpad(Cout);
    const int n1 = 32 * KPf, n2 = 32 * KPb;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n1 + n2; idx += gridDim.x * blockDim.x) {
        if (idx < n1) {
            const int i = idx / KPf, k = idx % KPf;
            float v = 0.f;
            if (i < Cout && k < Cin * 9) v = W[((size_t)i * Cin + k / 9) * 9 + k % 9];
            Wf[idx] = f2bf(v);
        } else if (Wb) {
            const int q = idx - n1;
            const int cc = q / KPb, k = q % KPb;
            float v = 0.f;
            if (cc < Cin && k < Cout * 9) {
                const int o = k / 9, t = k % 9;
                v = W[((size_t)o * Cin + cc) * 9 + (8 - t)];
            }
            Wb[q] = f2bf(v);
        }
    }
}

// ------------------------------------------------------------------ training data ------------
// dst[i][k] = src[idx[i]][k] (grid-stride over count * row_len).
__global__ __launch_bounds__(256) void k_gather_rows(const float* __restrict__ src, long long row_len,
                                                     const int* __restrict__ idx, long long total,
                                                     float* __restrict__ dst) {
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long long)gridDim.x * 256) {
        const long long i = t / row_len, k = t % row_len;
        dst[t] = src[(long long)idx[i] * row_len + k];
    }
}

// Bilinear upsampling at cell centres (source coordinate (d + 1/2) in/out - 1/2, clamped at 0;
// the upper neighbour clamped to the last cell), one fine cell per thread (grid-stride).
__global__ __launch_bounds__(256) void k_upsample_bilinear(const double* __restrict__ cz, int hc, int wc, int ny,
                                                           int nx, long long total, double* __restrict__ fine) {
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long long)gridDim.x * 256) {
        const int x = (int)(t % nx);
        const int y = (int)((t / nx) % ny);
        const long long plane = t / ((long long)nx * ny);
        const double sy = fmax(((double)y + 0.5) * hc / ny - 0.5, 0.0);
        const double sx = fmax(((double)x + 0.5) * wc / nx - 0.5, 0.0);
        const int y0 = min((int)sy, hc - 1), x0 = min((int)sx, wc - 1);
        const int y1 = min(y0 + 1, hc - 1), x1 = min(x0 + 1, wc - 1);
        const double ay = sy - y0, ax = sx - x0;
        const double* p = cz + plane * hc * wc;
        const double top = (1.0 - ax) * p[y0 * wc + x0] + ax * p[y0 * wc + x1];
        const double bot = (1.0 - ax) * p[y1 * wc + x0] + ax * p[y1 * wc + x1];
        fine[t] = (1.0 - ay) * top + ay * bot;
    }
}

// ------------------------------------------------------------------ coarse grid helpers ------
// out[c][I][J] = mean over the F x F block of (a - b - d) (b, d optional), FP64 in, FP32 out.
// One block per (chunk of CW columns, coarse row I, channel c), CW a multiple of F: the 256 threads
// split into 256 / CW row groups, each summing its rows of the block's F fine rows for one column
// (coalesced along x), then the F x F sums of the chunk's coarse cells are formed from LDS in a
// fixed order.
__host__ __device__ constexpr int pool_chunk(int F) { return F <= 64 ? F * (64 / F) : F; }

__global__ __launch_bounds__(256) void k_pool(const double* __restrict__ a, const double* __restrict__ bsub,
                                              const double* __restrict__ dsub, float* __restrict__ out, int C, int ny,
                                              int nx, int F) {
    __shared__ double part[256];
    const int CW = pool_chunk(F);
    const int NRG = 256 / CW;
    const int Hc = ny / F, Wc = nx / F;
    const int x0 = blockIdx.x * CW, I = blockIdx.y, c = blockIdx.z;
    const int ncols = min(CW, nx - x0);
    const int rg = threadIdx.x / CW, col = threadIdx.x % CW;
    double s = 0.0;
    if (rg < NRG && col < ncols) {
        const size_t base = ((size_t)c * ny + (size_t)I * F) * nx + x0 + col;
        for (int u = rg; u < F; u += NRG) {
            const size_t o = base + (size_t)u * nx;
            double val = a[o];
            if (bsub) val -= bsub[o];
            if (dsub) val -= dsub[o];
            s += val;
        }
    }
    part[threadIdx.x] = s;
    __syncthreads();
    const int ncells = ncols / F;
    for (int J = threadIdx.x; J < ncells; J += 256) {
        double t = 0.0;
        for (int g = 0; g < NRG; ++g)
            for (int q = 0; q < F; ++q) t += part[g * CW + J * F + q];
        out[((size_t)c * Hc + I) * Wc + x0 / F + J] = (float)(t / ((double)F * F));
    }
}

// One block per (channel, coarse row): column sums over the F fine rows, then F-wide groups into
// coarse cells; also the block's sum of v^2 for the RMS (partial[blockIdx], fixed order later).
__global__ __launch_bounds__(256) void k_pool_norm(const double* __restrict__ v, float* __restrict__ out,
                                                   double* __restrict__ partial, int ny, int nx, int F) {
    __shared__ double colsum[512];
    __shared__ double sh[4];
    const int Hc = ny / F, Wc = nx / F;
    const int c = blockIdx.x / Hc, I = blockIdx.x % Hc;
    double sq = 0.0;
    for (int x = threadIdx.x; x < nx; x += 256) {
        double cs = 0.0;
#pragma unroll 8
        for (int u = 0; u < F; ++u) {
            const double val = v[((size_t)c * ny + I * F + u) * nx + x];
            cs += val;
            sq += val * val;
        }
        colsum[x] = cs;
    }
    __syncthreads();
    for (int J = threadIdx.x; J < Wc; J += 256) {
        double t = 0.0;
        for (int q = 0; q < F; ++q) t += colsum[J * F + q];
        out[((size_t)c * Hc + I) * Wc + J] = (float)(t / ((double)F * F));
    }
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_down(sq, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Single block: n2 = sum of the np partials in a fixed order; st = [s, 1/s], s = sqrt(n2 / n).
__global__ __launch_bounds__(256) void k_scale_from_partials(const double* __restrict__ partial, int np, double n,
                                                             float* __restrict__ st) {
    __shared__ double sh[4];
    double t = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) t += partial[i];
    for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double r = sqrt((sh[0] + sh[1] + sh[2] + sh[3]) / n);
        st[0] = (float)r;
        st[1] = r > 0.0 ? (float)(1.0 / r) : 0.f;
    }
}

// The whole network in one workgroup for a small coarse grid (Hc <= 32 rows, Wc <= 32).  The MFMA's 32
// columns hold whole coarse rows (one row of up to 32 pixels, two of up to 16, ...).
// Activations stay in LDS as BF16, channel-innermost ([pixel][channel], pixel stride NET_PS shorts,
// zero halo and zero padded channels), so that for one 3x3 tap the eight consecutive K values a
// lane feeds to the MFMA are one 16-byte LDS read.  The reduction index is tap-major,
// k = t * CP + c (CP: input channels rounded up to 8, so a K step never straddles taps).
// Every layer's weights are loaded into LDS up front (tap-major rows of stride KS, prepacked by
// k_pack_tapmajor), so the only global reads are that copy, the input and the biases.  One wave per
// group of coarse rows; the last layer writes FP32 [c][y][x] to global memory.
constexpr int NET_THREADS = 1024;
constexpr int NET_PS = 40;                  // pixel stride in shorts: 32 channels + 8 (16-byte aligned, bank spread)
__host__ __device__ constexpr int net_cp(int c) { return (c + 7) / 8 * 8; }
__host__ __device__ constexpr int net_ks(int cin) { return 9 * net_cp(cin) + 8; }   // weight row stride

// dst[i][k] (row stride KS) = weight of output i, tap t = k / CP, input channel c = k % CP, taken
// from the forward pack (k' = c*9 + t, stride KG); zero for padded channels and the row tail.
__global__ void k_pack_tapmajor(const unsigned short* __restrict__ wf, int cin, unsigned short* __restrict__ dst) {
    const int CP = net_cp(cin), KS = net_ks(cin), KG = kpad(cin);
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < 32 * KS; idx += gridDim.x * blockDim.x) {
        const int i = idx / KS, k = idx % KS;
        unsigned short v = 0;
        if (k < 9 * CP) {
            const int t = k / CP, c = k % CP;
            if (c < cin) v = wf[(size_t)i * KG + c * 9 + t];
        }
        dst[idx] = v;
    }
}

// One output row y of a layer: D[32 out][32 columns] = W[32][9 CP] x B[9 CP][32] on MFMA, the
// reduction walked tap by tap (t = 3 dy + dx) and, within a tap, 16 channels per MFMA (8 for a
// remainder), so every LDS address is a base plus an immediate offset.  Lanes past the row edge read a valid pixel
// (their outputs are discarded).
template <int CP>
__device__ __forceinline__ f32x16 net_row(const unsigned short* __restrict__ Wl, const unsigned short* __restrict__ src,
                                          int pix, int j, int hi, int Wc) {
    // K steps of 16 on v_mfma_f32_32x32x16_bf16 (lane l holds k = 8 (l / 32) .. +7 of row / column
    // l % 32), and for CP = 8 (mod 16) one last step of 8 on the 32x32x8 form (k = 4 (l / 32) .. +3).
    // pix: the halo-grid index of the pixel whose 3x3 neighbourhood starts this lane's column.
    // Two accumulators take alternate steps, so that two independent MFMA chains are in flight.
    constexpr int KS = net_ks(CP);
    constexpr int NCB = CP / 16 + (CP % 16 != 0 ? 1 : 0);   // MFMA steps per tap
    f32x16 acc[2];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        acc[0][r] = 0.f;
        acc[1][r] = 0.f;
    }
    const unsigned short* arow = Wl + j * KS;
    const unsigned short* brow = src + (size_t)pix * NET_PS;
#pragma unroll 1
    for (int dy = 0; dy < 3; ++dy) {
        const unsigned short* bd = brow + dy * (Wc + 2) * NET_PS;
        const unsigned short* ad = arow + 3 * dy * CP;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const unsigned short* at = ad + dx * CP;
            const unsigned short* bt = bd + dx * NET_PS;
#pragma unroll
            for (int cb = 0; cb < CP / 16; ++cb) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(at + cb * 16 + 8 * hi);
                const bf16x8 bv = *reinterpret_cast<const bf16x8*>(bt + cb * 16 + 8 * hi);
                f32x16& c = acc[(dx * NCB + cb) & 1];
                c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv, c, 0, 0, 0);
            }
            if constexpr (CP % 16 != 0) {
                const bf16x4 a = *reinterpret_cast<const bf16x4*>(at + (CP / 16) * 16 + 4 * hi);
                const bf16x4 bv = *reinterpret_cast<const bf16x4*>(bt + (CP / 16) * 16 + 4 * hi);
                f32x16& c = acc[(dx * NCB + CP / 16) & 1];
                c = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bv, c, 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[0][r] += acc[1][r];
    return acc[0];
}

template <int HID>
__device__ __forceinline__ void net_fused_block(const float* __restrict__ in, const float* __restrict__ in_scale,
                                                const unsigned short* __restrict__ wn, int nwn,
                                                const float* __restrict__ bias_all, int nbias,
                                                const int* __restrict__ meta, int layers, int C, int Hc, int Wc,
                                                float* __restrict__ out, float in_mul) {
    // in_mul: an extra factor on the input (with *in_scale).
    // meta: per layer [cin, cout, tap-major pack offset, bias offset into bias_all]; nwn: pack length
    // (multiple of 8 shorts); all of it is staged in LDS first, with every global load of the
    // prologue in flight together (the kernel is latency-bound: one workgroup).
    static_assert(HID <= 32 && NET_PS >= 32 + 8 && NET_PS % 8 == 0, "pixel stride");
    extern __shared__ __attribute__((aligned(16))) unsigned short lds[];
    __shared__ int smeta[4 * 8];
    __shared__ float sbias[8 * 32];
    const int P = (Hc + 2) * (Wc + 2);
    unsigned short* const act0 = lds;
    unsigned short* const act1 = lds + (size_t)P * NET_PS;
    unsigned short* Wall = lds + (size_t)2 * P * NET_PS;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    {
        const uint4* ws = reinterpret_cast<const uint4*>(wn);
        uint4* wd = reinterpret_cast<uint4*>(Wall);
        const int nw4 = nwn / 8;
        constexpr int U = 8;
        const uint4 zero4 = {0u, 0u, 0u, 0u};
        for (int base = 0; base < nw4; base += U * NET_THREADS) {
            uint4 r[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = base + tid + u * NET_THREADS;
                r[u] = idx < nw4 ? ws[idx] : zero4;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = base + tid + u * NET_THREADS;
                if (idx < nw4) wd[idx] = r[u];
            }
        }
        if (tid < 4 * layers) smeta[tid] = meta[tid];
        if (tid < nbias) sbias[tid] = bias_all[tid];
        // the input: thread t takes pixel t % (Hc Wc) of channels t / (Hc Wc), t / (Hc Wc) + cstep, ...
        // (Hc Wc <= NET_THREADS), so the index arithmetic is done once; the loads are issued now,
        // with the weights still in flight
        const int HW = Hc * Wc;
        const int cstep = NET_THREADS / HW;
        const int pin = tid % HW, c0 = tid / HW;
        const bool lane_in = tid < cstep * HW;
        const int yin = pin / Wc, xin0 = pin % Wc;
        constexpr int UI = 8;   // channels per thread per batch (C <= 17; cstep >= 1)
        float xin[UI];
#pragma unroll
        for (int u = 0; u < UI; ++u) {
            const int c = c0 + u * cstep;
            xin[u] = (lane_in && c < C) ? in[(size_t)c * HW + pin] : 0.f;
        }
        uint4* az = reinterpret_cast<uint4*>(lds);
        const uint4 zero = {0u, 0u, 0u, 0u};
        for (int idx = tid; idx < 2 * P * NET_PS / 8; idx += NET_THREADS) az[idx] = zero;
        const float sc = *in_scale * in_mul;
        __syncthreads();   // the zero fill of the activations is complete
        unsigned short* const arow = act0 + ((yin + 1) * (Wc + 2) + xin0 + 1) * NET_PS;
        for (int cb = 0; cb < C; cb += UI * cstep) {
            if (cb > 0) {
#pragma unroll
                for (int u = 0; u < UI; ++u) {
                    const int c = c0 + cb + u * cstep;
                    xin[u] = (lane_in && c < C) ? in[(size_t)c * HW + pin] : 0.f;
                }
            }
#pragma unroll
            for (int u = 0; u < UI; ++u) {
                const int c = c0 + cb + u * cstep;
                if (lane_in && c < C) arow[c] = f2bf(xin[u] * sc);
            }
        }
    }
    __syncthreads();
    // The 32 MFMA columns take RPM = 32 / PR coarse rows of PR = (Wc rounded up to a power of two)
    // pixels each: lane column j is pixel px = j % PR of row y0 + j / PR.  Columns past the grid
    // read a valid pixel and their outputs are dropped.
    const int j = lane & 31, hi = lane >> 5;
    int PR = 1;
    while (PR < Wc) PR <<= 1;
    const int RPM = 32 / PR;
    const int px = j % PR, ry = j / PR;
    for (int l = 0; l < layers; ++l) {
        const int cin = smeta[4 * l], cout = smeta[4 * l + 1];
        const unsigned short* Wl = Wall + smeta[4 * l + 2];
        const float* bias = sbias + smeta[4 * l + 3];
        const bool last = l == layers - 1;
        const int CP = net_cp(cin);
        const unsigned short* src = (l & 1) ? act1 : act0;
        unsigned short* dst = (l & 1) ? act0 : act1;
        for (int y0 = wave * RPM; y0 < Hc; y0 += (NET_THREADS / 64) * RPM) {
            const int y = y0 + ry;
            const bool valid = px < Wc && y < Hc;
            const int pin = (y < Hc ? y : Hc - 1) * (Wc + 2) + (px < Wc ? px : Wc - 1);
            f32x16 acc;
            if (CP == 32) acc = net_row<32>(Wl, src, pin, j, hi, Wc);
            else if (CP == 24) acc = net_row<24>(Wl, src, pin, j, hi, Wc);
            else if (CP == 16) acc = net_row<16>(Wl, src, pin, j, hi, Wc);
            else acc = net_row<8>(Wl, src, pin, j, hi, Wc);
            if (valid) {
                const int pix = (y + 1) * (Wc + 2) + px + 1;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int i0 = 8 * g + 4 * hi;
                    if (last) {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (i0 + r < cout) out[((size_t)(i0 + r) * Hc + y) * Wc + px] = acc[4 * g + r] + bias[i0 + r];
                    } else if (i0 < cout) {
                        bf16x4 o;
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            o[r] = (short)(i0 + r < cout ? f2bf(fmaxf(acc[4 * g + r] + bias[i0 + r], 0.f)) : 0);
                        *reinterpret_cast<bf16x4*>(dst + pix * NET_PS + i0) = o;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// The whole network as a kernel of its own: one workgroup of NET_THREADS threads.
template <int HID>
__global__ __launch_bounds__(NET_THREADS) void k_net_fused(const float* __restrict__ in, const float* __restrict__ in_scale,
                                                           const unsigned short* __restrict__ wn, int nwn,
                                                           const float* __restrict__ bias_all, int nbias,
                                                           const int* __restrict__ meta, int layers, int C, int Hc,
                                                           int Wc, float* __restrict__ out) {
    net_fused_block<HID>(in, in_scale, wn, nwn, bias_all, nbias, meta, layers, C, Hc, Wc, out, 1.0f);
}

// st[0] = s = sqrt(norm2 / n), st[1] = 1/s (0 if s == 0).
__global__ void k_scale_from_norm2(const double* __restrict__ norm2, double n, float* __restrict__ st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double r = sqrt(norm2[0] / n);
        st[0] = (float)r;
        st[1] = r > 0.0 ? (float)(1.0 / r) : 0.f;
    }
}

// z = v + s * (P y): P is bilinear interpolation from the coarse cell centres (coarse cell I
// spans fine cells I*F .. I*F+F-1), clamped to the outer coarse centres.
__device__ __forceinline__ void lerp_index(int i, int F, int nc, int& lo, int& hi, float& a) {
    const float xi = ((float)i + 0.5f) / (float)F - 0.5f;
    const float f0 = floorf(xi);
    a = xi - f0;
    const int i0 = (int)f0;
    lo = min(max(i0, 0), nc - 1);
    hi = min(max(i0 + 1, 0), nc - 1);
}

// One block row per fine row (blockIdx.y = c * ny + y), threads along x.
__global__ __launch_bounds__(256) void k_prolong_add(const double* __restrict__ v, const float* __restrict__ y,
                                                     const float* __restrict__ st, double* __restrict__ z, int C, int ny,
                                                     int nx, int F) {
    const int xx = blockIdx.x * 256 + threadIdx.x;
    if (xx >= nx) return;
    const int c = blockIdx.y / ny, yy = blockIdx.y % ny;
    const int Hc = ny / F, Wc = nx / F;
    const double s = st[0];
    int y0, y1, x0, x1;
    float ay, ax;
    lerp_index(yy, F, Hc, y0, y1, ay);
    lerp_index(xx, F, Wc, x0, x1, ax);
    const float* yc = y + (size_t)c * Hc * Wc;
    const float top = (1.f - ax) * yc[y0 * Wc + x0] + ax * yc[y0 * Wc + x1];
    const float bot = (1.f - ax) * yc[y1 * Wc + x0] + ax * yc[y1 * Wc + x1];
    const size_t i = (size_t)blockIdx.y * nx + xx;
    z[i] = v[i] + s * (double)((1.f - ay) * top + ay * bot);
}

// The flexible-GMRES solution update in one pass over x: x += sum_{v < nvec} V[v] y[v], then
// + s P comb (comb: the coarse combination sum_j y_j Y_j; s = st[0]), in the order and with the
// prolongation of k_combine followed by k_prolong_add.  One block row per fine row (blockIdx.y =
// c * ny + row), threads along x.  Nothing when skip is given and skip[2] (the device's
// non-finite flag) is set.
template <typename TV>
__global__ __launch_bounds__(256) void k_combine_prolong(double* __restrict__ x, const TV* __restrict__ V, size_t ld,
                                                        int nvec, const double* __restrict__ y,
                                                        const float* __restrict__ comb,
                                                        const float* __restrict__ st, int ny, int nx, int F,
                                                        const int* __restrict__ skip) {
    __shared__ double ys[RTE_KRYLOV_MAXVEC];
    if (skip && skip[2] != 0) return;
    for (int v = threadIdx.x; v < nvec; v += 256) ys[v] = y[v];
    __syncthreads();
    const int xx = blockIdx.x * 256 + threadIdx.x;
    if (xx >= nx) return;
    const int c = blockIdx.y / ny, yy = blockIdx.y % ny;
    const int Hc = ny / F, Wc = nx / F;
    int y0, y1, x0, x1;
    float ay, ax;
    lerp_index(yy, F, Hc, y0, y1, ay);
    lerp_index(xx, F, Wc, x0, x1, ax);
    const float* yc = comb + (size_t)c * Hc * Wc;
    const float top = (1.f - ax) * yc[y0 * Wc + x0] + ax * yc[y0 * Wc + x1];
    const float bot = (1.f - ax) * yc[y1 * Wc + x0] + ax * yc[y1 * Wc + x1];
    const size_t i = (size_t)blockIdx.y * nx + xx;
    double t = x[i];
#pragma unroll 8
    for (int v = 0; v < nvec; ++v) t += (double)V[(size_t)v * ld + i] * ys[v];
    const double s = st[0];
    x[i] = t + s * (double)((1.f - ay) * top + ay * bot);
}

// Block means of one block's columns into coarse[c][I][J]: part[] holds each thread's column sum
// over its rows (CW columns x RG row groups).  One wave per coarse cell sums its RG x F column
// partials in a fixed order (strided lanes, then a shuffle reduction).
__device__ __forceinline__ void pool_block_cells(const double* part, int CW, int RG, int F, int chunk, int c, int I,
                                                 int Hc, int Wc, float* __restrict__ coarse) {
    const int ncell = CW / F;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int q = wave; q < ncell; q += 4) {
        const int J = chunk * ncell + q;
        double t = 0.0;
        for (int e = lane; e < RG * F; e += 64) t += part[(e / F) * CW + q * F + (e % F)];
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
        if (lane == 0 && J < Wc) coarse[((size_t)c * Hc + I) * Wc + J] = (float)(t / ((double)F * F));
    }
}

// v = a w (in place allowed) and the F x F block means of v into coarse[c][I][J] (FP32).  Work
// unit: (channel, coarse row I, chunk of CW = max(F, 64) columns), so that a unit owns its coarse
// cells; 256 threads = CW columns x (256 / CW) row groups.  The grid strides over the units.
template <typename TW, typename TV>
__device__ __forceinline__ void scale_pool_units(const TW* __restrict__ w, TV* __restrict__ v, double a,
                                                 float* __restrict__ coarse, int C, int ny, int nx, int F) {
    __shared__ double part[256];
    const int CW = F > 64 ? F : 64;
    const int RG = 256 / CW;                       // row groups
    const int nchunk = (nx + CW - 1) / CW;
    const int Hc = ny / F, Wc = nx / F;
    const int nunit = C * Hc * nchunk;
    const int col = threadIdx.x % CW, rg = threadIdx.x / CW;
    const int rows = (F + RG - 1) / RG;
    for (int unit = blockIdx.x; unit < nunit; unit += gridDim.x) {
        const int chunk = unit % nchunk;
        const int I = (unit / nchunk) % Hc;
        const int c = unit / (nchunk * Hc);
        const int x = chunk * CW + col;
        double s = 0.0;
        if (x < nx) {
#pragma unroll 8
            for (int u = 0; u < rows; ++u) {
                const int r = rg * rows + u;
                if (r < F) {
                    const size_t o = ((size_t)c * ny + I * F + r) * nx + x;
                    const TV val = (TV)(a * (double)w[o]);   // the block means are of the stored values
                    v[o] = val;
                    s += (double)val;
                }
            }
        }
        part[threadIdx.x] = s;
        __syncthreads();
        pool_block_cells(part, CW, RG, F, chunk, c, I, Hc, Wc, coarse);
        __syncthreads();   // part is reused by the next unit
    }
}

// v = a w and its block means (scale_pool_units), a = *a_dev or a_host when a_dev is NULL.  With g
// given, block 0 also sets g = (g0, 0, ..., 0) (gn entries) and flags[0..nflags) = 0, the start
// of a restart cycle.
template <typename TW, typename TV>
__global__ __launch_bounds__(256) void k_scale_pool(const TW* __restrict__ w, TV* __restrict__ v,
                                                    const double* __restrict__ a_dev, double a_host,
                                                    float* __restrict__ coarse, int C, int ny, int nx, int F,
                                                    double* __restrict__ g, int gn, double g0,
                                                    int* __restrict__ flags, int nflags) {
    if (g && blockIdx.x == 0) {
        for (int i = threadIdx.x; i < gn; i += blockDim.x) g[i] = i == 0 ? g0 : 0.0;
        for (int i = threadIdx.x; i < nflags; i += blockDim.x) flags[i] = 0;
    }
    scale_pool_units(w, v, a_dev ? *a_dev : a_host, coarse, C, ny, nx, F);
}

// Stage 1 of the fused single pass (block 0: the Arnoldi column's bookkeeping) and, when the
// stored vector needs it, its rescale with the block means taken again.
template <typename TV>
__global__ __launch_bounds__(256) void k_rescale_pool_arn1(ArnoldiArgs t, TV* __restrict__ w,
                                                           float* __restrict__ coarse, int C, int ny, int nx, int F,
                                                           const double* __restrict__ partial, int nblk) {
    const double inv = arnoldi_stage1_in_rescale(t, partial, nblk);
    if (inv < 0.0) return;
    scale_pool_units(w, w, inv, coarse, C, ny, nx, F);
}

// Stage 1 of the fused single pass and the next step's network in one launch: block 1 runs the
// whole network (net_fused_block) on the block means the update just wrote; every other block
// takes part in stage 1 (block 0: the column's bookkeeping) and, when the device finds the stored
// vector's norm off, in w's rescale.  The rescale does not pool again: block 1 takes the same
// decision from the same partial sums and puts the rescale factor on the network's input instead
// (the block means are linear in w), so the network sees the block means of the final vector.
template <int HID, typename TV>
__global__ __launch_bounds__(NET_THREADS) void k_rescale_net(ArnoldiArgs t, TV* __restrict__ w, size_t n,
                                                             const double* __restrict__ partial, int nblk,
                                                             const float* __restrict__ in,
                                                             const float* __restrict__ in_scale,
                                                             const unsigned short* __restrict__ wn, int nwn,
                                                             const float* __restrict__ bias_all, int nbias,
                                                             const int* __restrict__ meta, int layers, int C, int Hc,
                                                             int Wc, float* __restrict__ out) {
    const double inv = arnoldi_stage1_in_rescale(t, partial, nblk);   // bookkeeping in block 0 only
    if (blockIdx.x == 1) {
        net_fused_block<HID>(in, in_scale, wn, nwn, bias_all, nbias, meta, layers, C, Hc, Wc, out,
                             inv < 0.0 ? 1.0f : (float)inv);
        return;
    }
    if (inv < 0.0) return;
    const size_t wb = blockIdx.x == 0 ? 0 : blockIdx.x - 1, nwb = gridDim.x - 1;
    const size_t stride = nwb * NET_THREADS;
    for (size_t i = wb * NET_THREADS + threadIdx.x; i < n; i += stride) w[i] = (TV)((double)w[i] * inv);
}

// k_rescale_net with the next apply's pass A beside the network.  The next Krylov vector's
// preconditioned form z = v + s P Y needs Y, the network's output, but the x-transform is linear:
// the blocks other than 0 (the column's bookkeeping) and 1 (the network) transform v alone, and
// pass B adds the x-spectrum of the correction (CorrB).  Those blocks take row tiles of PA_TR rows,
// one per 256-thread quarter, in a loop that every block runs the same number of times (a tile
// past the end loads only in-range addresses and stores nothing).  When the device finds the
// stored vector's norm off, each quarter folds the factor into pass A's scale and then rescales
// its own tile's rows, after the barrier that ends the tile, so no other thread still reads them.
constexpr int PA_TR = 4;
constexpr int PA_NQ = NET_THREADS / 256;
struct PassAJob {
    const cx<float>* twx;   // x twiddles of the FP32 apply
    cx<float>* work;        // its work buffer [C][NKS][ny]
    ChanScale sc;           // pass A's per-channel factors (operator A)
    int nx, ny, C, pack;
};
template <int PX>
constexpr size_t pass_a_job_lds() {
    return (size_t)(PX + PA_NQ * (PA_TR / 2) * (padded(PX) + 1)) * sizeof(cx<float>);
}
// ST1 false: the first step of a cycle, with no Arnoldi column to finish: the network of v_0's
// block means beside pass A of v_0, no rescale.
template <int HID, typename TV, int PX, bool ST1>
__global__ __launch_bounds__(NET_THREADS) void k_rescale_net_pa(ArnoldiArgs t, TV* __restrict__ w,
                                                                const double* __restrict__ partial, int nblk,
                                                                const float* __restrict__ in,
                                                                const float* __restrict__ in_scale,
                                                                const unsigned short* __restrict__ wn, int nwn,
                                                                const float* __restrict__ bias_all, int nbias,
                                                                const int* __restrict__ meta, int layers, int C,
                                                                int Hc, int Wc, float* __restrict__ out, PassAJob pj) {
    double inv = -1.0;
    if constexpr (ST1) inv = arnoldi_stage1_in_rescale(t, partial, nblk);   // bookkeeping in block 0 only
    if (blockIdx.x == 1) {
        net_fused_block<HID>(in, in_scale, wn, nwn, bias_all, nbias, meta, layers, C, Hc, Wc, out,
                             inv < 0.0 ? 1.0f : (float)inv);
        return;
    }
    if (blockIdx.x == 0) return;
    constexpr int LD = padded(PX) + 1;
    extern __shared__ __attribute__((aligned(16))) unsigned short lds[];
    cx<float>* tws = reinterpret_cast<cx<float>*>(lds);
    const int q = threadIdx.x >> 8, ltid = threadIdx.x & 255;
    cx<float>* buf = tws + PX + q * (PA_TR / 2) * LD;
    stage_twiddles<float, PX, NET_THREADS>(tws, pj.twx, threadIdx.x);
    const int nx = pj.nx, ny = pj.ny;
    const int NKS = pj.pack ? PX / 2 : PX / 2 + 1;
    const int ntr = (ny + PA_TR - 1) / PA_TR;
    const int ntiles = pj.C * ntr;
    const int G = gridDim.x - 2, b = blockIdx.x - 2;
    const int rounds = (ntiles + PA_NQ * G - 1) / (PA_NQ * G);
    const double f = inv < 0.0 ? 1.0 : inv;
    for (int k = 0; k < rounds; ++k) {
        const int tile = (k * G + b) * PA_NQ + q;
        const bool live = tile < ntiles;
        const int bc = live ? tile / ntr : 0;
        const int y0 = live ? (tile % ntr) * PA_TR : ny;
        pass_a_tile<float, PX, PA_TR, 256, TV, false>(w + (size_t)bc * ny * nx, pj.work + (size_t)bc * NKS * ny, nx,
                                                       ny, pj.sc.s[bc] * f, pj.pack, y0, buf, tws, ltid);
        __syncthreads();   // this tile's LDS reads end before the next tile's writes
        if (inv >= 0.0 && live) {
            TV* wr = w + (size_t)bc * ny * nx + (size_t)y0 * nx;
            const int cnt = min(PA_TR, ny - y0) * nx;
            for (int e = ltid; e < cnt; e += 256) wr[e] = (TV)((double)wr[e] * inv);
        }
    }
}

// The single Gram-Schmidt pass of the preconditioned Arnoldi step with its normalisation and the
// network's restriction fused: w = a (w - sum_v V[v] h[v]) (h = st0.st, a computed here by
// arnoldi_stage0_in_update, block 0 also running stage 0 of the column), the F x F block means of
// the new w into coarse (as k_scale_pool), and partial_norm[blk] = sum of the new w^2 over the
// block.  Same work units as k_scale_pool, one per block (every fine cell of the grid [C][ny][nx]
// with ny, nx multiples of F belongs to exactly one block).  PAIRS (even nx and ld, 16-byte
// aligned w and V): each thread takes two adjacent columns as 16-byte loads, so a row group is
// CW / 2 threads and the block covers twice the rows per step.
template <bool PAIRS, typename TV>
__global__ __launch_bounds__(256) void k_update_pool(TV* __restrict__ w, const TV* __restrict__ V, size_t ld,
                                                     int nvec, float* __restrict__ coarse,
                                                     double* __restrict__ partial_norm, int ny, int nx, int F,
                                                     ArnoldiArgs st0) {
    __shared__ double part[512];
    __shared__ double hs[256];
    __shared__ double nsh[4];
    __shared__ double a_sh;
    const int CW = F > 64 ? F : 64;
    constexpr int PW = PAIRS ? 2 : 1;              // columns per thread
    const int TPR = CW / PW;                       // threads per row group
    const int RG = 256 / TPR;                      // row groups
    const int nchunk = (nx + CW - 1) / CW;
    const int Hc = ny / F, Wc = nx / F;
    const int chunk = blockIdx.x % nchunk;
    const int I = (blockIdx.x / nchunk) % Hc;
    const int c = blockIdx.x / (nchunk * Hc);
    for (int v = threadIdx.x; v < nvec; v += 256) hs[v] = st0.st[v];
    __syncthreads();
    arnoldi_stage0_in_update(st0, hs, &a_sh);   // the normalising factor; stage 0 in block 0
    __syncthreads();
    const double a = a_sh;
    const int col = (threadIdx.x % TPR) * PW, rg = threadIdx.x / TPR;
    const int x = chunk * CW + col;
    const int rows = (F + RG - 1) / RG;
    const int nr = rg < RG ? min(rows, F - rg * rows) : 0;   // rows of this thread's group in the cell
    double s0 = 0.0, s1 = 0.0, q = 0.0;
    if (x < nx) {
        const size_t o0 = ((size_t)c * ny + I * F + rg * rows) * nx + x;
        if constexpr (PAIRS) {
            using P2 = typename pair_of<TV>::type;
            P2* w2 = reinterpret_cast<P2*>(w);
            const P2* V2 = reinterpret_cast<const P2*>(V);
            const size_t ldp = ld / 2;
#pragma unroll 2
            for (int u = 0; u < nr; ++u) {
                const size_t op = (o0 + (size_t)u * nx) / 2;
                const P2 wl = w2[op];
                double tx = (double)wl.x, ty = (double)wl.y;
                // eight basis loads issued before their multiplies (the subtraction order is v)
                int v = 0;
                for (; v + 8 <= nvec; v += 8) {
                    P2 b[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) b[q] = V2[(size_t)(v + q) * ldp + op];
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        tx -= (double)b[q].x * hs[v + q];
                        ty -= (double)b[q].y * hs[v + q];
                    }
                }
                if (v + 4 <= nvec) {
                    P2 b[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) b[q] = V2[(size_t)(v + q) * ldp + op];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        tx -= (double)b[q].x * hs[v + q];
                        ty -= (double)b[q].y * hs[v + q];
                    }
                    v += 4;
                }
                if (v + 2 <= nvec) {
                    const P2 b0 = V2[(size_t)v * ldp + op], b1 = V2[(size_t)(v + 1) * ldp + op];
                    tx -= (double)b0.x * hs[v];
                    ty -= (double)b0.y * hs[v];
                    tx -= (double)b1.x * hs[v + 1];
                    ty -= (double)b1.y * hs[v + 1];
                    v += 2;
                }
                if (v < nvec) {
                    const P2 b = V2[(size_t)v * ldp + op];
                    tx -= (double)b.x * hs[v];
                    ty -= (double)b.y * hs[v];
                }
                P2 t;
                t.x = (TV)(tx * a);
                t.y = (TV)(ty * a);
                w2[op] = t;
                const double ux = (double)t.x, uy = (double)t.y;   // sums of the stored values
                s0 += ux;
                s1 += uy;
                q += ux * ux + uy * uy;
            }
        } else {
#pragma unroll 2
            for (int u = 0; u < nr; ++u) {
                const size_t o = o0 + (size_t)u * nx;
                double t = (double)w[o];
#pragma unroll 8
                for (int v = 0; v < nvec; ++v) t -= (double)V[(size_t)v * ld + o] * hs[v];
                const TV tq = (TV)(t * a);
                w[o] = tq;
                const double u2 = (double)tq;
                s0 += u2;
                q += u2 * u2;
            }
        }
    }
    // part[rg * CW + column] = this thread's column sums (= part[PW * threadIdx.x + k])
    part[PW * threadIdx.x] = s0;
    if (PAIRS) part[PW * threadIdx.x + 1] = s1;
    // block sum of q: waves, then thread 0 in a fixed order
    for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off, 64);
    if ((threadIdx.x & 63) == 0) nsh[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) partial_norm[blockIdx.x] = (nsh[0] + nsh[1]) + (nsh[2] + nsh[3]);
    pool_block_cells(part, CW, RG, F, chunk, c, I, Hc, Wc, coarse);
}

// out[i] = sum_{j < k} y_j Y[j][i] over one coarse vector of n entries (y FP64 on the device).
__global__ void k_coarse_combine(const float* __restrict__ Y, const double* __restrict__ y, int k, int n,
                                 float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double t = 0.0;
    for (int j = 0; j < k; ++j) t += y[j] * (double)Y[(size_t)j * n + i];
    out[i] = (float)t;
}

// Training pair normalisation (single block): s^2 = |r|^2 / n (fine grid); x = xr/s, t = xt/s,
// w = F^2 s^2 / |e|^2 (|r|^2 in r2, |e|^2 in e2, both on the device).
__global__ __launch_bounds__(256) void k_pair_finish(float* __restrict__ xr, float* __restrict__ xt, int nco,
                                                     const double* __restrict__ r2, double nfine,
                                                     const double* __restrict__ e2, float* __restrict__ w, int F) {
    const double ms = r2[0] / nfine;
    const double sc = ms > 0.0 ? 1.0 / sqrt(ms) : 0.0;
    if (threadIdx.x == 0) w[0] = (e2[0] > 0.0) ? (float)((double)F * F * ms / e2[0]) : 0.f;
    for (int i = threadIdx.x; i < nco; i += 256) {
        xr[i] = (float)(xr[i] * sc);
        xt[i] = (float)(xt[i] * sc);
    }
}

// d = a - b (FP64)
__global__ void k_sub(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ d, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        d[i] = a[i] - b[i];
}

// ------------------------------------------------------------------ host dispatch ------------
static int conv_launch(int Cin, const float* in, const unsigned short* Wp, const float* bias, int Cout, float* out,
                       float* preact, const float* mask, bool relu, const float* in_scale, int B, int H, int W,
                       hipStream_t st) {
    const int tiles = B * ((H + 3) / 4) * ((W + 31) / 32);
    dim3 g(tiles), blk(256);
    switch (Cin) {
#define RTE_CV(CI)                                                                                         \
    case CI:                                                                                               \
        hipLaunchKernelGGL((k_conv3x3<CI>), g, blk, 0, st, in, Wp, bias, Cout, out, preact, mask, relu ? 1 : 0, \
                           in_scale, B, H, W);                                                             \
        return 0;
        RTE_CV(1) RTE_CV(3) RTE_CV(5) RTE_CV(7) RTE_CV(9) RTE_CV(11) RTE_CV(13) RTE_CV(15) RTE_CV(16) RTE_CV(17)
        RTE_CV(32)
#undef RTE_CV
    }
    return -1;
}

struct NetShape {
    int C = 0, hidden = 0, layers = 0;
    std::vector<int> cin, cout;
    std::vector<size_t> woff, boff;    // offsets of W_l and b_l in the packed parameters
    size_t nparam = 0;
    size_t pf_off_total = 0, pb_off_total = 0;
    std::vector<size_t> pf_off, pb_off;  // offsets of the bf16 packs
    void init(int C_, int hidden_, int layers_) {
        C = C_; hidden = hidden_; layers = layers_;
        cin.resize(layers); cout.resize(layers); woff.resize(layers); boff.resize(layers);
        pf_off.resize(layers); pb_off.resize(layers);
        size_t off = 0, pf = 0, pb = 0;
        for (int l = 0; l < layers; ++l) {
            cin[l] = l == 0 ? C : hidden;
            cout[l] = l == layers - 1 ? C : hidden;
            woff[l] = off; off += (size_t)cout[l] * cin[l] * 9;
            boff[l] = off; off += cout[l];
            pf_off[l] = pf; pf += (size_t)32 * kpad(cin[l]);
            pb_off[l] = pb; pb += (size_t)32 * kpad(cout[l]);
        }
        nparam = off; pf_off_total = pf; pb_off_total = pb;
    }
};

// Length in shorts of the tap-major weight pack of every layer (each layer's block 16-byte aligned).
static size_t tapmajor_len(const NetShape& sh, std::vector<int>* off = nullptr) {
    size_t t = 0;
    for (int l = 0; l < sh.layers; ++l) {
        if (off) off->push_back((int)t);
        t += (size_t)32 * net_ks(sh.cin[l]);
    }
    return t;
}
// LDS of the fused network kernel: two BF16 activation grids with halo plus every layer's weights.
static size_t fused_net_lds(const NetShape& sh, int Hc, int Wc) {
    return ((size_t)2 * (Hc + 2) * (Wc + 2) * NET_PS + tapmajor_len(sh)) * 2;
}
static bool fused_net_fits(const NetShape& sh, int Hc, int Wc) {
    // dynamic LDS plus the kernel's static meta and bias arrays within the 160 KiB of a workgroup
    return Hc <= 32 && Wc <= 32 && fused_net_lds(sh, Hc, Wc) <= 156 * 1024;
}

static bool valid_net(int C, int hidden, int layers) {
    return C >= 1 && C <= 17 && (C & 1) && (hidden == 16 || hidden == 32) && layers >= 2 && layers <= 8;
}

// ------------------------------------------------------------------ allocation-free forward ---
// rte_nn_forward_noalloc keeps its intermediate activations in this device array instead of the
// object's lazily allocated buffers.  Each GPU holds its own copy until the process ends.  Host
// code never passes the array's name to a kernel: it uses the device address resolved per device
// by scratch_resolve(), which rte_nn_create calls with the new object's device current.
static __device__ __align__(256) float scratch[RTE_NN_SCRATCH_BYTES / sizeof(float)];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_dev[kMaxScratchDevices] = {};

static int scratch_resolve(int dev) {
    if (dev < 0 || dev >= kMaxScratchDevices) return set_error(RTE_EUNSUPPORTED, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[dev]) return RTE_OK;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return set_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)", __FILE__,
                             __LINE__);
    }
    g_scratch_dev[dev] = (float*)p;
    return RTE_OK;
}

static float* scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_dev[dev];
}

}  // namespace rte

struct rte_nn {
    rte::NetShape sh;
    hipStream_t stream = nullptr;
    int device = 0;                    // device current at creation (where the parameters live)
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    unsigned short *wf = nullptr, *wb = nullptr;
    int step = 0;
    bool use_bias = true;
    size_t cap = 0;                    // activation capacity in floats per tensor
    std::vector<float*> act, pre;      // act[l]: input of layer l (act[0] unused), pre[l]: pre-activation
    float *gA = nullptr, *gB = nullptr;
    float* wpart = nullptr;            // per-tile partial weight gradients (k_conv3x3_wgrad)
    size_t wpart_cap = 0;              // its capacity in floats
    double* lossb = nullptr;
    int lossb_cap = 0;
};

namespace rte {

template <typename P>
static int nalloc(P** p, size_t count) {
    *p = nullptr;
    hipError_t e = hipMalloc((void**)p, count * sizeof(P));
    if (e != hipSuccess) { *p = nullptr; (void)hipGetLastError(); return set_error(RTE_ENOMEM, "hipMalloc failed"); }
    return RTE_OK;
}
template <typename P>
static void nfree(P*& p) { if (p) (void)hipFree((void*)p); p = nullptr; }

static void pack_all(const NetShape& sh, const float* params, unsigned short* wf, unsigned short* wb, hipStream_t st) {
    for (int l = 0; l < sh.layers; ++l)
        hipLaunchKernelGGL(k_pack, dim3(64), dim3(256), 0, st, params + sh.woff[l], sh.cin[l], sh.cout[l],
                           wf + sh.pf_off[l], wb ? wb + sh.pb_off[l] : (unsigned short*)nullptr);
}

static int ensure_acts(rte_nn* nn, size_t per_tensor, int B) {
    if (per_tensor <= nn->cap && B <= nn->lossb_cap) return RTE_OK;
    for (auto& a : nn->act) nfree(a);
    for (auto& a : nn->pre) nfree(a);
    nfree(nn->gA); nfree(nn->gB); nfree(nn->lossb);
    const int L = nn->sh.layers;
    nn->act.assign(L + 1, nullptr);
    nn->pre.assign(L, nullptr);
    int rc;
    for (int l = 1; l <= L; ++l) if ((rc = nalloc(&nn->act[l], per_tensor))) return rc;
    for (int l = 0; l < L; ++l) if ((rc = nalloc(&nn->pre[l], per_tensor))) return rc;
    if ((rc = nalloc(&nn->gA, per_tensor)) || (rc = nalloc(&nn->gB, per_tensor))) return rc;
    if ((rc = nalloc(&nn->lossb, (size_t)B))) return rc;
    nn->cap = per_tensor;
    nn->lossb_cap = B;
    return RTE_OK;
}

// Forward through all layers; act[l+1] = layer l output, pre[l] = its pre-activation.
static int net_forward(const NetShape& sh, const unsigned short* wf, const float* params_bias_base,
                       const std::vector<size_t>& boff, const float* x, const float* in_scale, float* const* act,
                       float* const* pre, int B, int H, int W, hipStream_t st) {
    const float* a = x;
    for (int l = 0; l < sh.layers; ++l) {
        const bool last = l == sh.layers - 1;
        if (conv_launch(sh.cin[l], a, wf + sh.pf_off[l], params_bias_base + boff[l], sh.cout[l], act[l + 1],
                        pre ? pre[l] : nullptr, nullptr, !last, l == 0 ? in_scale : nullptr, B, H, W, st))
            return set_error(RTE_EUNSUPPORTED, "unsupported convolution width");
        a = act[l + 1];
    }
    return RTE_OK;
}

// ------------------------------------------------------------------ preconditioner on ctx -----
void pc_free(rte_ctx* c) {
    if (c->pc_w) (void)hipFree(c->pc_w);
    c->pc_w = nullptr;
    nfree(c->pc_b);
    nfree(c->pc_act0);
    nfree(c->pc_act1);
    nfree(c->pc_coarse);
    nfree(c->pc_st);
    nfree(c->pc_nrm);
    nfree(c->pc_part);
    nfree(c->pc_meta);
    nfree(c->pc_wn);
    nfree(c->pc_bn);
    c->pc_wn_len = 0;
    c->pc_nbias = 0;
    nfree(c->pc_Y);
    c->pc_slots = 0;
    nfree(c->pc_phi);
    c->pc_phi_pack = -1;
    nfree(c->pc_coef);
    for (float& v : c->pc_coef_host) v = 0.f;
    c->pc_attached = false;
}

// The network on the coarse input c->pc_coarse (already the F x F block means of a unit-norm v,
// so s = 1 / sqrt(nvec) is in c->pc_st) into out [C][Hc][Wc].
static int pc_net(rte_ctx* c, float* out) {
    NetShape sh;
    sh.init(c->C, c->pc_hidden, c->pc_layers);
    const int F = c->pc_factor;
    const int Hc = c->ny / F, Wc = c->nx / F;
    hipStream_t st = c->stream;
    const unsigned short* wf = (const unsigned short*)c->pc_w;
    if (c->pc_wn) {
        const size_t lds = fused_net_lds(sh, Hc, Wc);
        const int nwn = (int)c->pc_wn_len;
        if (c->pc_hidden == 32)
            hipLaunchKernelGGL((k_net_fused<32>), dim3(1), dim3(NET_THREADS), lds, st, c->pc_coarse, c->pc_st + 1,
                               c->pc_wn, nwn, c->pc_bn, c->pc_nbias, c->pc_meta, sh.layers, c->C, Hc, Wc, out);
        else
            hipLaunchKernelGGL((k_net_fused<16>), dim3(1), dim3(NET_THREADS), lds, st, c->pc_coarse, c->pc_st + 1,
                               c->pc_wn, nwn, c->pc_bn, c->pc_nbias, c->pc_meta, sh.layers, c->C, Hc, Wc, out);
    } else {
        const float* a = c->pc_coarse;
        float* bufs[2] = {c->pc_act0, c->pc_act1};
        for (int l = 0; l < sh.layers; ++l) {
            const bool last = l == sh.layers - 1;
            float* o = last ? out : bufs[l & 1];
            if (conv_launch(sh.cin[l], a, wf + sh.pf_off[l], c->pc_b + sh.boff[l], sh.cout[l], o, nullptr, nullptr, !last,
                            l == 0 ? c->pc_st + 1 : nullptr, 1, Hc, Wc, st))
                return set_error(RTE_EUNSUPPORTED, "unsupported convolution width");
            a = o;
        }
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "pc_net", __FILE__, __LINE__);
}

size_t pc_coarse_len(const rte_ctx* c) {
    return (size_t)c->C * (c->ny / c->pc_factor) * (c->nx / c->pc_factor);
}

// p[0..3] = (a, b, c, d), in stream order (no host staging to keep alive, no wait on the host).
__global__ void k_set_floats4(float* __restrict__ p, float a, float b, float c, float d) {
    if (threadIdx.x == 0) {
        p[0] = a;
        p[1] = b;
        p[2] = c;
        p[3] = d;
    }
}

int pc_begin_solve(rte_ctx* c, int m) {
    const size_t nco = pc_coarse_len(c);
    if (c->pc_slots < m + 1) {
        nfree(c->pc_Y);
        c->pc_slots = 0;
        int rc = nalloc(&c->pc_Y, (size_t)(m + 2) * nco);
        if (rc) return rc;
        c->pc_slots = m + 1;
    }
    // s = RMS of a unit-norm vector = 1 / sqrt(nvec); the combine slot is pc_Y[m + 1]
    hipLaunchKernelGGL(k_set_floats4, dim3(1), dim3(64), 0, c->stream, c->pc_st,
                       (float)(1.0 / std::sqrt((double)c->nvec)), (float)std::sqrt((double)c->nvec), 0.f, 0.f);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "pc_begin_solve", __FILE__, __LINE__);
}

template <typename TW, typename TV>
void pc_scale_pool(rte_ctx* c, const TW* w, TV* v, const double* a_dev, double a_host, double* g, int gn,
                   double g0, int* flags, int nflags) {
    const int F = c->pc_factor;
    const int CW = F > 64 ? F : 64;
    const int nchunk = (c->nx + CW - 1) / CW;
    const int nunit = c->C * (c->ny / F) * nchunk;
    hipLaunchKernelGGL((k_scale_pool<TW, TV>), dim3(nunit), dim3(256), 0, c->stream, w, v, a_dev, a_host,
                       c->pc_coarse, c->C, c->ny, c->nx, F, g, gn, g0, flags, nflags);
}

template <typename TV>
void pc_rescale_pool_arn1(rte_ctx* c, const ArnoldiArgs& t, TV* w, const double* partial) {
    const int F = c->pc_factor;
    const int CW = F > 64 ? F : 64;
    const int nunit = c->C * (c->ny / F) * ((c->nx + CW - 1) / CW);
    // usually nothing to rescale, so a small grid
    hipLaunchKernelGGL(k_rescale_pool_arn1<TV>, dim3(std::min(nunit, 512)), dim3(256), 0, c->stream, t, w, c->pc_coarse,
                       c->C, c->ny, c->nx, F, partial, pc_update_pool_blocks(c));
}

int pc_update_pool_blocks(const rte_ctx* c) {
    const int F = c->pc_factor;
    const int CW = F > 64 ? F : 64;
    return c->C * (c->ny / F) * ((c->nx + CW - 1) / CW);
}

template <typename TV>
void pc_update_pool(rte_ctx* c, TV* w, const TV* V, int nvec, double* partial, double* norm_out,
                    const ArnoldiArgs& s0) {
    const int nblk = pc_update_pool_blocks(c);
    const bool pairs = c->nx % 2 == 0 && c->nvec % 2 == 0 && ((uintptr_t)w % 16) == 0 && ((uintptr_t)V % 16) == 0;
    if (pairs)
        hipLaunchKernelGGL((k_update_pool<true, TV>), dim3(nblk), dim3(256), 0, c->stream, w, V, c->nvec, nvec,
                           c->pc_coarse, partial, c->ny, c->nx, c->pc_factor, s0);
    else
        hipLaunchKernelGGL((k_update_pool<false, TV>), dim3(nblk), dim3(256), 0, c->stream, w, V, c->nvec, nvec,
                           c->pc_coarse, partial, c->ny, c->nx, c->pc_factor, s0);
    if (norm_out) reduce_partials(partial, nblk, norm_out, 1, c->stream);
}

int pc_net_slot(rte_ctx* c, int j) { return pc_net(c, c->pc_Y + (size_t)j * pc_coarse_len(c)); }

// Static LDS of k_rescale_net (Arnoldi column staging, reductions, network metadata) on top of the
// network's dynamic LDS, with some headroom.
constexpr size_t RESCALE_NET_STATIC_LDS = 12 * 1024;

bool pc_rescale_net_ok(const rte_ctx* c) {
    if (!c->pc_wn) return false;
    NetShape sh;
    sh.init(c->C, c->pc_hidden, c->pc_layers);
    const int F = c->pc_factor;
    return fused_net_lds(sh, c->ny / F, c->nx / F) + RESCALE_NET_STATIC_LDS <= 160 * 1024;
}

template <typename TV>
int pc_rescale_net(rte_ctx* c, const ArnoldiArgs& t, TV* w, const double* partial, int slot) {
    NetShape sh;
    sh.init(c->C, c->pc_hidden, c->pc_layers);
    const int F = c->pc_factor;
    const int Hc = c->ny / F, Wc = c->nx / F;
    const size_t lds = fused_net_lds(sh, Hc, Wc);
    const int nwn = (int)c->pc_wn_len;
    float* out = c->pc_Y + (size_t)slot * pc_coarse_len(c);
    // block 1 is the network; the others share stage 1 and the (rare) rescale
    const size_t want = (c->nvec + NET_THREADS - 1) / NET_THREADS;
    const unsigned grid = 2 + (unsigned)std::min<size_t>(want, 254);
    const int nblk = pc_update_pool_blocks(c);
    if (c->pc_hidden == 32)
        hipLaunchKernelGGL((k_rescale_net<32, TV>), dim3(grid), dim3(NET_THREADS), lds, c->stream, t, w, c->nvec, partial,
                           nblk, c->pc_coarse, c->pc_st + 1, c->pc_wn, nwn, c->pc_bn, c->pc_nbias, c->pc_meta,
                           sh.layers, c->C, Hc, Wc, out);
    else
        hipLaunchKernelGGL((k_rescale_net<16, TV>), dim3(grid), dim3(NET_THREADS), lds, c->stream, t, w, c->nvec, partial,
                           nblk, c->pc_coarse, c->pc_st + 1, c->pc_wn, nwn, c->pc_bn, c->pc_nbias, c->pc_meta,
                           sh.layers, c->C, Hc, Wc, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "pc_rescale_net", __FILE__, __LINE__);
}

bool pc_rescale_net_pa_ok(const rte_ctx* c) {
    if (!pc_rescale_net_ok(c) || c->dim != 2) return false;
    if (c->PX != 128 && c->PX != 256 && c->PX != 512 && c->PX != 1024) return false;
    NetShape sh;
    sh.init(c->C, c->pc_hidden, c->pc_layers);
    const size_t pa = pass_a_job_lds<1024>();   // the largest instantiation
    return std::max(fused_net_lds(sh, c->ny / c->pc_factor, c->nx / c->pc_factor), pa) + RESCALE_NET_STATIC_LDS <=
           160 * 1024;
}

template <int HID, typename TV, int PX>
static void launch_rescale_net_pa(rte_ctx* c, const ArnoldiArgs* t, TV* w, const double* partial, int nblk,
                                  int nwn, int layers, int Hc, int Wc, float* out, const PassAJob& pj, size_t lds) {
    lds = std::max(lds, pass_a_job_lds<PX>());
    // one block per CU: blocks 0 and 1 plus 254 pass-A blocks
    if (t)
        hipLaunchKernelGGL((k_rescale_net_pa<HID, TV, PX, true>), dim3(256), dim3(NET_THREADS), lds, c->stream, *t, w,
                           partial, nblk, c->pc_coarse, c->pc_st + 1, c->pc_wn, nwn, c->pc_bn, c->pc_nbias,
                           c->pc_meta, layers, c->C, Hc, Wc, out, pj);
    else
        hipLaunchKernelGGL((k_rescale_net_pa<HID, TV, PX, false>), dim3(256), dim3(NET_THREADS), lds, c->stream,
                           ArnoldiArgs{}, w, partial, nblk, c->pc_coarse, c->pc_st + 1, c->pc_wn, nwn, c->pc_bn,
                           c->pc_nbias, c->pc_meta, layers, c->C, Hc, Wc, out, pj);
}

template <typename TV>
int pc_rescale_net_pa(rte_ctx* c, const ArnoldiArgs* t, TV* w, const double* partial, int slot,
                      const ChanScale& sc, int pack) {
    NetShape sh;
    sh.init(c->C, c->pc_hidden, c->pc_layers);
    const int F = c->pc_factor;
    const int Hc = c->ny / F, Wc = c->nx / F;
    const size_t lds = fused_net_lds(sh, Hc, Wc);
    const int nwn = (int)c->pc_wn_len;
    float* out = c->pc_Y + (size_t)slot * pc_coarse_len(c);
    const int nblk = pc_update_pool_blocks(c);
    PassAJob pj;
    pj.twx = c->twf[0];
    pj.work = c->wf;
    pj.sc = sc;
    pj.nx = c->nx;
    pj.ny = c->ny;
    pj.C = c->C;
    pj.pack = pack;
#define RTE_PA_CASE(PXV)                                                                                         \
    case PXV:                                                                                                    \
        if (c->pc_hidden == 32)                                                                                  \
            launch_rescale_net_pa<32, TV, PXV>(c, t, w, partial, nblk, nwn, sh.layers, Hc, Wc, out, pj, lds);    \
        else                                                                                                     \
            launch_rescale_net_pa<16, TV, PXV>(c, t, w, partial, nblk, nwn, sh.layers, Hc, Wc, out, pj, lds);    \
        break;
    switch (c->PX) {
        RTE_PA_CASE(128) RTE_PA_CASE(256) RTE_PA_CASE(512) RTE_PA_CASE(1024)
        default: return set_error(RTE_EUNSUPPORTED, "pc_rescale_net_pa: padded x %d", c->PX);
    }
#undef RTE_PA_CASE
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "pc_rescale_net_pa", __FILE__, __LINE__);
}

#define RTE_PC_INST(TV)                                                                                           \
    template void pc_scale_pool<double, TV>(rte_ctx*, const double*, TV*, const double*, double, double*, int,    \
                                            double, int*, int);                                                 \
    template void pc_rescale_pool_arn1<TV>(rte_ctx*, const ArnoldiArgs&, TV*, const double*);                    \
    template void pc_update_pool<TV>(rte_ctx*, TV*, const TV*, int, double*, double*, const ArnoldiArgs&);       \
    template int pc_rescale_net<TV>(rte_ctx*, const ArnoldiArgs&, TV*, const double*, int);                     \
    template int pc_rescale_net_pa<TV>(rte_ctx*, const ArnoldiArgs*, TV*, const double*, int, const ChanScale&, int);
RTE_PC_INST(float)
RTE_PC_INST(double)
#undef RTE_PC_INST
template void pc_scale_pool<float, float>(rte_ctx*, const float*, float*, const double*, double, double*, int,
                                          double, int*, int);

const float* pc_slot(const rte_ctx* c, int j) { return c->pc_Y + (size_t)j * pc_coarse_len(c); }

// x += s P (sum_{j < k} y_j Y_j) with y on the device.
template <typename TV>
void pc_combine(rte_ctx* c, double* x, const TV* V, int k, const double* y_dev, const int* skip) {
    const size_t nco = pc_coarse_len(c);
    float* comb = c->pc_Y + (size_t)(c->pc_slots) * nco;
    hipLaunchKernelGGL(k_coarse_combine, dim3((unsigned)((nco + 255) / 256)), dim3(256), 0, c->stream, c->pc_Y, y_dev, k,
                       (int)nco, comb);
    hipLaunchKernelGGL((k_combine_prolong<TV>), dim3((c->nx + 255) / 256, c->C * c->ny), dim3(256), 0, c->stream, x, V,
                       c->nvec, k, y_dev, comb, c->pc_st, c->ny, c->nx, c->pc_factor, skip);
}
template void pc_combine<double>(rte_ctx*, double*, const double*, int, const double*, const int*);
template void pc_combine<float>(rte_ctx*, double*, const float*, int, const double*, const int*);

int pc_apply(rte_ctx* c, const double* v, double* z) {
    NetShape sh;
    sh.init(c->C, c->pc_hidden, c->pc_layers);
    const int F = c->pc_factor;
    const int Hc = c->ny / F, Wc = c->nx / F;
    hipStream_t st = c->stream;
    // restriction and the RMS of v in one pass
    hipLaunchKernelGGL(k_pool_norm, dim3(c->C * Hc), dim3(256), 0, st, v, c->pc_coarse, c->pc_part, c->ny, c->nx, F);
    hipLaunchKernelGGL(k_scale_from_partials, dim3(1), dim3(256), 0, st, c->pc_part, c->C * Hc, (double)c->nvec,
                       c->pc_st);
    const float* a = c->pc_coarse;
    const unsigned short* wf = (const unsigned short*)c->pc_w;
    if (c->pc_wn) {
        const size_t lds = fused_net_lds(sh, Hc, Wc);
        const int nwn = (int)c->pc_wn_len;
        if (c->pc_hidden == 32)
            hipLaunchKernelGGL((k_net_fused<32>), dim3(1), dim3(NET_THREADS), lds, st, c->pc_coarse, c->pc_st + 1,
                               c->pc_wn, nwn, c->pc_bn, c->pc_nbias, c->pc_meta, sh.layers, c->C, Hc, Wc, c->pc_act0);
        else
            hipLaunchKernelGGL((k_net_fused<16>), dim3(1), dim3(NET_THREADS), lds, st, c->pc_coarse, c->pc_st + 1,
                               c->pc_wn, nwn, c->pc_bn, c->pc_nbias, c->pc_meta, sh.layers, c->C, Hc, Wc, c->pc_act0);
        a = c->pc_act0;
    } else {
        // ping-pong activations: layer l writes act[(l % 2)]
        float* bufs[2] = {c->pc_act0, c->pc_act1};
        for (int l = 0; l < sh.layers; ++l) {
            const bool last = l == sh.layers - 1;
            float* o = bufs[l & 1];
            if (conv_launch(sh.cin[l], a, wf + sh.pf_off[l], c->pc_b + sh.boff[l], sh.cout[l], o, nullptr, nullptr, !last,
                            l == 0 ? c->pc_st + 1 : nullptr, 1, Hc, Wc, st))
                return set_error(RTE_EUNSUPPORTED, "unsupported convolution width");
            a = o;
        }
    }
    hipLaunchKernelGGL(k_prolong_add, dim3((c->nx + 255) / 256, c->C * c->ny), dim3(256), 0, st, v, a, c->pc_st, z,
                       c->C, c->ny, c->nx, F);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "pc_apply", __FILE__, __LINE__);
}

}  // namespace rte

using namespace rte;

extern "C" {

int rte_pc_attach(rte_ctx* c, const float* weights, int hidden, int layers, int factor) {
    if (!c) return set_error(RTE_EINVAL, "ctx is NULL");
    pc_free(c);
    if (!weights) return RTE_OK;
    if (c->dim != 2) return set_error(RTE_EUNSUPPORTED, "the learned preconditioner is 2D only");
    if (c->C > 17) return set_error(RTE_EUNSUPPORTED, "the learned preconditioner takes up to 17 channels (L <= 8)");
    if (!valid_net(c->C, hidden, layers)) return set_error(RTE_EINVAL, "bad network shape");
    if (factor < 1 || c->nx % factor || c->ny % factor) return set_error(RTE_EINVAL, "factor must divide n_x and n_y");
    if (c->nx > 512) return set_error(RTE_EUNSUPPORTED, "grid too wide for the restriction kernel");
    if (factor > 256) return set_error(RTE_EUNSUPPORTED, "coarsening factor above 256");
    NetShape sh;
    sh.init(c->C, hidden, layers);
    const int Hc = c->ny / factor, Wc = c->nx / factor;
    const size_t per = (size_t)std::max(hidden, c->C) * Hc * Wc;
    unsigned short* wf = nullptr;
    int rc;
    if ((rc = nalloc(&wf, sh.pf_off_total))) return rc;
    c->pc_w = wf;
    if ((rc = nalloc(&c->pc_b, sh.nparam)) || (rc = nalloc(&c->pc_act0, per)) || (rc = nalloc(&c->pc_act1, per)) ||
        (rc = nalloc(&c->pc_coarse, (size_t)c->C * Hc * Wc)) || (rc = nalloc(&c->pc_st, 4)) ||
        (rc = nalloc(&c->pc_nrm, 2)) || (rc = nalloc(&c->pc_part, (size_t)c->C * Hc)) ||
        (rc = nalloc(&c->pc_meta, (size_t)4 * layers))) {
        pc_free(c);
        return rc;
    }
    // biases are read from a full FP32 copy of the parameters (only the bias slices are used)
    hipError_t e = hipMemcpyAsync(c->pc_b, weights, sh.nparam * sizeof(float), hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) { pc_free(c); return set_hip_error(e, "pc weights", __FILE__, __LINE__); }
    pack_all(sh, weights, wf, nullptr, c->stream);
    std::vector<int> toff;
    const size_t tlen = tapmajor_len(sh, &toff);
    std::vector<int> boff_packed(layers);
    int nbias = 0;
    for (int l = 0; l < layers; ++l) { boff_packed[l] = nbias; nbias += sh.cout[l]; }
    if (fused_net_fits(sh, Hc, Wc)) {
        if ((rc = nalloc(&c->pc_wn, tlen)) || (rc = nalloc(&c->pc_bn, (size_t)nbias))) { pc_free(c); return rc; }
        c->pc_wn_len = tlen;
        c->pc_nbias = nbias;
        for (int l = 0; l < layers; ++l) {
            hipLaunchKernelGGL(k_pack_tapmajor, dim3(64), dim3(256), 0, c->stream, wf + sh.pf_off[l], sh.cin[l],
                               c->pc_wn + toff[l]);
            e = hipMemcpyAsync(c->pc_bn + boff_packed[l], weights + sh.boff[l], sh.cout[l] * sizeof(float),
                               hipMemcpyDeviceToDevice, c->stream);
            if (e != hipSuccess) { pc_free(c); return set_hip_error(e, "pc biases", __FILE__, __LINE__); }
        }
    }
    // meta: cin, cout, tap-major pack offset, bias offset (into the packed biases of the fused
    // kernel when it is used, else into the full parameter copy)
    std::vector<int> meta(4 * layers);
    for (int l = 0; l < layers; ++l) {
        meta[4 * l] = sh.cin[l];
        meta[4 * l + 1] = sh.cout[l];
        meta[4 * l + 2] = toff[l];
        meta[4 * l + 3] = c->pc_wn ? boff_packed[l] : (int)sh.boff[l];
    }
    e = hipMemcpyAsync(c->pc_meta, meta.data(), meta.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) { pc_free(c); return set_hip_error(e, "pc meta", __FILE__, __LINE__); }
    c->pc_hidden = hidden;
    c->pc_layers = layers;
    c->pc_factor = factor;
    c->pc_attached = true;
    e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "rte_pc_attach", __FILE__, __LINE__);
}

int rte_pc_apply(rte_ctx* c, const double* v, double* z) {
    if (!c || !v || !z || v == z) return set_error(RTE_EINVAL, "bad argument");
    if (!c->pc_attached) return set_error(RTE_EINVAL, "no preconditioner attached");
    return pc_apply(c, v, z);
}

int rte_nn_create(rte_nn** out, int C, int hidden, int layers, unsigned long long seed, int use_bias, void* stream) {
    if (!out) return set_error(RTE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!valid_net(C, hidden, layers)) return set_error(RTE_EINVAL, "bad network shape");
    int dev = 0;
    RTE_HIP_TRY(hipGetDevice(&dev));
    {
        const int rs = scratch_resolve(dev);
        if (rs) return rs;
    }
    rte_nn* nn = new rte_nn();
    nn->sh.init(C, hidden, layers);
    nn->device = dev;
    nn->stream = (hipStream_t)stream;
    nn->use_bias = use_bias != 0;
    const size_t np = nn->sh.nparam;
    int rc;
    if ((rc = nalloc(&nn->p, np)) || (rc = nalloc(&nn->g, np)) || (rc = nalloc(&nn->m, np)) || (rc = nalloc(&nn->v, np)) ||
        (rc = nalloc(&nn->wf, nn->sh.pf_off_total)) || (rc = nalloc(&nn->wb, nn->sh.pb_off_total))) {
        rte_nn_destroy(nn);
        return rc;
    }
    // He-normal weights (std = sqrt(2 / fan_in)), zero biases, seeded
    std::vector<float> h(np, 0.f);
    std::mt19937_64 gen(seed);
    for (int l = 0; l < layers; ++l) {
        std::normal_distribution<double> nd(0.0, std::sqrt(2.0 / (9.0 * nn->sh.cin[l])) * (l == layers - 1 ? 0.1 : 1.0));
        for (size_t i = 0; i < (size_t)nn->sh.cout[l] * nn->sh.cin[l] * 9; ++i) h[nn->sh.woff[l] + i] = (float)nd(gen);
    }
    hipError_t e = hipMemcpy(nn->p, h.data(), np * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(nn->m, 0, np * sizeof(float));
    if (e == hipSuccess) e = hipMemset(nn->v, 0, np * sizeof(float));
    if (e != hipSuccess) { rte_nn_destroy(nn); return set_hip_error(e, "rte_nn_create", __FILE__, __LINE__); }
    *out = nn;
    return RTE_OK;
}

void rte_nn_destroy(rte_nn* nn) {
    if (!nn) return;
    if (nn->stream) (void)hipStreamSynchronize(nn->stream);
    nfree(nn->p); nfree(nn->g); nfree(nn->m); nfree(nn->v); nfree(nn->wf); nfree(nn->wb);
    for (auto& a : nn->act) nfree(a);
    for (auto& a : nn->pre) nfree(a);
    nfree(nn->gA); nfree(nn->gB); nfree(nn->lossb); nfree(nn->wpart);
    delete nn;
}

int rte_nn_param_count(const rte_nn* nn, long long* count) {
    if (!nn || !count) return set_error(RTE_EINVAL, "NULL argument");
    *count = (long long)nn->sh.nparam;
    return RTE_OK;
}

int rte_nn_get_params(rte_nn* nn, float* dst) {
    if (!nn || !dst) return set_error(RTE_EINVAL, "NULL argument");
    RTE_HIP_TRY(hipMemcpyAsync(dst, nn->p, nn->sh.nparam * sizeof(float), hipMemcpyDeviceToDevice, nn->stream));
    return RTE_OK;
}

int rte_nn_set_params(rte_nn* nn, const float* src) {
    if (!nn || !src) return set_error(RTE_EINVAL, "NULL argument");
    RTE_HIP_TRY(hipMemcpyAsync(nn->p, src, nn->sh.nparam * sizeof(float), hipMemcpyDeviceToDevice, nn->stream));
    return RTE_OK;
}

int rte_nn_forward(rte_nn* nn, const float* x, int B, int H, int W, float* y) {
    if (!nn || !x || !y || B < 1 || H < 1 || W < 1) return set_error(RTE_EINVAL, "bad argument");
    int rc = ensure_acts(nn, (size_t)B * std::max(nn->sh.hidden, nn->sh.C) * H * W, B);
    if (rc) return rc;
    pack_all(nn->sh, nn->p, nn->wf, nullptr, nn->stream);
    std::vector<float*> act = nn->act;
    act[nn->sh.layers] = y;
    rc = net_forward(nn->sh, nn->wf, nn->p, nn->sh.boff, x, nullptr, act.data(), nullptr, B, H, W, nn->stream);
    if (rc) return rc;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "rte_nn_forward", __FILE__, __LINE__);
}

int rte_nn_forward_noalloc(rte_nn* nn, const float* x, int B, int H, int W, float* y) {
    if (!nn || !x || !y || B < 1 || H < 1 || W < 1) return set_error(RTE_EINVAL, "bad argument");
    const NetShape& sh = nn->sh;
    // layers 0..L-2 write intermediate activations, alternating between two halves of the array
    const size_t per = (size_t)B * std::max(sh.hidden, sh.C) * H * W;
    const size_t halves = sh.layers > 2 ? 2 : 1;
    if (per > RTE_NN_SCRATCH_BYTES / sizeof(float) / halves)
        return set_error(RTE_EINVAL, "batch*channels*H*W = %zu exceeds the allocation-free forward's limit of %zu "
                         "floats per activation", per, (size_t)RTE_NN_SCRATCH_BYTES / sizeof(float) / halves);
    float* base = scratch_ptr(nn->device);
    if (!base) return set_error(RTE_EDEVICE, "scratch not resolved for device %d", nn->device);
    const size_t half = RTE_NN_SCRATCH_BYTES / sizeof(float) / 2;
    float* act[9];
    for (int l = 1; l < sh.layers; ++l) act[l] = base + (size_t)((l - 1) & 1) * half;
    act[sh.layers] = y;
    act[0] = nullptr;
    pack_all(sh, nn->p, nn->wf, nullptr, nn->stream);
    int rc = net_forward(sh, nn->wf, nn->p, sh.boff, x, nullptr, act, nullptr, B, H, W, nn->stream);
    if (rc) return rc;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "rte_nn_forward_noalloc", __FILE__, __LINE__);
}

int rte_nn_loss_grad(rte_nn* nn, const float* x, const float* t, const float* w, int B, int H, int W, double* loss,
                     float* grad) {
    if (!nn || !x || !t || !w || B < 1 || H < 1 || W < 1) return set_error(RTE_EINVAL, "bad argument");
    const NetShape& sh = nn->sh;
    int rc = ensure_acts(nn, (size_t)B * std::max(sh.hidden, sh.C) * H * W, B);
    if (rc) return rc;
    hipStream_t st = nn->stream;
    pack_all(sh, nn->p, nn->wf, nn->wb, st);
    if ((rc = net_forward(sh, nn->wf, nn->p, sh.boff, x, nullptr, nn->act.data(), nn->pre.data(), B, H, W, st)))
        return rc;
    const int per = sh.C * H * W;
    hipLaunchKernelGGL(k_loss, dim3(B), dim3(256), 0, st, nn->act[sh.layers], t, w, nn->gA, nn->lossb, per, B);
    const size_t wneed = (size_t)wgrad_tiles(B, H, W) * 32 * wgrad_ktiles(WG_MAXCIN) * 32;
    if (wneed > nn->wpart_cap) {
        nfree(nn->wpart);
        nn->wpart_cap = 0;
        if ((rc = nalloc(&nn->wpart, wneed))) return rc;
        nn->wpart_cap = wneed;
    }
    // backward: gA holds dLoss/d(output of layer l)
    float* gcur = nn->gA;
    float* gnext = nn->gB;
    for (int l = sh.layers - 1; l >= 0; --l) {
        const float* a_in = l == 0 ? x : nn->act[l];
        const int ntiles = wgrad_tiles(B, H, W);
        const dim3 wg((unsigned)ntiles, (unsigned)((wgrad_ktiles(sh.cin[l]) + 3) / 4));
        hipLaunchKernelGGL(k_conv3x3_wgrad, wg, dim3(256), 0, st, a_in, gcur, nn->wpart, B, sh.cin[l], sh.cout[l], H,
                           W);
        const int nout = sh.cout[l] * (sh.cin[l] * 9 + 1);
        hipLaunchKernelGGL(k_wgrad_reduce, dim3((nout + 255) / 256), dim3(256), 0, st, nn->wpart, ntiles, sh.cin[l],
                           sh.cout[l], nn->g + sh.woff[l], nn->g + sh.boff[l]);
        if (l > 0) {   // data gradient, masked by the ReLU of layer l-1
            if (conv_launch(sh.cout[l], gcur, nn->wb + sh.pb_off[l], nullptr, sh.cin[l], gnext, nullptr, nn->pre[l - 1],
                            false, nullptr, B, H, W, st))
                return set_error(RTE_EUNSUPPORTED, "unsupported convolution width");
            std::swap(gcur, gnext);
        }
    }
    if (!nn->use_bias)
        for (int l = 0; l < sh.layers; ++l)
            RTE_HIP_TRY(hipMemsetAsync(nn->g + sh.boff[l], 0, sh.cout[l] * sizeof(float), st));
    std::vector<double> lb(B);
    RTE_HIP_TRY(hipMemcpyAsync(lb.data(), nn->lossb, B * sizeof(double), hipMemcpyDeviceToHost, st));
    if (grad) RTE_HIP_TRY(hipMemcpyAsync(grad, nn->g, sh.nparam * sizeof(float), hipMemcpyDeviceToDevice, st));
    RTE_HIP_TRY(hipStreamSynchronize(st));
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += lb[b];
    if (loss) *loss = s;
    return RTE_OK;
}

int rte_nn_adam_step(rte_nn* nn, float lr) {
    if (!nn || !(lr > 0.f)) return set_error(RTE_EINVAL, "bad argument");
    nn->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)nn->step), c2 = 1.f - std::pow(b2, (float)nn->step);
    const size_t n = nn->sh.nparam;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, nn->stream, nn->p, nn->g, nn->m, nn->v, n,
                       lr, b1, b2, c1, c2, 1e-8f);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "rte_nn_adam_step", __FILE__, __LINE__);
}

int rte_nn_gather_rows(const float* src, long long nrows, long long row_len, const int* idx, int count, float* dst,
                       void* hip_stream) {
    if (!src || !idx || !dst || nrows < 1 || row_len < 1 || count < 0) return set_error(RTE_EINVAL, "bad argument");
    const float* src_end = src + nrows * row_len;
    if (dst < src_end && src < dst + (long long)count * row_len) return set_error(RTE_EINVAL, "dst overlaps src");
    if (count == 0) return RTE_OK;
    const long long total = (long long)count * row_len;
    const unsigned nb = (unsigned)std::min<long long>((total + 255) / 256, 65535LL * 8);
    hipLaunchKernelGGL(k_gather_rows, dim3(nb), dim3(256), 0, (hipStream_t)hip_stream, src, row_len, idx, total, dst);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "rte_nn_gather_rows", __FILE__, __LINE__);
}

int rte_nn_upsample_bilinear(const double* coarse, int count, int C, int hc, int wc, int ny, int nx, double* fine,
                             void* hip_stream) {
    if (!coarse || !fine || count < 0 || C < 1 || hc < 1 || wc < 1 || ny < 1 || nx < 1)
        return set_error(RTE_EINVAL, "bad argument");
    const long long total = (long long)count * C * ny * nx;
    if (total == 0) return RTE_OK;
    const unsigned nb = (unsigned)std::min<long long>((total + 255) / 256, 65535LL * 8);
    hipLaunchKernelGGL(k_upsample_bilinear, dim3(nb), dim3(256), 0, (hipStream_t)hip_stream, coarse, hc, wc, ny, nx,
                       total, fine);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "rte_nn_upsample_bilinear", __FILE__, __LINE__);
}

int rte_pc_make_pairs(rte_ctx* c, const double* b, const double* xs, const double* xit, int count, int F, float* xo,
                      float* to, float* wo) {
    if (!c || !b || !xs || !xit || !xo || !to || !wo || count < 0) return set_error(RTE_EINVAL, "bad argument");
    if (c->dim != 2 || F < 1 || c->nx % F || c->ny % F) return set_error(RTE_EINVAL, "factor must divide n_x and n_y");
    if (F > 256) return set_error(RTE_EUNSUPPORTED, "coarsening factor above 256");
    const size_t n = c->nvec;
    const int Hc = c->ny / F, Wc = c->nx / F;
    const int nco = c->C * Hc * Wc;
    hipStream_t st = c->stream;
    for (int j = 0; j < count; ++j) {
        const double* xj = xit + (size_t)j * n;
        // r = b - A x_j into rv; e = x_star - x_j into t1
        int rc = apply_channels(c, APPLY_RESID, RTE_PREC_FP64, xj, b, c->rv, 1);
        if (rc) return rc;
        hipLaunchKernelGGL(k_sub, dim3(2048), dim3(256), 0, st, xs, xj, c->t1, n);
        krylov_dots(c->t1, n, 1, c->t1, n, c->partial, c->dsmall, false, st);
        krylov_dots(c->rv, n, 1, c->rv, n, c->partial, c->dsmall + 1, false, st);
        float* xr = xo + (size_t)j * nco;
        float* xt = to + (size_t)j * nco;
        const dim3 pg((unsigned)((c->nx + pool_chunk(F) - 1) / pool_chunk(F)), (unsigned)Hc, (unsigned)c->C);
        hipLaunchKernelGGL(k_pool, pg, dim3(256), 0, st, c->rv, (const double*)nullptr, (const double*)nullptr, xr,
                           c->C, c->ny, c->nx, F);
        hipLaunchKernelGGL(k_pool, pg, dim3(256), 0, st, c->t1, c->rv, (const double*)nullptr, xt, c->C, c->ny, c->nx,
                           F);
        hipLaunchKernelGGL(k_pair_finish, dim3(1), dim3(256), 0, st, xr, xt, nco, c->dsmall + 1, (double)n, c->dsmall,
                           wo + j, F);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "rte_pc_make_pairs", __FILE__, __LINE__);
}

}  // extern "C"
