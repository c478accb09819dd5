// 3D FFT apply (Sec. 2.3.1 with d = 3; Sec. 3.1.2 for the spherical-harmonic modes).
//
// u is C real fields [C][nz][ny][nx] (C = 1: isotropic; C = (L+1)^2: the real spherical-harmonic
// modes of sh3d.h).  Isotropic: the kernel h^3 exp(-mu_t r)/(4 pi r^2) has a real, even spectrum,
// stored as the octant Q3[kx][ky][kz] (scaled by 1/(PX PY PZ)).  Modes: the (a, b) block of the
// kernel, kappa(r) Y_a(w) Y_b(w), has a spectrum F_ab = i^(l_b - l_a) R_ab with R_ab real, stored as
// one octant per pair a <= b, and reflecting ky or kz multiplies it by the parities of Y_a and Y_b.
// Five passes per channel:
//   A  x-FFT (real-to-complex) of every row, per z-slab, stored T1[c][z][kx][y]   (2D pass A)
//   B  y-FFT of every (c, z, kx) column times the channel's factor of D, stored T2[c][kx][ky][z]
//   C  z-FFT of every (kx, ky) column of every channel, multiply by the spectrum (C > 1: the
//      mode coupling y_a = sum_b F_ab w_b per frequency), inverse z-FFT, in place
//   D  inverse y-FFT, stored back to T1[c][z][kx][y]
//   E  inverse x-FFT (complex-to-real), crop, y = u - v / v / residual           (2D pass C)
// Each pass reads and writes HBM in 128-byte runs: B and D move tiles of TZ consecutive z.
#include "apply3d.h"
#include "fft.h"
#include "sh3d.h"

namespace rte {

template <typename T, int PY, int TZ, int NTHR>
__global__ __launch_bounds__(NTHR) void k_pass3_b(const cx<T>* __restrict__ T1, cx<T>* __restrict__ T2,
                                                  const cx<T>* __restrict__ tw, int ny, int nz, int nkx, size_t t1sz,
                                                  size_t t2sz, ChanScale3 sc) {
    constexpr int LD = padded(PY) + 1;   // odd row pitch: the TZ transforms start on different banks
    __shared__ cx<T> buf[TZ * LD];
    __shared__ cx<T> tws[PY];
    const int tid = threadIdx.x;
    const int kx = blockIdx.x, z0 = blockIdx.y * TZ, ch = blockIdx.z;
    const T s = (T)sc.s[ch];
    T1 += ch * t1sz;
    T2 += ch * t2sz;
    stage_twiddles<T, PY, NTHR>(tws, tw, tid);
    __syncthreads();
    // rows y >= ny are zero padding: the first stage is computed from the loads
    fft_forward_padded<T, PY, TZ, LD, NTHR>(buf, tws, tid, [&](int zl, int y) {
        const int z = z0 + zl;
        return (z < nz && y < ny) ? scale(T1[((size_t)z * nkx + kx) * ny + y], s) : mk((T)0, (T)0);
    });
    for (int idx = tid; idx < TZ * PY; idx += NTHR) {
        const int zl = idx % TZ, ky = idx / TZ;
        const int z = z0 + zl;
        if (z < nz) T2[((size_t)kx * PY + ky) * nz + z] = buf[zl * LD + sw(ky)];
    }
}

template <typename T, int PZ, int NC, int NTHR>
__global__ __launch_bounds__(NTHR) void k_pass3_c(cx<T>* __restrict__ T2, const T* __restrict__ Q3,
                                                  const cx<T>* __restrict__ tw, int nz, int PY, size_t ncol) {
    constexpr int LD = padded(PZ) + 1;
    __shared__ cx<T> buf[NC * LD];
    __shared__ cx<T> tws[PZ];
    const int tid = threadIdx.x;
    const size_t c0 = (size_t)blockIdx.x * NC;
    const int HY = PY / 2 + 1, HZ = PZ / 2 + 1;
    stage_twiddles<T, PZ, NTHR>(tws, tw, tid);
    __syncthreads();
    // entries z >= nz are zero padding; only z < nz are kept after the inverse transform
    fft_forward_padded<T, PZ, NC, LD, NTHR>(buf, tws, tid, [&](int c, int z) {
        const size_t col = c0 + c;
        return (col < ncol && z < nz) ? T2[col * nz + z] : mk((T)0, (T)0);
    });
    // spectrum row of each of the block's columns, decoded once (col = kx PY + ky)
    __shared__ int qrow[NC];
    if (tid < NC) {
        const int col = (int)(c0 + tid);
        const int kx = col / PY, ky = col % PY;
        const int fy = ky <= PY / 2 ? ky : PY - ky;
        qrow[tid] = (col < (int)ncol) ? (kx * HY + fy) * HZ : -1;
    }
    __syncthreads();
    // the spectrum values of the thread's entries are loaded first, all in flight together
    constexpr int PERQ = (NC * PZ + NTHR - 1) / NTHR;
    T qv[PERQ];
#pragma unroll
    for (int u = 0; u < PERQ; ++u) {
        const int idx = tid + u * NTHR;
        const int c = idx / PZ, kz = idx % PZ;
        const int q = ((NC * PZ) % NTHR == 0 || idx < NC * PZ) ? qrow[c] : -1;
        const int fz = kz <= PZ / 2 ? kz : PZ - kz;
        qv[u] = q >= 0 ? Q3[(size_t)q + fz] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < PERQ; ++u) {
        const int idx = tid + u * NTHR;
        const int c = idx / PZ, kz = idx % PZ;
        if (((NC * PZ) % NTHR == 0 || idx < NC * PZ) && qrow[c] >= 0)
            buf[c * LD + sw(kz)] = scale(buf[c * LD + sw(kz)], qv[u]);
    }
    __syncthreads();
    fft_inverse_cropped<T, PZ, NC, LD, NTHR>(buf, tws, tid, [&](int c, int z, cx<T> v) {
        const size_t col = c0 + c;
        if (col < ncol && z < nz) T2[col * nz + z] = v;
    });
}

// Degree and reflection parities of the first 16 modes, as compile-time tables (sh3d.h).
constexpr int kShDeg[16] = {0, 1, 1, 1, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3};
constexpr int kShNegY[16] = {0, 1, 0, 0, 1, 1, 0, 0, 0, 1, 1, 1, 0, 0, 0, 0};   // m < 0
constexpr int kShNegZ[16] = {0, 0, 1, 0, 0, 1, 0, 1, 0, 0, 1, 0, 1, 0, 1, 0};   // l - |m| odd

template <typename T>
__device__ __forceinline__ cx<T> times_i_pow(cx<T> v, int q) {   // v i^q, q in 0..3
    return q == 0 ? v : q == 1 ? mul_i(v) : q == 2 ? mk(-v.re, -v.im) : mul_mi(v);
}

// Pass C with the mode coupling.  A block takes the column pair (kx, fy) and (kx, PY - fy), which
// read the same octant entries (fy = 0 and PY/2 are single columns): the z-FFT of all CH channels of
// both columns in LDS, then per frequency kz (one thread each, both columns)
//     w'_b = i^(l_b) s_b w_b,   y'_a = sum_b R_ab w'_b,   y_a = i^(-l_a) s_a y'_a,
// s_a = the parities of Y_a for the reflections that map (ky, kz) into the stored octant, which
// equals y_a = sum_b F_ab w_b; R_ba = (-1)^(l_a + l_b) R_ab supplies the lower triangle, and every
// R value read serves both columns.  Then the inverse z-FFT of every channel of both columns.
template <typename T, int PZ, int CH, int NTHR>
__global__ __launch_bounds__(NTHR) void k_pass3_c_sh(cx<T>* __restrict__ T2, const T* __restrict__ Q,
                                                     const cx<T>* __restrict__ tw, int nz, int PY, size_t t2sz,
                                                     size_t noct) {
    constexpr int LD = padded(PZ) + 1;
    __shared__ cx<T> buf[2 * CH * LD];
    __shared__ cx<T> tws[PZ];
    const int tid = threadIdx.x;
    const int HY = PY / 2 + 1, HZ = PZ / 2 + 1;
    const int kx = blockIdx.x / HY, fy = blockIdx.x % HY;
    const bool pair = fy > 0 && fy < PY / 2;
    const size_t col0 = (size_t)kx * PY + fy, col1 = (size_t)kx * PY + (PY - fy);
    stage_twiddles<T, PZ, NTHR>(tws, tw, tid);
    __syncthreads();
    // transforms 0..CH-1: column (kx, fy); CH..2CH-1: column (kx, PY - fy), zero when single
    fft_forward_padded<T, PZ, 2 * CH, LD, NTHR>(buf, tws, tid, [&](int t, int z) {
        const int c = t % CH;
        const bool second = t >= CH;
        return (z < nz && (!second || pair)) ? T2[c * t2sz + (second ? col1 : col0) * nz + z] : mk((T)0, (T)0);
    });
    const T* Qc = Q + ((size_t)kx * HY + fy) * HZ;
    for (int kz = tid; kz < PZ; kz += NTHR) {
        const bool negz = kz > PZ / 2;
        const int fz = negz ? PZ - kz : kz;
        cx<T> w0[CH], y0[CH], w1[CH], y1[CH];
#pragma unroll
        for (int b = 0; b < CH; ++b) {
            // first column: ky = fy <= PY/2 (no y reflection); second: ky = PY - fy (reflected)
            cx<T> v = buf[b * LD + sw(kz)];
            if (kShNegZ[b] && negz) v = mk(-v.re, -v.im);
            w0[b] = times_i_pow(v, kShDeg[b] & 3);
            cx<T> u = buf[(CH + b) * LD + sw(kz)];
            if (kShNegY[b] != (kShNegZ[b] && negz)) u = mk(-u.re, -u.im);
            w1[b] = times_i_pow(u, kShDeg[b] & 3);
            y0[b] = mk((T)0, (T)0);
            y1[b] = mk((T)0, (T)0);
        }
#pragma unroll
        for (int a = 0; a < CH; ++a) {
#pragma unroll
            for (int b = a; b < CH; ++b) {
                const T r = Qc[(size_t)(a * CH - a * (a - 1) / 2 + (b - a)) * noct + fz];
                y0[a].re = fma(r, w0[b].re, y0[a].re);
                y0[a].im = fma(r, w0[b].im, y0[a].im);
                y1[a].re = fma(r, w1[b].re, y1[a].re);
                y1[a].im = fma(r, w1[b].im, y1[a].im);
                if (b != a) {
                    const T rb = ((kShDeg[a] + kShDeg[b]) & 1) ? -r : r;
                    y0[b].re = fma(rb, w0[a].re, y0[b].re);
                    y0[b].im = fma(rb, w0[a].im, y0[b].im);
                    y1[b].re = fma(rb, w1[a].re, y1[b].re);
                    y1[b].im = fma(rb, w1[a].im, y1[b].im);
                }
            }
        }
#pragma unroll
        for (int a = 0; a < CH; ++a) {
            cx<T> v = times_i_pow(y0[a], (4 - (kShDeg[a] & 3)) & 3);
            if (kShNegZ[a] && negz) v = mk(-v.re, -v.im);
            buf[a * LD + sw(kz)] = v;
            cx<T> u = times_i_pow(y1[a], (4 - (kShDeg[a] & 3)) & 3);
            if (kShNegY[a] != (kShNegZ[a] && negz)) u = mk(-u.re, -u.im);
            buf[(CH + a) * LD + sw(kz)] = u;
        }
    }
    __syncthreads();
    fft_inverse_cropped<T, PZ, 2 * CH, LD, NTHR>(buf, tws, tid, [&](int t, int z, cx<T> v) {
        const int c = t % CH;
        const bool second = t >= CH;
        if (z < nz && (!second || pair)) T2[c * t2sz + (second ? col1 : col0) * nz + z] = v;
    });
}

template <typename T, int PY, int TZ, int NTHR>
__global__ __launch_bounds__(NTHR) void k_pass3_d(cx<T>* __restrict__ T1, const cx<T>* __restrict__ T2,
                                                  const cx<T>* __restrict__ tw, int ny, int nz, int nkx, size_t t1sz,
                                                  size_t t2sz) {
    constexpr int LD = padded(PY) + 1;   // odd row pitch: the TZ transforms start on different banks
    __shared__ cx<T> buf[TZ * LD];
    __shared__ cx<T> tws[PY];
    const int tid = threadIdx.x;
    const int kx = blockIdx.x, z0 = blockIdx.y * TZ, ch = blockIdx.z;
    T1 += ch * t1sz;
    T2 += ch * t2sz;
    stage_twiddles<T, PY, NTHR>(tws, tw, tid);
    // every load of the tile is issued before the first LDS store, so their latencies overlap
    constexpr int PER = (TZ * PY + NTHR - 1) / NTHR;
    cx<T> v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = tid + u * NTHR;
        const int zl = idx % TZ, ky = idx / TZ;
        const int z = z0 + zl;
        v[u] = ((TZ * PY) % NTHR == 0 || idx < TZ * PY) && z < nz ? T2[((size_t)kx * PY + ky) * nz + z]
                                                                   : mk((T)0, (T)0);
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = tid + u * NTHR;
        if ((TZ * PY) % NTHR == 0 || idx < TZ * PY) buf[(idx % TZ) * LD + sw(idx / TZ)] = v[u];
    }
    __syncthreads();
    // only rows y < ny are kept: the last inverse stage writes them directly
    fft_inverse_cropped<T, PY, TZ, LD, NTHR>(buf, tws, tid, [&](int zl, int y, cx<T> v) {
        const int z = z0 + zl;
        if (z < nz && y < ny) T1[((size_t)z * nkx + kx) * ny + y] = v;
    });
}

// z-rows per block of the y-passes: 8 (variant 0), 4 or 16 (variants 1, 2).  At 128^3 in FP32, 16
// and 4 rows were slower than 8: 15.1 / 22.3 and 19.4 / 27.0 us for the forward / inverse pass
// against 13.4 / 21.1.
template <typename T, int PY, int TZ>
static void launch3_bd_tz(const Apply3DArgs<T>& a, bool inverse) {
    const int nkx = a.PX / 2 + 1;
    const size_t t1sz = (size_t)a.nz * nkx * a.ny, t2sz = (size_t)nkx * a.PY * a.nz;
    dim3 grid(nkx, (a.nz + TZ - 1) / TZ, a.C);
    if (!inverse)
        hipLaunchKernelGGL((k_pass3_b<T, PY, TZ, 256>), grid, dim3(256), 0, a.stream, a.T1, a.T2, a.twy, a.ny, a.nz,
                           nkx, t1sz, t2sz, a.sc);
    else
        hipLaunchKernelGGL((k_pass3_d<T, PY, TZ, 256>), grid, dim3(256), 0, a.stream, a.T1, a.T2, a.twy, a.ny, a.nz,
                           nkx, t1sz, t2sz);
}

template <typename T, int PY>
static void launch3_bd(const Apply3DArgs<T>& a, bool inverse) {
    const int v = a.var[inverse ? 2 : 0];
    if (v == 1) launch3_bd_tz<T, PY, 4>(a, inverse);
    else if (v == 2) launch3_bd_tz<T, PY, 16>(a, inverse);
    else launch3_bd_tz<T, PY, 8>(a, inverse);
}

template <typename T, int PZ, int NC>
static void launch3_c_iso(const Apply3DArgs<T>& a, size_t ncol) {
    dim3 grid((unsigned)((ncol + NC - 1) / NC));
    hipLaunchKernelGGL((k_pass3_c<T, PZ, NC, 256>), grid, dim3(256), 0, a.stream, a.T2, a.Q3, a.twz, a.nz, a.PY, ncol);
}

template <typename T, int PZ>
static int launch3_c(const Apply3DArgs<T>& a) {
    const size_t ncol = (size_t)(a.PX / 2 + 1) * a.PY;
    if (a.C == 1) {
        constexpr int NC = PZ >= 2048 ? 1 : 2048 / PZ;
        if (a.var[1] == 1) launch3_c_iso<T, PZ, (NC > 1 ? NC / 2 : 1)>(a, ncol);
        else if (a.var[1] == 2) launch3_c_iso<T, PZ, 2 * NC>(a, ncol);
        else launch3_c_iso<T, PZ, NC>(a, ncol);
        return 0;
    }
    if constexpr (PZ > 256) {
        return -1;                                       // the mode coupling is built for padded z <= 256
    } else {
    const size_t t2sz = ncol * a.nz;
    const size_t noct = (size_t)(a.PX / 2 + 1) * (a.PY / 2 + 1) * (PZ / 2 + 1);
    const unsigned npairs = (unsigned)((a.PX / 2 + 1) * (a.PY / 2 + 1));   // blocks: (kx, fy) column pairs
    constexpr int NT = PZ >= 256 ? 256 : (PZ < 64 ? 64 : PZ);
    switch (a.C) {
#define RTE_CSH(CHN)                                                                                              \
    case CHN:                                                                                                     \
        hipLaunchKernelGGL((k_pass3_c_sh<T, PZ, CHN, NT>), dim3(npairs), dim3(NT), 0, a.stream, a.T2, a.Q3, a.twz,   \
                           a.nz, a.PY, t2sz, noct);                                                               \
        return 0;
        RTE_CSH(4) RTE_CSH(9) RTE_CSH(16)
#undef RTE_CSH
    }
    return -1;
    }
}

template <typename T>
int apply3d_pass(const Apply3DArgs<T>& a, int which) {
    const int P = which == 2 ? a.PZ : a.PY;
    switch (P) {
#define RTE_C3(PP)                                              \
    case PP:                                                    \
        if (which == 1) launch3_bd<T, PP>(a, false);            \
        else if (which == 3) launch3_bd<T, PP>(a, true);        \
        else return launch3_c<T, PP>(a);                        \
        return 0;
        RTE_C3(16) RTE_C3(32) RTE_C3(64) RTE_C3(128) RTE_C3(256) RTE_C3(512)
#undef RTE_C3
    }
    return -1;
}

template <typename T>
int apply3d_variant_count(int which, int C, int PZ) {
    (void)PZ;
    if (which == 1 || which == 3) return 3;
    if (which == 2) return C == 1 ? 3 : 1;
    return 0;
}
template int apply3d_variant_count<float>(int, int, int);
template int apply3d_variant_count<double>(int, int, int);

template int apply3d_pass<float>(const Apply3DArgs<float>&, int);
template int apply3d_pass<double>(const Apply3DArgs<double>&, int);

}  // namespace rte
