// 3D isotropic FFT apply (Sec. 2.3.1 with d = 3; the M = {0} case of Sec. 3.1.2).
//
// u is one real field [nz][ny][nx]; the kernel h^3 exp(-mu_t r)/(4 pi r^2) has a real, even
// spectrum, stored as the octant Q3[kx][ky][kz] (scaled by 1/(PX PY PZ)).  Five passes:
//   A  x-FFT (real-to-complex) of every row, per z-slab, stored T1[z][kx][y]   (2D pass A)
//   B  y-FFT of every (z, kx) column, stored transposed T2[kx][ky][z]
//   C  z-FFT of every (kx, ky) column, multiply by the spectrum, inverse z-FFT, in place
//   D  inverse y-FFT, stored back to T1[z][kx][y]
//   E  inverse x-FFT (complex-to-real), crop, y = u - mu_s v / v / residual   (2D pass C)
// Each pass reads and writes HBM in 128-byte runs: B and D move tiles of TZ consecutive z.
#include "apply3d.h"
#include "fft.h"

namespace rte {

template <typename T, int PY, int TZ, int NTHR>
__global__ __launch_bounds__(NTHR) void k_pass3_b(const cx<T>* __restrict__ T1, cx<T>* __restrict__ T2,
                                                  const cx<T>* __restrict__ tw, int ny, int nz, int nkx) {
    constexpr int LD = padded(PY) + 1;   // odd row pitch: the TZ transforms start on different banks
    __shared__ cx<T> buf[TZ * LD];
    __shared__ cx<T> tws[PY];
    const int tid = threadIdx.x;
    const int kx = blockIdx.x, z0 = blockIdx.y * TZ;
    stage_twiddles<T, PY, NTHR>(tws, tw, tid);
    __syncthreads();
    // rows y >= ny are zero padding: the first stage is computed from the loads
    fft_forward_padded<T, PY, TZ, LD, NTHR>(buf, tws, tid, [&](int zl, int y) {
        const int z = z0 + zl;
        return (z < nz && y < ny) ? T1[((size_t)z * nkx + kx) * ny + y] : mk((T)0, (T)0);
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
    for (int idx = tid; idx < NC * PZ; idx += NTHR) {
        const int c = idx / PZ, kz = idx % PZ;
        const int q = qrow[c];
        if (q >= 0) {
            const int fz = kz <= PZ / 2 ? kz : PZ - kz;
            buf[c * LD + sw(kz)] = scale(buf[c * LD + sw(kz)], Q3[(size_t)q + fz]);
        }
    }
    __syncthreads();
    fft_inverse_cropped<T, PZ, NC, LD, NTHR>(buf, tws, tid, [&](int c, int z, cx<T> v) {
        const size_t col = c0 + c;
        if (col < ncol && z < nz) T2[col * nz + z] = v;
    });
}

template <typename T, int PY, int TZ, int NTHR>
__global__ __launch_bounds__(NTHR) void k_pass3_d(cx<T>* __restrict__ T1, const cx<T>* __restrict__ T2,
                                                  const cx<T>* __restrict__ tw, int ny, int nz, int nkx) {
    constexpr int LD = padded(PY) + 1;   // odd row pitch: the TZ transforms start on different banks
    __shared__ cx<T> buf[TZ * LD];
    __shared__ cx<T> tws[PY];
    const int tid = threadIdx.x;
    const int kx = blockIdx.x, z0 = blockIdx.y * TZ;
    stage_twiddles<T, PY, NTHR>(tws, tw, tid);
    for (int idx = tid; idx < TZ * PY; idx += NTHR) {
        const int zl = idx % TZ, ky = idx / TZ;
        const int z = z0 + zl;
        buf[zl * LD + sw(ky)] = z < nz ? T2[((size_t)kx * PY + ky) * nz + z] : mk((T)0, (T)0);
    }
    __syncthreads();
    // only rows y < ny are kept: the last inverse stage writes them directly
    fft_inverse_cropped<T, PY, TZ, LD, NTHR>(buf, tws, tid, [&](int zl, int y, cx<T> v) {
        const int z = z0 + zl;
        if (z < nz && y < ny) T1[((size_t)z * nkx + kx) * ny + y] = v;
    });
}

// z-rows per block of the y-passes: eight in both precisions (in FP32, 16 and 4 rows were slower
// at 128^3: 15.1 / 22.3 and 19.4 / 27.0 us for the forward / inverse pass against 13.4 / 21.1)
template <typename T> constexpr int tz_rows() { return 8; }

template <typename T, int PY>
static void launch3_bd(const Apply3DArgs<T>& a, bool inverse) {
    constexpr int TZ = tz_rows<T>();
    const int nkx = a.PX / 2 + 1;
    dim3 grid(nkx, (a.nz + TZ - 1) / TZ);
    if (!inverse)
        hipLaunchKernelGGL((k_pass3_b<T, PY, TZ, 256>), grid, dim3(256), 0, a.stream, a.T1, a.T2, a.twy, a.ny, a.nz,
                           nkx);
    else
        hipLaunchKernelGGL((k_pass3_d<T, PY, TZ, 256>), grid, dim3(256), 0, a.stream, a.T1, a.T2, a.twy, a.ny, a.nz,
                           nkx);
}

template <typename T, int PZ>
static void launch3_c(const Apply3DArgs<T>& a) {
    constexpr int NC = PZ >= 2048 ? 1 : 2048 / PZ;
    const size_t ncol = (size_t)(a.PX / 2 + 1) * a.PY;
    dim3 grid((unsigned)((ncol + NC - 1) / NC));
    hipLaunchKernelGGL((k_pass3_c<T, PZ, NC, 256>), grid, dim3(256), 0, a.stream, a.T2, a.Q3, a.twz, a.nz, a.PY,
                       ncol);
}

template <typename T>
int apply3d_pass(const Apply3DArgs<T>& a, int which) {
    const int P = which == 2 ? a.PZ : a.PY;
    switch (P) {
#define RTE_C3(PP)                                              \
    case PP:                                                    \
        if (which == 1) launch3_bd<T, PP>(a, false);            \
        else if (which == 3) launch3_bd<T, PP>(a, true);        \
        else launch3_c<T, PP>(a);                               \
        return 0;
        RTE_C3(16) RTE_C3(32) RTE_C3(64) RTE_C3(128) RTE_C3(256) RTE_C3(512)
#undef RTE_C3
    }
    return -1;
}

template int apply3d_pass<float>(const Apply3DArgs<float>&, int);
template int apply3d_pass<double>(const Apply3DArgs<double>&, int);

}  // namespace rte
