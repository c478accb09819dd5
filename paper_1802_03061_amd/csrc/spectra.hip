// Precompute of the kernel spectra (the T_pre step of Sec. 2.4; the FFT of the kernel table that
// the convolution applies of Sec. 2.3.1 and 3.3.1 multiply by).  Everything here runs in FP64.
//
// 2D: for m = 0..2L the table K_m[oy][ox] on the PY x PX periodic grid holds
//       h^2 exp(-mu_t r)/(2 pi r) exp(i m theta),  r = h|o|, theta = polar angle of o,
// for offsets |ox| < nx, |oy| < ny (stored at o mod P), the exact self-cell integral c_m at o = 0
// and zero elsewhere (Sec. 2.3 Nystrom rule; circulant embedding of Sec. 2.3.1).  exp(i m theta)
// is formed as ((ox + i oy)/|o|)^m by repeated complex multiplication.  Its 2D FFT is kept on the
// quarter kx <= PX/2, ky <= PY/2 (the rest follows from the mirror symmetries), scaled by
// 1/(PX PY) so the apply's inverse FFTs need no normalisation.
// 3D (isotropic): K[oz][oy][ox] = h^3 exp(-mu_t r)/(4 pi r^2) is real and even in every axis, so its
// spectrum is real and even; the octant kx <= PX/2, ky <= PY/2, kz <= PZ/2 is kept.
#include <cmath>
#include <vector>

#include "fft.h"
#include "sh3d.h"
#include "spectra.h"

namespace rte {

// ------------------------------------------------------------------ host: quadrature -----------
// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on the three-term recurrence.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            // p1 = P_n(z), p0 = P_{n-1}(z)
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// (1 - exp(-mu R))/mu with its mu -> 0 limit.
static inline double one_minus_exp_over(double mu, double R) {
    return mu == 0.0 ? R : -std::expm1(-mu * R) / mu;
}

// Integral over the square cell [-h/2, h/2]^2 of exp(-mu_t r)/(2 pi r) exp(i m theta).  Radially
// exact; the angular integral reduces by the square's symmetry group to
// (4/pi) int_0^{pi/4} cos(m t) (1 - exp(-mu_t h/(2 cos t)))/mu_t dt when 4 | m, else 0.
double self_cell_2d(int m, double h, double mu_t) {
    if (m % 4 != 0) return 0.0;
    const double pi = 3.14159265358979323846;
    std::vector<double> x, w;
    gauss_legendre(64, x, w);
    double s = 0.0;
    for (size_t i = 0; i < x.size(); ++i) {
        const double t = 0.125 * pi * (x[i] + 1.0);     // [0, pi/4]
        const double R = 0.5 * h / std::cos(t);
        s += 0.125 * pi * w[i] * std::cos(m * t) * one_minus_exp_over(mu_t, R);
    }
    return 4.0 / pi * s;
}

// Integral over the cube [-h/2, h/2]^3 of exp(-mu_t r)/(4 pi r^2): the six faces seen from the
// centre, each face point (x, y, a) at distance rho contributing solid angle a/rho^3 dx dy, so
// (6/(4 pi)) int_{[-a,a]^2} (1 - exp(-mu_t rho))/mu_t a/rho^3 dx dy with a = h/2.
double self_cell_3d(double h, double mu_t) {
    const double pi = 3.14159265358979323846;
    const double a = 0.5 * h;
    std::vector<double> x, w;
    gauss_legendre(48, x, w);
    double s = 0.0;
    for (size_t i = 0; i < x.size(); ++i) {
        const double xi = 0.5 * a * (x[i] + 1.0);
        for (size_t j = 0; j < x.size(); ++j) {
            const double yj = 0.5 * a * (x[j] + 1.0);
            const double rho = std::sqrt(xi * xi + yj * yj + a * a);
            s += 0.25 * a * a * w[i] * w[j] * one_minus_exp_over(mu_t, rho) * a / (rho * rho * rho);
        }
    }
    return 6.0 / (4.0 * pi) * 4.0 * s;
}

// c[a M + b] = integral over the cube [-h/2, h/2]^3 of exp(-mu_t r)/(4 pi r^2) Y_a(w) Y_b(w), w the
// direction of the point from the centre: the radial part exactly, the sphere split by the six
// faces (face point p with |p_axis| = a: R = |p|, solid angle a/|p|^3 dA), each face integrated by
// Gauss-Legendre on its four quarters.
void self_cell_3d_pairs(int L, double h, double mu_t, std::vector<double>& c) {
    const int M = sh_modes(L);
    const double pi = 3.14159265358979323846;
    const double a = 0.5 * h;
    std::vector<double> x, w;
    gauss_legendre(48, x, w);
    std::vector<double> s, ws;          // nodes and weights on [-a, a], four quarters in two halves
    for (size_t i = 0; i < x.size(); ++i) { s.push_back(-0.5 * a * (x[i] + 1.0)); ws.push_back(0.5 * a * w[i]); }
    for (size_t i = 0; i < x.size(); ++i) { s.push_back(0.5 * a * (x[i] + 1.0)); ws.push_back(0.5 * a * w[i]); }
    c.assign((size_t)M * M, 0.0);
    std::vector<double> Y(M);
    for (int axis = 0; axis < 3; ++axis)
        for (int sg = -1; sg <= 1; sg += 2)
            for (size_t i = 0; i < s.size(); ++i)
                for (size_t j = 0; j < s.size(); ++j) {
                    double p[3];
                    p[axis] = sg * a;
                    p[(axis + 1) % 3] = s[i];
                    p[(axis + 2) % 3] = s[j];
                    const double rho = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
                    const double wgt = ws[i] * ws[j] * one_minus_exp_over(mu_t, rho) * a / (rho * rho * rho) / (4.0 * pi);
                    for (int q = 0; q < M; ++q) Y[q] = real_sh(q, p[0] / rho, p[1] / rho, p[2] / rho);
                    for (int q = 0; q < M; ++q)
                        for (int r = 0; r < M; ++r) c[(size_t)q * M + r] += wgt * Y[q] * Y[r];
                }
}

// The twiddle table of the length-P LDS FFT (fft.h) with radix schedule `sched`, in its per-stage
// layout: for every Stockham stage after the first (sub-transform length NS, radix R), the factors
// exp(-2 pi i k r / (NS R)) for k < NS, r = 1..R-1 at stage_tw_offset(P, NS, sched) + k (R - 1) + (r - 1).  The angle is computed
// in long double from the exact integer fraction (k r mod NS R) / (NS R), rounded to FP64, with
// the quarter points exact.
void twiddles(int P, std::vector<double>& re, std::vector<double>& im, int sched) {
    re.assign(P, 0.0);
    im.assign(P, 0.0);
    const long double pi = 3.141592653589793238462643383279502884L;
    int ns = 1, off = 0;
    while (ns < P) {
        const int R = fft_radix(P, ns, sched);
        if (ns > 1) {
            const int S = ns * R;
            for (int k = 0; k < ns; ++k)
                for (int r = 1; r < R; ++r) {
                    const int q = (k * r) % S;
                    double cr, ci;
                    if (4 * q == 0) { cr = 1; ci = 0; }
                    else if (4 * q == S) { cr = 0; ci = -1; }
                    else if (4 * q == 2 * S) { cr = -1; ci = 0; }
                    else if (4 * q == 3 * S) { cr = 0; ci = 1; }
                    else {
                        const long double ang = -2.0L * pi * (long double)q / (long double)S;
                        cr = (double)std::cos(ang);
                        ci = (double)std::sin(ang);
                    }
                    re[off + k * (R - 1) + (r - 1)] = cr;
                    im[off + k * (R - 1) + (r - 1)] = ci;
                }
            off += ns * (R - 1);
        }
        ns *= R;
    }
}

// ------------------------------------------------------------------ device kernels -------------
__global__ void k_table_2d(cx<double>* __restrict__ out, int PX, int PY, int nx, int ny, int m, double h,
                           double mu_t, double c_self) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)PX * PY) return;
    const int ix = (int)(idx % PX), iy = (int)(idx / PX);
    const int ox = ix < PX / 2 ? ix : ix - PX;
    const int oy = iy < PY / 2 ? iy : iy - PY;
    cx<double> v = mk(0.0, 0.0);
    if (ox > -nx && ox < nx && oy > -ny && oy < ny) {
        if (ox == 0 && oy == 0) {
            v = mk(c_self, 0.0);
        } else {
            const double rr = sqrt((double)ox * ox + (double)oy * oy);
            const double r = h * rr;
            const double mag = h * h * exp(-mu_t * r) / (2.0 * 3.14159265358979323846 * r);
            const cx<double> e1 = mk((double)ox / rr, (double)oy / rr);
            cx<double> e = mk(1.0, 0.0);
            for (int k = 0; k < m; ++k) e = e * e1;
            v = scale(e, mag);
        }
    }
    out[idx] = v;
}

__global__ void k_table_3d(cx<double>* __restrict__ out, int PX, int PY, int PZ, int nx, int ny, int nz,
                           double h, double mu_t, double c_self) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)PX * PY * PZ) return;
    const int ix = (int)(idx % PX);
    const int iy = (int)((idx / PX) % PY);
    const int iz = (int)(idx / ((size_t)PX * PY));
    const int ox = ix < PX / 2 ? ix : ix - PX;
    const int oy = iy < PY / 2 ? iy : iy - PY;
    const int oz = iz < PZ / 2 ? iz : iz - PZ;
    double v = 0.0;
    if (ox > -nx && ox < nx && oy > -ny && oy < ny && oz > -nz && oz < nz) {
        if (ox == 0 && oy == 0 && oz == 0) {
            v = c_self;
        } else {
            const double r2 = h * h * ((double)ox * ox + (double)oy * oy + (double)oz * oz);
            v = h * h * h * exp(-mu_t * sqrt(r2)) / (4.0 * 3.14159265358979323846 * r2);
        }
    }
    out[idx] = mk(v, 0.0);
}

// Table of the mode pair (a, b): h^3 exp(-mu_t r)/(4 pi r^2) Y_a(o/|o|) Y_b(o/|o|), c_self at o = 0.
__global__ void k_table_3d_pair(cx<double>* __restrict__ out, int PX, int PY, int PZ, int nx, int ny, int nz,
                                double h, double mu_t, double c_self, int a, int b) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)PX * PY * PZ) return;
    const int ix = (int)(idx % PX);
    const int iy = (int)((idx / PX) % PY);
    const int iz = (int)(idx / ((size_t)PX * PY));
    const int ox = ix < PX / 2 ? ix : ix - PX;
    const int oy = iy < PY / 2 ? iy : iy - PY;
    const int oz = iz < PZ / 2 ? iz : iz - PZ;
    double v = 0.0;
    if (ox > -nx && ox < nx && oy > -ny && oy < ny && oz > -nz && oz < nz) {
        if (ox == 0 && oy == 0 && oz == 0) {
            v = c_self;
        } else {
            const double rr = sqrt((double)ox * ox + (double)oy * oy + (double)oz * oz);
            const double r = h * rr;
            const double ux = ox / rr, uy = oy / rr, uz = oz / rr;
            v = h * h * h * exp(-mu_t * r) / (4.0 * 3.14159265358979323846 * r * r) * real_sh(a, ux, uy, uz) *
                real_sh(b, ux, uy, uz);
        }
    }
    out[idx] = mk(v, 0.0);
}

// In-place FFT of `rows` contiguous rows of length P.
template <typename T, int P, bool INV>
__global__ __launch_bounds__(256) void k_fft_rows(cx<T>* __restrict__ data, const cx<T>* __restrict__ tw,
                                                  size_t rows) {
    constexpr int RPB = P >= 2048 ? 1 : 2048 / P;
    constexpr int LD = padded(P) + 1;
    __shared__ cx<T> buf[RPB * LD];
    __shared__ cx<T> tws[P];
    const size_t r0 = (size_t)blockIdx.x * RPB;
    const int tid = threadIdx.x;
    stage_twiddles<T, P, 256>(tws, tw, tid);
    for (int idx = tid; idx < RPB * P; idx += 256) {
        const size_t r = r0 + idx / P;
        buf[(idx / P) * LD + sw(idx % P)] = r < rows ? data[r * P + idx % P] : mk((T)0, (T)0);
    }
    __syncthreads();
    block_fft<T, P, RPB, LD, 256, INV>(buf, tws, tid);
    for (int idx = tid; idx < RPB * P; idx += 256) {
        const size_t r = r0 + idx / P;
        if (r < rows) data[r * P + idx % P] = buf[(idx / P) * LD + sw(idx % P)];
    }
}

// out[c][r] = in[r][c] for a rows x cols matrix, 32 x 32 tiles through LDS.
template <typename E>
__global__ __launch_bounds__(256) void k_transpose(const E* __restrict__ in, E* __restrict__ out, size_t rows,
                                                   size_t cols) {
    __shared__ E tile[32][33];
    const size_t c0 = (size_t)blockIdx.x * 32, r0 = (size_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8) {
        const size_t r = r0 + k, c = c0 + tx;
        if (r < rows && c < cols) tile[k][tx] = in[r * cols + c];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const size_t c = c0 + k, r = r0 + tx;
        if (r < rows && c < cols) out[c * rows + r] = tile[tx][k];
    }
}

// Q[m][kx][fy] = s * F[kx][fy] (F is [PX][PY] after the y-transform), fy <= PY/2, kx <= PX/2.
__global__ void k_extract_quarter(const cx<double>* __restrict__ F, cx<float>* __restrict__ Qf,
                                  cx<double>* __restrict__ Qd, int PX, int PY, int m, double s) {
    const int KH = PY / 2 + 1, NK = PX / 2 + 1;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)NK * KH) return;
    const int kx = (int)(idx / KH), fy = (int)(idx % KH);
    const cx<double> v = scale(F[(size_t)kx * PY + fy], s);
    const size_t o = (size_t)m * NK * KH + idx;
    if (Qd) Qd[o] = v;
    if (Qf) Qf[o] = cvt<float>(v);
}

// 3D octant: data is [PY][PX][PZ] after three transforms; Q3[kx][ky][kz] = s Re data.
__global__ void k_extract_octant(const cx<double>* __restrict__ F, float* __restrict__ Qf, double* __restrict__ Qd,
                                 int PX, int PY, int PZ, double s) {
    const int HX = PX / 2 + 1, HY = PY / 2 + 1, HZ = PZ / 2 + 1;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)HX * HY * HZ) return;
    const int kz = (int)(idx % HZ);
    const int ky = (int)((idx / HZ) % HY);
    const int kx = (int)(idx / ((size_t)HZ * HY));
    const double v = s * F[((size_t)ky * PX + kx) * PZ + kz].re;
    if (Qd) Qd[idx] = v;
    if (Qf) Qf[idx] = (float)v;
}

// Octant of a mode pair's spectrum: data is [PY][PX][PZ] after three transforms;
// Q[kx][ky][kz] = s * Re(F / i^q), i.e. s times Re F, Im F, -Re F, -Im F for q = 0, 1, 2, 3.
__global__ void k_extract_octant_pair(const cx<double>* __restrict__ F, float* __restrict__ Qf,
                                      double* __restrict__ Qd, int PX, int PY, int PZ, double s, int q) {
    const int HX = PX / 2 + 1, HY = PY / 2 + 1, HZ = PZ / 2 + 1;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)HX * HY * HZ) return;
    const int kz = (int)(idx % HZ);
    const int ky = (int)((idx / HZ) % HY);
    const int kx = (int)(idx / ((size_t)HZ * HY));
    const cx<double> f = F[((size_t)ky * PX + kx) * PZ + kz];
    const double v = s * (q == 0 ? f.re : q == 1 ? f.im : q == 2 ? -f.re : -f.im);
    if (Qd) Qd[idx] = v;
    if (Qf) Qf[idx] = (float)v;
}

// ------------------------------------------------------------------ host drivers ---------------
template <typename T, bool INV>
static int fft_rows_dispatch(cx<T>* data, const cx<T>* tw, int P, size_t rows, hipStream_t st) {
    const int rpb = P >= 2048 ? 1 : 2048 / P;
    const unsigned nb = (unsigned)((rows + rpb - 1) / rpb);
    switch (P) {
#define RTE_FR(PP) case PP: hipLaunchKernelGGL((k_fft_rows<T, PP, INV>), dim3(nb), dim3(256), 0, st, data, tw, rows); return 0;
        RTE_FR(16) RTE_FR(32) RTE_FR(64) RTE_FR(128) RTE_FR(256) RTE_FR(512) RTE_FR(1024)
#undef RTE_FR
    }
    return -1;
}

int fft_rows_f64(cx<double>* data, const cx<double>* tw, int P, size_t rows, bool inverse, hipStream_t st) {
    return inverse ? fft_rows_dispatch<double, true>(data, tw, P, rows, st)
                   : fft_rows_dispatch<double, false>(data, tw, P, rows, st);
}

void transpose_c128(const cx<double>* in, cx<double>* out, size_t rows, size_t cols, hipStream_t st) {
    dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
    hipLaunchKernelGGL((k_transpose<cx<double>>), grid, dim3(256), 0, st, in, out, rows, cols);
}

int build_spectra_2d(const SpectraArgs2D& a) {
    const size_t NP = (size_t)a.PX * a.PY;
    const unsigned nb = (unsigned)((NP + 255) / 256);
    const int NK = a.PX / 2 + 1, KH = a.PY / 2 + 1;
    const double s = 1.0 / ((double)a.PX * a.PY);
    for (int m = 0; m <= 2 * a.L; ++m) {
        const double c = self_cell_2d(m, a.h, a.mu_t);
        hipLaunchKernelGGL(k_table_2d, dim3(nb), dim3(256), 0, a.stream, a.buf0, a.PX, a.PY, a.nx, a.ny, m, a.h,
                           a.mu_t, c);
        if (fft_rows_f64(a.buf0, a.twx, a.PX, a.PY, false, a.stream)) return -1;
        transpose_c128(a.buf0, a.buf1, a.PY, a.PX, a.stream);   // -> [PX][PY]
        if (fft_rows_f64(a.buf1, a.twy, a.PY, NK, false, a.stream)) return -1;
        const unsigned nq = (unsigned)(((size_t)NK * KH + 255) / 256);
        hipLaunchKernelGGL(k_extract_quarter, dim3(nq), dim3(256), 0, a.stream, a.buf1, a.Qf, a.Qd, a.PX, a.PY, m,
                           s);
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int build_spectrum_3d(const SpectraArgs3D& a) {
    const size_t NP = (size_t)a.PX * a.PY * a.PZ;
    const unsigned nb = (unsigned)((NP + 255) / 256);
    const double c = self_cell_3d(a.h, a.mu_t);
    hipLaunchKernelGGL(k_table_3d, dim3(nb), dim3(256), 0, a.stream, a.buf0, a.PX, a.PY, a.PZ, a.nx, a.ny, a.nz,
                       a.h, a.mu_t, c);
    // [PZ][PY][PX]: x-transform, rotate to [PX][PZ][PY], y-transform, rotate to [PY][PX][PZ], z-transform
    if (fft_rows_f64(a.buf0, a.twx, a.PX, (size_t)a.PZ * a.PY, false, a.stream)) return -1;
    transpose_c128(a.buf0, a.buf1, (size_t)a.PZ * a.PY, a.PX, a.stream);
    if (fft_rows_f64(a.buf1, a.twy, a.PY, (size_t)a.PX * a.PZ, false, a.stream)) return -1;
    transpose_c128(a.buf1, a.buf0, (size_t)a.PX * a.PZ, a.PY, a.stream);
    if (fft_rows_f64(a.buf0, a.twz, a.PZ, (size_t)a.PY * a.PX, false, a.stream)) return -1;
    const size_t no = (size_t)(a.PX / 2 + 1) * (a.PY / 2 + 1) * (a.PZ / 2 + 1);
    const double s = 1.0 / ((double)a.PX * a.PY * a.PZ);
    hipLaunchKernelGGL(k_extract_octant, dim3((unsigned)((no + 255) / 256)), dim3(256), 0, a.stream, a.buf0, a.Qf,
                       a.Qd, a.PX, a.PY, a.PZ, s);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int build_spectra_3d_sh(const SpectraArgs3D& a, int L) {
    const int M = sh_modes(L);
    std::vector<double> cself;
    self_cell_3d_pairs(L, a.h, a.mu_t, cself);
    const size_t NP = (size_t)a.PX * a.PY * a.PZ;
    const unsigned nb = (unsigned)((NP + 255) / 256);
    const size_t no = (size_t)(a.PX / 2 + 1) * (a.PY / 2 + 1) * (a.PZ / 2 + 1);
    const double s = 1.0 / ((double)a.PX * a.PY * a.PZ);
    for (int p = 0; p < M; ++p)
        for (int q = p; q < M; ++q) {
            hipLaunchKernelGGL(k_table_3d_pair, dim3(nb), dim3(256), 0, a.stream, a.buf0, a.PX, a.PY, a.PZ, a.nx,
                               a.ny, a.nz, a.h, a.mu_t, cself[(size_t)p * M + q], p, q);
            if (fft_rows_f64(a.buf0, a.twx, a.PX, (size_t)a.PZ * a.PY, false, a.stream)) return -1;
            transpose_c128(a.buf0, a.buf1, (size_t)a.PZ * a.PY, a.PX, a.stream);
            if (fft_rows_f64(a.buf1, a.twy, a.PY, (size_t)a.PX * a.PZ, false, a.stream)) return -1;
            transpose_c128(a.buf1, a.buf0, (size_t)a.PX * a.PZ, a.PY, a.stream);
            if (fft_rows_f64(a.buf0, a.twz, a.PZ, (size_t)a.PY * a.PX, false, a.stream)) return -1;
            const size_t off = sh_pair_index(p, q, M) * no;
            const int ph = (((sh_degree(q) - sh_degree(p)) % 4) + 4) % 4;
            hipLaunchKernelGGL(k_extract_octant_pair, dim3((unsigned)((no + 255) / 256)), dim3(256), 0, a.stream,
                               a.buf0, a.Qf ? a.Qf + off : nullptr, a.Qd ? a.Qd + off : nullptr, a.PX, a.PY, a.PZ, s,
                               ph);
        }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace rte
