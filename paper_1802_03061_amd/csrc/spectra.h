// Setup: self-cell integrals, twiddle tables and FP64 kernel spectra.
#pragma once
#include <vector>

#include "common.h"

namespace rte {

double self_cell_2d(int m, double h, double mu_t);
double self_cell_3d(double h, double mu_t);
void twiddles(int P, std::vector<double>& re, std::vector<double>& im, int sched = 0);

struct SpectraArgs2D {
    int nx, ny, PX, PY, L;
    double h, mu_t;
    cx<double>* buf0;         // PX*PY scratch
    cx<double>* buf1;         // PX*PY scratch
    const cx<double>* twx;    // FP64 twiddles, PX
    const cx<double>* twy;    // FP64 twiddles, PY
    cx<float>* Qf;            // [2L+1][PX/2+1][PY/2+1] or null
    cx<double>* Qd;           // same shape or null
    hipStream_t stream;
};
int build_spectra_2d(const SpectraArgs2D& a);

struct SpectraArgs3D {
    int nx, ny, nz, PX, PY, PZ;
    double h, mu_t;
    cx<double>* buf0;         // PX*PY*PZ scratch
    cx<double>* buf1;
    const cx<double>* twx;
    const cx<double>* twy;
    const cx<double>* twz;
    float* Qf;                // [PX/2+1][PY/2+1][PZ/2+1] or null
    double* Qd;
    hipStream_t stream;
};
int build_spectrum_3d(const SpectraArgs3D& a);

// 3D anisotropic (real spherical harmonics to degree L, M = (L+1)^2 modes, sh3d.h): for every
// mode pair a <= b the table h^3 kappa(h|o|) Y_a(o/|o|) Y_b(o/|o|) (exact cell integral at o = 0),
// its FP64 FFT, and one real number per octant frequency, R_ab = F_ab / i^(l_b - l_a) scaled by
// 1/(PX PY PZ), at Qf/Qd + pair(a, b) * octant with pair(a, b) = a M - a (a - 1)/2 + (b - a).
// The spectrum F_ab is real when l_a + l_b is even and imaginary otherwise, and reflecting ky or kz
// multiplies it by the two modes' parities (sh3d.h), so the octant and R determine it.
void self_cell_3d_pairs(int L, double h, double mu_t, std::vector<double>& c);   // c[a M + b]
int build_spectra_3d_sh(const SpectraArgs3D& a, int L);
inline size_t sh_pair_index(int a, int b, int M) { return (size_t)a * M - (size_t)a * (a - 1) / 2 + (b - a); }

int fft_rows_f64(cx<double>* data, const cx<double>* tw, int P, size_t rows, bool inverse, hipStream_t st);
void transpose_c128(const cx<double>* in, cx<double>* out, size_t rows, size_t cols, hipStream_t st);

}  // namespace rte
