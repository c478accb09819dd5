// Setup: self-cell integrals, twiddle tables and FP64 kernel spectra.
#pragma once
#include <vector>

#include "common.h"

namespace rte {

double self_cell_2d(int m, double h, double mu_t);
double self_cell_3d(double h, double mu_t);
void twiddles(int P, std::vector<double>& re, std::vector<double>& im);

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

int fft_rows_f64(cx<double>* data, const cx<double>* tw, int P, size_t rows, bool inverse, hipStream_t st);
void transpose_c128(const cx<double>* in, cx<double>* out, size_t rows, size_t cols, hipStream_t st);

}  // namespace rte
