// Host-side interface of the 2D FFT apply kernels.
#pragma once
#include "../../include/rte.h"
#include "common.h"

namespace rte {

enum { APPLY_A = 0, APPLY_KT = 1, APPLY_RESID = 2 };

struct ChanScale {
    double s[2 * RTE_MAX_L + 1];   // per-channel factor applied in pass A (D for operator A, 1 for K~)
};

// The coarse correction added in pass B instead of pass A (FP32 fused pass B, L <= 8).  Pass A
// has transformed the vector alone; pass B adds, to every column before its y-FFT, the
// x-spectrum of the correction cs P y scaled as pass A scales its input.  P is separable (an
// x- then a y-interpolation), so the x-spectrum of row yy of P y_c is (1 - a) G_c[r0] + a G_c[r1],
// with (r0, r1, a) the y-interpolation of row yy and G_c[R](kx) = sum_X y_c[R][X] phi[X][kx],
// phi[X] being the x-spectrum of the fine row of interpolation weights of coarse column X (its
// column 0 holds (phi(0), phi(PX/2)) when the work buffer is packed).
struct CorrB {
    const float* y = nullptr;       // coarse field [C][Hc][Wc], 16-byte aligned, Wc a multiple of 4
    const void* phi = nullptr;      // cx<float> [Wc][nkx], nkx = columns of the work buffer
    const float* coef = nullptr;    // [C] in device memory: pass A's factor of channel c times cs
    int Hc = 0, Wc = 0, F = 1;
};

template <typename T>
struct Apply2DArgs {
    int nx, ny, PX, PY, L, C;
    cx<T>* work;               // work buffer [nbatch][C][NKS][ny], NKS = pack ? PX/2 : PX/2+1
    cx<T>* work2;              // split pass B only: [nbatch][C][NKS][PY] (may be null otherwise)
    const cx<T>* Q;            // quarter spectra [2L+1][PX/2+1][PY/2+1], scaled by 1/(PX PY)
    const cx<T>* twx;          // exp(-2 pi i q/PX), q < PX
    const cx<T>* twy;          // exp(-2 pi i q/PY), q < PY
    hipStream_t stream;
    const cx<T>* twm = nullptr;   // L > 8: stage twiddles of the mode-axis FFT (length mode_fft_len(L))
    const cx<T>* twy1 = nullptr;  // y twiddles in the radix-32 schedule (fft.h, schedule 1)
    const cx<T>* twyh = nullptr;  // stage twiddles of length PY/2 (pass B split in halves)
    int pack = 0;              // 1: x-frequencies 0 and PX/2 share column 0 of the work buffer
    int var[3] = {0, 0, 0};    // kernel variant of passes A, B, C (see apply2d_variant_count)
    // The input's channels other than channel 0 are zero and pass A ran for channel 0 alone, so
    // pass B reads channel 0 only (split form: forward y-FFTs of channel 0 only; fused form: the
    // other channels' spectra start as zeros without loads).  The right-hand side K~ f.
    int single_in = 0;
    // Optional coarse correction (operator A, one batch entry): the input of the apply is taken as
    // x + cs P y, y = corr[C][ny/cF][nx/cF] (FP32), P = bilinear interpolation from the coarse
    // cell centres, clamped -- the flexible-GMRES vector z = v + s P N(R v / s) formed on the fly.
    const float* corr = nullptr;
    int cF = 1;
    double cs = 0.0;
    // Set (bcorr.y non-null): pass B adds the correction's x-spectrum (see CorrB); pass A is not
    // run by apply2d_from_b.
    CorrB bcorr;
};

// Kernel variants (same arithmetic, different tiling; results agree up to rounding):
//   passes A and C (PX >= 128): row tiles of 16, 8, 32 or 4 rows (FP32) / 8, 4, 16 or 2 rows (FP64)
//   pass B, fused form (PY >= 128): default threads and FFT grouping, 1024 threads with groups of
//   4 transforms (FP32 only), 256 threads, the register-resident form (FP32, 5+ channels), the
//   radix-32 schedule (PY >= 256), and all of a block's transforms in one FFT stage group where
//   the default grouping splits them (FP32, PY = 1024, L >= 6)
//   pass B, split form (FP64 with L > 4): three kernels through the full-length buffer, the
//   column split in halves, or the coupling fused with the inverse y-FFTs by channel groups
//   pass B, L > 8: the coupling as a mode-axis FFT or as a register-blocked direct sum
// Number of variants of `pass` (0 = A, 1 = B, 2 = C) for this shape and precision.
template <typename T>
int apply2d_variant_count(int pass, int L, int PX, int PY);

// One isotropic problem (C = 1) of a batched apply.  Pass A reads in (+ j * stride when jin is
// set, j read from the device), pass C writes out (+ (j + 1) * stride when jout is set) and reads
// in again (operator A, residual) and bvec (residual).  The x-frequencies 0 and PX/2 are always
// packed into column 0 of the work buffer.
template <typename T>
struct BatchProb {
    int nx, ny, PX, PY;
    double s;                  // pass-A factor: mu_s sigma_0 for A and the residual, 1 for K~
    cx<T>* work;               // [PX/2][ny]
    const cx<T>* Q;            // quarter spectrum [PX/2+1][PY/2+1], scaled by 1/(PX PY)
    const cx<T>* twx;
    const cx<T>* twy;
    const double* in;
    double* out;
    const double* bvec;
    size_t stride;
    int jin, jout;
};

// Batched passes over a list of (problem index, tile) items whose problems all have this PX
// (passes A, C: tiles of apply2d_batch_rows(var) rows) or this PY (pass B: groups of
// apply2d_batch_cols(PY, var) columns).  act[p] == 0 skips problem p (act may be NULL); dj (may be
// NULL) points to the Krylov column index j.  Variants (same arithmetic, different tiling; -1 when
// var is out of range): passes A and C share the row tile (the single-problem row tiles, padded
// x >= 128); pass B takes the fused form's columns per block with its threads or half of them, or
// twice or half the columns (padded y >= 128).
template <typename T>
int apply2d_batch_row_variants(int PX);
template <typename T>
int apply2d_batch_rows(int var);
template <typename T>
int apply2d_batch_col_variants(int PY);
template <typename T>
int apply2d_batch_cols(int PY, int var);
template <typename T>
int apply2d_batch_pass_a(int PX, const BatchProb<T>* probs, const int2* items, int nitems, const int* act,
                         const int* dj, int var, hipStream_t st);
template <typename T>
int apply2d_batch_pass_b(int PY, const BatchProb<T>* probs, const int2* items, int nitems, const int* act, int var,
                         hipStream_t st);
template <typename T>
int apply2d_batch_pass_c(int PX, const BatchProb<T>* probs, const int2* items, int nitems, const int* act,
                         const int* dj, int mode, int var, hipStream_t st);

// y = x - K~ D x (APPLY_A), K~ x (APPLY_KT) or b - (x - K~ D x) (APPLY_RESID) on nbatch channel
// vectors [nbatch][C][ny][nx] stored as TV (float64, or float32 with T = float; b is float64),
// computed with FFTs in precision T.
template <typename T, typename TV>
int apply2d(const Apply2DArgs<T>& a, const TV* x, const double* b, TV* y, int mode,
            const ChanScale& sc, int nbatch);
template <typename T, typename TV>
int apply2d_pass_a(const Apply2DArgs<T>& a, const TV* x, const ChanScale& sc, int nbatch);
template <typename T>
int apply2d_pass_b(const Apply2DArgs<T>& a, int nbatch);
// True when pass B for (L, PY) in precision T needs the work2 buffer.
template <typename T>
bool apply2d_needs_work2(int L, int PY);
// Whether the 2D work buffer must be unpacked (x-frequencies 0 and PX/2 in columns of their own
// instead of sharing column 0) for pass B of this (precision, L, PY) and pass-B variant.
template <typename T>
bool apply2d_unpacked(int L, int PY, int var_b);
template <typename T, typename TV>
int apply2d_pass_c(const Apply2DArgs<T>& a, const TV* x, const double* b, TV* y, int mode,
                   int nbatch);
// Whether pass B of this (precision, L, PY, pass-B variant) can add the coarse correction
// (CorrB): the FP32 fused form in LDS, not the register-resident variant.
template <typename T>
bool apply2d_b_corr_ok(int L, int PY, int var_b);
// Passes B and C of y = A (x + cs P y) for one batch entry, pass A having already written the
// x-spectrum of the scaled x alone into a.work; a.bcorr and a.corr describe the correction.
template <typename T, typename TV>
int apply2d_from_b(const Apply2DArgs<T>& a, const TV* x, TV* y);

}  // namespace rte
