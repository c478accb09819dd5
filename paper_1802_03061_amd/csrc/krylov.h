// Krylov vector kernels (host wrappers).  Sums and products are FP64; basis vectors (TV) are
// double, or float for the inner solve of the FP32 apply.
#pragma once
#include "common.h"

#define RTE_KRYLOV_NBLK 1024      // blocks of the fixed-order reductions
#define RTE_KRYLOV_MAXVEC 256     // basis vectors handled by one update/combine

namespace rte {

// Arguments of one Arnoldi column on the device (k_arnoldi in krylov.hip): the Hessenberg column
// j of a restart length m, the Givens rotations, the residual vector g and the flags.
struct ArnoldiArgs {
    int stage = 0, j = 0, m = 0, reorth = 0, fused = 0;
    double renorm_tol = 1e-10;
    double* st = nullptr;
    double* H = nullptr;
    double* cs = nullptr;
    double* sn = nullptr;
    double* g = nullptr;
    double* est = nullptr;
    double* inv = nullptr;
    int* flags = nullptr;
    double* est_out = nullptr;
    int* flags_out = nullptr;
};

// Blocks of the dot and update kernels for vectors of n entries (rows of their partial sums).
unsigned krylov_nblk(size_t n);
// out[v] = <V_v, w> for v < nvec (V_v = V + v*ld); out[nvec] = <w, w> if with_norm.  With out NULL
// only the per-block partial sums are written (row v of krylov_nblk(n) entries).
// partial needs (nvec + 1) * RTE_KRYLOV_NBLK doubles.
// active (device int, may be null): the kernels do nothing when *active == 0.
template <typename TV>
void krylov_dots(const TV* V, size_t ld, int nvec, const TV* w, size_t n, double* partial,
                 double* out, bool with_norm, hipStream_t st, const int* active = nullptr);
// w -= sum_v h[v] V_v (h on the device); *norm_out = <w, w> after the update (with norm_out NULL
// only partial row 0 is written).  With stage0 (the fused single pass, h = stage0->st) w is also
// multiplied by the normalising factor, see rescale_arn1.
template <typename TV>
void krylov_update(TV* w, const TV* V, size_t ld, int nvec, const double* h, size_t n, double* partial,
                   double* norm_out, hipStream_t st, const int* active = nullptr, const ArnoldiArgs* stage0 = nullptr);
template <typename TV>
void rescale_arn1(const ArnoldiArgs& t, TV* w, size_t n, const double* partial, int nblk, hipStream_t st);
// y = R^{-1} g for the leading k x k block (k <= RTE_MAX_RESTART) of the rotated Hessenberg
// matrix H (column-major, leading dimension ld) and rotated residual vector g, on the device
// With flags (the device Arnoldi flags), y = 0 instead when flags[2] (non-finite) is set.
void back_solve_dev(const double* H, int ld, const double* g, int k, double* y, hipStream_t st,
                    const int* flags = nullptr);
// g = (g0, 0, ..., 0) with n entries and flags[0..nflags) = 0, on the device
void init_g(double* g, int n, double g0, int* flags, int nflags, hipStream_t st);
// dst = (*a) src
template <typename TV>
void vec_scale_dev(TV* dst, const TV* src, const double* a, size_t n, hipStream_t st);
// out[v] = sum_b partial[v * nblk + b] for v < nout, in a fixed order
void reduce_partials(const double* partial, int nblk, double* out, int nout, hipStream_t st);
// One Arnoldi column on the device (see k_arnoldi in krylov.hip).
void arnoldi_run(const ArnoldiArgs& t, hipStream_t s);
// Fused single pass: krylov_update with stage0 (h = stage0->st) computes the normalising factor
// itself and runs stage 0 of the column; rescale_arn1, given the update's nblk per-block partial
// sums of the new norm, then runs stage 1 and rescales w when the device finds its norm off (see
// arnoldi_dev.h).
// x += sum_v y[v] Z_v (y on the device)
// (nothing when skip is given and skip[2], the device's non-finite flag, is set)
template <typename TV>
void krylov_combine(double* x, const TV* Z, size_t ld, int nvec, const double* y, size_t n, hipStream_t st,
                    const int* skip = nullptr);
// dst = a src (src FP64, dst rounded to TD)
template <typename TD>
void vec_scale(TD* dst, const double* src, double a, size_t n, hipStream_t st);
void vec_fill(double* dst, double a, size_t n, hipStream_t st);
void modes_to_channels(const void* x, double* ch, int L, size_t N, bool one_part, hipStream_t st);
void channels_to_modes(const double* ch, void* y, int L, size_t N, bool one_part, hipStream_t st);
// The same for modes in a real basis (3D spherical harmonics): n = channels x cells entries.
void modes_to_channels_real(const void* x, double* ch, size_t n, bool one_part, hipStream_t st);
void channels_to_modes_real(const double* ch, void* y, size_t n, bool one_part, hipStream_t st);
void nonfinite_scan(const double* x, size_t n, int* flag, hipStream_t st);

}  // namespace rte
