// FP64 Krylov vector kernels (host wrappers).
#pragma once
#include "common.h"

#define RTE_KRYLOV_NBLK 1024      // blocks of the fixed-order reductions
#define RTE_KRYLOV_MAXVEC 256     // basis vectors handled by one update/combine

namespace rte {

// out[v] = <V_v, w> for v < nvec (V_v = V + v*ld); out[nvec] = <w, w> if with_norm.
// partial needs (nvec + 1) * RTE_KRYLOV_NBLK doubles.
// active (device int, may be null): the kernels do nothing when *active == 0.
void krylov_dots(const double* V, size_t ld, int nvec, const double* w, size_t n, double* partial,
                 double* out, bool with_norm, hipStream_t st, const int* active = nullptr);
// w -= sum_v h[v] V_v (h on the device); *norm_out = <w, w> after the update.
void krylov_update(double* w, const double* V, size_t ld, int nvec, const double* h, size_t n, double* partial,
                   double* norm_out, hipStream_t st, const int* active = nullptr);
void vec_scale_dev(double* dst, const double* src, const double* a, size_t n, hipStream_t st);
// Device-side Arnoldi bookkeeping for column j (see k_arnoldi in krylov.hip).
// stage 1 also writes the iteration's estimate and (breakdown, non-finite) flags to est_out and
// flags_out (device-visible host memory, may be NULL) for the host's convergence check.
void arnoldi_step(int stage, int j, int m, double* st, double* H, double* cs, double* sn, double* g, double* est,
                  double* inv, int* flags, int reorth, hipStream_t s, double* est_out = nullptr,
                  int* flags_out = nullptr);
// x += sum_v y[v] Z_v (y on the device)
void krylov_combine(double* x, const double* Z, size_t ld, int nvec, const double* y, size_t n, hipStream_t st);
void vec_scale(double* dst, const double* src, double a, size_t n, hipStream_t st);
void vec_fill(double* dst, double a, size_t n, hipStream_t st);
void modes_to_channels(const void* x, double* ch, int L, size_t N, bool one_part, hipStream_t st);
void channels_to_modes(const double* ch, void* y, int L, size_t N, bool one_part, hipStream_t st);
void nonfinite_scan(const double* x, size_t n, int* flag, hipStream_t st);

}  // namespace rte
