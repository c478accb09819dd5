// Per-L entry points of pass B (one translation unit per L, see apply2d_b.hip).
#pragma once
#include "apply2d.h"

namespace rte {
#define RTE_DECL_PASSB(L)                                                     \
    template <typename T> int pass_b_L##L(const Apply2DArgs<T>& a, int nbatch); \
    template <typename T> bool pass_b_split_L##L(int PY);                         \
    template <typename T> int pass_b_variants_L##L(int PY);                       \
    template <typename T> bool pass_b_unpacked_L##L(int PY, int var);          \
    template <typename T> bool pass_b_corr_ok_L##L(int PY, int var);
RTE_DECL_PASSB(0) RTE_DECL_PASSB(1) RTE_DECL_PASSB(2) RTE_DECL_PASSB(3) RTE_DECL_PASSB(4)
RTE_DECL_PASSB(5) RTE_DECL_PASSB(6) RTE_DECL_PASSB(7) RTE_DECL_PASSB(8)
#undef RTE_DECL_PASSB

// Pass B for L > 8 (split form, unpacked work buffer, work2 required; apply2d_bm.hip): variant 0
// couples the modes by an FFT along the mode axis (twm: twiddles of length mode_fft_len(L)),
// variant 1 by the direct Toeplitz sum.
constexpr int PASSB_FUSED_MAX_L = 8;
inline int mode_fft_len(int L) { int p = 1; while (p < 4 * L + 1) p <<= 1; return p; }
template <typename T> int pass_b_large(const Apply2DArgs<T>& a, int nbatch);
}  // namespace rte
