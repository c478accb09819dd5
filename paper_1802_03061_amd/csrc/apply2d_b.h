// Per-L entry points of pass B (one translation unit per L, see apply2d_b.hip).
#pragma once
#include "apply2d.h"

namespace rte {
#define RTE_DECL_PASSB(L)                                                     \
    template <typename T> int pass_b_L##L(const Apply2DArgs<T>& a, int nbatch); \
    template <typename T> bool pass_b_split_L##L(int PY);                         \
    template <typename T> int pass_b_variants_L##L(int PY);                       \
    template <typename T> bool pass_b_unpacked_L##L(int PY, int var);
RTE_DECL_PASSB(0) RTE_DECL_PASSB(1) RTE_DECL_PASSB(2) RTE_DECL_PASSB(3) RTE_DECL_PASSB(4)
RTE_DECL_PASSB(5) RTE_DECL_PASSB(6) RTE_DECL_PASSB(7) RTE_DECL_PASSB(8)
#undef RTE_DECL_PASSB
}  // namespace rte
