// Learned right preconditioner: 3x3 convolution network kernels (see nn.hip).
#pragma once
#include "ctx.h"

namespace rte {
// z = v + ||v|| N(v / ||v||) on one channel vector (FP64 in/out, BF16 x BF16 -> FP32 inside).
int pc_apply(rte_ctx* c, const double* v, double* z);
void pc_free(rte_ctx* c);
}  // namespace rte
