// Learned right preconditioner: 3x3 convolution network kernels (see nn.hip).
#pragma once
#include "apply2d.h"
#include "ctx.h"
#include "krylov.h"

namespace rte {
// z = v + ||v|| N(v / ||v||) on one channel vector (FP64 in/out, BF16 x BF16 -> FP32 inside).
int pc_apply(rte_ctx* c, const double* v, double* z);
void pc_free(rte_ctx* c);

// Flexible GMRES without a stored Z basis: z_j = v_j + s P y_j is formed inside the apply from the
// coarse network output y_j (slot j), with s = 1 / sqrt(nvec) for the unit-norm v_j.
size_t pc_coarse_len(const rte_ctx* c);
int pc_begin_solve(rte_ctx* c, int m);                 // slots for m columns, s in c->pc_st
// v = a w + pool (a = *a_dev, or a_host when a_dev is NULL); v (and the basis) stored as TV.  With g
// given, the same launch sets g = (g0, 0, ...) (gn entries) and clears flags[0..nflags).
template <typename TW, typename TV>
void pc_scale_pool(rte_ctx* c, const TW* w, TV* v, const double* a_dev, double a_host, double* g = nullptr,
                   int gn = 0, double g0 = 0.0, int* flags = nullptr, int nflags = 0);
// The fused single pass of the preconditioned Arnoldi step: w = a (w - sum_{v < nvec} h[v] V_v)
// with h = s0.st and the normalising factor a computed on the device (stage 0 of the column in
// block 0), and the block means of the new w; *norm_out = <w, w> (partial: one double per block,
// pc_update_pool_blocks(c) of them; with norm_out NULL only those are written)
template <typename TV>
void pc_update_pool(rte_ctx* c, TV* w, const TV* V, int nvec, double* partial, double* norm_out,
                    const ArnoldiArgs& s0);
// stage 1 of the fused single pass and, when flagged by the device, w's rescale and new block means
template <typename TV>
void pc_rescale_pool_arn1(rte_ctx* c, const ArnoldiArgs& t, TV* w, const double* partial);
// Stage 1 with the flagged rescale (without new block means) and the network of the block means
// the update wrote, into output slot `slot`, in one launch; usable when pc_rescale_net_ok(c).
bool pc_rescale_net_ok(const rte_ctx* c);
template <typename TV>
int pc_rescale_net(rte_ctx* c, const ArnoldiArgs& t, TV* w, const double* partial, int slot);
// The same launch with the next apply's pass A (FP32, 2D) on its other blocks: the x-transform of
// w alone, scaled per channel by sc, into the FP32 work buffer (packed as `pack`); the apply of
// w is then finished by passes B (adding the coarse correction, CorrB) and C.  With t NULL (the
// first step of a cycle, w = v_0 and its block means already pooled) there is no stage 1: the
// network of v_0 beside its pass A.  Usable when pc_rescale_net_pa_ok(c).
bool pc_rescale_net_pa_ok(const rte_ctx* c);
template <typename TV>
int pc_rescale_net_pa(rte_ctx* c, const ArnoldiArgs* t, TV* w, const double* partial, int slot,
                      const ChanScale& sc, int pack);
int pc_update_pool_blocks(const rte_ctx* c);
int pc_net_slot(rte_ctx* c, int j);                    // Y_j = N(pooled v_j / s)
const float* pc_slot(const rte_ctx* c, int j);
// x += sum_{j < k} y_j V_j + s P sum_j y_j Y_j (basis and coarse network parts in one pass over x);
// nothing when skip is given and skip[2] (the device's non-finite flag) is set
template <typename TV>
void pc_combine(rte_ctx* c, double* x, const TV* V, int k, const double* y_dev, const int* skip = nullptr);
}  // namespace rte
