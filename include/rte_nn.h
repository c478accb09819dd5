/*
 * rte_nn.h -- the learned right preconditioner of the RTE library (a component the paper does not
 * have).  A stack of 3x3 convolutions (zero "same" padding, bias, ReLU after every layer but the
 * last) maps C = 2L+1 channels through `hidden` channels back to C channels.  As a
 * preconditioner it acts on a coarse grid:
 *
 *     z = v + s P N(R v / s),   R: F x F block average, P: bilinear interpolation from the coarse cell centres,
 *                               s: root-mean-square of v over all cells and channels,
 *
 * and flexible GMRES uses z_j for the Arnoldi vector v_j.  It is trained on pairs (residual r,
 * error e = x* - x) of plain GMRES iterates and pairs (A u, u) of noise u: with x = R r / s and
 * t = R(e - r) / s the network minimises w ||N(x) - t||^2, w = F^2 s^2 / ||e||^2, the coarse part
 * of ||r + s P N(x) - e||^2 / ||e||^2 (exactly so for a block-constant P, for which P R is the
 * orthogonal projector onto block-constant fields; a surrogate for the bilinear P used).
 *
 * Packed parameters (float32): for each layer l = 0..layers-1 the weights W_l[Cout][Cin][3][3]
 * followed by the bias b_l[Cout]; layer 0 is C -> hidden, the last hidden -> C.  Activations are
 * float32 [batch][channels][H][W].  Convolutions run on MFMA with BF16 operands and FP32
 * accumulation (forward and data gradient); weight gradients and Adam are FP32.
 * All pointers are device pointers; calls are asynchronous on the given stream unless noted.
 * Status codes are those of rte.h.
 */
#ifndef RTE_NN_H
#define RTE_NN_H

#include "rte.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rte_nn rte_nn;

/* channels in 1..17 (odd: 2L+1), hidden 16 or 32, layers in 2..8.  Weights are drawn with a
 * seeded He-normal initialiser on the host, biases start at zero; Adam moments start at zero.
 * use_bias = 0 keeps every bias at zero (their gradients are zeroed before each Adam step): the
 * network is then positively homogeneous, N(c x) = c N(x) for c > 0, and so is the
 * preconditioner, M(c v) = c M(v). */
int rte_nn_create(rte_nn** out, int channels, int hidden, int layers, unsigned long long seed,
                  int use_bias, void* hip_stream);
void rte_nn_destroy(rte_nn* nn);
int rte_nn_param_count(const rte_nn* nn, long long* count);
int rte_nn_get_params(rte_nn* nn, float* dst_dev);
int rte_nn_set_params(rte_nn* nn, const float* src_dev);

/* y = N(x) with the BF16 MFMA kernels; x, y: [batch][channels][H][W]. */
int rte_nn_forward(rte_nn* nn, const float* x_dev, int batch, int H, int W, float* y_dev);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops
 * that forbid hipMalloc): y = N(x) exactly as rte_nn_forward computes it, with the intermediate
 * activations in a fixed device array of RTE_NN_SCRATCH_BYTES that the library holds on each GPU
 * (resolved when an rte_nn is created on that GPU) instead of buffers allocated on first use.
 * It calls no hipMalloc, hipFree or other allocating routine.
 *   Limit: batch * max(hidden, channels) * H * W <= RTE_NN_SCRATCH_BYTES / 4 floats for a
 *   2-layer network, half that for deeper ones; larger inputs return RTE_EINVAL before any work.
 *   Every call on one GPU (any rte_nn object) shares that GPU's array: calls that overlap in time
 *   on one GPU, e.g. on two streams, race and give undefined results; calls ordered on one stream
 *   are safe.  Nothing in the array needs to start at zero: every activation is written before it
 *   is read.  Asynchronous on the object's stream. */
#define RTE_NN_SCRATCH_BYTES (32UL << 20)
int rte_nn_forward_noalloc(rte_nn* nn, const float* x_dev, int batch, int H, int W, float* y_dev);

/* loss = mean_b w_b ||N(x_b) - t_b||^2 and its parameter gradient (kept inside the object for
 * rte_nn_adam_step, and copied to grad_dev in the packed layout if not NULL).  Synchronises the
 * stream to return the loss. */
int rte_nn_loss_grad(rte_nn* nn, const float* x_dev, const float* t_dev, const float* w_dev, int batch,
                     int H, int W, double* loss, float* grad_dev);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the last gradient. */
int rte_nn_adam_step(rte_nn* nn, float lr);

/* Minibatch gather for training: dst[i] = src[idx[i]] for i < count, rows of row_len floats
 * (device arrays; idx: device int32, each in [0, nrows); dst may not overlap src).  An index out
 * of range is not checked on the device: the caller draws them in range.  Asynchronous on
 * `hip_stream` (NULL = default stream). */
int rte_nn_gather_rows(const float* src_dev, long long nrows, long long row_len, const int* idx_dev, int count,
                       float* dst_dev, void* hip_stream);

/* Bilinear upsampling of FP64 fields [count][C][hc][wc] to [count][C][ny][nx] at cell centres,
 * used to make the multiscale random fields of the training pairs: the source coordinate of fine
 * cell (y, x) is ((y + 1/2) hc / ny - 1/2, (x + 1/2) wc / nx - 1/2), clamped below at 0, and the
 * value interpolates linearly between the two nearest coarse cells (the upper index clamped to
 * the last cell).  Asynchronous on `hip_stream`. */
int rte_nn_upsample_bilinear(const double* coarse_dev, int count, int C, int hc, int wc, int ny, int nx,
                             double* fine_dev, void* hip_stream);

/* Training pairs from `count` iterates x_j of a solve of A x = b with solution x_star (all FP64
 * channel vectors of the context): r_j = b - A x_j (FP64 apply), e_j = x_star - x_j, written as
 * coarse inputs x_out[j] = R r_j / s_j, targets t_out[j] = R (e_j - r_j) / s_j ([count][C][Hc][Wc],
 * Hc = ny / factor, Wc = nx / factor; factor must divide both), s_j = ||r_j|| / sqrt(C ny nx), and
 * weights w_out[j] = factor^2 s_j^2 / ||e_j||^2.  With b = 0 and x_star = 0 an "iterate" -u gives
 * the pair (r, e) = (A u, u) without a solve. */
int rte_pc_make_pairs(rte_ctx* ctx, const double* b_dev, const double* x_star_dev, const double* x_iters_dev,
                      int count, int factor, float* x_out, float* t_out, float* w_out);

/* The network is attached to a solver context with rte_pc_attach (rte.h).  z = M v with the
 * attached preconditioner on one FP64 channel vector of the context (z may not alias v). */
int rte_pc_apply(rte_ctx* ctx, const double* v_dev, double* z_dev);

#ifdef __cplusplus
}
#endif
#endif /* RTE_NN_H */
