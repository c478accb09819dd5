// The opaque context behind rte_ctx (one problem: grid, coefficients, spectra, work buffers,
// Krylov basis and the optional learned preconditioner).
#pragma once
#include <vector>

#include "../../include/rte.h"
#include "common.h"

struct rte_ctx {
    unsigned long long id = 0;   // unique per context in the process (cached batch plans key on it)
    int dim = 2, nx = 0, ny = 0, nz = 1, L = 0, C = 1, M = 1, prec = RTE_PREC_FP64;
    double h = 0, mu_a = 0, mu_s = 0, mu_t = 0;
    std::vector<double> sigma;
    int PX = 0, PY = 0, PZ = 1;
    size_t ncell = 0, nvec = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    double t_setup_ms = 0;
    // kernel spectra: 2D quarter [C][PX/2+1][PY/2+1]; 3D octant [PX/2+1][PY/2+1][PZ/2+1]
    rte::cx<float>* Qf = nullptr;
    rte::cx<double>* Qd = nullptr;
    float* Q3f = nullptr;
    double* Q3d = nullptr;
    rte::cx<float>* twf[3] = {nullptr, nullptr, nullptr};
    rte::cx<double>* twd[3] = {nullptr, nullptr, nullptr};
    // 2D: y twiddles in the radix-32 schedule (pass-B variant), and of length PY/2 (pass B in halves)
    rte::cx<float>* twy1f = nullptr;
    rte::cx<double>* twy1d = nullptr;
    rte::cx<float>* twyhf = nullptr;
    rte::cx<double>* twyhd = nullptr;
    // 2D with L > 8: stage twiddles of the FFT along the mode axis (pass-B coupling)
    rte::cx<float>* twmf = nullptr;
    rte::cx<double>* twmd = nullptr;
    // FFT work buffers (2D: T and the split pass-B buffer; 3D: T1 and T2)
    rte::cx<float>* wf = nullptr;
    rte::cx<float>* wf2 = nullptr;
    rte::cx<double>* wd = nullptr;
    rte::cx<double>* wd2 = nullptr;
    // solver vectors (channel layout, FP64)
    double* xv = nullptr;
    double* rv = nullptr;
    double* bv = nullptr;
    double* t0 = nullptr;   // 2 vectors
    double* t1 = nullptr;   // 2 vectors
    int work_nb = 2;        // batch entries (right-hand sides) the FFT work buffers hold
    // several right-hand sides sharing the operator (rte_solve_multi): stacked x, r, b
    int multi_nb = 0;
    double* xm = nullptr;
    double* rm = nullptr;
    double* bm = nullptr;
    int* dflag = nullptr;
    // Krylov basis
    int krylov_m = 0;
    size_t krylov_n = 0;        // vector length the basis is sized for (a multiple of nvec)
    bool krylov_z = false;
    size_t krylov_vbytes = 0;   // bytes per basis entry the allocation was sized for
    // (m + 1) basis vectors of nvec entries: double, or float when an FP32 context solves with
    // opts.basis_fp32 (the inner solve then keeps its basis in the apply's precision)
    unsigned char* V = nullptr;
    double* Z = nullptr;
    double* partial = nullptr;
    double* dsmall = nullptr;
    double* arn = nullptr;      // device Arnoldi state (H, Givens, g, estimates)
    int* arn_flags = nullptr;   // [second pass, breakdown, non-finite, spare]
    double* hpipe = nullptr;    // pinned per-iteration residual estimates
    int* hpipe_flags = nullptr; // pinned per-iteration (breakdown, non-finite)
    double* hpipe_dev = nullptr;     // device addresses of the two (mapped) host arrays above
    int* hpipe_flags_dev = nullptr;
    rte_solve_opts opts{};
    // kernel variants of the 2D apply passes A, B, C (FP32 and FP64 applies), set by the autotuner
    int varf[3] = {0, 0, 0};
    int vard[3] = {0, 0, 0};
    // 3D: variants of passes A (x-FFT row tiles), B, C, D, E (inverse x-FFT row tiles)
    int var3f[5] = {0, 0, 0, 0, 0};
    int var3d[5] = {0, 0, 0, 0, 0};
    // learned preconditioner (see nn.hip)
    bool pc_attached = false;
    int pc_hidden = 0, pc_layers = 0, pc_factor = 1;
    void* pc_w = nullptr;       // BF16 weight packs, device
    float* pc_b = nullptr;      // FP32 parameter copy (biases read from it), device
    float* pc_act0 = nullptr;   // activation ping-pong buffers (coarse grid)
    float* pc_act1 = nullptr;
    float* pc_coarse = nullptr; // restricted input
    float* pc_st = nullptr;     // [s, 1/s]
    double* pc_nrm = nullptr;   // |v|^2
    double* pc_part = nullptr;  // per-block partial sums of v^2
    int* pc_meta = nullptr;     // per layer: cin, cout, tap-major pack offset, bias offset
    unsigned short* pc_wn = nullptr;   // tap-major BF16 weights of the single-workgroup network kernel
    size_t pc_wn_len = 0;              // its length in shorts
    float* pc_bn = nullptr;            // biases of every layer, contiguous (fused kernel)
    int pc_nbias = 0;
    float* pc_Y = nullptr;             // coarse network outputs of the current cycle (+ a combine slot)
    int pc_slots = 0;
    // x-spectra of the prolongation's weight rows [Wc][nkx] (FP32 apply, work buffer packed as
    // pc_phi_pack), for the coarse correction added in pass B
    rte::cx<float>* pc_phi = nullptr;
    int pc_phi_pack = -1;
    // the correction's per-channel factors (pass A's factor times 1/sqrt(nvec)), device, and the
    // host copy they were made from
    float* pc_coef = nullptr;
    float pc_coef_host[17] = {};
};

namespace rte {
// Basis of m + 1 vectors with vbytes per entry (and Z when need_z), kept when large enough.
int ensure_krylov(rte_ctx* c, int m, bool need_z, size_t vbytes, size_t n = 0);
int apply_channels(rte_ctx* c, int mode, int prec, const double* x, const double* b, double* y, int nbatch);
// Basis vector element type of a context.
template <typename TV>
inline TV* basis(rte_ctx* c) { return reinterpret_cast<TV*>(c->V); }
// Output step of a solve (e.g. the conversion of x to the caller's layout), enqueued on the
// context stream after every true residual, while the host waits for its norm; the last call
// follows the last change of x.
struct SolveFinish {
    void (*fn)(rte_ctx* c, void* arg) = nullptr;
    void* arg = nullptr;
};
// nb > 1: b and x are nb stacked channel vectors and the Krylov process runs on the stacked
// (block-diagonal) system, one batched apply per iteration.
int solve_core(rte_ctx* c, const double* b, double tol, int max_iter, double* x, rte_solve_info* info,
               double* rec, int max_rec, int* nrec, const SolveFinish* finish = nullptr, int nb = 1);
int autotune_2d(rte_ctx* c, int reps, bool use_cache);
}  // namespace rte

namespace rte {
int solve_batched_impl(int count, rte_ctx* const* ctxs, const double* const* f, const double* tol, int max_iter,
                       void* const* u, rte_solve_info* infos);
int time_batched_impl(int count, rte_ctx* const* ctxs, int reps, double* ms_total, int max_launch, int* n_launch,
                      double* ms_launch, int* launch_pass, int* launch_px, int* launch_py, int* launch_var);
int batched_set_variant(int pass, int variant);
void batched_forget(unsigned long long id);
}  // namespace rte
