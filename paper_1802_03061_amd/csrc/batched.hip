// Batched solve of many independent isotropic 2D problems (rte_solve_batched).
//
// Every problem is its own discrete system (I - mu_s K~) u = K~ f (Sec. 2.3, isotropic case of the
// angularly reduced equation) on its own grid, solved by restarted GMRES with FP64 iterative
// refinement exactly as the single-problem solver does, but all problems advance together:
//
//   * one inner iteration of every unconverged problem is a fixed sequence of launches -- pass A,
//     pass B and pass C of the FFT apply (one launch per padded grid size, over the row tiles or
//     column groups of all its problems), then the Krylov kernels over a global list of 4096-element
//     chunks of all problems' vectors, Givens rotations with one thread per problem, and a tick that
//     advances the column index j kept in device memory;
//   * the tiling of each size class's passes (row tiles of A and C, column groups of B) is chosen
//     when the plan is built, by timing the variants on all of the class's problems;
//   * that sequence is captured once into a HIP graph and replayed; a problem whose estimate meets
//     its target (or that reaches the restart length) clears its active flag on the device and its
//     blocks exit at once in later replays;
//   * between cycles the solution update x += V y, the FP64 true residual b - A x (batched FP64
//     apply) and its norms run for the problems still open, and the host decides which continue.
//
// Orthogonalisation is one classical Gram-Schmidt pass (the FP64 refinement bounds the effect of
// any loss of orthogonality).  Sums over chunks are taken in a fixed order, so results do not
// depend on scheduling.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "apply2d.h"
#include "ctx.h"

namespace rte {
namespace {

constexpr int BT = 256;                  // threads of the chunk kernels
constexpr int CHUNK = 4096;              // vector elements per chunk
constexpr int CPT = CHUNK / BT;          // elements per thread

struct Chunk {
    int p, off, len;
};

struct KryProb {
    double* V;          // (m + 1) x nvec Krylov basis
    double* x;          // solution
    double* r;          // residual
    const double* b;    // right-hand side
    double* H;          // (m + 1) x m Hessenberg (column-major, ld m + 1), R after the rotations
    double* cs;
    double* sn;
    double* g;          // m + 1
    double* y;          // m
    cx<double>* u;      // output modes (complex, L = 0)
    int nvec;
    int c0, nc;         // chunks of this problem
};

struct BState {
    double target;      // absolute inner target of the current cycle
    double est;         // residual estimate after the last iteration
    double inv;         // 1 / H[j+1][j], 0 at breakdown
    double rn;          // residual norm at the cycle start
    int jd;             // valid columns of the current cycle
    int iters;          // inner iterations so far
    int flags;          // bit 1: non-finite value
    int pad;
};

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

__device__ __forceinline__ double wave_sum(double s) {
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

// ---------------------------------------------------------------- inner iteration ------------

// partial[chunk][i] = <V_i, w> over the chunk for i <= j, w = V_{j+1} (the new apply output).
__global__ __launch_bounds__(BT) void kb_dots(const Chunk* __restrict__ ch, const KryProb* __restrict__ kp,
                                              const int* __restrict__ act, const int* __restrict__ dj,
                                              double* __restrict__ partial, int m) {
    __shared__ double red[(RTE_MAX_RESTART + 1) * 4];
    const Chunk c = ch[blockIdx.x];
    if (!act[c.p]) return;
    const KryProb& k = kp[c.p];
    const int j = *dj;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double* w = k.V + (size_t)(j + 1) * k.nvec + c.off;
    double wv[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int e = tid + u * BT;
        wv[u] = e < c.len ? w[e] : 0.0;
    }
#pragma unroll 2   // the next vector's loads go out while this one is summed
    for (int i = 0; i <= j; ++i) {
        const double* v = k.V + (size_t)i * k.nvec + c.off;
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int e = tid + u * BT;
            if (e < c.len) s += v[e] * wv[u];
        }
        s = wave_sum(s);
        if (lane == 0) red[i * 4 + wave] = s;
    }
    __syncthreads();
    for (int i = tid; i <= j; i += BT)
        partial[(size_t)blockIdx.x * (m + 1) + i] = (red[i * 4] + red[i * 4 + 1]) + (red[i * 4 + 2] + red[i * 4 + 3]);
}

// H[0..j][j] = sum over the problem's chunks (in chunk order); one block per problem.
__global__ __launch_bounds__(64) void kb_hcol(const KryProb* __restrict__ kp, const int* __restrict__ act,
                                              const int* __restrict__ dj, const double* __restrict__ partial, int m) {
    const int p = blockIdx.x;
    if (!act[p]) return;
    const KryProb& k = kp[p];
    const int j = *dj;
    for (int i = threadIdx.x; i <= j; i += 64) {
        double s = 0.0;
#pragma unroll 8
        for (int c = 0; c < k.nc; ++c) s += partial[(size_t)(k.c0 + c) * (m + 1) + i];
        k.H[(size_t)j * (m + 1) + i] = s;
    }
}

// w -= sum_i H[i][j] V_i over the chunk; part2[chunk] = |w|^2 over the chunk afterwards.
__global__ __launch_bounds__(BT) void kb_update(const Chunk* __restrict__ ch, const KryProb* __restrict__ kp,
                                                const int* __restrict__ act, const int* __restrict__ dj,
                                                double* __restrict__ part2, int m) {
    __shared__ double h[RTE_MAX_RESTART + 1];
    __shared__ double red[4];
    const Chunk c = ch[blockIdx.x];
    if (!act[c.p]) return;
    const KryProb& k = kp[c.p];
    const int j = *dj;
    const int tid = threadIdx.x;
    for (int i = tid; i <= j; i += BT) h[i] = k.H[(size_t)j * (m + 1) + i];
    __syncthreads();
    double* w = k.V + (size_t)(j + 1) * k.nvec + c.off;
    double wv[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int e = tid + u * BT;
        wv[u] = e < c.len ? w[e] : 0.0;
    }
#pragma unroll 2   // the next vector's loads go out while this one is subtracted
    for (int i = 0; i <= j; ++i) {
        const double hi = h[i];
        const double* v = k.V + (size_t)i * k.nvec + c.off;
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int e = tid + u * BT;
            if (e < c.len) wv[u] -= hi * v[e];
        }
    }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int e = tid + u * BT;
        if (e < c.len) {
            w[e] = wv[u];
            s += wv[u] * wv[u];
        }
    }
    s = wave_sum(s);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) part2[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// H[j+1][j] = |w|, the previous Givens rotations and a new one on column j, the residual vector
// g and the estimate |g[j+1]|; decides whether the problem keeps iterating.  One 64-lane block per
// problem: the lanes sum the chunk partials of |w|^2 and the squares of H[.][j] (fixed-order
// shuffle reduction), lane 0 applies the rotations.
__global__ __launch_bounds__(64) void kb_givens(const KryProb* __restrict__ kp, int* __restrict__ act,
                                                const int* __restrict__ dj, const double* __restrict__ part2,
                                                BState* __restrict__ bs, int m, int P,
                                                const int* __restrict__ dmax_iter) {
    const int p = blockIdx.x;
    if (p >= P || !act[p]) return;
    const KryProb& k = kp[p];
    const int j = *dj;
    const int lane = threadIdx.x;
    double* Hj = k.H + (size_t)j * (m + 1);
    double w2 = 0.0, h2 = 0.0;
    for (int c = lane; c < k.nc; c += 64) w2 += part2[k.c0 + c];
    for (int i = lane; i <= j; i += 64) h2 += Hj[i] * Hj[i];
    w2 = wave_sum(w2);
    h2 = wave_sum(h2);
    if (lane != 0) return;
    const int max_iter = *dmax_iter;
    BState& s = bs[p];
    w2 = w2 > 0.0 ? w2 : 0.0;
    const double hn = sqrt(w2);
    Hj[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double t = k.cs[i] * Hj[i] + k.sn[i] * Hj[i + 1];
        Hj[i + 1] = -k.sn[i] * Hj[i] + k.cs[i] * Hj[i + 1];
        Hj[i] = t;
    }
    const double den = hypot(Hj[j], Hj[j + 1]);
    if (den == 0.0) { k.cs[j] = 1.0; k.sn[j] = 0.0; }
    else { k.cs[j] = Hj[j] / den; k.sn[j] = Hj[j + 1] / den; }
    Hj[j] = den;
    Hj[j + 1] = 0.0;
    k.g[j + 1] = -k.sn[j] * k.g[j];
    k.g[j] = k.cs[j] * k.g[j];
    const double est = fabs(k.g[j + 1]);
    s.iters += 1;
    if (!isfinite(den) || !isfinite(est)) {   // drop column j and stop
        s.flags |= 2;
        s.jd = j;
        act[p] = 0;
        return;
    }
    // |w| before orthogonalisation is sqrt(|h|^2 + |w'|^2) in exact arithmetic
    const bool breakdown = !(hn > 1e-14 * sqrt(h2 + w2));
    s.jd = j + 1;
    s.est = est;
    s.inv = breakdown ? 0.0 : 1.0 / hn;
    if (breakdown || est <= s.target || j + 1 >= m || s.iters >= max_iter) act[p] = 0;
}

// V_{j+1} = w / H[j+1][j] for the problems still iterating.
__global__ __launch_bounds__(BT) void kb_scale_next(const Chunk* __restrict__ ch, const KryProb* __restrict__ kp,
                                                    const int* __restrict__ act, const int* __restrict__ dj,
                                                    const BState* __restrict__ bs) {
    const Chunk c = ch[blockIdx.x];
    if (!act[c.p]) return;
    const KryProb& k = kp[c.p];
    const double a = bs[c.p].inv;
    double* w = k.V + (size_t)(*dj + 1) * k.nvec + c.off;
    for (int e = threadIdx.x; e < c.len; e += BT) w[e] *= a;
}

// count[j] = the number of problems still iterating, then j += 1.  Single block.  count is
// device-visible host memory that the host polls (one write-once slot per step of the cycle).
__global__ __launch_bounds__(BT) void kb_tick(int* __restrict__ dj, const int* __restrict__ act, int P,
                                              int* __restrict__ count) {
    __shared__ int red[4];
    int s = 0;
    for (int p = threadIdx.x; p < P; p += BT) s += act[p] != 0;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int j = *dj;
        count[j] = red[0] + red[1] + red[2] + red[3];
        *dj = j + 1;
    }
}

// ---------------------------------------------------------------- cycle boundaries -----------

// what: 0 -> x = 0 and r = b; 1 -> V_0 = r / rn (active problems); 2 -> u = (x, 0)
__global__ __launch_bounds__(BT) void kb_vec(const Chunk* __restrict__ ch, const KryProb* __restrict__ kp,
                                             const int* __restrict__ mask, const BState* __restrict__ bs, int what) {
    const Chunk c = ch[blockIdx.x];
    if (mask && !mask[c.p]) return;
    const KryProb& k = kp[c.p];
    for (int e = threadIdx.x; e < c.len; e += BT) {
        const size_t o = (size_t)c.off + e;
        if (what == 0) {
            k.x[o] = 0.0;
            k.r[o] = k.b[o];
        } else if (what == 1) {
            k.V[o] = k.r[o] / bs[c.p].rn;
        } else {
            k.u[o] = mk(k.x[o], 0.0);
        }
    }
}

// part2[chunk] = |r|^2 over the chunk (problems in mask).
__global__ __launch_bounds__(BT) void kb_norm2(const Chunk* __restrict__ ch, const KryProb* __restrict__ kp,
                                               const int* __restrict__ mask, double* __restrict__ part2) {
    __shared__ double red[4];
    const Chunk c = ch[blockIdx.x];
    if (!mask[c.p]) return;
    const double* r = kp[c.p].r + c.off;
    double s = 0.0;
    for (int e = threadIdx.x; e < c.len; e += BT) s += r[e] * r[e];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part2[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out[p] = sum of the problem's chunk partials (problems in mask), one thread per problem.
__global__ void kb_sum_parts(const KryProb* __restrict__ kp, const int* __restrict__ mask,
                             const double* __restrict__ part2, double* __restrict__ out, int P) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P || !mask[p]) return;
    double s = 0.0;
    for (int c = 0; c < kp[p].nc; ++c) s += part2[kp[p].c0 + c];
    out[p] = s;
}

// Cycle start for the problems in act: g = (rn, 0, ...), j = 0.
__global__ void kb_cycle_start(const KryProb* __restrict__ kp, const int* __restrict__ act,
                               const BState* __restrict__ bs, int* __restrict__ dj, int m, int P) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) *dj = 0;
    if (p >= P || !act[p]) return;
    kp[p].g[0] = bs[p].rn;
    for (int i = 1; i <= m; ++i) kp[p].g[i] = 0.0;
}

// y = R^{-1} g over the cycle's jd columns (problems in mask without a non-finite value).
__global__ void kb_backsolve(const KryProb* __restrict__ kp, const int* __restrict__ mask,
                             const BState* __restrict__ bs, int m, int P) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P || !mask[p] || (bs[p].flags & 2)) return;
    const KryProb& k = kp[p];
    const int jd = bs[p].jd;
    for (int i = jd - 1; i >= 0; --i) {
        double s = k.g[i];
        for (int q = i + 1; q < jd; ++q) s -= k.H[(size_t)q * (m + 1) + i] * k.y[q];
        k.y[i] = s / k.H[(size_t)i * (m + 1) + i];
    }
}

// x += sum_{i < jd} y_i V_i over the chunk.
__global__ __launch_bounds__(BT) void kb_combine(const Chunk* __restrict__ ch, const KryProb* __restrict__ kp,
                                                 const int* __restrict__ mask, const BState* __restrict__ bs) {
    __shared__ double y[RTE_MAX_RESTART];
    const Chunk c = ch[blockIdx.x];
    if (!mask[c.p] || (bs[c.p].flags & 2)) return;
    const KryProb& k = kp[c.p];
    const int jd = bs[c.p].jd;
    if (jd <= 0) return;
    for (int i = threadIdx.x; i < jd; i += BT) y[i] = k.y[i];
    __syncthreads();
    for (int e = threadIdx.x; e < c.len; e += BT) {
        const size_t o = (size_t)c.off + e;
        double s = k.x[o];
#pragma unroll 8
        for (int i = 0; i < jd; ++i) s += y[i] * k.V[(size_t)i * k.nvec + o];
        k.x[o] = s;
    }
}

// ---------------------------------------------------------------- host side -----------------

struct SizeClass {
    int PX, PY;
    std::vector<int> probs;    // problems of this padded size, in order
    std::vector<int2> ac, b;   // (problem, row tile) and (problem, column group)
    int2* dac = nullptr;       // device lists, room for the most items of any variant
    int2* db = nullptr;
    int vr = 0, vb = 0;        // variants: row tiles of passes A and C, column groups of pass B
};

template <typename T>
BatchProb<T> batch_prob(const rte_ctx* c, const cx<T>* Q, const cx<T>* twx, const cx<T>* twy, cx<T>* work,
                        double s, const double* in, double* out, const double* bvec, int jin, int jout) {
    BatchProb<T> d;
    d.nx = c->nx; d.ny = c->ny; d.PX = c->PX; d.PY = c->PY;
    d.s = s;
    d.work = work; d.Q = Q; d.twx = twx; d.twy = twy;
    d.in = in; d.out = out; d.bvec = bvec;
    d.stride = c->nvec;
    d.jin = jin; d.jout = jout;
    return d;
}

template <typename T>
int apply_batch(const std::vector<SizeClass>& cls, const BatchProb<T>* probs, const int* mask, const int* dj, int mode,
                hipStream_t st) {
    for (const auto& k : cls)
        if (apply2d_batch_pass_a<T>(k.PX, probs, k.dac, (int)k.ac.size(), mask, dj, k.vr, st)) return -1;
    for (const auto& k : cls)
        if (apply2d_batch_pass_b<T>(k.PY, probs, k.db, (int)k.b.size(), mask, k.vb, st)) return -1;
    for (const auto& k : cls)
        if (apply2d_batch_pass_c<T>(k.PX, probs, k.dac, (int)k.ac.size(), mask, dj, mode, k.vr, st)) return -1;
    return 0;
}

#define BK_TRY(expr)                                                          \
    do {                                                                      \
        hipError_t e_ = (expr);                                               \
        if (e_ != hipSuccess) return set_hip_error(e_, #expr, __FILE__, __LINE__); \
    } while (0)

// Everything a batch needs that does not change between calls on the same contexts: the device
// arena (descriptors, item lists, chunk list, partial sums, Arnoldi slabs, state), the stream,
// pinned staging, events and the instantiated graph of one inner iteration.  Cached per process
// for a few context lists; dropped when any of its contexts is destroyed.
// The device buffers of a context a plan's descriptors point at (checked on every lookup).
std::vector<const void*> ctx_buffers(const rte_ctx* c) {
    return {c->V, c->xv, c->rv, c->bv, c->wd, c->Qd, c->twd[0], c->twd[1], c->wf, c->Qf, c->twf[0], c->twf[1]};
}

struct Plan {
    std::vector<unsigned long long> ids;   // context ids, in order
    std::vector<const void*> bufs;         // ctx_buffers of every context, in order
    int m = 0, prec = 0, P = 0, NCH = 0;
    size_t S = 0;
    std::vector<SizeClass> cls, cls_d;
    std::vector<KryProb> kp;
    std::vector<Chunk> chunks;
    char* arena = nullptr;
    Chunk* d_ch = nullptr;
    KryProb* d_kp = nullptr;
    BState* d_bs = nullptr;
    int *d_act = nullptr, *d_todo = nullptr, *d_j = nullptr, *d_maxit = nullptr;
    double *d_part = nullptr, *d_part2 = nullptr, *d_rn2 = nullptr, *d_slab = nullptr;
    void* d_it = nullptr;                  // BatchProb<T>[P] of the iteration
    BatchProb<double>* d_res = nullptr;
    BatchProb<double>* d_rhs = nullptr;
    hipStream_t st = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* pinned = nullptr;                // BState[P] | act[P] | todo[P] | rn2[P] | count[m + 1] (mapped)
    BState* h_bs = nullptr;
    int *h_act = nullptr, *h_todo = nullptr, *h_cnt = nullptr, *h_cnt_dev = nullptr;
    double* h_rn2 = nullptr;
    ~Plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (pinned) (void)hipHostFree(pinned);
        if (st) (void)hipStreamDestroy(st);
        if (arena) (void)hipFree(arena);
    }
};

// Most recently used last.  Never destroyed: its plans hold HIP resources, which must not be
// released from static destructors after the runtime may have shut down (the process exit
// reclaims them).
std::mutex g_plan_mu;
std::vector<std::unique_ptr<Plan>>& plans() {
    static auto* v = new std::vector<std::unique_ptr<Plan>>();
    return *v;
}
constexpr size_t MAX_PLANS = 4;

// Workgroups are dispatched round-robin over the 8 XCDs: block b runs on XCD b % 8.  Reorder an
// item list so that XCD k executes a contiguous run of the original list (neighbouring row tiles
// of a problem share 128-byte lines of its spectrum, which then meet in one L2).
std::vector<int2> xcd_order(const std::vector<int2>& in) {
    const size_t N = in.size(), q = N / 8, rem = N % 8;
    std::vector<int2> out(N);
    for (size_t b = 0; b < N; ++b) {
        const size_t k = b % 8, l = b / 8;
        out[b] = in[k * q + std::min(k, rem) + l];
    }
    return out;
}

template <typename X>
X* carve(char* base, size_t& used, size_t n) {
    const size_t off = (used + 255) / 256 * 256;
    used = off + n * sizeof(X);
    return reinterpret_cast<X*>(base + off);
}

// The (problem, row tile) and (problem, column group) items of size class k for row tiles of tr
// rows and groups of nc columns, in XCD order.
void fill_items(SizeClass& k, rte_ctx* const* ctxs, int tr, int nc) {
    k.ac.clear();
    k.b.clear();
    for (int p : k.probs) {
        for (int t = 0; t < (ctxs[p]->ny + tr - 1) / tr; ++t) k.ac.push_back(make_int2(p, t));
        for (int t = 0; t < (ctxs[p]->PX / 2 + nc - 1) / nc; ++t) k.b.push_back(make_int2(p, t));
    }
    k.ac = xcd_order(k.ac);
    k.b = xcd_order(k.b);
}

// Item-list room of size class k over every variant of precision T (the smallest tiles give the
// most items).
template <typename T>
std::pair<size_t, size_t> item_room(const SizeClass& k, rte_ctx* const* ctxs) {
    int tr = 1 << 30, nc = 1 << 30;
    for (int v = 0; v < apply2d_batch_row_variants<T>(k.PX); ++v) tr = std::min(tr, apply2d_batch_rows<T>(v));
    for (int v = 0; v < apply2d_batch_col_variants<T>(k.PY); ++v) nc = std::min(nc, apply2d_batch_cols<T>(k.PY, v));
    size_t nac = 0, nb = 0;
    for (int p : k.probs) {
        nac += (size_t)(ctxs[p]->ny + tr - 1) / tr;
        nb += (size_t)(ctxs[p]->PX / 2 + nc - 1) / nc;
    }
    return {nac, nb};
}

// Variants forced by rte_set_batched_variant (-1: tuned); guarded by g_plan_mu.
int g_force[2] = {-1, -1};

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Choose the row-tile variant (passes A and C together) and the column-group variant (pass B) of
// every size class of the iteration's item lists: the fastest (best of 3 runs of 5 launches) over
// all of the class's problems (every problem active, basis column 0 in, column 1 out) on the plan stream,
// unless forced by rte_set_batched_variant or disabled by RTE_AUTOTUNE=0 (variant 0).  Leaves the
// chosen lists on the device.
template <typename T>
int tune_plan(Plan& pl, rte_ctx* const* ctxs) {
    hipStream_t st = pl.st;
    const char* at = std::getenv("RTE_AUTOTUNE");
    const bool tune = !(at && at[0] == '0');
    constexpr int reps = 5, trials = 3;
    const BatchProb<T>* probs = (const BatchProb<T>*)pl.d_it;
    std::vector<int> ones(pl.P, 1);
    const int j0[2] = {0, 0};
    BK_TRY(hipMemcpyAsync(pl.d_act, ones.data(), sizeof(int) * pl.P, hipMemcpyHostToDevice, st));
    BK_TRY(hipMemcpyAsync(pl.d_j, j0, sizeof(int), hipMemcpyHostToDevice, st));
    BK_TRY(hipStreamSynchronize(st));
    EventPair ev;
    BK_TRY(hipEventCreate(&ev.a));
    BK_TRY(hipEventCreate(&ev.b));
    auto upload = [&](const SizeClass& k) -> int {
        BK_TRY(hipMemcpyAsync(k.dac, k.ac.data(), sizeof(int2) * k.ac.size(), hipMemcpyHostToDevice, st));
        BK_TRY(hipMemcpyAsync(k.db, k.b.data(), sizeof(int2) * k.b.size(), hipMemcpyHostToDevice, st));
        BK_TRY(hipStreamSynchronize(st));
        return RTE_OK;
    };
    auto launch = [&](const SizeClass& k, int which) {
        if (which == 1) return apply2d_batch_pass_b<T>(k.PY, probs, k.db, (int)k.b.size(), pl.d_act, k.vb, st);
        if (apply2d_batch_pass_a<T>(k.PX, probs, k.dac, (int)k.ac.size(), pl.d_act, pl.d_j, k.vr, st)) return -1;
        return apply2d_batch_pass_c<T>(k.PX, probs, k.dac, (int)k.ac.size(), pl.d_act, pl.d_j, APPLY_A, k.vr, st);
    };
    auto timed = [&](SizeClass& k, int which, double* ms) -> int {
        fill_items(k, ctxs, apply2d_batch_rows<T>(k.vr), apply2d_batch_cols<T>(k.PY, k.vb));
        if (int rc = upload(k)) return rc;
        if (launch(k, which)) return set_error(RTE_EUNSUPPORTED, "batched apply: unsupported size");   // warm-up
        for (int trial = 0; trial < trials; ++trial) {   // the best of a few runs of `reps` launches
            BK_TRY(hipEventRecord(ev.a, st));
            for (int r = 0; r < reps; ++r) (void)launch(k, which);
            BK_TRY(hipEventRecord(ev.b, st));
            BK_TRY(hipEventSynchronize(ev.b));
            float t = 0.f;
            BK_TRY(hipEventElapsedTime(&t, ev.a, ev.b));
            if (trial == 0 || t < *ms) *ms = t;
        }
        return RTE_OK;
    };
    for (auto& k : pl.cls) {
        const int nv[2] = {apply2d_batch_row_variants<T>(k.PX), apply2d_batch_col_variants<T>(k.PY)};
        int* var[2] = {&k.vr, &k.vb};
        for (int w = 0; w < 2; ++w) *var[w] = g_force[w] >= 0 && g_force[w] < nv[w] ? g_force[w] : 0;
        for (int w = 0; w < 2; ++w) {
            if (!tune || g_force[w] >= 0 || nv[w] < 2) continue;
            double best = 0.0;
            int bv = 0;
            for (int v = 0; v < nv[w]; ++v) {
                *var[w] = v;
                double ms = 0.0;
                if (int rc = timed(k, w, &ms)) return rc;
                if (v == 0 || ms < best) { best = ms; bv = v; }
            }
            *var[w] = bv;
        }
        fill_items(k, ctxs, apply2d_batch_rows<T>(k.vr), apply2d_batch_cols<T>(k.PY, k.vb));
        if (int rc = upload(k)) return rc;
    }
    return RTE_OK;
}

template <typename T>
int build_plan(Plan& pl, int P, rte_ctx* const* ctxs) {
    const int m = pl.m;
    std::map<std::pair<int, int>, int> cls_index;
    pl.kp.assign(P, KryProb{});
    for (int p = 0; p < P; ++p) {
        const rte_ctx* c = ctxs[p];
        KryProb& k = pl.kp[p];
        k.nvec = (int)c->nvec;
        k.c0 = (int)pl.chunks.size();
        for (int off = 0; off < k.nvec; off += CHUNK) pl.chunks.push_back({p, off, std::min(CHUNK, k.nvec - off)});
        k.nc = (int)pl.chunks.size() - k.c0;
        auto key = std::make_pair(c->PX, c->PY);
        if (!cls_index.count(key)) {
            cls_index[key] = (int)pl.cls.size();
            SizeClass sc;
            sc.PX = c->PX;
            sc.PY = c->PY;
            pl.cls.push_back(sc);
        }
        pl.cls[cls_index[key]].probs.push_back(p);
    }
    // the iteration uses precision T (its variants tuned below), the right-hand side and residual
    // FP64 with variant 0: separate item lists
    pl.cls_d = pl.cls;
    for (auto& k : pl.cls_d) fill_items(k, ctxs, apply2d_batch_rows<double>(0), apply2d_batch_cols<double>(k.PY, 0));
    std::vector<std::pair<size_t, size_t>> room;
    for (auto& k : pl.cls) room.push_back(item_room<T>(k, ctxs));
    const int NCH = pl.NCH = (int)pl.chunks.size();
    const size_t S = pl.S = (size_t)(m + 1) * m + 4 * (size_t)m + 2;   // Arnoldi slab per problem
    size_t items = 0;
    for (auto& r : room) items += r.first + r.second;
    for (auto& k : pl.cls_d) items += k.ac.size() + k.b.size();
    const size_t ntake = 16 + 4 * pl.cls.size();
    const size_t cap = 256 * ntake + sizeof(Chunk) * NCH + sizeof(KryProb) * P + sizeof(BState) * P +
                       sizeof(int) * (2 * P + 4) + sizeof(double) * ((size_t)NCH * (m + 2) + P + S * P) +
                       sizeof(int2) * items + sizeof(BatchProb<T>) * P + 2 * sizeof(BatchProb<double>) * P;
    BK_TRY(hipMalloc((void**)&pl.arena, cap));
    size_t used = 0;
    char* a = pl.arena;
    pl.d_ch = carve<Chunk>(a, used, NCH);
    pl.d_kp = carve<KryProb>(a, used, P);
    pl.d_bs = carve<BState>(a, used, P);
    pl.d_act = carve<int>(a, used, P);
    pl.d_todo = carve<int>(a, used, P);
    pl.d_j = carve<int>(a, used, 4);
    pl.d_maxit = pl.d_j + 2;
    pl.d_part = carve<double>(a, used, (size_t)NCH * (m + 1));
    pl.d_part2 = carve<double>(a, used, NCH);
    pl.d_rn2 = carve<double>(a, used, P);
    pl.d_slab = carve<double>(a, used, S * P);
    for (size_t i = 0; i < pl.cls.size(); ++i) {
        pl.cls[i].dac = carve<int2>(a, used, room[i].first);
        pl.cls[i].db = carve<int2>(a, used, room[i].second);
    }
    for (auto& k : pl.cls_d) { k.dac = carve<int2>(a, used, k.ac.size()); k.db = carve<int2>(a, used, k.b.size()); }
    pl.d_it = carve<BatchProb<T>>(a, used, P);
    pl.d_res = carve<BatchProb<double>>(a, used, P);
    pl.d_rhs = carve<BatchProb<double>>(a, used, P);
    if (used > cap) return set_error(RTE_EDEVICE, "batched arena overflow");
    BK_TRY(hipStreamCreateWithFlags(&pl.st, hipStreamNonBlocking));
    hipStream_t st = pl.st;
    // descriptors that do not depend on the call's sources and outputs
    std::vector<BatchProb<T>> it(P);
    std::vector<BatchProb<double>> res(P);
    for (int p = 0; p < P; ++p) {
        rte_ctx* c = ctxs[p];
        KryProb& k = pl.kp[p];
        double* sl = pl.d_slab + S * p;
        k.V = basis<double>(c); k.x = c->xv; k.r = c->rv; k.b = c->bv;
        k.H = sl;
        k.cs = sl + (size_t)(m + 1) * m;
        k.sn = k.cs + m;
        k.g = k.sn + m;
        k.y = k.g + m + 1;
        k.u = nullptr;
        const double s = c->mu_s * c->sigma[0];
        if constexpr (sizeof(T) == 4)
            it[p] = batch_prob<float>(c, c->Qf, c->twf[0], c->twf[1], c->wf, s, k.V, k.V, nullptr, 1, 1);
        else
            it[p] = batch_prob<double>(c, c->Qd, c->twd[0], c->twd[1], c->wd, s, k.V, k.V, nullptr, 1, 1);
        res[p] = batch_prob<double>(c, c->Qd, c->twd[0], c->twd[1], c->wd, s, c->xv, c->rv, c->bv, 0, 0);
    }
    BK_TRY(hipMemcpyAsync(pl.d_ch, pl.chunks.data(), sizeof(Chunk) * NCH, hipMemcpyHostToDevice, st));
    BK_TRY(hipMemcpyAsync(pl.d_it, it.data(), sizeof(BatchProb<T>) * P, hipMemcpyHostToDevice, st));
    BK_TRY(hipMemcpyAsync(pl.d_res, res.data(), sizeof(BatchProb<double>) * P, hipMemcpyHostToDevice, st));
    for (const auto& k : pl.cls_d) {
        BK_TRY(hipMemcpyAsync(k.dac, k.ac.data(), sizeof(int2) * k.ac.size(), hipMemcpyHostToDevice, st));
        BK_TRY(hipMemcpyAsync(k.db, k.b.data(), sizeof(int2) * k.b.size(), hipMemcpyHostToDevice, st));
    }
    BK_TRY(hipStreamSynchronize(st));   // host staging vectors go out of scope
    if (int rc = tune_plan<T>(pl, ctxs)) return rc;
    // pinned host staging; the active count is written by the tick kernel straight into it
    const size_t pin_bytes = sizeof(BState) * P + sizeof(int) * 2 * P + 8 + sizeof(double) * P + sizeof(int) * (m + 1) + 64;
    BK_TRY(hipHostMalloc(&pl.pinned, pin_bytes, hipHostMallocMapped | hipHostMallocCoherent));
    pl.h_bs = (BState*)pl.pinned;
    pl.h_act = (int*)(pl.h_bs + P);
    pl.h_todo = pl.h_act + P;
    pl.h_rn2 = (double*)(((uintptr_t)(pl.h_todo + P) + 7) / 8 * 8);
    pl.h_cnt = (int*)(pl.h_rn2 + P);
    BK_TRY(hipHostGetDevicePointer((void**)&pl.h_cnt_dev, pl.h_cnt, 0));
    // capture one inner iteration; replay i (i < m, the step index) writes its active count to
    // h_cnt[i], which the host polls one replay behind
    const unsigned gP = (unsigned)((P + 63) / 64);
    BK_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
    int crc = apply_batch<T>(pl.cls, (const BatchProb<T>*)pl.d_it, pl.d_act, pl.d_j, APPLY_A, st);
    hipLaunchKernelGGL(kb_dots, dim3(NCH), dim3(BT), 0, st, pl.d_ch, pl.d_kp, pl.d_act, pl.d_j, pl.d_part, m);
    hipLaunchKernelGGL(kb_hcol, dim3(P), dim3(64), 0, st, pl.d_kp, pl.d_act, pl.d_j, pl.d_part, m);
    hipLaunchKernelGGL(kb_update, dim3(NCH), dim3(BT), 0, st, pl.d_ch, pl.d_kp, pl.d_act, pl.d_j, pl.d_part2, m);
    hipLaunchKernelGGL(kb_givens, dim3(P), dim3(64), 0, st, pl.d_kp, pl.d_act, pl.d_j, pl.d_part2, pl.d_bs, m, P,
                       pl.d_maxit);
    hipLaunchKernelGGL(kb_scale_next, dim3(NCH), dim3(BT), 0, st, pl.d_ch, pl.d_kp, pl.d_act, pl.d_j, pl.d_bs);
    hipLaunchKernelGGL(kb_tick, dim3(1), dim3(BT), 0, st, pl.d_j, pl.d_act, P, pl.h_cnt_dev);
    hipError_t ce = hipStreamEndCapture(st, &pl.graph);
    if (crc) return set_error(RTE_EUNSUPPORTED, "batched apply: unsupported size");
    BK_TRY(ce);
    BK_TRY(hipGraphInstantiate(&pl.exec, pl.graph, nullptr, nullptr, 0));
    return RTE_OK;
}

template <typename T>
int run_plan(Plan& pl, rte_ctx* const* ctxs, const double* const* f, const double* tol, int max_iter, void* const* u,
             rte_solve_info* infos, double t0) {
    const int P = pl.P, m = pl.m, NCH = pl.NCH;
    const rte_ctx* c0 = ctxs[0];
    const int max_cycles = c0->opts.max_cycles;
    const bool mixed = c0->prec == RTE_PREC_FP32;
    // Per-cycle reduction of the FP32 inner solve, at most 3e-5 here: the problems advance in
    // lockstep, so a third cycle for a few of them holds the whole batch for another restart
    // (measured on the 128-problem workload: 24.1 ms per batch at 3e-5, 35.3 ms at 3e-4).
    const double inner_tol = std::min(c0->opts.inner_tol, 3e-5);
    hipStream_t st = pl.st;
    // per-call descriptors: sources (right-hand side apply) and outputs
    std::vector<BatchProb<double>> rhs(P);
    for (int p = 0; p < P; ++p) {
        rte_ctx* c = ctxs[p];
        rhs[p] = batch_prob<double>(c, c->Qd, c->twd[0], c->twd[1], c->wd, 1.0, f[p], c->bv, nullptr, 0, 0);
        pl.kp[p].u = (cx<double>*)u[p];
    }
    BK_TRY(hipMemcpyAsync(pl.d_rhs, rhs.data(), sizeof(BatchProb<double>) * P, hipMemcpyHostToDevice, st));
    BK_TRY(hipMemcpyAsync(pl.d_kp, pl.kp.data(), sizeof(KryProb) * P, hipMemcpyHostToDevice, st));
    const int mi[2] = {max_iter, 0};
    BK_TRY(hipMemcpyAsync(pl.d_maxit, mi, sizeof(int), hipMemcpyHostToDevice, st));
    const unsigned gP = (unsigned)((P + 63) / 64);
    BState* h_bs = pl.h_bs;
    int* h_act = pl.h_act;
    int* h_todo = pl.h_todo;
    double* h_rn2 = pl.h_rn2;
    // ---- right-hand sides b = K~ f (FP64), x = 0, r = b, |b|
    if (apply_batch<double>(pl.cls_d, pl.d_rhs, nullptr, nullptr, APPLY_KT, st))
        return set_error(RTE_EUNSUPPORTED, "batched apply: unsupported size");
    hipLaunchKernelGGL(kb_vec, dim3(NCH), dim3(BT), 0, st, pl.d_ch, pl.d_kp, nullptr, pl.d_bs, 0);
    for (int p = 0; p < P; ++p) h_todo[p] = 1;
    BK_TRY(hipMemcpyAsync(pl.d_todo, h_todo, sizeof(int) * P, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(kb_norm2, dim3(NCH), dim3(BT), 0, st, pl.d_ch, pl.d_kp, pl.d_todo, pl.d_part2);
    hipLaunchKernelGGL(kb_sum_parts, dim3(gP), dim3(64), 0, st, pl.d_kp, pl.d_todo, pl.d_part2, pl.d_rn2, P);
    BK_TRY(hipMemcpyAsync(h_rn2, pl.d_rn2, sizeof(double) * P, hipMemcpyDeviceToHost, st));
    BK_TRY(hipStreamSynchronize(st));
    std::vector<double> bn(P), rn(P), est(P);
    std::vector<int> status(P, RTE_NOT_CONVERGED), cycles(P, 0);
    memset(h_bs, 0, sizeof(BState) * P);
    for (int p = 0; p < P; ++p) {
        bn[p] = std::sqrt(h_rn2[p]);
        rn[p] = est[p] = bn[p];
        if (!std::isfinite(h_rn2[p])) { status[p] = RTE_ENUMERIC; h_todo[p] = 0; }
        else if (h_rn2[p] == 0.0) { status[p] = RTE_OK; h_todo[p] = 0; }
    }
    // ---- cycles
    int ncyc = 0;
    while (true) {
        bool any = false;
        for (int p = 0; p < P; ++p) any = any || h_todo[p];
        if (!any || ncyc >= max_cycles) break;
        ++ncyc;
        for (int p = 0; p < P; ++p) {
            h_act[p] = h_todo[p];
            if (!h_todo[p]) continue;
            ++cycles[p];
            double target = 0.5 * tol[p] * bn[p];
            if (mixed) target = std::max(target, inner_tol * rn[p]);
            h_bs[p].target = target;
            h_bs[p].rn = rn[p];
            h_bs[p].jd = 0;
            h_bs[p].inv = 0.0;
            h_bs[p].flags = 0;
        }
        BK_TRY(hipMemcpyAsync(pl.d_bs, h_bs, sizeof(BState) * P, hipMemcpyHostToDevice, st));
        BK_TRY(hipMemcpyAsync(pl.d_act, h_act, sizeof(int) * P, hipMemcpyHostToDevice, st));
        BK_TRY(hipMemcpyAsync(pl.d_todo, h_todo, sizeof(int) * P, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(kb_cycle_start, dim3(gP), dim3(64), 0, st, pl.d_kp, pl.d_act, pl.d_bs, pl.d_j, m, P);
        hipLaunchKernelGGL(kb_vec, dim3(NCH), dim3(BT), 0, st, pl.d_ch, pl.d_kp, pl.d_act, pl.d_bs, 1);
        // inner iterations: replay the graph; replay i's tick writes the active count into the
        // write-once slot h_cnt[i] (mapped host memory, -1 until written), which the host polls
        // while replay i + 1 runs.  No event per replay: a record costs an idle gap on the GPU.
        volatile int* cnt = pl.h_cnt;
        for (int i = 0; i < m; ++i) cnt[i] = -1;
        for (int i = 0; i < m; ++i) {
            BK_TRY(hipGraphLaunch(pl.exec, st));
            if (i >= 1) {
                const double tw = now_ms();
                while (cnt[i - 1] < 0) {
                    if (now_ms() - tw > 20.0) {   // a long replay: block on the stream instead
                        BK_TRY(hipStreamSynchronize(st));
                        if (cnt[i - 1] < 0) return set_error(RTE_EDEVICE, "batched step count missing");
                        break;
                    }
                }
                if (cnt[i - 1] == 0) break;   // every problem has stopped
            }
        }
        // x += V y, r = b - A x (FP64), |r|
        hipLaunchKernelGGL(kb_backsolve, dim3(gP), dim3(64), 0, st, pl.d_kp, pl.d_todo, pl.d_bs, m, P);
        hipLaunchKernelGGL(kb_combine, dim3(NCH), dim3(BT), 0, st, pl.d_ch, pl.d_kp, pl.d_todo, pl.d_bs);
        if (apply_batch<double>(pl.cls_d, pl.d_res, pl.d_todo, nullptr, APPLY_RESID, st))
            return set_error(RTE_EUNSUPPORTED, "batched apply: unsupported size");
        hipLaunchKernelGGL(kb_norm2, dim3(NCH), dim3(BT), 0, st, pl.d_ch, pl.d_kp, pl.d_todo, pl.d_part2);
        hipLaunchKernelGGL(kb_sum_parts, dim3(gP), dim3(64), 0, st, pl.d_kp, pl.d_todo, pl.d_part2, pl.d_rn2, P);
        BK_TRY(hipMemcpyAsync(h_rn2, pl.d_rn2, sizeof(double) * P, hipMemcpyDeviceToHost, st));
        BK_TRY(hipMemcpyAsync(h_bs, pl.d_bs, sizeof(BState) * P, hipMemcpyDeviceToHost, st));
        BK_TRY(hipStreamSynchronize(st));
        for (int p = 0; p < P; ++p) {
            if (!h_todo[p]) continue;
            if (h_bs[p].flags & 2 || !std::isfinite(h_rn2[p])) {
                status[p] = RTE_ENUMERIC;
                h_todo[p] = 0;
                continue;
            }
            est[p] = h_bs[p].est;
            rn[p] = std::sqrt(h_rn2[p]);
            if (rn[p] <= tol[p] * bn[p]) { status[p] = RTE_OK; h_todo[p] = 0; }
            else if (h_bs[p].iters >= max_iter) h_todo[p] = 0;
        }
    }
    // ---- outputs
    for (int p = 0; p < P; ++p) h_act[p] = 1;
    BK_TRY(hipMemcpyAsync(pl.d_act, h_act, sizeof(int) * P, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(kb_vec, dim3(NCH), dim3(BT), 0, st, pl.d_ch, pl.d_kp, pl.d_act, pl.d_bs, 2);
    BK_TRY(hipGetLastError());
    BK_TRY(hipStreamSynchronize(st));
    const double t_solve = now_ms() - t0;
    int worst = RTE_OK;
    for (int p = 0; p < P; ++p) {
        if (status[p] == RTE_ENUMERIC) worst = RTE_ENUMERIC;
        else if (status[p] == RTE_NOT_CONVERGED && worst == RTE_OK) worst = RTE_NOT_CONVERGED;
        if (!infos) continue;
        rte_solve_info& in = infos[p];
        memset(&in, 0, sizeof(in));
        in.iterations = h_bs[p].iters;
        in.cycles = cycles[p];
        in.applies = h_bs[p].iters + cycles[p];
        in.relres_est = bn[p] > 0 ? est[p] / bn[p] : 0.0;
        in.relres_true = bn[p] > 0 ? rn[p] / bn[p] : 0.0;
        in.t_setup_ms = ctxs[p]->t_setup_ms;
        in.t_solve_ms = t_solve;
        in.status = status[p];
    }
    if (worst == RTE_ENUMERIC) return set_error(RTE_ENUMERIC, "non-finite value in a batched problem");
    if (worst == RTE_NOT_CONVERGED) set_error(RTE_NOT_CONVERGED, "some batched problems did not converge");
    return worst;
}

template <typename T>
int solve_batched_t(int P, rte_ctx* const* ctxs, const double* const* f, const double* tol, int max_iter, void* const* u,
                    rte_solve_info* infos) {
    const double t0 = now_ms();
    const int m = ctxs[0]->opts.restart;
    for (int p = 0; p < P; ++p) {
        int rc = ensure_krylov(ctxs[p], m, false, sizeof(double));   // an FP64 basis in every precision
        if (rc) return rc;
        BK_TRY(hipStreamSynchronize(ctxs[p]->stream));
    }
    std::vector<unsigned long long> ids(P);
    std::vector<const void*> bufs;
    for (int p = 0; p < P; ++p) {
        ids[p] = ctxs[p]->id;
        const auto b = ctx_buffers(ctxs[p]);
        bufs.insert(bufs.end(), b.begin(), b.end());
    }
    std::lock_guard<std::mutex> lk(g_plan_mu);   // one batched solve at a time per process
    auto& g_plans = plans();
    Plan* pl = nullptr;
    for (size_t i = 0; i < g_plans.size(); ++i) {
        Plan& q = *g_plans[i];
        // the Krylov buffers a plan points at are reallocated when the restart length changes
        if (q.ids == ids && q.m == m && q.prec == ctxs[0]->prec && q.bufs == bufs) {
            std::unique_ptr<Plan> keep = std::move(g_plans[i]);
            g_plans.erase(g_plans.begin() + i);
            g_plans.push_back(std::move(keep));
            pl = g_plans.back().get();
            break;
        }
    }
    if (!pl) {
        std::unique_ptr<Plan> np(new (std::nothrow) Plan);
        if (!np) return set_error(RTE_ENOMEM, "host allocation failed");
        np->ids = ids;
        np->bufs = bufs;
        np->m = m;
        np->prec = ctxs[0]->prec;
        np->P = P;
        int rc = build_plan<T>(*np, P, ctxs);
        if (rc) return rc;
        if (g_plans.size() >= MAX_PLANS) g_plans.erase(g_plans.begin());
        g_plans.push_back(std::move(np));
        pl = g_plans.back().get();
    }
    return run_plan<T>(*pl, ctxs, f, tol, max_iter, u, infos, t0);
}

// Time the batched FP-T apply of one inner iteration (every problem active, input basis column 0):
// one launch per pass and padded size, each bracketed by events on the plan's stream.
template <typename T>
int time_plan(Plan& pl, int reps, double* ms_total, int max_launch, int* n_launch, double* ms_launch, int* launch_pass,
              int* launch_px, int* launch_py, int* launch_var) {
    hipStream_t st = pl.st;
    const int P = pl.P, ncls = (int)pl.cls.size(), nl = 3 * ncls;
    std::vector<int> ones(P, 1);
    const int j0[2] = {0, 0};
    BK_TRY(hipMemcpyAsync(pl.d_act, ones.data(), sizeof(int) * P, hipMemcpyHostToDevice, st));
    BK_TRY(hipMemcpyAsync(pl.d_j, j0, sizeof(int), hipMemcpyHostToDevice, st));
    std::vector<hipEvent_t> ev(nl + 1, nullptr);
    int rc = RTE_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) { rc = set_error(RTE_EDEVICE, "hipEventCreate failed"); break; }
    std::vector<double> acc(nl, 0.0);
    const BatchProb<T>* probs = (const BatchProb<T>*)pl.d_it;
    for (int r = 0; r < reps && !rc; ++r) {
        int q = 0;
        if (hipEventRecord(ev[0], st) != hipSuccess) { rc = set_error(RTE_EDEVICE, "hipEventRecord failed"); break; }
        for (int pass = 0; pass < 3 && !rc; ++pass)
            for (const auto& k : pl.cls) {
                int bad = pass == 0
                              ? apply2d_batch_pass_a<T>(k.PX, probs, k.dac, (int)k.ac.size(), pl.d_act, pl.d_j, k.vr, st)
                          : pass == 1
                              ? apply2d_batch_pass_b<T>(k.PY, probs, k.db, (int)k.b.size(), pl.d_act, k.vb, st)
                              : apply2d_batch_pass_c<T>(k.PX, probs, k.dac, (int)k.ac.size(), pl.d_act, pl.d_j,
                                                        APPLY_A, k.vr, st);
                if (bad) { rc = set_error(RTE_EUNSUPPORTED, "batched apply: unsupported size"); break; }
                if (hipEventRecord(ev[++q], st) != hipSuccess) { rc = set_error(RTE_EDEVICE, "hipEventRecord failed"); break; }
            }
        if (rc) break;
        if (hipEventSynchronize(ev[nl]) != hipSuccess) { rc = set_error(RTE_EDEVICE, "hipEventSynchronize failed"); break; }
        for (int i = 0; i < nl; ++i) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
            acc[i] += ms;
        }
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc) return rc;
    double tot = 0.0;
    for (int i = 0; i < nl; ++i) tot += acc[i] / reps;
    if (ms_total) *ms_total = tot;
    if (n_launch) *n_launch = nl;
    for (int i = 0; i < nl && i < max_launch; ++i) {
        if (ms_launch) ms_launch[i] = acc[i] / reps;
        if (launch_pass) launch_pass[i] = i / ncls;
        if (launch_px) launch_px[i] = pl.cls[i % ncls].PX;
        if (launch_py) launch_py[i] = pl.cls[i % ncls].PY;
        if (launch_var) launch_var[i] = i / ncls == 1 ? pl.cls[i % ncls].vb : pl.cls[i % ncls].vr;
    }
    return RTE_OK;
}

}  // namespace

int time_batched_impl(int count, rte_ctx* const* ctxs, int reps, double* ms_total, int max_launch, int* n_launch,
                      double* ms_launch, int* launch_pass, int* launch_px, int* launch_py, int* launch_var) {
    if (count < 1 || !ctxs || reps < 1 || max_launch < 0) return set_error(RTE_EINVAL, "bad argument");
    for (int i = 0; i < count; ++i)
        if (!ctxs[i]) return set_error(RTE_EINVAL, "problem %d: NULL context", i);
    std::vector<unsigned long long> ids(count);
    std::vector<const void*> bufs;
    for (int p = 0; p < count; ++p) {
        ids[p] = ctxs[p]->id;
        const auto b = ctx_buffers(ctxs[p]);
        bufs.insert(bufs.end(), b.begin(), b.end());
    }
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto& q : plans()) {
        if (q->ids == ids && q->m == ctxs[0]->opts.restart && q->prec == ctxs[0]->prec && q->bufs == bufs) {
            return q->prec == RTE_PREC_FP32
                       ? time_plan<float>(*q, reps, ms_total, max_launch, n_launch, ms_launch, launch_pass, launch_px,
                                          launch_py, launch_var)
                       : time_plan<double>(*q, reps, ms_total, max_launch, n_launch, ms_launch, launch_pass, launch_px,
                                           launch_py, launch_var);
        }
    }
    return set_error(RTE_EINVAL, "no batch plan for these contexts: call rte_solve_batched on them first");
}

// Force the batched variants of every later plan (pass 0: row tiles of passes A and C, 1: column
// groups of pass B; -1: tuned) and drop the cached plans.
int batched_set_variant(int pass, int variant) {
    if (pass < 0 || pass > 1 || variant < -1 || variant > 3) return set_error(RTE_EINVAL, "bad batched variant");
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_force[pass] = variant;
    plans().clear();
    return RTE_OK;
}

// A context is going away: drop every cached batch plan that refers to it.
void batched_forget(unsigned long long id) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto& g_plans = plans();
    for (size_t i = 0; i < g_plans.size();) {
        const auto& ids = g_plans[i]->ids;
        if (std::find(ids.begin(), ids.end(), id) != ids.end()) g_plans.erase(g_plans.begin() + i);
        else ++i;
    }
}

int solve_batched_impl(int count, rte_ctx* const* ctxs, const double* const* f, const double* tol, int max_iter,
                       void* const* u, rte_solve_info* infos) {
    if (count < 0 || (count > 0 && (!ctxs || !f || !tol || !u))) return set_error(RTE_EINVAL, "bad batched arguments");
    if (max_iter < 1) return set_error(RTE_EINVAL, "max_iter must be >= 1");
    if (count == 0) return RTE_OK;
    for (int i = 0; i < count; ++i) {
        if (!ctxs[i] || ctxs[i]->dim != 2 || ctxs[i]->L != 0)
            return set_error(RTE_EINVAL, "problem %d: batched solves take 2D isotropic contexts", i);
        if (!f[i] || !u[i]) return set_error(RTE_EINVAL, "problem %d: NULL source or output", i);
        if (!(tol[i] > 0.0) || !(tol[i] < 1.0)) return set_error(RTE_EINVAL, "problem %d: tol must be in (0, 1)", i);
        if (ctxs[i]->prec != ctxs[0]->prec || ctxs[i]->device != ctxs[0]->device)
            return set_error(RTE_EINVAL, "problem %d: batched contexts must share precision and device", i);
        for (int q = 0; q < i; ++q)
            if (ctxs[q] == ctxs[i]) return set_error(RTE_EINVAL, "problem %d: a context appears twice", i);
    }
    if (ctxs[0]->opts.restart > RTE_MAX_RESTART) return set_error(RTE_EINVAL, "restart too long");
    if (ctxs[0]->prec == RTE_PREC_FP32) return solve_batched_t<float>(count, ctxs, f, tol, max_iter, u, infos);
    return solve_batched_t<double>(count, ctxs, f, tol, max_iter, u, infos);
}

}  // namespace rte
