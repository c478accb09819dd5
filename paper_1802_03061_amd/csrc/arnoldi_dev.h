// Device side of one Arnoldi column (FP64): the Hessenberg / Givens bookkeeping after the
// Gram-Schmidt dots and update, and the two scalar rules of the fused single pass that every block
// of a kernel can evaluate on its own (identical inputs, identical operation order, identical bits).
#pragma once
#include "krylov.h"

namespace rte {

constexpr int ARN_MAXROW = RTE_KRYLOV_MAXVEC + 2;   // column entries

// Factor a = 1/|w - V h| of the fused update, from |w|^2 (w0) and |h|^2 (hh) with V orthonormal:
// 1/sqrt(w0 - hh), or 1 when the difference has lost more than five digits to cancellation (the
// flagged rescale then normalises).
__device__ __forceinline__ double fused_factor(double w0, double hh) {
    const double d = w0 - hh;
    return (w0 > 0.0 && d > 1e-5 * w0) ? 1.0 / sqrt(d) : 1.0;
}

// After the fused update wrote a (w - V h) with squared norm nu2: hn = |w - V h|, whether the
// stored vector needs a rescale (nu2 not 1 within tol), breakdown (hn below 1e-14 |w|), and the
// rescale factor inv (0 on breakdown).
__device__ __forceinline__ void fused_decision(double nu2, double a, double w0, double tol, double& hn, bool& renorm,
                                               bool& breakdown, double& inv) {
    const double w1 = nu2 > 0.0 ? nu2 : 0.0;
    hn = sqrt(w1) / a;
    renorm = !(fabs(w1 - 1.0) <= tol);
    breakdown = !(hn > 1e-14 * sqrt(w0 > 0.0 ? w0 : 0.0));
    inv = breakdown ? 0.0 : 1.0 / sqrt(w1);
}

// Sum of h[i]^2, i <= j, in index order (one thread).
__device__ __forceinline__ double sum_sq(const double* h, int j) {
    double hh = 0.0;
    for (int i = 0; i <= j; ++i) hh += h[i] * h[i];
    return hh;
}

// Stage 0 of the fused single pass inside an update kernel: every block's thread 0 computes the
// factor a from the reduced h (hs, in LDS) and |w|^2 (t.st[j+1]) and returns it through *a_sh; block 0
// also stores H[:, j] = h, flags[0] = 0, st[m+3] = |w|^2 and st[2m+5] = a.  The caller
// synchronises the block before reading *a_sh.
__device__ __forceinline__ void arnoldi_stage0_in_update(const ArnoldiArgs& t, const double* hs, double* a_sh) {
    if (threadIdx.x != 0) return;
    const int j = t.j, m = t.m;
    const double w0 = t.st[j + 1];
    const double a = fused_factor(w0, sum_sq(hs, j));
    *a_sh = a;
    if (blockIdx.x == 0) {
        double* Hj = t.H + (size_t)j * (m + 1);
        for (int i = 0; i <= j; ++i) Hj[i] = hs[i];
        t.flags[0] = 0;
        t.st[m + 3] = w0;
        t.st[2 * m + 5] = a;
    }
}

// One Arnoldi column, run by one block (the reductions it needs are done by k_reduce_partials).
//
// stage 0: after the first Gram-Schmidt pass, decide whether a second pass runs (reorth 2:
// always; 1: when the norm fell below 1/sqrt2 of its value; 0: never) and store h into H[:, j].
// stage 1: add the second pass, form H[j+1, j], apply the previous Givens rotations and a new
// one, update the residual vector g, and write the estimate |g[j+1]| and 1/H[j+1, j].
//
// fused (one pass only): the update also normalises.  Stage 0 then estimates the norm of
// w - V h as sqrt(|w|^2 - |h|^2) (orthonormal V) and stores the factor a = 1/estimate in
// st[2m+5] (a = 1 when the difference has lost more than five digits to cancellation).  The
// update writes a (w - V h) and its squared norm nu2 into st[j+2].  Stage 1 takes
// H[j+1, j] = 1/a, the exact factor of the stored vector; when nu2 is not 1 within renorm_tol (or
// on breakdown) it sets flags[3] and inv[j+1] = 1/sqrt(nu2), and the caller's rescale pass, which
// runs only under that flag, makes the stored vector unit-norm with H[j+1, j] = sqrt(nu2)/a.
// st layout: [0..m] h pass 1 | [m+1] |w|^2 | [m+2] |w1|^2 | [m+4..2m+4] h pass 2 | [2m+5] a
__device__ __forceinline__ void arnoldi_block(const ArnoldiArgs t) {
    __shared__ double red[ARN_MAXROW];
    __shared__ double hl[ARN_MAXROW], csl[ARN_MAXROW], snl[ARN_MAXROW];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int j = t.j, m = t.m;
    double* Hj = t.H + (size_t)j * (m + 1);
    if (t.stage == 0)   // h, |w|^2 (and |w1|^2 after a separate update) into LDS
        for (int i = tid; i <= j + 2; i += nt) red[i] = t.st[i];
    if (t.stage == 1) {   // the column and the rotations, loaded in parallel
        for (int i = tid; i <= j; i += nt) hl[i] = Hj[i];
        for (int i = tid; i < j; i += nt) {
            csl[i] = t.cs[i];
            snl[i] = t.sn[i];
        }
    }
    __syncthreads();
    if (tid != 0) return;
    // thread 0: the scalar bookkeeping, from registers and LDS (no reads of its own global writes)
    double* st = t.st;
    int* flags = t.flags;
    if (t.stage == 0) {
        // red holds h[0..j] and |w|^2 (and |w1|^2 when the update ran first)
        const double w0 = red[j + 1];
        double hh = 0.0;
        for (int i = 0; i <= j; ++i) {
            const double hi = red[i];
            Hj[i] = hi;
            hh += hi * hi;
        }
        flags[0] = (t.reorth == 2 || (t.reorth == 1 && red[j + 2] < 0.5 * w0)) ? 1 : 0;
        st[m + 3] = w0;   // |w|^2 before orthogonalisation
        if (t.fused) st[2 * m + 5] = fused_factor(w0, hh);
        return;
    }
    const int second = flags[0];
    const int prev_nonfinite = flags[2];
    const double w0 = st[m + 3];
    const double w1r = st[j + 2];
    const double a = t.fused ? st[2 * m + 5] : 1.0;
    const double gj = t.g[j];
    if (second) {
        const double* h2 = st + m + 4;
        for (int i = 0; i <= j; ++i) hl[i] += h2[i];
    }
    const double w1 = w1r > 0.0 ? w1r : 0.0;
    double hn, hval, inv;
    bool renorm = false, breakdown;
    if (t.fused) {
        fused_decision(w1r, a, w0, t.renorm_tol, hn, renorm, breakdown, inv);
        hval = renorm ? hn : 1.0 / a;
    } else {
        hn = sqrt(w1);
        hval = hn;
        breakdown = !(hn > 1e-14 * sqrt(w0 > 0.0 ? w0 : 0.0));
        inv = breakdown ? 0.0 : 1.0 / hn;
    }
    hl[j + 1] = hval;
    for (int i = 0; i < j; ++i) {
        const double x = csl[i] * hl[i] + snl[i] * hl[i + 1];
        hl[i + 1] = -snl[i] * hl[i] + csl[i] * hl[i + 1];
        hl[i] = x;
    }
    const double den = hypot(hl[j], hl[j + 1]);
    double cj, sj;
    if (den == 0.0) { cj = 1.0; sj = 0.0; }
    else { cj = hl[j] / den; sj = hl[j + 1] / den; }
    t.cs[j] = cj;
    t.sn[j] = sj;
    hl[j] = den;
    hl[j + 1] = 0.0;
    for (int i = 0; i <= j + 1; ++i) Hj[i] = hl[i];
    const double gn = -sj * gj;
    t.g[j + 1] = gn;
    t.g[j] = cj * gj;
    const double ej = fabs(gn);
    t.est[j] = ej;
    const bool nonfinite = !isfinite(den) || !isfinite(ej);
    // factor that makes the stored vector unit-norm (fused: relative to the scaled vector)
    t.inv[j + 1] = inv;
    flags[1] = breakdown ? 1 : 0;
    flags[3] = (breakdown || renorm) ? 1 : 0;
    if (nonfinite) flags[2] = 1;
    // the host polls est_out (a write-once slot): the flags go out first, behind a system fence
    if (t.flags_out) {
        t.flags_out[0] = breakdown ? 1 : 0;
        t.flags_out[1] = (nonfinite || prev_nonfinite) ? 1 : 0;
    }
    if (t.est_out) {
        __threadfence_system();
        *t.est_out = ej;
    }
}


// Sum of partial[0..nblk) over the whole block in a fixed order (thread-strided sums, four loads
// in flight per step, then a wave reduction and the wave results in index order); every block
// that calls it gets the same bits.  Valid in every thread.
__device__ __forceinline__ double block_sum_fixed(const double* __restrict__ partial, int nblk) {
    __shared__ double wsum[16];
    __shared__ double total;
    const int tid = threadIdx.x, nt = blockDim.x;
    double s = 0.0;
    int b = tid;
    for (; b + 3 * nt < nblk; b += 4 * nt) {
        const double a0 = partial[b], a1 = partial[b + nt], a2 = partial[b + 2 * nt], a3 = partial[b + 3 * nt];
        s += (a0 + a1) + (a2 + a3);
    }
    // at most three values are left per thread: loaded together rather than one after another
    {
        const double t0 = b < nblk ? partial[b] : 0.0;
        const double t1 = b + nt < nblk ? partial[b + nt] : 0.0;
        const double t2 = b + 2 * nt < nblk ? partial[b + 2 * nt] : 0.0;
        s += (t0 + t1) + t2;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((tid & 63) == 0) wsum[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < (nt + 63) / 64; ++w) t += wsum[w];
        total = t;
    }
    __syncthreads();
    return total;
}

// Stage 1 of the fused single pass inside the rescale kernel: every block adds up the update's
// per-block partial sums of nu2 (partial[0..nblk), fixed order) and decides from nu2, a
// (st[2m+5]) and |w|^2 (st[m+3]) whether the stored vector needs the rescale, and by which factor;
// block 0 also stores nu2 in st[j+2] and runs the column's bookkeeping (arnoldi_block).  Returns
// that factor, or a negative value when nothing is to be done; every thread of the block gets it.
__device__ __forceinline__ double arnoldi_stage1_in_rescale(const ArnoldiArgs& t, const double* partial, int nblk) {
    __shared__ double inv_sh;
    const double nu2 = block_sum_fixed(partial, nblk);
    if (threadIdx.x == 0) {
        double hn, inv;
        bool renorm, breakdown;
        fused_decision(nu2, t.st[2 * t.m + 5], t.st[t.m + 3], t.renorm_tol, hn, renorm, breakdown, inv);
        inv_sh = (renorm || breakdown) ? inv : -1.0;
        if (blockIdx.x == 0) t.st[t.j + 2] = nu2;   // read back by arnoldi_block in this thread
    }
    if (blockIdx.x == 0) arnoldi_block(t);
    __syncthreads();
    return inv_sh;
}

}  // namespace rte
