// Pass B of the 2D apply for one value of L (this file is compiled once per L = 0..8 with
// -DRTE_PASSB_L=<L>): FFT along y of every channel, per-frequency mode coupling with the kernel
// spectra, inverse FFT along y (Sec. 3.3.1: the kernel depends on x - y and on k' - k only, so
// the convolution over y and the sum over k' meet at each frequency).
//
// Fused form: the NCOL x C column spectra of a block live in LDS (C = 2L+1 channels, NCOL
// adjacent columns), transformed by one batched FFT; each thread then couples the modes at its
// frequencies and writes them back in place; one batched inverse FFT; store the first ny rows.
// Split form (FP64 when C x PY does not fit in LDS): forward y-FFTs to a full-length buffer,
// a pointwise coupling kernel, inverse y-FFTs.
//
// Coupling at frequency (kx, ky), for channels a_0 = u_0, (a_k, b_k) = sqrt2 (Re u_k, Im u_k):
//   W_{+-k} = (A_k +- i B_k)/sqrt2 (W_0 = A_0)   -- the complex modes
//   V_k = sum_{k'} Khat_{k'-k} W_{k'},  k = -L..L  -- Toeplitz in the mode index
//   out: A_0 = V_0, A_k = (V_k + V_{-k})/sqrt2, B_k = -i (V_k - V_{-k})/sqrt2
// with Khat read from the quarter table (see apply2d.hip for the symmetries).
#include "apply2d.h"
#include "apply2d_b.h"
#include "apply2d_tile.h"
#include "fft.h"
#include "passb_split.h"

#ifndef RTE_PASSB_L
#error "compile with -DRTE_PASSB_L=<L>"
#endif

namespace rte {

template <typename T, int L>
__device__ __forceinline__ void couple_modes(cx<T>* v /* C values, in/out */, const cx<T>* __restrict__ Q,
                                             size_t qstride_m, size_t qoff, bool flip) {
    constexpr int C = 2 * L + 1;
    const T r2 = (T)0.70710678118654752440084436210485;
    cx<T> W[C];   // complex modes k' = -L..L at index k' + L
    W[L] = v[0];
#pragma unroll
    for (int k = 1; k <= L; ++k) {
        const cx<T> a = v[2 * k - 1], bb = v[2 * k];
        W[L + k] = scale(a + mul_i(bb), r2);
        W[L - k] = scale(a - mul_i(bb), r2);
    }
    cx<T> V[C];
#pragma unroll
    for (int k = 0; k < C; ++k) V[k] = mk((T)0, (T)0);
    // V_k += Khat_m W_{k+m} and V_k += Khat_{-m} W_{k-m}, one kernel spectrum at a time
#pragma unroll
    for (int m = 0; m <= 2 * L; ++m) {
        cx<T> K = Q[m * qstride_m + qoff];
        if (flip) { K.im = -K.im; if (m & 1) { K.re = -K.re; K.im = -K.im; } }
#pragma unroll
        for (int k = -L; k + m <= L; ++k) cmac(V[k + L], K, W[k + m + L]);
        if (m > 0) {
            cx<T> Kn = conj(K);                     // Khat_{-m} = (-1)^m conj Khat_m
            if (m & 1) { Kn.re = -Kn.re; Kn.im = -Kn.im; }
#pragma unroll
            for (int k = -L + m; k <= L; ++k) cmac(V[k + L], Kn, W[k - m + L]);
        }
    }
    v[0] = V[L];
#pragma unroll
    for (int k = 1; k <= L; ++k) {
        v[2 * k - 1] = scale(V[L + k] + V[L - k], r2);
        v[2 * k] = scale(mul_mi(V[L + k] - V[L - k]), r2);
    }
}

// The same coupling reading the C channel values at base[c * stride] and writing the result back in
// place, accumulated diagonal by diagonal (one kernel spectrum K_m at a time, all 2L+1 outputs
// accumulating in parallel: 2L+1 independent FMA chains per thread).
template <typename T, int L>
__device__ __forceinline__ void couple_inplace(cx<T>* base, int stride, const cx<T>* __restrict__ Q,
                                                    size_t qstride_m, size_t qoff, bool flip) {
    constexpr int C = 2 * L + 1;
    const T r2 = (T)0.70710678118654752440084436210485;
    cx<T> W[C];
    W[L] = base[0];
#pragma unroll
    for (int k = 1; k <= L; ++k) {
        const cx<T> a = base[(2 * k - 1) * stride], bb = base[2 * k * stride];
        W[L + k] = scale(a + mul_i(bb), r2);
        W[L - k] = scale(a - mul_i(bb), r2);
    }
    cx<T> V[C];
#pragma unroll
    for (int k = 0; k < C; ++k) V[k] = mk((T)0, (T)0);
#pragma unroll
    for (int m = 0; m <= 2 * L; ++m) {
        cx<T> K = Q[m * qstride_m + qoff];
        if (flip) { K.im = -K.im; if (m & 1) { K.re = -K.re; K.im = -K.im; } }
        // V_k += Khat_m W_{k+m}; for m > 0 also V_k += Khat_{-m} W_{k-m}, Khat_{-m} = (-1)^m conj Khat_m
#pragma unroll
        for (int k = -L; k + m <= L; ++k) cmac(V[k + L], K, W[k + m + L]);
        if (m > 0) {
            cx<T> Kn = conj(K);
            if (m & 1) { Kn.re = -Kn.re; Kn.im = -Kn.im; }
#pragma unroll
            for (int k = -L + m; k <= L; ++k) cmac(V[k + L], Kn, W[k - m + L]);
        }
    }
    base[0] = V[L];
#pragma unroll
    for (int k = 1; k <= L; ++k) {
        base[(2 * k - 1) * stride] = scale(V[L + k] + V[L - k], r2);
        base[2 * k * stride] = scale(mul_mi(V[L + k] - V[L - k]), r2);
    }
}

// Column 0 of a packed work buffer holds z = d + i q with d, q the (real) x-frequency-0 and
// x-frequency-PX/2 sequences in y.  At y-frequency f (and its mirror -f):
// D = (Z(f) + conj Z(-f))/2 and Q = (Z(f) - conj Z(-f))/(2i) are their spectra; each is coupled
// with its own kernel column and Z(f) = D' + i Q', Z(-f) = conj D' + i conj Q' recombined
// (D' and Q' are spectra of real sequences).  p(c) addresses Z(f) of channel c, pm(c) Z(-f); the
// coupled D' is parked in the Z(f) slot while Q is coupled, to keep few values live.
template <typename T, int L, typename PF, typename PM>
__device__ __forceinline__ void couple_packed_pair(PF p, PM pm, const cx<T>* __restrict__ Q, size_t qstride_m,
                                                   size_t qoff_dc, size_t qoff_ny, bool self, bool single = false) {
    // single: only channel 0 of the input is non-zero (the others are not read)
    constexpr int C = 2 * L + 1;
    const cx<T> zero = mk((T)0, (T)0);
    cx<T> v[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const bool in = !single || c == 0;
        const cx<T> z = in ? *p(c) : zero, w = in ? conj(*pm(c)) : zero;
        v[c] = scale(z + w, (T)0.5);
    }
    couple_modes<T, L>(v, Q, qstride_m, qoff_dc, false);
    cx<T> q[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const bool in = !single || c == 0;
        const cx<T> z = in ? *p(c) : zero, w = in ? conj(*pm(c)) : zero;
        q[c] = scale(mul_mi(z - w), (T)0.5);
        *p(c) = v[c];                       // park D'
    }
    couple_modes<T, L>(q, Q, qstride_m, qoff_ny, false);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const cx<T> d = *p(c);
        *p(c) = d + mul_i(q[c]);
        if (!self) *pm(c) = conj(d) + mul_i(conj(q[c]));
    }
}

// Default group size of the fused pass's y-transforms: at most ~3 radix-8 butterflies per thread
// and stage.  Fewer groups mean fewer barriers but more live registers per thread.
template <int PY, int NF, int NTHR>
constexpr int default_group() {
    constexpr int g = (3 * NTHR * 8) / PY;
    return g >= NF ? NF : (g < 1 ? 1 : g);
}

// Fused pass B: NCOL columns x C channels per block, spectra resident in LDS.
// base: the batch entry's [C][nkx][ny] work buffer; nkx = its columns, nkq = columns of the kernel
// table (PX/2 + 1); kx0 = the block's first column.
template <typename T, int PY, int L, int NCOL, int NTHR, int GV = 0, int SCH = 0, bool CORR = false>
__device__ __forceinline__ void pass_b_cols(cx<T>* __restrict__ base, const cx<T>* __restrict__ Q, int ny, int nkx,
                                            int nkq, int pack, int kx0, cx<T>* spec, const cx<T>* tws,
                                            cx<T>* pairtmp, int tid, int single = 0, const CorrB* cb = nullptr) {
    // single: only channel 0 of the input is non-zero; the other channels are not read
    constexpr int C = 2 * L + 1;
    constexpr int NF = NCOL * C;
    constexpr int LD = padded(PY);
    constexpr int KH = PY / 2 + 1;
    constexpr int HY = PY / 2;
    const size_t cstride = (size_t)nkx * ny;
    // Forward y-FFT of the NF = NCOL * C column sequences into spec[(col * C + c) * LD + sw(.)].
    // Rows y >= ny (<= PY/2) are zero padding, so the first Stockham stage (radix R0, no twiddles)
    // is done in registers straight from the loads: butterfly j takes inputs y = j + r PY/R0, of
    // which only r < R0/2 can be non-zero, and writes its R0 outputs at j R0 + r.
    constexpr int R0 = fft_radix(PY, 1, SCH);
    constexpr int NB0 = PY / R0;
    constexpr int NBT = NF * NB0;
    constexpr int IT = (NBT + NTHR - 1) / NTHR;
    // The coarse correction's x-spectrum (CorrB): G[fc][R] = coef_c sum_X y_c[R][X] phi[X][kx] for
    // the block's columns, interpolated in y onto every loaded row.  A thread's first G item has
    // its (L2-resident) loads issued before the column loads, so that their latency hides behind
    // those.
    //   When a wave's transform index is the same for all its lanes (NB0 a multiple of 64) and the
    // same rows recur at every step it, each wave computes the G values of its own transforms
    // into private slots among the pad slots of spec (never written by the transforms, see sw)
    // and reads them back after a wave-level fence: no block barrier, so the waves' column loads
    // still overlap one another's first stage.  Otherwise G and a table of the rows'
    // y-interpolation go through spec, behind two barriers.
    constexpr int GU = 16;
    constexpr bool WAVEG = CORR && NB0 % 64 == 0 && NTHR % NB0 == 0 && NTHR <= NF * (PY / 16);
    T gy[CORR ? GU : 1];
    cx<T> gp[CORR ? GU : 1];
    int Hc = 1, Wc = 1;
    bool wg = false;
    const cx<T>* phi = nullptr;
    const int wave = tid >> 6, lane = tid & 63;
    // pad slot e (< 64) of this wave
    auto gslot = [&](int e) -> cx<T>* {
        const int q = wave * 64 + e;
        return spec + (q / (PY / 16)) * LD + 17 * (q % (PY / 16)) + 16;
    };
    if constexpr (CORR) {
        Hc = cb->Hc;
        Wc = cb->Wc;
        phi = reinterpret_cast<const cx<T>*>(cb->phi);
        wg = WAVEG && IT * Hc <= 64;
        int fc, R;
        bool ok;
        if (wg) {   // lane = it Hc + R
            const int itl = lane / Hc;
            R = lane % Hc;
            fc = (64 * wave + itl * NTHR) / NB0;
            ok = itl < IT && fc < NF;
        } else {
            fc = tid / Hc;
            R = tid % Hc;
            ok = tid < NF * Hc;
        }
        const int kx = kx0 + fc / C;
        ok = ok && kx < nkx;
        // Each lane reads its own coarse row as 16-byte loads (rows are whole float4s, CorrB), an
        // instruction touching a quarter of the cache lines that single floats would.  Every load
        // takes a clamped in-range index instead of a branch, and the sums below skip the values
        // out of range: per-load branches made the compiler wait for these loads before issuing
        // the column loads.
        const float4* y4 = reinterpret_cast<const float4*>(cb->y + (ok ? ((size_t)(fc % C) * Hc + R) * Wc : 0));
#pragma unroll
        for (int q = 0; q < GU / 4; ++q) {
            const float4 t = y4[4 * q < Wc ? q : 0];
            gy[4 * q] = (T)t.x;
            gy[4 * q + 1] = (T)t.y;
            gy[4 * q + 2] = (T)t.z;
            gy[4 * q + 3] = (T)t.w;
        }
#pragma unroll
        for (int u = 0; u < GU; ++u) gp[u] = phi[(ok && u < Wc) ? (size_t)u * nkx + kx : 0];
    }
    cx<T> ld[IT][R0 / 2];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int idx = tid + it * NTHR;
        const int j = idx % NB0, fc = idx / NB0;
        const int col = fc / C, c = fc % C;
        const int kx = kx0 + col;
        const bool ok = (NBT % NTHR == 0 || idx < NBT) && kx < nkx && (!single || c == 0);
        // every load takes a clamped in-range index instead of a branch, and the values out of
        // range are zeroed where they are first used (the first stage below): behind per-load
        // branches, or with a product right after each load, the compiler waited for the first
        // loads before issuing the rest
#pragma unroll
        for (int r = 0; r < R0 / 2; ++r) {
            const int y = j + r * NB0;
            ld[it][r] = base[(ok && y < ny) ? c * cstride + (size_t)kx * ny + y : 0];
        }
    }
    // keep the column loads issued ahead of the correction's arithmetic, which waits on its own
    // (earlier) loads only
    if constexpr (CORR) __builtin_amdgcn_sched_barrier(0);
    if (CORR && wg) {
        const int itl = lane / Hc, R = lane % Hc;
        const int fc = (64 * wave + itl * NTHR) / NB0;
        const int kx = kx0 + fc / C;
        T gr = 0, gi = 0;
        if (itl < IT && fc < NF && kx < nkx) {
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const T yv = u < Wc ? gy[u] : (T)0;
                gr += yv * gp[u].re;
                gi += yv * gp[u].im;
            }
            const float* yr = cb->y + ((size_t)(fc % C) * Hc + R) * Wc;
            for (int X = GU; X < Wc; ++X) {
                const T yv = (T)yr[X];
                const cx<T> ph = phi[(size_t)X * nkx + kx];
                gr += yv * ph.re;
                gi += yv * ph.im;
            }
            const T k = (T)cb->coef[fc % C];
            gr *= k;
            gi *= k;
        }
        *gslot(lane) = mk(gr, gi);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // this thread's rows (the same at every it): lower coarse row and weight of the upper one
        const int j = tid % NB0;
        const float invF = 1.f / (float)cb->F;
        int rlo[R0 / 2];
        T wt[R0 / 2];
#pragma unroll
        for (int r = 0; r < R0 / 2; ++r) {
            const float yi = ((float)(j + r * NB0) + 0.5f) * invF - 0.5f;
            const float f0 = floorf(yi);
            const int i0 = (int)f0;
            rlo[r] = min(max(i0, 0), Hc - 1);
            wt[r] = (i0 < 0 || i0 >= Hc - 1) ? (T)0 : (T)(yi - f0);
        }
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int idx = tid + it * NTHR;
            const int kx = kx0 + (idx / NB0) / C;
            const bool ok = (NBT % NTHR == 0 || idx < NBT) && kx < nkx;
#pragma unroll
            for (int r = 0; r < R0 / 2; ++r) {
                if (ok && j + r * NB0 < ny) {
                    const cx<T> g0 = *gslot(it * Hc + rlo[r]), g1 = *gslot(it * Hc + min(rlo[r] + 1, Hc - 1));
                    ld[it][r].re += g0.re + wt[r] * (g1.re - g0.re);
                    ld[it][r].im += g0.im + wt[r] * (g1.im - g0.im);
                }
            }
        }
    } else if constexpr (CORR) {
        for (int idx = tid; idx < NF * Hc; idx += NTHR) {
            const int fc = idx / Hc, R = idx % Hc;
            const int c = fc % C;
            const int kx = kx0 + fc / C;
            T gr = 0, gi = 0;
            if (kx < nkx) {
                if (idx == tid) {
#pragma unroll
                    for (int u = 0; u < GU; ++u) {
                        const T yv = u < Wc ? gy[u] : (T)0;
                        gr += yv * gp[u].re;
                        gi += yv * gp[u].im;
                    }
                }
                const float* yr = cb->y + ((size_t)c * Hc + R) * Wc;
                for (int X = idx == tid ? GU : 0; X < Wc; ++X) {
                    const T yv = (T)yr[X];
                    const cx<T> ph = phi[(size_t)X * nkx + kx];
                    gr += yv * ph.re;
                    gi += yv * ph.im;
                }
            }
            const T k = (T)cb->coef[c];
            spec[idx] = mk(k * gr, k * gi);
        }
        // the y-interpolation of every row (lerp_at) after G: (weight of the upper row, lower row);
        // rows clamped to one coarse row get weight 0
        cx<T>* rt = spec + NF * Hc;
        for (int y = tid; y < ny; y += NTHR) {
            int r0, r1;
            float ay;
            lerp_at(y, cb->F, Hc, r0, r1, ay);
            rt[y] = mk(r1 == r0 ? (T)0 : (T)ay, (T)r0);
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int idx = tid + it * NTHR;
            const int j = idx % NB0, fc = idx / NB0;
            const int kx = kx0 + fc / C;
            const bool ok = (NBT % NTHR == 0 || idx < NBT) && kx < nkx;
            const cx<T>* g = spec + fc * Hc;
#pragma unroll
            for (int r = 0; r < R0 / 2; ++r) {
                const int y = j + r * NB0;
                if (ok && y < ny) {
                    const cx<T> t = rt[y];
                    const int r0 = (int)t.im;
                    const cx<T> g0 = g[r0], g1 = g[min(r0 + 1, Hc - 1)];
                    ld[it][r].re += g0.re + t.re * (g1.re - g0.re);
                    ld[it][r].im += g0.im + t.re * (g1.im - g0.im);
                }
            }
        }
        __syncthreads();   // G is read before the first stage overwrites spec
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int idx = tid + it * NTHR;
        if (NBT % NTHR == 0 || idx < NBT) {
            const int j = idx % NB0, fc = idx / NB0;
            const int c = fc % C, kx = kx0 + fc / C;
            const bool ok = kx < nkx && (!single || c == 0);
            cx<T> v[R0];
#pragma unroll
            for (int r = 0; r < R0; ++r)
                v[r] = (r < R0 / 2 && ok && j + r * NB0 < ny) ? ld[it][r] : mk((T)0, (T)0);
            dft_small<T, R0, false>(v);
#pragma unroll
            for (int r = 0; r < R0; ++r) spec[fc * LD + sw(j * R0 + r)] = v[r];
        }
    }
    __syncthreads();
    // the default groups, or groups of GV transforms if given (the radix-32 schedule transforms
    // every sequence at once)
    constexpr int G0 = SCH == 1 ? NF : default_group<PY, NF, NTHR>();
    constexpr int G = GV > 0 ? (GV < NF ? GV : NF) : G0;
    block_fft_grouped_range<T, PY, NF, G, LD, NTHR, false, R0, PY, SCH>(spec, tws, tid);
    const size_t qs = (size_t)nkq * KH;
    // Frequencies are visited in the order [0, PY/4), [3PY/4, PY), [PY/4, 3PY/4): with PY/2 threads
    // a frequency and its mirror PY - f, which read the same quarter-table entries, fall in the
    // same sweep, so the second read finds the entries in L2.
#pragma unroll 1
    for (int idx = tid; idx < NCOL * PY; idx += NTHR) {
        const int fi = idx % PY, col = idx / PY;
        const int f = fi < PY / 4 ? fi : (fi < PY / 2 ? fi + PY / 2 : fi - PY / 4);
        const int kx = kx0 + col;
        if (kx >= nkx) continue;
        cx<T>* sp = spec + col * C * LD;
        if (pack && kx == 0) {
            if (f > HY) continue;
            const int fm = (PY - f) & (PY - 1);
            const bool self = fm == f;
            cx<T>* zf = sp + sw(f);
            cx<T>* zq = self ? pairtmp + (f == 0 ? 0 : C) : sp + sw(fm);   // where Q is coupled
            // split into the spectra D (kept at f) and Q of the two real sequences
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const cx<T> z = zf[c * LD], w = conj(self ? z : zq[c * LD]);
                zf[c * LD] = scale(z + w, (T)0.5);
                zq[c * (self ? 1 : LD)] = scale(mul_mi(z - w), (T)0.5);
            }
            couple_inplace<T, L>(zf, LD, Q, qs, (size_t)f, false);
            couple_inplace<T, L>(zq, self ? 1 : LD, Q, qs, (size_t)(nkq - 1) * KH + f, false);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const cx<T> d = zf[c * LD], q = zq[c * (self ? 1 : LD)];
                zf[c * LD] = d + mul_i(q);
                if (!self) zq[c * LD] = conj(d) + mul_i(conj(q));
            }
        } else {
            const bool flip = f > HY;
            const int fy = flip ? PY - f : f;
            couple_inplace<T, L>(sp + sw(f), LD, Q, qs, (size_t)kx * KH + fy, flip);
        }
    }
    __syncthreads();
    // Inverse y-FFT: every stage but the last in LDS; the last stage (sub-length NSL, radix RL) goes
    // straight to memory, where only its outputs y = j + r NSL < ny are kept.
    constexpr int NSL = fft_last_ns(PY, SCH);
    constexpr int RL = PY / NSL;
    block_fft_grouped_range<T, PY, NF, G, LD, NTHR, true, 1, NSL, SCH>(spec, tws, tid);
    constexpr int TWL = stage_tw_offset(PY, NSL, SCH);
    for (int idx = tid; idx < NF * NSL; idx += NTHR) {
        const int j = idx % NSL, fc = idx / NSL;
        const int col = fc / C, c = fc % C;
        const int kx = kx0 + col;
        cx<T> v[RL];
#pragma unroll
        for (int r = 0; r < RL; ++r) v[r] = spec[fc * LD + sw(j + r * NSL)];
        if constexpr (NSL > 1) {   // a single-stage transform has no twiddles
#pragma unroll
            for (int r = 1; r < RL; ++r) {
                cx<T> w = tws[TWL + j * (RL - 1) + (r - 1)];
                w.im = -w.im;
                v[r] = v[r] * w;
            }
        }
        dft_small<T, RL, true>(v);
        if (kx < nkx) {
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int y = j + r * NSL;
                if (y < ny) base[c * cstride + (size_t)kx * ny + y] = v[r];
            }
        }
    }
}

template <typename T, int PY, int L, int NCOL, int NTHR, int GV, int SCH = 0, bool CORR = false>
__global__ __launch_bounds__(NTHR) void k_pass_b_lds(cx<T>* __restrict__ Tb, const cx<T>* __restrict__ Q,
                                                     const cx<T>* __restrict__ tw, int ny, int nkx, int nkq,
                                                     int pack, int single, CorrB cb) {
    constexpr int C = 2 * L + 1;
    __shared__ cx<T> spec[NCOL * C * padded(PY)];
    __shared__ cx<T> tws[PY];
    __shared__ cx<T> pairtmp[2 * C];   // Q of the two self-mirrored frequencies of a packed column
    const int tid = threadIdx.x;
    stage_twiddles<T, PY, NTHR>(tws, tw, tid);
    pass_b_cols<T, PY, L, NCOL, NTHR, GV, SCH, CORR>(Tb + (size_t)blockIdx.y * C * nkx * ny, Q, ny, nkx, nkq, pack,
                                                blockIdx.x * NCOL, spec, tws, pairtmp, tid, single, &cb);
}

// Register-resident form (unpacked work buffer: x-frequencies 0 and PX/2 in columns of their
// own).  One column per block; each thread owns FPT y-frequencies: FPT = 1, PY threads, thread t
// owns t; FPT = 2, PY/2 threads, thread t owns the mirror pair (t, PY - t) (thread 0: 0 and PY/2),
// which read the same entries of the quarter kernel table.  The forward y-FFTs run G channels at a
// time through LDS and every thread keeps its frequencies of those channels in registers; the mode
// coupling then runs from registers; the inverse y-FFTs run G channels at a time again, each thread
// writing its coupled values back into LDS first.  LDS holds G transforms instead of all 2L+1.
// The mode coupling of couple_modes done in place on v: the channel pairs become the complex
// modes in their own slots (slot 0: W_0, slot 2k-1: W_k, slot 2k: W_-k), only the 2L+1
// accumulators are extra (fewer live registers when other columns' values are held too).
template <typename T, int L>
__device__ __forceinline__ constexpr int mode_slot(int k) { return k == 0 ? 0 : (k > 0 ? 2 * k - 1 : -2 * k); }

template <typename T, int L>
__device__ __forceinline__ void couple_regs(cx<T>* v, const cx<T>* __restrict__ Q, size_t qstride_m, size_t qoff,
                                            bool flip) {
    constexpr int C = 2 * L + 1;
    const T r2 = (T)0.70710678118654752440084436210485;
#pragma unroll
    for (int k = 1; k <= L; ++k) {
        const cx<T> a = v[2 * k - 1], bb = v[2 * k];
        v[2 * k - 1] = scale(a + mul_i(bb), r2);
        v[2 * k] = scale(a - mul_i(bb), r2);
    }
    cx<T> V[C];   // V_k at index k + L
#pragma unroll
    for (int k = 0; k < C; ++k) V[k] = mk((T)0, (T)0);
#pragma unroll
    for (int m = 0; m <= 2 * L; ++m) {
        cx<T> K = Q[m * qstride_m + qoff];
        if (flip) { K.im = -K.im; if (m & 1) { K.re = -K.re; K.im = -K.im; } }
#pragma unroll
        for (int k = -L; k + m <= L; ++k) cmac(V[k + L], K, v[mode_slot<T, L>(k + m)]);
        if (m > 0) {
            cx<T> Kn = conj(K);                     // Khat_{-m} = (-1)^m conj Khat_m
            if (m & 1) { Kn.re = -Kn.re; Kn.im = -Kn.im; }
#pragma unroll
            for (int k = -L + m; k <= L; ++k) cmac(V[k + L], Kn, v[mode_slot<T, L>(k - m)]);
        }
    }
    v[0] = V[L];
#pragma unroll
    for (int k = 1; k <= L; ++k) {
        v[2 * k - 1] = scale(V[L + k] + V[L - k], r2);
        v[2 * k] = scale(mul_mi(V[L + k] - V[L - k]), r2);
    }
}

template <typename T, int L, int FPT>
struct RegCol {
    cx<T> d[FPT][2 * L + 1];
};

template <typename T, int PY, int L, int G, int FPT, int C0>
__device__ __forceinline__ void reg_forward(RegCol<T, L, FPT>& r, const cx<T>* __restrict__ base, size_t cstride,
                                            int kx, int ny, int single, cx<T>* spec, const cx<T>* tws, int tid,
                                            const int* f) {
    constexpr int C = 2 * L + 1;
    constexpr int NG = (C - C0) < G ? (C - C0) : G;
    constexpr int LD = padded(PY);
    constexpr int NT = PY / FPT;
    __syncthreads();   // the previous group's reads of spec are done
    fft_forward_padded<T, PY, NG, LD, NT>(spec, tws, tid, [&](int g, int y) {
        const int c = C0 + g;
        return (y < ny && (!single || c == 0)) ? base[c * cstride + (size_t)kx * ny + y] : mk((T)0, (T)0);
    });
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int q = 0; q < FPT; ++q) r.d[q][C0 + g] = spec[g * LD + sw(f[q])];
    if constexpr (C0 + NG < C)
        reg_forward<T, PY, L, G, FPT, C0 + NG>(r, base, cstride, kx, ny, single, spec, tws, tid, f);
}

template <typename T, int PY, int L, int G, int FPT, int C0>
__device__ __forceinline__ void reg_inverse(const RegCol<T, L, FPT>& r, cx<T>* __restrict__ base, size_t cstride,
                                            int kx, int ny, cx<T>* spec, const cx<T>* tws, int tid, const int* f) {
    constexpr int C = 2 * L + 1;
    constexpr int NG = (C - C0) < G ? (C - C0) : G;
    constexpr int LD = padded(PY);
    constexpr int NT = PY / FPT;
    __syncthreads();   // the previous group's last-stage reads of spec are done
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int q = 0; q < FPT; ++q) spec[g * LD + sw(f[q])] = r.d[q][C0 + g];
    __syncthreads();
    fft_inverse_cropped<T, PY, NG, LD, NT>(spec, tws, tid, [&](int g, int y, cx<T> v) {
        if (y < ny) base[(C0 + g) * cstride + (size_t)kx * ny + y] = v;
    });
    if constexpr (C0 + NG < C) reg_inverse<T, PY, L, G, FPT, C0 + NG>(r, base, cstride, kx, ny, spec, tws, tid, f);
}

template <typename T, int PY, int L, int G, int FPT, int MINW>
__global__ __launch_bounds__(PY / FPT, MINW) void k_pass_b_reg(cx<T>* __restrict__ Tb, const cx<T>* __restrict__ Q,
                                                            const cx<T>* __restrict__ tw, int ny, int nkx, int nkq,
                                                            int single) {
    constexpr int C = 2 * L + 1;
    constexpr int NT = PY / FPT;
    constexpr int KH = PY / 2 + 1;
    constexpr int HY = PY / 2;
    __shared__ cx<T> spec[G * padded(PY)];
    __shared__ cx<T> tws[PY];
    const int tid = threadIdx.x;
    const int kx = blockIdx.x;
    cx<T>* base = Tb + (size_t)blockIdx.y * C * nkx * ny;
    const size_t cstride = (size_t)nkx * ny;
    const size_t qs = (size_t)nkq * KH;
    stage_twiddles<T, PY, NT>(tws, tw, tid);
    int f[FPT];
    if constexpr (FPT == 1) f[0] = tid;
    else { f[0] = tid; f[1] = tid == 0 ? HY : PY - tid; }
    RegCol<T, L, FPT> r;
    reg_forward<T, PY, L, G, FPT, 0>(r, base, cstride, kx, ny, single, spec, tws, tid, f);
    const size_t qk = (size_t)kx * KH;
#pragma unroll
    for (int q = 0; q < FPT; ++q) {
        const bool flip = f[q] > HY;
        couple_regs<T, L>(r.d[q], Q, qs, qk + (flip ? PY - f[q] : f[q]), flip);
    }
    reg_inverse<T, PY, L, G, FPT, 0>(r, base, cstride, kx, ny, spec, tws, tid, f);
}

#if RTE_PASSB_L == 0
// Batched isotropic form: one block per (problem, group of NCOL columns).
template <typename T, int PY, int NCOL, int NTHR>
__global__ __launch_bounds__(NTHR) void k_pass_b_batch(const BatchProb<T>* __restrict__ probs,
                                                       const int2* __restrict__ items, const int* __restrict__ act) {
    __shared__ cx<T> spec[NCOL * padded(PY)];
    __shared__ cx<T> tws[PY];
    __shared__ cx<T> pairtmp[2];
    const int2 item = items[blockIdx.x];
    const BatchProb<T>& d = probs[item.x];
    if (act && !act[item.x]) return;
    const int tid = threadIdx.x;
    stage_twiddles<T, PY, NTHR>(tws, d.twy, tid);
    pass_b_cols<T, PY, 0, NCOL, NTHR>(d.work, d.Q, d.ny, d.PX / 2, d.PX / 2 + 1, 1, item.y * NCOL, spec, tws, pairtmp,
                                      tid);
}
#endif

// Split form, step 2/3: pointwise coupling over all (kx, ky).
template <typename T, int PY, int L>
__global__ __launch_bounds__(256) void k_pass_b_couple(cx<T>* __restrict__ T2, const cx<T>* __restrict__ Q,
                                                       int nkx, int nkq, int pack, int single) {
    constexpr int C = 2 * L + 1;
    constexpr int KH = PY / 2 + 1;
    const int b = blockIdx.y;
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)nkx * PY) return;
    // Adjacent threads take the mirrored frequencies f and PY - f, which read the same entries of
    // the quarter spectra, so a wave fetches each once: q = 2p -> f = p, q = 2p + 1 -> f = PY - p
    // (p = 0 -> f = PY/2); a bijection of [0, PY).
    const int kx = (int)(idx / PY), q = (int)(idx % PY);
    const int fp = q >> 1;
    const int f = (q & 1) ? (fp == 0 ? PY / 2 : PY - fp) : fp;
    const size_t cstride = (size_t)nkx * PY;
    const size_t qs = (size_t)nkq * KH;
    cx<T>* p = T2 + (size_t)b * C * cstride + (size_t)kx * PY;
    if (pack && kx == 0) {
        if (f > PY / 2) return;
        const int fm = (PY - f) & (PY - 1);
        couple_packed_pair<T, L>([&](int c) { return p + c * cstride + f; }, [&](int c) { return p + c * cstride + fm; },
                                 Q, qs, (size_t)f, (size_t)(nkq - 1) * KH + f, fm == f, single != 0);
        return;
    }
    const bool flip = f > PY / 2;
    const int fy = flip ? PY - f : f;
    cx<T> v[C];
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = (single && c > 0) ? mk((T)0, (T)0) : p[c * cstride + f];
    couple_modes<T, L>(v, Q, qs, (size_t)kx * KH + fy, flip);
#pragma unroll
    for (int c = 0; c < C; ++c) p[c * cstride + f] = v[c];
}

// Split form, steps 2 and 3 fused, by groups of output channels.  The coupling of one column at
// one frequency needs every input channel, so the column's spectra (2L+1 channels of PY entries)
// stay in the full-length buffer; a block takes a column and a group of output channels (modes 0
// and 1, then the pairs of modes 2g and 2g + 1: at most 4 channels), couples those channels at
// every frequency into LDS and runs their inverse y-FFTs, writing the kept rows.  Against the
// separate coupling and inverse kernels this skips one write and one read of the full-length
// buffer; the groups of a column run on one XCD, so the re-reads of its spectra and of its kernel
// column hit L2.
template <int L>
constexpr int couple_groups() { return (L + 2) / 2; }
template <int L, int G>
struct CGroup {
    static constexpr int klo = G == 0 ? 0 : 2 * G;                         // modes klo .. khi
    static constexpr int khi = (G == 0 ? 1 : 2 * G + 1) > L ? L : (G == 0 ? 1 : 2 * G + 1);
    static constexpr int ch0 = klo == 0 ? 0 : 2 * klo - 1;                // channels ch0 .. 2 khi
    static constexpr int nch = 2 * khi + 1 - ch0;
};

// The output channels of group G of the mode coupling at one frequency (conventions of
// couple_modes: V_k = sum_m Khat_m W_{k+m}, Khat_{-m} = (-1)^m conj Khat_m) from the 2L+1 input
// channels v; out[i] is channel ch0 + i.
template <typename T, int L, int G>
__device__ __forceinline__ void couple_group(const cx<T>* v, cx<T>* out, const cx<T>* __restrict__ Q,
                                             size_t qstride_m, size_t qoff, bool flip) {
    using CG = CGroup<L, G>;
    constexpr int C = 2 * L + 1;
    constexpr int KH = CG::khi;
    const T r2 = (T)0.70710678118654752440084436210485;
    cx<T> W[C];   // complex modes k' = -L..L at index k' + L
    W[L] = v[0];
#pragma unroll
    for (int k = 1; k <= L; ++k) {
        const cx<T> a = v[2 * k - 1], bb = v[2 * k];
        W[L + k] = scale(a + mul_i(bb), r2);
        W[L - k] = scale(a - mul_i(bb), r2);
    }
    cx<T> V[2 * KH + 1];   // modes k = -khi..khi at index k + khi (|k| >= klo used)
#pragma unroll
    for (int k = 0; k < 2 * KH + 1; ++k) V[k] = mk((T)0, (T)0);
#pragma unroll
    for (int m = 0; m <= KH + L; ++m) {
        cx<T> K = Q[m * qstride_m + qoff];
        if (flip) { K.im = -K.im; if (m & 1) { K.re = -K.re; K.im = -K.im; } }
        cx<T> Kn = conj(K);
        if (m & 1) { Kn.re = -Kn.re; Kn.im = -Kn.im; }
#pragma unroll
        for (int k = -KH; k <= KH; ++k) {
            if (k > -CG::klo && k < CG::klo) continue;
            if (k + m >= -L && k + m <= L) cmac(V[k + KH], K, W[k + m + L]);
            if (m > 0 && k - m >= -L && k - m <= L) cmac(V[k + KH], Kn, W[k - m + L]);
        }
    }
#pragma unroll
    for (int k = CG::klo; k <= KH; ++k) {
        if (k == 0) {
            out[0] = V[KH];
        } else {
            out[2 * k - 1 - CG::ch0] = scale(V[KH + k] + V[KH - k], r2);
            out[2 * k - CG::ch0] = scale(mul_mi(V[KH + k] - V[KH - k]), r2);
        }
    }
}

// The coupled output channels of group G at frequency f of column kx into spec (channel i of the
// group at spec[i * LD + sw(f)]).  Column 0 of a packed buffer holds z = d + i q: its D and Q
// spectra at f are formed from Z(f) and Z(PY - f) and coupled with the first and the last kernel
// column, one after the other (Z'(f) = D'(f) + i Q'(f)).
template <typename T, int PY, int L, int G, int LD>
__device__ __forceinline__ void couple_group_at(const cx<T>* __restrict__ col, size_t cstride, cx<T>* spec,
                                                const cx<T>* __restrict__ Q, size_t qs, int kx, int nkq, int f,
                                                bool packed, bool single) {
    constexpr int C = 2 * L + 1;
    constexpr int NCH = CGroup<L, G>::nch;
    constexpr int KH = PY / 2 + 1;
    const bool flip = f > PY / 2;
    const int fy = flip ? PY - f : f;
    const cx<T> zero = mk((T)0, (T)0);
    cx<T> v[C], o[NCH];
    if (!packed) {
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = (single && c > 0) ? zero : col[c * cstride + f];
        couple_group<T, L, G>(v, o, Q, qs, (size_t)kx * KH + fy, flip);
    } else {
        // D (s = 0) then Q (s = 1), through one coupling body so that only one is live
        const int fm = (PY - f) & (PY - 1);
#pragma unroll
        for (int i = 0; i < NCH; ++i) o[i] = zero;
#pragma unroll 1
        for (int s = 0; s < 2; ++s) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const bool in = !single || c == 0;
                const cx<T> z = in ? col[c * cstride + f] : zero, w = in ? conj(col[c * cstride + fm]) : zero;
                v[c] = scale(s ? mul_mi(z - w) : z + w, (T)0.5);
            }
            cx<T> os[NCH];
            couple_group<T, L, G>(v, os, Q, qs, (s ? (size_t)(nkq - 1) * KH : (size_t)0) + fy, flip);
#pragma unroll
            for (int i = 0; i < NCH; ++i) o[i] = o[i] + (s ? mul_i(os[i]) : os[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < NCH; ++i) spec[i * LD + sw(f)] = o[i];
}

template <typename T, int PY, int L, int NTHR>
__global__ __launch_bounds__(NTHR, 2) void k_pass_b_couple_inv(cx<T>* __restrict__ Tb, const cx<T>* __restrict__ T2,
                                                                const cx<T>* __restrict__ Q,
                                                                const cx<T>* __restrict__ tw, int ny, int nkx,
                                                                int nkq, int pack, int single) {
    constexpr int C = 2 * L + 1;
    constexpr int NG = couple_groups<L>();
    constexpr int GM = 4;                 // channels of the largest group
    constexpr int LD = padded(PY);
    __shared__ cx<T> spec[GM * LD];
    // block b runs on XCD b % 8: the NG groups of column kx take the blocks
    // 8 (NG (kx / 8) + g) + kx % 8, all on the XCD of kx % 8
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int kx = (slot / NG) * 8 + xcd, g = slot % NG;
    if (kx >= nkx) return;   // the whole block
    const int b = blockIdx.y, tid = threadIdx.x;
    const size_t cstride = (size_t)nkx * PY;
    const cx<T>* col = T2 + (size_t)b * C * cstride + (size_t)kx * PY;
    const size_t qs = (size_t)nkq * (PY / 2 + 1);
    const bool packed = pack && kx == 0;
    for (int i = tid; i < GM * LD; i += NTHR) spec[i] = mk((T)0, (T)0);   // the unused channels
    __syncthreads();
#pragma unroll 1
    for (int f = tid; f < PY; f += NTHR) {
        switch (g) {
            case 0: couple_group_at<T, PY, L, 0, LD>(col, cstride, spec, Q, qs, kx, nkq, f, packed, single); break;
            case 1: if constexpr (NG > 1) couple_group_at<T, PY, L, 1, LD>(col, cstride, spec, Q, qs, kx, nkq, f, packed, single); break;
            case 2: if constexpr (NG > 2) couple_group_at<T, PY, L, 2, LD>(col, cstride, spec, Q, qs, kx, nkq, f, packed, single); break;
            case 3: if constexpr (NG > 3) couple_group_at<T, PY, L, 3, LD>(col, cstride, spec, Q, qs, kx, nkq, f, packed, single); break;
            default: if constexpr (NG > 4) couple_group_at<T, PY, L, 4, LD>(col, cstride, spec, Q, qs, kx, nkq, f, packed, single); break;
        }
    }
    __syncthreads();
    const int ch0 = g == 0 ? 0 : 4 * g - 1;
    const int nch = (g == 0 ? 3 : 4) < C - ch0 ? (g == 0 ? 3 : 4) : C - ch0;
    cx<T>* dst = Tb + (size_t)b * C * nkx * ny + (size_t)kx * ny;
    const size_t ostride = (size_t)nkx * ny;
    fft_inverse_cropped<T, PY, GM, LD, NTHR>(spec, tw, tid, [&](int fl, int y, cx<T> v) {
        if (fl < nch && y < ny) dst[(size_t)(ch0 + fl) * ostride + y] = v;
    });
}

// Pass B split in halves (for columns whose spectra do not fit LDS at once: FP64 with many modes).
// The first decimation-in-frequency stage splits the length-PY y-transform of a column into its
// even and odd frequencies, the length-PH = PY/2 transforms of x[n] and x[n] W^n (W =
// exp(-2 pi i / PY); x[n] = 0 for n >= ny, and ny <= PH).  A block takes one column and runs the two
// halves one after the other with one half's spectra of every channel in LDS: forward transform,
// the mode coupling at that half's frequencies f = 2k + h, inverse transform.  The inverse of the
// whole column is e[n] + W^-n o[n] (e, o the inverse transforms of the even and odd halves): the
// even half's e goes to the scratch buffer E ([batch][C][columns][ny], like the work buffer), and
// the odd half adds its part and writes the column.  HBM: the column is read twice and e written
// and read once, against three passes over a full-length buffer in the split form.
template <typename T, int PY, int L, int NTHR>
__global__ __launch_bounds__(NTHR) void k_pass_b_half(cx<T>* __restrict__ Tb, cx<T>* __restrict__ E,
                                                      const cx<T>* __restrict__ Q, const cx<T>* __restrict__ twh,
                                                      int ny, int nkx, int nkq, int pack, int single) {
    constexpr int C = 2 * L + 1;
    constexpr int PH = PY / 2;
    constexpr int LD = padded(PH);
    constexpr int KH = PY / 2 + 1;
    constexpr int HY = PY / 2;
    constexpr int G = (3 * NTHR * 8) / PH >= C ? C : ((3 * NTHR * 8) / PH < 1 ? 1 : (3 * NTHR * 8) / PH);
    __shared__ cx<T> spec[C * LD];
    __shared__ cx<T> tws[PH];
    const int tid = threadIdx.x;
    const int kx = blockIdx.x, b = blockIdx.y;
    const size_t cstride = (size_t)nkx * ny;
    cx<T>* base = Tb + (size_t)b * C * cstride + (size_t)kx * ny;
    cx<T>* ebase = E + (size_t)b * C * cstride + (size_t)kx * ny;
    const size_t qs = (size_t)nkq * KH;
    stage_twiddles<T, PH, NTHR>(tws, twh, tid);
    for (int h = 0; h < 2; ++h) {
#pragma unroll 1
        for (int n = tid; n < PH; n += NTHR) {
            cx<T> w = mk((T)1, (T)0);
            if (h == 1) {
                double sn, cs;
                sincospi(-2.0 * (double)n / (double)PY, &sn, &cs);
                w = mk((T)cs, (T)sn);
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const cx<T> v = (n < ny && (!single || c == 0)) ? base[c * cstride + n] : mk((T)0, (T)0);
                spec[c * LD + sw(n)] = h ? v * w : v;
            }
        }
        __syncthreads();
        block_fft_grouped<T, PH, C, G, LD, NTHR, false>(spec, tws, tid);
        if (pack && kx == 0) {
            // column 0 packs the x-frequencies 0 and PX/2: split each frequency pair (f, PY - f), both
            // in this half, into the two real sequences' spectra (D kept at f, Q moved to PY - f),
            // couple each with its kernel column, recombine.  The Q of the two self-mirrored
            // frequencies (0 and PY/2) go to the slots 16 and 33 of each channel row, which the
            // swizzle sw() never uses, so that every coupling has the channel stride LD.
#pragma unroll 1
            for (int k = tid; k < PH; k += NTHR) {
                const int f = 2 * k + h;
                if (f > HY) continue;
                const int fm = (PY - f) & (PY - 1);
                const bool self = fm == f;
                cx<T>* zf = spec + sw(k);
                cx<T>* zq = spec + (self ? (f == 0 ? 16 : 33) : sw((fm - h) / 2));
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const cx<T> z = zf[c * LD], w = conj(self ? z : zq[c * LD]);
                    zf[c * LD] = scale(z + w, (T)0.5);
                    zq[c * LD] = scale(mul_mi(z - w), (T)0.5);
                }
            }
            __syncthreads();
#pragma unroll 1
            for (int it = tid; it < 2 * PH; it += NTHR) {
                const int k = it >> 1, f = 2 * k + h;
                if (f > HY) continue;
                const int fm = (PY - f) & (PY - 1);
                const bool self = fm == f, isq = it & 1;
                cx<T>* z = spec + (!isq ? sw(k) : (self ? (f == 0 ? 16 : 33) : sw((fm - h) / 2)));
                couple_inplace<T, L>(z, LD, Q, qs, isq ? (size_t)(nkq - 1) * KH + f : (size_t)f, false);
            }
            __syncthreads();
#pragma unroll 1
            for (int k = tid; k < PH; k += NTHR) {
                const int f = 2 * k + h;
                if (f > HY) continue;
                const int fm = (PY - f) & (PY - 1);
                const bool self = fm == f;
                cx<T>* zf = spec + sw(k);
                cx<T>* zq = spec + (self ? (f == 0 ? 16 : 33) : sw((fm - h) / 2));
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const cx<T> d = zf[c * LD], q = zq[c * LD];
                    zf[c * LD] = d + mul_i(q);
                    if (!self) zq[c * LD] = conj(d) + mul_i(conj(q));
                }
            }
        } else {
            // frequencies in the order [0, PH/4), [3PH/4, PH), [PH/4, 3PH/4): a frequency and its
            // mirror, which read the same quarter-table entries, fall in the same sweep
#pragma unroll 1
            for (int ki = tid; ki < PH; ki += NTHR) {
                const int k = ki < PH / 4 ? ki : (ki < PH / 2 ? ki + PH / 2 : ki - PH / 4);
                const int f = 2 * k + h;
                const bool flip = f > HY;
                couple_inplace<T, L>(spec + sw(k), LD, Q, qs, (size_t)kx * KH + (flip ? PY - f : f), flip);
            }
        }
        __syncthreads();
        block_fft_grouped<T, PH, C, G, LD, NTHR, true>(spec, tws, tid);
#pragma unroll 1
        for (int n = tid; n < ny; n += NTHR) {
            cx<T> w = mk((T)1, (T)0);
            if (h == 1) {
                double sn, cs;
                sincospi(2.0 * (double)n / (double)PY, &sn, &cs);
                w = mk((T)cs, (T)sn);
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const cx<T> v = spec[c * LD + sw(n)];
                if (h == 0) ebase[c * cstride + n] = v;
                else base[c * cstride + n] = ebase[c * cstride + n] + v * w;
            }
        }
        __syncthreads();   // the next half overwrites the spectra
    }
}

template <typename T, int PY, int L>
constexpr bool half_fits() {
    // LDS of k_pass_b_half: one half of the column's spectra and the half-length twiddles
    return PY >= 64 && ((long)(2 * L + 1) * padded(PY / 2) + PY / 2) * (long)sizeof(cx<T>) <= 160 * 1024;
}

constexpr int lds_budget() { return 160 * 1024; }

template <typename T, int PY, int L>
constexpr int ncol_for() {
    return (2 * L + 1) >= 4 ? 1 : ((2 * L + 1) == 3 ? 2 : 4);
}
template <typename T, int PY, int L>
constexpr bool fused_fits() {
    // LDS: column spectra, twiddle table, and the pair scratch; FP64 with L > 4 is left to the
    // split form (the fused FP64 coupling does not fit the register budget)
    return ((long)ncol_for<T, PY, L>() * (2 * L + 1) * padded(PY) + PY + 2 * (2 * L + 1)) * (long)sizeof(cx<T>) <=
               lds_budget() &&
           (sizeof(T) == 4 || L <= 4);
}
template <typename T, int NFPY>
constexpr int nthr_for() {
    // about 8 elements per thread, at most 512 threads: the mode coupling keeps 2(2L+1) complex
    // values per thread live, which does not fit the 128-VGPR budget of 1024-thread blocks
    return NFPY / 8 >= 512 ? 512 : (NFPY / 8 >= 256 ? 256 : (NFPY / 8 >= 128 ? 128 : 64));
}

// Fused-form variants: 0 = default threads and grouping; 1 = 1024 threads, groups of 4 transforms
// (FP32 only); 2 = 256 threads.  Variants 1 and 2 exist for PY >= 128 when they have enough work.
template <typename T, int PY, int L>
constexpr bool reg_variant() {   // the register-resident form as an FP32 variant: padded y >= 128, 5+ channels
    return sizeof(T) == 4 && PY >= 128 && L >= 2;
}

template <typename T, int PY, int L>
constexpr int fused_variants_base() {
    constexpr int C = 2 * L + 1;
    constexpr int NF = ncol_for<T, PY, L>() * C * PY;
    if (PY < 128) return 1;
    return reg_variant<T, PY, L>() ? 4 : ((sizeof(T) == 4 && NF / 8 >= 1024) ? 3 : 2);
}
// The radix-32 schedule (fft.h, schedule 1) as the next variant, for padded y >= 256.
template <typename T, int PY, int L>
constexpr bool sched_variant() { return PY >= 256; }
// All of a block's transforms in one group, as the last variant, where the default grouping
// splits them (FP32 at padded y = 1024 and L >= 6: 12 + 5 transforms at L = 8).
template <typename T, int PY, int L>
constexpr bool onegroup_variant() {
    constexpr int NF = ncol_for<T, PY, L>() * (2 * L + 1);
    return default_group<PY, NF, nthr_for<T, NF * PY>()>() < NF;
}
template <typename T, int PY, int L>
constexpr int fused_variants() {
    return fused_variants_base<T, PY, L>() + (sched_variant<T, PY, L>() ? 1 : 0) +
           (onegroup_variant<T, PY, L>() ? 1 : 0);
}

template <typename T, int PY, int L, int NCOL, int NT, int GV, int SCH = 0>
static void launch_fused(const Apply2DArgs<T>& a, int nbatch, int nkx, int nkq) {
    dim3 grid((nkx + NCOL - 1) / NCOL, nbatch);
    if constexpr (sizeof(T) == 4) {
        if (a.bcorr.y) {
            hipLaunchKernelGGL((k_pass_b_lds<T, PY, L, NCOL, NT, GV, SCH, true>), grid, dim3(NT), 0, a.stream, a.work,
                               a.Q, SCH == 1 ? a.twy1 : a.twy, a.ny, nkx, nkq, a.pack, 0, a.bcorr);
            return;
        }
    }
    hipLaunchKernelGGL((k_pass_b_lds<T, PY, L, NCOL, NT, GV, SCH>), grid, dim3(NT), 0, a.stream, a.work, a.Q,
                       SCH == 1 ? a.twy1 : a.twy, a.ny, nkx, nkq, a.pack, a.single_in, a.bcorr);
}

// Whether pass B of this (precision, PY, variant) adds the coarse correction (CorrB): the FP32
// fused forms in LDS.
template <typename T, int PY>
static bool corr_ok_py(int var) {
    constexpr int L = RTE_PASSB_L;
    if constexpr (sizeof(T) == 4 && fused_fits<T, PY, L>()) return !(reg_variant<T, PY, L>() && var == 3);
    else return false;
}

template <typename T, int PY>
static int launch_py(const Apply2DArgs<T>& a, int nbatch) {
    constexpr int L = RTE_PASSB_L;
    constexpr int C = 2 * L + 1;
    if (a.bcorr.y && (!corr_ok_py<T, PY>(a.var[1]) || a.single_in)) return -6;
    const int nkq = a.PX / 2 + 1;
    const int nkx = a.pack ? a.PX / 2 : nkq;
    if constexpr (fused_fits<T, PY, L>()) {
        constexpr int NCOL = ncol_for<T, PY, L>();
        constexpr int NT = nthr_for<T, NCOL * C * PY>();
        constexpr int NV = fused_variants_base<T, PY, L>();
        if constexpr (sched_variant<T, PY, L>()) {
            if (a.var[1] == NV) {
                if (!a.twy1) return -5;
                launch_fused<T, PY, L, NCOL, NT, 0, 1>(a, nbatch, nkx, nkq);
                return 0;
            }
        }
        if constexpr (reg_variant<T, PY, L>()) {
            if (a.var[1] == 3) {   // the work buffer is unpacked for this variant (apply2d_pack)
                if (a.pack) return -4;
                dim3 grid(nkx, nbatch);
                hipLaunchKernelGGL((k_pass_b_reg<T, PY, L, 4, 1, 4>), grid, dim3(PY), 0, a.stream, a.work, a.Q, a.twy,
                                   a.ny, nkx, nkq, a.single_in);
                return 0;
            }
        }
        if constexpr (NV >= 3) {
            if (a.var[1] == 1) { launch_fused<T, PY, L, NCOL, 1024, 4>(a, nbatch, nkx, nkq); return 0; }
        }
        if constexpr (NV >= 2) {
            if (a.var[1] == 2) { launch_fused<T, PY, L, NCOL, 256, 0>(a, nbatch, nkx, nkq); return 0; }
        }
        if constexpr (onegroup_variant<T, PY, L>()) {
            if (a.var[1] == NV + (sched_variant<T, PY, L>() ? 1 : 0)) {
                launch_fused<T, PY, L, NCOL, NT, NCOL * C>(a, nbatch, nkx, nkq);
                return 0;
            }
        }
        launch_fused<T, PY, L, NCOL, NT, 0>(a, nbatch, nkx, nkq);
        return 0;
    } else {
        if (!a.work2) return -2;
        if (a.single_in && nbatch != 1) return -3;
        if constexpr (half_fits<T, PY, L>()) {
            if (a.var[1] == 1) {   // split in halves
                if (!a.twyh) return -5;
                dim3 grid(nkx, nbatch);
                hipLaunchKernelGGL((k_pass_b_half<T, PY, L, 256>), grid, dim3(256), 0, a.stream, a.work, a.work2, a.Q,
                                   a.twyh, a.ny, nkx, nkq, a.pack, a.single_in);
                return 0;
            }
        }
        const size_t nseq = (size_t)nbatch * C * nkx;
        split_fft<T, PY, false>(a.work, a.work2, a.twy, a.ny, a.single_in ? (size_t)nkx : nseq, a.stream);  // single_in: channel 0 only
        if constexpr (L >= 1) {
            // the coupling fused with the inverse: the tuned choice, and always for a single input
            // channel (the right-hand side K~ f), where it reads one channel of the full-length
            // buffer instead of writing and reading all of them
            if (a.var[1] == (half_fits<T, PY, L>() ? 2 : 1) || a.single_in) {
                constexpr int NG = couple_groups<L>();
                dim3 g3((unsigned)(((nkx + 7) / 8) * 8 * NG), nbatch);
                hipLaunchKernelGGL((k_pass_b_couple_inv<T, PY, L, 256>), g3, dim3(256), 0, a.stream, a.work,
                                   a.work2, a.Q, a.twy, a.ny, nkx, nkq, a.pack, a.single_in);
                return 0;
            }
        }
        dim3 g2((unsigned)(((size_t)nkx * PY + 255) / 256), nbatch);
        hipLaunchKernelGGL((k_pass_b_couple<T, PY, L>), g2, dim3(256), 0, a.stream, a.work2, a.Q, nkx, nkq,
                           a.pack, a.single_in);
        split_fft<T, PY, true>(a.work, a.work2, a.twy, a.ny, nseq, a.stream);
        return 0;
    }
}

template <typename T, int PY>
static int variants_py() {
    if constexpr (fused_fits<T, PY, RTE_PASSB_L>()) return fused_variants<T, PY, RTE_PASSB_L>();
    // split form; split in halves; the coupling fused with the inverse y-FFTs
    return (half_fits<T, PY, RTE_PASSB_L>() ? 2 : 1) + (RTE_PASSB_L >= 1 ? 1 : 0);
}

template <typename T>
static int launch_pass_b_impl(const Apply2DArgs<T>& a, int nbatch) {
    switch (a.PY) {
        case 16: return launch_py<T, 16>(a, nbatch);
        case 32: return launch_py<T, 32>(a, nbatch);
        case 64: return launch_py<T, 64>(a, nbatch);
        case 128: return launch_py<T, 128>(a, nbatch);
        case 256: return launch_py<T, 256>(a, nbatch);
        case 512: return launch_py<T, 512>(a, nbatch);
        case 1024: return launch_py<T, 1024>(a, nbatch);
    }
    return -1;
}

#define RTE_CAT2(a, b) a##b
#define RTE_CAT(a, b) RTE_CAT2(a, b)
#if RTE_PASSB_L == 0
// Batched pass-B variants (padded y >= 128): 0 = the fused form's columns per block and threads;
// 1 = the same columns with half the threads; 2 = twice the columns; 3 = half the columns.
template <typename T, int PY, int NCOL>
constexpr bool batch_b_fits() {
    return ((long)NCOL * padded(PY) + PY + 2) * (long)sizeof(cx<T>) <= lds_budget();
}
template <typename T, int PY>
constexpr int batch_b_variants() {
    return PY < 128 ? 1 : (batch_b_fits<T, PY, 2 * ncol_for<T, PY, 0>()>() ? 4 : 2);
}
template <typename T, int PY, int NCOL, int NT>
static void launch_b_batch_nc(const BatchProb<T>* probs, const int2* items, int nitems, const int* act,
                              hipStream_t st) {
    static_assert(batch_b_fits<T, PY, NCOL>(), "batched pass-B columns exceed the LDS budget");
    hipLaunchKernelGGL((k_pass_b_batch<T, PY, NCOL, NT>), dim3(nitems), dim3(NT), 0, st, probs, items, act);
}
template <typename T, int PY>
static void launch_b_batch(const BatchProb<T>* probs, const int2* items, int nitems, const int* act, int var,
                           hipStream_t st) {
    static_assert(fused_fits<T, PY, 0>(), "isotropic pass B is always fused");
    constexpr int NCOL = ncol_for<T, PY, 0>();
    constexpr int NT = nthr_for<T, NCOL * PY>();
    if constexpr (batch_b_variants<T, PY>() >= 2) {
        if (var == 1) return launch_b_batch_nc<T, PY, NCOL, (NT / 2 > 64 ? NT / 2 : 64)>(probs, items, nitems, act, st);
    }
    if constexpr (batch_b_variants<T, PY>() >= 4) {
        if (var == 2) return launch_b_batch_nc<T, PY, 2 * NCOL, nthr_for<T, 2 * NCOL * PY>()>(probs, items, nitems,
                                                                                            act, st);
        if (var == 3) return launch_b_batch_nc<T, PY, NCOL / 2, nthr_for<T, NCOL / 2 * PY>()>(probs, items, nitems,
                                                                                            act, st);
    }
    launch_b_batch_nc<T, PY, NCOL, NT>(probs, items, nitems, act, st);
}
template <typename T>
int apply2d_batch_col_variants(int PY) {
    switch (PY) {
        case 128: return batch_b_variants<T, 128>();
        case 256: return batch_b_variants<T, 256>();
        case 512: return batch_b_variants<T, 512>();
        case 1024: return batch_b_variants<T, 1024>();
        default: return 1;
    }
}
template <typename T>
int apply2d_batch_cols(int PY, int var) {
    constexpr int NCOL = ncol_for<T, 1024, 0>();   // the same for every PY when C = 1
    if (var < 0 || var >= apply2d_batch_col_variants<T>(PY)) return 0;
    return var == 2 ? 2 * NCOL : var == 3 ? NCOL / 2 : NCOL;
}
template <typename T>
int apply2d_batch_pass_b(int PY, const BatchProb<T>* probs, const int2* items, int nitems, const int* act, int var,
                         hipStream_t st) {
    if (nitems <= 0) return 0;
    if (var < 0 || var >= apply2d_batch_col_variants<T>(PY)) return -1;
    switch (PY) {
        case 16: launch_b_batch<T, 16>(probs, items, nitems, act, var, st); break;
        case 32: launch_b_batch<T, 32>(probs, items, nitems, act, var, st); break;
        case 64: launch_b_batch<T, 64>(probs, items, nitems, act, var, st); break;
        case 128: launch_b_batch<T, 128>(probs, items, nitems, act, var, st); break;
        case 256: launch_b_batch<T, 256>(probs, items, nitems, act, var, st); break;
        case 512: launch_b_batch<T, 512>(probs, items, nitems, act, var, st); break;
        case 1024: launch_b_batch<T, 1024>(probs, items, nitems, act, var, st); break;
        default: return -1;
    }
    return 0;
}
template int apply2d_batch_col_variants<float>(int);
template int apply2d_batch_col_variants<double>(int);
template int apply2d_batch_cols<float>(int, int);
template int apply2d_batch_cols<double>(int, int);
template int apply2d_batch_pass_b<float>(int, const BatchProb<float>*, const int2*, int, const int*, int,
                                         hipStream_t);
template int apply2d_batch_pass_b<double>(int, const BatchProb<double>*, const int2*, int, const int*, int,
                                          hipStream_t);
#endif

// Whether pass B takes the work buffer unpacked (x-frequencies 0 and PX/2 in columns of their own)
// for this (precision, PY, pass-B variant): the register-resident forms.
template <typename T, int PY>
static bool unpacked_py(int var) {
    constexpr int L = RTE_PASSB_L;
    if constexpr (fused_fits<T, PY, L>()) return reg_variant<T, PY, L>() && var == 3;
    else return false;
}
template <typename T>
bool RTE_CAT(pass_b_unpacked_L, RTE_PASSB_L)(int PY, int var) {
    switch (PY) {
        case 16: return unpacked_py<T, 16>(var);
        case 32: return unpacked_py<T, 32>(var);
        case 64: return unpacked_py<T, 64>(var);
        case 128: return unpacked_py<T, 128>(var);
        case 256: return unpacked_py<T, 256>(var);
        case 512: return unpacked_py<T, 512>(var);
        case 1024: return unpacked_py<T, 1024>(var);
    }
    return false;
}
template bool RTE_CAT(pass_b_unpacked_L, RTE_PASSB_L)<float>(int, int);
template bool RTE_CAT(pass_b_unpacked_L, RTE_PASSB_L)<double>(int, int);

template <typename T>
bool RTE_CAT(pass_b_corr_ok_L, RTE_PASSB_L)(int PY, int var) {
    switch (PY) {
        case 16: return corr_ok_py<T, 16>(var);
        case 32: return corr_ok_py<T, 32>(var);
        case 64: return corr_ok_py<T, 64>(var);
        case 128: return corr_ok_py<T, 128>(var);
        case 256: return corr_ok_py<T, 256>(var);
        case 512: return corr_ok_py<T, 512>(var);
        case 1024: return corr_ok_py<T, 1024>(var);
    }
    return false;
}
template bool RTE_CAT(pass_b_corr_ok_L, RTE_PASSB_L)<float>(int, int);
template bool RTE_CAT(pass_b_corr_ok_L, RTE_PASSB_L)<double>(int, int);

#define RTE_PASSB_FN RTE_CAT(pass_b_L, RTE_PASSB_L)
#define RTE_PASSB_VARIANTS RTE_CAT(pass_b_variants_L, RTE_PASSB_L)
template <typename T>
int RTE_PASSB_VARIANTS(int PY) {
    switch (PY) {
        case 16: return variants_py<T, 16>();
        case 32: return variants_py<T, 32>();
        case 64: return variants_py<T, 64>();
        case 128: return variants_py<T, 128>();
        case 256: return variants_py<T, 256>();
        case 512: return variants_py<T, 512>();
        case 1024: return variants_py<T, 1024>();
    }
    return 0;
}
template int RTE_PASSB_VARIANTS<float>(int);
template int RTE_PASSB_VARIANTS<double>(int);

template <>
int RTE_PASSB_FN<float>(const Apply2DArgs<float>& a, int nbatch) { return launch_pass_b_impl<float>(a, nbatch); }
template <>
int RTE_PASSB_FN<double>(const Apply2DArgs<double>& a, int nbatch) { return launch_pass_b_impl<double>(a, nbatch); }

// Whether the split (3-kernel) form is used for this (precision, PY): the caller then provides
// work2 of nbatch * C * (PX/2+1) * PY elements.
template <>
bool RTE_CAT(pass_b_split_L, RTE_PASSB_L)<float>(int PY) {
    switch (PY) {
        case 16: return !fused_fits<float, 16, RTE_PASSB_L>();
        case 32: return !fused_fits<float, 32, RTE_PASSB_L>();
        case 64: return !fused_fits<float, 64, RTE_PASSB_L>();
        case 128: return !fused_fits<float, 128, RTE_PASSB_L>();
        case 256: return !fused_fits<float, 256, RTE_PASSB_L>();
        case 512: return !fused_fits<float, 512, RTE_PASSB_L>();
        default: return !fused_fits<float, 1024, RTE_PASSB_L>();
    }
}
template <>
bool RTE_CAT(pass_b_split_L, RTE_PASSB_L)<double>(int PY) {
    switch (PY) {
        case 16: return !fused_fits<double, 16, RTE_PASSB_L>();
        case 32: return !fused_fits<double, 32, RTE_PASSB_L>();
        case 64: return !fused_fits<double, 64, RTE_PASSB_L>();
        case 128: return !fused_fits<double, 128, RTE_PASSB_L>();
        case 256: return !fused_fits<double, 256, RTE_PASSB_L>();
        case 512: return !fused_fits<double, 512, RTE_PASSB_L>();
        default: return !fused_fits<double, 1024, RTE_PASSB_L>();
    }
}

}  // namespace rte
