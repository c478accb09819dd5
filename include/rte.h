/*
 * rte.h -- C ABI of the MI355X (gfx950) solver for the steady-state radiative transfer equation
 * in a homogeneous medium, in the angularly reduced Fredholm form of Fan, An and Ying,
 * "Fast algorithms for integral formulations of steady-state radiative transfer equation".
 *
 * The discrete problem (Sec. 3.3, eq. ani_discretization and eq. ani_AU; the isotropic u-form
 * of eq. iso_Fredholm discretised per Sec. 2.3) is
 *
 *     A u = (I - K~ D) u = K~ g,      g_{j,k} = f(x_j) delta_{k0},   D = diag_k(mu_s sigma_hat_k)
 *
 * on the cell centres x_j of a uniform grid of square (cubic) cells of side h.  K~ couples output
 * mode k at x_i to input mode k' at x_j by h^d kappa(|x_i-x_j|) exp(i (k'-k) theta_ij), with
 * kappa(r) = exp(-mu_t r)/(2 pi r) in 2D and exp(-mu_t r)/(4 pi r^2) in 3D and theta_ij the polar
 * angle of x_i - x_j (eq. ani_2d_operator); the diagonal entry is the exact cell integral of the
 * singular kernel over the cell (Sec. 2.3, eq. iso_discretization).  The operator is applied by
 * zero-padded FFT convolution (Sec. 2.3.1 and 3.3.1) and the system is solved by GMRES.
 *
 * 3D anisotropic scattering (Sec. 3.1.2, eq. ani_3d_Fredholm, re-derived in real spherical
 * harmonics): mode a = l^2 + l + m (l = 0..L, m = -l..l, M = (L+1)^2) is the coefficient of the
 * real harmonic Y_a normalised to unit mean square over the sphere (Y_00 = 1,
 * (Y_{1,-1}, Y_{1,0}, Y_{1,1}) = sqrt(3) (y, z, x); for m > 0, Y_{l,+-m} is
 * sqrt(2 (2l+1) (l-m)!/(l+m)!) times the associated Legendre function without the Condon-Shortley
 * phase times cos(m phi) / sin(m phi); Y_{l,0} = sqrt(2l+1) P_l(cos theta)), u_a = mean over
 * directions of Phi Y_a.  K~ couples output mode a at x_i to input mode b at x_j by
 * h^3 kappa(|x_i - x_j|) Y_a(w) Y_b(w), w = (x_i - x_j)/|x_i - x_j|, and
 * D = diag_a(mu_s sigma_hat_l(a)) with sigma_hat_l = (1/2) int_{-1}^{1} sigma(t) P_l(t) dt the
 * Legendre coefficients of the phase function normalised to unit mean (Henyey-Greenstein: g^l).
 *
 * Conventions shared by every entry point
 *   - All arrays are device pointers (hipMalloc'd or torch CUDA tensors) owned by the caller and
 *     borrowed for the duration of the call; all work is enqueued on the context's stream.
 *   - Grids: 2D arrays are [ny][nx] (x fastest), 3D arrays [nz][ny][nx].
 *   - RTE_LAYOUT_MODES: complex128 (interleaved re,im doubles) [M][ny][nx], mode k = -L..L at
 *     index k+L (M = 2L+1).  Any complex vector is accepted.  3D: M = (L+1)^2,
 *     [M][nz][ny][nx], mode a = l^2 + l + m (the solution's modes are real; imaginary parts are
 *     carried through the real operator).
 *   - RTE_LAYOUT_CHANNELS: real float64 [C][ny][nx], C = 2L+1, the image of a real angular flux
 *     (u_{-k} = conj u_k): channel 0 = Re u_0, channel 2k-1 = sqrt(2) Re u_k,
 *     channel 2k = sqrt(2) Im u_k (k = 1..L).  With the sqrt(2) the Euclidean norm of the channel
 *     vector equals the norm of the full mode vector.  3D: C = (L+1)^2, [C][nz][ny][nx], channel
 *     a = Re u_a.
 *   - Status: every int-returning function returns RTE_OK (0) on success, a positive value for a
 *     completed call with a caveat, a negative value on error; it never throws or aborts.
 *     rte_last_error() gives a thread-local message for the last non-OK status.
 */
#ifndef RTE_H
#define RTE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rte_ctx rte_ctx;

typedef struct {
    int dim;        /* 2 or 3 */
    int n[3];       /* cells along x, y, z (n[2] ignored in 2D); each >= 2 */
    double h;       /* cell side > 0; the domain is [0, n_x h] x [0, n_y h] (x [0, n_z h]) */
} rte_grid;

enum {
    RTE_OK = 0,
    RTE_NOT_CONVERGED = 1,   /* solve stopped at max_iter / max_cycles; output holds best iterate */
    RTE_EINVAL = -1,         /* bad argument; nothing was enqueued */
    RTE_ENOMEM = -2,         /* device allocation failed */
    RTE_EDEVICE = -3,        /* HIP runtime error */
    RTE_ENUMERIC = -4,       /* NaN or Inf in the residual */
    RTE_EUNSUPPORTED = -5    /* valid request outside what this build implements */
};

enum { RTE_PREC_FP32 = 0,    /* FFT apply in FP32/complex64 (FP32 accumulation); Krylov in FP64 */
       RTE_PREC_FP64 = 1 };  /* everything in FP64 */

enum { RTE_OP_A = 0,         /* y = x - K~ D x        (eq. ani_AU) */
       RTE_OP_KT = 1 };      /* y = K~ x              (step T.1 when x = g) */

enum { RTE_LAYOUT_MODES = 0, RTE_LAYOUT_CHANNELS = 1 };

typedef struct {
    int iterations;      /* inner (F)GMRES iterations, all cycles */
    int applies;         /* operator applies, all precisions */
    int cycles;          /* refinement cycles (true-residual checks) */
    int pc_used;         /* 1 if the attached preconditioner was used */
    int pc_fallback;     /* 1 if the solve fell back to plain GMRES */
    double relres_est;   /* last Arnoldi estimate of the relative residual */
    double relres_true;  /* ||b - A x|| / ||b|| with the FP64 apply, at exit */
    double t_setup_ms;   /* time of rte_setup for this context */
    double t_solve_ms;   /* wall time of this solve (batched: of the whole batch) */
    int status;          /* this problem's outcome: RTE_OK, RTE_NOT_CONVERGED or RTE_ENUMERIC */
} rte_solve_info;

typedef struct {
    int restart;         /* Krylov dimension per cycle, 1..RTE_MAX_RESTART (default 64) */
    int max_cycles;      /* refinement cycles (default 8) */
    double inner_tol;    /* per-cycle relative reduction for the FP32 inner solve (default 3e-4:
                            both refinement cycles stay short, and a step's Gram-Schmidt cost
                            grows with its position in the cycle; rte_solve_batched takes at most
                            3e-5, since its problems advance in lockstep and a third cycle for a
                            few of them costs the whole batch; ignored for RTE_PREC_FP64, whose
                            cycles run to the requested tol) */
    int reorth;          /* classical Gram-Schmidt passes: 0 = one pass (default; each restart
                            cycle ends with an FP64 true-residual check), 1 = a second pass when
                            the norm drops below 1/sqrt(2) of its value, 2 = always two passes.
                            With one pass the update also normalises the new basis vector, by
                            1/sqrt(|w|^2 - |h|^2), and it is rescaled in a second pass only when its
                            measured norm is off 1 by more than 1e-8 (FP32 apply) or 1e-10 (FP64) */
    int use_pc;          /* 1: flexible GMRES with the attached preconditioner (default 1 if one
                            is attached) */
    int basis_fp32;      /* RTE_PREC_FP32 only: 1 stores the inner solve's Krylov basis (and the
                            apply's output) in FP32, halving the Gram-Schmidt traffic; dot
                            products, the update arithmetic, the Hessenberg matrix, the rotations,
                            the solution and the true residual stay FP64.  The basis then stays
                            orthogonal to FP32 rounding only, below the per-cycle reduction
                            inner_tol, and the FP64 true residual still decides convergence.
                            0 (default): FP64 basis.  Ignored for RTE_PREC_FP64. */
} rte_solve_opts;

/* Largest 2D mode count L (M = 2L+1 = 65 modes).  Up to L = 8 pass B couples the modes in
 * registers per y-frequency; above, the coupling runs as a convolution along the mode axis by
 * FFTs of length 64, 128 or 256 (the kernel depends on k' - k only, Sec. 3.3.1), or as the direct
 * Toeplitz sum, whichever the autotuner times faster.  The learned preconditioner takes L <= 8. */
#define RTE_MAX_L 32
#define RTE_MAX_L3 3      /* largest spherical-harmonic degree of a 3D context (M = 16 modes) */
#define RTE_MAX_RESTART 128

/* Create a context: validates the problem, allocates the device state and precomputes the
 * kernel spectra in FP64 on the device (the T_pre step of Sec. 2.4).
 *   g          grid (2D: any n_x, n_y in [2, 512]; 3D: n in [2, 256] for L = 0, [2, 128] for
 *              L = 1..RTE_MAX_L3)
 *   mu_a, mu_s absorption and scattering coefficients, >= 0, mu_a + mu_s > 0 (assumption C2)
 *   sigma_hat  host array of L+1 real Fourier coefficients of the phase function (Sec. 3.1.1,
 *              eq. ani_Fouriermode; sigma_hat_{-k} = sigma_hat_k), sigma_hat[0] == 1 (C3) and
 *              |sigma_hat[k]| <= 1; may be NULL when L == 0.  3D: its Legendre coefficients
 *              sigma_hat_l, l = 0..L, with the same conditions
 *   L          2D: number of retained modes on each side, 0..RTE_MAX_L (M = 2L+1, up to 65); 3D: largest
 *              spherical-harmonic degree, 0..RTE_MAX_L3 (M = (L+1)^2)
 *   prec       RTE_PREC_FP32 or RTE_PREC_FP64
 *   hip_stream hipStream_t to enqueue on (NULL = default stream)
 * Errors: RTE_EINVAL (before any device work), RTE_EUNSUPPORTED (3D with L > RTE_MAX_L3, oversize grid),
 * RTE_ENOMEM, RTE_EDEVICE.  On error *out is NULL. */
int rte_setup(rte_ctx** out, const rte_grid* g, double mu_a, double mu_s,
              const double* sigma_hat, int L, int prec, void* hip_stream);

/* y = op(x) in the given layout.  prec selects the apply precision: RTE_PREC_FP64 is always
 * available; RTE_PREC_FP32 needs a context created with RTE_PREC_FP32.  x and y are FP64
 * (complex128 or float64 per layout) and may not alias.  Asynchronous on the context stream. */
int rte_apply(rte_ctx* ctx, int op, int layout, int prec, const void* x_dev, void* y_dev);

/* b = K~ g for g = f delta_{k0} (step T.1).  f_dev: float64 [ny][nx] ([nz][ny][nx]);
 * b_dev: FP64 in the given layout.  Uses the FP64 apply.  Asynchronous. */
int rte_rhs(rte_ctx* ctx, const double* f_dev, int layout, void* b_dev);

/* The scattering term of the solved flux at ntheta equispaced angles theta_q = 2 pi q / ntheta
 * (Sec. 3.1, eq. ani_2d_scattering, times mu_s):
 *     S[q][y][x] = Re( mu_s sum_{k=-L..L} sigma_hat_|k| u_k(x) e^{i k theta_q} )
 * the right-hand side that, with f, gives the angular flux by one transport sweep (Sec. 1).
 *   layout   RTE_LAYOUT_MODES (u complex128 [M][ny][nx], any complex vector; the real part of
 *            the sum is written) or RTE_LAYOUT_CHANNELS (u float64 [C][ny][nx])
 *   ntheta   1 .. 2^24
 *   S_dev    float64 [ntheta][ny][nx], caller-owned; may not overlap u
 * 2D contexts only (3D: RTE_EUNSUPPORTED).  Asynchronous on the context stream. */
int rte_scattering_term(rte_ctx* ctx, int layout, const void* u_dev, int ntheta, double* S_dev);

/* Replace the solver options (NULL restores the defaults). */
int rte_set_solve_opts(rte_ctx* ctx, const rte_solve_opts* opts);

/* Solve A u = K~ g to ||b - A u||_2 / ||b||_2 <= tol (true residual, FP64 apply) with
 * GMRES from u = 0, FP32 or FP64 inner applies per the context precision and FP64
 * iterative refinement.  f_dev: float64 source at the cell centres; u_dev: complex128 modes
 * (RTE_LAYOUT_MODES).  max_iter bounds the total inner iterations.  Synchronises the stream.
 * Returns RTE_OK, RTE_NOT_CONVERGED (u holds the best iterate), RTE_ENUMERIC or an error.
 * f = 0 gives u = 0 and RTE_OK.  info may be NULL.  u is written during the solve (after each
 * true residual); after an error its content is unspecified. */
int rte_solve(rte_ctx* ctx, const double* f_dev, double tol, int max_iter, void* u_dev,
              rte_solve_info* info);

/* An anisotropic source f(x, v) given by its angular modes g (Sec. 4: the right-hand side becomes
 * F T^{-1} f, which for a source with the retained modes only is K~ g with g in every mode, the
 * same K~ as the solve's): b = K~ g with the FP64 apply.  layout RTE_LAYOUT_MODES: g and b complex128
 * [M][..] (2D: the modes of a real source, g_{-k} = conj g_k; only k >= 0 are read);
 * RTE_LAYOUT_CHANNELS: float64 [C][..].  g and b may not alias.  Asynchronous. */
int rte_rhs_source(rte_ctx* ctx, const void* g_dev, int layout, void* b_dev);

/* Solve A u = K~ g for the anisotropic source g of rte_rhs_source, as rte_solve does for an
 * isotropic one: u in the same layout as g (modes: complex128 [M][..]; channels: float64 [C][..]),
 * written after every true residual.  Synchronises the stream; returns as rte_solve. */
int rte_solve_source(rte_ctx* ctx, const void* g_dev, int layout, double tol, int max_iter, void* u_dev,
                     rte_solve_info* info);

/* Several sources sharing one medium (the case the paper names for reusing one operator,
 * Sec. 2.3.2): solve A u_s = K~ g(f_s) for s < nrhs with this context's operator, as one GMRES on
 * the stacked block-diagonal system with every right-hand side scaled to unit norm (global GMRES):
 * each iteration applies A to all nrhs vectors in one batched launch per pass and runs one
 * Gram-Schmidt step on the stacked vector.  Stopping at a stacked relative residual of
 * tol / sqrt(number of non-zero sources) bounds every source's relative residual by tol; each
 * source's FP64 true residual is computed at the end and reported in infos[s].relres_true (its
 * status is RTE_NOT_CONVERGED if it exceeds tol).  f[s]: float64 sources at the cell centres;
 * u[s]: complex128 modes (RTE_LAYOUT_MODES); nrhs in 1..RTE_MAX_RHS.  Work buffers grow to nrhs
 * right-hand sides on first use.  The learned preconditioner is not used.  infos may be NULL.
 * Synchronises the stream.  Returns RTE_OK if every source converged, RTE_NOT_CONVERGED,
 * RTE_ENUMERIC or an error. */
#define RTE_MAX_RHS 64
int rte_solve_multi(rte_ctx* ctx, int nrhs, const double* const* f_dev, double tol, int max_iter,
                    void* const* u_dev, rte_solve_info* infos);

/* Solve A x = b for a right-hand side b given in RTE_LAYOUT_CHANNELS (float64), x in the same
 * layout.  If x_iterates is not NULL, the first inner cycle's iterates are recorded there
 * (x_iterates[j] = the iterate after j+1 inner iterations, up to max_record vectors of the
 * channel size) for generating preconditioner training pairs; *n_recorded gets their count.
 * x, b and the max_record vectors at x_iterates must not overlap (x is cleared before b is
 * read): overlapping storage is RTE_EINVAL. */
int rte_solve_rhs(rte_ctx* ctx, const double* b_dev, double tol, int max_iter, double* x_dev,
                  rte_solve_info* info, double* x_iterates, int max_record, int* n_recorded);

/* Solve `count` independent problems (contexts may differ in grid and coefficients; all must be
 * 2D isotropic (L = 0) contexts created on the same device and stream).  All problems advance
 * together: every pass is one launch over the tiles of all unconverged problems, and one inner
 * iteration is captured once into a HIP graph and replayed.  f_dev[i], u_dev[i] as in rte_solve;
 * tol[i] per problem; infos may be NULL.  Returns RTE_OK if all converged, RTE_NOT_CONVERGED if
 * some did not, or an error. */
int rte_solve_batched(int count, rte_ctx* const* ctxs, const double* const* f_dev,
                      const double* tol, int max_iter, void* const* u_dev, rte_solve_info* infos);

/* Attach a learned right preconditioner for flexible GMRES: the coarse-grid correction
 * z = v + s P N(R v / s) of rte_nn.h (R: factor x factor block average, P: bilinear interpolation from
 * the coarse cell centres, s: RMS of v, N: `layers` 3x3 convolutions C -> hidden -> ... -> C with ReLU
 * between, C = 2L+1).  weights_dev: packed float32 parameters (layout in rte_nn.h); the context
 * keeps a BF16 copy.  factor must divide n_x and n_y.  NULL detaches.  2D contexts with L <= 8
 * only (3D, or L > 8: RTE_EUNSUPPORTED).  A preconditioned cycle that does not end the solve and
 * fails to cut the true residual 10x (or to reach twice its own target, when that asks for less),
 * or that produces a non-finite value, is followed by plain GMRES (info.pc_fallback = 1).  With
 * the FP32 apply (padded x 128..1024) each Arnoldi step runs the next apply's x-transforms beside
 * the network and adds the correction's x-spectrum in the y-pass instead (the same z up to FP32
 * rounding); environment RTE_PC_EARLY_A=0 keeps the correction in the x-pass.  Environment
 * RTE_RENORM_TOL overrides the tolerance on |v_{j+1}|^2 - 1 beyond which a solve rescales the new
 * Krylov vector (default 1e-8 with the FP32 apply, 1e-10 with FP64; negative: every step). */
int rte_pc_attach(rte_ctx* ctx, const float* weights_dev, int hidden, int layers, int factor);

/* Time `reps` back-to-back applies (op, RTE_LAYOUT_CHANNELS, prec) on the context stream with
 * HIP events.  ms_total: whole apply; ms_pass[0..4]: per kernel of the apply (2D: passes A, B, C;
 * 3D: five passes; unused entries 0).  Input/output are internal buffers. */
int rte_time_apply(rte_ctx* ctx, int op, int prec, int reps, double* ms_total, double* ms_pass);

/* As rte_time_apply for the batched apply of nrhs stacked channel vectors that rte_solve_multi runs
 * every iteration (each pass one launch over all nrhs right-hand sides; nrhs in 1..RTE_MAX_RHS).
 * Grows the work buffers to nrhs right-hand sides as rte_solve_multi does.  Synchronises. */
int rte_time_apply_multi(rte_ctx* ctx, int nrhs, int op, int prec, int reps, double* ms_total, double* ms_pass);

/* Time the batched apply of one inner iteration of rte_solve_batched over the same contexts (in
 * the same order; a batch plan must exist, i.e. rte_solve_batched ran on them): every problem
 * active, one launch per pass (A, B, C) and padded grid size, `reps` times, each launch bracketed
 * by HIP events on the batch stream.  Outputs: *ms_total the average time of the whole batched
 * apply; for launch i < min(*n_launch, max_launch): ms_launch[i] its average time, launch_pass[i]
 * (0 = A, 1 = B, 2 = C), launch_px[i], launch_py[i] the padded grid of the problems it covers and
 * launch_var[i] the kernel variant it runs (rte_set_batched_variant); any output array may be
 * NULL.  Launches are ordered pass A over the size classes, then B, then C; size classes in the
 * order their first problem appears.  Overwrites the first two basis columns of each problem.
 * RTE_EINVAL without a plan for these contexts.  Synchronises the batch stream. */
int rte_time_batched_apply(int count, rte_ctx* const* ctxs, int reps, double* ms_total, int max_launch,
                           int* n_launch, double* ms_launch, int* launch_pass, int* launch_px, int* launch_py,
                           int* launch_var);

/* Kernel variants of the batched apply, per padded grid size of a batch (same arithmetic, equal
 * results up to rounding).  pass 0: the row tile of passes A and C (4 variants for a padded x >= 128,
 * as the single-problem row tiles); pass 1: the columns per block of pass B (the default columns and
 * threads, half the threads, twice or half the columns; padded y >= 128).  When rte_solve_batched
 * builds the plan of a new list of contexts it times the variants of every size class on all of
 * its problems and keeps the fastest (environment RTE_AUTOTUNE=0: variant 0).  This call forces
 * `variant` (0..3; a size class with fewer variants takes variant 0) or restores tuning (-1) for
 * plans built afterwards, and drops the cached plans.  The setting is process-wide.  RTE_EINVAL if
 * pass or variant is out of range. */
int rte_set_batched_variant(int pass, int variant);

/* Kernel variants of the apply (prec = RTE_PREC_FP32 or RTE_PREC_FP64 apply).  2D: pass 0 = A,
 * 1 = B, 2 = C; 3D: pass 0 = A (x-FFT), 1 = B (y-FFT), 2 = C (z-FFT with the spectrum or the mode
 * coupling), 3 = D (inverse y-FFT), 4 = E (inverse x-FFT).  Variants differ only in tiling (row
 * tiles, z-rows or columns per block, thread counts, FFT grouping, radix schedule, how the FP64
 * pass B with many modes stages its full-length spectra, the coupling method for many modes): the
 * same arithmetic, equal results up to rounding.  rte_setup of a 2D
 * context with n_x or n_y >= 128, or of a 3D context with a side >= 64, picks the fastest variant of
 * every pass by timing them on the context's buffers, once per (precision, L, grid) per process
 * (environment RTE_AUTOTUNE=0: keep variant 0).  rte_autotune re-times them (`reps` launches each;
 * synchronises the stream); rte_set_variant forces one (RTE_EINVAL if the pass or variant is out of
 * range); rte_get_variant reports the current one and how many exist. */
int rte_autotune(rte_ctx* ctx, int reps);
int rte_set_variant(rte_ctx* ctx, int prec, int pass, int variant);
int rte_get_variant(const rte_ctx* ctx, int prec, int pass, int* variant, int* count);

/* Sizes: *channels = *modes = 2L+1 (2D) or (L+1)^2 (3D), *cells = n_x n_y (n_z). */
int rte_query(const rte_ctx* ctx, int* channels, int* modes, long long* cells);

/* Pack complex modes (must be conjugate-symmetric) into channels, and back. FP64, asynchronous. */
int rte_modes_to_channels(rte_ctx* ctx, const void* modes_dev, double* channels_dev);
int rte_channels_to_modes(rte_ctx* ctx, const double* channels_dev, void* modes_dev);

void rte_destroy(rte_ctx* ctx);
const char* rte_last_error(void);
const char* rte_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RTE_H */
