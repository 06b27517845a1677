/*
 * recon.h - C ABI of the MI355X (gfx950) regularised spiral-MRI reconstruction.
 *
 * Method (Boubertakh, Giovannelli, De Cesare, Herment, "Regularized
 * reconstruction of MR images from spiral acquisitions"):
 *
 *   minimise J(x) = ||y - A x||^2 + lambda * sum phi(|D x|)
 *
 *   A   exact non-uniform DFT of Section 2, Eq. ModDirect:
 *         (A x)_l = (1/N) sum_{n,m} x[n][m] exp(+i 2 pi (kx_l m + ky_l n))
 *   D   first-order pixel differences in both directions (Section 3.3,
 *       Omega_1), non-periodic
 *   phi hyperbolic sqrt(delta^2 + t^2) (edge preserving, convex), or the
 *       paper's Huber function, or Hunt's quadratic
 *
 * The data term is evaluated in the image domain (Section 3.4, Eq. NewCritLS):
 * b = A^H y (the paper's D, Eq. AnnMatGD) and the trajectory-only Gram kernel
 * (the paper's G, Eq. DG) are computed once by exact sums; every iteration
 * applies Q = A^H A as a zero-padded L x L FFT, a pointwise product with the
 * real spectrum of the circulant-embedded kernel, an inverse FFT and a crop
 * (the gradient 2 f*G - 2D of Appendix B).  The minimiser is the paper's
 * pseudo-conjugate gradient with a Polak-Ribiere correction (Section 3.3),
 * with a half-quadratic majorant step length.
 *
 * Conventions
 *   - complex data are interleaved float pairs (re, im) ("complex64");
 *   - an image is row-major [N][N]: row n pairs with k_y, column m with k_x;
 *   - a batch of B frames is [B][N][N] (images) or [B][M] (samples);
 *   - a trajectory is host float64 [M][2] = (k_x, k_y) in cycles/pixel with
 *     |k_x|, |k_y| <= 0.5 (Section 2: F = [1, 1], k normalised to
 *     [-0.5, 0.5]).
 *
 * Memory ownership
 *   The library never allocates or frees device memory.  The caller provides
 *   the plan memory (recon_plan_bytes), the solver workspace
 *   (recon_workspace_bytes) and every input/output buffer; all device pointers
 *   must be 256-byte aligned device allocations on the current device.
 *   A plan handle is a small host object (recon_plan_destroy frees it, not
 *   the caller's plan memory).
 *
 * Streams and errors
 *   Every call enqueues work on `stream` (a hipStream_t, NULL = default
 *   stream) and returns without synchronising.  Arguments are validated
 *   before any launch; on error nothing is enqueued and a status != RECON_OK
 *   is returned, with a detail string from recon_last_error() (per thread).
 *   A plan is read-only after recon_gram_kernel and may be shared by several
 *   streams; a workspace may only be used by one call at a time.
 */
#ifndef RECON_H
#define RECON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct recon_plan_s* recon_plan_t;

typedef enum {
  RECON_OK = 0,
  RECON_E_ARG = 1,        /* null pointer, bad enum, negative count */
  RECON_E_RANGE = 2,      /* N, L, M, k or a size outside the supported range */
  RECON_E_NOMEM = 3,      /* caller buffer smaller than the *_bytes query */
  RECON_E_HIP = 4,        /* HIP runtime error (detail in recon_last_error) */
  RECON_E_STATE = 5,      /* call order violated (e.g. solve before gram) */
  RECON_E_NONFINITE = 6   /* per-frame status: a NaN/Inf appeared */
} recon_status_t;

/* Operand precision of the NUDFT contractions (adjoint / forward). */
typedef enum {
  RECON_FP32 = 0,         /* FP32 operands, FP32 MFMA, FP32 accumulation */
  RECON_BF16X3 = 1,       /* split bf16 hi+lo operands, 3 products, FP32 acc. */
  RECON_FP16X3 = 2,       /* split fp16 hi+lo operands, 3 products, FP32 acc. */
  RECON_FP64 = 3,         /* adjoint with FP64 phasors, products and MFMA
                             accumulation, rounded to FP32 once (accurate
                             form); the forward model stays FP32 */
  /* Flag OR'ed into RECON_FP64: run the iteration of recon_solve and of the
   * slot pools in FP64 (b, x, r, d, the row-transform intermediate, the
   * FFTs, the penalty stencil and the Gram spectrum; b is not rounded to
   * FP32).  The iterate after a fixed budget of iterations can amplify
   * per-step rounding by orders of magnitude when the minimisation is far
   * from converged; this form keeps it at FP64 level.  Inputs and outputs
   * (y, x0, x, exported fields) stay complex64.  Requires L <= 1024; the
   * workspace (recon_workspace_bytes with the same prec) is about twice as
   * large.  recon_gram_apply, recon_adjoint and recon_forward are unchanged. */
  RECON_ITER_FP64 = 16
} recon_prec_t;

/* Penalty phi(s), s = |difference| (Section 3.3). */
typedef enum {
  RECON_PHI_HYPERBOLIC = 0,  /* sqrt(delta^2 + s^2) */
  RECON_PHI_HUBER = 1,       /* s^2 if s <= delta else 2 delta s - delta^2 */
  RECON_PHI_QUADRATIC = 2    /* s^2 (delta unused) */
} recon_phi_t;

/* Per-frame result of recon_solve, written to device memory. */
typedef struct {
  double J;            /* criterion at the returned x */
  double grad_ratio;   /* ||grad J(x)|| / ||grad J(x0)|| */
  double gnorm0;       /* ||grad J(x0)|| */
  int32_t iters_done;  /* iterations run */
  int32_t status;      /* RECON_OK or RECON_E_NONFINITE */
} recon_stats_t;

/* Supported ranges: 2 <= N <= 1024, L a power of two with 2N-1 <= L <= 2048
 * (L <= 1024 with RECON_ITER_FP64), 64 <= L, 1 <= M <= 2^31-1, 1 <= B. */

/* ---- sizes (host only, no device work) ---------------------------------- */

/* Bytes of device memory a plan needs (trajectory, phasor tables for the
 * NUDFT contractions, FFT twiddles, Gram spectrum).  0 on invalid sizes. */
size_t recon_plan_bytes(int64_t M, int32_t N, int32_t L, int32_t prec);

/* Bytes of scratch device memory recon_gram_kernel needs (split-K partial
 * sums of the Gram kernel and the L x L embedding). */
size_t recon_gram_workspace_bytes(int64_t M, int32_t N, int32_t L);

/* Bytes of device workspace for recon_solve / recon_gram_apply /
 * recon_adjoint / recon_forward on B frames of plan geometry (N, L, M) and
 * precision prec (the plan's, including RECON_ITER_FP64).  0 on invalid
 * sizes or precision. */
size_t recon_workspace_bytes(int64_t M, int32_t N, int32_t L, int32_t B, int32_t prec);

/* ---- plan --------------------------------------------------------------- */

/* Section 2: validates the trajectory (finite, |k| <= 0.5), copies it to the
 * device and builds the FP32 (and, for split precisions, hi/lo) phasor
 * tables exp(i 2 pi k j) of the separable NUDFT.  traj: host float64
 * [M][2] (kx, ky).  L = 0 selects the smallest power of two >= 2N-1 (and
 * >= 64).  plan_mem: device, >= recon_plan_bytes(M, N, L, prec); owned by
 * the caller, must outlive the plan.  The tables are built asynchronously
 * on `stream`; *out is valid on return. */
recon_status_t recon_plan(const double* traj, int64_t M, int32_t N, int32_t L,
                          int32_t prec, void* plan_mem, size_t plan_mem_bytes,
                          void* stream, recon_plan_t* out);

/* Geometry of a plan (any out pointer may be NULL). */
recon_status_t recon_plan_info(recon_plan_t plan, int64_t* M, int32_t* N,
                               int32_t* L, int32_t* prec);

void recon_plan_destroy(recon_plan_t plan);

/* Section 3.4 Eq. DG and Appendix A.1 Eq. AnnMatG: the trajectory-only
 * kernel.  Computes the lag kernel h[a][b] = (1/N^2) sum_l
 * exp(-i 2 pi (ky_l a + kx_l b)), a, b in [-(N-1), N-1] (h[a][b] is the
 * paper's G[-b][-a]) with FP64 MFMA accumulation over all samples, embeds it
 * circularly in L x L, takes its 2D FFT in FP64 and keeps the real spectrum
 * (rounded once to FP32) inside the plan.  Must be called once before recon_solve /
 * recon_gram_apply.  ws: device scratch >= recon_gram_workspace_bytes.
 * Optional outputs (NULL to skip): khat_out device float32 [L][L] (p, q),
 * the unscaled real spectrum; lag_out device complex128 [2N-1][2N-1]
 * indexed [a + N-1][b + N-1]. */
recon_status_t recon_gram_kernel(recon_plan_t plan, void* ws, size_t ws_bytes,
                                 float* khat_out, double* lag_out,
                                 void* stream);

/* ---- operators ---------------------------------------------------------- */

/* Batch limit: with a plan whose adjoint precision is RECON_FP32,
 * RECON_BF16X3 or RECON_FP16X3, recon_adjoint, recon_forward, recon_solve
 * and recon_solve_begin accept at most 64 frames per call (RECON_E_ARG
 * above, before anything is launched); split larger batches into calls of
 * <= 64 frames.  Plans with the FP64 adjoint have no such limit. */

/* Appendix A.2, Eq. AnnMatGD: b[f] = A^H y[f], the paper's D
 * ("DFT of the data"), as an MFMA contraction over the M samples.
 * y: device complex64 [B][M]; b: device complex64 [B][N][N];
 * yy_out: optional device float64 [B] receiving ||y[f]||^2.
 * ws: device workspace >= recon_workspace_bytes(M, N, L, B). */
recon_status_t recon_adjoint(recon_plan_t plan, const float* y, int32_t B,
                             float* b, double* yy_out, void* ws,
                             size_t ws_bytes, void* stream);

/* Section 2, Eq. ModDirect (noise-free): y[f] = A x[f] as an MFMA
 * contraction.  x: device complex64 [B][N][N]; y: device complex64 [B][M]. */
recon_status_t recon_forward(recon_plan_t plan, const float* x, int32_t B,
                             float* y, void* ws, size_t ws_bytes,
                             void* stream);

/* Section 3.4 / Appendix B: Qv[f] = A^H A v[f] by the zero-padded L x L FFT
 * with the plan's Gram spectrum.  v, Qv: device complex64 [B][N][N]
 * (may not alias).  Requires recon_gram_kernel. */
recon_status_t recon_gram_apply(recon_plan_t plan, const float* v, int32_t B,
                                float* Qv, void* ws, size_t ws_bytes,
                                void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * Gram apply as recon_gram_apply, with its row-transform intermediate in a
 * fixed 64 MiB device array inside the library instead of a caller
 * workspace.  Nothing is allocated by the call: each GPU the library runs on
 * holds its own copy of the array until the process ends (its address is
 * looked up on the first call on a device).  B * N * L * 8 bytes must not
 * exceed recon_gram_apply_noalloc_max_bytes() (64 MiB; RECON_E_RANGE
 * otherwise, before anything is launched).  The caller still provides v and
 * Qv.  All calls on one GPU share the array, so calls that overlap on one
 * GPU (different streams, or threads without ordering) race; calls on one
 * stream are ordered and safe. */
size_t recon_gram_apply_noalloc_max_bytes(void);
recon_status_t recon_gram_apply_noalloc(recon_plan_t plan, const float* v, int32_t B, float* Qv,
                                        void* stream);

/* ---- solver ------------------------------------------------------------- */

/* Section 3.3: minimise ||y - A x||^2 + lambda sum phi(|D x|) for B frames
 * sharing the plan's trajectory, with `iters` iterations of the
 * pseudo-conjugate gradient (Polak-Ribiere, PR+ with restart) and the
 * half-quadratic majorant step, starting from x0 = 0 (x_in_is_x0 = 0) or from
 * the contents of x (x_in_is_x0 = 1).  Computes b = A^H y itself.
 * y: device complex64 [B][M]; x: device complex64 [B][N][N] (in/out);
 * stats: optional device recon_stats_t [B].  Requires recon_gram_kernel.
 * lambda >= 0, delta > 0 (ignored for the quadratic penalty), iters >= 0. */
recon_status_t recon_solve(recon_plan_t plan, const float* y, int32_t B,
                           double lambda, double delta, int32_t iters,
                           int32_t phi, float* x, int32_t x_in_is_x0,
                           void* ws, size_t ws_bytes, recon_stats_t* stats,
                           void* stream);

/* Resumable form of recon_solve for the same workspace (used to inspect the
 * iteration state between iterations), with the full criterion of Section
 * 3.3: J(x) = ||y - A x||^2 + lambda sum phi(|D x|) + lambda0 sum
 * phi_alpha0(|x|), the second sum being the background penalty Omega_0 with
 * the Huber function of threshold alpha0 (lambda0 = 0 turns it off, as in
 * recon_solve; lambda0 >= 0, and alpha0 > 0 when lambda0 > 0).
 *   recon_solve_begin: b = A^H y (or b given: y == NULL and b_in != NULL),
 *                      initial state from x0 (x0 == NULL means zeros);
 *   recon_solve_iterate: run `iters` more iterations;
 *   recon_solve_end:   objective and stats, copy x to x_out.
 * recon_solve_export copies one state field of the current iterate to `out`
 * (device complex64 [B][N][N]): 0 = x, 1 = r (= Q x - b), 2 = g (gradient),
 * 3 = d (search direction for the next iteration), 4 = b. */
recon_status_t recon_solve_begin(recon_plan_t plan, const float* y,
                                 const float* b_in, int32_t B, double lambda,
                                 double delta, double lambda0, double alpha0,
                                 int32_t phi, const float* x0, void* ws,
                                 size_t ws_bytes, void* stream);
/* recon_solve_begin with b given in FP64: b device complex128 [B][N][N],
 * for plans with RECON_ITER_FP64 (other plans: RECON_E_ARG).  The FP64
 * iteration amplifies perturbations of b (Section 3.4's D) by up to ~4e5 on
 * the 256^2 workload, so a b computed in FP64 elsewhere (the NUFFT form of
 * D, recon_grid_adjoint64) is handed over without rounding it to complex64.
 * b is read before the call's work completes on `stream` (stream-ordered);
 * the objective's constant ||y||^2 is taken as 0, as with b_in above. */
recon_status_t recon_solve_begin_b64(recon_plan_t plan, const double* b, int32_t B,
                                     double lambda, double delta, double lambda0,
                                     double alpha0, int32_t phi, const float* x0, void* ws,
                                     size_t ws_bytes, void* stream);
recon_status_t recon_solve_iterate(recon_plan_t plan, int32_t iters, void* ws,
                                   size_t ws_bytes, void* stream);
recon_status_t recon_solve_end(recon_plan_t plan, float* x_out,
                               recon_stats_t* stats, void* ws, size_t ws_bytes,
                               void* stream);
recon_status_t recon_solve_export(recon_plan_t plan, int32_t field, float* out,
                                  void* ws, size_t ws_bytes, void* stream);

/* ---- half-quadratic solver (Section 5's alternative to the pseudo-CG) --- */

/* The paper's conclusion (Section 5) names a dual / half-quadratic
 * optimisation [Idier01b] as a way to reduce the cost of the
 * conjugate-gradient minimisation.  This is its multiplicative
 * (Geman-Reynolds) form on the same criterion, operators and workspace:
 * `outer` times, the penalty weights w = phi'(s)/s of the differences
 * s = |D xbar| (and of the background term) are frozen at the current image
 * xbar, and `inner` steps of linear conjugate gradients (exact steps,
 * Polak-Ribiere coefficient with the descent safeguard, first direction -g)
 * decrease the quadratic surrogate
 *   ||y - A x||^2 + lam sum (w/2)|D x|^2 [+ lam0 sum (w0/2)|x|^2] + const,
 * which lies above J and touches it at xbar, so J decreases at every outer
 * iteration.  Each inner step applies Q once.
 *   recon_hq_workspace_bytes: workspace of the half-quadratic solver (the
 *                      recon_workspace_bytes layout plus one image); 0 on
 *                      invalid sizes or precision.
 *   recon_solve_hq:    as recon_solve (x0 = 0 or the contents of x), with
 *                      outer x inner steps; stats.grad_ratio is the true
 *                      gradient's norm ratio at the result.
 *   recon_solve_hq_iterate: outer x inner more steps after recon_solve_begin
 *                      (background term, b given, x0) on a workspace of
 *                      recon_hq_workspace_bytes; recon_solve_end and
 *                      recon_solve_export then apply as after
 *                      recon_solve_iterate.  Slot pools are rejected. */
size_t recon_hq_workspace_bytes(int64_t M, int32_t N, int32_t L, int32_t B, int32_t prec);
recon_status_t recon_solve_hq(recon_plan_t plan, const float* y, int32_t B, double lambda,
                              double delta, int32_t outer, int32_t inner, int32_t phi, float* x,
                              int32_t x_in_is_x0, void* ws, size_t ws_bytes,
                              recon_stats_t* stats, void* stream);
recon_status_t recon_solve_hq_iterate(recon_plan_t plan, int32_t outer, int32_t inner, void* ws,
                                      size_t ws_bytes, void* stream);

/* ---- convolution gridding and non-uniform FFT -------------------------- */

/* Section 1 describes the gridding reconstruction the method is compared
 * with: weighting of the samples for their non-uniform density, resampling
 * onto a Cartesian grid with a convolution kernel, an FFT, and correction of
 * the kernel's apodization; Section 4.1 uses a 7 x 7 Kaiser-Bessel kernel.
 * Section 5 proposes the same non-uniform FFT machinery to speed up the
 * precomputation of D = A^H y and of the Gram kernel.  All of it runs in
 * FP64 on the device:
 *   type-1 sum  out[n][m] = sum_l c_l exp(-i 2 pi (ky_l (n - h) + kx_l (m - h)))
 *   c spread onto a G x G grid with phi(g1 - G ky) phi(g2 - G kx), the
 *   Kaiser-Bessel kernel phi(t) = I0(beta sqrt(1 - (2t/W)^2)), |t| <= W/2;
 *   forward 2D FFT; outputs divided by the kernel's Fourier transform.
 * With grid oversampling G/N >= 2 and the default beta
 * (pi sqrt(W^2 / s^2 (s - 1/2)^2 - 0.8), s = G/N) the relative error of the
 * sums is bounded by about 4 / I0(beta): 4e-4 (W = 5), 3.5e-6 (W = 7),
 * 3.4e-8 (W = 9), 3.3e-10 (W = 11), 3.1e-12 (W = 13), 3.0e-14 (W = 15),
 * from the kernel's jump at the edge of its support.
 *
 * A grid plan holds, in caller memory (recon_grid_bytes), the trajectory,
 * the per-sample kernel weights and footprints, per-tile sample lists (built
 * on the host: the plan call synchronises `stream`), the apodization
 * correction and the FFT twiddles.  traj: host float64 [M][2] (kx, ky) as
 * for recon_plan; N: output size (N x N), 2 N <= G; G: power of two in
 * [64, 2048] (0: the smallest >= 2N); W: kernel width in [2, 16]; beta: the
 * kernel's shape (0: the default above).  M <= 2^29 - 1.
 *   recon_grid_adjoint: out[f] = (1/N) sum_l w_l y[f]_l exp(-i 2 pi (kx_l m + ky_l n)),
 *       n, m < N (Eq. AnnMatGD with weights; w == NULL means 1): with
 *       density weights it is the gridding reconstruction, without them the
 *       NUFFT form of D.  y: device complex64 [B][M]; w: device float64 [M];
 *       out: device complex64 [B][N][N]; ws >= recon_grid_workspace_bytes(B).
 *   recon_grid_adjoint64: the same sums with out device complex128
 *       [B][N][N] (no final rounding; for recon_solve_begin_b64).
 *   recon_grid_density: density-compensation weights by the fixed-point
 *       iteration of Pipe and Menon (the paper's [Pipe99]): from w = 1,
 *       `iters` times w <- w / (I S w) with S the spreading of real weights
 *       and I its adjoint (interpolation); finally scaled by
 *       phi_hat(0)^4 / (G/N)^2 so that a uniform Cartesian grid of spacing
 *       1/N gets weights ~1.  w: device float64 [M] (output).
 *   recon_gram_kernel_nufft: the plan's Gram kernel (as recon_gram_kernel)
 *       with the lag kernel h[a][b] = (1/N^2) sum_l exp(-i 2 pi (ky a + kx b))
 *       computed by a type-1 sum on 2N outputs (grid of 4N rounded up to a
 *       power of two, N <= 512) instead of the exact sums; within the bound
 *       above for width W.  ws >= recon_gram_nufft_workspace_bytes (which
 *       also holds that sum's own grid plan; the call synchronises `stream`). */
typedef struct recon_grid_s* recon_grid_t;
size_t recon_grid_bytes(int64_t M, int32_t N, int32_t G, int32_t W);
recon_status_t recon_grid_plan(const double* traj, int64_t M, int32_t N, int32_t G, int32_t W,
                               double beta, void* mem, size_t mem_bytes, void* stream,
                               recon_grid_t* out);
recon_status_t recon_grid_info(recon_grid_t grid, int32_t* G, int32_t* W, double* beta);
void recon_grid_destroy(recon_grid_t grid);
size_t recon_grid_workspace_bytes(recon_grid_t grid, int32_t B);
recon_status_t recon_grid_adjoint(recon_grid_t grid, const float* y, const double* w, int32_t B,
                                  float* out, void* ws, size_t ws_bytes, void* stream);
recon_status_t recon_grid_adjoint64(recon_grid_t grid, const float* y, const double* w, int32_t B,
                                    double* out, void* ws, size_t ws_bytes, void* stream);
recon_status_t recon_grid_density(recon_grid_t grid, int32_t iters, double* w, void* ws,
                                  size_t ws_bytes, void* stream);
size_t recon_gram_nufft_workspace_bytes(int64_t M, int32_t N, int32_t L, int32_t W);
recon_status_t recon_gram_kernel_nufft(recon_plan_t plan, int32_t W, void* ws, size_t ws_bytes,
                                       float* khat_out, double* lag_out, void* stream);

/* ---- slot pools: continuous batching of independent frames ------------- */

/* A slot pool is a workspace sized for B frames (recon_workspace_bytes(B))
 * whose frames ("slots") start and finish at different times.  All slots
 * share one plan (trajectory, N, L) and one penalty kind; lambda, delta and
 * the iteration budget are per slot.  Every iteration kernel runs on all B
 * slots of the pool and skips, as a whole block, the slots that are idle or
 * already done, so a frame that joins the pool at any iteration follows
 * exactly the sequence of operations of recon_solve with B = 1 and x0 = 0
 * (Section 3.3 of the paper): its result is bitwise equal to that solve.
 *
 *   recon_pool_reset:  bind the workspace to a pool of B idle slots.
 *   recon_pool_admit:  start a frame in an idle (or retired) slot: ||y||^2,
 *                      b = A^H y and the initial state, with a budget of
 *                      `iters` iterations from the pool's current iteration
 *                      counter, and its own lambda, delta, lambda0, alpha0
 *                      (as recon_solve_begin).  y: device complex64 [M] (the
 *                      plan's sample order).  RECON_E_STATE if the slot is
 *                      still running.
 *   recon_pool_step:   run `iters` iterations of the pool (all running slots
 *                      advance; slots whose budget is used up stay frozen).
 *   recon_pool_retire: objective/stats of a finished slot (stats: device
 *                      recon_stats_t, may be NULL) and a copy of its image
 *                      to x_out (device complex64 [N][N], may be NULL).
 *                      RECON_E_STATE while the slot still has iterations
 *                      left.  The slot is idle afterwards.
 *   recon_pool_iteration: the pool's iteration counter (iterations run by
 *                      recon_pool_step since the reset), -1 on error.
 * All calls are stream-ordered on `stream`; calls on one pool must not
 * overlap (host-side state is updated at call time).  recon_solve_iterate,
 * recon_solve_end and recon_solve_export reject a pool workspace. */
recon_status_t recon_pool_reset(recon_plan_t plan, int32_t B, int32_t phi,
                                void* ws, size_t ws_bytes, void* stream);
recon_status_t recon_pool_admit(recon_plan_t plan, int32_t slot, const float* y,
                                double lambda, double delta, double lambda0,
                                double alpha0, int32_t iters, void* ws,
                                size_t ws_bytes, void* stream);
recon_status_t recon_pool_step(recon_plan_t plan, int32_t iters, void* ws,
                               size_t ws_bytes, void* stream);
recon_status_t recon_pool_retire(recon_plan_t plan, int32_t slot, float* x_out,
                                 recon_stats_t* stats, void* ws,
                                 size_t ws_bytes, void* stream);
int64_t recon_pool_iteration(recon_plan_t plan, void* ws);

/* ---- diagnostics -------------------------------------------------------- */

/* Kernel timing trace (HIP events around every launch of one kernel kind on
 * the launching stream).  kernel: -1 = off, 0 = direction + row FFT,
 * 1 = column pass, 2 = inverse row FFT of recon_gram_apply, 3 = CG update
 * (inverse row FFT + update), 4 = adjoint contraction (all launches of one
 * recon_adjoint or solve), 5 = Gram contraction, 6 = forward contraction.  capacity
 * bounds the number of recorded launches (later ones are not recorded).
 * Creating the events allocates no device buffers.  recon_trace_read waits
 * for the recorded events and writes up to n durations (ms) to ms_out; it
 * returns the number written, or -1 on error.  Tracing is process-wide and
 * not thread-safe against concurrent solves. */
recon_status_t recon_trace_enable(int32_t kernel, int32_t capacity);
int32_t recon_trace_read(float* ms_out, int32_t n);
/* Several kinds at once: bit k of `mask` enables kind k (as numbered above),
 * each with its own `capacity` records; mask 0 turns tracing off.
 * recon_trace_read_kind reads the durations of one enabled kind (0 if the
 * kind is not enabled, -1 on error); recon_trace_read reads the lowest
 * enabled kind. */
recon_status_t recon_trace_enable_set(uint32_t mask, int32_t capacity);
int32_t recon_trace_read_kind(int32_t kernel, float* ms_out, int32_t n);

const char* recon_status_string(recon_status_t s);
/* Detail of the last error on the calling thread ("" if none). */
const char* recon_last_error(void);
/* Library version string. */
const char* recon_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RECON_H */
