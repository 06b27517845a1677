// Host-side launchers of the HIP kernels (defined in the .hip files).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace recon {

// Operand precisions of the split NUDFT contractions (values of recon_prec_t).
constexpr int RECON_PREC_BF16X3 = 1;
constexpr int RECON_PREC_FP16X3 = 2;

// Per-frame parameters (device array, one entry per frame).  A frame takes
// part in iteration k of its workspace only while k < stop_at (slot pools of
// the serving path; plain solves use INT32_MAX).
struct FrameParam {
  double lam;     // weight of the difference penalty Omega_1
  double delta;   // its threshold
  double lam0;    // weight of the background penalty Omega_0 (0: off)
  double alpha0;  // its Huber threshold
  int32_t stop_at;
  int32_t pad;
};

// Rows handled by one 256-thread block of the row-FFT kernels: one team of
// L/V threads per row (V = 16 values per thread at L = 1024, 8 otherwise).
inline int fft_rows_per_block(int L) { return (L == 1024 ? 4096 : 2048) / L; }
// Columns handled by one block of the column kernel (f64: the FP64 form).
int fft_cols_per_block(int L, bool f64);

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// Every kernel of the Gram apply and of the iteration exists for float2 (the
// FP32 iteration) and, for L <= 1024, double2 (the FP64 iteration: state,
// transforms and spectrum in FP64); the double2 overloads take the plan's
// FP64 twiddles and spectrum.

// ---- Gram apply (Section 3.4) ------------------------------------------------
// Row pass: T[f][n][:] = FFT_L(zero-padded v[f][n][:]) for n < N.
hipError_t launch_rowfft_plain(int L, int N, int B, const float2* v, float2* T,
                               const float2* tw, hipStream_t s);
hipError_t launch_rowfft_plain(int L, int N, int B, const double2* v, double2* T,
                               const double2* tw, hipStream_t s);
// Column pass (in place): column q of T[f] -> IFFT_L(khat_s[q][:] * FFT_L(col)),
// rows n < N kept.  khat_s is the transposed spectrum scaled by 1/L^2.
// p3 (optional, [B][L / cols_per_block]) receives per-block partials of
// sum khat_s |FFT_L(col)|^2 = Re<v, Q v> (Parseval).
hipError_t launch_colpass(int L, int N, int B, float2* T, const float* khat_s, double* p3,
                          const float2* tw, const FrameParam* fp, int k, hipStream_t s);
hipError_t launch_colpass(int L, int N, int B, double2* T, const double* khat_s, double* p3,
                          const double2* tw, const FrameParam* fp, int k, hipStream_t s);
// Row inverse pass: out[f][n][m] = IFFT_L(T[f][n][:])[m] for m < N.
hipError_t launch_rowifft(int L, int N, int B, const float2* T, float2* out,
                          const float2* tw, const FrameParam* fp, int k, hipStream_t s);
hipError_t launch_rowifft(int L, int N, int B, const double2* T, double2* out,
                          const double2* tw, const FrameParam* fp, int k, hipStream_t s);


// ---- CG kernels (Section 3.3) -------------------------------------------------
// Rows per block of the iteration kernels (one FFT team of L/8 threads per row).
// The step-length partials p1 and the update partials p4 have cdiv(N, rows)
// entries per frame.
// Direction: g = 2 r + grad R(x) (recomputed), d_new = -g + beta d_old (beta
// from the update partials, PR+ with restart), partials Re<g, d_new> and
// sum w(x)|D d_new|^2, and the row pass of the Gram apply on d_new.
// xb non-null: the inner step of the half-quadratic minimiser, every penalty
// weight (edges and background) frozen at the image xb.
hipError_t launch_dir_rowfft(int L, int phi, int N, int B, const float2* r,
                             const float2* d_old, float2* d_new, const float2* x, float2* T,
                             const double* p4, int nb4, double* p1, const FrameParam* fp,
                             const float2* tw, int k, bool bg, hipStream_t s,
                             const float2* xb = nullptr);
hipError_t launch_dir_rowfft(int L, int phi, int N, int B, const double2* r,
                             const double2* d_old, double2* d_new, const double2* x, double2* T,
                             const double* p4, int nb4, double* p1, const FrameParam* fp,
                             const double2* tw, int k, bool bg, hipStream_t s,
                             const double2* xb = nullptr);
// Row inverse pass of the Gram apply fused with the update: Qd = rows of
// IFFT(T) cropped; alpha from the partials; x_new = x + alpha d,
// r += alpha Qd; partials for beta from g_old (recomputed from r, x) and
// g_new = 2 r + grad R(x_new).  bg: some frame of the launch has the
// background penalty on (lam0 > 0); without it the term is compiled out.
// xb non-null: the half-quadratic inner step (weights frozen at xb).
hipError_t launch_update(int L, int phi, int N, int B, const float2* T, const float2* x_old,
                         float2* x_new, const float2* d, float2* r, const double* p1, int nb1,
                         const double* p3, int nb3, double* p4, const FrameParam* fp,
                         const float2* tw, int k, bool bg, hipStream_t s,
                         const float2* xb = nullptr);
hipError_t launch_update(int L, int phi, int N, int B, const double2* T, const double2* x_old,
                         double2* x_new, const double2* d, double2* r, const double* p1, int nb1,
                         const double* p3, int nb3, double* p4, const FrameParam* fp,
                         const double2* tw, int k, bool bg, hipStream_t s,
                         const double2* xb = nullptr);
// Initial state: x = x0 (or 0), r = Qx0 - b (Qx0 NULL: -b), d = 0; partials
// such that the first direction is -g, g = 2r + grad R(x0).  R rows per block.
hipError_t launch_init(int phi, int N, int R, int B, const float2* b,
                       const float2* x0, const float2* qx0, float2* x,
                       float2* r, float2* d, double* p4,
                       double* pg0, const FrameParam* fp, hipStream_t s);
hipError_t launch_init(int phi, int N, int R, int B, const double2* b,
                       const double2* x0, const double2* qx0, double2* x,
                       double2* r, double2* d, double* p4,
                       double* pg0, const FrameParam* fp, hipStream_t s);
hipError_t launch_zero_f64(size_t n, double* p, hipStream_t s);
hipError_t launch_set_params(int B, double lam, double delta, double lam0, double alpha0,
                             int stop_at, FrameParam* fp, hipStream_t s);
// n complex values widened to FP64 / rounded to FP32.
hipError_t launch_widen(size_t n, const float2* in, double2* out, hipStream_t s);
hipError_t launch_narrow(size_t n, const double2* in, float2* out, hipStream_t s);
// Objective partials and final statistics.
hipError_t launch_objective(int phi, int N, int R, int B, const float2* x,
                            const float2* b, const float2* r, double* pobj,
                            const FrameParam* fp, hipStream_t s);
hipError_t launch_objective(int phi, int N, int R, int B, const double2* x,
                            const double2* b, const double2* r, double* pobj,
                            const FrameParam* fp, hipStream_t s);
hipError_t launch_stats(int B, const double* pobj, int nbo, const double* p4,
                        int nb4, const double* pg0, int nbg, const double* yy,
                        int iters, const FrameParam* fp, void* stats,
                        hipStream_t s);
// The gradient (dir = 0) or the pending direction -g + beta d_old (dir = 1,
// as the next direction kernel would form it) of the current iterate.
hipError_t launch_export(int phi, int N, int R, int B, const float2* x, const float2* r,
                         const float2* d_old, const double* p4, int nb4, const FrameParam* fp,
                         float2* out, int dir, hipStream_t s);
hipError_t launch_export(int phi, int N, int R, int B, const double2* x, const double2* r,
                         const double2* d_old, const double* p4, int nb4, const FrameParam* fp,
                         float2* out, int dir, hipStream_t s);

// ---- half-quadratic minimisation (Section 5's dual alternative) -------------
// xb = x (weights frozen at the current image) and zeroed update partials.
hipError_t launch_hq_freeze(int N, int B, int nb4, const float2* x, float2* xb, double* p4,
                            hipStream_t s);
hipError_t launch_hq_freeze(int N, int B, int nb4, const double2* x, double2* xb, double* p4,
                            hipStream_t s);
// The inner steps run launch_dir_rowfft, launch_colpass and launch_update
// with xb given.
// p4 = [|grad J(x)|^2, 0, 0, 0] per block (the true gradient, weights from x).
hipError_t launch_hq_gnorm(int phi, int N, int R, int B, const float2* x, const float2* r,
                           double* p4, const FrameParam* fp, bool bg, hipStream_t s);
hipError_t launch_hq_gnorm(int phi, int N, int R, int B, const double2* x, const double2* r,
                           double* p4, const FrameParam* fp, bool bg, hipStream_t s);

// ---- NUDFT (Section 2, Appendix A.2) -------------------------------------------
// Phasor tables E[l][j] = exp(i 2 pi k_l j), j < N, FP32 complex, for both
// axes: ex from k_x, ey from k_y.  k: device float64 [M][2].
hipError_t launch_tables_f32(int64_t M, int N, const double* k, float2* ex,
                             float2* ey, hipStream_t s);
// Adjoint: b[f][n][m] = (1/N) sum_l conj(ey[l][n]) y[f][l] conj(ex[l][m]).
// Split-K over `splits` sample ranges into part[s][f][n][m] when splits > 1.
int adjoint_splits(int64_t M, int N);
int adjoint_group(int64_t M, int N);
// split-K count and frames per launch of the FP64 adjoint (its own shape)
int adjoint64_splits(int64_t M, int N);
int adjoint64_group(int64_t M, int N);
hipError_t launch_adjoint_f32(int64_t M, int N, int B, const float2* ex,
                              const float2* ey, const float2* y, float2* b,
                              float2* part, hipStream_t s);
hipError_t launch_forward_f32(int64_t M, int N, int B, const float2* ex,
                              const float2* ey, const float2* x, float2* y,
                              hipStream_t s);
// ||y_f||^2 per frame (FP64, fixed order); part: scratch of
// sumsq_parts() doubles per frame.
int sumsq_parts();
hipError_t launch_sumsq(int64_t M, int B, const float2* y, double* part, double* yy,
                        hipStream_t s);

// ---- split-precision NUDFT (BF16 x3 / FP16 x3) ------------------------------
// Padded table geometry (multiples of the 32-wide MFMA k-step).
int64_t split_pad_M(int64_t M);
int split_pad_N(int N);
// at: [4][N][Mp] 16-bit (hi/lo of Re Ey, hi/lo of -Im Ey, l contiguous);
// xs: [4][M][Np] 16-bit (hi/lo of Re Ex, hi/lo of Im Ex, m contiguous).
hipError_t launch_tables_split(int prec, int64_t M, int N, const double* k, void* at, void* xs,
                               hipStream_t s);
// sc: per-frame scale scratch [B]; part: split-K partials [splits][group][N][N].
hipError_t launch_adjoint_split(int prec, int64_t M, int N, int B, const void* at,
                                const float2* ex, const float2* y, float* sc, float2* b,
                                float2* part, hipStream_t s);
hipError_t launch_forward_split(int prec, int64_t M, int N, int B, const void* xs,
                                const float2* ey, const float2* x, float* sc, float2* y,
                                hipStream_t s);

// ---- Gram kernel (Eq. DG, FP64) ----------------------------------------------
int gram_splits(int64_t M, int N);
// Four real products over the samples of split s:
// part[s][0..3][a][b] = sum_l (Yr Xr, Yi Xi, Yr Xi, Yi Xr) with
// Y = exp(-i 2 pi ky a), X = exp(-i 2 pi kx b), a, b < N.
hipError_t launch_gram_f64(int64_t M, int N, const double* k, double* part,
                           int splits, hipStream_t s);
// Reduce the split partials, scale by 1/N^2, assemble h over the full lag
// range (conjugate symmetry), optionally export it (lag_out complex128
// [2N-1][2N-1]) and embed it circularly into emb [L][L] (FP64 complex).
hipError_t launch_gram_assemble(int N, int L, const double* part, int splits,
                                double* lag_out, double2* emb, hipStream_t s);
// FP64 2D FFT of the embedding (emb is overwritten, tmp is scratch of the
// same size), then khat_s[q][p] = Re K[p][q] / L^2 (FP32, transposed),
// optionally khat_out[p][q] = Re K[p][q] and khat64_s (khat_s in FP64).
hipError_t launch_spectrum_f64(int L, double2* emb, double2* tmp, float* khat_s,
                               float* khat_out, double* khat64_s, hipStream_t s);
// Adjoint accumulated in FP64 (phasors generated in FP64 from k); b FP32.
// part: split-K partials, FP64 complex [splits][group][N][N].
// FP64 phase tables of the accurate adjoint: phase_record(N) double2 per
// sample and axis (unit step, in-tile offsets, tile bases), ph[2][M][R].
int phase_record(int N);
hipError_t launch_phase_tables_f64(int64_t M, int N, const double* k, double2* ph, hipStream_t s);
hipError_t launch_adjoint_f64(int64_t M, int N, int B, const double2* ph, const float2* y,
                              float2* b, double2* part, hipStream_t s);
hipError_t launch_adjoint_f64(int64_t M, int N, int B, const double2* ph, const float2* y,
                              double2* b, double2* part, hipStream_t s);

// ---- convolution gridding / non-uniform FFT (Sections 1, 4.1, 5) -----------
// Per-sample Kaiser-Bessel weights wy, wx [M][W], footprint origins base
// [M] (mod G) and sample phases pf [M] (exp(-i 2 pi (kx + ky) h) or 1).
hipError_t launch_grid_weights(int64_t M, int G, int W, double beta, int h, int phase,
                               const double* k, int2* base, double* wy, double* wx, double2* pf,
                               hipStream_t s);
// grid[f][G][G] = spread of c = scale * w * pf * y[f] (y != NULL, B frames) or
// of c = scale * w (y == NULL, one grid); toff/tent: per-tile sample lists.
hipError_t launch_grid_spread(int G, int W, int B, int64_t M, const int* toff, const int* tent,
                              const int2* base, const double* wy, const double* wx,
                              const double2* pf, const float2* y, const double* w, double scale,
                              double2* grid, hipStream_t s);
// out[f][n][m] = FFT2(grid[f])[(n-h) mod G][(m-h) mod G] * deap[n] * deap[m].
hipError_t launch_grid_fft(int G, int Nout, int h, int B, const double2* grid, double2* rows,
                           const double* deap, float2* out, const double2* tw, hipStream_t s);
hipError_t launch_grid_fft(int G, int Nout, int h, int B, const double2* grid, double2* rows,
                           const double* deap, double2* out, const double2* tw, hipStream_t s);
// w[l] <- w[l] / Re(interpolation of grid at sample l) * scale.
hipError_t launch_dcf_update(int G, int W, int64_t M, const int2* base, const double* wy,
                             const double* wx, const double2* grid, double* w, double scale,
                             hipStream_t s);
hipError_t launch_fill_f64(size_t n, double v, double* p, hipStream_t s);
// Circular L x L embedding of the lags |a|, |b| <= N-1 of a 2N x 2N type-1
// output (lag a at row a + N), optional export [2N-1][2N-1] complex128.
hipError_t launch_lag_embed(int N, int L, const double2* lag2n, double* lag_out, double2* emb,
                            hipStream_t s);

}  // namespace recon
