// One iteration of the pseudo-conjugate gradient (Section 3.3) around the
// Toeplitz Gram apply (Section 3.4), as two row kernels on either side of
// the column pass:
//
//   k_dir_rowfft   g = 2 r + lam D^T(w(Dx) Dx)          (recomputed, not stored)
//                  d = -g + beta d_old                   (PR+ with restart)
//                  partials Re<g, d>, sum w(|Dx|) |Dd|^2 (step length)
//                  T[n][:] = FFT_L(pad d[n][:])          (row pass)
//   k_colpass      column FFT, x khat, column IFFT, <d, Qd> partials
//   k_update       Qd[n][:] = IFFT_L(T[n][:]) cropped    (row inverse pass)
//                  alpha = -Re<g, d> / (2 Re<d, Qd> + lam sum w |Dd|^2)
//                  x += alpha d, r += alpha Qd, g_new = 2 r + lam grad R(x),
//                  partials |g_new|^2, Re<g_new, g>, Re<g_new, d>, |g|^2
//
// A block owns ROWS = 256 / T image rows, one FFT team (T = L/V threads, V
// values each) per row; thread t of the team owns the pixels m = t + e T
// (e < V/2) of its row,
// which is exactly the layout the FFT team takes in and gives out, so pixel
// data, the transform and the update stay in registers.  The global loads
// of a thread (own pixels and its share of the one- or two-row halos that
// the stencil needs) are issued together before their first use; the FP64
// update of a large batch instead loads each image just before it is needed,
// which keeps it at four blocks per CU.  The gradient is rebuilt from r and
// x wherever it is needed with the same operations in the same order, so
// every copy of it is bitwise the same.  With a frozen image xb both row
// kernels run the inner step of the half-quadratic minimiser instead.
#include "fft.hpp"
#include "kernels.hpp"
#include "stencil.hpp"

namespace recon {

template <int L>
struct RowCfg {
  static constexpr int TT = FftShape<L>::T;  // threads per row team
  static constexpr int ROWS = 256 / TT;   // rows per block
  static constexpr int W = L / 2;         // widest image row (N <= L/2)
  static constexpr int EPT = W / TT;      // own pixels per thread (V / 2)
  static constexpr int HX2 = (2 * W + 255) / 256;  // two-row halo elements per thread
};

// Logical (row block, frame) of this workgroup.  Workgroups are dispatched
// round-robin over the 8 XCDs (linear id w runs on XCD w % 8).  The row blocks
// of each frame are cut into 8 contiguous ranges, one per XCD: neighbouring
// row blocks, which read each other's rows as stencil halos, mostly share an
// L2, and every frame is spread over the whole chip, so that a launch in which
// only some frames are active (a partly filled serving pool) still keeps every
// XCD busy.  A frame whose row-block count is not a multiple of 8 keeps the
// plain order, which rotates consecutive blocks over the XCDs.
__device__ __forceinline__ void xcd_tile(int& bx, int& f) {
  const int nbx = gridDim.x;
  f = blockIdx.y;
  bx = (nbx % 8 == 0) ? (blockIdx.x % 8) * (nbx / 8) + blockIdx.x / 8 : blockIdx.x;
}

// ------------------------------------------------------- direction + rows
// HQ: one inner step of the half-quadratic minimiser instead (the weights
// and the background weight frozen at the image xb; gradient and curvature of
// the quadratic surrogate): an extra tile of xb rows beside the x tile.
template <int L, int PHI, typename C, bool BG, bool HQ>
__global__ __launch_bounds__(256) void k_dir_rowfft(
    int N, const C* __restrict__ r, const C* __restrict__ d_old, C* __restrict__ d_new,
    const C* __restrict__ x, C* __restrict__ T, const double* __restrict__ p4, int nb4,
    double* __restrict__ p1, const FrameParam* __restrict__ fp, const C* __restrict__ twg,
    int kit, const C* __restrict__ xb) {
  using RC = RowCfg<L>;
  using R = real_t<C>;
  constexpr int TT = RC::TT, ROWS = RC::ROWS, W = RC::W, EPT = RC::EPT;
  constexpr int XT = (ROWS + 3) * W;      // x rows n0-1 .. n0+ROWS+1
  constexpr int DT = (ROWS + 1) * W;      // d rows n0 .. n0+ROWS (over the x tile)
  constexpr int FFTB = ROWS * fft_team_lds<L, C>();
  constexpr int SH = (XT > FFTB) ? XT : FFTB;
  static_assert(DT <= XT, "d tile aliases the x tile");
  // halo element j of a thread: row j / W, column j % W (W a power of two)
  constexpr int HX = (3 * W + 255) / 256;  // x halo elements per thread (3 rows)
  constexpr int HD = (W + 255) / 256;      // r, d halo elements per thread (1 row)
  // FP64: twiddles as running powers in registers (TwPow),
  // loaded just before the transform, instead of an 8-16 KB LDS table
  constexpr bool TWP = sizeof(C) == 16 && L <= 1024;
  int bx, f;
  xcd_tile(bx, f);
  if (kit >= fp[f].stop_at) return;  // frame idle in this iteration (block-uniform)
  __shared__ C tw[TWP ? 1 : L];
  __shared__ C sh[SH];
  // HQ: xb rows n0-1 .. n0+ROWS (the last x row's partner comes from memory);
  // ROWS + 2 rows keep the FP64 kernel at L = 512 within three blocks per CU
  constexpr int BT = (ROWS + 2) * W;
  __shared__ C sbt[HQ ? BT : 1];
  __shared__ double red[3 * 4];
  __shared__ R sbeta;
  C* Xt = sh;  // tile row i <-> image row n0 - 1 + i (stride N)
  C* Dt = sh;  // after the gradients: tile row i <-> image row n0 + i
  C* Bt = sbt;  // HQ: xb, rows as the x tile
  const int n0 = bx * ROWS;
  const size_t fo = (size_t)f * N * N;
  const int team = threadIdx.x / TT, t = threadIdx.x % TT;
  const int n = n0 + team;
  const C zero = cmk<C>(0, 0);

  // -- loads: own pixels, then the halo rows
  C xo[EPT], ro[EPT], dv[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int m = t + e * TT;
    const size_t idx = (n < N && m < N) ? fo + (size_t)n * N + m : 0;
    xo[e] = x[idx];
    ro[e] = r[idx];
    dv[e] = d_old[idx];
  }
  C hx[HX], hr[HD], hd[HD];
#pragma unroll
  for (int s = 0; s < HX; ++s) {
    const int j = threadIdx.x + s * 256;
    const int sel = j / W, m = j % W;  // sel 0: n0-1, 1: n0+ROWS, 2: n0+ROWS+1
    const int img = sel == 0 ? n0 - 1 : n0 + ROWS + sel - 1;
    const bool ok = j < 3 * W && m < N && img >= 0 && img < N;
    hx[s] = x[ok ? fo + (size_t)img * N + m : 0];
  }
#pragma unroll
  for (int s = 0; s < HD; ++s) {
    const int m = threadIdx.x + s * 256;
    const bool ok = m < N && n0 + ROWS < N;
    const size_t idx = ok ? fo + (size_t)(n0 + ROWS) * N + m : 0;
    hr[s] = r[idx];
    hd[s] = d_old[idx];
  }
  if constexpr (!TWP) load_twiddles<L>(tw, twg);

  // beta of the Polak-Ribiere (PR+) correction, with restart, from the
  // update kernel's partials [|g|^2, Re<g, g_old>, Re<g, d_old>, |g_old|^2].
  // (one wavefront reduces, the block reads the value after the next barrier)
  if (threadIdx.x < 64) {
    double g4[4], none[1];
    wave_sum_partials2<4, 0, 1>(p4 + (size_t)f * nb4 * 4, nb4, g4, nullptr, 0, none);
    const double gg = g4[0], ggo = g4[1], gdo = g4[2], gg_old = g4[3];
    double beta = 0.0;
    if (gg_old > 0.0) beta = fmax(0.0, (gg - ggo) / gg_old);
    if (-gg + beta * gdo >= 0.0) beta = 0.0;  // not a descent direction: restart
    if (threadIdx.x == 0) sbeta = (R)beta;
  }
  const R lam = (R)fp[f].lam, delta = (R)fp[f].delta;
  const R lam0 = (R)fp[f].lam0, alpha0 = (R)fp[f].alpha0;

  // -- x tile
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int m = t + e * TT;
    if (n < N && m < N) Xt[(team + 1) * N + m] = xo[e];
  }
#pragma unroll
  for (int s = 0; s < HX; ++s) {
    const int j = threadIdx.x + s * 256;
    const int sel = j / W, m = j % W;
    const int img = sel == 0 ? n0 - 1 : n0 + ROWS + sel - 1;
    if (j < 3 * W && m < N && img >= 0 && img < N) Xt[(img - n0 + 1) * N + m] = hx[s];
  }
  if constexpr (HQ) {  // xb straight into its tile (no register copies)
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int m = t + e * TT;
      if (n < N && m < N) Bt[(team + 1) * N + m] = xb[fo + (size_t)n * N + m];
    }
#pragma unroll
    for (int s = 0; s < RC::HX2; ++s) {
      const int j = threadIdx.x + s * 256;
      const int sel = j / W, m = j % W;  // sel 0: n0-1, 1: n0+ROWS
      const int img = sel == 0 ? n0 - 1 : n0 + ROWS;
      if (j < 2 * W && m < N && img >= 0 && img < N)
        Bt[(img - n0 + 1) * N + m] = xb[fo + (size_t)img * N + m];
    }
  }
  __syncthreads();
  const R bf = sbeta;

  // -- gradient and new direction: own rows and the halo row n0 + ROWS
  double gd = 0.0, cv0 = 0.0;
  C dn[EPT], dh[HD];
  R wdn[EPT], wrt[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int m = t + e * TT;
    dn[e] = zero;
    wdn[e] = wrt[e] = 0;
    if (n < N && m < N) {
      const C* mid = Xt + (team + 1) * N;
      C g;
      C wx = xo[e];  // the image the background weight is taken at
      if constexpr (HQ) {
        const C* bmid = Bt + (team + 1) * N;
        const C div = divergence_frozen_fw<PHI>(
            n > 0 ? mid - N : nullptr, mid, n + 1 < N ? mid + N : nullptr,
            n > 0 ? bmid - N : nullptr, bmid, n + 1 < N ? bmid + N : nullptr, m, N, delta,
            wdn[e], wrt[e]);
        wx = bmid[m];
        g = grad_frozen<BG>(ro[e], div, xo[e], wx, lam, lam0, alpha0);
      } else {
        const C div = divergence_fw<PHI>(n > 0 ? mid - N : nullptr, mid,
                                         n + 1 < N ? mid + N : nullptr, m, N, delta, wdn[e],
                                         wrt[e]);
        g = grad_full<BG>(ro[e], div, xo[e], lam, lam0, alpha0);
      }
      dn[e] = cmk<C>(rfma(bf, dv[e].x, -g.x), rfma(bf, dv[e].y, -g.y));
      d_new[fo + (size_t)n * N + m] = dn[e];
      gd += (double)g.x * (double)dn[e].x + (double)g.y * (double)dn[e].y;
      // background curvature w0(|x|) |d|^2 (majorant of Omega_0 along d;
      // HQ: the frozen w0(|xb|))
      if constexpr (BG) cv0 += (double)bg_weight(wx, lam0, alpha0) * (double)c_abs2(dn[e]);
    }
  }
  if (n0 + ROWS < N) {
    const int nh = n0 + ROWS;
#pragma unroll
    for (int s = 0; s < HD; ++s) {
      const int m = threadIdx.x + s * 256;
      if (m < N) {
        const C* mid = Xt + (ROWS + 1) * N;
        C g;
        if constexpr (HQ) {
          const C* bmid = Bt + (ROWS + 1) * N;
          const C div = divergence_frozen<PHI>(
              mid - N, mid, nh + 1 < N ? mid + N : nullptr, bmid - N, bmid,
              nh + 1 < N ? xb + fo + (size_t)(nh + 1) * N : nullptr, m, N, delta);
          g = grad_frozen<BG>(hr[s], div, mid[m], bmid[m], lam, lam0, alpha0);
        } else {
          const C div =
              divergence<PHI>(mid - N, mid, nh + 1 < N ? mid + N : nullptr, m, N, delta);
          g = grad_full<BG>(hr[s], div, mid[m], lam, lam0, alpha0);
        }
        dh[s] = cmk<C>(rfma(bf, hd[s].x, -g.x), rfma(bf, hd[s].y, -g.y));
      }
    }
  }
  __syncthreads();  // every read of the x tile is done: the d tile replaces it
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int m = t + e * TT;
    if (n < N && m < N) Dt[team * N + m] = dn[e];
  }
  if (n0 + ROWS < N) {
#pragma unroll
    for (int s = 0; s < HD; ++s) {
      const int m = threadIdx.x + s * 256;
      if (m < N) Dt[ROWS * N + m] = dh[s];
    }
  }
  __syncthreads();

  // -- curvature of the half-quadratic majorant along d (own rows)
  double cv = 0.0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int m = t + e * TT;
    if (n < N && m < N) {
      // the weights of the pixel's forward edges come from the divergence
      const C e0 = Dt[team * N + m];
      if (n + 1 < N) {
        const C te = c_sub(Dt[(team + 1) * N + m], e0);
        cv += (double)wdn[e] * (double)c_abs2(te);
      }
      if (m + 1 < N) {
        const C te = c_sub(Dt[team * N + m + 1], e0);
        cv += (double)wrt[e] * (double)c_abs2(te);
      }
    }
  }
  {
    double v3[3] = {gd, cv, cv0};
    block_partials_store<3>(v3, red);  // summed by thread 0 at the end
  }
  __syncthreads();  // the tiles are free; the wave sums are in red

  // -- row FFT of d (team layout in = own pixels)
  C val[FftShape<L>::V];
#pragma unroll
  for (int e = 0; e < EPT; ++e) val[e] = dn[e];
  if constexpr (TWP) {
    TwPow<L, C> twp;
    twp.load(twg, t);
    fft_team<L, false, true>(val, t, sh + team * fft_team_lds<L, C>(), twp);
  } else {
    fft_team<L, false, true>(val, t, sh + team * fft_team_lds<L, C>(), tw);
  }
  if (n < N) {
    C* out = T + ((size_t)f * N + n) * L;
#pragma unroll
    for (int e = 0; e < FftShape<L>::V; ++e) out[t + e * TT] = val[e];
  }
  if (threadIdx.x == 0) {
    double v3[3];
    block_partials_sum<3>(v3, red);
    double* o = p1 + ((size_t)f * gridDim.x + bx) * 3;
    o[0] = v3[0];
    o[1] = v3[1];
    o[2] = v3[2];
  }
}

// ------------------------------------------------ inverse rows + update
// Loads of the update kernel: a thread's own pixels of one image, and its
// share of the two halo rows (n0 - 1 and n0 + ROWS) of one image.
template <int L, typename C>
__device__ __forceinline__ void load_own(int N, size_t fo, int n, int t, const C* __restrict__ src,
                                         C (&dst)[RowCfg<L>::EPT]) {
#pragma unroll
  for (int e = 0; e < RowCfg<L>::EPT; ++e) {
    const int m = t + e * RowCfg<L>::TT;
    dst[e] = src[(n < N && m < N) ? fo + (size_t)n * N + m : 0];
  }
}
template <int L, typename C>
__device__ __forceinline__ void load_halo2(int N, size_t fo, int n0, const C* __restrict__ src,
                                           C (&dst)[RowCfg<L>::HX2]) {
  constexpr int ROWS = RowCfg<L>::ROWS, W = RowCfg<L>::W;
#pragma unroll
  for (int s = 0; s < RowCfg<L>::HX2; ++s) {
    const int j = threadIdx.x + s * 256;
    const int sel = j / W, m = j % W;  // sel 0: n0-1, 1: n0+ROWS
    const int img = sel == 0 ? n0 - 1 : n0 + ROWS;
    const bool ok = j < 2 * W && m < N && img >= 0 && img < N;
    dst[s] = src[ok ? fo + (size_t)img * N + m : 0];
  }
}

// HQ: the update of an inner half-quadratic step (weights frozen at xb; an
// extra tile of xb rows).  EARLY: the FP64 form with every load up front
// (small batches, where occupancy does not matter and each load's latency
// is on the launch's critical path).
template <int L, int PHI, typename C, bool BG, bool HQ, bool EARLY = false>
__global__ __launch_bounds__(256) void k_update(
    int N, const C* __restrict__ T, const C* __restrict__ x_old, C* __restrict__ x_new,
    const C* __restrict__ d, C* __restrict__ r, const double* __restrict__ p1, int nb1,
    const double* __restrict__ p3, int nb3, double* __restrict__ p4,
    const FrameParam* __restrict__ fp, const C* __restrict__ twg, int kit,
    const C* __restrict__ xb) {
  using RC = RowCfg<L>;
  using R = real_t<C>;
  constexpr int TT = RC::TT, ROWS = RC::ROWS, W = RC::W, EPT = RC::EPT;
  constexpr int XT = (ROWS + 2) * W;      // rows n0-1 .. n0+ROWS
  constexpr int FFTB = ROWS * fft_team_lds<L, C>();
  constexpr int HX = RC::HX2;  // halo elements per thread (2 rows, j -> j/W, j%W)
  // The x tile and the transform buffers share LDS: the inverse transform
  // runs first.
  constexpr int SH = XT > FFTB ? XT : FFTB;
  // FP32 at L <= 512: the thread's twiddles in registers instead of an LDS
  // table (11% faster; the FP64 form has no registers to spare, and the
  // direction kernel gained nothing from it)
  constexpr bool TWR = sizeof(C) == 8 && L <= 512;
  // FP64: running powers (TwPow), one twiddle per pass and butterfly
  constexpr bool TWP = sizeof(C) == 16 && L <= 1024;
  int bx, f;
  xcd_tile(bx, f);
  if (kit >= fp[f].stop_at) return;
  __shared__ C tw[(TWR || TWP) ? 1 : L];
  __shared__ C sh[SH];
  __shared__ C sbt[HQ ? XT : 1];
  __shared__ double red[4 * 4];
  __shared__ R salpha;
  C* Xt = sh;                      // x, then x + alpha d (in place); row i <-> image row n0-1+i
  C* fb = sh;                      // exchange buffers of the row transforms
  C* Bt = sbt;                     // HQ: xb, rows as the x tile
  const int n0 = bx * ROWS;
  const size_t fo = (size_t)f * N * N;
  const int team = threadIdx.x / TT, t = threadIdx.x % TT;
  const int n = n0 + team;

  // -- loads: the transformed row, own pixels, halo rows
  C val[FftShape<L>::V];
  {
    const C* row = T + ((size_t)f * N + (n < N ? n : 0)) * L;
#pragma unroll
    for (int e = 0; e < FftShape<L>::V; ++e) val[e] = row[t + e * TT];
  }
  // LATE (the FP64 form): each image is loaded just before its first use,
  // after the inverse transform, so that few of them are live at once.  At
  // L <= 512 that leaves 125 registers and, with the transform buffers
  // aliased to the x tile, <= 33 KB of LDS: 4 blocks per CU (an earlier form
  // with all loads up front and separate buffers held 3; the update at 256^2
  // went from 0.216 to 0.192 ms per 128 frames).
  constexpr bool LATE = sizeof(C) == 16 && !EARLY;
  // FP64: the new x is stored after the block's last barrier, which would
  // otherwise wait for those stores to complete, from the tile (the FP32 form
  // stores it in the last loop: the longer-lived tile costs it a wave)
  constexpr bool XLAST = sizeof(C) == 16;
  C xo[EPT], dv[EPT], ro[EPT];
  C hx[HX], hd[HX];
  if constexpr (!LATE) {
    load_own<L>(N, fo, n, t, x_old, xo);
    load_own<L>(N, fo, n, t, d, dv);
    load_own<L>(N, fo, n, t, r, ro);
    load_halo2<L>(N, fo, n0, x_old, hx);
    load_halo2<L>(N, fo, n0, d, hd);
  }
  TwRegs<(TWR ? L : 64), C> twr;
  TwPow<(TWP ? L : 64), C> twp;
  if constexpr (TWR) twr.load(twg, t);
  else if constexpr (TWP) twp.load(twg, t);
  else load_twiddles<L>(tw, twg);

  // Step length: exact minimiser of the half-quadratic majorant along d
  // (one wavefront reduces, the block reads it after the barrier).
  const R lam = (R)fp[f].lam, delta = (R)fp[f].delta;
  const R lam0 = (R)fp[f].lam0, alpha0 = (R)fp[f].alpha0;
  if (threadIdx.x < 64) {
    double s1[3], s3[1];
    wave_sum_partials2<3, 1, 2>(p1 + (size_t)f * nb1 * 3, nb1, s1, p3 + (size_t)f * nb3, nb3,
                                s3);
    const double gd = s1[0], cvv = s1[1], cv0 = s1[2], dqd = s3[0];
    const double den = 2.0 * dqd + fp[f].lam * cvv + (BG ? fp[f].lam0 * cv0 : 0.0);
    const double alpha = (gd == 0.0) ? 0.0 : -gd / den;
    if (threadIdx.x == 0) salpha = (R)alpha;
  }

  // -- Qd row: inverse FFT, first N outputs (v[e], e < V/2, are pixels t + e T)
  // (register twiddles: each team starts as soon as its row is in; the step
  // length is read after a later barrier)
  if constexpr (!TWR && !TWP) __syncthreads();  // the LDS twiddle table
  if constexpr (TWR) fft_team<L, true, false>(val, t, fb + team * fft_team_lds<L, C>(), twr);
  else if constexpr (TWP) fft_team<L, true, false>(val, t, fb + team * fft_team_lds<L, C>(), twp);
  else fft_team<L, true, false>(val, t, fb + team * fft_team_lds<L, C>(), tw);
  __syncthreads();  // the transform buffers become the x tile
  if constexpr (LATE) {
    load_own<L>(N, fo, n, t, x_old, xo);
    load_halo2<L>(N, fo, n0, x_old, hx);
  }

  // Old x: tile, divergence and gradient at the start of the iteration.
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int m = t + e * TT;
    if (n < N && m < N) Xt[(team + 1) * N + m] = xo[e];
  }
#pragma unroll
  for (int s = 0; s < HX; ++s) {
    const int j = threadIdx.x + s * 256;
    const int sel = j / W, m = j % W;
    const int img = sel == 0 ? n0 - 1 : n0 + ROWS;
    if (j < 2 * W && m < N && img >= 0 && img < N) Xt[(img - n0 + 1) * N + m] = hx[s];
  }
  if constexpr (HQ) {  // the xb tile, same rows, straight from memory
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int m = t + e * TT;
      if (n < N && m < N) Bt[(team + 1) * N + m] = xb[fo + (size_t)n * N + m];
    }
#pragma unroll
    for (int s = 0; s < HX; ++s) {
      const int j = threadIdx.x + s * 256;
      const int sel = j / W, m = j % W;
      const int img = sel == 0 ? n0 - 1 : n0 + ROWS;
      if (j < 2 * W && m < N && img >= 0 && img < N)
        Bt[(img - n0 + 1) * N + m] = xb[fo + (size_t)img * N + m];
    }
  }
  __syncthreads();  // x tile, twiddles, step length
  const R af = salpha;
  // go: the old gradient (LATE: the old divergence; the gradient is formed
  // in the last loop, with the same operations)
  C go[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int m = t + e * TT;
    go[e] = cmk<C>(0, 0);
    if (n < N && m < N) {
      const C* mo = Xt + (team + 1) * N;
      if constexpr (HQ) {
        const C* bm = Bt + (team + 1) * N;
        const C div_o = divergence_frozen<PHI>(
            n > 0 ? mo - N : nullptr, mo, n + 1 < N ? mo + N : nullptr,
            n > 0 ? bm - N : nullptr, bm, n + 1 < N ? bm + N : nullptr, m, N, delta);
        if constexpr (LATE) go[e] = div_o;
        else go[e] = grad_frozen<BG>(ro[e], div_o, xo[e], bm[m], lam, lam0, alpha0);
      } else {
        const C div_o = divergence<PHI>(n > 0 ? mo - N : nullptr, mo,
                                        n + 1 < N ? mo + N : nullptr, m, N, delta);
        if constexpr (LATE) go[e] = div_o;
        else go[e] = grad_full<BG>(ro[e], div_o, xo[e], lam, lam0, alpha0);
      }
    }
  }
  __syncthreads();  // every read of the old x is done

  // New x = x + alpha d, in place (each thread rewrites the entries it wrote;
  // LATE reads its old values back from the tile).
  if constexpr (LATE) {
    load_own<L>(N, fo, n, t, d, dv);
    load_halo2<L>(N, fo, n0, d, hd);
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int m = t + e * TT;
    if (n < N && m < N) {
      C* p = Xt + (team + 1) * N + m;
      *p = c_axpy(af, dv[e], LATE ? *p : xo[e]);
    }
  }
#pragma unroll
  for (int s = 0; s < HX; ++s) {
    const int j = threadIdx.x + s * 256;
    const int sel = j / W, m = j % W;
    const int img = sel == 0 ? n0 - 1 : n0 + ROWS;
    if (j < 2 * W && m < N && img >= 0 && img < N) {
      C* p = Xt + (img - n0 + 1) * N + m;
      *p = c_axpy(af, hd[s], LATE ? *p : hx[s]);
    }
  }

  __syncthreads();  // new x tile complete
  if constexpr (LATE) {
    load_own<L>(N, fo, n, t, r, ro);
    if (BG && lam0 != 0) load_own<L>(N, fo, n, t, x_old, xo);  // the background term needs x
  }

  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int m = t + e * TT;
    if (n < N && m < N) {
      const size_t idx = fo + (size_t)n * N + m;
      const C* mn = Xt + (team + 1) * N;
      const C rn = c_axpy(af, val[e], ro[e]);
      C goe, gn;
      if constexpr (HQ) {
        const C* bm = Bt + (team + 1) * N;
        const C div_n = divergence_frozen<PHI>(
            n > 0 ? mn - N : nullptr, mn, n + 1 < N ? mn + N : nullptr,
            n > 0 ? bm - N : nullptr, bm, n + 1 < N ? bm + N : nullptr, m, N, delta);
        goe = LATE ? grad_frozen<BG>(ro[e], go[e], xo[e], bm[m], lam, lam0, alpha0) : go[e];
        gn = grad_frozen<BG>(rn, div_n, mn[m], bm[m], lam, lam0, alpha0);
      } else {
        const C div_n = divergence<PHI>(n > 0 ? mn - N : nullptr, mn,
                                        n + 1 < N ? mn + N : nullptr, m, N, delta);
        goe = LATE ? grad_full<BG>(ro[e], go[e], xo[e], lam, lam0, alpha0) : go[e];
        gn = grad_full<BG>(rn, div_n, mn[m], lam, lam0, alpha0);
      }
      if constexpr (!XLAST) x_new[idx] = mn[m];
      r[idx] = rn;
      const double gx = gn.x, gy = gn.y;
      acc[0] += gx * gx + gy * gy;
      acc[1] += gx * (double)goe.x + gy * (double)goe.y;
      acc[2] += gx * (double)dv[e].x + gy * (double)dv[e].y;
      acc[3] += (double)goe.x * (double)goe.x + (double)goe.y * (double)goe.y;
    }
  }
  block_partials_store<4>(acc, red);
  __syncthreads();
  if constexpr (XLAST) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int m = t + e * TT;
      if (n < N && m < N) x_new[fo + (size_t)n * N + m] = Xt[(team + 1) * N + m];
    }
  }
  if (threadIdx.x == 0) {
    block_partials_sum<4>(acc, red);
    double* o = p4 + ((size_t)f * gridDim.x + bx) * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = acc[k];
  }
}

// ------------------------------------------------------------------ launchers
// (the FP64 iteration, C = double2, is built for L <= 1024)
#define RECON_ITER_L_SWITCH(L_, CALL)                    \
  switch (L_) {                                          \
    case 64: { constexpr int LL = 64; CALL; } break;     \
    case 128: { constexpr int LL = 128; CALL; } break;   \
    case 256: { constexpr int LL = 256; CALL; } break;   \
    case 512: { constexpr int LL = 512; CALL; } break;   \
    case 1024: { constexpr int LL = 1024; CALL; } break; \
    case 2048: {                                         \
      if constexpr (sizeof(C) == 8) {                    \
        constexpr int LL = 2048;                         \
        CALL;                                            \
      }                                                  \
    } break;                                             \
    default: return hipErrorInvalidValue;                \
  }
#define RECON_ITER_PHI_SWITCH(PHI_, CALL)             \
  switch (PHI_) {                                     \
    case 0: { constexpr int PP = 0; CALL; } break;    \
    case 1: { constexpr int PP = 1; CALL; } break;    \
    case 2: { constexpr int PP = 2; CALL; } break;    \
    default: return hipErrorInvalidValue;             \
  }

template <typename C, bool BG, bool HQ>
static hipError_t dir_rowfft_t(int L, int phi, int N, int B, const C* r, const C* d_old,
                               C* d_new, const C* x, C* T, const double* p4, int nb4, double* p1,
                               const FrameParam* fp, const C* tw, int k, const C* xb,
                               hipStream_t s) {
  dim3 grid(cdiv(N, fft_rows_per_block(L)), B);
  RECON_ITER_PHI_SWITCH(phi, RECON_ITER_L_SWITCH(L, (k_dir_rowfft<LL, PP, C, BG, HQ><<<grid, 256, 0, s>>>(
                                                        N, r, d_old, d_new, x, T, p4, nb4, p1,
                                                        fp, tw, k, xb))));
  return hipGetLastError();
}

template <typename C>
static hipError_t dir_rowfft_any(int L, int phi, int N, int B, const C* r, const C* d_old,
                                 C* d_new, const C* x, C* T, const double* p4, int nb4, double* p1,
                                 const FrameParam* fp, const C* tw, int k, bool bg, const C* xb,
                                 hipStream_t s) {
  if (N > L / 2) return hipErrorInvalidValue;
  if (sizeof(C) == 16 && L > 1024) return hipErrorInvalidValue;
  if (xb)
    return bg ? dir_rowfft_t<C, true, true>(L, phi, N, B, r, d_old, d_new, x, T, p4, nb4, p1, fp,
                                            tw, k, xb, s)
              : dir_rowfft_t<C, false, true>(L, phi, N, B, r, d_old, d_new, x, T, p4, nb4, p1, fp,
                                             tw, k, xb, s);
  return bg ? dir_rowfft_t<C, true, false>(L, phi, N, B, r, d_old, d_new, x, T, p4, nb4, p1, fp,
                                           tw, k, xb, s)
            : dir_rowfft_t<C, false, false>(L, phi, N, B, r, d_old, d_new, x, T, p4, nb4, p1, fp,
                                            tw, k, xb, s);
}

template <typename C, bool BG, bool HQ, bool EARLY = false>
static hipError_t update_t(int L, int phi, int N, int B, const C* T, const C* x_old, C* x_new,
                           const C* d, C* r, const double* p1, int nb1, const double* p3, int nb3,
                           double* p4, const FrameParam* fp, const C* tw, int k, const C* xb,
                           hipStream_t s) {
  dim3 grid(cdiv(N, fft_rows_per_block(L)), B);
  RECON_ITER_PHI_SWITCH(phi, RECON_ITER_L_SWITCH(L, (k_update<LL, PP, C, BG, HQ, EARLY><<<grid, 256, 0, s>>>(
                                                        N, T, x_old, x_new, d, r, p1, nb1, p3,
                                                        nb3, p4, fp, tw, k, xb))));
  return hipGetLastError();
}

// Batches up to this many frames take the FP64 update with every load up
// front (the same arithmetic in the same order, so the same bits): at 256^2
// 28.1 against 29.0 us per iteration for one frame, 36.7 against 37.5 for
// four; at eight frames the late loads are ahead (47.2 against 49.6).
constexpr int kEarlyUpdateMaxB = 4;

template <typename C>
static hipError_t update_any(int L, int phi, int N, int B, const C* T, const C* x_old, C* x_new,
                             const C* d, C* r, const double* p1, int nb1, const double* p3,
                             int nb3, double* p4, const FrameParam* fp, const C* tw, int k,
                             bool bg, const C* xb, hipStream_t s) {
  if (N > L / 2) return hipErrorInvalidValue;
  if (sizeof(C) == 16 && L > 1024) return hipErrorInvalidValue;
  if (xb)
    return bg ? update_t<C, true, true>(L, phi, N, B, T, x_old, x_new, d, r, p1, nb1, p3, nb3, p4,
                                        fp, tw, k, xb, s)
              : update_t<C, false, true>(L, phi, N, B, T, x_old, x_new, d, r, p1, nb1, p3, nb3,
                                         p4, fp, tw, k, xb, s);
  if constexpr (sizeof(C) == 16) {
    if (B <= kEarlyUpdateMaxB)
      return bg ? update_t<C, true, false, true>(L, phi, N, B, T, x_old, x_new, d, r, p1, nb1, p3,
                                                 nb3, p4, fp, tw, k, xb, s)
                : update_t<C, false, false, true>(L, phi, N, B, T, x_old, x_new, d, r, p1, nb1,
                                                  p3, nb3, p4, fp, tw, k, xb, s);
  }
  return bg ? update_t<C, true, false>(L, phi, N, B, T, x_old, x_new, d, r, p1, nb1, p3, nb3, p4,
                                       fp, tw, k, xb, s)
            : update_t<C, false, false>(L, phi, N, B, T, x_old, x_new, d, r, p1, nb1, p3, nb3, p4,
                                        fp, tw, k, xb, s);
}

hipError_t launch_dir_rowfft(int L, int phi, int N, int B, const float2* r,
                             const float2* d_old, float2* d_new, const float2* x, float2* T,
                             const double* p4, int nb4, double* p1, const FrameParam* fp,
                             const float2* tw, int k, bool bg, hipStream_t s, const float2* xb) {
  return dir_rowfft_any(L, phi, N, B, r, d_old, d_new, x, T, p4, nb4, p1, fp, tw, k, bg, xb, s);
}
hipError_t launch_dir_rowfft(int L, int phi, int N, int B, const double2* r,
                             const double2* d_old, double2* d_new, const double2* x, double2* T,
                             const double* p4, int nb4, double* p1, const FrameParam* fp,
                             const double2* tw, int k, bool bg, hipStream_t s,
                             const double2* xb) {
  return dir_rowfft_any(L, phi, N, B, r, d_old, d_new, x, T, p4, nb4, p1, fp, tw, k, bg, xb, s);
}

hipError_t launch_update(int L, int phi, int N, int B, const float2* T, const float2* x_old,
                         float2* x_new, const float2* d, float2* r, const double* p1, int nb1,
                         const double* p3, int nb3, double* p4, const FrameParam* fp,
                         const float2* tw, int k, bool bg, hipStream_t s, const float2* xb) {
  return update_any(L, phi, N, B, T, x_old, x_new, d, r, p1, nb1, p3, nb3, p4, fp, tw, k, bg, xb,
                    s);
}
hipError_t launch_update(int L, int phi, int N, int B, const double2* T, const double2* x_old,
                         double2* x_new, const double2* d, double2* r, const double* p1, int nb1,
                         const double* p3, int nb3, double* p4, const FrameParam* fp,
                         const double2* tw, int k, bool bg, hipStream_t s, const double2* xb) {
  return update_any(L, phi, N, B, T, x_old, x_new, d, r, p1, nb1, p3, nb3, p4, fp, tw, k, bg, xb,
                    s);
}

}  // namespace recon
