// Gram operator Q = A^H A applied in the image domain (Section 3.4 and
// Appendix B): the data-term gradient is a linear 2D correlation of the
// image with the trajectory-only kernel, evaluated exactly as
//
//   Q v = crop_N( IFFT_L( khat * FFT_L( pad_L(v) ) ) ),   L >= 2N - 1,
//
// in three streaming passes over an N x L intermediate (only the N non-zero
// rows of the padded image are transformed along rows, and only the N kept
// rows are produced along columns):
//   row pass      v[N][N]  -> T[N][L]      (row FFTs, first half of inputs zero)
//   column pass   T[N][L]  -> T[N][L]      (column FFT, x khat, column IFFT,
//                                           in place, tiles staged in LDS)
//   row inverse   T[N][L]  -> Qv[N][N]     (row IFFTs, first N outputs kept)
// Inside the iteration the row passes are fused with the conjugate-gradient
// direction and update kernels (iterate.hip); the <d, Qd> partial is taken
// in the column pass (Parseval).
#include "fft.hpp"
#include "kernels.hpp"
#include "stencil.hpp"

namespace recon {

// Exchange buffers of one team inside a block-shared array.
template <int L, typename C>
__device__ __forceinline__ C* team_buf(C* base, int team) {
  return base + team * fft_team_lds<L, C>();
}

// ----------------------------------------------------------------- row pass
template <int L, typename C>
__global__ __launch_bounds__(256) void k_rowfft_plain(int N, const C* __restrict__ v,
                                                      C* __restrict__ T,
                                                      const C* __restrict__ twg) {
  using S = FftShape<L>;
  constexpr int ROWS = 256 / S::T;
  __shared__ C tw[L];
  __shared__ C bufs[ROWS * fft_team_lds<L, C>()];
  const int f = blockIdx.y;
  const int team = threadIdx.x / S::T, t = threadIdx.x % S::T;
  const int n = blockIdx.x * ROWS + team;
  load_twiddles<L>(tw, twg);
  C val[S::V];
  const C* row = v + ((size_t)f * N + n) * N;
#pragma unroll
  for (int e = 0; e < S::V / 2; ++e) {
    const int p = t + e * S::T;
    val[e] = (n < N && p < N) ? row[p] : cmk<C>(0, 0);
  }
  __syncthreads();
  fft_team<L, false, true>(val, t, team_buf<L>(bufs, team), tw);
  if (n < N) {
    C* out = T + ((size_t)f * N + n) * L;
#pragma unroll
    for (int e = 0; e < S::V; ++e) out[t + e * S::T] = val[e];
  }
}

// ---------------------------------------------------------------- column pass
// Block = COLS columns of frame f, THREADS threads (TEAMS = THREADS / (L/8)
// columns transformed at once).  With p3 != NULL the block also writes the
// partial sum over its columns of khat_s |FFT(pad col)|^2, which by Parseval
// is its share of Re<v, Q v>.  FP64 elements (ES = 2) halve the columns per
// block (and the threads at L = 512) so that the tile stays within LDS.
template <int L, int ES = 1>
// (FP64 at L = 512 and 1024 has its own kernel, k_colpass_f64 below.)
struct ColCfg {
  static_assert(ES == 1 || L <= 256, "FP64 at L >= 512 uses k_colpass_f64");
  static constexpr int T = FftShape<L>::T;
  static constexpr int THREADS = (L == 512 && ES == 1) ? 512 : 256;
  static constexpr int TEAMS = THREADS / T;
  static constexpr int COLS = ((L <= 64) ? 32 : (L <= 512 ? 16 : 8)) / ES;
  static_assert(COLS % TEAMS == 0 || TEAMS > COLS, "columns per block vs teams");
};

template <int L, typename C>
__global__ __launch_bounds__((ColCfg<L, sizeof(C) / 8>::THREADS)) void k_colpass(
    int N, C* __restrict__ T, const real_t<C>* __restrict__ khat_s, double* __restrict__ p3,
    const C* __restrict__ twg, const FrameParam* __restrict__ fp, int kit) {
  using S = FftShape<L>;
  using CC = ColCfg<L, sizeof(C) / 8>;
  using R = real_t<C>;
  if (fp && kit >= fp[blockIdx.y].stop_at) return;
  constexpr int COLS = CC::COLS;
  constexpr int TEAMS = CC::TEAMS;
  constexpr int NT = CC::THREADS;
  // Column-major tile: column c at tile[c * TS + n].  TS = 2 (mod 16) puts
  // consecutive columns 4 (FP32) or 8 (FP64) 4-byte banks apart, so the 16
  // FP32 (8 FP64) columns of one row that the row-wise staging touches per
  // LDS cycle (consecutive threads -> consecutive columns) hit distinct
  // banks; the column-wise FFT gathers (consecutive threads -> consecutive
  // rows) are unit-stride.
  // INCOL (FP64, wave-local teams): while a team transforms its column, the
  // column's values are in registers, so the column itself (TS >= the
  // component-wise exchange buffer) serves as the team's exchange buffer.
  constexpr bool INCOL = sizeof(C) == 16 && FftSync<L>::WAVE_LOCAL;
  constexpr int TS0 = L / 2 + 2;
  constexpr int TS = (INCOL && fft_team_lds<L, C>() > TS0)
                         ? (fft_team_lds<L, C>() + 15) / 16 * 16 + 2 : TS0;
  constexpr int NBUF = INCOL ? 1 : TEAMS * fft_team_lds<L, C>();
  // FP32 at L <= 512: twiddles in registers (TwRegs) instead of an LDS table
  constexpr bool TWR = sizeof(C) == 8 && L <= 512;
  __shared__ C tw[TWR ? 1 : L];
  __shared__ C tile[COLS * TS];
  __shared__ C bufs[NBUF];
  __shared__ double red[NT / 64];
  const int f = blockIdx.y;
  // Row segments shorter than a cache line (FP32 at L >= 1024: 8 columns,
  // 64 bytes), or a kernel spectrum larger than an XCD's L2 (L >= 1024): a
  // frame's column blocks go to the 8 XCDs in contiguous ranges (workgroups
  // are dispatched round-robin over the XCDs), so the two halves of a line
  // are read by neighbouring blocks that share an L2, and each XCD reads
  // only its eighth of the spectrum's columns.
  int bx = blockIdx.x;
  if constexpr (COLS * sizeof(C) < 128 || L >= 1024) {
    const int nbx = gridDim.x;
    if (nbx % 8 == 0) bx = (blockIdx.x % 8) * (nbx / 8) + blockIdx.x / 8;
  }
  const int q0 = bx * COLS;
  C* Tf = T + (size_t)f * N * L;
  double dqd = 0.0;
  // Stage the block's columns: every load of a thread is issued before the
  // first LDS store (static count: N <= L/2).
  constexpr int SMAX = (L / 2) * COLS / NT;
  C stg[SMAX];
#pragma unroll
  for (int s = 0; s < SMAX; ++s) {
    const int i = threadIdx.x + s * NT;
    const int n = i / COLS, c = i - n * COLS;
    stg[s] = Tf[(n < N ? (size_t)n * L : 0) + q0 + c];
  }
  const int team = threadIdx.x / S::T, t = threadIdx.x % S::T;
  TwRegs<(TWR ? L : 64), C> twr;
  if constexpr (TWR) twr.load(twg, t);
  else load_twiddles<L>(tw, twg);
#pragma unroll
  for (int s = 0; s < SMAX; ++s) {
    const int i = threadIdx.x + s * NT;
    const int n = i / COLS, c = i - n * COLS;
    if (n < N) tile[c * TS + n] = stg[s];
  }
  __syncthreads();
  C* tb = INCOL ? nullptr : team_buf<L>(bufs, team);
  // Wave-local teams touch only their own columns and buffers: no block
  // barrier inside the loop.  Multi-wave teams synchronise inside the FFT.
#pragma unroll 1
  for (int c0 = 0; c0 < COLS; c0 += TEAMS) {
    const int c = c0 + team;
    const bool active = c < COLS;  // uniform per team
    // INCOL teams exchange through their own column: a team without a column
    // skips the round (wave-local teams, so no barrier is missed).
    if (INCOL && !active) continue;
    C val[S::V];
#pragma unroll
    for (int e = 0; e < S::V / 2; ++e) {
      const int p = t + e * S::T;
      val[e] = (active && p < N) ? tile[c * TS + p] : cmk<C>(0, 0);
    }
    // the column's kernel values are loaded before the transform, so that
    // their latency is hidden behind it
    const R* kq = khat_s + (size_t)(q0 + (active ? c : 0)) * L;
    R kvv[S::V];
#pragma unroll
    for (int e = 0; e < S::V; ++e) kvv[e] = kq[t + e * S::T];
    // (INCOL: the reads above precede the exchange writes within the wave)
    if constexpr (TWR) fft_team<L, false, true>(val, t, INCOL ? tile + c * TS : tb, twr);
    else fft_team<L, false, true>(val, t, INCOL ? tile + c * TS : tb, tw);
    R acc = 0;
#pragma unroll
    for (int e = 0; e < S::V; ++e) {
      const R kv = kvv[e];
      acc = rfma(kv, c_abs2(val[e]), acc);
      val[e] = c_scale(val[e], kv);
    }
    if (active) dqd += (double)acc;
    if constexpr (!FftSync<L>::WAVE_LOCAL) __syncthreads();
    if constexpr (TWR) fft_team<L, true, false>(val, t, INCOL ? tile + c * TS : tb, twr);
    else fft_team<L, true, false>(val, t, INCOL ? tile + c * TS : tb, tw);
    if (active) {
#pragma unroll
      for (int e = 0; e < S::V / 2; ++e) {
        const int p = t + e * S::T;
        if (p < N) tile[c * TS + p] = val[e];
      }
    }
    if constexpr (!FftSync<L>::WAVE_LOCAL) __syncthreads();
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < SMAX; ++s) {
    const int i = threadIdx.x + s * NT;
    const int n = i / COLS, c = i - n * COLS;
    if (n < N) Tf[(size_t)n * L + q0 + c] = tile[c * TS + n];
  }
  if (p3) {
    double v1[1] = {dqd};
    block_partials_store<1>(v1, red);
    __syncthreads();
    if (threadIdx.x == 0) {
      block_partials_sum<1>(v1, red);
      p3[(size_t)f * gridDim.x + bx] = v1[0];
    }
  }
}

// FP64 at L = 512 and 1024.  A block takes COLS adjacent columns (four at
// L = 512, two at 1024), one wave-local team (64 threads) per column.  The
// columns' rows are read and written with lanes along the row segments
// (COLS lanes per segment, 64 rows per instruction): read one column per
// lane, the same bytes took 1.6 x as long at L = 512 (125 against 79 us per
// 128-frame launch with no transform at all).  Each column goes through LDS
// to and from its team in the team's own exchange buffer (N <= L/2 values
// fit in it); the block barriers are the two around the transforms and the
// one of the <d, Qd> partial sum.
// Twiddles as running powers (TwPow).  L = 512: 124 registers without
// spills, 4 waves per SIMD (3 with TwRegs: 138-174).  L = 1024 (16 values per
// thread): ~250 registers, 2 waves per SIMD, the kernel values loaded after
// the forward transform; 314 -> 233-240 us per 32-frame launch against the
// earlier 8-column form with a staging tile and an LDS twiddle table.  The
// blocks that share a 128-byte row segment are mapped to one XCD.
template <int L>
struct Col64 {
  static constexpr int COLS = L == 1024 ? 2 : 4;
  static constexpr int THREADS = 64 * COLS;
  static constexpr bool LATEK = L == 1024;  // kernel values after the forward transform
};

template <int L>
__global__ __launch_bounds__(Col64<L>::THREADS) __attribute__((amdgpu_waves_per_eu(L == 512 ? 4 : 2)))
void k_colpass_f64(int N, double2* __restrict__ T, const double* __restrict__ khat_s,
                   double* __restrict__ p3, const double2* __restrict__ twg,
                   const FrameParam* __restrict__ fp, int kit) {
  using C = double2;
  using S = FftShape<L>;
  constexpr int COLS = Col64<L>::COLS, NT = Col64<L>::THREADS;
  constexpr int V = S::V;
  // team stride: the exchange buffer plus two elements, so that the columns
  // of one row (written by adjacent lanes) fall in different LDS banks
  constexpr int TB = fft_team_lds<L, C>() + 2;
  constexpr int RPI = NT / COLS;     // rows per staging instruction (64)
  constexpr int NS = (L / 2) / RPI;  // staging loads per thread
  static_assert(S::T == 64 && NT / S::T == COLS, "one wave-local team per column");
  static_assert(TB >= L / 2, "a column fits in its team's buffer");
  if (fp && kit >= fp[blockIdx.y].stop_at) return;
  __shared__ C bufs[COLS * TB];
  __shared__ double red[COLS];
  const int f = blockIdx.y;
  int bx = blockIdx.x;
  if (gridDim.x % 8 == 0) bx = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
  const int q0 = bx * COLS;
  C* Tf = T + (size_t)f * N * L;
  const int team = threadIdx.x / 64, t = threadIdx.x % 64;
  const int ci = threadIdx.x % COLS, ri = threadIdx.x / COLS;  // staging: column, first row
  C ld[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int n = ri + RPI * s;
    ld[s] = n < N ? Tf[(size_t)n * L + q0 + ci] : cmk<C>(0, 0);
  }
  TwPow<L, C> tw;
  tw.load(twg, t);
  const double* kq = khat_s + (size_t)(q0 + team) * L;
  double kv[V];
  if constexpr (!Col64<L>::LATEK) {
#pragma unroll
    for (int e = 0; e < V; ++e) kv[e] = kq[t + e * 64];
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) bufs[ci * TB + ri + RPI * s] = ld[s];
  __syncthreads();
  C* tb = bufs + team * TB;
  C val[V];
#pragma unroll
  for (int e = 0; e < V / 2; ++e) val[e] = tb[t + 64 * e];
  // (the reads above precede the transform's exchange writes within the wave)
  fft_team<L, false, true>(val, t, tb, tw);
  if constexpr (Col64<L>::LATEK) {
#pragma unroll
    for (int e = 0; e < V; ++e) kv[e] = kq[t + e * 64];
  }
  double acc = 0;
#pragma unroll
  for (int e = 0; e < V; ++e) {
    acc = fma(kv[e], c_abs2(val[e]), acc);
    val[e] = c_scale(val[e], kv[e]);
  }
  fft_team<L, true, false>(val, t, tb, tw);
#pragma unroll
  for (int e = 0; e < V / 2; ++e) tb[t + 64 * e] = val[e];
  if (p3) {
    double v1[1] = {acc};
    block_partials_store<1>(v1, red);
  }
  __syncthreads();  // the columns and the wave sums are in LDS
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int n = ri + RPI * s;
    if (n < N) Tf[(size_t)n * L + q0 + ci] = bufs[ci * TB + ri + RPI * s];
  }
  if (p3 && threadIdx.x == 0) {
    double v1[1];
    block_partials_sum<1>(v1, red);
    p3[(size_t)f * gridDim.x + bx] = v1[0];
  }
}

// --------------------------------------------------------- row inverse pass
template <int L, typename C>
__global__ __launch_bounds__(256) void k_rowifft(int N, const C* __restrict__ T,
                                                 C* __restrict__ out, const C* __restrict__ twg,
                                                 const FrameParam* __restrict__ fp, int kit) {
  using S = FftShape<L>;
  constexpr int ROWS = 256 / S::T;
  if (fp && kit >= fp[blockIdx.y].stop_at) return;
  __shared__ C tw[L];
  __shared__ C bufs[ROWS * fft_team_lds<L, C>()];
  const int f = blockIdx.y;
  const int team = threadIdx.x / S::T, t = threadIdx.x % S::T;
  const int n = blockIdx.x * ROWS + team;
  load_twiddles<L>(tw, twg);
  C val[S::V];
  const C* row = T + ((size_t)f * N + n) * L;
#pragma unroll
  for (int e = 0; e < S::V; ++e) val[e] = (n < N) ? row[t + e * S::T] : cmk<C>(0, 0);
  __syncthreads();
  fft_team<L, true, false>(val, t, team_buf<L>(bufs, team), tw);
  if (n < N) {
    const size_t ro = ((size_t)f * N + n) * N;
#pragma unroll
    for (int e = 0; e < S::V / 2; ++e) {
      const int p = t + e * S::T;
      if (p < N) out[ro + p] = val[e];
    }
  }
}

// ------------------------------------------------------------------ launchers
// (the FP64 forms, C = double2, are built for L <= 1024)
#define RECON_L_SWITCH(L_, CALL)                         \
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

int fft_cols_per_block(int L, bool f64) {
  if (f64 && L == 512) return Col64<512>::COLS;
  if (f64 && L == 1024) return Col64<1024>::COLS;
  switch (L) {
    case 64: return f64 ? ColCfg<64, 2>::COLS : ColCfg<64>::COLS;
    case 128: return f64 ? ColCfg<128, 2>::COLS : ColCfg<128>::COLS;
    case 256: return f64 ? ColCfg<256, 2>::COLS : ColCfg<256>::COLS;
    case 512: return ColCfg<512>::COLS;
    case 1024: return ColCfg<1024>::COLS;
    case 2048: return ColCfg<2048>::COLS;
    default: return 1;
  }
}

template <typename C>
static hipError_t rowfft_plain_any(int L, int N, int B, const C* v, C* T, const C* tw,
                                   hipStream_t s) {
  if (sizeof(C) == 16 && L > 1024) return hipErrorInvalidValue;
  dim3 grid(cdiv(N, fft_rows_per_block(L)), B);
  RECON_L_SWITCH(L, (k_rowfft_plain<LL, C><<<grid, 256, 0, s>>>(N, v, T, tw)));
  return hipGetLastError();
}

// The generic column kernel (FP64 at L >= 512 goes to k_colpass_f64 and is
// not built here).
template <int LL, typename C>
static void colpass_generic(dim3 grid, int N, C* T, const real_t<C>* khat_s, double* p3,
                            const C* tw, const FrameParam* fp, int k, hipStream_t s) {
  if constexpr (sizeof(C) == 8 || LL <= 256)
    k_colpass<LL, C><<<grid, ColCfg<LL, sizeof(C) / 8>::THREADS, 0, s>>>(N, T, khat_s, p3, tw,
                                                                          fp, k);
}

template <typename C>
static hipError_t colpass_any(int L, int N, int B, C* T, const real_t<C>* khat_s, double* p3,
                              const C* tw, const FrameParam* fp, int k, hipStream_t s) {
  if (sizeof(C) == 16 && L > 1024) return hipErrorInvalidValue;
  if constexpr (sizeof(C) == 16) {
    if (L == 512 || L == 1024) {
      if (N > L / 2) return hipErrorInvalidValue;
      if (L == 512)
        k_colpass_f64<512><<<dim3(L / Col64<512>::COLS, B), Col64<512>::THREADS, 0, s>>>(
            N, T, khat_s, p3, tw, fp, k);
      else
        k_colpass_f64<1024><<<dim3(L / Col64<1024>::COLS, B), Col64<1024>::THREADS, 0, s>>>(
            N, T, khat_s, p3, tw, fp, k);
      return hipGetLastError();
    }
  }
  dim3 grid(L / fft_cols_per_block(L, sizeof(C) == 16), B);
  RECON_L_SWITCH(L, (colpass_generic<LL, C>(grid, N, T, khat_s, p3, tw, fp, k, s)));
  return hipGetLastError();
}

template <typename C>
static hipError_t rowifft_any(int L, int N, int B, const C* T, C* out, const C* tw,
                              const FrameParam* fp, int k, hipStream_t s) {
  if (sizeof(C) == 16 && L > 1024) return hipErrorInvalidValue;
  dim3 grid(cdiv(N, fft_rows_per_block(L)), B);
  RECON_L_SWITCH(L, (k_rowifft<LL, C><<<grid, 256, 0, s>>>(N, T, out, tw, fp, k)));
  return hipGetLastError();
}

hipError_t launch_rowfft_plain(int L, int N, int B, const float2* v, float2* T,
                               const float2* tw, hipStream_t s) {
  return rowfft_plain_any(L, N, B, v, T, tw, s);
}
hipError_t launch_rowfft_plain(int L, int N, int B, const double2* v, double2* T,
                               const double2* tw, hipStream_t s) {
  return rowfft_plain_any(L, N, B, v, T, tw, s);
}

hipError_t launch_colpass(int L, int N, int B, float2* T, const float* khat_s, double* p3,
                          const float2* tw, const FrameParam* fp, int k, hipStream_t s) {
  return colpass_any(L, N, B, T, khat_s, p3, tw, fp, k, s);
}
hipError_t launch_colpass(int L, int N, int B, double2* T, const double* khat_s, double* p3,
                          const double2* tw, const FrameParam* fp, int k, hipStream_t s) {
  return colpass_any(L, N, B, T, khat_s, p3, tw, fp, k, s);
}

hipError_t launch_rowifft(int L, int N, int B, const float2* T, float2* out,
                          const float2* tw, const FrameParam* fp, int k, hipStream_t s) {
  return rowifft_any(L, N, B, T, out, tw, fp, k, s);
}
hipError_t launch_rowifft(int L, int N, int B, const double2* T, double2* out,
                          const double2* tw, const FrameParam* fp, int k, hipStream_t s) {
  return rowifft_any(L, N, B, T, out, tw, fp, k, s);
}

}  // namespace recon
