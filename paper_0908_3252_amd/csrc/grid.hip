// Convolution gridding with a Kaiser-Bessel kernel: the gridding
// reconstruction the paper compares against (Section 1: density weighting,
// resampling onto a Cartesian grid with a kernel, FFT, apodization
// correction; Section 4.1: 7 x 7 Kaiser-Bessel kernel) and the non-uniform
// FFT that Section 5 proposes for the precomputation of D = A^H y and of the
// Gram kernel.  All arithmetic in FP64.
//
// Type-1 sum on an Nout x Nout output with offset h, grid of G points per
// axis (G >= 2 Nout, a power of two), kernel width W:
//   out[n][m] = sum_l c_l exp(-i 2 pi (ky_l (n - h) + kx_l (m - h)))
//     c on the grid:  grid[g1][g2] = sum_l c_l phi(g1 - G ky_l) phi(g2 - G kx_l)
//     forward 2D FFT of the grid, outputs (n - h) mod G kept,
//     divided by phi_hat((n - h)/G) phi_hat((m - h)/G).
//
// Spreading is a gather: the grid is cut into 32 x 32 tiles, the samples
// whose W x W footprint touches a tile are listed per tile when the plan is
// made (on the host), and one block owns one tile, so every grid point is
// written once by one thread, in a fixed order (no atomics; results are
// reproducible and do not depend on the batch size).  The kernel weights of
// every sample (W per axis) are computed once per plan.
#include "fft.hpp"
#include "kernels.hpp"

namespace recon {

constexpr int GTILE = 32;   // grid tile side
constexpr int GCH = 64;     // samples staged per round
constexpr int GFR = 4;      // frames per spreading block

// Modified Bessel function I0 by its power series (x <= 40: at most ~80
// terms to FP64 precision).
__device__ __forceinline__ double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 200; ++k) {
    term *= q / ((double)k * (double)k);
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

// Per-sample kernel weights wy[l][i] = phi(g0y + i - G ky), wx likewise
// (i < W, g0 = floor(G k - W/2) + 1), footprint origins base[l] = (g0y mod G,
// g0x mod G), and the sample phase pf[l] = exp(-i 2 pi (kx + ky) h) (phase
// != 0) or 1.
__global__ void k_grid_weights(int64_t M, int G, int W, double beta, int h, int phase,
                               const double* __restrict__ k, int2* __restrict__ base,
                               double* __restrict__ wy, double* __restrict__ wx,
                               double2* __restrict__ pf) {
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < M;
       l += (int64_t)gridDim.x * blockDim.x) {
    const double kx = k[2 * l], ky = k[2 * l + 1];
    const double uy = (double)G * ky, ux = (double)G * kx;
    const double g0y = floor(uy - 0.5 * W) + 1.0, g0x = floor(ux - 0.5 * W) + 1.0;
    for (int i = 0; i < W; ++i) {
      const double ty = 2.0 * (g0y + i - uy) / W, tx = 2.0 * (g0x + i - ux) / W;
      const double ay = 1.0 - ty * ty, ax = 1.0 - tx * tx;
      wy[l * W + i] = ay >= 0.0 ? bessel_i0(beta * sqrt(ay)) : 0.0;
      wx[l * W + i] = ax >= 0.0 ? bessel_i0(beta * sqrt(ax)) : 0.0;
    }
    const int iy = (int)(((int64_t)g0y % G + G) % G), ix = (int)(((int64_t)g0x % G + G) % G);
    base[l] = make_int2(iy, ix);
    if (phase) {
      const double t = turn_frac(kx, (double)h) + turn_frac(ky, (double)h);
      pf[l] = phasor_f64(-t);
    } else {
      pf[l] = make_double2(1.0, 0.0);
    }
  }
}

// Spreading source: MODE 0 complex64 data [B][M] (times pf, scale and the
// optional real weights w), MODE 1 the real weights w alone (density
// compensation).
template <int MODE>
__global__ __launch_bounds__(256) void k_spread(int G, int W, int B, int64_t M,
                                                const int* __restrict__ toff,
                                                const int* __restrict__ tent,
                                                const int2* __restrict__ base,
                                                const double* __restrict__ wy,
                                                const double* __restrict__ wx,
                                                const double2* __restrict__ pf,
                                                const float2* __restrict__ y,
                                                const double* __restrict__ w, double scale,
                                                double2* __restrict__ grid) {
  __shared__ double sy[GCH][16], sx[GCH][16];
  __shared__ int2 sb[GCH];
  __shared__ double2 sc[GFR][GCH];
  const int ntx = G / GTILE;
  const int tile = blockIdx.x;
  const int ty0 = (tile / ntx) * GTILE, tx0 = (tile % ntx) * GTILE;
  const int f0 = blockIdx.y * GFR;
  const int nf = min(GFR, B - f0);
  const int r = threadIdx.x >> 3, c0 = (threadIdx.x & 7) * 4;
  const int gy = ty0 + r;
  double2 acc[GFR][4];
#pragma unroll
  for (int f = 0; f < GFR; ++f)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[f][j] = make_double2(0.0, 0.0);
  const int e0 = toff[tile], e1 = toff[tile + 1];
  for (int e = e0; e < e1; e += GCH) {
    const int cnt = min(GCH, e1 - e);
    for (int i = threadIdx.x; i < cnt * W; i += 256) {
      const int s = i / W, j = i - s * W;
      const int64_t l = tent[e + s];
      sy[s][j] = wy[l * W + j];
      sx[s][j] = wx[l * W + j];
    }
    if (threadIdx.x < cnt) {
      const int64_t l = tent[e + threadIdx.x];
      sb[threadIdx.x] = base[l];
      if constexpr (MODE == 0) {
        const double2 p = pf[l];
        const double wl = (w ? w[l] : 1.0) * scale;
        for (int f = 0; f < nf; ++f) {
          const float2 v = y[(size_t)(f0 + f) * M + l];
          sc[f][threadIdx.x] = make_double2(wl * ((double)v.x * p.x - (double)v.y * p.y),
                                            wl * ((double)v.x * p.y + (double)v.y * p.x));
        }
      } else {
        sc[0][threadIdx.x] = make_double2(w[l] * scale, 0.0);
      }
    }
    __syncthreads();
    for (int s = 0; s < cnt; ++s) {
      const int2 b = sb[s];
      const int dy = (gy - b.x) & (G - 1);
      if (dy >= W) continue;
      const double wyv = sy[s][dy];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int dx = (tx0 + c0 + j - b.y) & (G - 1);
        if (dx < W) {
          const double wv = wyv * sx[s][dx];
#pragma unroll
          for (int f = 0; f < GFR; ++f) {
            if (f < nf) {
              acc[f][j].x = fma(wv, sc[f][s].x, acc[f][j].x);
              acc[f][j].y = fma(wv, sc[f][s].y, acc[f][j].y);
            }
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int f = 0; f < GFR; ++f) {
    if (f < nf) {
      double2* gf = grid + (size_t)(f0 + f) * G * G + (size_t)gy * G + tx0 + c0;
#pragma unroll
      for (int j = 0; j < 4; ++j) gf[j] = acc[f][j];
    }
  }
}

// Forward FFT of every grid row; the Nout kept frequencies (p - h mod G in
// [-h, Nout - h)) go to rows[f][g][q], q = (p + h) mod G.
template <int G>
__global__ __launch_bounds__(256) void k_grid_rows(int Nout, int h, const double2* __restrict__ grid,
                                                   double2* __restrict__ rows,
                                                   const double2* __restrict__ twg) {
  using S = FftShape<G>;
  constexpr int TEAMS = 256 / S::T;
  constexpr bool TWR = S::V == 8 && G >= 2048;  // LDS budget: twiddles in registers
  __shared__ double2 tw[TWR ? 1 : S::TWN];
  __shared__ double2 bufs[TEAMS * fft_team_lds<G, double2>()];
  const int f = blockIdx.y;
  const int team = threadIdx.x / S::T, t = threadIdx.x % S::T;
  const int g = blockIdx.x * TEAMS + team;
  double2 v[S::V];
  const double2* src = grid + ((size_t)f * G + g) * G;
#pragma unroll
  for (int e = 0; e < S::V; ++e) v[e] = src[t + e * S::T];
  double2* tb = bufs + team * fft_team_lds<G, double2>();
  if constexpr (TWR) {
    TwRegs<G, double2> twr;
    twr.load(twg, t);
    fft_team<G, false, false>(v, t, tb, twr);
  } else {
    load_twiddles<G>(tw, twg);
    __syncthreads();
    fft_team<G, false, false>(v, t, tb, tw);
  }
  double2* dst = rows + ((size_t)f * G + g) * Nout;
#pragma unroll
  for (int e = 0; e < S::V; ++e) {
    const int q = (t + e * S::T + h) & (G - 1);
    if (q < Nout) dst[q] = v[e];
  }
}

// Forward FFT of the kept columns, kept rows, apodization correction:
// out[f][n][q] = FFT(rows[f][:][q])[(n - h) mod G] * deap[n] * deap[q].
template <int G, typename O>
__global__ __launch_bounds__(256) void k_grid_cols(int Nout, int h, const double2* __restrict__ rows,
                                                   const double* __restrict__ deap,
                                                   O* __restrict__ out,
                                                   const double2* __restrict__ twg) {
  using S = FftShape<G>;
  constexpr int TEAMS = 256 / S::T;
  constexpr bool TWR = S::V == 8 && G >= 2048;
  __shared__ double2 tw[TWR ? 1 : S::TWN];
  __shared__ double2 bufs[TEAMS * fft_team_lds<G, double2>()];
  const int f = blockIdx.y;
  const int team = threadIdx.x / S::T, t = threadIdx.x % S::T;
  const int q = blockIdx.x * TEAMS + team;
  const bool active = q < Nout;  // uniform per team; multi-wave teams are whole blocks
  double2 v[S::V];
  const double2* src = rows + (size_t)f * G * Nout + (active ? q : 0);
#pragma unroll
  for (int e = 0; e < S::V; ++e) v[e] = src[(size_t)(t + e * S::T) * Nout];
  double2* tb = bufs + team * fft_team_lds<G, double2>();
  if constexpr (TWR) {
    TwRegs<G, double2> twr;
    twr.load(twg, t);
    fft_team<G, false, false>(v, t, tb, twr);
  } else {
    load_twiddles<G>(tw, twg);
    __syncthreads();
    fft_team<G, false, false>(v, t, tb, tw);
  }
  if (!active) return;
  const double dq = deap[q];
  O* of = out + (size_t)f * Nout * Nout;
#pragma unroll
  for (int e = 0; e < S::V; ++e) {
    const int n = (t + e * S::T + h) & (G - 1);
    if (n < Nout) {
      const double s = deap[n] * dq;
      of[(size_t)n * Nout + q] = cmk<O>((real_t<O>)(v[e].x * s), (real_t<O>)(v[e].y * s));
    }
  }
}

// Interpolation (the adjoint of spreading) of a real-weight grid at every
// sample, and the density-compensation update w <- w / Re(I S w); the last
// round also applies the final scale.
__global__ void k_dcf_update(int G, int W, int64_t M, const int2* __restrict__ base,
                             const double* __restrict__ wy, const double* __restrict__ wx,
                             const double2* __restrict__ grid, double* __restrict__ w,
                             double scale) {
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < M;
       l += (int64_t)gridDim.x * blockDim.x) {
    const int2 b = base[l];
    double acc = 0.0;
    for (int i = 0; i < W; ++i) {
      const double* row = reinterpret_cast<const double*>(grid + (size_t)((b.x + i) & (G - 1)) * G);
      double ra = 0.0;
      for (int j = 0; j < W; ++j) ra = fma(wx[l * W + j], row[2 * ((b.y + j) & (G - 1))], ra);
      acc = fma(wy[l * W + i], ra, acc);
    }
    w[l] = w[l] / acc * scale;
  }
}

__global__ void k_fill_f64(size_t n, double v, double* __restrict__ p) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Lag kernel from the 2N x 2N type-1 output (lag a = n - N, b = m - N):
// circular embedding into L x L (lags |a|, |b| <= N-1) and the optional
// export [a + N-1][b + N-1].
__global__ void k_lag_embed(int N, int L, const double2* __restrict__ lag2n,
                            double* __restrict__ lag_out, double2* __restrict__ emb) {
  const int total = L * L;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int p = i / L, q = i - p * L;
    const int a = (p < N) ? p : ((p > L - N) ? p - L : INT32_MAX);
    const int b = (q < N) ? q : ((q > L - N) ? q - L : INT32_MAX);
    double2 v = make_double2(0.0, 0.0);
    if (a != INT32_MAX && b != INT32_MAX) {
      v = lag2n[(size_t)(a + N) * (2 * N) + (b + N)];
      if (lag_out) {
        const size_t o = ((size_t)(a + N - 1) * (2 * N - 1) + (b + N - 1)) * 2;
        lag_out[o] = v.x;
        lag_out[o + 1] = v.y;
      }
    }
    emb[i] = v;
  }
}

// ------------------------------------------------------------------ launchers
static unsigned grid_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 16384) b = 16384;
  return (unsigned)(b < 1 ? 1 : b);
}

hipError_t launch_grid_weights(int64_t M, int G, int W, double beta, int h, int phase,
                               const double* k, int2* base, double* wy, double* wx, double2* pf,
                               hipStream_t s) {
  if (W < 2 || W > 16) return hipErrorInvalidValue;
  k_grid_weights<<<grid_blocks(M), 256, 0, s>>>(M, G, W, beta, h, phase, k, base, wy, wx, pf);
  return hipGetLastError();
}

hipError_t launch_grid_spread(int G, int W, int B, int64_t M, const int* toff, const int* tent,
                              const int2* base, const double* wy, const double* wx,
                              const double2* pf, const float2* y, const double* w, double scale,
                              double2* grid, hipStream_t s) {
  if (G < 2 * GTILE || (G & (G - 1)) || W > 16) return hipErrorInvalidValue;
  const int ntiles = (G / GTILE) * (G / GTILE);
  if (y) {
    dim3 g(ntiles, cdiv(B, GFR));
    k_spread<0><<<g, 256, 0, s>>>(G, W, B, M, toff, tent, base, wy, wx, pf, y, w, scale, grid);
  } else {
    dim3 g(ntiles, 1);
    k_spread<1><<<g, 256, 0, s>>>(G, W, 1, M, toff, tent, base, wy, wx, pf, nullptr, w, scale,
                                  grid);
  }
  return hipGetLastError();
}

template <int G, typename O>
static hipError_t grid_fft_t(int Nout, int h, int B, const double2* grid, double2* rows,
                             const double* deap, O* out, const double2* tw, hipStream_t s) {
  constexpr int TEAMS = 256 / FftShape<G>::T;
  k_grid_rows<G><<<dim3(G / TEAMS, B), 256, 0, s>>>(Nout, h, grid, rows, tw);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_grid_cols<G, O><<<dim3(cdiv(Nout, TEAMS), B), 256, 0, s>>>(Nout, h, rows, deap, out, tw);
  return hipGetLastError();
}

template <typename O>
static hipError_t grid_fft_any(int G, int Nout, int h, int B, const double2* grid, double2* rows,
                               const double* deap, O* out, const double2* tw, hipStream_t s) {
  if (Nout > G / 2) return hipErrorInvalidValue;
  switch (G) {
    case 64: return grid_fft_t<64>(Nout, h, B, grid, rows, deap, out, tw, s);
    case 128: return grid_fft_t<128>(Nout, h, B, grid, rows, deap, out, tw, s);
    case 256: return grid_fft_t<256>(Nout, h, B, grid, rows, deap, out, tw, s);
    case 512: return grid_fft_t<512>(Nout, h, B, grid, rows, deap, out, tw, s);
    case 1024: return grid_fft_t<1024>(Nout, h, B, grid, rows, deap, out, tw, s);
    case 2048: return grid_fft_t<2048>(Nout, h, B, grid, rows, deap, out, tw, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_grid_fft(int G, int Nout, int h, int B, const double2* grid, double2* rows,
                           const double* deap, float2* out, const double2* tw, hipStream_t s) {
  return grid_fft_any(G, Nout, h, B, grid, rows, deap, out, tw, s);
}
hipError_t launch_grid_fft(int G, int Nout, int h, int B, const double2* grid, double2* rows,
                           const double* deap, double2* out, const double2* tw, hipStream_t s) {
  return grid_fft_any(G, Nout, h, B, grid, rows, deap, out, tw, s);
}

hipError_t launch_dcf_update(int G, int W, int64_t M, const int2* base, const double* wy,
                             const double* wx, const double2* grid, double* w, double scale,
                             hipStream_t s) {
  k_dcf_update<<<grid_blocks(M), 256, 0, s>>>(G, W, M, base, wy, wx, grid, w, scale);
  return hipGetLastError();
}

hipError_t launch_fill_f64(size_t n, double v, double* p, hipStream_t s) {
  k_fill_f64<<<grid_blocks((int64_t)n), 256, 0, s>>>(n, v, p);
  return hipGetLastError();
}

hipError_t launch_lag_embed(int N, int L, const double2* lag2n, double* lag_out, double2* emb,
                            hipStream_t s) {
  k_lag_embed<<<grid_blocks((int64_t)L * L), 256, 0, s>>>(N, L, lag2n, lag_out, emb);
  return hipGetLastError();
}

}  // namespace recon
