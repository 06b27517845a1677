// Adjoint NUDFT b = A^H y accumulated in FP64 on the matrix cores
// (Appendix A.2, Eq. AnnMatGD), the accurate form of the "DFT of the data".
//
//   b[n][m] = (1/N) sum_l conj(Ey[l][n]) * (y_l conj(Ex[l][m]))
//
// The perturbation of b propagates into the iterate with a large gain (the
// criterion is ill-conditioned), so this form keeps every phasor, product and
// partial sum in FP64 and rounds b to FP32 once at the end.
//
// Phasors come from per-plan FP64 phase tables, one record per sample and
// axis: exp(-i 2 pi k) (unit step), exp(-i 2 pi k 4j) for j < 16 (offsets
// inside a 64-wide tile) and exp(-i 2 pi k 64t) for the tiles t.  A thread
// forms exp(-i 2 pi k (64t + 4j + v)), v < 4, as tile x offset followed by
// three unit steps: four complex products instead of sincospi evaluations
// (on this chip FP64 vector work competes with the FP64 matrix pipe), with a
// relative error of a few 1e-16.
#include <map>
#include <mutex>
#include <utility>

#include "common.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace recon {

constexpr int AT = 64;        // output tile
constexpr int AK = 16;        // samples per LDS stage
constexpr int ALD = AT + 16;  // padded LDS row (doubles)

__device__ __forceinline__ double2 z_mul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

int phase_record(int N) { return 17 + (N + AT - 1) / AT; }

// ph[a][l][r], a = 0 (k_x), 1 (k_y); r = 0: exp(-i 2 pi k), 1 + j:
// exp(-i 2 pi k 4j) (j < 16), 17 + t: exp(-i 2 pi k AT t).  Every entry from
// the exactly reduced FP64 phase.
__global__ void k_phase_tables_f64(int64_t M, int R, const double* __restrict__ k,
                                   double2* __restrict__ ph) {
  const int64_t total = 2 * M * R;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t al = i / R;
    const int r = (int)(i - al * R);
    const int a = (int)(al / M);
    const int64_t l = al - (int64_t)a * M;
    const double kv = k[2 * l + a];
    const double j = r == 0 ? 1.0 : (r <= 16 ? 4.0 * (r - 1) : (double)AT * (r - 17));
    ph[i] = phasor_f64(-turn_frac(kv, j));
  }
}

hipError_t launch_phase_tables_f64(int64_t M, int N, const double* k, double2* ph, hipStream_t s) {
  const int R = phase_record(N);
  int64_t blocks = (2 * M * R + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_phase_tables_f64<<<(int)blocks, 256, 0, s>>>(M, R, k, ph);
  return hipGetLastError();
}

// Phase-table records and datum of sample l for one thread: unit steps,
// tile bases (tiles tn, tm) and in-tile offsets (index jo) of both axes.
// Samples outside the split (l >= l_end, or an empty trailing split) read
// sample 0 instead; the caller zeroes their contribution.
__device__ __forceinline__ void adj_fetch(int64_t M, int R, const double2* __restrict__ ph,
                                          const float2* __restrict__ yf, int64_t l,
                                          int64_t l_end, int tn, int tm, int jo, double2& sy,
                                          double2& ty, double2& oy, double2& sx, double2& tx,
                                          double2& ox, float2& yv) {
  const int64_t lc = l < l_end ? l : 0;
  const double2* rx = ph + (size_t)lc * R;
  const double2* ry = ph + ((size_t)M + lc) * R;
  sy = ry[0];
  ty = ry[17 + tn];
  oy = ry[1 + jo];
  sx = rx[0];
  tx = rx[17 + tm];
  ox = rx[1 + jo];
  yv = yf[lc];
}

// grid: (n-tiles, m-tiles * frames, splits).  O: float2 (b for the FP32
// iteration) or double2 (b kept in FP64 for the FP64 iteration).
template <typename O>
__global__ __launch_bounds__(256) void k_adjoint_f64(int64_t M, int N, int B, int splits,
                                                     const double2* __restrict__ ph,
                                                     int R,
                                                     const float2* __restrict__ y,
                                                     double2* __restrict__ part,
                                                     O* __restrict__ out, double scale) {
  __shared__ double Ar[AK][ALD], Ai[AK][ALD], Zr[AK][ALD], Zi[AK][ALD];
  const int mt = (N + AT - 1) / AT;
  const int n0 = blockIdx.x * AT;
  const int f = blockIdx.y / mt;
  const int m0 = (blockIdx.y % mt) * AT;
  const int s = blockIdx.z;
  const int64_t per = ((M + splits - 1) / splits + AK - 1) / AK * AK;
  const int64_t l_begin = (int64_t)s * per;
  const int64_t l_end = (l_begin + per < M) ? l_begin + per : M;
  const float2* yf = y + (size_t)f * M;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
  v4d cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) { cr[a][b] = v4d{0, 0, 0, 0}; ci[a][b] = v4d{0, 0, 0, 0}; }

  const int lr = tid >> 4, lc = (tid & 15) * 4;
  // Stage inputs of this thread (sample l0 + lr), loaded one stage ahead so
  // that the loads are in flight during the previous stage's products.
  double2 sy, ty, oy, sx, tx, ox;
  float2 yv;
  adj_fetch(M, R, ph, yf, l_begin + lr, l_end, n0 / AT, m0 / AT, lc / 4, sy, ty, oy, sx, tx, ox,
            yv);
  for (int64_t l0 = l_begin; l0 < l_end; l0 += AK) {
    const int64_t l = l0 + lr;
    const bool lv = l < l_end;
    double2 ea[4], ez[4];
    {
      const double2 yd = make_double2(yv.x, yv.y);
      // conj(Ey[l][n]) = exp(-i 2 pi ky n), n = n0 + lc + v
      ea[0] = z_mul(ty, oy);
#pragma unroll
      for (int v = 1; v < 4; ++v) ea[v] = z_mul(ea[v - 1], sy);
      // y_l conj(Ex[l][m]) = y_l exp(-i 2 pi kx m), m = m0 + lc + v
      double2 e = z_mul(tx, ox);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (v) e = z_mul(e, sx);
        ez[v] = z_mul(yd, e);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const bool an = lv && (n0 + lc + v) < N, am = lv && (m0 + lc + v) < N;
      Ar[lr][lc + v] = an ? ea[v].x : 0.0;
      Ai[lr][lc + v] = an ? ea[v].y : 0.0;
      Zr[lr][lc + v] = am ? ez[v].x : 0.0;
      Zi[lr][lc + v] = am ? ez[v].y : 0.0;
    }
    __syncthreads();
    if (l0 + AK < l_end)
      adj_fetch(M, R, ph, yf, l0 + AK + lr, l_end, n0 / AT, m0 / AT, lc / 4, sy, ty, oy, sx, tx,
                ox, yv);
#pragma unroll
    for (int kk = 0; kk < AK; kk += 4) {
      const int kr = kk + (lane >> 4), cc = lane & 15;
      double ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        ar[a] = Ar[kr][wi + 16 * a + cc];
        ai[a] = Ai[kr][wi + 16 * a + cc];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        br[b] = Zr[kr][wj + 16 * b + cc];
        bi[b] = Zi[kr][wj + 16 * b + cc];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          // A * Z with A = conj(Ey):  re = Ar Zr - Ai Zi,  im = Ar Zi + Ai Zr
          cr[a][b] = mfma_f64_16x16x4(ar[a], br[b], cr[a][b]);
          cr[a][b] = mfma_f64_16x16x4(-ai[a], bi[b], cr[a][b]);
          ci[a][b] = mfma_f64_16x16x4(ar[a], bi[b], ci[a][b]);
          ci[a][b] = mfma_f64_16x16x4(ai[a], br[b], ci[a][b]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = n0 + wi + 16 * a + mfma16_row_f64(lane, r);
        const int m = m0 + wj + 16 * b + mfma16_col(lane);
        if (n < N && m < N) {
          const size_t o = (size_t)n * N + m;
          if (splits == 1) {
            out[(size_t)f * N * N + o] = cmk<O>((real_t<O>)(cr[a][b][r] * scale),
                                                (real_t<O>)(ci[a][b][r] * scale));
          } else {
            part[((size_t)s * B + f) * (size_t)N * N + o] = make_double2(cr[a][b][r], ci[a][b][r]);
          }
        }
      }
}

template <typename O>
__global__ void k_split_reduce_f64(size_t count, int splits, const double2* __restrict__ part,
                                   O* __restrict__ b, double scale) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x) {
    double2 acc = part[i];
    for (int s = 1; s < splits; ++s) {
      const double2 v = part[(size_t)s * count + i];
      acc.x += v.x;
      acc.y += v.y;
    }
    b[i] = cmk<O>((real_t<O>)(acc.x * scale), (real_t<O>)(acc.y * scale));
  }
}

// Launch shape of this adjoint: split-K count and frames per launch, chosen
// so that a launch (tiles x splits x frames blocks) fills whole waves of
// resident blocks.  The kernel holds 3 blocks per CU (register-bound), 768
// on the 256 CUs; a launch of 1024 blocks ran one full wave and then a third
// of one with two thirds of the chip idle.  Among shapes of equal wave
// efficiency the one that also fills the chip for a single frame (a served
// request) and then the one with the fewest blocks is taken; each split keeps
// at least 8 stages of AK samples and the split-K partials of a launch stay
// within 64 MiB (splits x frames x N^2 complex128 values <= 4 Mi).  Depends
// on (M, N) only, so every frame's sums are taken in the same order whatever
// the batch.
constexpr int ADJ64_RESIDENT = 3 * 256;

static void adjoint64_shape_search(int64_t M, int N, int* splits, int* group) {
  const int64_t tiles = (int64_t)cdiv(N, AT) * cdiv(N, AT);
  int64_t max_sp = (M + 8 * AK - 1) / (8 * AK);
  if (max_sp > 192) max_sp = 192;
  if (max_sp < 1) max_sp = 1;
  auto eff = [](int64_t blocks) {
    const int64_t waves = (blocks + ADJ64_RESIDENT - 1) / ADJ64_RESIDENT;
    // efficiency in percent, rounded down
    return (int)(100 * blocks / (waves * ADJ64_RESIDENT));
  };
  int best_sp = 1, best_g = 1, best_e = -1, best_e1 = -1;
  int64_t best_blocks = 0;
  const int64_t max_part = (int64_t)1 << 22;  // complex128 partials per launch
  for (int g = 1; g <= 16; ++g)
    for (int64_t sp = 1; sp <= max_sp; ++sp) {
      if (sp > 1 && sp * g * N * N > max_part) break;
      const int64_t blocks = tiles * sp * g;
      const int e = eff(blocks), e1 = eff(tiles * sp);
      const bool better = e > best_e || (e == best_e && e1 > best_e1) ||
                          (e == best_e && e1 == best_e1 && blocks < best_blocks);
      if (better) {
        best_e = e;
        best_e1 = e1;
        best_blocks = blocks;
        best_sp = (int)sp;
        best_g = g;
      }
    }
  *splits = best_sp;
  *group = best_g;
}

// The search above, remembered per (M, N): workspace layouts and launches
// ask for the shape on every call.
static void adjoint64_shape(int64_t M, int N, int* splits, int* group) {
  static std::mutex mu;
  static std::map<std::pair<int64_t, int>, std::pair<int, int>> memo;
  const std::pair<int64_t, int> key(M, N);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = memo.find(key);
    if (it != memo.end()) {
      *splits = it->second.first;
      *group = it->second.second;
      return;
    }
  }
  adjoint64_shape_search(M, N, splits, group);
  std::lock_guard<std::mutex> lk(mu);
  memo[key] = std::make_pair(*splits, *group);
}

int adjoint64_splits(int64_t M, int N) {
  int sp, g;
  adjoint64_shape(M, N, &sp, &g);
  return sp;
}

int adjoint64_group(int64_t M, int N) {
  int sp, g;
  adjoint64_shape(M, N, &sp, &g);
  return sp == 1 ? (1 << 30) : g;
}

template <typename O>
static hipError_t adjoint_f64_any(int64_t M, int N, int B, const double2* ph, const float2* y,
                                  O* b, double2* part, hipStream_t s) {
  const int sp = adjoint64_splits(M, N);
  const int R = phase_record(N);
  if (sp == 1) {
    dim3 grid(cdiv(N, AT), cdiv(N, AT) * B, 1);
    k_adjoint_f64<O><<<grid, 256, 0, s>>>(M, N, B, 1, ph, R, y, nullptr, b, 1.0 / (double)N);
    return hipGetLastError();
  }
  const int G = adjoint64_group(M, N);
  for (int f0 = 0; f0 < B; f0 += G) {
    const int g = (B - f0 < G) ? B - f0 : G;
    dim3 grid(cdiv(N, AT), cdiv(N, AT) * g, sp);
    k_adjoint_f64<O><<<grid, 256, 0, s>>>(M, N, g, sp, ph, R, y + (size_t)f0 * M, part,
                                          (O*)nullptr, 1.0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t count = (size_t)g * N * N;
    size_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_split_reduce_f64<O><<<(int)blocks, 256, 0, s>>>(count, sp, part, b + (size_t)f0 * N * N,
                                                     1.0 / (double)N);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_adjoint_f64(int64_t M, int N, int B, const double2* ph, const float2* y,
                              float2* b, double2* part, hipStream_t s) {
  return adjoint_f64_any(M, N, B, ph, y, b, part, s);
}
hipError_t launch_adjoint_f64(int64_t M, int N, int B, const double2* ph, const float2* y,
                              double2* b, double2* part, hipStream_t s) {
  return adjoint_f64_any(M, N, B, ph, y, b, part, s);
}

// ---------------------------------------------------------------------------
// FP64 FFT of the rows of an [rows][L] array (in place), for the plan-time
// spectrum of the Gram kernel: one block per row, radix-2 Stockham passes in
// LDS (ping-pong), twiddles exp(-2 pi i t / L) computed in FP64.
__global__ __launch_bounds__(256) void k_fft_rows_f64(int L, int logL, double2* __restrict__ data) {
  extern __shared__ double2 sbuf[];  // 2 L entries
  double2* a = sbuf;
  double2* bb = sbuf + L;
  double2* row = data + (size_t)blockIdx.x * L;
  for (int i = threadIdx.x; i < L; i += blockDim.x) a[i] = row[i];
  __syncthreads();
  int Ns = 1;
  for (int p = 0; p < logL; ++p) {
    for (int j = threadIdx.x; j < L / 2; j += blockDim.x) {
      const int kk = j & (Ns - 1);
      const double2 x0 = a[j], x1 = a[j + L / 2];
      double sn, cs;
      sincospi(-(double)kk / (double)Ns, &sn, &cs);  // exp(-2 pi i kk / (2 Ns))
      const double2 t = z_mul(x1, make_double2(cs, sn));
      const int base = (j - kk) * 2 + kk;
      bb[base] = make_double2(x0.x + t.x, x0.y + t.y);
      bb[base + Ns] = make_double2(x0.x - t.x, x0.y - t.y);
    }
    __syncthreads();
    double2* tmp = a;
    a = bb;
    bb = tmp;
    Ns *= 2;
  }
  for (int i = threadIdx.x; i < L; i += blockDim.x) row[i] = a[i];
}

__global__ void k_transpose_f64(int L, const double2* __restrict__ in, double2* __restrict__ out) {
  __shared__ double2 t[32][33];
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
  for (int j = threadIdx.y; j < 32; j += blockDim.y) {
    const int r = y0 + j, c = x0 + threadIdx.x;
    if (r < L && c < L) t[j][threadIdx.x] = in[(size_t)r * L + c];
  }
  __syncthreads();
  for (int j = threadIdx.y; j < 32; j += blockDim.y) {
    const int r = x0 + j, c = y0 + threadIdx.x;
    if (r < L && c < L) out[(size_t)r * L + c] = t[threadIdx.x][j];
  }
}

// khat_s[q][p] = Re(spec_t[q][p]) / L^2 ; khat_out[p][q] = Re(spec_t[q][p]);
// khat64_s (optional): khat_s without the rounding to FP32.
__global__ void k_khat_finish_f64(int L, const double2* __restrict__ spec_t,
                                  float* __restrict__ khat_s, float* __restrict__ khat_out,
                                  double* __restrict__ khat64_s) {
  const double inv = 1.0 / ((double)L * (double)L);
  const int total = L * L;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int q = i / L, p = i - q * L;
    const double v = spec_t[i].x;
    khat_s[i] = (float)(v * inv);
    if (khat64_s) khat64_s[i] = v * inv;
    if (khat_out) khat_out[(size_t)p * L + q] = (float)v;
  }
}

hipError_t launch_spectrum_f64(int L, double2* emb, double2* tmp, float* khat_s, float* khat_out,
                               double* khat64_s, hipStream_t s) {
  int logL = 0;
  while ((1 << logL) < L) ++logL;
  const size_t shm = 2 * (size_t)L * sizeof(double2);
  k_fft_rows_f64<<<L, 256, shm, s>>>(L, logL, emb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 tg(cdiv(L, 32), cdiv(L, 32));
  k_transpose_f64<<<tg, dim3(32, 8), 0, s>>>(L, emb, tmp);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_fft_rows_f64<<<L, 256, shm, s>>>(L, logL, tmp);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  int blocks = cdiv(L * L, 256);
  if (blocks > 65536) blocks = 65536;
  k_khat_finish_f64<<<blocks, 256, 0, s>>>(L, tmp, khat_s, khat_out, khat64_s);
  return hipGetLastError();
}

}  // namespace recon
