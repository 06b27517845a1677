// Exact non-uniform DFT as separable complex contractions on the matrix
// cores (Section 2, Eq. ModDirect; Appendix A.2, Eq. AnnMatGD).
//
// With the phasor tables Ex[l][m] = exp(i 2 pi kx_l m) and
// Ey[l][n] = exp(i 2 pi ky_l n):
//   adjoint  b[n][m] = (1/N) sum_l conj(Ey[l][n]) * (y_l conj(Ex[l][m]))
//            = (1/N) (Ey^H . diag(y) . conj(Ex))[n][m]   -- GEMM, K = M samples
//   forward  y_l = (1/N) sum_n Ey[l][n] * P[n][l],  P = X . Ex^T -- GEMM, K = N,
//            followed by an Ey-weighted reduction over n in the epilogue.
// Complex products are four real MFMA products with FP32 accumulation.
// Frames of a batch share the tables: the adjoint folds frames into the
// output column dimension, the forward into the grid.
#include "common.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace recon {

constexpr int NT = 64;        // output tile (rows and columns) per block
constexpr int KT = 16;        // samples per LDS stage
constexpr int LDP = NT + 16;  // padded LDS row (floats): 4 k-rows hit distinct banks

// ----------------------------------------------------------------- tables
__global__ void k_tables_f32(int64_t M, int N, const double* __restrict__ k,
                             float2* __restrict__ ex, float2* __restrict__ ey) {
  const int64_t total = M * N;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = i / N;
    const int j = (int)(i - l * N);
    ex[i] = phasor_f32(turn_frac(k[2 * l + 0], (double)j));
    ey[i] = phasor_f32(turn_frac(k[2 * l + 1], (double)j));
  }
}

// ------------------------------------------------------------------ adjoint
// grid: (n-tiles, m-tiles * B, splits).  Block computes the complex tile
// C[n0:n0+64][m0:m0+64] of frame f over its sample range.
__global__ __launch_bounds__(256) void k_adjoint_f32(int64_t M, int N, int B, int splits,
                                                     const float2* __restrict__ ex,
                                                     const float2* __restrict__ ey,
                                                     const float2* __restrict__ y,
                                                     float2* __restrict__ out, float scale) {
  __shared__ float Er[KT][LDP], Ei[KT][LDP], Zr[KT][LDP], Zi[KT][LDP];
  const int mt = (N + NT - 1) / NT;
  const int n0 = blockIdx.x * NT;
  const int f = blockIdx.y / mt;
  const int m0 = (blockIdx.y % mt) * NT;
  const int s = blockIdx.z;
  const int64_t per = ((M + splits - 1) / splits + KT - 1) / KT * KT;
  const int64_t l_begin = (int64_t)s * per;
  const int64_t l_end = (l_begin + per < M) ? l_begin + per : M;
  const float2* yf = y + (size_t)f * M;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wi = (w >> 1) * 32, wj = (w & 1) * 32;  // wave sub-tile origin
  v4f cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) { cr[a][b] = v4f{0, 0, 0, 0}; ci[a][b] = v4f{0, 0, 0, 0}; }

  // loader mapping: 16 rows (samples) x 64 columns, 4 consecutive per thread
  const int lr = tid >> 4, lc = (tid & 15) * 4;
  for (int64_t l0 = l_begin; l0 < l_end; l0 += KT) {
    const int64_t l = l0 + lr;
    const bool lv = l < l_end;
    const float2 yv = lv ? yf[l] : make_float2(0.f, 0.f);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int n = n0 + lc + c, m = m0 + lc + c;
      const float2 e = (lv && n < N) ? ey[(size_t)l * N + n] : make_float2(0.f, 0.f);
      const float2 x = (lv && m < N) ? ex[(size_t)l * N + m] : make_float2(0.f, 0.f);
      Er[lr][lc + c] = e.x;
      Ei[lr][lc + c] = e.y;
      const float2 z = c_mulc(yv, x);  // y_l conj(Ex[l][m])
      Zr[lr][lc + c] = z.x;
      Zi[lr][lc + c] = z.y;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4) {
      const int kr = kk + (lane >> 4), cc = lane & 15;
      float ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        ar[a] = Er[kr][wi + 16 * a + cc];
        ai[a] = Ei[kr][wi + 16 * a + cc];
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
          // conj(E) * Z:  re = Er Zr + Ei Zi,  im = Er Zi - Ei Zr
          cr[a][b] = mfma_f32_16x16x4(ar[a], br[b], cr[a][b]);
          cr[a][b] = mfma_f32_16x16x4(ai[a], bi[b], cr[a][b]);
          ci[a][b] = mfma_f32_16x16x4(ar[a], bi[b], ci[a][b]);
          ci[a][b] = mfma_f32_16x16x4(-ai[a], br[b], ci[a][b]);
        }
    }
    __syncthreads();
  }
  // store: out[s][f][n][m]
  float2* o = out + ((size_t)s * B + f) * (size_t)N * N;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = n0 + wi + 16 * a + mfma16_row(lane, r);
        const int m = m0 + wj + 16 * b + mfma16_col(lane);
        if (n < N && m < N) o[(size_t)n * N + m] = make_float2(cr[a][b][r] * scale, ci[a][b][r] * scale);
      }
}

// b[f] = scale * sum_s part[s][f] in split order.
__global__ void k_split_reduce(size_t count, int splits, const float2* __restrict__ part,
                               float2* __restrict__ b, float scale) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x) {
    float2 acc = part[i];
    for (int s = 1; s < splits; ++s) acc = c_add(acc, part[(size_t)s * count + i]);
    b[i] = c_scale(acc, scale);
  }
}

// ------------------------------------------------------------------ forward
// grid: (l-tiles, B).  For each 64-row n-tile: P[n][l] = sum_m x[n][m] Ex[l][m]
// (MFMA, K = m in stages of FKT), then acc[l] += sum_n Ey[l][n] P[n][l];
// y[l] = acc / N.
//
// Both operands are staged in LDS in their natural row-major form, one plane
// per real component: X as [n][m] and Ex as [l][m] (row = MFMA row/column
// index, contiguous = contraction index), row stride FLS = FKT + 4 floats so
// that a fragment read (16 consecutive rows x 4 consecutive k) hits 64
// distinct banks.  Global loads are coalesced (16 lanes per 32-element row)
// and the next stage is prefetched into registers while the current one is
// multiplied.  The epilogue's Ey tile reuses the staging memory.
constexpr int FKT = 32;
constexpr int FLS = FKT + 4;

// Global -> registers: rows sr + 16 q (q < 4) of the x and Ex tiles, two
// consecutive contraction indices from sc.  Out-of-range elements are loaded
// from a clamped in-range address and zeroed only when stored (fwd_stash),
// so nothing waits for the loads before the current stage's products.
__device__ __forceinline__ void fwd_fetch(int64_t M, int N, const float2* __restrict__ xf,
                                          const float2* __restrict__ ex, int64_t l0, int n0,
                                          int m0, int sr, int sc, float2 (&px)[8],
                                          float2 (&pe)[8]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int n = n0 + sr + 16 * q;
    const int64_t l = l0 + sr + 16 * q;
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int m = m0 + sc + v;
      px[2 * q + v] = xf[(n < N && m < N) ? (size_t)n * N + m : 0];
      pe[2 * q + v] = ex[(l < M && m < N) ? (size_t)l * N + m : 0];
    }
  }
}

// Registers -> LDS planes (row-major, stride FLS), zeroing out-of-range
// elements of the stage (n0, m0).
__device__ __forceinline__ void fwd_stash(int64_t M, int N, int64_t l0, int n0, int m0,
                                          float* Xr, float* Xi, float* Er, float* Ei, int sr,
                                          int sc, const float2 (&px)[8], const float2 (&pe)[8]) {
  const float2 zero = make_float2(0.f, 0.f);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int n = n0 + sr + 16 * q;
    const int64_t l = l0 + sr + 16 * q;
    const bool m0ok = m0 + sc < N, m1ok = m0 + sc + 1 < N;
    const float2 x0 = (n < N && m0ok) ? px[2 * q] : zero;
    const float2 x1 = (n < N && m1ok) ? px[2 * q + 1] : zero;
    const float2 e0 = (l < M && m0ok) ? pe[2 * q] : zero;
    const float2 e1 = (l < M && m1ok) ? pe[2 * q + 1] : zero;
    const int o = (sr + 16 * q) * FLS + sc;
    *reinterpret_cast<float2*>(Xr + o) = make_float2(x0.x, x1.x);
    *reinterpret_cast<float2*>(Xi + o) = make_float2(x0.y, x1.y);
    *reinterpret_cast<float2*>(Er + o) = make_float2(e0.x, e1.x);
    *reinterpret_cast<float2*>(Ei + o) = make_float2(e0.y, e1.y);
  }
}

__global__ __launch_bounds__(256) void k_forward_f32(int64_t M, int N,
                                                     const float2* __restrict__ ex,
                                                     const float2* __restrict__ ey,
                                                     const float2* __restrict__ x,
                                                     float2* __restrict__ y, float scale) {
  constexpr int PLANE = NT * FLS;            // floats per operand plane
  constexpr int OPS = 4 * PLANE;             // Xr, Xi, Er, Ei
  constexpr int EPS = NT * (NT + 1) * 2;     // Ey tile [64][65] complex, in floats
  constexpr int SH = OPS > EPS ? OPS : EPS;
  __shared__ __attribute__((aligned(16))) float sm[SH];
  __shared__ float2 red[4][2][16];
  float* Xr = sm;
  float* Xi = sm + PLANE;
  float* Er = sm + 2 * PLANE;
  float* Ei = sm + 3 * PLANE;
  float2* Et = reinterpret_cast<float2*>(sm);
  const int f = blockIdx.y;
  const int64_t l0 = (int64_t)blockIdx.x * NT;
  const float2* xf = x + (size_t)f * N * N;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
  // staging map: rows sr + 16 q (q < 4), two consecutive k from sc
  const int sr = tid >> 4, sc = (tid & 15) * 2;
  const float2 zero = make_float2(0.f, 0.f);
  float2 px[8], pe[8];
  float2 yacc[2] = {zero, zero};
  v4f pr[2][2], pi[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) { pr[a][b] = v4f{0, 0, 0, 0}; pi[a][b] = v4f{0, 0, 0, 0}; }
  const int nmt = (N + FKT - 1) / FKT;  // stages per n-tile
  const int stages = ((N + NT - 1) / NT) * nmt;
  fwd_fetch(M, N, xf, ex, l0, 0, 0, sr, sc, px, pe);
  for (int st = 0; st < stages; ++st) {
    const int n0 = (st / nmt) * NT;
    fwd_stash(M, N, l0, n0, (st % nmt) * FKT, Xr, Xi, Er, Ei, sr, sc, px, pe);
    __syncthreads();
    if (st + 1 < stages)
      fwd_fetch(M, N, xf, ex, l0, ((st + 1) / nmt) * NT, ((st + 1) % nmt) * FKT, sr, sc, px, pe);
#pragma unroll
    for (int kk = 0; kk < FKT; kk += 4) {
      const int kr = kk + (lane >> 4), cr = lane & 15;
      float ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        ar[a] = Xr[(wi + 16 * a + cr) * FLS + kr];
        ai[a] = Xi[(wi + 16 * a + cr) * FLS + kr];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        br[b] = Er[(wj + 16 * b + cr) * FLS + kr];
        bi[b] = Ei[(wj + 16 * b + cr) * FLS + kr];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          // x * Ex:  re = xr er - xi ei,  im = xr ei + xi er
          pr[a][b] = mfma_f32_16x16x4(ar[a], br[b], pr[a][b]);
          pr[a][b] = mfma_f32_16x16x4(-ai[a], bi[b], pr[a][b]);
          pi[a][b] = mfma_f32_16x16x4(ar[a], bi[b], pi[a][b]);
          pi[a][b] = mfma_f32_16x16x4(ai[a], br[b], pi[a][b]);
        }
    }
    if (st % nmt == nmt - 1) {
      // Epilogue of the n-tile: acc[l] += sum_n Ey[l][n] P[n][l].
      __syncthreads();  // staging reads done before Et overwrites them
      for (int idx = tid; idx < NT * NT; idx += 256) {
        const int j = idx / NT, i = idx % NT;
        const int64_t l = l0 + j;
        const int n = n0 + i;
        Et[j * (NT + 1) + i] = (l < M && n < N) ? ey[(size_t)l * N + n] : zero;
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int j = wj + 16 * b + mfma16_col(lane);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = wi + 16 * a + mfma16_row(lane, r);
            yacc[b] = c_add(yacc[b], c_mul(Et[j * (NT + 1) + i],
                                           make_float2(pr[a][b][r], pi[a][b][r])));
          }
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) { pr[a][b] = v4f{0, 0, 0, 0}; pi[a][b] = v4f{0, 0, 0, 0}; }
    }
    __syncthreads();  // before the next stage overwrites the staging area
  }
  // Reduce over the row groups of a wave (lanes l, l^16, l^32, l^48) and
  // over the two waves sharing a column range.
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    float2 v = yacc[b];
    v.x += __shfl_xor(v.x, 16, 64);
    v.y += __shfl_xor(v.y, 16, 64);
    v.x += __shfl_xor(v.x, 32, 64);
    v.y += __shfl_xor(v.y, 32, 64);
    yacc[b] = v;
  }
  if (lane < 16) {
    red[w][0][lane] = yacc[0];
    red[w][1][lane] = yacc[1];
  }
  __syncthreads();
  if (tid < NT) {
    const int jb = tid / 32, rem = tid % 32, b = rem / 16, c = rem % 16;
    // waves 0 and 2 hold columns 0..31 (wj = 0), waves 1 and 3 columns 32..63
    const int wa = jb, wb = jb + 2;
    const float2 v = c_add(red[wa][b][c], red[wb][b][c]);
    const int64_t l = l0 + tid;
    if (l < M) y[(size_t)f * M + l] = c_scale(v, scale);
  }
}

// ||y_f||^2 in two fixed-order stages: block (s, f) sums chunk s of frame f
// into part[f][s]; the finisher sums the SUMSQ_PARTS partials of a frame.
constexpr int SUMSQ_PARTS = 64;

__global__ void k_sumsq(int64_t M, int64_t chunk, const float2* __restrict__ y,
                        double* __restrict__ part) {
  __shared__ double red[4];
  const int s = blockIdx.x, f = blockIdx.y;
  const int64_t lo = (int64_t)s * chunk;
  const int64_t hi = lo + chunk < M ? lo + chunk : M;
  double acc[1] = {0.0};
  for (int64_t l = lo + threadIdx.x; l < hi; l += blockDim.x) {
    const float2 v = y[(size_t)f * M + l];
    acc[0] += (double)v.x * v.x + (double)v.y * v.y;
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) part[(size_t)f * SUMSQ_PARTS + s] = acc[0];
}

__global__ void k_sumsq_finish(const double* __restrict__ part, double* __restrict__ yy) {
  const double v = wave_sum_partials(part + (size_t)blockIdx.x * SUMSQ_PARTS, SUMSQ_PARTS, 1);
  if (threadIdx.x == 0) yy[blockIdx.x] = v;
}

// ------------------------------------------------------------------ launchers
hipError_t launch_tables_f32(int64_t M, int N, const double* k, float2* ex, float2* ey,
                             hipStream_t s) {
  const int64_t total = M * N;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_tables_f32<<<(int)blocks, 256, 0, s>>>(M, N, k, ex, ey);
  return hipGetLastError();
}

// Split-K geometry depends only on (M, N), never on the batch size, so a
// frame's adjoint is bitwise the same alone or inside any batch.
int adjoint_splits(int64_t M, int N) {
  const int64_t tiles = (int64_t)cdiv(N, NT) * cdiv(N, NT);
  int64_t sp = (1024 + tiles - 1) / tiles;               // aim for >= 1024 blocks
  const int64_t max_by_k = (M + 8 * KT - 1) / (8 * KT);  // >= 8 stages per split
  if (sp > max_by_k) sp = max_by_k;
  if (sp > 64) sp = 64;
  if (sp < 1) sp = 1;
  return (int)sp;
}

// Frames per launch when split-K partials are used (bounds their memory).
int adjoint_group(int64_t M, int N) {
  const int sp = adjoint_splits(M, N);
  if (sp == 1) return 1 << 30;
  const int64_t tiles = (int64_t)cdiv(N, NT) * cdiv(N, NT);
  int64_t g = (1024 + tiles * sp - 1) / (tiles * sp);
  if (g < 1) g = 1;
  if (g > 8) g = 8;
  return (int)g;
}

hipError_t launch_adjoint_f32(int64_t M, int N, int B, const float2* ex, const float2* ey,
                              const float2* y, float2* b, float2* part, hipStream_t s) {
  const int sp = adjoint_splits(M, N);
  const float inv_n = 1.0f / (float)N;
  if (sp == 1) {
    dim3 grid(cdiv(N, NT), cdiv(N, NT) * B, 1);
    k_adjoint_f32<<<grid, 256, 0, s>>>(M, N, B, 1, ex, ey, y, b, inv_n);
    return hipGetLastError();
  }
  const int G = adjoint_group(M, N);
  for (int f0 = 0; f0 < B; f0 += G) {
    const int g = (B - f0 < G) ? B - f0 : G;
    dim3 grid(cdiv(N, NT), cdiv(N, NT) * g, sp);
    k_adjoint_f32<<<grid, 256, 0, s>>>(M, N, g, sp, ex, ey, y + (size_t)f0 * M, part, 1.0f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t count = (size_t)g * N * N;
    size_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_split_reduce<<<(int)blocks, 256, 0, s>>>(count, sp, part, b + (size_t)f0 * N * N, inv_n);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_forward_f32(int64_t M, int N, int B, const float2* ex, const float2* ey,
                              const float2* x, float2* y, hipStream_t s) {
  dim3 grid((unsigned)((M + NT - 1) / NT), B);
  k_forward_f32<<<grid, 256, 0, s>>>(M, N, ex, ey, x, y, 1.0f / (float)N);
  return hipGetLastError();
}

int sumsq_parts() { return SUMSQ_PARTS; }

hipError_t launch_sumsq(int64_t M, int B, const float2* y, double* part, double* yy,
                        hipStream_t s) {
  const int64_t chunk = (M + SUMSQ_PARTS - 1) / SUMSQ_PARTS;
  k_sumsq<<<dim3(SUMSQ_PARTS, B), 256, 0, s>>>(M, chunk, y, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_sumsq_finish<<<B, 64, 0, s>>>(part, yy);
  return hipGetLastError();
}

}  // namespace recon
