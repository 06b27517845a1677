// Split-precision NUDFT contractions on the matrix cores (BF16 x3, FP16 x3).
//
// Every operand value v is carried as v = hi + lo with hi = round(v) and
// lo = round(v - hi) in bf16 (8-bit significand, pair ~16 bits) or fp16
// (11-bit significand, pair ~22 bits), and each real product as
//   a b ~= a_hi b_hi + a_hi b_lo + a_lo b_hi        (lo * lo dropped)
// with FP32 accumulation in 16x16x32 MFMA.  The trajectory phasors are split
// once per plan (from FP64 values) into planes of hi/lo real/imaginary parts;
// the per-frame operand (the data y for the adjoint, the image x for the
// forward model) is split on the fly after a per-frame power-of-two scaling
// that keeps the fp16 parts in range.
//
//   adjoint  b[n][m] = (1/N) sum_l conj(Ey[l][n]) (y_l conj(Ex[l][m]))
//   forward  y_l = (1/N) sum_n Ey[l][n] sum_m x[n][m] Ex[l][m]
// (Section 2 Eq. ModDirect and Appendix A.2 Eq. AnnMatGD.)
#include "common.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace recon {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int PREC>
struct Split;
template <>
struct Split<RECON_PREC_BF16X3> {
  using T = __bf16;
  using V = bf16x8;
  static __device__ __forceinline__ v4f mfma(V a, V b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Split<RECON_PREC_FP16X3> {
  using T = _Float16;
  using V = f16x8;
  static __device__ __forceinline__ v4f mfma(V a, V b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

template <int PREC>
__device__ __forceinline__ unsigned short bits(typename Split<PREC>::T v) {
  return __builtin_bit_cast(unsigned short, v);
}

// hi/lo parts of x (FP32 or FP64 source).
template <int PREC, class F>
__device__ __forceinline__ void split2(F x, unsigned short& hi, unsigned short& lo) {
  using T = typename Split<PREC>::T;
  const T h = (T)x;
  const T l = (T)(x - (F)h);
  hi = bits<PREC>(h);
  lo = bits<PREC>(l);
}

// Eight 16-bit values packed for one 16-byte LDS store.
__device__ __forceinline__ u32x4 pack8(const unsigned short (&h)[8]) {
  return (u32x4){(unsigned)h[0] | ((unsigned)h[1] << 16), (unsigned)h[2] | ((unsigned)h[3] << 16),
                 (unsigned)h[4] | ((unsigned)h[5] << 16), (unsigned)h[6] | ((unsigned)h[7] << 16)};
}

template <class V>
__device__ __forceinline__ V vneg(V a) {
  u32x4 u = __builtin_bit_cast(u32x4, a);
  u ^= (u32x4){0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  return __builtin_bit_cast(V, u);
}

constexpr int ST = 64;        // output tile
constexpr int SK = 32;        // k per stage (one MFMA k-step)
constexpr int SLD = SK + 8;   // LDS row stride in 16-bit elements (80 bytes)

// ------------------------------------------------------------------ tables
// at[p][n][l] (l < Mp, zero padded): p = 0/1 hi/lo of Re Ey, 2/3 hi/lo of
// -Im Ey  (the adjoint's conj(Ey)^T);
// xs[p][l][m] (m < Np, zero padded): p = 0/1 hi/lo of Re Ex, 2/3 of Im Ex.
template <int PREC>
__global__ void k_tables_split(int64_t M, int N, int64_t Mp, int Np, const double* __restrict__ k,
                               unsigned short* __restrict__ at, unsigned short* __restrict__ xs) {
  const int64_t total = Mp * (int64_t)Np;
  const size_t pa = (size_t)N * Mp, px = (size_t)M * Np;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = i / Np;
    const int j = (int)(i - l * Np);
    const bool valid = l < M && j < N;
    double2 ey = make_double2(0.0, 0.0), ex = make_double2(0.0, 0.0);
    if (valid) {
      ey = phasor_f64(turn_frac(k[2 * l + 1], (double)j));
      ex = phasor_f64(turn_frac(k[2 * l + 0], (double)j));
    }
    unsigned short h, lo;
    if (j < N) {
      const size_t o = (size_t)j * Mp + l;
      split2<PREC>(ey.x, h, lo);
      at[o] = h;
      at[pa + o] = lo;
      split2<PREC>(-ey.y, h, lo);
      at[2 * pa + o] = h;
      at[3 * pa + o] = lo;
    }
    if (l < M) {
      const size_t o = (size_t)l * Np + j;
      split2<PREC>(ex.x, h, lo);
      xs[o] = h;
      xs[px + o] = lo;
      split2<PREC>(ex.y, h, lo);
      xs[2 * px + o] = h;
      xs[3 * px + o] = lo;
    }
  }
}

// Per-frame power-of-two scale s = 2^-ceil(log2(max |component|)) (1 if zero).
__global__ void k_frame_scale(int64_t count, const float2* __restrict__ v, float* __restrict__ sc) {
  __shared__ float red[4];
  const int f = blockIdx.x;
  float m = 0.f;
  for (int64_t i = threadIdx.x; i < count; i += blockDim.x) {
    const float2 a = v[(size_t)f * count + i];
    m = fmaxf(m, fmaxf(fabsf(a.x), fabsf(a.y)));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, red[w]);
    m = fmaxf(m, red[0]);
    sc[f] = (m > 0.f && isfinite(m)) ? exp2f(-ceilf(log2f(m))) : 1.f;
  }
}

// One 16x16 complex block product with split operands.
// A = (ar_h, ar_l, ai_h, ai_l), B = (br_h, br_l, bi_h, bi_l):
// cr += Ar Br - Ai Bi ; ci += Ar Bi + Ai Br.
template <int PREC>
__device__ __forceinline__ void cplx_split_mma(const typename Split<PREC>::V (&A)[4],
                                               const typename Split<PREC>::V (&nAi)[2],
                                               const typename Split<PREC>::V (&Bv)[4], v4f& cr,
                                               v4f& ci) {
  using S = Split<PREC>;
  cr = S::mfma(A[0], Bv[0], cr);
  cr = S::mfma(A[0], Bv[1], cr);
  cr = S::mfma(A[1], Bv[0], cr);
  cr = S::mfma(nAi[0], Bv[2], cr);
  cr = S::mfma(nAi[0], Bv[3], cr);
  cr = S::mfma(nAi[1], Bv[2], cr);
  ci = S::mfma(A[0], Bv[2], ci);
  ci = S::mfma(A[0], Bv[3], ci);
  ci = S::mfma(A[1], Bv[2], ci);
  ci = S::mfma(A[2], Bv[0], ci);
  ci = S::mfma(A[2], Bv[1], ci);
  ci = S::mfma(A[3], Bv[0], ci);
}

// ------------------------------------------------------------------ adjoint
// grid: (n-tiles, m-tiles * frames, splits).  Samples [l_begin, l_end) of
// split s; the output is unnormalised when splits > 1 (partials).
template <int PREC>
__global__ __launch_bounds__(256) void k_adjoint_split(
    int64_t M, int64_t Mp, int N, int B, int splits, const unsigned short* __restrict__ at,
    const float2* __restrict__ ex, const float2* __restrict__ y, const float* __restrict__ sc,
    float2* __restrict__ out) {
  using V = typename Split<PREC>::V;
  __shared__ __attribute__((aligned(16))) unsigned short As[4][ST][SLD];
  __shared__ __attribute__((aligned(16))) unsigned short Zs[4][ST][SLD];
  const int mt = (N + ST - 1) / ST;
  const int n0 = blockIdx.x * ST;
  const int f = blockIdx.y / mt;
  const int m0 = (blockIdx.y % mt) * ST;
  const int s = blockIdx.z;
  const int64_t per = ((M + splits - 1) / splits + SK - 1) / SK * SK;
  const int64_t l_begin = (int64_t)s * per;
  const int64_t l_end = (l_begin + per < M) ? l_begin + per : M;
  const float2* yf = y + (size_t)f * M;
  const float ys = sc[f];
  const size_t pa = (size_t)N * Mp;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
  v4f cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) { cr[a][b] = v4f{0, 0, 0, 0}; ci[a][b] = v4f{0, 0, 0, 0}; }
  // A staging: thread -> (plane, row), 64 bytes; Z staging: thread -> (m, 8 samples)
  const int ap = tid >> 6, arow = tid & 63;
  const int zm = tid & 63, zg = tid >> 6;
  for (int64_t l0 = l_begin; l0 < l_end; l0 += SK) {
    {
      u32x4* dst = reinterpret_cast<u32x4*>(&As[ap][arow][0]);
      const int n = n0 + arow;
      if (n < N) {
        const u32x4* src = reinterpret_cast<const u32x4*>(at + ap * pa + (size_t)n * Mp + l0);
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = src[q];  // padded table: always in bounds
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = (u32x4){0u, 0u, 0u, 0u};
      }
    }
    {
      unsigned short zr_h[8], zr_l[8], zi_h[8], zi_l[8];
      const int m = m0 + zm;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int64_t l = l0 + 8 * zg + v;
        float2 z = make_float2(0.f, 0.f);
        if (l < l_end && m < N) {
          const float2 yv = c_scale(yf[l], ys);
          z = c_mulc(yv, ex[(size_t)l * N + m]);  // y_l conj(Ex[l][m])
        }
        split2<PREC>(z.x, zr_h[v], zr_l[v]);
        split2<PREC>(z.y, zi_h[v], zi_l[v]);
      }
      *reinterpret_cast<u32x4*>(&Zs[0][zm][8 * zg]) = pack8(zr_h);
      *reinterpret_cast<u32x4*>(&Zs[1][zm][8 * zg]) = pack8(zr_l);
      *reinterpret_cast<u32x4*>(&Zs[2][zm][8 * zg]) = pack8(zi_h);
      *reinterpret_cast<u32x4*>(&Zs[3][zm][8 * zg]) = pack8(zi_l);
    }
    __syncthreads();
    const int r16 = lane & 15, g = lane >> 4;
    V Bf[2][4];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int p = 0; p < 4; ++p)
        Bf[b][p] = *reinterpret_cast<const V*>(&Zs[p][wj + 16 * b + r16][8 * g]);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      V Af[4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
        Af[p] = *reinterpret_cast<const V*>(&As[p][wi + 16 * a + r16][8 * g]);
      const V nAi[2] = {vneg(Af[2]), vneg(Af[3])};
#pragma unroll
      for (int b = 0; b < 2; ++b) cplx_split_mma<PREC>(Af, nAi, Bf[b], cr[a][b], ci[a][b]);
    }
    __syncthreads();
  }
  const float scale = (splits == 1) ? 1.0f / ((float)N * ys) : 1.0f / ys;
  float2* o = out + ((size_t)s * B + f) * (size_t)N * N;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = n0 + wi + 16 * a + mfma16_row(lane, r);
        const int m = m0 + wj + 16 * b + mfma16_col(lane);
        if (n < N && m < N)
          o[(size_t)n * N + m] = make_float2(cr[a][b][r] * scale, ci[a][b][r] * scale);
      }
}

__global__ void k_split_reduce_f32(size_t count, int splits, const float2* __restrict__ part,
                                   float2* __restrict__ b, float scale) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x) {
    float2 acc = part[i];
    for (int s = 1; s < splits; ++s) acc = c_add(acc, part[(size_t)s * count + i]);
    b[i] = c_scale(acc, scale);
  }
}

// ------------------------------------------------------------------ forward
// grid: (l-tiles, frames).  For each n-tile, P[n][l] = sum_m x[n][m] Ex[l][m]
// with split MFMA, then acc[l] += sum_n Ey[l][n] P[n][l] (FP32).
template <int PREC>
__global__ __launch_bounds__(256) void k_forward_split(int64_t M, int N, int Np,
                                                       const unsigned short* __restrict__ xs,
                                                       const float2* __restrict__ ey,
                                                       const float2* __restrict__ x,
                                                       const float* __restrict__ sc,
                                                       float2* __restrict__ y) {
  using V = typename Split<PREC>::V;
  constexpr int OPS = 2 * 4 * ST * SLD * 2;         // bytes of As + Bs
  constexpr int EPI = ST * (ST + 1) * 8;             // bytes of the Ey tile
  constexpr int SHB = OPS > EPI ? OPS : EPI;
  __shared__ __attribute__((aligned(16))) unsigned char smem[SHB];
  __shared__ float2 red[4][2][16];
  auto As = reinterpret_cast<unsigned short(*)[ST][SLD]>(smem);
  auto Bs = reinterpret_cast<unsigned short(*)[ST][SLD]>(smem + 4 * ST * SLD * 2);
  auto Et = reinterpret_cast<float2(*)[ST + 1]>(smem);
  const int f = blockIdx.y;
  const int64_t l0 = (int64_t)blockIdx.x * ST;
  const float2* xf = x + (size_t)f * N * N;
  const float xsc = sc[f];
  const size_t px = (size_t)M * Np;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
  const int r16 = lane & 15, g = lane >> 4;
  float2 yacc[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
  const int xr = tid >> 2, xg = tid & 3;     // x staging: row, 8-column group
  const int bp = tid >> 6, brow = tid & 63;  // Ex staging: plane, row

  for (int n0 = 0; n0 < N; n0 += ST) {
    v4f pr[2][2], pi[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) { pr[a][b] = v4f{0, 0, 0, 0}; pi[a][b] = v4f{0, 0, 0, 0}; }
    for (int m0 = 0; m0 < N; m0 += SK) {
      {
        const int n = n0 + xr;
        unsigned short h[4][8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const int m = m0 + 8 * xg + v;
          const float2 xv = (n < N && m < N) ? c_scale(xf[(size_t)n * N + m], xsc)
                                             : make_float2(0.f, 0.f);
          split2<PREC>(xv.x, h[0][v], h[1][v]);
          split2<PREC>(xv.y, h[2][v], h[3][v]);
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) *reinterpret_cast<u32x4*>(&As[p][xr][8 * xg]) = pack8(h[p]);
      }
      {
        u32x4* dst = reinterpret_cast<u32x4*>(&Bs[bp][brow][0]);
        const int64_t l = l0 + brow;
        if (l < M) {
          const u32x4* src = reinterpret_cast<const u32x4*>(xs + bp * px + (size_t)l * Np + m0);
#pragma unroll
          for (int q = 0; q < 4; ++q) dst[q] = src[q];  // Np is a multiple of 32
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) dst[q] = (u32x4){0u, 0u, 0u, 0u};
        }
      }
      __syncthreads();
      V Bf[2][4];
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int p = 0; p < 4; ++p)
          Bf[b][p] = *reinterpret_cast<const V*>(&Bs[p][wj + 16 * b + r16][8 * g]);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        V Af[4];
#pragma unroll
        for (int p = 0; p < 4; ++p)
          Af[p] = *reinterpret_cast<const V*>(&As[p][wi + 16 * a + r16][8 * g]);
        const V nAi[2] = {vneg(Af[2]), vneg(Af[3])};
#pragma unroll
        for (int b = 0; b < 2; ++b) cplx_split_mma<PREC>(Af, nAi, Bf[b], pr[a][b], pi[a][b]);
      }
      __syncthreads();
    }
    for (int idx = tid; idx < ST * ST; idx += 256) {
      const int j = idx / ST, i = idx % ST;
      const int64_t l = l0 + j;
      const int n = n0 + i;
      Et[j][i] = (l < M && n < N) ? ey[(size_t)l * N + n] : make_float2(0.f, 0.f);
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
          yacc[b] = c_add(yacc[b], c_mul(Et[j][i], make_float2(pr[a][b][r], pi[a][b][r])));
        }
    }
    __syncthreads();
  }
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
  if (tid < ST) {
    const int jb = tid / 32, rem = tid % 32, b = rem / 16, c = rem % 16;
    const float2 v = c_add(red[jb][b][c], red[jb + 2][b][c]);
    const int64_t l = l0 + tid;
    if (l < M) y[(size_t)f * M + l] = c_scale(v, 1.0f / ((float)N * xsc));
  }
}

// ------------------------------------------------------------------ launchers
int64_t split_pad_M(int64_t M) { return (M + SK - 1) / SK * SK; }
int split_pad_N(int N) { return (N + SK - 1) / SK * SK; }

hipError_t launch_tables_split(int prec, int64_t M, int N, const double* k, void* at, void* xs,
                               hipStream_t s) {
  const int64_t Mp = split_pad_M(M);
  const int Np = split_pad_N(N);
  int64_t blocks = (Mp * Np + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  auto* a = static_cast<unsigned short*>(at);
  auto* x = static_cast<unsigned short*>(xs);
  if (prec == RECON_PREC_BF16X3)
    k_tables_split<RECON_PREC_BF16X3><<<(int)blocks, 256, 0, s>>>(M, N, Mp, Np, k, a, x);
  else if (prec == RECON_PREC_FP16X3)
    k_tables_split<RECON_PREC_FP16X3><<<(int)blocks, 256, 0, s>>>(M, N, Mp, Np, k, a, x);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_adjoint_split(int prec, int64_t M, int N, int B, const void* at, const float2* ex,
                                const float2* y, float* sc, float2* b, float2* part,
                                hipStream_t s) {
  const int64_t Mp = split_pad_M(M);
  k_frame_scale<<<B, 256, 0, s>>>(M, y, sc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int sp = adjoint_splits(M, N);
  const auto* a = static_cast<const unsigned short*>(at);
  auto run = [&](int g, const float2* yy, const float* scc, float2* o, int splits) {
    dim3 grid(cdiv(N, ST), cdiv(N, ST) * g, splits);
    if (prec == RECON_PREC_BF16X3)
      k_adjoint_split<RECON_PREC_BF16X3><<<grid, 256, 0, s>>>(M, Mp, N, g, splits, a, ex, yy, scc, o);
    else
      k_adjoint_split<RECON_PREC_FP16X3><<<grid, 256, 0, s>>>(M, Mp, N, g, splits, a, ex, yy, scc, o);
    return hipGetLastError();
  };
  if (sp == 1) return run(B, y, sc, b, 1);
  const int G = adjoint_group(M, N);
  for (int f0 = 0; f0 < B; f0 += G) {
    const int g = (B - f0 < G) ? B - f0 : G;
    e = run(g, y + (size_t)f0 * M, sc + f0, part, sp);
    if (e != hipSuccess) return e;
    const size_t count = (size_t)g * N * N;
    size_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_split_reduce_f32<<<(int)blocks, 256, 0, s>>>(count, sp, part, b + (size_t)f0 * N * N,
                                                  1.0f / (float)N);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_forward_split(int prec, int64_t M, int N, int B, const void* xs, const float2* ey,
                                const float2* x, float* sc, float2* y, hipStream_t s) {
  k_frame_scale<<<B, 256, 0, s>>>((int64_t)N * N, x, sc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int Np = split_pad_N(N);
  dim3 grid((unsigned)((M + ST - 1) / ST), B);
  const auto* t = static_cast<const unsigned short*>(xs);
  if (prec == RECON_PREC_BF16X3)
    k_forward_split<RECON_PREC_BF16X3><<<grid, 256, 0, s>>>(M, N, Np, t, ey, x, sc, y);
  else
    k_forward_split<RECON_PREC_FP16X3><<<grid, 256, 0, s>>>(M, N, Np, t, ey, x, sc, y);
  return hipGetLastError();
}

}  // namespace recon
