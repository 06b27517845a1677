// Shared device helpers: complex arithmetic on interleaved float pairs,
// wavefront reductions, and the phase of the separable NUDFT phasors.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace recon {

constexpr int WAVE = 64;

__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * b
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 c_mulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
// conj(a) * b
__device__ __forceinline__ float2 c_cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.x, b.y, -a.y * b.x));
}
__device__ __forceinline__ float c_abs2(float2 a) { return fmaf(a.x, a.x, a.y * a.y); }

// The same operations on FP64 complex values (the FP64 iteration).
__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_scale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double c_abs2(double2 a) { return fma(a.x, a.x, a.y * a.y); }

// Real type of an interleaved complex type, construction and fused
// multiply-add for either precision of the iteration.
template <typename C> struct CxTraits;
template <> struct CxTraits<float2> { using R = float; };
template <> struct CxTraits<double2> { using R = double; };
template <typename C> using real_t = typename CxTraits<C>::R;

template <typename C>
__device__ __forceinline__ C cmk(real_t<C> re, real_t<C> im) {
  if constexpr (sizeof(C) == 8) return make_float2(re, im);
  else return make_double2(re, im);
}
__device__ __forceinline__ float rfma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double rfma(double a, double b, double c) { return fma(a, b, c); }
// a * s + c for complex a, c and real s.
template <typename C>
__device__ __forceinline__ C c_axpy(real_t<C> s, C a, C c) {
  return cmk<C>(rfma(s, a.x, c.x), rfma(s, a.y, c.y));
}
// Complex value rounded to FP32 / widened from FP32.
__device__ __forceinline__ float2 to_f32(float2 a) { return a; }
__device__ __forceinline__ float2 to_f32(double2 a) { return make_float2((float)a.x, (float)a.y); }
template <typename C>
__device__ __forceinline__ C from_f32(float2 a) { return cmk<C>(a.x, a.y); }

// Sum over the 64 lanes of a wavefront in a fixed tree order (xor
// butterflies), so the result is identical on every lane and every run.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Deterministic block reduction of NV doubles per thread.  `red` is LDS of
// at least NV * (blockDim.x / 64) doubles.  Result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[i * nw + w] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int k = 0; k < nw; ++k) s += red[i * nw + k];
      v[i] = s;
    }
  }
  __syncthreads();
}

// The two halves of block_sum for an LDS `red` that the kernel fills only
// once: block_partials_store sums each wave's values and lane 0 stores them;
// after the caller's next block barrier, thread 0 adds the stored values with
// block_partials_sum.  The same additions in the same order as block_sum,
// with one barrier (the caller's) instead of three.
template <int NV>
__device__ __forceinline__ void block_partials_store(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[i * nw + w] = v[i];
  }
}

template <int NV>
__device__ __forceinline__ void block_partials_sum(double (&v)[NV], const double* red) {
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += red[i * nw + k];
    v[i] = s;
  }
}

// Fixed-order sum of `n` partials p[0], p[stride], ... by one wavefront;
// every lane of the calling wave receives the same value.
__device__ __forceinline__ double wave_sum_partials(const double* p, int n, int stride) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int i = lane; i < n; i += WAVE) s += p[(size_t)i * stride];
  return wave_sum(s);
}

// Fixed-order sums of interleaved partial series by one wavefront: series q
// of set A is pa[i * NA + q], i < na, and of set B pb[i * NB + q], i < nb.
// The additions and their order are those of wave_sum_partials(pa + q, na,
// NA) and wave_sum_partials(pb + q, nb, NB) for every q; the loads of the
// first K rounds of both sets are issued before any is added, so that the
// sums wait for one memory round trip rather than one per series and round.
template <int NA, int NB, int K = 4>
__device__ __forceinline__ void wave_sum_partials2(const double* pa, int na, double (&oa)[NA],
                                                   const double* pb, int nb,
                                                   double (&ob)[NB > 0 ? NB : 1]) {
  const int lane = threadIdx.x & 63;
  double va[K][NA], vb[K][NB > 0 ? NB : 1];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = lane + k * WAVE;
#pragma unroll
    for (int q = 0; q < NA; ++q) va[k][q] = i < na ? pa[(size_t)i * NA + q] : 0.0;
#pragma unroll
    for (int q = 0; q < NB; ++q) vb[k][q] = i < nb ? pb[(size_t)i * NB + q] : 0.0;
  }
  double sa[NA], sb[NB > 0 ? NB : 1];
#pragma unroll
  for (int q = 0; q < NA; ++q) sa[q] = 0.0;
#pragma unroll
  for (int q = 0; q < NB; ++q) sb[q] = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = lane + k * WAVE;
#pragma unroll
    for (int q = 0; q < NA; ++q)
      if (i < na) sa[q] += va[k][q];
#pragma unroll
    for (int q = 0; q < NB; ++q)
      if (i < nb) sb[q] += vb[k][q];
  }
  for (int i = lane + K * WAVE; i < na; i += WAVE) {
#pragma unroll
    for (int q = 0; q < NA; ++q) sa[q] += pa[(size_t)i * NA + q];
  }
  for (int i = lane + K * WAVE; i < nb; i += WAVE) {
#pragma unroll
    for (int q = 0; q < NB; ++q) sb[q] += pb[(size_t)i * NB + q];
  }
#pragma unroll
  for (int q = 0; q < NA; ++q) oa[q] = wave_sum(sa[q]);
#pragma unroll
  for (int q = 0; q < NB; ++q) ob[q] = wave_sum(sb[q]);
}

// Reduced phase of exp(i 2 pi k j): t = k*j - rint(k*j) in [-1/2, 1/2],
// evaluated in FP64 (the rounding error of k*j is below 2^-53 * |k j|).
__device__ __forceinline__ double turn_frac(double k, double j) {
  double p = k * j;
  return p - rint(p);
}

// exp(i 2 pi t) in FP32 from an FP64 turn fraction.
__device__ __forceinline__ float2 phasor_f32(double t) {
  float s, c;
  sincospif((float)(2.0 * t), &s, &c);
  return make_float2(c, s);
}

__device__ __forceinline__ double2 phasor_f64(double t) {
  double s, c;
  sincospi(2.0 * t, &s, &c);
  return make_double2(c, s);
}

}  // namespace recon
