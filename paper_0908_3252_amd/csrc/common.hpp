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

// Fixed-order sum of `n` partials p[0], p[stride], ... by one wavefront;
// every lane of the calling wave receives the same value.
__device__ __forceinline__ double wave_sum_partials(const double* p, int n, int stride) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int i = lane; i < n; i += WAVE) s += p[(size_t)i * stride];
  return wave_sum(s);
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
