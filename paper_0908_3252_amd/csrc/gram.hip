// Trajectory-only Gram kernel (Section 3.4, Eq. DG; Appendix A.1,
// Eq. AnnMatG) accumulated in FP64 on the matrix cores, and its circulant
// spectrum.
//
// Lag kernel of Q = A^H A (row n <-> ky, column m <-> kx):
//   h[a][b] = (1/N^2) sum_l exp(-i 2 pi (ky_l a + kx_l b)) = G[-b][-a]
// With Y[l][a] = exp(-i 2 pi ky_l a) and X[l][b] = exp(-i 2 pi kx_l b)
// for a, b in [0, N), four real products over the samples
//   RR = sum Yr Xr, II = sum Yi Xi, RI = sum Yr Xi, IR = sum Yi Xr
// give the whole lag range through the conjugate symmetry of h:
//   h[a][ b] = (RR - II) + i (RI + IR)      (Y X)
//   h[a][-b] = (RR + II) + i (IR - RI)      (Y conj X)
//   h[-a][-b] = conj h[a][b],  h[-a][b] = conj h[a][-b].
// The phasors are generated on the fly in FP64 from the exact reduced phase
// (no tables), staged in LDS, and contracted with 16x16x4 FP64 MFMA.
#include "common.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace recon {

constexpr int GT = 64;        // lag tile (a and b) per block
constexpr int GK = 16;        // samples per LDS stage
constexpr int GLD = GT + 16;  // padded LDS row (doubles)

__global__ __launch_bounds__(256) void k_gram_f64(int64_t M, int N, const double* __restrict__ k,
                                                  double* __restrict__ part, int splits) {
  __shared__ double Yr[GK][GLD], Yi[GK][GLD], Xr[GK][GLD], Xi[GK][GLD];
  const int a0 = blockIdx.x * GT, b0 = blockIdx.y * GT, s = blockIdx.z;
  const int64_t per = ((M + splits - 1) / splits + GK - 1) / GK * GK;
  const int64_t l_begin = (int64_t)s * per;
  const int64_t l_end = (l_begin + per < M) ? l_begin + per : M;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
  v4d acc[4][2][2];  // [RR, II, RI, IR][a-block][b-block]
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[p][a][b] = v4d{0, 0, 0, 0};

  const int lr = tid >> 4, lc = (tid & 15) * 4;  // 16 samples x 64 lags
  for (int64_t l0 = l_begin; l0 < l_end; l0 += GK) {
    const int64_t l = l0 + lr;
    const bool lv = l < l_end;
    const double kx = lv ? k[2 * l + 0] : 0.0, ky = lv ? k[2 * l + 1] : 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int ia = a0 + lc + c, ib = b0 + lc + c;
      double2 yv = make_double2(0.0, 0.0), xv = make_double2(0.0, 0.0);
      if (lv && ia < N) yv = phasor_f64(-turn_frac(ky, (double)ia));
      if (lv && ib < N) xv = phasor_f64(-turn_frac(kx, (double)ib));
      Yr[lr][lc + c] = yv.x;
      Yi[lr][lc + c] = yv.y;
      Xr[lr][lc + c] = xv.x;
      Xi[lr][lc + c] = xv.y;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const int kr = kk + (lane >> 4), cc = lane & 15;
      double yr[2], yi[2], xr[2], xi[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        yr[a] = Yr[kr][wi + 16 * a + cc];
        yi[a] = Yi[kr][wi + 16 * a + cc];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        xr[b] = Xr[kr][wj + 16 * b + cc];
        xi[b] = Xi[kr][wj + 16 * b + cc];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc[0][a][b] = mfma_f64_16x16x4(yr[a], xr[b], acc[0][a][b]);
          acc[1][a][b] = mfma_f64_16x16x4(yi[a], xi[b], acc[1][a][b]);
          acc[2][a][b] = mfma_f64_16x16x4(yr[a], xi[b], acc[2][a][b]);
          acc[3][a][b] = mfma_f64_16x16x4(yi[a], xr[b], acc[3][a][b]);
        }
    }
    __syncthreads();
  }
  const size_t plane = (size_t)N * N;
  double* o = part + (size_t)s * 4 * plane;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ia = a0 + wi + 16 * a + mfma16_row_f64(lane, r);
          const int ib = b0 + wj + 16 * b + mfma16_col(lane);
          if (ia < N && ib < N) o[p * plane + (size_t)ia * N + ib] = acc[p][a][b][r];
        }
}

// h at lag (a, b), |a|, |b| < N, from the reduced products (FP64).
__device__ __forceinline__ double2 lag_value(int a, int b, int N, const double* __restrict__ part,
                                             int splits, double inv) {
  const int aa = a < 0 ? -a : a, bb = b < 0 ? -b : b;
  const size_t plane = (size_t)N * N, idx = (size_t)aa * N + bb;
  double rr = 0.0, ii = 0.0, ri = 0.0, ir = 0.0;
  for (int s = 0; s < splits; ++s) {
    const double* p = part + (size_t)s * 4 * plane;
    rr += p[idx];
    ii += p[plane + idx];
    ri += p[2 * plane + idx];
    ir += p[3 * plane + idx];
  }
  // (a >= 0, b >= 0): Y X ; (a >= 0, b < 0): Y conj X ; negative a: conjugates.
  double re, im;
  if ((a >= 0 && b >= 0) || (a <= 0 && b <= 0)) {
    re = rr - ii;
    im = ri + ir;
    if (a < 0 || (a == 0 && b < 0)) im = -im;  // h[-a][-b] = conj h[a][b]
  } else {
    re = rr + ii;
    im = ir - ri;
    if (a < 0) im = -im;  // h[-a][b] = conj h[a][-b]
  }
  return make_double2(re * inv, im * inv);
}

__global__ void k_gram_assemble(int N, int L, const double* __restrict__ part, int splits,
                                double* __restrict__ lag_out, double2* __restrict__ emb) {
  const double inv = 1.0 / ((double)N * (double)N);
  const int total = L * L;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int p = i / L, q = i - p * L;
    const int a = (p < N) ? p : ((p > L - N) ? p - L : INT32_MAX);
    const int b = (q < N) ? q : ((q > L - N) ? q - L : INT32_MAX);
    double2 v = make_double2(0.0, 0.0);
    if (a != INT32_MAX && b != INT32_MAX) {
      const double2 h = lag_value(a, b, N, part, splits, inv);
      v = h;
      if (lag_out) {
        const size_t o = ((size_t)(a + N - 1) * (2 * N - 1) + (b + N - 1)) * 2;
        lag_out[o] = h.x;
        lag_out[o + 1] = h.y;
      }
    }
    emb[i] = v;
  }
}

// ------------------------------------------------------------------ launchers
int gram_splits(int64_t M, int N) {
  const int64_t tiles = (int64_t)cdiv(N, GT) * cdiv(N, GT);
  int64_t sp = (512 + tiles - 1) / tiles;
  const int64_t max_by_k = (M + 8 * GK - 1) / (8 * GK);
  if (sp > max_by_k) sp = max_by_k;
  if (sp > 64) sp = 64;
  if (sp < 1) sp = 1;
  return (int)sp;
}

hipError_t launch_gram_f64(int64_t M, int N, const double* k, double* part, int splits,
                           hipStream_t s) {
  dim3 grid(cdiv(N, GT), cdiv(N, GT), splits);
  k_gram_f64<<<grid, 256, 0, s>>>(M, N, k, part, splits);
  return hipGetLastError();
}

hipError_t launch_gram_assemble(int N, int L, const double* part, int splits, double* lag_out,
                                double2* emb, hipStream_t s) {
  int blocks = cdiv(L * L, 256);
  if (blocks > 65536) blocks = 65536;
  k_gram_assemble<<<blocks, 256, 0, s>>>(N, L, part, splits, lag_out, emb);
  return hipGetLastError();
}

}  // namespace recon
