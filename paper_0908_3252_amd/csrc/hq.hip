// Half-quadratic minimisation (the dual / half-quadratic alternative to the
// conjugate gradient named in Section 5; multiplicative Geman-Reynolds form).
//
// Outer iteration at the current image xbar: the penalty weights
// w = phi'(s)/s of the differences s = |D xbar| (and w0 of the background
// term) are frozen, and linear conjugate gradients decrease the quadratic
// surrogate
//   S(x) = ||y - A x||^2 + lam sum (w/2) |D x|^2 + lam0 sum (w0/2) |x|^2 + const
// from xbar.  An inner step is the conjugate-gradient step of iterate.hip
// (direction + row transforms, column pass, inverse rows + update) with every
// weight taken from xbar: alpha = -Re<g,d> / (2 Re<d,Qd> + lam sum w|Dd|^2 +
// lam0 sum w0|d|^2) is then the exact minimiser of S along d.  This file
// holds the kernels around the inner steps:
//   k_hq_freeze  xbar = x, update partials zeroed (the first direction of
//                the inner problem is -g)
//   k_hq_gnorm   |grad J(x)|^2 of the true criterion, for the statistics
// Every reduction is a per-block FP64 partial summed in a fixed order, as in
// the conjugate-gradient kernels.
#include "kernels.hpp"
#include "stencil.hpp"

namespace recon {

// Weight of the edge between pixels a and b of xbar.
template <int PHI, typename C>
__device__ __forceinline__ real_t<C> edge_w(const C* __restrict__ xb, size_t a, size_t b,
                                            real_t<C> delta) {
  return pen_weight<PHI>(c_abs2(c_sub(xb[b], xb[a])), delta);
}

// (D^T (w(D xbar) . D x))[n][m] at global index i (the operations and order
// of divergence_fw, with the weights taken from xbar).  xv(j): x at index j.
template <int PHI, typename C, typename XF>
__device__ __forceinline__ C div_frozen(XF xv, const C* __restrict__ xb, size_t i, int n, int m,
                                        int N, real_t<C> delta) {
  const C c = xv(i);
  C acc = cmk<C>(0, 0);
  if (n > 0) acc = c_add(acc, c_scale(c_sub(c, xv(i - N)), edge_w<PHI>(xb, i - N, i, delta)));
  if (n + 1 < N) acc = c_sub(acc, c_scale(c_sub(xv(i + N), c), edge_w<PHI>(xb, i, i + N, delta)));
  if (m > 0) acc = c_add(acc, c_scale(c_sub(c, xv(i - 1)), edge_w<PHI>(xb, i - 1, i, delta)));
  if (m + 1 < N) acc = c_sub(acc, c_scale(c_sub(xv(i + 1), c), edge_w<PHI>(xb, i, i + 1, delta)));
  return acc;
}

// xbar = x (freeze the weights); zero the update partials of every frame
// (beta = 0: the first direction of the inner problem is -g).
template <typename C>
__global__ void k_hq_freeze(size_t n_img, const C* __restrict__ x, C* __restrict__ xb,
                            size_t n_p4, double* __restrict__ p4) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_img;
       i += (size_t)gridDim.x * blockDim.x) {
    xb[i] = x[i];
    if (i < n_p4) p4[i] = 0.0;
  }
}

// |g|^2 of the true gradient at x (xbar = x) into the first update partial
// of every block (the others zero): the statistics' gradient norm.
template <int PHI, typename C, bool BG>
__global__ __launch_bounds__(256) void k_hq_gnorm(int N, int ROWS, const C* __restrict__ x,
                                                  const C* __restrict__ r, double* __restrict__ p4,
                                                  const FrameParam* __restrict__ fp) {
  using R = real_t<C>;
  __shared__ double red[1 * 4];
  const int f = blockIdx.y, n0 = blockIdx.x * ROWS;
  const size_t fo = (size_t)f * N * N;
  const R lam = (R)fp[f].lam, delta = (R)fp[f].delta;
  const R lam0 = (R)fp[f].lam0, alpha0 = (R)fp[f].alpha0;
  auto xv = [x](size_t j) { return x[j]; };
  double acc[1] = {0.0};
  const int own = min(ROWS, N - n0);
  for (int i = threadIdx.x; i < own * N; i += 256) {
    const int rr = i / N, m = i - rr * N, n = n0 + rr;
    const size_t idx = fo + (size_t)n * N + m;
    const C div = div_frozen<PHI>(xv, x, idx, n, m, N, delta);
    const C g = grad_frozen<BG>(r[idx], div, x[idx], x[idx], lam, lam0, alpha0);
    acc[0] += (double)g.x * (double)g.x + (double)g.y * (double)g.y;
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) {
    double* o = p4 + ((size_t)f * gridDim.x + blockIdx.x) * 4;
    o[0] = acc[0];
    o[1] = o[2] = o[3] = 0.0;
  }
}

// ------------------------------------------------------------------ launchers
#define RECON_HQ_PHI_SWITCH(PHI_, CALL)               \
  switch (PHI_) {                                     \
    case 0: { constexpr int PP = 0; CALL; } break;    \
    case 1: { constexpr int PP = 1; CALL; } break;    \
    case 2: { constexpr int PP = 2; CALL; } break;    \
    default: return hipErrorInvalidValue;             \
  }

template <typename C>
static hipError_t hq_freeze_any(int N, int B, int nb4, const C* x, C* xb, double* p4,
                                hipStream_t s) {
  const size_t n = (size_t)B * N * N;
  const size_t np4 = (size_t)B * nb4 * 4;
  const size_t work = n > np4 ? n : np4;
  size_t blocks = (work + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (n < np4) return hipErrorInvalidValue;  // the copy loop also zeroes p4
  k_hq_freeze<C><<<(unsigned)blocks, 256, 0, s>>>(n, x, xb, np4, p4);
  return hipGetLastError();
}

template <typename C>
static hipError_t hq_gnorm_any(int phi, int N, int R, int B, const C* x, const C* r, double* p4,
                               const FrameParam* fp, bool bg, hipStream_t s) {
  dim3 grid(cdiv(N, R), B);
  if (bg) {
    RECON_HQ_PHI_SWITCH(phi, (k_hq_gnorm<PP, C, true><<<grid, 256, 0, s>>>(N, R, x, r, p4, fp)));
  } else {
    RECON_HQ_PHI_SWITCH(phi, (k_hq_gnorm<PP, C, false><<<grid, 256, 0, s>>>(N, R, x, r, p4, fp)));
  }
  return hipGetLastError();
}

hipError_t launch_hq_freeze(int N, int B, int nb4, const float2* x, float2* xb, double* p4,
                            hipStream_t s) {
  return hq_freeze_any(N, B, nb4, x, xb, p4, s);
}
hipError_t launch_hq_freeze(int N, int B, int nb4, const double2* x, double2* xb, double* p4,
                            hipStream_t s) {
  return hq_freeze_any(N, B, nb4, x, xb, p4, s);
}
hipError_t launch_hq_gnorm(int phi, int N, int R, int B, const float2* x, const float2* r,
                           double* p4, const FrameParam* fp, bool bg, hipStream_t s) {
  return hq_gnorm_any(phi, N, R, B, x, r, p4, fp, bg, s);
}
hipError_t launch_hq_gnorm(int phi, int N, int R, int B, const double2* x, const double2* r,
                           double* p4, const FrameParam* fp, bool bg, hipStream_t s) {
  return hq_gnorm_any(phi, N, R, B, x, r, p4, fp, bg, s);
}

}  // namespace recon
