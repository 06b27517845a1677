// Half-quadratic minimisation (the dual / half-quadratic alternative to the
// conjugate gradient named in Section 5; multiplicative Geman-Reynolds form).
//
// Outer iteration at the current image xbar: the penalty weights
// w = phi'(s)/s of the differences s = |D xbar| (and w0 of the background
// term) are frozen, and linear conjugate gradients decrease the quadratic
// surrogate
//   S(x) = ||y - A x||^2 + lam sum (w/2) |D x|^2 + lam0 sum (w0/2) |x|^2 + const
// from xbar.  One inner step:
//   k_hq_dir     g = 2 r + lam D^T(w . D x) + lam0 w0 x, beta (PR+, restart),
//                d = -g + beta d_old; g and d stored; partials Re<g, d>,
//                sum w0 |d|^2
//   k_hq_curv    partials sum w |D d|^2
//   Gram apply   Q d (row FFTs, column pass with the <d, Qd> partials,
//                row inverse: the kernels of toeplitz.hip)
//   k_hq_update  alpha = -Re<g,d> / (2 Re<d,Qd> + lam sum w|Dd|^2 + lam0 sum w0|d|^2),
//                x += alpha d, r += alpha Q d, g_new with the frozen weights,
//                partials for beta
// The weights are recomputed from xbar where needed (one image instead of
// two weight planes); neighbouring pixels are read through the caches.
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

// Surrogate gradient 2 r + lam div + lam0 w0(|xbar|) x (the form of grad_full).
template <bool BG, typename C>
__device__ __forceinline__ C grad_frozen(C r, C div, C x, C xbv, real_t<C> lam, real_t<C> lam0,
                                         real_t<C> alpha0) {
  C g = cmk<C>(rfma(lam, div.x, 2 * r.x), rfma(lam, div.y, 2 * r.y));
  if constexpr (BG) {
    if (lam0 != 0) {
      const real_t<C> w = lam0 * pen_weight<1>(c_abs2(xbv), alpha0);
      g = cmk<C>(rfma(w, x.x, g.x), rfma(w, x.y, g.y));
    }
  }
  return g;
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

template <int PHI, typename C, bool BG>
__global__ __launch_bounds__(256) void k_hq_dir(int N, int ROWS, const C* __restrict__ r,
                                                const C* __restrict__ d_old, C* __restrict__ d_new,
                                                C* __restrict__ g_out, const C* __restrict__ x,
                                                const C* __restrict__ xb,
                                                const double* __restrict__ p4, int nb4,
                                                double* __restrict__ p1,
                                                const FrameParam* __restrict__ fp) {
  using R = real_t<C>;
  __shared__ double red[2 * 4];
  __shared__ R sbeta;
  const int f = blockIdx.y, n0 = blockIdx.x * ROWS;
  const size_t fo = (size_t)f * N * N;
  // beta (PR+ with restart) from the update partials, as k_dir_rowfft forms it
  if (threadIdx.x < 64) {
    const double* pf = p4 + (size_t)f * nb4 * 4;
    const double gg = wave_sum_partials(pf + 0, nb4, 4);
    const double ggo = wave_sum_partials(pf + 1, nb4, 4);
    const double gdo = wave_sum_partials(pf + 2, nb4, 4);
    const double gg_old = wave_sum_partials(pf + 3, nb4, 4);
    double beta = 0.0;
    if (gg_old > 0.0) beta = fmax(0.0, (gg - ggo) / gg_old);
    if (-gg + beta * gdo >= 0.0) beta = 0.0;
    if (threadIdx.x == 0) sbeta = (R)beta;
  }
  __syncthreads();
  const R bf = sbeta;
  const R lam = (R)fp[f].lam, delta = (R)fp[f].delta;
  const R lam0 = (R)fp[f].lam0, alpha0 = (R)fp[f].alpha0;
  auto xv = [x](size_t j) { return x[j]; };
  double acc[2] = {0.0, 0.0};
  const int own = min(ROWS, N - n0);
  for (int i = threadIdx.x; i < own * N; i += 256) {
    const int rr = i / N, m = i - rr * N, n = n0 + rr;
    const size_t idx = fo + (size_t)n * N + m;
    const C div = div_frozen<PHI>(xv, xb, idx, n, m, N, delta);
    const C xbv = xb[idx];
    const C g = grad_frozen<BG>(r[idx], div, x[idx], xbv, lam, lam0, alpha0);
    const C dv = d_old[idx];
    const C dn = cmk<C>(rfma(bf, dv.x, -g.x), rfma(bf, dv.y, -g.y));
    d_new[idx] = dn;
    g_out[idx] = g;
    acc[0] += (double)g.x * (double)dn.x + (double)g.y * (double)dn.y;
    if constexpr (BG) acc[1] += (double)bg_weight(xbv, lam0, alpha0) * (double)c_abs2(dn);
  }
  block_sum<2>(acc, red);
  if (threadIdx.x == 0) {
    double* o = p1 + ((size_t)f * gridDim.x + blockIdx.x) * 3;
    o[0] = acc[0];
    o[2] = acc[1];
  }
}

// sum w(D xbar) |D d|^2 over the forward edges of the block's pixels.
template <int PHI, typename C>
__global__ __launch_bounds__(256) void k_hq_curv(int N, int ROWS, const C* __restrict__ d,
                                                 const C* __restrict__ xb, double* __restrict__ p1,
                                                 const FrameParam* __restrict__ fp) {
  using R = real_t<C>;
  __shared__ double red[1 * 4];
  const int f = blockIdx.y, n0 = blockIdx.x * ROWS;
  const size_t fo = (size_t)f * N * N;
  const R delta = (R)fp[f].delta;
  double acc[1] = {0.0};
  const int own = min(ROWS, N - n0);
  for (int i = threadIdx.x; i < own * N; i += 256) {
    const int rr = i / N, m = i - rr * N, n = n0 + rr;
    const size_t idx = fo + (size_t)n * N + m;
    const C e0 = d[idx];
    if (n + 1 < N) {
      const C te = c_sub(d[idx + N], e0);
      acc[0] += (double)edge_w<PHI>(xb, idx, idx + N, delta) * (double)c_abs2(te);
    }
    if (m + 1 < N) {
      const C te = c_sub(d[idx + 1], e0);
      acc[0] += (double)edge_w<PHI>(xb, idx, idx + 1, delta) * (double)c_abs2(te);
    }
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) p1[((size_t)f * gridDim.x + blockIdx.x) * 3 + 1] = acc[0];
}

template <int PHI, typename C, bool BG>
__global__ __launch_bounds__(256) void k_hq_update(
    int N, int ROWS, const C* __restrict__ x_old, C* __restrict__ x_new, const C* __restrict__ d,
    C* __restrict__ r, const C* __restrict__ qd, const C* __restrict__ g_old,
    const C* __restrict__ xb, const double* __restrict__ p1, int nb1,
    const double* __restrict__ p3, int nb3, double* __restrict__ p4,
    const FrameParam* __restrict__ fp) {
  using R = real_t<C>;
  __shared__ double red[4 * 4];
  __shared__ R salpha;
  const int f = blockIdx.y, n0 = blockIdx.x * ROWS;
  const size_t fo = (size_t)f * N * N;
  if (threadIdx.x < 64) {
    const double* q1 = p1 + (size_t)f * nb1 * 3;
    const double gd = wave_sum_partials(q1 + 0, nb1, 3);
    const double cvv = wave_sum_partials(q1 + 1, nb1, 3);
    const double cv0 = wave_sum_partials(q1 + 2, nb1, 3);
    const double dqd = wave_sum_partials(p3 + (size_t)f * nb3, nb3, 1);
    const double den = 2.0 * dqd + fp[f].lam * cvv + (BG ? fp[f].lam0 * cv0 : 0.0);
    const double alpha = (gd == 0.0) ? 0.0 : -gd / den;
    if (threadIdx.x == 0) salpha = (R)alpha;
  }
  __syncthreads();
  const R af = salpha;
  const R lam = (R)fp[f].lam, delta = (R)fp[f].delta;
  const R lam0 = (R)fp[f].lam0, alpha0 = (R)fp[f].alpha0;
  // x + alpha d, formed the same way wherever a pixel is needed
  auto xv = [x_old, d, af](size_t j) { return c_axpy(af, d[j], x_old[j]); };
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int own = min(ROWS, N - n0);
  for (int i = threadIdx.x; i < own * N; i += 256) {
    const int rr = i / N, m = i - rr * N, n = n0 + rr;
    const size_t idx = fo + (size_t)n * N + m;
    const C div_n = div_frozen<PHI>(xv, xb, idx, n, m, N, delta);
    const C xn = xv(idx);
    const C rn = c_axpy(af, qd[idx], r[idx]);
    const C gn = grad_frozen<BG>(rn, div_n, xn, xb[idx], lam, lam0, alpha0);
    const C go = g_old[idx];
    const C dv = d[idx];
    x_new[idx] = xn;
    r[idx] = rn;
    const double gx = gn.x, gy = gn.y;
    acc[0] += gx * gx + gy * gy;
    acc[1] += gx * (double)go.x + gy * (double)go.y;
    acc[2] += gx * (double)dv.x + gy * (double)dv.y;
    acc[3] += (double)go.x * (double)go.x + (double)go.y * (double)go.y;
  }
  block_sum<4>(acc, red);
  if (threadIdx.x == 0) {
    double* o = p4 + ((size_t)f * gridDim.x + blockIdx.x) * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = acc[k];
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
static hipError_t hq_dir_any(int phi, int N, int R, int B, const C* r, const C* d_old, C* d_new,
                             C* g, const C* x, const C* xb, const double* p4, int nb4, double* p1,
                             const FrameParam* fp, bool bg, hipStream_t s) {
  dim3 grid(cdiv(N, R), B);
  if (bg) {
    RECON_HQ_PHI_SWITCH(phi, (k_hq_dir<PP, C, true><<<grid, 256, 0, s>>>(
                                 N, R, r, d_old, d_new, g, x, xb, p4, nb4, p1, fp)));
  } else {
    RECON_HQ_PHI_SWITCH(phi, (k_hq_dir<PP, C, false><<<grid, 256, 0, s>>>(
                                 N, R, r, d_old, d_new, g, x, xb, p4, nb4, p1, fp)));
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  RECON_HQ_PHI_SWITCH(phi, (k_hq_curv<PP, C><<<grid, 256, 0, s>>>(N, R, d_new, xb, p1, fp)));
  return hipGetLastError();
}

template <typename C>
static hipError_t hq_update_any(int phi, int N, int R, int B, const C* x_old, C* x_new,
                                const C* d, C* r, const C* qd, const C* g_old, const C* xb,
                                const double* p1, int nb1, const double* p3, int nb3, double* p4,
                                const FrameParam* fp, bool bg, hipStream_t s) {
  dim3 grid(cdiv(N, R), B);
  if (bg) {
    RECON_HQ_PHI_SWITCH(phi, (k_hq_update<PP, C, true><<<grid, 256, 0, s>>>(
                                 N, R, x_old, x_new, d, r, qd, g_old, xb, p1, nb1, p3, nb3, p4,
                                 fp)));
  } else {
    RECON_HQ_PHI_SWITCH(phi, (k_hq_update<PP, C, false><<<grid, 256, 0, s>>>(
                                 N, R, x_old, x_new, d, r, qd, g_old, xb, p1, nb1, p3, nb3, p4,
                                 fp)));
  }
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
hipError_t launch_hq_dir(int phi, int N, int R, int B, const float2* r, const float2* d_old,
                         float2* d_new, float2* g, const float2* x, const float2* xb,
                         const double* p4, int nb4, double* p1, const FrameParam* fp, bool bg,
                         hipStream_t s) {
  return hq_dir_any(phi, N, R, B, r, d_old, d_new, g, x, xb, p4, nb4, p1, fp, bg, s);
}
hipError_t launch_hq_dir(int phi, int N, int R, int B, const double2* r, const double2* d_old,
                         double2* d_new, double2* g, const double2* x, const double2* xb,
                         const double* p4, int nb4, double* p1, const FrameParam* fp, bool bg,
                         hipStream_t s) {
  return hq_dir_any(phi, N, R, B, r, d_old, d_new, g, x, xb, p4, nb4, p1, fp, bg, s);
}
hipError_t launch_hq_update(int phi, int N, int R, int B, const float2* x_old, float2* x_new,
                            const float2* d, float2* r, const float2* qd, const float2* g_old,
                            const float2* xb, const double* p1, int nb1, const double* p3,
                            int nb3, double* p4, const FrameParam* fp, bool bg, hipStream_t s) {
  return hq_update_any(phi, N, R, B, x_old, x_new, d, r, qd, g_old, xb, p1, nb1, p3, nb3, p4, fp,
                       bg, s);
}
hipError_t launch_hq_update(int phi, int N, int R, int B, const double2* x_old, double2* x_new,
                            const double2* d, double2* r, const double2* qd,
                            const double2* g_old, const double2* xb, const double* p1, int nb1,
                            const double* p3, int nb3, double* p4, const FrameParam* fp, bool bg,
                            hipStream_t s) {
  return hq_update_any(phi, N, R, B, x_old, x_new, d, r, qd, g_old, xb, p1, nb1, p3, nb3, p4, fp,
                       bg, s);
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
