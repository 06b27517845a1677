// Pseudo-conjugate-gradient kernels (Section 3.3) around the Gram apply.
//
// One iteration (per frame, all frames of a batch in the same launches):
//   dir+row pass : beta (PR+, restart) from the previous update's partials,
//                  d = -g + beta d_old, partials Re<g,d>, sum w(|Dx|)|Dd|^2,
//                  row FFTs of d                       (toeplitz.hip)
//   column pass  : Gram spectrum product                (toeplitz.hip)
//   row inverse  : Qd, partial Re<d, Qd>                (toeplitz.hip)
//   update       : alpha = -Re<g,d> / (2 Re<d,Qd> + lam sum w|Dd|^2)
//                  x += alpha d ; r += alpha Qd (r = Qx - b)
//                  g = 2 r + lam D^T(w(|Dx|) Dx)  (gradient, Appendix B and
//                  the penalty gradient), partials for beta   (this file)
// All reductions are per-block FP64 partials summed in a fixed order by the
// consumer kernel, so results do not depend on scheduling or batch size.
// x and d are double-buffered because the stencils read neighbouring rows
// that other blocks of the same launch overwrite.
#include "kernels.hpp"
#include "stencil.hpp"

namespace recon {

__global__ void k_zero_f64(size_t n, double* p) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void k_set_params(int B, double lam, double delta, double lam0, double alpha0,
                             int stop_at, FrameParam* fp) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f < B) fp[f] = FrameParam{lam, delta, lam0, alpha0, stop_at, 0};
}

// Complex values widened to the FP64 iteration, or rounded back to FP32.
template <typename O, typename I>
__global__ void k_convert(size_t n, const I* __restrict__ in, O* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const I v = in[i];
    out[i] = cmk<O>((real_t<O>)v.x, (real_t<O>)v.y);
  }
}

template <int PHI, typename C>
__global__ __launch_bounds__(256) void k_init(
    int N, int ROWS, const C* __restrict__ b, const C* __restrict__ x0,
    const C* __restrict__ qx0, C* __restrict__ x, C* __restrict__ r,
    C* __restrict__ d, double* __restrict__ p4,
    double* __restrict__ pg0, const FrameParam* __restrict__ fp) {
  using R = real_t<C>;
  extern __shared__ __align__(16) unsigned char init_lds[];
  C* xt = reinterpret_cast<C*>(init_lds);
  __shared__ double red[1 * 4];
  const int f = blockIdx.y;
  const int n0 = blockIdx.x * ROWS;
  const size_t fo = (size_t)f * N * N;
  const R lam = (R)fp[f].lam, delta = (R)fp[f].delta;
  const R lam0 = (R)fp[f].lam0, alpha0 = (R)fp[f].alpha0;
  const int r_lo = max(n0 - 1, 0), r_hi = min(n0 + ROWS + 1, N);
  for (int i = threadIdx.x; i < (r_hi - r_lo) * N; i += 256) {
    const int rr = i / N, m = i - rr * N;
    const size_t idx = fo + (size_t)(r_lo + rr) * N + m;
    xt[(r_lo + rr - (n0 - 1)) * N + m] = x0 ? x0[idx] : cmk<C>(0, 0);
  }
  __syncthreads();
  double acc[1] = {0.0};
  const int own = min(ROWS, N - n0);
  for (int i = threadIdx.x; i < own * N; i += 256) {
    const int rr = i / N, m = i - rr * N;
    const int n = n0 + rr;
    const size_t idx = fo + (size_t)n * N + m;
    const C* mid = xt + (rr + 1) * N;
    const C* up = (n > 0) ? mid - N : nullptr;
    const C* dn = (n + 1 < N) ? mid + N : nullptr;
    const C div = divergence<PHI>(up, mid, dn, m, N, delta);
    const C bv = b[idx];
    const C q = qx0 ? qx0[idx] : cmk<C>(0, 0);
    const C rn = c_sub(q, bv);
    const C gn = grad_full(rn, div, mid[m], lam, lam0, alpha0);
    x[idx] = mid[m];
    r[idx] = rn;
    d[idx] = cmk<C>(0, 0);
    acc[0] += (double)gn.x * (double)gn.x + (double)gn.y * (double)gn.y;
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) {
    double* o = p4 + ((size_t)f * gridDim.x + blockIdx.x) * 4;
    // |g|^2 with zero history: beta = 0, so the first direction is -g.
    o[0] = acc[0];
    o[1] = 0.0;
    o[2] = 0.0;
    o[3] = 0.0;
    pg0[(size_t)f * gridDim.x + blockIdx.x] = acc[0];
  }
}

// Criterion J = ||y||^2 - 2 Re<x, b> + Re<x, Qx> + lam sum phi(|Dx|)
// + lam0 sum phi_alpha0(|x|) (Section 3.4, Eq. NewCritLS; the background term
// of Section 3.3, Huber) with Qx = r + b:
// partials [Re<x, b>, Re<x, r>, sum phi, sum phi_alpha0] per block.
template <int PHI, typename C>
__global__ __launch_bounds__(256) void k_objective(int N, int ROWS, const C* __restrict__ x,
                                                   const C* __restrict__ b,
                                                   const C* __restrict__ r,
                                                   double* __restrict__ pobj,
                                                   const FrameParam* __restrict__ fp) {
  __shared__ double red[4 * 4];
  const int f = blockIdx.y;
  const int n0 = blockIdx.x * ROWS;
  const size_t fo = (size_t)f * N * N;
  const double delta = fp[f].delta, alpha0 = fp[f].alpha0;
  const bool bg = fp[f].lam0 != 0.0;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int own = min(ROWS, N - n0);
  for (int i = threadIdx.x; i < own * N; i += 256) {
    const int rr = i / N, m = i - rr * N;
    const int n = n0 + rr;
    const size_t idx = fo + (size_t)n * N + m;
    const C xv = x[idx], bv = b[idx], rv = r[idx];
    acc[0] += (double)xv.x * bv.x + (double)xv.y * bv.y;
    acc[1] += (double)xv.x * rv.x + (double)xv.y * rv.y;
    if (bg) acc[3] += pen_phi<1>((double)xv.x * xv.x + (double)xv.y * xv.y, alpha0);
    if (n + 1 < N) {
      const C xd = x[idx + N];
      const double tx = (double)xd.x - xv.x, ty = (double)xd.y - xv.y;
      acc[2] += pen_phi<PHI>(tx * tx + ty * ty, delta);
    }
    if (m + 1 < N) {
      const C xr = x[idx + 1];
      const double tx = (double)xr.x - xv.x, ty = (double)xr.y - xv.y;
      acc[2] += pen_phi<PHI>(tx * tx + ty * ty, delta);
    }
  }
  block_sum<4>(acc, red);
  if (threadIdx.x == 0) {
    double* o = pobj + ((size_t)f * gridDim.x + blockIdx.x) * 4;
    o[0] = acc[0];
    o[1] = acc[1];
    o[2] = acc[2];
    o[3] = acc[3];
  }
}

struct StatsOut {
  double J, grad_ratio, gnorm0;
  int32_t iters_done, status;
};

__global__ void k_stats(int B, const double* __restrict__ pobj, int nbo,
                        const double* __restrict__ p4, int nb4,
                        const double* __restrict__ pg0, int nbg,
                        const double* __restrict__ yy, int iters,
                        const FrameParam* __restrict__ fp, StatsOut* __restrict__ st) {
  // one wavefront per frame
  const int f = blockIdx.x;
  if (f >= B) return;
  const double xb = wave_sum_partials(pobj + (size_t)f * nbo * 4 + 0, nbo, 4);
  const double xr = wave_sum_partials(pobj + (size_t)f * nbo * 4 + 1, nbo, 4);
  const double ph = wave_sum_partials(pobj + (size_t)f * nbo * 4 + 2, nbo, 4);
  const double ph0 = wave_sum_partials(pobj + (size_t)f * nbo * 4 + 3, nbo, 4);
  const double gg = wave_sum_partials(p4 + (size_t)f * nb4 * 4, nb4, 4);
  const double g0 = wave_sum_partials(pg0 + (size_t)f * nbg, nbg, 1);
  if (threadIdx.x == 0) {
    const double J = yy[f] - xb + xr + fp[f].lam * ph + fp[f].lam0 * ph0;
    StatsOut o;
    o.J = J;
    o.gnorm0 = sqrt(g0);
    o.grad_ratio = (g0 > 0.0) ? sqrt(gg / g0) : 0.0;
    o.iters_done = iters;
    o.status = (isfinite(J) && isfinite(gg)) ? 0 : 6;
    st[f] = o;
  }
}

// The gradient g = 2 r + lam D^T(w(Dx) Dx) of the current iterate, or the
// pending direction -g + beta d_old (as the next direction kernel forms
// it), into out.  Rows n0-1 .. n0+ROWS of x are staged in LDS.
template <int PHI, typename C>
__global__ __launch_bounds__(256) void k_export(int N, int ROWS, const C* __restrict__ x,
                                                const C* __restrict__ r,
                                                const C* __restrict__ d_old,
                                                const double* __restrict__ p4, int nb4,
                                                const FrameParam* __restrict__ fp,
                                                float2* __restrict__ out, int dir) {
  using R = real_t<C>;
  extern __shared__ __align__(16) unsigned char exp_lds[];
  C* xt = reinterpret_cast<C*>(exp_lds);
  const int f = blockIdx.y;
  const int n0 = blockIdx.x * ROWS;
  const size_t fo = (size_t)f * N * N;
  const R lam = (R)fp[f].lam, delta = (R)fp[f].delta;
  const R lam0 = (R)fp[f].lam0, alpha0 = (R)fp[f].alpha0;
  R bf = 0;
  if (dir) {
    const double* pf = p4 + (size_t)f * nb4 * 4;
    const double gg = wave_sum_partials(pf + 0, nb4, 4);
    const double ggo = wave_sum_partials(pf + 1, nb4, 4);
    const double gdo = wave_sum_partials(pf + 2, nb4, 4);
    const double gg_old = wave_sum_partials(pf + 3, nb4, 4);
    double beta = 0.0;
    if (gg_old > 0.0) beta = fmax(0.0, (gg - ggo) / gg_old);
    if (-gg + beta * gdo >= 0.0) beta = 0.0;
    bf = (R)beta;
  }
  const int r_lo = max(n0 - 1, 0), r_hi = min(n0 + ROWS + 1, N);
  for (int i = threadIdx.x; i < (r_hi - r_lo) * N; i += 256) {
    const int rr = i / N, m = i - rr * N;
    xt[(r_lo + rr - (n0 - 1)) * N + m] = x[fo + (size_t)(r_lo + rr) * N + m];
  }
  __syncthreads();
  const int own = min(ROWS, N - n0);
  for (int i = threadIdx.x; i < own * N; i += 256) {
    const int rr = i / N, m = i - rr * N;
    const int n = n0 + rr;
    const size_t idx = fo + (size_t)n * N + m;
    const C* mid = xt + (rr + 1) * N;
    const C div = divergence<PHI>(n > 0 ? mid - N : nullptr, mid,
                                  n + 1 < N ? mid + N : nullptr, m, N, delta);
    const C rv = r[idx];
    const C g = grad_full(rv, div, mid[m], lam, lam0, alpha0);
    if (dir) {
      const C dv = d_old[idx];
      out[idx] = to_f32(cmk<C>(rfma(bf, dv.x, -g.x), rfma(bf, dv.y, -g.y)));
    } else {
      out[idx] = to_f32(g);
    }
  }
}

// ------------------------------------------------------------------ launchers
#define RECON_PHI_SWITCH(PHI_, CALL)                  \
  switch (PHI_) {                                     \
    case 0: { constexpr int PP = 0; CALL; } break;    \
    case 1: { constexpr int PP = 1; CALL; } break;    \
    case 2: { constexpr int PP = 2; CALL; } break;    \
    default: return hipErrorInvalidValue;             \
  }

hipError_t launch_zero_f64(size_t n, double* p, hipStream_t s) {
  k_zero_f64<<<(unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096), 256, 0, s>>>(n, p);
  return hipGetLastError();
}

hipError_t launch_set_params(int B, double lam, double delta, double lam0, double alpha0,
                             int stop_at, FrameParam* fp, hipStream_t s) {
  k_set_params<<<cdiv(B, 256), 256, 0, s>>>(B, lam, delta, lam0, alpha0, stop_at, fp);
  return hipGetLastError();
}

template <typename C>
static hipError_t init_any(int phi, int N, int R, int B, const C* b, const C* x0, const C* qx0,
                           C* x, C* r, C* d, double* p4, double* pg0, const FrameParam* fp,
                           hipStream_t s) {
  dim3 grid(cdiv(N, R), B);
  const size_t shm = (size_t)(R + 2) * N * sizeof(C);
  RECON_PHI_SWITCH(phi, (k_init<PP, C><<<grid, 256, shm, s>>>(N, R, b, x0, qx0, x, r, d, p4,
                                                              pg0, fp)));
  return hipGetLastError();
}
hipError_t launch_init(int phi, int N, int R, int B, const float2* b, const float2* x0,
                       const float2* qx0, float2* x, float2* r, float2* d,
                       double* p4, double* pg0, const FrameParam* fp, hipStream_t s) {
  return init_any(phi, N, R, B, b, x0, qx0, x, r, d, p4, pg0, fp, s);
}
hipError_t launch_init(int phi, int N, int R, int B, const double2* b, const double2* x0,
                       const double2* qx0, double2* x, double2* r, double2* d,
                       double* p4, double* pg0, const FrameParam* fp, hipStream_t s) {
  return init_any(phi, N, R, B, b, x0, qx0, x, r, d, p4, pg0, fp, s);
}

template <typename C>
static hipError_t objective_any(int phi, int N, int R, int B, const C* x, const C* b, const C* r,
                                double* pobj, const FrameParam* fp, hipStream_t s) {
  dim3 grid(cdiv(N, R), B);
  RECON_PHI_SWITCH(phi, (k_objective<PP, C><<<grid, 256, 0, s>>>(N, R, x, b, r, pobj, fp)));
  return hipGetLastError();
}
hipError_t launch_objective(int phi, int N, int R, int B, const float2* x, const float2* b,
                            const float2* r, double* pobj, const FrameParam* fp,
                            hipStream_t s) {
  return objective_any(phi, N, R, B, x, b, r, pobj, fp, s);
}
hipError_t launch_objective(int phi, int N, int R, int B, const double2* x, const double2* b,
                            const double2* r, double* pobj, const FrameParam* fp,
                            hipStream_t s) {
  return objective_any(phi, N, R, B, x, b, r, pobj, fp, s);
}

hipError_t launch_stats(int B, const double* pobj, int nbo, const double* p4, int nb4,
                         const double* pg0, int nbg, const double* yy, int iters,
                         const FrameParam* fp, void* stats, hipStream_t s) {
  k_stats<<<B, 64, 0, s>>>(B, pobj, nbo, p4, nb4, pg0, nbg, yy, iters, fp,
                           reinterpret_cast<StatsOut*>(stats));
  return hipGetLastError();
}

template <typename C>
static hipError_t export_any(int phi, int N, int R, int B, const C* x, const C* r,
                             const C* d_old, const double* p4, int nb4, const FrameParam* fp,
                             float2* out, int dir, hipStream_t s) {
  dim3 grid(cdiv(N, R), B);
  const size_t shm = (size_t)(R + 2) * N * sizeof(C);
  RECON_PHI_SWITCH(phi, (k_export<PP, C><<<grid, 256, shm, s>>>(N, R, x, r, d_old, p4, nb4, fp,
                                                                out, dir)));
  return hipGetLastError();
}
hipError_t launch_export(int phi, int N, int R, int B, const float2* x, const float2* r,
                         const float2* d_old, const double* p4, int nb4, const FrameParam* fp,
                         float2* out, int dir, hipStream_t s) {
  return export_any(phi, N, R, B, x, r, d_old, p4, nb4, fp, out, dir, s);
}
hipError_t launch_export(int phi, int N, int R, int B, const double2* x, const double2* r,
                         const double2* d_old, const double* p4, int nb4, const FrameParam* fp,
                         float2* out, int dir, hipStream_t s) {
  return export_any(phi, N, R, B, x, r, d_old, p4, nb4, fp, out, dir, s);
}

template <typename O, typename I>
static hipError_t convert_any(size_t n, const I* in, O* out, hipStream_t s) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks == 0) return hipSuccess;
  k_convert<O, I><<<(unsigned)blocks, 256, 0, s>>>(n, in, out);
  return hipGetLastError();
}
hipError_t launch_widen(size_t n, const float2* in, double2* out, hipStream_t s) {
  return convert_any(n, in, out, s);
}
hipError_t launch_narrow(size_t n, const double2* in, float2* out, hipStream_t s) {
  return convert_any(n, in, out, s);
}

}  // namespace recon
