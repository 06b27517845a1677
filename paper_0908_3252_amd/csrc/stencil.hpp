// Edge-preserving penalty on first-order pixel differences (Section 3.3).
//
// phi acts on the modulus s = |t| of each complex difference t; the
// gradient and the half-quadratic majorant use the weight w(s) = phi'(s)/s:
//   PHI 0  hyperbolic  phi = sqrt(delta^2 + s^2)     w = 1/sqrt(delta^2 + s^2)
//   PHI 1  Huber       phi = s^2 (s <= delta), 2 delta s - delta^2 otherwise
//                      w = 2 (s <= delta), 2 delta / s otherwise
//   PHI 2  quadratic   phi = s^2                     w = 2
#pragma once
#include "common.hpp"

namespace recon {

template <int PHI>
__device__ __forceinline__ float pen_weight(float s2, float delta) {
  if constexpr (PHI == 0) {
    return rsqrtf(fmaf(delta, delta, s2));
  } else if constexpr (PHI == 1) {
    return (s2 <= delta * delta) ? 2.f : 2.f * delta * rsqrtf(s2);
  } else {
    return 2.f;
  }
}

// FP64 weights (the FP64 iteration): the FP64 reciprocal square root
// (hardware estimate plus one refinement, within about an ulp) instead of a
// square root followed by a division, about a fifth of the instructions.
template <int PHI>
__device__ __forceinline__ double pen_weight(double s2, double delta) {
  if constexpr (PHI == 0) {
    return rsqrt(fma(delta, delta, s2));
  } else if constexpr (PHI == 1) {
    return (s2 <= delta * delta) ? 2.0 : 2.0 * delta * rsqrt(s2);
  } else {
    return 2.0;
  }
}

template <int PHI>
__device__ __forceinline__ double pen_phi(double s2, double delta) {
  if constexpr (PHI == 0) {
    return sqrt(delta * delta + s2);
  } else if constexpr (PHI == 1) {
    return (s2 <= delta * delta) ? s2 : 2.0 * delta * sqrt(s2) - delta * delta;
  } else {
    return s2;
  }
}

// w(|t|) t for the difference t = b - a.
template <int PHI, typename C>
__device__ __forceinline__ C wdiff(C a, C b, real_t<C> delta) {
  const C t = c_sub(b, a);
  return c_scale(t, pen_weight<PHI>(c_abs2(t), delta));
}

// (D^T (w . D x))[n][m] from a tile holding rows n-1, n, n+1 of x:
// up/mid/dn point at column 0 of those rows (up/dn may be null at the image
// border).  Vertical differences exist for rows 0..N-2, horizontal for
// columns 0..N-2 (non-periodic).  Also returns the weights of the pixel's
// forward edges (down: (n, m)-(n+1, m), right: (n, m)-(n, m+1); 0 where the
// edge does not exist), which the curvature of the majorant reuses.
template <int PHI, typename C>
__device__ __forceinline__ C divergence_fw(const C* up, const C* mid, const C* dn, int m, int N,
                                           real_t<C> delta, real_t<C>& w_dn, real_t<C>& w_rt) {
  const C c = mid[m];
  C acc = cmk<C>(0, 0);
  w_dn = 0;
  w_rt = 0;
  if (up) acc = c_add(acc, wdiff<PHI>(up[m], c, delta));
  if (dn) {
    const C t = c_sub(dn[m], c);
    w_dn = pen_weight<PHI>(c_abs2(t), delta);
    acc = c_sub(acc, c_scale(t, w_dn));
  }
  if (m > 0) acc = c_add(acc, wdiff<PHI>(mid[m - 1], c, delta));
  if (m + 1 < N) {
    const C t = c_sub(mid[m + 1], c);
    w_rt = pen_weight<PHI>(c_abs2(t), delta);
    acc = c_sub(acc, c_scale(t, w_rt));
  }
  return acc;
}

// The same without the weights (one code path, so the same values).
template <int PHI, typename C>
__device__ __forceinline__ C divergence(const C* up, const C* mid, const C* dn, int m, int N,
                                        real_t<C> delta) {
  real_t<C> w_dn, w_rt;
  return divergence_fw<PHI>(up, mid, dn, m, N, delta, w_dn, w_rt);
}

// (D^T (w(D xb) . D x))[n][m] with the weights frozen at the image xb (the
// half-quadratic surrogate of Section 5's alternative minimiser): rows n-1,
// n, n+1 of x (up/mid/dn) and of xb (bup/bmid/bdn), null at the image border
// as above; the edges in the order of divergence_fw.  Also returns the
// frozen weights of the pixel's forward edges.
template <int PHI, typename C>
__device__ __forceinline__ C divergence_frozen_fw(const C* up, const C* mid, const C* dn,
                                                  const C* bup, const C* bmid, const C* bdn,
                                                  int m, int N, real_t<C> delta,
                                                  real_t<C>& w_dn, real_t<C>& w_rt) {
  const C c = mid[m], cb = bmid[m];
  C acc = cmk<C>(0, 0);
  w_dn = 0;
  w_rt = 0;
  if (up) {
    const real_t<C> w = pen_weight<PHI>(c_abs2(c_sub(cb, bup[m])), delta);
    acc = c_add(acc, c_scale(c_sub(c, up[m]), w));
  }
  if (dn) {
    w_dn = pen_weight<PHI>(c_abs2(c_sub(bdn[m], cb)), delta);
    acc = c_sub(acc, c_scale(c_sub(dn[m], c), w_dn));
  }
  if (m > 0) {
    const real_t<C> w = pen_weight<PHI>(c_abs2(c_sub(cb, bmid[m - 1])), delta);
    acc = c_add(acc, c_scale(c_sub(c, mid[m - 1]), w));
  }
  if (m + 1 < N) {
    w_rt = pen_weight<PHI>(c_abs2(c_sub(bmid[m + 1], cb)), delta);
    acc = c_sub(acc, c_scale(c_sub(mid[m + 1], c), w_rt));
  }
  return acc;
}

template <int PHI, typename C>
__device__ __forceinline__ C divergence_frozen(const C* up, const C* mid, const C* dn,
                                               const C* bup, const C* bmid, const C* bdn, int m,
                                               int N, real_t<C> delta) {
  real_t<C> w_dn, w_rt;
  return divergence_frozen_fw<PHI>(up, mid, dn, bup, bmid, bdn, m, N, delta, w_dn, w_rt);
}

// Gradient of the criterion at one pixel (Appendix B): g = 2 r + lam div
// + lam0 w0(|x|) x, where div = (D^T (w . D x))[n][m] and the background
// term of Section 3.3 (Omega_0 = sum phi_alpha0(|x|), Huber) is on when
// lam0 != 0.  Every kernel forms the gradient through this one function, so
// every copy of it is bitwise the same.
// BG = false compiles the term out (launches where no frame uses it).
template <bool BG = true, typename C>
__device__ __forceinline__ C grad_full(C r, C div, C x, real_t<C> lam, real_t<C> lam0,
                                       real_t<C> alpha0) {
  C g = cmk<C>(rfma(lam, div.x, 2 * r.x), rfma(lam, div.y, 2 * r.y));
  if constexpr (BG) {
    if (lam0 != 0) {
      const real_t<C> w = lam0 * pen_weight<1>(c_abs2(x), alpha0);
      g = cmk<C>(rfma(w, x.x, g.x), rfma(w, x.y, g.y));
    }
  }
  return g;
}

// Gradient of the half-quadratic surrogate at one pixel: 2 r + lam div +
// lam0 w0(|xb|) x, div from divergence_frozen (the form of grad_full with the
// background weight frozen at xb).
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

// Weight of the background term at one pixel (0 when it is off).
template <bool BG = true, typename C>
__device__ __forceinline__ real_t<C> bg_weight(C x, real_t<C> lam0, real_t<C> alpha0) {
  if constexpr (BG) return lam0 != 0 ? pen_weight<1>(c_abs2(x), alpha0) : real_t<C>(0);
  else return real_t<C>(0);
}

}  // namespace recon
