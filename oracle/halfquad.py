"""Half-quadratic minimisation of the regularised criterion (oracle, FP64).

Section 5 of the paper names a dual (half-quadratic) optimisation [Idier01b]
as a way to cut the cost of the conjugate-gradient minimisation of Section
3.3.  This is its multiplicative (Geman-Reynolds) form, written out:

  outer iteration, at the current image xbar:
    1. freeze the half-quadratic weights w_i = phi'(s_i) / s_i of the
       differences s_i = |(D xbar)_i| (and w0_p = phi0'(|xbar_p|) / |xbar_p|
       of the background term when lam0 > 0);
    2. decrease the quadratic surrogate
         S(x; xbar) = ||y - A x||^2
                      + lam  sum_i [phi(s_i) + (w_i / 2) (|(D x)_i|^2 - s_i^2)]
                      + lam0 sum_p [phi0(|xbar_p|) + (w0_p / 2) (|x_p|^2 - |xbar_p|^2)]
       by `inner` steps of linear conjugate gradients started at xbar, on
       the image-domain form of the data term (Section 3.4):
         gradient  g = 2 (Q x - b) + lam D^T (w . D x) + lam0 w0 . x
         step      alpha = -Re<g, d> / (2 Re<d, Q d> + lam sum w |D d|^2
                                                    + lam0 sum w0 |d|^2)
                   (the exact minimiser of the quadratic along d)
         direction d = -g first, then d = -g_new + beta d with the
                   Polak-Ribiere coefficient clipped at zero (for a
                   quadratic with exact steps it equals the Fletcher-Reeves
                   one) and the same descent safeguard as Section 3.3's
                   iteration.
  S(.; xbar) lies above J and touches it at xbar (phi(sqrt(rho)) is concave
  in rho), and linear CG decreases S from xbar, so J decreases at every
  outer iteration.

The minimiser of one surrogate solves the linear system
    (2 A^H A + lam D^T W D + lam0 W0) x = 2 A^H y,
which ``surrogate_minimiser_dense`` forms explicitly for tiny images.
"""
from __future__ import annotations

import numpy as np

from . import penalty, solver, toeplitz


def _dot(a, b):
    return np.sum(np.conj(a) * b)


def frozen_weights(xbar, delta, kind="hyperbolic", lam0=0.0, alpha0=1.0,
                   kind0="huber"):
    """(wv, wh, w0): weights of the vertical and horizontal differences of
    xbar and of its pixels (w0 = None without the background term)."""
    dv, dh = penalty.diff(xbar)
    wv = penalty.weight(np.abs(dv), delta, kind)
    wh = penalty.weight(np.abs(dh), delta, kind)
    w0 = penalty.weight(np.abs(xbar), alpha0, kind0) if lam0 else None
    return wv, wh, w0


def surrogate_grad(x, r, W, lam, lam0=0.0):
    """2 r + lam D^T (w . D x) + lam0 w0 . x, with r = Q x - b."""
    wv, wh, w0 = W
    dv, dh = penalty.diff(x)
    g = 2.0 * r + lam * penalty.diff_adjoint(wv * dv, wh * dh)
    if lam0:
        g = g + lam0 * w0 * x
    return g


def surrogate_curv(d, W, lam, lam0=0.0):
    """lam sum w |D d|^2 + lam0 sum w0 |d|^2."""
    wv, wh, w0 = W
    ev, eh = penalty.diff(d)
    c = lam * (np.sum(wv * np.abs(ev) ** 2) + np.sum(wh * np.abs(eh) ** 2))
    if lam0:
        c = c + lam0 * np.sum(w0 * np.abs(d) ** 2)
    return c


def solve(b, K, lam, delta, outer, inner, kind="hyperbolic", x0=None,
          lam0=0.0, alpha0=1.0, kind0="huber", trace=None):
    """`outer` half-quadratic iterations of `inner` linear-CG steps each,
    from x0 (zeros by default).  trace: optional list receiving, after every
    outer iteration, the image and the number of operator applications."""
    b = np.asarray(b, dtype=np.complex128)
    N = b.shape[-1]

    def Q(v):
        return toeplitz.apply_gram(v, K, N)

    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = Q(x) - b
    applies = 0
    for _ in range(outer):
        W = frozen_weights(x, delta, kind, lam0, alpha0, kind0)
        g = surrogate_grad(x, r, W, lam, lam0)
        d = -g
        for _i in range(inner):
            Qd = Q(d)
            applies += 1
            gd = np.real(_dot(g, d))
            curv = 2.0 * np.real(_dot(d, Qd)) + surrogate_curv(d, W, lam, lam0)
            alpha = 0.0 if gd == 0.0 else -gd / curv
            x = x + alpha * d
            r = r + alpha * Qd
            g_new = surrogate_grad(x, r, W, lam, lam0)
            beta = solver.pr_plus_beta(g_new, g)
            d, _ = solver.next_direction(g_new, d, beta)
            g = g_new
        if trace is not None:
            trace.append(dict(x=x, applies=applies))
    return x


def surrogate_minimiser_dense(y, k, N, xbar, lam, delta, kind="hyperbolic",
                              lam0=0.0, alpha0=1.0, kind0="huber"):
    """Minimiser of S(.; xbar) from the explicit matrix of Section 2 and an
    explicit difference matrix: (2 A^H A + lam D^T W D + lam0 W0) x = 2 A^H y
    (tiny N; differences ordered as penalty.diff flattens them)."""
    from . import nudft
    H = nudft.dense_matrix(k, N)
    n2 = N * N
    rows = []
    for n in range(N - 1):
        for m in range(N):
            e = np.zeros(n2)
            e[(n + 1) * N + m], e[n * N + m] = 1.0, -1.0
            rows.append(e)
    for n in range(N):
        for m in range(N - 1):
            e = np.zeros(n2)
            e[n * N + m + 1], e[n * N + m] = 1.0, -1.0
            rows.append(e)
    Dm = np.array(rows)
    wv, wh, w0 = frozen_weights(xbar, delta, kind, lam0, alpha0, kind0)
    Wd = np.concatenate([wv.ravel(), wh.ravel()])
    A = 2.0 * H.conj().T @ H + lam * (Dm.T @ (Wd[:, None] * Dm))
    if lam0:
        A = A + lam0 * np.diag(w0.ravel())
    return np.linalg.solve(A, 2.0 * H.conj().T @ y).reshape(N, N)
