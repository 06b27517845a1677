"""Regularised criterion and its gradient (oracle, FP64).

J(x) = ||y - A x||^2 + lam * Omega_1(x) + lam0 * Omega_0(x)   (Section 3.3)

Two evaluations of the data term:

* direct:     ||y - A x||^2 with the exact forward model (Eq. CritLS);
* rewritten:  ||y||^2 - 2 Re<x, b> + Re<x, Q x>, b = A^H y, Q = A^H A
              (Eq. NewCritLS; the paper writes the last term as sum C G with
              the image correlation C, which is the same number).

Gradient (Appendix B), real gradient packed as complex (2 dJ/d conj x):

    grad J = 2 (Q x - b) + lam * D^T (w(Dx) * Dx) + lam0 * w0(x) * x.
"""
from __future__ import annotations

import numpy as np

from . import nudft, penalty, toeplitz


def penalty_value(x, lam, delta, kind="hyperbolic", lam0=0.0, alpha0=1.0,
                  kind0="huber"):
    v = lam * penalty.smooth_value(x, delta, kind)
    if lam0:
        v = v + lam0 * penalty.background_value(x, alpha0, kind0)
    return v


def penalty_grad(x, lam, delta, kind="hyperbolic", lam0=0.0, alpha0=1.0,
                 kind0="huber"):
    g = lam * penalty.smooth_grad(x, delta, kind)
    if lam0:
        g = g + lam0 * penalty.background_grad(x, alpha0, kind0)
    return g


def J_direct(x, y, k, lam, delta, kind="hyperbolic", **kw):
    r = y - nudft.forward(x, k)
    return (np.abs(r) ** 2).sum(axis=-1) + penalty_value(x, lam, delta, kind, **kw)


def J_rewritten(x, yy, b, Qx, lam, delta, kind="hyperbolic", **kw):
    """yy = ||y||^2, b = A^H y, Qx = Q x."""
    data = (yy - 2.0 * np.real(np.sum(np.conj(x) * b, axis=(-2, -1)))
            + np.real(np.sum(np.conj(x) * Qx, axis=(-2, -1))))
    return data + penalty_value(x, lam, delta, kind, **kw)


def grad(x, b, K, lam, delta, kind="hyperbolic", **kw):
    N = x.shape[-1]
    return 2.0 * (toeplitz.apply_gram(x, K, N) - b) + penalty_grad(
        x, lam, delta, kind, **kw)


def image_correlation(x: np.ndarray) -> np.ndarray:
    """Appendix A.1's C[u, v] = sum_{p,q} f[p,q] conj f[p-u, q-v] with
    f[p, q] = x[n=q, m=p]; returned as [u + N-1, v + N-1] (plain loops)."""
    N = x.shape[-1]
    C = np.zeros((2 * N - 1, 2 * N - 1), dtype=np.complex128)
    for u in range(-(N - 1), N):
        for v in range(-(N - 1), N):
            s = 0.0 + 0.0j
            for p in range(max(0, u), min(N - 1, N - 1 + u) + 1):
                for q in range(max(0, v), min(N - 1, N - 1 + v) + 1):
                    s += x[q, p] * np.conj(x[q - v, p - u])
            C[u + N - 1, v + N - 1] = s
    return C
