"""Trajectory-only Gram quantities (oracle, FP64).

The paper's matrix (Section 3.4, Eq. DG; Appendix A.1, Eq. AnnMatG):

    G[u, v] = (1/N^2) * sum_l exp(+i 2 pi (kx_l u + ky_l v)),  u, v in [1-N, N-1]

For the image-domain Gram operator Q = A^H A with x[n, m] (row n <-> ky):

    (Q x)[n, m] = sum_{n', m'} (1/N^2) sum_l exp(i 2 pi (kx (m'-m) + ky (n'-n))) x[n', m']
                = sum_{a, b} h[a, b] x[n - a, m - b]

a linear convolution with the lag kernel

    h[a, b] = (1/N^2) * sum_l exp(-i 2 pi (ky_l a + kx_l b)) = G[-b, -a],

a, b in [-(N-1), N-1].  G and h are conjugate centro-symmetric
(h[-a, -b] = conj h[a, b]); the paper calls this a Hermitian symmetry.

``khat`` places h circularly on an L x L grid (lag a at index a mod L,
other slots zero) and takes its 2D DFT; because of the conjugate symmetry the
spectrum is real, and the linear convolution is exact for L >= 2N - 1.
"""
from __future__ import annotations

import numpy as np

_CHUNK = 4096


def lag_kernel(k: np.ndarray, N: int) -> np.ndarray:
    """h as complex128 [2N-1, 2N-1], entry [a + N-1, b + N-1]."""
    lags = np.arange(-(N - 1), N, dtype=np.float64)
    h = np.zeros((2 * N - 1, 2 * N - 1), dtype=np.complex128)
    M = k.shape[0]
    for s in range(0, M, _CHUNK):
        e = min(M, s + _CHUNK)
        Fy = np.exp(-2j * np.pi * np.outer(k[s:e, 1], lags))   # [c, a]
        Fx = np.exp(-2j * np.pi * np.outer(k[s:e, 0], lags))   # [c, b]
        h += Fy.T @ Fx
    return h / (N * N)


def paper_G(k: np.ndarray, N: int) -> np.ndarray:
    """The paper's G as complex128 [2N-1, 2N-1], entry [u + N-1, v + N-1]."""
    lags = np.arange(-(N - 1), N, dtype=np.float64)
    G = np.zeros((2 * N - 1, 2 * N - 1), dtype=np.complex128)
    M = k.shape[0]
    for s in range(0, M, _CHUNK):
        e = min(M, s + _CHUNK)
        Ex = np.exp(2j * np.pi * np.outer(k[s:e, 0], lags))    # [c, u]
        Ey = np.exp(2j * np.pi * np.outer(k[s:e, 1], lags))    # [c, v]
        G += Ex.T @ Ey
    return G / (N * N)


def circulant_embed(h: np.ndarray, N: int, L: int) -> np.ndarray:
    """L x L array with h[a, b] at [a mod L, b mod L] (requires L >= 2N-1)."""
    if L < 2 * N - 1:
        raise ValueError("L must be >= 2N-1")
    c = np.zeros((L, L), dtype=np.complex128)
    idx = np.arange(-(N - 1), N) % L
    c[np.ix_(idx, idx)] = h
    return c


def khat(k: np.ndarray, N: int, L: int, h: np.ndarray | None = None,
         return_complex: bool = False) -> np.ndarray:
    """Real L x L spectrum of the circulant-embedded lag kernel."""
    if h is None:
        h = lag_kernel(k, N)
    K = np.fft.fft2(circulant_embed(h, N, L))
    return K if return_complex else K.real.copy()


def lag_at(k: np.ndarray, N: int, a, b) -> np.ndarray:
    """h[a, b] at the given lag pairs by the direct sum over samples
    (Eq. DG with the lag convention above); a, b integer arrays in
    [-(N-1), N-1].  For spot checks at sizes where the full kernel is costly."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    out = np.empty(a.shape[0], dtype=np.complex128)
    for i in range(a.shape[0]):
        out[i] = np.sum(np.exp(-2j * np.pi * (k[:, 1] * a[i] + k[:, 0] * b[i])))
    return out / (N * N)


def _lag_sum(t: np.ndarray, N: int) -> np.ndarray:
    """sum_{a=-(N-1)}^{N-1} exp(-i 2 pi a t), a real number: the geometric
    series in closed form sin((2N-1) pi t) / sin(pi t) (period 1 in t; the
    limit 2N-1 where sin(pi t) vanishes)."""
    t = np.asarray(t, dtype=np.float64)
    t = t - np.round(t)                      # same value, |t| <= 1/2
    s = np.sin(np.pi * t)
    out = np.full(t.shape, float(2 * N - 1))
    nz = np.abs(t) > 1e-9
    out[nz] = np.sin((2 * N - 1) * np.pi * t[nz]) / s[nz]
    # |t| <= 1e-9: the series differs from 2N-1 by about 2 pi^2 t^2 N^3 / 3,
    # a relative 1e-11 or less for N <= 1024
    return out


def khat_at(k: np.ndarray, N: int, L: int, p, q) -> np.ndarray:
    """Khat[p, q] (the spectrum ``khat`` returns) at given frequency pairs.

    Khat[p, q] = sum_{a,b} h[a, b] exp(-i 2 pi (p a + q b) / L)
               = (1/N^2) sum_l S(ky_l + p/L) S(kx_l + q/L),
    S the lag sum over [-(N-1), N-1] (real), so the value is real."""
    p = np.asarray(p, dtype=np.float64).ravel()
    q = np.asarray(q, dtype=np.float64).ravel()
    out = np.empty(p.shape[0], dtype=np.float64)
    for i in range(p.shape[0]):
        out[i] = np.sum(_lag_sum(k[:, 1] + p[i] / L, N) * _lag_sum(k[:, 0] + q[i] / L, N))
    return out / (N * N)
