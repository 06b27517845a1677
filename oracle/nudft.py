"""Exact non-uniform DFT (oracle, FP64).

Forward model, Section 2, Eq. ModDirect (noise-free part):

    (A x)_l = (1/N) * sum_{n,m=0}^{N-1} x[n, m] * exp(+i 2 pi (kx_l m + ky_l n))

with x[n, m] row n (paired with k_y) and column m (paired with k_x), F = [1, 1]
and k normalised to [-0.5, 0.5].  Its adjoint is the paper's D matrix
(Eq. AnnMatGD, Appendix A.2):

    (A^H y)[n, m] = (1/N) * sum_l y_l * exp(-i 2 pi (kx_l m + ky_l n)).

Both are evaluated with separable FP64 phase tables
Ex[l, m] = exp(+i 2 pi kx_l m) and Ey[l, n] = exp(+i 2 pi ky_l n) and BLAS
matrix products, chunked over samples to bound memory.  ``dense_matrix``
forms the M x N^2 matrix H of Section 2 explicitly (tiny N only).
"""
from __future__ import annotations

import numpy as np

_CHUNK = 8192


def _tables(kcol: np.ndarray, N: int) -> np.ndarray:
    """exp(+i 2 pi k j) for j = 0..N-1, shape [len(k), N]."""
    j = np.arange(N, dtype=np.float64)
    return np.exp(2j * np.pi * np.outer(kcol, j))


def forward(x: np.ndarray, k: np.ndarray) -> np.ndarray:
    """y = A x.  x: [..., N, N] complex; k: [M, 2] (kx, ky).  Returns [..., M]."""
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[-1]
    assert x.shape[-2] == N
    lead = x.shape[:-2]
    xf = x.reshape((-1, N, N))
    M = k.shape[0]
    y = np.empty((xf.shape[0], M), dtype=np.complex128)
    for s in range(0, M, _CHUNK):
        e = min(M, s + _CHUNK)
        Ex = _tables(k[s:e, 0], N)            # [c, N] over m
        Ey = _tables(k[s:e, 1], N)            # [c, N] over n
        # P[f, n, l] = sum_m x[f, n, m] Ex[l, m]
        P = xf @ Ex.T
        # y[f, l] = (1/N) sum_n Ey[l, n] P[f, n, l]
        y[:, s:e] = np.einsum("ln,fnl->fl", Ey, P) / N
    return y.reshape(lead + (M,))


def adjoint(y: np.ndarray, k: np.ndarray, N: int) -> np.ndarray:
    """b = A^H y (the paper's D).  y: [..., M]; returns [..., N, N]."""
    y = np.asarray(y, dtype=np.complex128)
    lead = y.shape[:-1]
    yf = y.reshape((-1, y.shape[-1]))
    M = k.shape[0]
    assert yf.shape[1] == M
    b = np.zeros((yf.shape[0], N, N), dtype=np.complex128)
    for s in range(0, M, _CHUNK):
        e = min(M, s + _CHUNK)
        cEx = np.conj(_tables(k[s:e, 0], N))   # [c, m]
        cEy = np.conj(_tables(k[s:e, 1], N))   # [c, n]
        for f in range(yf.shape[0]):
            # b[n, m] += sum_l conj(Ey[l,n]) y_l conj(Ex[l,m])
            b[f] += cEy.T @ (yf[f, s:e, None] * cEx)
    return (b / N).reshape(lead + (N, N))


def dense_matrix(k: np.ndarray, N: int) -> np.ndarray:
    """Explicit H (M x N^2), column index n*N + m (row-major x[n, m])."""
    n, m = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    n = n.reshape(-1).astype(np.float64)
    m = m.reshape(-1).astype(np.float64)
    ph = np.outer(k[:, 0], m) + np.outer(k[:, 1], n)
    return np.exp(2j * np.pi * ph) / N


def adjoint_at(y: np.ndarray, k: np.ndarray, N: int, n, m) -> np.ndarray:
    """Entries (A^H y)[n_i, m_i] by the direct sum of Eq. AnnMatGD.
    y: [M]; n, m integer arrays.  For spot checks at large sizes."""
    y = np.asarray(y, dtype=np.complex128)
    n = np.asarray(n).ravel()
    m = np.asarray(m).ravel()
    out = np.empty(n.shape[0], dtype=np.complex128)
    for i in range(n.shape[0]):
        out[i] = np.sum(y * np.exp(-2j * np.pi * (k[:, 0] * m[i] + k[:, 1] * n[i])))
    return out / N
