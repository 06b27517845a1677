"""Gram operator Q = A^H A (oracle, FP64).

Section 3.4 rewrites the data term so that only image-domain products are
needed; its gradient (Appendix B) is a 2D convolution of the image with the
trajectory-only kernel, evaluated by FFT.  The convolution is linear (not
circular) over the N x N support, so it is exact after zero padding to any
L >= 2N - 1:

    Q v = crop_N( IFFT_L( khat * FFT_L( pad_L(v) ) ) ).

``dense_gram`` forms A^H A from the explicit matrix of Section 2 (tiny N).
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft

from . import nudft

_WORKERS = os.cpu_count() or 1


def apply_gram(v: np.ndarray, K: np.ndarray, N: int) -> np.ndarray:
    """Q v for v [..., N, N] given the L x L spectrum K (from gram.khat)."""
    L = K.shape[0]
    v = np.asarray(v, dtype=np.complex128)
    pad = np.zeros(v.shape[:-2] + (L, L), dtype=np.complex128)
    pad[..., :N, :N] = v
    out = scipy.fft.ifft2(K * scipy.fft.fft2(pad, axes=(-2, -1), workers=_WORKERS),
                          axes=(-2, -1), workers=_WORKERS)
    return out[..., :N, :N].copy()


def dense_gram(k: np.ndarray, N: int) -> np.ndarray:
    """Explicit A^H A, N^2 x N^2, index n*N + m."""
    H = nudft.dense_matrix(k, N)
    return H.conj().T @ H
