"""Convolution gridding and its NUFFT use (oracle, FP64).

Section 1 of the paper describes the gridding reconstruction the method is
compared with, in four steps: weighting of the samples for the non-uniform
sampling density, resampling onto a Cartesian grid with a convolution
kernel, an FFT, and correction of the kernel's apodization; Section 4.1
uses a 7 x 7 Kaiser-Bessel kernel [O'Sullivan85] and measures the
quadratic error in a region ROI1 and the variance in a flat region ROI2.
Section 5 proposes the same machinery (a non-uniform FFT [Dale01]) to
accelerate the exact precomputations of D = A^H y and of the Gram kernel.

Conventions (the image and sample order of Eq. ModDirect):

* the grid has G points per axis; a sample at k (cycles/pixel) sits at the
  grid coordinate u = G k; the kernel phi (width W grid points) is
  separable, phi2(g - u) = phi(g1 - G ky) phi(g2 - G kx), and grid indices
  wrap modulo G;
* Kaiser-Bessel kernel phi(t) = I0(beta sqrt(1 - (2t/W)^2)) for |t| <= W/2,
  with the closed-form transform
      phi_hat(nu) = W sinh(sqrt(beta^2 - (pi W nu)^2)) / sqrt(beta^2 - (pi W nu)^2)
  (sin/sqrt beyond the cut-off); beta from the minimal-oversampling rule
  beta = pi sqrt(W^2 / s^2 (s - 1/2)^2 - 0.8), s = G / Nout;
* type-1 sum on Nout x Nout outputs with offset h (default Nout // 2):
      out[n][m] = sum_l c_l exp(-i 2 pi (ky_l (n - h) + kx_l (m - h)))
  approximated by spreading c onto the grid, a forward 2D DFT of the grid
  and division by phi_hat((n - h)/G) phi_hat((m - h)/G).  By Poisson
  summation the error is the aliased part of phi_hat, small when the
  outputs stay within |n - h| <= Nout/2 << G/2.
"""
from __future__ import annotations

import math

import numpy as np

from . import nudft


def kb_beta(W: int, sigma: float) -> float:
    """Kaiser-Bessel shape for width W (grid points) at oversampling sigma."""
    return math.pi * math.sqrt((W / sigma) ** 2 * (sigma - 0.5) ** 2 - 0.8)


def kb(t, W: int, beta: float):
    t = np.asarray(t, dtype=np.float64)
    a = 1.0 - (2.0 * t / W) ** 2
    out = np.zeros_like(t)
    inside = a >= 0.0
    out[inside] = np.i0(beta * np.sqrt(a[inside]))
    return out


def kb_hat(nu, W: int, beta: float):
    """Continuous Fourier transform of kb (closed form)."""
    nu = np.asarray(nu, dtype=np.float64)
    z2 = beta * beta - (math.pi * W * nu) ** 2
    out = np.empty_like(nu)
    pos = z2 > 1e-12
    neg = z2 < -1e-12
    mid = ~(pos | neg)
    z = np.sqrt(z2[pos])
    out[pos] = W * np.sinh(z) / z
    z = np.sqrt(-z2[neg])
    out[neg] = W * np.sin(z) / z
    out[mid] = W
    return out


def spread(k, c, G: int, W: int, beta: float):
    """grid[g1][g2] = sum_l c_l phi(g1 - G ky_l) phi(g2 - G kx_l), g mod G.
    c: [..., M] complex; returns [..., G, G]."""
    c = np.asarray(c, dtype=np.complex128)
    grid = np.zeros(c.shape[:-1] + (G, G), dtype=np.complex128)
    offs = np.arange(W)
    for l in range(k.shape[0]):
        uy, ux = G * k[l, 1], G * k[l, 0]
        gy = np.floor(uy - W / 2.0) + 1 + offs          # the W grid points with |g - u| < W/2
        gx = np.floor(ux - W / 2.0) + 1 + offs
        wy = kb(gy - uy, W, beta)
        wx = kb(gx - ux, W, beta)
        iy = gy.astype(np.int64) % G
        ix = gx.astype(np.int64) % G
        grid[..., iy[:, None], ix[None, :]] += c[..., l, None, None] * np.outer(wy, wx)
    return grid


def interp(k, grid, W: int, beta: float):
    """The adjoint of ``spread`` (real kernel): out_l = sum_g phi2(g - u_l) grid[g]."""
    G = grid.shape[-1]
    out = np.zeros(grid.shape[:-2] + (k.shape[0],), dtype=np.complex128)
    offs = np.arange(W)
    for l in range(k.shape[0]):
        uy, ux = G * k[l, 1], G * k[l, 0]
        gy = np.floor(uy - W / 2.0) + 1 + offs
        gx = np.floor(ux - W / 2.0) + 1 + offs
        wy = kb(gy - uy, W, beta)
        wx = kb(gx - ux, W, beta)
        iy = gy.astype(np.int64) % G
        ix = gx.astype(np.int64) % G
        out[..., l] = np.sum(grid[..., iy[:, None], ix[None, :]] * np.outer(wy, wx),
                             axis=(-2, -1))
    return out


def type1(k, c, Nout: int, G: int, W: int, beta: float | None = None, h: int | None = None):
    """out[n][m] ~ sum_l c_l exp(-i 2 pi (ky_l (n - h) + kx_l (m - h)))."""
    if beta is None:
        beta = kb_beta(W, G / Nout)
    if h is None:
        h = Nout // 2
    grid = spread(k, c, G, W, beta)
    F = np.fft.fft2(grid, axes=(-2, -1))
    n = np.arange(Nout) - h
    idx = n % G
    corr = 1.0 / kb_hat(n / G, W, beta)
    return F[..., idx[:, None], idx[None, :]] * np.outer(corr, corr)


def type1_exact(k, c, Nout: int, h: int | None = None):
    """The sum type1 approximates, by direct summation (reference)."""
    if h is None:
        h = Nout // 2
    n = np.arange(Nout) - h
    Ey = np.exp(-2j * np.pi * np.outer(k[:, 1], n))     # [M, Nout]
    Ex = np.exp(-2j * np.pi * np.outer(k[:, 0], n))
    c = np.asarray(c, dtype=np.complex128)
    return np.einsum("...l,ln,lm->...nm", c, Ey, Ex)


def adjoint_nufft(y, k, N: int, G: int | None = None, W: int = 7, beta: float | None = None,
                  w=None):
    """b[n][m] = (1/N) sum_l w_l y_l exp(-i 2 pi (kx_l m + ky_l n)) by type1
    (Eq. AnnMatGD with density weights w, 1 by default): the sample phase
    exp(-i 2 pi (kx + ky) h) moves the outputs to n - h."""
    G = 2 * N if G is None else G
    h = N // 2
    y = np.asarray(y, dtype=np.complex128)
    c = y * np.exp(-2j * np.pi * (k[:, 0] + k[:, 1]) * h) / N
    if w is not None:
        c = c * w
    return type1(k, c, N, G, W, beta, h)


def lag_kernel_nufft(k, N: int, G: int | None = None, W: int = 7, beta: float | None = None):
    """The Gram lag kernel h[a][b] = (1/N^2) sum_l exp(-i 2 pi (ky a + kx b)),
    a, b in [-(N-1), N-1] (gram.lag_kernel), by type1 on 2N outputs with
    offset N; returned as [a + N-1][b + N-1]."""
    G = 4 * N if G is None else G
    c = np.full(k.shape[0], 1.0 / (N * N), dtype=np.complex128)
    out = type1(k, c, 2 * N, G, W, beta, N)
    return out[1:, 1:]


def density_weights(k, N: int, iters: int, G: int | None = None, W: int = 7,
                    beta: float | None = None):
    """Sampling-density compensation by the fixed-point iteration of Pipe and
    Menon (the paper's [Pipe99]): w <- w / (I S w), S = spread, I = its
    adjoint, from w = 1; then scaled by phi_hat(0)^4 / sigma^2 (sigma = G/N),
    the factor that gives weight 1 to a sample of a uniform Cartesian grid of
    spacing 1/N (for uniform density rho, I S w = w rho phi_hat(0)^4 / G^2)."""
    G = 2 * N if G is None else G
    sigma = G / N
    if beta is None:
        beta = kb_beta(W, sigma)
    w = np.ones(k.shape[0])
    for _ in range(iters):
        d = interp(k, spread(k, w.astype(np.complex128), G, W, beta), W, beta).real
        w = w / d
    return w * kb_hat(np.array([0.0]), W, beta)[0] ** 4 / sigma ** 2


def gridding_recon(y, k, N: int, w, G: int | None = None, W: int = 7,
                   beta: float | None = None):
    """Section 1's gridding reconstruction: density weights, KB resampling,
    FFT, apodization correction (= the weighted adjoint by type1)."""
    return adjoint_nufft(y, k, N, G, W, beta, w=w)


def roi_metrics(x, x_ref, roi1, roi2):
    """Section 4.1's figures of merit: the quadratic error sum |x - x_ref|^2
    over ROI1 (divided by its pixel count) and the variance of x over the
    flat region ROI2 (mean |x - mean x|^2).  roi1, roi2: boolean masks."""
    x = np.asarray(x)
    e = np.abs(x - x_ref) ** 2
    q = float(e[roi1].mean())
    v = x[roi2]
    return q, float(np.mean(np.abs(v - v.mean()) ** 2))


def exact_adjoint(y, k, N, w=None):
    """Weighted exact adjoint (1/N) sum_l w_l y_l exp(-i 2 pi (kx m + ky n))."""
    y = np.asarray(y, dtype=np.complex128)
    return nudft.adjoint(y if w is None else y * w, k, N)
