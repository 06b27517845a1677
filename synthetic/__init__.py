"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module draws *inputs only*: k-space trajectories, ellipse phantoms and
unit-variance noise draws.  It holds none of the reconstruction arithmetic
(no Fourier operator, no Gram kernel, no penalty), so that the oracle and the
HIP path can both consume the same inputs without sharing any method code.

The paper's own data sets (the simulated two-vessel phantom of Section 4.1 and
the GEMS phantom acquisition of Section 4.2) are not available; the recipes
below stand in for them with the shapes the paper and the workload
configurations use (interleaved spirals, k normalised to [-0.5, 0.5],
complex images on an N x N grid, complex white Gaussian noise, Section 2).

Conventions (Section 2, Eq. ModDirect): the image x is stored row-major as
x[n, m], row n paired with k_y and column m paired with k_x; a trajectory is
an array k of shape [M, 2] holding (k_x, k_y) per sample in cycles/pixel.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "spiral_trajectory",
    "ellipse_phantom",
    "noise_draws",
    "Problem",
    "make_problem",
    "make_frames",
    "serving_requests",
    "CONFIGS",
]


def spiral_trajectory(N: int, interleaves: int, samples: int, R: float = 1.0,
                      density: str = "clv") -> np.ndarray:
    """Archimedean interleaved spiral, k in cycles/pixel with |k| < 0.5.

    Interleave j in [0, I), sample s in [0, S); sample index l = j*S + s.
    radius r = 0.5*tau, angle theta = 2*pi*T*tau + 2*pi*j/I, with T = N/(2*I*R)
    turns so that adjacent arms are R/N apart radially (R = angular
    undersampling factor).  density 'clv' (uniform density): tau = sqrt(s/S);
    'cav' (density ~ 1/|k|): tau = s/S.

    Returns float64 array [M, 2] of (k_x, k_y).
    """
    if interleaves < 1 or samples < 1 or N < 2:
        raise ValueError("need N >= 2, interleaves >= 1, samples >= 1")
    I, S = int(interleaves), int(samples)
    T = N / (2.0 * I * R)
    s = np.arange(S, dtype=np.float64) / S
    if density == "clv":
        tau = np.sqrt(s)
    elif density == "cav":
        tau = s
    else:
        raise ValueError(f"unknown density {density!r}")
    j = np.arange(I, dtype=np.float64)[:, None]
    theta = 2.0 * math.pi * T * tau[None, :] + 2.0 * math.pi * j / I
    r = 0.5 * tau[None, :]
    k = np.empty((I, S, 2), dtype=np.float64)
    k[..., 0] = r * np.cos(theta)
    k[..., 1] = r * np.sin(theta)
    return k.reshape(I * S, 2)


def ellipse_phantom(N: int, K: int, rng: np.random.Generator,
                    drift: float = 0.0, drift_dirs: Optional[np.ndarray] = None
                    ) -> np.ndarray:
    """Sum of K random ellipses, each with a constant complex value.

    centre = N/2 + U(-0.3N, 0.3N)^2, semi-axes U(0.05N, 0.25N)^2,
    rotation U(0, pi), amplitude U(0.1, 1), phase U(0, 2pi).  Pixel (n, m) has
    position (x = m, y = n) and receives amp*exp(i*phase) of every ellipse that
    contains it.  ``drift`` (pixels) shifts every centre by drift*u_e where u_e
    is the ellipse's unit vector from ``drift_dirs`` [K, 2].

    Returns complex128 [N, N].
    """
    cx = N / 2 + rng.uniform(-0.3 * N, 0.3 * N, size=K)
    cy = N / 2 + rng.uniform(-0.3 * N, 0.3 * N, size=K)
    ax = rng.uniform(0.05 * N, 0.25 * N, size=K)
    ay = rng.uniform(0.05 * N, 0.25 * N, size=K)
    rot = rng.uniform(0.0, math.pi, size=K)
    amp = rng.uniform(0.1, 1.0, size=K)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=K)
    if drift and drift_dirs is not None:
        cx = cx + drift * drift_dirs[:, 0]
        cy = cy + drift * drift_dirs[:, 1]
    img = np.zeros((N, N), dtype=np.complex128)
    for e in range(K):
        c, s = math.cos(rot[e]), math.sin(rot[e])
        # Only pixels inside the ellipse's bounding box (plus a one-pixel
        # margin) can satisfy the test; the test itself is unchanged.
        hx = math.hypot(ax[e] * c, ay[e] * s) + 1.0
        hy = math.hypot(ax[e] * s, ay[e] * c) + 1.0
        m0, m1 = max(0, int(math.floor(cx[e] - hx))), min(N, int(math.ceil(cx[e] + hx)) + 1)
        n0, n1 = max(0, int(math.floor(cy[e] - hy))), min(N, int(math.ceil(cy[e] + hy)) + 1)
        if m0 >= m1 or n0 >= n1:
            continue
        yy, xx = np.meshgrid(np.arange(n0, n1, dtype=np.float64),
                             np.arange(m0, m1, dtype=np.float64), indexing="ij")
        dx, dy = xx - cx[e], yy - cy[e]
        u = (c * dx + s * dy) / ax[e]
        v = (-s * dx + c * dy) / ay[e]
        inside = (u * u + v * v) <= 1.0
        img[n0:n1, m0:m1][inside] += amp[e] * complex(math.cos(ph[e]), math.sin(ph[e]))
    return img


def noise_draws(M: int, rng: np.random.Generator) -> np.ndarray:
    """Unit complex Gaussian draws xi + i*eta (xi, eta ~ N(0, 1) iid), [M]."""
    z = rng.standard_normal((2, M))
    return z[0] + 1j * z[1]


@dataclass
class Problem:
    """One reconstruction problem's inputs (no measured data yet).

    The measured data are y = y0 + sigma*noise with y0 the exact forward model
    of ``x_true`` and sigma = noise_c * max|y0|; forming y0 needs the Fourier
    operator, which each side (oracle or GPU) applies itself.
    """
    name: str
    N: int
    k: np.ndarray                  # [M, 2] float64 (kx, ky)
    x_true: np.ndarray             # [F, N, N] complex128
    noise: np.ndarray              # [F, M] complex128 unit draws
    noise_c: float
    lam: float
    delta: float
    iters: int
    L: int
    extra: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.k.shape[0])

    @property
    def frames(self) -> int:
        return int(self.x_true.shape[0])

    def measured(self, y0: np.ndarray) -> np.ndarray:
        """y = y0 + sigma*noise, sigma = noise_c*max|y0| per frame."""
        y0 = np.asarray(y0)
        sig = self.noise_c * np.abs(y0).max(axis=-1, keepdims=True)
        return y0 + sig * self.noise[: y0.shape[0]]


# Workload recipes (image size, spiral, phantom, noise, penalty, iterations).
CONFIGS = {
    1: dict(name="tiny", N=32, K=10, I=4, S=256, R=1.0, density="clv",
            c=0.01, delta=0.05, lam=0.02, iters=200, L=64, frames=1, drift=0.0),
    2: dict(name="plain256", N=256, K=40, I=16, S=2048, R=2.0, density="clv",
            c=0.02, delta=0.02, lam=0.01, iters=300, L=512, frames=1, drift=0.0),
    3: dict(name="series256", N=256, K=40, I=16, S=2048, R=2.0, density="clv",
            c=0.02, delta=0.02, lam=0.01, iters=300, L=512, frames=128, drift=2.0),
    5: dict(name="large512", N=512, K=40, I=64, S=4096, R=1.0, density="cav",
            c=0.02, delta=0.01, lam=0.005, iters=500, L=1024, frames=32, drift=2.0),
}


def make_frames(cfg: int, frames: Optional[int] = None, first: int = 0,
                **overrides) -> Problem:
    """Inputs of workload ``cfg`` for frames [first, first+frames).

    Frame f of a series draws its phantom from default_rng([cfg, f]) with every
    ellipse centre shifted by drift*(f/(F-1))*u_e (u_e seeded unit vectors
    from default_rng([cfg, 99991])), then its noise from the same generator.
    Single-frame workloads use default_rng(cfg): phantom first, then noise.
    """
    p = dict(CONFIGS[cfg])
    p.update(overrides)
    N = p["N"]
    k = spiral_trajectory(N, p["I"], p["S"], p["R"], p["density"])
    M = k.shape[0]
    F_total = p["frames"]
    F = F_total - first if frames is None else frames
    xs, ns = [], []
    if F_total == 1 and first == 0 and F == 1:
        rng = np.random.default_rng(cfg)
        xs.append(ellipse_phantom(N, p["K"], rng))
        ns.append(noise_draws(M, rng))
    else:
        drng = np.random.default_rng([cfg, 99991])
        ang = drng.uniform(0.0, 2.0 * math.pi, size=p["K"])
        dirs = np.stack([np.cos(ang), np.sin(ang)], axis=1)
        denom = max(F_total - 1, 1)
        for f in range(first, first + F):
            rng = np.random.default_rng([cfg, f])
            xs.append(ellipse_phantom(N, p["K"], rng,
                                      drift=p["drift"] * f / denom,
                                      drift_dirs=dirs))
            ns.append(noise_draws(M, rng))
    return Problem(name=p["name"], N=N, k=k, x_true=np.stack(xs),
                   noise=np.stack(ns), noise_c=p["c"], lam=p["lam"],
                   delta=p["delta"], iters=p["iters"], L=p["L"],
                   extra=dict(cfg=cfg, first=first))


def make_problem(cfg: int, **overrides) -> Problem:
    """All frames of workload ``cfg`` (single-frame workloads: one frame)."""
    return make_frames(cfg, **overrides)


def serving_requests(count: int, rate: float, seed: int = 4):
    """Poisson stream of serving requests (workload 4).

    Request i draws from default_rng([seed, i]): N ~ U{64,128,192,256,384},
    interleaves ~ U{8,16,32}, S = N^2/16 samples per interleave, R = 2, uniform
    density, K = 20 ellipses, lambda ~ U[0.005, 0.05], delta ~ U[0.01, 0.1],
    noise c = 0.01, 300 iterations, L = 2N.  Arrival gaps are exponential with
    mean 1/rate, drawn from default_rng([seed, 'gaps'-stream]).
    Yields dicts with arrival time and inputs (trajectory keyed by (N, I)).
    """
    grng = np.random.default_rng([seed, 7777777])
    t = 0.0
    out = []
    for i in range(count):
        t += grng.exponential(1.0 / rate)
        rng = np.random.default_rng([seed, i])
        N = int(rng.choice([64, 128, 192, 256, 384]))
        I = int(rng.choice([8, 16, 32]))
        lam = float(rng.uniform(0.005, 0.05))
        delta = float(rng.uniform(0.01, 0.1))
        S = N * N // 16
        x = ellipse_phantom(N, 20, rng)
        nz = noise_draws(I * S, rng)
        out.append(dict(id=i, arrival=t, N=N, I=I, S=S, R=2.0, lam=lam,
                        delta=delta, iters=300, L=2 * N, noise_c=0.01,
                        x_true=x, noise=nz))
    return out


def roi_masks(x_true: np.ndarray, radius: int = 2):
    """Regions of interest of a phantom for the gridding comparison (the
    paper's ROI1, a central square, and ROI2, a region of constant value).

    ROI1: the central square of side N/4.  ROI2: the pixels whose whole
    (2 radius + 1)^2 neighbourhood holds one non-zero value, restricted to
    the value that covers the most such pixels (a flat interior region of
    the piecewise-constant phantom).  Returns two boolean [N, N] masks."""
    N = x_true.shape[-1]
    roi1 = np.zeros((N, N), dtype=bool)
    a = N // 2 - N // 8
    roi1[a:a + N // 4, a:a + N // 4] = True
    flat = x_true != 0
    for dn in range(-radius, radius + 1):
        for dm in range(-radius, radius + 1):
            sh = np.roll(np.roll(x_true, dn, axis=0), dm, axis=1)
            flat &= sh == x_true
    flat[:radius, :] = flat[-radius:, :] = False
    flat[:, :radius] = flat[:, -radius:] = False
    vals, counts = np.unique(x_true[flat], return_counts=True)
    roi2 = flat & (x_true == vals[np.argmax(counts)]) if len(vals) else flat
    return roi1, roi2
