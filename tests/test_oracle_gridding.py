"""Pins of the oracle's gridding / NUFFT module (Section 1's four gridding
steps with Section 4.1's Kaiser-Bessel kernel; Section 5's NUFFT
precomputation of D and of the Gram kernel).

* the kernel's closed-form transform against numerical quadrature;
* spread and interpolation are adjoint;
* the type-1 sum against direct summation, within the bound set by the
  kernel's edge jump: the truncated Kaiser-Bessel kernel jumps from 1 to 0
  at |t| = W/2 while its peak is I0(beta), so its transform has a slowly
  decaying tail of relative size ~1/I0(beta) that aliases into the
  passband; the relative L2 error is held to 4 / I0(beta);
* the NUFFT forms of D = A^H y and of the lag kernel against the exact
  sums (same bound), on random and full Cartesian trajectories;
* the density weights of the Pipe-Menon iteration: the fixed point
  I S w = 1 is approached, uniform Cartesian sampling gets weights ~1,
  radial sampling gets weights ~ |k| (its density falls as 1/|k|);
* the ROI figures of merit on a hand-worked example;
* planted mistakes (phase offset of the wrong sign, no apodization
  correction, transposed kernel weights) fail these pins.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import gram, gridding as gr


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def bound(W, sigma=2.0):
    return 4.0 / float(np.i0(gr.kb_beta(W, sigma)))


@pytest.mark.parametrize("W", [5, 7, 11])
def test_kb_transform_closed_form(W):
    from scipy.integrate import quad
    beta = gr.kb_beta(W, 2.0)
    for nu in (0.0, 0.07, 0.21, 0.5, 0.93, 1.7):
        num, _ = quad(lambda t: float(gr.kb(np.array([t]), W, beta)[0]) * math.cos(2 * math.pi * nu * t),
                      -W / 2, W / 2, limit=200, epsabs=1e-13, epsrel=1e-13)
        ref = float(gr.kb_hat(np.array([nu]), W, beta)[0])
        assert abs(num - ref) <= 1e-9 * abs(gr.kb_hat(np.array([0.0]), W, beta)[0]), (nu, num, ref)


def test_spread_and_interp_are_adjoint():
    rng = np.random.default_rng(2)
    k = rng.uniform(-0.5, 0.5, (40, 2))
    c = rand_c(rng, 40)
    G, W = 32, 7
    beta = gr.kb_beta(W, 2.0)
    g = rand_c(rng, G, G)
    lhs = np.vdot(gr.spread(k, c, G, W, beta), g)
    rhs = np.vdot(c, gr.interp(k, g, W, beta))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("W", [5, 7, 9, 11])
def test_type1_within_edge_bound(W):
    rng = np.random.default_rng(W)
    k = rng.uniform(-0.5, 0.5, (300, 2))
    c = rand_c(rng, 300)
    for Nout, h in ((16, 8), (15, 7)):   # outputs within |n - h| <= Nout/2 (the passband)
        out = gr.type1(k, c, Nout, 2 * Nout, W, h=h)
        ref = gr.type1_exact(k, c, Nout, h=h)
        assert rel(out, ref) < bound(W), (W, Nout, rel(out, ref))


@pytest.mark.parametrize("W", [7, 11])
def test_nufft_adjoint_and_lag_kernel_against_exact_sums(W):
    rng = np.random.default_rng(30 + W)
    N, M = 16, 500
    k = rng.uniform(-0.5, 0.5, (M, 2))
    y = rand_c(rng, 2, M)
    b = oracle.adjoint(y, k, N)
    bn = gr.adjoint_nufft(y, k, N, W=W)
    assert rel(bn, b) < bound(W)
    h = gram.lag_kernel(k, N)
    hn = gr.lag_kernel_nufft(k, N, W=W)
    assert rel(hn, h) < bound(W)


def test_cartesian_adjoint_is_the_inverse_dft():
    """Section 3.1: on the full Cartesian grid A^H A = I; the NUFFT adjoint of
    A x returns x within the bound."""
    N = 12
    p = np.arange(-N // 2, N // 2)
    P, Q = np.meshgrid(p, p, indexing="ij")
    k = np.stack([P.ravel() / N, Q.ravel() / N], axis=1)
    rng = np.random.default_rng(4)
    x = rand_c(rng, N, N)
    xb = gr.adjoint_nufft(oracle.forward(x, k), k, N, W=9)
    assert rel(xb, x) < bound(9)


def test_density_weights():
    N = 16
    # fixed point approached
    rng = np.random.default_rng(6)
    k = rng.uniform(-0.45, 0.45, (400, 2))
    G, W = 2 * N, 7
    beta = gr.kb_beta(W, 2.0)
    res = []
    for it in (1, 5, 20):
        w = gr.density_weights(k, N, it)
        scale = gr.kb_hat(np.array([0.0]), W, beta)[0] ** 4 / 4.0
        isw = gr.interp(k, gr.spread(k, (w / scale).astype(complex), G, W, beta), W, beta).real
        res.append(np.median(np.abs(isw - 1.0)))
    assert res[2] < res[1] < res[0] and res[2] < 0.01, res
    # uniform Cartesian sampling: weights ~ 1
    p = np.arange(-N // 2, N // 2)
    P, Q = np.meshgrid(p, p, indexing="ij")
    kc = np.stack([P.ravel() / N, Q.ravel() / N], axis=1)
    wc = gr.density_weights(kc, N, 20)
    assert abs(np.median(wc) - 1.0) < 0.01, np.median(wc)
    # radial sampling (density ~ 1/|k|): weights ~ |k| away from the centre
    ang = np.arange(64) * np.pi / 64
    rad = (np.arange(32) - 15.5) / 32
    kr = np.stack([np.outer(np.cos(ang), rad).ravel(), np.outer(np.sin(ang), rad).ravel()], 1)
    wr = gr.density_weights(kr, N, 20)
    kk = np.hypot(kr[:, 0], kr[:, 1])
    mid = (kk > 0.12) & (kk < 0.38)
    ratio = wr[mid] / kk[mid]
    assert np.std(ratio) / np.mean(ratio) < 0.05, np.std(ratio) / np.mean(ratio)


def test_roi_metrics_hand_example():
    x = np.array([[1, 2], [3, 4 + 1j]], dtype=complex)
    ref = np.array([[1, 1], [1, 1]], dtype=complex)
    r1 = np.array([[True, True], [False, False]])
    r2 = np.array([[False, True], [True, False]])
    q, v = gr.roi_metrics(x, ref, r1, r2)
    assert q == pytest.approx((0 + 1) / 2)
    assert v == pytest.approx(((2 - 2.5) ** 2 + (3 - 2.5) ** 2) / 2)


def test_planted_gridding_mistakes_are_caught(monkeypatch):
    rng = np.random.default_rng(8)
    N, M, W = 16, 300, 9
    k = rng.uniform(-0.5, 0.5, (M, 2))
    y = rand_c(rng, M)
    b = oracle.adjoint(y, k, N)
    h = N // 2
    # phase offset with the wrong sign
    c = y * np.exp(+2j * np.pi * (k[:, 0] + k[:, 1]) * h) / N
    assert rel(gr.type1(k, c, N, 2 * N, W, h=h), b) > 1e-2
    # no apodization correction
    with monkeypatch.context() as mp:
        mp.setattr(gr, "kb_hat", lambda nu, W, beta: np.ones_like(np.asarray(nu, dtype=float)))
        assert rel(gr.adjoint_nufft(y, k, N, W=W), b) > 1e-2
    # transposed kernel weights in the interpolation
    orig = gr.kb
    beta = gr.kb_beta(W, 2.0)
    g = rand_c(rng, 2 * N, 2 * N)
    lhs = np.vdot(gr.spread(k, y, 2 * N, W, beta), g)
    with monkeypatch.context() as mp:
        mp.setattr(gr, "kb", lambda t, W_, beta_: orig(np.asarray(t)[::-1], W_, beta_))
        rhs = np.vdot(y, gr.interp(k, g, W, beta))
    assert abs(lhs - rhs) > 1e-6 * abs(lhs)
