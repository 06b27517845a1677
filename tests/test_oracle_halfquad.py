"""Pins of the oracle's half-quadratic minimiser (Section 5's dual /
half-quadratic alternative to the conjugate gradient).

Each inner problem is a quadratic whose minimiser has a dense closed form;
the outer iterations must decrease J monotonically (majorise-minimise) and
reach the same unique minimiser (Section 3.3: J is strictly convex) as the
pseudo-conjugate gradient and an independent quasi-Newton solver.
"""
import numpy as np
import pytest

import oracle
from oracle import criterion, halfquad, penalty, solver


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _case(seed=5, N=5, M=40):
    rng = np.random.default_rng(seed)
    k = rng.uniform(-0.5, 0.5, size=(M, 2))
    y = rand_c(rng, M)
    xbar = rand_c(rng, N, N)
    return k, y, N, xbar


def _inner_pin_error(kind, lam0):
    """Relative max error of one outer iteration with 2 N^2 + 10 inner steps
    (linear CG, enough to solve the quadratic) against the dense solve."""
    k, y, N, xbar = _case()
    lam, delta, alpha0 = 0.3, 0.2, 0.5
    ref = halfquad.surrogate_minimiser_dense(y, k, N, xbar, lam, delta, kind, lam0=lam0,
                                             alpha0=alpha0)
    x = halfquad.solve(oracle.adjoint(y, k, N), oracle.khat(k, N, 2 * N), lam, delta, 1,
                       2 * N * N + 10, kind, x0=xbar, lam0=lam0, alpha0=alpha0)
    return float(np.abs(x - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("kind", ["hyperbolic", "huber"])
@pytest.mark.parametrize("lam0", [0.0, 0.2])
def test_inner_problem_is_the_dense_surrogate_minimiser(kind, lam0):
    assert _inner_pin_error(kind, lam0) < 1e-10


def test_outer_iterations_decrease_J_and_reach_the_minimiser():
    k, y, N, _ = _case()
    lam, delta = 0.3, 0.2
    b = oracle.adjoint(y, k, N)
    K = oracle.khat(k, N, 2 * N)
    trace = []
    x = halfquad.solve(b, K, lam, delta, 60, 8, trace=trace)
    J = np.array([criterion.J_direct(t["x"], y, k, lam, delta) for t in trace])
    assert np.all(np.diff(J) <= 1e-12 * abs(J[0]))
    assert trace[-1]["applies"] == 60 * 8
    xs = solver.solve(b, K, lam, delta, 800)
    np.testing.assert_allclose(x, xs, atol=1e-10 * np.abs(xs).max())


def test_planted_half_quadratic_mistakes_are_caught(monkeypatch):
    """Weights recomputed from the moving image instead of frozen, and the
    surrogate's weight taken without its factor 1/2, each fail a pin."""
    delta = 0.2
    with monkeypatch.context() as mp:
        mp.setattr(halfquad, "surrogate_grad",
                   lambda x, r, W, lam, lam0=0.0: 2.0 * r + lam * penalty.smooth_grad(x, delta))
        assert _inner_pin_error("hyperbolic", 0.0) > 1e-4
    orig = halfquad.surrogate_grad
    with monkeypatch.context() as mp:
        mp.setattr(halfquad, "surrogate_grad",
                   lambda x, r, W, lam, lam0=0.0: orig(x, r, W, 2.0 * lam, lam0))
        assert _inner_pin_error("hyperbolic", 0.0) > 1e-4
