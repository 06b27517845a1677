"""Pins of the FP64 oracle against facts fixed by the paper and mathematics.

Each test names the passage it follows.  None of them re-types the oracle's
own formula: they use hand-worked values, library routines on special cases
(numpy's 2D DFT), explicit dense matrices, invariants (adjoint identity,
symmetry), closed forms (Dirichlet spectrum of the Gram kernel), finite
differences, a dense linear solve and an independent quasi-Newton minimiser.
"""
import cmath
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import criterion, gram, nudft, penalty, solver, toeplitz
import synthetic

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rand_k(rng, M):
    return rng.uniform(-0.5, 0.5, size=(M, 2))


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ---------------------------------------------------------------- forward model

def test_hand_worked_n2():
    """Section 2 Eq. ModDirect, Appendix A Eqs. AnnMatGD / AnnMatG, by hand."""
    g = json.load(open(os.path.join(GOLD, "hand_n2.json")))
    k = np.array(g["k"], dtype=np.float64)
    x = np.array(g["x_re"]) + 1j * np.array(g["x_im"])
    y = oracle.forward(x, k)
    np.testing.assert_allclose(y, np.array(g["y_re"]) + 1j * np.array(g["y_im"]),
                               atol=1e-15)
    s = np.array(g["s_re"]) + 1j * np.array(g["s_im"])
    D = oracle.adjoint(s, k, g["N"])
    np.testing.assert_allclose(D, np.array(g["D_re"]) + 1j * np.array(g["D_im"]),
                               atol=1e-15)
    G = oracle.paper_G(k, g["N"])
    np.testing.assert_allclose(G, np.array(g["G_re"]) + 1j * np.array(g["G_im"]),
                               atol=1e-15)


def test_forward_bruteforce_loops():
    """Eq. ModDirect summed with pure-Python loops on a tiny case."""
    rng = np.random.default_rng(1)
    N, M = 3, 5
    k = rand_k(rng, M)
    x = rand_c(rng, N, N)
    y = oracle.forward(x, k)
    for l in range(M):
        s = 0j
        for n in range(N):
            for m in range(N):
                s += x[n, m] * cmath.exp(2j * math.pi * (k[l, 0] * m + k[l, 1] * n))
        assert abs(y[l] - s / N) < 1e-14


@pytest.mark.parametrize("N,M", [(4, 9), (8, 200), (16, 1000)])
def test_P1_adjoint_identity(N, M):
    """<A x, y> = <x, A^H y> (Appendix A.2: D is the adjoint of the model)."""
    rng = np.random.default_rng(N)
    k = rand_k(rng, M)
    x = rand_c(rng, 2, N, N)
    y = rand_c(rng, 2, M)
    lhs = np.sum(np.conj(oracle.forward(x, k)) * y, axis=-1)
    rhs = np.sum(np.conj(x) * oracle.adjoint(y, k, N), axis=(-2, -1))
    np.testing.assert_allclose(lhs, rhs, rtol=1e-13)


def cart_grid(N):
    p = np.arange(-N // 2, N // 2)
    P, Qg = np.meshgrid(p, p, indexing="ij")      # P: kx index, Qg: ky index
    k = np.stack([P.reshape(-1) / N, Qg.reshape(-1) / N], axis=1)
    return k, P.reshape(-1), Qg.reshape(-1)


@pytest.mark.parametrize("N", [4, 8, 6])
def test_P2_full_cartesian_is_dft(N):
    """Section 3.1: on the complete Cartesian grid H is the (inverse) DFT
    matrix, H^H H = I, so G is a delta and the Gram spectrum is 1."""
    rng = np.random.default_rng(3)
    k, P, Qg = cart_grid(N)
    x = rand_c(rng, N, N)
    y = oracle.forward(x, k)
    ref = np.fft.ifft2(x, norm="ortho")
    np.testing.assert_allclose(y, ref[Qg % N, P % N], atol=1e-13)
    H = oracle.dense_matrix(k, N)
    np.testing.assert_allclose(H.conj().T @ H, np.eye(N * N), atol=1e-13)
    h = gram.lag_kernel(k, N)
    delta = np.zeros_like(h)
    delta[N - 1, N - 1] = 1.0
    np.testing.assert_allclose(h, delta, atol=1e-13)
    for L in (2 * N - 1, 2 * N):
        np.testing.assert_allclose(gram.khat(k, N, L), np.ones((L, L)), atol=1e-13)
        np.testing.assert_allclose(
            toeplitz.apply_gram(x, gram.khat(k, N, L), N), x, atol=1e-13)


@pytest.mark.parametrize("N", [2, 3, 5, 8])
def test_P3_toeplitz_equals_dense_gram(N):
    """Section 3.4 / Appendix B: the FFT evaluation of the Gram operator equals
    the explicit A^H A, for any zero padding L >= 2N-1."""
    rng = np.random.default_rng(10 + N)
    k = rand_k(rng, 3 * N * N)
    Qd = toeplitz.dense_gram(k, N)
    v = rand_c(rng, N, N)
    ref = (Qd @ v.reshape(-1)).reshape(N, N)
    for L in (2 * N - 1, 2 * N, 2 * N + 3):
        K = gram.khat(k, N, L)
        np.testing.assert_allclose(toeplitz.apply_gram(v, K, N), ref,
                                   rtol=0, atol=1e-12 * np.abs(ref).max())
    with pytest.raises(ValueError):
        gram.khat(k, N, 2 * N - 2)


def test_P4_criterion_rewriting():
    """Eq. NewCritLS and Appendix A: ||y - Ax||^2 = ||y||^2 - 2Re<x,D> + sum C G,
    with C the image correlation (brute-force loops) and G from Eq. AnnMatG."""
    rng = np.random.default_rng(4)
    N, M = 5, 40
    k = rand_k(rng, M)
    x = rand_c(rng, N, N)
    y = rand_c(rng, M)
    C = criterion.image_correlation(x)
    G = oracle.paper_G(k, N)
    yx = oracle.forward(x, k)
    np.testing.assert_allclose(np.sum(np.abs(yx) ** 2), np.sum(C * G).real,
                               rtol=1e-12)
    assert abs(np.sum(C * G).imag) < 1e-10
    b = oracle.adjoint(y, k, N)
    K = oracle.khat(k, N, 2 * N)
    Qx = oracle.apply_gram(x, K, N)
    lhs = np.sum(np.abs(y - yx) ** 2)
    rhs = (np.sum(np.abs(y) ** 2) - 2 * np.real(np.sum(np.conj(x) * b))
           + np.sum(C * G).real)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)
    Jd = criterion.J_direct(x, y, k, 0.3, 0.1)
    Jr = criterion.J_rewritten(x, np.sum(np.abs(y) ** 2), b, Qx, 0.3, 0.1)
    np.testing.assert_allclose(Jd, Jr, rtol=1e-12)


def dirichlet(theta, N):
    """sum_{a=-(N-1)}^{N-1} exp(-i 2 pi a theta) = sin((2N-1) pi t)/sin(pi t)."""
    theta = np.asarray(theta, dtype=np.float64)
    s = np.sin(np.pi * theta)
    out = np.empty_like(theta)
    small = np.abs(s) < 1e-12
    out[~small] = np.sin((2 * N - 1) * np.pi * theta[~small]) / s[~small]
    # limit: +-(2N-1) at integer theta (sign (-1)^{theta (2N-2)} = +1)
    out[small] = 2 * N - 1
    return out


@pytest.mark.parametrize("N,L", [(4, 8), (5, 9), (8, 19)])
def test_P5_gram_properties_and_closed_form(N, L):
    """Section 3.4: G depends on the trajectory only, is conjugate
    centro-symmetric (the paper's 'Hermitian symmetry') and G(0,0) = M/N^2;
    its circulant spectrum equals the closed Dirichlet form
    Khat[p, q] = (1/N^2) sum_l Dir(ky_l + p/L) Dir(kx_l + q/L)."""
    rng = np.random.default_rng(5 + N)
    M = 37
    k = rand_k(rng, M)
    h = gram.lag_kernel(k, N)
    G = gram.paper_G(k, N)
    assert abs(h[N - 1, N - 1] - M / N ** 2) < 1e-13
    np.testing.assert_allclose(h[::-1, ::-1], np.conj(h), atol=1e-14)
    # h[a, b] = G[-b, -a]
    np.testing.assert_allclose(h, G[::-1, ::-1].T, atol=1e-14)
    Kc = gram.khat(k, N, L, return_complex=True)
    assert np.abs(Kc.imag).max() < 1e-12 * np.abs(Kc.real).max()
    p = np.arange(L) / L
    U = dirichlet(k[:, 1][:, None] + p[None, :], N)   # [M, L] over p (rows)
    V = dirichlet(k[:, 0][:, None] + p[None, :], N)   # [M, L] over q (cols)
    ref = U.T @ V / N ** 2
    np.testing.assert_allclose(Kc.real, ref, atol=1e-11 * np.abs(ref).max())
    # one sample at k = 0 gives h = 1/N^2 everywhere
    h0 = gram.lag_kernel(np.zeros((1, 2)), N)
    np.testing.assert_allclose(h0, np.full_like(h0, 1 / N ** 2), atol=1e-16)


# ---------------------------------------------------------------- penalty

def test_differences_ramp_and_adjoint():
    """Section 3.3 first-order differences: a ramp a*n + b*m has constant
    differences; D^T is the adjoint of D."""
    N = 7
    n, m = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    x = (0.5 - 2j) * n + (1.5 + 0.25j) * m
    dv, dh = penalty.diff(x)
    assert dv.shape == (N - 1, N) and dh.shape == (N, N - 1)
    np.testing.assert_allclose(dv, np.full(dv.shape, 0.5 - 2j))
    np.testing.assert_allclose(dh, np.full(dh.shape, 1.5 + 0.25j))
    rng = np.random.default_rng(6)
    x = rand_c(rng, N, N)
    tv, th = rand_c(rng, N - 1, N), rand_c(rng, N, N - 1)
    dv, dh = penalty.diff(x)
    lhs = np.sum(np.conj(dv) * tv) + np.sum(np.conj(dh) * th)
    rhs = np.sum(np.conj(x) * penalty.diff_adjoint(tv, th))
    assert abs(lhs - rhs) < 1e-12


def test_penalty_special_values():
    """Huber (Section 3.3) joins x^2 and 2 alpha|x| - alpha^2 continuously at
    alpha; the hyperbolic penalty equals delta at 0 and ~|t| far away."""
    a = 0.7
    s = np.array([0.0, 0.3, a, 2.0])
    np.testing.assert_allclose(penalty.phi(s, a, "huber"),
                               [0.0, 0.09, a * a, 2 * a * 2.0 - a * a])
    np.testing.assert_allclose(penalty.phi(np.array([0.0]), 0.3), [0.3])
    assert abs(penalty.phi(np.array([1e6]), 0.3)[0] - 1e6) < 1e-6
    # weights: phi'(s)/s by central differences
    for kind in penalty.PHIS:
        for s0 in (0.2, 1.3):
            h = 1e-6
            dphi = (penalty.phi(np.array([s0 + h]), a, kind)
                    - penalty.phi(np.array([s0 - h]), a, kind))[0] / (2 * h)
            assert abs(dphi / s0 - penalty.weight(np.array([s0]), a, kind)[0]) < 1e-6


@pytest.mark.parametrize("kind", ["hyperbolic", "huber", "quadratic"])
def test_P6_gradient_finite_differences(kind):
    """Appendix B gradient (2 f*G - 2D) plus the penalty gradient, against
    central differences of J in the real and imaginary part of pixels."""
    rng = np.random.default_rng(7)
    N, M = 6, 60
    k = rand_k(rng, M)
    y = rand_c(rng, M)
    x = rand_c(rng, N, N)
    lam, delta = 0.37, 0.4
    kw = dict(lam0=0.2, alpha0=0.5, kind0="huber")
    b = oracle.adjoint(y, k, N)
    K = oracle.khat(k, N, 2 * N)
    g = criterion.grad(x, b, K, lam, delta, kind, **kw)
    h = 1e-6
    for (n, m) in [(0, 0), (2, 3), (5, 5), (4, 1)]:
        for unit in (1.0, 1j):
            e = np.zeros((N, N), dtype=np.complex128)
            e[n, m] = unit * h
            jp = criterion.J_direct(x + e, y, k, lam, delta, kind, **kw)
            jm = criterion.J_direct(x - e, y, k, lam, delta, kind, **kw)
            fd = (jp - jm) / (2 * h)
            an = g[n, m].real if unit == 1.0 else g[n, m].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (kind, n, m, unit)


# ---------------------------------------------------------------- solver

def test_P7_quadratic_closed_form():
    """Quadratic penalty (Hunt): the minimiser is (A^H A + lam D^T D)^{-1} A^H y
    (Section 3's least-squares closed form with the penalty added)."""
    rng = np.random.default_rng(8)
    N, M = 6, 30
    k = rand_k(rng, M)
    y = rand_c(rng, M)
    lam = 0.05
    ref = solver.solve_quadratic_dense(y, k, N, lam)
    b = oracle.adjoint(y, k, N)
    K = oracle.khat(k, N, 2 * N)
    x = solver.solve(b, K, lam, 1.0, 400, kind="quadratic")
    np.testing.assert_allclose(x, ref, atol=1e-10 * np.abs(ref).max())


def test_mm_step_decreases_and_is_exact_for_quadratic():
    """The majorise-minimise step never increases J; for the quadratic
    penalty it is the exact minimiser along d (zero directional derivative)."""
    rng = np.random.default_rng(9)
    N, M = 8, 90
    k = rand_k(rng, M)
    y = rand_c(rng, M)
    b = oracle.adjoint(y, k, N)
    K = oracle.khat(k, N, 2 * N)
    yy = np.sum(np.abs(y) ** 2)
    for kind in ("hyperbolic", "huber", "quadratic"):
        x = rand_c(rng, N, N)
        r = oracle.apply_gram(x, K, N) - b
        g = 2 * r + criterion.penalty_grad(x, 0.3, 0.2, kind)
        d = -g + 0.3 * rand_c(rng, N, N)
        (x1, r1, g1, d1), sc = solver.step_from_state(x, r, g, d, K, 0.3, 0.2, kind)
        J0 = criterion.J_direct(x, y, k, 0.3, 0.2, kind)
        J1 = criterion.J_direct(x1, y, k, 0.3, 0.2, kind)
        assert J1 < J0
        np.testing.assert_allclose(r1 + b, oracle.apply_gram(x1, K, N), atol=1e-10)
        if kind == "quadratic":
            assert abs(np.real(np.sum(np.conj(g1) * d))) < 1e-9 * np.sum(np.abs(g) ** 2)


def test_P8_monotone_and_vanishing_gradient_tiny_workload():
    """Section 3.3: J is convex with a unique minimum; the iteration decreases
    J monotonically and drives the gradient to zero (32x32 workload)."""
    p = synthetic.make_problem(1)
    y = p.measured(oracle.forward(p.x_true, p.k))[0]
    b = oracle.adjoint(y, p.k, p.N)
    K = oracle.khat(p.k, p.N, p.L)
    x, h = solver.solve(b, K, p.lam, p.delta, p.iters,
                        yy=float(np.sum(np.abs(y) ** 2)), history=True)
    J = np.array(h["J"])
    assert np.all(np.diff(J) <= 1e-12 * abs(J[0]))
    assert h["gnorm"][-1] / h["gnorm"][0] < 1e-8
    # the end point matches the direct criterion evaluation
    np.testing.assert_allclose(J[-1], criterion.J_direct(x, y, p.k, p.lam, p.delta),
                               rtol=1e-10)


def _tiny_hyperbolic(seed=11, N=6, M=40):
    rng = np.random.default_rng(seed)
    k = rand_k(rng, M)
    y = rand_c(rng, M)
    return k, y, N


def test_P9_unique_minimiser_from_two_starts():
    k, y, N = _tiny_hyperbolic()
    lam, delta = 0.2, 0.3
    b = oracle.adjoint(y, k, N)
    K = oracle.khat(k, N, 2 * N)
    xa = solver.solve(b, K, lam, delta, 600)
    xb = solver.solve(b, K, lam, delta, 600, x0=b)
    np.testing.assert_allclose(xa, xb, atol=1e-10 * np.abs(xa).max())


def test_P10_independent_quasi_newton():
    """scipy L-BFGS-B on (Re x, Im x) with the explicit matrix H reaches the
    same minimiser as the pseudo-CG iteration."""
    from scipy.optimize import minimize
    k, y, N = _tiny_hyperbolic()
    lam, delta = 0.2, 0.3
    H = oracle.dense_matrix(k, N)

    def fg(z):
        x = (z[: N * N] + 1j * z[N * N:]).reshape(N, N)
        res = H @ x.reshape(-1) - y
        dv = x[1:, :] - x[:-1, :]
        dh = x[:, 1:] - x[:, :-1]
        J = np.sum(np.abs(res) ** 2) + lam * (
            np.sum(np.sqrt(delta ** 2 + np.abs(dv) ** 2))
            + np.sum(np.sqrt(delta ** 2 + np.abs(dh) ** 2)))
        gd = 2 * (H.conj().T @ res).reshape(N, N)
        wv = dv / np.sqrt(delta ** 2 + np.abs(dv) ** 2)
        wh = dh / np.sqrt(delta ** 2 + np.abs(dh) ** 2)
        gp = np.zeros((N, N), dtype=complex)
        gp[1:, :] += wv
        gp[:-1, :] -= wv
        gp[:, 1:] += wh
        gp[:, :-1] -= wh
        g = gd + lam * gp
        return J, np.concatenate([g.real.reshape(-1), g.imag.reshape(-1)])

    res = minimize(fg, np.zeros(2 * N * N), jac=True, method="L-BFGS-B",
                   options=dict(maxiter=20000, gtol=1e-13, ftol=1e-16, maxcor=50))
    xq = (res.x[: N * N] + 1j * res.x[N * N:]).reshape(N, N)
    b = oracle.adjoint(y, k, N)
    K = oracle.khat(k, N, 2 * N)
    xs = solver.solve(b, K, lam, delta, 600)
    np.testing.assert_allclose(xs, xq, atol=1e-7 * np.abs(xq).max())


# ------------------------------------------------ iteration path (Section 3.3)

def _dense_normal_matrix(k, N, lam):
    """A^H A + lam D^T D from the explicit matrix of Section 2 and an explicit
    difference matrix (row-major pixel index n*N + m)."""
    A = nudft.dense_matrix(k, N)
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
    return A.conj().T @ A + lam * (Dm.T @ Dm)


def _linear_cg_metrics(first=10):
    """With the quadratic penalty the majorant step is the exact line
    minimiser, so the pseudo-CG of Section 3.3 must be linear CG on
    H = A^H A + lam D^T D over R^(2N^2) (inner product Re<a, b>): gradients
    mutually orthogonal, directions H-conjugate (H as a dense matrix, not
    the FFT form the oracle uses), and the gradient gone after 2 N^2 steps.
    Returns (worst orthogonality, worst conjugacy over the first `first`
    iterations, ||g_end|| / ||g_0||)."""
    rng = np.random.default_rng(3)
    N, M, lam = 4, 24, 0.02                 # condition number about 30
    k = rand_k(rng, M)
    y = rand_c(rng, M)
    H = _dense_normal_matrix(k, N, lam)
    trace = []
    solver.solve(oracle.adjoint(y, k, N), oracle.khat(k, N, 2 * N), lam, 1.0,
                 2 * N * N, kind="quadratic", trace=trace)
    G = [t["g"].ravel() for t in trace]
    D = [t["d"].ravel() for t in trace]

    def cosine(a, b, op=None):
        if op is None:
            return abs(np.real(np.vdot(a, b))) / (np.linalg.norm(a) * np.linalg.norm(b))
        return abs(np.real(np.vdot(a, op @ b))) / np.sqrt(
            np.real(np.vdot(a, op @ a)) * np.real(np.vdot(b, op @ b)))

    orth = max(cosine(G[i], G[j]) for i in range(first) for j in range(i))
    conj = max(cosine(D[i], D[j], H) for i in range(first) for j in range(i))
    return orth, conj, np.linalg.norm(G[-1]) / np.linalg.norm(G[0])


def test_linear_cg_pin_quadratic_penalty():
    """Section 3.3 with Hunt's quadratic penalty: PR+ with the exact step is
    linear conjugate gradients (orthogonal gradients, conjugate directions,
    termination within the 2 N^2 real dimensions)."""
    orth, conj, ratio = _linear_cg_metrics()
    assert orth < 1e-10 and conj < 1e-10, (orth, conj)
    assert ratio <= 1e-10, ratio


def _mm_pin(kind):
    """The step length of one iteration against the minimiser of the
    half-quadratic surrogate along d, built here from phi itself (its
    derivative by a fourth-order central difference), the dense forward
    matrix and a brute-force scalar minimisation:
        S(a) = ||y - A(x + a d)||^2
               + lam sum [phi(s) + (phi'(s) / (2 s)) (|D(x + a d)|^2 - s^2)],
    s = |D x|.  Returns (relative step error, min over a grid of S - J)."""
    from scipy.optimize import minimize_scalar
    rng = np.random.default_rng(21)
    N, M, lam, delta = 5, 50, 0.4, 0.3
    k = rand_k(rng, M)
    y = rand_c(rng, M)
    A = nudft.dense_matrix(k, N)
    b = oracle.adjoint(y, k, N)
    K = oracle.khat(k, N, 2 * N)
    x = rand_c(rng, N, N)
    r = oracle.apply_gram(x, K, N) - b
    g = 2 * r + criterion.penalty_grad(x, lam, delta, kind)
    d = -g + 0.3 * rand_c(rng, N, N)
    _, sc = solver.step_from_state(x, r, g, d, K, lam, delta, kind)

    def diffs(z):
        return np.concatenate([(z[1:, :] - z[:-1, :]).ravel(),
                               (z[:, 1:] - z[:, :-1]).ravel()])

    def phi(t):
        return penalty.phi(t, delta, kind)

    s = np.abs(diffs(x))
    h = 1e-5
    dphi = (-phi(s + 2 * h) + 8 * phi(s + h) - 8 * phi(s - h) + phi(s - 2 * h)) / (12 * h)
    w = dphi / s

    def S(a):
        z = x + a * d
        t = np.abs(diffs(z))
        return (np.sum(np.abs(y - A @ z.ravel()) ** 2)
                + lam * np.sum(phi(s) + 0.5 * w * (t ** 2 - s ** 2)))

    def J(a):
        z = x + a * d
        return np.sum(np.abs(y - A @ z.ravel()) ** 2) + lam * np.sum(phi(np.abs(diffs(z))))

    a_star = minimize_scalar(S, bracket=(0.0, 1e-3), tol=1e-14).x
    a = sc["alpha"]
    gap = min(S(t) - J(t) for t in np.linspace(-2 * a, 4 * a, 61))
    return abs(a - a_star) / abs(a_star), gap / abs(J(0.0))


@pytest.mark.parametrize("kind", ["hyperbolic", "huber"])
def test_mm_step_is_the_surrogate_minimiser(kind):
    """The step of Section 3.3's iteration minimises the half-quadratic
    majorant of J along d, and that majorant lies above J."""
    err, gap = _mm_pin(kind)
    assert err < 1e-8, err
    assert gap > -1e-13, gap


def _restart_state():
    """A state (x, r, g, d) whose next direction -g1 + beta d is not a
    descent direction: g is a small multiple of u, d = -u + c v with v the
    part of the true gradient orthogonal to u, so beta is huge and
    Re<g1, d> > 0."""
    rng = np.random.default_rng(7)
    N, M, lam, delta = 5, 40, 0.3, 0.2
    k = rand_k(rng, M)
    y = rand_c(rng, M)
    b = oracle.adjoint(y, k, N)
    K = oracle.khat(k, N, 2 * N)
    x = rand_c(rng, N, N)
    r = oracle.apply_gram(x, K, N) - b
    g_true = 2 * r + criterion.penalty_grad(x, lam, delta)
    u = rand_c(rng, N, N)
    v = g_true - np.real(np.vdot(u, g_true)) / np.real(np.vdot(u, u)) * u
    g = 1e-3 * u
    d = -u + 5.0 * v / np.linalg.norm(v) * np.linalg.norm(u)
    assert np.real(np.vdot(g, d)) < 0           # a descent direction for g
    return (x, r, g, d), K, lam, delta


def test_restart_gives_steepest_descent():
    """Section 3.3's restart: when -g1 + beta d is not a descent direction
    the next direction is exactly -g1; every direction is a descent one."""
    state, K, lam, delta = _restart_state()
    (x1, r1, g1, d1), sc = solver.step_from_state(*state, K, lam, delta)
    assert sc["beta"] > 0 and sc["restart"]
    assert np.array_equal(d1, -g1)
    assert np.real(np.vdot(g1, d1)) < 0


def test_planted_iteration_mistakes_are_caught(monkeypatch):
    """beta = 0, a wrong-sign beta, the majorant curvature taken with the
    weights of D d instead of D x, and a dropped restart each fail a pin."""
    orig_beta = solver.pr_plus_beta
    with monkeypatch.context() as mp:
        mp.setattr(solver, "pr_plus_beta", lambda gn, g: 0.0)
        orth, conj, ratio = _linear_cg_metrics()
        assert ratio > 1e-6 and conj > 1e-3
    with monkeypatch.context() as mp:
        mp.setattr(solver, "pr_plus_beta", lambda gn, g: -orig_beta(gn, g))
        orth, conj, ratio = _linear_cg_metrics()
        assert ratio > 1e-6 and conj > 1e-3
    orig_curv = penalty.smooth_curv
    with monkeypatch.context() as mp:
        mp.setattr(penalty, "smooth_curv",
                   lambda x, d, delta, kind="hyperbolic": orig_curv(d, d, delta, kind))
        for kind in ("hyperbolic", "huber"):
            err, _ = _mm_pin(kind)
            assert err > 1e-3, (kind, err)
    with monkeypatch.context() as mp:
        mp.setattr(solver, "next_direction", lambda gn, d, beta: (-gn + beta * d, False))
        state, K, lam, delta = _restart_state()
        (x1, r1, g1, d1), _ = solver.step_from_state(*state, K, lam, delta)
        assert np.real(np.vdot(g1, d1)) >= 0


# ---------------------------------------------------------------- planted mistakes

def test_planted_mistakes_are_caught(monkeypatch):
    """Plausible mistakes planted in the oracle fail at least one pin."""
    rng = np.random.default_rng(12)
    N, M = 5, 30
    k = rand_k(rng, M)
    x = rand_c(rng, N, N)
    y = rand_c(rng, M)
    # (1) swapped kx/ky in the forward model -> full Cartesian pin fails
    kc, P, Qg = cart_grid(4)
    xs = rand_c(rng, 4, 4)
    bad = oracle.forward(xs, kc[:, ::-1])
    assert np.abs(bad - np.fft.ifft2(xs, norm="ortho")[Qg % 4, P % 4]).max() > 1e-3
    # (2) wrong sign in the adjoint -> adjoint identity fails
    badb = np.conj(oracle.adjoint(np.conj(y), k, N))
    lhs = np.sum(np.conj(oracle.forward(x, k)) * y)
    assert abs(lhs - np.sum(np.conj(x) * badb)) > 1e-3
    # (3) transposed lag kernel -> dense Gram pin fails
    h = gram.lag_kernel(k, N)
    Kbad = np.fft.fft2(gram.circulant_embed(h.T, N, 2 * N)).real
    ref = (toeplitz.dense_gram(k, N) @ x.reshape(-1)).reshape(N, N)
    assert np.abs(toeplitz.apply_gram(x, Kbad, N) - ref).max() > 1e-3
    # (4) dropped penalty term in the gradient -> finite-difference pin fails
    b = oracle.adjoint(y, k, N)
    K = oracle.khat(k, N, 2 * N)
    gbad = 2 * (oracle.apply_gram(x, K, N) - b)
    e = np.zeros((N, N), dtype=complex)
    e[1, 1] = 1e-6
    fd = (criterion.J_direct(x + e, y, k, 0.5, 0.3)
          - criterion.J_direct(x - e, y, k, 0.5, 0.3)) / 2e-6
    assert abs(fd - gbad[1, 1].real) > 1e-4


def test_spot_check_entries_agree_with_full_forms():
    """The per-entry forms used for spot checks at large sizes agree with the
    full forms: adjoint_at (direct sum) with the table/GEMM adjoint, lag_at
    (direct sum) with lag_kernel, khat_at (closed-form geometric series per
    sample) with the FFT of the circulant embedding, including frequencies
    where a sample sits at an integer t (k = 0) and at the ends of the range."""
    rng = np.random.default_rng(41)
    N, L, M = 9, 19, 53
    k = rand_k(rng, M)
    k[0] = 0.0                      # t = p/L exactly at p = 0
    k[1] = (-0.5, 0.5)              # range ends
    y = rand_c(rng, M)
    b = nudft.adjoint(y, k, N)
    n = np.array([0, 8, 3, 8, 0])
    m = np.array([0, 8, 5, 0, 7])
    assert np.max(np.abs(nudft.adjoint_at(y, k, N, n, m) - b[n, m])) < 1e-13
    h = gram.lag_kernel(k, N)
    a = np.array([-(N - 1), 0, 3, N - 1, -2])
    bb = np.array([N - 1, 0, -4, -(N - 1), 1])
    assert np.max(np.abs(gram.lag_at(k, N, a, bb) - h[a + N - 1, bb + N - 1])) < 1e-15
    K = gram.khat(k, N, L)
    p = np.array([0, 0, 5, L - 1, 11, 18])
    q = np.array([0, 7, 0, L - 1, 3, 9])
    assert np.max(np.abs(gram.khat_at(k, N, L, p, q) - K[p, q])) < 1e-12 * np.abs(K).max()


def test_spot_check_planted_mistake_is_caught():
    """A sign error in the phase of the per-entry lag form is caught."""
    rng = np.random.default_rng(42)
    N, M = 6, 31
    k = rand_k(rng, M)
    h = gram.lag_kernel(k, N)
    a, b = np.array([2]), np.array([-3])
    wrong = np.sum(np.exp(+2j * np.pi * (k[:, 1] * a[0] + k[:, 0] * b[0]))) / N ** 2
    assert abs(wrong - h[a[0] + N - 1, b[0] + N - 1]) > 1e-3
    assert abs(gram.lag_at(k, N, a, b)[0] - h[a[0] + N - 1, b[0] + N - 1]) < 1e-15
