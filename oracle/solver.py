"""Minimisation of the regularised criterion (oracle, FP64).

Section 3.3 minimises the convex criterion with a pseudo-conjugate-gradient
method with a Polak-Ribiere correction, on the image-domain form of the data
term (Section 3.4).  The paper does not spell out its line search (it spends
three criterion evaluations per iteration, Section 4.2) and cites
half-quadratic work for faster schemes (Section 5).  The reading used here:

    x = x0 (zeros), r = Q x - b, g = 2 r + grad R(x), d = -g
    repeat iters times:
        Qd    = Q d
        alpha = -Re<g, d> / (2 Re<d, Qd> + lam sum w(Dx)|Dd|^2 [+ lam0 sum w0(x)|d|^2])
                (exact minimiser along d of the half-quadratic majorant of J,
                 which exists because sqrt(delta^2 + rho) is concave in
                 rho = |t|^2; J decreases monotonically)
        x    += alpha d ;  r += alpha Qd
        g_new = 2 r + grad R(x)
        beta  = max(0, Re<g_new, g_new - g> / <g, g>)      (Polak-Ribiere, PR+)
        d     = -g_new + beta d ;  g = g_new
        if Re<g, d> >= 0: d = -g                            (restart)

with <a, b> = sum conj(a) b.  ``ls_steps`` > 1 repeats the majorant step
along the same d (the paper's several criterion evaluations per iteration).
Guards: alpha = 0 when Re<g, d> = 0; beta = 0 when <g, g> = 0.
"""
from __future__ import annotations

import numpy as np

from . import criterion, penalty, toeplitz


def _dot(a, b):
    return np.sum(np.conj(a) * b)


def step_length(g, d, dQd, x, lam, delta, kind="hyperbolic", lam0=0.0,
                alpha0=1.0, kind0="huber"):
    """Minimiser along d of the half-quadratic majorant of J at x:
    alpha = -Re<g, d> / (2 Re<d, Qd> + lam sum w(|Dx|) |Dd|^2
                         [+ lam0 sum w0(|x|) |d|^2]),
    with dQd = Re<d, Q d> and alpha = 0 when Re<g, d> = 0."""
    gd = np.real(_dot(g, d))
    curv = 2.0 * dQd + lam * penalty.smooth_curv(x, d, delta, kind)
    if lam0:
        curv = curv + lam0 * penalty.background_curv(x, d, alpha0, kind0)
    return 0.0 if gd == 0.0 else -gd / curv


def pr_plus_beta(g_new, g):
    """Polak-Ribiere coefficient clipped at zero (PR+):
    beta = max(0, Re<g_new, g_new - g> / <g, g>), 0 when <g, g> = 0."""
    gg = np.real(_dot(g, g))
    return 0.0 if gg == 0.0 else max(0.0, np.real(_dot(g_new, g_new - g)) / gg)


def next_direction(g_new, d, beta):
    """d_new = -g_new + beta d, or -g_new (restart) when that is not a
    descent direction (Re<g_new, d_new> >= 0).  Returns (d_new, restarted)."""
    dn = -g_new + beta * d
    if np.real(_dot(g_new, dn)) >= 0.0:
        return -g_new, True
    return dn, False


def solve(b, K, lam, delta, iters, kind="hyperbolic", x0=None, yy=None,
          lam0=0.0, alpha0=1.0, kind0="huber", ls_steps=1, history=False,
          trace=None):
    """Run the fixed-budget minimisation for one frame.

    b: [N, N] complex (A^H y); K: [L, L] real Gram spectrum.
    Returns x, and with history=True also a dict with per-iteration J
    (needs yy = ||y||^2), ||g|| and the iteration state at the end.
    trace: optional list; receives the initial (x, g, d) and, after every
    iteration, (x, g, d, alpha, beta, restart) as dicts.
    """
    b = np.asarray(b, dtype=np.complex128)
    N = b.shape[-1]

    def Q(v):
        return toeplitz.apply_gram(v, K, N)

    pen = dict(lam0=lam0, alpha0=alpha0, kind0=kind0)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = Q(x) - b
    g = 2.0 * r + criterion.penalty_grad(x, lam, delta, kind, **pen)
    d = -g
    hist = dict(J=[], gnorm=[float(np.sqrt(np.real(_dot(g, g))))], restarts=0)
    if trace is not None:
        trace.append(dict(x=x, g=g, d=d))

    def J_now():
        return float(criterion.J_rewritten(x, yy, b, r + b, lam, delta, kind,
                                           **pen))

    if history and yy is not None:
        hist["J"].append(J_now())
    for _ in range(iters):
        Qd = Q(d)
        dQd = np.real(_dot(d, Qd))
        for _s in range(ls_steps):
            alpha = step_length(g, d, dQd, x, lam, delta, kind, **pen)
            x = x + alpha * d
            r = r + alpha * Qd
            g_new = 2.0 * r + criterion.penalty_grad(x, lam, delta, kind, **pen)
            if _s + 1 < ls_steps:
                g = g_new
        beta = pr_plus_beta(g_new, g)
        d, restarted = next_direction(g_new, d, beta)
        g = g_new
        hist["restarts"] += int(restarted)
        hist["gnorm"].append(float(np.sqrt(np.real(_dot(g, g)))))
        if trace is not None:
            trace.append(dict(x=x, g=g, d=d, alpha=alpha, beta=beta,
                              restart=restarted))
        if history and yy is not None:
            hist["J"].append(J_now())
    if history:
        hist["state"] = dict(x=x, r=r, g=g, d=d)
        return x, hist
    return x


def step_from_state(x, r, g, d, K, lam, delta, kind="hyperbolic"):
    """One iteration of ``solve`` from an explicit state (x, r, g, d).

    Returns the next state (x, r, g, d) and the scalars used.  The GPU path's
    own state can be advanced by this FP64 step and compared with the GPU's
    next state.
    """
    N = x.shape[-1]
    Qd = toeplitz.apply_gram(d, K, N)
    alpha = step_length(g, d, np.real(_dot(d, Qd)), x, lam, delta, kind)
    x1 = x + alpha * d
    r1 = r + alpha * Qd
    g1 = 2.0 * r1 + criterion.penalty_grad(x1, lam, delta, kind)
    beta = pr_plus_beta(g1, g)
    d1, restart = next_direction(g1, d, beta)
    return (x1, r1, g1, d1), dict(alpha=alpha, beta=beta, restart=restart,
                                  Qd=Qd)


def solve_quadratic_dense(y, k, N, lam):
    """Closed form for phi(s) = s^2: x = (A^H A + lam D^T D)^{-1} A^H y.

    Built from the explicit matrix H of Section 2 and an explicit difference
    matrix (tiny N); this is Section 3's least-squares closed form with the
    quadratic (Hunt) penalty added.
    """
    from . import nudft
    H = nudft.dense_matrix(k, N)
    n2 = N * N
    rows = []
    for n in range(N - 1):
        for m in range(N):
            e = np.zeros(n2)
            e[(n + 1) * N + m] = 1.0
            e[n * N + m] = -1.0
            rows.append(e)
    for n in range(N):
        for m in range(N - 1):
            e = np.zeros(n2)
            e[n * N + m + 1] = 1.0
            e[n * N + m] = -1.0
            rows.append(e)
    Dm = np.array(rows)
    A = H.conj().T @ H + lam * (Dm.T @ Dm)
    return np.linalg.solve(A, H.conj().T @ y).reshape(N, N)
