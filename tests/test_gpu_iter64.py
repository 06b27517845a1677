"""GPU parity of the FP64 iteration (plan precision FP64 | ITER_FP64).

The iterate after a fixed budget of iterations amplifies per-step rounding
when the minimisation is far from converged (on the 256^2 series, random
relative perturbations of 6e-8 per step move the 300-iteration iterate by
~1e-4).  With b, x, r, d, the transforms, the penalty stencil and the Gram
spectrum in FP64 the per-step errors are ~1e-15, so the GPU iterate follows
the FP64 oracle's to ~1e-10 or better; the bars below (1e-8 on the small
cases, 1e-6 at 256^2) sit far under the required 1e-4 so that a lost FP64
term (e.g. one FP32 rounding of lambda or of the spectrum, ~1e-8 per step)
fails them.  Results leave the library as complex64: final iterates are
compared with the oracle's rounded to complex64 (rel32), and the exported
state of the one-step check carries one FP32 rounding (~6e-8).
"""
import numpy as np
import pytest

import oracle
import synthetic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_0908_3252_amd import recon  # noqa: E402

P64 = recon.FP64_ITER64


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rel32(x, ref):
    """x (a complex64 result) against the FP64 reference rounded to complex64:
    only differences of the iterations themselves remain."""
    return rel(x, ref.astype(np.complex64).astype(np.complex128))


def _c1():
    p = synthetic.make_problem(1)
    y = p.measured(oracle.forward(p.x_true, p.k)).astype(np.complex64)
    return p, y


def test_initial_state_fp64_iteration():
    """x0 = 0: r = -b, g = -2b, d = 2b exactly (after the one rounding of the
    exported values), b within one FP32 rounding of the oracle's."""
    p, y = _c1()
    plan = recon.Plan(p.k, p.N, p.L, prec=P64)
    plan.gram_kernel()
    plan.begin(y=dev(y), lam=p.lam, delta=p.delta)
    b = host(plan.export("b"))
    e = rel(b, oracle.adjoint(y, p.k, p.N))
    print(f"b rel {e:.2e}")
    assert e < 1e-7
    np.testing.assert_array_equal(host(plan.export("r")), -b)
    np.testing.assert_array_equal(host(plan.export("g")), -2 * b)
    np.testing.assert_array_equal(host(plan.export("d")), 2 * b)
    np.testing.assert_array_equal(host(plan.export("x")), 0 * b)


def test_end_to_end_tiny_fp64_iteration():
    """32x32, 200 iterations: iterate and criterion against the oracle."""
    p, y = _c1()
    plan = recon.Plan(p.k, p.N, p.L, prec=P64)
    plan.gram_kernel()
    x, st = plan.solve(dev(y), p.lam, p.delta, p.iters)
    b = oracle.adjoint(y[0], p.k, p.N)
    K = oracle.khat(p.k, p.N, p.L)
    yy = float(np.sum(np.abs(y[0].astype(np.complex128)) ** 2))
    xo, h = oracle.solve(b, K, p.lam, p.delta, p.iters, yy=yy, history=True)
    e = rel32(host(x)[0], xo)
    dj = abs(st["J"][0] - h["J"][-1]) / abs(h["J"][-1])
    print(f"C1 FP64 iteration: rel {e:.2e}, J rel {dj:.2e}")
    assert e < 1e-8
    assert dj < 1e-10
    assert st["status"][0] == 0 and st["iters_done"][0] == p.iters


def test_one_step_shadow_fp64_iteration():
    """One FP64 oracle step from the GPU's (exported) state against the GPU's
    next state: only the rounding of the exports remains.  Early iterations
    only: once |g| << |2r| the gradient the oracle rebuilds from the rounded
    r and x cancels, and the export rounding (not the GPU step) dominates."""
    p, y = _c1()
    plan = recon.Plan(p.k, p.N, p.L, prec=P64)
    plan.gram_kernel()
    K = oracle.khat(p.k, p.N, p.L)
    plan.begin(y=dev(y), lam=p.lam, delta=p.delta)
    cur = 0
    for k_it in (0, 1, 3):
        if k_it > cur:
            plan.iterate(k_it - cur)
            cur = k_it
        st = {f: host(plan.export(f))[0] for f in ("x", "r", "g", "d")}
        (x1, r1, g1, d1), _ = oracle.solver.step_from_state(
            st["x"], st["r"], st["g"], st["d"], K, p.lam, p.delta)
        plan.iterate(1)
        cur += 1
        nx = {f: host(plan.export(f))[0] for f in ("x", "r", "g", "d")}
        for f, ref in (("x", x1), ("r", r1), ("g", g1), ("d", d1)):
            e = rel(nx[f], ref)
            print(f"after {k_it}: step {f} rel {e:.2e}")
            assert e < 1e-6, (k_it, f, e)


@pytest.mark.parametrize("phi", ["huber", "quadratic"])
def test_other_penalties_fp64_iteration(phi):
    rng = np.random.default_rng(21)
    N = 16
    k = synthetic.spiral_trajectory(N, 3, 120, 1.0)
    y = (rng.standard_normal((1, k.shape[0])) + 1j * rng.standard_normal((1, k.shape[0])))
    y = y.astype(np.complex64)
    lam, delta, iters = 0.05, 0.3, 150
    plan = recon.Plan(k, N, prec=P64)
    plan.gram_kernel()
    x, st = plan.solve(dev(y), lam, delta, iters, phi=phi)
    b = oracle.adjoint(y[0], k, N)
    K = oracle.khat(k, N, plan.L)
    xo = oracle.solve(b, K, lam, delta, iters, kind=phi)
    e = rel32(host(x)[0], xo)
    print(f"{phi}: rel {e:.2e}")
    assert e < 1e-8
    if phi == "quadratic":
        xc = oracle.solve_quadratic_dense(y[0], k, N, lam)
        assert rel(host(x)[0], xc) < 1e-6


def test_warm_start_fp64_iteration():
    """x0 (complex64) widened, r = Q x0 - b by the FP64 Gram apply."""
    p, y = _c1()
    rng = np.random.default_rng(3)
    x0 = (0.1 * (rng.standard_normal((1, p.N, p.N)) + 1j * rng.standard_normal((1, p.N, p.N))))
    x0 = x0.astype(np.complex64)
    plan = recon.Plan(p.k, p.N, p.L, prec=P64)
    plan.gram_kernel()
    x, _ = plan.solve(dev(y), p.lam, p.delta, 40, x0=dev(x0))
    b = oracle.adjoint(y[0], p.k, p.N)
    K = oracle.khat(p.k, p.N, p.L)
    xo = oracle.solve(b, K, p.lam, p.delta, 40, x0=x0[0])
    e = rel32(host(x)[0], xo)
    print(f"warm start rel {e:.2e}")
    assert e < 1e-8


@pytest.mark.parametrize("N,L", [(40, 1024), (300, 1024), (48, 128)])
def test_end_to_end_fp64_iteration_transforms(N, L):
    """Multi-wavefront FFT teams (L = 1024), a ragged N and a small L through
    the FP64 iteration."""
    rng = np.random.default_rng(N + L)
    k = (synthetic.spiral_trajectory(N, 12, 4096, 1.0) if N > 100
         else synthetic.spiral_trajectory(N, 4, 300, 2.0))
    x_true = synthetic.ellipse_phantom(N, 8, rng)
    y0 = oracle.forward(x_true, k)
    y = (y0 + 0.01 * np.abs(y0).max() * synthetic.noise_draws(k.shape[0], rng))[None]
    y = y.astype(np.complex64)
    lam, delta, iters = 0.02, 0.05, 40
    plan = recon.Plan(k, N, L, prec=P64)
    plan.gram_kernel()
    x, st = plan.solve(dev(y), lam, delta, iters)
    b = oracle.adjoint(y[0], k, N)
    K = oracle.khat(k, N, L)
    xo = oracle.solve(b, K, lam, delta, iters)
    e = rel32(host(x)[0], xo)
    print(f"N={N} L={L}: rel {e:.2e}")
    assert e < 1e-8
    assert st["status"][0] == 0


@pytest.mark.parametrize("N,L", [(64, 0), (100, 256), (40, 1024)])
def test_batch_invariance_fp64_iteration(N, L):
    """Each frame of a 6-frame batch equals its solve alone, bitwise.  The
    batch takes the update with late loads, the single frames the one with
    every load up front (batches of at most four frames)."""
    p = synthetic.make_frames(3, frames=6, N=N, S=256, I=8, K=10)
    y = p.measured(oracle.forward(p.x_true, p.k))
    print(f"batch invariance N={N} L={L or 'default'}", flush=True)
    plan = recon.Plan(p.k, p.N, L, prec=P64)
    plan.gram_kernel()
    xb, _ = plan.solve(dev(y), p.lam, p.delta, 30)
    for f in range(6):
        xf, _ = plan.solve(dev(y[f:f + 1]), p.lam, p.delta, 30)
        np.testing.assert_array_equal(host(xf)[0], host(xb)[f])


def test_fp64_iteration_rejections():
    """The FP64 iteration needs the FP64 adjoint and L <= 1024."""
    k = synthetic.spiral_trajectory(16, 2, 64, 1.0)
    with pytest.raises(recon.ReconError):
        recon.Plan(k, 16, 2048, prec=recon.FP64_ITER64)
    with pytest.raises(recon.ReconError):
        recon.Plan(k, 16, 64, prec=recon.FP32 | recon.ITER_FP64)
