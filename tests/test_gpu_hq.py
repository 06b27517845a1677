"""GPU parity of the half-quadratic solver (Section 5's dual /
half-quadratic alternative to the pseudo-conjugate gradient) against the
oracle's half-quadratic minimiser (oracle/halfquad.py, pinned by the CPU
tests against the dense closed form of every inner problem).

Bars: the FP64 iteration equals the oracle's iterate up to the final
rounding to complex64 (1e-8 on the small cases, 1e-6 at 256^2); the FP32
iteration on the converging 32^2 workload 1e-4.
"""
import numpy as np
import pytest

import oracle
from oracle import halfquad
import synthetic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_0908_3252_amd import recon  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rel32(x, ref):
    return rel(x, ref.astype(np.complex64).astype(np.complex128))


def _c1():
    p = synthetic.make_problem(1)
    y = p.measured(oracle.forward(p.x_true, p.k)).astype(np.complex64)
    return p, y


@pytest.mark.parametrize("prec", [recon.FP64_ITER64, recon.FP64])
@pytest.mark.parametrize("phi", ["hyperbolic", "huber"])
def test_hq_tiny_against_oracle(prec, phi):
    p, y = _c1()
    outer, inner = 20, 10
    print(f"HQ 32^2 {phi} prec={prec} {outer}x{inner}", flush=True)
    plan = recon.Plan(p.k, p.N, p.L, prec=prec)
    plan.gram_kernel()
    x, st = plan.solve_hq(dev(y), p.lam, p.delta, outer, inner, phi=phi)
    b = oracle.adjoint(y[0], p.k, p.N)
    K = oracle.khat(p.k, p.N, p.L)
    xo = halfquad.solve(b, K, p.lam, p.delta, outer, inner, kind=phi)
    xg = host(x)[0]
    e = rel32(xg, xo) if prec == recon.FP64_ITER64 else rel(xg, xo)
    Jo = oracle.criterion.J_direct(xo, y[0].astype(np.complex128), p.k, p.lam, p.delta, phi)
    dj = abs(st["J"][0] - Jo) / abs(Jo)
    print(f"  rel {e:.2e}, J rel diff {dj:.2e}, grad ratio {st['grad_ratio'][0]:.2e}, "
          f"iters {st['iters_done'][0]}")
    assert st["status"][0] == 0 and st["iters_done"][0] == outer * inner
    assert e < (1e-8 if prec == recon.FP64_ITER64 else 1e-4)
    # FP32 iteration: J is formed from the iteration's own residual r (updated
    # 200 times in FP32) and ||y||^2 - Re<x, b> cancel most of its digits
    assert dj < (1e-12 if prec == recon.FP64_ITER64 else 1e-4)


def test_hq_background_term_fp64_iteration():
    """Huber differences plus the Huber background penalty (the paper's full
    criterion) through the resumable form."""
    p, y = _c1()
    lam, alpha1, lam0, alpha0 = 0.02, 0.2, 0.05, 0.1
    plan = recon.Plan(p.k, p.N, p.L, prec=recon.FP64_ITER64)
    plan.gram_kernel()
    x, st = plan.solve_hq(dev(y), lam, alpha1, 12, 10, phi="huber", lam0=lam0, alpha0=alpha0)
    b = oracle.adjoint(y[0], p.k, p.N)
    K = oracle.khat(p.k, p.N, p.L)
    xo = halfquad.solve(b, K, lam, alpha1, 12, 10, kind="huber", lam0=lam0, alpha0=alpha0)
    e = rel32(host(x)[0], xo)
    print(f"HQ 32^2 full criterion: rel {e:.2e}")
    assert e < 1e-8
    assert st["status"][0] == 0


def test_hq_outer_iterations_decrease_J():
    """Majorise-minimise: J at the end of every outer iteration decreases."""
    p, y = _c1()
    plan = recon.Plan(p.k, p.N, p.L, prec=recon.FP64_ITER64)
    plan.gram_kernel()
    plan.begin(y=dev(y), lam=p.lam, delta=p.delta, hq=True)
    J = []
    for _ in range(15):
        plan.hq_iterate(1, 6)
        J.append(plan.end()[1]["J"][0])
    print("HQ J per outer iteration: " + ", ".join(f"{j:.8g}" for j in J[:6]) + " ...")
    assert np.all(np.diff(J) <= 1e-12 * abs(J[0]))


def test_hq_batch_invariance():
    """Each frame of a batch is bitwise its solve alone."""
    p = synthetic.make_frames(3, frames=3, N=48, S=256, I=6, K=8)
    y = p.measured(oracle.forward(p.x_true, p.k)).astype(np.complex64)
    plan = recon.Plan(p.k, p.N, prec=recon.FP64_ITER64)
    plan.gram_kernel()
    xb, _ = plan.solve_hq(dev(y), p.lam, p.delta, 4, 5)
    for f in range(3):
        xf, _ = plan.solve_hq(dev(y[f:f + 1]), p.lam, p.delta, 4, 5)
        np.testing.assert_array_equal(host(xf)[0], host(xb)[f])


def test_hq_plain_workload_256():
    """The benchmark's 256^2 frame: 30 outer x 10 inner steps, FP64 iteration,
    against the oracle's half-quadratic iterate."""
    p = synthetic.make_problem(2)
    y = p.measured(oracle.forward(p.x_true, p.k)).astype(np.complex64)
    outer, inner = 30, 10
    plan = recon.Plan(p.k, p.N, p.L, prec=recon.FP64_ITER64)
    plan.gram_kernel()
    x, st = plan.solve_hq(dev(y), p.lam, p.delta, outer, inner)
    b = oracle.adjoint(y[0], p.k, p.N)
    K = oracle.khat(p.k, p.N, p.L)
    xo = halfquad.solve(b, K, p.lam, p.delta, outer, inner)
    e = rel32(host(x)[0], xo)
    print(f"HQ 256^2 {outer}x{inner}: rel {e:.2e}, J {st['J'][0]:.10g}")
    assert e < 1e-6
    assert st["status"][0] == 0


@pytest.mark.parametrize("N,L,prec", [(40, 1024, recon.FP64_ITER64), (300, 1024, recon.FP64_ITER64),
                                      (100, 256, recon.FP64_ITER64), (48, 128, recon.FP64_ITER64),
                                      (100, 256, recon.FP64)])
def test_hq_transforms_and_ragged_sizes(N, L, prec):
    """The inner steps in the fused row kernels with the frozen-image tiles:
    multi-wavefront FFT teams (L = 1024), ragged N (row blocks that end
    inside the image, halo rows at both borders), a small L, with the
    background term on (its weight frozen as well)."""
    rng = np.random.default_rng(N + L + 7)
    k = (synthetic.spiral_trajectory(N, 6, 2048, 1.0) if N > 100
         else synthetic.spiral_trajectory(N, 4, 300, 2.0))
    x_true = synthetic.ellipse_phantom(N, 8, rng)
    y0 = oracle.forward(x_true, k)
    y = (y0 + 0.01 * np.abs(y0).max() * synthetic.noise_draws(k.shape[0], rng))[None]
    y = y.astype(np.complex64)
    lam, delta, lam0, alpha0, outer, inner = 0.02, 0.05, 0.01, 0.1, 4, 6
    print(f"HQ N={N} L={L} prec={prec} {outer}x{inner}", flush=True)
    plan = recon.Plan(k, N, L, prec=prec)
    plan.gram_kernel()
    x, st = plan.solve_hq(dev(y), lam, delta, outer, inner, lam0=lam0, alpha0=alpha0)
    b = oracle.adjoint(y[0], k, N)
    K = oracle.khat(k, N, L)
    xo = halfquad.solve(b, K, lam, delta, outer, inner, lam0=lam0, alpha0=alpha0)
    xg = host(x)[0]
    e = rel32(xg, xo) if prec == recon.FP64_ITER64 else rel(xg, xo)
    print(f"  rel {e:.2e}")
    assert st["status"][0] == 0 and st["iters_done"][0] == outer * inner
    assert e < (1e-8 if prec == recon.FP64_ITER64 else 1e-4)


def test_hq_rejections():
    p, y = _c1()
    plan = recon.Plan(p.k, p.N, p.L)
    plan.gram_kernel()
    lib = recon.load()
    ws, n = plan.workspace(1)          # the plain workspace is too small for HQ
    x = torch.empty((1, p.N, p.N), dtype=torch.complex64, device="cuda")
    yd = dev(y)
    st = lib.recon_solve_hq(plan.handle, yd.data_ptr(), 1, p.lam, p.delta, 2, 2, 0,
                            x.data_ptr(), 0, ws.data_ptr(), n, None, recon._stream())
    assert st == recon.E_NOMEM
    wsh, nh = plan.hq_workspace(1)
    st = lib.recon_solve_hq(plan.handle, yd.data_ptr(), 1, p.lam, p.delta, -1, 2, 0,
                            x.data_ptr(), 0, wsh.data_ptr(), nh, None, recon._stream())
    assert st == recon.E_ARG
