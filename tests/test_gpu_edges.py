"""GPU edge cases against the FP64 oracle: the smallest geometry (N = 2,
L = 64, a single sample), trajectories touching the edge of the k range and
the origin, lambda = 0, a zero iteration budget, and the largest geometry
(N = 1024, L = 2048).

Bars: operators as in the parity tests (a few FP32 roundings; FP64 adjoint
1e-7); iterates 1e-4 (FP32 iteration) or 1e-8 against the oracle's iterate
rounded to complex64 (FP64 iteration).
"""
import numpy as np
import pytest

import oracle
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


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("M", [1, 3])
@pytest.mark.parametrize("prec", [recon.FP32, recon.FP64, recon.FP64_ITER64])
def test_smallest_geometry(M, prec):
    """N = 2, L = 64 and one or three samples: every operator and a solve."""
    rng = np.random.default_rng(M + 10 * prec)
    N = 2
    k = rng.uniform(-0.5, 0.5, size=(M, 2))
    print(f"N=2 M={M} prec={prec}", flush=True)
    plan = recon.Plan(k, N, 64, prec=prec)
    plan.gram_kernel()
    y = rand_c(rng, 2, M).astype(np.complex64)
    b = host(plan.adjoint(dev(y)))
    eb = rel(b, oracle.adjoint(y, k, N))
    x = rand_c(rng, 2, N, N).astype(np.complex64)
    ey = rel(host(plan.forward(dev(x))), oracle.forward(x, k))
    K = oracle.khat(k, N, 64)
    eq = rel(host(plan.gram_apply(dev(x))), oracle.apply_gram(x, K, N))
    lam, delta, iters = 0.05, 0.1, 20
    xs, st = plan.solve(dev(y), lam, delta, iters)
    xo = np.array([oracle.solve(oracle.adjoint(y[f], k, N), K, lam, delta, iters)
                   for f in range(2)])
    es = rel32(host(xs), xo) if prec == recon.FP64_ITER64 else rel(host(xs), xo)
    print(f"  adjoint {eb:.2e} forward {ey:.2e} gram {eq:.2e} solve {es:.2e}")
    assert eb < (1e-7 if prec != recon.FP32 else 2e-6)
    assert ey < 2e-6 and eq < 5e-6
    assert es < (1e-8 if prec == recon.FP64_ITER64 else 1e-4)
    assert all(s == 0 for s in st["status"])


def test_k_range_edges():
    """Samples at k = 0 and on the edges |k| = 0.5 of the accepted range."""
    rng = np.random.default_rng(5)
    N = 24
    edge = np.array([[0.0, 0.0], [0.5, 0.0], [0.0, -0.5], [-0.5, 0.5], [0.5, 0.5],
                     [-0.5, -0.5], [0.25, -0.5]])
    k = np.concatenate([edge, rng.uniform(-0.5, 0.5, size=(200, 2))])
    for prec in (recon.FP32, recon.FP64):
        plan = recon.Plan(k, N, prec=prec)
        plan.gram_kernel()
        y = rand_c(rng, 1, k.shape[0]).astype(np.complex64)
        x = rand_c(rng, 1, N, N).astype(np.complex64)
        eb = rel(host(plan.adjoint(dev(y))), oracle.adjoint(y, k, N))
        ey = rel(host(plan.forward(dev(x))), oracle.forward(x, k))
        eq = rel(host(plan.gram_apply(dev(x))),
                 oracle.apply_gram(x, oracle.khat(k, N, plan.L), N))
        print(f"prec={prec}: adjoint {eb:.2e} forward {ey:.2e} gram {eq:.2e}")
        assert eb < 2e-6 and ey < 2e-6 and eq < 5e-6


@pytest.mark.parametrize("prec", [recon.FP64, recon.FP64_ITER64])
def test_lambda_zero(prec):
    """lambda = 0: the data term alone (the iteration is linear CG on Q x = b
    with the exact step).  Uniformly random samples, M = 4 N^2 (Gram condition
    number ~24): spiral trajectories leave the k-space corners empty and make
    the unregularised problem so ill-conditioned (~1e10) that its FP32
    iterate amplifies rounding past 1e-4."""
    rng = np.random.default_rng(9)
    N = 16
    k = rng.uniform(-0.5, 0.5, size=(4 * N * N, 2))
    y = rand_c(rng, 1, k.shape[0]).astype(np.complex64)
    plan = recon.Plan(k, N, prec=prec)
    plan.gram_kernel()
    x, st = plan.solve(dev(y), 0.0, 0.1, 40)
    xo = oracle.solve(oracle.adjoint(y[0], k, N), oracle.khat(k, N, plan.L), 0.0, 0.1, 40)
    e = rel32(host(x)[0], xo) if prec == recon.FP64_ITER64 else rel(host(x)[0], xo)
    print(f"lambda 0 prec={prec}: rel {e:.2e}")
    assert e < (1e-8 if prec == recon.FP64_ITER64 else 1e-4)
    assert st["status"][0] == 0


@pytest.mark.parametrize("prec", [recon.FP64, recon.FP64_ITER64])
def test_zero_iterations(prec):
    """iters = 0 returns x0 (zeros) with the criterion of x0: J = ||y||^2."""
    rng = np.random.default_rng(2)
    N = 16
    k = synthetic.spiral_trajectory(N, 2, 100, 1.0)
    y = rand_c(rng, 2, k.shape[0]).astype(np.complex64)
    plan = recon.Plan(k, N, prec=prec)
    plan.gram_kernel()
    x, st = plan.solve(dev(y), 0.02, 0.1, 0)
    assert np.all(host(x) == 0)
    yy = np.sum(np.abs(y.astype(np.complex128)) ** 2, axis=1)
    pen0 = 0.02 * 2 * N * (N - 1) * 0.1  # phi(0) = delta on every difference
    np.testing.assert_allclose(st["J"], yy + pen0, rtol=1e-12)
    assert all(st["iters_done"] == 0) and all(st["grad_ratio"] == 1.0)


def test_largest_geometry():
    """N = 1024, L = 2048 (the largest supported): the Gram apply in full and
    three iterations of the FP32 iteration against the oracle."""
    rng = np.random.default_rng(1024)
    N, L = 1024, 2048
    k = rng.uniform(-0.5, 0.5, size=(1024, 2))
    print("N=1024 L=2048 M=1024", flush=True)
    plan = recon.Plan(k, N, L, prec=recon.FP64)
    plan.gram_kernel()
    K = oracle.khat(k, N, L)
    v = (0.1 * rand_c(rng, 1, N, N)).astype(np.complex64)
    eq = rel(host(plan.gram_apply(dev(v))), oracle.apply_gram(v, K, N))
    x_true = synthetic.ellipse_phantom(N, 6, rng)
    y = oracle.forward(x_true, k)[None].astype(np.complex64)
    x, st = plan.solve(dev(y), 0.01, 0.05, 3)
    xo = oracle.solve(oracle.adjoint(y[0], k, N), K, 0.01, 0.05, 3)
    e = rel(host(x)[0], xo)
    print(f"  gram apply rel {eq:.2e}; 3 iterations rel {e:.2e}")
    assert eq < 5e-6
    assert e < 1e-4
    assert st["status"][0] == 0


@pytest.mark.parametrize("prec", [recon.FP32, recon.BF16X3, recon.FP16X3])
def test_batch_limit_without_fp64_adjoint(prec):
    """Plans with an FP32 or split-precision adjoint refuse more than 64 frames
    per adjoint, forward or solve call, before launching anything.  (Larger
    batches of these plans stay off the GPU: an unexplained fault at 128
    frames.)"""
    rng = np.random.default_rng(64)
    N = 16
    k = synthetic.spiral_trajectory(N, 2, 64, 1.0)
    plan = recon.Plan(k, N, prec=prec)
    plan.gram_kernel()
    y = dev(rand_c(rng, 65, k.shape[0]))
    x = dev(rand_c(rng, 65, N, N))
    with pytest.raises(recon.ReconError):
        plan.adjoint(y)
    with pytest.raises(recon.ReconError):
        plan.forward(x)
    with pytest.raises(recon.ReconError):
        plan.solve(y, 0.02, 0.1, 2)
    with pytest.raises(recon.ReconError):
        plan.begin(y=y, lam=0.02, delta=0.1)


def test_no_batch_limit_with_fp64_adjoint():
    """An FP64-adjoint plan takes 65 frames; frame 64 equals its lone result."""
    rng = np.random.default_rng(65)
    N = 16
    k = synthetic.spiral_trajectory(N, 2, 64, 1.0)
    plan = recon.Plan(k, N, prec=recon.FP64)
    plan.gram_kernel()
    y = dev(rand_c(rng, 65, k.shape[0]))
    b = host(plan.adjoint(y))
    b1 = host(plan.adjoint(y[64:65]))
    np.testing.assert_array_equal(b[64], b1[0])
