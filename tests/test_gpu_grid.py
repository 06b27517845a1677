"""GPU parity of the convolution gridding / non-uniform FFT module
(Section 1's gridding steps with Section 4.1's Kaiser-Bessel kernel; Section
5's NUFFT precomputation of D and of the Gram kernel) against the oracle's
gridding module (oracle/gridding.py, pinned by the CPU tests).

Both sides run the same FP64 approximation, so they agree to FP64 rounding
where the output is FP64 (lag kernel, density weights) and to one complex64
rounding where it is complex64 (images); against the exact sums both stay
within the kernel's edge-jump bound 4 / I0(beta).
"""
import numpy as np
import pytest

import oracle
from oracle import gram, gridding as gr
import synthetic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_0908_3252_amd import recon  # noqa: E402


def dev(a, dtype=np.complex64):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def bound(W, sigma):
    return 4.0 / float(np.i0(gr.kb_beta(W, sigma)))


# (N, trajectory, kernel width): several 32 x 32 grid tiles, ragged sample
# counts, an odd N (offset h = N // 2), the 256^2 workload's spiral
CASES = [
    ("n48_w7", 48, ("rand", 2900), 7),
    ("n45_w9", 45, ("rand", 1777), 9),
    ("n64_w5_spiral", 64, ("spiral", (8, 300, 1.0)), 5),
    ("n256_w7_workload", 256, ("spiral", (16, 2048, 2.0)), 7),
]


def traj(spec, N, seed):
    kind, arg = spec
    if kind == "rand":
        return np.random.default_rng(seed).uniform(-0.5, 0.5, (arg, 2))
    return synthetic.spiral_trajectory(N, *arg)


@pytest.mark.parametrize("name,N,spec,W", CASES)
def test_nufft_adjoint(name, N, spec, W):
    k = traj(spec, N, N)
    M = k.shape[0]
    print(f"{name}: N={N} M={M} W={W}", flush=True)
    gp = recon.GridPlan(k, N, W=W)
    rng = np.random.default_rng(N + W)
    B = 3
    y = rand_c(rng, B, M).astype(np.complex64)
    b = host(gp.adjoint(dev(y)))
    ref = gr.adjoint_nufft(y.astype(np.complex128), k, N, G=gp.G, W=W, beta=gp.beta)
    exact = oracle.adjoint(y.astype(np.complex128), k, N)
    e_or, e_ex = rel(b, ref), rel(b, exact)
    bd = max(bound(W, gp.G / N), 1e-7)
    print(f"  G={gp.G} beta={gp.beta:.3f}: vs oracle NUFFT {e_or:.2e}, vs exact sums {e_ex:.2e} "
          f"(bound {bd:.1e})")
    assert e_or < 2e-7
    assert e_ex < bd + 2e-7
    # batch invariance: frame 1 alone gives the same bits
    b1 = host(gp.adjoint(dev(y[1:2])))
    np.testing.assert_array_equal(b1[0], b[1])


def test_gridding_reconstruction_and_density():
    """Density weights (Pipe-Menon) and the weighted gridding image on the
    32^2 workload's spiral."""
    p = synthetic.make_problem(1)
    y = p.measured(oracle.forward(p.x_true, p.k)).astype(np.complex64)
    gp = recon.GridPlan(p.k, p.N, W=7)
    wg = gp.density(10).cpu().numpy()
    wo = gr.density_weights(p.k, p.N, 10, G=gp.G, W=7, beta=gp.beta)
    e = float(np.max(np.abs(wg - wo)) / np.max(np.abs(wo)))
    print(f"density weights, 10 iterations: max rel {e:.2e}")
    assert e < 1e-10
    img = host(gp.adjoint(dev(y), w=dev(wo, np.float64)))
    ref = gr.gridding_recon(y[0].astype(np.complex128), p.k, p.N, wo, G=gp.G, W=7, beta=gp.beta)
    e = rel(img[0], ref)
    print(f"gridding image: rel {e:.2e}")
    assert e < 2e-7


@pytest.mark.parametrize("N,W", [(24, 9), (40, 11)])
def test_nufft_gram_kernel(N, W):
    """Lag kernel and spectrum from the NUFFT against the oracle's NUFFT
    (FP64 both) and the exact sums (within the bound); the FP64 iteration
    on that spectrum equals the oracle's iterate on the same spectrum."""
    rng = np.random.default_rng(N)
    k = synthetic.spiral_trajectory(N, 4, 3 * N, 1.0)
    M = k.shape[0]
    plan = recon.Plan(k, N, prec=recon.FP64_ITER64)
    khat, lag = plan.gram_kernel_nufft(W, want_khat=True, want_lag=True)
    lag = lag.cpu().numpy()
    G = 64
    while G < 4 * N:
        G *= 2
    h_or = gr.lag_kernel_nufft(k, N, G=G, W=W)
    h_ex = gram.lag_kernel(k, N)
    e_or, e_ex = rel(lag, h_or), rel(lag, h_ex)
    print(f"N={N} M={M} W={W}: lag kernel vs oracle NUFFT {e_or:.2e}, vs exact {e_ex:.2e} "
          f"(bound {bound(W, G / (2 * N)):.1e})")
    assert e_or < 1e-12
    assert e_ex < bound(W, G / (2 * N))
    K = gram.khat(k, N, plan.L, h=h_or)
    ek = float(np.max(np.abs(khat.cpu().numpy() - K)) / np.max(np.abs(K)))
    assert ek < 2e-7
    x_true = synthetic.ellipse_phantom(N, 6, rng)
    y = oracle.forward(x_true, k) + 0.01 * synthetic.noise_draws(M, rng)
    y = y.astype(np.complex64)
    x, st = plan.solve(dev(y[None]), 0.02, 0.05, 40)
    xo = oracle.solve(oracle.adjoint(y.astype(np.complex128), k, N), K, 0.02, 0.05, 40)
    e = rel(host(x)[0], xo.astype(np.complex64).astype(np.complex128))
    print(f"  FP64 iteration on the NUFFT spectrum, 40 iterations: rel {e:.2e}")
    assert e < 1e-8


def test_nufft_large_workload_sampled():
    """The large workload's geometry (512^2, M = 262144): NUFFT adjoint and
    lag kernel (grid 2048) on sampled entries against the exact sums."""
    p = synthetic.make_frames(5, frames=1)
    N, k = p.N, p.k
    print(f"large: N={N} M={p.M}", flush=True)
    rng = np.random.default_rng(77)
    y = rand_c(rng, 1, p.M).astype(np.complex64)
    gp = recon.GridPlan(k, N, W=9)
    b = host(gp.adjoint(dev(y)))[0]
    n = np.concatenate([[0, N - 1, 0, N - 1], rng.integers(0, N, 60)])
    m = np.concatenate([[0, N - 1, N - 1, 0], rng.integers(0, N, 60)])
    ref = oracle.adjoint_at(y[0].astype(np.complex128), k, N, n, m)
    e = rel(b[n, m], ref)
    print(f"  adjoint, 64 sampled entries: rel {e:.2e}")
    assert e < max(bound(9, gp.G / N), 1e-7) + 2e-7
    plan = recon.Plan(k, N, p.L, prec=recon.FP64)
    _, lag = plan.gram_kernel_nufft(11, want_lag=True)
    lag = lag.cpu().numpy()
    a = np.concatenate([[0, N - 1, -(N - 1)], rng.integers(-(N - 1), N, 45)])
    bb = np.concatenate([[0, -(N - 1), N - 1], rng.integers(-(N - 1), N, 45)])
    ref = gram.lag_at(k, N, a, bb)
    e = rel(lag[a + N - 1, bb + N - 1], ref)
    print(f"  lag kernel (grid 2048), 48 sampled lags: rel {e:.2e}")
    assert e < bound(11, 2.0)


def test_grid_argument_checks():
    k = np.zeros((10, 2))
    with pytest.raises(recon.ReconError):
        recon.GridPlan(k, 40, G=64)            # 2N > G
    with pytest.raises(recon.ReconError):
        recon.GridPlan(k, 16, W=17)
    bad = k.copy()
    bad[3, 0] = 0.75
    with pytest.raises(recon.ReconError):
        recon.GridPlan(bad, 16)


@pytest.mark.parametrize("name,N,spec,W", [CASES[0], CASES[1]])
def test_nufft_adjoint_fp64_output(name, N, spec, W):
    """recon_grid_adjoint64: the same sums without the final rounding.  Its
    complex64 form is exactly the rounding of this result; against the
    oracle's NUFFT it agrees to FP64 rounding, against the exact sums within
    the bound."""
    k = traj(spec, N, N)
    M = k.shape[0]
    gp = recon.GridPlan(k, N, W=W)
    rng = np.random.default_rng(7 + N)
    y = rand_c(rng, 2, M).astype(np.complex64)
    b64 = gp.adjoint(dev(y), f64=True)
    b32 = gp.adjoint(dev(y))
    torch.cuda.synchronize()
    assert b64.dtype == torch.complex128
    np.testing.assert_array_equal(b64.to(torch.complex64).cpu().numpy(), b32.cpu().numpy())
    b = b64.cpu().numpy()
    ref = gr.adjoint_nufft(y.astype(np.complex128), k, N, G=gp.G, W=W, beta=gp.beta)
    exact = oracle.adjoint(y.astype(np.complex128), k, N)
    e_or, e_ex = rel(b, ref), rel(b, exact)
    print(f"{name}: FP64 output vs oracle NUFFT {e_or:.2e}, vs exact {e_ex:.2e} "
          f"(bound {bound(W, gp.G / N):.1e})")
    assert e_or < 1e-12
    assert e_ex < bound(W, gp.G / N) + 1e-12


def test_fp64_b_into_fp64_iteration():
    """recon_solve_begin_b64: the oracle's exact b (complex128) handed to the
    FP64 iteration without rounding gives the oracle's iterate (32^2 workload,
    200 iterations) to the final complex64 rounding; an FP32-iteration plan
    refuses an FP64 b."""
    p = synthetic.make_problem(1)
    y = p.measured(oracle.forward(p.x_true, p.k)).astype(np.complex64)
    b = oracle.adjoint(y[0].astype(np.complex128), p.k, p.N)
    plan = recon.Plan(p.k, p.N, p.L, prec=recon.FP64_ITER64)
    plan.gram_kernel()
    plan.begin(b=dev(b[None], np.complex128), lam=p.lam, delta=p.delta)
    plan.iterate(p.iters)
    x, st = plan.end()
    K = oracle.khat(p.k, p.N, p.L)
    xo = oracle.solve(b, K, p.lam, p.delta, p.iters)
    e = rel(host(x)[0], xo.astype(np.complex64).astype(np.complex128))
    print(f"FP64 b, 200 iterations: rel {e:.2e}")
    assert e < 1e-8
    assert st["status"][0] == 0
    p32 = recon.Plan(p.k, p.N, p.L, prec=recon.FP64)
    p32.gram_kernel()
    ws, n = p32.workspace(1)
    st = recon.load().recon_solve_begin_b64(p32._h, dev(b[None], np.complex128).data_ptr(), 1,
                                            p.lam, p.delta, 0.0, 1.0, 0, None, ws.data_ptr(),
                                            n, recon._stream())
    assert st == recon.E_ARG


def test_nufft_D_fp64_into_fp64_iteration():
    """Section 5's NUFFT D at W = 15 (bound 3.0e-14), kept in FP64, as the
    FP64 iteration's b on the 32^2 workload: the iterate stays at the
    oracle's exact-sums iterate to the final complex64 rounding."""
    p = synthetic.make_problem(1)
    y = p.measured(oracle.forward(p.x_true, p.k)).astype(np.complex64)
    gp = recon.GridPlan(p.k, p.N, W=15)
    b64 = gp.adjoint(dev(y), f64=True)
    b_ex = oracle.adjoint(y[0].astype(np.complex128), p.k, p.N)
    eb = rel(b64.cpu().numpy()[0], b_ex)
    plan = recon.Plan(p.k, p.N, p.L, prec=recon.FP64_ITER64)
    plan.gram_kernel()
    plan.begin(b=b64, lam=p.lam, delta=p.delta)
    plan.iterate(p.iters)
    x, st = plan.end()
    xo = oracle.solve(b_ex, oracle.khat(p.k, p.N, p.L), p.lam, p.delta, p.iters)
    e = rel(host(x)[0], xo.astype(np.complex64).astype(np.complex128))
    print(f"NUFFT D (W = 15) vs exact sums {eb:.2e}; FP64 iteration from it vs oracle {e:.2e}")
    assert eb < bound(15, gp.G / p.N) + 1e-13
    assert e < 1e-8
