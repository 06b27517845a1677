"""GPU: slot pools (continuous batching) against standalone solves.

A frame that joins a pool at any iteration, shares it with frames that start
and stop at other iterations, and leaves when its own budget is used up must
give bitwise the image and statistics of recon_solve on that frame alone
(B = 1, x0 = 0): every iteration kernel skips idle slots as whole blocks, and
each frame's arithmetic and reduction order do not depend on its slot or on
the pool's size.  The standalone solve is itself held to the FP64 oracle by
the parity tests.
"""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_0908_3252_amd import recon  # noqa: E402


def frames_for(N, I, S, R, F, seed):
    k = synthetic.spiral_trajectory(N, I, S, R)
    xs = []
    for f in range(F):
        rng = np.random.default_rng([seed, f])
        xs.append(synthetic.ellipse_phantom(N, 10, rng))
    return k, np.array(xs)


def measured(plan, xs, c, seed):
    x = torch.from_numpy(xs.astype(np.complex64)).cuda()
    y0 = plan.forward(x)
    rng = np.random.default_rng([seed, 77])
    nz = torch.from_numpy(synthetic.noise_draws(y0.numel(), rng).reshape(y0.shape)
                          .astype(np.complex64)).cuda()
    sig = c * y0.abs().amax(dim=1, keepdim=True)
    return (y0 + sig * nz).contiguous()


def bitwise(a, b):
    return torch.equal(a.contiguous().view(torch.float32), b.contiguous().view(torch.float32))


def standalone(plan, y, lam, delta, iters):
    x, st = plan.solve(y[None], lam, delta, iters)
    torch.cuda.synchronize()
    return x[0], st[0]


@pytest.mark.parametrize("prec", [recon.FP64, recon.FP64_ITER64])
@pytest.mark.parametrize("N,I,S,R,L", [(32, 4, 256, 1.0, 64), (48, 5, 199, 1.0, 128)])
def test_pool_matches_standalone_bitwise(N, I, S, R, L, prec):
    k, xs = frames_for(N, I, S, R, 6, seed=N)
    plan = recon.Plan(k, N, L, prec=prec)
    plan.gram_kernel()
    y = measured(plan, xs, 0.01, N)
    lam, delta = [0.02, 0.01, 0.03, 0.02, 0.015, 0.05], [0.05, 0.02, 0.1, 0.05, 0.03, 0.05]
    budget = [40, 25, 0, 30, 17, 9]
    print(f"pool N={N} L={L} prec={prec} slots=3 budgets={budget}", flush=True)
    pool = recon.Pool(plan, 3)
    out = {}

    def retire(slot, f):
        x = torch.empty((N, N), dtype=torch.complex64, device="cuda")
        st = torch.empty(recon.STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        pool.retire(slot, x, stats_out=st)
        out[f] = (x, st)

    pool.admit(0, y[0], lam[0], delta[0], budget[0])        # k = 0, stops at 40
    pool.step(10)
    pool.admit(1, y[1], lam[1], delta[1], budget[1])        # k = 10, stops at 35
    pool.step(7)
    pool.admit(2, y[2], lam[2], delta[2], budget[2])        # k = 17, zero budget
    retire(2, 2)
    pool.admit(2, y[3], lam[3], delta[3], budget[3])        # k = 17, stops at 47
    pool.step(18)                                           # k = 35
    retire(1, 1)
    pool.admit(1, y[4], lam[4], delta[4], budget[4])        # k = 35, stops at 52
    pool.step(5)                                            # k = 40
    retire(0, 0)
    pool.admit(0, y[5], lam[5], delta[5], budget[5])        # k = 40, stops at 49
    assert pool.iteration == 40
    pool.step(12)                                           # k = 52 (slot 0 froze at 49)
    retire(0, 5)
    retire(2, 3)
    retire(1, 4)
    torch.cuda.synchronize()
    for f in range(6):
        xr, sr = standalone(plan, y[f], lam[f], delta[f], budget[f])
        x, st = out[f]
        s = np.frombuffer(st.cpu().numpy().tobytes(), dtype=recon.STATS_DTYPE)[0]
        print(f"frame {f}: iters {s['iters_done']} J {s['J']:.6e} ref {sr['J']:.6e}")
        assert bitwise(x, xr), f"frame {f} differs from its standalone solve"
        assert s["iters_done"] == budget[f] == sr["iters_done"]
        assert s["J"] == sr["J"] and s["grad_ratio"] == sr["grad_ratio"]
        assert s["status"] == 0


def test_pool_plain_workload_shape_bitwise():
    """256 x 256, M = 32768 (the plain workload's trajectory), two frames
    admitted 13 iterations apart into a 4-slot pool."""
    p = synthetic.make_frames(3, frames=2)
    plan = recon.Plan(p.k, p.N, p.L, prec=recon.FP64)
    plan.gram_kernel()
    x = torch.from_numpy(p.x_true.astype(np.complex64)).cuda()
    y0 = plan.forward(x)
    nz = torch.from_numpy(p.noise.astype(np.complex64)).cuda()
    y = (y0 + p.noise_c * y0.abs().amax(dim=1, keepdim=True) * nz).contiguous()
    print("pool 256x256 M=32768 slots=4", flush=True)
    pool = recon.Pool(plan, 4)
    pool.admit(3, y[0], p.lam, p.delta, 30)
    pool.step(13)
    pool.admit(1, y[1], p.lam, p.delta, 30)
    pool.step(17)
    x0 = torch.empty((p.N, p.N), dtype=torch.complex64, device="cuda")
    pool.retire(3, x0)
    pool.step(13)
    x1 = torch.empty((p.N, p.N), dtype=torch.complex64, device="cuda")
    pool.retire(1, x1)
    for f, xg in ((0, x0), (1, x1)):
        xr, _ = standalone(plan, y[f], p.lam, p.delta, 30)
        assert bitwise(xg, xr), f"frame {f}"


@pytest.mark.parametrize("prec", [recon.FP64, recon.FP64_ITER64])
def test_pool_launch_range_follows_running_slots(prec):
    """A pool step launches over the slots up to the highest running one: a
    step with only slot 1 running (slots 2..5 idle), then slot 5 admitted
    while slot 1 still runs, then slot 1 finishing first.  Both results equal
    their standalone solves bit for bit."""
    p = synthetic.make_frames(3, frames=2, N=48, S=192, I=8, K=10)
    plan = recon.Plan(p.k, p.N, prec=prec)
    plan.gram_kernel()
    y0 = plan.forward(torch.from_numpy(p.x_true.astype(np.complex64)).cuda())
    nz = torch.from_numpy(p.noise.astype(np.complex64)).cuda()
    y = (y0 + p.noise_c * y0.abs().amax(dim=1, keepdim=True) * nz).contiguous()
    pool = recon.Pool(plan, 6)
    pool.admit(1, y[0], p.lam, p.delta, 20)   # k = 0, stops at 20
    pool.step(8)                              # launches cover slots 0..1
    pool.admit(5, y[1], p.lam, p.delta, 15)   # k = 8, stops at 23
    pool.step(12)                             # k = 20: slot 1 done
    x0 = torch.empty((p.N, p.N), dtype=torch.complex64, device="cuda")
    pool.retire(1, x0)
    pool.step(3)                              # k = 23: slots 0..5, slot 5 only
    x1 = torch.empty((p.N, p.N), dtype=torch.complex64, device="cuda")
    pool.retire(5, x1)
    pool.step(4)                              # nothing running: no launch
    for f, xg, it in ((0, x0, 20), (1, x1, 15)):
        xr, _ = standalone(plan, y[f], p.lam, p.delta, it)
        assert bitwise(xg, xr), f"frame {f}"


def test_pool_state_errors():
    N, L = 32, 64
    k, xs = frames_for(N, 4, 256, 1.0, 2, seed=5)
    plan = recon.Plan(k, N, L, prec=recon.FP64)
    plan.gram_kernel()
    y = measured(plan, xs, 0.01, 5)
    pool = recon.Pool(plan, 2)
    pool.admit(0, y[0], 0.02, 0.05, 5)
    with pytest.raises(recon.ReconError) as e:
        pool.admit(0, y[1], 0.02, 0.05, 5)       # slot busy
    assert e.value.status == recon.E_STATE
    with pytest.raises(recon.ReconError) as e:
        pool.retire(0)                            # budget not used up
    assert e.value.status == recon.E_STATE
    with pytest.raises(recon.ReconError) as e:
        pool.admit(2, y[1], 0.02, 0.05, 5)       # no such slot
    assert e.value.status == recon.E_RANGE
    with pytest.raises(recon.ReconError) as e:   # resumable-solve calls refuse a pool
        recon._check(recon.load().recon_solve_iterate(plan.handle, 1, pool.ws.data_ptr(),
                                                      pool.nbytes, recon._stream()))
    assert e.value.status == recon.E_STATE
    pool.step(5)
    pool.retire(0)
    torch.cuda.synchronize()


def test_scheduler_serves_mixed_requests_bitwise():
    """The serving loop on a short Poisson stream of mixed image sizes: every
    request completes and equals its standalone solve bitwise."""
    from paper_0908_3252_amd import serving
    wl = serving.make_workload(8, seed=11)
    print("serving 8 requests", [b["key"] for b in wl[0]], flush=True)
    out = serving.serve(400.0, wl, warmup_frac=0.0, chunk=20, streams=2, verify=8, seed=11)
    print(out)
    assert out["completed"] == 8
    assert out["status_ok"] == 8
    assert out["bitwise_equal_standalone"] == "8/8"
