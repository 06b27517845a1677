"""Every frame of the 128-frame 256^2 series (Section 4.2's dynamic
setting; 300 iterations of the pseudo-CG of Section 3.3, FP64 iteration)
against the FP64 oracle run frame by frame on oracle-made data.

On most frames the GPU and the oracle agree to ~1e-9 (the complex64 output
rounding aside).  On a few, the fixed-budget iterate is not determined by
the FP64 arithmetic to better than ~1e-3: the oracle itself moves that much
when b changes by 1e-14 (relative), with no restart involved, because the
trajectory amplifies perturbations by ~1e11 over the 300 iterations.  No
implementation that does not repeat the oracle's roundings step for step can
meet a fixed bar there.  The test therefore holds every frame to 1e-6, and a
frame that misses it to the oracle's own sensitivity there: with s the
oracle's move under a random 1e-14 change of b, the GPU's distance must stay
below 100 s (an effective perturbation of at most 1e-12 from the different
rounding order of its transforms and sums).  A frame off the oracle by more
than its own rounding sensitivity explains fails.  All frames must end finite
with status OK.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synthetic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_0908_3252_amd import recon  # noqa: E402

BAR = 1e-6          # GPU vs oracle, unless the oracle's own sensitivity explains more
PERTURB = 1e-14     # relative change of b that measures that sensitivity
EXPLAINED = 100.0   # GPU distance allowed per unit of the oracle's own move


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _workers():
    return max(1, min(16, os.cpu_count() or 1))


CHUNK = 16  # frames per test (progress is reported per chunk)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("first", list(range(0, 128, CHUNK)))
def test_series_frames_against_oracle(first):
    from threadpoolctl import threadpool_limits
    prob = synthetic.make_frames(3, frames=CHUNK, first=first)  # frames of the 128-frame series
    N, L, it = prob.N, prob.L, prob.iters
    F = prob.frames
    with threadpool_limits(limits=1), ThreadPoolExecutor(_workers()) as ex:
        y0 = np.concatenate(list(ex.map(lambda f: oracle.forward(prob.x_true[f:f + 1], prob.k),
                                        range(F))))
    y = prob.measured(y0).astype(np.complex64)
    print(f"series frames {first}..{first + F - 1}: N={N}, M={prob.M}, {it} iterations",
          flush=True)
    plan = recon.Plan(prob.k, N, L, prec=recon.FP64_ITER64)
    plan.gram_kernel()
    x, st = plan.solve(torch.from_numpy(y).cuda(), prob.lam, prob.delta, it)
    torch.cuda.synchronize()
    xg = x.cpu().numpy().astype(np.complex128)
    assert np.all(st["status"] == 0)
    assert np.all(np.isfinite(xg))
    K = oracle.khat(prob.k, N, L)
    yc = y.astype(np.complex128)

    def frame(f):
        b = oracle.adjoint(yc[f], prob.k, N)
        xo = oracle.solve(b, K, prob.lam, prob.delta, it)
        e = _rel(xg[f], xo.astype(np.complex64).astype(np.complex128))
        s = None
        if e > BAR:
            rng = np.random.default_rng(first + f)
            db = rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape)
            db *= PERTURB * np.linalg.norm(b) / np.linalg.norm(db)
            s = _rel(oracle.solve(b + db, K, prob.lam, prob.delta, it), xo)
        return first + f, e, s

    with threadpool_limits(limits=1), ThreadPoolExecutor(_workers()) as ex:
        res = list(ex.map(frame, range(F)))
    e = np.array([r[1] for r in res])
    print(f"GPU vs oracle: median {np.median(e):.2e}, max {e.max():.2e}; within 1e-4: "
          f"{(e <= 1e-4).sum()} / {F}, within {BAR:g}: {(e <= BAR).sum()} / {F}")
    bad = []
    for f, ef, sf in res:
        if ef <= BAR:
            continue
        print(f"  frame {f}: GPU vs oracle {ef:.2e}; oracle's own move under a {PERTURB:g} "
              f"change of b: {sf:.2e}")
        if ef > EXPLAINED * sf:
            bad.append((f, ef, sf))
    assert not bad, f"frames off the oracle beyond its own sensitivity: {bad}"
