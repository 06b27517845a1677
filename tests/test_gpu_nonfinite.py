"""GPU: a non-finite value in one frame stays in that frame.

Every reduction of the iteration is per frame (per-block partials summed by
the consumer for that frame only), so a NaN in one frame's data must leave
the other frames bitwise as their clean solves give them, and the poisoned
frame must report RECON_E_NONFINITE (6) in its statistics.  Checked for a
batched solve (B = 3, NaN in frame 1) and for a slot pool, with the FP32 and
the FP64 iteration.
"""
import numpy as np
import pytest

import oracle
import synthetic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_0908_3252_amd import recon  # noqa: E402

E_NONFINITE = 6


def _inputs():
    p = synthetic.make_frames(3, frames=3, N=48, S=256, I=6, K=8)
    y = p.measured(oracle.forward(p.x_true, p.k)).astype(np.complex64)
    return p, y


def bitwise(a, b):
    return torch.equal(a.contiguous().view(torch.float32), b.contiguous().view(torch.float32))


@pytest.mark.parametrize("prec", [recon.FP64, recon.FP64_ITER64])
def test_nan_frame_is_isolated_in_a_batch(prec):
    p, y = _inputs()
    plan = recon.Plan(p.k, p.N, prec=prec)
    plan.gram_kernel()
    clean = torch.from_numpy(y).cuda()
    bad = clean.clone()
    bad[1, 17] = complex(float("nan"), 0.0)
    print(f"batch of 3, NaN in frame 1, prec={prec}", flush=True)
    xc, stc = plan.solve(clean, p.lam, p.delta, 25)
    xb, stb = plan.solve(bad, p.lam, p.delta, 25)
    torch.cuda.synchronize()
    print(f"  status clean {list(stc['status'])}, poisoned {list(stb['status'])}")
    assert list(stc["status"]) == [0, 0, 0]
    assert stb["status"][1] == E_NONFINITE
    assert stb["status"][0] == 0 and stb["status"][2] == 0
    for f in (0, 2):
        assert bitwise(xb[f], xc[f]), f
        assert stb["J"][f] == stc["J"][f]


@pytest.mark.parametrize("prec", [recon.FP64, recon.FP64_ITER64])
def test_nan_slot_is_isolated_in_a_pool(prec):
    p, y = _inputs()
    plan = recon.Plan(p.k, p.N, prec=prec)
    plan.gram_kernel()
    yd = torch.from_numpy(y).cuda()
    bad = yd[1].clone()
    bad[5] = complex(float("inf"), 0.0)
    print(f"pool of 3 slots, Inf in slot 1, prec={prec}", flush=True)
    ref = []
    for f in (0, 2):
        x, st = plan.solve(yd[f:f + 1], p.lam, p.delta, 20)
        ref.append((x[0], st[0]))
    pool = recon.Pool(plan, 3)
    pool.admit(0, yd[0], p.lam, p.delta, 20)
    pool.admit(1, bad, p.lam, p.delta, 20)
    pool.step(4)
    pool.admit(2, yd[2], p.lam, p.delta, 20)
    pool.step(20)
    outs = {}
    for s in range(3):
        outs[s] = torch.empty((p.N, p.N), dtype=torch.complex64, device="cuda")
        pool.retire(s, outs[s])
    st = pool.read_stats([0, 1, 2])
    print(f"  pool statuses {list(st['status'])}")
    assert st["status"][1] == E_NONFINITE
    assert st["status"][0] == 0 and st["status"][2] == 0
    assert bitwise(outs[0], ref[0][0]) and bitwise(outs[2], ref[1][0])
    assert st["J"][0] == ref[0][1]["J"] and st["J"][2] == ref[1][1]["J"]
