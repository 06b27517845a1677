"""GPU: the allocation-free Gram apply (recon_gram_apply_noalloc) against
recon_gram_apply with a caller workspace, through the C ABI: two calls in a
row on one plan, the second with fewer frames, and a call on a second plan of
another geometry; both must give bitwise the workspace form's output (same
kernels, same inputs).  Oversized requests are refused before any launch."""
import ctypes

import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_0908_3252_amd import recon  # noqa: E402


def _plan(N, I, S, L=0):
    k = synthetic.spiral_trajectory(N, I, S, 2.0)
    plan = recon.Plan(k, N, L)
    plan.gram_kernel()
    return plan


def _apply_ws(lib, plan, v):
    B = v.shape[0]
    out = torch.empty_like(v)
    ws, n = plan.workspace(B)
    recon._check(lib.recon_gram_apply(plan.handle, v.data_ptr(), B, out.data_ptr(), ws.data_ptr(),
                                      n, recon._stream()))
    return out


def _apply_noalloc(lib, plan, v):
    B = v.shape[0]
    out = torch.empty_like(v)
    recon._check(lib.recon_gram_apply_noalloc(plan.handle, v.data_ptr(), B, out.data_ptr(),
                                              recon._stream()))
    return out


def bitwise(a, b):
    return torch.equal(a.contiguous().view(torch.float32), b.contiguous().view(torch.float32))


def test_noalloc_gram_apply_matches_workspace_form():
    lib = recon.load()
    assert lib.recon_gram_apply_noalloc_max_bytes() == 64 << 20
    rng = np.random.default_rng(5)
    p1 = _plan(256, 16, 2048)
    p2 = _plan(100, 8, 600)
    print(f"noalloc Gram apply: N=256 L={p1.L} B=40 then B=3; N=100 L={p2.L} B=5", flush=True)
    for plan, B in ((p1, 40), (p1, 3), (p2, 5)):
        v = torch.from_numpy((rng.standard_normal((B, plan.N, plan.N))
                              + 1j * rng.standard_normal((B, plan.N, plan.N))).astype(np.complex64)).cuda()
        a = _apply_noalloc(lib, plan, v)
        b = _apply_ws(lib, plan, v)
        torch.cuda.synchronize()
        assert bitwise(a, b), (plan.N, B)
    # 65 frames of 256 x 512 complex64 rows exceed the 64 MiB scratch
    v = torch.zeros((65, 256, 256), dtype=torch.complex64, device="cuda")
    out = torch.empty_like(v)
    st = lib.recon_gram_apply_noalloc(p1.handle, v.data_ptr(), 65, out.data_ptr(), recon._stream())
    assert st == recon.E_RANGE
    assert b"64 MiB" in lib.recon_last_error()
