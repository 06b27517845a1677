"""Host-side checks of the C ABI library (no GPU work).

The library must load, export every function include/recon.h declares, size
its buffers consistently, and reject invalid arguments before any launch.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_0908_3252_amd import recon

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "recon.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(recon_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = recon.load()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    # the binding wraps every declared function
    assert lib.recon_version().decode().startswith("recon-mi355x")


def test_size_queries():
    lib = recon.load()
    M, N = 32768, 256
    pb = lib.recon_plan_bytes(M, N, 512, recon.FP32)
    # trajectory + two FP32 phasor tables + twiddles + spectrum
    assert pb >= M * 16 + 2 * M * N * 8 + 512 * 8 + 512 * 512 * 4
    assert lib.recon_plan_bytes(M, N, 0, recon.FP32) == pb  # L = 0 -> 2N rounded to pow2
    w1 = lib.recon_workspace_bytes(M, N, 512, 1, recon.FP32)
    w8 = lib.recon_workspace_bytes(M, N, 512, 8, recon.FP32)
    assert w1 > 0 and w8 > 0
    # per frame: 8 N x N images + the N x L intermediate
    assert w8 >= 8 * (8 * N * N * 8 + N * 512 * 8)
    assert lib.recon_gram_workspace_bytes(M, N, 512) >= 2 * 512 * 512 * 8


def test_fp64_iteration_size_queries():
    """The FP64 iteration flag: FP64 adjoint and L <= 1024 only; the
    workspace holds complex128 images and intermediate."""
    lib = recon.load()
    M, N = 32768, 256
    P = recon.FP64_ITER64
    assert lib.recon_plan_bytes(M, N, 512, P) > lib.recon_plan_bytes(M, N, 512, recon.FP64)
    assert lib.recon_plan_bytes(M, 40, 2048, P) == 0
    assert lib.recon_plan_bytes(M, N, 512, recon.FP32 | recon.ITER_FP64) == 0
    assert lib.recon_workspace_bytes(M, 40, 2048, 1, P) == 0
    w32 = lib.recon_workspace_bytes(M, N, 512, 8, recon.FP64)
    w64 = lib.recon_workspace_bytes(M, N, 512, 8, P)
    # seven N x N images and the N x L intermediate per frame grow 8 -> 16 bytes
    assert w64 - w32 >= 8 * (7 * N * N * 8 + N * 512 * 8)


def test_hq_workspace_is_one_image_more():
    """The half-quadratic workspace adds the frozen image xbar (one N x N
    image per frame, 256-byte aligned) to the solve workspace."""
    lib = recon.load()
    M, N = 32768, 256
    for prec, es in ((recon.FP64, 8), (recon.FP64_ITER64, 16)):
        for B in (1, 8):
            w = lib.recon_workspace_bytes(M, N, 512, B, prec)
            h = lib.recon_hq_workspace_bytes(M, N, 512, B, prec)
            img = B * N * N * es
            assert img <= h - w < img + 256, (prec, B, h - w, img)
    assert lib.recon_hq_workspace_bytes(M, 40, 2048, 1, recon.FP64_ITER64) == 0


@pytest.mark.parametrize("M,N,L", [(10, 1, 64), (10, 2000, 4096), (10, 64, 96), (10, 64, 64),
                                   (0, 32, 64), (10, 32, 32)])
def test_invalid_geometry_sizes_are_zero(M, N, L):
    lib = recon.load()
    assert lib.recon_plan_bytes(M, N, L, 0) == 0
    assert lib.recon_workspace_bytes(M, N, L, 1, 0) == 0


def test_plan_rejects_bad_trajectory_before_any_launch():
    lib = recon.load()
    h = ctypes.c_void_p()
    k = np.zeros((4, 2))
    k[1, 0] = 0.75  # |k| > 0.5
    st = lib.recon_plan(k.ctypes.data, 4, 8, 64, 0, ctypes.c_void_p(256), 1 << 30, None,
                        ctypes.byref(h))
    assert st == recon.E_RANGE
    assert b"trajectory" in lib.recon_last_error()
    k[1, 0] = np.nan
    st = lib.recon_plan(k.ctypes.data, 4, 8, 64, 0, ctypes.c_void_p(256), 1 << 30, None,
                        ctypes.byref(h))
    assert st == recon.E_RANGE
    k[1, 0] = 0.1
    # plan memory too small
    st = lib.recon_plan(k.ctypes.data, 4, 8, 64, 0, ctypes.c_void_p(256), 16, None,
                        ctypes.byref(h))
    assert st == recon.E_NOMEM
    # null pointers and unknown precision
    assert lib.recon_plan(None, 4, 8, 64, 0, ctypes.c_void_p(256), 1 << 30, None,
                          ctypes.byref(h)) == recon.E_ARG
    assert lib.recon_plan(k.ctypes.data, 4, 8, 64, 7, ctypes.c_void_p(256), 1 << 30, None,
                          ctypes.byref(h)) == recon.E_ARG
    # L < 2N - 1
    assert lib.recon_plan(k.ctypes.data, 4, 40, 64, 0, ctypes.c_void_p(256), 1 << 30, None,
                          ctypes.byref(h)) == recon.E_RANGE


def test_status_strings():
    lib = recon.load()
    for s in range(7):
        assert lib.recon_status_string(s)


def test_fp64_b_and_grid_adjoint64_reject_null_arguments_before_any_launch():
    """recon_solve_begin_b64 and recon_grid_adjoint64 validate their pointers
    on the host (no plan, no device memory needed)."""
    lib = recon.load()
    # NULL plan / NULL b
    assert lib.recon_solve_begin_b64(None, ctypes.c_void_p(256), 1, 0.01, 0.02, 0.0, 1.0, 0,
                                     None, ctypes.c_void_p(256), 1 << 20, None) == recon.E_ARG
    assert lib.recon_solve_begin_b64(ctypes.c_void_p(256), None, 1, 0.01, 0.02, 0.0, 1.0, 0,
                                     None, ctypes.c_void_p(256), 1 << 20, None) == recon.E_ARG
    assert b"b" in lib.recon_last_error()
    # NULL grid plan, output or workspace
    assert lib.recon_grid_adjoint64(None, ctypes.c_void_p(256), None, 1, ctypes.c_void_p(256),
                                    ctypes.c_void_p(256), 1 << 20, None) == recon.E_ARG
