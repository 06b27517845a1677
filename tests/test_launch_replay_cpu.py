"""CPU replay of the global-memory extents of the launches that a batch of
non-FP64-adjoint frames runs (the case switched off after an unexplained GPU
fault: FP32 and split BF16 / FP16 x3 plans refuse more than 64 frames per
call).

For every launch of that sequence -- frame sums, the FP32 and split adjoint
contractions with their split-K reductions, the split frame scaling, the
FP32 and split forward contractions, and the initial state of the FP32
iteration -- the largest element index each kernel's grid and index
expressions reach in every buffer is computed on the host and compared with
the buffer's extent: the caller's y / x / b arrays, the plan regions and
the workspace regions of the library's own layouts.  The launch shapes
(split-K counts, frames per launch, padded table sizes) are taken from the
built library itself; the index expressions are those of the kernels
(nudft.hip, nudft_split.hip, cg.hip) written out in Python, and the region
sizes follow the layout functions of api.cpp.  It runs the sizes of the
256^2 series (M = 32768) at B = 64 and B = 128 and the serving sizes.

It also checks the earlier suspicion about the faulting run (an FP16 x3
forward model inside an FP64 plan, which has no split tables, so a split
launcher would read its tables at plan offset 0): such reads stay inside
the FP64 plan's memory, so they could give wrong values but not an access
fault.
"""
import ctypes
import os

import pytest

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_0908_3252_amd", "librecon.so")

C64, C128, F32, F64 = 8, 16, 4, 8
NT = 64          # FP32 adjoint / forward output tile
KT = 16          # FP32 adjoint samples per stage
ST, SK = 64, 32  # split contractions: tile, samples per stage
SUMSQ_BLOCKS = 64


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    L = ctypes.CDLL(LIB)

    def fn(name, res, *args):
        f = getattr(L, name)
        f.restype, f.argtypes = res, list(args)
        return f

    i64, i32 = ctypes.c_int64, ctypes.c_int32
    return dict(
        adj_splits=fn("_ZN5recon14adjoint_splitsEli", i32, i64, i32),
        adj_group=fn("_ZN5recon13adjoint_groupEli", i32, i64, i32),
        adj64_splits=fn("_ZN5recon16adjoint64_splitsEli", i32, i64, i32),
        adj64_group=fn("_ZN5recon15adjoint64_groupEli", i32, i64, i32),
        pad_M=fn("_ZN5recon11split_pad_MEl", i64, i64),
        pad_N=fn("_ZN5recon11split_pad_NEi", i32, i32),
        sumsq_parts=fn("_ZN5recon11sumsq_partsEv", i32),
        plan_bytes=fn("recon_plan_bytes", ctypes.c_size_t, i64, i32, i32, i32),
        ws_bytes=fn("recon_workspace_bytes", ctypes.c_size_t, i64, i32, i32, i32, i32),
    )


def cdiv(a, b):
    return -(-a // b)


class Buf:
    """A buffer of `n` elements; `touch` records the largest index used."""

    def __init__(self, name, n):
        self.name, self.n, self.hi = name, n, -1

    def touch(self, idx):
        assert idx >= 0, (self.name, idx)
        self.hi = max(self.hi, idx)

    def ok(self):
        return self.hi < self.n


def workspace_regions(lib, M, N, L, B):
    """Element extents of the workspace regions the sequence uses (the
    layout of api.cpp for the FP32 iteration)."""
    img = B * N * N
    sp, g = lib["adj_splits"](M, N), lib["adj_group"](M, N)
    a32 = sp * min(g, B) if sp > 1 else 0
    sp64, g64 = lib["adj64_splits"](M, N), lib["adj64_group"](M, N)
    a64 = sp64 * min(g64, B) if sp64 > 1 else 0
    rows = 2048 // L if L != 1024 else 4
    nb4 = cdiv(N, rows)
    return dict(b=img, x=img, r=img, d=img, qd=img,
                adj_c64=max(a32, a64) * N * N * C128 // C64,
                sc=B, yyp=B * lib["sumsq_parts"](), yy=B, p4=B * nb4 * 4, pg0=B * nb4), nb4


def replay_sumsq(M, B, y, yyp):
    chunk = cdiv(M, SUMSQ_BLOCKS)
    for f in (0, B - 1):
        for s in (0, SUMSQ_BLOCKS - 1):
            lo, hi = s * chunk, min(s * chunk + chunk, M)
            if hi > lo:
                y.touch(f * M + hi - 1)
            yyp.touch(f * SUMSQ_BLOCKS + s)


def replay_adjoint(M, N, B, splits, group, y, ex, ey, part, b, split_tables=None, sc=None):
    """FP32 adjoint (split_tables None) or split adjoint (tables (at, Mp))."""
    tile = NT if split_tables is None else ST
    kstep = KT if split_tables is None else SK
    per = cdiv(cdiv(M, splits), kstep) * kstep
    if splits == 1:
        groups = [(0, B)]
    else:
        groups = [(f0, min(group, B - f0)) for f0 in range(0, B, group)]
    for f0, g in groups:
        for s in range(splits):
            lb = s * per
            le = min(lb + per, M)
            if le <= lb:
                continue
            for f in (0, g - 1):
                y.touch((f0 + f) * M + le - 1)
                if sc is not None:
                    sc.touch(f0 + f)
                ex.touch((le - 1) * N + N - 1)
                if split_tables is None:
                    ey.touch((le - 1) * N + N - 1)
                else:
                    at, Mp = split_tables
                    # A staging: 32 consecutive samples of row n from l0 (<= le - 1)
                    l0 = lb + ((le - 1 - lb) // kstep) * kstep
                    at.touch(3 * N * Mp + (N - 1) * Mp + l0 + kstep - 1)
                n_hi = min(cdiv(N, tile) * tile, N) - 1
                o = part if splits > 1 else b
                base = (s * g + f) * N * N if splits > 1 else (f0 + f) * N * N
                o.touch(base + n_hi * N + n_hi)
        if splits > 1:
            count = g * N * N
            part.touch((splits - 1) * count + count - 1)
            b.touch(f0 * N * N + count - 1)


def replay_forward(M, N, B, x, ex, ey, y, split_tables=None, sc=None):
    for f in (0, B - 1):
        x.touch(f * N * N + (N - 1) * N + N - 1)
        if sc is not None:
            sc.touch(f)
        if split_tables is None:
            ex.touch((M - 1) * N + N - 1)
        else:
            xs, Np = split_tables
            m0 = ((N - 1) // SK) * SK
            xs.touch(3 * M * Np + (M - 1) * Np + m0 + SK - 1)
        ey.touch((M - 1) * N + N - 1)
        y.touch(f * M + M - 1)


def replay_init(N, B, nb4, ws_bufs):
    for name in ("b", "x", "r", "d"):
        ws_bufs[name].touch((B - 1) * N * N + N * N - 1)
    ws_bufs["p4"].touch(((B - 1) * nb4 + nb4 - 1) * 4 + 3)
    ws_bufs["pg0"].touch((B - 1) * nb4 + nb4 - 1)


@pytest.mark.parametrize("M,N,L,B", [(32768, 256, 512, 64), (32768, 256, 512, 128),
                                     (32768, 256, 512, 1), (2048, 64, 128, 64),
                                     (18432, 192, 512, 128), (294912, 384, 1024, 16)])
@pytest.mark.parametrize("split", [False, True])
def test_non_fp64_sequence_stays_in_bounds(lib, M, N, L, B, split):
    regions, nb4 = workspace_regions(lib, M, N, L, B)
    ws = {k: Buf(k, v) for k, v in regions.items()}
    y = Buf("y", B * M)
    x = Buf("x_out", B * N * N)
    yfit = Buf("y_fit", B * M)
    b = ws["b"]
    ex = Buf("ex", M * N)
    ey = Buf("ey", M * N)
    replay_sumsq(M, B, y, ws["yyp"])
    sp, g = lib["adj_splits"](M, N), lib["adj_group"](M, N)
    if split:
        Mp, Np = lib["pad_M"](M), lib["pad_N"](N)
        at = Buf("at", 4 * N * Mp)
        xs = Buf("xs", 4 * M * Np)
        replay_adjoint(M, N, B, sp, g, y, ex, ey, ws["adj_c64"], b, (at, Mp), ws["sc"])
        replay_forward(M, N, B, x, ex, ey, yfit, (xs, Np), ws["sc"])
        tables = [at, xs]
    else:
        replay_adjoint(M, N, B, sp, g, y, ex, ey, ws["adj_c64"], b)
        replay_forward(M, N, B, x, ex, ey, yfit)
        tables = []
    replay_init(N, B, nb4, ws)
    bad = [(buf.name, buf.hi, buf.n) for buf in [y, x, yfit, ex, ey] + tables + list(ws.values())
           if not buf.ok()]
    assert not bad, bad
    # the workspace the library asks for holds every region
    total = sum(v * (C64 if k not in ("sc", "yyp", "yy", "p4", "pg0") else F64)
                for k, v in regions.items())
    assert lib["ws_bytes"](M, N, L, B, 0) >= total


def test_split_tables_at_offset_zero_of_an_fp64_plan_stay_inside_it(lib):
    """A split forward launched on an FP64 plan (no split tables: the layout
    leaves their offsets at 0) would read 4 M Np 16-bit entries from the
    start of the plan: inside the plan's memory at the benchmark's size, so
    no access fault, only wrong values."""
    M, N, L = 32768, 256, 512
    Np = lib["pad_N"](N)
    reach = 4 * M * Np * 2
    plan_total = lib["plan_bytes"](M, N, L, 3)
    assert 0 < reach <= plan_total, (reach, plan_total)
