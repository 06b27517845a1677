"""ctypes binding of librecon.so (the C ABI in include/recon.h).

Argument marshalling only: every step of the reconstruction runs in the HIP
library.  PyTorch supplies device memory (complex64 / uint8 tensors) and the
current HIP stream.  The library must have been built (``build.py``); a
missing library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librecon.so")

OK, E_ARG, E_RANGE, E_NOMEM, E_HIP, E_STATE, E_NONFINITE = range(7)
FP32, BF16X3, FP16X3, FP64 = 0, 1, 2, 3
# Flag OR'ed into FP64: the iteration itself in FP64 (state, FFTs, spectrum).
ITER_FP64 = 16
FP64_ITER64 = FP64 | ITER_FP64
PHI = {"hyperbolic": 0, "huber": 1, "quadratic": 2}
FIELD = {"x": 0, "r": 1, "g": 2, "d": 3, "b": 4}

STATS_DTYPE = np.dtype([("J", "<f8"), ("grad_ratio", "<f8"), ("gnorm0", "<f8"),
                        ("iters_done", "<i4"), ("status", "<i4")])

_lib = None


class ReconError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"recon status {status}: {detail}")
        self.status = status


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          f"python -m paper_0908_3252_amd.build")
    lib = ctypes.CDLL(path)
    c = ctypes
    vp, i32, i64, sz, f64 = c.c_void_p, c.c_int32, c.c_int64, c.c_size_t, c.c_double
    sig = {
        "recon_plan_bytes": (sz, [i64, i32, i32, i32]),
        "recon_gram_workspace_bytes": (sz, [i64, i32, i32]),
        "recon_workspace_bytes": (sz, [i64, i32, i32, i32, i32]),
        "recon_plan": (i32, [vp, i64, i32, i32, i32, vp, sz, vp, c.POINTER(vp)]),
        "recon_plan_info": (i32, [vp, c.POINTER(i64), c.POINTER(i32), c.POINTER(i32),
                                  c.POINTER(i32)]),
        "recon_plan_destroy": (None, [vp]),
        "recon_gram_kernel": (i32, [vp, vp, sz, vp, vp, vp]),
        "recon_adjoint": (i32, [vp, vp, i32, vp, vp, vp, sz, vp]),
        "recon_forward": (i32, [vp, vp, i32, vp, vp, sz, vp]),
        "recon_gram_apply": (i32, [vp, vp, i32, vp, vp, sz, vp]),
        "recon_solve": (i32, [vp, vp, i32, f64, f64, i32, i32, vp, i32, vp, sz, vp, vp]),
        "recon_solve_begin": (i32, [vp, vp, vp, i32, f64, f64, f64, f64, i32, vp, vp, sz, vp]),
        "recon_solve_begin_b64": (i32, [vp, vp, i32, f64, f64, f64, f64, i32, vp, vp, sz, vp]),
        "recon_solve_iterate": (i32, [vp, i32, vp, sz, vp]),
        "recon_solve_end": (i32, [vp, vp, vp, vp, sz, vp]),
        "recon_solve_export": (i32, [vp, i32, vp, vp, sz, vp]),
        "recon_hq_workspace_bytes": (sz, [i64, i32, i32, i32, i32]),
        "recon_solve_hq": (i32, [vp, vp, i32, f64, f64, i32, i32, i32, vp, i32, vp, sz, vp,
                                 vp]),
        "recon_solve_hq_iterate": (i32, [vp, i32, i32, vp, sz, vp]),
        "recon_grid_bytes": (sz, [i64, i32, i32, i32]),
        "recon_grid_plan": (i32, [vp, i64, i32, i32, i32, f64, vp, sz, vp, c.POINTER(vp)]),
        "recon_grid_info": (i32, [vp, c.POINTER(i32), c.POINTER(i32), c.POINTER(f64)]),
        "recon_grid_destroy": (None, [vp]),
        "recon_grid_workspace_bytes": (sz, [vp, i32]),
        "recon_grid_adjoint": (i32, [vp, vp, vp, i32, vp, vp, sz, vp]),
        "recon_grid_adjoint64": (i32, [vp, vp, vp, i32, vp, vp, sz, vp]),
        "recon_grid_density": (i32, [vp, i32, vp, vp, sz, vp]),
        "recon_gram_nufft_workspace_bytes": (sz, [i64, i32, i32, i32]),
        "recon_gram_kernel_nufft": (i32, [vp, i32, vp, sz, vp, vp, vp]),
        "recon_gram_apply_noalloc_max_bytes": (sz, []),
        "recon_gram_apply_noalloc": (i32, [vp, vp, i32, vp, vp]),
        "recon_pool_reset": (i32, [vp, i32, i32, vp, sz, vp]),
        "recon_pool_admit": (i32, [vp, i32, vp, f64, f64, f64, f64, i32, vp, sz, vp]),
        "recon_pool_step": (i32, [vp, i32, vp, sz, vp]),
        "recon_pool_retire": (i32, [vp, i32, vp, vp, vp, sz, vp]),
        "recon_pool_iteration": (i64, [vp, vp]),
        "recon_trace_enable": (i32, [i32, i32]),
        "recon_trace_read": (i32, [c.POINTER(c.c_float), i32]),
        "recon_trace_enable_set": (i32, [c.c_uint32, i32]),
        "recon_trace_read_kind": (i32, [i32, c.POINTER(c.c_float), i32]),
        "recon_status_string": (c.c_char_p, [i32]),
        "recon_last_error": (c.c_char_p, []),
        "recon_version": (c.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != OK:
        lib = load()
        raise ReconError(status, lib.recon_last_error().decode())


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _dev_buf(nbytes: int):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


def default_L(N: int) -> int:
    L = 64
    while L < 2 * N - 1:
        L *= 2
    return L


class Plan:
    """A trajectory on the device plus its Gram spectrum (after gram_kernel)."""

    def __init__(self, k: np.ndarray, N: int, L: int = 0, prec: int = FP32):
        lib = load()
        k = np.ascontiguousarray(np.asarray(k, dtype=np.float64))
        if k.ndim != 2 or k.shape[1] != 2:
            raise ValueError("trajectory must have shape [M, 2]")
        self.M = int(k.shape[0])
        self.N = int(N)
        self.L = int(L) if L else default_L(N)
        self.prec = int(prec)
        nbytes = lib.recon_plan_bytes(self.M, self.N, self.L, self.prec)
        if nbytes == 0:
            raise ReconError(E_RANGE, "invalid plan geometry")
        self.mem = _dev_buf(nbytes)
        h = ctypes.c_void_p()
        _check(lib.recon_plan(k.ctypes.data, self.M, self.N, self.L, self.prec,
                              self.mem.data_ptr(), nbytes, _stream(), ctypes.byref(h)))
        self._h = h
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.recon_plan_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def workspace(self, B: int):
        """Device workspace for B frames (cached per B)."""
        if B not in self._ws:
            n = load().recon_workspace_bytes(self.M, self.N, self.L, B, self.prec)
            self._ws[B] = (_dev_buf(n), n)
        return self._ws[B]

    def hq_workspace(self, B: int):
        """Device workspace of the half-quadratic solver for B frames (cached
        per B; it also serves every call the plain workspace serves)."""
        key = ("hq", B)
        if key not in self._ws:
            n = load().recon_hq_workspace_bytes(self.M, self.N, self.L, B, self.prec)
            self._ws[key] = (_dev_buf(n), n)
        return self._ws[key]

    def gram_kernel(self, want_khat: bool = False, want_lag: bool = False):
        import torch
        lib = load()
        n = lib.recon_gram_workspace_bytes(self.M, self.N, self.L)
        ws = _dev_buf(n)
        khat = torch.empty((self.L, self.L), dtype=torch.float32, device="cuda") if want_khat else None
        lag = (torch.empty((2 * self.N - 1, 2 * self.N - 1), dtype=torch.complex128, device="cuda")
               if want_lag else None)
        _check(lib.recon_gram_kernel(self._h, ws.data_ptr(), n, _ptr(khat), _ptr(lag), _stream()))
        torch.cuda.current_stream().synchronize()
        del ws
        return khat, lag

    def gram_kernel_nufft(self, W: int = 11, want_khat: bool = False, want_lag: bool = False):
        """The Gram kernel with its lag kernel from a Kaiser-Bessel non-uniform
        FFT of width W instead of the exact sums."""
        import torch
        lib = load()
        n = lib.recon_gram_nufft_workspace_bytes(self.M, self.N, self.L, int(W))
        if n == 0:
            raise ReconError(E_RANGE, "invalid NUFFT Gram geometry")
        ws = _dev_buf(n)
        khat = torch.empty((self.L, self.L), dtype=torch.float32, device="cuda") if want_khat else None
        lag = (torch.empty((2 * self.N - 1, 2 * self.N - 1), dtype=torch.complex128, device="cuda")
               if want_lag else None)
        _check(lib.recon_gram_kernel_nufft(self._h, int(W), ws.data_ptr(), n, _ptr(khat),
                                           _ptr(lag), _stream()))
        torch.cuda.current_stream().synchronize()
        del ws
        return khat, lag

    def adjoint(self, y, want_yy: bool = False):
        import torch
        y = y.contiguous()
        B = y.shape[0]
        b = torch.empty((B, self.N, self.N), dtype=torch.complex64, device="cuda")
        yy = torch.empty(B, dtype=torch.float64, device="cuda") if want_yy else None
        ws, n = self.workspace(B)
        _check(load().recon_adjoint(self._h, y.data_ptr(), B, b.data_ptr(), _ptr(yy),
                                    ws.data_ptr(), n, _stream()))
        return (b, yy) if want_yy else b

    def forward(self, x):
        import torch
        x = x.contiguous()
        B = x.shape[0]
        y = torch.empty((B, self.M), dtype=torch.complex64, device="cuda")
        ws, n = self.workspace(B)
        _check(load().recon_forward(self._h, x.data_ptr(), B, y.data_ptr(), ws.data_ptr(), n,
                                    _stream()))
        return y

    def gram_apply(self, v):
        import torch
        v = v.contiguous()
        B = v.shape[0]
        out = torch.empty_like(v)
        ws, n = self.workspace(B)
        _check(load().recon_gram_apply(self._h, v.data_ptr(), B, out.data_ptr(), ws.data_ptr(),
                                       n, _stream()))
        return out

    def solve(self, y, lam: float, delta: float, iters: int, phi: str = "hyperbolic",
              x0=None, want_stats: bool = True, lam0: float = 0.0, alpha0: float = 1.0):
        """lam0 > 0 adds the background penalty lam0 sum phi_alpha0(|x|)
        (Huber), through the resumable entry points."""
        import torch
        y = y.contiguous()
        B = y.shape[0]
        if lam0:
            self.begin(y=y, lam=lam, delta=delta, phi=phi, x0=x0, lam0=lam0, alpha0=alpha0)
            self.iterate(iters)
            return self.end() if want_stats else self.end()[0]
        x = (x0.clone().contiguous() if x0 is not None else
             torch.empty((B, self.N, self.N), dtype=torch.complex64, device="cuda"))
        st = _dev_buf(B * STATS_DTYPE.itemsize) if want_stats else None
        ws, n = self.workspace(B)
        _check(load().recon_solve(self._h, y.data_ptr(), B, float(lam), float(delta), int(iters),
                                  PHI[phi], x.data_ptr(), 1 if x0 is not None else 0,
                                  ws.data_ptr(), n, _ptr(st), _stream()))
        if not want_stats:
            return x
        return x, stats_to_numpy(st, B)

    def solve_hq(self, y, lam: float, delta: float, outer: int, inner: int,
                 phi: str = "hyperbolic", x0=None, want_stats: bool = True, lam0: float = 0.0,
                 alpha0: float = 1.0):
        """Half-quadratic minimisation: `outer` weight freezes of `inner`
        linear-CG steps each (lam0 > 0: through the resumable entry points)."""
        import torch
        y = y.contiguous()
        B = y.shape[0]
        if lam0:
            self.begin(y=y, lam=lam, delta=delta, phi=phi, x0=x0, lam0=lam0, alpha0=alpha0,
                       hq=True)
            self.hq_iterate(outer, inner)
            return self.end() if want_stats else self.end()[0]
        x = (x0.clone().contiguous() if x0 is not None else
             torch.empty((B, self.N, self.N), dtype=torch.complex64, device="cuda"))
        st = _dev_buf(B * STATS_DTYPE.itemsize) if want_stats else None
        ws, n = self.hq_workspace(B)
        _check(load().recon_solve_hq(self._h, y.data_ptr(), B, float(lam), float(delta),
                                     int(outer), int(inner), PHI[phi], x.data_ptr(),
                                     1 if x0 is not None else 0, ws.data_ptr(), n, _ptr(st),
                                     _stream()))
        if not want_stats:
            return x
        return x, stats_to_numpy(st, B)

    # resumable form
    def begin(self, y=None, b=None, B=None, lam=0.0, delta=1.0, phi="hyperbolic", x0=None,
              lam0=0.0, alpha0=1.0, hq: bool = False):
        """hq: bind the half-quadratic workspace (for hq_iterate).  A complex128
        b (FP64-iteration plans) is handed over without rounding."""
        import torch
        src = y if y is not None else b
        B = src.shape[0] if B is None else B
        ws, n = self.hq_workspace(B) if hq else self.workspace(B)
        if y is None and b is not None and b.dtype == torch.complex128:
            _check(load().recon_solve_begin_b64(self._h, b.contiguous().data_ptr(), B, float(lam),
                                                float(delta), float(lam0), float(alpha0),
                                                PHI[phi], _ptr(x0), ws.data_ptr(), n,
                                                _stream()))
        else:
            _check(load().recon_solve_begin(self._h, _ptr(y), _ptr(b), B, float(lam),
                                            float(delta), float(lam0), float(alpha0), PHI[phi],
                                            _ptr(x0), ws.data_ptr(), n, _stream()))
        self._active = (B, hq)

    def _active_ws(self):
        B, hq = self._active
        return self.hq_workspace(B) if hq else self.workspace(B)

    @property
    def _active_B(self):
        return self._active[0]

    def iterate(self, iters: int):
        ws, n = self._active_ws()
        _check(load().recon_solve_iterate(self._h, int(iters), ws.data_ptr(), n, _stream()))

    def hq_iterate(self, outer: int, inner: int):
        ws, n = self._active_ws()
        _check(load().recon_solve_hq_iterate(self._h, int(outer), int(inner), ws.data_ptr(), n,
                                             _stream()))

    def export(self, field: str):
        import torch
        B = self._active_B
        out = torch.empty((B, self.N, self.N), dtype=torch.complex64, device="cuda")
        ws, n = self._active_ws()
        _check(load().recon_solve_export(self._h, FIELD[field], out.data_ptr(), ws.data_ptr(), n,
                                         _stream()))
        return out

    def end(self):
        import torch
        B = self._active_B
        x = torch.empty((B, self.N, self.N), dtype=torch.complex64, device="cuda")
        st = _dev_buf(B * STATS_DTYPE.itemsize)
        ws, n = self._active_ws()
        _check(load().recon_solve_end(self._h, x.data_ptr(), st.data_ptr(), ws.data_ptr(), n,
                                      _stream()))
        return x, stats_to_numpy(st, B)


class GridPlan:
    """Kaiser-Bessel convolution gridding on an N x N output (grid G, kernel
    width W): the density-weighted gridding reconstruction and the NUFFT form
    of A^H y."""

    def __init__(self, k: np.ndarray, N: int, G: int = 0, W: int = 7, beta: float = 0.0):
        lib = load()
        k = np.ascontiguousarray(np.asarray(k, dtype=np.float64))
        self.M = int(k.shape[0])
        self.N = int(N)
        nbytes = lib.recon_grid_bytes(self.M, self.N, int(G), int(W))
        if nbytes == 0:
            raise ReconError(E_RANGE, "invalid grid geometry")
        self.mem = _dev_buf(nbytes)
        h = ctypes.c_void_p()
        _check(lib.recon_grid_plan(k.ctypes.data, self.M, self.N, int(G), int(W), float(beta),
                                   self.mem.data_ptr(), nbytes, _stream(), ctypes.byref(h)))
        self._h = h
        g, w, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(lib.recon_grid_info(h, ctypes.byref(g), ctypes.byref(w), ctypes.byref(b)))
        self.G, self.W, self.beta = g.value, w.value, b.value
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.recon_grid_destroy(h)
            self._h = None

    def workspace(self, B: int):
        if B not in self._ws:
            n = load().recon_grid_workspace_bytes(self._h, B)
            self._ws[B] = (_dev_buf(n), n)
        return self._ws[B]

    def adjoint(self, y, w=None, f64: bool = False):
        """(1/N) sum_l w_l y_l exp(-i 2 pi (kx m + ky n)) for each frame of y
        (device complex64 [B][M]); w: device float64 [M] or None.  f64: the
        result as complex128 (no rounding to complex64)."""
        import torch
        y = y.contiguous()
        B = y.shape[0]
        out = torch.empty((B, self.N, self.N), dtype=torch.complex128 if f64 else torch.complex64,
                          device="cuda")
        ws, n = self.workspace(B)
        fn = load().recon_grid_adjoint64 if f64 else load().recon_grid_adjoint
        _check(fn(self._h, y.data_ptr(), _ptr(w), B, out.data_ptr(), ws.data_ptr(), n, _stream()))
        return out

    def density(self, iters: int = 20):
        """Pipe-Menon density-compensation weights (device float64 [M])."""
        import torch
        w = torch.empty(self.M, dtype=torch.float64, device="cuda")
        ws, n = self.workspace(1)
        _check(load().recon_grid_density(self._h, int(iters), w.data_ptr(), ws.data_ptr(), n,
                                         _stream()))
        return w


class Pool:
    """B reconstruction slots on one plan (continuous batching).

    Frames join (admit) and leave (retire) between chunks of iterations
    (step); each runs exactly its own iteration budget, and its result is
    bitwise the one recon_solve gives for that frame alone.  The pool owns
    its workspace and may run on its own stream (torch.cuda.Stream with the
    default priority), so pools of different plans can overlap.
    """

    def __init__(self, plan: "Plan", B: int, phi: str = "hyperbolic", stream=None):
        import torch
        lib = load()
        self.plan = plan
        self.B = int(B)
        self.phi = phi
        self.stream = stream
        self.nbytes = lib.recon_workspace_bytes(plan.M, plan.N, plan.L, self.B, plan.prec)
        with torch.cuda.stream(stream) if stream is not None else _nullctx():
            self.ws = _dev_buf(self.nbytes)
            self.stats = _dev_buf(self.B * STATS_DTYPE.itemsize)
        _check(lib.recon_pool_reset(plan.handle, self.B, PHI[phi], self.ws.data_ptr(),
                                    self.nbytes, self._s()))

    def _s(self):
        return self.stream.cuda_stream if self.stream is not None else _stream()

    @property
    def iteration(self) -> int:
        return int(load().recon_pool_iteration(self.plan.handle, self.ws.data_ptr()))

    def admit(self, slot: int, y, lam: float, delta: float, iters: int, lam0: float = 0.0,
              alpha0: float = 1.0):
        """Start frame y (device complex64 [M]) in `slot` with `iters` iterations.

        When the pool runs on its own stream, that stream first waits for
        the work already queued on the caller's current stream (which may
        still be producing y), and y is marked as used on the pool's stream
        so that its memory is not reused before the pool has read it."""
        if self.stream is not None:
            import torch
            cur = torch.cuda.current_stream()
            if cur != self.stream:
                self.stream.wait_stream(cur)
                y.record_stream(self.stream)
        _check(load().recon_pool_admit(self.plan.handle, int(slot), y.data_ptr(), float(lam),
                                       float(delta), float(lam0), float(alpha0), int(iters),
                                       self.ws.data_ptr(), self.nbytes, self._s()))

    def step(self, iters: int):
        _check(load().recon_pool_step(self.plan.handle, int(iters), self.ws.data_ptr(),
                                      self.nbytes, self._s()))

    def retire(self, slot: int, x_out=None, stats: bool = True, stats_out=None):
        """Write the finished slot's image to x_out (device complex64 [N][N])
        and its statistics to stats_out (device buffer of STATS_DTYPE.itemsize
        bytes) or, without one, to the pool's stats buffer (read_stats)."""
        if stats_out is not None:
            st = stats_out.data_ptr()
        elif stats:
            st = self.stats.data_ptr() + int(slot) * STATS_DTYPE.itemsize
        else:
            st = None
        _check(load().recon_pool_retire(self.plan.handle, int(slot), _ptr(x_out), st,
                                        self.ws.data_ptr(), self.nbytes, self._s()))

    def read_stats(self, slots) -> np.ndarray:
        """Statistics of retired slots (synchronises the pool's stream)."""
        import torch
        (self.stream or torch.cuda.current_stream()).synchronize()
        raw = self.stats.cpu().numpy()
        allst = np.frombuffer(raw.tobytes(), dtype=STATS_DTYPE)
        return allst[np.asarray(list(slots), dtype=np.int64)].copy()


class _nullctx:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


TRACE = {"dir_rowfft": 0, "colpass": 1, "rowifft": 2, "update": 3, "adjoint": 4, "gram": 5,
         "forward": 6}


def trace_enable(kernel: Optional[str], capacity: int = 4096):
    """Record HIP events around each launch of one kernel kind (None: off)."""
    _check(load().recon_trace_enable(-1 if kernel is None else TRACE[kernel], int(capacity)))


def trace_read(n: int = 1 << 16, kind: Optional[str] = None) -> np.ndarray:
    """Durations (ms) recorded for one kind (default: the lowest enabled)."""
    buf = (ctypes.c_float * n)()
    lib = load()
    m = lib.recon_trace_read(buf, n) if kind is None else lib.recon_trace_read_kind(TRACE[kind], buf, n)
    if m < 0:
        raise ReconError(E_HIP, "trace read failed")
    return np.array(buf[:m], dtype=np.float64)


def trace_enable_set(kinds, capacity: int = 4096):
    """Record events around the launches of several kinds at once."""
    mask = 0
    for k in kinds:
        mask |= 1 << TRACE[k]
    _check(load().recon_trace_enable_set(mask, int(capacity)))


def stats_to_numpy(st, B: int) -> np.ndarray:
    import torch
    torch.cuda.current_stream().synchronize()
    raw = st[: B * STATS_DTYPE.itemsize].cpu().numpy()
    return np.frombuffer(raw.tobytes(), dtype=STATS_DTYPE).copy()
