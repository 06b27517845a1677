"""Benchmark: regularised spiral-MRI reconstruction on one MI355X.

Workloads:
  series256 (default): 256 x 256 complex images, 16-interleave Archimedean
    spiral at 2x angular undersampling (M = 32768 samples), hyperbolic
    penalty delta = 0.02, lambda = 0.01, 300 pseudo-CG iterations, noise
    sigma = 0.02 max|y|; a batch of 128 frames sharing the trajectory.
  large512: 512 x 512 images, 64-interleave variable-density spiral
    (M = 262144), delta = 0.01, lambda = 0.005, 500 iterations, L = 1024,
    32 frames.

One step = the whole hot path for one batch: plan (trajectory upload and
phasor tables), FP64 Gram kernel and its spectrum, adjoint b = A^H y, all
iterations (Toeplitz Gram apply, penalty stencil, step length, updates),
objective and statistics, and the forward model of the result (data
consistency).  Inputs are resident in device memory when the timed region
starts.  value = reconstructions per second over the timed steps.

Prints one JSON line (see the metric contract in the repository docs).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synthetic  # noqa: E402

HBM_PEAK_GBS = 8000.0
# fp64i: FP64 adjoint and the FP64 iteration (state, FFTs, stencil, spectrum)
PRECS = {"fp64i": 3 | 16, "fp64": 3, "fp32": 0, "fp16x3": 2, "bf16x3": 1}
METRIC = "recons/sec + p50/p99 latency at 256^2 spiral, rel-L2<=1e-4 vs FP64 oracle"

# --criterion full: the paper's criterion with both penalties (Section 3.3),
# Huber for the differences and the background.  The paper's values
# (lambda1 0.1, alpha1 20, lambda0 0.5, alpha0 10 on its intensity scale) are
# carried over by their ratios (lambda0 = 5 lambda1, alpha0 = alpha1 / 2),
# with alpha1 at 0.08 of the synthetic images' unit amplitude (20 of 255) and
# lambda1 at the workload's lambda.
FULL = dict(phi=1, alpha1=0.08, lam0_factor=5.0, alpha0=0.04)


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


MFMA_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "fp16x3": 2500.0, "bf16x3": 2500.0}
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP64_VECTOR_PEAK_TFLOPS = 78.6
CSRC = os.path.join(ROOT, "paper_0908_3252_amd", "csrc")
TRAFFIC_DIR = os.path.join(ROOT, "profiles")


def kernel_bytes(kind: str, N: int, L: int, B: int, es: int = 8) -> float:
    """Algorithmic HBM bytes of one launch over B frames (each array moved
    once; stencil halo re-reads are not counted).  es: bytes of one complex
    element (8: FP32 iteration, 16: FP64 iteration)."""
    img = float(es) * N * N    # one image
    tmat = float(es) * N * L   # the N x L intermediate of one frame
    if kind == "colpass":      # read and write the intermediate, read the spectrum once
        return B * 2 * tmat + (es / 2.0) * L * L
    if kind == "dir_rowfft":   # read x, r, d_old; write d, intermediate
        return B * (4 * img + tmat)
    if kind == "update":       # read intermediate, x, d, r; write x, r
        return B * (tmat + 5 * img)
    raise ValueError(kind)


def kernel_flops(kind: str, N: int, M: int, L: int, B: int) -> float:
    """Algorithmic flops of one launch over B frames."""
    if kind in ("adjoint", "forward"):  # complex MAC = 8 real flops, N^2 M per frame
        return 8.0 * N * N * M * B
    if kind == "colpass":  # two length-L FFTs per column (5 L log2 L) + the real scaling
        return B * L * (2 * 5.0 * L * np.log2(L) + 6.0 * L)
    raise ValueError(kind)


def csrc_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kind: str, digest: str, prec: str = "fp64"):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this workload and precision (FETCH_SIZE and WRITE_SIZE per dispatch,
    each scaled by what the counter reads for a plain copy of known size), or
    None when the kernel sources have changed since the counters were taken."""
    suffix = "" if prec == "fp64" else f"_{prec}"
    path = os.path.join(TRAFFIC_DIR, f"traffic_{workload}{suffix}.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        f = line.split()
        if len(f) == 7 and f[0] == "traffic" and f[1] == kind:
            fetch_kib, write_kib, ffac, wfac, dig = map(str, f[2:])
            if dig != digest:
                return None
            return round((float(fetch_kib) * float(ffac) + float(write_kib) * float(wfac)) * 1024.0)
    return None


def synth_batch(plan, prob, B, torch):
    """y = A x_true + sigma * noise per frame, on the GPU (input synthesis)."""
    x_true = torch.from_numpy(prob.x_true.astype(np.complex64)).cuda()
    y0 = plan.forward(x_true)
    noise = torch.from_numpy(prob.noise.astype(np.complex64)).cuda()
    sig = prob.noise_c * y0.abs().amax(dim=1, keepdim=True)
    return (y0 + sig * noise).contiguous()


WORKLOADS = {
    "series256": dict(cfg=3, batch=128),
    "large512": dict(cfg=5, batch=32),
}


def cpu_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def host_info():
    """The host the oracle runs on: CPU model, cores, numpy / scipy versions and
    BLAS threads."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:  # pragma: no cover
        pass
    info = {"cpu_model": model, "cpu_count": os.cpu_count(), "numpy": np.__version__,
            "blas_threads": int(cpu_threads())}
    try:
        import scipy
        info["scipy"] = scipy.__version__
    except ImportError:  # pragma: no cover
        pass
    return info


def cpu_baseline_large(torch, recon, prec, sample_iters=40):
    """The FP64 oracle on frame 0 of the large workload: adjoint and Gram
    kernel in full plus a bounded number of iterations, timed on the host;
    the per-reconstruction time is setup + iterations scaled to the full
    budget.  (The 20-iteration GPU/oracle agreement is a parity test.)"""
    import oracle
    prob = synthetic.make_frames(5, frames=1)
    y = prob.measured(oracle.forward(prob.x_true, prob.k))
    t0 = time.perf_counter()
    b = oracle.adjoint(y[0], prob.k, prob.N)
    K = oracle.khat(prob.k, prob.N, prob.L)
    t1 = time.perf_counter()
    oracle.solve(b, K, prob.lam, prob.delta, sample_iters)
    t2 = time.perf_counter()
    per = (t1 - t0) + (t2 - t1) * prob.iters / sample_iters
    return dict(value=1.0 / per, unit="recons/sec", cores=int(cpu_threads()), kind="oracle",
                sample=(f"one 512x512 frame, M={prob.M}: adjoint + Gram kernel in full "
                        f"({t1 - t0:.1f} s) + {sample_iters} of {prob.iters} iterations "
                        f"({t2 - t1:.1f} s, scaled to {prob.iters}) in FP64 numpy"),
                seconds=t2 - t0), None, None


def criterion_args(args, prob):
    """(phi name, lambda, delta, lambda0, alpha0) of the benchmarked criterion."""
    if args.criterion == "full":
        return ("huber", prob.lam, FULL["alpha1"], FULL["lam0_factor"] * prob.lam,
                FULL["alpha0"])
    return ("hyperbolic", prob.lam, prob.delta, 0.0, 1.0)


def cpu_baseline(args, torch, recon, prec):
    """The FP64 oracle on one 256^2 frame (adjoint + Gram + all iterations),
    timed on the host, and the GPU result on the same frame against it."""
    import oracle
    if args.workload == "large512":
        return cpu_baseline_large(torch, recon, prec)
    threads = cpu_threads()
    prob = synthetic.make_problem(2)
    phi, lam, delta, lam0, alpha0 = criterion_args(args, prob)
    y = prob.measured(oracle.forward(prob.x_true, prob.k)).astype(np.complex64)
    t0 = time.perf_counter()
    b = oracle.adjoint(y[0], prob.k, prob.N)
    K = oracle.khat(prob.k, prob.N, prob.L)
    xo = oracle.solve(b, K, lam, delta, prob.iters, kind=phi, lam0=lam0, alpha0=alpha0,
                      kind0="huber")
    dt = time.perf_counter() - t0
    # GPU on the identical frame (oracle-made data)
    plan = recon.Plan(prob.k, prob.N, prob.L, prec=prec)
    plan.gram_kernel()
    xg, st = plan.solve(torch.from_numpy(y).cuda(), lam, delta, prob.iters, phi=phi, lam0=lam0,
                        alpha0=alpha0)
    torch.cuda.synchronize()
    xg = xg.cpu().numpy()[0].astype(np.complex128)
    rel = float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))
    return dict(value=1.0 / dt, unit="recons/sec", cores=int(threads), kind="oracle",
                sample=(f"one 256x256 frame, M={prob.M}: adjoint + Gram kernel + "
                        f"{prob.iters} iterations in FP64 numpy ({dt:.1f} s)"),
                seconds=dt), rel, (y[0], xo)


def cuda_ms(torch, fn, reps=3):
    """Median duration (ms) of fn() on the current stream (HIP events), after
    one untimed call."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


SERIES_FRAMES = (0, 42, 85, 127)


def _rel(torch, a, b):
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def _rel_frames(torch, a, b):
    """Relative L2 distance of every frame of a from the same frame of b."""
    d = torch.linalg.vector_norm(a - b, dim=(-2, -1)) / torch.linalg.vector_norm(b, dim=(-2, -1))
    return d.double().cpu().numpy()


def _rel_summary(e):
    return {"frames": int(e.size), "median": float(f"{np.median(e):.3e}"),
            "p90": float(f"{np.quantile(e, 0.9):.3e}"), "max": float(f"{e.max():.3e}"),
            "frames_over_1e-4": int((e >= 1e-4).sum())}


def extra_precision_form(c):
    """The precision form on the 128-frame series: FP32 and split BF16 / FP16
    x3 NUDFT contractions with the FP32 iteration (and the FP64 adjoint with
    the FP32 iteration), one whole step each (plan, Gram kernel, adjoint,
    iterations, forward model) in calls of 64 frames (these plans take at
    most 64 frames per call), against the FP64-iteration result of the main
    benchmark on frames 0, 42, 85, 127 (the parity tests hold that result to
    the FP64 oracle at 2.5e-8)."""
    torch, recon, lib = c["torch"], c["recon"], c["lib"]
    B, N, L, M, iters = c["B"], c["N"], c["L"], c["M"], c["iters"]
    y, xref = c["y"], c["x"]
    res = {}
    for name, prec in (("fp64_adjoint_fp32_iteration", recon.FP64), ("fp32", recon.FP32),
                       ("fp16x3", recon.FP16X3), ("bf16x3", recon.BF16X3)):
        plan = recon.Plan(c["k_host"], N, L, prec=prec)
        plan.gram_kernel()
        G = min(B, 64)
        ws, wsn = plan.workspace(G)
        pbytes = lib.recon_plan_bytes(M, N, L, prec)
        gws_n = lib.recon_gram_workspace_bytes(M, N, L)
        gws = torch.empty(gws_n, dtype=torch.uint8, device="cuda")
        xo = torch.empty((B, N, N), dtype=torch.complex64, device="cuda")
        yfit = torch.empty((B, M), dtype=torch.complex64, device="cuda")
        import ctypes

        def step():
            h = ctypes.c_void_p()
            recon._check(lib.recon_plan(c["k_host"].ctypes.data, M, N, L, prec,
                                        plan.mem.data_ptr(), pbytes, c["stream"], ctypes.byref(h)))
            try:
                recon._check(lib.recon_gram_kernel(h, gws.data_ptr(), gws_n, None, None,
                                                   c["stream"]))
                for f0 in range(0, B, G):
                    g = min(G, B - f0)
                    recon._check(lib.recon_solve(h, y[f0].data_ptr(), g, c["lam"], c["delta"],
                                                 iters, 0, xo[f0].data_ptr(), 0, ws.data_ptr(),
                                                 wsn, None, c["stream"]))
                    recon._check(lib.recon_forward(h, xo[f0].data_ptr(), g, yfit[f0].data_ptr(),
                                                   ws.data_ptr(), wsn, c["stream"]))
            finally:
                lib.recon_plan_destroy(h)

        ms = cuda_ms(torch, step, reps=3)
        errs = {f"f{f}": _rel(torch, xo[f], xref[f]) for f in SERIES_FRAMES if f < B}
        allf = _rel_frames(torch, xo, xref)
        res[name] = {"recons_per_sec": round(B / (ms * 1e-3), 2), "ms_per_step": round(ms, 3),
                     "calls_per_step": -(-B // G),
                     "rel_l2_vs_fp64_iteration": {k: float(f"{v:.3e}") for k, v in errs.items()},
                     "rel_l2_all_frames": _rel_summary(allf),
                     "meets_1e-4": bool(allf.max() < 1e-4)}
        del plan, ws, gws, xo, yfit
    return res


def extra_half_quadratic(c):
    """Section 5's half-quadratic alternative against the pseudo-CG on the
    128-frame batch (FP64 iteration): criterion J (median over frames) and
    time for the same numbers of Gram applications."""
    torch, recon = c["torch"], c["recon"]
    B, N, L = c["B"], c["N"], c["L"]
    plan = recon.Plan(c["k_host"], N, L, prec=recon.FP64_ITER64)
    plan.gram_kernel()
    y = c["y"]
    rows = []
    xs = {}
    for apps in (60, 150, 300):
        out = {"gram_applications": apps}
        res = {}
        ms = cuda_ms(torch, lambda: res.__setitem__("cg", plan.solve(y, c["lam"], c["delta"],
                                                                     apps)), reps=1)
        out["cg"] = {"ms": round(ms, 2), "J_median": float(np.median(res["cg"][1]["J"]))}
        outer = apps // 10
        ms = cuda_ms(torch, lambda: res.__setitem__("hq", plan.solve_hq(y, c["lam"], c["delta"],
                                                                        outer, 10)), reps=1)
        out["half_quadratic"] = {"outer": outer, "inner": 10, "ms": round(ms, 2),
                                 "J_median": float(np.median(res["hq"][1]["J"]))}
        out["J_hq_minus_J_cg_median"] = float(np.median(res["hq"][1]["J"] - res["cg"][1]["J"]))
        xs[apps] = (res["cg"][0], res["hq"][0])
        rows.append(out)
    cg300, hq300 = xs[300]
    return {"frames": B, "iteration": "fp64", "runs": rows,
            "rel_l2_hq_vs_cg_at_300_median": float(np.median(
                [_rel(torch, hq300[f], cg300[f]) for f in range(0, B, 16)]))}


def extra_gridding(c):
    """The paper's comparison (Section 4.1): Kaiser-Bessel gridding (W = 7,
    grid 2N, Pipe-Menon density weights) against the regularised
    reconstruction (the benchmark's FP64-iteration result), quadratic error
    in ROI1 (central square) and variance in ROI2 (a flat region) against
    the synthetic truth, on 8 frames."""
    torch, recon = c["torch"], c["recon"]
    prob, y, x, B, N = c["prob"], c["y"], c["x"], c["B"], c["N"]
    gp = recon.GridPlan(c["k_host"], N, W=7)
    box = {}
    ms_dcf = cuda_ms(torch, lambda: box.__setitem__("w", gp.density(10)), reps=1)
    w = box["w"]
    ms_grid = cuda_ms(torch, lambda: box.__setitem__("img", gp.adjoint(y, w)), reps=3)
    img = box["img"]
    frames = list(range(0, B, max(1, B // 8)))[:8]
    q_g, q_r, v_g, v_r = [], [], [], []
    for f in frames:
        xt = prob.x_true[f]
        roi1, roi2 = synthetic.roi_masks(xt)
        xg = img[f].cpu().numpy().astype(np.complex128)
        xr = x[f].cpu().numpy().astype(np.complex128)
        for arr, q, v in ((xg, q_g, v_g), (xr, q_r, v_r)):
            q.append(float(np.mean(np.abs(arr - xt)[roi1] ** 2)))
            vals = arr[roi2]
            v.append(float(np.mean(np.abs(vals - vals.mean()) ** 2)))
    return {"kernel_width": 7, "grid": gp.G, "beta": round(gp.beta, 4),
            "density_iterations": 10, "density_ms": round(ms_dcf, 3),
            "gridding_ms_per_batch": round(ms_grid, 3), "frames": B,
            "benchmark_frames": _roi_summary(q_g, q_r, v_g, v_r),
            "paper_like": _gridding_paper_like(c)}


def _roi_summary(q_g, q_r, v_g, v_r):
    return {"frames_scored": len(q_g),
            "roi1_quadratic_error": {"gridding_median": float(np.median(q_g)),
                                     "regularised_median": float(np.median(q_r)),
                                     "ratio_median": float(np.median(np.array(q_g) / np.array(q_r)))},
            "roi2_variance": {"gridding_median": float(np.median(v_g)),
                              "regularised_median": float(np.median(v_r)),
                              "ratio_median": float(np.median(np.array(v_g) / np.array(v_r)))}}


def _gridding_paper_like(c):
    """Section 4.1's comparison setting on synthetic data: 128 x 128 images
    (the paper's simulated model size), 10 interleaves of 512 samples (its
    error sweeps), noise-free and with noise c = 0.002 max|y| (about 25 dB),
    8 seeded 10-ellipse phantoms; regularised: hyperbolic lambda = 0.02,
    delta = 0.05, 300 iterations in FP64; gridding: Kaiser-Bessel W = 7,
    grid 256, 10 density iterations."""
    torch, recon = c["torch"], c["recon"]
    N, F = 128, 8
    k = np.ascontiguousarray(synthetic.spiral_trajectory(N, 10, 512, 1.0))
    xt = np.stack([synthetic.ellipse_phantom(N, 10, np.random.default_rng([6, f]))
                   for f in range(F)])
    plan = recon.Plan(k, N, prec=recon.FP64_ITER64)
    plan.gram_kernel()
    y0 = plan.forward(torch.from_numpy(xt.astype(np.complex64)).cuda())
    nz = torch.from_numpy(np.stack([synthetic.noise_draws(k.shape[0], np.random.default_rng([6, 100 + f]))
                                    for f in range(F)]).astype(np.complex64)).cuda()
    gp = recon.GridPlan(k, N, W=7)
    w = gp.density(10)
    out = {"image": N, "samples": int(k.shape[0]), "frames": F}
    for name, cn in (("noise_free", 0.0), ("c_0.002", 0.002)):
        y = (y0 + cn * y0.abs().amax(dim=1, keepdim=True) * nz).contiguous()
        xr, _ = plan.solve(y, 0.02, 0.05, 300)
        xg = gp.adjoint(y, w)
        torch.cuda.synchronize()
        q_g, q_r, v_g, v_r = [], [], [], []
        for f in range(F):
            roi1, roi2 = synthetic.roi_masks(xt[f])
            for arr, q, v in ((xg[f], q_g, v_g), (xr[f], q_r, v_r)):
                a = arr.cpu().numpy().astype(np.complex128)
                q.append(float(np.mean(np.abs(a - xt[f])[roi1] ** 2)))
                vals = a[roi2]
                v.append(float(np.mean(np.abs(vals - vals.mean()) ** 2)))
        out[name] = _roi_summary(q_g, q_r, v_g, v_r)
    return out


def extra_nufft(c):
    """Section 5's NUFFT precomputation (Kaiser-Bessel, W = 11, grid 2N for
    D = A^H y, 4N for the lag kernel) against the exact FP64-accumulated
    sums: time per 128-frame batch, relative difference, the whole step with
    the NUFFT D in complex64 (W = 11) and kept in FP64 (W = 15), each with
    every frame's distance from the exact-sums result, and one 256^2 frame
    solved with the FP64 iteration from the NUFFT D and spectrum against the
    oracle (exact sums)."""
    torch, recon = c["torch"], c["recon"]
    B, N, L, y = c["B"], c["N"], c["L"], c["y"]
    W = 11
    gp = recon.GridPlan(c["k_host"], N, W=W)
    exact = recon.Plan(c["k_host"], N, L, prec=recon.FP64_ITER64)
    box = {}
    ms_exact_b = cuda_ms(torch, lambda: box.__setitem__("be", exact.adjoint(y)), reps=3)
    ms_nufft_b = cuda_ms(torch, lambda: box.__setitem__("bn", gp.adjoint(y)), reps=3)
    eb = float(np.median([_rel(torch, box["bn"][f], box["be"][f]) for f in range(0, B, 8)]))
    ms_exact_g = cuda_ms(torch, lambda: exact.gram_kernel(), reps=3)
    nplan = recon.Plan(c["k_host"], N, L, prec=recon.FP64_ITER64)
    ms_nufft_g = cuda_ms(torch, lambda: nplan.gram_kernel_nufft(W), reps=3)
    _, lag_e = exact.gram_kernel(want_lag=True)
    _, lag_n = nplan.gram_kernel_nufft(W, want_lag=True)
    eg = _rel(torch, lag_n, lag_e)
    out = {"kernel_width": W, "grid_for_D": gp.G, "beta": round(gp.beta, 4),
           "stated_bound": float(f"{4.0 / float(np.i0(gp.beta)):.2e}"),
           "D_batch_ms": {"exact_fp64": round(ms_exact_b, 3), "nufft": round(ms_nufft_b, 3)},
           "D_rel_diff_median": float(f"{eb:.3e}"),
           "gram_kernel_ms": {"exact_fp64": round(ms_exact_g, 3),
                              "nufft_incl_host_binning": round(ms_nufft_g, 3)},
           "lag_kernel_rel_diff": float(f"{eg:.3e}")}
    # the benchmark's whole step with D from the NUFFT (plan, exact Gram kernel,
    # NUFFT D, FP64 iteration from that D, forward model), 128 frames
    lib = c["lib"]
    import ctypes
    M = c["M"]
    prec = recon.FP64_ITER64
    sp = recon.Plan(c["k_host"], N, L, prec=prec)
    sp.gram_kernel()
    pbytes = lib.recon_plan_bytes(M, N, L, prec)
    gws_n = lib.recon_gram_workspace_bytes(M, N, L)
    gws = torch.empty(gws_n, dtype=torch.uint8, device="cuda")
    ws, wsn = sp.workspace(B)
    gws2, gwsn2 = gp.workspace(B)
    bD = torch.empty((B, N, N), dtype=torch.complex64, device="cuda")
    xo = torch.empty((B, N, N), dtype=torch.complex64, device="cuda")
    yfit = torch.empty((B, M), dtype=torch.complex64, device="cuda")
    st = c["stream"]

    def step():
        h = ctypes.c_void_p()
        recon._check(lib.recon_plan(c["k_host"].ctypes.data, M, N, L, prec, sp.mem.data_ptr(),
                                    pbytes, st, ctypes.byref(h)))
        try:
            recon._check(lib.recon_gram_kernel(h, gws.data_ptr(), gws_n, None, None, st))
            recon._check(lib.recon_grid_adjoint(gp._h, y.data_ptr(), None, B, bD.data_ptr(),
                                                gws2.data_ptr(), gwsn2, st))
            recon._check(lib.recon_solve_begin(h, None, bD.data_ptr(), B, c["lam"], c["delta"],
                                               0.0, 1.0, 0, None, ws.data_ptr(), wsn, st))
            recon._check(lib.recon_solve_iterate(h, c["iters"], ws.data_ptr(), wsn, st))
            recon._check(lib.recon_solve_end(h, xo.data_ptr(), None, ws.data_ptr(), wsn, st))
            recon._check(lib.recon_forward(h, xo.data_ptr(), B, yfit.data_ptr(), ws.data_ptr(),
                                           wsn, st))
        finally:
            lib.recon_plan_destroy(h)

    ms = cuda_ms(torch, step, reps=3)
    errs = [_rel(torch, xo[f], c["x"][f]) for f in SERIES_FRAMES if f < B]
    out["step_with_nufft_D"] = {"recons_per_sec": round(B / (ms * 1e-3), 2),
                                "ms_per_step": round(ms, 3),
                                "rel_l2_vs_exact_sums_result_max": float(f"{max(errs):.3e}"),
                                "rel_l2_all_frames": _rel_summary(_rel_frames(torch, xo,
                                                                              c["x"]))}
    # the same step with D from a W = 15 NUFFT kept in FP64 (no rounding to
    # complex64 before the FP64 iteration)
    W64 = 15
    gp64 = recon.GridPlan(c["k_host"], N, W=W64)
    gws64, gwsn64 = gp64.workspace(B)
    bD64 = torch.empty((B, N, N), dtype=torch.complex128, device="cuda")

    def step64():
        h = ctypes.c_void_p()
        recon._check(lib.recon_plan(c["k_host"].ctypes.data, M, N, L, prec, sp.mem.data_ptr(),
                                    pbytes, st, ctypes.byref(h)))
        try:
            recon._check(lib.recon_gram_kernel(h, gws.data_ptr(), gws_n, None, None, st))
            recon._check(lib.recon_grid_adjoint64(gp64._h, y.data_ptr(), None, B,
                                                  bD64.data_ptr(), gws64.data_ptr(), gwsn64, st))
            recon._check(lib.recon_solve_begin_b64(h, bD64.data_ptr(), B, c["lam"], c["delta"],
                                                   0.0, 1.0, 0, None, ws.data_ptr(), wsn, st))
            recon._check(lib.recon_solve_iterate(h, c["iters"], ws.data_ptr(), wsn, st))
            recon._check(lib.recon_solve_end(h, xo.data_ptr(), None, ws.data_ptr(), wsn, st))
            recon._check(lib.recon_forward(h, xo.data_ptr(), B, yfit.data_ptr(), ws.data_ptr(),
                                           wsn, st))
        finally:
            lib.recon_plan_destroy(h)

    ms64 = cuda_ms(torch, step64, reps=3)
    ms_d64 = cuda_ms(torch, lambda: gp64.adjoint(y, f64=True), reps=3)
    out["step_with_nufft_D_fp64"] = {
        "kernel_width": W64, "beta": round(gp64.beta, 4),
        "stated_bound": float(f"{4.0 / float(np.i0(gp64.beta)):.2e}"),
        "D_batch_ms": round(ms_d64, 3),
        "recons_per_sec": round(B / (ms64 * 1e-3), 2), "ms_per_step": round(ms64, 3),
        "rel_l2_all_frames": _rel_summary(_rel_frames(torch, xo, c["x"]))}
    del gws64, bD64
    # control: the exact FP64 sums rounded to complex64 and passed in as D, to
    # separate the iterate's sensitivity to that rounding from the NUFFT's error
    be = exact.adjoint(y)
    sp.begin(b=be, lam=c["lam"], delta=c["delta"])
    sp.iterate(c["iters"])
    xe, _ = sp.end()
    out["exact_D_rounded_to_complex64"] = {
        "D_rel_diff_median_vs_nufft": float(f"{eb:.3e}"),
        "rel_l2_all_frames": _rel_summary(_rel_frames(torch, xe, c["x"]))}
    of = c.get("oracle_frame")
    if of is not None:
        y0, xo = of
        yd = torch.from_numpy(np.ascontiguousarray(y0[None], dtype=np.complex64)).cuda()
        pgp = recon.GridPlan(c["k_host"], N, W=W)
        b0 = pgp.adjoint(yd)
        nplan.begin(b=b0, lam=c["lam"], delta=c["delta"])
        nplan.iterate(c["iters"])
        xg, _ = nplan.end()
        xg = xg[0].cpu().numpy().astype(np.complex128)
        out["frame0_rel_l2_vs_oracle_exact_sums"] = float(
            f"{np.linalg.norm(xg - xo) / np.linalg.norm(xo):.3e}")
    return out


def extra_paper_shape(c):
    """The workload the paper times (Section 4.2: 256^2 image, 12 and 24
    spiral interleaves of 2048 samples, 50 iterations), one frame at a time
    on the GPU in the benchmark's precision, beside the paper's own timings
    on its hardware (context only): D took 30 s, 50 iterations 3 min."""
    torch, recon = c["torch"], c["recon"]
    N = 256
    rng = np.random.default_rng([2, 4242])
    xt = synthetic.ellipse_phantom(N, 40, rng)
    out = {"paper": {"D_s": 30.0, "iterations_50_s": 180.0,
                     "hardware": "Athlon 2.1 GHz (C) for D, Matlab for the iterations"}}
    for inter in (12, 24):
        k = np.ascontiguousarray(synthetic.spiral_trajectory(N, inter, 2048, 1.0))
        M = k.shape[0]
        plan = recon.Plan(k, N, 512, prec=c["prec"])
        ms_gram = cuda_ms(torch, lambda: plan.gram_kernel(), reps=3)
        y0 = plan.forward(torch.from_numpy(xt[None].astype(np.complex64)).cuda())
        noise = torch.from_numpy(synthetic.noise_draws(M, rng)[None].astype(np.complex64)).cuda()
        y = (y0 + 0.02 * y0.abs().amax() * noise).contiguous()
        ms_adj = cuda_ms(torch, lambda: plan.adjoint(y), reps=5)
        ms_solve = cuda_ms(torch, lambda: plan.solve(y, c["lam"], c["delta"], 50,
                                                      want_stats=False), reps=5)
        out[f"interleaves_{inter}"] = {"M": M, "gram_kernel_ms": round(ms_gram, 3),
                                       "D_ms": round(ms_adj, 3),
                                       "solve_50_ms_incl_D": round(ms_solve, 3)}
    return out


def extra_served_mixed(args, c):
    """The mixed-size served stream (N in {64..384}, 8/16/32 interleaves,
    Poisson arrivals) at the given rates, FP64 iteration and the precision
    forms (FP32, split FP16 / BF16 x3 with the FP32 iteration), each result
    compared with the FP64-iteration result of the same request."""
    from paper_0908_3252_amd import serving as srv
    wl = srv.make_workload(args.mixed_count, 4)
    runs = []
    for rate in [float(v) for v in args.mixed_rates.split(",")]:
        ref = None
        for prec in ("fp64i", "fp32", "fp16x3", "bf16x3"):
            if prec == "fp64i":
                o, ref = srv.serve(rate, wl, prec=prec, keep_results=True, verify=1)
            else:
                o = srv.serve(rate, wl, prec=prec, reference=ref, verify=1)
            keep = {k: o[k] for k in ("rate", "prec", "requests", "completed", "recons_per_sec",
                                      "p50_ms", "p99_ms", "status_ok", "bitwise_equal_standalone",
                                      "rel_l2_vs_reference") if k in o}
            for k in ("recons_per_sec", "p50_ms", "p99_ms"):
                if k in keep:
                    keep[k] = round(keep[k], 2)
            runs.append(keep)
            log(f"mixed {rate}/s {prec}: {keep}")
        ref = None
    return {"requests_per_rate": args.mixed_count, "runs": runs,
            "what": "arrival-to-result latency, first 10% excluded; rel_l2_vs_reference: each "
                    "result against the FP64-iteration result of the same request"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="series256", choices=list(WORKLOADS))
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--prec", default="fp64i", choices=list(PRECS),
                    help="NUDFT contraction precision (fp64: FP64-accumulated adjoint; "
                         "fp64i: that adjoint and the iteration in FP64)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-reps", type=int, default=10)
    ap.add_argument("--serve-rate", default="250,450",
                    help="served 256^2 request streams: comma list of Poisson arrival rates "
                         "per second (0: off)")
    ap.add_argument("--serve-count", type=int, default=600)
    ap.add_argument("--no-phases", action="store_true",
                    help="skip the separately timed phases (plan, adjoint, one apply, solve)")
    ap.add_argument("--serve-chunk", type=int, default=10,
                    help="iterations a served pool runs per scheduling step")
    ap.add_argument("--criterion", default="plain", choices=["plain", "full"],
                    help="plain: hyperbolic difference penalty (the workload's criterion); "
                         "full: the paper's criterion, Huber differences + background penalty")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the precision form, half-quadratic, gridding, NUFFT and mixed "
                         "serving sections (profiling runs)")
    ap.add_argument("--mixed-count", type=int, default=600,
                    help="requests per rate of the mixed-size served stream (0: off)")
    ap.add_argument("--mixed-rates", default="200,2000")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB "
                         "(reference kernel for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                                   "(frames and requests are independent, so more GPUs "
                                   "would each take a share of them with no exchange)"}))
        sys.exit(2)

    import torch
    from paper_0908_3252_amd import recon
    recon.load()
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration_mb:
        nb = args.copy_calibration_mb << 20
        src = torch.ones(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nb} bytes device to device")
        del src, dst
    wl = WORKLOADS[args.workload]
    B = args.batch or wl["batch"]
    prob = synthetic.make_frames(wl["cfg"], frames=B)  # drifting phantoms, shared trajectory
    iters = args.iters or prob.iters
    N, L, M = prob.N, prob.L, prob.M
    log(f"workload N={N} M={M} L={L} B={B} iters={iters}")

    # device-resident inputs and buffers (allocated once)
    lib = recon.load()
    prec = PRECS[args.prec]
    plan = recon.Plan(prob.k, N, L, prec=prec)
    plan.gram_kernel()
    y = synth_batch(plan, prob, B, torch)
    es = 16 if prec & recon.ITER_FP64 else 8
    k_host = np.ascontiguousarray(prob.k)
    plan_bytes = lib.recon_plan_bytes(M, N, L, prec)
    gws_bytes = lib.recon_gram_workspace_bytes(M, N, L)
    gws = torch.empty(gws_bytes, dtype=torch.uint8, device="cuda")
    ws, ws_bytes = plan.workspace(B)
    x = torch.empty((B, N, N), dtype=torch.complex64, device="cuda")
    yfit = torch.empty((B, M), dtype=torch.complex64, device="cuda")
    stats = torch.empty(B * recon.STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    import ctypes

    phi_name, c_lam, c_delta, c_lam0, c_alpha0 = criterion_args(args, prob)
    phi = recon.PHI[phi_name]

    def solve(h, yp, nb, xp, wsp, wsn, stp):
        if args.criterion == "plain":
            recon._check(lib.recon_solve(h, yp, nb, c_lam, c_delta, iters, phi, xp, 0, wsp, wsn,
                                         stp, stream))
            return
        recon._check(lib.recon_solve_begin(h, yp, None, nb, c_lam, c_delta, c_lam0, c_alpha0,
                                           phi, None, wsp, wsn, stream))
        recon._check(lib.recon_solve_iterate(h, iters, wsp, wsn, stream))
        recon._check(lib.recon_solve_end(h, xp, stp, wsp, wsn, stream))

    def step():
        h = ctypes.c_void_p()
        recon._check(lib.recon_plan(k_host.ctypes.data, M, N, L, prec, plan.mem.data_ptr(),
                                    plan_bytes, stream, ctypes.byref(h)))
        try:
            recon._check(lib.recon_gram_kernel(h, gws.data_ptr(), gws_bytes, None, None, stream))
            solve(h, y.data_ptr(), B, x.data_ptr(), ws.data_ptr(), ws_bytes, stats.data_ptr())
            recon._check(lib.recon_forward(h, x.data_ptr(), B, yfit.data_ptr(), ws.data_ptr(),
                                           ws_bytes, stream))
        finally:
            lib.recon_plan_destroy(h)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")

    kinds = ["adjoint", "forward", "dir_rowfft", "colpass", "update"]
    # events around the first 64 launches of each kind (every step's adjoint
    # and forward, the first 64 iterations' kernels): enough for the averages
    # without instrumenting every launch of the timed region
    recon.trace_enable_set(kinds, capacity=max(args.steps, 64))
    times = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"step {i + 1}/{args.steps}: {times[-1] * 1e3:.2f} ms")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    kms = {k: recon.trace_read(kind=k) for k in kinds}
    recon.trace_enable(None)
    st = recon.stats_to_numpy(stats, B)
    ms_step = 1e3 * total / args.steps
    value = B * args.steps / total

    # rooflines of the traced kernels (HIP events on the solve stream)
    digest = csrc_digest()
    rooflines = {}
    for k in kinds:
        d = kms[k]
        if not len(d):
            continue
        avg_ms = float(np.mean(d))
        per_step = 1 if k in ("adjoint", "forward") else iters  # launches per step
        ent = dict(avg_launch_ms=round(avg_ms, 5), launches_timed=int(len(d)),
                   ms_per_step=round(avg_ms * per_step, 3))
        if k in ("adjoint", "forward"):
            fl = kernel_flops(k, N, M, L, B)
            mp = "fp64" if args.prec == "fp64i" else args.prec
            peak = MFMA_PEAK_TFLOPS[mp if k == "adjoint" else
                                    ("fp32" if mp in ("fp32", "fp64") else mp)]
            ach = fl / (avg_ms * 1e-3) / 1e12
            ent.update(bound="mfma", achieved=round(ach, 2), peak=peak, unit="TFLOP/s",
                       frac=round(ach / peak, 4), algorithmic_flops_per_launch=fl)
        else:
            kb = kernel_bytes(k, N, L, B, es)
            ach = kb / (avg_ms * 1e-3) / 1e9
            ent.update(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                       frac=round(ach / HBM_PEAK_GBS, 4), algorithmic_bytes_per_launch=kb)
            # the same launch priced with complex64 elements (8 bytes), the
            # byte model of the FP32 iteration
            kb8 = kernel_bytes(k, N, L, B, 8)
            ent["frac_complex64_model"] = round(kb8 / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            if k == "colpass":
                fl = kernel_flops(k, N, M, L, B)
                vt = "fp64" if es == 16 else "fp32"
                vp = FP64_VECTOR_PEAK_TFLOPS if es == 16 else FP32_VECTOR_PEAK_TFLOPS
                ent[f"alu_{vt}_tflops"] = round(fl / (avg_ms * 1e-3) / 1e12, 2)
                ent[f"alu_frac_of_{vt}_vector_peak"] = round(
                    fl / (avg_ms * 1e-3) / 1e12 / vp, 4)
        ent["traffic"] = measured_traffic(args.workload, k, digest, args.prec)
        rooflines[k] = ent
    dominant = max(rooflines, key=lambda k: rooflines[k]["ms_per_step"])
    roofline = dict(rooflines[dominant])
    roofline["kernel"] = dominant
    roofline["basis"] = (f"algorithmic bytes with {es}-byte complex elements (the element size "
                         f"this iteration stores); frac_complex64_model prices the same launch "
                         f"with 8-byte elements")
    # one whole iteration (direction + column pass + update) against the
    # 176 N^2 bytes-per-frame model of the FP32 iteration
    it_ms = sum(rooflines[k]["avg_launch_ms"] for k in ("dir_rowfft", "colpass", "update")
                if k in rooflines)
    iteration_model = None
    if it_ms > 0:
        mb = 176.0 * N * N * B
        iteration_model = {"ms_per_iteration": round(it_ms, 5), "model_bytes": mb,
                           "frac_of_hbm_peak": round(mb / (it_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "what": "176 N^2 bytes per frame and iteration (complex64 state: "
                                   "Toeplitz apply 80 N^2 + stencil and updates 96 N^2)"}

    # single-frame latency (one 256^2 reconstruction, same hot path, B = 1)
    lat = []
    y1 = y[:1].contiguous()
    x1 = torch.empty((1, N, N), dtype=torch.complex64, device="cuda")
    ws1, ws1_bytes = plan.workspace(1)
    for i in range(args.latency_reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solve(plan.handle, y1.data_ptr(), 1, x1.data_ptr(), ws1.data_ptr(), ws1_bytes, None)
        torch.cuda.synchronize()
        if i:
            lat.append(time.perf_counter() - t0)
    # phases timed separately (events on the library's stream): plan + Gram
    # kernel, batched adjoint, one batched Toeplitz apply (the public FP32
    # apply, scored against the two-round-trip byte model), whole solve
    phases = None
    if not args.no_phases:
        def time_phase(fn, reps):
            fn()
            torch.cuda.synchronize()
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(reps)]
            for a, b_ in evs:
                a.record()
                fn()
                b_.record()
            torch.cuda.synchronize()
            t = np.array([a.elapsed_time(b_) for a, b_ in evs])
            return {"median_ms": round(float(np.median(t)), 4),
                    "p10_ms": round(float(np.percentile(t, 10)), 4),
                    "p90_ms": round(float(np.percentile(t, 90)), 4), "reps": reps}

        def plan_gram():
            h = ctypes.c_void_p()
            recon._check(lib.recon_plan(k_host.ctypes.data, M, N, L, prec, plan.mem.data_ptr(),
                                        plan_bytes, stream, ctypes.byref(h)))
            recon._check(lib.recon_gram_kernel(h, gws.data_ptr(), gws_bytes, None, None, stream))
            torch.cuda.current_stream().synchronize()
            lib.recon_plan_destroy(h)

        bq = torch.empty((B, N, N), dtype=torch.complex64, device="cuda")
        vq = x.clone()
        h0 = plan._h
        log("timing phases")
        ph_plan = time_phase(plan_gram, 5)
        ph_adj = time_phase(lambda: recon._check(lib.recon_adjoint(
            h0, y.data_ptr(), B, bq.data_ptr(), None, ws.data_ptr(), ws_bytes, stream)), 20)
        ph_app = time_phase(lambda: recon._check(lib.recon_gram_apply(
            h0, vq.data_ptr(), B, bq.data_ptr(), ws.data_ptr(), ws_bytes, stream)), 20)
        ph_solve = time_phase(lambda: solve(h0, y.data_ptr(), B, x.data_ptr(), ws.data_ptr(),
                                            ws_bytes, stats.data_ptr()), 5)
        app_bytes = B * 80 * N * N + 16 * N * N  # per apply: 80 N^2 per frame + K-hat once
        app_gbs = app_bytes / (ph_app["median_ms"] * 1e-3) / 1e9
        ph_app.update({"model_bytes": app_bytes, "achieved_gbs": round(app_gbs, 1),
                       "frac_of_hbm_peak": round(app_gbs / HBM_PEAK_GBS, 4),
                       "what": "v -> Q v on complex64 frames: row FFTs, column pass, row "
                               "inverse; bytes = v in + Qv out + the N x L intermediate "
                               "written and read twice (80 N^2 per frame) + K-hat"})
        ph_adj["achieved_tflops"] = round(8.0 * N * N * M * B / (ph_adj["median_ms"] * 1e-3)
                                          / 1e12, 2)
        phases = {"plan_and_gram_kernel": ph_plan, "adjoint_batch": ph_adj,
                  "toeplitz_apply_batch": ph_app, "solve_batch": ph_solve, "frames": B}
        del bq, vq

    # served stream of 256^2 requests (continuous batching): the benchmark's
    # frames arriving one by one (Poisson), each with its own 300 iterations
    served = []
    rates = [float(v) for v in str(args.serve_rate).split(",") if float(v) > 0]
    if rates and args.workload == "series256" and args.criterion == "plain":
        from paper_0908_3252_amd import serving as srv
        arr = np.cumsum(np.random.default_rng([4, 256]).exponential(1.0, size=args.serve_count))
        key = (N, 16)
        base = [dict(id=i, arrival=float(arr[i]), key=key, y=y[i % B], lam=c_lam, delta=c_delta,
                     iters=iters) for i in range(args.serve_count)]
        for rate in rates:
            log(f"serving {args.serve_count} requests at {rate}/s")
            res = srv.serve(rate, (base, {key: (k_host, N, L)}, {key: plan}),
                            prec=args.prec, verify=1, chunk=args.serve_chunk)
            served.append({"offered_per_sec": rate, "requests": args.serve_count,
                           "completed": res.get("completed", 0),
                           "recons_per_sec": round(res.get("recons_per_sec", 0.0), 2),
                           "p50_ms": round(res.get("p50_ms", float("nan")), 2),
                           "p99_ms": round(res.get("p99_ms", float("nan")), 2),
                           "chunk": args.serve_chunk, "status_ok": res["status_ok"],
                           "bitwise_equal_standalone": res.get("bitwise_equal_standalone")})
    crit = (f"hyperbolic delta={c_delta}, lambda={c_lam}" if args.criterion == "plain" else
            f"Huber differences alpha1={c_delta} lambda1={c_lam} + Huber background "
            f"alpha0={c_alpha0} lambda0={c_lam0}")
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "recons/sec",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64i" else "f32",
        "precision": {
            "fp64i": "f64 adjoint, Gram kernel, iterations, FFTs and reductions; f32 forward model",
            "fp64": "f32 iterations; f64-accumulated adjoint, f64 Gram and reductions",
            "fp32": "f32 (f64 Gram accumulation and reductions)",
            "fp16x3": "f32 iterations; fp16 hi+lo split NUDFT, f64 Gram and reductions",
            "bf16x3": "f32 iterations; bf16 hi+lo split NUDFT, f64 Gram and reductions"}[args.prec],
        "data": "synthetic",
        "config": {"workload": (f"256x256 spiral M={M} (16 interleaves, 2x angular "
                                f"undersampling), {crit}, {iters} iterations, batch of {B} "
                                f"frames sharing the trajectory, L={L}")
                               if args.workload == "series256"
                               else (f"512x512 variable-density spiral M={M} (64 interleaves), "
                                     f"{crit}, {iters} iterations, batch of {B} frames sharing "
                                     f"the trajectory, L={L}"),
                   "criterion": args.criterion,
                   "name": args.workload,
                   "global_batch": B, "image": N, "samples": M, "iters": iters,
                   "parallelism": "none (1 GPU)"},
        "latency_ms": {"p50": round(1e3 * float(np.percentile(times, 50)), 3),
                       "p99": round(1e3 * float(np.percentile(times, 99)), 3),
                       "what": f"one step = {B} reconstructions finishing together"},
        "phases": phases,
        "served_latency_256": {
            "what": "arrival-to-result latency of single 256^2 reconstructions (the frames "
                    "above, 300 iterations each) served by continuous batching, first 10% "
                    "excluded", "runs": served} if served else None,
        "single_frame_latency_ms": {"p50": round(1e3 * float(np.percentile(lat, 50)), 3),
                                    "p99": round(1e3 * float(np.percentile(lat, 99)), 3)},
        "roofline": roofline,
        "rooflines": rooflines,
        "iteration_model": iteration_model,
        "csrc_digest": digest,
        "status_ok_frames": int(np.sum(st["status"] == 0)),
        "grad_ratio_median": float(np.median(st["grad_ratio"])),
    }
    oracle_frame = None
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle, one frame)")
        cb, rel, oracle_frame = cpu_baseline(args, torch, recon, prec)
        out["cpu_baseline"] = {k: v for k, v in cb.items() if k != "seconds"}
        out["cpu_baseline"]["host"] = host_info()
        if rel is not None:
            out["rel_l2_vs_oracle_one_frame"] = rel
    if not args.no_extras and args.workload == "series256" and args.criterion == "plain":
        ctx = dict(torch=torch, recon=recon, lib=lib, prob=prob, y=y, x=x, B=B, N=N, L=L, M=M,
                   prec=prec,
                   iters=iters, k_host=k_host, lam=c_lam, delta=c_delta, stream=stream,
                   oracle_frame=oracle_frame)
        for name, fn in (("precision_form", extra_precision_form),
                         ("half_quadratic_vs_cg", extra_half_quadratic),
                         ("gridding_comparison", extra_gridding),
                         ("nufft_precompute", extra_nufft),
                         ("paper_shape", extra_paper_shape)):
            log(f"extra: {name}")
            out[name] = fn(ctx)
        if args.mixed_count > 0:
            log("extra: mixed-size served stream")
            out["served_mixed"] = extra_served_mixed(args, ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
