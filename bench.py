#!/usr/bin/env python3
"""Throughput of the 256x256 angular-spectrum + STFT32 + Doppler-moment path.

Workload: a stream of 65,536 uint8 frames of 256x256 (4 GiB, resident in
HBM before timing, like the paper's file mode), angular-spectrum
reconstruction at a fixed z, STFT window 32 / stride 32, M0/M1/M2 over
[3, 35] kHz at fs = 71.4 kHz.  One step = one pass of the whole path over the
whole stream.  The FP32 form is the headline value; the mixed form is timed
the same way and reported beside it.

Prints one JSON line.  ``--gpus`` above 1 is refused: this path runs on one
GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "input frames/s @256² AS+STFT32+M0 (FP32 vs mixed, % HBM peak); p99 latency"
HBM_PEAK_GBS = 8000.0
NY = NX = 256
W = 32


def bytes_per_pxf(prec: int, nb: int) -> dict:
    """Algorithmic bytes (read + write) per input pixel-frame of each kernel
    of the two orders, for u8 frames, W = stride = 32, nb band bins and three
    f32 moment images.  e = bytes of one stored complex value."""
    e = 8 if prec == 0 else 4
    return {
        # frames first: u8 in, half spectrum out; half in, full out; W full in, 3 images out
        "row_r2c": 1 + e / 2, "col_as": e / 2 + e, "rowinv_coef": e + 12 / W,
        # band first: W u8 in, nb bin fields out; nb fields in and out; nb in, 3 images out
        "band_rows": 1 + nb * e / W, "band_cols": 2 * nb * e / W, "band_power": nb * e / W + 12 / W,
    }


# library sources that build the kernels and launch shapes of this workload
# (the counter summary under profiles/ is tied to them)
PROFILED_SOURCES = ("api.cpp", "band.hip", "fft_lds.h", "gmem.h", "hv_ctx.h", "hv_internal.h", "spatial.hip",
                    "temporal.hip")


def source_sha() -> str:
    import hashlib
    d = os.path.join(ROOT, "paper_2508_03911_amd", "csrc")
    return hashlib.sha256(b"".join(open(os.path.join(d, f), "rb").read() for f in PROFILED_SOURCES)).hexdigest()[:16]


def measured_traffic(kernel: str, prec: str, field: str = "traffic_bytes_per_dispatch"):
    """HBM bytes per dispatch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, or the DRAM-labelled request counters), or
    None when the library sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_as_stft32_256x256.json")
    try:
        d = json.load(open(path))
    except OSError:
        return None
    if d.get("source_sha") != source_sha():
        return None
    k = d.get("kernels", {}).get(kernel, {}).get(prec)
    return None if k is None else k.get(field)


TRAFFIC_SOURCE = ("rocprofv3 FETCH_SIZE + WRITE_SIZE per dispatch (profiles/hbm_traffic_as_stft32_256x256.json), "
                  "scaled by the counts of a 1 GiB device copy; these count L2-to-fabric traffic, Infinity-Cache "
                  "hits included (no counter on this GPU separates them: the DRAM-labelled request counters "
                  "TCC_EA0_RDREQ_DRAM_32B / TCC_EA0_WRREQ_WRITE_DRAM_32B read the same bytes)")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_steps(ctx, hv, torch, x, opt, tp, prec, outs, steps):
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        ctx.hv_stft_moments(x, opt, tp, prec, out=outs)
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def kernel_profile(ctx, hv, torch, x, opt, tp, prec, outs, steps, frames):
    """Per-kernel average launch time from HIP events recorded around each
    launch on the stream, and the achieved algorithmic bandwidth."""
    ctx.set_timing(True)
    for _ in range(steps):
        ctx.hv_stft_moments(x, opt, tp, prec, out=outs)
    torch.cuda.synchronize()
    res = {}
    for name, bpp in bytes_per_pxf(prec, len(hv.band_bins(tp)[0])).items():
        ms, n = ctx.kernel_time(name)
        if n == 0:
            continue
        avg_ms = ms / n
        pxf_per_launch = frames * steps * NY * NX / n
        gbs = bpp * pxf_per_launch / (avg_ms * 1e-3) / 1e9
        res[name] = {"launches": n, "avg_ms": avg_ms, "total_ms_per_step": ms / steps,
                     "bytes_per_pixel_frame": bpp, "bytes_per_launch": bpp * pxf_per_launch, "achieved_GBs": gbs}
    ctx.set_timing(False)
    return res


# ---------------------------------------------------------------- CPU baseline
# The oracle runs in a pool of worker processes, one window range per task
# (windows are independent).  The workers are forked before this process
# touches the GPU and inherit the base block of the stream.

_ORACLE = {}


def _oracle_worker_init():
    from threadpoolctl import threadpool_limits
    _ORACLE["limits"] = threadpool_limits(1)  # one core per worker


def _oracle_ready(_):
    time.sleep(0.2)  # keep each worker busy so that every one answers
    return os.getpid()


def _oracle_windows(task):
    """The oracle's moments of windows j0 .. j1-1 of the stream (the base
    block replayed cyclically); returned only for windows of the first block
    (the rest repeat them), None otherwise."""
    from oracle import pipeline
    import numpy as np
    j0, j1 = task
    block, spec, z = _ORACLE["block"], _ORACLE["spec"], _ORACLE["z"]
    per = block.shape[0] // W
    frames = np.concatenate([block[(j % per) * W:(j % per + 1) * W] for j in range(j0, j1)])
    ref = pipeline.stft_moments(frames, pipeline.Optics(852e-9, spec.pitch, spec.pitch, -z), W, W, spec.fs,
                                3e3, 35e3)
    if j0 >= per:
        return None
    return j0, {k: ref[k] for k in ("m0", "m1", "m2")}


def oracle_pool(block, spec, z):
    """Fork the oracle workers now (before any GPU call): one per core of
    this process's CPU set, at most 16."""
    import concurrent.futures as cf
    import multiprocessing as mp
    _ORACLE.update(block=block, spec=spec, z=z)
    n = max(1, min(16, len(os.sched_getaffinity(0))))
    pool = cf.ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("fork"), initializer=_oracle_worker_init)
    pids = set(pool.map(_oracle_ready, range(2 * n)))
    return pool, n, len(pids)


def cpu_baseline(pool, workers, frames, block, spec, z, ctx, hv, torch, precision=None):
    """The FP64 oracle, unchanged, over the whole stream (every window of the
    `frames`-frame stream, one window range per task across `workers`
    processes, timed), and the relative L2 error of both GPU forms against
    it on the first block; with `precision` (from precision_case) also the
    errors of window 0 of the 1024 x 1024 Fresnel case, every output, both
    forms."""
    import numpy as np

    nwin = frames // W
    per = block.shape[0] // W
    tasks = [(j, min(nwin, j + 16)) for j in range(0, nwin, 16)]
    t0 = time.perf_counter()
    parts = [r for r in pool.map(_oracle_windows, tasks) if r is not None]
    dt = time.perf_counter() - t0
    ref = {k: np.concatenate([p[1][k] for p in sorted(parts, key=lambda p: p[0])])[:per] for k in ("m0", "m1", "m2")}
    sample = block
    opt = hv.Optics(852e-9, spec.pitch, spec.pitch, -z, hv.HV_AS)
    tp = hv.Temporal(W, W, spec.fs, 3e3, 35e3)
    xd = torch.from_numpy(sample).cuda()
    err = {}
    for order, tag in ((hv.HV_ORDER_FRAMES_FIRST, ""), (hv.HV_ORDER_BAND_FIRST, "band_first_")):
        ctx.set_stft_order(order)
        for prec, name in ((hv.HV_PREC_FP32, "fp32"), (hv.HV_PREC_MIXED, "mixed")):
            got = [t.cpu().numpy().astype(np.float64) for t in ctx.hv_stft_moments(xd, opt, tp, prec)]
            err[tag + name] = {k: float(np.linalg.norm(g - ref[k]) / np.linalg.norm(ref[k]))
                               for k, g in zip(("m0", "m1", "m2"), got)}
    ctx.set_stft_order(hv.HV_ORDER_FRAMES_FIRST)
    res = {"value": nwin * W / dt, "unit": "frames/s", "cores": int(workers), "kind": "oracle",
           "sample": f"the whole stream: {nwin * W} frames ({nwin} windows) of 256x256, numpy float64, "
                     f"{workers} worker processes with one BLAS thread each, 16 windows per task; GPU errors on "
                     f"the first {sample.shape[0]} frames (the rest repeat them)", "seconds": dt,
           "gpu_rel_l2_vs_oracle": err}
    if precision is not None:
        from oracle import optics as oopt, pca as opca, temporal as otemp
        pb, ps, w = precision["block"], precision["spec"], precision["window"]
        u = oopt.fresnel(pb.astype(np.float64), 852e-9, ps.pitch, ps.pitch, -ps.z)
        bins, freqs = otemp.band_bins(w, ps.fs, 2 * ps.fs / w, 31 * ps.fs / w)
        mom = [mm[0] for mm in otemp.moments(otemp.stft(u, w, w), bins, freqs)]
        pr = opca.pca_window(u, 1, 63)
        s_ref = otemp.stft(u, w, w)[0]
        from oracle import ssa as ossa
        sr = ossa.ssa_moments(u, w, w, ps.fs, 2 * ps.fs / w, 31 * ps.fs / w, 1, 63)
        rel = lambda a, b: float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
        res["precision_case_window0_rel_l2"] = {
            name: {"spectrum_all_64_bins": rel(g["spectrum"], s_ref[g["bins"]]),
                   "m0": rel(g["m"][0], mom[0]), "m1": rel(g["m"][1], mom[1]), "m2": rel(g["m"][2], mom[2]),
                   "covariance": rel(g["cov"], pr["cov"]), "eigvals": rel(g["eigvals"], pr["eigvals"]),
                   "pca_m0": rel(g["pca_m0"], pr["m0"]),
                   "ssa_m0": rel(g["ssa"][0], sr["m0"][0]), "ssa_m1": rel(g["ssa"][1], sr["m1"][0]),
                   "ssa_m2": rel(g["ssa"][2], sr["m2"][0])}
            for name, g in precision["gpu"].items()}
    return res


def serving(hv, torch, seconds, prec):
    """The mixed-size stream load: 4 slots each of 256x256 u8 at 71.4 kHz
    (W 16), 512x512 u8 at 20 kHz (W 32) and 1024x512 u16 at 5 kHz (W 64),
    Poisson arrivals at 6/s with Exp(2 s) lifetimes, z uniform in
    [0.1, 0.4] m, HBM budget 32 GiB, device-resident camera blocks."""
    from synth import holograms
    classes = []
    for cls in range(3):
        t0 = time.time()
        x, spec = holograms.stream_block(cls, cls)
        ny, nx, bits, fs, w, _ = holograms.STREAM_CLASSES[cls]
        classes.append(dict(ny=ny, nx=nx, raw_t=0, fps=fs, window=w, stride=w, f_lo=2 * fs / w,
                            f_hi=(w // 2 - 1) * fs / w, block=torch.from_numpy(x).cuda(), max_active=4,
                            ring_frames=0))
        log(f"stream class {cls}: block {x.shape} {x.dtype} in {time.time() - t0:.1f}s")
    ctx = hv.Context(0, hbm_budget=32 << 30)
    r = ctx.hv_replay_run(classes, wavelength=852e-9, pitch=20e-6, z_lo=0.1, z_hi=0.4, prec=prec, arrival_hz=6.0,
                          mean_life_s=2.0, duration_s=seconds, warmup_s=1.0, packet_frames=8, seed=5)
    ctx.close()
    return {"seconds": r["seconds"], "frames_per_s": r["frames_per_s"], "frames_offered": r["frames_offered"],
            "frames_in": r["frames_in"], "frames_dropped": r["frames_dropped"], "windows_done": r["windows_done"],
            "streams_admitted": r["streams_admitted"], "streams_refused": r["streams_refused"],
            "lat_p50_ms": r["lat_p50_ns"] / 1e6, "lat_p99_ms": r["lat_p99_ns"] / 1e6,
            "lat_max_ms": r["lat_max_ns"] / 1e6, "latency_samples": r["latency_samples"],
            "precision": "fp32" if prec == 0 else "mixed",
            "load": "12 slots (4 per class): 256x256 u8 71.4 kHz W16, 512x512 u8 20 kHz W32, "
                    "1024x512 u16 5 kHz W64; Poisson 6/s, Exp(2 s) lifetimes; budget 32 GiB"}


def he_normal_init(seed):
    """Initial network parameters in the library's storage order: per conv
    layer weight [co][ci][3][3] then bias, per FC layer weight [out][in] then
    bias; weights N(0, 2 / fan_in), biases zero."""
    import numpy as np
    rng = np.random.default_rng(seed)
    parts = []
    for co, ci, k in ((32, 1, 3), (32, 32, 3), (32, 32, 3), (32, 32, 3), (64, 32, 1), (2, 64, 1)):
        fan_in = ci * k * k
        parts += [rng.standard_normal(co * fan_in) * np.sqrt(2.0 / fan_in), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


# local scan seeded by the network: candidates (half over z +- AF_K sigma,
# half over one coarse step around the best of those)
AF_REFINE, AF_K = 12, 2.0


def autofocus(hv, torch, n_train, n_eval, epochs, batch=256, lr=1e-3):
    """Learned autofocus: train the CNN on n_train holograms synthesised on
    the GPU by the project's forward model (z uniform in [0.05, 0.5] m,
    quantised to 512 levels), evaluate on n_eval held-out holograms against
    the 128-candidate scan, with the scan as fallback for the 10 % least
    confident predictions."""
    import numpy as np

    lam, pitch = 852e-9, 20e-6
    z_mean, z_scale = 0.275, 0.45 / np.sqrt(12)
    ctx = hv.Context(0)

    def dataset(n, seed, base):
        rng = np.random.default_rng(seed)
        lv = rng.integers(0, 512, n // 16)
        z = np.repeat(0.05 + 0.45 * (lv + 0.5) / 512, 16)
        crops, holos = [], []
        for i in range(0, n, 4096):
            h = ctx.hv_af_synthesize(z[i:i + 4096], lam, pitch, seed=seed, index_base=base + i)
            crops.append(ctx.hv_af_crops(h))
            holos.append(h)
        return torch.cat(crops), holos, torch.from_numpy(z.astype(np.float32)).cuda()

    t0 = time.time()
    crops, holos, z = dataset(n_train, 1000, 0)
    del holos
    torch.cuda.synchronize()
    t_gen = time.time() - t0
    log(f"autofocus: {n_train} training holograms synthesised and cropped in {t_gen:.1f}s")
    init = he_normal_init(7)
    model = ctx.af_model(init, batch, z_mean, z_scale)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    g = torch.Generator(device="cuda").manual_seed(0)
    steps = epochs * (n_train // batch)
    curve = []
    torch.cuda.synchronize()
    t0 = time.time()
    for step in range(steps):
        idx = torch.randint(0, n_train, (batch,), device="cuda", generator=g)
        rate = lr if step < steps * 0.7 else lr * 0.1
        model.train_step(crops[idx].contiguous(), z[idx].contiguous(), rate, loss)
        if step % max(1, steps // 10) == 0 or step == steps - 1:
            curve.append(round(loss.item(), 4))
    torch.cuda.synchronize()
    t_train = time.time() - t0
    log(f"autofocus: {steps} steps in {t_train:.1f}s, loss {curve}")
    del crops
    _, eh, ez = dataset(n_eval, 9000000, 9000000)
    eh = torch.cat(eh)
    ez = ez.cpu().numpy()

    def timed(fn, reps=3):
        # one untimed call (tables, workspaces), then the median of `reps`
        r = fn()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return r, float(np.median(ts))

    (zs, _), t_scan = timed(lambda: ctx.hv_af_scan(eh, lam, pitch))
    (zn, sig, _, _), t_net = timed(lambda: model.predict(eh, lam, pitch, tau=1e9))
    tau = float(np.quantile(sig.cpu().numpy(), 0.9))
    (zf, _, used, nfb), t_fb = timed(lambda: model.predict(eh, lam, pitch, tau=tau))
    (zl, _, _, _), t_loc = timed(lambda: model.predict(eh, lam, pitch, tau=1e9, refine=AF_REFINE, refine_k=AF_K))
    (zlf, _, _, nlf), t_lf = timed(lambda: model.predict(eh, lam, pitch, tau=tau, refine=AF_REFINE, refine_k=AF_K))

    def err(zhat):
        e = np.abs(zhat.cpu().numpy() - ez) * 1e3
        return {"median_mm": float(np.median(e)), "p90_mm": float(np.quantile(e, 0.9)),
                "rms_mm": float(np.sqrt(np.mean(e ** 2)))}

    out = {"train_holograms": n_train, "eval_holograms": n_eval, "epochs": epochs, "steps": steps,
           "synth_seconds": t_gen, "train_seconds": t_train, "train_samples_per_s": steps * batch / t_train,
           "loss_curve": curve,
           "mean_predictor": {"median_mm": float(np.median(np.abs(ez - z_mean)) * 1e3)},
           "cnn": {**err(zn), "holograms_per_s": n_eval / t_net},
           "cnn_fallback": {**err(zf), "holograms_per_s": n_eval / t_fb, "fallback_fraction": nfb / n_eval,
                            "tau_m": tau},
           "cnn_local_scan": {**err(zl), "holograms_per_s": n_eval / t_loc, "candidates": AF_REFINE, "k_sigma": AF_K,
                              "speedup_vs_scan": t_scan / t_loc,
                              "median_vs_scan": float(np.median(np.abs(zl.cpu().numpy() - ez))
                                                      / np.median(np.abs(zs.cpu().numpy() - ez)))},
           "cnn_local_scan_fallback": {**err(zlf), "holograms_per_s": n_eval / t_lf,
                                       "fallback_fraction": nlf / n_eval, "speedup_vs_scan": t_scan / t_lf},
           "scan": {**err(zs), "holograms_per_s": n_eval / t_scan, "candidates": 128}}
    model.close()
    ctx.close()
    return out


# The paper's Table IV: frame sizes (ny, nx), frames per timed pass, and its
# file-mode fps on an RTX 4090 for the two pipelines (context, not targets).
TABLE_IV = (
    ((256, 256), 16384, {"as_hp_stft512": 88100, "fresnel_pca32": 53090}),
    ((512, 512), 4096, {"as_hp_stft512": 23100, "fresnel_pca32": 25200}),
    ((320, 512), 8192, {"as_hp_stft512": 35900, "fresnel_pca32": 37850}),
    ((384, 384), 8192, {"as_hp_stft512": 39000, "fresnel_pca32": 40270}),
    ((800, 1280), 2048, {"as_hp_stft512": 6100, "fresnel_pca32": 6650}),
)


def table_iv_inputs(torch):
    """Synthetic u8 stacks of the Table IV sizes resident in device memory: a
    base block from the generator (z drawn in [0.1, 0.4] m) replayed to the
    pass length."""
    from synth import holograms
    out = []
    for k, ((ny, nx), frames, paper) in enumerate(TABLE_IV):
        t0 = time.time()
        if (ny, nx) == (256, 256):
            block, spec = holograms.config_c2_block(2048)
        else:
            spec = holograms.HoloSpec(frames=64 if ny * nx <= 512 * 512 else 32, ny=ny, nx=nx,
                                      z=holograms.drawn_z(20 + k), fs=20e3, seed=20 + k)
            block = holograms.hologram_stack(spec)
        xb = torch.from_numpy(block).cuda()
        x = xb.repeat(frames // block.shape[0], 1, 1).contiguous()
        del xb
        log(f"Table IV input {ny}x{nx}: {block.shape[0]}-frame block in {time.time() - t0:.1f}s, {frames} frames")
        out.append(((ny, nx), x, spec, paper))
    return out


def _timed_passes(torch, fn, steps):
    fn()  # warm-up: plans and workspaces
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


MFMA_PEAK_TFLOPS = {"fp32": 157.3, "mixed": 2500.0}  # dense matrix peak of the operand type used


def precision_case(hv, torch, steps):
    """The precision-form workload: 4,096 uint16 (12-bit) frames of 1024 x 1024
    (a 64-frame synthetic block replayed 64 times, resident in HBM), Fresnel at
    z = 0.5 m, then (a) the STFT over windows of 64 (stride 64, bins 2..31 at
    fs 5 kHz) with its moments, (b) PCA over the same windows (components
    1..63) and (c) SSA + FFT over them (components 1..63, then the band
    moments).  Reports frames/s per form and the GEMM kernels' useful TFLOP/s
    against the matrix-core peak of their operand type; returns as well the
    GPU outputs of window 0 and the block, for the oracle check of the
    cpu_baseline leg."""
    import numpy as np
    from synth import holograms
    t0 = time.time()
    block, spec = holograms.config_c3(64)
    log(f"precision case: block {block.shape} in {time.time() - t0:.1f}s")
    x = torch.from_numpy(block).cuda().repeat(64, 1, 1).contiguous()
    n, ny, nx = x.shape
    w = 64
    opt = hv.Optics(852e-9, spec.pitch, spec.pitch, -spec.z, hv.HV_FRESNEL)
    fs = spec.fs
    tp = hv.Temporal(w, w, fs, 2 * fs / w, 31 * fs / w)
    nb = len(hv.band_bins(tp)[0])
    nwin = n // w
    npix = ny * nx
    # useful flops per pixel and window of each GEMM (real arithmetic on
    # (re, im)-interleaved operands, K = 2W)
    flops = {"field_coef": 2 * (2 * nb) * (2 * w), "gram": 2 * (2 * w) ** 2, "proj_energy": 2 * (2 * 63) * (2 * w),
             "ssa_moments": 2 * (2 * nb) * (2 * w)}
    ctx = hv.Context(0)
    out = {"workload": f"{n} uint16 frames of {nx}x{ny} (12-bit), Fresnel z={spec.z} m, W={w} stride {w}, "
                       f"{nb} band bins, PCA components 1..63", "frames": n}
    res_keep = {}
    for prec, name in ((hv.HV_PREC_FP32, "fp32"), (hv.HV_PREC_MIXED, "mixed")):
        stft = lambda: ctx.hv_stft_moments(x, opt, tp, prec)
        pca = lambda: ctx.hv_pca(x, opt, w, w, 1, 63, prec, want_eig=True)
        ssa = lambda: ctx.hv_ssa_moments(x, opt, tp, 1, 63, prec)
        ms_s = _timed_passes(torch, stft, steps)
        ms_p = _timed_passes(torch, pca, steps)
        ms_a = _timed_passes(torch, ssa, steps)
        kern = {}
        # per path: the launches of one pass, timed by events on their own
        # streams (two streams share the GPU, so a launch's time includes the
        # time it shares it)
        for path, fn in (("stft", stft), ("pca", pca), ("ssa", ssa)):
            ctx.set_timing(True)
            fn()
            torch.cuda.synchronize()
            kp = {}
            for k in ("fresnel_rows", "fresnel_cols", "field_coef", "gram", "jacobi", "proj_energy", "ssa_moments"):
                ms, cnt = ctx.kernel_time(k)
                if cnt == 0:
                    continue
                kp[k] = {"launches": cnt, "avg_ms": ms / cnt}
                if k in flops:
                    tf = flops[k] * npix * nwin / (ms * 1e-3) / 1e12
                    kp[k].update({"useful_TFLOPs": tf, "mfma_peak_TFLOPs": MFMA_PEAK_TFLOPS[name],
                                  "frac": tf / MFMA_PEAK_TFLOPS[name]})
            kern[path] = kp
        ctx.set_timing(False)
        # alone on one stream: the Fresnel passes (hv_propagate of one window's
        # frames, field written) and the DFT GEMM on that field in memory
        fld = torch.empty((w, ny, nx), dtype=torch.complex64, device="cuda")
        ctx.hv_propagate(x[:w], opt, prec, out=fld)
        torch.cuda.synchronize()
        ctx.set_timing(True)
        for _ in range(steps):
            ctx.hv_propagate(x[:w], opt, prec, out=fld)
        torch.cuda.synchronize()
        alone = {}
        in_b = 2  # u16 camera values
        cb = 8 if prec == hv.HV_PREC_FP32 else 4
        for k, bpp in (("fresnel_rows", in_b + cb), ("fresnel_cols", cb + 8)):
            ms, cnt = ctx.kernel_time(k)
            if cnt:
                gbs = bpp * npix * w / (ms / cnt * 1e-3) / 1e9
                alone[k] = {"avg_ms": ms / cnt, "bytes_per_launch": bpp * npix * w, "GBs": gbs,
                            "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
        ctx.set_timing(False)
        tp_f = hv.Temporal(w, w, fs, 2 * fs / w, 31 * fs / w)
        mo = [torch.empty((1, ny, nx), dtype=torch.float32, device="cuda") for _ in range(3)]
        ms_g = _timed_passes(torch, lambda: ctx.hv_stft_moments(fld, None, tp_f, prec, out=mo), steps)
        gemm_b = 8 * npix * w + 12 * npix
        alone["field_coef_c64_field"] = {"avg_ms": ms_g, "field_GBs": gemm_b / (ms_g * 1e-3) / 1e9,
                                         "frac_of_hbm_peak": gemm_b / (ms_g * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                         "useful_TFLOPs": flops["field_coef"] * npix / (ms_g * 1e-3) / 1e12}
        del fld, mo
        # PCA of one window: a single chunk, so its covariance, eigensolve and
        # projection run on one stream with nothing beside them
        ctx.hv_pca(x[:w], opt, w, w, 1, 63, prec)
        torch.cuda.synchronize()
        ctx.set_timing(True)
        for _ in range(steps):
            ctx.hv_pca(x[:w], opt, w, w, 1, 63, prec)
        torch.cuda.synchronize()
        for k in ("gram", "jacobi", "proj_energy"):
            ms, cnt = ctx.kernel_time(k)
            if cnt:
                alone[k + "_one_window"] = {"avg_ms": ms / cnt}
                if k in flops:
                    tf = flops[k] * npix / (ms / cnt * 1e-3) / 1e12
                    alone[k + "_one_window"].update({"useful_TFLOPs": tf, "frac": tf / MFMA_PEAK_TFLOPS[name]})
        ctx.set_timing(False)
        out[name] = {"stft_moments_frames_per_s": n / (ms_s * 1e-3), "pca_frames_per_s": n / (ms_p * 1e-3),
                     "ssa_fft_moments_frames_per_s": n / (ms_a * 1e-3), "kernels": kern, "kernels_alone": alone}
        log(f"precision case {name}: {out[name]}")
        m = [t[0].cpu().numpy().astype(np.float64) for t in stft()]
        r = ctx.hv_pca(x[:w], opt, w, w, 1, 63, prec, want_eig=True, want_cov=True)
        # every bin of window 0: the band [0, fs/2] taken on both sides
        tp_all = hv.Temporal(w, w, fs, 0.0, fs / 2, True)
        s_all = ctx.hv_stft_bins(x[:w], opt, tp_all, prec)[0].cpu().numpy()
        ra = ctx.hv_ssa_moments(x[:w], opt, tp, 1, 63, prec)
        res_keep[name] = {"m": m, "pca_m0": r["m0"][0].cpu().numpy().astype(np.float64),
                          "ssa": [ra[k][0].cpu().numpy().astype(np.float64) for k in ("m0", "m1", "m2")],
                          "eigvals": r["eigvals"][0].cpu().numpy(), "cov": r["cov"][0].cpu().numpy(),
                          "spectrum": s_all, "bins": hv.band_bins(tp_all)[0]}
        del s_all
    ctx.close()
    del x
    return out, {"block": block[:w], "spec": spec, "window": w, "gpu": res_keep}


def table_iv(hv, torch, inputs, steps):
    """The paper's Table IV Fresnel + PCA pipeline (window 32, stride 32,
    components 1..31) at its five frame sizes, file mode."""
    out = {}
    ctx = hv.Context(0)
    for (ny, nx), x, spec, paper in inputs:
        frames = x.shape[0]
        opt = hv.Optics(852e-9, spec.pitch, spec.pitch, -spec.z, hv.HV_FRESNEL)
        res = {}
        for prec, name in ((hv.HV_PREC_FP32, "fp32"), (hv.HV_PREC_MIXED, "mixed")):
            ms = _timed_passes(torch, lambda: ctx.hv_pca(x, opt, 32, 32, 1, 31, prec, want_eig=False), steps)
            res[name] = {"frames_per_s": frames / (ms * 1e-3), "ms_per_pass": ms,
                         "gigapixels_per_s": frames * ny * nx / (ms * 1e-3) / 1e9}
        log(f"table IV Fresnel+PCA32 {nx}x{ny}: {res}")
        out[f"{nx}x{ny}"] = {"frames": frames, **res, "paper_file_fps_rtx4090": paper["fresnel_pca32"]}
    ctx.close()
    return out


def table_iv_volume(hv, torch, inputs, steps, highpass=0.05):
    """The paper's Table IV angular spectrum + spatial high-pass filter +
    STFT 512/512 pipeline (every bin of every window rendered: |S_k|^2 as a
    float32 volume) at its five frame sizes, file mode.  The high-pass radius
    is not given in the paper; 0.05 cycles per pixel is used (the filter is a
    mask in the transfer table, so its value does not change the work)."""
    out = {}
    ctx = hv.Context(0)
    for (ny, nx), x, spec, paper in inputs:
        frames = x.shape[0]
        opt = hv.Optics(852e-9, spec.pitch, spec.pitch, -spec.z, hv.HV_AS, highpass)
        vol = torch.empty((frames // 512, 512, ny, nx), dtype=torch.float32, device="cuda")
        res = {}
        for prec, name in ((hv.HV_PREC_FP32, "fp32"), (hv.HV_PREC_MIXED, "mixed")):
            ms = _timed_passes(torch, lambda: ctx.hv_stft_volume(x, opt, 512, 512, prec, out=vol), steps)
            res[name] = {"frames_per_s": frames / (ms * 1e-3), "ms_per_pass": ms,
                         "gigavoxels_per_s": frames * ny * nx / (ms * 1e-3) / 1e9}
        log(f"table IV AS+HP+STFT512 {nx}x{ny}: {res}")
        out[f"{nx}x{ny}"] = {"frames": frames, "highpass_cycles_per_pixel": highpass, **res,
                             "paper_file_fps_rtx4090": paper["as_hp_stft512"]}
        del vol
    ctx.close()
    return out


def copy_rate(torch, reps: int = 10):
    """Device-to-device copy of 2 GiB by torch: read + write bytes per second,
    the practical HBM rate that the pass-level figure can be read against."""
    src = torch.empty(1 << 31, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    gbs = 2 * (1 << 31) * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    return {"GBs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS, "note": "torch copy of 2 GiB, read + write bytes"}


def bins_image_rate(ctx, hv, torch, reps: int = 10):
    """Magnitude and argument images (hv_bins_image) over the 14 band bins
    of 64 windows of the 256x256 stream: the spectrum [64][14][256][256] c64
    (470 MB) is read once and [64][256][256] float32 written, so the
    algorithmic bytes are 14 * 8 + 4 = 116 per pixel and window.  HIP events
    on the stream the kernel is launched on."""
    j, nb = 64, 14
    spec_t = torch.randn((j, nb, NY, NX), dtype=torch.complex64, device="cuda")
    out = torch.empty((j, NY, NX), dtype=torch.float32, device="cuda")
    nbytes = j * NY * NX * (nb * 8 + 4)
    res = {"workload": f"{j} windows x {nb} bins of {NY}x{NX} c64", "bytes_per_launch": nbytes}
    for kind, name in ((hv.HV_IMG_MAGNITUDE, "magnitude"), (hv.HV_IMG_ARGUMENT, "argument")):
        ctx.hv_bins_image(spec_t, kind, out=out)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            ctx.hv_bins_image(spec_t, kind, out=out)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        gbs = nbytes / (ms * 1e-3) / 1e9
        res[name] = {"ms_per_launch": ms, "GBs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS}
    del spec_t, out
    return res


def isolated_kernels(ctx, hv, torch, x, opt, steps, frames=8192):
    """The per-frame path's row and column kernels timed alone: hv_propagate
    (K1, K2, row inverse) on one stream over the first `frames` frames, with
    the same launch shapes as the headline, so no other stream shares the GPU
    during a launch.  Algorithmic bytes as in bytes_per_pxf."""
    xs = x[:frames]
    out = torch.empty((frames, NY, NX), dtype=torch.complex64, device="cuda")
    ctx.hv_propagate(xs, opt, hv.HV_PREC_FP32, out=out)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for _ in range(steps):
        ctx.hv_propagate(xs, opt, hv.HV_PREC_FP32, out=out)
    torch.cuda.synchronize()
    res = {}
    bpp = bytes_per_pxf(0, 14)
    for name in ("row_r2c", "col_as"):
        ms, n = ctx.kernel_time(name)
        if n == 0:
            continue
        per_launch = bpp[name] * NY * NX * frames * steps / n
        gbs = per_launch / (ms / n * 1e-3) / 1e9
        res[name] = {"launches": n, "avg_ms": ms / n, "bytes_per_launch": per_launch, "achieved_GBs": gbs,
                     "frac": gbs / HBM_PEAK_GBS}
    ctx.set_timing(False)
    del out
    return res


def host_ingest(hv, torch, block, spec, frames, steps):
    """The same 256x256 stream with its frames in pinned host memory and the
    moment images returned to pinned host memory: every frame crosses PCIe
    (the paper's camera-side path).  PCIe-inclusive context, not the
    headline value."""
    reps = frames // block.shape[0]
    xh = torch.empty((reps * block.shape[0],) + block.shape[1:], dtype=torch.uint8, pin_memory=True)
    src = torch.from_numpy(block)
    for r in range(reps):
        xh[r * block.shape[0]:(r + 1) * block.shape[0]].copy_(src)
    ctx = hv.Context(0)
    opt = hv.Optics(852e-9, spec.pitch, spec.pitch, -spec.z, hv.HV_AS)
    tp = hv.Temporal(W, W, spec.fs, 3e3, 35e3)
    res = {}
    for prec, name in ((hv.HV_PREC_FP32, "fp32"), (hv.HV_PREC_MIXED, "mixed")):
        out = ctx.hv_stft_moments_host(xh, opt, tp, prec)  # warm-up; allocates the pinned images
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.hv_stft_moments_host(xh, opt, tp, prec, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        res[name] = {"frames_per_s": xh.shape[0] / dt, "ms_per_pass": dt * 1e3,
                     "h2d_GBs": xh.numel() / dt / 1e9}
    ctx.close()
    log(f"host ingest: {res}")
    return {"frames": int(xh.shape[0]), **res,
            "note": "frames in pinned host memory, images back to pinned host memory; PCIe-inclusive"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=65536)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=20.0, help="stream-load replay length (0 = skip)")
    ap.add_argument("--af-train", type=int, default=200000, help="autofocus training holograms (0 = skip)")
    ap.add_argument("--af-eval", type=int, default=10000)
    ap.add_argument("--af-epochs", type=int, default=3)
    ap.add_argument("--no-table-iv", action="store_true", help="skip the Table IV measurements")
    ap.add_argument("--no-host-ingest", action="store_true", help="skip the pinned-host (PCIe) measurement")
    ap.add_argument("--no-precision-case", action="store_true", help="skip the 1024x1024 u16 Fresnel W64 case")
    ap.add_argument("--no-large-chunks", action="store_true",
                    help="skip the headline pass with chunks larger than the Infinity Cache")
    ap.add_argument("--precision-case-only", action="store_true",
                    help="run only the 1024x1024 u16 Fresnel W64 case and print its JSON")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device-to-device copy (scale factor for HBM counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the windows are independent, "
              "so N GPUs would each run this same per-GPU workload.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2508_03911_amd import hv
    from synth import holograms

    if args.precision_case_only:
        print(json.dumps({"precision_case": precision_case(hv, torch, max(1, args.steps // 3))[0]}), flush=True)
        return

    t0 = time.time()
    block, spec = holograms.config_c2_block(2048)
    log(f"generated base block {block.shape} in {time.time() - t0:.1f}s (z = {spec.z:.4f} m)")
    reps = args.frames // block.shape[0]
    frames = reps * block.shape[0]
    pool = None
    if not args.no_cpu_baseline:
        pool, workers, forked = oracle_pool(block, spec, spec.z)
        log(f"oracle pool: {workers} workers ({forked} answered)")
    xb = torch.from_numpy(block).cuda()
    x = xb.repeat(reps, 1, 1).contiguous()  # the stream replays the base block cyclically
    del xb
    ctx = hv.Context(0)
    opt = hv.Optics(852e-9, spec.pitch, spec.pitch, -spec.z, hv.HV_AS)
    tp = hv.Temporal(W, W, spec.fs, 3e3, 35e3)
    j = frames // W
    outs = [torch.empty((j, NY, NX), dtype=torch.float32, device="cuda") for _ in range(3)]

    def measure(order):
        ctx.set_stft_order(order)
        res = {}
        for prec in (hv.HV_PREC_FP32, hv.HV_PREC_MIXED):
            for _ in range(args.warmup):
                ctx.hv_stft_moments(x, opt, tp, prec, out=outs)
            ms = time_steps(ctx, hv, torch, x, opt, tp, prec, outs, args.steps)
            kern = kernel_profile(ctx, hv, torch, x, opt, tp, prec, outs, args.steps, frames)
            res[prec] = {"ms_per_step": ms, "frames_per_s": frames / (ms * 1e-3), "kernels": kern}
            log(f"order {order} prec {prec}: {ms:.3f} ms/step, {frames / (ms * 1e-3) / 1e6:.3f} M frames/s")
        ctx.set_stft_order(hv.HV_ORDER_FRAMES_FIRST)
        return res

    def large_chunks():
        """The headline pass with chunks of 512 and 1,024 frames: 384 / 768 MiB
        (FP32) of intermediate spectra per chunk, two chunks in flight, so
        every intermediate is evicted from the 256 MiB Infinity Cache before
        it is read back and the pass-level rate is a rate to and from HBM."""
        res = {}
        for chunk in (512, 1024):
            ctx.set_chunk_frames(chunk)
            for prec, name in ((hv.HV_PREC_FP32, "fp32"), (hv.HV_PREC_MIXED, "mixed")):
                ctx.hv_stft_moments(x, opt, tp, prec, out=outs)
                ms = time_steps(ctx, hv, torch, x, opt, tp, prec, outs, max(3, args.steps // 2))
                bpf = 25.375 if prec == hv.HV_PREC_FP32 else 13.375
                gbs = bpf * NY * NX * frames / (ms * 1e-3) / 1e9
                res[f"{name}_chunk{chunk}"] = {"frames_per_s": frames / (ms * 1e-3), "ms_per_step": ms,
                                               "pass_level_GBs": gbs, "frac": gbs / HBM_PEAK_GBS,
                                               "intermediate_MiB_per_chunk": chunk * NY * NX * 1.5 *
                                               (8 if prec == hv.HV_PREC_FP32 else 4) / 2 ** 20}
            log(f"chunk {chunk}: {res}")
        ctx.set_chunk_frames(0)
        return res

    def roofline(r):
        name, k = max(r["kernels"].items(), key=lambda kv: kv[1]["total_ms_per_step"])
        dram = measured_traffic(name, "fp32", "dram_read_bytes_per_dispatch")
        dramw = measured_traffic(name, "fp32", "dram_write_bytes_per_dispatch")
        return {"bound": "hbm", "kernel": name, "achieved": k["achieved_GBs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": k["achieved_GBs"] / HBM_PEAK_GBS, "traffic": measured_traffic(name, "fp32"),
                "traffic_source": TRAFFIC_SOURCE,
                "dram_labelled_bytes": None if dram is None or dramw is None else dram + dramw,
                "algorithmic_bytes_per_launch": k["bytes_per_launch"], "avg_launch_ms": k["avg_ms"]}

    def pass_level(r):
        bpf = sum(k["bytes_per_pixel_frame"] for k in r["kernels"].values())
        gbs = bpf * NY * NX * frames / (r["ms_per_step"] * 1e-3) / 1e9
        return {"GBs": gbs, "frac": gbs / HBM_PEAK_GBS, "bytes_per_pixel_frame": bpf}

    # the headline keeps the paper's order: every frame propagated, then the
    # temporal transform
    res = measure(hv.HV_ORDER_FRAMES_FIRST)
    fp32, mixed = res[hv.HV_PREC_FP32], res[hv.HV_PREC_MIXED]
    band = measure(hv.HV_ORDER_BAND_FIRST)
    bf32, bmix = band[hv.HV_PREC_FP32], band[hv.HV_PREC_MIXED]
    line = {
        "metric": METRIC,
        "value": fp32["frames_per_s"],
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"256x256 uint8 x {frames} frames resident in HBM; angular spectrum at z=-{spec.z:.4f} m; "
                               "STFT window 32 stride 32; M0/M1/M2 over [3,35] kHz at fs 71.4 kHz",
                   "frames": frames, "ny": NY, "nx": NX, "window": W, "stride": W, "precision": "fp32"},
        "roofline": roofline(fp32),
        "pass_level_hbm": pass_level(fp32),
        "mixed": {"value": mixed["frames_per_s"], "ms_per_step": mixed["ms_per_step"],
                  "speedup_vs_fp32": mixed["frames_per_s"] / fp32["frames_per_s"],
                  "kernels": mixed["kernels"]},
        "kernels_fp32": fp32["kernels"],
        "band_first_variant": {
            "label": "band-only variant, not the headline: the 14 band bins of each window are formed from its "
                     "raw frames and only those fields are propagated (the two linear steps swapped; same "
                     "moments up to rounding, see gpu_rel_l2_vs_oracle in cpu_baseline)",
            "value": bf32["frames_per_s"], "unit": "frames/s", "ms_per_step": bf32["ms_per_step"],
            "roofline": roofline(bf32), "pass_level_hbm": pass_level(bf32),
            "mixed": {"value": bmix["frames_per_s"], "ms_per_step": bmix["ms_per_step"],
                      "speedup_vs_fp32": bmix["frames_per_s"] / bf32["frames_per_s"], "kernels": bmix["kernels"]},
            "kernels_fp32": bf32["kernels"]},
        "pass_level_hbm_large_chunks": None if args.no_large_chunks else large_chunks(),
        "hbm_copy": copy_rate(torch),
        "kernels_alone_fp32": isolated_kernels(ctx, hv, torch, x, opt, max(1, args.steps // 2)),
        "bins_image": bins_image_rate(ctx, hv, torch),
    }
    if args.serve_seconds > 0:
        log(f"stream load replay for {args.serve_seconds:.0f}s ...")
        line["serving"] = serving(hv, torch, args.serve_seconds, hv.HV_PREC_FP32)
        log(f"serving: {line['serving']}")
    if not args.no_host_ingest:
        log("host ingest (PCIe) ...")
        line["host_ingest"] = host_ingest(hv, torch, block, spec, frames, max(1, args.steps // 3))
    if not args.no_table_iv:
        inputs = table_iv_inputs(torch)
        log("Table IV Fresnel + PCA32 ...")
        line["table_iv_fresnel_pca32"] = table_iv(hv, torch, inputs, max(1, args.steps // 2))
        log("Table IV AS + high-pass + STFT512 ...")
        line["table_iv_as_hp_stft512"] = table_iv_volume(hv, torch, inputs, max(1, args.steps // 2))
        del inputs
    precision = None
    if not args.no_precision_case:
        log("precision case (1024x1024 u16 Fresnel, W 64, STFT moments and PCA) ...")
        line["precision_case"], precision = precision_case(hv, torch, max(1, args.steps // 3))
    if args.af_train > 0:
        log("autofocus training and evaluation ...")
        line["autofocus"] = autofocus(hv, torch, args.af_train, args.af_eval, args.af_epochs)
        log(f"autofocus: {line['autofocus']}")
    if not args.no_cpu_baseline:
        log("timing the oracle over the stream ...")
        line["cpu_baseline"] = cpu_baseline(pool, workers, frames, block, spec, spec.z, ctx, hv, torch, precision)
        pool.shutdown()
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
