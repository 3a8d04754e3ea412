#!/usr/bin/env python3
"""Throughput of the fused DWT pan-sharpening kernels on one MI355X.

Primary line: Daubechies-4 on the Landsat-7-shaped scene, PAN 15872 x 14336,
6 MS bands (synthetic, seeded), inputs resident in HBM; one step = one fused
forward launch over all bands.  The other workloads (Haar on the same scene,
D4 8192 x 8192 with 3 bands, Haar 512 x 512, the 96-scene batch, 8-bit I/O,
kappa = 2, the paper's multi-pass pipeline, the adjoint and the
differentiation step) are reported under "workloads".  Prints exactly one
JSON line on stdout; progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --mode copy      # plain copy kernel (counter calibration)
    python bench.py --mode primary   # primary workload only (for profiling)
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fuse_d4_landsat_15872x14336_b6.json")

# The paper's own performance claim, quoted as context (other hardware, end-to-end
# cluster wall times including network transfers); not a target.
PAPER_CONTEXT = {
    "claim": "GPU cluster 2-18x faster than the CPU cluster over the four fusion methods (section 4, "
             "Tables 1-2, Fig. 4)",
    "hardware": "4 nodes x GeForce GTX 460 (GPU cluster) vs 4 nodes x Core 2 Quad Q8400, 4 GB RAM, "
                "1 Gbit/s Ethernet, MPICH2, Windows 7 x64 (CPU cluster)",
    "paper_times_s_16280x14960": {"haar_gpu_cluster": 3.61, "d4_gpu_cluster": 3.70,
                                  "haar_cpu_cluster": 11.6, "d4_cpu_cluster": 13.5},
    "note": "end-to-end wall time of a 4-node cluster including scatter/gather of 8-bit parts; band count not "
            "stated; context only, not comparable to one GPU's kernel time",
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algo_bytes(H, W, B):
    """PAN read once, MS read once, every output band written once."""
    return H * W * 4 + B * (H // 2) * (W // 2) * 4 + B * H * W * 4


class Prepared:
    """Pre-marshalled dwt_fuse_run call (keeps Python overhead out of the loop)."""

    def __init__(self, api, pan, ms, wavelet, out, gain=None):
        from paper_1803_00737_amd._lib import wavelet_id

        self.ctx = api.context(pan.device)
        self.ctx.bind_stream()
        H, W = pan.shape
        B = ms.shape[0]
        self.args = (self.ctx.handle, wavelet_id(wavelet), H, W, B,
                     ctypes.c_void_p(pan.data_ptr()), pan.stride(0),
                     ctypes.c_void_p(ms.data_ptr()), ms.stride(1), ms.stride(0),
                     ctypes.c_void_p(gain.data_ptr()) if gain is not None else None,
                     ctypes.c_void_p(out.data_ptr()), out.stride(1), out.stride(0))
        self.fn = self.ctx.lib.dwt_fuse_run
        self.keep = (pan, ms, out, gain)

    def __call__(self):
        st = self.fn(*self.args)
        if st != 0:
            self.ctx.check(st, "dwt_fuse_run")


class PreparedEx:
    """Pre-marshalled dwt_fuse_run_ex call (8-bit / kappa variants)."""

    def __init__(self, api, pan, ms, wavelet, out, kappa=1.0):
        from paper_1803_00737_amd import _lib

        self.ctx = api.context(pan.device)
        self.ctx.bind_stream()
        fmt = lambda t: _lib.U8 if t.dtype == api.torch.uint8 else _lib.F32  # noqa: E731
        self.opts = _lib.Opts(fmt(pan), fmt(out), kappa)
        H, W = pan.shape
        B = ms.shape[0]
        self.args = (self.ctx.handle, _lib.wavelet_id(wavelet), H, W, B,
                     ctypes.c_void_p(pan.data_ptr()), pan.stride(0),
                     ctypes.c_void_p(ms.data_ptr()), ms.stride(1), ms.stride(0), None,
                     ctypes.c_void_p(out.data_ptr()), out.stride(1), out.stride(0), ctypes.byref(self.opts))
        self.fn = self.ctx.lib.dwt_fuse_run_ex
        self.keep = (pan, ms, out)

    def __call__(self):
        st = self.fn(*self.args)
        if st != 0:
            self.ctx.check(st, "dwt_fuse_run_ex")


def u8_bytes(H, W, B):
    """8-bit PAN and MS read once, 8-bit output bands written once."""
    return H * W + B * (H // 2) * (W // 2) + B * H * W


def time_loop(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms per step


def primary_tile(ctx, wl):
    """The launch shape the context holds for the primary workload (the
    tuning table's entry for its key, as the library saves it), or None."""
    import math
    import tempfile

    key = "f%d_h%d_w%d_b%d_" % (1 if wl.wavelet == "d4" else 0, math.ceil(math.log2(wl.H)), math.ceil(math.log2(wl.W)),
                                min(wl.B, 8))
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "table.txt")
        ctx.tune_save(path)
        with open(path) as f:
            for line in f.read().splitlines()[1:]:
                if line.startswith(key):
                    return " ".join(line.split()[1:])
    return None


def read_traffic(tile):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel build with the launch shape this run
    uses (`tile`, from primary_tile; counters are kept for the shapes the
    tuner picks most often)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        from paper_1803_00737_amd.build import build_id

        if t.get("build_id") != build_id() or tile not in t.get("tiles", {}):
            return None
        return float(t["tiles"][tile]["traffic_bytes_per_launch"])
    except Exception:
        return None


def force_primary_tile(ctx, wl, tile):
    """Load a one-entry tuning table that gives the primary workload the
    launch shape `tile` ("seg_rows wpb nc order mode split bg", as the table
    stores it), so a profiler run can take counters for that shape."""
    import math
    import tempfile

    key = "f%d_h%d_w%d_b%d_p0" % (1 if wl.wavelet == "d4" else 0, math.ceil(math.log2(wl.H)),
                                 math.ceil(math.log2(wl.W)), min(wl.B, 8))
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "table.txt")
        ctx.tune_save(path)  # for the header line: the library build id and the device
        with open(path) as f:
            header = f.read().splitlines()[0]
        with open(path, "w") as f:
            f.write(header + "\n" + key + " " + tile + "\n")
        ctx.tune_load(path)


def copy_rate(torch, steps):
    """GB/s of a 1 GiB device-to-device copy with torch's copy kernel, for
    context (a grid-stride copy; one 16-byte element per thread with many
    short-lived workgroups streams faster on this GPU)."""
    n = 1 << 28  # 1 GiB of float32
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    ms = time_loop(torch, lambda: b.copy_(a), steps, 2)
    del a, b
    torch.cuda.empty_cache()
    return 2 * 4 * n / (ms * 1e-3) / 1e9, ms, n


def run_copy(torch, steps):
    gbs, ms, n = copy_rate(torch, steps)
    print(json.dumps({"mode": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n, "ms": ms, "GB/s": gbs}))


def _strip_rows(H, nstrips, rows):
    """nstrips strips of `rows` output rows at evenly spaced even offsets."""
    return [(2 * ((H // 2) * k // nstrips), 2 * ((H // 2) * k // nstrips) + rows) for k in range(nstrips)]


def cpu_baseline(pan, ms, wavelet, budget_s=12.0, max_passes=16):
    """The FP64 oracle as it stands (plain C, one thread) on a bounded sample of
    the primary workload: 8 strips of 248 output rows (1984 of the scene's rows,
    every column and band) at evenly spaced offsets, each computed by the
    oracle's row-strip entry point from the whole scene (the true wrap at the
    image border); whole passes over the sample until about budget_s seconds
    have run; rate = output pixels / time.  pan, ms: float64 host arrays."""
    import oracle

    H, W = pan.shape
    B = ms.shape[0]
    strips = _strip_rows(H, 8, 248)
    px = B * W * sum(b - a for a, b in strips)
    total, passes = 0.0, 0
    while passes < max_passes and (passes == 0 or total < budget_s):
        t0 = time.perf_counter()
        for a, b in strips:
            oracle.fuse_rows(wavelet, pan, ms, a, b)
        total += time.perf_counter() - t0
        passes += 1
    return {"value": passes * px / total / 1e6, "unit": "Mpix/s", "cores": 1, "kind": "oracle",
            "sample": "8 strips of 248 rows (1984 of %d rows, all %d columns and %d bands) of the primary scene, "
                      "row-strip FP64 oracle, 1 thread, %d passes in %.1f s" % (H, W, B, passes, total),
            "host": {"cpu": cpu_model(), "logical_cpus": os.cpu_count()}}


def cpu_oracle_rates(synth, pan, ms, wavelet, torch=None):
    """Further FP64-oracle rates beside the baseline figure (same oracle, as it
    stands, on the host cores): the Haar 512x512 scene (one thread); a
    row-strip sample of the D4 8192x8192 3-band scene (one thread); the
    baseline's sample of the primary scene with the other wavelet (one
    thread); and the baseline's sample on all host cores (at most 16, the host
    share of one GPU): its 8 strips cut into as many row strips as threads,
    each computed by the row-strip oracle (whose C calls release the
    interpreter lock).  pan, ms: the primary scene as float64 host arrays."""
    import concurrent.futures
    import oracle

    def rate(fn, px, budget_s):
        total, passes = 0.0, 0
        while passes == 0 or (total < budget_s and passes < 20):
            t0 = time.perf_counter()
            fn()
            total += time.perf_counter() - t0
            passes += 1
        return px * passes / total / 1e6, passes, total

    out = {}
    wl = synth.haar_512()
    p5, m5 = wl.make()
    r, n, t = rate(lambda: oracle.fuse("haar", p5, m5), wl.B * wl.H * wl.W, 1.0)
    out[wl.name] = {"Mpix/s": r, "threads": 1, "sample": "whole scene, %d passes, %.2f s" % (n, t)}
    # D4 8192 x 8192, 3 bands: the same kind of row-strip sample as the baseline's
    import numpy as np

    wl = synth.d4_8192()
    if torch is not None:  # generated on the GPU (numpy takes about a minute here), timed on the host
        pd, md = wl.make(device="cuda")
        p8, m8 = pd.cpu().numpy().astype(np.float64), md.cpu().numpy().astype(np.float64)
        del pd, md
        torch.cuda.empty_cache()
    else:
        p8, m8 = wl.make()
        p8, m8 = p8.astype(np.float64), m8.astype(np.float64)
    strips8 = _strip_rows(wl.H, 8, 248)
    px8 = wl.B * wl.W * sum(b - a for a, b in strips8)
    r, n, t = rate(lambda: [oracle.fuse_rows(wl.wavelet, p8, m8, a, b) for a, b in strips8], px8, 2.0)
    out[wl.name + "_sample"] = {"Mpix/s": r, "threads": 1,
                                "sample": "8 strips of 248 rows (1984 of %d rows, all columns and %d bands), "
                                          "%d passes, %.2f s" % (wl.H, wl.B, n, t)}
    del p8, m8
    H, W = pan.shape
    B = ms.shape[0]
    strips = _strip_rows(H, 8, 248)
    px = B * W * sum(b - a for a, b in strips)
    other = "haar" if wavelet == "d4" else "d4"
    r, n, t = rate(lambda: [oracle.fuse_rows(other, pan, ms, a, b) for a, b in strips], px, 4.0)
    out["primary_sample_" + other] = {"Mpix/s": r, "threads": 1,
                                      "sample": "the baseline's 8 x 248 rows, %s, %d passes, %.2f s" % (other, n, t)}
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    nt = max(1, min(16, ncpu))
    per = max(1, nt // len(strips))
    pieces = []
    for a, b in strips:
        cuts = [a + 2 * (((b - a) // 2) * k // per) for k in range(per + 1)]
        pieces += [(c0, c1) for c0, c1 in zip(cuts[:-1], cuts[1:]) if c1 > c0]
    with concurrent.futures.ThreadPoolExecutor(max_workers=nt) as ex:
        def all_cores_pass():
            list(ex.map(lambda q: oracle.fuse_rows(wavelet, pan, ms, q[0], q[1]), pieces))
        r, n, t = rate(all_cores_pass, px, 4.0)
    out["primary_sample_all_cores"] = {"Mpix/s": r, "threads": nt,
                                       "sample": "the baseline's 8 x 248 rows in %d row strips, %d passes, %.2f s"
                                                 % (len(pieces), n, t)}
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def launch_stats(torch, fn, n, flush=None):
    """Per-launch kernel times (ms) from an event pair around each launch on
    the current stream.  With `flush` (a device buffer larger than the L2 and
    the Infinity Cache together), the buffer is read before each launch, so
    that no input is left in a cache and no dirty line of the previous launch
    is left to be written back during the timed one (a write would leave its
    own dirty lines behind instead)."""
    s = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    fn()
    for e0, e1 in ev:
        if flush is not None:
            flush.sum()
        e0.record(s)
        fn()
        e1.record(s)
    torch.cuda.synchronize()
    t = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    return {"median_ms": t[len(t) // 2], "min_ms": t[0], "max_ms": t[-1], "launches": n}


def extras(torch, api, synth, steps, warmup, primary_call, only=None):
    """Every workload after the primary one (or those named in `only`)."""
    out = {}

    def want(name):
        return only is None or name in only

    dev = torch.device("cuda:0")
    if want("per_launch"):
        # Primary workload launch by launch: back to back, and with every input
        # and output evicted from the caches before each launch.
        flush = torch.ones(1 << 27, device=dev)  # 512 MiB
        n = max(10, steps // 2)
        out["primary_per_launch"] = {"back_to_back": launch_stats(torch, primary_call, n),
                                     "cache_flushed": launch_stats(torch, primary_call, n, flush)}
        log("primary per launch", out["primary_per_launch"])
        del flush
        torch.cuda.empty_cache()
    if want("d4_8192"):
        # D4 8192 x 8192, 3 bands.
        wl = synth.d4_8192()
        pan, ms = wl.make(device=dev)
        o = torch.empty((wl.B, wl.H, wl.W), device=dev)
        call = Prepared(api, pan, ms, wl.wavelet, o)
        call()  # tunes the launch shape for this size class unless tuning is off
        ms_t = time_loop(torch, call, steps, warmup)
        gbs = algo_bytes(wl.H, wl.W, wl.B) / (ms_t * 1e-3) / 1e9
        out[wl.name] = {"Mpix/s": wl.B * wl.H * wl.W / ms_t / 1e3, "ms": ms_t, "GB/s": gbs, "frac": gbs / HBM_PEAK_GBS,
                        "per_launch": launch_stats(torch, call, max(10, steps // 2))}
        flush = torch.ones(1 << 27, device=dev)  # 512 MiB: inputs evicted before each launch
        out[wl.name]["per_launch_cache_flushed"] = launch_stats(torch, call, max(10, steps // 2), flush)
        del flush
        log(wl.name, out[wl.name])
        del pan, ms, o, call
        torch.cuda.empty_cache()
    if want("haar_512"):
        # Haar 512x512, 1 band: launch-latency bound (fits in cache); Mpix/s only.
        wl = synth.haar_512()
        pan, ms = wl.make(device=dev)
        o = torch.empty((wl.B, wl.H, wl.W), device=dev)
        ms_t = time_loop(torch, Prepared(api, pan, ms, wl.wavelet, o), steps, warmup)
        out[wl.name] = {"Mpix/s": wl.B * wl.H * wl.W / ms_t / 1e3, "ms": ms_t}
        log(wl.name, out[wl.name])
    if want("haar_landsat"):
        # Haar on the Landsat-shaped scene (PAN detail computed once for 6 bands).
        wl = synth.landsat("haar")
        pan, ms = wl.make(device=dev)
        o = torch.empty((wl.B, wl.H, wl.W), device=dev)
        call = Prepared(api, pan, ms, wl.wavelet, o)
        call()
        ms_t = time_loop(torch, call, max(5, steps // 2), warmup)
        gbs = algo_bytes(wl.H, wl.W, wl.B) / (ms_t * 1e-3) / 1e9
        out[wl.name] = {"Mpix/s": wl.B * wl.H * wl.W / ms_t / 1e3, "ms": ms_t, "GB/s": gbs, "frac": gbs / HBM_PEAK_GBS}
        log(wl.name, out[wl.name])
        del pan, ms, o, call
        torch.cuda.empty_cache()
    if want("u8"):
        # 8-bit images in and out (the paper's 8-bit-per-pixel representation):
        # Landsat-shaped scene and the 8192^2 D4 scene.
        for wl in (synth.landsat("haar"), synth.landsat("d4"), synth.d4_8192()):
            pan, ms = wl.make(device=dev)
            p8, m8 = pan.to(torch.uint8), ms.to(torch.uint8)
            del pan, ms
            o8 = torch.empty((wl.B, wl.H, wl.W), dtype=torch.uint8, device=dev)
            call = PreparedEx(api, p8, m8, wl.wavelet, o8)
            call()  # tunes the launch shape for this size class unless tuning is off
            ms_t = time_loop(torch, call, max(5, steps // 2), warmup)
            gbs = u8_bytes(wl.H, wl.W, wl.B) / (ms_t * 1e-3) / 1e9
            out[wl.name + "_u8"] = {"Mpix/s": wl.B * wl.H * wl.W / ms_t / 1e3, "ms": ms_t, "GB/s": gbs,
                                    "frac": gbs / HBM_PEAK_GBS, "bytes_per_output_pixel": u8_bytes(wl.H, wl.W, wl.B) /
                                    (wl.B * wl.H * wl.W)}
            log(wl.name + "_u8", out[wl.name + "_u8"])
            del p8, m8, o8, call
            torch.cuda.empty_cache()
    if want("quality"):
        # DC-matched D4 (kappa = 2) and the quality diagnostics against the
        # scene's synthetic full-resolution truth, on the 8192^2 D4 scene.
        wl = synth.d4_8192()
        pan, ms = wl.make(device=dev)
        truth = wl.truth(pan)
        o = torch.empty((wl.B, wl.H, wl.W), device=dev)
        qual = {}
        for name, w, kappa in (("d4_kappa1", "d4", 1.0), ("d4_kappa2", "d4", 2.0), ("haar", "haar", 1.0)):
            api.fuse(pan, ms, w, out=o, kappa=kappa)
            q = api.quality(o, truth)
            qual[name] = {"rmse": q["rmse"], "ergas": q["ergas"]}
        call = PreparedEx(api, pan, ms, "d4", o, kappa=2.0)
        t_k2 = time_loop(torch, call, steps, warmup)
        t_q = time_loop(torch, lambda: api.quality(o, truth), max(3, steps // 10), 1)
        qual["fused_kappa2_ms"] = t_k2
        qual["fused_kappa2_Mpix/s"] = wl.B * wl.H * wl.W / t_k2 / 1e3
        qual["fused_kappa2_frac"] = algo_bytes(wl.H, wl.W, wl.B) / (t_k2 * 1e-3) / 1e9 / HBM_PEAK_GBS
        qual["quality_call_ms"] = t_q
        out["dc_matched_quality_" + wl.name] = qual
        log("dc matched / quality", qual)
        del pan, ms, truth, o, call
        torch.cuda.empty_cache()
    if want("batched"):
        # Batched: 96 uneven scenes, mixed wavelets, one persistent launch vs 96 launches.
        layout = synth.uneven_batch()
        scenes, preps = [], []
        px = 0
        nbytes = 0
        for sc in layout:
            pan, ms = synth.make_scene(sc.H, sc.W, sc.B, sc.seed, device=dev)
            o = torch.empty((sc.B, sc.H, sc.W), device=dev)
            scenes.append(dict(pan=pan, ms=ms, wavelet=sc.wavelet, out=o))
            preps.append(Prepared(api, pan, ms, sc.wavelet, o))
            px += sc.B * sc.H * sc.W
            nbytes += algo_bytes(sc.H, sc.W, sc.B)
        arr, _, keep = api.make_items(scenes)
        ctx = api.context(dev)
        ctx.bind_stream()
        lib = ctx.lib

        def per_image():
            for p in preps:
                p()

        def batched(flags):
            def f():
                st = lib.dwt_fuse_run_batched(ctx.handle, arr, len(scenes), flags)
                if st != 0:
                    ctx.check(st, "dwt_fuse_run_batched")
            return f

        bsteps = max(5, steps // 2)
        t_per = time_loop(torch, per_image, bsteps, warmup)
        t_bat = time_loop(torch, batched(0), bsteps, warmup)
        t_gra = time_loop(torch, batched(1), bsteps, warmup)
        out["uneven_96_batched"] = {
            "scenes": len(layout), "output_Mpix": px / 1e6,
            "per_image_ms": t_per, "batched_ms": t_bat, "batched_graph_ms": t_gra,
            "per_image_Mpix/s": px / t_per / 1e3, "batched_graph_Mpix/s": px / t_gra / 1e3,
            "batched_graph_GB/s": nbytes / (t_gra * 1e-3) / 1e9,
            "speedup_graph_vs_per_image": t_per / t_gra,
        }
        log("uneven_96", out["uneven_96_batched"])
        del scenes, preps, arr, keep
        torch.cuda.empty_cache()
    if want("multipass"):
        # The paper's own multi-pass pipeline (section 3) on the primary workload, as a comparator.
        wl = synth.d4_8192()
        pan, ms = wl.make(device=dev)
        o = torch.empty((wl.B, wl.H, wl.W), device=dev)
        t_mp = time_loop(torch, lambda: api.fuse_multipass(pan, ms, wl.wavelet, out=o), max(3, steps // 10), 1)
        t_fu = time_loop(torch, Prepared(api, pan, ms, wl.wavelet, o), steps, warmup)
        out["paper_multipass_" + wl.name] = {"multipass_ms": t_mp, "fused_ms": t_fu, "fused_speedup": t_mp / t_fu,
                                             "multipass_Mpix/s": wl.B * wl.H * wl.W / t_mp / 1e3}
        log("multipass", out["paper_multipass_" + wl.name])
        del pan, ms, o
        torch.cuda.empty_cache()
    if want("adjoint"):
        # Adjoint alone at the primary shape (D4 8192^2, 3 bands): gradients
        # w.r.t. PAN, MS and the 3 gains from one upstream gradient, one
        # pre-marshalled dwt_fuse_backward call per step; algorithmic bytes
        # H*W*(8 + 5B) (PAN and B upstream gradients read, grad_pan and B
        # quarter-size grad_ms written).
        wl = synth.d4_8192()
        pan, _ = wl.make(device=dev)
        H, W, B = wl.H, wl.W, wl.B
        gy = torch.randn((B, H, W), device=dev, generator=torch.Generator(device=dev).manual_seed(3))
        gain = torch.ones(B, device=dev)
        gp = torch.empty((H, W), device=dev)
        gm = torch.empty((B, H // 2, W // 2), device=dev)
        gg = torch.empty(B, device=dev)
        actx = api.context(dev)
        actx.bind_stream()
        alib = actx.lib
        bargs = (actx.handle, 1, H, W, B, ctypes.c_void_p(pan.data_ptr()), W, ctypes.c_void_p(gain.data_ptr()),
                 ctypes.c_void_p(gy.data_ptr()), W, H * W, ctypes.c_void_p(gp.data_ptr()),
                 ctypes.c_void_p(gm.data_ptr()), ctypes.c_void_p(gg.data_ptr()))
        ms_t = time_loop(torch, lambda: actx.check(alib.dwt_fuse_backward(*bargs), "dwt_fuse_backward"),
                         max(5, steps // 2), warmup)
        gbs = H * W * (8 + 5 * B) / (ms_t * 1e-3) / 1e9
        out["adjoint_d4_8192x8192_b3"] = {"ms": ms_t, "GB/s": gbs, "frac": gbs / HBM_PEAK_GBS}
        log("adjoint_d4_8192x8192_b3", out["adjoint_d4_8192x8192_b3"])
        del pan, gy, gp, gm, gg, bargs
        torch.cuda.empty_cache()

    if want("differentiation"):
        # Differentiation: 16 x 2048^2, 4 bands, D4: fused forward + adjoint
        # (gradients w.r.t. PAN, MS and the 4 gains) of every scene, as
        # pre-marshalled C-ABI calls (the Python autograd wrapper adds host time).
        # Two ways: one batched forward call and one batched adjoint call over the
        # 16 scenes; and per-scene calls issued round-robin on 4 streams, one
        # library context each, so one scene's kernels fill the ramp-up and tail
        # of another's (a 2048^2 launch is short).
        H = W = 2048
        B = 4
        NS = 4
        gain = torch.ones(B, device=dev)
        fwd_sc, bwd_sc = [], []
        for s in range(16):
            pan, ms = synth.make_scene(H, W, B, synth.seed_for(4, s), device=dev)
            gy = torch.randn((B, H, W), device=dev) * 1e-3
            o = torch.empty((B, H, W), device=dev)
            fwd_sc.append(dict(pan=pan, ms=ms, wavelet="d4", gain=gain, out=o))
            bwd_sc.append(dict(pan=pan, grad_out=gy, wavelet="d4", gain=gain))
        farr, _, fkeep = api.make_items(fwd_sc)
        barr, bouts, bkeep = api.make_bwd_items(bwd_sc)
        ctx = api.context(dev)
        ctx.bind_stream()
        lib = ctx.lib

        def fwd_bwd_batched():
            ctx.check(lib.dwt_fuse_run_batched(ctx.handle, farr, 16, 0), "dwt_fuse_run_batched")
            ctx.check(lib.dwt_fuse_backward_batched(ctx.handle, barr, 16), "dwt_fuse_backward_batched")

        streams = [torch.cuda.Stream() for _ in range(NS)]
        sctx = [api.Context(dev.index if dev.index is not None else 0) for _ in range(NS)]
        for c, st in zip(sctx, streams):
            c.bind_stream(st)
        calls = []
        for s, (f, b, (gp, gm, gg)) in enumerate(zip(fwd_sc, bwd_sc, bouts)):
            c = sctx[s % NS]
            fargs = (c.handle, 1, H, W, B, ctypes.c_void_p(f["pan"].data_ptr()), W, ctypes.c_void_p(f["ms"].data_ptr()),
                     W // 2, (H // 2) * (W // 2), ctypes.c_void_p(gain.data_ptr()), ctypes.c_void_p(f["out"].data_ptr()),
                     W, H * W)
            bargs = (c.handle, 1, H, W, B, ctypes.c_void_p(b["pan"].data_ptr()), W, ctypes.c_void_p(gain.data_ptr()),
                     ctypes.c_void_p(b["grad_out"].data_ptr()), W, H * W, ctypes.c_void_p(gp.data_ptr()),
                     ctypes.c_void_p(gm.data_ptr()), ctypes.c_void_p(gg.data_ptr()))
            calls.append(lambda a=fargs, c=c: c.check(lib.dwt_fuse_run(*a), "dwt_fuse_run"))
            calls.append(lambda a=bargs, c=c: c.check(lib.dwt_fuse_backward(*a), "dwt_fuse_backward"))

        def fwd_bwd_streams():
            cur = torch.cuda.current_stream()
            for st in streams:
                st.wait_stream(cur)
            for c in calls:
                c()
            for st in streams:
                cur.wait_stream(st)

        n = max(5, steps // 5)
        t_b = time_loop(torch, fwd_bwd_batched, n, 2)
        t_s = time_loop(torch, fwd_bwd_streams, n, 2)
        fb_bytes = 16 * (algo_bytes(H, W, B) + H * W * (8 + 5 * B))
        out["differentiation_16x2048_b4"] = {"fwd_bwd_ms": t_b, "scenes/s": 16 / (t_b * 1e-3),
                                             "GB/s": fb_bytes / (t_b * 1e-3) / 1e9,
                                             "frac": fb_bytes / (t_b * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                             "how": "one batched forward call + one batched adjoint call",
                                             "per_scene_calls_on_%d_streams_ms" % NS: t_s}
        log("differentiation", out["differentiation_16x2048_b4"])
        torch.cuda.synchronize()
        del calls, sctx, fkeep, bkeep, bouts, farr, barr, fwd_sc, bwd_sc
        torch.cuda.empty_cache()
    return out


def device_info(torch):
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", None), "compute_units": p.multi_processor_count,
            "hbm_GiB": round(p.total_memory / 2**30, 1), "hip": torch.version.hip}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", choices=["full", "primary", "copy"], default="full")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default=None,
                    help="comma-separated subset of the extra workloads (per_launch, d4_8192, haar_512, "
                         "haar_landsat, u8, quality, batched, multipass, adjoint, differentiation)")
    ap.add_argument("--no-tune", action="store_true", help="use the default tile instead of the autotuner")
    ap.add_argument("--tile", default=None,
                    help='primary workload only: its launch shape, "seg_rows wpb nc order mode split bg" '
                         "(as in a tuning table), instead of tuning")
    ap.add_argument("--tune-cache", default=None,
                    help="tuning table file: loaded if it exists (no tuning), else written after tuning "
                         "(after the primary workload, and again at the end with every workload's shapes)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.mode == "copy":
        run_copy(torch, args.steps)
        return

    from paper_1803_00737_amd import api, synth

    dev = torch.device("cuda:0")
    wl = synth.landsat("d4")
    log("generating", wl.name)
    pan, ms = wl.make(device=dev)
    out = torch.empty((wl.B, wl.H, wl.W), device=dev)
    ctx = api.context(dev)
    loaded = False
    if args.tile:
        force_primary_tile(ctx, wl, args.tile)
        loaded = True
        log("primary launch shape forced:", args.tile)
    elif args.tune_cache and os.path.exists(args.tune_cache):
        ctx.tune_load(args.tune_cache)
        loaded = True
        log("tuning table loaded from", args.tune_cache)
    elif not args.no_tune:
        ctx.set_tuning(True)
    torch.cuda.synchronize()
    call = Prepared(api, pan, ms, wl.wavelet, out)
    call()  # first call tunes the launch shape for this size class
    torch.cuda.synchronize()
    if args.tune_cache and not loaded and not args.no_tune:
        ctx.tune_save(args.tune_cache)
    ms_step = time_loop(torch, call, args.steps, args.warmup)
    tile = primary_tile(ctx, wl)
    nbytes = algo_bytes(wl.H, wl.W, wl.B)
    achieved = nbytes / (ms_step * 1e-3) / 1e9
    value = wl.B * wl.H * wl.W / ms_step / 1e3
    log("primary %.4f ms/step  %.0f Mpix/s  %.0f GB/s" % (ms_step, value, achieved))
    result = {
        "metric": "fused output Mpix/s (all bands) + % HBM peak, batched vs per-image, 1 GPU",
        "value": value,
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded blob/rectangle/noise scenes, uint8-valued float32)",
        "config": {"workload": wl.name, "wavelet": "d4", "H": wl.H, "W": wl.W, "bands": wl.B,
                   "parallelism": "single GPU",
                   "stands_in_for": "the paper's largest Landsat-7 PAN scene, 16280 x 14960 (section 4, Table 1)"},
        "device": device_info(torch),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": read_traffic(tile),
                     "launch_shape": tile,
                     "algorithmic_bytes_per_launch": nbytes,
                     "torch_copy_1GiB_GB/s": copy_rate(torch, 20)[0]},
        "paper_context": PAPER_CONTEXT,
    }
    if args.mode == "full":
        only = set(args.only.split(",")) if args.only else None
        result["workloads"] = extras(torch, api, synth, args.steps, args.warmup, call, only)
        if args.tune_cache and not loaded and not args.no_tune:
            ctx.tune_save(args.tune_cache)  # now with the shapes of every workload
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        import numpy as np

        pan_h = pan.cpu().numpy().astype(np.float64)
        ms_h = ms.cpu().numpy().astype(np.float64)
        del pan, ms, out, call
        torch.cuda.empty_cache()
        result["cpu_baseline"] = cpu_baseline(pan_h, ms_h, wl.wavelet)
        log("cpu baseline", result["cpu_baseline"])
        if args.mode == "full":
            result["cpu_oracle_rates"] = cpu_oracle_rates(synth, pan_h, ms_h, wl.wavelet, torch)
            log("cpu oracle rates", result["cpu_oracle_rates"])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
