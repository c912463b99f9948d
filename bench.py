#!/usr/bin/env python3
"""Throughput of the VCA hot path on one MI355X: 2160p frames/s for all seven
features, full w = 32 DCT and low-pass K = 16, with the forward kernel's
roofline position and the CPU oracle timed beside it.

A step is one pass of the whole path over one batch: vca_analyze_frames on the
600 device-resident frames of the synthetic 2160p 8-bit 4:2:0 workload
(5 scenes of 120 frames, hard cuts, texture sigma 0..60, global motion up to
16 px/frame) followed by vca_features for those 600 frames.

Prints one JSON line.  ``--gpus`` above 1 is refused: the path runs on one GPU.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "2160p frames/s, all 7 features (full vs low-pass DCT); % of int8-MFMA/HBM peak"
WIDTH, HEIGHT, FRAMES = 3840, 2160, 600
BLOCK = 32
MAX_BATCH = 600                 # one forward launch per step
HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
INT8_PEAK_TOPS = 5000.0         # MI355X dense int8 MFMA
FP16_PEAK_TFLOPS = 2500.0       # MI355X dense fp16 MFMA


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def frame_bytes(width: int, height: int, bit_depth: int = 8) -> int:
    """Algorithmic bytes of one 4:2:0 frame: every sample of Y, U and V once
    (3840x2160 8-bit: 12,441,600 B; 10-bit, uint16 samples: 24,883,200 B)."""
    return (width * height + 2 * (width // 2) * (height // 2)) * (1 if bit_depth == 8 else 2)


def block_count(width: int, height: int, w: int) -> int:
    return (width // w) * (height // w) + 2 * ((width // 2) // w) * ((height // 2) // w)


def int8_ops_per_frame(width: int, height: int, w: int, k: int = 0) -> int:
    """Algorithmic int8 ops (2 per multiply-add) of the two transform passes
    per frame: per block the horizontal pass w x K x w and the vertical pass
    K x K x w multiply-adds (3840x2160, w = 32: 1.573 G full, 0.590 G K = 16)."""
    K = k or w
    return block_count(width, height, w) * 2 * (w * K * w + K * K * w)


def mfma_issued_ops_per_frame(width: int, height: int, w: int, k: int = 0, bit_depth: int = 8) -> int:
    """int8 ops the forward kernel issues on MFMA per frame.  A unit of
    w / K sample tiles of 32 x 32 (one tile for the full transform) takes one
    32x32x32 horizontal-pass product per sample tile (two for 10-bit) and two
    vertical-pass products (hi and lo) shared by the unit."""
    pack = w // (k or w)
    tiles = block_count(width, height, w) * (w * w) / (32 * 32)
    per_tile = (1 if bit_depth == 8 else 2) + 2 / pack
    return int(tiles * per_tile * 2 * 32 * 32 * 32)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(sv, frames: int) -> dict:
    """The CPU oracle (plain C, int64 transform, FP64 features, OpenMP over
    frames) timed on this host: the 10 frames of the 720p patches workload in
    full, and the first `frames` frames of the 600-frame 2160p workload at
    full DCT and K = 16, each on every core this process may use and on one
    thread.  A reported baseline, not a target."""
    import oracle
    import synth
    cores = len(os.sched_getaffinity(0))
    video = sv.frames(0, frames)
    small = synth.patches_video()

    def timed(cfg, v, threads):
        t0 = time.perf_counter()
        oracle.analyze(cfg, v.y, v.u, v.v, threads=threads)
        return time.perf_counter() - t0

    full = oracle.Config(WIDTH, HEIGHT, 8, BLOCK, 0)
    k16 = oracle.Config(WIDTH, HEIGHT, 8, BLOCK, 16)
    c720 = oracle.Config(small.width, small.height, 8, BLOCK, 0)
    t_all = timed(full, video, cores)
    t_k16_all = timed(k16, video, cores)
    t_one = timed(full, video, 1)
    t_k16_one = timed(k16, video, 1)
    t720_all = timed(c720, small, cores)
    t720_one = timed(c720, small, 1)
    n720 = small.n_frames
    return {"value": frames / t_all, "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": f"first {frames} frames of the 600-frame 3840x2160 8-bit workload, w=32, "
                      f"full DCT, {cores} OpenMP threads (every core of this process's affinity), "
                      f"{t_all:.1f} s wall",
            "cpu": cpu_model(),
            "full_single_thread": frames / t_one,
            "lowpass_k16_all_cores": frames / t_k16_all,
            "lowpass_k16_single_thread": frames / t_k16_one,
            "patches_720p_all_cores": n720 / t720_all,
            "patches_720p_single_thread": n720 / t720_one,
            "detail": f"2160p: full {t_all:.2f} s ({cores} threads) / {t_one:.2f} s (1 thread), "
                      f"K=16 {t_k16_all:.2f} s / {t_k16_one:.2f} s for {frames} frames; "
                      f"720p patches workload ({n720} frames, full DCT) {t720_all:.3f} s / "
                      f"{t720_one:.3f} s"}


def run_mode(vca, dev, lowpass_k: int, steps: int, warmup: int, tune: bool,
             downsample: bool = False, block_size: int = BLOCK) -> dict:
    import torch
    an = vca.Analyzer(WIDTH, HEIGHT, block_size=block_size, lowpass_k=lowpass_k, timing=True,
                      max_batch=MAX_BATCH, downsample=downsample)
    planes = dev.planes()
    launch = an.tune(*planes, reps=2) if tune else an.tuned_launch()
    for _ in range(warmup):
        first = an.submit(*planes)
        an.features(first, FRAMES)
    an.timing(reset=True)
    torch.cuda.synchronize()
    step_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        first = an.submit(*planes)
        feats = an.features(first, FRAMES)   # waits for the step's launches
        step_ms.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tm = an.timing(reset=True)
    an.close()
    rec = launch_record(tm, steps * FRAMES / dt, dt * 1e3 / steps, WIDTH, HEIGHT, block_size,
                        lowpass_k, 8, downsample, launch, feats)
    rec["ms_per_step_median"] = statistics.median(step_ms)
    rec["fps_median"] = FRAMES / rec["ms_per_step_median"] * 1e3
    return rec


def launch_record(tm: dict, fps: float, ms_per_step: float, width: int, height: int, w: int,
                  k: int, bit_depth: int, downsample: bool, launch: dict, feats) -> dict:
    """Rates of the forward kernel from the library's HIP-event times: HBM
    against the frame's algorithmic bytes (every sample once), int8 matrix
    cores against the transform's algorithmic ops and against the ops issued
    (hi/lo split included)."""
    fwd_ms = tm["forward_ms"] / max(1, tm["forward_launches"])
    red_ms = tm["reduce_ms"] / max(1, tm["reduce_launches"])
    frames_per_launch = tm["frames"] / max(1, tm["forward_launches"])
    alg_bytes = frame_bytes(width, height, bit_depth) * frames_per_launch
    gbs = alg_bytes / (fwd_ms * 1e-3) / 1e9
    aw, ah = (width // 2, height // 2) if downsample else (width, height)
    alg_tops = int8_ops_per_frame(aw, ah, w, k) * frames_per_launch / (fwd_ms * 1e-3) / 1e12
    iss_tops = (mfma_issued_ops_per_frame(aw, ah, w, k, bit_depth) * frames_per_launch
                / (fwd_ms * 1e-3) / 1e12)
    return {
        "fps": fps,
        "ms_per_step": ms_per_step,
        "forward_kernel_ms": fwd_ms,
        "reduce_kernel_ms": red_ms,
        "frames_per_launch": frames_per_launch,
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None},
        "mfma": {"achieved": alg_tops, "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                 "frac": alg_tops / INT8_PEAK_TOPS, "ops": "algorithmic (transform multiply-adds x 2)",
                 "issued_achieved": iss_tops, "issued_frac": iss_tops / INT8_PEAK_TOPS},
        "last_features": [float(x) for x in feats[-1]],
        "launch": launch,
    }


TENBIT_FRAMES = 300


def run_tenbit(vca, steps: int, warmup: int, tune: bool) -> dict:
    """The 10-bit precision-stress workload: 300 frames of 3840x2160 and of
    1920x1080 10-bit 4:2:0 (uint16 samples), w = 32 and 16, full DCT, one
    launch per step.  Three stress frames (full-range noise, saturated edges
    and sign-matched worst-case blocks) repeat on the device as frames t % 3."""
    import numpy as np
    import torch
    import synth
    out = {}
    for width, height in ((3840, 2160), (1920, 1080)):
        for w in (32, 16):
            base = synth.stress_video(width, height, 3, cell=w, stream=300 + w)
            idx = torch.arange(TENBIT_FRAMES, device="cuda") % 3
            planes = [torch.from_numpy(p.view(np.int16)).cuda()[idx].contiguous()
                      for p in (base.y, base.u, base.v)]
            an = vca.Analyzer(width, height, bit_depth=10, block_size=w, timing=True,
                              max_batch=TENBIT_FRAMES)
            launch = an.tune(*planes, reps=2) if tune else an.tuned_launch()
            for _ in range(warmup):
                an.features(an.submit(*planes), TENBIT_FRAMES)
            an.timing(reset=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                feats = an.features(an.submit(*planes), TENBIT_FRAMES)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rec = launch_record(an.timing(reset=True), steps * TENBIT_FRAMES / dt, dt * 1e3 / steps,
                                width, height, w, 0, 10, False, launch, feats)
            an.close()
            del planes
            torch.cuda.empty_cache()
            rec.pop("last_features")
            rec["frame_bytes"] = frame_bytes(width, height, 10)
            out[f"{width}x{height}_w{w}"] = rec
            log(f"10-bit {width}x{height} w={w}: {rec['fps']:.0f} frames/s, forward "
                f"{rec['forward_kernel_ms']:.3f} ms, HBM {rec['roofline']['frac']:.3f}")
    return out


def plane_bytes(d: dict) -> int:
    """Algorithmic bytes of one frame of a stream (8-bit)."""
    return frame_bytes(d["width"], d["height"])


def small_streams(n: int = 256, frames: int = 8) -> list:
    """Many small live streams: n streams of 640x360 8-bit 4:2:0, `frames`
    frames each per step, block size 8, 16, 32 in turn."""
    return [dict(width=640, height=360, block_size=(8, 16, 32)[s % 3], n_frames=frames, stream=s + 1)
            for s in range(n)]


def run_batch(vca, steps: int, warmup: int, tune: bool, descs: list, workload: str) -> dict:
    """The streams `descs` in one graph-replayed round per step (one persistent
    launch per class of streams, each followed by its reduction; per_class
    gives each class's tuned forward time alone, arrangement whether the
    classes ran one after another or side by side),
    against the same streams analysed one after another by plain contexts
    (each on its own stream).  Both sides submit descriptors prepared once
    for the fixed frame buffers; the batch reads every stream's features
    with one call, the plain contexts with one call each."""
    import torch
    from synth.device import generated_scene_video
    log(f"generating {len(descs)} streams, {sum(d['n_frames'] for d in descs)} frames on the device")
    vids = [generated_scene_video(d["width"], d["height"], d["n_frames"], seed=3000 + d["stream"])
            for d in descs]
    torch.cuda.synchronize()
    frames = [v.planes() for v in vids]
    total_frames = sum(d["n_frames"] for d in descs)
    total_bytes = sum(plane_bytes(d) * d["n_frames"] for d in descs)
    cfg = [dict(width=d["width"], height=d["height"], block_size=d["block_size"],
                max_batch=d["n_frames"]) for d in descs]
    b = vca.Batch(cfg, timing=True)
    launch = b.tune(frames, reps=1) if tune else b.tuned_launch()
    per_class = b.class_times()
    arrangement = b.arrangement()
    prepared = b.prepare(frames)
    for _ in range(warmup):
        b.submit(prepared)
    b.timing(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        first = b.submit(prepared)
        b.features_many([(s, first[s], d["n_frames"]) for s, d in enumerate(descs)])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tm = b.timing(reset=True)
    b.close()
    # the same streams through plain contexts, one after another
    ans = [vca.Analyzer(d["width"], d["height"], block_size=d["block_size"], max_batch=d["n_frames"])
           for d in descs]
    preps = [an.prepare(*fr) for an, fr in zip(ans, frames)]
    for an, pf in zip(ans, preps):
        an.submit(pf)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        for an, pf in zip(ans, preps):
            an.submit(pf)
        for an, d in zip(ans, descs):
            an.features(an.submitted - d["n_frames"], d["n_frames"])
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t1
    for an in ans:
        an.close()
    dev_ms = tm["ms"] / max(1, tm["launches"])
    gbs = total_bytes / (dev_ms * 1e-3) / 1e9
    return {
        "workload": workload,
        "streams": len(descs), "frames_per_step": total_frames,
        "bytes_per_step": total_bytes,
        "value": steps * total_frames / dt, "unit": "frames/s",
        "ms_per_step": dt * 1e3 / steps,
        "device_ms_per_step": dev_ms,
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None},
        "plain_same_streams": {"value": steps * total_frames / dt_plain, "unit": "frames/s",
                               "ms_per_step": dt_plain * 1e3 / steps},
        "speedup_vs_plain": dt_plain / dt,
        "launch": launch,
        "per_class": per_class,
        "arrangement": arrangement,
    }


def run_latency(vca, dev, reps: int = 200) -> dict:
    """Frames arriving one at a time (a live stream): one device-resident
    2160p frame submitted and its features read back, full DCT, repeated;
    the median and 99th percentile of the host's wall time per frame."""
    import torch
    an = vca.Analyzer(WIDTH, HEIGHT, block_size=BLOCK, max_batch=1)
    y, u, v = dev.planes()
    frames = [an.prepare(y[i:i + 1], u[i:i + 1], v[i:i + 1]) for i in range(16)]
    for i in range(20):
        an.features(an.submit(frames[i % 16]), 1)
    torch.cuda.synchronize()
    ts = []
    for i in range(reps):
        t0 = time.perf_counter()
        an.features(an.submit(frames[i % 16]), 1)
        ts.append(time.perf_counter() - t0)
    an.close()
    ts.sort()
    return {"median_us": ts[len(ts) // 2] * 1e6, "p99_us": ts[int(len(ts) * 0.99) - 1] * 1e6,
            "frames": reps, "unit": "us per frame",
            "workload": "one 3840x2160 8-bit 4:2:0 frame per call, resident in HBM, w=32 full DCT, "
                        "vca_analyze_frames + vca_features"}


INGEST_FRAMES = 120   # host-resident frames per ingest step


def run_ingest(vca, dev, steps: int) -> dict:
    """End-to-end rate with the frames in host memory: the first 120 frames of
    the 2160p workload as pageable numpy planes through vca_analyze_frames
    (staged via pinned buffers, host-to-device copies overlapped with the
    analysis), and the same frames as a raw .yuv file in /tmp through
    vca_analyze_yuv_file (page cache warm).  PCIe-inclusive; never the
    headline value."""
    import os
    import tempfile
    import torch
    y, u, v = (p[:INGEST_FRAMES].cpu().numpy() for p in dev.planes())
    nbytes = y.nbytes + u.nbytes + v.nbytes
    an = vca.Analyzer(WIDTH, HEIGHT, block_size=BLOCK, max_batch=MAX_BATCH)
    an.features(an.submit_host(y, u, v), INGEST_FRAMES)            # warm-up (allocates staging)
    t0 = time.perf_counter()
    for _ in range(steps):
        first = an.submit_host(y, u, v)
        an.features(first, INGEST_FRAMES)
    dt_host = (time.perf_counter() - t0) / steps
    fd, path = tempfile.mkstemp(suffix=".yuv", dir="/tmp")
    os.close(fd)
    try:
        vca.write_yuv(path, y, u, v)
        an.features(an.submit_file(path), INGEST_FRAMES)            # warm the page cache
        t0 = time.perf_counter()
        for _ in range(steps):
            first = an.submit_file(path)
            an.features(first, INGEST_FRAMES)
        dt_file = (time.perf_counter() - t0) / steps
    finally:
        os.unlink(path)
    an.close()
    torch.cuda.synchronize()
    return {"value": INGEST_FRAMES / dt_host, "unit": "frames/s",
            "GBps": nbytes / dt_host / 1e9, "ms_per_step": dt_host * 1e3,
            "file_value": INGEST_FRAMES / dt_file, "file_GBps": nbytes / dt_file / 1e9,
            "frames_per_step": INGEST_FRAMES,
            "workload": f"{INGEST_FRAMES} frames 3840x2160 8-bit 4:2:0 in pageable host memory, "
                        "and as a raw .yuv file (page cache warm), w=32 full DCT",
            "what": "host-to-device inclusive: pinned double-buffered staging, copies on a "
                    "second stream overlapped with the analysis"}


def run_backward(vca, steps: int, warmup: int) -> dict:
    """Differentiable E_Y and h of 16 pairs of 1920x1080 8-bit-valued luma
    frames cast to float32, w = 32: one step is the forward and the backward
    through the autograd Function (dL/dx for given dL/dE, dL/dh).  Kernel
    times come from HIP events around the two C-ABI calls on the stream they
    are launched on; the plain integer path on the same frames (all seven
    features from Y, U and V) is timed beside it."""
    import ctypes
    import torch
    from paper_2304_12384_amd import _lib, grad
    from synth.device import generated_scene_video
    n_seq, seq_len, H, W, w = 16, 2, 1080, 1920, 32
    n = n_seq * seq_len
    dv = generated_scene_video(W, H, n, seed=4, scene_len=seq_len)
    x = dv.y.float().reshape(n_seq, seq_len, H, W).contiguous().requires_grad_(True)
    g = torch.Generator(device="cuda")
    g.manual_seed(12384)
    gE = torch.randn(n_seq, seq_len, device="cuda", generator=g)
    gh = torch.randn(n_seq, seq_len, device="cuda", generator=g)

    def step():
        E, h = vca.energy_features(x, block_size=w)
        return torch.autograd.grad((E, h), (x,), (gE, gh))[0]

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        gx = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    # the two C-ABI calls alone, preallocated buffers, events on their stream
    L = _lib.lib()
    xd = x.detach()
    cfg = grad._config(xd, w, 0, 8)
    ws = torch.empty(L.vca_grad_workspace(ctypes.byref(cfg)), device="cuda", dtype=torch.uint8)
    E = torch.empty(n, device="cuda")
    h = torch.empty(n, device="cuda")
    gxb = torch.empty_like(xd)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd_ms = bwd_ms = 0.0
    reps = max(steps, 5)
    for i in range(reps + 1):
        ev[0].record(stream)
        _lib.check(L.vca_energy_forward(ctypes.byref(cfg), xd.data_ptr(), E.data_ptr(), h.data_ptr(),
                                        ws.data_ptr(), stream.cuda_stream), "vca_energy_forward")
        ev[1].record(stream)
        _lib.check(L.vca_energy_backward(ctypes.byref(cfg), ws.data_ptr(), gE.data_ptr(),
                                         gh.data_ptr(), gxb.data_ptr(), stream.cuda_stream),
                   "vca_energy_backward")
        ev[2].record(stream)
        ev[2].synchronize()
        if i > 0:                       # the first pass builds the operand tables
            fwd_ms += ev[0].elapsed_time(ev[1]) / reps
            bwd_ms += ev[1].elapsed_time(ev[2]) / reps
    assert torch.equal(gxb, gx), "C-ABI backward differs from the autograd path"
    # the forward call alone, back to back: its reads then find no dirty
    # gradient lines of a preceding backward call waiting to be written back
    fwd_alone_ms = 0.0
    for i in range(reps + 1):
        ev[0].record(stream)
        _lib.check(L.vca_energy_forward(ctypes.byref(cfg), xd.data_ptr(), E.data_ptr(), h.data_ptr(),
                                        ws.data_ptr(), stream.cuda_stream), "vca_energy_forward")
        ev[1].record(stream)
        ev[1].synchronize()
        if i > 0:
            fwd_alone_ms += ev[0].elapsed_time(ev[1]) / reps

    an = vca.Analyzer(W, H, block_size=w, max_batch=n)
    for _ in range(warmup):
        an.features(an.submit(dv.y, dv.u, dv.v), n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        an.features(an.submit(dv.y, dv.u, dv.v), n)
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t0
    an.close()

    tiles = (W // w) * (H // w) * n                # w = 32: one 32 x 32 tile per block
    bytes_fwd = tiles * (w * w * 4 + 256)          # samples read, coefficient signs written
    bytes_bwd = tiles * (256 + w * w * 4)          # signs read, dL/dx written
    # fp16 matrix-core work as issued: forward 6 (integer-valued samples: one
    # digit, 2 horizontal + 4 vertical products), backward 10 products of
    # 32x32x16 per tile
    f16_fwd = tiles * 6 * 2 * 32 * 32 * 16
    f16_bwd = tiles * 10 * 2 * 32 * 32 * 16
    bw_gbs = bytes_bwd / (bwd_ms * 1e-3) / 1e9
    fw_gbs = bytes_fwd / (fwd_ms * 1e-3) / 1e9
    fa_gbs = bytes_fwd / (fwd_alone_ms * 1e-3) / 1e9
    pair_gbs = (bytes_fwd + bytes_bwd) / ((fwd_ms + bwd_ms) * 1e-3) / 1e9
    return {
        "value": steps * n / dt, "unit": "frames/s",
        "workload": f"{n_seq} pairs of {W}x{H} float32 luma (8-bit values), w={w}, "
                    "forward + backward of E_Y and h",
        "ms_per_step": dt * 1e3 / steps,
        "forward_kernel_ms": fwd_ms, "backward_kernel_ms": bwd_ms,
        "roofline": {"bound": "hbm", "achieved": bw_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": bw_gbs / HBM_PEAK_GBS, "traffic": None},
        "backward_mfma_f16": {"achieved": f16_bwd / (bwd_ms * 1e-3) / 1e12, "peak": FP16_PEAK_TFLOPS,
                              "unit": "TFLOP/s"},
        "forward_hbm": {"achieved": fw_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": fw_gbs / HBM_PEAK_GBS},
        "forward_alone": {"ms": fwd_alone_ms, "achieved": fa_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": fa_gbs / HBM_PEAK_GBS,
                          "what": "forward calls back to back, no backward call between them"},
        "pair_hbm": {"achieved": pair_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": pair_gbs / HBM_PEAK_GBS, "bytes": bytes_fwd + bytes_bwd,
                     "what": "forward + backward call: both calls' algorithmic bytes over both kernels' time"},
        "forward_mfma_f16": {"achieved": f16_fwd / (fwd_ms * 1e-3) / 1e12, "peak": FP16_PEAK_TFLOPS,
                             "unit": "TFLOP/s"},
        "plain_same_frames": {"value": steps * n / dt_plain, "unit": "frames/s",
                              "what": "integer path, all 7 features of the same frames (YUV)"},
        "ratio_vs_plain": dt_plain / dt,
    }


KERNEL_SOURCES = ("vca.hip", "vca_strip.h", "vca_tile.h", "vca_host.h", "vca_reduce.h")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_forward_kernels.md")


def kernel_sources_sha() -> str:
    """SHA-256 over the plain path's kernel sources, to tell whether byte
    counters taken earlier still describe the kernel being timed."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2304_12384_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per forward launch from the committed counter summary (the
    JSON block of the traffic profile), or None when that summary is missing
    or was taken on different kernel sources."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    start = text.find("```json")
    if start < 0:
        return None
    end = text.find("```", start + 7)
    try:
        data = json.loads(text[start + 7:end])
    except ValueError:
        return None
    if data.get("kernel_sources_sha256") != kernel_sources_sha():
        return None
    return {mode: v["hbm_bytes_per_launch"] for mode, v in data.items() if isinstance(v, dict)}


def attach_traffic(line: dict, traffic) -> None:
    """Sets roofline.traffic of each record the traffic summary covers (the
    head line is the full-DCT record unless only K = 16 ran)."""
    if not traffic:
        return
    head = "full" if line.get("config", {}).get("lowpass_k", 0) == 0 else "lowpass"
    spots = [(head, line), ("lowpass", line.get("lowpass_k16")),
             ("downsample", line.get("lowpass_downsample"))]
    for k in ("w16", "w8"):
        spots.append((k, (line.get("block_sizes_8bit") or {}).get(k)))
    for k in ("3840x2160_w32", "3840x2160_w16"):
        spots.append(("tenbit_" + k, (line.get("tenbit_stress") or {}).get(k)))
    for mode, entry in spots:
        if isinstance(entry, dict) and "roofline" in entry and mode in traffic:
            entry["roofline"]["traffic"] = traffic[mode]


def calibration_copy(mib: int) -> dict:
    """One plain device kernel that reads `mib` MiB and writes as many
    (bitwise NOT of uint8, a kernel of its own name in a counter run), its
    source written before a 1 GiB flush buffer so that it is read from HBM:
    the reference that scales FETCH_SIZE / WRITE_SIZE readings to bytes."""
    import torch
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(7)
    dst = torch.empty_like(src)
    flush = torch.empty(1 << 30, dtype=torch.uint8, device="cuda").fill_(1)
    torch.cuda.synchronize()
    del flush
    t0 = time.perf_counter()
    torch.bitwise_not(src, out=dst)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"bytes": n, "ms": dt * 1e3, "kernel": "bitwise_not (uint8)"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10,
                    help="untimed launches per mode first: the launch time settles over about ten")
    ap.add_argument("--cpu-frames", type=int, default=60,
                    help="2160p frames of the oracle's bounded CPU sample (0 skips it)")
    ap.add_argument("--modes",
                    default="full,lowpass,downsample,blocksizes,tenbit,ingest,batch,backward",
                    help="comma list of full, lowpass (K = 16 crop), downsample (the paper's 2x "
                         "downsampled low-pass), blocksizes (w = 16 and 8, full DCT), tenbit "
                         "(the 10-bit stress workload), ingest (frames from host memory and a "
                         ".yuv file), batch, backward")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of MIB MiB from a cold source (the "
                         "known-size reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the analysis has no multi-GPU path); "
              f"got --gpus {args.gpus}", file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    import paper_2304_12384_amd as vca
    import synth
    from synth.device import scene_to_device

    # Python's cyclic collector is off for the rest of the run (collected
    # once here): a full collection over torch's object graph stalls the host
    # for tens of milliseconds at random steps, which is the interpreter's
    # cost, not the path's.  Collecting per mode instead would idle the GPU
    # between the autotuner and the timed steps and start them at a lowered
    # clock.
    gc.collect()
    gc.disable()
    results = {}
    modes = args.modes.split(",")
    sv = dev = None
    if any(m in modes for m in ("full", "lowpass", "downsample", "blocksizes", "ingest")) \
            or args.cpu_frames > 0:
        log("generating the 600-frame 2160p synthetic workload")
        sv = synth.scene_video(WIDTH, HEIGHT, FRAMES)
        dev = scene_to_device(sv)
        torch.cuda.synchronize()
        log(f"frames resident on the device: {dev.nbytes / 1e9:.2f} GB")
    for mode in (m for m in modes if m in ("full", "lowpass", "downsample")):
        k = 16 if mode == "lowpass" else 0
        log(f"timing mode={mode} steps={args.steps} warmup={args.warmup}")
        results[mode] = run_mode(vca, dev, k, args.steps, args.warmup, not args.no_tune,
                                 downsample=mode == "downsample")
        log(f"mode={mode}: {results[mode]['fps']:.0f} frames/s, forward kernel "
            f"{results[mode]['forward_kernel_ms']:.3f} ms/launch, launch {results[mode]['launch']}")
    sizes = {}
    if "blocksizes" in modes:
        for w in (16, 8):
            log(f"timing block size w={w} (full DCT)")
            r = run_mode(vca, dev, 0, args.steps, args.warmup, not args.no_tune, block_size=w)
            r.pop("last_features")
            sizes[f"w{w}"] = r
            log(f"w={w}: {r['fps']:.0f} frames/s, forward kernel {r['forward_kernel_ms']:.3f} ms/launch")
    latency = None
    if "full" in modes:
        latency = run_latency(vca, dev)
        log(f"single-frame latency: median {latency['median_us']:.1f} us, "
            f"p99 {latency['p99_us']:.1f} us")
    tenbit = None
    if "tenbit" in modes:
        log("timing the 10-bit precision-stress workload")
        tenbit = run_tenbit(vca, args.steps, args.warmup, not args.no_tune)
    ingest = None
    if "ingest" in modes:
        log("timing host-resident ingest")
        ingest = run_ingest(vca, dev, max(2, args.steps // 8))
        log(f"ingest: {ingest['value']:.0f} frames/s from host memory ({ingest['GBps']:.1f} GB/s), "
            f"{ingest['file_value']:.0f} frames/s from a .yuv file")
    batch = batch_small = None
    if "batch" in modes:
        del dev
        torch.cuda.empty_cache()
        log("timing the batched form")
        batch = run_batch(vca, max(2, args.steps // 4), 1, not args.no_tune, synth.batch_streams(64),
                          "64 streams, resolution 360p..2160p, w in {8, 16, 32}, 30-300 frames "
                          "each (drawn per stream), 8-bit 4:2:0")
        log(f"batched: {batch['value']:.0f} frames/s over {batch['streams']} streams, "
            f"{batch['speedup_vs_plain']:.2f}x the plain path")
        torch.cuda.empty_cache()
        batch_small = run_batch(vca, max(20, args.steps), 3, not args.no_tune, small_streams(),
                                "256 streams of 640x360 8-bit 4:2:0, 8 frames each per step, "
                                "w = 8, 16, 32 in turn")
        log(f"batched, small streams: {batch_small['value']:.0f} frames/s over "
            f"{batch_small['streams']} streams, {batch_small['speedup_vs_plain']:.2f}x the plain path")

    backward = None
    if "backward" in modes:
        torch.cuda.empty_cache()
        log("timing the backward form")
        backward = run_backward(vca, max(50, 5 * args.steps), 20)
        log(f"backward: {backward['value']:.0f} frames/s forward+backward, kernels "
            f"{backward['forward_kernel_ms']:.3f} + {backward['backward_kernel_ms']:.3f} ms "
            f"(pair {backward['pair_hbm']['frac']:.2f} of HBM; forward alone "
            f"{backward['forward_alone']['ms']:.3f} ms, {backward['forward_alone']['frac']:.2f})")

    cpu = None
    if args.cpu_frames > 0:
        log(f"timing the CPU oracle on {args.cpu_frames} frames")
        cpu = cpu_baseline(sv, args.cpu_frames)

    copy = calibration_copy(args.calibrate_copy) if args.calibrate_copy > 0 else None

    if not results:
        print(json.dumps({"metric": METRIC, "batched": batch, "batched_small_streams": batch_small,
                          "backward": backward,
                          "host_ingest": ingest, "calibration_copy": copy}), flush=True)
        return 0
    head = results.get("full") or next(iter(results.values()))
    line = {
        "metric": METRIC,
        "value": head["fps"],
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "ms_per_step_median": head["ms_per_step_median"],
        "value_median": head["fps_median"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"{FRAMES} frames 3840x2160 8-bit YUV 4:2:0 per step, w=32, "
                               f"{'full DCT' if 'full' in results else 'low-pass K=16'}",
                   "frames_per_step": FRAMES, "block_size": BLOCK,
                   "lowpass_k": 0 if "full" in results else 16},
        "roofline": head["roofline"],
        "mfma": head["mfma"],
        "forward_kernel_ms": head["forward_kernel_ms"],
        "reduce_kernel_ms": head["reduce_kernel_ms"],
        "launch": head["launch"],
        "cpu_baseline": cpu,
    }
    if "downsample" in results and "full" in results:
        ds = results["downsample"]
        line["lowpass_downsample"] = {"value": ds["fps"], "unit": "frames/s",
                                      "ms_per_step": ds["ms_per_step"], "roofline": ds["roofline"],
                                      "mfma": ds["mfma"], "forward_kernel_ms": ds["forward_kernel_ms"],
                                      "launch": ds["launch"],
                                      "what": "planes downsampled 2x (2x2 mean), full 32x32 DCT"}
    if "lowpass" in results and "full" in results:
        lp = results["lowpass"]
        line["lowpass_k16"] = {"value": lp["fps"], "unit": "frames/s",
                               "ms_per_step": lp["ms_per_step"], "roofline": lp["roofline"],
                               "mfma": lp["mfma"], "forward_kernel_ms": lp["forward_kernel_ms"],
                               "launch": lp["launch"]}
    if copy is not None:
        line["calibration_copy"] = copy
    if sizes:
        line["block_sizes_8bit"] = {k: {"value": v["fps"], "unit": "frames/s",
                                        "ms_per_step": v["ms_per_step"], "roofline": v["roofline"],
                                        "mfma": v["mfma"], "forward_kernel_ms": v["forward_kernel_ms"],
                                        "launch": v["launch"]} for k, v in sizes.items()}
        line["block_sizes_8bit"]["workload"] = ("the same 600 frames of 3840x2160 8-bit 4:2:0, "
                                                "full DCT, one launch per step")
    if tenbit is not None:
        line["tenbit_stress"] = {k: {"value": v["fps"], "unit": "frames/s",
                                     "ms_per_step": v["ms_per_step"], "roofline": v["roofline"],
                                     "mfma": v["mfma"], "forward_kernel_ms": v["forward_kernel_ms"],
                                     "frame_bytes": v["frame_bytes"], "launch": v["launch"]}
                                 for k, v in tenbit.items()}
        line["tenbit_stress"]["workload"] = (f"{TENBIT_FRAMES} frames of 10-bit 4:2:0 (uint16) per "
                                             "step, full DCT: full-range noise, saturated edges "
                                             "and sign-matched worst-case blocks")
    if latency is not None:
        line["single_frame_latency"] = latency
    if ingest is not None:
        line["host_ingest"] = ingest
    if batch is not None:
        line["batched"] = batch
        line["batched_small_streams"] = batch_small
    if backward is not None:
        line["backward"] = backward
    attach_traffic(line, measured_traffic())
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
