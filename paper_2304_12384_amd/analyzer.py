"""Python face of the VCA library: one ``Analyzer`` per video stream.

Frames are torch tensors already on the GPU (uint8 for 8-bit, uint16 stored
as int16/uint16 for 10-bit); every step of the analysis runs in the HIP
library through the C ABI, on the caller's current torch stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from . import _lib
from ._lib import VcaConfig, VcaFrames, check

FEATURE_NAMES = ("E_Y", "h", "L_Y", "E_U", "E_V", "L_U", "L_V")


def block_counts(width: int, height: int, block_size: int = 32, bit_depth: int = 8,
                 lowpass_k: int = 0, downsample: bool = False) -> tuple[int, int, int]:
    cfg = _config(width, height, bit_depth, block_size, lowpass_k, 0,
                  _lib.VCA_F_DOWNSAMPLE if downsample else 0, 0, 0)
    out = (ctypes.c_int32 * 3)()
    check(_lib.lib().vca_block_counts(ctypes.byref(cfg), out), "vca_block_counts")
    return out[0], out[1], out[2]


def _config(width, height, bit_depth, block_size, lowpass_k, device, flags, max_batch,
            feature_capacity) -> VcaConfig:
    return VcaConfig(ctypes.sizeof(VcaConfig), width, height, bit_depth, 420, block_size,
                     lowpass_k, device, flags, max_batch, feature_capacity)


def _plane_geometry(t: torch.Tensor, bps: int):
    if t.dim() == 2:
        t = t.unsqueeze(0)
    if t.dim() != 3 or t.stride(2) != 1:
        raise ValueError("planes must be [n, rows, cols] with unit column stride")
    if not t.is_cuda:
        raise ValueError("frames must be device tensors")
    if t.element_size() != bps:
        raise ValueError(f"expected {bps}-byte samples, got {t.dtype}")
    return t, t.stride(1) * bps, t.stride(0) * bps


class PreparedFrames:
    """Frame descriptors of device buffers, validated once by ``prepare`` of
    one Analyzer or Batch and submitted any number of times (the caller
    refills the buffers in between; they stay referenced here)."""
    __slots__ = ("owner", "frames", "counts", "keep")

    def __init__(self, owner, frames, counts, keep):
        self.owner, self.frames, self.counts, self.keep = owner, frames, counts, keep


class Analyzer:
    """Wraps one ``vca_ctx``.

    >>> an = Analyzer(3840, 2160, block_size=32)
    >>> an.submit(y, u, v)          # y: [n, H, W] uint8 cuda tensor, u/v: [n, H/2, W/2]
    >>> feats = an.features(0, n)   # numpy [n, 7] float32
    """

    def __init__(self, width: int, height: int, *, bit_depth: int = 8, block_size: int = 32,
                 lowpass_k: int = 0, device: int | None = None, keep_coeffs: bool = False,
                 validate: bool = False, timing: bool = False, max_batch: int = 0,
                 feature_capacity: int = 0, downsample: bool = False,
                 stream: torch.cuda.Stream | None = None):
        if device is None:
            device = torch.cuda.current_device()
        flags = ((_lib.VCA_F_KEEP_COEFFS if keep_coeffs else 0) |
                 (_lib.VCA_F_VALIDATE if validate else 0) | (_lib.VCA_F_TIMING if timing else 0) |
                 (_lib.VCA_F_DOWNSAMPLE if downsample else 0))
        self.cfg = _config(width, height, bit_depth, block_size, lowpass_k, device, flags,
                           max_batch, feature_capacity)
        self.width, self.height, self.bit_depth = width, height, bit_depth
        self.block_size = block_size
        self.k = block_size if lowpass_k == 0 else lowpass_k
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._ctx = ctypes.c_void_p()
        check(_lib.lib().vca_open(ctypes.byref(self.cfg), ctypes.c_void_p(self.stream.cuda_stream),
                                  ctypes.byref(self._ctx)), "vca_open")
        self.counts = block_counts(width, height, block_size, bit_depth, lowpass_k, downsample)
        self._keep = []   # frame tensors referenced until their work is known to be done

    # ------------------------------------------------------------------ calls
    def close(self) -> None:
        if self._ctx:
            _lib.lib().vca_close(self._ctx)
            self._ctx = ctypes.c_void_p()
        self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def submitted(self) -> int:
        return int(_lib.lib().vca_frames_submitted(self._ctx))

    def prepare(self, y: torch.Tensor, u: torch.Tensor, v: torch.Tensor) -> PreparedFrames:
        """Validates device planes once; ``submit`` takes the result in place
        of the planes."""
        bps = 1 if self.bit_depth == 8 else 2
        y, py, fy = _plane_geometry(y, bps)
        u, pu, fu = _plane_geometry(u, bps)
        v, pv, fv = _plane_geometry(v, bps)
        if pu != pv or fu != fv:
            raise ValueError("U and V must share pitch and frame stride")
        n = y.shape[0]
        if u.shape[0] != n or v.shape[0] != n:
            raise ValueError("planes hold different frame counts")
        if y.shape[1:] != (self.height, self.width):
            raise ValueError(f"luma shape {tuple(y.shape[1:])} != {(self.height, self.width)}")
        if u.shape[1:] != (self.height // 2, self.width // 2) or v.shape[1:] != u.shape[1:]:
            raise ValueError("chroma planes must be [n, H/2, W/2]")
        fr = VcaFrames(y.data_ptr(), u.data_ptr(), v.data_ptr(), py, pu, fy, fu, 1)
        return PreparedFrames(self, fr, n, (y, u, v))

    def submit(self, y, u: torch.Tensor | None = None, v: torch.Tensor | None = None) -> int:
        """Enqueues frames (asynchronous): device planes y, u, v, or a
        ``prepare`` result of this Analyzer.  Returns the index of the first
        frame."""
        p = y if isinstance(y, PreparedFrames) else self.prepare(y, u, v)
        if p.owner is not self:
            raise ValueError("frames prepared by another Analyzer")
        first = self.submitted
        check(_lib.lib().vca_analyze_frames(self._ctx, ctypes.byref(p.frames), p.counts),
              "vca_analyze_frames", self._ctx)
        self._keep = p.keep
        return first

    def submit_host(self, y, u, v) -> int:
        """Enqueues host-resident frames (numpy arrays or CPU tensors, [n, H, W]
        and [n, H/2, W/2], uint8 or 16-bit); the library stages them through
        pinned buffers and returns once they are copied.  Returns the index of
        the first frame."""
        planes = [_host_plane(p, self.bit_depth) for p in (y, u, v)]
        (ya, py, fy), (ua, pu, fu), (va, pv, fv) = planes
        n = ya.shape[0]
        if ua.shape[0] != n or va.shape[0] != n:
            raise ValueError("planes hold different frame counts")
        if ya.shape[1:] != (self.height, self.width):
            raise ValueError(f"luma shape {ya.shape[1:]} != {(self.height, self.width)}")
        if ua.shape[1:] != (self.height // 2, self.width // 2) or va.shape[1:] != ua.shape[1:]:
            raise ValueError("chroma planes must be [n, H/2, W/2]")
        if pu != pv or fu != fv:
            raise ValueError("U and V must share pitch and frame stride")
        fr = VcaFrames(ya.ctypes.data, ua.ctypes.data, va.ctypes.data, py, pu, fy, fu, 0)
        first = self.submitted
        check(_lib.lib().vca_analyze_frames(self._ctx, ctypes.byref(fr), n), "vca_analyze_frames",
              self._ctx)
        return first

    def submit_file(self, path: str, first: int = 0, count: int | None = None) -> int:
        """Enqueues frames [first, first + count) of a raw 4:2:0 .yuv file of this
        resolution and bit depth (count None: to the end of the file)."""
        if count is None:
            bps = 1 if self.bit_depth == 8 else 2
            frame = (self.width * self.height + 2 * (self.width // 2) * (self.height // 2)) * bps
            count = os.path.getsize(path) // frame - first
        start = self.submitted
        check(_lib.lib().vca_analyze_yuv_file(self._ctx, os.fsencode(path), first, count),
              "vca_analyze_yuv_file", self._ctx)
        return start

    def features(self, first: int, count: int) -> np.ndarray:
        """Features of frames [first, first + count) as float32 [count, 7]; waits."""
        out = np.zeros((count, 7), np.float32)
        check(_lib.lib().vca_features(self._ctx, first, count, out.ctypes.data_as(ctypes.c_void_p)),
              "vca_features", self._ctx)
        return out

    def analyze(self, y: torch.Tensor, u: torch.Tensor, v: torch.Tensor) -> np.ndarray:
        first = self.submit(y, u, v)
        return self.features(first, self.submitted - first)

    def block_coeffs(self, frame: int) -> np.ndarray:
        """int16 [C_Y + C_U + C_V, K, K] of a frame of the most recent call."""
        total = sum(self.counts)
        out = np.zeros((total, self.k, self.k), np.int16)
        check(_lib.lib().vca_block_coeffs(self._ctx, frame, out.ctypes.data_as(ctypes.c_void_p),
                                          out.size), "vca_block_coeffs", self._ctx)
        return out

    def block_stats(self, frame: int) -> tuple[np.ndarray, np.ndarray]:
        """(H float64, DC int32), each [C_Y + C_U + C_V], of a frame of the last launch."""
        total = sum(self.counts)
        h = np.zeros(total, np.float64)
        dc = np.zeros(total, np.int32)
        check(_lib.lib().vca_block_stats(self._ctx, frame, h.ctypes.data_as(ctypes.c_void_p),
                                         dc.ctypes.data_as(ctypes.c_void_p), total),
              "vca_block_stats", self._ctx)
        return h, dc

    def block_maps(self, first: int, count: int) -> dict:
        """Per-block maps of frames [first, first + count) of the last launch as
        device tensors on the context's stream: ``h`` float64 [count, C_Y + C_U + C_V],
        ``dc`` int32 (same shape), ``dh`` float64 [count, C_Y] = |H_t - H_{t-1}| of
        the luma blocks (0 for a frame without a previous one)."""
        total = sum(self.counts)
        dev = torch.device("cuda", self.device)
        with torch.cuda.stream(self.stream):
            h = torch.empty((count, total), dtype=torch.float64, device=dev)
            dc = torch.empty((count, total), dtype=torch.int32, device=dev)
            dh = torch.empty((count, self.counts[0]), dtype=torch.float64, device=dev)
        check(_lib.lib().vca_block_maps(self._ctx, first, count, ctypes.c_void_p(h.data_ptr()),
                                        ctypes.c_void_p(dc.data_ptr()), ctypes.c_void_p(dh.data_ptr())),
              "vca_block_maps", self._ctx)
        return {"h": h, "dc": dc, "dh": dh}

    def timing(self, reset: bool = False) -> dict:
        """Kernel times measured with HIP events on the context's stream."""
        t = _lib.VcaTiming()
        check(_lib.lib().vca_get_timing(self._ctx, ctypes.byref(t), int(reset)), "vca_get_timing",
              self._ctx)
        return {f: getattr(t, f) for f, _ in t._fields_}

    def reset(self) -> None:
        check(_lib.lib().vca_reset(self._ctx), "vca_reset", self._ctx)

    def tune(self, y: torch.Tensor, u: torch.Tensor, v: torch.Tensor, reps: int = 3) -> dict:
        """Autotunes the launch shape on these frames (see vca_tune)."""
        fr = _frames(self, y, u, v)
        check(_lib.lib().vca_tune(self._ctx, ctypes.byref(fr), y.shape[0], reps), "vca_tune", self._ctx)
        return self.tuned_launch()

    def tuned_launch(self) -> dict:
        d, g, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        check(_lib.lib().vca_tuned_launch(self._ctx, ctypes.byref(d), ctypes.byref(g), ctypes.byref(ms)),
              "vca_tuned_launch", self._ctx)
        return {"depth": d.value, "groups_per_cu": g.value, "ms": ms.value}


def analyze_noalloc(y: torch.Tensor, u: torch.Tensor, v: torch.Tensor, out: torch.Tensor, *,
                    bit_depth: int = 8, block_size: int = 32, lowpass_k: int = 0,
                    downsample: bool = False, stream: torch.cuda.Stream | None = None) -> None:
    """``vca_analyze_noalloc``: features of device frames y, u, v ([n, H, W],
    [n, H/2, W/2]) as one fresh sequence into ``out`` (float32 device tensor
    [n, 7], contiguous), enqueued on ``stream`` (default: the current one) with
    no device allocation by the library."""
    bps = 1 if bit_depth == 8 else 2
    y, py, fy = _plane_geometry(y, bps)
    u, pu, fu = _plane_geometry(u, bps)
    v, pv, fv = _plane_geometry(v, bps)
    if pu != pv or fu != fv:
        raise ValueError("U and V must share pitch and frame stride")
    n = y.shape[0]
    if u.shape[0] != n or v.shape[0] != n:
        raise ValueError("planes hold different frame counts")
    if not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
            and tuple(out.shape) == (n, 7)):
        raise ValueError("out must be a contiguous float32 device tensor [n, 7]")
    height, width = y.shape[1], y.shape[2]
    cfg = _config(width, height, bit_depth, block_size, lowpass_k, y.device.index,
                  _lib.VCA_F_DOWNSAMPLE if downsample else 0, 0, 0)
    fr = VcaFrames(y.data_ptr(), u.data_ptr(), v.data_ptr(), py, pu, fy, fu, 1)
    if stream is None:
        stream = torch.cuda.current_stream(y.device)
    check(_lib.lib().vca_analyze_noalloc(ctypes.byref(cfg), ctypes.byref(fr), n,
                                         ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(stream.cuda_stream)),
          "vca_analyze_noalloc")


def _host_plane(p, bit_depth):
    """(contiguous-row numpy array, pitch, frame stride) of a host plane."""
    if hasattr(p, "is_cuda"):
        if p.is_cuda:
            raise ValueError("submit_host takes host arrays")
        p = p.numpy()
    a = np.asarray(p)
    if a.ndim != 3:
        raise ValueError("planes must be [n, rows, columns]")
    bps = 1 if bit_depth == 8 else 2
    if a.itemsize != bps:
        raise ValueError(f"expected {bps}-byte samples, got {a.dtype}")
    if a.strides[2] != bps:
        a = np.ascontiguousarray(a)
    return a, a.strides[1], a.strides[0]


def read_yuv(path: str, width: int, height: int, bit_depth: int = 8, first: int = 0,
             count: int | None = None):
    """Frames [first, first + count) of a raw 4:2:0 .yuv file as numpy planes
    (y [n, H, W], u and v [n, H/2, W/2]; uint8, or uint16 for 10-bit)."""
    dt = np.uint8 if bit_depth == 8 else np.uint16
    bps = np.dtype(dt).itemsize
    frame = (width * height + 2 * (width // 2) * (height // 2)) * bps
    if count is None:
        count = os.path.getsize(path) // frame - first
    y = np.empty((count, height, width), dt)
    u = np.empty((count, height // 2, width // 2), dt)
    v = np.empty_like(u)
    check(_lib.lib().vca_read_yuv(os.fsencode(path), width, height, bit_depth, first, count,
                                  y.ctypes.data, u.ctypes.data, v.ctypes.data), "vca_read_yuv")
    return y, u, v


def write_yuv(path: str, y, u, v) -> None:
    """Writes planes ([n, H, W], [n, H/2, W/2]) as a raw 4:2:0 .yuv file."""
    with open(path, "wb") as f:
        for t in range(y.shape[0]):
            for p in (y[t], u[t], v[t]):
                f.write(np.ascontiguousarray(p).astype(p.dtype.newbyteorder("<"), copy=False).tobytes())


def _frames(owner, y, u, v) -> VcaFrames:
    """Validated frame descriptor of device planes for a stream of `owner`'s
    geometry (width, height, bit_depth attributes)."""
    bps = 1 if owner.bit_depth == 8 else 2
    y, py, fy = _plane_geometry(y, bps)
    u, pu, fu = _plane_geometry(u, bps)
    v, pv, fv = _plane_geometry(v, bps)
    if pu != pv or fu != fv:
        raise ValueError("U and V must share pitch and frame stride")
    n = y.shape[0]
    if u.shape[0] != n or v.shape[0] != n:
        raise ValueError("planes hold different frame counts")
    if y.shape[1:] != (owner.height, owner.width):
        raise ValueError(f"luma shape {tuple(y.shape[1:])} != {(owner.height, owner.width)}")
    if u.shape[1:] != (owner.height // 2, owner.width // 2) or v.shape[1:] != u.shape[1:]:
        raise ValueError("chroma planes must be [n, H/2, W/2]")
    return VcaFrames(y.data_ptr(), u.data_ptr(), v.data_ptr(), py, pu, fy, fu, 1)


class _StreamGeom:
    def __init__(self, width, height, bit_depth):
        self.width, self.height, self.bit_depth = width, height, bit_depth


class Batch:
    """Wraps one ``vca_batch``: many streams analysed by one graph-replayed
    round (one persistent launch per class of streams).

    >>> b = Batch([dict(width=1920, height=1080, block_size=16), dict(width=640, height=360)])
    >>> b.submit([(y0, u0, v0), (y1, u1, v1)])
    >>> b.features(0, 0, n0)
    """

    def __init__(self, streams: list, *, device: int | None = None, timing: bool = False,
                 stream: torch.cuda.Stream | None = None):
        if device is None:
            device = torch.cuda.current_device()
        n = len(streams)
        cfgs = (VcaConfig * n)()
        self.geoms = []
        for s, d in enumerate(streams):
            flags = (_lib.VCA_F_TIMING if timing else 0) | (_lib.VCA_F_VALIDATE if d.get("validate") else 0)
            cfgs[s] = _config(d["width"], d["height"], d.get("bit_depth", 8), d.get("block_size", 32),
                              d.get("lowpass_k", 0), device, flags, d.get("max_batch", 0),
                              d.get("feature_capacity", 0))
            self.geoms.append(_StreamGeom(d["width"], d["height"], d.get("bit_depth", 8)))
        self.n = n
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._b = ctypes.c_void_p()
        check(_lib.lib().vca_open_batch(cfgs, n, ctypes.c_void_p(self.stream.cuda_stream),
                                        ctypes.byref(self._b)), "vca_open_batch")
        self._keep = []
        self._submitted = [0] * n     # mirrors vca_batch_submitted

    def close(self) -> None:
        if self._b:
            _lib.lib().vca_close_batch(self._b)
            self._b = ctypes.c_void_p()
        self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _descr(self, frames):
        if len(frames) != self.n:
            raise ValueError(f"expected {self.n} frame sets")
        fr = (VcaFrames * self.n)()
        counts = (ctypes.c_int32 * self.n)()
        keep = []
        for s, f in enumerate(frames):
            if f is None:
                fr[s] = VcaFrames(None, None, None, 0, 0, 0, 0, 1)
                counts[s] = 0
                continue
            y, u, v = f
            fr[s] = _frames(self.geoms[s], y, u, v)
            counts[s] = y.shape[0] if y.dim() == 3 else 1
            keep += [y, u, v]
        return fr, counts, keep

    def submitted(self, s: int) -> int:
        return int(_lib.lib().vca_batch_submitted(self._b, s))

    def prepare(self, frames: list) -> PreparedFrames:
        """Validates every stream's device planes once; ``submit`` takes the
        result in place of the list."""
        fr, counts, keep = self._descr(frames)
        return PreparedFrames(self, fr, counts, keep)

    def submit(self, frames) -> list:
        """frames[s] = (y, u, v) device planes of stream s, or None; or a
        ``prepare`` result of this Batch.  Returns the index of each stream's
        first submitted frame (asynchronous)."""
        p = frames if isinstance(frames, PreparedFrames) else self.prepare(frames)
        if p.owner is not self:
            raise ValueError("frames prepared by another Batch")
        first = list(self._submitted)
        st = _lib.lib().vca_analyze_batch(self._b, p.frames, p.counts)
        if st == 0:
            self._submitted = [f + c for f, c in zip(first, p.counts)]
        else:   # a failure may come after some rounds were enqueued
            self._submitted = [self.submitted(s) for s in range(self.n)]
        check(st, "vca_analyze_batch", batch=self._b)
        self._keep = p.keep
        return first

    def features(self, s: int, first: int, count: int) -> np.ndarray:
        out = np.zeros((count, 7), np.float32)
        check(_lib.lib().vca_batch_features(self._b, s, first, count,
                                            out.ctypes.data_as(ctypes.c_void_p)),
              "vca_batch_features", batch=self._b)
        return out

    def features_many(self, requests: list) -> list:
        """Features of several (stream, first, count) requests in one call,
        waiting once: a list of numpy [count, 7] arrays in request order."""
        n = len(requests)
        streams = np.fromiter((r[0] for r in requests), np.int32, n)
        first = np.fromiter((r[1] for r in requests), np.int64, n)
        count = np.fromiter((r[2] for r in requests), np.int32, n)
        out = np.zeros((int(count.sum()), 7), np.float32)
        check(_lib.lib().vca_batch_features_many(
            self._b, n, streams.ctypes.data_as(ctypes.c_void_p), first.ctypes.data_as(ctypes.c_void_p),
            count.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p)),
            "vca_batch_features_many", batch=self._b)
        return np.split(out, np.cumsum(count)[:-1]) if n else []

    def tune(self, frames: list, reps: int = 3) -> dict:
        fr, counts, keep = self._descr(frames)
        check(_lib.lib().vca_tune_batch(self._b, fr, counts, reps), "vca_tune_batch", batch=self._b)
        return self.tuned_launch()

    def tuned_launch(self) -> dict:
        d, g, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        check(_lib.lib().vca_batch_tuned_launch(self._b, ctypes.byref(d), ctypes.byref(g),
                                                ctypes.byref(ms)), "vca_batch_tuned_launch",
              batch=self._b)
        return {"depth": d.value, "groups_per_cu": g.value, "ms": ms.value}

    def class_times(self) -> dict:
        """Tuned forward launch of each class present: {"b8_w32_k32": {"ms", "depth",
        "groups_per_cu", "waves", "chunk_strips"}, ...} (device time of the class's
        launch alone)."""
        ms = (ctypes.c_double * 18)()
        dp, gp, wv, ch = [(ctypes.c_int32 * 18)() for _ in range(4)]
        check(_lib.lib().vca_batch_class_times(self._b, ms, dp, gp, wv, ch), "vca_batch_class_times",
              batch=self._b)
        out = {}
        for k in range(18):
            if dp[k] <= 0:
                continue
            bits = 10 if k >= 9 else 8
            w = (32, 16, 8)[(k // 3) % 3]
            kk = w // (1, 2, 4)[k % 3]
            out[f"b{bits}_w{w}_k{kk}"] = {"ms": ms[k], "depth": dp[k], "groups_per_cu": gp[k],
                                         "waves": wv[k], "chunk_strips": ch[k]}
        return out

    def arrangement(self) -> dict:
        """How a round runs its classes: {"serial": bool, "serial_ms", "parallel_ms"}
        (the tuned round times of either arrangement, reductions included, 0 if
        not measured)."""
        sr, sm, pm = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double()
        check(_lib.lib().vca_batch_arrangement(self._b, ctypes.byref(sr), ctypes.byref(sm),
                                               ctypes.byref(pm)), "vca_batch_arrangement",
              batch=self._b)
        return {"serial": bool(sr.value), "serial_ms": sm.value, "parallel_ms": pm.value}

    def set_class_shape(self, cls: str, depth: int, groups_per_cu: int, waves: int,
                        chunk_strips: int) -> None:
        """Pins class `cls` ("b8_w16_k16", as class_times names them) to a launch
        shape in place of the tuned one."""
        bits, w, kk = (int(x[1:]) for x in cls.split("_"))
        k = (9 if bits == 10 else 0) + 3 * {32: 0, 16: 1, 8: 2}[w] + {w: 0, w // 2: 1, w // 4: 2}[kk]
        check(_lib.lib().vca_batch_set_class_shape(self._b, k, depth, groups_per_cu, waves,
                                                   chunk_strips), "vca_batch_set_class_shape",
              batch=self._b)

    def set_arrangement(self, serial: bool) -> None:
        """Runs the later rounds' classes one after another (True) or side by
        side (False), in place of the tuned choice."""
        check(_lib.lib().vca_batch_set_arrangement(self._b, int(serial)),
              "vca_batch_set_arrangement", batch=self._b)

    def timing(self, reset: bool = False) -> dict:
        ms, n, fr = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        check(_lib.lib().vca_batch_timing(self._b, ctypes.byref(ms), ctypes.byref(n),
                                          ctypes.byref(fr), int(reset)), "vca_batch_timing",
              batch=self._b)
        return {"ms": ms.value, "launches": n.value, "frames": fr.value}

    def reset(self, stream: int = -1) -> None:
        check(_lib.lib().vca_reset_batch(self._b, stream), "vca_reset_batch", batch=self._b)
