"""TEST INFRASTRUCTURE ONLY: Python face of the plain CPU oracle.

The oracle computes the seven per-frame VCA features of Menon et al. (GMSys
2023), Section 2, and the block transform behind them, in exact int64
arithmetic and FP64 (``oracle/vcaref.c`` holds the arithmetic and lists the
readings taken where the paper is silent).  Only ``tests/``, the smoke check
and the benchmark's ``cpu_baseline`` leg may import this package.  It shares no
code with ``paper_2304_12384_amd`` and never imports it.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# VCAREF_LIB names another build of vcaref.c (the mutation tests plant a
# mistake in a copy and check that the pins catch it).
LIB_PATH = os.environ.get("VCAREF_LIB") or os.path.join(HERE, "libvcaref.so")

FEATURE_NAMES = ("E_Y", "h", "L_Y", "E_U", "E_V", "L_U", "L_V")

_lib = None


class _Config(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("bit_depth", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("lowpass_k", ctypes.c_int32)]


class OracleError(RuntimeError):
    pass


def lib() -> ctypes.CDLL:
    """Loads the built oracle library, building it only if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.vcaref_dct_matrix.argtypes = [ctypes.c_int32, P]
        L.vcaref_weights.argtypes = [ctypes.c_int32, P]
        L.vcaref_block_transform.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P]
        L.vcaref_block_counts.argtypes = [ctypes.POINTER(_Config), P]
        L.vcaref_analyze.argtypes = [ctypes.POINTER(_Config), P, P, P, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_int32, ctypes.c_int32, P, P, P, P, P]
        for f in (L.vcaref_dct_matrix, L.vcaref_weights, L.vcaref_block_transform,
                  L.vcaref_block_counts, L.vcaref_analyze):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str) -> None:
    if rc == -2:
        raise OracleError(f"{what}: sample outside [0, 2^bit_depth - 1]")
    if rc != 0:
        raise OracleError(f"{what}: invalid argument (code {rc})")


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def dct_matrix(w: int) -> np.ndarray:
    """Integer DCT matrix C_w, rows = frequencies (int64, w x w)."""
    out = np.zeros((w, w), np.int32)
    _check(lib().vcaref_dct_matrix(w, _ptr(out)), "dct_matrix")
    return out.astype(np.int64)


def weights(w: int) -> np.ndarray:
    """Energy weights W[i][j] (float64, w x w)."""
    out = np.zeros((w, w), np.float64)
    _check(lib().vcaref_weights(w, _ptr(out)), "weights")
    return out


def block_transform(x: np.ndarray, bit_depth: int, k: int | None = None) -> np.ndarray:
    """Top-left K x K integer coefficients of one w x w block of raw samples."""
    x = np.ascontiguousarray(x, dtype=np.int32)
    w = x.shape[0]
    assert x.shape == (w, w)
    K = w if not k else k
    out = np.zeros((K, K), np.int64)
    _check(lib().vcaref_block_transform(_ptr(x), w, K, bit_depth, _ptr(out)), "block_transform")
    return out


@dataclass
class Config:
    width: int
    height: int
    bit_depth: int = 8
    block_size: int = 32
    lowpass_k: int = 0

    def _c(self) -> _Config:
        return _Config(self.width, self.height, self.bit_depth, self.block_size, self.lowpass_k)

    @property
    def k(self) -> int:
        return self.block_size if self.lowpass_k == 0 else self.lowpass_k


def block_counts(cfg: Config) -> tuple[int, int, int]:
    out = np.zeros(3, np.int32)
    _check(lib().vcaref_block_counts(ctypes.byref(cfg._c()), _ptr(out)), "block_counts")
    return int(out[0]), int(out[1]), int(out[2])


@dataclass
class Result:
    features: np.ndarray            # [n, 7] float64: E_Y, h, L_Y, E_U, E_V, L_U, L_V
    block_h: np.ndarray | None      # [n, C_Y + C_U + C_V] float64
    block_dc: np.ndarray | None     # [n, C_Y + C_U + C_V] int64
    coeffs: np.ndarray | None       # [n, C_Y + C_U + C_V, K, K] int32


def analyze(cfg: Config, y: np.ndarray, u: np.ndarray, v: np.ndarray, *,
            h_prev: np.ndarray | None = None, threads: int = 1,
            want_blocks: bool = False, want_coeffs: bool = False) -> Result:
    """Features of n frames given as [n, H, W] (Y) and [n, H/2, W/2] (U, V)
    arrays of uint8 (8-bit) or uint16 (10-bit) samples."""
    dt = np.uint8 if cfg.bit_depth == 8 else np.uint16
    planes = [np.ascontiguousarray(p, dtype=dt) for p in (y, u, v)]
    if planes[0].ndim == 2:
        planes = [p[None] for p in planes]
    n = planes[0].shape[0]
    assert planes[0].shape[1:] == (cfg.height, cfg.width), planes[0].shape
    assert planes[1].shape == planes[2].shape == (n, cfg.height // 2, cfg.width // 2)
    cy, cu, cv = block_counts(cfg)
    total = cy + cu + cv
    K = cfg.k
    feats = np.zeros((n, 7), np.float64)
    bh = np.zeros((n, total), np.float64) if want_blocks else None
    bdc = np.zeros((n, total), np.int64) if want_blocks else None
    co = np.zeros((n, total, K, K), np.int32) if want_coeffs else None
    hp = None
    if h_prev is not None:
        hp = np.ascontiguousarray(h_prev, dtype=np.float64)
        assert hp.shape == (cy,)
    rc = lib().vcaref_analyze(
        ctypes.byref(cfg._c()), _ptr(planes[0]), _ptr(planes[1]), _ptr(planes[2]),
        cfg.width, cfg.width // 2, cfg.width * cfg.height, (cfg.width // 2) * (cfg.height // 2),
        n, threads, _ptr(hp), _ptr(feats), _ptr(bh), _ptr(bdc), _ptr(co))
    _check(rc, "analyze")
    return Result(feats, bh, bdc, co)


# --------------------------------------------------------------- downsampling
# The paper's own low-pass option (Section 2, optimisation (3)) evaluates the
# features on the video spatially downsampled by two.  The filter is not
# stated; the reading taken here: each output sample is the mean of a 2 x 2
# input block, rounded half up, in integer arithmetic, on every plane.  Frame
# dimensions must be multiples of 4 so that the result is 4:2:0 video of
# half the width and height.

def downsample(plane: np.ndarray) -> np.ndarray:
    """[..., H, W] uint8/uint16 -> [..., H/2, W/2] of (a + b + c + d + 2) >> 2,
    a..d the 2 x 2 block (H, W even)."""
    p = np.asarray(plane)
    assert p.shape[-1] % 2 == 0 and p.shape[-2] % 2 == 0, p.shape
    q = p.astype(np.int64)
    s = q[..., 0::2, 0::2] + q[..., 0::2, 1::2] + q[..., 1::2, 0::2] + q[..., 1::2, 1::2]
    return ((s + 2) >> 2).astype(p.dtype)


def analyze_downsampled(cfg: Config, y: np.ndarray, u: np.ndarray, v: np.ndarray,
                        **kw) -> Result:
    """The features of video (cfg.width x cfg.height) after 2x downsampling
    of every plane: analyze() on the (width/2 x height/2) 4:2:0 video."""
    if cfg.width % 4 or cfg.height % 4:
        raise OracleError("downsampling needs width and height divisible by 4")
    half = Config(cfg.width // 2, cfg.height // 2, cfg.bit_depth, cfg.block_size, cfg.lowpass_k)
    return analyze(half, downsample(y), downsample(u), downsample(v), **kw)
