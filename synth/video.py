"""Seeded synthetic video recipes.

Every recipe is deterministic in (recipe index, stream) through NumPy's PCG64
seeded with ``SEED_BASE + 1000 * recipe + stream``.  Frames come back as
planar arrays: Y of shape [H, W] and U, V of shape [H/2, W/2], uint8 for 8-bit
and uint16 for 10-bit samples.

Recipes (the workloads the paper measures are UHD 8-bit 4:2:0 videos; these
stand in for them with the same shapes and sample ranges):
  * ``patches_video``: a linear luma gradient with Gaussian-noise patches that
    translate 2 px per frame, smooth sinusoidal chroma with fresh uniform noise.
  * ``scene_video``: scenes of ``scene_len`` frames, each a crop window moving
    with a constant global motion over a noisy gradient canvas; a hard cut
    starts a new canvas.  Frames are crops of a few canvases, so a device can
    rebuild them cheaply from the canvases and the offsets (``SceneVideo``).
  * ``stress_video``: 10-bit blocks of full-range noise, saturated edges and
    cosine-sign patterns that drive transform intermediates to their extremes.
  * ``soft_frames``: float frames with fractional values, as a pre-processing
    filter would produce them: a separable binomial blur of given frames with
    seeded per-frame sub-sample weights.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2304_12384


def make_rng(recipe: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + 1000 * recipe + stream))


def _to_samples(a: np.ndarray, bit_depth: int) -> np.ndarray:
    maxv = (1 << bit_depth) - 1
    out = np.clip(np.rint(a), 0, maxv)
    return out.astype(np.uint8 if bit_depth == 8 else np.uint16)


@dataclass
class Video:
    """Frames held in host memory: y [n, H, W], u and v [n, H/2, W/2]."""
    y: np.ndarray
    u: np.ndarray
    v: np.ndarray
    bit_depth: int

    @property
    def n_frames(self) -> int:
        return self.y.shape[0]

    @property
    def width(self) -> int:
        return self.y.shape[2]

    @property
    def height(self) -> int:
        return self.y.shape[1]

    def frames(self, t0: int = 0, t1: int | None = None) -> "Video":
        t1 = self.n_frames if t1 is None else t1
        return Video(self.y[t0:t1], self.u[t0:t1], self.v[t0:t1], self.bit_depth)


def patches_video(width: int = 1280, height: int = 720, n_frames: int = 10, *,
                  recipe: int = 0, stream: int = 0, n_patches: int = 12) -> Video:
    """Linear luma gradient 16 + 219 (0.6 x/W + 0.4 y/H) plus ``n_patches``
    rectangular Gaussian-noise patches (sides 64..256 px, sigma in 4..40) that
    move +2 px per frame in x; chroma 128 + 60 sin(2 pi x/lx + phi) cos(2 pi y/ly)
    (periods 160..320 chroma px) plus fresh uniform noise in [-8, 8] per frame."""
    rng = make_rng(recipe, stream)
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float64)
    base = 16.0 + 219.0 * (0.6 * xx / width + 0.4 * yy / height)
    patches = []
    for _ in range(n_patches):
        ph = int(rng.integers(64, 257))
        pw = int(rng.integers(64, 257))
        y0 = int(rng.integers(0, max(1, height - ph)))
        x0 = int(rng.integers(0, max(1, width - pw)))
        sigma = float(rng.integers(4, 41))
        patches.append((y0, x0, sigma * rng.standard_normal((ph, pw))))
    ch, cw = height // 2, width // 2
    cy, cx = np.mgrid[0:ch, 0:cw].astype(np.float64)
    chroma_fields = []
    for _ in range(2):
        lx, ly = rng.uniform(160, 320, size=2)
        phi = rng.uniform(0, 2 * np.pi)
        chroma_fields.append(128.0 + 60.0 * np.sin(2 * np.pi * cx / lx + phi) * np.cos(2 * np.pi * cy / ly))
    Y = np.empty((n_frames, height, width), np.uint8)
    U = np.empty((n_frames, ch, cw), np.uint8)
    V = np.empty((n_frames, ch, cw), np.uint8)
    for t in range(n_frames):
        f = base.copy()
        for (y0, x0, noise) in patches:
            ph, pw = noise.shape
            xs = x0 + 2 * t
            if xs >= width:
                continue
            span = min(pw, width - xs)
            f[y0:y0 + ph, xs:xs + span] += noise[:, :span]
        Y[t] = _to_samples(f, 8)
        U[t] = _to_samples(chroma_fields[0] + rng.integers(-8, 9, size=(ch, cw)), 8)
        V[t] = _to_samples(chroma_fields[1] + rng.integers(-8, 9, size=(ch, cw)), 8)
    return Video(Y, U, V, 8)


@dataclass
class SceneVideo:
    """Frames as crops of per-scene canvases.

    Frame t belongs to scene ``t // scene_len``; its luma is
    ``canvas_y[oy:oy+H, ox:ox+W]`` and its chroma
    ``canvas_u[oy//2 : oy//2 + H/2, ox//2 : ox//2 + W/2]`` (same for V) with
    ``(oy, ox) = offsets[t]``."""
    width: int
    height: int
    n_frames: int
    bit_depth: int
    scene_len: int
    canvases: list = field(default_factory=list)   # [(Y, U, V)] per scene
    offsets: np.ndarray = None                     # [n_frames, 2] (oy, ox) luma
    params: list = field(default_factory=list)     # per-scene (sigma, dy, dx)

    def scene_of(self, t: int) -> int:
        return t // self.scene_len

    def frame(self, t: int):
        cy, cu, cv = self.canvases[self.scene_of(t)]
        oy, ox = (int(a) for a in self.offsets[t])
        H, W = self.height, self.width
        return (cy[oy:oy + H, ox:ox + W], cu[oy // 2:oy // 2 + H // 2, ox // 2:ox // 2 + W // 2],
                cv[oy // 2:oy // 2 + H // 2, ox // 2:ox // 2 + W // 2])

    def frames(self, t0: int = 0, t1: int | None = None) -> Video:
        t1 = self.n_frames if t1 is None else t1
        ys, us, vs = zip(*(self.frame(t) for t in range(t0, t1)))
        return Video(np.stack(ys), np.stack(us), np.stack(vs), self.bit_depth)


def scene_video(width: int = 3840, height: int = 2160, n_frames: int = 600, *,
                scene_len: int = 120, bit_depth: int = 8, recipe: int = 1, stream: int = 0,
                max_sigma: float = 60.0, max_motion: int = 16) -> SceneVideo:
    """Scenes of ``scene_len`` frames with a hard cut between scenes.  Per scene:
    texture sigma ~ U(0, max_sigma) of Gaussian noise over a random linear
    gradient, global motion (dy, dx) ~ U{-max_motion..max_motion}^2 px/frame."""
    rng = make_rng(recipe, stream)
    scale = float(1 << (bit_depth - 8))
    n_scenes = (n_frames + scene_len - 1) // scene_len
    sv = SceneVideo(width, height, n_frames, bit_depth, scene_len)
    offsets = np.zeros((n_frames, 2), np.int64)
    for s in range(n_scenes):
        sigma = float(rng.uniform(0.0, max_sigma))
        dy, dx = (int(a) for a in rng.integers(-max_motion, max_motion + 1, size=2))
        frames_here = min(scene_len, n_frames - s * scene_len)
        travel_y, travel_x = abs(dy) * (frames_here - 1), abs(dx) * (frames_here - 1)
        Hc = height + travel_y + (travel_y & 1)
        Wc = width + travel_x + (travel_x & 1)
        yy, xx = np.mgrid[0:Hc, 0:Wc].astype(np.float32)
        a = float(rng.uniform(0.2, 0.8))
        lo, hi = float(rng.uniform(16, 80)), float(rng.uniform(160, 235))
        grad = lo + (hi - lo) * (a * xx / Wc + (1 - a) * yy / Hc)
        del yy, xx
        cy_ = grad + np.float32(sigma) * rng.standard_normal((Hc, Wc), dtype=np.float32)
        del grad
        canvas_y = _to_samples(cy_ * np.float32(scale), bit_depth)
        del cy_
        chroma = []
        ch, cw = Hc // 2, Wc // 2
        gy, gx = np.mgrid[0:ch, 0:cw].astype(np.float32)
        for _ in range(2):
            lx, ly = rng.uniform(80, 400, size=2)
            phi = rng.uniform(0, 2 * np.pi)
            f = 128.0 + 50.0 * np.sin(2 * np.pi * gx / lx + phi) * np.cos(2 * np.pi * gy / ly)
            f = f + np.float32(sigma / 2) * rng.standard_normal((ch, cw), dtype=np.float32)
            chroma.append(_to_samples(f * np.float32(scale), bit_depth))
        del gy, gx
        sv.canvases.append((canvas_y, chroma[0], chroma[1]))
        sv.params.append((sigma, dy, dx))
        oy0 = 0 if dy >= 0 else travel_y
        ox0 = 0 if dx >= 0 else travel_x
        for t in range(frames_here):
            offsets[s * scene_len + t] = (oy0 + dy * t, ox0 + dx * t)
    sv.offsets = offsets
    return sv


def _stress_plane(rng: np.random.Generator, h: int, w_: int, cell: int) -> np.ndarray:
    """One 10-bit plane tiled with cell x cell blocks of three kinds: 40%
    uniform noise in [0, 1023], 40% saturated edges (0 / 1023 split along a
    random line), 20% cosine-sign patterns (1023 where cos(pi l (2n+1)/(2 cell))
    >= 0 along rows, columns or both, else 0)."""
    nby, nbx = h // cell, w_ // cell
    out = rng.integers(0, 1024, size=(h, w_)).astype(np.uint16)
    kind = rng.choice(3, size=(nby, nbx), p=[0.4, 0.4, 0.2])
    yy, xx = np.mgrid[0:cell, 0:cell].astype(np.float64)
    theta = rng.uniform(0, 2 * np.pi, size=(nby, nbx))
    offs = rng.uniform(-cell / 3, cell / 3, size=(nby, nbx))
    freq = rng.integers(1, cell, size=(nby, nbx, 2))
    orient = rng.integers(0, 3, size=(nby, nbx))
    flip = rng.integers(0, 2, size=(nby, nbx))
    c = (cell - 1) / 2.0
    dist = (np.cos(theta)[..., None, None] * (xx - c) + np.sin(theta)[..., None, None] * (yy - c)
            - offs[..., None, None])
    edge = np.where(dist > 0, 1023, 0)
    ch = np.cos(np.pi * freq[..., 0, None, None] * (2 * xx + 1) / (2 * cell))
    cv = np.cos(np.pi * freq[..., 1, None, None] * (2 * yy + 1) / (2 * cell))
    o = orient[..., None, None]
    prod = np.where(o == 0, ch, np.where(o == 1, cv, ch * cv))
    sign = np.where((prod >= 0) ^ (flip[..., None, None] == 1), 1023, 0)
    k = kind[..., None, None]
    blocks = np.where(k == 1, edge, sign)                            # [nby, nbx, cell, cell]
    grid = blocks.transpose(0, 2, 1, 3).reshape(nby * cell, nbx * cell).astype(np.uint16)
    region = out[:nby * cell, :nbx * cell]
    mask = np.repeat(np.repeat(kind != 0, cell, axis=0), cell, axis=1)
    region[mask] = grid[mask]
    return out


def stress_video(width: int, height: int, n_frames: int, *, cell: int = 32,
                 recipe: int = 2, stream: int = 0) -> Video:
    """10-bit precision-stress frames (independent frames, no motion)."""
    rng = make_rng(recipe, stream)
    Y = np.stack([_stress_plane(rng, height, width, cell) for _ in range(n_frames)])
    U = np.stack([_stress_plane(rng, height // 2, width // 2, cell) for _ in range(n_frames)])
    V = np.stack([_stress_plane(rng, height // 2, width // 2, cell) for _ in range(n_frames)])
    return Video(Y, U, V, 10)


RESOLUTIONS = ((640, 360), (1280, 720), (1920, 1080), (2560, 1440), (3840, 2160))


def batch_streams(n_streams: int = 64, *, recipe: int = 3, min_frames: int = 30,
                  max_frames: int = 300, block_sizes=(8, 16, 32)):
    """Stream descriptors for the batched workload: per stream a resolution
    drawn uniformly from RESOLUTIONS, a block size from ``block_sizes`` and a
    frame count from [min_frames, max_frames].  Returns a list of dicts with
    keys width, height, block_size, n_frames, stream (the content seed)."""
    rng = make_rng(recipe, 0)
    out = []
    for s in range(n_streams):
        W, H = RESOLUTIONS[int(rng.integers(0, len(RESOLUTIONS)))]
        out.append(dict(width=W, height=H, block_size=int(rng.choice(block_sizes)),
                        n_frames=int(rng.integers(min_frames, max_frames + 1)), stream=s + 1))
    return out


def soft_frames(x: np.ndarray, *, recipe: int = 5, stream: int = 0) -> np.ndarray:
    """Non-integer frames from frames x [..., H, W]: each frame blurred along
    columns and rows with a seeded 3-tap kernel [a, 1, a] / (1 + 2a),
    a ~ U(0.1, 0.4) per frame and direction (edges replicated), so values
    stay in the input range and almost none is an integer.  Returned as
    float64 holding float32 values (what a float32 filter output is)."""
    rng = make_rng(recipe, stream)
    x = np.asarray(x, np.float64)
    flat = x.reshape(-1, *x.shape[-2:])
    out = np.empty_like(flat)
    for i, f in enumerate(flat):
        ay, ax = rng.uniform(0.1, 0.4, size=2)
        ky = np.array([ay, 1.0, ay]) / (1.0 + 2 * ay)
        kx = np.array([ax, 1.0, ax]) / (1.0 + 2 * ax)
        p = np.pad(f, 1, mode="edge")
        g = ky[0] * p[:-2, :] + ky[1] * p[1:-1, :] + ky[2] * p[2:, :]
        out[i] = kx[0] * g[:, :-2] + kx[1] * g[:, 1:-1] + kx[2] * g[:, 2:]
    return out.reshape(x.shape).astype(np.float32).astype(np.float64)
