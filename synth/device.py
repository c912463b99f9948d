"""Builds synthetic frames in device memory from ``SceneVideo`` canvases.

Only data movement (uploads and slicing copies with torch) and input
filtering; no analysis arithmetic.  Frame t of the result equals
``SceneVideo.frame(t)``.
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass
class DeviceVideo:
    y: "object"      # torch tensor [n, H, W]
    u: "object"      # torch tensor [n, H/2, W/2]
    v: "object"
    bit_depth: int

    def planes(self, t0: int = 0, t1: int | None = None):
        t1 = self.y.shape[0] if t1 is None else t1
        return self.y[t0:t1], self.u[t0:t1], self.v[t0:t1]

    @property
    def n_frames(self) -> int:
        return self.y.shape[0]

    @property
    def nbytes(self) -> int:
        return sum(p.numel() * p.element_size() for p in (self.y, self.u, self.v))


def scene_to_device(sv, device="cuda", t0: int = 0, t1: int | None = None) -> DeviceVideo:
    import torch
    t1 = sv.n_frames if t1 is None else t1
    n = t1 - t0
    dt = torch.uint8 if sv.bit_depth == 8 else torch.int16
    H, W = sv.height, sv.width
    y = torch.empty((n, H, W), dtype=dt, device=device)
    u = torch.empty((n, H // 2, W // 2), dtype=dt, device=device)
    v = torch.empty((n, H // 2, W // 2), dtype=dt, device=device)
    cache = {}
    for t in range(t0, t1):
        s = sv.scene_of(t)
        if s not in cache:
            cache.clear()
            cache[s] = [torch.from_numpy(c.view("int16") if c.dtype.itemsize == 2 else c).to(device)
                        for c in sv.canvases[s]]
        cy, cu, cv = cache[s]
        oy, ox = (int(a) for a in sv.offsets[t])
        y[t - t0].copy_(cy[oy:oy + H, ox:ox + W])
        u[t - t0].copy_(cu[oy // 2:oy // 2 + H // 2, ox // 2:ox // 2 + W // 2])
        v[t - t0].copy_(cv[oy // 2:oy // 2 + H // 2, ox // 2:ox // 2 + W // 2])
    return DeviceVideo(y, u, v, sv.bit_depth)


def generated_scene_video(width: int, height: int, n_frames: int, *, seed: int,
                          scene_len: int = 120, max_sigma: float = 60.0, max_motion: int = 16,
                          device="cuda") -> DeviceVideo:
    """8-bit scene video generated directly in device memory (for workloads too
    large to draw on the host): the recipe of ``scene_video`` -- per scene a
    noisy random gradient canvas (sigma ~ U(0, max_sigma)) cropped along a
    constant global motion (|dx|, |dy| <= max_motion px/frame), a hard cut
    every ``scene_len`` frames -- with torch's generator seeded by ``seed``.
    Frames are inputs only; a host check copies the frames it needs back."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    H, W = height, width
    y = torch.empty((n_frames, H, W), dtype=torch.uint8, device=device)
    u = torch.empty((n_frames, H // 2, W // 2), dtype=torch.uint8, device=device)
    v = torch.empty((n_frames, H // 2, W // 2), dtype=torch.uint8, device=device)

    def rand(*shape):
        return torch.rand(shape, generator=g, device=device)

    for s0 in range(0, n_frames, scene_len):
        frames_here = min(scene_len, n_frames - s0)
        sigma = float(rand(1)) * max_sigma
        dy, dx = (int(a) for a in (rand(2) * (2 * max_motion + 1)).floor().long() - max_motion)
        ty, tx = abs(dy) * (frames_here - 1), abs(dx) * (frames_here - 1)
        Hc, Wc = H + ty + (ty & 1), W + tx + (tx & 1)
        a = 0.2 + 0.6 * float(rand(1))
        lo, hi = 16 + 64 * float(rand(1)), 160 + 75 * float(rand(1))
        yy = torch.arange(Hc, device=device, dtype=torch.float32)[:, None] / Hc
        xx = torch.arange(Wc, device=device, dtype=torch.float32)[None, :] / Wc
        cy = lo + (hi - lo) * (a * xx + (1 - a) * yy)
        cy = cy + sigma * torch.randn((Hc, Wc), generator=g, device=device)
        canvas_y = cy.round_().clamp_(0, 255).to(torch.uint8)
        del cy
        ch, cw = Hc // 2, Wc // 2
        gy = torch.arange(ch, device=device, dtype=torch.float32)[:, None]
        gx = torch.arange(cw, device=device, dtype=torch.float32)[None, :]
        canv_c = []
        for _ in range(2):
            lx, ly = (80 + 320 * rand(2)).tolist()
            phi = float(rand(1)) * 6.283185307
            f = 128.0 + 50.0 * torch.sin(6.283185307 * gx / lx + phi) * torch.cos(6.283185307 * gy / ly)
            f = f + (sigma / 2) * torch.randn((ch, cw), generator=g, device=device)
            canv_c.append(f.round_().clamp_(0, 255).to(torch.uint8))
        oy0 = 0 if dy >= 0 else ty
        ox0 = 0 if dx >= 0 else tx
        for t in range(frames_here):
            oy, ox = oy0 + dy * t, ox0 + dx * t
            y[s0 + t].copy_(canvas_y[oy:oy + H, ox:ox + W])
            u[s0 + t].copy_(canv_c[0][oy // 2:oy // 2 + H // 2, ox // 2:ox // 2 + W // 2])
            v[s0 + t].copy_(canv_c[1][oy // 2:oy // 2 + H // 2, ox // 2:ox // 2 + W // 2])
        del canvas_y, canv_c
    return DeviceVideo(y, u, v, 8)


def soft_device_frames(x, seed: int):
    """Device analogue of ``video.soft_frames``: float32 frames [..., H, W]
    blurred along rows and columns with a 3-tap kernel whose side weight is
    drawn per frame from torch's generator seeded by ``seed``."""
    import torch
    g = torch.Generator(device=x.device)
    g.manual_seed(seed)
    shape = x.shape
    f = x.reshape(-1, 1, *shape[-2:]).float()
    a = 0.1 + 0.3 * torch.rand((f.shape[0], 2), generator=g, device=x.device)
    out = torch.empty_like(f)
    for i in range(f.shape[0]):
        ay, ax = float(a[i, 0]), float(a[i, 1])
        ky = torch.tensor([ay, 1.0, ay], device=x.device) / (1.0 + 2 * ay)
        kx = torch.tensor([ax, 1.0, ax], device=x.device) / (1.0 + 2 * ax)
        p = torch.nn.functional.pad(f[i:i + 1], (1, 1, 1, 1), mode="replicate")
        p = torch.nn.functional.conv2d(p, ky.view(1, 1, 3, 1))
        out[i:i + 1] = torch.nn.functional.conv2d(p, kx.view(1, 1, 1, 3))
    return out.reshape(shape).contiguous()
