"""Builds synthetic frames in device memory from ``SceneVideo`` canvases.

Only data movement (uploads and slicing copies with torch); no analysis
arithmetic.  Frame t of the result equals ``SceneVideo.frame(t)``.
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
