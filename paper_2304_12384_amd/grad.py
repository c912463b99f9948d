"""Differentiable luma texture energy E_Y and gradient h (Section 2 of the
paper names both features) as a ``torch.autograd.Function``.

Forward and backward run in the HIP library (``vca_energy_forward`` and
``vca_energy_backward`` of include/vca.h) on the caller's current stream;
this module only marshals tensors.  The features are those of the block
transform with its two roundings dropped (scale 2^-(2 log2 w + B - 3)), so
they are piecewise linear in the samples and the backward is
C^T (W o sign(Y)) C per block, with sign(0) = 0.  The forward keeps the
coefficient signs in its workspace; the backward reads those, not x.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import VcaGradConfig, check


def _config(x: torch.Tensor, block_size: int, lowpass_k: int, bit_depth: int) -> VcaGradConfig:
    n_seq, seq_len, height, width = x.shape
    return VcaGradConfig(ctypes.sizeof(VcaGradConfig), width, height, block_size, lowpass_k,
                         bit_depth, n_seq, seq_len, x.device.index, x.stride(2), x.stride(1))


def _prepare(x: torch.Tensor) -> torch.Tensor:
    """[B, T, H, W] float32 on the device, rows 16-byte aligned, frames dense
    along T (padding the row pitch to a multiple of 4 floats if needed)."""
    if x.dim() != 4:
        raise ValueError("x must be [batch, frames, height, width]")
    if not x.is_cuda or x.dtype != torch.float32:
        raise ValueError("x must be a float32 device tensor")
    B, T, H, W = x.shape
    pitch = (W + 3) // 4 * 4
    ok = (x.stride(3) == 1 and x.stride(2) == pitch and x.stride(1) == H * pitch
          and x.stride(0) == T * H * pitch and x.data_ptr() % 16 == 0)
    if ok:
        return x
    buf = torch.empty(B, T, H, pitch, device=x.device, dtype=torch.float32)
    buf[..., :W].copy_(x)
    return buf[..., :W]


class VCAEnergyFn(torch.autograd.Function):
    """(E, h) = VCAEnergyFn.apply(x, block_size, lowpass_k, bit_depth);
    x: [B, T, H, W] float32 luma, E and h: [B, T] float32 (h[:, 0] = 0)."""

    @staticmethod
    def forward(ctx, x, block_size=32, lowpass_k=0, bit_depth=8):
        xp = _prepare(x.detach())
        cfg = _config(xp, block_size, lowpass_k, bit_depth)
        L = _lib.lib()
        n_ws = L.vca_grad_workspace(ctypes.byref(cfg))   # bytes
        if n_ws < 0:
            raise ValueError(f"unsupported configuration {tuple(x.shape)}, w={block_size}, "
                             f"K={lowpass_k}, B={bit_depth}")
        B, T = x.shape[:2]
        E = torch.empty(B, T, device=x.device, dtype=torch.float32)
        h = torch.empty(B, T, device=x.device, dtype=torch.float32)
        ws = torch.empty(n_ws, device=x.device, dtype=torch.uint8)
        if ws.data_ptr() % 256:
            raise RuntimeError("workspace allocation is not 256-byte aligned")
        stream = torch.cuda.current_stream(x.device).cuda_stream
        check(L.vca_energy_forward(ctypes.byref(cfg), xp.data_ptr(), E.data_ptr(), h.data_ptr(),
                                   ws.data_ptr(), stream), "vca_energy_forward")
        ctx.save_for_backward(xp, ws)
        ctx.geom = (block_size, lowpass_k, bit_depth)
        return E, h

    @staticmethod
    def backward(ctx, gE, gh):
        xp, ws = ctx.saved_tensors
        block_size, lowpass_k, bit_depth = ctx.geom
        B, T = xp.shape[:2]
        gE = (torch.zeros(B, T, device=xp.device) if gE is None else gE).float().contiguous()
        gh = (torch.zeros(B, T, device=xp.device) if gh is None else gh).float().contiguous()
        cfg = _config(xp, block_size, lowpass_k, bit_depth)
        gx = torch.empty(xp.shape[:3] + (xp.stride(2),), device=xp.device, dtype=torch.float32)
        stream = torch.cuda.current_stream(xp.device).cuda_stream
        check(_lib.lib().vca_energy_backward(ctypes.byref(cfg), ws.data_ptr(), gE.data_ptr(),
                                             gh.data_ptr(), gx.data_ptr(), stream),
              "vca_energy_backward")
        return gx[..., :xp.shape[3]], None, None, None


def energy_features(x: torch.Tensor, block_size: int = 32, lowpass_k: int = 0,
                    bit_depth: int = 8):
    """Differentiable (E_Y, h) of x: [B, T, H, W] float32 luma on the GPU."""
    return VCAEnergyFn.apply(x, block_size, lowpass_k, bit_depth)
