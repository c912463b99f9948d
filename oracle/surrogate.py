"""TEST INFRASTRUCTURE ONLY: FP64 reference of the differentiable luma
surrogate of the VCA texture energy E_Y and its gradient h (Section 2 of
Menon et al., GMSys 2023, names both features).

The paper's transform rounds; for gradients the rounding is dropped: per
w x w luma block X,
    Y = C X C^T * 2^-(s1 + s2),   s1 + s2 = 2 log2 w + B - 3,
the unrounded composition of the two integer passes, and
    H = sum_{(i,k) != (0,0), i,k < K} W_ik |Y_ik|,
    E = sum_blocks H / (C_Y w^2),
    h_t = sum_blocks |H_t - H_{t-1}| / (C_Y w^2),  h_0 = 0 within a sequence.
The subgradient of |.| at 0 is 0 (torch's sign(0) = 0).  Written with plain
PyTorch CPU ops in float64 so that autograd of this function is the
reference gradient.  Only the tests and the benchmark's CPU leg may import it.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import dct_matrix, weights


def scale(w: int, bit_depth: int = 8) -> float:
    return 2.0 ** -(2 * int(math.log2(w)) + bit_depth - 3)


def weight_mask(w: int, k: int | None = None) -> np.ndarray:
    """Energy weights with the DC weight and the weights outside K x K at 0."""
    K = w if not k else k
    W = weights(w).copy()
    W[0, 0] = 0.0
    W[K:, :] = 0.0
    W[:, K:] = 0.0
    return W


def block_energies(x: torch.Tensor, w: int, k: int | None = None, bit_depth: int = 8) -> torch.Tensor:
    """x: [..., H, W] float64 luma -> H: [..., nby, nbx] block energies."""
    nby, nbx = x.shape[-2] // w, x.shape[-1] // w
    xb = x[..., :nby * w, :nbx * w]
    xb = xb.reshape(*x.shape[:-2], nby, w, nbx, w).transpose(-3, -2)   # [..., nby, nbx, w, w]
    C = torch.as_tensor(dct_matrix(w), dtype=torch.float64)
    Y = C @ xb @ C.T * scale(w, bit_depth)
    Wm = torch.as_tensor(weight_mask(w, k), dtype=torch.float64)
    return (Wm * Y.abs()).sum(dim=(-2, -1))


def energy_features(x: torch.Tensor, w: int = 32, k: int | None = None, bit_depth: int = 8):
    """x: [B, T, H, W] float64.  Returns (E, h), each [B, T]."""
    Hb = block_energies(x, w, k, bit_depth)
    cy = Hb.shape[-1] * Hb.shape[-2]
    norm = 1.0 / (cy * w * w)
    E = Hb.sum(dim=(-2, -1)) * norm
    dh = (Hb[:, 1:] - Hb[:, :-1]).abs().sum(dim=(-2, -1)) * norm
    h = torch.cat([torch.zeros_like(E[:, :1]), dh], dim=1)     # no predecessor: h = 0
    return E, h


def reference_gradient(x: np.ndarray, gE: np.ndarray, gh: np.ndarray, w: int = 32,
                       k: int | None = None, bit_depth: int = 8):
    """Autograd (float64) of sum(gE * E + gh * h) with respect to x."""
    xt = torch.tensor(np.asarray(x, np.float64), requires_grad=True)
    E, h = energy_features(xt, w, k, bit_depth)
    loss = (E * torch.as_tensor(gE, dtype=torch.float64)).sum() + \
           (h * torch.as_tensor(gh, dtype=torch.float64)).sum()
    loss.backward()
    return E.detach().numpy(), h.detach().numpy(), xt.grad.numpy()
