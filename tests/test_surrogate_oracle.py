"""Pins of the FP64 surrogate used as the gradient reference: agreement with
the integer transform up to its rounding, invariances the definition fixes,
and central finite differences against its autograd gradient."""
import numpy as np
import pytest
import torch

import oracle
from oracle import surrogate


@pytest.mark.parametrize("w", [8, 16, 32])
@pytest.mark.parametrize("B", [8, 10])
def test_surrogate_close_to_integer_transform(w, B):
    """Unrounded C X C^T 2^-(s1+s2) differs from the two rounded passes by at
    most the propagated rounding: 1/2 in T scaled by sum|C|/2^s2, plus 1/2."""
    rng = np.random.default_rng(w + B)
    C = oracle.dct_matrix(w).astype(np.float64)
    s2 = int(np.log2(w)) + 6
    bound = 0.5 * np.abs(C).sum(axis=1).max() / 2 ** s2 + 0.5 + 1e-9
    for _ in range(10):
        X = rng.integers(0, 1 << B, size=(w, w))
        Ys = C @ X @ C.T * surrogate.scale(w, B)
        assert np.abs(Ys - oracle.block_transform(X, B)).max() <= bound


def frames(rng, b, t, h, w_):
    return torch.tensor(rng.integers(0, 256, size=(b, t, h, w_)).astype(np.float64))


@pytest.mark.parametrize("w", [8, 32])
def test_dc_invariance_and_homogeneity(w):
    rng = np.random.default_rng(1)
    x = frames(rng, 2, 3, 64, 96)
    E, h = surrogate.energy_features(x, w)
    E2, h2 = surrogate.energy_features(x + 37.5, w)       # constant shift: DC only
    E3, h3 = surrogate.energy_features(2.5 * x, w)        # |.| is positively homogeneous
    np.testing.assert_allclose(E2, E, rtol=1e-12)
    np.testing.assert_allclose(h2, h, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(E3, 2.5 * E, rtol=1e-12)
    np.testing.assert_allclose(h3, 2.5 * h, rtol=1e-12, atol=1e-12)
    assert (h[:, 0] == 0).all()


def test_gradient_sums_to_zero_per_block():
    """The DC direction carries no weight, so every block's gradient sums to 0."""
    rng = np.random.default_rng(2)
    x = rng.integers(0, 256, size=(1, 2, 64, 64)).astype(np.float64)
    _, _, g = surrogate.reference_gradient(x, np.ones((1, 2)), np.ones((1, 2)), w=16)
    sums = g.reshape(1, 2, 4, 16, 4, 16).sum(axis=(3, 5))
    assert np.abs(sums).max() < 1e-12 * np.abs(g).max() * 256


@pytest.mark.parametrize("w,k", [(32, None), (16, 8)])
def test_autograd_matches_central_differences(w, k):
    rng = np.random.default_rng(3)
    x = rng.integers(0, 256, size=(1, 2, 64, 64)).astype(np.float64)
    gE = rng.normal(size=(1, 2))
    gh = rng.normal(size=(1, 2))
    _, _, g = surrogate.reference_gradient(x, gE, gh, w=w, k=k)

    def loss(xv):
        E, h = surrogate.energy_features(torch.tensor(xv), w, k)
        return float((E.numpy() * gE).sum() + (h.numpy() * gh).sum())

    d = 1e-2
    checked = 0
    for _ in range(40):
        idx = tuple(int(rng.integers(0, s)) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += d
        xm[idx] -= d
        fd = (loss(xp) - loss(xm)) / (2 * d)
        # the loss is piecewise linear in one pixel: skip kinks inside [-d, d]
        xp2, xm2 = x.copy(), x.copy()
        xp2[idx] += d / 2
        xm2[idx] -= d / 2
        fd2 = (loss(xp2) - loss(xm2)) / d
        if abs(fd - fd2) > 1e-5 * (abs(fd) + 1e-9):
            continue
        assert fd == pytest.approx(g[idx], rel=1e-5, abs=1e-12)
        checked += 1
    assert checked >= 30


def test_single_frame_sequences_have_zero_h():
    rng = np.random.default_rng(4)
    x = frames(rng, 3, 1, 32, 64)
    E, h = surrogate.energy_features(x, 16)
    assert E.shape == h.shape == (3, 1)
    assert (h == 0).all() and (E > 0).all()
    _, _, g = surrogate.reference_gradient(x.numpy(), np.ones((3, 1)), np.ones((3, 1)), w=16)
    _, _, g_e = surrogate.reference_gradient(x.numpy(), np.ones((3, 1)), np.zeros((3, 1)), w=16)
    np.testing.assert_array_equal(g, g_e)      # h carries no gradient without a predecessor
