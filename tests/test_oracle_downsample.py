"""Pins of the 2x-downsampling low-pass oracle (Section 2, optimisation (3),
with the 2 x 2 round-half-up mean as the reading of the unstated filter)."""
import numpy as np
import pytest

import oracle


def brute_downsample(p):
    """Pure-Python loops over one 2-D plane."""
    H, W = p.shape
    out = np.zeros((H // 2, W // 2), p.dtype)
    for y in range(H // 2):
        for x in range(W // 2):
            s = int(p[2 * y, 2 * x]) + int(p[2 * y, 2 * x + 1]) + int(p[2 * y + 1, 2 * x]) \
                + int(p[2 * y + 1, 2 * x + 1])
            out[y, x] = (s + 2) // 4
    return out


@pytest.mark.parametrize("dtype,top", [(np.uint8, 255), (np.uint16, 1023)])
def test_downsample_matches_loops_and_rounds_half_up(dtype, top):
    rng = np.random.default_rng(3)
    p = rng.integers(0, top + 1, size=(14, 22)).astype(dtype)
    np.testing.assert_array_equal(oracle.downsample(p), brute_downsample(p))
    # sums 4k + 2 round up, 4k + 1 down
    two = np.array([[0, 1], [0, 1]], dtype)      # sum 2 -> 1
    one = np.array([[0, 1], [0, 0]], dtype)      # sum 1 -> 0
    three = np.array([[1, 1], [0, 1]], dtype)    # sum 3 -> 1
    assert oracle.downsample(two)[0, 0] == 1 and oracle.downsample(one)[0, 0] == 0
    assert oracle.downsample(three)[0, 0] == 1
    full = np.full((2, 2), top, dtype)
    assert oracle.downsample(full)[0, 0] == top   # no overflow at the top of the range


def upsample(p):
    return np.repeat(np.repeat(p, 2, axis=-2), 2, axis=-1)


@pytest.mark.parametrize("w,B", [(32, 8), (16, 10), (8, 8)])
def test_downsampled_analysis_of_an_upsampled_video_is_the_plain_analysis(w, B):
    """Duplicating every sample 2 x 2 and downsampling gives the original
    back, so the features equal the plain analysis of the original."""
    rng = np.random.default_rng(w + B)
    top = (1 << B) - 1
    dt = np.uint8 if B == 8 else np.uint16
    W, H, n = 128, 96, 3
    y = rng.integers(0, top + 1, size=(n, H, W)).astype(dt)
    u = rng.integers(0, top + 1, size=(n, H // 2, W // 2)).astype(dt)
    v = rng.integers(0, top + 1, size=(n, H // 2, W // 2)).astype(dt)
    small = oracle.Config(W, H, B, w)
    big = oracle.Config(2 * W, 2 * H, B, w)
    ref = oracle.analyze(small, y, u, v, want_blocks=True)
    got = oracle.analyze_downsampled(big, upsample(y), upsample(u), upsample(v), want_blocks=True)
    np.testing.assert_array_equal(got.features, ref.features)
    np.testing.assert_array_equal(got.block_dc, ref.block_dc)
    np.testing.assert_array_equal(got.block_h, ref.block_h)


def test_constant_video_after_downsampling():
    """A constant plane stays constant: E = h = 0 and L as for the constant."""
    W, H = 256, 128
    y = np.full((2, H, W), 90, np.uint8)
    u = np.full((2, H // 2, W // 2), 130, np.uint8)
    v = np.full((2, H // 2, W // 2), 20, np.uint8)
    got = oracle.analyze_downsampled(oracle.Config(W, H, 8, 16), y, u, v).features
    ref = oracle.analyze(oracle.Config(W // 2, H // 2, 8, 16), y[:, ::2, ::2], u[:, ::2, ::2],
                         v[:, ::2, ::2]).features
    np.testing.assert_array_equal(got, ref)
    assert (got[:, [0, 1, 3, 4]] == 0).all()


def test_block_counts_of_the_half_size_video():
    cfg = oracle.Config(3840, 2160, 8, 32)
    half = oracle.Config(1920, 1080, 8, 32)
    assert oracle.block_counts(half) == (60 * 33, 30 * 16, 30 * 16)
    with pytest.raises(oracle.OracleError):
        oracle.analyze_downsampled(oracle.Config(130, 64, 8, 8), np.zeros((1, 64, 130), np.uint8),
                                   np.zeros((1, 32, 65), np.uint8), np.zeros((1, 32, 65), np.uint8))
