"""Per-block feature maps (vca_block_maps) against the oracle's per-block
results: H and DC of every block, and |H_t - H_(t-1)| of every luma block,
the summand of h (Section 2 of the paper).

Bar: DC bit-exact, H within 1e-12 relative (both FP64), |dH| within 1e-12 of
the oracle's H scale, and the luma map summed and normalised equal to the
oracle's h within 1e-9 relative.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import print_case, to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2304_12384_amd as vca_mod
    return vca_mod


@pytest.fixture(scope="module")
def patches():
    return synth.patches_video()


def oracle_blocks(video, w, k):
    cfg = oracle.Config(video.width, video.height, video.bit_depth, w, k)
    return oracle.analyze(cfg, video.y, video.u, video.v, threads=8, want_blocks=True)


def check_maps(maps, ref, frames, prev_frame, c_y, w):
    """maps of `frames` (global indices); prev_frame[i] = index of the frame
    before frames[i] or None."""
    h = maps["h"].cpu().numpy()
    dc = maps["dc"].cpu().numpy()
    dh = maps["dh"].cpu().numpy()
    scale = ref.block_h[:, :c_y].max()
    for i, t in enumerate(frames):
        assert (dc[i] == ref.block_dc[t]).all(), f"DC differs, frame {t}"
        np.testing.assert_allclose(h[i], ref.block_h[t], rtol=1e-12, atol=0)
        p = prev_frame[i]
        want = np.zeros(c_y) if p is None else np.abs(ref.block_h[t, :c_y] - ref.block_h[p, :c_y])
        np.testing.assert_allclose(dh[i], want, rtol=0, atol=1e-12 * scale)
        # the map sums to the feature h
        h_feat = dh[i].sum() / (c_y * w * w)
        if ref.features[t, 1] == 0.0:
            assert h_feat == 0.0
        else:
            assert h_feat == pytest.approx(ref.features[t, 1], rel=1e-9)


@pytest.mark.parametrize("w,k", [(32, 0), (32, 16), (16, 0), (8, 4)])
def test_maps_across_calls(vca, patches, w, k):
    """Two calls (4 + 6 frames): the second call's first frame takes its
    previous luma H from the state the first call left."""
    print_case(test="block_maps", w=w, k=k)
    ref = oracle_blocks(patches, w, k)
    c_y = vca.block_counts(patches.width, patches.height, w, 8, k)[0]
    y, u, v = to_device(patches)
    an = vca.Analyzer(patches.width, patches.height, block_size=w, lowpass_k=k)
    an.submit(y[:4], u[:4], v[:4])
    first = an.submit(y[4:], u[4:], v[4:])
    maps = an.block_maps(first, 6)
    torch.cuda.synchronize()
    check_maps(maps, ref, list(range(4, 10)), [3, 4, 5, 6, 7, 8], c_y, w)
    # a sub-range
    sub = an.block_maps(first + 2, 3)
    torch.cuda.synchronize()
    check_maps(sub, ref, [6, 7, 8], [5, 6, 7], c_y, w)
    an.close()


def test_maps_first_frame_reset_and_chunks(vca, patches):
    print_case(test="block_maps_reset_chunks")
    ref = oracle_blocks(patches, 32, 0)
    c_y = vca.block_counts(patches.width, patches.height)[0]
    y, u, v = to_device(patches)
    # first frames after open: no previous frame
    an = vca.Analyzer(patches.width, patches.height)
    an.submit(y, u, v)
    maps = an.block_maps(0, 10)
    torch.cuda.synchronize()
    check_maps(maps, ref, list(range(10)), [None] + list(range(9)), c_y, 32)
    # after a reset the next frame has no previous frame either
    an.reset()
    an.submit(y[:3], u[:3], v[:3])
    maps = an.block_maps(10, 3)
    torch.cuda.synchronize()
    assert (maps["dh"][0] == 0).all()
    check_maps({"h": maps["h"][1:], "dc": maps["dc"][1:], "dh": maps["dh"][1:]}, ref, [1, 2], [0, 1],
               c_y, 32)
    an.close()
    # chunks of 3 frames: only the last launch (frame 9) is exported; its
    # previous frame comes from the state of the launch before
    an = vca.Analyzer(patches.width, patches.height, max_batch=3)
    an.submit(y, u, v)
    maps = an.block_maps(9, 1)
    torch.cuda.synchronize()
    check_maps(maps, ref, [9], [8], c_y, 32)
    with pytest.raises(vca.VcaError):
        an.block_maps(8, 1)
    with pytest.raises(vca.VcaError):
        an.block_maps(9, 2)
    an.close()


def test_maps_optional_outputs_and_argument_errors(vca, patches):
    print_case(test="block_maps_args")
    from paper_2304_12384_amd import _lib
    ref = oracle_blocks(patches, 32, 0)
    y, u, v = to_device(patches)
    an = vca.Analyzer(patches.width, patches.height)
    an.submit(y, u, v)
    total = sum(an.counts)
    dc = torch.zeros((2, total), dtype=torch.int32, device="cuda")
    L = _lib.lib()
    assert L.vca_block_maps(an._ctx, 3, 2, None, ctypes.c_void_p(dc.data_ptr()), None) == 0
    torch.cuda.synchronize()
    assert (dc.cpu().numpy() == ref.block_dc[3:5]).all()
    assert L.vca_block_maps(an._ctx, 3, 2, None, None, None) == _lib.VCA_ERR_INVALID_ARG
    assert L.vca_block_maps(an._ctx, 3, 0, None, ctypes.c_void_p(dc.data_ptr()), None) == \
        _lib.VCA_ERR_INVALID_ARG
    assert L.vca_block_maps(an._ctx, 3, 2, None, ctypes.c_void_p(dc.data_ptr() + 4), None) == \
        _lib.VCA_ERR_INVALID_ARG
    assert L.vca_block_maps(an._ctx, -1, 2, None, ctypes.c_void_p(dc.data_ptr()), None) == \
        _lib.VCA_ERR_STATE
    an.close()
