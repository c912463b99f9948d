"""The allocation-free entry point (vca_analyze_noalloc) against the context
path (vca_open / vca_analyze_frames / vca_features) on the same frames.

Both run the same kernels, so the features must agree bit for bit (the bar
for them is 1e-5 relative against the oracle; equality is stronger).  Two
calls in a row, the second smaller, so the second call starts from the
first call's leftovers in the shared device array; the first call spans two
internal launches, so h crosses a launch boundary inside the array.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from synth.device import generated_scene_video
from tests.gpu_util import assert_features_close, print_case, to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2304_12384_amd as vca_mod
    return vca_mod


def frames_per_launch(width, height, w):
    """Frames one internal launch holds (the header's sizing rule)."""
    cy = (width // w) * (height // w)
    total = cy + 2 * ((width // 2 // w) * (height // 2 // w))
    state = (8 * cy + 255) // 256 * 256
    avail = (32 << 20) - 9 * (16 << 10) - 2 * state
    return avail // (12 * total + 256)


def context_features(vca, planes, *, bit_depth=8, w=32, k=0):
    y, u, v = planes
    an = vca.Analyzer(y.shape[2], y.shape[1], bit_depth=bit_depth, block_size=w, lowpass_k=k)
    feats = an.analyze(y, u, v)
    an.close()
    return feats


def noalloc_features(vca, planes, *, bit_depth=8, w=32, k=0):
    from paper_2304_12384_amd.analyzer import analyze_noalloc
    y, u, v = planes
    out = torch.full((y.shape[0], 7), float("nan"), dtype=torch.float32, device=y.device)
    analyze_noalloc(y, u, v, out, bit_depth=bit_depth, block_size=w, lowpass_k=k)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_two_calls_second_smaller(vca):
    # call 1: 2160p, w = 8, more frames than one launch holds
    per_launch = frames_per_launch(3840, 2160, 8)
    n1 = per_launch + 7
    print_case(test="noalloc", call=1, res="3840x2160", w=8, frames=n1, per_launch=per_launch)
    big = generated_scene_video(3840, 2160, n1, seed=7, scene_len=per_launch + 3)
    ref1 = context_features(vca, big.planes(), w=8)
    got1 = noalloc_features(vca, big.planes(), w=8)
    assert np.isfinite(got1).all()
    assert got1.tobytes() == ref1.tobytes()
    assert got1[0, 1] == 0.0 and (got1[1:, 1] > 0).any()
    del big
    # call 2: smaller (720p, w = 32, K = 16, 6 frames), also against the oracle
    video = synth.patches_video(1280, 720, 6)
    print_case(test="noalloc", call=2, res="1280x720", w=32, k=16, frames=6)
    planes = to_device(video)
    ref2 = context_features(vca, planes, k=16)
    got2 = noalloc_features(vca, planes, k=16)
    assert got2.tobytes() == ref2.tobytes()
    orc = oracle.analyze(oracle.Config(1280, 720, 8, 32, 16), video.y, video.u, video.v).features
    assert_features_close(got2, orc)


def test_10bit_after_8bit(vca):
    video = synth.stress_video(1920, 1080, 3)
    planes = to_device(video)
    print_case(test="noalloc", res="1920x1080", bits=10, w=16, frames=3)
    ref = context_features(vca, planes, bit_depth=10, w=16)
    got = noalloc_features(vca, planes, bit_depth=10, w=16)
    assert got.tobytes() == ref.tobytes()
    orc = oracle.analyze(oracle.Config(1920, 1080, 10, 16, 0), video.y, video.u, video.v).features
    assert_features_close(got, orc)


def test_rejections(vca):
    from paper_2304_12384_amd import _lib
    L = _lib.lib()
    y = torch.zeros((1, 64, 64), dtype=torch.uint8, device="cuda")
    u = torch.zeros((1, 32, 32), dtype=torch.uint8, device="cuda")
    out = torch.zeros((1, 7), dtype=torch.float32, device="cuda")
    fr = _lib.VcaFrames(y.data_ptr(), u.data_ptr(), u.data_ptr(), 64, 32, 64 * 64, 32 * 32, 1)
    for flags in (_lib.VCA_F_KEEP_COEFFS, _lib.VCA_F_VALIDATE, _lib.VCA_F_TIMING):
        cfg = _lib.VcaConfig(ctypes.sizeof(_lib.VcaConfig), 64, 64, 8, 420, 8, 0, 0, flags, 0, 0)
        assert L.vca_analyze_noalloc(ctypes.byref(cfg), ctypes.byref(fr), 1,
                                     ctypes.c_void_p(out.data_ptr()), None) == _lib.VCA_ERR_UNSUPPORTED
    cfg = _lib.VcaConfig(ctypes.sizeof(_lib.VcaConfig), 64, 64, 8, 420, 8, 0, 0, 0, 0, 0)
    misaligned = ctypes.c_void_p(out.data_ptr() + 2)
    assert L.vca_analyze_noalloc(ctypes.byref(cfg), ctypes.byref(fr), 1, misaligned,
                                 None) == _lib.VCA_ERR_INVALID_ARG
    host = _lib.VcaFrames(y.data_ptr(), u.data_ptr(), u.data_ptr(), 64, 32, 64 * 64, 32 * 32, 0)
    assert L.vca_analyze_noalloc(ctypes.byref(cfg), ctypes.byref(host), 1,
                                 ctypes.c_void_p(out.data_ptr()), None) == _lib.VCA_ERR_INVALID_ARG
