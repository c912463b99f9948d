"""The paper's own low-pass option (2x downsampling, then the full w x w
transform) on the GPU against the oracle: features, and per block the exact
DC and the energy H."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_features_close, print_case, to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2304_12384_amd as vca_mod
    return vca_mod


CASES = [
    # (width, height, w, bit depth, frames)
    (1280, 720, 32, 8, 4),       # half size 640x360: luma 20x11 blocks, chroma 10x5
    (1920, 1080, 16, 8, 3),      # half 960x540: partial strips, 33.75 block rows
    (1344, 776, 8, 8, 3),        # half 672x388: w = 8, partial 32x32 tiles on both edges
    (1280, 720, 16, 10, 3),
    (1056, 600, 8, 10, 2),       # half 528x300
    (3840, 2160, 32, 8, 2),
]


def frames(width, height, B, n, seed):
    if B == 8:
        return synth.patches_video(width, height, n, stream=seed)
    return synth.stress_video(width, height, n, cell=16, stream=seed)


@pytest.mark.parametrize("case", CASES)
def test_downsampled_features_and_blocks_match_oracle(vca, case):
    W, H, w, B, n = case
    print_case(test="downsample", size=(W, H), w=w, bits=B, n=n)
    vid = frames(W, H, B, n, seed=40 + CASES.index(case))
    y, u, v = to_device(vid)
    an = vca.Analyzer(W, H, bit_depth=B, block_size=w, downsample=True, max_batch=n)
    an.submit(y, u, v)
    got = an.features(0, n)
    cfg = oracle.Config(W, H, B, w)
    ref = oracle.analyze_downsampled(cfg, vid.y, vid.u, vid.v, threads=8, want_blocks=True)
    assert_features_close(got, ref.features)
    for f in (0, n - 1):
        h, dc = an.block_stats(f)
        np.testing.assert_array_equal(dc, ref.block_dc[f])
        np.testing.assert_allclose(h, ref.block_h[f], rtol=1e-12, atol=0)
    an.close()


def test_downsampled_h_chains_across_calls_and_tunes(vca):
    W, H, w = 1280, 720, 32
    print_case(test="downsample_calls")
    vid = frames(W, H, 8, 6, seed=77)
    y, u, v = to_device(vid)
    an = vca.Analyzer(W, H, block_size=w, downsample=True, max_batch=4)
    choice = an.tune(y[:4], u[:4], v[:4], reps=1)
    assert choice["depth"] in (1, 2, 4)
    an.submit(y[:2], u[:2], v[:2])
    an.submit(y[2:], u[2:], v[2:])          # 4 frames in one launch after 2
    got = an.features(0, 6)
    an.close()
    ref = oracle.analyze_downsampled(oracle.Config(W, H, 8, w), vid.y, vid.u, vid.v, threads=8)
    assert_features_close(got, ref.features)
