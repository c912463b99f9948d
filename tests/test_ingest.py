"""Host-resident frames and raw .yuv files through the staged ingest
(pinned double buffers, copies on a second stream) against the CPU oracle
-- features to 1e-5 (exact zeros), the last launch's block DC bit-exact and
H to 1e-12 -- and against the same frames analysed from device memory
(features bitwise equal), h chained across staging batches and calls."""
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


@pytest.fixture(scope="module")
def patches():
    return synth.patches_video()


def check_against_oracle(an, feats, video, first_frame, t0, t1, w=32):
    """Features of frames [t0, t1) of ``video`` (analysed as one sequence, the
    first at context frame ``first_frame``) and the block maps of the last
    analysed frame against the oracle."""
    cfg = oracle.Config(video.width, video.height, video.bit_depth, w, 0)
    ref = oracle.analyze(cfg, video.y[t0:t1], video.u[t0:t1], video.v[t0:t1], threads=8,
                         want_blocks=True)
    assert_features_close(feats, ref.features)
    last = first_frame + (t1 - t0) - 1
    maps = an.block_maps(last, 1)
    torch.cuda.synchronize()
    assert (maps["dc"].cpu().numpy()[0] == ref.block_dc[-1]).all()
    np.testing.assert_allclose(maps["h"].cpu().numpy()[0], ref.block_h[-1], rtol=1e-12, atol=0)
    if t1 - t0 > 1:
        cy = maps["dh"].shape[1]   # luma blocks come first
        dh_ref = np.abs(ref.block_h[-1][:cy] - ref.block_h[-2][:cy])
        # both energies within 1e-12 relative: the difference within 2e-12 of the larger
        np.testing.assert_allclose(maps["dh"].cpu().numpy()[0], dh_ref, rtol=0,
                                   atol=2e-12 * ref.block_h[-2:, :cy].max())


def device_features(vca, video, first=0, count=None, **kw):
    count = video.n_frames - first if count is None else count
    an = vca.Analyzer(video.width, video.height, bit_depth=video.bit_depth, **kw)
    y, u, v = to_device(video)
    an.submit(y[first:first + count], u[first:first + count], v[first:first + count])
    f = an.features(0, count)
    an.close()
    return f


@pytest.mark.parametrize("max_batch", [3, 0])
def test_host_frames_match_device_frames(vca, patches, max_batch):
    """max_batch 3: four staging batches of at most 3 frames through two slots."""
    print_case(test="ingest_host", max_batch=max_batch)
    ref = device_features(vca, patches)
    an = vca.Analyzer(patches.width, patches.height, max_batch=max_batch)
    an.submit_host(patches.y[:4], patches.u[:4], patches.v[:4])
    an.submit_host(patches.y[4:], patches.u[4:], patches.v[4:])   # h chains across calls
    f = an.features(0, 10)
    check_against_oracle(an, f, patches, 0, 0, 10)
    an.close()
    assert f.tobytes() == ref.tobytes()


def test_host_frames_with_row_padding_and_10_bit(vca):
    print_case(test="ingest_host_strided_10bit")
    video = synth.stress_video(256, 128, 5)
    ref = device_features(vca, video, block_size=16)
    # planes inside wider rows (pitch 256 + 40 samples) and reused buffers
    pad = lambda p: np.pad(p, ((0, 0), (0, 0), (0, 40)))[:, :, :p.shape[2]]
    y, u, v = pad(video.y), pad(video.u), pad(video.v)
    assert y.strides[1] != y.shape[2] * 2
    an = vca.Analyzer(video.width, video.height, bit_depth=10, block_size=16, max_batch=2)
    an.submit_host(y, u, v)
    f = an.features(0, 5)
    check_against_oracle(an, f, video, 0, 0, 5, w=16)
    an.close()
    assert f.tobytes() == ref.tobytes()


def test_yuv_file_matches_device_frames(vca, patches, tmp_path):
    print_case(test="ingest_file")
    path = str(tmp_path / "patches.yuv")
    vca.write_yuv(path, patches.y, patches.u, patches.v)
    ref = device_features(vca, patches, first=2, count=7)
    an = vca.Analyzer(patches.width, patches.height, max_batch=4)
    first = an.submit_file(path, first=2, count=7)
    f = an.features(first, 7)
    check_against_oracle(an, f, patches, first, 2, 9)
    # the rest of the file after a reset
    an.reset()
    first = an.submit_file(path, first=9)
    g = an.features(first, 1)
    check_against_oracle(an, g, patches, first, 9, 10)
    an.close()
    assert f.tobytes() == ref.tobytes()
    assert g.tobytes() == device_features(vca, patches, first=9, count=1).tobytes()


def test_ingest_errors(vca, patches, tmp_path):
    print_case(test="ingest_errors")
    path = str(tmp_path / "short.yuv")
    vca.write_yuv(path, patches.y[:2], patches.u[:2], patches.v[:2])
    an = vca.Analyzer(patches.width, patches.height)
    with pytest.raises(vca.VcaError):
        an.submit_file(path, first=1, count=2)
    with pytest.raises(vca.VcaError):
        an.submit_file(str(tmp_path / "missing.yuv"), count=1)
    assert an.submitted == 0
    an.close()
    keep = vca.Analyzer(patches.width, patches.height, keep_coeffs=True, max_batch=4)
    with pytest.raises(vca.VcaError):
        keep.submit_host(patches.y[:2], patches.u[:2], patches.v[:2])
    keep.close()
