"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Bar: every DCT coefficient and block DC bit-exact, block energies H within
1e-12 relative (both FP64), the seven features within 1e-5 relative (exact
zero where the oracle gives zero).
"""
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


def run_gpu(vca, video, *, k=0, w=32, keep=False, max_batch=0, splits=None):
    an = vca.Analyzer(video.width, video.height, bit_depth=video.bit_depth, block_size=w,
                      lowpass_k=k, keep_coeffs=keep, max_batch=max_batch)
    y, u, v = to_device(video)
    n = video.n_frames
    splits = splits or [n]
    t0 = 0
    coeffs, stats = [], []
    for part in splits:
        an.submit(y[t0:t0 + part], u[t0:t0 + part], v[t0:t0 + part])
        if keep:
            coeffs += [an.block_coeffs(t0 + i) for i in range(part)]
        t0 += part
    feats = an.features(0, n)
    if keep:
        stats = [an.block_stats(i) for i in range(n - splits[-1], n)]
    an.close()
    return feats, coeffs, stats


def oracle_run(video, *, k=0, w=32, threads=8, coeffs=False):
    cfg = oracle.Config(video.width, video.height, video.bit_depth, w, k)
    return oracle.analyze(cfg, video.y, video.u, video.v, threads=threads, want_blocks=True,
                          want_coeffs=coeffs)


@pytest.mark.parametrize("k", [0, 16, 8])
def test_patches_720p_bit_exact(vca, patches, k):
    print_case(test="patches_720p", k=k, frames=patches.n_frames)
    ref = oracle_run(patches, k=k, coeffs=True)
    feats, coeffs, stats = run_gpu(vca, patches, k=k, keep=True, max_batch=16)
    for t in range(patches.n_frames):
        assert (coeffs[t].astype(np.int32) == ref.coeffs[t]).all(), f"coefficients differ, frame {t}"
    for t, (h, dc) in enumerate(stats):
        assert (dc == ref.block_dc[t]).all()
        np.testing.assert_allclose(h, ref.block_h[t], rtol=1e-12, atol=0)
    assert_features_close(feats, ref.features)


def test_scene_cut_2160p_bit_exact(vca):
    sv = synth.scene_video(3840, 2160, 122)
    video = sv.frames(118, 122)                  # crosses the hard cut at frame 120
    for k in (0, 16):
        print_case(test="scene_cut_2160p", k=k)
        ref = oracle_run(video, k=k, coeffs=True)
        feats, coeffs, _ = run_gpu(vca, video, k=k, keep=True, max_batch=4)
        for t in range(video.n_frames):
            assert (coeffs[t].astype(np.int32) == ref.coeffs[t]).all(), f"frame {t}, k={k}"
        assert_features_close(feats, ref.features)


@pytest.fixture(scope="module")
def uhd600():
    """The 600-frame 2160p workload the benchmark times, once on the host (for
    the oracle) and once on the device."""
    from synth.device import scene_to_device
    sv = synth.scene_video(3840, 2160, 600)
    return sv, scene_to_device(sv)


@pytest.mark.parametrize("mode", ["full", "k16", "downsample"])
def test_2160p_bench_launch_sampled(vca, uhd600, mode):
    """600 UHD frames in the benchmark's launch configuration (one launch,
    tuned as the benchmark tunes it) for each mode it times: full DCT,
    low-pass K = 16 and the paper's 2x downsampled low-pass.  Sampled frames
    (around every scene cut, first and last) checked against the oracle:
    features to 1e-5, every block's DC bit-exact and H to 1e-12."""
    sv, buf = uhd600
    k = 16 if mode == "k16" else 0
    ds = mode == "downsample"
    an = vca.Analyzer(3840, 2160, block_size=32, lowpass_k=k, max_batch=600, downsample=ds)
    print_case(test="bench_launch_600x2160p", mode=mode)
    an.tune(*buf.planes(), reps=1)
    an.submit(*buf.planes())
    feats = an.features(an.submitted - 600, 600)
    first = an.submitted - 600
    sampled = (0, 1, 119, 120, 121, 240, 359, 480, 599)
    maps = {t: an.block_maps(first + t, 1) for t in sampled}
    torch.cuda.synchronize()
    an.close()
    for t in sampled:
        t0 = max(0, t - 1)
        v = sv.frames(t0, t + 1)
        if ds:
            cfg = oracle.Config(3840, 2160, 8, 32, 0)
            ref = oracle.analyze_downsampled(cfg, v.y, v.u, v.v, threads=8, want_blocks=True)
        else:
            ref = oracle_run(v, k=k, threads=8)
        assert_features_close(feats[t:t + 1], ref.features[-1][None])
        assert (maps[t]["dc"].cpu().numpy()[0] == ref.block_dc[-1]).all(), f"frame {t}"
        np.testing.assert_allclose(maps[t]["h"].cpu().numpy()[0], ref.block_h[-1], rtol=1e-12, atol=0)


def test_call_boundaries_reset_and_chunking(vca, patches):
    print_case(test="call_boundaries")
    whole, _, _ = run_gpu(vca, patches)
    split, _, _ = run_gpu(vca, patches, splits=[3, 1, 6])
    chunked, _, _ = run_gpu(vca, patches, max_batch=3)
    assert (whole == split).all()
    assert (whole == chunked).all()
    an = vca.Analyzer(patches.width, patches.height)
    y, u, v = to_device(patches)
    an.submit(y[:4], u[:4], v[:4])
    an.reset()
    an.submit(y[4:], u[4:], v[4:])
    f = an.features(0, 10)
    an.close()
    assert f[4, 1] == 0.0
    assert (f[5:] == whole[5:]).all()
    assert (f[:4] == whole[:4]).all()


def test_features_read_while_later_calls_are_queued(vca, patches):
    """A feature read waits for the launch that produced the frames asked for,
    not for the whole stream: reading call i's frames after call i + 1 was
    queued gives call i's features, also with one launch per frame
    (max_batch 1) and for frames older than every launch the context still
    remembers (30 launches queued, frames 0-2 read last)."""
    print_case(test="features_pipelined")
    y, u, v = to_device(patches)
    for mb in (0, 1):
        ref_an = vca.Analyzer(patches.width, patches.height, max_batch=mb)
        for _ in range(3):
            ref_an.submit(y, u, v)
        ref = ref_an.features(0, 30)
        ref_an.close()
        an = vca.Analyzer(patches.width, patches.height, max_batch=mb)
        got, prev = [], None
        for _ in range(3):
            first = an.submit(y, u, v)
            if prev is not None:
                got.append(an.features(prev, 10))
            prev = first
        got.append(an.features(prev, 10))
        oldest = an.features(0, 3)
        an.close()
        assert np.concatenate(got).tobytes() == ref.tobytes(), f"max_batch {mb}"
        assert oldest.tobytes() == ref[:3].tobytes()


def test_static_sequence_and_determinism(vca, patches):
    print_case(test="static_sequence")
    rep = synth.Video(np.repeat(patches.y[:1], 5, 0), np.repeat(patches.u[:1], 5, 0),
                      np.repeat(patches.v[:1], 5, 0), 8)
    f, _, _ = run_gpu(vca, rep)
    assert (f[:, 1] == 0.0).all()
    assert (f == f[0]).all()
    a, _, _ = run_gpu(vca, patches)
    b, _, _ = run_gpu(vca, patches)
    assert a.tobytes() == b.tobytes()


@pytest.mark.parametrize("size", [(64, 64), (104, 72), (1000, 568), (1920, 1080)])
def test_small_and_ragged_frames(vca, size):
    width, height = size
    print_case(test="ragged", width=width, height=height)
    rng = np.random.default_rng(width + height)
    n = 3
    pitch = (width + 15) // 16 * 16 + 16          # padded pitch, 16-byte multiple
    cpitch = (width // 2 + 15) // 16 * 16 + 16
    y = rng.integers(0, 256, size=(n, height, pitch), dtype=np.uint8)
    u = rng.integers(0, 256, size=(n, height // 2, cpitch), dtype=np.uint8)
    v = rng.integers(0, 256, size=(n, height // 2, cpitch), dtype=np.uint8)
    yd, ud, vd = (torch.from_numpy(a).cuda() for a in (y, u, v))
    crop = synth.Video(y[:, :, :width], u[:, :, :width // 2], v[:, :, :width // 2], 8)
    for k in (0, 16):
        an = vca.Analyzer(width, height, lowpass_k=k, keep_coeffs=True, max_batch=n)
        an.submit(yd[:, :, :width], ud[:, :, :width // 2], vd[:, :, :width // 2])
        co = [an.block_coeffs(t) for t in range(n)]
        f = an.features(0, n)
        an.close()
        ref = oracle_run(crop, k=k, coeffs=True)
        for t in range(n):
            assert (co[t].astype(np.int32) == ref.coeffs[t]).all()
        assert_features_close(f, ref.features)


def test_argument_errors(vca, patches):
    from paper_2304_12384_amd import VcaError
    an = vca.Analyzer(patches.width, patches.height)
    y, u, v = to_device(patches)
    with pytest.raises(VcaError):                 # frames not yet submitted
        an.features(0, 1)
    wide = torch.zeros((2, 720, 1288), dtype=torch.uint8, device="cuda")
    with pytest.raises(VcaError):                 # pitch 1288 is not a 16-byte multiple
        an.submit(wide[:, :, :1280], u[:2], v[:2])
    an.submit(y[:2], u[:2], v[:2])
    with pytest.raises(VcaError):
        an.features(1, 2)
    assert an.features(0, 2).shape == (2, 7)
    with pytest.raises(VcaError):                 # not opened with keep_coeffs
        an.block_coeffs(0)
    an.close()


@pytest.mark.parametrize("w,k", [(32, 0), (16, 8), (8, 0)])
def test_8k_frames_strip_path(vca, w, k):
    """7680x4320 (the largest common frame size; 32 strips per luma tile
    row): every block's DC exact and H to 1e-12 through the production strip
    kernels, features to 1e-5."""
    print_case(test="8k", w=w, k=k)
    rng = np.random.default_rng(8000 + w + k)
    width, height, n = 7680, 4320, 2
    y = rng.integers(0, 256, size=(n, height, width), dtype=np.uint8)
    u = rng.integers(0, 256, size=(n, height // 2, width // 2), dtype=np.uint8)
    v = rng.integers(0, 256, size=(n, height // 2, width // 2), dtype=np.uint8)
    video = synth.Video(y, u, v, 8)
    an = vca.Analyzer(width, height, block_size=w, lowpass_k=k)
    an.submit(*to_device(video))
    f = an.features(0, n)
    maps = an.block_maps(0, n)
    torch.cuda.synchronize()
    an.close()
    ref = oracle_run(video, k=k, w=w)
    assert (maps["dc"].cpu().numpy() == ref.block_dc).all()
    np.testing.assert_allclose(maps["h"].cpu().numpy(), ref.block_h, rtol=1e-12, atol=0)
    assert_features_close(f, ref.features)


def test_empty_submission_is_a_no_op(vca, patches):
    print_case(test="empty_submission")
    an = vca.Analyzer(patches.width, patches.height)
    y, u, v = to_device(patches)
    assert an.submit(y[:0], u[:0], v[:0]) == 0
    assert an.submitted == 0
    an.submit(y, u, v)
    f = an.features(0, 10)
    assert an.submit_host(patches.y[:0], patches.u[:0], patches.v[:0]) == 10
    assert an.submitted == 10
    an.close()
    ref, _, _ = run_gpu(vca, patches)
    assert f.tobytes() == ref.tobytes()
