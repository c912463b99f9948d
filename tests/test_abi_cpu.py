"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/vca.h declares, and rejects bad configurations before it
touches a device."""
import ctypes
import os
import re

import pytest

from paper_2304_12384_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "vca.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vca_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert names, "no declarations parsed"
    assert sorted(_lib.EXPORTS) == names
    L = _lib.lib()
    for n in names:
        assert getattr(L, n) is not None


def test_header_structs_match_binding():
    assert ctypes.sizeof(_lib.VcaConfig) == 44
    assert ctypes.sizeof(_lib.VcaFrameFeatures) == 28
    assert ctypes.sizeof(_lib.VcaFrames) == 3 * 8 + 4 * 8 + 8


def test_status_strings():
    for code, name in [(0, "VCA_OK"), (1, "VCA_ERR_INVALID_ARG"), (2, "VCA_ERR_UNSUPPORTED"),
                       (3, "VCA_ERR_OOM"), (4, "VCA_ERR_DEVICE"), (5, "VCA_ERR_STATE")]:
        assert _lib.status_str(code) == name


def cfg(**kw):
    base = dict(width=3840, height=2160, bit_depth=8, chroma_format=420, block_size=32,
                lowpass_k=0, device=0, flags=0, max_batch=0, feature_capacity=0)
    base.update(kw)
    c = _lib.VcaConfig()
    c.struct_size = kw.pop("struct_size", ctypes.sizeof(_lib.VcaConfig))
    for k, v in base.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("w,res,counts", [
    (32, (3840, 2160), (8040, 1980, 1980)), (16, (1920, 1080), (8040, 1980, 1980)),
    (8, (640, 360), (3600, 880, 880)), (32, (1280, 720), (880, 220, 220))])
def test_block_counts(w, res, counts):
    out = (ctypes.c_int32 * 3)()
    c = cfg(width=res[0], height=res[1], block_size=w)
    assert _lib.lib().vca_block_counts(ctypes.byref(c), out) == 0
    assert tuple(out) == counts


@pytest.mark.parametrize("bad", [
    dict(block_size=4), dict(block_size=64), dict(bit_depth=9), dict(chroma_format=444),
    dict(width=3841), dict(height=0), dict(width=62, block_size=32), dict(lowpass_k=3),
    dict(lowpass_k=64), dict(max_batch=-1), dict(flags=0x80), dict(struct_size=12),
    dict(device=-1)])
def test_bad_config_rejected_before_device(bad):
    c = cfg(**bad)
    out = (ctypes.c_int32 * 3)()
    assert _lib.lib().vca_block_counts(ctypes.byref(c), out) == _lib.VCA_ERR_INVALID_ARG
    ctx = ctypes.c_void_p(1234)
    assert _lib.lib().vca_open(ctypes.byref(c), None, ctypes.byref(ctx)) == _lib.VCA_ERR_INVALID_ARG
    assert not ctx.value


@pytest.mark.parametrize("mb,cap", [(8, 4), (0, 255), (300, 299)])
def test_feature_ring_smaller_than_a_launch_rejected(mb, cap):
    """A ring that cannot hold one launch's frames (after the defaults:
    max_batch 256 plain, 300 batched) is refused before the device is
    touched."""
    c = cfg(max_batch=mb, feature_capacity=cap)
    ctx = ctypes.c_void_p(1234)
    assert _lib.lib().vca_open(ctypes.byref(c), None, ctypes.byref(ctx)) == _lib.VCA_ERR_INVALID_ARG
    assert not ctx.value
    b = ctypes.c_void_p(1234)
    assert _lib.lib().vca_open_batch(ctypes.byref(c), 1, None, ctypes.byref(b)) == \
        _lib.VCA_ERR_INVALID_ARG
    assert not b.value


def test_null_arguments():
    L = _lib.lib()
    assert L.vca_open(None, None, None) == _lib.VCA_ERR_INVALID_ARG
    assert L.vca_analyze_frames(None, None, 0) == _lib.VCA_ERR_INVALID_ARG
    assert L.vca_features(None, 0, 0, None) == _lib.VCA_ERR_INVALID_ARG
    assert L.vca_reset(None) == _lib.VCA_ERR_INVALID_ARG
    assert L.vca_block_maps(None, 0, 1, None, None, None) == _lib.VCA_ERR_INVALID_ARG
    assert L.vca_batch_features(None, 0, 0, 0, None) == _lib.VCA_ERR_INVALID_ARG
    assert L.vca_batch_features_many(None, 0, None, None, None, None) == _lib.VCA_ERR_INVALID_ARG
    assert L.vca_frames_submitted(None) == -1
    assert L.vca_last_error(None) == b""
    L.vca_close(None)


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.lib()


def grad_cfg(**kw):
    base = dict(width=1920, height=1080, block_size=32, lowpass_k=0, bit_depth=8, n_seq=16,
                seq_len=2, device=0, pitch=1920, fstride=1920 * 1080)
    base.update(kw)
    c = _lib.VcaGradConfig()
    c.struct_size = base.pop("struct_size", ctypes.sizeof(_lib.VcaGradConfig))
    for k, v in base.items():
        setattr(c, k, v)
    return c


def test_grad_config_layout_and_workspace():
    assert ctypes.sizeof(_lib.VcaGradConfig) == 56
    L = _lib.lib()
    def ws(blocks, tiles):   # FP64 block energies, 256-byte aligned, then 256 B of masks per tile
        return (blocks * 8 + 255) // 256 * 256 + tiles * 256
    assert L.vca_grad_workspace(ctypes.byref(grad_cfg())) == ws(60 * 33 * 32, 60 * 33 * 32)
    assert L.vca_grad_workspace(ctypes.byref(grad_cfg(block_size=8, lowpass_k=2, n_seq=1, seq_len=3))) \
        == ws(240 * 135 * 3, 60 * 34 * 3)


@pytest.mark.parametrize("bad", [
    dict(block_size=4), dict(lowpass_k=3), dict(lowpass_k=64), dict(bit_depth=12),
    dict(width=16), dict(n_seq=0), dict(seq_len=0), dict(pitch=1000), dict(pitch=1922),
    dict(fstride=1920 * 1000), dict(fstride=1922), dict(n_seq=40000, seq_len=2),
    dict(struct_size=40), dict(device=-1)])
def test_bad_grad_config_rejected_before_device(bad):
    c = grad_cfg(**bad)
    L = _lib.lib()
    assert L.vca_grad_workspace(ctypes.byref(c)) == -1
    p = ctypes.c_void_p(1 << 20)   # never dereferenced: the configuration fails first
    assert L.vca_energy_forward(ctypes.byref(c), p, p, p, p, None) == _lib.VCA_ERR_INVALID_ARG
    assert L.vca_energy_backward(ctypes.byref(c), p, p, p, p, None) == _lib.VCA_ERR_INVALID_ARG


def test_grad_null_and_misaligned_arguments():
    L = _lib.lib()
    c = grad_cfg()
    p = ctypes.c_void_p(1 << 20)
    odd = ctypes.c_void_p((1 << 20) + 4)
    assert L.vca_grad_workspace(None) == -1
    assert L.vca_energy_forward(ctypes.byref(c), None, p, p, p, None) == _lib.VCA_ERR_INVALID_ARG
    assert L.vca_energy_forward(ctypes.byref(c), odd, p, p, p, None) == _lib.VCA_ERR_INVALID_ARG
    assert L.vca_energy_forward(ctypes.byref(c), p, p, p, None, None) == _lib.VCA_ERR_INVALID_ARG
    assert L.vca_energy_forward(ctypes.byref(c), p, p, p, odd, None) == _lib.VCA_ERR_INVALID_ARG
    assert L.vca_energy_backward(ctypes.byref(c), p, p, p, odd, None) == _lib.VCA_ERR_INVALID_ARG
    assert L.vca_energy_backward(ctypes.byref(c), odd, p, p, p, None) == _lib.VCA_ERR_INVALID_ARG
    assert L.vca_energy_backward(ctypes.byref(c), None, p, p, p, None) == _lib.VCA_ERR_INVALID_ARG


def test_downsample_flag_block_counts_and_rejections():
    L = _lib.lib()
    out = (ctypes.c_int32 * 3)()
    c = cfg(flags=_lib.VCA_F_DOWNSAMPLE)
    assert L.vca_block_counts(ctypes.byref(c), out) == 0
    assert tuple(out) == (60 * 33, 30 * 16, 30 * 16)   # the 1920x1080 half-size video
    for bad in (dict(width=3842), dict(height=2162), dict(lowpass_k=16),
                dict(width=120, height=120)):             # width / 4 < w
        c = cfg(flags=_lib.VCA_F_DOWNSAMPLE, **bad)
        assert L.vca_block_counts(ctypes.byref(c), out) == _lib.VCA_ERR_INVALID_ARG, bad
    c = cfg(flags=_lib.VCA_F_DOWNSAMPLE | _lib.VCA_F_KEEP_COEFFS)
    assert L.vca_block_counts(ctypes.byref(c), out) == _lib.VCA_ERR_UNSUPPORTED
    ctx = ctypes.c_void_p(1234)
    assert L.vca_open(ctypes.byref(c), None, ctypes.byref(ctx)) == _lib.VCA_ERR_UNSUPPORTED
    assert not ctx.value


def test_noalloc_rejects_before_touching_a_device():
    """vca_analyze_noalloc refuses, without a device, what its fixed array cannot
    hold (one 8192 x 8192 frame at w = 8 needs more than the 32 MiB) and the
    flags it does not support; a bad config is an invalid argument."""
    L = _lib.lib()
    fr = _lib.VcaFrames(16, 16, 16, 8192, 4096, 8192 * 8192, 4096 * 4096, 1)
    out = ctypes.c_void_p(256)
    big = cfg(width=8192, height=8192, block_size=8)
    assert L.vca_analyze_noalloc(ctypes.byref(big), ctypes.byref(fr), 1, out, None) == \
        _lib.VCA_ERR_UNSUPPORTED
    for flags in (_lib.VCA_F_KEEP_COEFFS, _lib.VCA_F_VALIDATE, _lib.VCA_F_TIMING):
        c = cfg(flags=flags)
        assert L.vca_analyze_noalloc(ctypes.byref(c), ctypes.byref(fr), 1, out, None) == \
            _lib.VCA_ERR_UNSUPPORTED
    bad = cfg(block_size=12)
    assert L.vca_analyze_noalloc(ctypes.byref(bad), ctypes.byref(fr), 1, out, None) == \
        _lib.VCA_ERR_INVALID_ARG
    ok = cfg(width=8192, height=4096, block_size=8)
    # zero frames: nothing to do, no device needed
    assert L.vca_analyze_noalloc(ctypes.byref(ok), ctypes.byref(fr), 0, None, None) == _lib.VCA_OK
    assert L.vca_analyze_noalloc(ctypes.byref(ok), ctypes.byref(fr), 1, None, None) == \
        _lib.VCA_ERR_INVALID_ARG
