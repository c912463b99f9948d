"""Host-only part of the host ingest: the raw .yuv reader (vca_read_yuv)
against numpy, and its argument checks.  No device is touched."""
import numpy as np
import pytest

from paper_2304_12384_amd import VcaError, read_yuv, write_yuv


def planes(rng, n, w, h, bit_depth):
    top = (1 << bit_depth) - 1
    dt = np.uint8 if bit_depth == 8 else np.uint16
    y = rng.integers(0, top + 1, (n, h, w)).astype(dt)
    u = rng.integers(0, top + 1, (n, h // 2, w // 2)).astype(dt)
    v = rng.integers(0, top + 1, (n, h // 2, w // 2)).astype(dt)
    return y, u, v


@pytest.mark.parametrize("w,h,bits", [(70, 38, 8), (64, 48, 10), (2, 2, 8)])
def test_read_yuv_round_trip(tmp_path, w, h, bits):
    rng = np.random.default_rng(w * h + bits)
    y, u, v = planes(rng, 5, w, h, bits)
    path = str(tmp_path / "clip.yuv")
    write_yuv(path, y, u, v)
    # the file is plain I420: frame t = Y rows, U rows, V rows
    raw = np.fromfile(path, dtype=y.dtype)
    per = w * h + 2 * (w // 2) * (h // 2)
    assert raw.size == 5 * per
    assert (raw[per:per + w * h].reshape(h, w) == y[1]).all()
    ry, ru, rv = read_yuv(path, w, h, bits)
    assert (ry == y).all() and (ru == u).all() and (rv == v).all()
    ry, ru, rv = read_yuv(path, w, h, bits, first=1, count=3)
    assert (ry == y[1:4]).all() and (ru == u[1:4]).all() and (rv == v[1:4]).all()
    ry, ru, rv = read_yuv(path, w, h, bits, first=5, count=0)
    assert ry.shape == (0, h, w)


def test_read_yuv_errors(tmp_path):
    rng = np.random.default_rng(3)
    y, u, v = planes(rng, 2, 16, 8, 8)
    path = str(tmp_path / "two.yuv")
    write_yuv(path, y, u, v)
    with pytest.raises(VcaError):
        read_yuv(path, 16, 8, 8, first=1, count=2)          # past the end
    with pytest.raises(VcaError):
        read_yuv(str(tmp_path / "missing.yuv"), 16, 8, 8, count=1)
    with pytest.raises(VcaError):
        read_yuv(path, 15, 8, 8, count=1)                     # odd width
    with pytest.raises(VcaError):
        read_yuv(path, 16, 8, 12, count=1)                    # bit depth
