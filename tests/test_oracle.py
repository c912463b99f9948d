"""Pins of the CPU oracle against things other than itself.

The paper (Section 2) names the seven features and the low-pass DCT option
but prints no worked example, so every pin here comes from mathematics: the
orthonormal DCT-II of a library routine, closed forms of the integer transform
on constant and single-basis blocks (through the Gram matrix C C^T), brute
force in pure Python on tiny frames, and invariants of the features (constant
frames, static sequences, grid edges, call boundaries).
"""
import math

import numpy as np
import pytest
import scipy.fft

import oracle
from tests import brute

WS = (4, 8, 16, 32)


def shifts(w, B):
    lw = int(math.log2(w))
    return lw + B - 9, lw + 6


def orthonormal_dct(w):
    return scipy.fft.dct(np.eye(w), norm="ortho", axis=0)   # rows = frequencies


# ----------------------------------------------------------------- matrix C_w
@pytest.mark.parametrize("w", WS)
def test_matrix_structure(w):
    C = oracle.dct_matrix(w)
    assert (C[0] == 64).all()
    assert (C[1:].sum(axis=1) == 0).all()
    assert np.abs(C).max() <= 90                 # every entry fits int8
    for k in range(w):                           # DCT-II parity about the centre
        assert (C[k, ::-1] == (-1) ** k * C[k]).all()


@pytest.mark.parametrize("w", WS)
def test_matrix_near_scaled_orthonormal_dct(w):
    C = oracle.dct_matrix(w)
    ref = 64.0 * math.sqrt(w) * orthonormal_dct(w)
    assert np.abs(C - ref).max() <= 1.37
    assert (np.sign(C) == np.sign(np.round(ref, 9))).all()


@pytest.mark.parametrize("w,max_off", [(4, 0), (8, 50), (16, 188), (32, 376)])
def test_matrix_gram(w, max_off):
    C = oracle.dct_matrix(w)
    G = C @ C.T
    assert np.abs(np.diag(G) / (4096.0 * w) - 1.0).max() < 2e-3
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() == max_off
    assert (off[::2, 1::2] == 0).all() and (off[1::2, ::2] == 0).all()   # even/odd rows


@pytest.mark.parametrize("w", (4, 8, 16))
def test_matrix_embedding(w):
    C32 = oracle.dct_matrix(32)
    assert (oracle.dct_matrix(w) == C32[:: 32 // w, :w]).all()


# ------------------------------------------------------------ block transform
def random_block(rng, w, B):
    kind = rng.integers(0, 3)
    maxv = (1 << B) - 1
    if kind == 0:
        return rng.integers(0, maxv + 1, size=(w, w))
    if kind == 1:
        yy, xx = np.mgrid[0:w, 0:w]
        th = rng.uniform(0, 2 * np.pi)
        return np.where(np.cos(th) * (xx - w / 2) + np.sin(th) * (yy - w / 2) > 0, maxv, 0)
    return np.clip(rng.normal(maxv / 2, maxv / 6, size=(w, w)).round(), 0, maxv).astype(np.int64)


@pytest.mark.parametrize("w", WS)
@pytest.mark.parametrize("B", (8, 10))
def test_transform_matches_brute_force(w, B):
    rng = np.random.default_rng(100 + w + B)
    C = oracle.dct_matrix(w).tolist()
    for K in sorted({w, max(1, w // 2), max(1, w // 4)}):
        for _ in range(6):
            X = random_block(rng, w, B)
            got = oracle.block_transform(X, B, K)
            want = brute.block_coeffs(X.tolist(), C, w, K, B)
            assert got.tolist() == want


@pytest.mark.parametrize("w", WS)
@pytest.mark.parametrize("B", (8, 10))
def test_constant_block_closed_form(w, B):
    for v in (0, 1, 77, (1 << (B - 1)), (1 << B) - 1):
        Y = oracle.block_transform(np.full((w, w), v), B)
        assert Y[0, 0] == (1 << (15 - B)) * v
        Y[0, 0] = 0
        assert not Y.any()


def _gram_prediction(w, B, l0, a, orientation):
    """Exact coefficients of X = 2^(B-1) + a C[l0] laid along rows ("v": the
    pattern varies with the row index m) or columns ("h": with n)."""
    C = oracle.dct_matrix(w)
    G = C @ C.T
    s1, s2 = shifts(w, B)
    Y = np.zeros((w, w), np.int64)
    Y[0, 0] = 1 << 14
    if orientation == "v":
        # rows of T are 2^(15-B) X[m] exactly, rounding happens once, vertically
        for i in range(1, w):
            Y[i, 0] = ((1 << (15 - B)) * a * G[i, l0] + (1 << (s2 - 1))) >> s2
    else:
        # rounding happens in the horizontal pass; the vertical pass is exact
        for k in range(1, w):
            Y[0, k] = (a * G[k, l0] + (1 << (s1 - 1))) >> s1
    return Y


@pytest.mark.parametrize("w", WS)
@pytest.mark.parametrize("B,a", [(8, 1), (10, 1), (10, 5)])
def test_single_basis_pattern_gram_closed_form(w, B, a):
    """Pins the matrix, the pass order (horizontal first), the orientation of
    the output (row index = vertical frequency) and both rounding shifts."""
    C = oracle.dct_matrix(w)
    for l0 in range(1, w):
        col = (1 << (B - 1)) + a * C[l0]
        Xv = np.repeat(col[:, None], w, axis=1)        # varies with m
        Xh = np.repeat(col[None, :], w, axis=0)        # varies with n
        assert (oracle.block_transform(Xv, B) == _gram_prediction(w, B, l0, a, "v")).all()
        assert (oracle.block_transform(Xh, B) == _gram_prediction(w, B, l0, a, "h")).all()


@pytest.mark.parametrize("w", (8, 16, 32))
def test_exactly_one_coefficient_subset(w):
    """An integer basis pattern lights exactly one AC coefficient precisely for
    the rows where the integer matrix is exactly orthogonal to all others."""
    C = oracle.dct_matrix(w)
    G = C @ C.T
    lit = set()
    for l0 in range(1, w):
        X = np.repeat(((1 << 7) + C[l0])[:, None], w, axis=1)
        Y = oracle.block_transform(X, 8)
        Y[0, 0] = 0
        nz = list(zip(*np.nonzero(Y)))
        if nz == [(l0, 0)]:
            lit.add(l0)
        orthogonal = all(G[i, l0] == 0 for i in range(1, w) if i != l0)
        assert (l0 in lit) == orthogonal
    assert lit == {w // 4, w // 2, 3 * w // 4}


@pytest.mark.parametrize("w", (8, 16, 32))
@pytest.mark.parametrize("B", (8, 10))
def test_cosine_pattern_energy_concentrates(w, B):
    """A rounded 2-D cosine of vertical frequency p and horizontal frequency q
    puts almost all AC energy at Y[p][q]."""
    rng = np.random.default_rng(7 * w + B)
    amp = 0.45 * (1 << B)
    m = np.arange(w)
    for _ in range(10):
        p, q = (int(t) for t in rng.integers(0, w, size=2))
        if p == 0 and q == 0:
            continue
        X = np.round((1 << (B - 1)) + amp * np.outer(np.cos(np.pi * p * (2 * m + 1) / (2 * w)),
                                                     np.cos(np.pi * q * (2 * m + 1) / (2 * w))))
        Y = oracle.block_transform(X.astype(np.int64), B).astype(np.float64)
        Y[0, 0] = 0
        e = Y ** 2
        assert np.unravel_index(np.argmax(e), e.shape) == (p, q)
        assert e[p, q] >= 0.97 * e.sum()


@pytest.mark.parametrize("w", (8, 16, 32))
@pytest.mark.parametrize("B", (8, 10))
def test_transform_approximates_orthonormal_dct(w, B):
    """Y ~ (2^(15-B) / w) D X D^T with D the orthonormal DCT-II."""
    rng = np.random.default_rng(11 * w + B)
    worst, sq, cnt = 0.0, 0.0, 0
    for _ in range(40):
        X = random_block(rng, w, B)
        ref = (2.0 ** (15 - B) / w) * scipy.fft.dctn(X.astype(np.float64), norm="ortho")
        err = oracle.block_transform(X, B) - ref
        worst = max(worst, np.abs(err).max())
        sq += (err ** 2).sum()
        cnt += err.size
    assert worst <= 1e-2 * 2 ** 15
    assert math.sqrt(sq / cnt) <= 3e-3 * 2 ** 15


@pytest.mark.parametrize("w", (8, 16, 32))
@pytest.mark.parametrize("B", (8, 10))
def test_lowpass_is_crop_of_full(w, B):
    rng = np.random.default_rng(5 * w + B)
    for _ in range(10):
        X = random_block(rng, w, B)
        full = oracle.block_transform(X, B)
        for K in (1, w // 4, w // 2):
            assert (oracle.block_transform(X, B, K) == full[:K, :K]).all()


def test_block_transform_range_error():
    X = np.zeros((8, 8), np.int64)
    X[3, 3] = 1024
    with pytest.raises(oracle.OracleError):
        oracle.block_transform(X, 10)
    X[3, 3] = 256
    with pytest.raises(oracle.OracleError):
        oracle.block_transform(X, 8)


# -------------------------------------------------------------------- weights
@pytest.mark.parametrize("w", (8, 16, 32))
def test_weights(w):
    W = oracle.weights(w)
    assert W[w - 1, w - 1] == 1.0
    assert W[0, 0] == pytest.approx(math.exp(1.0 - 1.0 / w ** 4), rel=1e-15)
    assert (W == W.T).all()
    assert W.min() >= 1.0 and W.max() <= math.e
    prod = np.outer(np.arange(1, w + 1), np.arange(1, w + 1)).ravel()
    order = np.argsort(prod, kind="stable")
    assert (np.diff(W.ravel()[order]) <= 0).all()   # decreasing in (i+1)(j+1)


# ------------------------------------------------------------------- features
def tiny_frames(rng, n, width, height, B, static=False):
    maxv = (1 << B) - 1
    dt = np.uint8 if B == 8 else np.uint16
    y0 = rng.integers(0, maxv + 1, size=(height, width))
    frames = []
    for t in range(n):
        y = y0 if static else rng.integers(0, maxv + 1, size=(height, width))
        u = rng.integers(0, maxv + 1, size=(height // 2, width // 2))
        v = rng.integers(0, maxv + 1, size=(height // 2, width // 2))
        frames.append((y.astype(dt), u.astype(dt), v.astype(dt)))
    return frames


def run_oracle(frames, cfg, **kw):
    y = np.stack([f[0] for f in frames])
    u = np.stack([f[1] for f in frames])
    v = np.stack([f[2] for f in frames])
    return oracle.analyze(cfg, y, u, v, want_blocks=True, **kw)


@pytest.mark.parametrize("w", (8, 16, 32))
@pytest.mark.parametrize("B", (8, 10))
@pytest.mark.parametrize("size", [(64, 64), (96, 64)])
def test_features_match_brute_force(w, B, size):
    width, height = size
    rng = np.random.default_rng(w * 1000 + B * 10 + width)
    frames = tiny_frames(rng, 3, width, height, B)
    C = oracle.dct_matrix(w).tolist()
    for K in sorted({w, w // 2}):
        cfg = oracle.Config(width, height, B, w, 0 if K == w else K)
        res = run_oracle(frames, cfg)
        want, wantH = brute.features([tuple(p.tolist() for p in f) for f in frames], C, w, K, B)
        np.testing.assert_allclose(res.features, np.array(want), rtol=1e-12, atol=0)
        np.testing.assert_allclose(res.block_h, np.array(wantH), rtol=1e-12, atol=0)


@pytest.mark.parametrize("w", (8, 16, 32))
@pytest.mark.parametrize("B", (8, 10))
def test_constant_frames_closed_form(w, B):
    vals = (3, 200, 97) if B == 8 else (1023, 5, 640)
    dt = np.uint8 if B == 8 else np.uint16
    for width, height in ((128, 64), (160, 96)):
        cfg = oracle.Config(width, height, B, w)
        y = np.full((2, height, width), vals[0], dt)
        u = np.full((2, height // 2, width // 2), vals[1], dt)
        v = np.full((2, height // 2, width // 2), vals[2], dt)
        f = oracle.analyze(cfg, y, u, v).features
        for t in range(2):
            assert f[t, 0] == 0.0 and f[t, 3] == 0.0 and f[t, 4] == 0.0 and f[t, 1] == 0.0
            for idx, val in ((2, vals[0]), (5, vals[1]), (6, vals[2])):
                assert f[t, idx] == pytest.approx(math.sqrt((1 << (15 - B)) * val) / (w * w),
                                                  rel=1e-14)


@pytest.mark.parametrize("w", (8, 32))
def test_static_sequence_has_zero_h(w):
    rng = np.random.default_rng(3)
    frames = tiny_frames(rng, 4, 128, 96, 8, static=True)
    f = run_oracle(frames, oracle.Config(128, 96, 8, w)).features
    assert (f[:, 1] == 0.0).all()
    assert (f[:, 0] > 0).all()


def test_h_of_single_block_change():
    rng = np.random.default_rng(4)
    w = 16
    frames = tiny_frames(rng, 1, 128, 64, 8)
    y1 = frames[0][0].copy()
    y1[16:32, 48:64] = rng.integers(0, 256, size=(16, 16))
    frames.append((y1, frames[0][1], frames[0][2]))
    cfg = oracle.Config(128, 64, 8, w)
    res = run_oracle(frames, cfg)
    cy = 8 * 4
    k = 1 * 8 + 3                           # block row 1, column 3
    Xa = frames[0][0][16:32, 48:64].astype(np.int64)
    Xb = y1[16:32, 48:64].astype(np.int64)
    C = oracle.dct_matrix(w).tolist()
    Ha = brute.block_energy(brute.block_coeffs(Xa.tolist(), C, w, w, 8), w)
    Hb = brute.block_energy(brute.block_coeffs(Xb.tolist(), C, w, w, 8), w)
    assert res.block_h[0, k] == pytest.approx(Ha, rel=1e-13)
    assert res.features[1, 1] == pytest.approx(abs(Hb - Ha) / (cy * w * w), rel=1e-12)
    assert res.features[0, 1] == 0.0


def test_call_boundary_continuity():
    rng = np.random.default_rng(5)
    frames = tiny_frames(rng, 6, 96, 64, 8)
    cfg = oracle.Config(96, 64, 8, 16)
    whole = run_oracle(frames, cfg)
    a = run_oracle(frames[:4], cfg)
    cy = oracle.block_counts(cfg)[0]
    b = run_oracle(frames[4:], cfg, h_prev=a.block_h[-1, :cy])
    assert (np.concatenate([a.features, b.features]) == whole.features).all()


def test_pixels_outside_block_grid_are_ignored():
    rng = np.random.default_rng(6)
    width, height, w = 104, 72, 32        # luma 3x2 blocks + margins; chroma 1x1 + margins
    frames = tiny_frames(rng, 2, width, height, 8)
    cfg = oracle.Config(width, height, 8, w)
    ref = run_oracle(frames, cfg).features
    changed = []
    for (y, u, v) in frames:
        y, u, v = y.copy(), u.copy(), v.copy()
        y[64:, :] = 255 - y[64:, :]
        y[:, 96:] = 0
        u[32:, :] = 7
        u[:, 32:] = 9
        v[32:, 32:] = 255
        changed.append((y, u, v))
    assert (run_oracle(changed, cfg).features == ref).all()


@pytest.mark.parametrize("width,height,w,counts", [
    (3840, 2160, 32, (8040, 1980, 1980)), (1280, 720, 32, (880, 220, 220)),
    (1920, 1080, 16, (8040, 1980, 1980)), (640, 360, 8, (3600, 880, 880)),
    (2560, 1440, 32, (3600, 880, 880))])
def test_block_counts(width, height, w, counts):
    assert oracle.block_counts(oracle.Config(width, height, 8, w)) == counts


def test_lowpass_equals_full_on_band_limited_content():
    """Blocks whose only AC coefficient lies inside the K x K corner give the
    same energy with and without the low-pass option."""
    w, B, K = 32, 8, 16
    C = oracle.dct_matrix(w)
    width, height = 128, 64
    y = np.zeros((height, width), np.uint8)
    for bx, l0 in enumerate((8, 0, 8, 8)):          # l0 = w/4 lights one AC coefficient
        col = 128 + (C[l0] if l0 else 0)
        y[:32, bx * 32:(bx + 1) * 32] = np.repeat(np.asarray(col)[:, None] * np.ones(1), 32, axis=1) \
            if l0 else 128
        y[32:, bx * 32:(bx + 1) * 32] = 40 + 10 * bx
    u = np.full((height // 2, width // 2), 128, np.uint8)
    full = oracle.analyze(oracle.Config(width, height, B, w), y[None], u[None], u[None]).features
    low = oracle.analyze(oracle.Config(width, height, B, w, K), y[None], u[None], u[None]).features
    assert full[0, 0] > 0
    assert (full == low).all()


def test_threads_do_not_change_results():
    rng = np.random.default_rng(8)
    frames = tiny_frames(rng, 5, 128, 64, 10)
    cfg = oracle.Config(128, 64, 10, 8)
    a = run_oracle(frames, cfg, threads=1)
    b = run_oracle(frames, cfg, threads=4)
    assert (a.features == b.features).all() and (a.block_h == b.block_h).all()


def test_analyze_rejects_bad_input():
    dt = np.uint16
    y = np.zeros((1, 64, 64), dt)
    u = np.zeros((1, 32, 32), dt)
    y[0, 5, 5] = 1024
    with pytest.raises(oracle.OracleError):
        oracle.analyze(oracle.Config(64, 64, 10, 8), y, u, u)
    with pytest.raises(oracle.OracleError):      # chroma smaller than one block
        oracle.block_counts(oracle.Config(64, 40, 8, 32))
    with pytest.raises(oracle.OracleError):
        oracle.block_counts(oracle.Config(64, 64, 9, 8))
