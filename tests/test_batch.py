"""Batched form: one persistent, graph-replayed launch over many uneven
streams gives, per stream, exactly the features of the plain path (itself
bit-exact against the oracle), and matches the oracle on spot checks."""
import os

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


STREAMS = [
    dict(width=640, height=360, block_size=8, n=7),
    dict(width=1280, height=720, block_size=32, lowpass_k=16, n=12),
    dict(width=1920, height=1080, block_size=16, n=5),
    dict(width=640, height=360, block_size=32, n=9),
    dict(width=2560, height=1440, block_size=8, lowpass_k=4, n=3),
    dict(width=3840, height=2160, block_size=32, n=4),
    dict(width=1056, height=568, block_size=16, lowpass_k=8, n=6),
    dict(width=1920, height=1080, block_size=16, bit_depth=10, n=3),
    dict(width=1280, height=720, block_size=8, bit_depth=10, lowpass_k=2, n=2),
]


def make_frames(d, seed):
    if d.get("bit_depth", 8) == 10:
        return to_device(synth.stress_video(d["width"], d["height"], d["n"], cell=d["block_size"],
                                            stream=seed))
    dv = generated_scene_video(d["width"], d["height"], d["n"], seed=seed, scene_len=4)
    return dv.y, dv.u, dv.v


@pytest.fixture(scope="module")
def frames(vca):
    return [make_frames(d, 1000 + i) for i, d in enumerate(STREAMS)]


def plain_features(vca, d, planes, calls):
    an = vca.Analyzer(d["width"], d["height"], bit_depth=d.get("bit_depth", 8),
                      block_size=d["block_size"], lowpass_k=d.get("lowpass_k", 0))
    for _ in range(calls):
        an.submit(*planes)
    f = an.features(0, calls * d["n"])
    an.close()
    return f


@pytest.mark.parametrize("serial", [True, False], ids=["serial", "side_by_side"])
def test_batch_graph_replays_match_plain(vca, frames, serial):
    """Both arrangements of the classes in a round (one after another, side
    by side on parallel graph branches) give the plain path's features."""
    print_case(test="batch_vs_plain", streams=len(STREAMS), serial=serial)
    calls = 3
    b = vca.Batch(STREAMS)
    b.set_arrangement(serial)
    assert b.arrangement()["serial"] == serial
    for c in range(calls):
        b.submit(list(frames))
        # eager work and a synchronisation between graph replays
        x = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
        assert float((x * 2).sum()) > 0
        torch.cuda.synchronize()
    got = [b.features(s, 0, calls * d["n"]) for s, d in enumerate(STREAMS)]
    b.close()
    for s, d in enumerate(STREAMS):
        ref = plain_features(vca, d, frames[s], calls)
        assert got[s].tobytes() == ref.tobytes(), f"stream {s} ({d}) differs from the plain path"


def test_batch_features_read_while_later_rounds_are_queued(vca, frames):
    """vca_batch_features waits for the round that produced the frames asked
    for: the first call's features read after a second call was queued (one
    frame per round: 24 rounds, more than the batch remembers) equal the plain
    path's."""
    print_case(test="batch_pipelined")
    one = [dict(d, max_batch=1) for d in STREAMS]
    b = vca.Batch(one)
    first = b.submit(list(frames))
    b.submit(list(frames))
    got = [b.features(s, first[s], d["n"]) for s, d in enumerate(STREAMS)]
    second = [b.features(s, d["n"], d["n"]) for s, d in enumerate(STREAMS)]
    b.close()
    for s, d in enumerate(STREAMS):
        ref = plain_features(vca, d, frames[s], 2)
        assert got[s].tobytes() == ref[:d["n"]].tobytes(), f"stream {s} ({d})"
        assert second[s].tobytes() == ref[d["n"]:].tobytes(), f"stream {s} ({d})"


def test_batch_features_many_and_prepared_frames(vca, frames):
    """vca_batch_features_many returns, request by request, what
    vca_batch_features returns (two calls, several rounds each, requests out
    of stream order, repeated and empty); prepared frames submit exactly as
    the planes they were prepared from; bad requests fail before anything is
    copied."""
    print_case(test="batch_features_many")
    small = [dict(d, max_batch=4) for d in STREAMS]
    b = vca.Batch(small)
    p = b.prepare(list(frames))
    b.submit(p)
    b.submit(list(frames))
    reqs = [(s, 0, 2 * d["n"]) for s, d in reversed(list(enumerate(STREAMS)))]
    reqs += [(1, 3, 5), (1, 0, 0), (0, STREAMS[0]["n"], 1)]
    got = b.features_many(reqs)
    for (s, f, c), g in zip(reqs, got):
        assert g.shape == (c, 7)
        assert g.tobytes() == b.features(s, f, c).tobytes(), (s, f, c)
    for s, d in enumerate(STREAMS):
        ref = plain_features(vca, d, frames[s], 2)
        assert b.features(s, 0, 2 * d["n"]).tobytes() == ref.tobytes(), f"stream {s}"
    with pytest.raises(vca.VcaError):
        b.features_many([(0, 0, 1), (len(STREAMS), 0, 1)])
    with pytest.raises(vca.VcaError):
        b.features_many([(0, 0, 2 * STREAMS[0]["n"] + 1)])
    assert b.features_many([]) == []
    other = vca.Batch(small)
    with pytest.raises(ValueError):
        other.submit(p)
    other.close()
    b.close()
    # the plain path's prepared frames
    d = STREAMS[1]
    an = vca.Analyzer(d["width"], d["height"], block_size=d["block_size"], lowpass_k=d.get("lowpass_k", 0))
    pf = an.prepare(*frames[1])
    an.submit(pf)
    an.submit(*frames[1])
    assert an.features(0, 2 * d["n"]).tobytes() == plain_features(vca, d, frames[1], 2).tobytes()
    an.close()


def test_batch_oracle_spot_checks(vca, frames):
    print_case(test="batch_oracle")
    b = vca.Batch(STREAMS)
    b.submit(list(frames))
    for s in (0, 1, 4, 7):
        d = STREAMS[s]
        got = b.features(s, 0, d["n"])
        y, u, v = (p.cpu().numpy() for p in frames[s])
        if d.get("bit_depth", 8) == 10:
            y, u, v = (a.view(np.uint16) for a in (y, u, v))
        cfg = oracle.Config(d["width"], d["height"], d.get("bit_depth", 8), d["block_size"],
                            d.get("lowpass_k", 0))
        ref = oracle.analyze(cfg, y, u, v, threads=8).features
        assert_features_close(got, ref)
    b.close()


def test_batch_rounds_empty_streams_and_signature_change(vca, frames):
    print_case(test="batch_rounds")
    small = [dict(d, max_batch=2) for d in STREAMS[:4]]
    b = vca.Batch(small)
    sub = [frames[s] for s in range(4)]
    b.submit(sub)                                     # rounds of 2 frames
    b.submit([sub[0], None, sub[2], None])            # streams 1 and 3 idle
    b.submit([None, sub[1], None, sub[3]])
    for s, d in enumerate(small):
        n = d["n"]
        got = b.features(s, 0, 2 * n)
        ref = plain_features(vca, d, frames[s], 2)
        assert got.tobytes() == ref.tobytes(), f"stream {s}"
    b.close()


@pytest.mark.skip(reason="crashed the host (segmentation fault inside vca_analyze_batch) when the "
                         "batch evicted cached graphs, both before and after giving each capture "
                         "its own branch streams and events; eviction is switched off (no cached "
                         "graph is destroyed before close, rounds beyond the cache run in line) "
                         "and this case is not run again until the cause is shown")
def test_batch_graph_cache_eviction(vca, frames):
    """Ten launch signatures in turn, more than an eight-entry graph cache
    held when this case crashed: rounds of varying frame counts (idle
    streams included), alternating the arrangement; every stream's features
    equal the plain path's over the same sequence of frames."""
    print_case(test="batch_graph_eviction")
    ds = STREAMS[:3]
    b = vca.Batch([dict(d, max_batch=8) for d in ds])
    plain = [vca.Analyzer(d["width"], d["height"], bit_depth=d.get("bit_depth", 8),
                          block_size=d["block_size"], lowpass_k=d.get("lowpass_k", 0)) for d in ds]
    total = [0] * len(ds)
    for i in range(20):
        b.set_arrangement(i % 2 == 0)
        sub = []
        for s, d in enumerate(ds):
            c = (i * (s + 2) + s) % 5                  # 0..4 frames, 0 = idle
            c = min(c, d["n"])
            if c == 0:
                sub.append(None)
                continue
            a = (i * 3 + s) % (d["n"] - c + 1)
            planes = tuple(t[a:a + c] for t in frames[s])
            sub.append(planes)
            plain[s].submit(*planes)
            total[s] += c
        b.submit(sub)
    for s in range(len(ds)):
        assert total[s] > 0
        got = b.features(s, 0, total[s])
        ref = plain[s].features(0, total[s])
        assert got.tobytes() == ref.tobytes(), f"stream {s}"
        plain[s].close()
    b.close()


def test_batch_tune_and_no_graph_path(vca, frames, monkeypatch):
    print_case(test="batch_tune")
    sub = list(frames[:6])
    b = vca.Batch(STREAMS[:6])
    choice = b.tune(sub, reps=1)
    assert choice["depth"] in (1, 2, 4) and choice["groups_per_cu"] >= 1 and choice["ms"] > 0
    arr = b.arrangement()
    assert arr["serial_ms"] > 0 and arr["parallel_ms"] > 0
    assert arr["serial"] == (arr["serial_ms"] <= arr["parallel_ms"])
    times = b.class_times()
    assert set(times) == {"b8_w8_k8", "b8_w32_k16", "b8_w16_k16", "b8_w32_k32", "b8_w8_k4"}
    assert all(t["ms"] > 0 and t["depth"] in (1, 2, 4) and t["groups_per_cu"] >= 1 and
               t["waves"] in (4, 8) and t["chunk_strips"] in (8, 16, 32, 64) for t in times.values())
    b.submit(sub)
    tuned = [b.features(s, 0, d["n"]) for s, d in enumerate(STREAMS[:6])]
    b.close()
    monkeypatch.setenv("VCA_BATCH_NO_GRAPH", "1")
    for serial in (True, False):
        b2 = vca.Batch(STREAMS[:6])
        b2.set_arrangement(serial)
        b2.submit(sub)
        b2.submit(sub)
        eager = [b2.features(s, 0, 2 * d["n"]) for s, d in enumerate(STREAMS[:6])]
        b2.close()
        for s, d in enumerate(STREAMS[:6]):
            assert tuned[s].tobytes() == eager[s][:d["n"]].tobytes(), (serial, s)
            ref = plain_features(vca, d, frames[s], 2)
            assert eager[s].tobytes() == ref.tobytes(), (serial, s)
    with pytest.raises(vca.VcaError):
        b3 = vca.Batch(STREAMS[:1])
        try:
            b3.set_arrangement(2)
        finally:
            b3.close()


def test_batch_tune_between_rounds_keeps_features_and_state(vca, frames):
    """Tuning after a round (its arrangement timing runs whole rounds with
    their reductions) leaves the features already computed and the h state
    alone, even with feature rings of one round, whose slots the tuning
    rounds would reuse: both rounds still match the plain path."""
    print_case(test="batch_tune_between_rounds")
    streams = [dict(d, max_batch=d["n"], feature_capacity=d["n"]) for d in STREAMS[:4]]
    sub = list(frames[:4])
    b = vca.Batch(streams)
    b.submit(sub)
    first = [b.features(s, 0, d["n"]) for s, d in enumerate(streams)]
    b.tune(sub, reps=1)
    assert b.arrangement()["serial_ms"] > 0
    again = [b.features(s, 0, d["n"]) for s, d in enumerate(streams)]
    b.submit(sub)
    second = [b.features(s, d["n"], d["n"]) for s, d in enumerate(streams)]
    b.close()
    for s, d in enumerate(streams):
        ref = plain_features(vca, d, frames[s], 2)
        assert again[s].tobytes() == first[s].tobytes(), s
        assert first[s].tobytes() == ref[:d["n"]].tobytes(), s
        assert second[s].tobytes() == ref[d["n"]:].tobytes(), s


@pytest.mark.parametrize("waves,chunk", [(8, 8), (4, 64), (8, 16)])
def test_batch_class_shapes(vca, frames, waves, chunk):
    """Every class pinned to 4 or 8 wavefronts per workgroup and 8 to 64
    strips per chunk gives the plain path's features (two rounds, so h
    crosses a round); bad shapes fail before any launch."""
    print_case(test="batch_class_shapes", waves=waves, chunk=chunk)
    b = vca.Batch(STREAMS)
    classes = {f"b{d.get('bit_depth', 8)}_w{d['block_size']}_k{d.get('lowpass_k', 0) or d['block_size']}"
               for d in STREAMS}
    for i, cls in enumerate(sorted(classes)):
        b.set_class_shape(cls, (1, 2, 4)[i % 3], i % 3, waves, chunk)
    b.submit(list(frames))
    b.submit(list(frames))
    got = [b.features(s, 0, 2 * d["n"]) for s, d in enumerate(STREAMS)]
    for bad in ((3, 0, 4, 32), (2, -1, 4, 32), (2, 0, 6, 32), (2, 0, 4, 24)):
        with pytest.raises(vca.VcaError):
            b.set_class_shape("b8_w32_k32", *bad)
    b.close()
    for s, d in enumerate(STREAMS):
        assert got[s].tobytes() == plain_features(vca, d, frames[s], 2).tobytes(), f"stream {s} ({d})"


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_batch_random_mixes(vca, seed):
    """Seeded random mixes of 5-9 streams (width and height, w, K, bit depth
    and frame count drawn per stream; some streams share a class, some
    classes hold one stream), two calls each: every stream's features equal
    the plain path's bytes."""
    rng = np.random.default_rng(seed)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    descs, planes = [], []
    for _ in range(int(rng.integers(5, 10))):
        w = int(rng.choice([8, 16, 32]))
        k = int(rng.choice([0, w // 2, w // 4]))
        bits = int(rng.choice([8, 10]))
        width = 32 * int(rng.integers(max(2, w // 16 + 1), 40))
        height = 2 * int(rng.integers(w, 200))
        n = int(rng.integers(1, 7))
        top = (1 << bits) - 1
        dt = torch.uint8 if bits == 8 else torch.int16
        pl = tuple(torch.randint(0, top + 1, (n, hh, ww), device="cuda", generator=g).to(dt)
                   for hh, ww in ((height, width), (height // 2, width // 2), (height // 2, width // 2)))
        descs.append(dict(width=width, height=height, block_size=w, lowpass_k=k, bit_depth=bits, n=n))
        planes.append(pl)
    print_case(test="batch_random_mix", seed=seed,
               streams=[(d["width"], d["height"], d["block_size"], d["lowpass_k"], d["bit_depth"], d["n"])
                        for d in descs])
    b = vca.Batch(descs)
    b.submit(planes)
    b.submit(planes)
    got = [b.features(s, 0, 2 * d["n"]) for s, d in enumerate(descs)]
    b.close()
    for s, d in enumerate(descs):
        ref = plain_features(vca, d, planes[s], 2)
        assert got[s].tobytes() == ref.tobytes(), f"stream {s} ({d})"


def test_plain_tune(vca, frames):
    print_case(test="plain_tune")
    d = STREAMS[5]
    an = vca.Analyzer(d["width"], d["height"], block_size=d["block_size"])
    choice = an.tune(*frames[5], reps=1)
    assert choice["depth"] in (1, 2, 4) and choice["groups_per_cu"] >= 1
    an.submit(*frames[5])
    f = an.features(0, d["n"])
    an.close()
    assert f.tobytes() == plain_features(vca, d, frames[5], 1).tobytes()


def test_batch_10bit_validation(vca):
    """A validating 10-bit stream in a batch: a sample above 1023 inside its
    block grid fails that stream's features only."""
    from paper_2304_12384_amd import VcaError
    print_case(test="batch_10bit_validation")
    rng = np.random.default_rng(21)
    def planes(w, h, bits, n):
        top = (1 << bits) - 1
        dt = np.uint8 if bits == 8 else np.uint16
        ps = [rng.integers(0, top + 1, (n, hh, ww)).astype(dt) for hh, ww in ((h, w), (h // 2, w // 2),
                                                                            (h // 2, w // 2))]
        return ps
    p10 = planes(256, 128, 10, 2)
    p8 = planes(320, 192, 8, 2)
    p10[0][1, 64, 100] = 1024
    dev10 = [torch.from_numpy(a.view(np.int16)).cuda() for a in p10]
    dev8 = [torch.from_numpy(a).cuda() for a in p8]
    b = vca.Batch([dict(width=256, height=128, bit_depth=10, block_size=16, validate=True),
                   dict(width=320, height=192, block_size=32)])
    b.submit([tuple(dev10), tuple(dev8)])
    assert b.features(1, 0, 2).shape == (2, 7)
    with pytest.raises(VcaError):
        b.features(0, 0, 2)
    # the mark is frame 1's: frame 0 of the same stream still reads, and so
    # does the next round's clean frame
    assert b.features(0, 0, 1).shape == (1, 7)
    b.submit([(dev10[0][:1], dev10[1][:1], dev10[2][:1]), tuple(dev8)])
    assert b.features(0, 2, 1).shape == (1, 7)
    b.close()
