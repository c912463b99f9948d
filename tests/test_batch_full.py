"""The batched form at full size, in the benchmark's launch configuration:
64 uneven 8-bit 4:2:0 streams (resolution 360p..2160p, w in {8, 16, 32},
30-300 frames: 10,764 frames, 45.5 GB generated on the device), tuned, one
graph-replayed launch.

Every frame's seven features equal, bit for bit, those of the same stream
analysed by a plain context (itself held bit-exact to the oracle by the
parity tests); one frame per stream, with the frame before it for h, is
checked against the oracle directly (features within 1e-5 relative).
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_features_close, print_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2304_12384_amd as vca_mod
    return vca_mod


def sampled_frame(s, n):
    """One frame per stream: the first, the last, or the first after a scene
    cut (every 120 frames) where the stream is long enough."""
    return (0, n - 1, 120 if n > 120 else n // 2)[s % 3]


def test_batch_64_streams_bench_launch(vca):
    from synth.device import generated_scene_video
    descs = synth.batch_streams(64)
    print_case(test="batch_full", streams=len(descs), frames=sum(d["n_frames"] for d in descs))
    vids = [generated_scene_video(d["width"], d["height"], d["n_frames"], seed=3000 + d["stream"])
            for d in descs]
    frames = [v.planes() for v in vids]
    cfg = [dict(width=d["width"], height=d["height"], block_size=d["block_size"],
                max_batch=d["n_frames"]) for d in descs]
    b = vca.Batch(cfg)
    b.tune(frames, reps=1)
    first = b.submit(frames)
    got = [b.features(s, first[s], d["n_frames"]) for s, d in enumerate(descs)]
    b.close()

    for s, (d, fr) in enumerate(zip(descs, frames)):
        an = vca.Analyzer(d["width"], d["height"], block_size=d["block_size"],
                          max_batch=d["n_frames"])
        an.submit(*fr)
        ref = an.features(0, d["n_frames"])
        an.close()
        assert got[s].tobytes() == ref.tobytes(), f"stream {s} ({d}) differs from the plain path"

    for s, (d, fr) in enumerate(zip(descs, frames)):
        t = sampled_frame(s, d["n_frames"])
        t0 = max(0, t - 1)
        y, u, v = (p[t0:t + 1].cpu().numpy() for p in fr)
        ocfg = oracle.Config(d["width"], d["height"], 8, d["block_size"], 0)
        ref = oracle.analyze(ocfg, y, u, v, threads=8).features
        assert_features_close(got[s][t:t + 1], ref[-1][None])
    del frames, vids
    torch.cuda.empty_cache()
