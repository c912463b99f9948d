"""bench.py's fixed arithmetic and its refusal of several GPUs, on the CPU.

The roofline figures divide the algorithmic bytes (or matrix-core
operations) per frame by a measured kernel time; these pin those per-frame
numbers to values worked out by hand from the block grid of Section 2's
block DCT (complete w x w blocks anchored at the origin, 4:2:0 chroma).
"""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_frame_bytes():
    # every sample of Y (3840 x 2160) and of U and V (1920 x 1080) once
    assert bench.frame_bytes(3840, 2160) == 12_441_600
    assert bench.frame_bytes(3840, 2160, 10) == 24_883_200       # uint16 samples
    assert bench.frame_bytes(1920, 1080, 10) == 6_220_800
    assert bench.frame_bytes(1280, 720) == 1_382_400


def test_algorithmic_int8_ops_per_2160p_frame():
    blocks = 120 * 67 + 2 * 60 * 33     # w = 32, complete blocks only
    assert bench.block_count(3840, 2160, 32) == blocks == 12_000
    # per block w*K*w + K*K*w multiply-adds, 2 ops each
    assert bench.int8_ops_per_frame(3840, 2160, 32) == blocks * 2 * 2 * 32 ** 3
    assert bench.int8_ops_per_frame(3840, 2160, 32) == 1_572_864_000
    assert bench.int8_ops_per_frame(3840, 2160, 32, 16) == blocks * 2 * (16 * 32 * 32 + 16 * 16 * 32)
    assert bench.int8_ops_per_frame(3840, 2160, 32, 16) == 589_824_000


def test_matrix_core_issued_ops_per_2160p_frame():
    product = 2 * 32 * 32 * 32        # int8 ops of one 32x32x32 product
    tiles = 120 * 67 + 2 * 60 * 33     # w = 32: one block per 32 x 32 tile
    # full transform: horizontal pass + hi and lo vertical passes per tile
    assert bench.mfma_issued_ops_per_frame(3840, 2160, 32) == tiles * 3 * product
    # K = 16: two sample tiles share one pair of vertical-pass products
    assert bench.mfma_issued_ops_per_frame(3840, 2160, 32, 16) == tiles * 2 * product
    # K = 8: four sample tiles share them
    assert bench.mfma_issued_ops_per_frame(3840, 2160, 32, 8) == tiles * 6 // 4 * product
    # w = 16: four blocks per 32 x 32 tile
    tiles16 = (240 * 135 + 2 * 120 * 67) // 4
    assert bench.mfma_issued_ops_per_frame(3840, 2160, 16) == tiles16 * 3 * product
    # 10-bit: two horizontal-pass products per tile
    assert bench.mfma_issued_ops_per_frame(3840, 2160, 32, 0, 10) == tiles * 4 * product


def test_small_streams_workload():
    d = bench.small_streams()
    assert len(d) == 256
    assert {(s["width"], s["height"], s["n_frames"]) for s in d} == {(640, 360, 8)}
    assert [s["block_size"] for s in d[:6]] == [8, 16, 32, 8, 16, 32]


def test_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_summary_parses_and_attaches():
    """The committed traffic summary parses (it is ignored once the kernel
    sources no longer hash to its recorded value), and each covered record
    of a bench line gets its own per-launch bytes."""
    t = bench.measured_traffic()
    assert t is None or {"full", "lowpass", "w16", "w8"} <= set(t)
    line = {"config": {"lowpass_k": 0}, "roofline": {},
            "lowpass_k16": {"roofline": {}}, "lowpass_downsample": {"roofline": {}},
            "block_sizes_8bit": {"w16": {"roofline": {}}, "w8": {"roofline": {}}, "workload": "x"},
            "tenbit_stress": {"3840x2160_w32": {"roofline": {}}, "workload": "y"}}
    bench.attach_traffic(line, {"full": 1, "lowpass": 2, "downsample": 3, "w16": 4, "w8": 5,
                                "tenbit_3840x2160_w32": 6})
    assert line["roofline"]["traffic"] == 1
    assert line["lowpass_k16"]["roofline"]["traffic"] == 2
    assert line["lowpass_downsample"]["roofline"]["traffic"] == 3
    assert line["block_sizes_8bit"]["w16"]["roofline"]["traffic"] == 4
    assert line["block_sizes_8bit"]["w8"]["roofline"]["traffic"] == 5
    assert line["tenbit_stress"]["3840x2160_w32"]["roofline"]["traffic"] == 6
    only_k16 = {"config": {"lowpass_k": 16}, "roofline": {}}
    bench.attach_traffic(only_k16, {"full": 1, "lowpass": 2})
    assert only_k16["roofline"]["traffic"] == 2
    bench.attach_traffic(only_k16, None)
