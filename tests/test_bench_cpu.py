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


def test_algorithmic_bytes_per_2160p_frame():
    # w = 32: 120 x 67 luma blocks and 2 x 60 x 33 chroma blocks of 1024 samples
    assert bench.algorithmic_bytes_per_frame(3840, 2160, 32) == (120 * 67 + 2 * 60 * 33) * 1024
    assert bench.algorithmic_bytes_per_frame(3840, 2160, 32) == 12_288_000
    # w = 16: 240 x 135 and 2 x 120 x 67 blocks of 256 samples
    assert bench.algorithmic_bytes_per_frame(3840, 2160, 16) == (240 * 135 + 2 * 120 * 67) * 256
    # w = 8 covers every sample of a 2160p frame
    assert bench.algorithmic_bytes_per_frame(3840, 2160, 8) == 3840 * 2160 * 3 // 2


def test_downsampled_bytes_per_2160p_frame():
    # the half-size video's blocks (60 x 33 luma, 2 x 30 x 16 chroma), each
    # analysed sample the mean of four input samples
    assert bench.downsampled_bytes_per_frame(3840, 2160, 32) == 4 * (60 * 33 + 2 * 30 * 16) * 1024
    assert bench.downsampled_bytes_per_frame(3840, 2160, 32) == 12_042_240


def test_matrix_core_ops_per_2160p_frame():
    product = 2 * 32 * 32 * 32        # int8 ops of one 32x32x32 product
    tiles = 120 * 67 + 2 * 60 * 33     # w = 32: one block per 32 x 32 tile
    # full transform: horizontal pass + hi and lo vertical passes per tile
    assert bench.mfma_ops_per_frame(3840, 2160, 32) == tiles * 3 * product
    # K = 16: two sample tiles share one pair of vertical-pass products
    assert bench.mfma_ops_per_frame(3840, 2160, 32, 16) == tiles * 2 * product
    # K = 8: four sample tiles share them
    assert bench.mfma_ops_per_frame(3840, 2160, 32, 8) == tiles * 6 // 4 * product
    # w = 16: four blocks per 32 x 32 tile
    tiles16 = (240 * 135 + 2 * 120 * 67) // 4
    assert bench.mfma_ops_per_frame(3840, 2160, 16) == tiles16 * 3 * product


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
