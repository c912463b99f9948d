"""Seeded synthetic YUV 4:2:0 video for the tests, the smoke check and the benchmark.

This package only draws pixels.  It holds none of the analyser's arithmetic,
so both the HIP path and the CPU oracle can be fed from it.
"""
from .video import (SEED_BASE, Video, SceneVideo, make_rng, patches_video, scene_video,
                    stress_video, batch_streams)

__all__ = ["SEED_BASE", "Video", "SceneVideo", "make_rng", "patches_video", "scene_video",
           "stress_video", "batch_streams"]
