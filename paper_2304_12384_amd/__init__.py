"""MI355X (gfx950) Video Complexity Analyzer.

Per-frame block-DCT complexity features (E_Y, h, L_Y, E_U, E_V, L_U, L_V) of
Menon et al., "Green Video Complexity Analysis for Efficient Encoding in
Adaptive Video Streaming", Section 2, computed by hand-written HIP kernels
behind the C ABI in include/vca.h.
"""
from ._lib import VcaError, EXPORTS, LIB_PATH
from .analyzer import (Analyzer, Batch, PreparedFrames, FEATURE_NAMES, analyze_noalloc, block_counts,
                       read_yuv, write_yuv)
from .grad import VCAEnergyFn, energy_features

__all__ = ["Analyzer", "Batch", "PreparedFrames", "FEATURE_NAMES", "analyze_noalloc", "block_counts",
           "read_yuv", "write_yuv",
           "VcaError", "EXPORTS", "LIB_PATH",
           "VCAEnergyFn", "energy_features"]
