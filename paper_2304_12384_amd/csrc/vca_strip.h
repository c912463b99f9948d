// vca_strip.h -- strips of 32 x 32 tiles, the work unit of the plain and the
// batched forward kernels.
//
// A strip is a run of up to kStrip consecutive tiles of one plane of one
// frame: for w = 32 (a tile is one block) on planes at least kStrip blocks
// wide, kStrip consecutive blocks in raster order, wrapping at most once
// from one block row to the next, so that only the plane's last strip can be
// short; otherwise up to kStrip tiles of one tile row.  A wavefront decodes a strip once (scalar loads of one plane record),
// addresses every tile as a scalar base + a 32-bit lane offset computed once
// per strip, and transforms the strip in units of kPack = w / K tiles that
// share one MFMA tile (vca_tile.h, packed layout).  For w = 32 the FP64
// energy shares of the strip's tiles are reduced together at the end of the
// strip.
#pragma once

#include "vca_host.h"
#include "vca_tile.h"

namespace vca {

constexpr int kStrip = 8;   // tiles per strip

// One plane as the strip decoder sees it.
// 64 bytes, so that the strip decoder reads a record with one wide scalar
// load.
struct alignas(16) StripPlane {
  const uint8_t* plane;    // first sample of frame 0
  int64_t fstride;         // bytes between frames
  int32_t pitch;           // bytes between rows
  int32_t nbx, nby, ntx;   // blocks per row / column, tiles per row
  int32_t spr;             // strips per tile row; 0: the strips follow the raster
                           // order of blocks (w = 32 and nbx >= kStrip)
  int32_t scnt;            // strips per plane
  int32_t boff;            // index of the plane's first block within a frame
  int32_t cnt;             // blocks of the plane
  FastDiv div_spr;         // / spr (row strips)
  FastDiv div_nbx;         // / nbx (raster-order strips)
};
static_assert(sizeof(StripPlane) == 64, "one 64-byte record per plane");

// The strips of a run of frames of one video.
struct StripGeom {
  StripPlane sp[3];
  int32_t strips_per_frame;
  FastDiv div_spf;         // / strips_per_frame
  int32_t per_frame;       // blocks per frame
  int32_t blk_base;        // output index of block 0 of the run's frame 0
  int32_t frame_base;      // index of the run's frame 0 in the launch's frame flags
};

// Host: strips of frames starting at base[P] (Y, U, V) with the given frame
// strides and pitches, outputs from block blk_base on.
inline StripGeom make_strip_geom(const Geometry& g, const uint8_t* const base[3],
                                 const int64_t fstride[3], const int64_t pitch[3],
                                 int32_t blk_base, int32_t frame_base = 0) {
  StripGeom G{};
  for (int P = 0; P < 3; P++) {
    StripPlane& sp = G.sp[P];
    sp.plane = base[P];
    sp.fstride = fstride[P];
    sp.pitch = (int32_t)pitch[P];
    sp.nbx = g.nbx[P];
    sp.nby = g.nby[P];
    sp.ntx = g.ntx[P];
    sp.cnt = g.cnt[P];
    // w = 32 on planes at least kStrip blocks wide: strips of kStrip
    // consecutive blocks along the raster order (at most one row wrap each)
    const bool linear = g.w == kTile && sp.nbx >= kStrip;
    const int32_t spr = (g.ntx[P] + kStrip - 1) / kStrip;
    sp.spr = linear ? 0 : spr;
    sp.scnt = linear ? (sp.cnt + kStrip - 1) / kStrip : spr * (g.tcnt[P] / g.ntx[P]);
    sp.boff = g.boff[P];
    sp.div_spr = make_fastdiv((uint32_t)spr);
    sp.div_nbx = make_fastdiv((uint32_t)sp.nbx);
  }
  G.strips_per_frame = G.sp[0].scnt + G.sp[1].scnt + G.sp[2].scnt;
  G.div_spf = make_fastdiv((uint32_t)G.strips_per_frame);
  G.per_frame = g.per_frame;
  G.blk_base = blk_base;
  G.frame_base = frame_base;
  return G;
}

struct StripWork {
  const uint8_t* base;  // first sample of the strip's first tile
  int64_t wrap_delta;   // w = 32: bytes from the end of a block row to the next row's start
  int32_t wrap_t;       // w = 32: tiles t >= wrap_t lie on the next block row
  int32_t pitch;
  int32_t n;            // tiles in the strip, 1..kStrip
  int32_t out0;         // output index of block (0, 0) of the first tile
  int32_t out_row;      // output index step between block rows
  int32_t vr;           // block rows of the strip inside the grid
  int32_t vc_last;      // block columns of the last tile inside the grid
  int32_t row0;         // output index of block (0, 0) of the strip's tile row
  int32_t frame;        // the strip's frame in the launch's frame flags
};

// Strip `id` (frame-major, then Y, U, V, then tile rows, then strips along a
// row).
template <int kBits, int kW, bool kDs = false>
__device__ inline StripWork decode_strip(const StripGeom& G, int id) {
  constexpr int kBps = kBits == 8 ? 1 : 2;
  constexpr int kBpt = kTile / kW;
  constexpr int kScale = kDs ? 2 : 1;   // input samples per analysed sample, each way
  const int f = (int)fastdiv((uint32_t)id, G.div_spf);
  int r = id - f * G.strips_per_frame;
  int P = 0;
  if (r >= G.sp[0].scnt) {
    r -= G.sp[0].scnt;
    P = 1;
    if (r >= G.sp[1].scnt) {
      r -= G.sp[1].scnt;
      P = 2;
    }
  }
  const StripPlane& pl = G.sp[P];
  if constexpr (kW == kTile) {
    // blocks i0 .. i0 + n - 1 in raster order: linear strips of kStrip
    // blocks, else the strips of each block row
    int i0, by, c0, n;
    if (pl.spr == 0) {
      i0 = r * kStrip;
      by = (int)fastdiv((uint32_t)i0, pl.div_nbx);
      c0 = i0 - by * pl.nbx;
      n = min(kStrip, pl.cnt - i0);
    } else {
      by = (int)fastdiv((uint32_t)r, pl.div_spr);
      c0 = (r - by * pl.spr) * kStrip;
      i0 = by * pl.nbx + c0;
      n = min(kStrip, pl.nbx - c0);
    }
    StripWork w;
    w.pitch = pl.pitch;
    w.n = n;
    w.base = pl.plane + f * pl.fstride + (int64_t)by * kTile * kScale * w.pitch + c0 * kTile * kBps * kScale;
    w.wrap_t = pl.nbx - c0;
    w.wrap_delta = (int64_t)kTile * kScale * w.pitch - (int64_t)pl.nbx * kTile * kBps * kScale;
    w.vr = 1;
    w.vc_last = 1;
    w.out0 = G.blk_base + f * G.per_frame + pl.boff + i0;
    w.row0 = w.out0;
    w.out_row = pl.nbx;
    w.frame = G.frame_base + f;
    return w;
  }
  const int ty = (int)fastdiv((uint32_t)r, pl.div_spr);
  const int tx0 = (r - ty * pl.spr) * kStrip;
  StripWork w;
  w.pitch = pl.pitch;
  w.wrap_t = kStrip;
  w.wrap_delta = 0;
  w.n = min(kStrip, pl.ntx - tx0);
  const int by0 = ty * kBpt, bx0 = tx0 * kBpt;
  w.base = pl.plane + f * pl.fstride + (int64_t)by0 * kW * kScale * w.pitch + bx0 * kW * kBps * kScale;
  w.vr = min(kBpt, pl.nby - by0);
  w.vc_last = min(kBpt, pl.nbx - (tx0 + w.n - 1) * kBpt);
  w.out0 = G.blk_base + f * G.per_frame + pl.boff + by0 * pl.nbx + bx0;
  w.row0 = w.out0 - bx0;
  w.out_row = pl.nbx;
  w.frame = G.frame_base + f;
  return w;
}

// Byte offsets of a lane's samples inside the tiles of a strip (scalar tile
// base + 32-bit lane offset keeps every load in the saddr form): `a` (and,
// for 10-bit, `b`) for full tiles, and the same for the strip's last tile.
// Rows past the block grid (bottom tile row) and 16-byte pieces past it (last
// tile of a row) are redirected to the strip's first valid row / the lane's
// first valid piece: a piece that starts inside the block grid lies inside
// the row's pitch (a multiple of 16 bytes), so every access stays in bounds;
// the redirected data only feeds blocks that are discarded.
struct LaneOffsets {
  uint32_t a, b, last_a, last_b;
};

// Downsampled (kDs): the analysed row r comes from input rows 2r and 2r + 1
// (the second at + pitch), output columns c..c+7 from input columns 2c..2c+15;
// `a` and `b` are the byte offsets of the pieces of output columns 16g..16g+7
// and 16g+8..16g+15 (whole tiles), last_a / last_b the same for the strip's
// last tile, redirected like the plain layout's pieces.
template <int kBits, int kW, bool kDs = false>
__device__ inline LaneOffsets lane_offsets(const StripWork& s, int lane) {
  constexpr int kBps = kBits == 8 ? 1 : 2;
  constexpr int kScale = kDs ? 2 : 1;
  const int r = lane & 31, g = lane >> 5;
  const int rows = s.vr * kW;
  const uint32_t roff =
      __umul24((uint32_t)(kScale * (kW == 32 || r < rows ? r : 0)), (uint32_t)s.pitch);
  LaneOffsets o;
  o.a = roff + 16 * g * kBps * kScale;
  o.b = o.a + 8 * kBps * kScale;
  if (kW == 32) {            // a w = 32 tile is one complete block
    o.last_a = o.a;
    o.last_b = o.b;
  } else {
    const int cols = s.vc_last * kW;
    const int c0 = 16 * g < cols ? 16 * g : 0;
    const int c1 = 16 * g + 8 < cols ? 16 * g + 8 : c0;
    o.last_a = roff + c0 * kBps * kScale;
    o.last_b = roff + c1 * kBps * kScale;
  }
  return o;
}

// 2 x 2 means, rounded half up, of two input rows' dwords: 8-bit, four input
// samples per dword -> output samples 2q, 2q + 1 of the piece in the 16-bit
// halves, as (sum + 2) (shift still to come).
__device__ inline uint32_t sum4_u8(uint32_t r0, uint32_t r1) {
  const uint32_t e0 = __builtin_amdgcn_perm(r0, r0, 0x0C020C00u);   // bytes 0, 2 -> halves
  const uint32_t o0 = __builtin_amdgcn_perm(r0, r0, 0x0C030C01u);   // bytes 1, 3
  const uint32_t e1 = __builtin_amdgcn_perm(r1, r1, 0x0C020C00u);
  const uint32_t o1 = __builtin_amdgcn_perm(r1, r1, 0x0C030C01u);
  return e0 + e1 + o0 + o1 + 0x00020002u;   // each half <= 1022 + 2: no carry across
}

// Four output samples (bytes) from two dwords of 16-bit (sum + 2).
__device__ inline uint32_t pack4_u8(uint32_t s01, uint32_t s23) {
  const uint32_t a = (s01 >> 2) & 0x00FF00FFu, b = (s23 >> 2) & 0x00FF00FFu;
  return __builtin_amdgcn_perm(b, a, 0x06040200u);
}

// 10-bit: one dword of each row (two input samples each) -> one output sample,
// with any bit above 1023 of the inputs carried into bits 10..15 (so that a
// validation of the output samples sees it).
__device__ inline uint32_t mean4_u16(uint32_t r0, uint32_t r1) {
  const uint32_t s = r0 + r1;                       // two 16-bit sums <= 2046 each
  const uint32_t t = (s & 0xFFFFu) + (s >> 16) + 2u;
  return ((t >> 2) & 0x3FFu) | (((r0 | r1) & 0xFC00FC00u) ? 0xFC00u : 0u);
}

template <int kBits>
__device__ inline TileData downsample_tile(const uint8_t* row0, uint32_t oa, uint32_t ob,
                                           int64_t pitch) {
  const uint8_t* row1 = row0 + pitch;
  TileData d;
  if (kBits == 8) {
    // pieces: 16 input bytes -> 8 output samples
    const v4i a0 = *reinterpret_cast<const v4i*>(row0 + oa);
    const v4i a1 = *reinterpret_cast<const v4i*>(row1 + oa);
    const v4i b0 = *reinterpret_cast<const v4i*>(row0 + ob);
    const v4i b1 = *reinterpret_cast<const v4i*>(row1 + ob);
    d.a[0] = (int)pack4_u8(sum4_u8(a0[0], a1[0]), sum4_u8(a0[1], a1[1]));
    d.a[1] = (int)pack4_u8(sum4_u8(a0[2], a1[2]), sum4_u8(a0[3], a1[3]));
    d.a[2] = (int)pack4_u8(sum4_u8(b0[0], b1[0]), sum4_u8(b0[1], b1[1]));
    d.a[3] = (int)pack4_u8(sum4_u8(b0[2], b1[2]), sum4_u8(b0[3], b1[3]));
  } else {
    // pieces: 32 input bytes (16 samples) -> 8 output samples
    v4i in0[4], in1[4];
    in0[0] = *reinterpret_cast<const v4i*>(row0 + oa);
    in0[1] = *reinterpret_cast<const v4i*>(row0 + oa + 16);
    in0[2] = *reinterpret_cast<const v4i*>(row0 + ob);
    in0[3] = *reinterpret_cast<const v4i*>(row0 + ob + 16);
    in1[0] = *reinterpret_cast<const v4i*>(row1 + oa);
    in1[1] = *reinterpret_cast<const v4i*>(row1 + oa + 16);
    in1[2] = *reinterpret_cast<const v4i*>(row1 + ob);
    in1[3] = *reinterpret_cast<const v4i*>(row1 + ob + 16);
    uint32_t out[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const int piece = k / 2, q = (k % 2) * 2;
      const uint32_t lo = mean4_u16((uint32_t)in0[piece][q], (uint32_t)in1[piece][q]);
      const uint32_t hi = mean4_u16((uint32_t)in0[piece][q + 1], (uint32_t)in1[piece][q + 1]);
      out[k] = lo | (hi << 16);
    }
    d.a = v4i{(int)out[0], (int)out[1], (int)out[2], (int)out[3]};
    d.b = v4i{(int)out[4], (int)out[5], (int)out[6], (int)out[7]};
  }
  return d;
}

// First sample of tile t of a strip (scalar): w = 32 tiles follow the raster
// order of blocks and may continue on the next block row (once).
template <int kBits, int kW, bool kDs = false>
__device__ inline const uint8_t* tile_base(const StripWork& s, int t) {
  constexpr int kBps = kBits == 8 ? 1 : 2;
  constexpr int kScale = kDs ? 2 : 1;
  const uint8_t* b = s.base + t * (kTile * kBps * kScale);
  if constexpr (kW == kTile) b += t >= s.wrap_t ? s.wrap_delta : 0;
  return b;
}

template <int kBits, int kW, bool kDs = false>
__device__ inline TileData strip_load(const StripWork& s, const LaneOffsets& o, int t) {
  const bool last = kW != 32 && t == s.n - 1;
  if constexpr (kDs) {
    return downsample_tile<kBits>(tile_base<kBits, kW, true>(s, t), last ? o.last_a : o.a,
                                  last ? o.last_b : o.b, s.pitch);
  }
  const uint8_t* base = tile_base<kBits, kW>(s, t);
  TileData d;
  d.a = *reinterpret_cast<const v4i*>(base + (last ? o.last_a : o.a));
  if (kBits != 8) d.b = *reinterpret_cast<const v4i*>(base + (last ? o.last_b : o.b));
  return d;
}

// Strips are taken in runs of kRunLen consecutive strip ids (kRun unless a
// launch is too small to fill the device with runs that long): this
// wavefront runs run0, run0 + run_stride, ... (strips below `end`).  Consecutive strips
// own consecutive output ranges when w = 32 (a tile is a block and the tile
// grid is the block grid), so a run's H and DC are gathered into the lanes
// (lane i = block i of the run) and stored with one store each at the run's
// end: a store's completion counts in vmcnt like a load's, and one per strip
// stalled the loads queued behind it.
//
// Loads: ring slot u % kDepth holds unit u of the strip until its horizontal
// pass, and is then refilled with unit u + kDepth, which may lie in the next
// strip (units per strip % kDepth == 0, so ring slots line up across
// strips).  Every unit issues the same loads whatever the strip length (tile
// indices are clamped into the strip, and the last strip prefetches itself
// again), so the compiler waits for exactly the oldest unit's loads; the
// missing tiles of a short strip are transformed but never stored.
//
// w = 16 and 8: a tile holds several blocks, each spread over 2 K lanes
// with one FP64 share per block row.  Each unit's shares (and the lanes'
// row-0 coefficients, the DC candidates) go to a per-wavefront LDS area,
// lane-major, with no arithmetic; every LdsGroup units the lanes read them
// back block by block (RedMap below), sum a block's shares in 8-term chunks
// and combine a block's chunks across adjacent lanes, and one lane per block
// writes its H and DC into the segment of the tile row being walked (block
// row x block column, up to seg_cols(w) columns) -- copied out with
// row-contiguous stores when the next strip leaves the tile row, would
// overflow it, or the run ends.
constexpr int kRun = 8;   // strips per run (w = 32: at most 64 blocks, one per lane)

// Block columns of a staged segment (w = 16, 8): 3 KiB of H and DC.
constexpr int seg_cols(int w) { return w == 16 ? 128 : 64; }

// LDS bytes of one wavefront's staging area: w = 32, the DC of the run's 64
// blocks; else the shares of one group (4 KiB), the DC candidates of one
// group (2 KiB), then the segment's FP64 H and int32 DC.
constexpr int kLdsShareBytes = 8 * 64 * 8;   // LdsGroup units x block rows = 8 share rows
constexpr int kLdsDcBytes = 8 * 64 * 4;
constexpr int stage_bytes(int w) {
  return w == 32 ? 64 * 4 : kLdsShareBytes + kLdsDcBytes + (kTile / w) * seg_cols(w) * 12;
}

// The LDS reduction of w = 16, 8 units: per group of kGroup units, share
// row (ul, b) holds the 64 lanes' shares of block row b of unit ul.  Block
// beta = ((ul * kBpt + b) * kBpt + bc) * kPack + q of the group owns the
// lanes g * 32 + bc * w + q * K + k (g = 0, 1; k < K) of its share row.  The
// 64 reader lanes take kPer terms each: with 2 K >= kPer, kLanes = 2 K / kPer
// adjacent lanes share a block (chunk = lane % kLanes); otherwise a lane
// sums kBlocks = kPer / (2 K) consecutive blocks (consecutive q).
template <int kW, int kK>
struct RedMap {
  static constexpr int kBpt = kTile / kW;
  static constexpr int kPack = kW / kK;
  static constexpr int kUnits = kStrip / kPack;
  static constexpr int kGroup = (8 / kBpt) < kUnits ? (8 / kBpt) : kUnits;
  static constexpr int kPer = kGroup * kBpt;                 // terms per reader lane
  static constexpr int kLanes = 2 * kK >= kPer ? 2 * kK / kPer : 1;
  static constexpr int kBlocks = 2 * kK >= kPer ? 1 : kPer / (2 * kK);
  static constexpr int kNb = kGroup * kPack * kBpt * kBpt;   // blocks per group
  static_assert(kNb == 64 / kLanes * kBlocks, "every block read exactly once");
  static_assert(kPer % 2 == 0 && kK % 2 == 0, "terms read in aligned pairs");

  // Byte offset of the reader's term pair p (terms 2p, 2p + 1 of its
  // chunk, or of its blocks) from the reader's first term.
  static constexpr int pair_offset(int p) {
    if (kBlocks > 1) {                       // p: block p / (K), g and k within it
      const int per_block = kK;              // pairs per block: 2 K terms
      const int blk = p / per_block, r = p % per_block;
      return blk * kK * 8 + (r / (kK / 2)) * 32 * 8 + (r % (kK / 2)) * 16;
    }
    if (kK >= kPer) return p * 16;           // the chunk lies in one g half
    return (2 * p / kK) * 32 * 8 + (2 * p % kK) * 8;   // chunk = whole block, both halves
  }
  // The reader lane's first block and chunk, its share-row offset and the
  // block's (ul, b, bc, q).
  int beta, chunk, ul, b, bc, q;
  __device__ explicit RedMap(int lane) {
    beta = kBlocks > 1 ? lane * kBlocks : lane / kLanes;
    chunk = kBlocks > 1 ? 0 : lane % kLanes;
    q = beta % kPack;
    bc = (beta / kPack) % kBpt;
    b = (beta / (kPack * kBpt)) % kBpt;
    ul = beta / (kPack * kBpt * kBpt);
  }
  // byte offset of the reader's first term in the share area
  __device__ int first_term() const {
    const int t0 = chunk * kPer;             // term index within the block
    const int g = t0 / kK, k = t0 % kK;
    return ((ul * kBpt + b) * 64 + g * 32 + bc * kW + q * kK + k) * 8;
  }
  // byte offset of the block's DC candidate (lane g = 0, k = 0) in the DC area
  __device__ int dc_slot(int extra) const {
    return ((ul * kBpt + b) * 64 + bc * kW + (q + extra) * kK) * 4;
  }
};

// Coefficient export (VCA_F_KEEP_COEFFS, tests): the K x K coefficients of
// the blocks of unit u of strip S, DC corrected, at ((block * K + i) * K + k)
// of out.coeffs -- the same registers coeff_energy weighs, so the export shows
// exactly what the production walk computed.
template <int kBits, int kW, int kK, class PC>
__device__ inline void store_unit_coeffs(const TileOut& o, const StripWork& S, int u, const PC& pc,
                                         const v16i& dh, const v16i& dl, int lane) {
  constexpr int kS2 = ilog2c(kW) + 6;
  constexpr int kBpt = kTile / kW;
  constexpr int kPack = kW / kK;
  constexpr int kDcAdd = kBits == 8 ? kDcOffset : 0;
  const int c = lane & 31, g = lane >> 5;
  const int bc = c / kW, cc = c % kW, kk = cc % kK;
  const int t = u * kPack + cc / kK;   // the lane's sample tile within the strip
  const int vc = t == S.n - 1 ? S.vc_last : kBpt;
  if (t >= S.n || bc >= vc) return;
#pragma unroll
  for (int j = 0; j < 16; j++) {
    if (!reg_used(j, kW, kK)) continue;
    const int m = reg_row(j, g), br = m / kW, ii = m % kW;
    if (ii >= kK || br >= S.vr) continue;
    const int yv = (int)((uint32_t)dh[j] * 256u + (uint32_t)dl[j]) >> kS2;
    const int64_t blk = S.out0 + br * S.out_row + t * kBpt + bc;
    o.coeffs[(blk * kK + ii) * kK + kk] = (int16_t)(yv + (ii == 0 && kk == 0 ? kDcAdd : 0));
  }
}

template <int kBits, int kW, int kK, int kDepthMax, bool kDs = false, bool kValidate = false,
          int kRunLen = kRun, bool kKeep = false>
__device__ __forceinline__ void run_strips(const StripGeom& G, const TileOut& out,
                                           const PackConsts<kW, kK>& pc, int run0, int run_stride,
                                           int end, int lane, uint8_t* stage) {
  constexpr int kPack = kW / kK;
  constexpr int kUnits = kStrip / kPack;
  constexpr int kDepth = kDepthMax < kUnits ? kDepthMax : kUnits;
  constexpr int kBpt = kTile / kW;
  static_assert(kUnits % kDepth == 0, "ring slots must line up across strips");
  constexpr int kDcAdd = kBits == 8 ? kDcOffset : 0;
  struct Unit {
    TileData t[kPack];
  };
  const int c = lane & 31, g = lane >> 5;
  const int cc = c % kW, q = cc / kK;   // lane's column and tile within its unit

  auto load_unit = [&](const StripWork& S, const LaneOffsets& O, int u) {
    Unit d;
#pragma unroll
    for (int i = 0; i < kPack; i++) d.t[i] = strip_load<kBits, kW, kDs>(S, O, min(u * kPack + i, S.n - 1));
    return d;
  };
  // the strip after `id` in this wavefront's sequence
  auto next_id = [&](int id) {
    return (id + 1) % kRunLen != 0 ? id + 1 : id + 1 + (run_stride - 1) * kRunLen;
  };

  int id = run0 * kRunLen;
  if (id >= end) return;
  StripWork S = decode_strip<kBits, kW, kDs>(G, id);
  LaneOffsets O = lane_offsets<kBits, kW, kDs>(S, lane);
  Unit ring[kDepth];
#pragma unroll
  for (int u = 0; u < kDepth; u++) ring[u] = load_unit(S, O, u);
  const v16i c2 = stage2_bias<kW>(lane);
  // w = 32: the current run's blocks, lane i holding block run_out0 + i;
  // w < 32: the staged segment starts at block run_out0 (row 0 of its tile row)
  double hrun = 0.0;
  int run_out0 = S.out0;
  uint32_t seen = 0;   // kValidate: OR of every sample of the current strip
  constexpr int kSeg = seg_cols(kW);
  int* st_run_dc = reinterpret_cast<int*>(stage);              // w = 32: [64] DC of the run
  // w < 32: the group's shares and DC candidates, then the segment
  double* st_share = reinterpret_cast<double*>(stage);         // [share row][64 lanes]
  int* st_dcc = reinterpret_cast<int*>(stage + kLdsShareBytes);  // [share row][64 lanes]
  double* st_h = reinterpret_cast<double*>(stage + kLdsShareBytes + kLdsDcBytes);  // [kBpt][kSeg]
  int* st_dc = reinterpret_cast<int*>(st_h + kBpt * kSeg);     // [kBpt][kSeg]
  using RM = RedMap<kW, kK>;
  // w < 32, per reader lane: its first share and DC candidate (bytes), its
  // first block's tile within the group (past every tile for lanes that
  // read a later chunk: they never write), block column and segment row
  int red_first = 0, red_dc = 0, red_t = 0, red_bc = 0, red_row = 0;
  if constexpr (kW != 32) {
    const RM rm(lane);
    red_first = rm.first_term();
    red_dc = rm.dc_slot(0);
    red_t = rm.chunk == 0 ? rm.ul * kPack + rm.q : 1 << 20;
    red_bc = rm.bc;
    red_row = rm.b * kSeg;
  }

  while (true) {
    const int id2 = next_id(id);
    const bool more = id2 < end;
    StripWork S2 = S;
    LaneOffsets O2 = O;
    if (more) {
      S2 = decode_strip<kBits, kW, kDs>(G, id2);
      O2 = lane_offsets<kBits, kW, kDs>(S2, lane);
    }
    double hs[kUnits];
    int dcs[kUnits];
    // energies of unit u of this strip from its vertical-pass accumulators
    auto finish = [&](int u, const v16i& dh, const v16i& dl) {
      double h[kBpt];
      int dc[kBpt];
      coeff_energy<kBits, kW, kK>(pc, dh, dl, h, dc);
      if constexpr (kKeep) store_unit_coeffs<kBits, kW, kK>(out, S, u, pc, dh, dl, lane);
      if constexpr (kW == 32) {
        hs[u] = h[0];
        dcs[u] = dc[0];
      } else {
        // the unit's shares and DC candidates into the group's share rows
        const int ul = u % RM::kGroup;
#pragma unroll
        for (int b = 0; b < kBpt; b++) {
          st_share[(ul * kBpt + b) * 64 + lane] = h[b];
          st_dcc[(ul * kBpt + b) * 64 + lane] = dc[b];
        }
        if (ul == RM::kGroup - 1) {
          // the group's blocks: sum each reader's terms, then its chunks
          const uint8_t* sh = reinterpret_cast<const uint8_t*>(st_share) + red_first;
          constexpr int kPairs = RM::kPer / 2 / RM::kBlocks;   // pairs per block
          double sum[RM::kBlocks];
#pragma unroll
          for (int k = 0; k < RM::kBlocks; k++) {
#pragma unroll
            for (int p = 0; p < kPairs; p++) {
              const double2 v =
                  *reinterpret_cast<const double2*>(sh + RM::pair_offset(k * kPairs + p));
              sum[k] = p == 0 ? v.x + v.y : sum[k] + (v.x + v.y);
            }
            if constexpr (RM::kLanes >= 2) sum[k] += dpp64<kDppXor1>(sum[k]);
            if constexpr (RM::kLanes >= 4) sum[k] += dpp64<kDppXor2>(sum[k]);
          }
          // one writer per block: its H and DC into the segment
          const int t0 = (u / RM::kGroup) * RM::kGroup * kPack + red_t;
#pragma unroll
          for (int k = 0; k < RM::kBlocks; k++) {
            const int t = t0 + k;   // the block's tile within the strip
            const int vc = t == S.n - 1 ? S.vc_last : kBpt;
            if (t < S.n && red_bc < vc) {
              const int col = S.out0 - run_out0 + t * kBpt + red_bc;
              st_h[red_row + col] = sum[k];
              st_dc[red_row + col] = st_dcc[(red_dc >> 2) + k * kK] + kDcAdd;
            }
          }
        }
      }
    };
#pragma unroll
    for (int u = 0; u < kUnits; u++) {
      const Unit d = ring[u % kDepth];
      const int v = u + kDepth;   // the unit whose loads go out now
      ring[u % kDepth] = v < kUnits ? load_unit(S, O, v) : load_unit(S2, O2, v - kUnits);
      v16i dh, dl;
      mfma2(pc.a2, split2<kBits, kW>(stage1_sum<kBits>(stage1_acc<kBits, kW, kPack>(pc.b1, d.t, seen))),
            c2, dh, dl);
      finish(u, dh, dl);
    }
    if constexpr (kW == 32) {
      // Sum each tile's shares; tile_lane(t) is a lane holding tile t's total.
      double h;
      auto tile_lane = [](int t) {
        if constexpr (kPack == 2) return 32 * (t >> 2) + 8 * ((t >> 1) & 1) + 16 * (t & 1);
        else return 8 * t;
      };
      if constexpr (kPack == 1) h = reduce_scatter8(hs, lane);
      else if constexpr (kPack == 2) h = reduce_scatter4x2(hs, lane);
      else h = reduce_scatter2x4(hs);
      // gather into the run's lanes: lane run position + t <- tile t
      const int t = lane - (S.out0 - run_out0);
      const bool in_strip = t >= 0 && t < S.n;
      const double ht = __shfl(h, in_strip ? tile_lane(t) : lane);
      if (in_strip) hrun = ht;
      // DC of tile u * kPack + q (register dcs[u] of the lane with c = q K,
      // g = 0) into the wavefront's LDS row at run position + tile, read back
      // by lane = position at the run's end; positions past the strip's last
      // tile are rewritten by the next strip of the run or not stored
      const int pos0 = S.out0 - run_out0;
      if (g == 0 && cc % kK == 0) {
#pragma unroll
        for (int u = 0; u < kUnits; u++) st_run_dc[pos0 + u * kPack + q] = dcs[u];
      }
      if (!more || id2 % kRunLen == 0) {   // the run ends with this strip
        if (lane < S.out0 - run_out0 + S.n) {
          out.blk_h[run_out0 + lane] = hrun;
          out.blk_dc[run_out0 + lane] = st_run_dc[lane] + kDcAdd;
        }
        run_out0 = S2.out0;
      }
    }
    if constexpr (kW != 32) {
      // copy the segment out when the next strip leaves it
      const bool leave = !more || id2 % kRunLen == 0 || S2.row0 != S.row0 ||
                         S2.out0 - run_out0 + kStrip * kBpt > kSeg;
      if (leave) {
        const int cols = S.out0 - run_out0 + (S.n - 1) * kBpt + S.vc_last;
        for (int b = 0; b < S.vr; b++) {
          for (int cb = 0; cb < cols; cb += 64) {
            const int col = cb + lane;
            if (col < cols) {
              out.blk_h[run_out0 + b * S.out_row + col] = st_h[b * kSeg + col];
              out.blk_dc[run_out0 + b * S.out_row + col] = st_dc[b * kSeg + col];
            }
          }
        }
        run_out0 = S2.out0;
      }
    }
    // kValidate: a flagged sample of the strip marks its frame (the
    // reduction moves the mark into the frame's slot of the feature ring)
    if constexpr (kValidate) {
      if (out.validate && (seen & kOver10Bits)) out.err_flag[S.frame] = 1;
      seen = 0;
    }
    if (!more) break;
    id = id2;
    S = S2;
    O = O2;
  }
}

}  // namespace vca
