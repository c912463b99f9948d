// vca_tile.h -- the 32 x 32 MFMA tile of the VCA forward transform (gfx950).
//
// A tile is a 32 x 32 region of one plane holding (32/w)^2 blocks of w x w
// (w in {8, 16, 32}).  One wavefront transforms one tile:
//   * lane (r + 32 g) loads row r, samples 16g..16g+15 of the tile;
//   * horizontal pass T = X' Cd^T on v_mfma_i32_32x32x32_i8, Cd the
//     block-diagonal matrix diag(C_w, ..., C_w); 8-bit: X' = X - 128 as one
//     int8 byte; 10-bit: X = 256 t + lo, t in [0, 4], two int8 products;
//   * the accumulator (lane = column k, register j = row
//     m_j = 8 (j/4) + 4 g + j%4) is already the B-operand layout of the
//     vertical pass once its 16-bit values are split into int8 bytes;
//   * vertical pass Y = Cd T on two int8 MFMAs (hi and lo bytes of T);
//   * per lane, FP64 sums of W |Y| per block row, reduced over the lanes of
//     a block (permlane swaps and DPP) to the block energy H; DC is read in
//     place.
// Transform definition (Section 2 of the paper names the block-DCT features;
// the integer transform is the H.265 core transform): per block
//   T = floor((X C^T + 2^(s1-1)) / 2^s1),  s1 = log2 w + B - 9
//   Y = floor((C T   + 2^(s2-1)) / 2^s2),  s2 = log2 w + 6.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

namespace vca {

constexpr int kTile = 32;           // MFMA tile edge (samples)
constexpr int kDcOffset = 1 << 14;  // DC removed by the -2^(B-1) sample offset, exact for all w, B

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

// Row of coefficient register j in lane half g.
constexpr int reg_row(int j, int g) { return 8 * (j / 4) + 4 * g + (j % 4); }

// Register j holds a coefficient inside some block's K x K corner.
constexpr bool reg_used(int j, int w, int K) {
  return (reg_row(j, 0) % w) < K || (reg_row(j, 1) % w) < K;
}

// Register j holds the first row (i % w == 0) of a block for lanes with g = 0.
constexpr bool reg_block_row0(int j, int w) { return j % 4 == 0 && (8 * (j / 4)) % w == 0; }

// ---------------------------------------------------------------- host side
// Integer stand-ins for 64*sqrt(2)*cos(pi*t/64), t = 0..32 (H.265 core
// transform values; t = 32 is the zero of the cosine).
constexpr int kCosQuarter[33] = {90, 90, 90, 90, 89, 88, 87, 85, 83, 82, 80, 78, 75, 73, 70, 67, 64,
                                 61, 57, 54, 50, 46, 43, 38, 36, 31, 25, 22, 18, 13, 9,  4,  0};

// Entry (k, n) of the 32-point matrix via the quadrant of the angle k(2n+1).
inline int mat32(int k, int n) {
  if (k == 0) return 64;
  const int t = (k * (2 * n + 1)) & 127;
  if (t <= 32) return kCosQuarter[t];
  if (t <= 64) return -kCosQuarter[64 - t];
  if (t <= 96) return -kCosQuarter[t - 64];
  return kCosQuarter[128 - t];
}

// w-point matrix: the 32-point one restricted to every (32/w)-th row.
inline int matw(int w, int k, int n) { return mat32(k * (kTile / w), n); }

// Entry (a, b) of the 32 x 32 block-diagonal matrix diag(C_w, ..., C_w).
inline int matd(int w, int a, int b) { return a / w == b / w ? matw(w, a % w, b % w) : 0; }

// Energy weight of coefficient (i, k) of a w x w block (1-based frequencies).
inline double weight(int w, int i, int k) {
  const double q = (double)((i + 1) * (k + 1)) / (double)(w * w);
  return std::exp(std::fabs(q * q - 1.0));
}

// Per-lane MFMA operands and weights of the tile for block size w and
// low-pass size K: b1 = stage-1 B operand (16 bytes per lane), a2 = stage-2
// A operand (16 bytes per lane), wt[j * 64 + lane] = weight of the
// coefficient in register j of the lane (0 outside the K x K corners and at
// every DC).
inline void build_tile_tables(int w, int K, std::vector<int8_t>& b1, std::vector<int8_t>& a2,
                              std::vector<double>& wt) {
  b1.assign(64 * 16, 0);
  a2.assign(64 * 16, 0);
  wt.assign(16 * 64, 0.0);
  for (int lane = 0; lane < 64; lane++) {
    const int c = lane & 31, g = lane >> 5;
    for (int j = 0; j < 16; j++) {
      // stage 1: B[n][k] = Cd[k][n], n = 16 g + j (the samples each lane loads)
      b1[lane * 16 + j] = (int8_t)matd(w, c, 16 * g + j);
      // stage 2: A[i][m] = Cd[i][m], m = the row held by accumulator register j
      const int m = reg_row(j, g);
      a2[lane * 16 + j] = (int8_t)matd(w, c, m);
      // weight of output (i, k) = (m, c) held by register j of lane (c + 32 g)
      const int ii = m % w, kk = c % w;
      wt[j * 64 + lane] = (ii < K && kk < K && !(ii == 0 && kk == 0)) ? weight(w, ii, kk) : 0.0;
    }
  }
}

// Tables of the packed layout used when K < w: one 32 x 32 MFMA tile holds
// kPack = w / K sample tiles, sample tile p owning lanes whose column c has
// (c % w) / K == p.  b1p[(p * 64 + lane) * 16 + j] = stage-1 B operand of
// sample tile p (Cd row bc*w + kk, zero in other tiles' columns), wt as in
// build_tile_tables for the coefficient (row % w, c % w % K) of the lane's
// tile.  With K == w this is build_tile_tables' b1 and wt.
inline void build_packed_tables(int w, int K, std::vector<int8_t>& b1p, std::vector<double>& wt) {
  const int pack = w / K;
  b1p.assign((size_t)pack * 64 * 16, 0);
  wt.assign(16 * 64, 0.0);
  for (int lane = 0; lane < 64; lane++) {
    const int c = lane & 31, g = lane >> 5;
    const int bc = c / w, cc = c % w, p = cc / K, kk = cc % K;
    for (int j = 0; j < 16; j++) {
      const int n = 16 * g + j;   // the sample column this lane's byte j multiplies
      b1p[((size_t)p * 64 + lane) * 16 + j] = (int8_t)(n / w == bc ? matw(w, kk, n % w) : 0);
      const int ii = reg_row(j, g) % w;
      wt[j * 64 + lane] = (ii < K && !(ii == 0 && kk == 0)) ? weight(w, ii, kk) : 0.0;
    }
  }
}

// Division by an invariant d (Granlund-Montgomery, round-up multiplier):
// n / d = (umulhi(n, m) + n) >> l for 0 <= n < 2^31, with l = ceil(log2 d)
// and m = floor(2^32 (2^l - d) / d) + 1.  Keeps tile-id decoding scalar.
struct FastDiv {
  uint32_t m;
  uint32_t l;
};

inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) l++;
  const uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
  return FastDiv{(uint32_t)m, l};
}

// -------------------------------------------------------------- device side
__device__ inline uint32_t fastdiv(uint32_t n, FastDiv d) { return (__umulhi(n, d.m) + n) >> d.l; }

__device__ inline uint32_t perm_b32(uint32_t hi_src, uint32_t lo_src, uint32_t sel) {
  return __builtin_amdgcn_perm(hi_src, lo_src, sel);
}

// Raw samples of one lane: 8-bit uses a (16 samples), 10-bit a and b
// (8 uint16 samples each).
struct TileData {
  v4i a;
  v4i b;
};

// Outputs of the forward kernels.
struct TileOut {
  double* blk_h;      // block energies
  int32_t* blk_dc;    // block DC coefficients
  int16_t* coeffs;    // optional K x K coefficients per block
  int32_t* err_flag;  // per frame of the launch: set to 1 when a 10-bit sample of
                      // the frame exceeds 1023 (validation on)
  int32_t validate;
};

// A v16i with every element v, built at the matrix-core call that takes it
// as the accumulator input (zero is encoded in the instruction; other values
// the compiler copies into registers once per strip).
template <int kV>
__device__ __forceinline__ v16i splat16() {
  v16i c;
#pragma unroll
  for (int j = 0; j < 16; j++) c[j] = kV;
  return c;
}

// 10-bit samples need no offset: x = 256 t + lo with lo the sign-extended low
// byte and t = (x + 128) >> 8 in [0, 4], both int8.  The raw horizontal-pass
// result stays within [-2^14, 2^15) (its first column is at most 32 * 1023),
// so the T >> 8 byte of the split still fits int8, and DC needs no
// correction.  A pair of samples x0 | x1 << 16 gives t0 and t1 in bytes 0 and
// 2 of ((pair + 0x00800080) >> 8).
__device__ __forceinline__ void operands10(const TileData& d, v4i& hi, v4i& lo) {
  uint32_t tv[8];
#pragma unroll
  for (int q = 0; q < 4; q++) {
    tv[q] = ((uint32_t)d.a[q] + 0x00800080u) >> 8;
    tv[4 + q] = ((uint32_t)d.b[q] + 0x00800080u) >> 8;
  }
  lo[0] = (int)perm_b32((uint32_t)d.a[1], (uint32_t)d.a[0], 0x06040200u);
  lo[1] = (int)perm_b32((uint32_t)d.a[3], (uint32_t)d.a[2], 0x06040200u);
  lo[2] = (int)perm_b32((uint32_t)d.b[1], (uint32_t)d.b[0], 0x06040200u);
  lo[3] = (int)perm_b32((uint32_t)d.b[3], (uint32_t)d.b[2], 0x06040200u);
#pragma unroll
  for (int q = 0; q < 4; q++) hi[q] = (int)perm_b32(tv[2 * q + 1], tv[2 * q], 0x06040200u);
}

// 10-bit validation: the OR of a lane's samples; a bit in 0xFC00FC00 marks a
// sample above 1023.  Callers accumulate it and test it once per strip run
// (a conditional store per unit split the unit loop into branches and
// doubled the register allocation of the w = 32 kernels).
__device__ __forceinline__ uint32_t samples_or(const TileData& d) {
  uint32_t any = 0;
#pragma unroll
  for (int q = 0; q < 4; q++) any |= (uint32_t)d.a[q] | (uint32_t)d.b[q];
  return any;
}

constexpr uint32_t kOver10Bits = 0xFC00FC00u;

// Horizontal-pass accumulators of one unit: 8-bit needs lo only; 10-bit
// keeps the products of the high (t) and low bytes apart until the split,
// T_raw = 256 hi + lo.
struct Acc1 {
  v16i lo;
  v16i hi;
};

// Horizontal pass of kPack sample tiles into one accumulator: tile p's
// B operand b1[p] puts its coefficients in its own lanes (kPack = 1: the
// plain tile).  The first product adds the rounding 2^(s1-1).
template <int kBits, int kW, int kPack>
__device__ __forceinline__ Acc1 stage1_acc(const v4i (&b1)[kPack],
                                           const TileData (&d)[kPack], uint32_t& seen) {
  constexpr int kS1 = ilog2c(kW) + kBits - 9;
  Acc1 r;
  if (kBits == 8) {
    r.lo = __builtin_amdgcn_mfma_i32_32x32x32_i8(d[0].a ^ (int)0x80808080, b1[0],
                                                 splat16<1 << (kS1 - 1)>(), 0, 0, 0);   // x - 128
#pragma unroll
    for (int p = 1; p < kPack; p++)
      r.lo = __builtin_amdgcn_mfma_i32_32x32x32_i8(d[p].a ^ (int)0x80808080, b1[p], r.lo, 0, 0, 0);
  } else {
#pragma unroll
    for (int p = 0; p < kPack; p++) {
      v4i hi, lo;
      operands10(d[p], hi, lo);
      seen |= samples_or(d[p]);
      if (p == 0) {
        r.hi = __builtin_amdgcn_mfma_i32_32x32x32_i8(hi, b1[p], splat16<0>(), 0, 0, 0);
        r.lo = __builtin_amdgcn_mfma_i32_32x32x32_i8(lo, b1[p], splat16<1 << (kS1 - 1)>(), 0, 0, 0);
      } else {
        r.hi = __builtin_amdgcn_mfma_i32_32x32x32_i8(hi, b1[p], r.hi, 0, 0, 0);
        r.lo = __builtin_amdgcn_mfma_i32_32x32x32_i8(lo, b1[p], r.lo, 0, 0, 0);
      }
    }
  }
  return r;
}

// The rounded-up horizontal-pass accumulator X' Cd^T + 2^(s1-1).
template <int kBits>
__device__ __forceinline__ v16i stage1_sum(const Acc1& a) {
  if (kBits == 8) return a.lo;
  v16i d1;
#pragma unroll
  for (int j = 0; j < 16; j++) d1[j] = (int)((uint32_t)a.hi[j] * 256u + (uint32_t)a.lo[j]);
  return d1;
}

// Split of the horizontal-pass result and the vertical pass.  Exact split of
// T (-2^14 <= T < 2^15 for every w and B):
//   T = 256 T_hi + u,  T_hi = T >> 8 in [-64, 127],  u = T & 255,
// C T = 256 C T_hi + C (u - 128) + 128 C 1, the last term being 128 * 64 w
// on each block's row 0 and 0 elsewhere: exactly +128 after the 2^s2
// scaling.  Both the vertical pass's rounding 2^(s2-1) and that +128 ride in
// the hi accumulator's initial value (2^(s2-9), plus 2^(s2-1) on each
// block's row 0), so Y = (256 dh + dl) >> s2.
struct Split {
  v4i hi;   // T >> 8 bytes
  v4i lo;   // (T & 255) - 128 bytes
};

template <int kBits, int kW>
__device__ __forceinline__ Split split2(const v16i& d1) {
  constexpr int kS1 = ilog2c(kW) + kBits - 9;
  Split sp;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    // T of registers 4q..4q+3 in the low 16 bits of s0..s3: a 64-bit shift
    // of a register pair moves both (the upper word's low bits land above
    // bit 16 of the lower word, which the byte selection below ignores)
    uint64_t p01 = (((uint64_t)(uint32_t)d1[4 * q + 1] << 32) | (uint32_t)d1[4 * q + 0]) >> kS1;
    uint64_t p23 = (((uint64_t)(uint32_t)d1[4 * q + 3] << 32) | (uint32_t)d1[4 * q + 2]) >> kS1;
    // (empty asm, no instruction: keeps the compiler from splitting each
    // shift into two 32-bit ones; not volatile, so it does not pin the
    // schedule)
    asm("" : "+v"(p01), "+v"(p23));
    const uint32_t s0 = (uint32_t)p01, s1 = (uint32_t)(p01 >> 32);
    const uint32_t s2 = (uint32_t)p23, s3 = (uint32_t)(p23 >> 32);
    const uint32_t b01 = perm_b32(s1, s0, 0x05010400u);   // s0.b0 s1.b0 s0.b1 s1.b1
    const uint32_t b23 = perm_b32(s3, s2, 0x05010400u);
    sp.lo[q] = (int)(perm_b32(b23, b01, 0x05040100u) ^ 0x80808080u);   // u - 128
    sp.hi[q] = (int)perm_b32(b23, b01, 0x07060302u);                     // T >> 8
  }
  return sp;
}

// Vertical pass: dh = Cd T_hi + c2 (stage2_bias: the rounding and the +128
// of each block's row 0) and dl = Cd (u - 128).
__device__ __forceinline__ void mfma2(const v4i& a2, const Split& sp, const v16i& c2, v16i& dh,
                                      v16i& dl) {
  dh = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2, sp.hi, c2, 0, 0, 0);
  dl = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2, sp.lo, splat16<0>(), 0, 0, 0);
}

// Initial value of the vertical pass's hi accumulator: the rounding
// 2^(s2-1) / 256 in every element, plus the +128 of each block's row 0
// (128 * 2^s2 / 256 in the registers holding a row 0, lanes g = 0).  Kept in
// registers for the whole strip walk (the empty asm makes it an opaque
// register value, so the compiler neither rebuilds it for every product nor
// copies it in).
template <int kW>
__device__ __forceinline__ v16i stage2_bias(int lane) {
  constexpr int kS2 = ilog2c(kW) + 6;
  v16i c2 = splat16<1 << (kS2 - 9)>();
  if (lane < 32) {
#pragma unroll
    for (int j = 0; j < 16; j++)
      if (reg_block_row0(j, kW)) c2[j] += 1 << (kS2 - 1);
  }
  asm volatile("" : "+v"(c2));
  return c2;
}

// ------------------------------------------------------- w = 32 strips
// A 32 x 32 tile is one block: its energy is a sum over all 64 lanes.  The
// functions below reduce the lanes' FP64 shares of eight tiles at once.

__device__ inline uint32_t lo32(double v) { return (uint32_t)__double_as_longlong(v); }
__device__ inline uint32_t hi32(double v) { return (uint32_t)(__double_as_longlong(v) >> 32); }
__device__ inline double mk64(uint32_t hi, uint32_t lo) {
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// a + b after exchanging the upper 32 lanes of a with the lower 32 lanes of
// b: lanes 0..31 get the two-half sum of a, lanes 32..63 that of b.
__device__ inline double fold32(double a, double b) {
  const auto l = __builtin_amdgcn_permlane32_swap(lo32(a), lo32(b), false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi32(a), hi32(b), false, false);
  return mk64(h[0], l[0]) + mk64(h[1], l[1]);
}

// The same over 16-lane rows: odd rows of a swap with even rows of b; lanes
// with bit 4 clear get the row-pair sum of a, the others that of b.
__device__ inline double fold16(double a, double b) {
  const auto l = __builtin_amdgcn_permlane16_swap(lo32(a), lo32(b), false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi32(a), hi32(b), false, false);
  return mk64(h[0], l[0]) + mk64(h[1], l[1]);
}

// v read from another lane of the same 16-lane row through DPP (every
// pattern used reads a lane of the same row, so no lane keeps an old value).
template <int kCtrl>
__device__ inline double dpp64(double v) {
  const uint32_t l = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo32(v), kCtrl, 0xf, 0xf, true);
  const uint32_t h = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi32(v), kCtrl, 0xf, 0xf, true);
  return mk64(h, l);
}

constexpr int kDppXor1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // lane i <-> 7 - i within each 8 lanes
constexpr int kDppRor8 = 0x128;        // lane i <- lane (i + 8) mod 16 in its row

// Sums v[t] over all 64 lanes for t = 0..7; lane l receives the total of
// tile l >> 3 (every lane of each group of eight holds it).
__device__ inline double reduce_scatter8(const double (&v)[8], int lane) {
  // halves: lanes < 32 keep tiles 0..3, the others 4..7
  const double a0 = fold32(v[0], v[4]), a1 = fold32(v[1], v[5]);
  const double a2 = fold32(v[2], v[6]), a3 = fold32(v[3], v[7]);
  // rows: bit 4 of the lane picks tile pair (0, 1) or (2, 3) of the half
  const double b0 = fold16(a0, a2), b1 = fold16(a1, a3);
  // bit 3 picks the tile; its partner 8 lanes away sends the other one
  const bool odd = (lane & 8) != 0;
  const double keep = odd ? b1 : b0, send = odd ? b0 : b1;
  double c = keep + dpp64<kDppRor8>(send);
  // all eight lanes of the group
  c += dpp64<kDppXor1>(c);
  c += dpp64<kDppXor2>(c);
  c += dpp64<kDppHalfMirror>(c);
  return c;
}

// Sums over all 64 lanes for 4 units of two w = 32, K = 16 tiles (unit u
// holds tile 2u in lanes with bit 4 clear, 2u + 1 in the others); lane l
// receives the total of tile 4 b5 + 2 b3 + b4 (b_i = bit i of l).
__device__ inline double reduce_scatter4x2(const double (&v)[4], int lane) {
  const double e0 = fold32(v[0], v[2]), e1 = fold32(v[1], v[3]);   // units 0|2, 1|3
  const bool odd = (lane & 8) != 0;
  const double keep = odd ? e1 : e0, send = odd ? e0 : e1;
  double c = keep + dpp64<kDppRor8>(send);
  c += dpp64<kDppXor1>(c);
  c += dpp64<kDppXor2>(c);
  c += dpp64<kDppHalfMirror>(c);
  return c;
}

// The same for 2 units of four w = 32, K = 8 tiles (unit u holds tile
// 4u + q in lanes with (l >> 3) & 3 == q): lane l receives tile l >> 3.
__device__ inline double reduce_scatter2x4(const double (&v)[2]) {
  double c = fold32(v[0], v[1]);
  c += dpp64<kDppXor1>(c);
  c += dpp64<kDppXor2>(c);
  c += dpp64<kDppHalfMirror>(c);
  return c;
}

// Per-wavefront constants of the packed layout (kPack = w / K sample tiles
// per MFMA tile; kPack = 1 is the plain tile).
template <int kW, int kK>
struct PackConsts {
  static constexpr int kPack = kW / kK;
  v4i b1[kPack];      // stage-1 B operand of each sample tile
  v4i a2;             // stage-2 A operand
  double wt[16];      // weights (only registers in use are loaded)

  __device__ void load(const v4i* tab_b1p, const v4i* tab_a2, const double* tab_w, int lane) {
#pragma unroll
    for (int p = 0; p < kPack; p++) b1[p] = tab_b1p[p * 64 + lane];
    a2 = tab_a2[lane];
#pragma unroll
    for (int j = 0; j < 16; j++)
      if (reg_used(j, kW, kK)) wt[j] = tab_w[j * 64 + lane];
  }
};

// Energies of one packed unit from its vertical-pass accumulators: h[b] =
// this lane's FP64 share of the energy of block row b of its sample tile,
// dc[b] = the coefficient in register row (b, 0) (the block's DC where the
// lane is a DC lane: c % K == 0, g = 0).
template <int kBits, int kW, int kK, class PC>
__device__ __forceinline__ void coeff_energy(const PC& pc, const v16i& dh, const v16i& dl,
                                             double (&h)[kTile / kW], int (&dc)[kTile / kW]) {
  constexpr int kS2 = ilog2c(kW) + 6;
  constexpr int kBpt = kTile / kW;
  double acc[kBpt];
#pragma unroll
  for (int b = 0; b < kBpt; b++) {
    acc[b] = 0.0;
    dc[b] = 0;
  }
#pragma unroll
  for (int j = 0; j < 16; j++) {
    if (!reg_used(j, kW, kK)) continue;
    const int yv = (int)((uint32_t)dh[j] * 256u + (uint32_t)dl[j]) >> kS2;
    const int br = (8 * (j / 4)) / kW;
    if (reg_block_row0(j, kW)) dc[br] = yv;
    acc[br] = fma(pc.wt[j], fabs((double)yv), acc[br]);
  }
#pragma unroll
  for (int b = 0; b < kBpt; b++) h[b] = acc[b];
}

// ----------------------------------------------------- w = 16, 8 blocks
// In the packed layout a block's energy is spread over the 2 kK lanes of its
// (block column, sample tile) group -- kK consecutive lanes in each half --
// one share per block row held in h[0 .. kBpt - 1].  rows_reduce sums every
// row's shares over its group and leaves row rows_lane_row(lane) in each
// lane: the halves split the rows first (lanes < 32 keep the first half of
// the rows), then, with four rows, the top in-group lane bit picks one of
// the remaining two, and the other in-group bits are summed over.

// 8-lane pairing across bit 2 (lane i with 7 - i), 4-lane pairing across
// bit 1, 2-lane pairing across bit 0.
template <int kLanes>
__device__ inline double dpp_top(double v) {
  if constexpr (kLanes == 16) return dpp64<kDppRor8>(v);
  else if constexpr (kLanes == 8) return dpp64<kDppHalfMirror>(v);
  else if constexpr (kLanes == 4) return dpp64<kDppXor2>(v);
  else return dpp64<kDppXor1>(v);
}

// Sum over the low log2(kLanes) lane bits (DPP inside 16-lane rows).
template <int kLanes>
__device__ inline double dpp_allreduce(double v) {
  if constexpr (kLanes >= 2) v += dpp64<kDppXor1>(v);
  if constexpr (kLanes >= 4) v += dpp64<kDppXor2>(v);
  if constexpr (kLanes >= 8) v += dpp64<kDppHalfMirror>(v);
  if constexpr (kLanes >= 16) v += dpp64<kDppRor8>(v);
  return v;
}

template <int kW, int kK>
__device__ inline int rows_lane_row(int lane) {
  constexpr int kBpt = kTile / kW;
  const int half = lane >> 5;
  if constexpr (kBpt == 2) return half;
  else return 2 * half + ((lane & (kK / 2)) ? 1 : 0);
}

template <int kW, int kK>
__device__ inline double rows_reduce(const double (&h)[kTile / kW], int lane) {
  constexpr int kBpt = kTile / kW;
  static_assert(kBpt == 2 || kBpt == 4, "w = 16 or 8");
  if constexpr (kBpt == 2) {
    return dpp_allreduce<kK>(fold32(h[0], h[1]));
  } else {
    const double r01 = fold32(h[0], h[2]);   // halves: rows 0 | 2
    const double r23 = fold32(h[1], h[3]);   //         rows 1 | 3
    const bool top = (lane & (kK / 2)) != 0;
    const double keep = top ? r23 : r01, send = top ? r01 : r23;
    return dpp_allreduce<kK / 2>(keep + dpp_top<kK>(send));
  }
}

}  // namespace vca
