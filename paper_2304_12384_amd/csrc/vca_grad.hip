// vca_grad.hip -- differentiable luma texture energy E_Y and its temporal
// gradient h (Section 2 of the paper names both features) on gfx950.
//
// For gradients the transform's roundings are dropped: per w x w block X,
//   Y = C X C^T * 2^-(s1+s2),  s1 + s2 = 2 log2 w + B - 3,
//   H = sum W_ik |Y_ik| (DC and coefficients outside K x K weigh 0),
//   E = sum_blocks H / (C_Y w^2),  h_t = sum_blocks |H_t - H_{t-1}| / (C_Y w^2).
// d/dX of H is 2^-(s1+s2) C^T (W o sign(Y)) C, with sign(0) = 0.
//
// One wavefront per 32 x 32 tile (block-diagonal Cd for w < 32), on fp16
// matrix cores (v_mfma_f32_32x32x16_f16, FP32 accumulation) with operands
// split into fp16 integers, so that every product and partial sum is an
// integer below 2^24 and the accumulators are exact:
//   forward  the samples as fixed-point digits x = a + 2^-11 b + 2^-22 c + r
//            (a = rint(x), |b|, |c| <= 1024, |r| <= 2^-23 and r = 0 for
//            |x| >= 2 or x on the 2^-22 grid); per digit T = X Cd^T, split
//            as T = 4096 t_h + t_l; Y assembled in FP64 from four exact
//            accumulators (see tile_acc), so Y, sign(Y) and Y = 0 are
//            exact for such samples (|x| < 2^11).  Tiles of integer samples
//            have b = c = 0 and skip their products.  Block energies in
//            FP64; per tile the signs of the coefficients go to the
//            workspace as sixteen 2-bit fields per lane.
//   backward S = W o sign(Y) from the masks (W = w0 + w1, two fp16 parts),
//            U = S^T Cd, G^T = Cd^T U (U in three fp16 parts), both chained
//            in registers, then each block of G times its upstream factor
//            c = (dL/dE_t + dL/dh_t sgn(H_t - H_{t-1})
//                 - dL/dh_{t+1} sgn(H_{t+1} - H_t)) 2^-(s1+s2) / (C_Y w^2).
//            The backward reads 256 bytes of masks per tile instead of the
//            4 KiB tile of samples, and does not repeat the forward passes;
//            it writes each gradient tile as whole 128-byte rows (through
//            LDS) with streaming stores, so no dirty gradient lines are left
//            in the memory-side cache for the next forward call's reads.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/vca.h"
#include "vca_host.h"
#include "vca_tile.h"

using namespace vca;

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __fp16 h2 __attribute__((ext_vector_type(2)));

namespace {

constexpr int kGWaves = 4;
constexpr int kGThreads = 64 * kGWaves;

// Eight fp16 operand values of one lane (one MFMA slot each), packed.
struct H8 {
  uint32_t w[4];
};

// Per-lane operand tables and weights.  Slot s of MFMA h of lane (c + 32 g):
//   b1: 2^-12 Cd[c][16 g + 8 h + s]  (stage 1 B; the lane's samples 16 g..)
//   a2: Cd[c][m_{8h+s}(g)]           (stage 2 A; T rows held in registers)
//   a2x2: 2^-11 a2                    (stage 2 A of the 2 t_h digit products)
//   ct: Cd[m_{8h+s}(g)][c]           (backward: B of S^T Cd and A of Cd^T U)
// The 2^-12 of b1 makes the horizontal pass T / 4096 (its split needs no
// scaling); a2x2 and wd carry the matching powers of two, so every value is
// the unscaled one times a power of two and rounds alike.
struct alignas(16) GradTables {
  H8 b1[2][64];
  H8 a2[2][64];
  H8 a2x2[2][64];
  H8 ct[2][64];
  double wd[16][64];   // weight * 2^-(s1+s2) * 4096 of coefficient register j (energy)
  float w0[16][64];    // weight = w0 + w1, both fp16 values (backward)
  float w1[16][64];
};

struct GradParams {
  const float* x;
  float* gx;
  double* blk_h;        // [frames][C_Y]
  uint32_t* masks;      // [tiles][64]: bits 2j, 2j + 1 sign(Y_j) as a 2-bit signed field
  const float* gE;      // [frames]
  const float* gh;      // [frames]
  const GradTables* tab;
  int64_t pitch;        // floats
  int64_t fstride;      // floats
  int32_t nbx, nby, ntx, tiles_per_frame, per_frame;
  FastDiv div_tpf, div_ntx;
  int32_t n_frames, seq_len;
  float grad_scale;     // 2^-(s1+s2) / (C_Y w^2)
};

template <int kW>
struct FTile {
  int64_t origin;       // float offset of the tile origin
  int32_t f, vr, vc, out0;
};

template <int kW>
__device__ inline FTile<kW> decode_ftile(const GradParams& p, int id) {
  constexpr int kBpt = kTile / kW;
  FTile<kW> t;
  t.f = (int)fastdiv((uint32_t)id, p.div_tpf);
  const int r = id - t.f * p.tiles_per_frame;
  const int ty = (int)fastdiv((uint32_t)r, p.div_ntx);
  const int tx = r - ty * p.ntx;
  const int by0 = ty * kBpt, bx0 = tx * kBpt;
  t.origin = t.f * p.fstride + (int64_t)by0 * kW * p.pitch + bx0 * kW;
  t.vr = min(kBpt, p.nby - by0);
  t.vc = min(kBpt, p.nbx - bx0);
  t.out0 = t.f * p.per_frame + by0 * p.nbx + bx0;
  return t;
}

// Lane (r + 32 g) loads row r, samples 16g..16g+15 of the tile; rows and
// 16-byte pieces outside the valid blocks are redirected in bounds (a piece
// that starts inside the block grid lies inside the row's pitch).
template <int kW>
__device__ inline void load_ftile(const GradParams& p, const FTile<kW>& t, int lane, float x[16]) {
  const int r = lane & 31, g = lane >> 5;
  const int rows = t.vr * kW, cols = t.vc * kW;
  const float* row = p.x + t.origin + (int64_t)(r < rows ? r : 0) * p.pitch;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int c = 16 * g + 4 * q;
    const v4f v = *reinterpret_cast<const v4f*>(row + (c < cols ? c : 0));
    x[4 * q + 0] = v[0];
    x[4 * q + 1] = v[1];
    x[4 * q + 2] = v[2];
    x[4 * q + 3] = v[3];
  }
}

__device__ inline uint32_t pk(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(a, b));   // toward zero
}
__device__ inline float lo_of(uint32_t p) { return (float)__builtin_bit_cast(h2, p).x; }
__device__ inline float hi_of(uint32_t p) { return (float)__builtin_bit_cast(h2, p).y; }

// v = p0 + p1 + p2 exactly in fp16 parts (each part keeps the leading 11
// significant bits of what is left; three parts hold an FP32 significand,
// down to fp16's smallest subnormal).
__device__ inline void split3(const float* v, H8& p0, H8& p1, H8& p2) {
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const float a = v[2 * q], b = v[2 * q + 1];
    const uint32_t u0 = pk(a, b);
    const float ra = a - lo_of(u0), rb = b - hi_of(u0);
    const uint32_t u1 = pk(ra, rb);
    p0.w[q] = u0;
    p1.w[q] = u1;
    p2.w[q] = pk(ra - lo_of(u1), rb - hi_of(u1));
  }
}

__device__ inline v16f mma(const H8& a, const H8& b, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, a), __builtin_bit_cast(v8h, b),
                                                c, 0, 0, 0);
}

__device__ inline H8 ld8(const H8 (&t)[64], int lane) {
  const v4i v = *reinterpret_cast<const v4i*>(&t[lane]);
  H8 h;
  h.w[0] = (uint32_t)v[0];
  h.w[1] = (uint32_t)v[1];
  h.w[2] = (uint32_t)v[2];
  h.w[3] = (uint32_t)v[3];
  return h;
}

// Fixed-point digits of a lane's 16 samples: x = a + 2^-11 b + 2^-22 c + r
// with a = rint(x), b = rint((x - a) 2^11), c = rint((x - a - 2^-11 b) 2^22),
// each an integer of magnitude <= 2048 (exact in fp16; |x| < 2^11), and
// |r| <= 2^-23 (r = 0 unless x is off the 2^-22 grid, i.e. |x| < 2).
// digit(x, 0, ..) gives a (and whether some sample is not an integer),
// digit(x, 1, ..) gives b and digit(x, 2, ..) c, each in two halves of 8.
__device__ inline bool digit(const float (&x)[16], int which, H8 (&d)[2]) {
  bool frac = false;
#pragma unroll
  for (int h = 0; h < 2; h++) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      float v[2];
#pragma unroll
      for (int e = 0; e < 2; e++) {
        const float xv = x[8 * h + 2 * q + e];
        const float ia = rintf(xv);
        float r = xv - ia;                                   // exact, |r| <= 1/2
        if (which == 0) {
          frac |= xv != ia;
          v[e] = ia;
        } else {
          const float ib = rintf(r * 2048.f);
          if (which == 1) {
            v[e] = ib;
          } else {
            r = fmaf(-ib, 1.f / 2048.f, r);                  // exact, |r| <= 2^-12
            v[e] = rintf(r * 4194304.f);
          }
        }
      }
      d[h].w[q] = pk(v[0], v[1]);
    }
  }
  return frac;
}

// Horizontal pass of one digit, T / 4096 = X (2^-12 Cd)^T (|T| <= 2048 * 2048 =
// 2^22, an integer, so T / 4096 is exact in FP32).
__device__ inline v16f stage1(const H8 (&b1)[2], const H8 (&xd)[2]) {
  v16f t = {};
  t = mma(xd[0], b1[0], t);
  t = mma(xd[1], b1[1], t);
  return t;
}

// Vertical-pass operands of registers 8h..8h+7 of t = T / 4096: T = 4096 th +
// tl with th = rint(t) (|th| <= 1024, an integer) and tl / 4096 = t - th
// (|tl| <= 2048 an integer, so tl / 4096 is exact in fp16).
__device__ inline void split_t(const v16f& t, int h, H8& th, H8& tl) {
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int j = 8 * h + 2 * q;
    const float ha = rintf(t[j]), hb = rintf(t[j + 1]);
    th.w[q] = pk(ha, hb);
    tl.w[q] = pk(t[j] - ha, t[j + 1] - hb);
  }
}

// Y (without the 2^-(s1+s2) scale) of a tile in the accumulator layout
// (lane = column, register j = row m_j) as
//   Y = 4096 A1 + A2 + 2^-11 A3 + 2^-22 A4,
//   A1 = Cd t_h(a),  A2 = Cd t_l(a) + 2Cd t_h(b),
//   A3 = Cd t_l(b) + 2Cd t_h(c),  A4 = Cd t_l(c),
// where t(d) is the horizontal pass of digit d.  |t_h(b)|, |t_h(c)| <= 512,
// so A2 and A3 stay below 2^23 and every accumulator is an exact integer.
// The accumulators hold A1 and A2 / 4096, A3 / 4096, A4 / 4096 (the t_l
// operands and a2x2 carry the 2^-12), so Y / 4096 is formed.
// kFrac = false: integer samples (b = c = 0), A1 and A2 only.
struct YAcc {
  v16f a1, a2, a3, a4;
};

template <bool kFrac>
__device__ inline YAcc tile_acc(const H8 (&b1)[2], const H8 (&a2)[2], const H8 (&a2x2)[2],
                                const float (&x)[16], const H8 (&xa)[2]) {
  YAcc y;
  y.a1 = v16f{};
  y.a2 = v16f{};
  v16f t = stage1(b1, xa);
#pragma unroll
  for (int h = 0; h < 2; h++) {
    H8 th, tl;
    split_t(t, h, th, tl);
    y.a1 = mma(a2[h], th, y.a1);
    y.a2 = mma(a2[h], tl, y.a2);
  }
  if constexpr (kFrac) {
    H8 xd[2];
    y.a3 = v16f{};
    y.a4 = v16f{};
    digit(x, 1, xd);
    t = stage1(b1, xd);
#pragma unroll
    for (int h = 0; h < 2; h++) {
      H8 th, tl;
      split_t(t, h, th, tl);
      y.a2 = mma(a2x2[h], th, y.a2);
      y.a3 = mma(a2[h], tl, y.a3);
    }
    digit(x, 2, xd);
    t = stage1(b1, xd);
#pragma unroll
    for (int h = 0; h < 2; h++) {
      H8 th, tl;
      split_t(t, h, th, tl);
      y.a3 = mma(a2x2[h], th, y.a3);
      y.a4 = mma(a2[h], tl, y.a4);
    }
  }
  return y;
}

// Coefficient j of the tile / 4096 from its accumulators, exactly (up to one
// FP64 rounding in the last term).
template <bool kFrac>
__device__ inline double coeff(const YAcc& y, int j) {
  double v = (double)y.a1[j] + (double)y.a2[j];
  if constexpr (kFrac) {
    v = fma(0x1p-11, (double)y.a3[j], v);
    v = fma(0x1p-22, (double)y.a4[j], v);
  }
  return v;
}

template <int kW, int kK>
__global__ __launch_bounds__(kGThreads) void energy_fwd_kernel(GradParams p) {
  constexpr int kBpt = kTile / kW;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 31;
  double wd[16];
#pragma unroll
  for (int j = 0; j < 16; j++) wd[j] = reg_used(j, kW, kK) ? p.tab->wd[j][lane] : 0.0;
  H8 b1[2], a2[2], a2x2[2];
#pragma unroll
  for (int h = 0; h < 2; h++) {
    b1[h] = ld8(p.tab->b1[h], lane);
    a2[h] = ld8(p.tab->a2[h], lane);
    a2x2[h] = ld8(p.tab->a2x2[h], lane);
  }
  const int total = p.n_frames * p.tiles_per_frame;
  const int stride = gridDim.x * kGWaves;
  int id = blockIdx.x * kGWaves + wave;
  if (id >= total) return;
  // Energies and coefficient signs of tile `id` (samples x), from the exact
  // coefficients.  sign(Y_j) goes into bits 2j, 2j + 1 of the lane's mask as
  // a 2-bit signed field (1, 0 or -1), shifted in from the top one field per
  // register.  Adding +0.0 turns a -0 into +0; a nonzero coefficient is far
  // above the subnormal range, so the high word of its FP64 value is a
  // positive or negative integer other than 0x80000000, and its clamp to
  // [-1, 1] is the sign.
  auto energy = [&](const YAcc& y, double (&h)[kBpt], uint32_t& mask, auto frac) {
    constexpr bool kFrac = decltype(frac)::value;
#pragma unroll
    for (int j = 0; j < 16; j++) {
      if (!reg_used(j, kW, kK)) {
        mask >>= 2;
        continue;
      }
      const double v = coeff<kFrac>(y, j) + 0.0;
      h[(8 * (j / 4)) / kW] = fma(wd[j], fabs(v), h[(8 * (j / 4)) / kW]);
      const int hi = (int)(__builtin_bit_cast(uint64_t, v) >> 32);
      int sg;   // the clamp as one instruction (written as min/max it compiles to two selects)
      asm("v_med3_i32 %0, %1, -1, 1" : "=v"(sg) : "v"(hi));
      mask = __builtin_amdgcn_alignbit((uint32_t)sg, mask, 2);
    }
  };
  auto tile = [&](const FTile<kW>& t, const float (&x)[16], int id) {
    H8 xa[2];
    const bool frac_lane = digit(x, 0, xa);
    double h[kBpt];
#pragma unroll
    for (int b = 0; b < kBpt; b++) h[b] = 0.0;
    uint32_t mask = 0;
    // one branch per tile for the whole wavefront: integer samples skip the
    // products of the fraction digits
    if (__builtin_amdgcn_ballot_w64(frac_lane) != 0) {
      energy(tile_acc<true>(b1, a2, a2x2, x, xa), h, mask, std::true_type{});
    } else {
      energy(tile_acc<false>(b1, a2, a2x2, x, xa), h, mask, std::false_type{});
    }
    p.masks[(int64_t)id * 64 + lane] = mask;
    // Each block's shares lie in the kW lanes of its block column in both
    // halves, one per block row in h[]; they are summed across lanes with
    // permlane swaps and DPP (no LDS round trips), leaving one block per
    // lane group, which one lane of the group stores.
    if constexpr (kW == 32) {
      double v = fold32(h[0], h[0]);
      v = dpp_allreduce<16>(fold16(v, v));
      if (lane == 0) p.blk_h[t.out0] = v;
    } else {
      const double v = rows_reduce<kW, kW>(h, lane);
      const int row = rows_lane_row<kW, kW>(lane), col = r / kW;
      if ((lane & (kW == 16 ? 15 : 3)) == 0 && row < t.vr && col < t.vc)
        p.blk_h[t.out0 + row * p.nbx + col] = v;
    }
  };
  // Two sample buffers in turn: the next tile's loads are issued before this
  // tile is transformed and stay there (a scheduling barrier keeps the
  // compiler from sinking them below the matrix products), and the loop is
  // unrolled by two so that no buffer is copied (a copy would wait for the
  // loads).  Past the end the last tile loads itself again, so every step
  // issues the same loads.
  FTile<kW> ta = decode_ftile<kW>(p, id), tb;
  float xa[16], xb[16];
  load_ftile<kW>(p, ta, lane, xa);
  for (;;) {
    tb = decode_ftile<kW>(p, min(id + stride, total - 1));
    load_ftile<kW>(p, tb, lane, xb);
    __builtin_amdgcn_sched_barrier(0);
    tile(ta, xa, id);
    if ((id += stride) >= total) break;
    ta = decode_ftile<kW>(p, min(id + stride, total - 1));
    load_ftile<kW>(p, ta, lane, xa);
    __builtin_amdgcn_sched_barrier(0);
    tile(tb, xb, id);
    if ((id += stride) >= total) break;
  }
}

// One workgroup per frame: E and h from the block energies (fixed order).
__global__ __launch_bounds__(256) void energy_reduce_kernel(const double* blk_h, int32_t per_frame,
                                                            int32_t seq_len, double norm, float* E,
                                                            float* h) {
  __shared__ double red[2][256];
  const int f = blockIdx.x, t = threadIdx.x;
  const double* H = blk_h + (int64_t)f * per_frame;
  const bool first = f % seq_len == 0;
  double se = 0.0, sh = 0.0;
  for (int b = t; b < per_frame; b += 256) {
    se += H[b];
    if (!first) sh += fabs(H[b] - H[b - per_frame]);
  }
  red[0][t] = se;
  red[1][t] = sh;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) {
      red[0][t] += red[0][t + w];
      red[1][t] += red[1][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    E[f] = (float)(red[0][0] * norm);
    h[f] = (float)(red[1][0] * norm);
  }
}

__device__ inline float sgn(double v) { return v > 0.0 ? 1.f : (v < 0.0 ? -1.f : 0.f); }

template <int kW, int kK>
__global__ __launch_bounds__(kGThreads) void energy_bwd_kernel(GradParams p) {
  constexpr int kBpt = kTile / kW;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 31, g = lane >> 5;
  float w0[16], w1[16];
#pragma unroll
  for (int j = 0; j < 16; j++) {
    w0[j] = reg_used(j, kW, kK) ? p.tab->w0[j][lane] : 0.f;
    w1[j] = reg_used(j, kW, kK) ? p.tab->w1[j][lane] : 0.f;
  }
  H8 ct[2];
#pragma unroll
  for (int h = 0; h < 2; h++) ct[h] = ld8(p.tab->ct[h], lane);
  // one 32 x 32 gradient tile per wavefront, rows padded to 36 floats: the
  // eight lanes of one 16-byte piece of eight rows (the writes) and the eight
  // lanes of one row (the reads) fall in different banks
  constexpr int kStageRow = 36;
  __shared__ __attribute__((aligned(16))) float stage_all[kGWaves][32 * kStageRow];
  float* const stage = stage_all[wave];
  const int total = p.n_frames * p.tiles_per_frame;
  const int stride = gridDim.x * kGWaves;
  // a tile's inputs: its sign masks; per block column of the lane's block
  // row, H of the block in this, the previous and the next frame (the
  // block's own index where a neighbour frame is not used); and the frame's
  // upstream gradients dL/dE_t, dL/dh_t and dL/dh_{t+1} (the last index
  // clamped; a term whose frame is not used is dropped where it is applied).
  // Every load is unconditional, so the compiler can count what is in flight.
  struct In {
    FTile<kW> t;
    uint32_t mask;
    double hc[kBpt], hp[kBpt], hn[kBpt];
    float gE, gh, ghn;
  };
  auto fetch = [&](int tid) {
    In in;
    in.t = decode_ftile<kW>(p, tid);
    in.mask = p.masks[(int64_t)tid * 64 + lane];
    const int f = in.t.f, pos = f % p.seq_len;
    in.gE = p.gE[f];
    in.gh = p.gh[f];
    in.ghn = p.gh[min(f + 1, p.n_frames - 1)];
    const int br = min(r / kW, in.t.vr - 1);
#pragma unroll
    for (int b = 0; b < kBpt; b++) {
      const int idx = in.t.out0 + br * p.nbx + min(b, in.t.vc - 1);
      in.hc[b] = p.blk_h[idx];
      in.hp[b] = p.blk_h[pos > 0 ? idx - p.per_frame : idx];
      in.hn[b] = p.blk_h[pos + 1 < p.seq_len ? idx + p.per_frame : idx];
    }
    return in;
  };
  // dL/dx of one tile from its inputs
  auto tile = [&](const In& cur) {
    const FTile<kW> t = cur.t;
    const uint32_t mask = cur.mask;
    // S = W o sign(Y): lane (c + 32 g) register j is coefficient (m_j, c);
    // as S^T's A operand, slot s of MFMA h is register 8 h + s
    v16f u = {};
#pragma unroll
    for (int h = 0; h < 2; h++) {
      H8 s0, s1;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        float a[2][2];
#pragma unroll
        for (int e = 0; e < 2; e++) {
          const int j = 8 * h + 2 * q + e;
          // the builtin's result type is unsigned: the field, sign-extended, as int
          const float sg = (float)(int)__builtin_amdgcn_sbfe(mask, 2 * j, 2);
          a[0][e] = sg * w0[j];
          a[1][e] = sg * w1[j];
        }
        s0.w[q] = pk(a[0][0], a[0][1]);
        s1.w[q] = pk(a[1][0], a[1][1]);
      }
      u = mma(s0, ct[h], u);
      u = mma(s1, ct[h], u);
    }
    // G^T = Cd^T U: U's register 8 h + s is the B operand's slot s
    v16f gt = {};
#pragma unroll
    for (int h = 0; h < 2; h++) {
      float uv[8];
#pragma unroll
      for (int s = 0; s < 8; s++) uv[s] = u[8 * h + s];
      H8 u0, u1, u2;
      split3(uv, u0, u1, u2);
      gt = mma(ct[h], u0, gt);
      gt = mma(ct[h], u1, gt);
      gt = mma(ct[h], u2, gt);
    }
    // upstream factor of each block: lane's pixel row r is in block row
    // r / w; register j's pixel column m_j in block column m_j / w
    const int f = t.f;
    const int pos = f % p.seq_len;
    const bool has_prev = pos > 0, has_next = pos + 1 < p.seq_len;
    const float gE = cur.gE;
    const float ghf = has_prev ? cur.gh : 0.f;
    const float ghn = has_next ? cur.ghn : 0.f;
    float cb[kBpt];
#pragma unroll
    for (int b = 0; b < kBpt; b++) {
      float c = gE;
      if (has_prev) c += ghf * sgn(cur.hc[b] - cur.hp[b]);
      if (has_next) c -= ghn * sgn(cur.hn[b] - cur.hc[b]);
      cb[b] = c * p.grad_scale;
    }
    // pixel (r, m_j): registers 4q..4q+3 are columns 8q + 4g + 0..3.  The
    // scaled tile goes through the wavefront's LDS area and comes back as
    // whole rows: store q of lane 8 rho + pi writes piece pi (16 bytes) of row
    // 8 q + rho, so each store instruction covers eight full 128-byte rows.
    // Whole-row streaming stores go on to HBM during this kernel; 16-byte
    // pieces of 32 rows per instruction leave the gradients as dirty lines
    // in the memory-side cache, written back while the next forward call
    // reads its samples.
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int col = 8 * q + 4 * g;
      const float c = cb[col / kW];
      const v4f v = {gt[4 * q] * c, gt[4 * q + 1] * c, gt[4 * q + 2] * c, gt[4 * q + 3] * c};
      *reinterpret_cast<v4f*>(&stage[r * kStageRow + col]) = v;
    }
    const int rows = t.vr * kW, cols = t.vc * kW;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int row = 8 * q + (lane >> 3), col = 4 * (lane & 7);
      const v4f v = *reinterpret_cast<const v4f*>(&stage[row * kStageRow + col]);
      if (row < rows && col < cols)
        __builtin_nontemporal_store(v, reinterpret_cast<v4f*>(p.gx + t.origin + (int64_t)row * p.pitch + col));
    }
  };
  // Two input sets in turn, as in the forward kernel: the next tile's loads
  // are issued before this tile is transformed and stay there, and no set
  // is copied.  Past the end the last tile is fetched again.
  int id = blockIdx.x * kGWaves + wave;
  if (id >= total) return;
  In ia = fetch(id), ib;
  for (;;) {
    ib = fetch(min(id + stride, total - 1));
    __builtin_amdgcn_sched_barrier(0);
    tile(ia);
    if ((id += stride) >= total) break;
    ia = fetch(min(id + stride, total - 1));
    __builtin_amdgcn_sched_barrier(0);
    tile(ib);
    if ((id += stride) >= total) break;
  }
}

// Pixels outside the block grid (rows >= nby w, or columns >= nbx w) take no
// part in any block: their gradient is 0.  One grid-stride loop per frame.
__global__ __launch_bounds__(256) void zero_border_kernel(float* gx, int64_t pitch, int64_t fstride,
                                                          int32_t width, int32_t height,
                                                          int32_t grid_w, int32_t grid_h) {
  float* frame = gx + (int64_t)blockIdx.y * fstride;
  const int64_t bottom = (int64_t)(height - grid_h) * width;
  const int32_t right_w = width - grid_w;
  const int64_t total = bottom + (int64_t)grid_h * right_w;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    int64_t row, col;
    if (i < bottom) {
      row = grid_h + i / width;
      col = i % width;
    } else {
      const int64_t j = i - bottom;
      row = j / right_w;
      col = grid_w + j % right_w;
    }
    frame[row * pitch + col] = 0.f;
  }
}

uint16_t half_bits(float v) {
  const _Float16 h = (_Float16)v;
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}

void put8(H8& dst, const float (&v)[8]) {
  for (int q = 0; q < 4; q++) dst.w[q] = half_bits(v[2 * q]) | ((uint32_t)half_bits(v[2 * q + 1]) << 16);
}

void build_grad_tables(int w, int K, int bit_depth, GradTables& t) {
  std::vector<int8_t> b1, a2;
  std::vector<double> wt;
  build_tile_tables(w, K, b1, a2, wt);   // weights with DC and non-K x K at 0
  const double sc = std::ldexp(1.0, -(2 * ilog2c(w) + bit_depth - 3));
  for (int lane = 0; lane < 64; lane++) {
    const int c = lane & 31, g = lane >> 5;
    for (int h = 0; h < 2; h++) {
      float vb1[8], va2[8], va2x2[8], vct[8];
      for (int s = 0; s < 8; s++) {
        const int m = reg_row(8 * h + s, g);
        vb1[s] = std::ldexp((float)matd(w, c, 16 * g + 8 * h + s), -12);
        va2[s] = (float)matd(w, c, m);
        va2x2[s] = std::ldexp(va2[s], -11);
        vct[s] = (float)matd(w, m, c);
      }
      put8(t.b1[h][lane], vb1);
      put8(t.a2[h][lane], va2);
      put8(t.a2x2[h][lane], va2x2);
      put8(t.ct[h][lane], vct);
    }
    for (int j = 0; j < 16; j++) {
      const double wv = wt[j * 64 + lane];
      t.wd[j][lane] = std::ldexp(wv * sc, 12);
      const float hi = (float)(_Float16)(float)wv;      // nearest fp16
      const float lo = (float)(_Float16)(float)(wv - (double)hi);
      t.w0[j][lane] = hi;
      t.w1[j][lane] = lo;
    }
  }
}

using GradKernel = void (*)(GradParams);

template <int W>
GradKernel pick_grad(int K, bool bwd) {
  if (K == W) return bwd ? energy_bwd_kernel<W, W> : energy_fwd_kernel<W, W>;
  if (K == W / 2) return bwd ? energy_bwd_kernel<W, W / 2> : energy_fwd_kernel<W, W / 2>;
  if (K == W / 4) return bwd ? energy_bwd_kernel<W, W / 4> : energy_fwd_kernel<W, W / 4>;
  return nullptr;
}

GradKernel select_grad(int w, int K, bool bwd) {
  if (w == 32) return pick_grad<32>(K, bwd);
  if (w == 16) return pick_grad<16>(K, bwd);
  if (w == 8) return pick_grad<8>(K, bwd);
  return nullptr;
}

vca_status check_grad_config(const vca_grad_config* c) {
  if (!c || c->struct_size != sizeof(vca_grad_config)) return VCA_ERR_INVALID_ARG;
  const int w = c->block_size;
  if (w != 8 && w != 16 && w != 32) return VCA_ERR_INVALID_ARG;
  const int k = c->lowpass_k;
  if (k != 0 && k != w && k != w / 2 && k != w / 4) return VCA_ERR_INVALID_ARG;
  if (c->bit_depth != 8 && c->bit_depth != 10) return VCA_ERR_INVALID_ARG;
  if (c->width < w || c->height < w || c->n_seq <= 0 || c->seq_len <= 0 || c->device < 0)
    return VCA_ERR_INVALID_ARG;
  if ((int64_t)c->n_seq * c->seq_len > 65535) return VCA_ERR_INVALID_ARG;
  if (c->pitch < c->width || c->pitch % 4 || c->fstride % 4) return VCA_ERR_INVALID_ARG;
  if ((int64_t)c->n_seq * c->seq_len > 1 && c->fstride < c->pitch * c->height) return VCA_ERR_INVALID_ARG;
  const int64_t blocks = (int64_t)(c->width / w) * (c->height / w) * c->n_seq * c->seq_len;
  if (blocks > (int64_t)INT32_MAX / 2) return VCA_ERR_INVALID_ARG;
  return VCA_OK;
}

// Workspace layout: FP64 block energies of every frame, then the sign masks
// (64 words per tile), 256-byte aligned.
struct WorkspaceLayout {
  int64_t h_bytes, mask_off, bytes;
};

WorkspaceLayout workspace_layout(const vca_grad_config* c) {
  const int w = c->block_size, bpt = kTile / w;
  const int64_t nbx = c->width / w, nby = c->height / w;
  const int64_t tiles = ((nbx + bpt - 1) / bpt) * ((nby + bpt - 1) / bpt);
  const int64_t frames = (int64_t)c->n_seq * c->seq_len;
  WorkspaceLayout L;
  L.h_bytes = nbx * nby * frames * (int64_t)sizeof(double);
  L.mask_off = (L.h_bytes + 255) / 256 * 256;
  L.bytes = L.mask_off + tiles * frames * 64 * (int64_t)sizeof(uint32_t);
  return L;
}

// Tables live in device memory per (device, w, K, bit depth); built once per
// process and kept until it ends.
struct GradTableCache {
  std::mutex mu;
  std::map<std::tuple<int, int, int, int>, GradTables*> map;
};

GradTableCache& table_cache() {
  static GradTableCache c;
  return c;
}

vca_status get_tables(const vca_grad_config* c, int K, const GradTables** out) {
  GradTableCache& tc = table_cache();
  std::lock_guard<std::mutex> lk(tc.mu);
  const auto key = std::make_tuple(c->device, c->block_size, K, c->bit_depth);
  auto it = tc.map.find(key);
  if (it != tc.map.end()) {
    *out = it->second;
    return VCA_OK;
  }
  GradTables* h = new (std::nothrow) GradTables();
  if (!h) return VCA_ERR_OOM;
  build_grad_tables(c->block_size, K, c->bit_depth, *h);
  GradTables* d = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&d), sizeof(GradTables)) != hipSuccess) {
    delete h;
    return VCA_ERR_OOM;
  }
  const hipError_t e = hipMemcpy(d, h, sizeof(GradTables), hipMemcpyHostToDevice);
  delete h;
  if (e != hipSuccess) {
    (void)hipFree(d);
    return VCA_ERR_DEVICE;
  }
  tc.map[key] = d;
  *out = d;
  return VCA_OK;
}

vca_status prepare(const vca_grad_config* c, void* workspace, GradParams& p) {
  const int w = c->block_size, K = c->lowpass_k == 0 ? w : c->lowpass_k;
  const int bpt = kTile / w;
  p.pitch = c->pitch;
  p.fstride = c->fstride;
  p.nbx = c->width / w;
  p.nby = c->height / w;
  p.ntx = (p.nbx + bpt - 1) / bpt;
  p.tiles_per_frame = p.ntx * ((p.nby + bpt - 1) / bpt);
  p.per_frame = p.nbx * p.nby;
  p.div_tpf = make_fastdiv((uint32_t)p.tiles_per_frame);
  p.div_ntx = make_fastdiv((uint32_t)p.ntx);
  p.n_frames = c->n_seq * c->seq_len;
  p.seq_len = c->seq_len;
  p.grad_scale = (float)(std::ldexp(1.0, -(2 * ilog2c(w) + c->bit_depth - 3)) /
                         ((double)p.per_frame * w * w));
  const WorkspaceLayout L = workspace_layout(c);
  p.blk_h = static_cast<double*>(workspace);
  p.masks = reinterpret_cast<uint32_t*>(static_cast<char*>(workspace) + L.mask_off);
  return get_tables(c, K, &p.tab);
}

// Workgroups of `kern` that fit on device `dev` at once: CUs x resident
// groups per CU, computed once per (kernel, device) -- the queries cost more
// host time than these short launches themselves.
hipError_t occupancy_slots(GradKernel kern, int dev, int* slots) {
  static std::mutex m;
  static std::map<std::pair<const void*, int>, int> cache;
  std::lock_guard<std::mutex> lock(m);
  const auto key = std::make_pair(reinterpret_cast<const void*>(kern), dev);
  auto it = cache.find(key);
  if (it == cache.end()) {
    int resident = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, kern, kGThreads, 0);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    it = cache.emplace(key, cus * std::max(1, resident)).first;
  }
  *slots = it->second;
  return hipSuccess;
}

vca_status launch_grad(const vca_grad_config* c, const GradParams& p, bool bwd, hipStream_t st) {
  const int w = c->block_size, K = c->lowpass_k == 0 ? w : c->lowpass_k;
  GradKernel kern = select_grad(w, K, bwd);
  if (!kern) return VCA_ERR_UNSUPPORTED;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return VCA_ERR_DEVICE;
  int slots = 0;   // resident workgroups on the whole device (cached per kernel and device)
  if (occupancy_slots(kern, dev, &slots) != hipSuccess) return VCA_ERR_DEVICE;
  const int64_t groups = ((int64_t)p.n_frames * p.tiles_per_frame + kGWaves - 1) / kGWaves;
  const int grid = (int)std::min<int64_t>(groups, (int64_t)slots);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kGThreads), 0, st, p);
  return hipGetLastError() == hipSuccess ? VCA_OK : VCA_ERR_DEVICE;
}

}  // namespace

extern "C" {

int64_t vca_grad_workspace(const vca_grad_config* c) {
  if (check_grad_config(c) != VCA_OK) return -1;
  return workspace_layout(c).bytes;
}

vca_status vca_energy_forward(const vca_grad_config* c, const float* x, float* E, float* h,
                              void* workspace, void* hip_stream) {
  if (!x || ((uintptr_t)x & 15) || !E || !h || !workspace || ((uintptr_t)workspace & 255))
    return VCA_ERR_INVALID_ARG;
  vca_status s = check_grad_config(c);
  if (s != VCA_OK) return s;
  DeviceGuard guard(c->device);
  GradParams p{};
  if ((s = prepare(c, workspace, p)) != VCA_OK) return s;
  p.x = x;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  if ((s = launch_grad(c, p, false, st)) != VCA_OK) return s;
  const double norm = 1.0 / ((double)p.per_frame * c->block_size * c->block_size);
  hipLaunchKernelGGL(energy_reduce_kernel, dim3(p.n_frames), dim3(256), 0, st, p.blk_h, p.per_frame,
                     p.seq_len, norm, E, h);
  return hipGetLastError() == hipSuccess ? VCA_OK : VCA_ERR_DEVICE;
}

vca_status vca_energy_backward(const vca_grad_config* c, const void* workspace, const float* grad_E,
                               const float* grad_h, float* grad_x, void* hip_stream) {
  if (!workspace || ((uintptr_t)workspace & 255) || !grad_E || !grad_h || !grad_x ||
      ((uintptr_t)grad_x & 15))
    return VCA_ERR_INVALID_ARG;
  vca_status s = check_grad_config(c);
  if (s != VCA_OK) return s;
  DeviceGuard guard(c->device);
  GradParams p{};
  if ((s = prepare(c, const_cast<void*>(workspace), p)) != VCA_OK) return s;
  p.gE = grad_E;
  p.gh = grad_h;
  p.gx = grad_x;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  if ((s = launch_grad(c, p, true, st)) != VCA_OK) return s;
  const int w = c->block_size;
  const int grid_w = p.nbx * w, grid_h = p.nby * w;
  const int64_t border = (int64_t)(c->height - grid_h) * c->width + (int64_t)grid_h * (c->width - grid_w);
  if (border > 0) {
    const int gx_blocks = (int)std::min<int64_t>((border + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_border_kernel, dim3(gx_blocks, p.n_frames), dim3(256), 0, st, grad_x,
                       c->pitch, c->fstride, c->width, c->height, grid_w, grid_h);
    if (hipGetLastError() != hipSuccess) return VCA_ERR_DEVICE;
  }
  return VCA_OK;
}

}  // extern "C"
