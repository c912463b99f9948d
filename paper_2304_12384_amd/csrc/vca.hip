// vca.hip -- MI355X (gfx950) Video Complexity Analyzer: kernels and C ABI.
//
// Computes the per-frame block-DCT features of Menon et al. (GMSys 2023),
// Section 2 (E_Y, h, L_Y, E_U, E_V, L_U, L_V) and the low-pass option of the
// same section.  The definitions implemented are stated in include/vca.h.
//
// Data path per 32 x 32 tile (one wavefront per tile):
//   1. one 16-byte global load per lane: lane (r + 32 g) reads row r, bytes
//      16g..16g+15 of the tile (8-bit samples), offset by -128 into int8;
//   2. horizontal pass T = X' C^T on one v_mfma_i32_32x32x32_i8 with the
//      rounding bias preloaded in the accumulator;
//   3. the accumulator (lane = column k, 16 rows per lane) is split into
//      int8 hi/lo bytes in registers -- exactly the B-operand layout of the
//      vertical pass, so T never leaves the register file;
//   4. vertical pass Y = C T as two int8 MFMAs (hi, lo) recombined exactly;
//   5. per lane: FP64 weighted sum of |Y|; one wavefront reduction gives the
//      block energy H; lane 0 holds DC (offset corrected by +2^14).
// A second kernel reduces the per-block H and DC of each frame, in a fixed
// order, to the seven features (FP64 sums, FP32 output).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/vca.h"

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

namespace {

constexpr int kTile = 32;           // MFMA tile edge (pixels)
constexpr int kWavesPerGroup = 4;   // wavefronts per workgroup
constexpr int kGroupThreads = 64 * kWavesPerGroup;
constexpr int kDcOffset = 1 << 14;  // DC lost by the -2^(B-1) sample offset, exact for all w, B

// ---------------------------------------------------------------- the matrix
// Integer stand-ins for 64*sqrt(2)*cos(pi*t/64), t = 0..32 (H.265 core
// transform values; t = 32 is the zero of the cosine).
constexpr int kCosQuarter[33] = {90, 90, 90, 90, 89, 88, 87, 85, 83, 82, 80, 78, 75, 73, 70, 67, 64,
                                 61, 57, 54, 50, 46, 43, 38, 36, 31, 25, 22, 18, 13, 9,  4,  0};

// Entry (k, n) of the 32-point matrix via the quadrant of the angle k(2n+1).
int mat32(int k, int n) {
  if (k == 0) return 64;
  int t = (k * (2 * n + 1)) & 127;
  if (t <= 32) return kCosQuarter[t];
  if (t <= 64) return -kCosQuarter[64 - t];
  if (t <= 96) return -kCosQuarter[t - 64];
  return kCosQuarter[128 - t];
}

// w-point matrix: the 32-point one restricted to every (32/w)-th row.
int matw(int w, int k, int n) { return mat32(k * (kTile / w), n); }

int log2i(int v) {
  int s = 0;
  while ((1 << s) < v) s++;
  return s;
}

// ------------------------------------------------------------ kernel params
// Division by an invariant d (Granlund-Montgomery, round-up multiplier):
// n / d = (umulhi(n, m) + n) >> l for 0 <= n < 2^31, with l = ceil(log2 d)
// and m = floor(2^32 (2^l - d) / d) + 1.  Keeps block-id decoding on the
// scalar unit.
struct FastDiv {
  uint32_t m;
  uint32_t l;
};

FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) l++;
  const uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
  return FastDiv{(uint32_t)m, l};
}

struct FwdParams {
  const uint8_t* plane[3];
  int64_t pitch[3];
  int64_t fstride[3];
  int32_t nbx[3];          // blocks per row of each plane
  int32_t cnt[3];          // blocks per plane
  int32_t per_frame;       // cnt[0] + cnt[1] + cnt[2]
  FastDiv div_frame;       // / per_frame
  FastDiv div_nbx[3];      // / nbx[P]
  int32_t n_frames;
  int32_t k;               // low-pass size (w when full)
  const v4i* tab_b1;       // [64] stage-1 B operand (C^T) per lane
  const v4i* tab_a2;       // [64] stage-2 A operand (C, rows permuted) per lane
  const double* tab_w;     // [16][64] weight per (accumulator register, lane)
  double* blk_h;           // [n_frames][per_frame]
  int32_t* blk_dc;         // [n_frames][per_frame]
  int16_t* coeffs;         // optional [n_frames][per_frame][k][k]
};

struct ReduceParams {
  const double* blk_h;
  const int32_t* blk_dc;
  const double* state_in;  // luma H of the frame before frame 0, or null (h = 0)
  double* state_out;       // receives luma H of the last frame
  float* ring;             // [capacity][7]
  int64_t first_frame;     // global index of frame 0 of this launch
  int64_t capacity;
  int32_t cnt[3];
  int32_t per_frame;
  int32_t n_frames;
  double inv_norm[3];      // 1 / (C_P w^2)
};

// ------------------------------------------------------------------ kernels
__device__ inline uint32_t perm_b32(uint32_t hi_src, uint32_t lo_src, uint32_t sel) {
  return __builtin_amdgcn_perm(hi_src, lo_src, sel);
}

__device__ inline uint32_t fastdiv(uint32_t n, FastDiv d) { return (__umulhi(n, d.m) + n) >> d.l; }

// The 16 bytes lane (r + 32 g) loads for block `id` of a launch;
// lane_off[P] = r * pitch[P] + 16 g.  The block's base address is
// wave-uniform (scalar); the load uses it with a 32-bit per-lane offset.
__device__ inline v4i load_block(const FwdParams& p, int id, const uint32_t lane_off[2]) {
  const int f = (int)fastdiv((uint32_t)id, p.div_frame);
  int b = id - f * p.per_frame;
  int P = 0;
  if (b >= p.cnt[0]) {
    b -= p.cnt[0];
    P = 1;
    if (b >= p.cnt[1]) {
      b -= p.cnt[1];
      P = 2;
    }
  }
  const int by = (int)fastdiv((uint32_t)b, p.div_nbx[P]);
  const int bx = b - by * p.nbx[P];
  const uint8_t* base = p.plane[P] + f * p.fstride[P] + (int64_t)by * kTile * p.pitch[P] + bx * kTile;
  return *reinterpret_cast<const v4i*>(base + lane_off[P == 0 ? 0 : 1]);
}

// Blocks each wavefront keeps in flight ahead of the one it transforms.
#ifndef VCA_PREFETCH_DEPTH
#define VCA_PREFETCH_DEPTH 2
#endif

// Per-wavefront constants of the full-tile transform.
template <int kRegs>
struct TileConsts {
  v4i b1;            // stage-1 B operand (C^T)
  v4i a2;            // stage-2 A operand (C, contraction order of the accumulator rows)
  double wt[kRegs];  // weight of the coefficient in each accumulator register
  int row0_fix;      // +128 on coefficient row 0 (lanes 0..31, register 0)
};

// Transform, energy and DC of one 32 x 32 block whose 16 bytes per lane are
// in x (8-bit samples).  Exact split of the horizontal-pass result T
// (|T| <= 2^14):
//   T = 256 * T_hi + u,  T_hi = T >> 8 in [-64, 63],  u = T & 255 in [0, 255]
// so that C T = 256 * C T_hi + C (u - 128) + 128 * C 1.  Both T_hi and u - 128
// are int8; the last term is 128 * 64 * 32 on coefficient row 0 (the DC row)
// and 0 elsewhere, i.e. exactly +128 after the 2^11 scaling of the vertical
// pass.  With the vertical pass's rounding 2^(s2-1) folded into the hi
// accumulator as 2^(s2-9), both accumulator biases are MFMA inline constants.
template <int kBits, int kRegs, bool kKeep>
__device__ __forceinline__ void fwd32_block(const FwdParams& p, const TileConsts<kRegs>& tc,
                                            v4i x, int id, int lane) {
  constexpr int kS1 = 5 + kBits - 9;   // log2(32) + B - 9
  constexpr int kS2 = 5 + 6;           // log2(32) + 6
  v16i c1, c2;
#pragma unroll
  for (int j = 0; j < 16; j++) {
    c1[j] = 1 << (kS1 - 1);            // rounding of the horizontal pass
    c2[j] = 1 << (kS2 - 9);            // 256 * 2^(s2-9) = 2^(s2-1): rounding of the vertical pass
  }
  const v16i zero = {};
  x ^= (int)0x80808080;                // x - 128 as int8

  const v16i d1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(x, tc.b1, c1, 0, 0, 0);

  v4i tlo, thi;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const uint32_t s0 = (uint32_t)(d1[4 * q + 0] >> kS1);
    const uint32_t s1 = (uint32_t)(d1[4 * q + 1] >> kS1);
    const uint32_t s2 = (uint32_t)(d1[4 * q + 2] >> kS1);
    const uint32_t s3 = (uint32_t)(d1[4 * q + 3] >> kS1);
    const uint32_t p01 = perm_b32(s1, s0, 0x05010400u);   // s0.b0 s1.b0 s0.b1 s1.b1
    const uint32_t p23 = perm_b32(s3, s2, 0x05010400u);
    tlo[q] = (int)(perm_b32(p23, p01, 0x05040100u) ^ 0x80808080u);   // u - 128
    thi[q] = (int)perm_b32(p23, p01, 0x07060302u);                     // T >> 8
  }
  const v16i dh = __builtin_amdgcn_mfma_i32_32x32x32_i8(tc.a2, thi, c2, 0, 0, 0);
  const v16i dl = __builtin_amdgcn_mfma_i32_32x32x32_i8(tc.a2, tlo, zero, 0, 0, 0);

  double h0 = 0.0, h1 = 0.0;
  int y0 = 0;
#pragma unroll
  for (int j = 0; j < kRegs; j++) {
    int yv = (int)((uint32_t)dh[j] * 256u + (uint32_t)dl[j]) >> kS2;
    if (j == 0) {
      yv += tc.row0_fix;
      y0 = yv;
    }
    if (j & 1)
      h1 = fma(tc.wt[j], fabs((double)yv), h1);
    else
      h0 = fma(tc.wt[j], fabs((double)yv), h0);
    if (kKeep) {
      const int kk = p.k;
      const int g = lane >> 5, r = lane & 31;
      const int i = 8 * (j >> 2) + 4 * g + (j & 3);
      if (i < kk && r < kk) {
        const int out = yv + ((i == 0 && r == 0) ? kDcOffset : 0);
        p.coeffs[((int64_t)id * kk + i) * kk + r] = (int16_t)out;
      }
    }
  }
  double h = h0 + h1;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) h += __shfl_xor(h, off);
  if (lane == 0) {
    p.blk_h[id] = h;
    p.blk_dc[id] = y0 + kDcOffset;
  }
}

// Full-tile forward kernel, w = 32, 8-bit samples.  One wavefront per block;
// the grid loops over all blocks of all frames of the launch, each wavefront
// keeping VCA_PREFETCH_DEPTH blocks in flight in a register ring (the loop
// body is unrolled over the ring, so no registers move).
// kRegs: accumulator registers that hold coefficients inside the K x K corner
// (16: K = 32, 8: K = 16, 4: K = 8); kKeep: also store the coefficients.
template <int kBits, int kRegs, bool kKeep>
__global__ __launch_bounds__(kGroupThreads) void fwd32_kernel(FwdParams p) {
  constexpr int kDepth = VCA_PREFETCH_DEPTH;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 31;             // tile row loaded by this lane / output column
  const int g = lane >> 5;             // half of the row loaded by this lane
  const uint32_t lane_off[2] = {(uint32_t)(r * p.pitch[0] + 16 * g),
                                (uint32_t)(r * p.pitch[1] + 16 * g)};

  TileConsts<kRegs> tc;
  tc.b1 = p.tab_b1[lane];
  tc.a2 = p.tab_a2[lane];
#pragma unroll
  for (int j = 0; j < kRegs; j++) tc.wt[j] = p.tab_w[j * 64 + lane];
  tc.row0_fix = g == 0 ? 128 : 0;

  const int total = p.n_frames * p.per_frame;
  const int stride = gridDim.x * kWavesPerGroup;
  int id = blockIdx.x * kWavesPerGroup + wave;
  v4i ring[kDepth];
#pragma unroll
  for (int s = 0; s < kDepth; s++) {
    const int nid = id + s * stride;
    ring[s] = nid < total ? load_block(p, nid, lane_off) : v4i{};
  }
  while (id < total) {
#pragma unroll
    for (int s = 0; s < kDepth; s++) {
      if (id < total) {
        const v4i x = ring[s];
        const int nid = id + kDepth * stride;
        if (nid < total) ring[s] = load_block(p, nid, lane_off);
        fwd32_block<kBits, kRegs, kKeep>(p, tc, x, id, lane);
        id += stride;
      }
    }
  }
}

// One workgroup per frame: fixed-order FP64 sums of H, sqrt(DC) and |dH|.
__global__ __launch_bounds__(256) void reduce_kernel(ReduceParams p) {
  __shared__ double red[7][256];
  const int f = blockIdx.x;
  const int t = threadIdx.x;
  const double* H = p.blk_h + (int64_t)f * p.per_frame;
  const int32_t* DC = p.blk_dc + (int64_t)f * p.per_frame;
  const double* prev = f > 0 ? H - p.per_frame : p.state_in;
  double s[7] = {0, 0, 0, 0, 0, 0, 0};   // H_Y H_U H_V L_Y L_U L_V dH
  const int e0 = p.cnt[0], e1 = p.cnt[0] + p.cnt[1];
  for (int b = t; b < p.per_frame; b += 256) {
    const int P = b < e0 ? 0 : (b < e1 ? 1 : 2);
    const double hb = H[b];
    s[P] += hb;
    s[3 + P] += sqrt((double)DC[b]);
    if (P == 0 && prev) s[6] += fabs(hb - prev[b]);
  }
#pragma unroll
  for (int q = 0; q < 7; q++) red[q][t] = s[q];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int q = 0; q < 7; q++) red[q][t] += red[q][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    float* o = p.ring + ((p.first_frame + f) % p.capacity) * 7;
    o[0] = (float)(red[0][0] * p.inv_norm[0]);
    o[1] = (float)(red[6][0] * p.inv_norm[0]);
    o[2] = (float)(red[3][0] * p.inv_norm[0]);
    o[3] = (float)(red[1][0] * p.inv_norm[1]);
    o[4] = (float)(red[2][0] * p.inv_norm[2]);
    o[5] = (float)(red[4][0] * p.inv_norm[1]);
    o[6] = (float)(red[5][0] * p.inv_norm[2]);
  }
  if (f == p.n_frames - 1)
    for (int b = t; b < p.cnt[0]; b += 256) p.state_out[b] = H[b];
}

}  // namespace

// =================================================================== host side
struct vca_ctx {
  vca_config cfg{};
  int K = 0;
  int32_t cnt[3] = {0, 0, 0};
  int32_t nbx[3] = {0, 0, 0};
  int32_t per_frame = 0;
  int device = 0;
  int num_cus = 0;
  int groups_per_cu = 0;           // 0: as many as fit (VCA_GROUPS_PER_CU overrides)
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // device tables and state
  v4i* tab_b1 = nullptr;
  v4i* tab_a2 = nullptr;
  double* tab_w = nullptr;
  double* blk_h = nullptr;
  int32_t* blk_dc = nullptr;
  int16_t* coeffs = nullptr;
  double* state[2] = {nullptr, nullptr};
  float* ring = nullptr;
  int cur_state = 0;
  bool has_prev = false;
  int64_t submitted = 0;
  int64_t last_chunk_first = -1;  // global index of frame 0 of the most recent launch
  int32_t last_chunk_len = 0;
  int64_t last_call_first = -1;
  int32_t last_call_len = 0;
  // VCA_F_TIMING: one (start, middle, end) event triple per launch pair
  std::vector<hipEvent_t> ev_pool;
  std::vector<int32_t> ev_frames;
  size_t ev_used = 0;
  std::string err;
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int now = -1;
    if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
  }
};

vca_status fail(vca_ctx* c, vca_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

vca_status hip_fail(vca_ctx* c, hipError_t e, const char* what) {
  return fail(c, VCA_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                     \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr);   \
  } while (0)

vca_status check_config(const vca_config* cfg) {
  if (!cfg) return VCA_ERR_INVALID_ARG;
  if (cfg->struct_size != sizeof(vca_config)) return VCA_ERR_INVALID_ARG;
  const int w = cfg->block_size;
  if (w != 8 && w != 16 && w != 32) return VCA_ERR_INVALID_ARG;
  if (cfg->bit_depth != 8 && cfg->bit_depth != 10) return VCA_ERR_INVALID_ARG;
  if (cfg->chroma_format != 420) return VCA_ERR_INVALID_ARG;
  if (cfg->width <= 0 || cfg->height <= 0 || cfg->width % 2 || cfg->height % 2)
    return VCA_ERR_INVALID_ARG;
  if (cfg->width / 2 < w || cfg->height / 2 < w) return VCA_ERR_INVALID_ARG;
  const int k = cfg->lowpass_k;
  if (k != 0 && k != w && k != w / 2 && k != w / 4) return VCA_ERR_INVALID_ARG;
  if (cfg->max_batch < 0 || cfg->feature_capacity < 0 || cfg->device < 0)
    return VCA_ERR_INVALID_ARG;
  if (cfg->flags & ~(VCA_F_KEEP_COEFFS | VCA_F_VALIDATE | VCA_F_TIMING)) return VCA_ERR_INVALID_ARG;
  return VCA_OK;
}

template <typename T>
vca_status dev_alloc(vca_ctx* c, T** p, size_t count) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
  if (e == hipErrorOutOfMemory) return fail(c, VCA_ERR_OOM, "hipMalloc: out of device memory");
  if (e != hipSuccess) return hip_fail(c, e, "hipMalloc");
  return VCA_OK;
}

// Per-lane operand and weight tables for the 32 x 32 tile.
void build_tables(int w, int K, std::vector<int8_t>& b1, std::vector<int8_t>& a2,
                  std::vector<double>& wt) {
  b1.assign(64 * 16, 0);
  a2.assign(64 * 16, 0);
  wt.assign(16 * 64, 0.0);
  for (int lane = 0; lane < 64; lane++) {
    const int c = lane & 31, g = lane >> 5;
    for (int j = 0; j < 16; j++) {
      // stage 1: B[n][k] = C[k][n] with n = 16 g + j (the bytes each lane loads)
      b1[lane * 16 + j] = (int8_t)matw(w, c, 16 * g + j);
      // stage 2: A[i][m] = C[i][m] with m = the row held by accumulator register j
      const int m = 8 * (j >> 2) + 4 * g + (j & 3);
      a2[lane * 16 + j] = (int8_t)matw(w, c, m);
      // weight of output (i, k) held by register j of lane (k + 32 g)
      const int i = m;
      double wv = 0.0;
      if (i < K && c < K && !(i == 0 && c == 0)) {
        const double q = (double)((i + 1) * (c + 1)) / (double)(w * w);
        wv = std::exp(std::fabs(q * q - 1.0));
      }
      wt[j * 64 + lane] = wv;
    }
  }
}

}  // namespace

extern "C" {

vca_status vca_block_counts(const vca_config* cfg, int32_t counts[3]) {
  if (!counts) return VCA_ERR_INVALID_ARG;
  vca_status s = check_config(cfg);
  if (s != VCA_OK) return s;
  const int w = cfg->block_size;
  counts[0] = (cfg->width / w) * (cfg->height / w);
  counts[1] = (cfg->width / 2 / w) * (cfg->height / 2 / w);
  counts[2] = counts[1];
  return VCA_OK;
}

const char* vca_status_str(vca_status s) {
  switch (s) {
    case VCA_OK: return "VCA_OK";
    case VCA_ERR_INVALID_ARG: return "VCA_ERR_INVALID_ARG";
    case VCA_ERR_UNSUPPORTED: return "VCA_ERR_UNSUPPORTED";
    case VCA_ERR_OOM: return "VCA_ERR_OOM";
    case VCA_ERR_DEVICE: return "VCA_ERR_DEVICE";
    case VCA_ERR_STATE: return "VCA_ERR_STATE";
  }
  return "VCA_ERR_UNKNOWN";
}

const char* vca_last_error(const vca_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

int64_t vca_frames_submitted(const vca_ctx* ctx) { return ctx ? ctx->submitted : -1; }

void vca_close(vca_ctx* ctx) {
  if (!ctx) return;
  {
    DeviceGuard g(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    void* bufs[] = {ctx->tab_b1, ctx->tab_a2, ctx->tab_w, ctx->blk_h, ctx->blk_dc,
                    ctx->coeffs, ctx->state[0], ctx->state[1], ctx->ring};
    for (void* b : bufs)
      if (b) (void)hipFree(b);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  }
  delete ctx;
}

vca_status vca_open(const vca_config* cfg, void* hip_stream, vca_ctx** out) {
  if (!out) return VCA_ERR_INVALID_ARG;
  *out = nullptr;
  vca_status s = check_config(cfg);
  if (s != VCA_OK) return s;
  if (cfg->block_size != 32 || cfg->bit_depth != 8) return VCA_ERR_UNSUPPORTED;

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return VCA_ERR_DEVICE;
  if (cfg->device >= ndev) return VCA_ERR_INVALID_ARG;

  vca_ctx* c = new (std::nothrow) vca_ctx();
  if (!c) return VCA_ERR_OOM;
  c->cfg = *cfg;
  if (c->cfg.max_batch == 0) c->cfg.max_batch = 256;
  if (c->cfg.feature_capacity == 0) c->cfg.feature_capacity = 65536;
  const int w0 = cfg->block_size;
  const int64_t per_frame0 =
      (int64_t)(cfg->width / w0) * (cfg->height / w0) + 2 * (int64_t)(cfg->width / 2 / w0) * (cfg->height / 2 / w0);
  if ((int64_t)c->cfg.max_batch * per_frame0 > (int64_t)INT32_MAX / 2) {
    delete c;
    return VCA_ERR_INVALID_ARG;   // block ids of one launch must fit int32
  }
  const int w = cfg->block_size;
  c->K = cfg->lowpass_k == 0 ? w : cfg->lowpass_k;
  vca_block_counts(cfg, c->cnt);
  c->nbx[0] = cfg->width / w;
  c->nbx[1] = c->nbx[2] = cfg->width / 2 / w;
  c->per_frame = c->cnt[0] + c->cnt[1] + c->cnt[2];
  c->device = cfg->device;

  auto bail = [&](vca_status st) {
    vca_close(c);
    return st;
  };
  DeviceGuard guard(c->device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return bail(VCA_ERR_DEVICE);
  c->num_cus = prop.multiProcessorCount;
  if (const char* e = std::getenv("VCA_GROUPS_PER_CU")) c->groups_per_cu = std::atoi(e);
  if (hip_stream) {
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(VCA_ERR_DEVICE);
    c->own_stream = true;
  }
  const size_t mb = (size_t)c->cfg.max_batch;
  if ((s = dev_alloc(c, &c->tab_b1, 64)) != VCA_OK) return bail(s);
  if ((s = dev_alloc(c, &c->tab_a2, 64)) != VCA_OK) return bail(s);
  if ((s = dev_alloc(c, &c->tab_w, 16 * 64)) != VCA_OK) return bail(s);
  if ((s = dev_alloc(c, &c->blk_h, mb * c->per_frame)) != VCA_OK) return bail(s);
  if ((s = dev_alloc(c, &c->blk_dc, mb * c->per_frame)) != VCA_OK) return bail(s);
  if ((s = dev_alloc(c, &c->state[0], c->cnt[0])) != VCA_OK) return bail(s);
  if ((s = dev_alloc(c, &c->state[1], c->cnt[0])) != VCA_OK) return bail(s);
  if ((s = dev_alloc(c, &c->ring, (size_t)c->cfg.feature_capacity * 7)) != VCA_OK) return bail(s);
  if (cfg->flags & VCA_F_KEEP_COEFFS)
    if ((s = dev_alloc(c, &c->coeffs, mb * c->per_frame * c->K * c->K)) != VCA_OK) return bail(s);

  std::vector<int8_t> b1, a2;
  std::vector<double> wt;
  build_tables(w, c->K, b1, a2, wt);
  if (hipMemcpy(c->tab_b1, b1.data(), b1.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->tab_a2, a2.data(), a2.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->tab_w, wt.data(), wt.size() * sizeof(double), hipMemcpyHostToDevice) !=
          hipSuccess)
    return bail(VCA_ERR_DEVICE);
  *out = c;
  return VCA_OK;
}

vca_status vca_reset(vca_ctx* ctx) {
  if (!ctx) return VCA_ERR_INVALID_ARG;
  ctx->has_prev = false;
  return VCA_OK;
}

vca_status vca_analyze_frames(vca_ctx* ctx, const vca_frames* fr, int32_t n_frames) {
  if (!ctx || !fr || n_frames < 0) return fail(ctx, VCA_ERR_INVALID_ARG, "null argument or n < 0");
  if (!fr->on_device) return fail(ctx, VCA_ERR_UNSUPPORTED, "host-resident frames");
  if (n_frames == 0) return VCA_OK;
  const vca_config& cfg = ctx->cfg;
  const int bps = cfg.bit_depth == 8 ? 1 : 2;
  if (!fr->y || !fr->u || !fr->v) return fail(ctx, VCA_ERR_INVALID_ARG, "null plane pointer");
  if (fr->pitch_y < (int64_t)cfg.width * bps || fr->pitch_uv < (int64_t)cfg.width / 2 * bps)
    return fail(ctx, VCA_ERR_INVALID_ARG, "pitch smaller than a row");
  if (fr->pitch_y > (1 << 26) || fr->pitch_uv > (1 << 26))
    return fail(ctx, VCA_ERR_INVALID_ARG, "pitch above 64 MiB");   // lane offsets are 32-bit
  if (n_frames > 1 && (fr->fstride_y < fr->pitch_y * cfg.height ||
                       fr->fstride_uv < fr->pitch_uv * (cfg.height / 2)))
    return fail(ctx, VCA_ERR_INVALID_ARG, "frame stride smaller than a frame");
  const uintptr_t align = (uintptr_t)fr->y | (uintptr_t)fr->u | (uintptr_t)fr->v |
                          (uintptr_t)fr->pitch_y | (uintptr_t)fr->pitch_uv |
                          (uintptr_t)fr->fstride_y | (uintptr_t)fr->fstride_uv;
  if (align & 15) return fail(ctx, VCA_ERR_INVALID_ARG, "planes, pitches and strides need 16-byte alignment");
  if ((cfg.flags & VCA_F_KEEP_COEFFS) && n_frames > cfg.max_batch)
    return fail(ctx, VCA_ERR_INVALID_ARG, "VCA_F_KEEP_COEFFS: n_frames exceeds max_batch");

  DeviceGuard guard(ctx->device);
  const int w = cfg.block_size;
  const double ww = (double)w * w;
  ctx->last_call_first = ctx->submitted;
  ctx->last_call_len = n_frames;
  for (int32_t done = 0; done < n_frames;) {
    const int32_t n = std::min<int32_t>(cfg.max_batch, n_frames - done);
    FwdParams fp{};
    const uint8_t* base[3] = {static_cast<const uint8_t*>(fr->y), static_cast<const uint8_t*>(fr->u),
                              static_cast<const uint8_t*>(fr->v)};
    const int64_t fs[3] = {fr->fstride_y, fr->fstride_uv, fr->fstride_uv};
    const int64_t pt[3] = {fr->pitch_y, fr->pitch_uv, fr->pitch_uv};
    for (int P = 0; P < 3; P++) {
      fp.plane[P] = base[P] + fs[P] * done;
      fp.pitch[P] = pt[P];
      fp.fstride[P] = fs[P];
      fp.nbx[P] = ctx->nbx[P];
      fp.cnt[P] = ctx->cnt[P];
      fp.div_nbx[P] = make_fastdiv((uint32_t)ctx->nbx[P]);
    }
    fp.div_frame = make_fastdiv((uint32_t)ctx->per_frame);
    fp.per_frame = ctx->per_frame;
    fp.n_frames = n;
    fp.k = ctx->K;
    fp.tab_b1 = ctx->tab_b1;
    fp.tab_a2 = ctx->tab_a2;
    fp.tab_w = ctx->tab_w;
    fp.blk_h = ctx->blk_h;
    fp.blk_dc = ctx->blk_dc;
    fp.coeffs = ctx->coeffs;
    const int64_t waves = (int64_t)n * ctx->per_frame;
    const int64_t groups_needed = (waves + kWavesPerGroup - 1) / kWavesPerGroup;
    const bool keep = ctx->coeffs != nullptr;
    const int regs = ctx->K == 32 ? 16 : (ctx->K == 16 ? 8 : 4);
    void (*kern)(FwdParams) = nullptr;
    if (regs == 16) kern = keep ? fwd32_kernel<8, 16, true> : fwd32_kernel<8, 16, false>;
    if (regs == 8) kern = keep ? fwd32_kernel<8, 8, true> : fwd32_kernel<8, 8, false>;
    if (regs == 4) kern = keep ? fwd32_kernel<8, 4, true> : fwd32_kernel<8, 4, false>;
    // Persistent grid: exactly as many workgroups as can be resident at once,
    // so no workgroup waits for another to drain before it starts its loop.
    int resident = 0;
    HIP_TRY(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, kern, kGroupThreads, 0));
    resident = std::max(1, resident);
    if (ctx->groups_per_cu > 0) resident = std::min(resident, ctx->groups_per_cu);
    const int grid = (int)std::min<int64_t>(groups_needed, (int64_t)ctx->num_cus * resident);
    hipEvent_t* ev = nullptr;
    if (cfg.flags & VCA_F_TIMING) {
      if (ctx->ev_used + 3 > ctx->ev_pool.size()) {
        for (int e = 0; e < 3; e++) {
          hipEvent_t h;
          HIP_TRY(ctx, hipEventCreate(&h));
          ctx->ev_pool.push_back(h);
        }
      }
      ev = &ctx->ev_pool[ctx->ev_used];
      ctx->ev_frames.push_back(n);
      ctx->ev_used += 3;
      HIP_TRY(ctx, hipEventRecord(ev[0], ctx->stream));
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kGroupThreads), 0, ctx->stream, fp);
    HIP_TRY(ctx, hipGetLastError());
    if (ev) HIP_TRY(ctx, hipEventRecord(ev[1], ctx->stream));

    ReduceParams rp{};
    rp.blk_h = ctx->blk_h;
    rp.blk_dc = ctx->blk_dc;
    rp.state_in = ctx->has_prev ? ctx->state[ctx->cur_state] : nullptr;
    rp.state_out = ctx->state[ctx->cur_state ^ 1];
    rp.ring = ctx->ring;
    rp.first_frame = ctx->submitted;
    rp.capacity = cfg.feature_capacity;
    for (int P = 0; P < 3; P++) {
      rp.cnt[P] = ctx->cnt[P];
      rp.inv_norm[P] = 1.0 / ((double)ctx->cnt[P] * ww);
    }
    rp.per_frame = ctx->per_frame;
    rp.n_frames = n;
    hipLaunchKernelGGL(reduce_kernel, dim3(n), dim3(256), 0, ctx->stream, rp);
    HIP_TRY(ctx, hipGetLastError());
    if (ev) HIP_TRY(ctx, hipEventRecord(ev[2], ctx->stream));
    ctx->cur_state ^= 1;
    ctx->has_prev = true;
    ctx->last_chunk_first = ctx->submitted;
    ctx->last_chunk_len = n;
    ctx->submitted += n;
    done += n;
  }
  return VCA_OK;
}

vca_status vca_features(vca_ctx* ctx, int64_t first, int32_t count, vca_frame_features* out) {
  if (!ctx || count < 0 || first < 0 || (count > 0 && !out))
    return fail(ctx, VCA_ERR_INVALID_ARG, "bad vca_features arguments");
  if (first + count > ctx->submitted) return fail(ctx, VCA_ERR_STATE, "frame not yet submitted");
  const int64_t cap = ctx->cfg.feature_capacity;
  if (first < ctx->submitted - cap) return fail(ctx, VCA_ERR_STATE, "frame left the feature ring");
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  int64_t done = 0;
  while (done < count) {
    const int64_t slot = (first + done) % cap;
    const int64_t n = std::min<int64_t>(count - done, cap - slot);
    HIP_TRY(ctx, hipMemcpy(reinterpret_cast<float*>(out) + done * 7, ctx->ring + slot * 7,
                           (size_t)n * 7 * sizeof(float), hipMemcpyDeviceToHost));
    done += n;
  }
  return VCA_OK;
}

vca_status vca_get_timing(vca_ctx* ctx, vca_timing* out, int32_t reset) {
  if (!ctx || !out) return fail(ctx, VCA_ERR_INVALID_ARG, "null argument");
  if (!(ctx->cfg.flags & VCA_F_TIMING)) return fail(ctx, VCA_ERR_STATE, "opened without VCA_F_TIMING");
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  vca_timing t{};
  for (size_t i = 0; i + 3 <= ctx->ev_used; i += 3) {
    float a = 0.f, b = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&a, ctx->ev_pool[i], ctx->ev_pool[i + 1]));
    HIP_TRY(ctx, hipEventElapsedTime(&b, ctx->ev_pool[i + 1], ctx->ev_pool[i + 2]));
    t.forward_ms += a;
    t.reduce_ms += b;
    t.forward_launches++;
    t.reduce_launches++;
    t.frames += ctx->ev_frames[i / 3];
  }
  *out = t;
  if (reset) {
    ctx->ev_used = 0;
    ctx->ev_frames.clear();
  }
  return VCA_OK;
}

vca_status vca_block_coeffs(vca_ctx* ctx, int64_t frame, int16_t* out, size_t capacity) {
  if (!ctx || !out) return fail(ctx, VCA_ERR_INVALID_ARG, "null argument");
  if (!ctx->coeffs) return fail(ctx, VCA_ERR_STATE, "context opened without VCA_F_KEEP_COEFFS");
  if (frame < ctx->last_chunk_first || frame >= ctx->last_chunk_first + ctx->last_chunk_len)
    return fail(ctx, VCA_ERR_STATE, "frame not in the most recent call");
  const size_t per = (size_t)ctx->per_frame * ctx->K * ctx->K;
  if (capacity < per) return fail(ctx, VCA_ERR_INVALID_ARG, "output buffer too small");
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  HIP_TRY(ctx, hipMemcpy(out, ctx->coeffs + (frame - ctx->last_chunk_first) * per,
                         per * sizeof(int16_t), hipMemcpyDeviceToHost));
  return VCA_OK;
}

vca_status vca_block_stats(vca_ctx* ctx, int64_t frame, double* h_out, int32_t* dc_out,
                           size_t capacity) {
  if (!ctx || (!h_out && !dc_out)) return fail(ctx, VCA_ERR_INVALID_ARG, "null argument");
  if (frame < ctx->last_chunk_first || frame >= ctx->last_chunk_first + ctx->last_chunk_len)
    return fail(ctx, VCA_ERR_STATE, "frame not in the most recent launch");
  if (capacity < (size_t)ctx->per_frame) return fail(ctx, VCA_ERR_INVALID_ARG, "output buffer too small");
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  const int64_t off = (frame - ctx->last_chunk_first) * ctx->per_frame;
  if (h_out)
    HIP_TRY(ctx, hipMemcpy(h_out, ctx->blk_h + off, ctx->per_frame * sizeof(double),
                           hipMemcpyDeviceToHost));
  if (dc_out)
    HIP_TRY(ctx, hipMemcpy(dc_out, ctx->blk_dc + off, ctx->per_frame * sizeof(int32_t),
                           hipMemcpyDeviceToHost));
  return VCA_OK;
}

}  // extern "C"
