// vca.hip -- MI355X (gfx950) Video Complexity Analyzer: plain path and C ABI.
//
// Computes the per-frame block-DCT features of Menon et al. (GMSys 2023),
// Section 2 (E_Y, h, L_Y, E_U, E_V, L_U, L_V) and the low-pass option of the
// same section, for 8/10-bit 4:2:0 video and block sizes 8, 16, 32.  The
// definitions implemented are stated in include/vca.h.
//
// Kernels:
//   fwd_kernel     persistent grid over all 32 x 32 tiles of all frames of a
//                  launch; one wavefront per tile (vca_tile.h) with a
//                  register ring of tiles in flight; per-block H and DC out.
//   reduce_kernel  one workgroup per frame: fixed-order FP64 sums of H,
//                  sqrt(DC) and |H_p - H_{p-1}| into the seven features.

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
#include "vca_tile.h"

using namespace vca;

namespace {

constexpr int kWavesPerGroup = 4;   // wavefronts per workgroup
constexpr int kGroupThreads = 64 * kWavesPerGroup;

// Tiles each wavefront keeps in flight ahead of the one it transforms.
#ifndef VCA_PREFETCH_DEPTH
#define VCA_PREFETCH_DEPTH 2
#endif

struct FwdParams {
  const uint8_t* plane[3];
  int32_t pitch[3];        // bytes between rows
  int64_t fstride[3];      // bytes between frames
  int32_t nbx[3], nby[3];  // blocks per row / column of each plane
  int32_t ntx[3];          // tiles per row
  int32_t tcnt[3];         // tiles per plane
  int32_t boff[3];         // index of the plane's first block within a frame
  int32_t tiles_per_frame;
  int32_t per_frame;       // blocks per frame
  FastDiv div_tpf;         // / tiles_per_frame
  FastDiv div_ntx[3];      // / ntx[P]
  int32_t n_frames;
  const v4i* tab_b1;
  const v4i* tab_a2;
  const double* tab_w;
  TileOut out;
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

// Tile `id` of a launch (frame-major, then Y, U, V, then raster order).
template <int kBits, int kW>
__device__ inline TileWork decode_tile(const FwdParams& p, int id) {
  constexpr int kBps = kBits == 8 ? 1 : 2;
  constexpr int kBpt = kTile / kW;
  const int f = (int)fastdiv((uint32_t)id, p.div_tpf);
  int t = id - f * p.tiles_per_frame;
  int P = 0;
  if (t >= p.tcnt[0]) {
    t -= p.tcnt[0];
    P = 1;
    if (t >= p.tcnt[1]) {
      t -= p.tcnt[1];
      P = 2;
    }
  }
  const int ty = (int)fastdiv((uint32_t)t, p.div_ntx[P]);
  const int tx = t - ty * p.ntx[P];
  const int by0 = ty * kBpt, bx0 = tx * kBpt;
  TileWork w;
  w.pitch = p.pitch[P];
  w.base = p.plane[P] + f * p.fstride[P] + (int64_t)by0 * kW * w.pitch + bx0 * kW * kBps;
  w.vr = min(kBpt, p.nby[P] - by0);
  w.vc = min(kBpt, p.nbx[P] - bx0);
  w.out0 = f * p.per_frame + p.boff[P] + by0 * p.nbx[P] + bx0;
  w.out_row = p.nbx[P];
  return w;
}

// Persistent forward kernel: each wavefront walks tiles id, id + S, ...
// (S = all wavefronts of the grid), keeping VCA_PREFETCH_DEPTH tiles in
// flight in a register ring (the loop body is unrolled over the ring, so no
// registers move).
template <int kBits, int kW, int kK, bool kKeep>
__global__ __launch_bounds__(kGroupThreads) void fwd_kernel(FwdParams p) {
  constexpr int kDepth = VCA_PREFETCH_DEPTH;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  TileConsts<kW, kK> tc;
  tc.load(p.tab_b1, p.tab_a2, p.tab_w, lane);

  const int total = p.n_frames * p.tiles_per_frame;
  const int stride = gridDim.x * kWavesPerGroup;
  int id = blockIdx.x * kWavesPerGroup + wave;
  TileData ring[kDepth];
#pragma unroll
  for (int s = 0; s < kDepth; s++) {
    const int nid = id + s * stride;
    if (nid < total) ring[s] = load_tile<kBits, kW>(decode_tile<kBits, kW>(p, nid), lane);
  }
  while (id < total) {
#pragma unroll
    for (int s = 0; s < kDepth; s++) {
      if (id < total) {
        const TileData d = ring[s];
        const int nid = id + kDepth * stride;
        if (nid < total) ring[s] = load_tile<kBits, kW>(decode_tile<kBits, kW>(p, nid), lane);
        fwd_tile<kBits, kW, kK, kKeep>(p.out, tc, d, decode_tile<kBits, kW>(p, id), lane);
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
  int32_t nby[3] = {0, 0, 0};
  int32_t ntx[3] = {0, 0, 0};
  int32_t tcnt[3] = {0, 0, 0};
  int32_t per_frame = 0;
  int32_t tiles_per_frame = 0;
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
  int32_t* err_flag = nullptr;
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

// Kernel for (bit depth, w, K, coefficient export).
using FwdKernel = void (*)(FwdParams);

template <int B, int W, int K>
FwdKernel pick_keep(bool keep) {
  return keep ? fwd_kernel<B, W, K, true> : fwd_kernel<B, W, K, false>;
}

template <int B, int W>
FwdKernel pick_k(int K, bool keep) {
  if (K == W) return pick_keep<B, W, W>(keep);
  if (K == W / 2) return pick_keep<B, W, W / 2>(keep);
  if (K == W / 4) return pick_keep<B, W, W / 4>(keep);
  return nullptr;
}

template <int B>
FwdKernel pick_w(int w, int K, bool keep) {
  if (w == 32) return pick_k<B, 32>(K, keep);
  if (w == 16) return pick_k<B, 16>(K, keep);
  if (w == 8) return pick_k<B, 8>(K, keep);
  return nullptr;
}

FwdKernel select_fwd_kernel(int bits, int w, int K, bool keep) {
  return bits == 8 ? pick_w<8>(w, K, keep) : (bits == 10 ? pick_w<10>(w, K, keep) : nullptr);
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
    void* bufs[] = {ctx->tab_b1, ctx->tab_a2, ctx->tab_w, ctx->blk_h,    ctx->blk_dc,
                    ctx->coeffs, ctx->err_flag, ctx->state[0], ctx->state[1], ctx->ring};
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
  const int bpt = kTile / w;
  for (int P = 0; P < 3; P++) {
    const int pw = P == 0 ? cfg->width : cfg->width / 2;
    const int ph = P == 0 ? cfg->height : cfg->height / 2;
    c->nbx[P] = pw / w;
    c->nby[P] = ph / w;
    c->ntx[P] = (c->nbx[P] + bpt - 1) / bpt;
    c->tcnt[P] = c->ntx[P] * ((c->nby[P] + bpt - 1) / bpt);
  }
  c->per_frame = c->cnt[0] + c->cnt[1] + c->cnt[2];
  c->tiles_per_frame = c->tcnt[0] + c->tcnt[1] + c->tcnt[2];
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
  if ((s = dev_alloc(c, &c->err_flag, 1)) != VCA_OK) return bail(s);
  if (hipMemset(c->err_flag, 0, sizeof(int32_t)) != hipSuccess) return bail(VCA_ERR_DEVICE);
  if (cfg->flags & VCA_F_KEEP_COEFFS)
    if ((s = dev_alloc(c, &c->coeffs, mb * c->per_frame * c->K * c->K)) != VCA_OK) return bail(s);

  std::vector<int8_t> b1, a2;
  std::vector<double> wt;
  build_tile_tables(w, c->K, b1, a2, wt);
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
  if (fr->pitch_y >= (1 << 23) || fr->pitch_uv >= (1 << 23))
    return fail(ctx, VCA_ERR_INVALID_ARG, "pitch of 8 MiB or more");   // 24-bit lane offsets
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
    int32_t boff = 0;
    for (int P = 0; P < 3; P++) {
      fp.plane[P] = base[P] + fs[P] * done;
      fp.pitch[P] = (int32_t)pt[P];
      fp.fstride[P] = fs[P];
      fp.nbx[P] = ctx->nbx[P];
      fp.nby[P] = ctx->nby[P];
      fp.ntx[P] = ctx->ntx[P];
      fp.tcnt[P] = ctx->tcnt[P];
      fp.boff[P] = boff;
      boff += ctx->cnt[P];
      fp.div_ntx[P] = make_fastdiv((uint32_t)ctx->ntx[P]);
    }
    fp.tiles_per_frame = ctx->tiles_per_frame;
    fp.per_frame = ctx->per_frame;
    fp.div_tpf = make_fastdiv((uint32_t)ctx->tiles_per_frame);
    fp.n_frames = n;
    fp.tab_b1 = ctx->tab_b1;
    fp.tab_a2 = ctx->tab_a2;
    fp.tab_w = ctx->tab_w;
    fp.out.blk_h = ctx->blk_h;
    fp.out.blk_dc = ctx->blk_dc;
    fp.out.coeffs = ctx->coeffs;
    fp.out.err_flag = ctx->err_flag;
    fp.out.validate = (cfg.flags & VCA_F_VALIDATE) && cfg.bit_depth == 10 ? 1 : 0;
    const int64_t waves = (int64_t)n * ctx->tiles_per_frame;
    const int64_t groups_needed = (waves + kWavesPerGroup - 1) / kWavesPerGroup;
    void (*kern)(FwdParams) = select_fwd_kernel(cfg.bit_depth, cfg.block_size, ctx->K, ctx->coeffs != nullptr);
    if (!kern) return fail(ctx, VCA_ERR_UNSUPPORTED, "no kernel for this configuration");
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
  if (ctx->cfg.flags & VCA_F_VALIDATE) {
    int32_t bad = 0;
    HIP_TRY(ctx, hipMemcpy(&bad, ctx->err_flag, sizeof(bad), hipMemcpyDeviceToHost));
    if (bad) return fail(ctx, VCA_ERR_STATE, "a 10-bit sample above 1023 was submitted");
  }
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
