// vca.hip -- MI355X (gfx950) Video Complexity Analyzer: plain path and C ABI.
//
// Computes the per-frame block-DCT features of Menon et al. (GMSys 2023),
// Section 2 (E_Y, h, L_Y, E_U, E_V, L_U, L_V) and the low-pass option of the
// same section, for 8/10-bit 4:2:0 video and block sizes 8, 16, 32.  The
// definitions implemented are stated in include/vca.h.
//
// Kernels:
//   strip_kernel   persistent grid over the strips of 32 x 32 tiles of all
//                  frames of a launch (vca_strip.h): wavefronts walk runs of
//                  strips with a register ring of tiles in flight; per-block
//                  H and DC out (and, for tests, the K x K coefficients).
//   reduce_kernel  one workgroup per frame (vca_reduce.h).
// Launch shape (ring depth, workgroups per CU) comes from vca_tune's
// measurements when the context was tuned, else from fixed defaults.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/vca.h"
#include "vca_host.h"
#include "vca_ingest.h"
#include "vca_reduce.h"
#include "vca_strip.h"
#include "vca_tile.h"

using namespace vca;

namespace {

constexpr int kWavesPerGroup = 4;   // wavefronts per workgroup
constexpr int kGroupThreads = 64 * kWavesPerGroup;
constexpr int kDefaultDepth = 2;    // tiles in flight per wavefront when untuned
constexpr int kDefaultMaxBatch = 256;     // vca_config.max_batch = 0
constexpr int kDefaultCapacity = 65536;   // vca_config.feature_capacity = 0

int effective(int32_t v, int32_t dflt) { return v == 0 ? dflt : v; }

struct FwdParams {
  int32_t n_frames;
  StripGeom geom;          // the launch's frames as strips
  const v4i* tab_a2;       // stage-2 operand per lane
  const v4i* tab_b1p;      // w / K stage-1 operands per lane (packed layout; K = w: one)
  const double* tab_wp;    // weights of the packed layout
  TileOut out;
};

// Persistent forward kernel over strips (vca_strip.h): wavefront i of S
// takes the runs of kRunLen strips i, i + S, ...
// kDs: the planes are downsampled by two on the fly (VCA_F_DOWNSAMPLE);
// kValidate (10-bit): samples above 1023 mark their frame; kKeep: the K x K
// coefficients of every block are exported as well (VCA_F_KEEP_COEFFS).
template <int kBits, int kW, int kK, int kDepth, bool kDs, bool kValidate, int kRunLen = kRun,
          bool kKeep = false>
__global__ __launch_bounds__(kGroupThreads) void strip_kernel(FwdParams p) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int kStage = stage_bytes(kW) > 0 ? stage_bytes(kW) : 16;
  __shared__ __attribute__((aligned(16))) uint8_t stage[kWavesPerGroup][kStage];
  PackConsts<kW, kK> pc;
  pc.load(p.tab_b1p, p.tab_a2, p.tab_wp, lane);
  run_strips<kBits, kW, kK, kDepth, kDs, kValidate, kRunLen, kKeep>(
      p.geom, p.out, pc, blockIdx.x * kWavesPerGroup + wave, gridDim.x * kWavesPerGroup,
      p.n_frames * p.geom.strips_per_frame, lane, stage[wave]);
}

__global__ __launch_bounds__(kReduceThreads) void reduce_kernel(ReduceParams p) {
  reduce_frame(p, blockIdx.x);
}

// Per-block maps of `count` frames starting at frame f0 of the last launch:
// H and DC copied, |H_t - H_{t-1}| for luma blocks (prev = the frame before
// f0 of the launch, the state buffer, or none).
struct MapsParams {
  const double* blk_h;
  const int32_t* blk_dc;
  const double* prev;   // luma H of the frame before f0, or null
  double* h_out;
  int32_t* dc_out;
  double* dh_out;
  int64_t per_frame;
  int64_t cnt_y;
  int64_t f0;           // first frame, relative to the launch
  int64_t count;
};

constexpr int kMapsThreads = 256;

__global__ __launch_bounds__(kMapsThreads) void block_maps_kernel(MapsParams p) {
  const int64_t i = (int64_t)blockIdx.y;   // frame of the range
  const int64_t f = p.f0 + i;
  const double* H = p.blk_h + f * p.per_frame;
  const int32_t* DC = p.blk_dc + f * p.per_frame;
  const double* prev = f > 0 ? H - p.per_frame : p.prev;
  for (int64_t b = (int64_t)blockIdx.x * kMapsThreads + threadIdx.x; b < p.per_frame;
       b += (int64_t)gridDim.x * kMapsThreads) {
    if (p.h_out) p.h_out[i * p.per_frame + b] = H[b];
    if (p.dc_out) p.dc_out[i * p.per_frame + b] = DC[b];
    if (p.dh_out && b < p.cnt_y) p.dh_out[i * p.cnt_y + b] = prev ? fabs(H[b] - prev[b]) : 0.0;
  }
}

// Kernel for (bit depth, w, K, downsampling, ring depth, validation, run
// length, coefficient export).
using FwdKernel = void (*)(FwdParams);

// validate (10-bit only): the validating kernel, one depth.  short_runs:
// runs of one strip for launches too small to fill the device with runs of
// kRun (one depth, the untuned default; one for validation).  keep: the
// exporting variant of the same walk (runs as the launch size picks them,
// ring depth 4 or the untuned default, validation decided at run time).
template <int B, int W, int K, bool kDs>
FwdKernel pick_depth(int depth, bool validate, bool short_runs, bool keep) {
  if constexpr (!kDs) {
    if (keep)
      return short_runs ? strip_kernel<B, W, K, kDefaultDepth, false, (B != 8), 1, true>
                        : strip_kernel<B, W, K, 4, false, (B != 8), kRun, true>;
  } else {
    if (keep) return nullptr;
  }
  if constexpr (B != 8) {
    if (validate) return short_runs ? strip_kernel<B, W, K, 1, kDs, true, 1> : strip_kernel<B, W, K, 1, kDs, true>;
  }
  if (short_runs) return strip_kernel<B, W, K, kDefaultDepth, kDs, false, 1>;
  if (depth == 1) return strip_kernel<B, W, K, 1, kDs, false>;
  if (depth >= 4) return strip_kernel<B, W, K, 4, kDs, false>;   // capped at the units per strip
  return strip_kernel<B, W, K, 2, kDs, false>;
}

template <int B, int W>
FwdKernel pick_k(int K, bool keep, bool ds, int depth, bool v, bool sr) {
  if (ds) return K == W ? pick_depth<B, W, W, true>(depth, v, sr, keep) : nullptr;
  if (K == W) return pick_depth<B, W, W, false>(depth, v, sr, keep);
  if (K == W / 2) return pick_depth<B, W, W / 2, false>(depth, v, sr, keep);
  if (K == W / 4) return pick_depth<B, W, W / 4, false>(depth, v, sr, keep);
  return nullptr;
}

template <int B>
FwdKernel pick_w(int w, int K, bool keep, bool ds, int depth, bool v, bool sr) {
  if (w == 32) return pick_k<B, 32>(K, keep, ds, depth, v, sr);
  if (w == 16) return pick_k<B, 16>(K, keep, ds, depth, v, sr);
  if (w == 8) return pick_k<B, 8>(K, keep, ds, depth, v, sr);
  return nullptr;
}

FwdKernel select_fwd_kernel(int bits, int w, int K, bool keep, bool ds, int depth, bool validate,
                            bool short_runs = false) {
  return bits == 8 ? pick_w<8>(w, K, keep, ds, depth, false, short_runs)
                   : (bits == 10 ? pick_w<10>(w, K, keep, ds, depth, validate, short_runs) : nullptr);
}

}  // namespace

// =================================================================== host side
struct vca_ctx {
  vca_config cfg{};
  Geometry geo;
  int device = 0;
  int num_cus = 0;
  int env_groups_per_cu = 0;       // VCA_GROUPS_PER_CU caps workgroups per CU
  LaunchChoice tuned;              // set by vca_tune
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // device tables and state
  v4i* tab_a2 = nullptr;
  v4i* tab_b1p = nullptr;
  double* tab_wp = nullptr;
  double* blk_h = nullptr;
  int32_t* blk_dc = nullptr;
  int16_t* coeffs = nullptr;
  int32_t* frame_err = nullptr;    // per frame of a launch: validation marks (device)
  int32_t* err_ring = nullptr;     // device view of err_ring_host
  int32_t* err_ring_host = nullptr;   // pinned, mapped: [feature_capacity] marks
  double* state[2] = {nullptr, nullptr};
  float* ring = nullptr;           // device view of ring_host
  float* ring_host = nullptr;      // pinned, mapped: [feature_capacity][7]
  int cur_state = 0;
  bool has_prev = false;
  bool last_chunk_prev = false;    // the last launch's first frame had a previous frame
  int64_t submitted = 0;
  int64_t last_chunk_first = -1;  // global index of frame 0 of the most recent launch
  int32_t last_chunk_len = 0;
  DoneMarks done;                  // completion of the recent launches
  // VCA_F_TIMING: one (start, middle, end) event triple per launch pair
  std::vector<hipEvent_t> ev_pool;
  std::vector<int32_t> ev_frames;
  size_t ev_used = 0;
  // host-resident frames: two staging slots (pinned host + device), filled
  // by the worker pool and copied on copy_stream; created on first use
  struct IngestSlot {
    uint8_t* pinned = nullptr;
    uint8_t* dev = nullptr;
    hipEvent_t copied = nullptr;   // its host-to-device copy is done
    hipEvent_t used = nullptr;     // the analysis reading it is done
    bool busy = false;
  };
  IngestSlot ing[2];
  int32_t ing_batch = 0;           // frames per slot
  int ing_next = 0;
  hipStream_t copy_stream = nullptr;
  std::unique_ptr<WorkerPool> pool;
  std::string err;
};

namespace {

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

template <typename T>
vca_status dev_alloc(vca_ctx* c, T** p, size_t count) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
  if (e == hipErrorOutOfMemory) return fail(c, VCA_ERR_OOM, "hipMalloc: out of device memory");
  if (e != hipSuccess) return hip_fail(c, e, "hipMalloc");
  return VCA_OK;
}

// Forward-launch parameters for frames [done, done + n) of a call.
FwdParams make_fwd_params(const vca_ctx* ctx, const vca_frames* fr, int32_t done, int32_t n) {
  FwdParams fp{};
  const uint8_t* base[3] = {static_cast<const uint8_t*>(fr->y), static_cast<const uint8_t*>(fr->u),
                            static_cast<const uint8_t*>(fr->v)};
  const int64_t fs[3] = {fr->fstride_y, fr->fstride_uv, fr->fstride_uv};
  const int64_t pt[3] = {fr->pitch_y, fr->pitch_uv, fr->pitch_uv};
  const uint8_t* first[3];
  for (int P = 0; P < 3; P++) first[P] = base[P] + fs[P] * done;
  fp.geom = make_strip_geom(ctx->geo, first, fs, pt, 0);
  fp.n_frames = n;
  fp.tab_a2 = ctx->tab_a2;
  fp.tab_b1p = ctx->tab_b1p;
  fp.tab_wp = ctx->tab_wp;
  fp.out.blk_h = ctx->blk_h;
  fp.out.blk_dc = ctx->blk_dc;
  fp.out.coeffs = ctx->coeffs;
  fp.out.err_flag = ctx->frame_err;
  fp.out.validate = (ctx->cfg.flags & VCA_F_VALIDATE) && ctx->cfg.bit_depth == 10 ? 1 : 0;
  return fp;
}

// Enqueues one forward launch of the strip kernel for (bits, w, K, ds) with
// the given ring depth and workgroup cap on `stream`.  allow_short = false:
// always runs of kRun (the autotuner times those; the tuned depth applies to
// them only).  On failure `err` receives the message.
vca_status enqueue_fwd(const Geometry& geo, int num_cus, hipStream_t stream, const FwdParams& fp,
                       int depth, int groups_per_cu, bool keep, bool validate, bool allow_short,
                       std::string& err) {
  // A launch whose runs of kRun strips would give fewer than four
  // wavefronts per CU (a frame or two at 2160p) takes runs of one strip, so
  // that a single frame spreads over the device instead of 47 workgroups.
  // The coefficient export follows the same rule, so it shows both walks.
  const int64_t strips = (int64_t)fp.n_frames * fp.geom.strips_per_frame;
  const bool short_runs = allow_short && (strips + kRun - 1) / kRun < 4 * (int64_t)num_cus;
  FwdKernel kern = select_fwd_kernel(geo.bits, geo.w, geo.K, keep, geo.ds, depth, validate, short_runs);
  if (!kern) {
    err = "no kernel for this configuration";
    return VCA_ERR_UNSUPPORTED;
  }
  // Persistent grid: at most as many workgroups as can be resident at once,
  // so no workgroup waits for another to drain before it starts its loop.
  int resident = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, kern, kGroupThreads, 0);
  if (e == hipSuccess) {
    resident = std::max(1, resident);
    if (groups_per_cu > 0) resident = std::min(resident, groups_per_cu);
    const int64_t waves = short_runs ? strips : (strips + kRun - 1) / kRun;
    const int64_t groups_needed = (waves + kWavesPerGroup - 1) / kWavesPerGroup;
    const int grid = (int)std::min<int64_t>(groups_needed, (int64_t)num_cus * resident);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kGroupThreads), 0, stream, fp);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    err = std::string("forward launch: ") + hipGetErrorString(e);
    return VCA_ERR_DEVICE;
  }
  return VCA_OK;
}

// The same for a context's configuration and stream.
vca_status launch_fwd(vca_ctx* ctx, const FwdParams& fp, int depth, int groups_per_cu,
                      bool allow_short = true, bool validate = true) {
  return enqueue_fwd(ctx->geo, ctx->num_cus, ctx->stream, fp, depth, groups_per_cu,
                     ctx->coeffs != nullptr, validate && (ctx->cfg.flags & VCA_F_VALIDATE) != 0,
                     allow_short, ctx->err);
}

std::string tune_key(int num_cus, const vca_config& cfg, const Geometry& geo) {
  char key[160];
  std::snprintf(key, sizeof(key), "gfx950/cu%d/plain/b%d/w%d/k%d%s/%dx%d", num_cus, cfg.bit_depth,
                cfg.block_size, geo.K, geo.ds ? "/ds" : "", cfg.width, cfg.height);
  return key;
}

std::string tune_key(const vca_ctx* ctx) { return tune_key(ctx->num_cus, ctx->cfg, ctx->geo); }

}  // namespace

extern "C" {

vca_status vca_block_counts(const vca_config* cfg, int32_t counts[3]) {
  if (!counts) return VCA_ERR_INVALID_ARG;
  vca_status s = check_config(cfg);
  if (s != VCA_OK) return s;
  Geometry g;
  g.init(*cfg);
  for (int P = 0; P < 3; P++) counts[P] = g.cnt[P];
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
    void* bufs[] = {ctx->tab_a2,   ctx->tab_b1p,  ctx->tab_wp,   ctx->blk_h,    ctx->blk_dc,
                    ctx->coeffs,   ctx->state[0], ctx->state[1], ctx->frame_err};
    for (void* b : bufs)
      if (b) (void)hipFree(b);
    if (ctx->ring_host) (void)hipHostFree(ctx->ring_host);
    if (ctx->err_ring_host) (void)hipHostFree(ctx->err_ring_host);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    ctx->done.destroy();
    if (ctx->copy_stream) (void)hipStreamSynchronize(ctx->copy_stream);
    for (auto& sl : ctx->ing) {
      if (sl.pinned) (void)hipHostFree(sl.pinned);
      if (sl.dev) (void)hipFree(sl.dev);
      if (sl.copied) (void)hipEventDestroy(sl.copied);
      if (sl.used) (void)hipEventDestroy(sl.used);
    }
    if (ctx->copy_stream) (void)hipStreamDestroy(ctx->copy_stream);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  }
  delete ctx;
}

vca_status vca_open(const vca_config* cfg, void* hip_stream, vca_ctx** out) {
  if (!out) return VCA_ERR_INVALID_ARG;
  *out = nullptr;
  vca_status s = check_config(cfg);
  if (s != VCA_OK) return s;
  // one launch's frames must not share ring slots
  if (effective(cfg->feature_capacity, kDefaultCapacity) < effective(cfg->max_batch, kDefaultMaxBatch))
    return VCA_ERR_INVALID_ARG;

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return VCA_ERR_DEVICE;
  if (cfg->device >= ndev) return VCA_ERR_INVALID_ARG;

  vca_ctx* c = new (std::nothrow) vca_ctx();
  if (!c) return VCA_ERR_OOM;
  c->cfg = *cfg;
  c->cfg.max_batch = effective(c->cfg.max_batch, kDefaultMaxBatch);
  c->cfg.feature_capacity = effective(c->cfg.feature_capacity, kDefaultCapacity);
  c->geo.init(*cfg);
  if ((int64_t)c->cfg.max_batch * c->geo.per_frame > (int64_t)INT32_MAX / 2) {
    delete c;
    return VCA_ERR_INVALID_ARG;   // block ids of one launch must fit int32
  }
  c->device = cfg->device;

  auto bail = [&](vca_status st) {
    vca_close(c);
    return st;
  };
  DeviceGuard guard(c->device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return bail(VCA_ERR_DEVICE);
  c->num_cus = prop.multiProcessorCount;
  if (const char* e = std::getenv("VCA_GROUPS_PER_CU")) c->env_groups_per_cu = std::atoi(e);
  if (hip_stream) {
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(VCA_ERR_DEVICE);
    c->own_stream = true;
  }
  if (c->done.init(1) != hipSuccess) return bail(VCA_ERR_DEVICE);
  const size_t mb = (size_t)c->cfg.max_batch;
  const int K = c->geo.K;
  if ((s = dev_alloc(c, &c->tab_a2, 64)) != VCA_OK) return bail(s);
  if ((s = dev_alloc(c, &c->tab_b1p, (size_t)(cfg->block_size / K) * 64)) != VCA_OK) return bail(s);
  if ((s = dev_alloc(c, &c->tab_wp, 16 * 64)) != VCA_OK) return bail(s);
  if ((s = dev_alloc(c, &c->blk_h, mb * c->geo.per_frame)) != VCA_OK) return bail(s);
  if ((s = dev_alloc(c, &c->blk_dc, mb * c->geo.per_frame)) != VCA_OK) return bail(s);
  if ((s = dev_alloc(c, &c->state[0], c->geo.cnt[0])) != VCA_OK) return bail(s);
  if ((s = dev_alloc(c, &c->state[1], c->geo.cnt[0])) != VCA_OK) return bail(s);
  if ((s = dev_alloc(c, &c->frame_err, mb)) != VCA_OK) return bail(s);
  if (hipMemset(c->frame_err, 0, mb * sizeof(int32_t)) != hipSuccess) return bail(VCA_ERR_DEVICE);
  if (host_mapped_alloc((size_t)c->cfg.feature_capacity * 7 * sizeof(float),
                        reinterpret_cast<void**>(&c->ring_host),
                        reinterpret_cast<void**>(&c->ring)) != hipSuccess ||
      host_mapped_alloc((size_t)c->cfg.feature_capacity * sizeof(int32_t),
                        reinterpret_cast<void**>(&c->err_ring_host),
                        reinterpret_cast<void**>(&c->err_ring)) != hipSuccess)
    return bail(VCA_ERR_OOM);
  if (cfg->flags & VCA_F_KEEP_COEFFS)
    if ((s = dev_alloc(c, &c->coeffs, mb * c->geo.per_frame * K * K)) != VCA_OK) return bail(s);

  std::vector<int8_t> b1, a2;
  std::vector<double> wt;
  build_tile_tables(cfg->block_size, K, b1, a2, wt);
  std::vector<int8_t> b1p;
  std::vector<double> wtp;
  build_packed_tables(cfg->block_size, K, b1p, wtp);
  if (hipMemcpy(c->tab_a2, a2.data(), a2.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->tab_b1p, b1p.data(), b1p.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->tab_wp, wtp.data(), wtp.size() * sizeof(double), hipMemcpyHostToDevice) !=
          hipSuccess)
    return bail(VCA_ERR_DEVICE);
  TuneCache::get().find(tune_key(c), &c->tuned);
  *out = c;
  return VCA_OK;
}

vca_status vca_reset(vca_ctx* ctx) {
  if (!ctx) return VCA_ERR_INVALID_ARG;
  ctx->has_prev = false;
  return VCA_OK;
}

}  // extern "C"

namespace {

// Enqueues the analysis of n_frames validated device frames.
vca_status analyze_device(vca_ctx* ctx, const vca_frames* fr, int32_t n_frames) {
  const vca_config& cfg = ctx->cfg;
  const double ww = (double)cfg.block_size * cfg.block_size;
  const int depth = ctx->tuned.depth > 0 ? ctx->tuned.depth : kDefaultDepth;
  const int gpc = ctx->env_groups_per_cu > 0 ? ctx->env_groups_per_cu : ctx->tuned.groups_per_cu;
  for (int32_t done = 0; done < n_frames;) {
    const int32_t n = std::min<int32_t>(cfg.max_batch, n_frames - done);
    const FwdParams fp = make_fwd_params(ctx, fr, done, n);
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
    vca_status s = launch_fwd(ctx, fp, depth, gpc);
    if (s != VCA_OK) return s;
    if (ev) HIP_TRY(ctx, hipEventRecord(ev[1], ctx->stream));

    ReduceParams rp{};
    rp.blk_h = ctx->blk_h;
    rp.blk_dc = ctx->blk_dc;
    rp.state_in = ctx->has_prev ? ctx->state[ctx->cur_state] : nullptr;
    rp.state_out = ctx->state[ctx->cur_state ^ 1];
    rp.ring = ctx->ring;
    rp.frame_err = (cfg.flags & VCA_F_VALIDATE) ? ctx->frame_err : nullptr;
    rp.err_ring = ctx->err_ring;
    rp.first_frame = ctx->submitted;
    rp.capacity = cfg.feature_capacity;
    for (int P = 0; P < 3; P++) {
      rp.cnt[P] = ctx->geo.cnt[P];
      rp.inv_norm[P] = 1.0 / ((double)ctx->geo.cnt[P] * ww);
    }
    rp.per_frame = ctx->geo.per_frame;
    rp.n_frames = n;
    hipLaunchKernelGGL(reduce_kernel, dim3(n), dim3(kReduceThreads), 0, ctx->stream, rp);
    HIP_TRY(ctx, hipGetLastError());
    if (ev) HIP_TRY(ctx, hipEventRecord(ev[2], ctx->stream));
    ctx->last_chunk_prev = ctx->has_prev;
    ctx->cur_state ^= 1;
    ctx->has_prev = true;
    ctx->last_chunk_first = ctx->submitted;
    ctx->last_chunk_len = n;
    ctx->submitted += n;
    HIP_TRY(ctx, ctx->done.record(ctx->stream, &ctx->submitted));
    done += n;
  }
  return VCA_OK;
}

// Staging layout of one ingest slot: planes of ing_batch frames, Y then U
// then V, rows padded to 16 bytes (the device path's alignment rule).
struct SlotLayout {
  int64_t pitch_y, pitch_uv, fstride_y, fstride_uv, off_u, off_v, bytes;
};

SlotLayout slot_layout(const vca_config& cfg, int32_t batch) {
  const YuvLayout L = YuvLayout::of(cfg.width, cfg.height, cfg.bit_depth);
  SlotLayout s;
  s.pitch_y = (L.row_y + 15) / 16 * 16;
  s.pitch_uv = (L.row_uv + 15) / 16 * 16;
  s.fstride_y = s.pitch_y * L.rows_y;
  s.fstride_uv = s.pitch_uv * L.rows_uv;
  s.off_u = s.fstride_y * batch;
  s.off_v = s.off_u + s.fstride_uv * batch;
  s.bytes = s.off_v + s.fstride_uv * batch;
  return s;
}

constexpr int64_t kIngestSlotBytes = 64ll << 20;   // target staging per slot

vca_status ingest_setup(vca_ctx* ctx) {
  if (ctx->copy_stream) return VCA_OK;
  const SlotLayout one = slot_layout(ctx->cfg, 1);
  ctx->ing_batch = (int32_t)std::max<int64_t>(
      1, std::min<int64_t>(kIngestSlotBytes / one.bytes, ctx->cfg.max_batch));
  const SlotLayout sl = slot_layout(ctx->cfg, ctx->ing_batch);
  for (auto& slot : ctx->ing) {
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&slot.pinned), (size_t)sl.bytes,
                                 hipHostMallocDefault);
    if (e != hipSuccess) return fail(ctx, VCA_ERR_OOM, "hipHostMalloc: staging buffer");
    vca_status s = dev_alloc(ctx, &slot.dev, (size_t)sl.bytes);
    if (s != VCA_OK) return s;
    HIP_TRY(ctx, hipEventCreateWithFlags(&slot.copied, hipEventDisableTiming));
    HIP_TRY(ctx, hipEventCreateWithFlags(&slot.used, hipEventDisableTiming));
  }
  ctx->pool.reset(new WorkerPool(ingest_threads()));
  HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking));
  return VCA_OK;
}

// Analyses n_frames frames that `fill` writes into host memory: fill(first,
// count, dst, part, parts) writes part `part` of `parts` of frames [first,
// first + count) of the run.  Double-buffered: while the device copies slot
// s and analyses the other slot's frames, the pool fills the next batch.
template <class Fill>
vca_status analyze_staged(vca_ctx* ctx, int32_t n_frames, Fill fill) {
  vca_status st = ingest_setup(ctx);
  if (st != VCA_OK) return st;
  const SlotLayout sl = slot_layout(ctx->cfg, ctx->ing_batch);
  for (int32_t done = 0; done < n_frames;) {
    const int32_t b = std::min(ctx->ing_batch, n_frames - done);
    vca_ctx::IngestSlot& slot = ctx->ing[ctx->ing_next];
    ctx->ing_next ^= 1;
    // the pinned buffer is free once its previous copy has finished
    if (slot.busy) HIP_TRY(ctx, hipEventSynchronize(slot.copied));
    const PlanarDst dst{slot.pinned, slot.pinned + sl.off_u, slot.pinned + sl.off_v,
                        sl.pitch_y,  sl.pitch_uv,            sl.fstride_y,
                        sl.fstride_uv};
    std::atomic<bool> ok{true};
    const int parts = ctx->pool->size();
    ctx->pool->run([&](int part) {
      if (!fill(done, b, dst, part, parts)) ok = false;
    });
    if (!ok) return fail(ctx, VCA_ERR_INVALID_ARG, "reading the frames failed");
    // the device buffer is free once the analysis of its previous batch is done
    if (slot.busy) HIP_TRY(ctx, hipStreamWaitEvent(ctx->copy_stream, slot.used, 0));
    // copy the used part of each plane region
    HIP_TRY(ctx, hipMemcpyAsync(slot.dev, slot.pinned, (size_t)(sl.fstride_y * b),
                                hipMemcpyHostToDevice, ctx->copy_stream));
    HIP_TRY(ctx, hipMemcpyAsync(slot.dev + sl.off_u, slot.pinned + sl.off_u,
                                (size_t)(sl.fstride_uv * b), hipMemcpyHostToDevice, ctx->copy_stream));
    HIP_TRY(ctx, hipMemcpyAsync(slot.dev + sl.off_v, slot.pinned + sl.off_v,
                                (size_t)(sl.fstride_uv * b), hipMemcpyHostToDevice, ctx->copy_stream));
    HIP_TRY(ctx, hipEventRecord(slot.copied, ctx->copy_stream));
    HIP_TRY(ctx, hipStreamWaitEvent(ctx->stream, slot.copied, 0));
    vca_frames df{};
    df.y = slot.dev;
    df.u = slot.dev + sl.off_u;
    df.v = slot.dev + sl.off_v;
    df.pitch_y = sl.pitch_y;
    df.pitch_uv = sl.pitch_uv;
    df.fstride_y = sl.fstride_y;
    df.fstride_uv = sl.fstride_uv;
    df.on_device = 1;
    st = analyze_device(ctx, &df, b);
    if (st != VCA_OK) return st;
    HIP_TRY(ctx, hipEventRecord(slot.used, ctx->stream));
    slot.busy = true;
    done += b;
  }
  return VCA_OK;
}

}  // namespace

extern "C" {

vca_status vca_analyze_frames(vca_ctx* ctx, const vca_frames* fr, int32_t n_frames) {
  if (!ctx || !fr || n_frames < 0) return fail(ctx, VCA_ERR_INVALID_ARG, "null argument or n < 0");
  if (n_frames == 0) return VCA_OK;
  const vca_config& cfg = ctx->cfg;
  if ((cfg.flags & VCA_F_KEEP_COEFFS) && n_frames > cfg.max_batch)
    return fail(ctx, VCA_ERR_INVALID_ARG, "VCA_F_KEEP_COEFFS: n_frames exceeds max_batch");
  DeviceGuard guard(ctx->device);
  if (fr->on_device) {
    if (const char* msg = check_frames(cfg, fr, n_frames)) return fail(ctx, VCA_ERR_INVALID_ARG, msg);
    return analyze_device(ctx, fr, n_frames);
  }
  if (const char* msg = check_host_frames(cfg, fr, n_frames)) return fail(ctx, VCA_ERR_INVALID_ARG, msg);
  if ((cfg.flags & VCA_F_KEEP_COEFFS) && n_frames > 0)
    return fail(ctx, VCA_ERR_UNSUPPORTED, "VCA_F_KEEP_COEFFS with host-resident frames");
  const YuvLayout L = YuvLayout::of(cfg.width, cfg.height, cfg.bit_depth);
  const vca_frames src = *fr;
  return analyze_staged(ctx, n_frames, [&](int32_t first, int32_t b, const PlanarDst& d, int part,
                                           int parts) {
    int64_t y0, y1, c0, c1;
    band(L.rows_y, part, parts, y0, y1);
    band(L.rows_uv, part, parts, c0, c1);
    for (int32_t i = 0; i < b; i++) {
      const int64_t f = first + i;
      copy_rows(d.y + i * d.fstride_y, d.pitch_y,
                static_cast<const uint8_t*>(src.y) + f * src.fstride_y, src.pitch_y, L.row_y, y0, y1);
      copy_rows(d.u + i * d.fstride_uv, d.pitch_uv,
                static_cast<const uint8_t*>(src.u) + f * src.fstride_uv, src.pitch_uv, L.row_uv, c0, c1);
      copy_rows(d.v + i * d.fstride_uv, d.pitch_uv,
                static_cast<const uint8_t*>(src.v) + f * src.fstride_uv, src.pitch_uv, L.row_uv, c0, c1);
    }
    return true;
  });
}

vca_status vca_analyze_yuv_file(vca_ctx* ctx, const char* path, int64_t first_frame,
                                int32_t n_frames) {
  if (!ctx || !path || first_frame < 0 || n_frames < 0)
    return fail(ctx, VCA_ERR_INVALID_ARG, "null argument or negative frame range");
  if (n_frames == 0) return VCA_OK;
  const vca_config& cfg = ctx->cfg;
  if (cfg.flags & VCA_F_KEEP_COEFFS)
    return fail(ctx, VCA_ERR_UNSUPPORTED, "VCA_F_KEEP_COEFFS with host-resident frames");
  const YuvLayout L = YuvLayout::of(cfg.width, cfg.height, cfg.bit_depth);
  const int64_t avail = yuv_frames_in_file(path, L);
  if (avail < 0) return fail(ctx, VCA_ERR_INVALID_ARG, std::string("cannot open ") + path);
  if (first_frame + n_frames > avail)
    return fail(ctx, VCA_ERR_INVALID_ARG, "the file holds fewer frames than requested");
  const int fd = ::open(path, O_RDONLY);
  if (fd < 0) return fail(ctx, VCA_ERR_INVALID_ARG, std::string("cannot open ") + path);
  DeviceGuard guard(ctx->device);
  const vca_status st = analyze_staged(
      ctx, n_frames, [&](int32_t first, int32_t b, const PlanarDst& d, int part, int parts) {
        return read_yuv_part(fd, L, first_frame + first, b, d, part, parts);
      });
  ::close(fd);
  return st;
}

vca_status vca_read_yuv(const char* path, int32_t width, int32_t height, int32_t bit_depth,
                        int64_t first_frame, int32_t n_frames, void* y, void* u, void* v) {
  if (!path || !y || !u || !v || first_frame < 0 || n_frames < 0) return VCA_ERR_INVALID_ARG;
  if (width <= 0 || height <= 0 || (width & 1) || (height & 1) || (bit_depth != 8 && bit_depth != 10))
    return VCA_ERR_INVALID_ARG;
  const YuvLayout L = YuvLayout::of(width, height, bit_depth);
  const int64_t avail = yuv_frames_in_file(path, L);
  if (avail < 0 || first_frame + n_frames > avail) return VCA_ERR_INVALID_ARG;
  const int fd = ::open(path, O_RDONLY);
  if (fd < 0) return VCA_ERR_INVALID_ARG;
  const PlanarDst d{static_cast<uint8_t*>(y), static_cast<uint8_t*>(u), static_cast<uint8_t*>(v),
                    L.row_y, L.row_uv, L.plane_y, L.plane_uv};
  const bool ok = read_yuv_part(fd, L, first_frame, n_frames, d, 0, 1);
  ::close(fd);
  return ok ? VCA_OK : VCA_ERR_INVALID_ARG;
}

vca_status vca_tune(vca_ctx* ctx, const vca_frames* fr, int32_t n_frames, int32_t reps) {
  if (!ctx || !fr || n_frames <= 0 || reps <= 0)
    return fail(ctx, VCA_ERR_INVALID_ARG, "bad vca_tune arguments");
  if (!fr->on_device) return fail(ctx, VCA_ERR_UNSUPPORTED, "host-resident frames");
  if (const char* msg = check_frames(ctx->cfg, fr, n_frames)) return fail(ctx, VCA_ERR_INVALID_ARG, msg);
  if (ctx->coeffs) return fail(ctx, VCA_ERR_STATE, "contexts with VCA_F_KEEP_COEFFS are not tuned");
  DeviceGuard guard(ctx->device);
  const int32_t n = std::min<int32_t>(n_frames, ctx->cfg.max_batch);
  const FwdParams fp = make_fwd_params(ctx, fr, 0, n);
  hipEvent_t a, b;
  HIP_TRY(ctx, hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(ctx, VCA_ERR_DEVICE, "hipEventCreate");
  }
  LaunchChoice best;
  best.ms = 1e30;
  vca_status st = VCA_OK;
  // the tuning launches overwrite the per-block results of the last call
  ctx->last_chunk_len = 0;
  for (int depth = 1; depth <= 4 && st == VCA_OK; depth *= 2) {
    int resident = 0;
    FwdKernel kern =
        select_fwd_kernel(ctx->cfg.bit_depth, ctx->cfg.block_size, ctx->geo.K, false, ctx->geo.ds, depth,
                          false);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, kern, kGroupThreads, 0) != hipSuccess)
      resident = 1;
    for (int gpc = 1; gpc <= std::max(1, resident) && st == VCA_OK; gpc++) {
      // the non-validating kernel: tuning frames leave no validation marks
      st = launch_fwd(ctx, fp, depth, gpc, false, false);   // warm-up
      if (st != VCA_OK) break;
      if (hipEventRecord(a, ctx->stream) != hipSuccess) {
        st = fail(ctx, VCA_ERR_DEVICE, "hipEventRecord");
        break;
      }
      for (int r = 0; r < reps && st == VCA_OK; r++) st = launch_fwd(ctx, fp, depth, gpc, false, false);
      if (st != VCA_OK) break;
      if (hipEventRecord(b, ctx->stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess) {
        st = fail(ctx, VCA_ERR_DEVICE, "hipEventRecord/Synchronize");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, a, b);
      ms /= reps;
      if (ms < best.ms) best = LaunchChoice{depth, gpc, ms};
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != VCA_OK) return st;
  ctx->tuned = best;
  TuneCache::get().put(tune_key(ctx), best);
  return VCA_OK;
}

vca_status vca_tuned_launch(const vca_ctx* ctx, int32_t* depth, int32_t* groups_per_cu, double* ms) {
  if (!ctx) return VCA_ERR_INVALID_ARG;
  if (depth) *depth = ctx->tuned.depth;
  if (groups_per_cu) *groups_per_cu = ctx->tuned.groups_per_cu;
  if (ms) *ms = ctx->tuned.ms;
  return VCA_OK;
}

vca_status vca_features(vca_ctx* ctx, int64_t first, int32_t count, vca_frame_features* out) {
  if (!ctx || count < 0 || first < 0 || (count > 0 && !out))
    return fail(ctx, VCA_ERR_INVALID_ARG, "bad vca_features arguments");
  if (first + count > ctx->submitted) return fail(ctx, VCA_ERR_STATE, "frame not yet submitted");
  const int64_t cap = ctx->cfg.feature_capacity;
  if (first < ctx->submitted - cap) return fail(ctx, VCA_ERR_STATE, "frame left the feature ring");
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, ctx->done.wait(0, first + count, ctx->stream));
  // the rings are host memory the kernels wrote before the launch that
  // produced the last frame asked for completed (later launches may still
  // run: they write other ring slots)
  if (ctx->cfg.flags & VCA_F_VALIDATE) {
    const volatile int32_t* marks = ctx->err_ring_host;
    for (int64_t f = first; f < first + count; f++)
      if (marks[f % cap])
        return fail(ctx, VCA_ERR_STATE,
                    "frame " + std::to_string(f) + " holds a 10-bit sample above 1023");
  }
  int64_t done = 0;
  while (done < count) {
    const int64_t slot = (first + done) % cap;
    const int64_t n = std::min<int64_t>(count - done, cap - slot);
    std::memcpy(reinterpret_cast<float*>(out) + done * 7, ctx->ring_host + slot * 7,
                (size_t)n * 7 * sizeof(float));
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
  const size_t per = (size_t)ctx->geo.per_frame * ctx->geo.K * ctx->geo.K;
  if (capacity < per) return fail(ctx, VCA_ERR_INVALID_ARG, "output buffer too small");
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  HIP_TRY(ctx, hipMemcpy(out, ctx->coeffs + (frame - ctx->last_chunk_first) * per,
                         per * sizeof(int16_t), hipMemcpyDeviceToHost));
  return VCA_OK;
}

vca_status vca_block_maps(vca_ctx* ctx, int64_t first_frame, int32_t count, double* h_dev,
                          int32_t* dc_dev, double* dh_dev) {
  if (!ctx || count <= 0 || (!h_dev && !dc_dev && !dh_dev))
    return fail(ctx, VCA_ERR_INVALID_ARG, "null context, count <= 0 or no output");
  if (first_frame < ctx->last_chunk_first ||
      first_frame + count > ctx->last_chunk_first + ctx->last_chunk_len)
    return fail(ctx, VCA_ERR_STATE, "frames not in the most recent launch");
  if (((uintptr_t)h_dev | (uintptr_t)dh_dev | (uintptr_t)dc_dev) & 7)
    return fail(ctx, VCA_ERR_INVALID_ARG, "outputs must be 8-byte aligned");
  DeviceGuard guard(ctx->device);
  MapsParams mp{};
  mp.blk_h = ctx->blk_h;
  mp.blk_dc = ctx->blk_dc;
  // the launch's reduction read the previous frame's luma H from the state
  // buffer it did not write, which the next launch has not touched yet
  mp.prev = ctx->last_chunk_prev ? ctx->state[ctx->cur_state ^ 1] : nullptr;
  mp.h_out = h_dev;
  mp.dc_out = dc_dev;
  mp.dh_out = dh_dev;
  mp.per_frame = ctx->geo.per_frame;
  mp.cnt_y = ctx->geo.cnt[0];
  mp.f0 = first_frame - ctx->last_chunk_first;
  mp.count = count;
  const int gx = (int)std::min<int64_t>((mp.per_frame + kMapsThreads - 1) / kMapsThreads, 64);
  hipLaunchKernelGGL(block_maps_kernel, dim3(gx, count), dim3(kMapsThreads), 0, ctx->stream, mp);
  HIP_TRY(ctx, hipGetLastError());
  return VCA_OK;
}

vca_status vca_block_stats(vca_ctx* ctx, int64_t frame, double* h_out, int32_t* dc_out,
                           size_t capacity) {
  if (!ctx || (!h_out && !dc_out)) return fail(ctx, VCA_ERR_INVALID_ARG, "null argument");
  if (frame < ctx->last_chunk_first || frame >= ctx->last_chunk_first + ctx->last_chunk_len)
    return fail(ctx, VCA_ERR_STATE, "frame not in the most recent launch");
  const int32_t per = ctx->geo.per_frame;
  if (capacity < (size_t)per) return fail(ctx, VCA_ERR_INVALID_ARG, "output buffer too small");
  DeviceGuard guard(ctx->device);
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  const int64_t off = (frame - ctx->last_chunk_first) * per;
  if (h_out)
    HIP_TRY(ctx, hipMemcpy(h_out, ctx->blk_h + off, per * sizeof(double), hipMemcpyDeviceToHost));
  if (dc_out)
    HIP_TRY(ctx, hipMemcpy(dc_out, ctx->blk_dc + off, per * sizeof(int32_t), hipMemcpyDeviceToHost));
  return VCA_OK;
}

}  // extern "C"

// ====================================================== allocation-free form
// vca_analyze_noalloc runs the plain path's kernels with every buffer they
// need beyond the caller's frames and feature output placed in `scratch`, a
// fixed array each device holds while the process runs:
//   [0, kNaTablesBytes)  operand and weight tables of the nine (w, K)
//                        classes, kNaClassBytes apart, uploaded once per
//                        device on its first call;
//   then                 per-launch block energies (FP64) and DC (int32) of
//                        up to n_max frames, and two luma-H state buffers
//                        (the previous launch's last frame for h).
// Host code reaches the array only through the address hipGetSymbolAddress
// returned for the current device.
namespace {

constexpr size_t kNaScratchBytes = 32ull << 20;
constexpr size_t kNaClassBytes = 16 << 10;           // a2 1 KiB + b1p <= 4 KiB + weights 8 KiB
constexpr size_t kNaTablesBytes = 9 * kNaClassBytes;
constexpr int kNaMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kNaScratchBytes];

struct NaDevice {
  uint8_t* ptr = nullptr;   // this device's copy of `scratch`
  int num_cus = 0;
};

std::mutex na_mu;
NaDevice na_dev[kNaMaxDevices];

int na_class(int w, int K) { return 3 * (w == 8 ? 0 : (w == 16 ? 1 : 2)) + (K == w ? 0 : (K == w / 2 ? 1 : 2)); }

// Once per device, with that device current: the array's device address,
// then the tables of every class (synchronous copies; nothing is allocated).
vca_status na_setup(int device, NaDevice* out, std::string& err) {
  std::lock_guard<std::mutex> lk(na_mu);
  NaDevice& d = na_dev[device];
  if (!d.ptr) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return VCA_ERR_DEVICE;
    }
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    for (int w = 8; w <= 32 && e == hipSuccess; w *= 2) {
      for (int K = w; K >= w / 4 && e == hipSuccess; K /= 2) {
        std::vector<int8_t> b1, a2, b1p;
        std::vector<double> wt, wtp;
        build_tile_tables(w, K, b1, a2, wt);
        build_packed_tables(w, K, b1p, wtp);
        uint8_t* base = static_cast<uint8_t*>(ptr) + na_class(w, K) * kNaClassBytes;
        e = hipMemcpy(base, a2.data(), a2.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(base + 1024, b1p.data(), b1p.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
          e = hipMemcpy(base + 5120, wtp.data(), wtp.size() * sizeof(double), hipMemcpyHostToDevice);
      }
    }
    if (e != hipSuccess) {
      err = std::string("scratch set-up: ") + hipGetErrorString(e);
      return VCA_ERR_DEVICE;
    }
    d.num_cus = cus;
    d.ptr = static_cast<uint8_t*>(ptr);
  }
  *out = d;
  return VCA_OK;
}

}  // namespace

extern "C" {

vca_status vca_analyze_noalloc(const vca_config* cfg, const vca_frames* fr, int32_t n_frames,
                               float* features_dev, void* hip_stream) {
  vca_status s = check_config(cfg);
  if (s != VCA_OK) return s;
  if (!fr || n_frames < 0 || (n_frames > 0 && !features_dev) || ((uintptr_t)features_dev & 3))
    return VCA_ERR_INVALID_ARG;
  if (cfg->flags & (VCA_F_KEEP_COEFFS | VCA_F_VALIDATE | VCA_F_TIMING)) return VCA_ERR_UNSUPPORTED;
  if (cfg->device >= kNaMaxDevices) return VCA_ERR_UNSUPPORTED;
  Geometry geo;
  geo.init(*cfg);
  // frames per launch that fit beside the tables and the two state buffers
  const size_t state_bytes = (size_t)geo.cnt[0] * sizeof(double);
  const size_t per_frame_bytes = (size_t)geo.per_frame * (sizeof(double) + sizeof(int32_t));
  const size_t avail = kNaScratchBytes - kNaTablesBytes - 2 * ((state_bytes + 255) / 256 * 256);
  const int64_t n_max = (int64_t)(avail / (per_frame_bytes + 256));
  if (n_max < 1) return VCA_ERR_UNSUPPORTED;   // one frame's block results exceed the array
  if (n_frames == 0) return VCA_OK;
  if (fr->on_device != 1) return VCA_ERR_INVALID_ARG;
  if (check_frames(*cfg, fr, n_frames)) return VCA_ERR_INVALID_ARG;

  DeviceGuard guard(cfg->device);
  std::string na_err;   // stays empty (no allocation) unless a HIP call fails
  NaDevice dev;
  if ((s = na_setup(cfg->device, &dev, na_err)) != VCA_OK) return s;
  uint8_t* tab = dev.ptr + na_class(geo.w, geo.K) * kNaClassBytes;
  uint8_t* cur = dev.ptr + kNaTablesBytes;
  double* state[2];
  state[0] = reinterpret_cast<double*>(cur);
  cur += (state_bytes + 255) / 256 * 256;
  state[1] = reinterpret_cast<double*>(cur);
  cur += (state_bytes + 255) / 256 * 256;
  const int32_t n_launch = (int32_t)std::min<int64_t>(n_max, n_frames);
  double* blk_h = reinterpret_cast<double*>(cur);
  int32_t* blk_dc = reinterpret_cast<int32_t*>(cur + ((size_t)n_launch * geo.per_frame * sizeof(double) + 255) / 256 * 256);

  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  LaunchChoice tuned;
  TuneCache::get().find(tune_key(dev.num_cus, *cfg, geo), &tuned);
  const int depth = tuned.depth > 0 ? tuned.depth : kDefaultDepth;
  const double ww = (double)cfg->block_size * cfg->block_size;
  int cur_state = 0;
  for (int32_t done = 0; done < n_frames;) {
    const int32_t n = std::min<int32_t>(n_launch, n_frames - done);
    FwdParams fp{};
    const uint8_t* first[3] = {static_cast<const uint8_t*>(fr->y) + fr->fstride_y * done,
                               static_cast<const uint8_t*>(fr->u) + fr->fstride_uv * done,
                               static_cast<const uint8_t*>(fr->v) + fr->fstride_uv * done};
    const int64_t fs[3] = {fr->fstride_y, fr->fstride_uv, fr->fstride_uv};
    const int64_t pt[3] = {fr->pitch_y, fr->pitch_uv, fr->pitch_uv};
    fp.geom = make_strip_geom(geo, first, fs, pt, 0);
    fp.n_frames = n;
    fp.tab_a2 = reinterpret_cast<const v4i*>(tab);
    fp.tab_b1p = reinterpret_cast<const v4i*>(tab + 1024);
    fp.tab_wp = reinterpret_cast<const double*>(tab + 5120);
    fp.out.blk_h = blk_h;
    fp.out.blk_dc = blk_dc;
    if ((s = enqueue_fwd(geo, dev.num_cus, stream, fp, depth, tuned.groups_per_cu, false, false, true,
                         na_err)) != VCA_OK)
      return s;
    ReduceParams rp{};
    rp.blk_h = blk_h;
    rp.blk_dc = blk_dc;
    rp.state_in = done > 0 ? state[cur_state] : nullptr;   // h = 0 for the call's first frame
    rp.state_out = state[cur_state ^ 1];
    rp.ring = features_dev;
    rp.first_frame = done;
    rp.capacity = n_frames;
    for (int P = 0; P < 3; P++) {
      rp.cnt[P] = geo.cnt[P];
      rp.inv_norm[P] = 1.0 / ((double)geo.cnt[P] * ww);
    }
    rp.per_frame = geo.per_frame;
    rp.n_frames = n;
    hipLaunchKernelGGL(reduce_kernel, dim3(n), dim3(kReduceThreads), 0, stream, rp);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      na_err = std::string("reduce launch: ") + hipGetErrorString(e);
      return VCA_ERR_DEVICE;
    }
    cur_state ^= 1;
    done += n;
  }
  return VCA_OK;
}

}  // extern "C"
