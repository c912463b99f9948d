// vca_batch.hip -- batched form of the VCA forward path (gfx950).
//
// Many independent video streams of different resolution, block size, bit
// depth and frame count are analysed in one round of launches: the streams
// are grouped by class (bit depth, w, K), and each class present gets ONE
// persistent launch of a kernel specialised for it (its own register budget;
// ring depth, wavefronts per workgroup, workgroups per CU and strips per
// chunk chosen by vca_tune_batch).  Its wavefronts take chunks of the class's
// flat list (runs of consecutive strips of one stream, vca_strip.h; a
// stream's chunks are contiguous) from the class's device counter, so that
// waves that drew cheap chunks take more and all finish together, and run
// the plain path's strip loop.  After a class's forward launch, a reduction
// launch turns each of the class's (stream, frame) pairs into its seven
// features (vca_reduce.h).  The classes run one after another or side by
// side on forked streams (the tuned arrangement).  A round's launches are
// captured once into a hipGraph per signature and replayed; per call only
// the descriptor tables (frame pointers, state buffers) are uploaded.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/vca.h"
#include "vca_host.h"
#include "vca_reduce.h"
#include "vca_strip.h"
#include "vca_tile.h"

using namespace vca;

namespace {

constexpr int kDefaultWaves = 4;   // wavefronts per workgroup of a class launch (or 8)
constexpr int kKinds = 18;          // bit depth {8, 10} x w {32, 16, 8} x K {w, w/2, w/4}
constexpr int32_t kDefaultMaxBatch = 300;    // frames per stream and round (max_batch = 0)
constexpr int32_t kDefaultCapacity = 4096;   // feature ring per stream (feature_capacity = 0)

inline int kind_of(int bits, int w, int K) {
  const int wi = w == 32 ? 0 : (w == 16 ? 1 : 2);
  const int ki = K == w ? 0 : (K == w / 2 ? 1 : 2);
  return ((bits == 10 ? 1 : 0) * 3 + wi) * 3 + ki;
}

// Device-side description of one stream for one launch.
struct StreamDesc {
  StripGeom geom;                  // the stream's frames of this launch as strips
  int32_t kind;
  int32_t strips;                  // strips of the stream in this launch
  int32_t chunk_begin, chunk_end;  // the stream's chunks in the launch's flat list
  int32_t validate;
  int32_t stream;                  // index of the stream
};

using ConstDesc = __attribute__((address_space(4))) const StreamDesc;

// Consecutive strips of one stream handed to a wavefront at a time (a
// multiple of kRun, so chunks start on a run boundary): 32 unless tuned to
// one of kChunkChoices.
constexpr int kDefaultChunk = 32;
constexpr int kChunkChoices[] = {8, 16, 32, 64};
constexpr int kMaxPack = 4;        // w / K at most

// Descriptors and chunks of one class, ranges in the launch's flat lists
// (ordered by class, then stream).
struct KindRange {
  int32_t desc_begin, desc_end;
  int32_t chunk_begin, chunk_end;
  int32_t chunk_strips;   // strips per chunk
};

struct BatchParams {
  const StreamDesc* streams;   // in flat order (by class, then stream)
  KindRange kr;                // the class's descriptors and chunks
  const v4i* tab_b1p;    // the class's packed stage-1 operands [kMaxPack][64]
  const v4i* tab_a2;     // [64]
  const double* tab_wp;  // [16][64] packed-layout weights
  double* blk_h;
  int32_t* blk_dc;
  int32_t* err_flag;      // per frame of the round (StripGeom::frame_base + frame):
                          // a validated 10-bit sample above 1023
  int32_t* queue;         // the class's next chunk (relative to kr.chunk_begin); zero at launch
};

struct BatchReduceParams {
  const ReduceParams* red;    // the class's streams; red[s].frame_begin = first workgroup of s
  int32_t n_streams;
};

// The next chunk of the class for the calling wavefront (one atomic per
// wavefront, result broadcast).  Chunks are handed out in increasing order.
__device__ __forceinline__ int next_chunk(int32_t* queue, int lane) {
  int c = 0;
  if (lane == 0) c = __hip_atomic_fetch_add(queue, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_amdgcn_readfirstlane(c);
}

// Persistent kernel of one class: every wavefront draws the class's chunks
// until its list is exhausted.  The class's descriptors are contiguous and a
// wavefront's chunks only grow, so its stream search only moves forward.
template <int kBits, int kW, int kK, int kDepth, int kWaves>
__global__ __launch_bounds__(64 * kWaves) void batch_class_kernel(BatchParams p) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int kStage = stage_bytes(kW);
  __shared__ __attribute__((aligned(16))) uint8_t stage_mem[kWaves][kStage];
  TileOut o;
  o.blk_h = p.blk_h;
  o.blk_dc = p.blk_dc;
  o.coeffs = nullptr;
  o.err_flag = p.err_flag;
  o.validate = 0;
  PackConsts<kW, kK> pc;
  pc.load(p.tab_b1p, p.tab_a2, p.tab_wp, lane);
  // The descriptors stay unchanged while the launch runs: reading them
  // through the constant address space gives scalar loads, as for a kernel
  // argument, where generic loads would be vector loads whose wait also
  // drains the tile prefetch ring.
  const ConstDesc* streams = (const ConstDesc*)p.streams;
  int d = p.kr.desc_begin;
  for (int c = p.kr.chunk_begin + next_chunk(p.queue, lane); c < p.kr.chunk_end;
       c = p.kr.chunk_begin + next_chunk(p.queue, lane)) {
    while (d < p.kr.desc_end - 1 && c >= streams[d].chunk_end) d++;
    o.validate = streams[d].validate;
    const int s0 = (c - streams[d].chunk_begin) * p.kr.chunk_strips;
    const int s1 = min(s0 + p.kr.chunk_strips, streams[d].strips);
    run_strips<kBits, kW, kK, kDepth, false, (kBits != 8)>(
        *(const StripGeom*)&streams[d].geom, o, pc, s0 / kRun, 1, s1, lane,
        stage_mem[wave]);
  }
}

// Zeroes the classes' chunk counters ahead of the forward launches (a kernel
// node rather than a memset, so the captured graph holds kernels only).
__global__ void queue_reset_kernel(int32_t* queue) {
  if (threadIdx.x < kKinds) queue[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kReduceThreads) void batch_reduce_kernel(BatchReduceParams p) {
  // stream of this workgroup: the last s with red[s].frame_begin <= blockIdx.x
  int lo = 0, hi = p.n_streams - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (p.red[mid].frame_begin <= b) lo = mid;
    else hi = mid - 1;
  }
  reduce_frame(p.red[lo], b - p.red[lo].frame_begin);
}

using BatchKernel = void (*)(BatchParams);

template <int B, int W, int K, int V>
BatchKernel pick_class_depth(int depth) {
  if (depth == 1) return batch_class_kernel<B, W, K, 1, V>;
  if (depth >= 4) return batch_class_kernel<B, W, K, 4, V>;
  return batch_class_kernel<B, W, K, 2, V>;
}

template <int B, int W, int K>
BatchKernel pick_class_waves(int depth, int waves) {
  return waves == 8 ? pick_class_depth<B, W, K, 8>(depth) : pick_class_depth<B, W, K, 4>(depth);
}

template <int B, int W>
BatchKernel pick_class_k(int ki, int depth, int waves) {
  if (ki == 0) return pick_class_waves<B, W, W>(depth, waves);
  if (ki == 1) return pick_class_waves<B, W, W / 2>(depth, waves);
  return pick_class_waves<B, W, W / 4>(depth, waves);
}

template <int B>
BatchKernel pick_class_w(int wi, int ki, int depth, int waves) {
  if (wi == 0) return pick_class_k<B, 32>(ki, depth, waves);
  if (wi == 1) return pick_class_k<B, 16>(ki, depth, waves);
  return pick_class_k<B, 8>(ki, depth, waves);
}

// Kernel of class `kind` (kind_of numbering) with the given ring depth and
// wavefronts per workgroup (4 or 8).
BatchKernel class_kernel_for(int kind, int depth, int waves) {
  const int ki = kind % 3, wi = (kind / 3) % 3;
  return kind < 9 ? pick_class_w<8>(wi, ki, depth, waves) : pick_class_w<10>(wi, ki, depth, waves);
}

}  // namespace

struct vca_batch {
  int n = 0;
  std::vector<vca_config> cfgs;
  std::vector<Geometry> geos;
  int device = 0;
  int num_cus = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t capture = nullptr;   // private stream the graph is captured on
  // tables for every kind
  v4i* tab_b1p = nullptr;
  v4i* tab_a2 = nullptr;
  double* tab_wp = nullptr;
  // per-stream device state
  double* blk_h = nullptr;
  int32_t* blk_dc = nullptr;
  std::vector<int64_t> blk_base;   // per stream, into blk_h / blk_dc
  double* state = nullptr;
  std::vector<int64_t> state_off;  // per stream: two buffers of C_Y doubles
  float* rings = nullptr;          // device view of rings_host
  float* rings_host = nullptr;     // pinned, mapped
  std::vector<int64_t> ring_off;   // per stream, in floats
  int32_t* frame_err = nullptr;    // per frame of a round: validation marks (device)
  int32_t* err_rings = nullptr;    // device view of err_rings_host
  int32_t* err_rings_host = nullptr;   // pinned, mapped: per stream [feature_capacity] marks
  int32_t* queue = nullptr;        // [kKinds] chunk counters of the forward launches
  std::vector<int> cur_state;
  std::vector<char> has_prev;
  std::vector<int64_t> submitted;
  DoneMarks done;                  // completion of the recent rounds
  // descriptors (device + pinned staging)
  StreamDesc* d_streams = nullptr;
  ReduceParams* d_red = nullptr;
  StreamDesc* h_streams = nullptr;
  ReduceParams* h_red = nullptr;
  hipEvent_t uploaded = nullptr;   // staging buffers reusable once this completes
  bool upload_pending = false;
  // executable graphs of the launch signatures met so far (frames per stream,
  // per-class launch shapes, arrangement), up to kMaxGraphs
  struct CachedGraph {
    std::vector<int32_t> sig;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<CachedGraph> graphs;
  bool use_graph = true;
  KindRange kinds[kKinds] = {};    // flat-list ranges of the current round
  int32_t kind_frames[kKinds] = {};   // frames of each class in the current round
  int64_t kind_blocks[kKinds] = {};   // blocks of each class in the current round
  hipStream_t branch[kKinds] = {};    // one per class launched, forked from the launch stream
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kKinds] = {};
  hipEvent_t fwd_ev[kKinds] = {};     // serial arrangement: class j's forward launch done
  int serial = 1;                     // classes one after another (1) or side by side (0)
  double serial_ms = 0.0, parallel_ms = 0.0;   // tuned whole rounds of either arrangement
  LaunchChoice kind_tuned[kKinds];    // per class: ring depth, workgroups per CU, ms
  LaunchChoice tuned;                 // summary: the most expensive class's shape, total ms
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int64_t> ev_frames;
  size_t ev_used = 0;
  std::string err;
};

namespace {

vca_status bfail(vca_batch* b, vca_status s, const std::string& msg) {
  if (b) b->err = msg;
  return s;
}

#define BHIP_TRY(b, expr)                                                        \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess)                                                        \
      return bfail((b), VCA_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
vca_status balloc(vca_batch* b, T** p, size_t count) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
  if (e == hipErrorOutOfMemory) return bfail(b, VCA_ERR_OOM, "hipMalloc: out of device memory");
  if (e != hipSuccess) return bfail(b, VCA_ERR_DEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
  return VCA_OK;
}

// Executable graphs a batch keeps.  None is destroyed before the batch is
// closed: destroying a cached graph and then capturing another crashed the
// host inside the HIP runtime (both with the graph's launch possibly still
// pending and after draining the stream), so a round whose signature finds
// the cache full runs its launches eagerly, in line on the batch's stream.
constexpr size_t kMaxGraphs = 16;

// Destroys every cached graph (at close, once the batch's stream has
// drained).
void drop_graphs(vca_batch* b) {
  for (auto& c : b->graphs) {
    if (c.exec) (void)hipGraphExecDestroy(c.exec);
    if (c.graph) (void)hipGraphDestroy(c.graph);
  }
  b->graphs.clear();
}

// Launch shape of class k: tuned, else ring depth 2, 4 wavefronts per
// workgroup, as many workgroups per CU as fit and 32 strips per chunk.
LaunchChoice class_choice(const vca_batch* b, int k) {
  LaunchChoice c = b->kind_tuned[k];
  if (c.depth <= 0) c = LaunchChoice{2, 0, 0.0, kDefaultWaves, kDefaultChunk};
  if (c.waves != 4 && c.waves != 8) c.waves = kDefaultWaves;
  if (c.chunk <= 0 || c.chunk % kRun != 0) c.chunk = kDefaultChunk;
  return c;
}

// Fills the staging descriptors for one round: stream s analyses frames
// [off[s], off[s] + cnt[s]) of its call.  Returns the number of chunks and of
// frames of the round.
void fill_descriptors(vca_batch* b, const vca_frames* fr, const int32_t* off, const int32_t* cnt,
                      int32_t* total_chunks, int32_t* total_frames) {
  int32_t chunks = 0, frames = 0, i = 0;
  // each stream's frames are numbered from its first reduction workgroup on
  std::vector<int32_t> frame_begin(b->n);
  for (int s = 0; s < b->n; s++) {
    frame_begin[s] = frames;
    frames += cnt[s];
  }
  frames = 0;
  for (int k = 0; k < kKinds; k++) {
    KindRange& kr = b->kinds[k];
    kr.desc_begin = i;
    kr.chunk_begin = chunks;
    kr.chunk_strips = class_choice(b, k).chunk;
    for (int s = 0; s < b->n; s++) {
      const Geometry& g = b->geos[s];
      const vca_config& c = b->cfgs[s];
      if (kind_of(c.bit_depth, c.block_size, g.K) != k) continue;
      StreamDesc& sd = b->h_streams[i++];
      std::memset(&sd, 0, sizeof(sd));
      const uint8_t* base[3] = {static_cast<const uint8_t*>(fr[s].y), static_cast<const uint8_t*>(fr[s].u),
                                static_cast<const uint8_t*>(fr[s].v)};
      const int64_t fs[3] = {fr[s].fstride_y, fr[s].fstride_uv, fr[s].fstride_uv};
      const int64_t pt[3] = {fr[s].pitch_y, fr[s].pitch_uv, fr[s].pitch_uv};
      const uint8_t* first[3];
      for (int P = 0; P < 3; P++) first[P] = cnt[s] > 0 ? base[P] + fs[P] * off[s] : nullptr;
      sd.geom = make_strip_geom(g, first, fs, pt, (int32_t)b->blk_base[s], frame_begin[s]);
      sd.kind = k;
      sd.strips = cnt[s] * sd.geom.strips_per_frame;
      sd.chunk_begin = chunks;
      chunks += (sd.strips + kr.chunk_strips - 1) / kr.chunk_strips;
      sd.chunk_end = chunks;
      sd.validate = (c.flags & VCA_F_VALIDATE) && c.bit_depth == 10 ? 1 : 0;
      sd.stream = s;
    }
    kr.desc_end = i;
    kr.chunk_end = chunks;
  }
  // reduction records in the flat order (by class, then stream); each
  // class's reduction launch numbers its workgroups from 0
  for (int k = 0; k < kKinds; k++) {
    int32_t kframes = 0;
    int64_t kblocks = 0;
    for (int i2 = b->kinds[k].desc_begin; i2 < b->kinds[k].desc_end; i2++) {
      const int s = b->h_streams[i2].stream;
      const Geometry& g = b->geos[s];
      const vca_config& c = b->cfgs[s];
      ReduceParams& rp = b->h_red[i2];
      std::memset(&rp, 0, sizeof(rp));
      const double ww = (double)c.block_size * c.block_size;
      rp.blk_h = b->blk_h + b->blk_base[s];
      rp.blk_dc = b->blk_dc + b->blk_base[s];
      double* st = b->state + b->state_off[s];
      rp.state_in = b->has_prev[s] ? st + (int64_t)b->cur_state[s] * g.cnt[0] : nullptr;
      rp.state_out = st + (int64_t)(b->cur_state[s] ^ 1) * g.cnt[0];
      rp.ring = b->rings + b->ring_off[s];
      rp.frame_err = (c.flags & VCA_F_VALIDATE) ? b->frame_err + frame_begin[s] : nullptr;
      rp.err_ring = b->err_rings + b->ring_off[s] / 7;
      rp.first_frame = b->submitted[s];
      rp.capacity = c.feature_capacity;
      for (int P = 0; P < 3; P++) {
        rp.cnt[P] = g.cnt[P];
        rp.inv_norm[P] = 1.0 / ((double)g.cnt[P] * ww);
      }
      rp.per_frame = g.per_frame;
      rp.n_frames = cnt[s];
      rp.frame_begin = kframes;
      kframes += cnt[s];
      kblocks += (int64_t)cnt[s] * g.per_frame;
      frames += cnt[s];
    }
    b->kind_frames[k] = kframes;
    b->kind_blocks[k] = kblocks;
  }
  *total_chunks = chunks;
  *total_frames = frames;
}

// Enqueues class k's forward launch on st.
vca_status launch_forward(vca_batch* b, hipStream_t st, int k, const LaunchChoice& lc) {
  const KindRange& kr = b->kinds[k];
  const int waves = lc.waves == 8 ? 8 : 4;
  BatchKernel kern = class_kernel_for(k, lc.depth, waves);
  int resident = 0;
  BHIP_TRY(b, hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, kern, 64 * waves, 0));
  resident = std::max(1, resident);
  if (lc.groups_per_cu > 0) resident = std::min(resident, lc.groups_per_cu);
  const int64_t groups = ((int64_t)(kr.chunk_end - kr.chunk_begin) + waves - 1) / waves;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(groups, (int64_t)b->num_cus * resident));
  BatchParams bp{};
  bp.streams = b->d_streams;
  bp.kr = kr;
  bp.tab_b1p = b->tab_b1p + k * kMaxPack * 64;
  bp.tab_a2 = b->tab_a2 + k * 64;
  bp.tab_wp = b->tab_wp + k * 16 * 64;
  bp.blk_h = b->blk_h;
  bp.blk_dc = b->blk_dc;
  bp.err_flag = b->frame_err;
  bp.queue = b->queue + k;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * waves), 0, st, bp);
  BHIP_TRY(b, hipGetLastError());
  return VCA_OK;
}

// Enqueues class k's reduction (features and h state of its streams) on st.
vca_status launch_reduce(vca_batch* b, hipStream_t st, int k) {
  const KindRange& kr = b->kinds[k];
  if (b->kind_frames[k] <= 0) return VCA_OK;
  BatchReduceParams rp{b->d_red + kr.desc_begin, kr.desc_end - kr.desc_begin};
  hipLaunchKernelGGL(batch_reduce_kernel, dim3(b->kind_frames[k]), dim3(kReduceThreads), 0, st, rp);
  BHIP_TRY(b, hipGetLastError());
  return VCA_OK;
}

// Classes with work in the current round.
int present_classes(const vca_batch* b, int* list) {
  int n = 0;
  for (int k = 0; k < kKinds; k++)
    if (b->kinds[k].chunk_end > b->kinds[k].chunk_begin) list[n++] = k;
  return n;
}

// Streams and events of the forks (created before any capture).
vca_status ensure_branches(vca_batch* b, int n) {
  if (!b->fork_ev) BHIP_TRY(b, hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
  for (int j = 0; j < n; j++) {
    if (!b->branch[j]) BHIP_TRY(b, hipStreamCreateWithFlags(&b->branch[j], hipStreamNonBlocking));
    if (!b->join_ev[j]) BHIP_TRY(b, hipEventCreateWithFlags(&b->join_ev[j], hipEventDisableTiming));
    if (!b->fwd_ev[j]) BHIP_TRY(b, hipEventCreateWithFlags(&b->fwd_ev[j], hipEventDisableTiming));
  }
  return VCA_OK;
}

// The classes of the current round on st, after the counters are reset.
// Parallel: each class's forward launch (and, with_reduce, its reduction) on
// a branch of its own, all forked from st.  Serial: the forward launches one
// after another on st (the class with the most blocks first), each class's
// reduction on a branch forked after its forward launch, so that it overlaps
// the next class.  Either way every branch joins st again.
vca_status enqueue_classes(vca_batch* b, hipStream_t st, bool serial, bool with_reduce) {
  int list[kKinds];
  const int n = present_classes(b, list);
  hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, st, b->queue);
  BHIP_TRY(b, hipGetLastError());
  if (n == 0) return VCA_OK;
  vca_status s = VCA_OK;
  if (serial) {
    // most blocks first: the last class's reduction is the one left
    // exposed, and a reduction's cost follows the blocks it sums
    std::stable_sort(list, list + n,
                     [b](int x, int y) { return b->kind_blocks[x] > b->kind_blocks[y]; });
    for (int j = 0; j < n; j++) {
      if ((s = launch_forward(b, st, list[j], class_choice(b, list[j]))) != VCA_OK) return s;
      if (!with_reduce) continue;
      BHIP_TRY(b, hipEventRecord(b->fwd_ev[j], st));
      BHIP_TRY(b, hipStreamWaitEvent(b->branch[j], b->fwd_ev[j], 0));
      if ((s = launch_reduce(b, b->branch[j], list[j])) != VCA_OK) return s;
      BHIP_TRY(b, hipEventRecord(b->join_ev[j], b->branch[j]));
    }
    if (with_reduce)
      for (int j = 0; j < n; j++) BHIP_TRY(b, hipStreamWaitEvent(st, b->join_ev[j], 0));
    return VCA_OK;
  }
  BHIP_TRY(b, hipEventRecord(b->fork_ev, st));
  for (int j = 0; j < n; j++) {
    BHIP_TRY(b, hipStreamWaitEvent(b->branch[j], b->fork_ev, 0));
    if ((s = launch_forward(b, b->branch[j], list[j], class_choice(b, list[j]))) != VCA_OK) return s;
    if (with_reduce && (s = launch_reduce(b, b->branch[j], list[j])) != VCA_OK) return s;
    BHIP_TRY(b, hipEventRecord(b->join_ev[j], b->branch[j]));
  }
  for (int j = 0; j < n; j++) BHIP_TRY(b, hipStreamWaitEvent(st, b->join_ev[j], 0));
  return VCA_OK;
}

// One round on st in the batch's arrangement of classes.
vca_status enqueue_round(vca_batch* b, hipStream_t st) {
  return enqueue_classes(b, st, b->serial != 0, true);
}

// One round on st alone, with no branch: every class's forward launch and
// then its reduction, class after class (rounds whose signature finds the
// graph cache full).
vca_status enqueue_round_in_line(vca_batch* b, hipStream_t st) {
  int list[kKinds];
  const int n = present_classes(b, list);
  hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, st, b->queue);
  BHIP_TRY(b, hipGetLastError());
  vca_status s = VCA_OK;
  for (int j = 0; j < n; j++) {
    if ((s = launch_forward(b, st, list[j], class_choice(b, list[j]))) != VCA_OK) return s;
    if ((s = launch_reduce(b, st, list[j])) != VCA_OK) return s;
  }
  return VCA_OK;
}

// Copies the staging descriptors to the device on the batch's stream.
vca_status upload_descriptors(vca_batch* b) {
  BHIP_TRY(b, hipMemcpyAsync(b->d_streams, b->h_streams, sizeof(StreamDesc) * b->n,
                             hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipMemcpyAsync(b->d_red, b->h_red, sizeof(ReduceParams) * b->n,
                             hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipEventRecord(b->uploaded, b->stream));
  b->upload_pending = true;
  return VCA_OK;
}

vca_status wait_staging(vca_batch* b) {
  if (b->upload_pending) {
    BHIP_TRY(b, hipEventSynchronize(b->uploaded));
    b->upload_pending = false;
  }
  return VCA_OK;
}

std::string batch_tune_key(const vca_batch* b) {
  std::string k = "gfx950/cu" + std::to_string(b->num_cus) + "/batch";
  for (int s = 0; s < b->n; s++) {
    const vca_config& c = b->cfgs[s];
    k += "/" + std::to_string(c.bit_depth) + "b" + std::to_string(c.block_size) + "w" +
         std::to_string(b->geos[s].K) + "k" + std::to_string(c.width) + "x" + std::to_string(c.height);
  }
  // keys stay short: hash the stream list
  uint64_t h = 1469598103934665603ull;
  for (char ch : k) h = (h ^ (uint8_t)ch) * 1099511628211ull;
  char buf[96];
  std::snprintf(buf, sizeof(buf), "gfx950/cu%d/batch/n%d/%016llx", b->num_cus, b->n,
                (unsigned long long)h);
  return buf;
}

std::string class_tune_key(const vca_batch* b, int k) { return batch_tune_key(b) + "/k" + std::to_string(k); }

// Per-class shapes cached for this stream list (from an earlier vca_tune_batch
// in the process or the VCA_TUNE_CACHE file), and their summary.
void load_tuned(vca_batch* b) {
  double total = 0.0, worst = -1.0;
  for (int k = 0; k < kKinds; k++) {
    if (!TuneCache::get().find(class_tune_key(b, k), &b->kind_tuned[k])) continue;
    total += b->kind_tuned[k].ms;
    if (b->kind_tuned[k].ms > worst) {
      worst = b->kind_tuned[k].ms;
      b->tuned = b->kind_tuned[k];
    }
  }
  if (worst >= 0.0) b->tuned.ms = total;
  // the arrangement of the classes: serial unless side by side measured
  // faster over whole rounds
  LaunchChoice par, ser;
  if (TuneCache::get().find(batch_tune_key(b) + "/parallel_round", &par) &&
      TuneCache::get().find(batch_tune_key(b) + "/serial_round", &ser)) {
    b->parallel_ms = par.ms;
    b->serial_ms = ser.ms;
    b->serial = ser.ms <= par.ms ? 1 : 0;
  }
}

// Validation marks of frames [first, first + count) of a stream (whose round
// has completed): a message if one of them held a 10-bit sample above 1023.
const char* invalid_frames(const vca_batch* b, int32_t s, int64_t first, int32_t count) {
  if (!(b->cfgs[s].flags & VCA_F_VALIDATE)) return nullptr;
  const int64_t cap = b->cfgs[s].feature_capacity;
  const volatile int32_t* marks = b->err_rings_host + b->ring_off[s] / 7;
  for (int64_t f = first; f < first + count; f++)
    if (marks[f % cap]) return "a requested frame holds a 10-bit sample above 1023";
  return nullptr;
}

vca_status check_batch_frames(vca_batch* b, const vca_frames* fr, const int32_t* n_frames) {
  if (!fr || !n_frames) return bfail(b, VCA_ERR_INVALID_ARG, "null argument");
  for (int s = 0; s < b->n; s++) {
    if (n_frames[s] < 0) return bfail(b, VCA_ERR_INVALID_ARG, "negative frame count");
    if (n_frames[s] == 0) continue;
    if (!fr[s].on_device) return bfail(b, VCA_ERR_UNSUPPORTED, "host-resident frames");
    if (const char* msg = check_frames(b->cfgs[s], &fr[s], n_frames[s]))
      return bfail(b, VCA_ERR_INVALID_ARG, "stream " + std::to_string(s) + ": " + msg);
  }
  return VCA_OK;
}

}  // namespace

extern "C" {

void vca_close_batch(vca_batch* b) {
  if (!b) return;
  {
    DeviceGuard g(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    void* bufs[] = {b->tab_b1p, b->tab_a2,    b->tab_wp, b->blk_h,  b->blk_dc,
                    b->state,   b->d_streams, b->d_red,  b->queue, b->frame_err};
    for (void* p : bufs)
      if (p) (void)hipFree(p);
    if (b->rings_host) (void)hipHostFree(b->rings_host);
    if (b->err_rings_host) (void)hipHostFree(b->err_rings_host);
    if (b->h_streams) (void)hipHostFree(b->h_streams);
    if (b->h_red) (void)hipHostFree(b->h_red);
    if (b->uploaded) (void)hipEventDestroy(b->uploaded);
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    for (int k = 0; k < kKinds; k++) {
      if (b->join_ev[k]) (void)hipEventDestroy(b->join_ev[k]);
      if (b->fwd_ev[k]) (void)hipEventDestroy(b->fwd_ev[k]);
      if (b->branch[k]) (void)hipStreamDestroy(b->branch[k]);
    }
    for (hipEvent_t e : b->ev_pool) (void)hipEventDestroy(e);
    b->done.destroy();
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  }
  delete b;
}

vca_status vca_open_batch(const vca_config* cfgs, int32_t n_streams, void* hip_stream,
                          vca_batch** out) {
  if (!out) return VCA_ERR_INVALID_ARG;
  *out = nullptr;
  if (!cfgs || n_streams <= 0) return VCA_ERR_INVALID_ARG;
  for (int s = 0; s < n_streams; s++) {
    vca_status st = check_config(&cfgs[s]);
    if (st == VCA_OK && (cfgs[s].flags & VCA_F_DOWNSAMPLE)) st = VCA_ERR_UNSUPPORTED;
    if (st != VCA_OK) return st;
    // one round's frames of a stream must not share ring slots
    const int32_t mb = cfgs[s].max_batch ? cfgs[s].max_batch : kDefaultMaxBatch;
    const int32_t cap = cfgs[s].feature_capacity ? cfgs[s].feature_capacity : kDefaultCapacity;
    if (cap < mb) return VCA_ERR_INVALID_ARG;
    if (cfgs[s].flags & VCA_F_KEEP_COEFFS) return VCA_ERR_UNSUPPORTED;
    if (cfgs[s].device != cfgs[0].device) return VCA_ERR_INVALID_ARG;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return VCA_ERR_DEVICE;
  if (cfgs[0].device >= ndev) return VCA_ERR_INVALID_ARG;

  vca_batch* b = new (std::nothrow) vca_batch();
  if (!b) return VCA_ERR_OOM;
  b->n = n_streams;
  b->device = cfgs[0].device;
  b->cfgs.assign(cfgs, cfgs + n_streams);
  b->geos.resize(n_streams);
  b->blk_base.resize(n_streams);
  b->state_off.resize(n_streams);
  b->ring_off.resize(n_streams);
  b->cur_state.assign(n_streams, 0);
  b->has_prev.assign(n_streams, 0);
  b->submitted.assign(n_streams, 0);
  int64_t blk = 0, st_total = 0, ring_total = 0, round_frames = 0;
  for (int s = 0; s < n_streams; s++) {
    vca_config& c = b->cfgs[s];
    if (c.max_batch == 0) c.max_batch = kDefaultMaxBatch;
    if (c.feature_capacity == 0) c.feature_capacity = kDefaultCapacity;
    round_frames += c.max_batch;
    b->geos[s].init(c);
    if (c.flags & VCA_F_TIMING) b->timing = true;
    b->blk_base[s] = blk;
    blk += (int64_t)c.max_batch * b->geos[s].per_frame;
    b->state_off[s] = st_total;
    st_total += 2 * (int64_t)b->geos[s].cnt[0];
    b->ring_off[s] = ring_total;
    ring_total += (int64_t)c.feature_capacity * 7;
  }
  auto bail = [&](vca_status st) {
    vca_close_batch(b);
    return st;
  };
  if (blk > (int64_t)INT32_MAX / 2) return bail(VCA_ERR_INVALID_ARG);   // block ids fit int32
  DeviceGuard guard(b->device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, b->device) != hipSuccess) return bail(VCA_ERR_DEVICE);
  b->num_cus = prop.multiProcessorCount;
  if (hip_stream) {
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(VCA_ERR_DEVICE);
    b->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess)
    return bail(VCA_ERR_DEVICE);
  if (hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming) != hipSuccess ||
      b->done.init(n_streams) != hipSuccess)
    return bail(VCA_ERR_DEVICE);
  vca_status s;
  if ((s = balloc(b, &b->tab_b1p, kKinds * kMaxPack * 64)) != VCA_OK) return bail(s);
  if ((s = balloc(b, &b->tab_a2, kKinds * 64)) != VCA_OK) return bail(s);
  if ((s = balloc(b, &b->tab_wp, kKinds * 16 * 64)) != VCA_OK) return bail(s);
  if ((s = balloc(b, &b->blk_h, (size_t)blk)) != VCA_OK) return bail(s);
  if ((s = balloc(b, &b->blk_dc, (size_t)blk)) != VCA_OK) return bail(s);
  if ((s = balloc(b, &b->state, (size_t)st_total)) != VCA_OK) return bail(s);
  if (host_mapped_alloc((size_t)ring_total * sizeof(float), reinterpret_cast<void**>(&b->rings_host),
                        reinterpret_cast<void**>(&b->rings)) != hipSuccess ||
      host_mapped_alloc((size_t)(ring_total / 7) * sizeof(int32_t),
                        reinterpret_cast<void**>(&b->err_rings_host),
                        reinterpret_cast<void**>(&b->err_rings)) != hipSuccess)
    return bail(VCA_ERR_OOM);
  if ((s = balloc(b, &b->frame_err, (size_t)round_frames)) != VCA_OK) return bail(s);
  if (hipMemset(b->frame_err, 0, (size_t)round_frames * sizeof(int32_t)) != hipSuccess)
    return bail(VCA_ERR_DEVICE);
  if ((s = balloc(b, &b->d_streams, n_streams)) != VCA_OK) return bail(s);
  if ((s = balloc(b, &b->d_red, n_streams)) != VCA_OK) return bail(s);
  if ((s = balloc(b, &b->queue, kKinds)) != VCA_OK) return bail(s);
  if (hipHostMalloc(reinterpret_cast<void**>(&b->h_streams), sizeof(StreamDesc) * n_streams, 0) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&b->h_red), sizeof(ReduceParams) * n_streams, 0) != hipSuccess)
    return bail(VCA_ERR_OOM);

  // operand and weight tables of every kind (packed layout)
  std::vector<int8_t> b1all((size_t)kKinds * kMaxPack * 64 * 16, 0), a2all(kKinds * 64 * 16);
  std::vector<double> wall(kKinds * 16 * 64);
  for (int bits : {8, 10})
    for (int w : {32, 16, 8})
      for (int kd : {1, 2, 4}) {
        const int kind = kind_of(bits, w, w / kd);
        std::vector<int8_t> b1, a2, b1p;
        std::vector<double> wt, wtp;
        build_tile_tables(w, w / kd, b1, a2, wt);
        build_packed_tables(w, w / kd, b1p, wtp);
        std::copy(b1p.begin(), b1p.end(), b1all.begin() + (size_t)kind * kMaxPack * 64 * 16);
        std::copy(a2.begin(), a2.end(), a2all.begin() + kind * 64 * 16);
        std::copy(wtp.begin(), wtp.end(), wall.begin() + kind * 16 * 64);
      }
  if (hipMemcpy(b->tab_b1p, b1all.data(), b1all.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->tab_a2, a2all.data(), a2all.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->tab_wp, wall.data(), wall.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return bail(VCA_ERR_DEVICE);
  if (const char* e = std::getenv("VCA_BATCH_NO_GRAPH")) b->use_graph = !(e[0] == '1');
  load_tuned(b);
  *out = b;
  return VCA_OK;
}

vca_status vca_analyze_batch(vca_batch* b, const vca_frames* frames, const int32_t* n_frames) {
  if (!b) return VCA_ERR_INVALID_ARG;
  vca_status st = check_batch_frames(b, frames, n_frames);
  if (st != VCA_OK) return st;
  DeviceGuard guard(b->device);
  std::vector<int32_t> off(b->n, 0), cnt(b->n, 0);
  for (;;) {
    bool any = false;
    for (int s = 0; s < b->n; s++) {
      cnt[s] = std::min<int32_t>(b->cfgs[s].max_batch, n_frames[s] - off[s]);
      any |= cnt[s] > 0;
    }
    if (!any) break;
    if ((st = wait_staging(b)) != VCA_OK) return st;
    int32_t chunks = 0, nfr = 0;
    fill_descriptors(b, frames, off.data(), cnt.data(), &chunks, &nfr);
    if ((st = upload_descriptors(b)) != VCA_OK) return st;
    {
      int list[kKinds];
      if ((st = ensure_branches(b, present_classes(b, list))) != VCA_OK) return st;
    }
    hipEvent_t* ev = nullptr;
    if (b->timing) {
      if (b->ev_used + 2 > b->ev_pool.size()) {
        for (int e = 0; e < 2; e++) {
          hipEvent_t h;
          BHIP_TRY(b, hipEventCreate(&h));
          b->ev_pool.push_back(h);
        }
      }
      ev = &b->ev_pool[b->ev_used];
      b->ev_frames.push_back(nfr);
      b->ev_used += 2;
      BHIP_TRY(b, hipEventRecord(ev[0], b->stream));
    }
    if (b->use_graph) {
      std::vector<int32_t> sig(cnt);
      for (int k = 0; k < kKinds; k++) {
        const LaunchChoice lc = class_choice(b, k);
        sig.push_back(lc.depth);
        sig.push_back(lc.groups_per_cu);
        sig.push_back(lc.waves);
        sig.push_back(lc.chunk);
      }
      sig.push_back(b->serial);
      vca_batch::CachedGraph* hit = nullptr;
      for (auto& c : b->graphs)
        if (c.sig == sig) hit = &c;
      const bool eager = !hit && b->graphs.size() >= kMaxGraphs;   // cache full
      if (!hit && !eager) {
        BHIP_TRY(b, hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
        st = enqueue_round(b, b->capture);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(b->capture, &g);
        if (st != VCA_OK) {
          if (g) (void)hipGraphDestroy(g);
          return st;
        }
        if (ec != hipSuccess) return bfail(b, VCA_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
        hipGraphExec_t x = nullptr;
        const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
          (void)hipGraphDestroy(g);
          return bfail(b, VCA_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
        }
        b->graphs.push_back(vca_batch::CachedGraph{sig, g, x});
        hit = &b->graphs.back();
      }
      if (eager) {
        if ((st = enqueue_round_in_line(b, b->stream)) != VCA_OK) return st;
      } else {
        BHIP_TRY(b, hipGraphLaunch(hit->exec, b->stream));
      }
    } else {
      if ((st = enqueue_round(b, b->stream)) != VCA_OK) return st;
    }
    if (ev) BHIP_TRY(b, hipEventRecord(ev[1], b->stream));
    for (int s = 0; s < b->n; s++) {
      if (cnt[s] <= 0) continue;
      b->cur_state[s] ^= 1;
      b->has_prev[s] = 1;
      b->submitted[s] += cnt[s];
      off[s] += cnt[s];
    }
    BHIP_TRY(b, b->done.record(b->stream, b->submitted.data()));
  }
  return VCA_OK;
}

vca_status vca_tune_batch(vca_batch* b, const vca_frames* frames, const int32_t* n_frames, int32_t reps) {
  if (!b || reps <= 0) return bfail(b, VCA_ERR_INVALID_ARG, "bad vca_tune_batch arguments");
  vca_status st = check_batch_frames(b, frames, n_frames);
  if (st != VCA_OK) return st;
  DeviceGuard guard(b->device);
  std::vector<int32_t> off(b->n, 0), cnt(b->n, 0);
  for (int s = 0; s < b->n; s++) cnt[s] = std::min<int32_t>(b->cfgs[s].max_batch, n_frames[s]);
  if ((st = wait_staging(b)) != VCA_OK) return st;
  int32_t chunks = 0, nfr = 0;
  hipEvent_t e0, e1;
  BHIP_TRY(b, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return bfail(b, VCA_ERR_DEVICE, "hipEventCreate");
  }
  // the round's descriptors with the classes' current chunk sizes (no
  // validation while tuning: no reduction follows to collect the marks)
  auto refill = [&]() -> vca_status {
    vca_status r = wait_staging(b);
    if (r != VCA_OK) return r;
    fill_descriptors(b, frames, off.data(), cnt.data(), &chunks, &nfr);
    for (int i = 0; i < b->n; i++) b->h_streams[i].validate = 0;
    return upload_descriptors(b);
  };
  // class k's forward launch alone with shape lc: its mean time over reps
  // launches after one warm-up (features and h state are untouched)
  auto time_class = [&](int k, const LaunchChoice& lc, double* ms_out) -> vca_status {
    auto once = [&]() {
      hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, b->stream, b->queue);
      return launch_forward(b, b->stream, k, lc);
    };
    vca_status r = once();
    if (r != VCA_OK) return r;
    if (hipEventRecord(e0, b->stream) != hipSuccess) return bfail(b, VCA_ERR_DEVICE, "hipEventRecord");
    for (int i = 0; i < reps && r == VCA_OK; i++) r = once();
    if (r != VCA_OK) return r;
    if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return bfail(b, VCA_ERR_DEVICE, "hipEventRecord/Synchronize");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *ms_out = ms / reps;
    return VCA_OK;
  };
  // each class alone: every (ring depth, wavefronts per workgroup,
  // workgroups per CU) at the default chunk size, then every chunk size at
  // the best of those
  st = refill();
  int list[kKinds];
  const int n = st == VCA_OK ? present_classes(b, list) : 0;
  for (int j = 0; j < n && st == VCA_OK; j++) {
    const int k = list[j];
    LaunchChoice best;
    best.ms = 1e30;
    for (int waves = 4; waves <= 8 && st == VCA_OK; waves += 4) {
      for (int depth = 1; depth <= 4 && st == VCA_OK; depth *= 2) {
        int resident = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, class_kernel_for(k, depth, waves), 64 * waves,
                                                         0) != hipSuccess)
          resident = 1;
        for (int gpc = 1; gpc <= std::max(1, resident) && st == VCA_OK; gpc++) {
          const LaunchChoice lc{depth, gpc, 0.0, waves, class_choice(b, k).chunk};
          double ms = 0.0;
          if ((st = time_class(k, lc, &ms)) != VCA_OK) break;
          if (ms < best.ms) best = LaunchChoice{depth, gpc, ms, waves, lc.chunk};
        }
      }
    }
    const int chunk0 = best.chunk;
    for (int chunk : kChunkChoices) {
      if (st != VCA_OK || chunk == chunk0) continue;
      LaunchChoice lc = best;
      lc.chunk = chunk;
      b->kind_tuned[k] = lc;   // the descriptors follow the class's chunk size
      double ms = 0.0;
      if ((st = refill()) != VCA_OK || (st = time_class(k, lc, &ms)) != VCA_OK) break;
      if (ms < best.ms) best = LaunchChoice{lc.depth, lc.groups_per_cu, ms, lc.waves, chunk};
    }
    if (st == VCA_OK) {
      b->kind_tuned[k] = best;
      TuneCache::get().put(class_tune_key(b, k), best);
      st = refill();
    }
  }
  // then the arrangement of the tuned classes, one after another or side by
  // side: whole rounds, reductions included (in the serial arrangement they
  // run beside the next class's forward launch, which decides between the
  // two).  The reductions' features and marks go to a scratch area and
  // their h state to the buffer the next round overwrites, so no stream's
  // features or state change.
  double arr_ms[2] = {0.0, 0.0};
  void* scratch = nullptr;
  if (st == VCA_OK && n > 1) st = ensure_branches(b, n);
  if (st == VCA_OK && n > 1) {
    int64_t cap = 1;
    for (int s = 0; s < b->n; s++) cap = std::max<int64_t>(cap, b->cfgs[s].feature_capacity);
    if (hipMalloc(&scratch, (size_t)cap * 8 * sizeof(float)) != hipSuccess) {
      scratch = nullptr;
      st = bfail(b, VCA_ERR_OOM, "hipMalloc (tuning scratch)");
    } else if ((st = wait_staging(b)) == VCA_OK) {
      for (int i = 0; i < b->n; i++) {
        b->h_red[i].ring = static_cast<float*>(scratch);
        b->h_red[i].err_ring = reinterpret_cast<int32_t*>(static_cast<float*>(scratch) + cap * 7);
      }
      st = upload_descriptors(b);
    }
  }
  // one warm-up round of each, then at least four rounds of each in turn,
  // so that a drift of the clock over the tuning falls on both alike
  const int arr_reps = std::max(reps, 4);
  for (int serial = 0; serial < 2 && st == VCA_OK && n > 1; serial++)
    st = enqueue_classes(b, b->stream, serial != 0, true);
  for (int r = 0; r < 2 * arr_reps && st == VCA_OK && n > 1; r++) {
    const int serial = r & 1;
    if (hipEventRecord(e0, b->stream) != hipSuccess) { st = bfail(b, VCA_ERR_DEVICE, "hipEventRecord"); break; }
    if ((st = enqueue_classes(b, b->stream, serial != 0, true)) != VCA_OK) break;
    if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      st = bfail(b, VCA_ERR_DEVICE, "hipEventRecord/Synchronize");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    arr_ms[serial] += ms / arr_reps;
  }
  if (scratch) {
    // every launch that writes the scratch area has finished before it goes
    if (hipStreamSynchronize(b->stream) != hipSuccess && st == VCA_OK)
      st = bfail(b, VCA_ERR_DEVICE, "hipStreamSynchronize");
    (void)hipFree(scratch);
    if (st == VCA_OK) st = refill();   // the real feature rings back in the descriptors
  }
  if (st == VCA_OK && n > 1) {
    TuneCache::get().put(batch_tune_key(b) + "/parallel_round", LaunchChoice{1, 0, arr_ms[0]});
    TuneCache::get().put(batch_tune_key(b) + "/serial_round", LaunchChoice{1, 0, arr_ms[1]});
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != VCA_OK) return st;
  load_tuned(b);
  return VCA_OK;
}

vca_status vca_batch_tuned_launch(const vca_batch* b, int32_t* depth, int32_t* groups_per_cu, double* ms) {
  if (!b) return VCA_ERR_INVALID_ARG;
  if (depth) *depth = b->tuned.depth;
  if (groups_per_cu) *groups_per_cu = b->tuned.groups_per_cu;
  if (ms) *ms = b->tuned.ms;
  return VCA_OK;
}

vca_status vca_batch_class_times(const vca_batch* b, double* ms, int32_t* depth,
                                 int32_t* groups_per_cu, int32_t* waves, int32_t* chunk_strips) {
  if (!b) return VCA_ERR_INVALID_ARG;
  for (int k = 0; k < kKinds; k++) {
    const LaunchChoice& t = b->kind_tuned[k];
    const bool tuned = t.depth > 0;
    if (ms) ms[k] = tuned ? t.ms : 0.0;
    if (depth) depth[k] = tuned ? t.depth : 0;
    if (groups_per_cu) groups_per_cu[k] = tuned ? t.groups_per_cu : 0;
    if (waves) waves[k] = tuned ? class_choice(b, k).waves : 0;
    if (chunk_strips) chunk_strips[k] = tuned ? class_choice(b, k).chunk : 0;
  }
  return VCA_OK;
}

vca_status vca_batch_arrangement(const vca_batch* b, int32_t* serial, double* serial_ms,
                                double* parallel_ms) {
  if (!b) return VCA_ERR_INVALID_ARG;
  if (serial) *serial = b->serial;
  if (serial_ms) *serial_ms = b->serial_ms;
  if (parallel_ms) *parallel_ms = b->parallel_ms;
  return VCA_OK;
}

vca_status vca_batch_set_class_shape(vca_batch* b, int32_t cls, int32_t depth, int32_t groups_per_cu,
                                     int32_t waves, int32_t chunk_strips) {
  if (!b) return VCA_ERR_INVALID_ARG;
  const bool chunk_ok = std::find(std::begin(kChunkChoices), std::end(kChunkChoices), chunk_strips) !=
                        std::end(kChunkChoices);
  if (cls < 0 || cls >= kKinds || (depth != 1 && depth != 2 && depth != 4) || groups_per_cu < 0 ||
      (waves != 4 && waves != 8) || !chunk_ok)
    return bfail(b, VCA_ERR_INVALID_ARG, "bad class shape");
  b->kind_tuned[cls] = LaunchChoice{depth, groups_per_cu, 0.0, waves, chunk_strips};
  return VCA_OK;
}

vca_status vca_batch_set_arrangement(vca_batch* b, int32_t serial) {
  if (!b || (serial != 0 && serial != 1)) return bfail(b, VCA_ERR_INVALID_ARG, "serial must be 0 or 1");
  b->serial = serial;
  return VCA_OK;
}

vca_status vca_batch_features(vca_batch* b, int32_t stream, int64_t first, int32_t count,
                              vca_frame_features* out) {
  if (!b || stream < 0 || stream >= b->n || count < 0 || first < 0 || (count > 0 && !out))
    return bfail(b, VCA_ERR_INVALID_ARG, "bad vca_batch_features arguments");
  if (first + count > b->submitted[stream]) return bfail(b, VCA_ERR_STATE, "frame not yet submitted");
  const int64_t cap = b->cfgs[stream].feature_capacity;
  if (first < b->submitted[stream] - cap) return bfail(b, VCA_ERR_STATE, "frame left the feature ring");
  DeviceGuard guard(b->device);
  BHIP_TRY(b, b->done.wait(stream, first + count, b->stream));
  // the rings are host memory the kernels wrote before the round that
  // produced the last frame asked for completed
  if (const char* bad = invalid_frames(b, stream, first, count)) return bfail(b, VCA_ERR_STATE, bad);
  const float* ring = b->rings_host + b->ring_off[stream];
  int64_t done = 0;
  while (done < count) {
    const int64_t slot = (first + done) % cap;
    const int64_t n = std::min<int64_t>(count - done, cap - slot);
    std::memcpy(reinterpret_cast<float*>(out) + done * 7, ring + slot * 7, (size_t)n * 7 * sizeof(float));
    done += n;
  }
  return VCA_OK;
}

vca_status vca_batch_features_many(vca_batch* b, int32_t n_requests, const int32_t* streams,
                                   const int64_t* first, const int32_t* count,
                                   vca_frame_features* out) {
  if (!b || n_requests < 0 || (n_requests > 0 && (!streams || !first || !count || !out)))
    return bfail(b, VCA_ERR_INVALID_ARG, "bad vca_batch_features_many arguments");
  int rank = 0;
  for (int32_t r = 0; r < n_requests; r++) {
    const int32_t s = streams[r];
    if (s < 0 || s >= b->n || count[r] < 0 || first[r] < 0)
      return bfail(b, VCA_ERR_INVALID_ARG, "request " + std::to_string(r) + ": bad stream or range");
    if (first[r] + count[r] > b->submitted[s])
      return bfail(b, VCA_ERR_STATE, "request " + std::to_string(r) + ": frame not yet submitted");
    if (first[r] < b->submitted[s] - b->cfgs[s].feature_capacity)
      return bfail(b, VCA_ERR_STATE, "request " + std::to_string(r) + ": frame left the feature ring");
    rank = std::max(rank, b->done.cover(s, first[r] + count[r]));
  }
  DeviceGuard guard(b->device);
  BHIP_TRY(b, b->done.wait_rank(rank, b->stream));
  float* dst = reinterpret_cast<float*>(out);
  for (int32_t r = 0; r < n_requests; r++) {
    const int32_t s = streams[r];
    if (const char* bad = invalid_frames(b, s, first[r], count[r]))
      return bfail(b, VCA_ERR_STATE, "stream " + std::to_string(s) + ": " + bad);
    const int64_t cap = b->cfgs[s].feature_capacity;
    const float* ring = b->rings_host + b->ring_off[s];
    for (int64_t done = 0; done < count[r];) {
      const int64_t slot = (first[r] + done) % cap;
      const int64_t n = std::min<int64_t>(count[r] - done, cap - slot);
      std::memcpy(dst, ring + slot * 7, (size_t)n * 7 * sizeof(float));
      dst += n * 7;
      done += n;
    }
  }
  return VCA_OK;
}

vca_status vca_batch_timing(vca_batch* b, double* total_ms, int64_t* launches, int64_t* frames,
                            int32_t reset) {
  if (!b) return VCA_ERR_INVALID_ARG;
  if (!b->timing) return bfail(b, VCA_ERR_STATE, "no stream opened with VCA_F_TIMING");
  DeviceGuard guard(b->device);
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  double ms = 0.0;
  int64_t n = 0, fr = 0;
  for (size_t i = 0; i + 2 <= b->ev_used; i += 2) {
    float t = 0.f;
    BHIP_TRY(b, hipEventElapsedTime(&t, b->ev_pool[i], b->ev_pool[i + 1]));
    ms += t;
    n++;
    fr += b->ev_frames[i / 2];
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = n;
  if (frames) *frames = fr;
  if (reset) {
    b->ev_used = 0;
    b->ev_frames.clear();
  }
  return VCA_OK;
}

vca_status vca_reset_batch(vca_batch* b, int32_t stream) {
  if (!b || stream < -1 || stream >= b->n) return VCA_ERR_INVALID_ARG;
  for (int s = 0; s < b->n; s++)
    if (stream < 0 || s == stream) b->has_prev[s] = 0;
  return VCA_OK;
}

int64_t vca_batch_submitted(const vca_batch* b, int32_t stream) {
  if (!b || stream < 0 || stream >= b->n) return -1;
  return b->submitted[stream];
}

const char* vca_batch_last_error(const vca_batch* b) { return b ? b->err.c_str() : ""; }

}  // extern "C"
