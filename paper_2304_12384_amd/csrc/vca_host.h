// vca_host.h -- host-side helpers shared by the plain and batched paths:
// configuration checks, plane/tile geometry, device allocation, error
// reporting, and the launch-parameter autotuner's cache.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/vca.h"
#include "vca_reduce.h"
#include "vca_tile.h"

namespace vca {

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

inline vca_status check_config(const vca_config* cfg) {
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
  if (cfg->flags & ~(VCA_F_KEEP_COEFFS | VCA_F_VALIDATE | VCA_F_TIMING | VCA_F_DOWNSAMPLE))
    return VCA_ERR_INVALID_ARG;
  if (cfg->flags & VCA_F_DOWNSAMPLE) {
    if (cfg->width % 4 || cfg->height % 4 || cfg->width / 4 < w || cfg->height / 4 < w)
      return VCA_ERR_INVALID_ARG;
    if (k != 0 && k != w) return VCA_ERR_INVALID_ARG;
    if (cfg->flags & VCA_F_KEEP_COEFFS) return VCA_ERR_UNSUPPORTED;
  }
  return VCA_OK;
}

// Block and tile geometry of one video configuration.
struct Geometry {
  int w = 0, K = 0, bits = 0;
  int32_t nbx[3] = {0, 0, 0}, nby[3] = {0, 0, 0}, cnt[3] = {0, 0, 0};
  int32_t ntx[3] = {0, 0, 0}, tcnt[3] = {0, 0, 0}, boff[3] = {0, 0, 0};
  int32_t per_frame = 0;        // blocks per frame
  int32_t tiles_per_frame = 0;  // 32 x 32 tiles per frame

  bool ds = false;               // planes downsampled by two before the analysis

  void init(const vca_config& cfg) {
    w = cfg.block_size;
    K = cfg.lowpass_k == 0 ? w : cfg.lowpass_k;
    bits = cfg.bit_depth;
    ds = (cfg.flags & VCA_F_DOWNSAMPLE) != 0;
    const int vw = ds ? cfg.width / 2 : cfg.width, vh = ds ? cfg.height / 2 : cfg.height;
    const int bpt = kTile / w;
    per_frame = tiles_per_frame = 0;
    for (int P = 0; P < 3; P++) {
      const int pw = P == 0 ? vw : vw / 2;
      const int ph = P == 0 ? vh : vh / 2;
      nbx[P] = pw / w;
      nby[P] = ph / w;
      cnt[P] = nbx[P] * nby[P];
      ntx[P] = (nbx[P] + bpt - 1) / bpt;
      tcnt[P] = ntx[P] * ((nby[P] + bpt - 1) / bpt);
      boff[P] = per_frame;
      per_frame += cnt[P];
      tiles_per_frame += tcnt[P];
    }
  }
};

// Checks a frame descriptor against a configuration (16-byte alignment,
// pitches, strides).  Returns a message, or nullptr when the frames are valid.
inline const char* check_frames(const vca_config& cfg, const vca_frames* fr, int32_t n_frames) {
  const int bps = cfg.bit_depth == 8 ? 1 : 2;
  if (!fr->on_device) return "host-resident frames are not supported";
  if (!fr->y || !fr->u || !fr->v) return "null plane pointer";
  if (fr->pitch_y < (int64_t)cfg.width * bps || fr->pitch_uv < (int64_t)cfg.width / 2 * bps)
    return "pitch smaller than a row";
  if (fr->pitch_y >= (1 << 23) || fr->pitch_uv >= (1 << 23))
    return "pitch of 8 MiB or more";  // lane offsets are 24-bit products
  if (n_frames > 1 && (fr->fstride_y < fr->pitch_y * cfg.height ||
                       fr->fstride_uv < fr->pitch_uv * (cfg.height / 2)))
    return "frame stride smaller than a frame";
  const uintptr_t align = (uintptr_t)fr->y | (uintptr_t)fr->u | (uintptr_t)fr->v |
                          (uintptr_t)fr->pitch_y | (uintptr_t)fr->pitch_uv |
                          (uintptr_t)fr->fstride_y | (uintptr_t)fr->fstride_uv;
  if (align & 15) return "planes, pitches and strides need 16-byte alignment";
  return nullptr;
}

// Host-resident frames (vca_frames.on_device == 0): any alignment, the
// same row and frame-stride rules.  nullptr when valid.
inline const char* check_host_frames(const vca_config& cfg, const vca_frames* fr, int32_t n_frames) {
  const int bps = cfg.bit_depth == 8 ? 1 : 2;
  if (fr->on_device) return "device frames";
  if (!fr->y || !fr->u || !fr->v) return "null plane pointer";
  if (fr->pitch_y < (int64_t)cfg.width * bps || fr->pitch_uv < (int64_t)cfg.width / 2 * bps)
    return "pitch smaller than a row";
  if (n_frames > 1 && (fr->fstride_y < fr->pitch_y * cfg.height ||
                       fr->fstride_uv < fr->pitch_uv * (cfg.height / 2)))
    return "frame stride smaller than a frame";
  return nullptr;
}

// Pinned host memory the device reads and writes directly (fine-grained,
// mapped), zeroed: the feature rings and error flags live there, so reading
// features after a stream synchronisation is a host memcpy, not a device
// copy per call.  Freed with hipHostFree(*host).
inline hipError_t host_mapped_alloc(size_t bytes, void** host, void** dev) {
  hipError_t e = hipHostMalloc(host, bytes ? bytes : 1, hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) return e;
  std::memset(*host, 0, bytes ? bytes : 1);
  return hipHostGetDevicePointer(dev, *host, 0);
}

// Completion marks of the most recent launches on one stream.  After each
// launch an event is recorded together with, per video stream, the number of
// frames submitted up to and including that launch; a feature read then waits
// for the oldest launch that covers the frames it asks for instead of
// draining the whole stream, so a caller can queue the next batch before
// reading the last one.  A read older than every remembered mark waits for
// the oldest remembered launch (later than needed, never earlier).
class DoneMarks {
 public:
  static constexpr int kMarks = 16;

  hipError_t init(int n_streams) {
    n_ = n_streams;
    end_.assign((size_t)kMarks * n_streams, 0);
    for (int i = 0; i < kMarks; i++) {
      hipError_t e = hipEventCreateWithFlags(&ev_[i], hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  void destroy() {
    for (hipEvent_t& e : ev_)
      if (e) {
        (void)hipEventDestroy(e);
        e = nullptr;
      }
  }
  // ends[s]: frames of stream s submitted up to and including the launch
  // just enqueued on `stream`.
  hipError_t record(hipStream_t stream, const int64_t* ends) {
    const int i = next_;
    hipError_t e = hipEventRecord(ev_[i], stream);
    if (e != hipSuccess) return e;
    std::copy(ends, ends + n_, end_.begin() + (size_t)i * n_);
    next_ = (next_ + 1) % kMarks;
    used_ = std::min(used_ + 1, kMarks);
    return hipSuccess;
  }
  // Age rank (0 = oldest remembered) of the oldest launch after which every
  // frame of stream s below `upto` has been written, or kMarks if no
  // remembered launch covers it.
  int cover(int s, int64_t upto) const {
    for (int k = 0; k < used_; k++)
      if (end_[(size_t)slot(k) * n_ + s] >= upto) return k;
    return kMarks;
  }
  // Blocks until the launch of age rank k has completed (k = kMarks: until
  // the stream drains).  Launches complete in order, so this also covers
  // every older one.
  hipError_t wait_rank(int k, hipStream_t stream) const {
    if (k >= used_) return hipStreamSynchronize(stream);
    return hipEventSynchronize(ev_[slot(k)]);
  }
  // Blocks until every frame of stream s below `upto` has been written.
  hipError_t wait(int s, int64_t upto, hipStream_t stream) const {
    return wait_rank(cover(s, upto), stream);
  }

 private:
  int slot(int k) const { return (next_ - used_ + k + kMarks) % kMarks; }
  int n_ = 0;
  hipEvent_t ev_[kMarks] = {};
  std::vector<int64_t> end_;
  int next_ = 0, used_ = 0;
};

// Launch parameters chosen by the autotuner (depth 0 = not tuned).
struct LaunchChoice {
  int depth = 0;          // work units in flight per wavefront (1..4)
  int groups_per_cu = 0;  // 0: as many as fit
  double ms = 0.0;
  int waves = 0;          // batched form: wavefronts per workgroup (0: the default)
  int chunk = 0;          // batched form: strips per chunk (0: the default)
};

// Process-wide cache of tuned launch choices, optionally persisted to the
// text file named by VCA_TUNE_CACHE (one "key depth groups ms [waves chunk]"
// per line).
class TuneCache {
 public:
  static TuneCache& get() {
    static TuneCache c;
    return c;
  }
  bool find(const std::string& key, LaunchChoice* out) {
    std::lock_guard<std::mutex> lk(mu_);
    load_once();
    auto it = map_.find(key);
    if (it == map_.end()) return false;
    *out = it->second;
    return true;
  }
  void put(const std::string& key, const LaunchChoice& c) {
    std::lock_guard<std::mutex> lk(mu_);
    load_once();
    map_[key] = c;
    const char* path = std::getenv("VCA_TUNE_CACHE");
    if (!path || !*path) return;
    if (FILE* f = std::fopen(path, "w")) {
      for (const auto& kv : map_)
        std::fprintf(f, "%s %d %d %.6f %d %d\n", kv.first.c_str(), kv.second.depth,
                     kv.second.groups_per_cu, kv.second.ms, kv.second.waves, kv.second.chunk);
      std::fclose(f);
    }
  }

 private:
  void load_once() {
    if (loaded_) return;
    loaded_ = true;
    const char* path = std::getenv("VCA_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512], key[256];
    while (std::fgets(line, sizeof(line), f)) {
      LaunchChoice c;
      const int n = std::sscanf(line, "%255s %d %d %lf %d %d", key, &c.depth, &c.groups_per_cu, &c.ms,
                                &c.waves, &c.chunk);
      if (n != 4 && n != 6) continue;
      if (n == 4) c.waves = c.chunk = 0;
      if (c.depth >= 1 && c.depth <= 4 && c.groups_per_cu >= 0 && (c.waves == 0 || c.waves == 4 || c.waves == 8) &&
          c.chunk >= 0 && c.chunk <= 1024 && c.chunk % 8 == 0)
        map_[key] = c;
    }
    std::fclose(f);
  }
  std::mutex mu_;
  bool loaded_ = false;
  std::map<std::string, LaunchChoice> map_;
};

}  // namespace vca
