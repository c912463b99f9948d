// vca_ingest.h -- host side of host-resident frame ingest: planar 4:2:0
// frame layouts, a raw .yuv file reader, and a small worker pool that fills
// pinned staging buffers in parallel.  No device code.
#pragma once

#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace vca {

// One frame's planes as stored in a raw .yuv file (I420: Y rows, then U,
// then V, rows without padding; 10-bit samples as little-endian uint16).
struct YuvLayout {
  int64_t row_y, row_uv;     // bytes per row
  int64_t rows_y, rows_uv;   // rows per plane
  int64_t plane_y, plane_uv; // bytes per plane
  int64_t frame;             // bytes per frame

  static YuvLayout of(int32_t width, int32_t height, int32_t bit_depth) {
    const int64_t bps = bit_depth == 8 ? 1 : 2;
    YuvLayout l;
    l.row_y = width * bps;
    l.row_uv = (width / 2) * bps;
    l.rows_y = height;
    l.rows_uv = height / 2;
    l.plane_y = l.row_y * l.rows_y;
    l.plane_uv = l.row_uv * l.rows_uv;
    l.frame = l.plane_y + 2 * l.plane_uv;
    return l;
  }
};

// Where the planes of frame i of a batch live in memory.
struct PlanarDst {
  uint8_t* y;
  uint8_t* u;
  uint8_t* v;
  int64_t pitch_y, pitch_uv;       // bytes between rows
  int64_t fstride_y, fstride_uv;   // bytes between frames
};

// Runs f(0 .. size-1) on a fixed set of threads (f(0) on the caller) and
// waits for all of them.  Not reentrant; one pool per context.
class WorkerPool {
 public:
  explicit WorkerPool(int n) : n_(std::max(1, n)) {
    for (int i = 1; i < n_; i++) threads_.emplace_back([this, i] { loop(i); });
  }
  ~WorkerPool() {
    {
      std::lock_guard<std::mutex> lock(m_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : threads_) t.join();
  }
  WorkerPool(const WorkerPool&) = delete;
  WorkerPool& operator=(const WorkerPool&) = delete;

  int size() const { return n_; }

  void run(const std::function<void(int)>& f) {
    {
      std::lock_guard<std::mutex> lock(m_);
      job_ = &f;
      pending_ = n_ - 1;
      gen_++;
    }
    cv_.notify_all();
    f(0);
    std::unique_lock<std::mutex> lock(m_);
    done_.wait(lock, [this] { return pending_ == 0; });
    job_ = nullptr;
  }

 private:
  void loop(int i) {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(int)>* f;
      {
        std::unique_lock<std::mutex> lock(m_);
        cv_.wait(lock, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
        f = job_;
      }
      (*f)(i);
      {
        std::lock_guard<std::mutex> lock(m_);
        if (--pending_ == 0) done_.notify_one();
      }
    }
  }

  int n_;
  std::vector<std::thread> threads_;
  std::mutex m_;
  std::condition_variable cv_, done_;
  const std::function<void(int)>* job_ = nullptr;
  int pending_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};

// Row band [r0, r1) of `rows` split `parts` ways.
inline void band(int64_t rows, int part, int parts, int64_t& r0, int64_t& r1) {
  r0 = rows * part / parts;
  r1 = rows * (part + 1) / parts;
}

// Copies rows [r0, r1) of a plane (src pitch sp) to dst (pitch dp), `row`
// bytes each.
inline void copy_rows(uint8_t* dst, int64_t dp, const uint8_t* src, int64_t sp, int64_t row,
                      int64_t r0, int64_t r1) {
  if (r1 <= r0) return;
  if (dp == row && sp == row) {
    std::memcpy(dst + r0 * row, src + r0 * row, (size_t)((r1 - r0) * row));
    return;
  }
  for (int64_t r = r0; r < r1; r++) std::memcpy(dst + r * dp, src + r * sp, (size_t)row);
}

// Reads rows [r0, r1) of one plane from fd at byte offset `off` (tight rows
// in the file) into dst with pitch dp.  Returns false on a short read.
inline bool pread_rows(int fd, int64_t off, uint8_t* dst, int64_t dp, int64_t row, int64_t r0,
                       int64_t r1) {
  auto read_all = [&](uint8_t* p, int64_t n, int64_t at) {
    while (n > 0) {
      const ssize_t got = ::pread(fd, p, (size_t)n, (off_t)at);
      if (got < 0 && errno == EINTR) continue;
      if (got <= 0) return false;
      p += got;
      n -= got;
      at += got;
    }
    return true;
  };
  if (r1 <= r0) return true;
  if (dp == row) return read_all(dst + r0 * row, (r1 - r0) * row, off + r0 * row);
  for (int64_t r = r0; r < r1; r++)
    if (!read_all(dst + r * dp, row, off + r * row)) return false;
  return true;
}

// Reads frames [first, first + n) of an open .yuv file into dst, split over
// `parts` row bands (part `part` of them).  Returns false on a short read.
inline bool read_yuv_part(int fd, const YuvLayout& L, int64_t first, int32_t n, const PlanarDst& d,
                          int part, int parts) {
  int64_t y0, y1, c0, c1;
  band(L.rows_y, part, parts, y0, y1);
  band(L.rows_uv, part, parts, c0, c1);
  for (int32_t i = 0; i < n; i++) {
    const int64_t base = (first + i) * L.frame;
    if (!pread_rows(fd, base, d.y + i * d.fstride_y, d.pitch_y, L.row_y, y0, y1)) return false;
    if (!pread_rows(fd, base + L.plane_y, d.u + i * d.fstride_uv, d.pitch_uv, L.row_uv, c0, c1))
      return false;
    if (!pread_rows(fd, base + L.plane_y + L.plane_uv, d.v + i * d.fstride_uv, d.pitch_uv, L.row_uv,
                    c0, c1))
      return false;
  }
  return true;
}

// Frames in the file at `path`, or -1 if it cannot be opened.
inline int64_t yuv_frames_in_file(const char* path, const YuvLayout& L) {
  struct stat st;
  if (::stat(path, &st) != 0) return -1;
  return (int64_t)st.st_size / L.frame;
}

inline int ingest_threads() {
  const unsigned hw = std::thread::hardware_concurrency();
  return (int)std::min<unsigned>(8, std::max<unsigned>(1, hw / 2));
}

}  // namespace vca
