// Host-side check of the ingest helpers (paper_2304_12384_amd/csrc/vca_ingest.h),
// built by tests/test_host_sanitizers.py with AddressSanitizer + UBSan and with
// ThreadSanitizer: raw I420 frames read in row bands split over 1..8 parts
// (the parts run on a WorkerPool, as host ingest runs them), into tight and
// pitched destinations, and row-band copies between pitched buffers; every
// byte is compared with the file, and a short file must be reported.
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <vector>
#include <fcntl.h>
#include <unistd.h>

#include "../../paper_2304_12384_amd/csrc/vca_ingest.h"

using namespace vca;

static int fail(const char* what) {
  std::fprintf(stderr, "FAIL: %s\n", what);
  return 1;
}

int main() {
  WorkerPool pool(4);
  const int W = 328, H = 202, n = 5;
  for (int bits : {8, 10}) {
    const YuvLayout L = YuvLayout::of(W, H, bits);
    std::vector<uint8_t> file((size_t)L.frame * n);
    for (size_t i = 0; i < file.size(); i++) file[i] = (uint8_t)((i * 2654435761u) >> 11);
    char path[] = "/tmp/vca_ingest_checkXXXXXX";
    const int wfd = mkstemp(path);
    if (wfd < 0 || write(wfd, file.data(), file.size()) != (ssize_t)file.size()) return fail("write");
    close(wfd);
    if (yuv_frames_in_file(path, L) != n) return fail("frame count");
    const int fd = open(path, O_RDONLY);
    for (int pad : {0, 48}) {                       // tight and pitched destinations
      const int64_t py = L.row_y + pad, pc = L.row_uv + pad;
      for (int first = 0; first < n; first++)
        for (int cnt = 1; first + cnt <= n; cnt++)
          for (int parts = 1; parts <= 8; parts++) {
            std::vector<uint8_t> y((size_t)py * L.rows_y * cnt, 0xEE), u((size_t)pc * L.rows_uv * cnt, 0xEE),
                v((size_t)pc * L.rows_uv * cnt, 0xEE);
            const PlanarDst d{y.data(), u.data(), v.data(), py, pc, py * L.rows_y, pc * L.rows_uv};
            std::vector<char> ok(parts, 0);
            const std::function<void(int)> job = [&](int i) {
              for (int p = i; p < parts; p += pool.size()) ok[p] = read_yuv_part(fd, L, first, cnt, d, p, parts);
            };
            pool.run(job);
            for (char o : ok)
              if (!o) return fail("read_yuv_part");
            for (int t = 0; t < cnt; t++) {
              const uint8_t* src = file.data() + (size_t)(first + t) * L.frame;
              for (int64_t r = 0; r < L.rows_y; r++)
                if (std::memcmp(y.data() + t * py * L.rows_y + r * py, src + r * L.row_y, L.row_y)) return fail("Y");
              for (int64_t r = 0; r < L.rows_uv; r++) {
                if (std::memcmp(u.data() + t * pc * L.rows_uv + r * pc, src + L.plane_y + r * L.row_uv, L.row_uv))
                  return fail("U");
                if (std::memcmp(v.data() + t * pc * L.rows_uv + r * pc, src + L.plane_y + L.plane_uv + r * L.row_uv,
                                L.row_uv))
                  return fail("V");
              }
              for (int64_t r = 0; r < L.rows_y && pad; r++)
                for (int k = 0; k < pad; k++)
                  if (y[t * py * L.rows_y + r * py + L.row_y + k] != 0xEE) return fail("Y padding written");
            }
          }
    }
    // frames past the end of the file: a short read
    {
      std::vector<uint8_t> y((size_t)L.plane_y * 2), u((size_t)L.plane_uv * 2), v((size_t)L.plane_uv * 2);
      const PlanarDst d{y.data(), u.data(), v.data(), L.row_y, L.row_uv, L.plane_y, L.plane_uv};
      if (read_yuv_part(fd, L, n - 1, 2, d, 0, 1)) return fail("short read not reported");
    }
    close(fd);
    unlink(path);
    // row-band copies between pitched buffers
    for (int parts = 1; parts <= 8; parts++) {
      const int64_t rows = 37, row = 100, sp = 128, dp = 112;
      std::vector<uint8_t> src(sp * rows), dst(dp * rows, 0);
      for (size_t i = 0; i < src.size(); i++) src[i] = (uint8_t)(i * 7 + 3);
      for (int p = 0; p < parts; p++) {
        int64_t r0, r1;
        band(rows, p, parts, r0, r1);
        copy_rows(dst.data(), dp, src.data(), sp, row, r0, r1);
      }
      for (int64_t r = 0; r < rows; r++)
        if (std::memcmp(dst.data() + r * dp, src.data() + r * sp, row)) return fail("copy_rows");
    }
  }
  std::puts("ingest check ok");
  return 0;
}
