// Host-only check of the launch-shape cache file (VCA_TUNE_CACHE): lines of
// the current six-field form and of the older four-field form load, invalid
// shapes are dropped, and put() writes every entry back in the six-field
// form.  Run by tests/test_tune_cache_cpu.py; calls no HIP function.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "../../paper_2304_12384_amd/csrc/vca_host.h"

using vca::LaunchChoice;
using vca::TuneCache;

static int failures = 0;
#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      std::printf("FAILED line %d: %s\n", __LINE__, #cond);          \
      failures++;                                                     \
    }                                                                 \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  const char* path = argv[1];
  if (FILE* f = std::fopen(path, "w")) {
    std::fputs("plain/3840x2160 4 3 1.875000 0 0\n", f);    // six fields
    std::fputs("batch/k0 2 1 0.500000 8 16\n", f);          // six fields, batched shape
    std::fputs("old/key 2 2 1.250000\n", f);                // four fields (older files)
    std::fputs("bad/depth 5 1 1.0 0 0\n", f);               // depth outside 1..4
    std::fputs("bad/waves 2 1 1.0 6 8\n", f);               // waves neither 4 nor 8
    std::fputs("bad/chunk 2 1 1.0 4 12\n", f);              // chunk not a multiple of 8
    std::fputs("bad/fields 2 1\n", f);                      // too few fields
    std::fputs("\n", f);
    std::fclose(f);
  } else {
    return 2;
  }
  setenv("VCA_TUNE_CACHE", path, 1);
  TuneCache& c = TuneCache::get();
  LaunchChoice lc;
  CHECK(c.find("plain/3840x2160", &lc) && lc.depth == 4 && lc.groups_per_cu == 3 && lc.ms == 1.875 &&
        lc.waves == 0 && lc.chunk == 0);
  CHECK(c.find("batch/k0", &lc) && lc.depth == 2 && lc.groups_per_cu == 1 && lc.waves == 8 && lc.chunk == 16);
  CHECK(c.find("old/key", &lc) && lc.depth == 2 && lc.groups_per_cu == 2 && lc.ms == 1.25 && lc.waves == 0 &&
        lc.chunk == 0);
  CHECK(!c.find("bad/depth", &lc));
  CHECK(!c.find("bad/waves", &lc));
  CHECK(!c.find("bad/chunk", &lc));
  CHECK(!c.find("bad/fields", &lc));
  CHECK(!c.find("missing", &lc));
  // put() rewrites the file with every entry in the six-field form
  LaunchChoice n;
  n.depth = 1;
  n.groups_per_cu = 2;
  n.ms = 0.25;
  n.waves = 4;
  n.chunk = 32;
  c.put("new/key", n);
  CHECK(c.find("new/key", &lc) && lc.depth == 1 && lc.waves == 4 && lc.chunk == 32);
  FILE* f = std::fopen(path, "r");
  CHECK(f != nullptr);
  int lines = 0, six = 0;
  bool saw_old = false, saw_new = false;
  char line[512];
  while (f && std::fgets(line, sizeof(line), f)) {
    char key[256];
    int d, g, w, k;
    double ms;
    lines++;
    if (std::sscanf(line, "%255s %d %d %lf %d %d", key, &d, &g, &ms, &w, &k) == 6) six++;
    if (std::strncmp(line, "old/key 2 2 1.250000 0 0", 24) == 0) saw_old = true;
    if (std::strncmp(line, "new/key 1 2 0.250000 4 32", 25) == 0) saw_new = true;
  }
  if (f) std::fclose(f);
  CHECK(lines == 4 && six == 4);   // the three valid entries loaded and the new one
  CHECK(saw_old && saw_new);
  if (failures == 0) std::printf("tune cache check ok\n");
  return failures == 0 ? 0 : 1;
}
