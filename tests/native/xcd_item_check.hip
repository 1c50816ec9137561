// Host-side check of the persistent-grid item walk (xcd_item): for every grid
// size G and item count `total` in the ranges given on the command line, the
// workgroups 0..G-1 visit every item in [0, total) exactly once.  Prints the
// number of failing (G, total) pairs and exits non-zero if there is any.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "mhd_fft.h"

int main(int argc, char** argv) {
  const int gmax = argc > 1 ? std::atoi(argv[1]) : 64;
  const int tmax = argc > 2 ? std::atoi(argv[2]) : 300;
  int bad = 0;
  for (int G = 1; G <= gmax; ++G) {
    for (int total = 0; total <= tmax; ++total) {
      std::vector<int> seen(total, 0);
      bool ok = true;
      for (int w = 0; w < G && ok; ++w) {
        for (int64_t k = 0;; ++k) {
          const int64_t it = mhd::xcd_item(w, G, k, total);
          if (it < 0) break;
          if (it >= total) { ok = false; break; }
          ++seen[it];
        }
      }
      for (int i = 0; i < total && ok; ++i) ok = seen[i] == 1;
      if (!ok) {
        if (bad < 10) std::printf("G=%d total=%d: items missed or repeated\n", G, total);
        ++bad;
      }
    }
  }
  std::printf("failing pairs: %d\n", bad);
  return bad ? 1 : 0;
}
