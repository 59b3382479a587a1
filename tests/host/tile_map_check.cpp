// Host check of the compositing launches' block -> tile map: for every tile
// capacity in a range, the render_grid(total) blocks hit each tile index in
// [0, total) exactly once, every XCD (block % 8) receives a share of the
// tiles within one chunk of the others, and no block maps past its grid.
#include <cstdio>
#include <vector>

#include "blend.hpp"

int main() {
  for (int64_t total = 1; total <= 40000; total += (total < 2000 ? 1 : 97)) {
    const int64_t grid = pvg::render_grid(total);
    std::vector<int> hit(static_cast<size_t>(grid), 0);
    int64_t per_xcd[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t b = 0; b < grid; ++b) {
      const int64_t t = pvg::xcd_tile(b, total);
      if (t < 0 || t >= grid) { std::printf("total %lld: block %lld -> %lld outside the grid\n", (long long)total, (long long)b, (long long)t); return 1; }
      hit[static_cast<size_t>(t)]++;
      if (t < total) per_xcd[b & 7]++;
    }
    for (int64_t t = 0; t < grid; ++t)
      if (hit[static_cast<size_t>(t)] != 1) { std::printf("total %lld: tile %lld hit %d times\n", (long long)total, (long long)t, hit[static_cast<size_t>(t)]); return 1; }
    int64_t lo = per_xcd[0], hi = per_xcd[0];
    for (int x = 1; x < 8; ++x) { lo = per_xcd[x] < lo ? per_xcd[x] : lo; hi = per_xcd[x] > hi ? per_xcd[x] : hi; }
    if (hi - lo > pvg::xcd_chunk(total)) { std::printf("total %lld: XCD shares %lld..%lld\n", (long long)total, (long long)lo, (long long)hi); return 1; }
  }
  std::printf("tile map ok\n");
  return 0;
}
