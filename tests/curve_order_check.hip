// Host-side check of the point order's curve key (order.hip): the keys form a
// Hilbert curve through the 2^10 x 2^10 x 2^10 grid.  Built and run by
// test_curve_order.py; prints "ok" or the first failure.
#include "order.hip"

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

int main() {
  using lsg::hilbert_key;
  const uint32_t last = (1u << 30) - 1;
  // the curve runs from the origin to the far end of the x axis
  if (hilbert_key(0, 0, 0) != 0u) return printf("key(0,0,0) = %u\n", hilbert_key(0, 0, 0)), 1;
  if (hilbert_key(1023, 0, 0) != last) return printf("key(1023,0,0) is not the last key\n"), 1;
  // the first 2^18 keys fill the 64^3 cube at the origin, each once
  std::vector<uint32_t> keys;
  keys.reserve(1u << 18);
  for (uint32_t x = 0; x < 64; ++x)
    for (uint32_t y = 0; y < 64; ++y)
      for (uint32_t z = 0; z < 64; ++z) keys.push_back(hilbert_key(x, y, z));
  std::sort(keys.begin(), keys.end());
  for (uint32_t i = 0; i < keys.size(); ++i)
    if (keys[i] != i) return printf("64^3 corner: key %u at rank %u\n", keys[i], i), 1;
  // consecutive keys are face neighbours: of the six face neighbours of a
  // cell with key k, one has key k - 1 and one key k + 1 (at the ends, one)
  std::mt19937 rng(12345);
  std::uniform_int_distribution<uint32_t> u(0, 1023);
  const int d[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
  for (int s = 0; s < 1000000; ++s) {
    const uint32_t c[3] = {u(rng), u(rng), u(rng)};
    const uint32_t k = hilbert_key(c[0], c[1], c[2]);
    int prev = 0, next = 0;
    for (const auto &o : d) {
      const int64_t a = (int64_t)c[0] + o[0], b = (int64_t)c[1] + o[1], e = (int64_t)c[2] + o[2];
      if (a < 0 || b < 0 || e < 0 || a > 1023 || b > 1023 || e > 1023) continue;
      const uint32_t kn = hilbert_key((uint32_t)a, (uint32_t)b, (uint32_t)e);
      prev += k > 0 && kn == k - 1;
      next += k < last && kn == k + 1;
    }
    if (prev != (k > 0 ? 1 : 0) || next != (k < last ? 1 : 0))
      return printf("cell (%u,%u,%u) key %u: %d / %d neighbours with key -1 / +1\n", c[0], c[1],
                    c[2], k, prev, next),
             1;
  }
  printf("ok\n");
  return 0;
}
