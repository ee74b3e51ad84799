// Host-side check of the pair kernel's block -> work-item order (estep.hip,
// item_order): a bijection on the items of a problem; block i (run on XCD
// i mod 8) gets the x-th contiguous run of items; with c items per group the
// blocks of one XCD take, within a segment of groups, every group's first
// item, then every group's second, and so on.  Built and run by
// test_item_order.py; prints "ok" or the first failure.
#include "estep.hip"

#include <cstdio>
#include <vector>

int main() {
  using lsg::item_order;
  const int cases[][2] = {{1, 1},   {7, 1},    {8, 1},    {100, 1},  {391, 21}, {157, 26},
                          {16, 1},  {3, 5},    {1, 7},    {100, 3},  {8, 100},  {1000, 9},
                          {5, 4},   {64, 128}, {33, 33},  {2047, 3}, {12, 0}};
  for (const auto &cs : cases) {
    const int ng = cs[0], c = cs[1];
    const int n = c > 0 ? ng * c : ng;  // c = 0: groups of different item counts
    std::vector<int> seen(n, 0), at(n);
    for (int i = 0; i < n; ++i) {
      const int t = item_order(i, n, c);
      if (t < 0 || t >= n) return printf("n %d c %d: block %d -> item %d out of range\n", n, c, i, t), 1;
      if (seen[t]++) return printf("n %d c %d: item %d taken twice\n", n, c, t), 1;
      at[i] = t;
    }
    // each XCD's blocks cover one contiguous run of items
    for (int x = 0; x < 8 && c <= 1; ++x) {
      int lo = n, hi = -1, cnt = 0;
      for (int i = x; i < n; i += 8) {
        lo = at[i] < lo ? at[i] : lo;
        hi = at[i] > hi ? at[i] : hi;
        ++cnt;
      }
      if (cnt > 0 && hi - lo + 1 != cnt) return printf("n %d: XCD %d's items not contiguous\n", n, x), 1;
    }
    // chunk-major: consecutive blocks of an XCD take the same item of
    // consecutive groups, or move on to the next item of the segment's first
    if (c > 1) {
      for (int x = 0; x < 8; ++x)
        for (int i = x; i + 8 < n; i += 8) {
          const int a = at[i], b = at[i + 8];
          const bool next_group = b / c == a / c + 1 && b % c == a % c;
          const bool next_item = b % c == a % c + 1;
          const bool new_run = b / c > a / c;  // the XCD's run moved on
          if (!next_group && !next_item && !new_run)
            return printf("n %d c %d: blocks %d, %d -> items %d, %d\n", n, c, i, i + 8, a, b), 1;
        }
    }
  }
  printf("ok\n");
  return 0;
}
