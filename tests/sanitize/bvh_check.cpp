// Host BVH builder under AddressSanitizer / UndefinedBehaviorSanitizer
// (test infrastructure): builds trees over seeded random and degenerate box
// sets and checks the structure: every primitive in exactly one leaf, leaf
// sizes within max_leaf, each node's box containing its primitives' boxes,
// skip indices past the node's subtree.  Prints "ok" and exits 0, or
// reports the first violation and exits 1.
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <random>
#include <vector>

#include "../../paper_2305_04403_amd/csrc/bvh_build.hpp"

using wobhost::Box;

static bool contains(const Box& outer, const Box& inner, int dim) {
  for (int a = 0; a < dim; ++a)
    if (inner.lo[a] < outer.lo[a] || inner.hi[a] > outer.hi[a]) return false;
  return true;
}

static int check(int dim, const std::vector<Box>& boxes, int max_leaf, const char* name) {
  const wobhost::Bvh b = wobhost::build_bvh(dim, boxes, max_leaf);
  const int64_t n = (int64_t)boxes.size(), nn = (int64_t)b.nodes.size();
  std::vector<int> seen(n, 0);
  if ((int64_t)b.order.size() != n) {
    std::printf("%s: order has %zu entries for %lld primitives\n", name, b.order.size(), (long long)n);
    return 1;
  }
  for (int64_t i = 0; i < nn; ++i) {
    const wobhost::FlatNode& f = b.nodes[i];
    if (f.skip <= i || f.skip > nn) {
      std::printf("%s: node %lld skip %d\n", name, (long long)i, f.skip);
      return 1;
    }
    if (f.child < 0) {
      if (f.count < 1 || f.count > max_leaf || f.first < 0 || f.first + f.count > n) {
        std::printf("%s: leaf %lld first %d count %d\n", name, (long long)i, f.first, f.count);
        return 1;
      }
      for (int j = f.first; j < f.first + f.count; ++j) {
        const int32_t id = b.order[j];
        if (id < 0 || id >= n) {
          std::printf("%s: order entry %d = %d\n", name, j, id);
          return 1;
        }
        ++seen[id];
        if (!contains(f.box, boxes[id], dim)) {
          std::printf("%s: leaf %lld box misses primitive %d\n", name, (long long)i, id);
          return 1;
        }
      }
    } else if (f.child != i + 1 || f.child >= nn || !contains(f.box, b.nodes[f.child].box, dim)) {
      std::printf("%s: interior %lld child %d\n", name, (long long)i, f.child);
      return 1;
    }
  }
  for (int64_t id = 0; id < n; ++id)
    if (seen[id] != 1) {
      std::printf("%s: primitive %lld in %d leaves\n", name, (long long)id, seen[id]);
      return 1;
    }
  return 0;
}

int main() {
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> u(-1.0, 1.0), s(0.0, 0.05);
  int bad = 0;
  for (int dim = 2; dim <= 3; ++dim) {
    for (int n : {1, 2, 3, 7, 8, 9, 64, 1000, 5000}) {
      std::vector<Box> boxes(n);
      for (Box& b : boxes) {
        for (int a = 0; a < 3; ++a) {
          const double c = a < dim ? u(rng) : 0.0, h = a < dim ? s(rng) : 0.0;
          b.lo[a] = c - h;
          b.hi[a] = c + h;
        }
      }
      char name[64];
      std::snprintf(name, sizeof(name), "random dim %d n %d", dim, n);
      bad |= check(dim, boxes, 8, name);
      bad |= check(dim, boxes, 1, name);
    }
    // every box identical (no split separates them)
    std::vector<Box> same(500);
    for (Box& b : same)
      for (int a = 0; a < 3; ++a) {
        b.lo[a] = a < dim ? 0.25 : 0.0;
        b.hi[a] = a < dim ? 0.5 : 0.0;
      }
    bad |= check(dim, same, 8, "identical boxes");
    // a staircase: boxes along a line with doubling gaps (a deep tree)
    std::vector<Box> stair(300);
    for (int i = 0; i < 300; ++i)
      for (int a = 0; a < 3; ++a) {
        const double c = a == 0 ? std::ldexp(1.0, i / 10) * (1.0 + 0.01 * i) : 0.0;
        stair[i].lo[a] = c;
        stair[i].hi[a] = a < dim ? c + 0.001 : 0.0;
      }
    bad |= check(dim, stair, 8, "staircase");
    // flat boxes (zero extent on one axis): a mesh face parallel to an axis
    std::vector<Box> flat(2000);
    for (Box& b : flat)
      for (int a = 0; a < 3; ++a) {
        const double c = a == 0 ? 0.0 : (a < dim ? u(rng) : 0.0);
        b.lo[a] = c;
        b.hi[a] = a == 0 ? c : c + (a < dim ? s(rng) : 0.0);
      }
    bad |= check(dim, flat, 8, "flat boxes");
  }
  if (!bad) std::printf("ok\n");
  return bad;
}
