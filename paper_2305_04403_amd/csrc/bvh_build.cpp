// Binned-SAH BVH builder with pre-order skip-index layout (see bvh_build.hpp).
#include "bvh_build.hpp"

#include <algorithm>
#include <cmath>
#include <limits>

namespace wobhost {

namespace {

constexpr int kBins = 32;
// SAH costs of visiting an interior node (one record: the two child boxes)
// and of one primitive test.  Measured on the 20,480-triangle icosphere
// benchmark, leaves of at most 4, primitive cost 0.5 / 0.75 / 1 / 1.5: 75.9 /
// 75.0 / 75.9 / 80.6 ms per solve (50 / 53 / 56 / 60 interior nodes and 23 /
// 17 / 14 / 11 triangles per line); leaves of at most 2, 0.5 / 0.75 / 1:
// 69.0 / 68.9 / 69.1 ms.
constexpr double kNodeCost = 1.0;
constexpr double kPrimCost = 0.75;
// Below this depth subtrees are split at the centroid median, which bounds
// the depth by kSahDepth + log2(n) whatever the geometry (the traversal stack
// holds one entry per level; 32 + 26 levels keep it under 64 entries).
constexpr int32_t kSahDepth = 32;

void grow(Box& b, const Box& o) {
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = std::min(b.lo[a], o.lo[a]);
    b.hi[a] = std::max(b.hi[a], o.hi[a]);
  }
}

Box empty_box() {
  Box b;
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = std::numeric_limits<double>::infinity();
    b.hi[a] = -std::numeric_limits<double>::infinity();
  }
  return b;
}

struct Builder {
  int dim;
  int max_leaf;
  const std::vector<Box>& boxes;
  std::vector<double> cen;  // centroid per primitive, 3 per entry
  Bvh out;

  Builder(int d, int ml, const std::vector<Box>& b) : dim(d), max_leaf(ml), boxes(b) {
    cen.resize(3 * b.size());
    for (size_t i = 0; i < b.size(); ++i)
      for (int a = 0; a < 3; ++a) cen[3 * i + a] = 0.5 * (b[i].lo[a] + b[i].hi[a]);
  }

  void make_leaf(int32_t idx, int32_t first, int32_t count) {
    FlatNode& n = out.nodes[idx];
    n.first = first;
    n.count = count;
    n.child = -1 - ((first << 3) | (count - 1));
    out.max_leaf = std::max(out.max_leaf, count);
    out.n_leaves += 1;
  }

  void build(int32_t first, int32_t count, int32_t depth) {
    const int32_t idx = (int32_t)out.nodes.size();
    out.nodes.push_back(FlatNode{});
    out.depth = std::max(out.depth, depth);
    Box nb = empty_box(), cb = empty_box();
    for (int32_t i = first; i < first + count; ++i) {
      const int32_t p = out.order[i];
      grow(nb, boxes[p]);
      Box c;
      for (int a = 0; a < 3; ++a) c.lo[a] = c.hi[a] = cen[3 * p + a];
      grow(cb, c);
    }
    out.nodes[idx].box = nb;
    out.nodes[idx].count = 0;

    if (count == 1) {
      make_leaf(idx, first, count);
      out.nodes[idx].skip = (int32_t)out.nodes.size();
      return;
    }

    if (depth >= kSahDepth && count > max_leaf) {
      int axis = 0;
      for (int a = 1; a < dim; ++a)
        if (cb.hi[a] - cb.lo[a] > cb.hi[axis] - cb.lo[axis]) axis = a;
      auto* beg = out.order.data() + first;
      const int32_t half = count / 2;
      std::nth_element(beg, beg + half, beg + count,
                       [&](int32_t p, int32_t q) { return cen[3 * p + axis] < cen[3 * q + axis]; });
      out.nodes[idx].child = idx + 1;
      build(first, half, depth + 1);
      build(first + half, count - half, depth + 1);
      out.nodes[idx].skip = (int32_t)out.nodes.size();
      return;
    }

    // binned SAH over every axis
    const double parent = std::max(box_measure(nb, dim), 1e-300);
    double best_cost = std::numeric_limits<double>::infinity();
    int best_axis = -1, best_split = -1;
    for (int a = 0; a < dim; ++a) {
      const double ext = cb.hi[a] - cb.lo[a];
      if (!(ext > 0.0)) continue;
      int cnt[kBins] = {0};
      Box bb[kBins];
      for (int k = 0; k < kBins; ++k) bb[k] = empty_box();
      const double scale = kBins / ext;
      for (int32_t i = first; i < first + count; ++i) {
        const int32_t p = out.order[i];
        int k = (int)((cen[3 * p + a] - cb.lo[a]) * scale);
        k = std::min(std::max(k, 0), kBins - 1);
        cnt[k] += 1;
        grow(bb[k], boxes[p]);
      }
      double right_area[kBins];
      int right_cnt[kBins];
      Box acc = empty_box();
      int c = 0;
      for (int k = kBins - 1; k > 0; --k) {
        grow(acc, bb[k]);
        c += cnt[k];
        right_area[k] = c ? box_measure(acc, dim) : 0.0;
        right_cnt[k] = c;
      }
      acc = empty_box();
      c = 0;
      for (int k = 1; k < kBins; ++k) {
        grow(acc, bb[k - 1]);
        c += cnt[k - 1];
        if (c == 0 || right_cnt[k] == 0) continue;
        const double cost = kNodeCost + kPrimCost *
                                            (box_measure(acc, dim) * c + right_area[k] * right_cnt[k]) /
                                            parent;
        if (cost < best_cost) {
          best_cost = cost;
          best_axis = a;
          best_split = k;
        }
      }
    }

    const double leaf_cost = kPrimCost * count;
    int32_t mid = -1;
    if (best_axis >= 0 && (count > max_leaf || best_cost < leaf_cost)) {
      const double ext = cb.hi[best_axis] - cb.lo[best_axis];
      const double scale = kBins / ext;
      auto* beg = out.order.data() + first;
      auto* end = beg + count;
      auto* m = std::partition(beg, end, [&](int32_t p) {
        int k = (int)((cen[3 * p + best_axis] - cb.lo[best_axis]) * scale);
        k = std::min(std::max(k, 0), kBins - 1);
        return k < best_split;
      });
      mid = (int32_t)(m - out.order.data());
    } else if (count > max_leaf) {
      // centroids coincide on every axis: split the list in half
      mid = first + count / 2;
    }

    if (mid < 0 || mid == first || mid == first + count) {
      if (count <= max_leaf) {
        make_leaf(idx, first, count);
        out.nodes[idx].skip = (int32_t)out.nodes.size();
        return;
      }
      mid = first + count / 2;
    }
    out.nodes[idx].child = idx + 1;
    build(first, mid - first, depth + 1);
    build(mid, first + count - mid, depth + 1);
    out.nodes[idx].skip = (int32_t)out.nodes.size();
  }
};

}  // namespace

double box_measure(const Box& b, int dim) {
  const double dx = b.hi[0] - b.lo[0], dy = b.hi[1] - b.lo[1];
  if (dim == 2) return 2.0 * (dx + dy);
  const double dz = b.hi[2] - b.lo[2];
  return 2.0 * (dx * dy + dy * dz + dz * dx);
}

Bvh build_bvh(int dim, const std::vector<Box>& prim_boxes, int max_leaf) {
  Builder b(dim, std::min(std::max(max_leaf, 1), 8), prim_boxes);
  const int32_t n = (int32_t)prim_boxes.size();
  b.out.order.resize(n);
  for (int32_t i = 0; i < n; ++i) b.out.order[i] = i;
  b.out.nodes.reserve(2 * (size_t)n);
  if (n > 0) b.build(0, n, 1);
  return std::move(b.out);
}

}  // namespace wobhost
