// Host-side bounding-volume hierarchy for all-hits line queries.
//
// The paper only asks for an "all-hits" ray query over the boundary
// (Sec. 4.4.1); the acceleration structure is this library's own design: a
// binary BVH built with the binned surface-area heuristic and laid out in
// pre-order with a skip ("escape") index per node.  The device records are
// derived from it (wob.hip: 4-wide interior records with binary16 boxes,
// walked with a short per-lane stack; a line query visits every box it
// meets and needs no front-to-back order).
#pragma once

#include <cstdint>
#include <vector>

namespace wobhost {

struct Box {
  double lo[3];
  double hi[3];
};

struct FlatNode {
  Box box;
  int32_t skip;   // first node after this subtree (n_nodes at the end)
  int32_t child;  // >= 0: first child (interior); < 0: leaf code -1 - ((first << 3) | (count - 1))
  int32_t first;  // leaf: first entry of `order`
  int32_t count;  // leaf: number of primitives (<= 8); 0 for interior nodes
};

struct Bvh {
  std::vector<FlatNode> nodes;
  std::vector<int32_t> order;  // leaf order -> original primitive id
  int32_t depth = 0;
  int32_t max_leaf = 0;
  int64_t n_leaves = 0;
};

// Measure of the lines meeting a convex set is proportional to its surface
// area (3D) or perimeter (2D) (Cauchy-Crofton), so the SAH weights children by it.
double box_measure(const Box& b, int dim);

// Build over primitive boxes (dim 2 or 3). max_leaf <= 8.
Bvh build_bvh(int dim, const std::vector<Box>& prim_boxes, int max_leaf);

}  // namespace wobhost
