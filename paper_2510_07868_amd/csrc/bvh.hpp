// Host BVH builder interface.
#pragma once
#include <stdint.h>

#include <vector>

#include "bvh_layout.hpp"

namespace nrrs {

struct BvhOut {
  std::vector<float> nodes;      // 16 floats per node: child0 lo/hi, child1 lo/hi, links
  std::vector<uint32_t> order;   // BVH position -> original triangle index
  uint64_t n_nodes = 0;
  int max_depth = 0;             // levels from the root to the deepest leaf
  // The same tree collapsed to 4 children per node: 32 floats per node, child-major per
  // component: lo.x[4], hi.x[4], lo.y[4], hi.y[4], lo.z[4], hi.z[4], link[4], unused[4].
  std::vector<float> nodes4;
  uint64_t n_nodes4 = 0;
  int max_depth4 = 0;
};


// Child link: bit 31 set = leaf with first = (link >> 3) & 0x0fffffff and count = (link & 7) + 1
// triangles in BVH order; otherwise the index of an internal node.  Node 0 is the root.
// wide: also collapse the tree into out.nodes4.
int build_bvh(const float* verts, const uint32_t* tris, uint64_t nt, BvhOut& out, bool wide = true);

// The same binned-SAH tree over axis-aligned boxes (6 floats per item: lo xyz, hi xyz); leaf
// links then index items in out.order.  No 4-wide copy.
int build_bvh_boxes(const float* boxes, uint64_t n, BvhOut& out);

// Collapses out.nodes (BVH2) into out.nodes4: each 4-wide node takes the two children of a
// BVH2 node and repeatedly opens its largest-area inner child until it has four children.
void collapse_bvh4(BvhOut& out);

}  // namespace nrrs
