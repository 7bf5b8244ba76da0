// Host BVH builder interface.
#pragma once
#include <stdint.h>

#include <vector>

namespace nrrs {

struct BvhOut {
  std::vector<float> nodes;      // 16 floats per node: child0 lo/hi, child1 lo/hi, links
  std::vector<uint32_t> order;   // BVH position -> original triangle index
  uint64_t n_nodes = 0;
  int max_depth = 0;             // levels from the root to the deepest leaf
};

// Child link: bit 31 set = leaf with first = (link >> 3) & 0x0fffffff and count = (link & 7) + 1
// triangles in BVH order; otherwise the index of an internal node.  Node 0 is the root.
int build_bvh(const float* verts, const uint32_t* tris, uint64_t nt, BvhOut& out);

}  // namespace nrrs
