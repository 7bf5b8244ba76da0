// Constants of the BVH layouts shared by the host builder and the traversal kernels.
#pragma once
#include <stdint.h>

namespace nrrs {

constexpr int kMaxBvhDepth = 62;                // deepest BVH2 level the traversal stack is sized for
constexpr int kMaxBvh4Depth = 30;               // deepest 4-wide level (3 stack entries per level)
constexpr uint32_t kEmptyChild4 = 0x7FFFFFFFu;  // link of an unused 4-wide child slot
// Triangles per leaf at most: the shared leaf phase gives each parked leaf a group of this many
// lanes (16 leaves per 64-lane round).
constexpr uint32_t kLeafMaxTris = 4;

}  // namespace nrrs
