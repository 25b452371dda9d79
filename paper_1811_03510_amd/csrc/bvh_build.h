// Host BVH construction over patch boxes: binary, one patch per leaf, splits
// chosen approximately by the surface area heuristic with binning (the
// hierarchy the paper traverses, Sec. 4).
#pragma once

#include <cstdint>
#include <vector>

namespace ccs {

struct BuildBox {
  float lo[3], hi[3];
};

struct BvhOutput {
  std::vector<float> nodes;           // 16 floats per node (see ccs_internal.h)
  std::vector<uint32_t> perm;         // record (leaf order) -> input patch index
  std::vector<int32_t> leaf_parent;   // record -> (node << 1 | side)
  std::vector<int32_t> node_parent;   // node -> (parent << 1 | side), -1 for the root
  uint32_t max_depth = 0;             // deepest leaf (root children have depth 1)
};

// max_depth_limit bounds the traversal stack: below depth `sah_depth` splits
// follow the SAH, deeper ones split at the object median of the widest axis.
BvhOutput build_bvh(const std::vector<BuildBox>& boxes, uint32_t sah_depth, int n_threads);

}  // namespace ccs
