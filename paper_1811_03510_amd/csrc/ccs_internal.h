// Internal interface between the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ccs.h"

namespace ccs {

// BVH node: 64 bytes = 4 float4.
//   f[0] = (lo0.x, lo0.y, lo0.z, hi0.x)
//   f[1] = (hi0.y, hi0.z, lo1.x, lo1.y)
//   f[2] = (lo1.z, hi1.x, hi1.y, hi1.z)
//   f[3] = (child0, child1, -, -) as int bits: >= 0 internal node, < 0 patch
//          record ~child (one patch per leaf).  An empty child has lo > hi.
struct DeviceScene {
  const float4* nodes;
  float* recs;               // n x kRecFloats
  uint32_t n_patches;
  uint32_t n_nodes;
  int leaf_depth;
  const uint32_t* perm;      // record -> original index
  const uint32_t* inv_perm;  // original index -> record
  const int32_t* leaf_parent;  // record -> (node << 1 | side)
  const int32_t* node_parent;  // node -> (parent << 1 | side), -1 for the root
  uint32_t* arrivals;        // n_nodes counters for the bottom-up refit
  uint32_t n_cus;            // compute units of the device
  uint32_t n_frames;         // frames: copies of recs and node boxes sharing one topology
  size_t frame_rec_floats;   // floats per frame in recs (n_patches * kRecFloats)
  size_t frame_node_f4;      // float4s per frame in nodes (n_nodes * 4)
};

// Rays of one launch: up to kMaxBatches batches, each with its own frame, ray
// array and hit array; ray k of the launch belongs to batch b when
// prefix[b] <= k < prefix[b + 1].  Passed by value as a kernel argument.
constexpr int kMaxBatches = 32;
struct BatchTable {
  uint32_t n_batches;
  uint32_t prefix[kMaxBatches + 1];
  uint32_t frame[kMaxBatches];
  const ccs_ray* rays[kMaxBatches];
  ccs_hit* hits[kMaxBatches];
};

// Phase thresholds of the persistent intersection kernel (see trace.hip) and
// the launch's ray-queue counter.
struct LaunchParams {
  uint32_t fetch_min, traverse_min, grid_min, traverse_steps;
  uint32_t* queue;
};

int max_waves_per_cu(bool counted);
hipError_t launch_intersect(const DeviceScene& s, const BatchTable& bt, uint32_t* counters, const LaunchParams& lp,
                            uint32_t waves_per_cu, hipStream_t stream);
hipError_t launch_refit(const DeviceScene& s, const float* cp_world, hipStream_t stream);
hipError_t launch_bounce(const DeviceScene& s, const ccs_ray* rays, const ccs_hit* hits, const float* uniforms,
                         uint32_t n, ccs_ray* out, hipStream_t stream);

}  // namespace ccs
