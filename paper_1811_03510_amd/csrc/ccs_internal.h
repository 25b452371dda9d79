// Internal interface between the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ccs.h"

namespace ccs {

// Child-ordering network as matrix-core operand fragments (layout in policy.h).
constexpr int kPolicyParams = 1732;
constexpr int kPolicyWTiles = 8, kPolicyBTiles = 5;
struct PolicyDev {
  const uint2* w;   // kPolicyWTiles * 64 lanes x 4 bfloat16
  const float4* b;  // kPolicyBTiles * 64 lanes x 4 fp32
};

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
  const uint32_t* level_nodes;  // node indices sorted by depth (refit order; offsets on the host)
  uint32_t n_cus;            // compute units of the device
  uint32_t n_frames;         // frames: copies of recs and node boxes sharing one topology
  size_t frame_rec_floats;   // floats per frame in recs (n_patches * kRecFloats)
  size_t frame_node_f4;      // float4s per frame in nodes (n_nodes * 4)
  PolicyDev policy;          // set: learned child ordering (see policy.h); w == nullptr: closest first
  float4* frames;            // patch-local frames: 3 rows per record (per frame), row 0's w = the box pad;
                             // nullptr: world frame
  size_t frame_frames_f4;    // float4s per frame in frames (n_patches * 3)
  bool single_box;           // Alg. 3 steps test only the current domain's box (ablation; closest first)
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
  uint32_t fetch_min, traverse_min, grid_min, traverse_steps, decide_min;
  uint32_t* queue;
};

// BVH depth the learned variant's node stack holds (its LDS also holds a 64-byte
// decision slot per lane; with 32 levels a wave's LDS stays within 1/12 of the
// CU's, so 12 waves fit as in the closest-first variant, which holds
// kMaxBvhDepth).  SAH builds of the 1M- and 8M-patch benchmark scenes are 27 and
// 29 levels deep.
constexpr uint32_t kMaxBvhDepth = 48;
constexpr uint32_t kMaxBvhDepthLearned = 32;

// Leaf depths up to kMaxLeafDepth32 run with 32-bit path codes; deeper ones (up to
// CCS_MAX_LEAF_DEPTH) with 64-bit codes, closest-first order only.
constexpr uint32_t kMaxLeafDepth32 = 16;
int max_waves_per_cu(bool counted, bool learned, bool single_box, bool deep);
hipError_t launch_intersect(const DeviceScene& s, const BatchTable& bt, uint32_t* counters, const LaunchParams& lp,
                            uint32_t waves_per_cu, hipStream_t stream);
hipError_t launch_refit(const DeviceScene& s, const float* cp_world, const uint32_t* level_offsets,
                        uint32_t n_levels, hipStream_t stream);
hipError_t launch_policy_pack(const float* params, uint2* w, float4* b, hipStream_t stream);
hipError_t launch_policy_infer(const PolicyDev& P, const float* x, uint32_t n, float* z, hipStream_t stream);
hipError_t launch_record(const DeviceScene& s, const ccs_ray* rays, const ccs_hit* hits, uint32_t n, float* feats,
                         uint8_t* labels, hipStream_t stream);
hipError_t launch_mlp_grad(const float* theta, const float* X, const uint8_t* Y, uint32_t n, uint32_t batch,
                           uint64_t pos0, uint64_t pa, uint64_t pc, int bf16, float* partial, float* lossp,
                           hipStream_t stream);
hipError_t launch_mlp_reduce(const float* partial, const float* lossp, uint32_t nblk, float* grad, float* loss,
                             hipStream_t stream);
hipError_t launch_mlp_adam(float* theta, float* m, float* v, const float* partial, const float* lossp, uint32_t nblk,
                           float lr, float beta1, float beta2, float eps, float c1, float c2, float* loss,
                           hipStream_t stream);
hipError_t launch_fill(float* p, uint32_t n, float value, hipStream_t stream);
// Rows of the gradient entry point that allocates nothing: at most
// kGradScratchBlocks blocks of 64 (1.7 MiB of device scratch per device).
constexpr uint32_t kGradScratchBlocks = 256;
hipError_t grad_scratch(float** partial, float** lossp);
constexpr int kDebugGridFloats = 160;
hipError_t launch_debug_grids(const DeviceScene& s, const uint32_t* patch, const uint32_t* code,
                              const uint32_t* depth, uint32_t n, float* out, hipStream_t stream);
hipError_t launch_bounce(const DeviceScene& s, const ccs_ray* rays, const ccs_hit* hits, const float* uniforms,
                         uint32_t n, ccs_ray* out, hipStream_t stream);
// Ray compaction (compact.hip): blocks of 256 rays; work holds 1 + compact_blocks(n) words.
inline uint32_t compact_blocks(uint32_t n) { return (uint32_t)(((uint64_t)n + 255u) / 256u); }
hipError_t launch_compact_rays(const ccs_ray* rays, uint32_t n, ccs_ray* out, uint32_t* index, uint32_t* work,
                               hipStream_t stream);

}  // namespace ccs
