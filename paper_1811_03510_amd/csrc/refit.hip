// Refit of an existing scene to moved control points (animation playback).
// Topology is kept; anchors stay at their create-time values.
//
//   k_refit_patches  one thread per patch record: the 20 world points are read
//                    as 15 16-byte loads, the anchored record is written as 15
//                    16-byte stores, and the patch's hull box goes into its
//                    parent node's child slot;
//   k_refit_level    one launch per BVH depth, deepest first: each node of that
//                    depth unions its two child slots into its own slot in its
//                    parent.
// Launch boundaries order the levels, so no thread ever waits on another and no
// device-wide fence is needed (each XCD's L2 is written back at kernel end).

#include "ccs_internal.h"
#include "patch_math.h"

namespace ccs {

constexpr int kRefitBlock = 256;

__device__ __forceinline__ void write_child_box(float4* nodes, int node, int side, const float lo[3],
                                                const float hi[3]) {
  float* f = reinterpret_cast<float*>(nodes + 4 * (size_t)node);
  const int base = side ? 6 : 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    f[base + k] = lo[k];
    f[base + 3 + k] = hi[k];
  }
}

__global__ __launch_bounds__(kRefitBlock) void k_refit_patches(DeviceScene s, const float* __restrict__ cp) {
  const uint32_t r = blockIdx.x * kRefitBlock + threadIdx.x;
  if (r >= s.n_patches) return;
  float4* rec = reinterpret_cast<float4*>(s.recs + (size_t)r * kRecFloats);
  const float4 meta = rec[15];  // anchor xyz, meta bits: unchanged
  const bool greg = (__float_as_uint(meta.w) & kGregoryBit) != 0;
  const float4* src = reinterpret_cast<const float4*>(cp + (size_t)s.perm[r] * 60);  // 240 B, 16-B aligned
  float p[60];
#pragma unroll
  for (int q = 0; q < 15; ++q) {
    const float4 v = src[q];
    p[4 * q] = v.x;
    p[4 * q + 1] = v.y;
    p[4 * q + 2] = v.z;
    p[4 * q + 3] = v.w;
  }
  float lo[3] = {p[0], p[1], p[2]}, hi[3] = {p[0], p[1], p[2]};
#pragma unroll
  for (int sl = 1; sl < 20; ++sl) {
    if (sl >= 16 && !greg) break;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], p[3 * sl + a]);
      hi[a] = fmaxf(hi[a], p[3 * sl + a]);
    }
  }
  const float anc[3] = {meta.x, meta.y, meta.z};
  float out[60];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int sl = 0; sl < 16; ++sl) out[16 * a + sl] = p[3 * sl + a] - anc[a];
#pragma unroll
    for (int j = 0; j < 4; ++j) out[48 + 4 * a + j] = p[3 * (16 + j) + a] - anc[a];
  }
#pragma unroll
  for (int q = 0; q < 15; ++q) rec[q] = make_float4(out[4 * q], out[4 * q + 1], out[4 * q + 2], out[4 * q + 3]);
  float4* nodes = const_cast<float4*>(s.nodes);
  const int link = s.leaf_parent[r];
  write_child_box(nodes, link >> 1, link & 1, lo, hi);
  if (s.n_patches == 1) write_child_box(nodes, 0, 1, lo, hi);  // a lone patch occupies both slots of the root
}

__global__ __launch_bounds__(kRefitBlock) void k_refit_level(float4* __restrict__ nodes,
                                                             const uint32_t* __restrict__ ids, uint32_t count,
                                                             const int32_t* __restrict__ node_parent) {
  const uint32_t i = blockIdx.x * kRefitBlock + threadIdx.x;
  if (i >= count) return;
  const uint32_t node = ids[i];
  const int link = node_parent[node];
  if (link < 0) return;  // the root has no slot to fill
  const float4 a = nodes[4 * (size_t)node], b = nodes[4 * (size_t)node + 1], c = nodes[4 * (size_t)node + 2];
  const float lo[3] = {fminf(a.x, b.z), fminf(a.y, b.w), fminf(a.z, c.x)};
  const float hi[3] = {fmaxf(a.w, c.y), fmaxf(b.x, c.z), fmaxf(b.y, c.w)};
  write_child_box(nodes, link >> 1, link & 1, lo, hi);
}

hipError_t launch_refit(const DeviceScene& s, const float* cp_world, const uint32_t* level_offsets,
                        uint32_t n_levels, hipStream_t stream) {
  if (s.n_patches == 0) return hipSuccess;
  hipLaunchKernelGGL(k_refit_patches, dim3((s.n_patches + kRefitBlock - 1) / kRefitBlock), dim3(kRefitBlock), 0,
                     stream, s, cp_world);
  float4* nodes = const_cast<float4*>(s.nodes);
  for (uint32_t d = n_levels; d-- > 1;) {  // deepest level first; level 0 is the root
    const uint32_t lo = level_offsets[d], count = level_offsets[d + 1] - lo;
    if (count == 0) continue;
    hipLaunchKernelGGL(k_refit_level, dim3((count + kRefitBlock - 1) / kRefitBlock), dim3(kRefitBlock), 0, stream,
                       nodes, s.level_nodes + lo, count, s.node_parent);
  }
  return hipGetLastError();
}

}  // namespace ccs
