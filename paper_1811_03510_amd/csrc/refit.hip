// Refit of an existing scene to moved control points (animation playback):
// anchored records and patch boxes are recomputed per patch, then node boxes are
// refitted bottom-up in one launch.  Each leaf thread writes its box into its
// parent's child slot and walks up; at every node the second thread to arrive
// (atomic arrival counter) unions both child slots and continues, the first stops.

#include "ccs_internal.h"
#include "patch_math.h"

namespace ccs {

constexpr int kRefitBlock = 256;

__global__ __launch_bounds__(kRefitBlock) void k_zero(uint32_t* __restrict__ p, uint32_t n) {
  const uint32_t i = blockIdx.x * kRefitBlock + threadIdx.x;
  if (i < n) p[i] = 0u;
}

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

__global__ __launch_bounds__(kRefitBlock) void k_refit(DeviceScene s, const float* __restrict__ cp) {
  const uint32_t r = blockIdx.x * kRefitBlock + threadIdx.x;
  if (r >= s.n_patches) return;
  float* rec = s.recs + (size_t)r * kRecFloats;
  const uint32_t meta = __float_as_uint(rec[63]);
  const bool greg = (meta & kGregoryBit) != 0;
  const float ax = rec[60], ay = rec[61], az = rec[62];
  const float* src = cp + (size_t)s.perm[r] * 60;
  float lo[3] = {src[0], src[1], src[2]}, hi[3] = {src[0], src[1], src[2]};
  for (int slot = 0; slot < 20; ++slot) {
    const float x = src[3 * slot], y = src[3 * slot + 1], z = src[3 * slot + 2];
    if (slot < 16 || greg) {
      lo[0] = fminf(lo[0], x); lo[1] = fminf(lo[1], y); lo[2] = fminf(lo[2], z);
      hi[0] = fmaxf(hi[0], x); hi[1] = fmaxf(hi[1], y); hi[2] = fmaxf(hi[2], z);
    }
    if (slot < 16) {
      rec[slot] = x - ax;
      rec[16 + slot] = y - ay;
      rec[32 + slot] = z - az;
    } else {
      rec[48 + slot - 16] = x - ax;
      rec[52 + slot - 16] = y - ay;
      rec[56 + slot - 16] = z - az;
    }
  }
  float4* nodes = const_cast<float4*>(s.nodes);
  int link = s.leaf_parent[r];
  write_child_box(nodes, link >> 1, link & 1, lo, hi);
  if (s.n_patches == 1) {  // a lone patch occupies both slots of the root
    write_child_box(nodes, 0, 1, lo, hi);
    return;
  }
  for (;;) {
    const int node = link >> 1;
    __threadfence();
    if (atomicAdd(&s.arrivals[node], 1u) == 0u) return;  // sibling subtree still pending
    __threadfence();
    const volatile float* f = reinterpret_cast<const volatile float*>(nodes + 4 * (size_t)node);
    for (int k = 0; k < 3; ++k) {
      lo[k] = fminf(f[k], f[6 + k]);
      hi[k] = fmaxf(f[3 + k], f[9 + k]);
    }
    link = s.node_parent[node];
    if (link < 0) return;  // root
    write_child_box(nodes, link >> 1, link & 1, lo, hi);
  }
}

hipError_t launch_refit(const DeviceScene& s, const float* cp_world, hipStream_t stream) {
  if (s.n_patches == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3((s.n_nodes + kRefitBlock - 1) / kRefitBlock), dim3(kRefitBlock), 0, stream,
                     s.arrivals, s.n_nodes);
  hipLaunchKernelGGL(k_refit, dim3((s.n_patches + kRefitBlock - 1) / kRefitBlock), dim3(kRefitBlock), 0, stream, s,
                     cp_world);
  return hipGetLastError();
}

}  // namespace ccs
