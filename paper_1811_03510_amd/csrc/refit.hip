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
// With patch-local frames the per-patch pass also recomputes each patch's frame
// and stores the record in it.  Compiled without floating-point contraction, so
// every refit of the same points gives the same bits.

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
    const bool in = sl < 16 || greg;  // a Bezier patch's hull is that of its 16 points
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = in ? fminf(lo[a], p[3 * sl + a]) : lo[a];
      hi[a] = in ? fmaxf(hi[a], p[3 * sl + a]) : hi[a];
    }
  }
  const float anc[3] = {meta.x, meta.y, meta.z};
  float out[60];
  if (s.frames) {
    // patch-local frame, in double: r0 = unit(p30 - p00), r1 = unit of (p03 - p00)
    // without its r0 part, r2 = r0 x r1; the identity for a degenerate u or v edge.
    // Rows are stored in fp32 and the anchored points are mapped by the stored rows
    // (in double, rounded once), so that rays mapped by the same rows see exactly
    // the mapped patch.
    double eu[3], ev[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      eu[a] = (double)p[9 + a] - (double)p[a];
      ev[a] = (double)p[36 + a] - (double)p[a];
    }
    const double lu = sqrt(eu[0] * eu[0] + eu[1] * eu[1] + eu[2] * eu[2]);
    const double lv = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
    double m[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    if (lu > 0.0 && lv > 0.0) {
      const double iu = 1.0 / lu;
      const double r0[3] = {iu * eu[0], iu * eu[1], iu * eu[2]};
      const double dv = ev[0] * r0[0] + ev[1] * r0[1] + ev[2] * r0[2];
      const double w[3] = {ev[0] - dv * r0[0], ev[1] - dv * r0[1], ev[2] - dv * r0[2]};
      const double lw = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
      if (lw > 1e-9 * lv) {
        const double iw = 1.0 / lw;
        const double r1[3] = {iw * w[0], iw * w[1], iw * w[2]};
        m[0][0] = r0[0]; m[0][1] = r0[1]; m[0][2] = r0[2];
        m[1][0] = r1[0]; m[1][1] = r1[1]; m[1][2] = r1[2];
        m[2][0] = r0[1] * r1[2] - r0[2] * r1[1];
        m[2][1] = r0[2] * r1[0] - r0[0] * r1[2];
        m[2][2] = r0[0] * r1[1] - r0[1] * r1[0];
      }
    }
    float rf[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) rf[a][b] = (float)m[a][b];
#pragma unroll
    for (int sl = 0; sl < 20; ++sl) {
      const double q[3] = {(double)p[3 * sl] - (double)anc[0], (double)p[3 * sl + 1] - (double)anc[1],
                           (double)p[3 * sl + 2] - (double)anc[2]};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float v = (float)((double)rf[a][0] * q[0] + (double)rf[a][1] * q[1] + (double)rf[a][2] * q[2]);
        if (sl < 16)
          out[16 * a + sl] = v;
        else
          out[48 + 4 * a + (sl - 16)] = v;
      }
    }
    // gap-closing pad (Sec. 3.4): 2^-19 of the patch's largest extent in its frame;
    // every subdivision box of the patch is grown by it on all sides
    float ext = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float l = out[16 * a], h = out[16 * a];
#pragma unroll
      for (int sl = 1; sl < 16; ++sl) {
        l = fminf(l, out[16 * a + sl]);
        h = fmaxf(h, out[16 * a + sl]);
      }
      if (greg) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          l = fminf(l, out[48 + 4 * a + j]);
          h = fmaxf(h, out[48 + 4 * a + j]);
        }
      }
      ext = fmaxf(ext, h - l);
    }
    const float pad = ldexpf(ext, -19);
#pragma unroll
    for (int a = 0; a < 3; ++a)
      s.frames[3 * (size_t)r + a] = make_float4(rf[a][0], rf[a][1], rf[a][2], a == 0 ? pad : 0.0f);
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int sl = 0; sl < 16; ++sl) out[16 * a + sl] = p[3 * sl + a] - anc[a];
#pragma unroll
      for (int j = 0; j < 4; ++j) out[48 + 4 * a + j] = p[3 * (16 + j) + a] - anc[a];
    }
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
