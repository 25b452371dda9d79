// Kernels of the learned child ordering that share the intersection kernel's
// arithmetic: trace recording (policy inputs at the nodes on the path to each
// ray's reported leaf), stand-alone inference, and packing of the network into
// matrix-core operand fragments.  Compiled with the intersection kernel's
// floating-point flags so that inputs are formed exactly as during traversal.

#include "ccs_internal.h"
#include "patch_math.h"
#include "policy.h"

namespace ccs {

// Per (ray, level k): the node of depth 2k holding the ray's reported leaf.  Its
// grid is recomputed for its domain (crop, or Alg. 2 on a Gregory patch), split
// along u, and both halves are slab-tested (without a cap); when both are met
// the node is a decision of the policy and the record gets
// its inputs and, as label, the grandchild holding the leaf.  Otherwise (and
// for rays that missed) the label is 255 and the inputs are zero.
__global__ __launch_bounds__(64) void k_record(DeviceScene s, const ccs_ray* __restrict__ rays,
                                               const ccs_hit* __restrict__ hits, uint32_t n,
                                               float* __restrict__ feats, uint8_t* __restrict__ labels) {
  const uint32_t L = (uint32_t)s.leaf_depth;
  const uint64_t idx = (uint64_t)blockIdx.x * 64 + threadIdx.x;
  if (idx >= (uint64_t)n * L) return;
  const uint32_t r = (uint32_t)(idx / L), k = (uint32_t)(idx % L);
  float f[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) f[q] = 0.0f;
  uint32_t label = 255u;
  const float4 h = reinterpret_cast<const float4*>(hits)[r];
  const uint32_t id = __float_as_uint(h.y);
  if (id < s.n_patches) {
    const float4* r4 = reinterpret_cast<const float4*>(rays + r);
    const float4 ro = r4[0], rd = r4[1];
    const float* rec = s.recs + (size_t)s.inv_perm[id] * kRecFloats;
    const float4 meta = reinterpret_cast<const float4*>(rec)[15];
    const bool greg = (__float_as_uint(meta.w) & kGregoryBit) != 0;
    float pox, poy, poz, ptmin, pt0;  // pt0 unused: no cap here
    float dxp = rd.x, dyp = rd.y, dzp = rd.z;  // direction in the frame the patch is subdivided in
    if (!s.frames) patch_frame(meta, ro.x, ro.y, ro.z, rd.x, rd.y, rd.z, ro.w, pox, poy, poz, ptmin, pt0);
    if (s.frames) {
      const float4* fr = s.frames + 3 * (size_t)s.inv_perm[id];
      const float4 r0 = fr[0], r1 = fr[1], r2 = fr[2];
      patch_frame_rows(meta, r0, r1, r2, ro.x, ro.y, ro.z, rd.x, rd.y, rd.z, ro.w, pox, poy, poz, dxp, dyp, dzp,
                       ptmin, pt0);
      pox += r0.w;  // the box pad, as in the intersection kernel
      poy += r0.w;
      poz += r0.w;
    }
    // the reported (u, v) is a leaf centre (2i + 1) 2^-(L+1): scaling by 2^L is exact
    const float scale = __uint_as_float((127u + L) << 23);
    const uint32_t iu = (uint32_t)(h.z * scale), iv = (uint32_t)(h.w * scale);
    const float size = __uint_as_float((127u - k) << 23);
    const float u0 = (float)(iu >> (L - k)) * size, v0 = (float)(iv >> (L - k)) * size;
    PatchPts P;
    load_grid(rec, P, greg);
    float qx[4][4], qy[4][4], qz[4][4], dx, dy, dz;
    calc_points_and_d(P, greg, u0, u0 + size, v0, v0 + size, qx, qy, qz, dx, dy, dz);
    if (s.frames) {
      const float pad2 = 2.0f * s.frames[3 * (size_t)s.inv_perm[id]].w;
      dx += pad2;
      dy += pad2;
      dz += pad2;
    }
    Grid G;
    orient(qx, false, G.x);
    orient(qy, false, G.y);
    orient(qz, false, G.z);
    Row7 e[4];
    SlabPair sp = {ptmin, __builtin_inff(), ptmin, __builtin_inff()};
    // reciprocals rounded back to a direction, exactly as the intersection kernel sees it
    const float ix = safe_inv(dxp), iy = safe_inv(dyp), iz = safe_inv(dzp);
    split_fold(G.x, pox, ix, dx, e, sp);
    split_fold(G.y, poy, iy, dy, e, sp);
    split_fold(G.z, poz, iz, dz, e, sp);
    // no cap: the reported hit lies on the boxes' boundary as often as not, and a
    // capped test there would turn on rounding
    const bool ha = sp.na <= widen_far(sp.fa), hb = sp.nb <= widen_far(sp.fb);
    if (ha && hb) {
      const float sx[4] = {qx[0][0], qx[3][0], qx[0][3], qx[3][3]};
      const float sy[4] = {qy[0][0], qy[3][0], qy[0][3], qy[3][3]};
      const float sz[4] = {qz[0][0], qz[3][0], qz[0][3], qz[3][3]};
      const float fdx = s.frames ? __builtin_amdgcn_rcpf(ix) : rd.x, fdy = s.frames ? __builtin_amdgcn_rcpf(iy) : rd.y,
                  fdz = s.frames ? __builtin_amdgcn_rcpf(iz) : rd.z;
      policy_features(policy_raw(sx, sy, sz, 0u, sp), pox, poy, poz, fdx, fdy, fdz, (int)(2 * k), (int)L, greg, f);
      label = 2u * ((iu >> (L - 1 - k)) & 1u) + ((iv >> (L - 1 - k)) & 1u);
    }
  }
  float4* o = reinterpret_cast<float4*>(feats + idx * 16);
#pragma unroll
  for (int q = 0; q < 4; ++q) o[q] = make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
  labels[idx] = (uint8_t)label;
}

// Network inference for n input rows, one wave per 64 rows, through the same
// wave-wide routine the intersection kernel uses.
__global__ __launch_bounds__(64) void k_policy_infer(PolicyDev P, const float* __restrict__ x, uint32_t n,
                                                     float* __restrict__ z) {
  __shared__ __align__(16) uint32_t feat[64 * 8];
  const int lane = threadIdx.x;
  const uint64_t row = (uint64_t)blockIdx.x * 64 + lane;
  const bool in = row < n;
  float f[16];
  if (in) {
    const float4* xi = reinterpret_cast<const float4*>(x + row * 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 v = xi[q];
      f[4 * q] = v.x;
      f[4 * q + 1] = v.y;
      f[4 * q + 2] = v.z;
      f[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 16; ++q) f[q] = 0.0f;
  }
  policy_store_inputs<8>(feat, lane, f);
  policy_wave<8>(P, feat, __ballot(in), lane);
  if (in) {
    const float4 lg = reinterpret_cast<const float4*>(feat)[2 * lane];
    reinterpret_cast<float4*>(z)[row] = lg;
  }
}

// Operand fragments from the fp32 parameters (layout in policy.h).  Thread
// (tile, lane); weights rounded to bfloat16, biases kept in fp32.
__global__ __launch_bounds__(64) void k_policy_pack(const float* __restrict__ th, uint2* __restrict__ w,
                                                    float4* __restrict__ b) {
  const int tile = blockIdx.x, lane = threadIdx.x;
  const int r = lane & 15, g = lane >> 4;
  if (tile < kPolicyWTiles) {
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 4 * g + i;
      if (tile < 2) {
        v[i] = th[kPolicyW1 + (16 * tile + r) * 16 + k];
      } else if (tile < 6) {
        const int rt = (tile - 2) >> 1, ct = (tile - 2) & 1;
        v[i] = th[kPolicyW2 + (16 * rt + r) * 32 + 16 * ct + k];
      } else {
        const int ct = tile - 6;
        v[i] = r < 4 ? th[kPolicyW3 + r * 32 + 16 * ct + k] : 0.0f;
      }
    }
    w[tile * 64 + lane] = make_uint2(bf16_pair(v[0], v[1]), bf16_pair(v[2], v[3]));
  } else {
    const int bt = tile - kPolicyWTiles;
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 4 * g + i;
      if (bt < 2)
        v[i] = th[kPolicyB1 + 16 * bt + row];
      else if (bt < 4)
        v[i] = th[kPolicyB2 + 16 * (bt - 2) + row];
      else
        v[i] = row < 4 ? th[kPolicyB3 + row] : 0.0f;
    }
    b[bt * 64 + lane] = make_float4(v[0], v[1], v[2], v[3]);
  }
}

hipError_t launch_policy_pack(const float* params, uint2* w, float4* b, hipStream_t stream) {
  hipLaunchKernelGGL(k_policy_pack, dim3(kPolicyWTiles + kPolicyBTiles), dim3(64), 0, stream, params, w, b);
  return hipGetLastError();
}

hipError_t launch_policy_infer(const PolicyDev& P, const float* x, uint32_t n, float* z, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_policy_infer, dim3((n + 63) / 64), dim3(64), 0, stream, P, x, n, z);
  return hipGetLastError();
}

hipError_t launch_record(const DeviceScene& s, const ccs_ray* rays, const ccs_hit* hits, uint32_t n, float* feats,
                         uint8_t* labels, hipStream_t stream) {
  const uint64_t total = (uint64_t)n * (uint64_t)s.leaf_depth;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_record, dim3((uint32_t)((total + 63) / 64)), dim3(64), 0, stream, s, rays, hits, n, feats,
                     labels);
  return hipGetLastError();
}

}  // namespace ccs
