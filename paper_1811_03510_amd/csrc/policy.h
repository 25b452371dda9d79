// Learned child ordering: the policy's inputs and its wave-wide inference on
// the matrix cores.
//
// The closest-first rule of Alg. 3 (Sec. 3.3) picks, after each split, the half
// whose box the ray enters first.  The learned policy replaces that pick at
// nodes of even depth (the split runs along u) where both u-halves are hit: a
// 16-32-32-4 ReLU network ranks the node's four grandchildren (u-half, v-half),
// the lane descends into the u-half of the top-ranked one and, one split later,
// into its v-half when both v-halves are hit.  Only halves whose boxes are hit
// are ever entered and nothing else of Alg. 3 changes, so the traversal still
// finds the closest leaf; the order only changes how soon.
//
// Inputs (16), free of position, orientation and scale:
//   0..11  the node grid's corner points (u0,v0), (u1,v0), (u0,v1), (u1,v1),
//          minus the ray's entry point into the node box, in the frame
//          (e1, e2, d/|d|) of Duff et al. 2017, divided by s, the largest of
//          these 12 magnitudes
//   12, 13 entry and exit distance of the lower minus the upper u-half,
//          times |d| / s, clamped to [-4, 4] and divided by 4
//   14     depth / 2L;  15: 1 on a Gregory patch
// Network: parameters fp32 in the order W1 (32x16, row = unit), b1, W2
// (32x32), b2, W3 (4x32), b3; inference rounds inputs, weights and hidden
// activations to bfloat16 (nearest, ties to even) and accumulates in fp32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ccs_internal.h"
#include "patch_math.h"

namespace ccs {

constexpr int kPolicyW1 = 0, kPolicyB1 = 512, kPolicyW2 = 544, kPolicyB2 = 1568, kPolicyW3 = 1600, kPolicyB3 = 1728;
// Matrix-core operand fragments of the network for one wave (PolicyDev): 8
// weight tiles of 64 lanes x 4 bfloat16 (W1 rows 0-15, 16-31; W2 (row tile,
// column tile) (0,0), (0,1), (1,0), (1,1); W3 (zero-padded to 16 rows) column
// tiles 0, 1) and 5 bias tiles of 64 lanes x 4 fp32 (b1 rows 0-15, 16-31; b2 the
// same; b3).  Lane l of a weight tile holds row l & 15, columns 4 (l >> 4) .. +3;
// lane l of a bias tile holds rows 4 (l >> 4) .. +3.

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t bf16_bits(float x) {  // round to nearest, ties to even (finite x)
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ uint32_t bf16_pair(float lo, float hi) { return bf16_bits(lo) | (bf16_bits(hi) << 16); }

__device__ __forceinline__ bf16x4 as_bf16x4(uint2 v) {
  bf16x4 r;
  __builtin_memcpy(&r, &v, 8);
  return r;
}

// The per-node values the inputs are formed from (PolicyRaw): the node grid's
// corner points in canonical (u, v) order (u0,v0), (u1,v0), (u0,v1), (u1,v1),
// and the raw (uncapped) slab entry and exit of the lower and the upper u-half.
struct PolicyRaw {
  float cx[4], cy[4], cz[4];
  float n_lo, n_up, x_lo, x_up;
};

// PolicyRaw of a node at even depth from its corners in storage order (first,
// second index) = (0,0), (3,0), (0,3), (3,3) (the first index runs along u;
// mirror bit 0 / 1: u / v stored reversed) and the slab results of the two
// u-halves in storage order.
__device__ __forceinline__ PolicyRaw policy_raw(const float sx[4], const float sy[4], const float sz[4],
                                                uint32_t mirror, const SlabPair& sp) {
  const bool mu = (mirror & 1u) != 0, mv = (mirror & 2u) != 0;
  PolicyRaw r;
  r.n_lo = mu ? sp.nb : sp.na;
  r.n_up = mu ? sp.na : sp.nb;
  r.x_lo = mu ? sp.fb : sp.fa;
  r.x_up = mu ? sp.fa : sp.fb;
  // storage order to canonical (u, v) order by selects (no indexing by a run-time value)
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r.cx[k] = sx[k];
    r.cy[k] = sy[k];
    r.cz[k] = sz[k];
  }
#pragma unroll
  for (int k = 0; k < 4; k += 2) {  // u reversed: swap (0,1) and (2,3)
    float t;
    t = r.cx[k]; r.cx[k] = mu ? r.cx[k + 1] : t; r.cx[k + 1] = mu ? t : r.cx[k + 1];
    t = r.cy[k]; r.cy[k] = mu ? r.cy[k + 1] : t; r.cy[k + 1] = mu ? t : r.cy[k + 1];
    t = r.cz[k]; r.cz[k] = mu ? r.cz[k + 1] : t; r.cz[k + 1] = mu ? t : r.cz[k + 1];
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {  // v reversed: swap (0,2) and (1,3)
    float t;
    t = r.cx[k]; r.cx[k] = mv ? r.cx[k + 2] : t; r.cx[k + 2] = mv ? t : r.cx[k + 2];
    t = r.cy[k]; r.cy[k] = mv ? r.cy[k + 2] : t; r.cy[k + 2] = mv ? t : r.cy[k + 2];
    t = r.cz[k]; r.cz[k] = mv ? r.cz[k + 2] : t; r.cz[k + 2] = mv ? t : r.cz[k + 2];
  }
  return r;
}

// The 16 inputs from PolicyRaw, a ray with origin o and direction d in the patch
// frame, the node's depth and the patch type.
__device__ __forceinline__ void policy_features(const PolicyRaw& r, float ox, float oy, float oz, float dx,
                                                float dy, float dz, int depth, int leaf_depth, bool gregory,
                                                float f[16]) {
  // the inputs end as bfloat16 (8 significant bits): the hardware square root and
  // reciprocals (within 1 ulp of fp32) are ample, and the training records are
  // formed by this same code
  const float t_in = fminf(r.n_lo, r.n_up);
  const float dl = __builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz);
  const float il = __builtin_amdgcn_rcpf(dl);
  const float nx = dx * il, ny = dy * il, nz = dz * il;
  // Duff et al. 2017, branch-free orthonormal basis around n
  const float sg = copysignf(1.0f, nz);
  const float a = -__builtin_amdgcn_rcpf(sg + nz);
  const float b = nx * ny * a;
  const float e1x = 1.0f + sg * nx * nx * a, e1y = sg * b, e1z = -sg * nx;
  const float e2x = b, e2y = sg + ny * ny * a, e2z = -ny;
  const float px = ox + t_in * dx, py = oy + t_in * dy, pz = oz + t_in * dz;
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float qx = r.cx[k] - px, qy = r.cy[k] - py, qz = r.cz[k] - pz;
    f[3 * k + 0] = qx * e1x + qy * e1y + qz * e1z;
    f[3 * k + 1] = qx * e2x + qy * e2y + qz * e2z;
    f[3 * k + 2] = qx * nx + qy * ny + qz * nz;
    s = fmaxf(s, fmaxf(fabsf(f[3 * k]), fmaxf(fabsf(f[3 * k + 1]), fabsf(f[3 * k + 2]))));
  }
  s = fmaxf(s, 1e-30f);
  const float is = __builtin_amdgcn_rcpf(s);
#pragma unroll
  for (int k = 0; k < 12; ++k) f[k] *= is;
  const float sc = dl * is;
  f[12] = fminf(fmaxf((r.n_lo - r.n_up) * sc, -4.0f), 4.0f) * 0.25f;
  f[13] = fminf(fmaxf((r.x_lo - r.x_up) * sc, -4.0f), 4.0f) * 0.25f;
  f[14] = (float)depth * __builtin_amdgcn_rcpf((float)(2 * leaf_depth));
  f[15] = gregory ? 1.0f : 0.0f;
}

// The values policy_raw takes (corners and slab results in storage order)
// through a lane's 64-byte slot of LDS: the intersection kernel keeps them there
// between the split that meets a decision and the decision itself.
__device__ __forceinline__ void policy_store_node(uint32_t* slots, int lane, const float sx[4], const float sy[4],
                                                  const float sz[4], const SlabPair& sp) {
  float4* o = reinterpret_cast<float4*>(slots + lane * 16);
  o[0] = make_float4(sx[0], sx[1], sx[2], sx[3]);
  o[1] = make_float4(sy[0], sy[1], sy[2], sy[3]);
  o[2] = make_float4(sz[0], sz[1], sz[2], sz[3]);
  o[3] = make_float4(sp.na, sp.fa, sp.nb, sp.fb);
}
__device__ __forceinline__ PolicyRaw policy_load_node(const uint32_t* slots, int lane, uint32_t mirror) {
  const float4* i = reinterpret_cast<const float4*>(slots + lane * 16);
  const float4 a = i[0], b = i[1], c = i[2], d = i[3];
  const float sx[4] = {a.x, a.y, a.z, a.w}, sy[4] = {b.x, b.y, b.z, b.w}, sz[4] = {c.x, c.y, c.z, c.w};
  const SlabPair sp = {d.x, d.y, d.z, d.w};
  return policy_raw(sx, sy, sz, mirror, sp);
}

// One 16-sample column tile of the network on the matrix cores, computed
// transposed (H^T = W X^T) so that each layer's accumulator layout is the next
// layer's B operand: lane l holds, for sample (l & 15) of the tile, inputs
// 4 (l >> 4) .. +3 in `x`, and receives in the returned vector, when l < 16,
// the tile's logits 0..3 of sample l.  Must be executed by the whole wave.
__device__ __forceinline__ f32x4 policy_tile(const PolicyDev& P, bf16x4 x, int lane) {
  const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  bf16x4 h1[2], h2[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(as_bf16x4(P.w[t * 64 + lane]), x, zero, 0, 0, 0);
    const float4 bb = P.b[t * 64 + lane];
    uint2 hv;
    hv.x = bf16_pair(fmaxf(acc[0] + bb.x, 0.0f), fmaxf(acc[1] + bb.y, 0.0f));
    hv.y = bf16_pair(fmaxf(acc[2] + bb.z, 0.0f), fmaxf(acc[3] + bb.w, 0.0f));
    h1[t] = as_bf16x4(hv);
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(as_bf16x4(P.w[(2 + 2 * t) * 64 + lane]), h1[0], zero, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(as_bf16x4(P.w[(3 + 2 * t) * 64 + lane]), h1[1], acc, 0, 0, 0);
    const float4 bb = P.b[(2 + t) * 64 + lane];
    uint2 hv;
    hv.x = bf16_pair(fmaxf(acc[0] + bb.x, 0.0f), fmaxf(acc[1] + bb.y, 0.0f));
    hv.y = bf16_pair(fmaxf(acc[2] + bb.z, 0.0f), fmaxf(acc[3] + bb.w, 0.0f));
    h2[t] = as_bf16x4(hv);
  }
  f32x4 z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(as_bf16x4(P.w[6 * 64 + lane]), h2[0], zero, 0, 0, 0);
  z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(as_bf16x4(P.w[7 * 64 + lane]), h2[1], z, 0, 0, 0);
  const float4 bb = P.b[4 * 64 + lane];
  z[0] += bb.x;
  z[1] += bb.y;
  z[2] += bb.z;
  z[3] += bb.w;
  return z;
}

// A lane's 16 inputs as bfloat16 pairs into the first 32 bytes of its slot of
// `feat` (kSlot words per slot).
template <int kSlot>
__device__ __forceinline__ void policy_store_inputs(uint32_t* feat, int lane, const float f[16]) {
  uint4* o = reinterpret_cast<uint4*>(feat + lane * kSlot);
  o[0] = make_uint4(bf16_pair(f[0], f[1]), bf16_pair(f[2], f[3]), bf16_pair(f[4], f[5]), bf16_pair(f[6], f[7]));
  o[1] = make_uint4(bf16_pair(f[8], f[9]), bf16_pair(f[10], f[11]), bf16_pair(f[12], f[13]),
                    bf16_pair(f[14], f[15]));
}

// The network for every lane whose bit is set in `need`: lane s's inputs are
// read from its slot of `feat` (LDS, 64 slots of kSlot >= 8 words) and its four
// logits are written back to the first 16 bytes of the slot.  Column tiles
// without a requesting lane are skipped.  Must be executed by the whole wave.
template <int kSlot>
__device__ __forceinline__ void policy_wave(const PolicyDev& P, uint32_t* feat, uint64_t need, int lane) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (((need >> (16 * c)) & 0xFFFFull) == 0) continue;
    const uint2 xv = *reinterpret_cast<const uint2*>(feat + (16 * c + (lane & 15)) * kSlot + 2 * (lane >> 4));
    const f32x4 z = policy_tile(P, as_bf16x4(xv), lane);
    if (lane < 16)
      *reinterpret_cast<float4*>(feat + (16 * c + lane) * kSlot) = make_float4(z[0], z[1], z[2], z[3]);
  }
}

// Index of the largest logit, ties to the lower index.
__device__ __forceinline__ uint32_t policy_top(float z0, float z1, float z2, float z3) {
  uint32_t k = 0;
  float m = z0;
  if (z1 > m) { k = 1; m = z1; }
  if (z2 > m) { k = 2; m = z2; }
  if (z3 > m) { k = 3; }
  return k;
}

}  // namespace ccs
