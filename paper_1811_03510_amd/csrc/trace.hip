// Closest-hit kernel: BVH traversal over patch boxes and, per candidate patch,
// the stackless hierarchical subdivision of Alg. 3 (Sec. 3.3) in fp32.
//
// One ray per lane, wave64, one wave per block.  The BVH node stack lives in
// LDS, interleaved by lane.  Traversal and patch intersection alternate in a
// while-while structure: every lane traverses until it reaches a candidate
// patch (or finishes), then the lanes holding a candidate run Alg. 3 together.
//
// Alg. 3 state per lane (registers only, no stack):
//   code  interleaved path bits of the current domain; split k (u at even k)
//         owns bit 2L-1-k and is set when the upper half was taken;
//   trail same bit layout; a set bit marks a pending sibling (both halves hit);
//   depth number of splits on the path (next axis: u iff depth is even);
//   G     the current grid (lower bounding grid for a Gregory patch), held so
//         that the split runs along its first index; mirror bits per axis;
//   d     the Gregory displacement of the current domain (0 for Bezier).
// Backtracking takes the lowest set trail bit (the deepest pending level, one
// count-trailing-zeros for both axes at once), flips that path bit, clears the
// bits below it, and recomputes the grid of the new domain from the patch.
// A pair of leaf children is resolved at its parent: the closer one hit is
// recorded, its sibling cannot be closer (Sec. 3.3) and is never queued.

#include "ccs_internal.h"
#include "patch_math.h"

namespace ccs {

constexpr int kBlock = 64;
constexpr int kStack = 48;

struct Best {
  float t;
  uint32_t id;
  float u, v;
};

struct Counts {
  uint32_t node, cand, split, backtrack, greg, leaf, crop, cand_greg;
};

__device__ __forceinline__ float safe_inv(float d) {
  // a zero component gets a huge finite reciprocal: the slab of that axis is then
  // unbounded for origins between the planes and empty otherwise, without 0*inf
  return d == 0.0f ? copysignf(1e30f, d) : __frcp_rn(d);
}

// Bounds of the current grid's two halves and the slab tests against them.
struct StepResult {
  Split1 sx, sy, sz;
  float ta, tb;
  bool ha, hb;
};

template <bool kStats>
__device__ __forceinline__ void intersect_patch(const float* __restrict__ rec, float wox, float woy, float woz,
                                                const RayP& wr, int L, Best& best, Counts& cnt) {
  const float4 meta = reinterpret_cast<const float4*>(rec)[15];
  const uint32_t mbits = __float_as_uint(meta.w);
  const bool greg = (mbits & kGregoryBit) != 0;
  const uint32_t pid = mbits & kIdMask;
  if (kStats) cnt.cand_greg += greg ? 1u : 0u;
  RayP r;
  r.ox = wox - meta.x;
  r.oy = woy - meta.y;
  r.oz = woz - meta.z;
  r.ix = wr.ix;
  r.iy = wr.iy;
  r.iz = wr.iz;
  r.cx = -r.ox * r.ix;
  r.cy = -r.oy * r.iy;
  r.cz = -r.oz * r.iz;
  r.tmin = wr.tmin;

  const int L2 = 2 * L;
  const float leaf_scale = __uint_as_float((uint32_t)(127 - L) << 23);  // 2^-L
  Grid G;
  float dx, dy, dz;
  uint32_t code = 0, trail = 0, mirror = 0;
  int depth = 0;
  bool need_grid = true;

  for (;;) {
    if (need_grid && !greg && depth == 0) {
      // Bezier root: the grid is the patch itself
      PatchPts P;
      load_grid(rec, P, false);
      orient(P.x, false, G.x);
      orient(P.y, false, G.y);
      orient(P.z, false, G.z);
      dx = dy = dz = 0.0f;
      need_grid = false;
    }
    if (need_grid) {
      // domain of the node at `depth`: pos from the path code, sizes from the depth
      const float u0 = (float)compact_even(code >> 1) * leaf_scale;
      const float v0 = (float)compact_even(code) * leaf_scale;
      const float su = __uint_as_float((uint32_t)(127 - ((depth + 1) >> 1)) << 23);
      const float sv = __uint_as_float((uint32_t)(127 - (depth >> 1)) << 23);
      PatchPts P;
      load_grid(rec, P, greg);
      float qx[4][4], qy[4][4], qz[4][4];
      calc_points_and_d(P, greg, u0, u0 + su, v0, v0 + sv, qx, qy, qz, dx, dy, dz);
      const bool along_v = (depth & 1) != 0;
      orient(qx, along_v, G.x);
      orient(qy, along_v, G.y);
      orient(qz, along_v, G.z);
      mirror = 0;
      need_grid = false;
      if (kStats && greg) cnt.greg++;
    }
    if (kStats) cnt.split++;
    const Split1 sx = split_component(G.x);
    const Split1 sy = split_component(G.y);
    const Split1 sz = split_component(G.z);
    const float ta = slab(r, sx.lo_a, sy.lo_a, sz.lo_a, sx.hi_a + dx, sy.hi_a + dy, sz.hi_a + dz, best.t);
    const float tb = slab(r, sx.lo_b, sy.lo_b, sz.lo_b, sx.hi_b + dx, sy.hi_b + dy, sz.hi_b + dz, best.t);
    const bool ha = ta != __builtin_inff(), hb = tb != __builtin_inff();
    const int axis = depth & 1;
    const bool mir = ((mirror >> axis) & 1u) != 0;
    const bool h_lo = mir ? hb : ha, h_up = mir ? ha : hb;
    const float t_lo = mir ? tb : ta, t_up = mir ? ta : tb;
    const bool go_up = h_up && (!h_lo || t_up < t_lo);
    const uint32_t bit = 1u << (L2 - 1 - depth);
    bool backtrack = !(ha || hb);
    if (!backtrack) {
      if (depth == L2 - 1) {
        const float tf = go_up ? t_up : t_lo;
        if (tf < best.t || (tf == best.t && pid < best.id)) {
          const uint32_t lc = code | (go_up ? bit : 0u);
          best.t = tf;
          best.id = pid;
          best.u = (float)(2u * compact_even(lc >> 1) + 1u) * (0.5f * leaf_scale);
          best.v = (float)(2u * compact_even(lc) + 1u) * (0.5f * leaf_scale);
          if (kStats) cnt.leaf++;
        }
        backtrack = true;
      } else {
        if (ha && hb) trail |= bit;
        if (go_up) code |= bit;
        const bool second = go_up != mir;
        take_half(sx, second, G.x);
        take_half(sy, second, G.y);
        take_half(sz, second, G.z);
        if (second) mirror ^= (1u << axis);
        depth++;
        need_grid = greg;  // Alg. 3 recomputes a Gregory grid at every node
      }
    }
    if (backtrack) {
      if (trail == 0) break;
      const int b = __builtin_ctz(trail);
      const uint32_t tb_bit = 1u << b;
      trail ^= tb_bit;
      code = (code ^ tb_bit) & ~(tb_bit - 1u);
      depth = L2 - b;
      need_grid = true;
      if (kStats) {
        cnt.backtrack++;
        cnt.crop += greg ? 0u : 1u;
      }
    }
  }
}

__device__ __forceinline__ void node_boxes(const float4* __restrict__ nodes, int idx, float4& a, float4& b, float4& c,
                                           int& c0, int& c1) {
  const float4* n = nodes + 4 * (size_t)idx;
  a = n[0];
  b = n[1];
  c = n[2];
  const float4 d = n[3];
  c0 = __float_as_int(d.x);
  c1 = __float_as_int(d.y);
}

template <bool kStats>
__global__ __launch_bounds__(kBlock) void k_intersect(DeviceScene s, const ccs_ray* __restrict__ rays, uint32_t n,
                                                      ccs_hit* __restrict__ hits, uint32_t* __restrict__ counters) {
  __shared__ int stack[kStack * kBlock];
  const int lane = threadIdx.x;
  const uint32_t i = blockIdx.x * kBlock + lane;
  if (i >= n) return;
  const float4* r4 = reinterpret_cast<const float4*>(rays + i);
  const float4 ro = r4[0], rd = r4[1];
  Best best = {rd.w, kNoHit, 0.0f, 0.0f};
  Counts cnt = {0, 0, 0, 0, 0, 0, 0, 0};
  const bool finite = isfinite(ro.x) && isfinite(ro.y) && isfinite(ro.z) && isfinite(rd.x) && isfinite(rd.y) &&
                      isfinite(rd.z) && !isnan(ro.w) && !isnan(rd.w);
  const bool valid = finite && !(rd.x == 0.0f && rd.y == 0.0f && rd.z == 0.0f) && ro.w <= rd.w &&
                     s.n_nodes > 0;
  RayP wr;
  wr.ox = ro.x;
  wr.oy = ro.y;
  wr.oz = ro.z;
  wr.ix = safe_inv(rd.x);
  wr.iy = safe_inv(rd.y);
  wr.iz = safe_inv(rd.z);
  wr.cx = -ro.x * wr.ix;
  wr.cy = -ro.y * wr.iy;
  wr.cz = -ro.z * wr.iz;
  wr.tmin = ro.w;

  // state: cur >= 0 internal node to visit; cur < 0 patch record ~cur; done when !alive
  int cur = 0;
  bool alive = valid;
  int sp = 0;
  while (alive) {
    // traversal until a candidate patch is reached or the stack runs dry
    while (alive && cur >= 0) {
      if (kStats) cnt.node++;
      float4 a, b, c;
      int c0, c1;
      node_boxes(s.nodes, cur, a, b, c, c0, c1);
      const float t0 = slab(wr, a.x, a.y, a.z, a.w, b.x, b.y, best.t);
      const float t1 = slab(wr, b.z, b.w, c.x, c.y, c.z, c.w, best.t);
      const bool h0 = t0 != __builtin_inff(), h1 = t1 != __builtin_inff();
      if (h0 && h1) {
        const bool first1 = t1 < t0;
        // the host rejects BVHs deeper than kStack, so sp < kStack always holds here
        if (sp < kStack) {
          stack[sp * kBlock + lane] = first1 ? c0 : c1;
          ++sp;
        }
        cur = first1 ? c1 : c0;
      } else if (h0 || h1) {
        cur = h0 ? c0 : c1;
      } else if (sp > 0) {
        --sp;
        cur = stack[sp * kBlock + lane];
      } else {
        alive = false;
      }
    }
    if (alive) {
      if (kStats) cnt.cand++;
      const uint32_t r = (uint32_t)(~cur);
      intersect_patch<kStats>(s.recs + (size_t)r * kRecFloats, ro.x, ro.y, ro.z, wr, s.leaf_depth, best, cnt);
      if (sp > 0) {
        --sp;
        cur = stack[sp * kBlock + lane];
      } else {
        alive = false;
      }
    }
  }
  const bool hit = best.id != kNoHit;
  float4 h;
  h.x = hit ? best.t : __builtin_inff();
  h.y = __uint_as_float(best.id);
  h.z = hit ? best.u : 0.0f;
  h.w = hit ? best.v : 0.0f;
  reinterpret_cast<float4*>(hits)[i] = h;
  if (kStats) {
    uint4* c = reinterpret_cast<uint4*>(counters + 8 * (size_t)i);
    c[0] = make_uint4(cnt.node, cnt.cand, cnt.split, cnt.backtrack);
    c[1] = make_uint4(cnt.greg, cnt.leaf, cnt.crop, cnt.cand_greg);
  }
}

hipError_t launch_intersect(const DeviceScene& s, const ccs_ray* rays, uint32_t n, ccs_hit* hits, uint32_t* counters,
                            hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const dim3 grid((n + kBlock - 1) / kBlock), block(kBlock);
  if (counters)
    hipLaunchKernelGGL(k_intersect<true>, grid, block, 0, stream, s, rays, n, hits, counters);
  else
    hipLaunchKernelGGL(k_intersect<false>, grid, block, 0, stream, s, rays, n, hits, nullptr);
  return hipGetLastError();
}

}  // namespace ccs
