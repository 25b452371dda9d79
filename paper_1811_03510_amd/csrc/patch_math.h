// Device-side patch arithmetic for the gfx950 intersector (fp32, registers).
//
// Patch records (kRecFloats floats, 256-byte aligned, BVH-leaf order):
//   [ 0,16) x of grid slots 0..15, [16,32) y, [32,48) z   (anchored: p - anchor)
//   [48,52) x of P^v for the inner points, [52,56) y, [56,60) z (anchored)
//   [60,63) anchor (world), [63] meta bits: original patch index | kGregoryBit
// Slot(i, j) = 4*j + i, i along u, j along v.  Inner slots 5, 6, 9, 10 hold P^u.
//
// The working grid G[a][b] is held so that the next split always runs along the
// first index a (Sec. 3.5: transposing after every split and recomputation lets
// all lanes split along one direction).  A chosen child is written back
// transposed; an upper child is kept mirrored (a3 first) so that choosing it
// costs three selects per row instead of four.  Per parametric axis one mirror
// bit records whether register order runs against the parameter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccs {

constexpr int kRecFloats = 64;
constexpr uint32_t kGregoryBit = 0x80000000u;
constexpr uint32_t kIdMask = 0x7FFFFFFFu;
constexpr uint32_t kNoHit = 0xFFFFFFFFu;

struct Grid {
  float x[4][4], y[4][4], z[4][4];
};

struct Box {
  float lx, ly, lz, hx, hy, hz;
};

__device__ __forceinline__ float mid(float a, float b) { return (a + b) * 0.5f; }
__device__ __forceinline__ float min4(float a, float b, float c, float d) { return fminf(fminf(a, b), fminf(c, d)); }
__device__ __forceinline__ float max4(float a, float b, float c, float d) { return fmaxf(fmaxf(a, b), fmaxf(c, d)); }

// Seven de Casteljau points of one cubic split at 1/2: a0, m01, m012, m, m123, m23, a3.
struct Row7 {
  float v[7];
};

__device__ __forceinline__ Row7 casteljau_half(float a0, float a1, float a2, float a3) {
  Row7 r;
  float m01 = mid(a0, a1), m12 = mid(a1, a2), m23 = mid(a2, a3);
  float m012 = mid(m01, m12), m123 = mid(m12, m23);
  r.v[0] = a0;
  r.v[1] = m01;
  r.v[2] = m012;
  r.v[3] = mid(m012, m123);
  r.v[4] = m123;
  r.v[5] = m23;
  r.v[6] = a3;
  return r;
}

// Running slab test of the two child boxes, one component at a time, so that a
// component's box bounds die as soon as they are folded in.  na/fa: entry and
// exit of the register-first half so far, nb/fb: of the second half.
struct SlabPair {
  float na, fa, nb, fb;
};

// Splits component g, folds its child intervals [lo, hi + d] into s, and returns
// the seven points of every row.  Each half's bounds over its 16 points are
// linear chains of two-value steps, which the compiler folds into one
// three-operand min / max per two points (min and max are exact, so the order
// does not change the bounds).
__device__ __forceinline__ void split_fold(const float g[4][4], float o, float inv, float d, Row7 e[4], SlabPair& s) {
#pragma unroll
  for (int b = 0; b < 4; ++b) e[b] = casteljau_half(g[0][b], g[1][b], g[2][b], g[3][b]);
  float la = fminf(e[0].v[0], e[0].v[1]), ha = fmaxf(e[0].v[0], e[0].v[1]);
  float lb = fminf(e[0].v[3], e[0].v[4]), hb = fmaxf(e[0].v[3], e[0].v[4]);
  la = fminf(fminf(la, e[0].v[2]), e[0].v[3]);
  ha = fmaxf(fmaxf(ha, e[0].v[2]), e[0].v[3]);
  lb = fminf(fminf(lb, e[0].v[5]), e[0].v[6]);
  hb = fmaxf(fmaxf(hb, e[0].v[5]), e[0].v[6]);
#pragma unroll
  for (int b = 1; b < 4; ++b) {
    la = fminf(fminf(la, e[b].v[0]), e[b].v[1]);
    la = fminf(fminf(la, e[b].v[2]), e[b].v[3]);
    ha = fmaxf(fmaxf(ha, e[b].v[0]), e[b].v[1]);
    ha = fmaxf(fmaxf(ha, e[b].v[2]), e[b].v[3]);
    lb = fminf(fminf(lb, e[b].v[3]), e[b].v[4]);
    lb = fminf(fminf(lb, e[b].v[5]), e[b].v[6]);
    hb = fmaxf(fmaxf(hb, e[b].v[3]), e[b].v[4]);
    hb = fmaxf(fmaxf(hb, e[b].v[5]), e[b].v[6]);
  }
  const float a0 = (la - o) * inv, a1 = (ha + d - o) * inv;
  const float b0 = (lb - o) * inv, b1 = (hb + d - o) * inv;
  s.na = fmaxf(s.na, fminf(a0, a1));
  s.fa = fminf(s.fa, fmaxf(a0, a1));
  s.nb = fmaxf(s.nb, fminf(b0, b1));
  s.fb = fminf(s.fb, fmaxf(b0, b1));
}

// The box of one component of a whole grid, [min, max + d], folded into the
// slab interval (na, fa) of s (the fields nb, fb are left alone).
__device__ __forceinline__ void grid_fold(const float g[4][4], float o, float inv, float d, SlabPair& s) {
  float lo = fminf(g[0][0], g[0][1]), hi = fmaxf(g[0][0], g[0][1]);
  lo = fminf(fminf(lo, g[0][2]), g[0][3]);
  hi = fmaxf(fmaxf(hi, g[0][2]), g[0][3]);
#pragma unroll
  for (int a = 1; a < 4; ++a) {
    lo = fminf(fminf(lo, g[a][0]), g[a][1]);
    lo = fminf(fminf(lo, g[a][2]), g[a][3]);
    hi = fmaxf(fmaxf(hi, g[a][0]), g[a][1]);
    hi = fmaxf(fmaxf(hi, g[a][2]), g[a][3]);
  }
  const float a0 = (lo - o) * inv, a1 = (hi + d - o) * inv;
  s.na = fmaxf(s.na, fminf(a0, a1));
  s.fa = fminf(s.fa, fmaxf(a0, a1));
}

// Chosen half written back transposed: new G[b][k] = point k of row b, the
// second half taken mirrored (a3, m23, m123, m).
__device__ __forceinline__ void take_half(const Row7 e[4], bool second, float g[4][4]) {
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    g[b][0] = second ? e[b].v[6] : e[b].v[0];
    g[b][1] = second ? e[b].v[5] : e[b].v[1];
    g[b][2] = second ? e[b].v[4] : e[b].v[2];
    g[b][3] = e[b].v[3];
  }
}

// ---------------------------------------------------------------- ray / box
struct RayP {  // a ray in some frame: origin, reciprocal direction, tmin
  float ox, oy, oz;
  float ix, iy, iz;  // 1/d (zero components replaced by +-1e30)
  float tmin;
};

// Widening of the far distance that makes the fp32 slab test conservative
// against rounding (robust BVH traversal of Ize 2013, cited in Sec. 3.4).  A
// distance is formed as (plane - o) * (1/d): the difference and the product are
// rounded once each (u = 2^-24 relative), and 1/d comes from the hardware
// reciprocal, within 1 ulp (2u relative), so each distance carries at most
// gamma_4 = 4u / (1 - 4u) of relative error and an entry can exceed its exit by
// rounding alone by 2 gamma_4 of the exit's magnitude.  (A precomputed -o/d
// would carry an error relative to |o|/|d|, not to the distance.)
// kFarScale = 1 + 5 * 2^-23, the first fp32 value above 1 + 2 gamma_4.
constexpr float kFarScale = 1.0f + 5.0f * 1.1920929e-7f;
// The same widening for a negative far distance (patch-frame distances are measured
// from the ray's point closest to the patch anchor, so a box the ray leaves before
// that point has a negative far distance): 1 - 10 * 2^-24, below 1 - 2 gamma_4.
constexpr float kFarShrink = 1.0f - 10.0f * 5.9604645e-8f;

// A far distance moved outwards by 2 gamma_4 of its magnitude, whatever its sign
// (a plain product by kFarScale would pull a negative one inwards, and a box of zero
// thickness, where entry equals exit, would then be missed).
__device__ __forceinline__ float widen_far(float f) { return f * (f >= 0.0f ? kFarScale : kFarShrink); }

// Reciprocal of a direction component from the hardware reciprocal (within
// 1 ulp), branch-free; a zero component gets a huge finite reciprocal, so that the
// slab of that axis is unbounded for origins between the planes and empty
// otherwise, without 0 * inf.
__device__ __forceinline__ float safe_inv(float d) {
  const float r = __builtin_amdgcn_rcpf(d);
  return d == 0.0f ? copysignf(1e30f, d) : r;
}

// Patch frame of a ray: anchored at the patch's anchor, origin moved along the
// ray to (about) the point closest to the anchor, computed in double and rounded
// once.  Distances inside the patch are then of the patch's size, so their
// rounding, and the conservative widening of the slab test that covers it, are
// relative to the patch rather than to the distance from the ray origin (Sec.
// 3.4: anchoring for precision).  Any t0 gives the same ray; patch-frame
// distances are world distances minus t0.
__device__ __forceinline__ void patch_frame(float4 anchor, float ox, float oy, float oz, float dx, float dy, float dz,
                                            float tmin, float& pox, float& poy, float& poz, float& ptmin, float& t0) {
  const float qx = anchor.x - ox, qy = anchor.y - oy, qz = anchor.z - oz;
  t0 = (qx * dx + qy * dy + qz * dz) * __builtin_amdgcn_rcpf(dx * dx + dy * dy + dz * dz);
  pox = (float)fma((double)t0, (double)dx, (double)ox - (double)anchor.x);
  poy = (float)fma((double)t0, (double)dy, (double)oy - (double)anchor.y);
  poz = (float)fma((double)t0, (double)dz, (double)oz - (double)anchor.z);
  ptmin = (float)((double)tmin - (double)t0);
}

// Patch frame of a ray in a patch-local frame (rows r0, r1, r2): the anchored
// origin of patch_frame and the direction are mapped by the rows in double and
// rounded once, so that the mapped ray is as exact as the stored mapped patch
// (rounding a mapped direction twice would tilt it, and a grazing ray would then
// meet the surface leaves away).
__device__ __forceinline__ void patch_frame_rows(float4 anchor, float4 r0, float4 r1, float4 r2, float ox, float oy,
                                                 float oz, float dx, float dy, float dz, float tmin, float& pox,
                                                 float& poy, float& poz, float& pdx, float& pdy, float& pdz,
                                                 float& ptmin, float& t0) {
  const float qx = anchor.x - ox, qy = anchor.y - oy, qz = anchor.z - oz;
  t0 = (qx * dx + qy * dy + qz * dz) * __builtin_amdgcn_rcpf(dx * dx + dy * dy + dz * dz);
  const double ax = fma((double)t0, (double)dx, (double)ox - (double)anchor.x);
  const double ay = fma((double)t0, (double)dy, (double)oy - (double)anchor.y);
  const double az = fma((double)t0, (double)dz, (double)oz - (double)anchor.z);
  const double ex = dx, ey = dy, ez = dz;
  pox = (float)fma((double)r0.z, az, fma((double)r0.y, ay, (double)r0.x * ax));
  poy = (float)fma((double)r1.z, az, fma((double)r1.y, ay, (double)r1.x * ax));
  poz = (float)fma((double)r2.z, az, fma((double)r2.y, ay, (double)r2.x * ax));
  pdx = (float)fma((double)r0.z, ez, fma((double)r0.y, ey, (double)r0.x * ex));
  pdy = (float)fma((double)r1.z, ez, fma((double)r1.y, ey, (double)r1.x * ex));
  pdz = (float)fma((double)r2.z, ez, fma((double)r2.y, ey, (double)r2.x * ex));
  ptmin = (float)((double)tmin - (double)t0);
}

// Closed slab test on [tmin, cap]; returns the entry distance or +inf when missed.
__device__ __forceinline__ float slab(const RayP& r, float lx, float ly, float lz, float hx, float hy, float hz,
                                      float cap) {
  const float tx0 = (lx - r.ox) * r.ix, tx1 = (hx - r.ox) * r.ix;
  const float ty0 = (ly - r.oy) * r.iy, ty1 = (hy - r.oy) * r.iy;
  const float tz0 = (lz - r.oz) * r.iz, tz1 = (hz - r.oz) * r.iz;
  const float nr = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), r.tmin));
  float fr = widen_far(fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1)));
  fr = fminf(fr, cap);
  return nr <= fr ? nr : __builtin_inff();
}

// ------------------------------------------------------------ crop (blossom)
// Rows of the 4x4 matrix taking cubic Bezier points to those of the restriction
// to [t0, t1]: row k is the blossom of the Bernstein basis at (t0^(3-k), t1^k).
// Entries are non-negative and each row sums to 1, so the crop is a convex
// combination of the original points (no cancellation).
struct Crop4 {
  float m[4][4];
};

__device__ __forceinline__ Crop4 crop_matrix(float t0, float t1) {
  float s0 = 1.0f - t0, s1 = 1.0f - t1;
  Crop4 c;
  float s00 = s0 * s0, t00 = t0 * t0, s11 = s1 * s1, t11 = t1 * t1, ts0 = t0 * s0, ts1 = t1 * s1;
  c.m[0][0] = s00 * s0;
  c.m[0][1] = 3.0f * ts0 * s0;
  c.m[0][2] = 3.0f * ts0 * t0;
  c.m[0][3] = t00 * t0;
  c.m[1][0] = s00 * s1;
  c.m[1][1] = fmaf(2.0f * ts0, s1, s00 * t1);
  c.m[1][2] = fmaf(t00, s1, 2.0f * ts0 * t1);
  c.m[1][3] = t00 * t1;
  c.m[2][0] = s0 * s11;
  c.m[2][1] = fmaf(t0, s11, 2.0f * s0 * ts1);
  c.m[2][2] = fmaf(2.0f * t0, ts1, s0 * t11);
  c.m[2][3] = t0 * t11;
  c.m[3][0] = s11 * s1;
  c.m[3][1] = 3.0f * ts1 * s1;
  c.m[3][2] = 3.0f * ts1 * t1;
  c.m[3][3] = t11 * t1;
  return c;
}

// q[i][j] (i along u, j along v) = restriction of p (p[i][j]) to [u0,u1] x [v0,v1].
__device__ __forceinline__ void crop_component(const float p[4][4], const Crop4& mu, const Crop4& mv,
                                               float q[4][4]) {
  float r[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      r[i][j] = fmaf(mu.m[i][3], p[3][j], fmaf(mu.m[i][2], p[2][j], fmaf(mu.m[i][1], p[1][j], mu.m[i][0] * p[0][j])));
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      q[i][j] = fmaf(mv.m[j][3], r[i][3], fmaf(mv.m[j][2], r[i][2], fmaf(mv.m[j][1], r[i][1], mv.m[j][0] * r[i][0])));
}

// Store q (canonical [i][j]) into the working grid oriented for a split along
// u (axis 0: G = q) or v (axis 1: G = q^T).
__device__ __forceinline__ void orient(const float q[4][4], bool along_v, float g[4][4]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) g[a][b] = (a == b) ? q[a][b] : (along_v ? q[b][a] : q[a][b]);
}

// Maximum over [t0, t1] of the Bernstein weight B_1 (k = 1) or B_2 (k = 2) of
// degree 3: evaluated at the peak 1/3 resp. 2/3 clamped into the interval (Alg. 2).
__device__ __forceinline__ float wbar1(float t0, float t1) {
  float t = fminf(fmaxf(0.33333334f, t0), t1);
  float s = 1.0f - t;
  return 3.0f * t * s * s;
}
__device__ __forceinline__ float wbar2(float t0, float t1) {
  float t = fminf(fmaxf(0.6666667f, t0), t1);
  return 3.0f * t * t * (1.0f - t);
}

// Patch points loaded from a record: the 16 grid points p[i][j] and, for a
// Gregory patch, the four P^v (inner order (1,1), (2,1), (1,2), (2,2)).
struct PatchPts {
  float x[4][4], y[4][4], z[4][4];
  float vx[4], vy[4], vz[4];
};

__device__ __forceinline__ void load_grid(const float* __restrict__ rec, PatchPts& P, bool gregory) {
  const float4* r4 = reinterpret_cast<const float4*>(rec);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float4 x = r4[j], y = r4[4 + j], z = r4[8 + j];
    P.x[0][j] = x.x; P.x[1][j] = x.y; P.x[2][j] = x.z; P.x[3][j] = x.w;
    P.y[0][j] = y.x; P.y[1][j] = y.y; P.y[2][j] = y.z; P.y[3][j] = y.w;
    P.z[0][j] = z.x; P.z[1][j] = z.y; P.z[2][j] = z.z; P.z[3][j] = z.w;
  }
  if (gregory) {
    float4 vx = r4[12], vy = r4[13], vz = r4[14];
    P.vx[0] = vx.x; P.vx[1] = vx.y; P.vx[2] = vx.z; P.vx[3] = vx.w;
    P.vy[0] = vy.x; P.vy[1] = vy.y; P.vy[2] = vy.z; P.vy[3] = vy.w;
    P.vz[0] = vz.x; P.vz[1] = vz.y; P.vz[2] = vz.z; P.vz[3] = vz.w;
  }
}

// calcPointsAndD (Alg. 2) on [u0,u1] x [v0,v1]: the lower bounding Bezier grid
// restricted to the domain (canonical orientation) and the displacement d of the
// upper bound.  For a Bezier patch d = 0 and the grid is the plain restriction.
// Inner point k of a Gregory patch is bounded by the blends A, B at its smallest
// and largest weight on P^u over the domain (the weight is monotone in u and v,
// Sec. 3.2); A = P^v + lam (P^u - P^v), lam = du / (du + dv) at the extreme corner.
__device__ __forceinline__ void calc_points_and_d(const PatchPts& P, bool gregory, float u0, float u1, float v0,
                                                  float v1, float qx[4][4], float qy[4][4], float qz[4][4],
                                                  float& dx, float& dy, float& dz) {
  float gx[4][4], gy[4][4], gz[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      gx[i][j] = P.x[i][j];
      gy[i][j] = P.y[i][j];
      gz[i][j] = P.z[i][j];
    }
  dx = dy = dz = 0.0f;
  if (gregory) {
    const float wu1 = wbar1(u0, u1), wu2 = wbar2(u0, u1), wv1 = wbar1(v0, v1), wv2 = wbar2(v0, v1);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = (k & 1) ? 2 : 1, j = (k & 2) ? 2 : 1;
      const float dul = (i == 1) ? u0 : 1.0f - u1, duh = (i == 1) ? u1 : 1.0f - u0;
      const float dvl = (j == 1) ? v0 : 1.0f - v1, dvh = (j == 1) ? v1 : 1.0f - v0;
      // hardware reciprocal (1 ulp): moves A, B by a rounding-sized amount, like the crop itself
      const float lam_lo = dul * __builtin_amdgcn_rcpf(dul + dvh), lam_hi = duh * __builtin_amdgcn_rcpf(duh + dvl);
      const float w = ((i == 1) ? wu1 : wu2) * ((j == 1) ? wv1 : wv2);
      const float px = P.x[i][j], py = P.y[i][j], pz = P.z[i][j];
      const float ex = px - P.vx[k], ey = py - P.vy[k], ez = pz - P.vz[k];
      const float ax = fmaf(lam_lo, ex, P.vx[k]), bx = fmaf(lam_hi, ex, P.vx[k]);
      const float ay = fmaf(lam_lo, ey, P.vy[k]), by = fmaf(lam_hi, ey, P.vy[k]);
      const float az = fmaf(lam_lo, ez, P.vz[k]), bz = fmaf(lam_hi, ez, P.vz[k]);
      gx[i][j] = fminf(ax, bx);
      gy[i][j] = fminf(ay, by);
      gz[i][j] = fminf(az, bz);
      dx = fmaf(w, fabsf(ax - bx), dx);
      dy = fmaf(w, fabsf(ay - by), dy);
      dz = fmaf(w, fabsf(az - bz), dz);
    }
  }
  const Crop4 mu = crop_matrix(u0, u1), mv = crop_matrix(v0, v1);
  crop_component(gx, mu, mv, qx);
  crop_component(gy, mu, mv, qy);
  crop_component(gz, mu, mv, qz);
}

// One component (x, y or z) of calc_points_and_d, with the same operations in
// the same order: rc holds the record's 16 grid values of the component (slot
// 4j + i at rc[4j + i]), rv its four P^v values.  Used when the three components
// of a lane's grid are computed by three lanes.
__device__ __forceinline__ void calc_component(const float* __restrict__ rc, const float* __restrict__ rv,
                                               bool gregory, float u0, float u1, float v0, float v1, float q[4][4],
                                               float& d) {
  float g[4][4];
  const float4* r4 = reinterpret_cast<const float4*>(rc);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float4 x = r4[j];
    g[0][j] = x.x;
    g[1][j] = x.y;
    g[2][j] = x.z;
    g[3][j] = x.w;
  }
  d = 0.0f;
  if (gregory) {
    const float4 pv = *reinterpret_cast<const float4*>(rv);
    const float vv[4] = {pv.x, pv.y, pv.z, pv.w};
    const float wu1 = wbar1(u0, u1), wu2 = wbar2(u0, u1), wv1 = wbar1(v0, v1), wv2 = wbar2(v0, v1);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = (k & 1) ? 2 : 1, j = (k & 2) ? 2 : 1;
      const float dul = (i == 1) ? u0 : 1.0f - u1, duh = (i == 1) ? u1 : 1.0f - u0;
      const float dvl = (j == 1) ? v0 : 1.0f - v1, dvh = (j == 1) ? v1 : 1.0f - v0;
      const float lam_lo = dul * __builtin_amdgcn_rcpf(dul + dvh), lam_hi = duh * __builtin_amdgcn_rcpf(duh + dvl);
      const float w = ((i == 1) ? wu1 : wu2) * ((j == 1) ? wv1 : wv2);
      const float e = g[i][j] - vv[k];
      const float a = fmaf(lam_lo, e, vv[k]), b = fmaf(lam_hi, e, vv[k]);
      g[i][j] = fminf(a, b);
      d = fmaf(w, fabsf(a - b), d);
    }
  }
  const Crop4 mu = crop_matrix(u0, u1), mv = crop_matrix(v0, v1);
  crop_component(g, mu, mv, q);
}

// Position of the r-th set bit (from 0) of m; r < popcount(m).
__device__ __forceinline__ uint32_t nth_set_bit(uint64_t m, uint32_t r) {
  uint32_t pos = 0;
  uint32_t c = (uint32_t)__popc((uint32_t)m);
  if (r >= c) {
    r -= c;
    m >>= 32;
    pos = 32;
  }
  uint32_t x = (uint32_t)m;
#pragma unroll
  for (int w = 16; w >= 1; w >>= 1) {
    c = (uint32_t)__popc(x & ((1u << w) - 1u));
    if (r >= c) {
      r -= c;
      x >>= w;
      pos += (uint32_t)w;
    }
  }
  return pos;
}

// Bits of a 2L-bit interleaved path code: split k (0-based, u at even k) owns bit
// 2L-1-k, so u bits sit at odd and v bits at even positions.
__device__ __forceinline__ uint32_t compact_even(uint32_t x) {
  x &= 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0F0F0F0Fu;
  x = (x | (x >> 4)) & 0x00FF00FFu;
  x = (x | (x >> 8)) & 0x0000FFFFu;
  return x;
}
// The same for a 64-bit code (leaf depths above 16): the even bits of the high
// word follow those of the low word.
__device__ __forceinline__ uint32_t compact_even(uint64_t x) {
  return compact_even((uint32_t)x) | (compact_even((uint32_t)(x >> 32)) << 16);
}

}  // namespace ccs
