// Secondary rays from hits (Sec. 3.3): the origin o + t d is moved along the
// unit surface normal (turned against d) by the L1 size of the box of the leaf
// domain containing (u, v); the direction is cosine-weighted about the normal.

#include "ccs_internal.h"
#include "patch_math.h"

namespace ccs {

constexpr int kBounceBlock = 256;

__device__ __forceinline__ void bern3(float t, float b[4], float db[4]) {
  const float s = 1.0f - t;
  b[0] = s * s * s;
  b[1] = 3.0f * t * s * s;
  b[2] = 3.0f * t * t * s;
  b[3] = t * t * t;
  db[0] = -3.0f * s * s;
  db[1] = 3.0f * s * s - 6.0f * t * s;
  db[2] = 6.0f * t * s - 3.0f * t * t;
  db[3] = 3.0f * t * t;
}

// f_u and f_v of a Bezier or Gregory patch at (u, v); a Gregory patch adds the
// derivative of the blend weight of each inner point.
__device__ void patch_partials(const PatchPts& P, bool greg, float u, float v, float fu[3], float fv[3]) {
  float bu[4], du[4], bv[4], dv[4];
  bern3(u, bu, du);
  bern3(v, bv, dv);
  float gx[4][4], gy[4][4], gz[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      gx[i][j] = P.x[i][j];
      gy[i][j] = P.y[i][j];
      gz[i][j] = P.z[i][j];
    }
  float lu[4] = {0, 0, 0, 0}, lv[4] = {0, 0, 0, 0};
  if (greg) {
    for (int k = 0; k < 4; ++k) {
      const int i = (k & 1) ? 2 : 1, j = (k & 2) ? 2 : 1;
      const float a = (i == 1) ? u : 1.0f - u, b = (j == 1) ? v : 1.0f - v;
      const float den = a + b;
      const float ex = P.x[i][j] - P.vx[k], ey = P.y[i][j] - P.vy[k], ez = P.z[i][j] - P.vz[k];
      if (den > 0.0f) {
        const float lam = a / den;
        gx[i][j] = fmaf(lam, ex, P.vx[k]);
        gy[i][j] = fmaf(lam, ey, P.vy[k]);
        gz[i][j] = fmaf(lam, ez, P.vz[k]);
        const float inv2 = 1.0f / (den * den);
        lu[k] = ((i == 1) ? 1.0f : -1.0f) * b * inv2;
        lv[k] = -((j == 1) ? 1.0f : -1.0f) * a * inv2;
      } else {
        gx[i][j] = fmaf(0.5f, ex, P.vx[k]);
        gy[i][j] = fmaf(0.5f, ey, P.vy[k]);
        gz[i][j] = fmaf(0.5f, ez, P.vz[k]);
      }
    }
  }
  for (int c = 0; c < 3; ++c) {
    fu[c] = 0.0f;
    fv[c] = 0.0f;
  }
  for (int j = 0; j < 4; ++j)
    for (int i = 0; i < 4; ++i) {
      const float wu = du[i] * bv[j], wv = bu[i] * dv[j];
      fu[0] = fmaf(wu, gx[i][j], fu[0]);
      fu[1] = fmaf(wu, gy[i][j], fu[1]);
      fu[2] = fmaf(wu, gz[i][j], fu[2]);
      fv[0] = fmaf(wv, gx[i][j], fv[0]);
      fv[1] = fmaf(wv, gy[i][j], fv[1]);
      fv[2] = fmaf(wv, gz[i][j], fv[2]);
    }
  if (greg) {
    for (int k = 0; k < 4; ++k) {
      const int i = (k & 1) ? 2 : 1, j = (k & 2) ? 2 : 1;
      const float w = bu[i] * bv[j];
      const float ex = P.x[i][j] - P.vx[k], ey = P.y[i][j] - P.vy[k], ez = P.z[i][j] - P.vz[k];
      fu[0] = fmaf(w * lu[k], ex, fu[0]);
      fu[1] = fmaf(w * lu[k], ey, fu[1]);
      fu[2] = fmaf(w * lu[k], ez, fu[2]);
      fv[0] = fmaf(w * lv[k], ex, fv[0]);
      fv[1] = fmaf(w * lv[k], ey, fv[1]);
      fv[2] = fmaf(w * lv[k], ez, fv[2]);
    }
  }
}

__global__ __launch_bounds__(kBounceBlock) void k_bounce(DeviceScene s, const ccs_ray* __restrict__ rays,
                                                         const ccs_hit* __restrict__ hits,
                                                         const float* __restrict__ uniforms, uint32_t n,
                                                         ccs_ray* __restrict__ out) {
  const uint32_t i = blockIdx.x * kBounceBlock + threadIdx.x;
  if (i >= n) return;
  const ccs_hit h = hits[i];
  ccs_ray o;
  if (h.patch_id >= s.n_patches || !isfinite(h.t)) {
    o.ox = o.oy = o.oz = 0.0f;
    o.tmin = 0.0f;
    o.dx = o.dy = 0.0f;
    o.dz = 1.0f;
    o.tmax = -1.0f;
    out[i] = o;
    return;
  }
  const ccs_ray r = rays[i];
  const uint32_t rec_idx = s.inv_perm[h.patch_id];
  const float* rec = s.recs + (size_t)rec_idx * kRecFloats;
  const bool greg = (__float_as_uint(rec[63]) & kGregoryBit) != 0;
  PatchPts P;
  load_grid(rec, P, greg);
  float fu[3], fv[3];
  patch_partials(P, greg, h.u, h.v, fu, fv);
  float nx = fu[1] * fv[2] - fu[2] * fv[1];
  float ny = fu[2] * fv[0] - fu[0] * fv[2];
  float nz = fu[0] * fv[1] - fu[1] * fv[0];
  if (s.frames) {  // record in the patch's frame: the normal back to world space (rows transposed)
    const float4 r0 = s.frames[3 * (size_t)rec_idx], r1 = s.frames[3 * (size_t)rec_idx + 1],
                 r2 = s.frames[3 * (size_t)rec_idx + 2];
    const float lx = nx, ly = ny, lz = nz;
    nx = r0.x * lx + r1.x * ly + r2.x * lz;
    ny = r0.y * lx + r1.y * ly + r2.y * lz;
    nz = r0.z * lx + r1.z * ly + r2.z * lz;
  }
  const float inv_len = 1.0f / sqrtf(nx * nx + ny * ny + nz * nz);
  nx *= inv_len;
  ny *= inv_len;
  nz *= inv_len;
  if (nx * r.dx + ny * r.dy + nz * r.dz > 0.0f) {
    nx = -nx;
    ny = -ny;
    nz = -nz;
  }
  // leaf domain containing (u, v); its box is taken in the frame the patch is subdivided in
  const uint32_t leaf = (1u << 23) >> s.leaf_depth;
  const uint32_t pu = min((uint32_t)floorf(h.u * 8388608.0f) & ~(leaf - 1u), (1u << 23) - leaf);
  const uint32_t pv = min((uint32_t)floorf(h.v * 8388608.0f) & ~(leaf - 1u), (1u << 23) - leaf);
  const float unit = 1.0f / 8388608.0f;
  float qx[4][4], qy[4][4], qz[4][4], dx, dy, dz;
  calc_points_and_d(P, greg, pu * unit, (pu + leaf) * unit, pv * unit, (pv + leaf) * unit, qx, qy, qz, dx, dy, dz);
  float lo[3] = {qx[0][0], qy[0][0], qz[0][0]}, hi[3] = {qx[0][0], qy[0][0], qz[0][0]};
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      lo[0] = fminf(lo[0], qx[a][b]); hi[0] = fmaxf(hi[0], qx[a][b]);
      lo[1] = fminf(lo[1], qy[a][b]); hi[1] = fmaxf(hi[1], qy[a][b]);
      lo[2] = fminf(lo[2], qz[a][b]); hi[2] = fmaxf(hi[2], qz[a][b]);
    }
  float off = (hi[0] + dx - lo[0]) + (hi[1] + dy - lo[1]) + (hi[2] + dz - lo[2]);
  if (s.frames) off += 6.0f * s.frames[3 * (size_t)rec_idx].w;  // the box pad on both sides of 3 axes
  o.ox = fmaf(off, nx, fmaf(h.t, r.dx, r.ox));
  o.oy = fmaf(off, ny, fmaf(h.t, r.dy, r.oy));
  o.oz = fmaf(off, nz, fmaf(h.t, r.dz, r.oz));
  o.tmin = 0.0f;
  // cosine-weighted direction: polar map of the unit disk lifted to the hemisphere
  const float u1 = uniforms[2 * (size_t)i], u2 = uniforms[2 * (size_t)i + 1];
  const float rr = sqrtf(u1), z = sqrtf(fmaxf(0.0f, 1.0f - u1));
  float sp, cp;
  sincosf(6.2831855f * u2, &sp, &cp);
  const float sign = nz >= 0.0f ? 1.0f : -1.0f;
  const float a = -1.0f / (sign + nz);
  const float bb = nx * ny * a;
  const float tx = 1.0f + sign * nx * nx * a, ty = sign * bb, tz = -sign * nx;
  const float bx = bb, by = sign + ny * ny * a, bz = -ny;
  const float lx = rr * cp, ly = rr * sp;
  o.dx = lx * tx + ly * bx + z * nx;
  o.dy = lx * ty + ly * by + z * ny;
  o.dz = lx * tz + ly * bz + z * nz;
  o.tmax = __builtin_inff();
  out[i] = o;
}

hipError_t launch_bounce(const DeviceScene& s, const ccs_ray* rays, const ccs_hit* hits, const float* uniforms,
                         uint32_t n, ccs_ray* out, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bounce, dim3((n + kBounceBlock - 1) / kBounceBlock), dim3(kBounceBlock), 0, stream, s, rays,
                     hits, uniforms, n, out);
  return hipGetLastError();
}

}  // namespace ccs
