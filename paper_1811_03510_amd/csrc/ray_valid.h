// Which rays the intersection kernel traces, shared with the ray compaction so
// that both decide alike: finite origin and direction, tmin and tmax not NaN, a
// nonzero direction and tmin <= tmax.  Both files are compiled assuming no NaN
// arithmetic, and the optimizer turns mask-and-compare tests on a float's bits
// into floating-point classifications, which that assumption then lets it
// simplify (a NaN would pass as finite).  So the bits pass through an empty asm
// statement first, which the optimizer cannot see through: the tests stay
// integer tests on the stored bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccs {

__device__ __forceinline__ uint32_t opaque_bits(float x) {
  uint32_t u = __float_as_uint(x);
  asm volatile("" : "+v"(u));
  return u;
}
__device__ __forceinline__ bool finite_bits(float x) { return (opaque_bits(x) & 0x7F800000u) != 0x7F800000u; }
__device__ __forceinline__ bool nan_bits(float x) { return (opaque_bits(x) & 0x7FFFFFFFu) > 0x7F800000u; }

// ro = (origin, tmin), rd = (direction, tmax).  The comparisons run after the NaN
// tests, with the kernel's fp32 denormals flushed to zero.
__device__ __forceinline__ bool ray_traced(const float4& ro, const float4& rd) {
  const bool finite = finite_bits(ro.x) && finite_bits(ro.y) && finite_bits(ro.z) && finite_bits(rd.x) &&
                      finite_bits(rd.y) && finite_bits(rd.z) && !nan_bits(ro.w) && !nan_bits(rd.w);
  return finite && !(rd.x == 0.0f && rd.y == 0.0f && rd.z == 0.0f) && ro.w <= rd.w;
}

}  // namespace ccs
