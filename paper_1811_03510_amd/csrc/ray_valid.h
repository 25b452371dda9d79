// Which rays the intersection kernel traces, shared with the ray compaction so
// that both decide alike: finite origin and direction, tmin and tmax not NaN, a
// nonzero direction and tmin <= tmax.  Both files are compiled assuming no NaN
// arithmetic, and the optimizer turns mask-and-compare tests on a float's bits
// into floating-point classifications, which that assumption then lets it
// simplify (a NaN would pass as finite).  So the tested integers pass through an
// empty asm statement, which the optimizer cannot see through: the tests stay
// integer tests on the stored bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccs {

__device__ __forceinline__ uint32_t bits(float x) { return __float_as_uint(x); }

// ro = (origin, tmin), rd = (direction, tmax).  A component is infinite or NaN iff its
// exponent field is all ones, so the origin and direction are finite iff the largest
// of their six exponent fields is not; tmin and tmax are not NaN iff neither
// magnitude exceeds infinity's.  The two integers go through the asm statement; the
// comparisons that follow run after those tests, with fp32 denormals flushed to zero
// as in the intersection kernel.
__device__ __forceinline__ bool ray_traced(const float4& ro, const float4& rd) {
  constexpr uint32_t kExp = 0x7F800000u, kMag = 0x7FFFFFFFu;
  uint32_t e = max(max(max(bits(ro.x) & kExp, bits(ro.y) & kExp), max(bits(ro.z) & kExp, bits(rd.x) & kExp)),
                   max(bits(rd.y) & kExp, bits(rd.z) & kExp));
  uint32_t t = max(bits(ro.w) & kMag, bits(rd.w) & kMag);
  asm volatile("" : "+v"(e), "+v"(t));
  return e != kExp && t <= kExp && !(rd.x == 0.0f && rd.y == 0.0f && rd.z == 0.0f) && ro.w <= rd.w;
}

}  // namespace ccs
