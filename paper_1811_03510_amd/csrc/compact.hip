// Stream compaction of ray arrays: the rays the intersection kernel traces
// (its validity test, below) are copied in input order to a dense array with
// their input indices, so that a path tracer's later bounce levels, where most
// pixels' paths have ended (Sec. 4: a bounce of a missed ray is inactive), are
// traced without cycling through their inactive rays.
//
// Three launches over blocks of 256 rays: per-block counts, one exclusive scan
// of the counts (a single workgroup walking them with a running carry), and the
// scatter, where each ray's place is its block's offset plus its rank among the
// active rays before it in the block (wave ballots).  The order is the input
// order, so the result is deterministic.  The test of a traced ray is the
// intersection kernel's own (ray_valid.h), and this file is compiled with that
// kernel's floating-point flags (denormals flushed), so both decide alike.

#include "ccs_internal.h"
#include "ray_valid.h"

namespace ccs {

constexpr int kCompactBlock = 256;
constexpr int kCompactWaves = kCompactBlock / 64;
constexpr int kScanThreads = 1024;

__device__ __forceinline__ bool traced_at(const ccs_ray* rays, uint32_t i, uint32_t n, float4& ro, float4& rd) {
  if (i >= n) return false;
  const float4* r4 = reinterpret_cast<const float4*>(rays + i);
  ro = r4[0];
  rd = r4[1];
  return ray_traced(ro, rd);
}

// Active rays of each block: work[1 + block].
__global__ __launch_bounds__(kCompactBlock) void k_compact_count(const ccs_ray* __restrict__ rays, uint32_t n,
                                                                 uint32_t* __restrict__ work) {
  __shared__ uint32_t s_wave[kCompactWaves];
  const uint32_t i = blockIdx.x * kCompactBlock + threadIdx.x;
  float4 ro, rd;
  const uint64_t m = __ballot(traced_at(rays, i, n, ro, rd));
  if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x >> 6] = (uint32_t)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t c = 0;
    for (int w = 0; w < kCompactWaves; ++w) c += s_wave[w];
    work[1 + blockIdx.x] = c;
  }
}

// Exclusive scan of the nb block counts in place; work[0] = their sum.
__global__ __launch_bounds__(kScanThreads) void k_compact_scan(uint32_t nb, uint32_t* __restrict__ work) {
  __shared__ uint32_t s_wave[kScanThreads / 64];
  __shared__ uint32_t s_carry;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < nb; base += kScanThreads) {
    const uint32_t k = base + threadIdx.x;
    const uint32_t v = k < nb ? work[1 + k] : 0u;
    // inclusive scan within the wave
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)x, d);
      if (lane >= d) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    uint32_t before = s_carry;
    for (int w = 0; w < wave; ++w) before += s_wave[w];
    if (k < nb) work[1 + k] = before + x - v;
    __syncthreads();
    if (threadIdx.x == kScanThreads - 1) s_carry = before + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) work[0] = s_carry;
}

// Active ray i goes to out[offset of its block + its rank in the block].
__global__ __launch_bounds__(kCompactBlock) void k_compact_scatter(const ccs_ray* __restrict__ rays, uint32_t n,
                                                                   const uint32_t* __restrict__ work,
                                                                   ccs_ray* __restrict__ out,
                                                                   uint32_t* __restrict__ index) {
  __shared__ uint32_t s_wave[kCompactWaves];
  const uint32_t i = blockIdx.x * kCompactBlock + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float4 ro, rd;
  const bool act = traced_at(rays, i, n, ro, rd);
  const uint64_t m = __ballot(act);
  if (lane == 0) s_wave[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  if (act) {
    uint32_t pos = work[1 + blockIdx.x] + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    for (int w = 0; w < wave; ++w) pos += s_wave[w];
    float4* o4 = reinterpret_cast<float4*>(out + pos);
    o4[0] = ro;
    o4[1] = rd;
    index[pos] = i;
  }
}

__global__ void k_compact_empty(uint32_t* work) { work[0] = 0u; }

hipError_t launch_compact_rays(const ccs_ray* rays, uint32_t n, ccs_ray* out, uint32_t* index, uint32_t* work,
                               hipStream_t stream) {
  if (n == 0) {
    hipLaunchKernelGGL(k_compact_empty, dim3(1), dim3(1), 0, stream, work);
    return hipGetLastError();
  }
  const uint32_t nb = compact_blocks(n);
  hipLaunchKernelGGL(k_compact_count, dim3(nb), dim3(kCompactBlock), 0, stream, rays, n, work);
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(kScanThreads), 0, stream, nb, work);
  hipLaunchKernelGGL(k_compact_scatter, dim3(nb), dim3(kCompactBlock), 0, stream, rays, n, work, out, index);
  return hipGetLastError();
}

}  // namespace ccs
