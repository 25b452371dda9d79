// Training of the child-ordering network: loss, backpropagation and Adam, on
// the GPU.  One block of 64 threads takes 64 samples of a minibatch: each
// thread runs its sample forward and backward (weights in LDS), then the block
// sums every parameter's gradient over its samples in a fixed order and writes
// one partial row; a second kernel adds the rows in block order (deterministic),
// divides by the number of labelled samples and applies the update.
//
// Network and parameter order as in policy.h.  In bfloat16 mode the inputs,
// the weights and the hidden activations are rounded to bfloat16 as in
// inference, sums stay fp32 and gradients pass straight through the roundings
// to the fp32 master weights.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "policy.h"

namespace ccs {

constexpr int kMlpBlock = 64;

__device__ __forceinline__ float bf16_value(float x) { return __uint_as_float(bf16_bits(x) << 16); }

// Minibatch sample k of the affine permutation (a * pos + c) mod n, gcd(a, n) = 1.
__device__ __forceinline__ uint32_t perm_index(uint64_t pos, uint64_t a, uint64_t c, uint32_t n) {
  return (uint32_t)((a * (pos % n) + c) % n);
}

__global__ __launch_bounds__(kMlpBlock) void k_mlp_grad(const float* __restrict__ theta, const float* __restrict__ X,
                                                        const uint8_t* __restrict__ Y, uint32_t n, uint32_t batch,
                                                        uint64_t pos0, uint64_t pa, uint64_t pc, int bf16,
                                                        float* __restrict__ partial, float* __restrict__ lossp) {
  __shared__ float w[kPolicyParams];
  __shared__ float act[kMlpBlock][80];  // x (16), h1 (32), h2 (32)
  __shared__ float del[kMlpBlock][68];  // d1 (32), d2 (32), d3 (4): gradients at the pre-activations
  __shared__ float red[kMlpBlock][2];
  const int tid = threadIdx.x;
  for (int p = tid; p < kPolicyParams; p += kMlpBlock) {
    const bool is_w = p < kPolicyB1 || (p >= kPolicyW2 && p < kPolicyB2) || (p >= kPolicyW3 && p < kPolicyB3);
    const float v = theta[p];
    w[p] = (bf16 && is_w) ? bf16_value(v) : v;
  }
  __syncthreads();
  const uint32_t k = blockIdx.x * kMlpBlock + tid;
  uint32_t label = 255u;
  uint32_t row = 0;
  if (k < batch) {
    row = perm_index(pos0 + k, pa, pc, n);
    label = Y[row];
  }
  const bool lab = label < 4u;
  float x[16], h1[32], h2[32];
  uint32_t m1 = 0, m2 = 0;  // ReLU masks
  float loss = 0.0f;
  float d3[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if (lab) {
    const float4* xr = reinterpret_cast<const float4*>(X + (size_t)row * 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 v = xr[q];
      x[4 * q] = v.x;
      x[4 * q + 1] = v.y;
      x[4 * q + 2] = v.z;
      x[4 * q + 3] = v.w;
    }
    if (bf16) {
#pragma unroll
      for (int q = 0; q < 16; ++q) x[q] = bf16_value(x[q]);
    }
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      float a = w[kPolicyB1 + u];
#pragma unroll
      for (int q = 0; q < 16; ++q) a = fmaf(w[kPolicyW1 + u * 16 + q], x[q], a);
      if (a > 0.0f) m1 |= 1u << u;
      const float h = fmaxf(a, 0.0f);
      h1[u] = bf16 ? bf16_value(h) : h;
    }
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      float a = w[kPolicyB2 + u];
#pragma unroll
      for (int q = 0; q < 32; ++q) a = fmaf(w[kPolicyW2 + u * 32 + q], h1[q], a);
      if (a > 0.0f) m2 |= 1u << u;
      const float h = fmaxf(a, 0.0f);
      h2[u] = bf16 ? bf16_value(h) : h;
    }
    float z[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      float a = w[kPolicyB3 + o];
#pragma unroll
      for (int q = 0; q < 32; ++q) a = fmaf(w[kPolicyW3 + o * 32 + q], h2[q], a);
      z[o] = a;
    }
    const float zm = fmaxf(fmaxf(z[0], z[1]), fmaxf(z[2], z[3]));
    float e[4], se = 0.0f;
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      e[o] = expf(z[o] - zm);
      se += e[o];
    }
    const float zy = label == 0 ? z[0] : label == 1 ? z[1] : label == 2 ? z[2] : z[3];
    loss = logf(se) + zm - zy;
#pragma unroll
    for (int o = 0; o < 4; ++o) d3[o] = e[o] / se - (label == (uint32_t)o ? 1.0f : 0.0f);
  } else {
#pragma unroll
    for (int q = 0; q < 16; ++q) x[q] = 0.0f;
#pragma unroll
    for (int q = 0; q < 32; ++q) h1[q] = h2[q] = 0.0f;
  }
  // backward to the pre-activations
  float d2[32], d1[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    float g = 0.0f;
#pragma unroll
    for (int o = 0; o < 4; ++o) g = fmaf(w[kPolicyW3 + o * 32 + q], d3[o], g);
    d2[q] = ((m2 >> q) & 1u) ? g : 0.0f;
  }
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    float g = 0.0f;
#pragma unroll
    for (int u = 0; u < 32; ++u) g = fmaf(w[kPolicyW2 + u * 32 + q], d2[u], g);
    d1[q] = ((m1 >> q) & 1u) ? g : 0.0f;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) act[tid][q] = x[q];
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    act[tid][16 + q] = h1[q];
    act[tid][48 + q] = h2[q];
    del[tid][q] = d1[q];
    del[tid][32 + q] = d2[q];
  }
#pragma unroll
  for (int o = 0; o < 4; ++o) del[tid][64 + o] = d3[o];
  red[tid][0] = loss;
  red[tid][1] = lab ? 1.0f : 0.0f;
  __syncthreads();
  // parameter gradients summed over the block's samples in sample order
  for (int p = tid; p < kPolicyParams; p += kMlpBlock) {
    int di, ai;  // delta column, activation column (-1: bias)
    if (p < kPolicyB1) {
      di = p / 16;
      ai = p % 16;
    } else if (p < kPolicyW2) {
      di = p - kPolicyB1;
      ai = -1;
    } else if (p < kPolicyB2) {
      di = 32 + (p - kPolicyW2) / 32;
      ai = 16 + (p - kPolicyW2) % 32;
    } else if (p < kPolicyW3) {
      di = 32 + (p - kPolicyB2);
      ai = -1;
    } else if (p < kPolicyB3) {
      di = 64 + (p - kPolicyW3) / 32;
      ai = 48 + (p - kPolicyW3) % 32;
    } else {
      di = 64 + (p - kPolicyB3);
      ai = -1;
    }
    float g = 0.0f;
    if (ai < 0) {
      for (int t = 0; t < kMlpBlock; ++t) g += del[t][di];
    } else {
      for (int t = 0; t < kMlpBlock; ++t) g = fmaf(del[t][di], act[t][ai], g);
    }
    partial[(size_t)blockIdx.x * kPolicyParams + p] = g;
  }
  if (tid == 0) {
    float ls = 0.0f, cn = 0.0f;
    for (int t = 0; t < kMlpBlock; ++t) {
      ls += red[t][0];
      cn += red[t][1];
    }
    lossp[2 * blockIdx.x] = ls;
    lossp[2 * blockIdx.x + 1] = cn;
  }
}

// Sum of the partial rows in block order, divided by the labelled count.
__device__ __forceinline__ float reduce_rows(const float* partial, const float* lossp, uint32_t nblk, int p,
                                             float& cnt, float& loss) {
  float g = 0.0f, c = 0.0f, l = 0.0f;
  for (uint32_t b = 0; b < nblk; ++b) {
    g += partial[(size_t)b * kPolicyParams + p];
    c += lossp[2 * b + 1];
    l += lossp[2 * b];
  }
  cnt = c;
  loss = l;
  return g / fmaxf(c, 1.0f);
}

__global__ __launch_bounds__(kMlpBlock) void k_mlp_reduce(const float* __restrict__ partial,
                                                          const float* __restrict__ lossp, uint32_t nblk,
                                                          float* __restrict__ grad, float* __restrict__ loss_out) {
  const int p = blockIdx.x * kMlpBlock + threadIdx.x;
  if (p >= kPolicyParams) return;
  float cnt, loss;
  grad[p] = reduce_rows(partial, lossp, nblk, p, cnt, loss);
  if (p == 0 && loss_out) *loss_out = loss / fmaxf(cnt, 1.0f);
}

// Adam with bias corrections c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ __launch_bounds__(kMlpBlock) void k_mlp_adam(float* __restrict__ theta, float* __restrict__ m,
                                                        float* __restrict__ v, const float* __restrict__ partial,
                                                        const float* __restrict__ lossp, uint32_t nblk, float lr,
                                                        float beta1, float beta2, float eps, float c1, float c2,
                                                        float* __restrict__ loss_out) {
  const int p = blockIdx.x * kMlpBlock + threadIdx.x;
  if (p >= kPolicyParams) return;
  float cnt, loss;
  const float g = reduce_rows(partial, lossp, nblk, p, cnt, loss);
  const float mm = beta1 * m[p] + (1.0f - beta1) * g;
  const float vv = beta2 * v[p] + (1.0f - beta2) * g * g;
  m[p] = mm;
  v[p] = vv;
  theta[p] -= lr * (mm * c1) / (sqrtf(vv * c2) + eps);
  if (p == 0 && loss_out) *loss_out = loss / fmaxf(cnt, 1.0f);
}

__global__ void k_fill(float* __restrict__ p, uint32_t n, float value) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

hipError_t launch_mlp_grad(const float* theta, const float* X, const uint8_t* Y, uint32_t n, uint32_t batch,
                           uint64_t pos0, uint64_t pa, uint64_t pc, int bf16, float* partial, float* lossp,
                           hipStream_t stream) {
  const uint32_t nblk = (batch + kMlpBlock - 1) / kMlpBlock;
  hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(kMlpBlock), 0, stream, theta, X, Y, n, batch, pos0, pa, pc, bf16,
                     partial, lossp);
  return hipGetLastError();
}

hipError_t launch_mlp_reduce(const float* partial, const float* lossp, uint32_t nblk, float* grad, float* loss,
                             hipStream_t stream) {
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kPolicyParams + kMlpBlock - 1) / kMlpBlock), dim3(kMlpBlock), 0, stream,
                     partial, lossp, nblk, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* theta, float* m, float* v, const float* partial, const float* lossp, uint32_t nblk,
                           float lr, float beta1, float beta2, float eps, float c1, float c2, float* loss,
                           hipStream_t stream) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((kPolicyParams + kMlpBlock - 1) / kMlpBlock), dim3(kMlpBlock), 0, stream,
                     theta, m, v, partial, lossp, nblk, lr, beta1, beta2, eps, c1, c2, loss);
  return hipGetLastError();
}

hipError_t launch_fill(float* p, uint32_t n, float value, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, stream, p, n, value);
  return hipGetLastError();
}

// Gradient scratch of the entry point that allocates nothing: partial rows of
// kGradScratchBlocks blocks, then their (loss, count) pairs.  One copy per device,
// held until the process ends; every call on a device shares it.
static __device__ __align__(256) float scratch[kGradScratchBlocks * (kPolicyParams + 2)];

hipError_t grad_scratch(float** partial, float** lossp) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static float* base[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!base[dev]) {
    // the array's address on the current device (its host-side name is not a device address)
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    base[dev] = static_cast<float*>(p);
  }
  *partial = base[dev];
  *lossp = base[dev] + (size_t)kGradScratchBlocks * kPolicyParams;
  return hipSuccess;
}

}  // namespace ccs
