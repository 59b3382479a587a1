// L1 term of the training loss (Sec. 3.4 objective): scale * sum_i |a_i - b_i|
// and its gradient scale * sign(a_i - b_i) with respect to a, in one pass
// over a and b.  kL1Blocks workgroups stride over the data (so the partial
// sums depend only on n), each writes one partial sum, and one workgroup
// adds the partials in FP64 in a fixed order: the loss is the same on every
// run.  HBM-bound: 8 bytes read and 4 written per element.
#include "pvg_internal.hpp"

namespace pvg {

namespace {

constexpr int kL1Threads = 256;

__device__ __forceinline__ float l1_grad(float d, float scale) {
  // torch's |.| adjoint: sign(d), 0 at d = 0, NaN for NaN
  return d > 0.0f ? scale : (d < 0.0f ? -scale : (d == 0.0f ? 0.0f : d));
}

__device__ __forceinline__ float block_sum(float v, float* lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  float s = 0.0f;
  if (threadIdx.x == 0)
    for (int w = 0; w < kL1Threads / 64; ++w) s += lds[w];
  return s;
}

template <bool kVec>
__global__ void __launch_bounds__(kL1Threads) k_l1(const float* __restrict__ a, const float* __restrict__ b, int64_t n,
                                                   float scale, float* __restrict__ grad, float* partials) {
  __shared__ float lds[kL1Threads / 64];
  float acc = 0.0f;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kL1Threads;
  const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kL1Threads + threadIdx.x;
  if (kVec) {
    const int64_t n4 = n / 4;
    for (int64_t i = t0; i < n4; i += stride) {
      const float4 x = reinterpret_cast<const float4*>(a)[i], y = reinterpret_cast<const float4*>(b)[i];
      const float d0 = x.x - y.x, d1 = x.y - y.y, d2 = x.z - y.z, d3 = x.w - y.w;
      acc += (fabsf(d0) + fabsf(d1)) + (fabsf(d2) + fabsf(d3));
      if (grad)
        reinterpret_cast<float4*>(grad)[i] =
            make_float4(l1_grad(d0, scale), l1_grad(d1, scale), l1_grad(d2, scale), l1_grad(d3, scale));
    }
  } else {
    for (int64_t i = t0; i < n; i += stride) {
      const float d = a[i] - b[i];
      acc += fabsf(d);
      if (grad) grad[i] = l1_grad(d, scale);
    }
  }
  const float s = block_sum(acc, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kL1Threads) k_l1_total(const float* __restrict__ partials, int count, float scale,
                                                         float* loss) {
  __shared__ double lds[kL1Threads];
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += kL1Threads) s += static_cast<double>(partials[i]);
  lds[threadIdx.x] = s;
  __syncthreads();
  for (int h = kL1Threads / 2; h > 0; h >>= 1) {
    if (static_cast<int>(threadIdx.x) < h) lds[threadIdx.x] += lds[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = static_cast<float>(lds[0] * static_cast<double>(scale));
}

}  // namespace

hipError_t launch_l1(const float* a, const float* b, int64_t n, float scale, float* loss, float* grad,
                     float* partials, hipStream_t s) {
  const bool vec = n % 4 == 0 && (reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
                                  reinterpret_cast<uintptr_t>(grad)) % 16 == 0;
  hipLaunchKernelGGL(vec ? k_l1<true> : k_l1<false>, dim3(kL1Blocks), dim3(kL1Threads), 0, s, a, b, n, scale, grad,
                     partials);
  hipLaunchKernelGGL(k_l1_total, dim3(1), dim3(kL1Threads), 0, s, partials, kL1Blocks, scale, loss);
  return hipGetLastError();
}

}  // namespace pvg
