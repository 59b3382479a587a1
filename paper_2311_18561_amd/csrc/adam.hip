// Fused Adam over every parameter row of the Gaussians (the optimizer of
// Sec. 4: Adam with per-parameter learning rates).  The renderer takes
// activated values (s, o, beta, l > 0, o < 1); the optimizer steps in the
// unconstrained space those come from: log s, logit o, log beta, log l, and
// the identity for mu, q, SH, v and tau.  One thread per Gaussian walks all
// 17 + 3K rows (coalesced across the wave per row): chain the gradient into
// that space, update the two moments, take the bias-corrected step, map the
// value back.  Memory-bound: per row and Gaussian 4 B of parameter and of
// gradient read, 8 B of moments read and written, 4 B of parameter written.
#include "pvg_internal.hpp"

namespace pvg {

namespace {

enum Kind : int { kIdent = 0, kLog = 1, kLogit = 2 };

// The step u is taken on the unconstrained value without forming it:
// exp(log x - u) = x exp(-u) and sigmoid(logit x - u) = x / (x + (1 - x) exp(u)),
// so a zero step leaves x bit for bit and no log / exp round trip adds error.
__device__ __forceinline__ void adam_row(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                         float* __restrict__ v, int kind, float lr, const AdamCfg& c) {
  const float x = *p;
  const float graw = kind == kLog ? *g * x : kind == kLogit ? *g * (x * (1.0f - x)) : *g;
  const float mn = c.beta1 * *m + (1.0f - c.beta1) * graw;
  const float vn = c.beta2 * *v + (1.0f - c.beta2) * (graw * graw);
  *m = mn;
  *v = vn;
  const float u = lr * (mn / c.bc1) / (sqrtf(vn / c.bc2) + c.eps);
  if (u == 0.0f) return;
  *p = kind == kLog ? x * expf(-u) : kind == kLogit ? x / (x + (1.0f - x) * expf(u)) : x - u;
}

__global__ void __launch_bounds__(256) k_adam(SceneOut s, pvg_gaussians_grad g, float* __restrict__ m,
                                              float* __restrict__ v, AdamCfg c) {
  const int64_t n = s.n;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const int K3 = 3 * (s.degree + 1) * (s.degree + 1);
  int64_t row = 0;  // moments: [17 + 3K][n] in the order mu, scale, rot, sh, opacity, vel, period, tau, beta
  auto step = [&](float* prow, const float* grow, int rows, int kind, float lr) {
    for (int r = 0; r < rows; ++r, ++row)
      adam_row(prow + r * n + i, grow + r * n + i, m + row * n + i, v + row * n + i, kind, lr, c);
  };
  step(s.mu, g.mu, 3, kIdent, c.lr[0]);
  step(s.scale, g.scale, 3, kLog, c.lr[1]);
  step(s.rot, g.rot, 4, kIdent, c.lr[2]);
  step(s.sh, g.sh, 3, kIdent, c.lr[3]);                  // degree-0 coefficients
  step(s.sh + 3 * n, g.sh + 3 * n, K3 - 3, kIdent, c.lr[4]);  // the higher degrees
  step(s.opacity, g.opacity, 1, kLogit, c.lr[5]);
  step(s.vel, g.vel, 3, kIdent, c.lr[6]);
  step(s.period, g.period, 1, kLog, c.lr[7]);
  step(s.tau, g.tau, 1, kIdent, c.lr[8]);
  step(s.beta, g.beta, 1, kLog, c.lr[9]);
}

// o = min(o, cap) and the opacity row's moments cleared (the opacity reset of
// Sec. 4, after which the optimizer starts that row afresh).
__global__ void __launch_bounds__(256) k_opacity_reset(float* __restrict__ o, float* __restrict__ m,
                                                       float* __restrict__ v, int64_t n, float cap) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  o[i] = fminf(o[i], cap);
  m[i] = 0.0f;
  v[i] = 0.0f;
}

// Plain Adam on a dense array (the learnable sky cube map of Sec. 3.4, whose
// texels are taken as they are): four texels per thread, the same update as
// adam_row's identity case.
__global__ void __launch_bounds__(256) k_adam_dense(float* __restrict__ p, const float* __restrict__ g,
                                                    float* __restrict__ m, float* __restrict__ v, int64_t count,
                                                    float lr, AdamCfg c) {
  const int64_t i0 = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) * 4;
  if (i0 >= count) return;
  if (i0 + 4 <= count && (reinterpret_cast<uintptr_t>(p + i0) & 15) == 0 &&
      (reinterpret_cast<uintptr_t>(g + i0) & 15) == 0 && (reinterpret_cast<uintptr_t>(m + i0) & 15) == 0 &&
      (reinterpret_cast<uintptr_t>(v + i0) & 15) == 0) {
    float4 pp = *reinterpret_cast<const float4*>(p + i0);
    const float4 gg = *reinterpret_cast<const float4*>(g + i0);
    float4 mm = *reinterpret_cast<const float4*>(m + i0);
    float4 vv = *reinterpret_cast<const float4*>(v + i0);
    float* pe = &pp.x;
    const float* ge = &gg.x;
    float* me = &mm.x;
    float* ve = &vv.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) adam_row(pe + k, ge + k, me + k, ve + k, kIdent, lr, c);
    *reinterpret_cast<float4*>(p + i0) = pp;
    *reinterpret_cast<float4*>(m + i0) = mm;
    *reinterpret_cast<float4*>(v + i0) = vv;
    return;
  }
  for (int64_t i = i0; i < min(i0 + 4, count); ++i) adam_row(p + i, g + i, m + i, v + i, kIdent, lr, c);
}

}  // namespace

hipError_t launch_adam_dense(float* p, const float* g, float* m, float* v, int64_t count, float lr, const AdamCfg& c,
                             hipStream_t st) {
  if (count == 0) return hipSuccess;
  const int64_t blocks = (count + 1023) / 1024;
  hipLaunchKernelGGL(k_adam_dense, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, p, g, m, v, count, lr, c);
  return hipGetLastError();
}

hipError_t launch_adam(const SceneOut& s, const pvg_gaussians_grad& g, float* m, float* v, const AdamCfg& c,
                       hipStream_t st) {
  if (s.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>((s.n + 255) / 256)), dim3(256), 0, st, s, g, m, v, c);
  return hipGetLastError();
}

hipError_t launch_opacity_reset(float* o, float* m_row, float* v_row, int64_t n, float cap, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_opacity_reset, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, o, m_row,
                     v_row, n, cap);
  return hipGetLastError();
}

}  // namespace pvg
