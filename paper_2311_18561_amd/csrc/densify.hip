// Position-aware adaptive control (Sec. 3.3, Eq. (9); split rules of the
// implementation details in the appendix).  Per Gaussian, from the view-space
// gradient statistics accumulated by the adjoint:
//   gamma(mu) = 1 if |mu| < 2 r, else |mu| / r - 1;
//   densify if accumulated norm / count >= threshold; then clone when
//   max(s) <= g gamma(mu), else split;  prune when max(s) > b gamma(mu) (or
//   o < min_opacity).
// A clone copies every parameter.  A split replaces the Gaussian by two
// children k = 0, 1 with scales decay * s, tau + dtau_k, beta * beta_decay and
// mean mu + R(q) (s * eps_k) + dtau_k v~, where dtau_k = beta eps_k3 and
// v~ = v exp(-beta / (2 l)); eps comes from the caller ([8][n] normal draws).
// Every output (the kept original, its clone, the two children) is pruned by
// its own parameters.  Outputs are ordered by parent index, and within a
// parent: original, clone, child 0, child 1.
//
// Three kernels, HBM-bound: the plan writes one code byte per Gaussian (bit 0
// original kept, 1 clone kept, 2 and 3 children kept) and per-block output
// counts; one block scans the block counts; the apply kernel re-derives each
// Gaussian's offset from the block offset and an in-block scan of the codes
// and writes its outputs.  All decisions are FP32 without contraction, with
// correctly rounded division and square root and the exponential taken in
// FP64 and rounded once, so they are reproducible off the GPU.
#include "pvg_internal.hpp"

namespace pvg {

namespace {

constexpr int kDB = 256;  // Gaussians per block of the plan and apply kernels

struct Child {
  float mu[3], scale[3], tau, beta;
};

__device__ __forceinline__ float gamma_of(float x, float y, float z, float r) {
  const float nrm = sqrtf((x * x + y * y) + z * z);
  return nrm < 2.0f * r ? 1.0f : nrm / r - 1.0f;
}

__device__ __forceinline__ bool pruned(float x, float y, float z, float smax, float o, const DensifyCfg& c) {
  return smax > c.prune_scale * gamma_of(x, y, z, c.radius) || o < c.min_opacity;
}

__device__ __forceinline__ float max3(float a, float b, float c) { return fmaxf(fmaxf(a, b), c); }

// The split child k of Gaussian i.
__device__ void make_child(const Scene& s, const float* __restrict__ noise, int64_t i, int k, const DensifyCfg& c,
                           Child& ch) {
  const int64_t n = s.n;
  const float qw = s.rot[i], qx = s.rot[n + i], qy = s.rot[2 * n + i], qz = s.rot[3 * n + i];
  const float qn = sqrtf(((qw * qw + qx * qx) + qy * qy) + qz * qz);
  const float w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
  const float R[9] = {1.0f - 2.0f * (y * y + z * z), 2.0f * (x * y - w * z), 2.0f * (x * z + w * y),
                      2.0f * (x * y + w * z), 1.0f - 2.0f * (x * x + z * z), 2.0f * (y * z - w * x),
                      2.0f * (x * z - w * y), 2.0f * (y * z + w * x), 1.0f - 2.0f * (x * x + y * y)};
  float a[3];
  for (int d = 0; d < 3; ++d) a[d] = s.scale[d * n + i] * noise[(4 * k + d) * n + i];
  const float beta = s.beta[i], l = s.period[i];
  const float e = static_cast<float>(exp(static_cast<double>(-(beta / (2.0f * l)))));
  const float dtau = beta * noise[(4 * k + 3) * n + i];
  for (int d = 0; d < 3; ++d) {
    const float off = (R[3 * d] * a[0] + R[3 * d + 1] * a[1]) + R[3 * d + 2] * a[2];
    const float vb = s.vel[d * n + i] * e;
    ch.mu[d] = (s.mu[d * n + i] + off) + dtau * vb;
    ch.scale[d] = c.scale_decay * s.scale[d * n + i];
  }
  ch.tau = s.tau[i] + dtau;
  ch.beta = c.beta_decay * beta;
}

__device__ uint32_t decide(const Scene& s, const float* __restrict__ gacc, const float* __restrict__ gcnt,
                           const float* __restrict__ noise, int64_t i, const DensifyCfg& c) {
  const int64_t n = s.n;
  const float mx = s.mu[i], my = s.mu[n + i], mz = s.mu[2 * n + i];
  const float smax = max3(s.scale[i], s.scale[n + i], s.scale[2 * n + i]);
  const float o = s.opacity[i];
  const float cnt = gcnt[i];
  const float avg = cnt > 0.0f ? gacc[i] / cnt : 0.0f;
  const bool dens = avg >= c.grad_threshold;
  const float gam = gamma_of(mx, my, mz, c.radius);
  const bool clone = dens && smax <= c.clone_scale * gam;
  const bool split = dens && !clone;
  const bool keep = !pruned(mx, my, mz, smax, o, c);
  uint32_t code = 0;
  if (!split && keep) code |= 1u;
  if (clone && keep) code |= 2u;
  if (split) {
    for (int k = 0; k < 2; ++k) {
      Child ch;
      make_child(s, noise, i, k, c, ch);
      if (!pruned(ch.mu[0], ch.mu[1], ch.mu[2], max3(ch.scale[0], ch.scale[1], ch.scale[2]), o, c))
        code |= 4u << k;
    }
  }
  return code;
}

// Exclusive prefix over the block of v (0..4 per thread); returns the block total in *total.
__device__ uint32_t block_exclusive(uint32_t v, uint32_t* s_wave, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  uint32_t base = 0, sum = 0;
  for (int w = 0; w < kDB / 64; ++w) {
    if (w < wave) base += s_wave[w];
    sum += s_wave[w];
  }
  *total = sum;
  return base + x - v;
}

__global__ void __launch_bounds__(kDB) k_densify_plan(Scene s, const float* __restrict__ gacc,
                                                      const float* __restrict__ gcnt, const float* __restrict__ noise,
                                                      DensifyCfg c, uint8_t* codes, uint32_t* block_count) {
  __shared__ uint32_t s_wave[kDB / 64];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kDB + threadIdx.x;
  uint32_t code = 0;
  if (i < s.n) {
    code = decide(s, gacc, gcnt, noise, i, c);
    codes[i] = static_cast<uint8_t>(code);
  }
  uint32_t total;
  block_exclusive(static_cast<uint32_t>(__popc(code)), s_wave, &total);
  if (threadIdx.x == 0) block_count[blockIdx.x] = total;
}

// One block: exclusive offsets of nb block counts in place, total into *out_total.
__global__ void __launch_bounds__(1024) k_densify_scan(uint32_t* block_count, int64_t nb,
                                                       unsigned long long* out_total) {
  __shared__ unsigned long long s_sum[1024];
  const int64_t per = (nb + 1023) / 1024;
  const int64_t b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
  unsigned long long mine = 0;
  for (int64_t b = b0; b < b1; ++b) mine += block_count[b];
  s_sum[threadIdx.x] = mine;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const unsigned long long add = threadIdx.x >= off ? s_sum[threadIdx.x - off] : 0ull;
    __syncthreads();
    s_sum[threadIdx.x] += add;
    __syncthreads();
  }
  unsigned long long run = s_sum[threadIdx.x] - mine;
  for (int64_t b = b0; b < b1; ++b) {
    const uint32_t cnt = block_count[b];
    block_count[b] = static_cast<uint32_t>(run);
    run += cnt;
  }
  if (threadIdx.x == 1023) *out_total = s_sum[1023];
}

// Rows are copied eight at a time, all loads before the stores, so a thread
// keeps eight loads in flight instead of waiting on each row in turn.
__device__ __forceinline__ void copy_rows(const float* __restrict__ src, float* __restrict__ dst, int rows,
                                          int64_t n, int64_t n_out, int64_t i, int64_t j) {
  for (int r0 = 0; r0 < rows; r0 += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = r0 + u < rows ? src[(r0 + u) * n + i] : 0.0f;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (r0 + u < rows) dst[(r0 + u) * n_out + j] = v[u];
  }
}

constexpr int kExtraRowsPerBlock = 32;  // carried rows per blockIdx.y slice of the apply grid

// blockIdx.y = 0 writes the parameters; blockIdx.y = 1, 2, ... each write
// kExtraRowsPerBlock of the carried rows.  Every block re-derives its
// Gaussians' output offsets from the codes.
__global__ void __launch_bounds__(kDB) k_densify_apply(Scene s, const float* __restrict__ noise, DensifyCfg c,
                                                       const uint8_t* __restrict__ codes,
                                                       const uint32_t* __restrict__ block_off, SceneOut out,
                                                       const float* __restrict__ extra_in,
                                                       float* __restrict__ extra_out, int32_t n_extra) {
  __shared__ uint32_t s_wave[kDB / 64];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kDB + threadIdx.x;
  const uint32_t code = i < s.n ? codes[i] : 0u;
  uint32_t total;
  const uint32_t local = block_exclusive(static_cast<uint32_t>(__popc(code)), s_wave, &total);
  if (code == 0) return;
  const int64_t n = s.n, m = out.n;
  const int64_t j0 = static_cast<int64_t>(block_off[blockIdx.x]) + local;
  if (blockIdx.y > 0) {  // a slice of the carried rows: kept for the original, zero for new points
    const int r0 = (blockIdx.y - 1) * kExtraRowsPerBlock;
    const int rows = min(kExtraRowsPerBlock, n_extra - r0);
    int64_t j = j0;
    for (int slot = 0; slot < 4; ++slot) {
      if (!(code & (1u << slot))) continue;
      if (j >= m) return;
      if (slot == 0) {
        copy_rows(extra_in + static_cast<int64_t>(r0) * n, extra_out + static_cast<int64_t>(r0) * m, rows, n, m, i,
                  j);
      } else {
        for (int r = 0; r < rows; ++r) extra_out[(r0 + r) * m + j] = 0.0f;
      }
      ++j;
    }
    return;
  }
  const int K3 = 3 * (s.degree + 1) * (s.degree + 1);
  int64_t j = j0;
  for (int slot = 0; slot < 4; ++slot) {
    if (!(code & (1u << slot))) continue;
    if (j >= m) return;  // the host checks out.n against the plan's total; never write past it
    copy_rows(s.rot, out.rot, 4, n, m, i, j);
    copy_rows(s.sh, out.sh, K3, n, m, i, j);
    copy_rows(s.vel, out.vel, 3, n, m, i, j);
    out.opacity[j] = s.opacity[i];
    out.period[j] = s.period[i];
    if (slot < 2) {  // the original or its clone: every parameter as it is
      copy_rows(s.mu, out.mu, 3, n, m, i, j);
      copy_rows(s.scale, out.scale, 3, n, m, i, j);
      out.tau[j] = s.tau[i];
      out.beta[j] = s.beta[i];
    } else {
      Child ch;
      make_child(s, noise, i, slot - 2, c, ch);
      for (int d = 0; d < 3; ++d) {
        out.mu[d * m + j] = ch.mu[d];
        out.scale[d * m + j] = ch.scale[d];
      }
      out.tau[j] = ch.tau;
      out.beta[j] = ch.beta;
    }
    ++j;
  }
}

// Static / dynamic split (Sec. 3.2: a threshold on the staticness rho =
// beta / l separates static from dynamic points).  Static when rho >=
// threshold (FP32, correctly rounded division).  The plan counts static
// Gaussians per block (scanned by k_densify_scan); the apply kernel writes a
// static Gaussian at its rank among the static ones and a dynamic one at
// i minus the number of static Gaussians before it, so both sets keep index
// order.
__device__ __forceinline__ bool is_static(const Scene& s, int64_t i, float thr) {
  return s.beta[i] / s.period[i] >= thr;
}

__global__ void __launch_bounds__(kDB) k_static_plan(Scene s, float thr, uint32_t* block_count) {
  __shared__ uint32_t s_wave[kDB / 64];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kDB + threadIdx.x;
  const uint32_t st = (i < s.n && is_static(s, i, thr)) ? 1u : 0u;
  uint32_t total;
  block_exclusive(st, s_wave, &total);
  if (threadIdx.x == 0) block_count[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kDB) k_static_apply(Scene s, float thr, const uint32_t* __restrict__ block_off,
                                                      SceneOut os, SceneOut od) {
  __shared__ uint32_t s_wave[kDB / 64];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kDB + threadIdx.x;
  const bool st = i < s.n && is_static(s, i, thr);
  uint32_t total;
  const uint32_t local = block_exclusive(st ? 1u : 0u, s_wave, &total);
  if (i >= s.n) return;
  const int64_t before = static_cast<int64_t>(block_off[blockIdx.x]) + local;  // static Gaussians before i
  const SceneOut& o = st ? os : od;
  const int64_t j = st ? before : i - before;
  if (j >= o.n) return;  // the host sizes both outputs from the plan's count
  const int64_t n = s.n, m = o.n;
  const int K3 = 3 * (s.degree + 1) * (s.degree + 1);
  copy_rows(s.mu, o.mu, 3, n, m, i, j);
  copy_rows(s.scale, o.scale, 3, n, m, i, j);
  copy_rows(s.rot, o.rot, 4, n, m, i, j);
  copy_rows(s.sh, o.sh, K3, n, m, i, j);
  copy_rows(s.vel, o.vel, 3, n, m, i, j);
  o.opacity[j] = s.opacity[i];
  o.period[j] = s.period[i];
  o.tau[j] = s.tau[i];
  o.beta[j] = s.beta[i];
}

}  // namespace

hipError_t launch_static_plan(const Scene& s, float thr, void* tmp, hipStream_t st) {
  const int64_t nb = (s.n + kDB - 1) / kDB;
  uint32_t* bc = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(tmp) + ((s.n + 255) / 256) * 256);
  unsigned long long* total = densify_total_ptr(tmp, s.n);
  if (s.n == 0) return launch_fill_u32(reinterpret_cast<uint32_t*>(total), 0u, 2, st);
  hipLaunchKernelGGL(k_static_plan, dim3(static_cast<unsigned>(nb)), dim3(kDB), 0, st, s, thr, bc);
  hipLaunchKernelGGL(k_densify_scan, dim3(1), dim3(1024), 0, st, bc, nb, total);
  return hipGetLastError();
}

hipError_t launch_static_apply(const Scene& s, float thr, const void* tmp, const SceneOut& os, const SceneOut& od,
                               hipStream_t st) {
  if (s.n == 0) return hipSuccess;
  const int64_t nb = (s.n + kDB - 1) / kDB;
  const uint32_t* bo =
      reinterpret_cast<const uint32_t*>(static_cast<const uint8_t*>(tmp) + ((s.n + 255) / 256) * 256);
  hipLaunchKernelGGL(k_static_apply, dim3(static_cast<unsigned>(nb)), dim3(kDB), 0, st, s, thr, bo, os, od);
  return hipGetLastError();
}

size_t densify_tmp_bytes(int64_t n) {
  const int64_t nb = (n + kDB - 1) / kDB;
  return static_cast<size_t>(((n + 255) / 256) * 256) + static_cast<size_t>(nb) * 4 + 256;
}

// tmp: [codes: n bytes, padded to 256][block counts / offsets: nb u32][total: u64]
hipError_t launch_densify_plan(const Scene& s, const float* gacc, const float* gcnt, const float* noise,
                               const DensifyCfg& c, void* tmp, hipStream_t st) {
  const int64_t nb = (s.n + kDB - 1) / kDB;
  uint8_t* codes = static_cast<uint8_t*>(tmp);
  uint32_t* bc = reinterpret_cast<uint32_t*>(codes + ((s.n + 255) / 256) * 256);
  unsigned long long* total = reinterpret_cast<unsigned long long*>(
      reinterpret_cast<char*>(bc) + ((nb * 4 + 7) / 8) * 8);
  if (s.n == 0) return launch_fill_u32(reinterpret_cast<uint32_t*>(total), 0u, 2, st);
  hipLaunchKernelGGL(k_densify_plan, dim3(static_cast<unsigned>(nb)), dim3(kDB), 0, st, s, gacc, gcnt, noise, c,
                     codes, bc);
  hipLaunchKernelGGL(k_densify_scan, dim3(1), dim3(1024), 0, st, bc, nb, total);
  return hipGetLastError();
}

unsigned long long* densify_total_ptr(void* tmp, int64_t n) {
  const int64_t nb = (n + kDB - 1) / kDB;
  char* bc = static_cast<char*>(tmp) + ((n + 255) / 256) * 256;
  return reinterpret_cast<unsigned long long*>(bc + ((nb * 4 + 7) / 8) * 8);
}

hipError_t launch_densify_apply(const Scene& s, const float* noise, const DensifyCfg& c, const void* tmp,
                                const SceneOut& out, const float* extra_in, float* extra_out, int32_t n_extra,
                                hipStream_t st) {
  if (s.n == 0 || out.n == 0) return hipSuccess;
  const int64_t nb = (s.n + kDB - 1) / kDB;
  const uint8_t* codes = static_cast<const uint8_t*>(tmp);
  const uint32_t* bo = reinterpret_cast<const uint32_t*>(codes + ((s.n + 255) / 256) * 256);
  const unsigned slices = 1u + static_cast<unsigned>((n_extra + kExtraRowsPerBlock - 1) / kExtraRowsPerBlock);
  hipLaunchKernelGGL(k_densify_apply, dim3(static_cast<unsigned>(nb), slices), dim3(kDB), 0, st, s, noise, c, codes,
                     bo, out, extra_in, extra_out, n_extra);
  return hipGetLastError();
}

}  // namespace pvg
