// SSIM term of the training loss (Sec. 3.4 objective, weight lambda_r): the
// structural similarity of Wang et al. with an 11 x 11 Gaussian window
// (sigma 1.5), zero padding and C1 = 0.01^2, C2 = 0.03^2, per channel and
// pixel:
//   S = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sxx + syy + C2))
// with mx = G*x, sxx = G*(x^2) - mx^2, sxy = G*(x y) - mx my (G* the window).
// y (the target) takes no gradient.
//
// One 256-thread workgroup per 32 x 32 pixel tile and channel.  The forward
// stages the tile's 42 x 42 halo of x and y in LDS, filters the five maps
// separably (rows into LDS, then columns), and writes S and the three
// partial derivatives dS/dmx, dS/d(G*x^2), dS/d(G*xy) that the adjoint
// needs.  The adjoint stages the upstream gradient times those partials on
// the halo, filters them the same way (the window is symmetric, so the
// zero-padded filter is its own adjoint) and forms
//   dL/dx = G*(g dS/dmx) + 2 x G*(g dS/dExx) + y G*(g dS/dExy).
#include <cmath>

#include "pvg_internal.hpp"

namespace pvg {

namespace {

constexpr int kR = 5;              // window radius
// 32 x 32 tiles (four outputs per thread): each kernel's haloed inputs are
// the bulk of its reads, and a 42 x 42 halo is 1.7 times its tile where a
// 26 x 26 one (16 x 16 tiles) is 2.6 times.
constexpr int kT = 32;
constexpr int kTH = kT + 2 * kR;  // 42
constexpr float kC1 = 0.0001f, kC2 = 0.0009f;

struct Window {
  float w[2 * kR + 1];
};

// Workgroup b takes tile (b mod 8) * per + b / 8: workgroups are dealt to the
// eight XCDs in turn, so each XCD gets a contiguous band of tiles and the
// halos that neighbouring tiles share stay in its L2.  Tiles past the end
// (the grid is 8 per) exit at once.
__device__ __forceinline__ int64_t band_tile(int64_t b, int64_t total) {
  const int64_t per = (total + 7) / 8;
  return (b % 8) * per + b / 8;
}

// The SSIM kernels may fuse multiply-adds and use the hardware reciprocal:
// no decision depends on their rounding (the bar is a tolerance), and with
// contraction off they were bound by the separate multiplies and adds of the
// window sums and the IEEE division sequences.
__global__ void __launch_bounds__(256) k_ssim_fwd(const float* __restrict__ x, const float* __restrict__ y, int H,
                                                  int W, int GX, int64_t ntiles, Window win,
                                                  float* __restrict__ smap, float* __restrict__ part) {
#pragma clang fp contract(fast)
  __shared__ float s_src[5][kTH][kTH];
  __shared__ float s_h[5][kTH][kT];
  const int ch = blockIdx.y;
  const int64_t HW = static_cast<int64_t>(H) * W;
  const float* xc = x + ch * HW;
  const float* yc = y + ch * HW;
  const int64_t tile = band_tile(blockIdx.x, ntiles);
  if (tile >= ntiles) return;  // the whole workgroup, before any barrier
  const int x0 = static_cast<int>(tile % GX) * kT - kR, y0 = static_cast<int>(tile / GX) * kT - kR;
  for (int e = threadIdx.x; e < kTH * kTH; e += 256) {
    const int r = e / kTH, c = e % kTH;
    const int py = y0 + r, px = x0 + c;
    float a = 0.0f, b = 0.0f;
    if (py >= 0 && py < H && px >= 0 && px < W) {
      a = xc[static_cast<int64_t>(py) * W + px];
      b = yc[static_cast<int64_t>(py) * W + px];
    }
    s_src[0][r][c] = a;
    s_src[1][r][c] = b;
    s_src[2][r][c] = a * a;
    s_src[3][r][c] = b * b;
    s_src[4][r][c] = a * b;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kTH * kT; e += 256) {
    const int r = e / kT, c = e % kT;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k <= 2 * kR; ++k) acc += win.w[k] * s_src[m][r][c + k];
      s_h[m][r][c] = acc;
    }
  }
  __syncthreads();
  const int64_t CHW = static_cast<int64_t>(gridDim.y) * HW;
  const int tc = threadIdx.x % kT, tr0 = threadIdx.x / kT;  // rows tr0 + (256 / kT) j
#pragma unroll
  for (int j = 0; j < kT * kT / 256; ++j) {
    const int tr = tr0 + (256 / kT) * j;
    float f[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k <= 2 * kR; ++k) acc += win.w[k] * s_h[m][tr + k][tc];
      f[m] = acc;
    }
    const int py = y0 + kR + tr, px = x0 + kR + tc;
    if (py >= H || px >= W) continue;
    const float mx = f[0], my = f[1];
    const float sxx = f[2] - mx * mx, syy = f[3] - my * my, sxy = f[4] - mx * my;
    const float A = 2.0f * mx * my + kC1, B = 2.0f * sxy + kC2;
    const float Cc = mx * mx + my * my + kC1, D = sxx + syy + kC2;
    // C >= C1 and D near sxx + syy + C2 > 0: neither is ever 0
    const float iC = __builtin_amdgcn_rcpf(Cc), iD = __builtin_amdgcn_rcpf(D);
    const float Q = iC * iD;
    const float S = (A * B) * Q;
    const int64_t o = ch * HW + static_cast<int64_t>(py) * W + px;
    if (smap) smap[o] = S;
    // dS/dmx (through A, B, C, D), dS/d(G*x^2) (through D), dS/d(G*xy) (through
    // B); no division by A or B, which may pass through 0
    part[o] = 2.0f * my * (B - A) * Q + 2.0f * mx * S * (iD - iC);
    part[CHW + o] = -S * iD;
    part[2 * CHW + o] = 2.0f * A * Q;
  }
}

__global__ void __launch_bounds__(256) k_ssim_bwd(const float* __restrict__ g, const float* __restrict__ x,
                                                  const float* __restrict__ y, const float* __restrict__ part, int H,
                                                  int W, int GX, int64_t ntiles, Window win, float* __restrict__ dx) {
#pragma clang fp contract(fast)
  __shared__ float s_src[3][kTH][kTH];
  __shared__ float s_h[3][kTH][kT];
  const int ch = blockIdx.y;
  const int64_t HW = static_cast<int64_t>(H) * W;
  const int64_t CHW = static_cast<int64_t>(gridDim.y) * HW;
  const int64_t tile = band_tile(blockIdx.x, ntiles);
  if (tile >= ntiles) return;  // the whole workgroup, before any barrier
  const int x0 = static_cast<int>(tile % GX) * kT - kR, y0 = static_cast<int>(tile / GX) * kT - kR;
  for (int e = threadIdx.x; e < kTH * kTH; e += 256) {
    const int r = e / kTH, c = e % kTH;
    const int py = y0 + r, px = x0 + c;
    float q0 = 0.0f, q1 = 0.0f, q2 = 0.0f;
    if (py >= 0 && py < H && px >= 0 && px < W) {
      const int64_t o = ch * HW + static_cast<int64_t>(py) * W + px;
      const float gg = g[o];
      q0 = gg * part[o];
      q1 = gg * part[CHW + o];
      q2 = gg * part[2 * CHW + o];
    }
    s_src[0][r][c] = q0;
    s_src[1][r][c] = q1;
    s_src[2][r][c] = q2;
  }
  __syncthreads();
  // rows: kTH x kT outputs per map
  for (int e = threadIdx.x; e < kTH * kT; e += 256) {
    const int r = e / kT, c = e % kT;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k <= 2 * kR; ++k) acc += win.w[k] * s_src[m][r][c + k];
      s_h[m][r][c] = acc;
    }
  }
  __syncthreads();
  const int tc = threadIdx.x % kT, tr0 = threadIdx.x / kT;  // rows tr0 + 8 j
#pragma unroll
  for (int j = 0; j < kT / 8; ++j) {
    const int tr = tr0 + 8 * j;
    float f[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k <= 2 * kR; ++k) acc += win.w[k] * s_h[m][tr + k][tc];
      f[m] = acc;
    }
    const int py = y0 + kR + tr, px = x0 + kR + tc;
    if (py < H && px < W) {
      const int64_t o = ch * HW + static_cast<int64_t>(py) * W + px;
      dx[o] = f[0] + 2.0f * x[o] * f[1] + y[o] * f[2];
    }
  }
}

Window gaussian_window() {
  Window win;
  double w[2 * kR + 1], sum = 0.0;
  for (int k = 0; k <= 2 * kR; ++k) {
    const double d = k - kR;
    w[k] = std::exp(-(d * d) / (2.0 * 1.5 * 1.5));
    sum += w[k];
  }
  for (int k = 0; k <= 2 * kR; ++k) win.w[k] = static_cast<float>(w[k] / sum);
  return win;
}

}  // namespace

hipError_t launch_ssim_fwd(const float* x, const float* y, int C, int H, int W, float* smap, float* part,
                           hipStream_t st) {
  if (static_cast<int64_t>(H) * W * C == 0) return hipSuccess;
  const int GX = (W + kT - 1) / kT, GY = (H + kT - 1) / kT;
  const int64_t ntiles = static_cast<int64_t>(GX) * GY;
  hipLaunchKernelGGL(k_ssim_fwd, dim3(static_cast<unsigned>(8 * ((ntiles + 7) / 8)), C), dim3(256), 0, st, x, y, H,
                     W, GX, ntiles, gaussian_window(), smap, part);
  return hipGetLastError();
}

hipError_t launch_ssim_bwd(const float* g, const float* x, const float* y, const float* part, int C, int H, int W,
                           float* dx, hipStream_t st) {
  if (static_cast<int64_t>(H) * W * C == 0) return hipSuccess;
  const int GX = (W + kT - 1) / kT, GY = (H + kT - 1) / kT;
  const int64_t ntiles = static_cast<int64_t>(GX) * GY;
  hipLaunchKernelGGL(k_ssim_bwd, dim3(static_cast<unsigned>(8 * ((ntiles + 7) / 8)), C), dim3(256), 0, st, g, x, y,
                     part, H, W, GX, ntiles, gaussian_window(), dx);
  return hipGetLastError();
}

}  // namespace pvg
