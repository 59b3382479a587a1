// Per-tile alpha blending (Sec. 3.1, Eq. (3)) and its adjoint on gfx950.
//
// One 64-lane wavefront owns one 16x16 tile; lane l shades the four pixels of
// column l % 16 in rows l / 16 + {0, 4, 8, 12}.  The tile's depth-ordered list
// is walked in batches of 64 Gaussians: each lane gathers one Gaussian's
// record (2D mean, conic, opacity, colour) into LDS and every lane then reads
// the batch back as broadcasts.  A pixel stops before the Gaussian that would
// take its transmittance below 1e-4; the wave leaves the list as soon as a
// ballot shows all 256 pixels done.
//
// The adjoint walks the list backwards from the wave's last contributor,
// recovering each pixel's transmittance by division, sums the four pixels'
// screen-space gradients per lane, reduces them across the wave and issues one
// set of 9 global atomics per (Gaussian, tile).
//
// Tiles are assigned so that each of the eight XCDs (which receive workgroups
// round-robin) works on one contiguous band of tiles, keeping the Gaussians
// shared by neighbouring tiles in that XCD's L2.
#include "pvg_internal.hpp"

namespace pvg {

__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t total) {
  const int64_t per = (total + 7) / 8;
  return (b % 8) * per + b / 8;
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
  return x;
}

// alpha of a (pixel, Gaussian) pair; the exact arithmetic is shared by the
// forward and the adjoint so that both take the same branch decisions.
struct Pair {
  float dx, dy, power, G, raw, alpha;
};
__device__ __forceinline__ bool eval_pair(float gx, float gy, float A, float B, float C, float op, float px, float py,
                                          Pair& p) {
  p.dx = gx - px;
  p.dy = gy - py;
  p.power = -0.5f * (A * (p.dx * p.dx) + C * (p.dy * p.dy)) - B * (p.dx * p.dy);
  if (p.power > 0.0f) return false;
  p.G = expf(p.power);
  p.raw = op * p.G;
  p.alpha = fminf(kAlphaMax, p.raw);
  return !(p.alpha < kAlphaMin);
}

constexpr int kPix = 4;  // pixels per lane

__global__ void __launch_bounds__(64) k_render_fwd(ViewSet vs, Geom geom, const uint32_t* __restrict__ vals,
                                                   const uint32_t* __restrict__ ranges,
                                                   unsigned long long* pair_counter) {
  __shared__ float2 s_xy[64];
  __shared__ float4 s_co[64];
  __shared__ float4 s_rgb[64];
  const int64_t ntiles = live_tiles(vs);
  const int64_t tile = xcd_tile(blockIdx.x, ntiles);
  if (tile >= ntiles) return;
  const View& v = view_at(vs, view_of_tile(vs, tile));
  const int64_t local = tile - v.tile_off;
  const int tx = static_cast<int>(local % v.GX), ty = static_cast<int>(local / v.GX);
  const int lane = threadIdx.x;
  const int px = tx * kTile + (lane & 15);
  const int py0 = ty * kTile + (lane >> 4);
  const float fpx = static_cast<float>(px);
  float T[kPix], Cr[kPix], Cg[kPix], Cb[kPix];
  int last[kPix];
  bool done[kPix];
#pragma unroll
  for (int k = 0; k < kPix; ++k) {
    T[k] = 1.0f; Cr[k] = 0.0f; Cg[k] = 0.0f; Cb[k] = 0.0f; last[k] = 0;
    done[k] = !(px < v.W && py0 + 4 * k < v.H);
  }
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
  long long evaluated = 0;
  for (uint32_t b0 = start; b0 < end; b0 += 64) {
    const bool active = !(done[0] && done[1] && done[2] && done[3]);
    if (!__any(active)) break;
    const uint32_t idx = b0 + lane;
    if (idx < end) {
      const uint32_t g = vals[idx];
      s_xy[lane] = reinterpret_cast<const float2*>(geom.xy)[g];
      s_co[lane] = reinterpret_cast<const float4*>(geom.conic_op)[g];
      s_rgb[lane] = make_float4(geom.rgb[3 * g], geom.rgb[3 * g + 1], geom.rgb[3 * g + 2], 0.0f);
    }
    __syncthreads();
    const int cnt = static_cast<int>(min(64u, end - b0));
    for (int j = 0; j < cnt; ++j) {
      const bool act = !(done[0] && done[1] && done[2] && done[3]);
      if (!__any(act)) break;
      const float2 m = s_xy[j];
      const float4 co = s_co[j];
      const float4 c = s_rgb[j];
      const int pos = static_cast<int>(b0 - start) + j + 1;
#pragma unroll
      for (int k = 0; k < kPix; ++k) {
        if (done[k]) continue;
        ++evaluated;
        Pair p;
        if (!eval_pair(m.x, m.y, co.x, co.y, co.z, co.w, fpx, static_cast<float>(py0 + 4 * k), p)) continue;
        const float Tn = T[k] * (1.0f - p.alpha);
        if (Tn < kTMin) {
          done[k] = true;
          continue;
        }
        const float w = p.alpha * T[k];
        Cr[k] = Cr[k] + c.x * w;
        Cg[k] = Cg[k] + c.y * w;
        Cb[k] = Cb[k] + c.z * w;
        T[k] = Tn;
        last[k] = pos;
      }
    }
    __syncthreads();
  }
  const int64_t HW = static_cast<int64_t>(v.W) * v.H;
#pragma unroll
  for (int k = 0; k < kPix; ++k) {
    const int py = py0 + 4 * k;
    if (px < v.W && py < v.H) {
      const int64_t o = static_cast<int64_t>(py) * v.W + px;
      v.img[o] = Cr[k] + T[k] * v.bg[0];
      v.img[HW + o] = Cg[k] + T[k] * v.bg[1];
      v.img[2 * HW + o] = Cb[k] + T[k] * v.bg[2];
      v.final_T[o] = T[k];
      v.n_contrib[o] = last[k];
    }
  }
  if (pair_counter) {
    long long e = evaluated;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    if (lane == 0) atomicAdd(pair_counter, static_cast<unsigned long long>(e));
  }
}

__global__ void __launch_bounds__(64) k_render_bwd(ViewSet vs, Geom geom, const uint32_t* __restrict__ vals,
                                                   const uint32_t* __restrict__ ranges, float* g2d,
                                                   unsigned long long* pair_counter) {
  __shared__ float2 s_xy[64];
  __shared__ float4 s_co[64];
  __shared__ float4 s_rgb[64];
  __shared__ uint32_t s_g[64];
  __shared__ float s_acc[64][9];
  __shared__ int s_any[64];
  const int64_t ntiles = live_tiles(vs);
  const int64_t tile = xcd_tile(blockIdx.x, ntiles);
  if (tile >= ntiles) return;
  const View& v = view_at(vs, view_of_tile(vs, tile));
  const int64_t local = tile - v.tile_off;
  const int tx = static_cast<int>(local % v.GX), ty = static_cast<int>(local / v.GX);
  const int lane = threadIdx.x;
  const int px = tx * kTile + (lane & 15);
  const int py0 = ty * kTile + (lane >> 4);
  const float fpx = static_cast<float>(px);
  const int64_t HW = static_cast<int64_t>(v.W) * v.H;
  float T[kPix], rr[kPix], gr[kPix], gg[kPix], gb[kPix];
  int last[kPix];
  int lmax = 0;
#pragma unroll
  for (int k = 0; k < kPix; ++k) {
    const int py = py0 + 4 * k;
    if (px < v.W && py < v.H) {
      const int64_t o = static_cast<int64_t>(py) * v.W + px;
      T[k] = v.final_T[o];
      last[k] = v.n_contrib[o];
      gr[k] = v.dL_dimg[o];
      gg[k] = v.dL_dimg[HW + o];
      gb[k] = v.dL_dimg[2 * HW + o];
    } else {
      T[k] = 1.0f; last[k] = 0; gr[k] = 0.0f; gg[k] = 0.0f; gb[k] = 0.0f;
    }
    rr[k] = v.bg[0] * gr[k] + v.bg[1] * gg[k] + v.bg[2] * gb[k];
    lmax = max(lmax, last[k]);
  }
  lmax = wave_max(lmax);
  const uint32_t start = ranges[2 * tile];
  lmax = min(lmax, static_cast<int>(ranges[2 * tile + 1] - start));  // never read past the tile's list
  long long evaluated = 0;
  for (int hi = lmax; hi > 0; hi -= 64) {
    const int lo = max(0, hi - 64);
    const int cnt = hi - lo;
    if (lane < cnt) {
      const uint32_t g = vals[start + lo + lane];
      s_g[lane] = g;
      s_xy[lane] = reinterpret_cast<const float2*>(geom.xy)[g];
      s_co[lane] = reinterpret_cast<const float4*>(geom.conic_op)[g];
      s_rgb[lane] = make_float4(geom.rgb[3 * g], geom.rgb[3 * g + 1], geom.rgb[3 * g + 2], 0.0f);
    }
    __syncthreads();
    for (int j = cnt - 1; j >= 0; --j) {
      const int pos = lo + j;  // 0-based list position
      const float2 m = s_xy[j];
      const float4 co = s_co[j];
      const float4 c = s_rgb[j];
      float a[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) a[q] = 0.0f;
      bool any = false;
#pragma unroll
      for (int k = 0; k < kPix; ++k) {
        if (pos >= last[k]) continue;
        ++evaluated;
        Pair p;
        if (!eval_pair(m.x, m.y, co.x, co.y, co.z, co.w, fpx, static_cast<float>(py0 + 4 * k), p)) continue;
        any = true;
        T[k] = T[k] / (1.0f - p.alpha);
        const float cg = c.x * gr[k] + c.y * gg[k] + c.z * gb[k];
        const float dalpha = T[k] * (cg - rr[k]);
        const float w = p.alpha * T[k];
        a[6] += w * gr[k];
        a[7] += w * gg[k];
        a[8] += w * gb[k];
        rr[k] = p.alpha * cg + (1.0f - p.alpha) * rr[k];
        if (!(p.raw > kAlphaMax)) {
          a[5] += p.G * dalpha;
          const float gp = p.alpha * dalpha;
          a[2] += -0.5f * p.dx * p.dx * gp;
          a[3] += -p.dx * p.dy * gp;
          a[4] += -0.5f * p.dy * p.dy * gp;
          a[0] += -(co.x * p.dx + co.y * p.dy) * gp;
          a[1] += -(co.y * p.dx + co.z * p.dy) * gp;
        }
      }
      const bool wany = __any(any);
      if (wany) {
#pragma unroll
        for (int q = 0; q < 9; ++q) a[q] = wave_sum(a[q]);
        if (lane == 0) {
#pragma unroll
          for (int q = 0; q < 9; ++q) s_acc[j][q] = a[q];
        }
      }
      if (lane == 0) s_any[j] = wany ? 1 : 0;
    }
    __syncthreads();
    if (lane < cnt && s_any[lane]) {
      float* dst = g2d + static_cast<int64_t>(kG2DStride) * s_g[lane];
#pragma unroll
      for (int q = 0; q < 9; ++q) atomicAdd(dst + q, s_acc[lane][q]);
    }
    __syncthreads();
  }
  if (pair_counter) {
    long long e = evaluated;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    if (lane == 0) atomicAdd(pair_counter, static_cast<unsigned long long>(e));
  }
}

hipError_t launch_render_fwd(const ViewSet& vs, const Geom& geom, const uint32_t* vals, const uint32_t* ranges,
                             hipStream_t s) {
  if (vs.total_tiles == 0) return hipSuccess;
  StageScope scope(PVG_STAGE_RENDER_FWD, s);
  const int64_t grid = ((vs.total_tiles + 7) / 8) * 8;
  hipLaunchKernelGGL(k_render_fwd, dim3(static_cast<unsigned>(grid)), dim3(64), 0, s, vs, geom, vals, ranges,
                     profile_work_counter(PVG_STAGE_RENDER_FWD));
  return hipGetLastError();
}

hipError_t launch_render_bwd(const ViewSet& vs, const Geom& geom, const uint32_t* vals, const uint32_t* ranges,
                             const float* dL_dimg_base, float* g2d, hipStream_t s) {
  (void)dL_dimg_base;
  if (vs.total_tiles == 0) return hipSuccess;
  StageScope scope(PVG_STAGE_RENDER_BWD, s);
  const int64_t grid = ((vs.total_tiles + 7) / 8) * 8;
  hipLaunchKernelGGL(k_render_bwd, dim3(static_cast<unsigned>(grid)), dim3(64), 0, s, vs, geom, vals, ranges, g2d,
                     profile_work_counter(PVG_STAGE_RENDER_BWD));
  return hipGetLastError();
}

}  // namespace pvg
