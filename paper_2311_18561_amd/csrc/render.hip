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
// screen-space gradients per lane and reduces them across the wave.  Each
// (Gaussian, tile) pair's nine sums are stored, without atomics, at the pair's
// index in emission order (a Gaussian's pairs are contiguous there) and
// flagged in a byte array; a gather kernel then adds each Gaussian's flagged
// pairs.  Device-scope float atomics resolve
// at the memory side on this chip and cost three times the rest of the
// kernel, and the atomic-free sums are bitwise reproducible.
//
// Tiles are assigned so that each of the eight XCDs (which receive workgroups
// round-robin) works on one contiguous band of tiles, keeping the Gaussians
// shared by neighbouring tiles in that XCD's L2.
#include "pvg_math.hpp"

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

// Sums ten per-lane values over the wave by halving: a half-wave swap adds
// two values at once (lanes 0-31 keep the sums of the even-indexed values,
// 32-63 of the odd ones), a row swap does the same between the two 16-lane
// rows of each half, and DPP folds the last three values within each row.
// Afterwards every lane of row r (lanes 16r .. 16r+15) holds, in out[k], the
// wave total of value 4k + 2(r & 1) + (r >> 1) (indices >= 10 are padding).
__device__ __forceinline__ float swap_sum32(float x, float y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap_sum16(float x, float y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float dpp_add(float x, int ctrl) {
  switch (ctrl) {  // the control word must be a compile-time constant
    case 0x128: return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xf, 0xf, false));
    case 0x124: return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x124, 0xf, 0xf, false));
    case 0x4e: return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4e, 0xf, 0xf, false));
    default: return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xb1, 0xf, 0xf, false));
  }
}
__device__ __forceinline__ void wave_sum10(const float a[10], float out[3]) {
  float h[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) h[m] = swap_sum32(a[2 * m], a[2 * m + 1]);
  out[0] = swap_sum16(h[0], h[1]);
  out[1] = swap_sum16(h[2], h[3]);
  out[2] = swap_sum16(h[4], 0.0f);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    out[k] = dpp_add(out[k], 0x128);  // row_ror:8
    out[k] = dpp_add(out[k], 0x124);  // row_ror:4
    out[k] = dpp_add(out[k], 0x4e);   // quad_perm [2,3,0,1]
    out[k] = dpp_add(out[k], 0xb1);   // quad_perm [1,0,3,2]
  }
}

// The same for sixteen values: out[k] (k < 4) of the lanes of row r holds the
// wave total of value 4k + 2(r & 1) + (r >> 1).
__device__ __forceinline__ void wave_sum16(const float a[16], float out[4]) {
  float h[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) h[m] = swap_sum32(a[2 * m], a[2 * m + 1]);
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = swap_sum16(h[2 * k], h[2 * k + 1]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    out[k] = dpp_add(out[k], 0x128);  // row_ror:8
    out[k] = dpp_add(out[k], 0x124);  // row_ror:4
    out[k] = dpp_add(out[k], 0x4e);   // quad_perm [2,3,0,1]
    out[k] = dpp_add(out[k], 0xb1);   // quad_perm [1,0,3,2]
  }
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
  return x;
}

// The pair exponent in base 2.  With the conic (A, B, C) scaled once per
// Gaussian into q = -log2(e) (A / 2, B, C / 2), the exponent of Eq. (3)'s
// 2D Gaussian at offset (dx, dy) is power = ln 2 * p2 with
//   p2 = q.x dx^2 + q.y dx dy + q.z dy^2 = (q.z dy + q.y dx) dy + q.x dx^2,
// so alpha = o 2^p2 takes the hardware base-2 exponential directly.  A lane
// forms c1 = q.y dx and c0 = q.x dx^2 once per Gaussian (its four pixels
// share dx) and then two FMAs per pixel.  The rounding differs from the
// natural-base form by a few ulps relative to the terms' magnitudes; a skip
// or stop decision can then go the other way only where its exact value sits
// within that of a threshold.  The forward and the adjoint share this
// function, so they take every decision alike.
constexpr float kLog2e = 1.44269504088896341f;

__device__ __forceinline__ float4 pair_coefs(float A, float B, float C, float o) {
  return make_float4(-0.5f * kLog2e * A, -kLog2e * B, -0.5f * kLog2e * C, o);
}

__device__ __forceinline__ float pair_exp2(float qz, float c1, float c0, float dy) {
  return fmaf(fmaf(qz, dy, c1), dy, c0);
}

constexpr int kPix = 4;  // pixels per lane

// kCh: also blend each Gaussian's camera depth, mean velocity and
// staticness into the channels the view asks for (the flexible rendering of
// Sec. 3.1, with these in place of the colour).
template <bool kCount, bool kCulled, bool kCh>
__global__ void __launch_bounds__(64) k_render_fwd(ViewSet vs, Geom geom, const uint32_t* __restrict__ vals,
                                                   const uint32_t* __restrict__ ranges,
                                                   unsigned long long* pair_counter) {
  __shared__ float2 s_xy[64];
  __shared__ float4 s_co[64];
  __shared__ float4 s_rgb[64];  // rgb and the list position (as int bits)
  __shared__ float s_z[kCh ? 64 : 1];
  __shared__ float4 s_fv[kCh ? 64 : 1];  // v~ and rho
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
  float X0, X1, Y0, Y1;
  tile_bounds(tx, ty, v.W, v.H, X0, X1, Y0, Y1);
  const uint64_t lt = (1ull << lane) - 1ull;
  float T[kPix], Cr[kPix], Cg[kPix], Cb[kPix], Dz[kPix], V0[kPix], V1[kPix], V2[kPix], Rh[kPix];
  float Aw[kPix];  // sum T alpha, the normalized depth's denominator
  int last[kPix];
  bool act[kPix];
#pragma unroll
  for (int k = 0; k < kPix; ++k) {
    T[k] = 1.0f; Cr[k] = 0.0f; Cg[k] = 0.0f; Cb[k] = 0.0f; last[k] = 0;
    Dz[k] = 0.0f; V0[k] = 0.0f; V1[k] = 0.0f; V2[k] = 0.0f; Rh[k] = 0.0f; Aw[k] = 0.0f;
    act[k] = px < v.W && py0 + 4 * k < v.H;
  }
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
  long long evaluated = 0;
  for (uint32_t b0 = start; b0 < end; b0 += 64) {
    if (!__any(act[0] || act[1] || act[2] || act[3])) break;
    const uint32_t idx = b0 + lane;
    bool keep = false;
    float2 m;
    float4 co, c;
    float z = 0.0f;
    float4 fv = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (idx < end) {
      const uint32_t g = vals[idx];
      m = reinterpret_cast<const float2*>(geom.xy)[g];
      co = reinterpret_cast<const float4*>(geom.conic_op)[g];
      c = make_float4(geom.rgb[3 * g], geom.rgb[3 * g + 1], geom.rgb[3 * g + 2],
                      __int_as_float(static_cast<int>(idx - start) + 1));
      if (kCh) {
        z = geom.depth[g];
        if (geom.feat) fv = reinterpret_cast<const float4*>(geom.feat)[g];
      }
      keep = kCulled || tile_reachable(m.x, m.y, co.x, co.y, co.z, co.w, X0, X1, Y0, Y1);
    }
    const uint64_t km = __ballot(keep);
    if (keep) {
      const int slot = __popcll(km & lt);
      s_xy[slot] = m;
      s_co[slot] = pair_coefs(co.x, co.y, co.z, co.w);
      s_rgb[slot] = c;
      if (kCh) {
        s_z[slot] = z;
        s_fv[slot] = fv;
      }
    }
    __syncthreads();
    const int cnt = __popcll(km);
    for (int j = 0; j < cnt; ++j) {
      if (!__any(act[0] || act[1] || act[2] || act[3])) break;
      const float2 gm = s_xy[j];
      const float4 gc = s_co[j];
      const float4 cc = s_rgb[j];
      const float gz = kCh ? s_z[j] : 0.0f;
      const float4 gv = kCh ? s_fv[j] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      const int pos = __float_as_int(cc.w);
      const float dx = gm.x - fpx;
      const float c1 = gc.y * dx, c0 = (gc.x * dx) * dx;
#pragma unroll
      for (int k = 0; k < kPix; ++k) {
        if (kCount) evaluated += act[k] ? 1 : 0;
        const float dy = gm.y - static_cast<float>(py0 + 4 * k);
        const float p2 = pair_exp2(gc.z, c1, c0, dy);
        const float alpha = fminf(kAlphaMax, gc.w * __builtin_amdgcn_exp2f(p2));
        const bool ok = act[k] && !(p2 > 0.0f) && !(alpha < kAlphaMin);
        const float Tn = T[k] * (1.0f - alpha);
        const bool stop = ok && Tn < kTMin;
        const bool use = ok && !stop;
        const float w = use ? alpha * T[k] : 0.0f;
        Cr[k] = fmaf(cc.x, w, Cr[k]);
        Cg[k] = fmaf(cc.y, w, Cg[k]);
        Cb[k] = fmaf(cc.z, w, Cb[k]);
        if (kCh) {
          Dz[k] = fmaf(gz, w, Dz[k]);
          Aw[k] += w;
          V0[k] = fmaf(gv.x, w, V0[k]);
          V1[k] = fmaf(gv.y, w, V1[k]);
          V2[k] = fmaf(gv.z, w, V2[k]);
          Rh[k] = fmaf(gv.w, w, Rh[k]);
        }
        T[k] = use ? Tn : T[k];
        last[k] = use ? pos : last[k];
        act[k] = act[k] && !stop;
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
      if (v.opacity_img) v.opacity_img[o] = 1.0f - T[k];
      if (kCh) {
        // every contributor has alpha >= 1/255, so the sum is 0 exactly when none did
        if (v.depth_img) v.depth_img[o] = !v.depth_norm ? Dz[k] : (Aw[k] > 0.0f ? Dz[k] / Aw[k] : 0.0f);
        if (v.vbar_img) {
          v.vbar_img[o] = V0[k];
          v.vbar_img[HW + o] = V1[k];
          v.vbar_img[2 * HW + o] = V2[k];
        }
        if (v.rho_img) v.rho_img[o] = Rh[k];
      }
    }
  }
  if (kCount && pair_counter) {
    long long e = evaluated;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    if (lane == 0) atomicAdd(pair_counter, static_cast<unsigned long long>(e));
  }
}

// kCh: the view also carries upstream gradients of the depth, velocity and
// staticness channels and/or of final_T (each may be null); records then hold
// five more sums (d z, d v~, d rho).
template <bool kCount, bool kCulled, bool kCh>
__global__ void __launch_bounds__(64) k_render_bwd(ViewSet vs, Geom geom, Lists lists, float* rec,
                                                   uint8_t* vis, unsigned long long* pair_counter) {
  // The gradient arithmetic may fuse multiply-adds.  Every branch decision
  // (exponent sign, alpha thresholds) comes from pair_coefs, pair_exp2 (its
  // FMAs explicit) and single products, which fuse with nothing, so the
  // adjoint takes the forward's.
#pragma clang fp contract(fast)
  const uint32_t* __restrict__ vals = lists.vals;
  const uint32_t* __restrict__ ranges = lists.ranges;
  const uint32_t* __restrict__ first = lists.first;
  __shared__ float2 s_xy[64];
  __shared__ float4 s_co[64];
  __shared__ float4 s_q[64];    // pair_coefs of the conic and the opacity
  __shared__ float4 s_rgb[64];  // rgb and the 0-based list position (as int bits)
  __shared__ uint32_t s_g[64];
  __shared__ float s_acc[64][kRecFloats];
  __shared__ float s_z[kCh ? 64 : 1];
  __shared__ float4 s_fv[kCh ? 64 : 1];
  __shared__ int s_any[64];
  constexpr int kSums = kCh ? 14 : 9;  // also the record stride
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
  float X0, X1, Y0, Y1;
  tile_bounds(tx, ty, v.W, v.H, X0, X1, Y0, Y1);
  const uint64_t lt = (1ull << lane) - 1ull;
  const int64_t HW = static_cast<int64_t>(v.W) * v.H;
  float T[kPix], rr[kPix], gr[kPix], gg[kPix], gb[kPix];
  float gd[kPix], gv0[kPix], gv1[kPix], gv2[kPix], gh[kPix];  // channel gradients: z, v~, rho
  int last[kPix];
  int lmax = 0;
#pragma unroll
  for (int k = 0; k < kPix; ++k) {
    const int py = py0 + 4 * k;
    float gt = 0.0f;
    gd[k] = 0.0f; gv0[k] = 0.0f; gv1[k] = 0.0f; gv2[k] = 0.0f; gh[k] = 0.0f;
    if (px < v.W && py < v.H) {
      const int64_t o = static_cast<int64_t>(py) * v.W + px;
      T[k] = v.final_T[o];
      last[k] = v.n_contrib[o];
      gr[k] = v.dL_dimg[o];
      gg[k] = v.dL_dimg[HW + o];
      gb[k] = v.dL_dimg[2 * HW + o];
      if (kCh) {
        if (v.dL_dT) gt = v.dL_dT[o];
        if (v.dL_dO) gt -= v.dL_dO[o];  // O = 1 - final_T
        if (v.dL_ddepth) {
          gd[k] = v.dL_ddepth[o];
          if (v.depth_norm) {
            // D / A with A = sum T alpha = 1 - final_T: d/dD = 1 / A and, the
            // sum telescoping, d/d final_T = (D / A) / A
            const float A = 1.0f - T[k];
            const float ia = A > 0.0f ? 1.0f / A : 0.0f;
            gt = fmaf(gd[k] * v.depth_img[o], ia, gt);
            gd[k] *= ia;
          }
        }
        if (v.dL_dvbar) {
          gv0[k] = v.dL_dvbar[o];
          gv1[k] = v.dL_dvbar[HW + o];
          gv2[k] = v.dL_dvbar[2 * HW + o];
        }
        if (v.dL_drho) gh[k] = v.dL_drho[o];
      }
    } else {
      T[k] = 1.0f; last[k] = 0; gr[k] = 0.0f; gg[k] = 0.0f; gb[k] = 0.0f;
    }
    // the blend behind the last contributor: the background colour, and for
    // final_T a channel that is 0 on every Gaussian and 1 behind them all
    rr[k] = v.bg[0] * gr[k] + v.bg[1] * gg[k] + v.bg[2] * gb[k] + gt;
    lmax = max(lmax, last[k]);
  }
  lmax = wave_max(lmax);
  const uint32_t start = ranges[2 * tile];
  lmax = min(lmax, static_cast<int>(ranges[2 * tile + 1] - start));  // never read past the tile's list
  long long evaluated = 0;
  for (int hi = lmax; hi > 0; hi -= 64) {
    const int lo = max(0, hi - 64);
    bool keep = false;
    uint32_t g = 0;
    float2 m;
    float4 co, c;
    float z = 0.0f;
    float4 fv = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (lane < hi - lo) {
      g = vals[start + lo + lane];
      m = reinterpret_cast<const float2*>(geom.xy)[g];
      co = reinterpret_cast<const float4*>(geom.conic_op)[g];
      c = make_float4(geom.rgb[3 * g], geom.rgb[3 * g + 1], geom.rgb[3 * g + 2], __int_as_float(lo + lane));
      if (kCh) {
        z = geom.depth[g];
        if (geom.feat) fv = reinterpret_cast<const float4*>(geom.feat)[g];
      }
      keep = kCulled || tile_reachable(m.x, m.y, co.x, co.y, co.z, co.w, X0, X1, Y0, Y1);
    }
    const uint64_t km = __ballot(keep);
    if (keep) {
      const int slot = __popcll(km & lt);
      s_g[slot] = g;
      s_xy[slot] = m;
      s_co[slot] = co;
      s_q[slot] = pair_coefs(co.x, co.y, co.z, co.w);
      s_rgb[slot] = c;
      if (kCh) {
        s_z[slot] = z;
        s_fv[slot] = fv;
      }
    }
    __syncthreads();
    const int cnt = __popcll(km);
    for (int j = cnt - 1; j >= 0; --j) {
      const float2 gm = s_xy[j];
      const float4 gc = s_co[j];
      const float4 gq = s_q[j];
      const float4 cc = s_rgb[j];
      const float gz = kCh ? s_z[j] : 0.0f;
      const float4 gf = kCh ? s_fv[j] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      const int pos = __float_as_int(cc.w);
      // The lane's four pixels share the column offset dx.  Per pixel the
      // power gradient is gp = alpha dL/dalpha (zero where the pair is unused
      // or alpha is clamped); the lane sums s0 = sum gp, s1 = sum gp dy and
      // s2 = sum gp dy^2, from which the moments of gp in (dx, dy) follow.
      // An unused pair takes alpha = 0, which leaves T (rcp(1) is exact)
      // and the colour behind it unchanged, so no selects are needed.
      const float dx = gm.x - fpx;
      const float c1 = gq.y * dx, c0 = (gq.x * dx) * dx;
      float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, cr = 0.0f, cgr = 0.0f, cb = 0.0f;
      float cz = 0.0f, cv0 = 0.0f, cv1 = 0.0f, cv2 = 0.0f, ch = 0.0f;
      bool any = false;
#pragma unroll
      for (int k = 0; k < kPix; ++k) {
        const bool inr = pos < last[k];
        if (kCount) evaluated += inr ? 1 : 0;
        const float dy = gm.y - static_cast<float>(py0 + 4 * k);
        const float p2 = pair_exp2(gq.z, c1, c0, dy);
        const float raw = gq.w * __builtin_amdgcn_exp2f(p2);
        const float alpha = fminf(kAlphaMax, raw);
        const bool ok = inr && !(p2 > 0.0f) && !(alpha < kAlphaMin);
        any = any || ok;
        const float au = ok ? alpha : 0.0f;
        const float om = 1.0f - au;
        T[k] *= __builtin_amdgcn_rcpf(om);
        float cg = cc.x * gr[k] + cc.y * gg[k] + cc.z * gb[k];
        if (kCh) {  // the channels blend like a colour
          cg = fmaf(gz, gd[k], cg);
          cg = fmaf(gf.x, gv0[k], cg);
          cg = fmaf(gf.y, gv1[k], cg);
          cg = fmaf(gf.z, gv2[k], cg);
          cg = fmaf(gf.w, gh[k], cg);
        }
        const float dal = T[k] * (cg - rr[k]);
        const float w = au * T[k];
        cr = fmaf(w, gr[k], cr);
        cgr = fmaf(w, gg[k], cgr);
        cb = fmaf(w, gb[k], cb);
        if (kCh) {
          cz = fmaf(w, gd[k], cz);
          cv0 = fmaf(w, gv0[k], cv0);
          cv1 = fmaf(w, gv1[k], cv1);
          cv2 = fmaf(w, gv2[k], cv2);
          ch = fmaf(w, gh[k], ch);
        }
        rr[k] = fmaf(au, cg, om * rr[k]);
        const float gp = (raw > kAlphaMax ? 0.0f : au) * dal;
        s0 += gp;
        s1 = fmaf(dy, gp, s1);
        s2 = fmaf(dy * dy, gp, s2);
      }
      // power = -(A dx^2 + C dy^2)/2 - B dx dy and d(mean) = d(dx, dy); the
      // exponential's own gradient, sum G dL/dalpha over unclamped pairs, is
      // s0 / o (there alpha = o G)
      float a[16];
      {
        const float sx = dx * s0;
        a[0] = -(gc.x * sx + gc.y * s1);
        a[1] = -(gc.y * sx + gc.z * s1);
        a[2] = -0.5f * (dx * sx);
        a[3] = -(dx * s1);
        a[4] = -0.5f * s2;
        a[5] = gc.w > 0.0f ? s0 * __builtin_amdgcn_rcpf(gc.w) : 0.0f;
        a[6] = cr;
        a[7] = cgr;
        a[8] = cb;
        a[9] = cz;  // the channel sums are 0 without channels
        a[10] = cv0;
        a[11] = cv1;
        a[12] = cv2;
        a[13] = ch;
        a[14] = 0.0f;
        a[15] = 0.0f;
      }
      const bool wany = __any(any);
      if (wany) {
        if (kCh) {
          float red[4];
          wave_sum16(a, red);
          if ((lane & 15) == 0) {
            const int r = lane >> 4;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int q = 4 * k + 2 * (r & 1) + (r >> 1);
              if (q < kSums) s_acc[j][q] = red[k];
            }
          }
        } else {
          float red[3];
          wave_sum10(a, red);
          if ((lane & 15) == 0) {
            const int r = lane >> 4;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              const int q = 4 * k + 2 * (r & 1) + (r >> 1);
              if (q < kSums) s_acc[j][q] = red[k];
            }
          }
        }
      }
      if (lane == 0) s_any[j] = wany ? 1 : 0;
    }
    __syncthreads();
    if (keep && s_any[__popcll(km & lt)] != 0) {
      // record of this (Gaussian, tile) pair at its emission-order index,
      // flagged for the gather (pairs no pixel used keep flag 0, no record)
      const int slot = __popcll(km & lt);
      uint32_t e;
      if (kCulled) {  // the tile's rank among the Gaussian's reached tiles
        const uint32_t ri = lists.row_base[g] + static_cast<uint32_t>(ty);
        e = static_cast<uint32_t>(min<int64_t>(lists.capacity, 0xffffffffll));  // skipped below
        if (static_cast<int64_t>(ri) < lists.capacity) {  // false only for lists not from these records
          const uint2 rw = lists.rows[ri];
          e = rw.x + static_cast<uint32_t>(tx - static_cast<int>(rw.y & 0xffffu));
        }
      } else {
        int32_t rect[4];
        tile_rect(m.x, m.y, geom.radius[g], v.GX, v.GY, rect);
        e = first[g] + static_cast<uint32_t>((ty - rect[1]) * (rect[2] - rect[0]) + (tx - rect[0]));
      }
      if (static_cast<int64_t>(e) < lists.capacity) {
        float* dst = rec + kSums * static_cast<int64_t>(e);
#pragma unroll
        for (int q = 0; q < kSums; ++q) dst[q] = s_acc[slot][q];
        vis[e] = 1;
      }
    }
    __syncthreads();
  }
  if (kCount && pair_counter) {
    long long e = evaluated;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    if (lane == 0) atomicAdd(pair_counter, static_cast<unsigned long long>(e));
  }
}

// Sum of one Gaussian's flagged records in [e0, e0 + cnt) by one thread,
// reading the flags 16 at a time.  The emission order keeps a Gaussian's
// pairs contiguous.
template <int kSums>
__device__ __forceinline__ void gather_range(uint32_t e0, uint32_t cnt, const float* __restrict__ rec,
                                             const uint8_t* __restrict__ vis, float acc[16]) {
#pragma unroll
  for (int c = 0; c < 16; ++c) acc[c] = 0.0f;
  const uint32_t e1 = e0 + cnt;
  for (uint32_t b = e0 & ~15u; b < e1; b += 16) {
    const uint4 w = *reinterpret_cast<const uint4*>(vis + b);
    const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const uint32_t e = b + static_cast<uint32_t>(j);
      if (((words[j >> 2] >> (8 * (j & 3))) & 0xffu) && e >= e0 && e < e1) {
        const float* r = rec + kSums * static_cast<int64_t>(e);  // records are kSums floats apart
#pragma unroll
        for (int q = 0; q < kSums; ++q) acc[q] += r[q];
      }
    }
  }
}

constexpr uint32_t kShortRange = 48;  // Gaussians with more listed pairs are gathered by a whole wave

// Sum of one Gaussian's flagged records in [e0, e0 + cnt) by a whole wave:
// each round, lane l reads the 16 flags at b + 16 l (1024 pairs per round),
// the wave compacts the flagged indices into its LDS list `idx` (a wave
// prefix sum of the lanes' counts gives each lane its slots), and the lanes
// then take the listed records 64 at a time.  A near-camera splat with
// thousands of listed tiles thus needs a few rounds instead of one round per
// 64 flags.  Every lane returns its partial sums; the caller reduces them.
template <int kSums>
__device__ __forceinline__ void gather_range_wave(uint32_t e0, uint32_t cnt, int lane,
                                                  const float* __restrict__ rec,
                                                  const uint8_t* __restrict__ vis, uint32_t* idx,
                                                  float acc[16]) {
#pragma unroll
  for (int c = 0; c < 16; ++c) acc[c] = 0.0f;
  const uint32_t e1 = e0 + cnt;
  for (uint32_t b = e0 & ~15u; b < e1; b += 1024) {
    const uint32_t mb = b + 16u * static_cast<uint32_t>(lane);
    uint32_t words[4] = {0u, 0u, 0u, 0u};
    if (mb < e1) {
      const uint4 w = *reinterpret_cast<const uint4*>(vis + mb);
      words[0] = w.x; words[1] = w.y; words[2] = w.z; words[3] = w.w;
    }
    uint32_t bits = 0;  // bit j: pair mb + j is flagged and inside the range
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const uint32_t e = mb + static_cast<uint32_t>(j);
      if (((words[j >> 2] >> (8 * (j & 3))) & 0xffu) && e >= e0 && e < e1) bits |= 1u << j;
    }
    const int c = __popc(bits);
    int incl = c;  // inclusive prefix over the lanes
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off, 64);
      if (lane >= off) incl += y;
    }
    const int total = __shfl(incl, 63, 64);
    int slot = incl - c;
    while (bits) {
      const int j = __ffs(bits) - 1;
      bits &= bits - 1u;
      idx[slot++] = mb + static_cast<uint32_t>(j);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int k = lane; k < total; k += 64) {
      const float* r = rec + kSums * static_cast<int64_t>(idx[k]);
#pragma unroll
      for (int q = 0; q < kSums; ++q) acc[q] += r[q];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Per visible Gaussian: the index range of its pairs (first[g] and the
// listed count: its rectangle's tiles, or, for culled lists, up to the end
// of its last row) and the sum of the flagged records.
// kCh: the records hold the five channel sums too (d z, d v~, d rho); g2d
// slots 9..13 receive them, or zeros.
template <bool kCulled, bool kCh>
__global__ void __launch_bounds__(256) k_grad_gather(ViewSet vs, Geom geom, Lists lists,
                                                     const float* __restrict__ rec,
                                                     const uint8_t* __restrict__ vis, float* g2d) {
  constexpr int kSums = kCh ? 14 : 9;
  __shared__ uint32_t s_queue[256][3];
  __shared__ uint32_t s_idx[4][1024];  // per wave: flagged pair indices of one round
  __shared__ int s_qn;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) s_qn = 0;
  __syncthreads();
  const int64_t gi = static_cast<int64_t>(blockIdx.x) * 256 + tid;
  const bool visible = gi < live_gauss(vs) && geom.radius[gi] > 0;
  uint32_t e0 = 0, cnt = 0;
  if (visible) {
    e0 = lists.first[gi];
    if (kCulled) {  // (lists of an overflowed sort hold nothing; the bound below keeps reads inside)
      const View& v = view_at(vs, view_of_gauss(vs, gi));
      const float2 m = reinterpret_cast<const float2*>(geom.xy)[gi];
      int32_t rect[4];
      tile_rect(m.x, m.y, geom.radius[gi], v.GX, v.GY, rect);
      const uint32_t ri = lists.row_base[gi] + static_cast<uint32_t>(rect[3] - 1);
      if (static_cast<int64_t>(ri) < lists.capacity) {
        const uint2 rw = lists.rows[ri];
        cnt = rw.x + (rw.y >> 16) - e0;
      }
    } else {
      cnt = geom.tiles[gi];
    }
    const uint64_t cap = static_cast<uint64_t>(lists.capacity);
    if (static_cast<uint64_t>(e0) > cap || static_cast<uint64_t>(cnt) > cap - e0) cnt = 0;
  }
  if (visible && cnt <= kShortRange) {
    float acc[16];
    gather_range<kSums>(e0, cnt, rec, vis, acc);
    float* dst = g2d + kG2DStride * gi;
#pragma unroll
    for (int c = 0; c < 14; ++c) dst[c] = acc[c];
  } else if (visible) {
    const int q = atomicAdd(&s_qn, 1);
    s_queue[q][0] = static_cast<uint32_t>(gi);
    s_queue[q][1] = e0;
    s_queue[q][2] = cnt;
  }
  __syncthreads();
  const int qn = s_qn;
  for (int qi = wid; qi < qn; qi += 4) {
    const uint32_t g = s_queue[qi][0];
    float acc[16], red[4];
    gather_range_wave<kSums>(s_queue[qi][1], s_queue[qi][2], lane, rec, vis, s_idx[wid], acc);
    wave_sum16(acc, red);
    if ((lane & 15) == 0) {
      const int r = lane >> 4;
      float* dst = g2d + kG2DStride * static_cast<int64_t>(g);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int qq = 4 * k + 2 * (r & 1) + (r >> 1);
        if (qq < 14) dst[qq] = red[k];
      }
    }
  }
}

hipError_t launch_render_fwd(const ViewSet& vs, const Geom& geom, const uint32_t* vals, const uint32_t* ranges,
                             bool culled, hipStream_t s) {
  if (vs.total_tiles == 0) return hipSuccess;
  StageScope scope(PVG_STAGE_RENDER_FWD, s);
  const dim3 grid(static_cast<unsigned>(((vs.total_tiles + 7) / 8) * 8));
  unsigned long long* cnt = profile_work_counter(PVG_STAGE_RENDER_FWD);
  // channels are single-view only
  const bool depth = !vs.table && (vs.one.depth_img || vs.one.vbar_img || vs.one.rho_img);
  auto k = depth ? (cnt ? (culled ? k_render_fwd<true, true, true> : k_render_fwd<true, false, true>)
                        : (culled ? k_render_fwd<false, true, true> : k_render_fwd<false, false, true>))
                 : (cnt ? (culled ? k_render_fwd<true, true, false> : k_render_fwd<true, false, false>)
                        : (culled ? k_render_fwd<false, true, false> : k_render_fwd<false, false, false>));
  hipLaunchKernelGGL(k, grid, dim3(64), 0, s, vs, geom, vals, ranges, cnt);
  return hipGetLastError();
}

hipError_t launch_render_bwd(const ViewSet& vs, const Geom& geom, const Lists& lists, float* rec, uint8_t* vis,
                             int64_t vis_bytes, float* g2d, hipStream_t s) {
  if (vs.total_tiles == 0) return hipSuccess;
  const bool culled = lists.culled;
  // channel gradients are single-view only
  const bool ch =
      !vs.table && (vs.one.dL_ddepth || vs.one.dL_dT || vs.one.dL_dO || vs.one.dL_dvbar || vs.one.dL_drho);
  {
    StageScope scope(PVG_STAGE_RENDER_BWD, s);
    // clear the flags (a fill kernel: no memset node in a captured graph)
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(vis), 0u, vis_bytes / 4, s);
    if (e != hipSuccess) return e;
    const dim3 grid(static_cast<unsigned>(((vs.total_tiles + 7) / 8) * 8));
    unsigned long long* cnt = profile_work_counter(PVG_STAGE_RENDER_BWD);
    auto k = ch ? (cnt ? (culled ? k_render_bwd<true, true, true> : k_render_bwd<true, false, true>)
                       : (culled ? k_render_bwd<false, true, true> : k_render_bwd<false, false, true>))
                : (cnt ? (culled ? k_render_bwd<true, true, false> : k_render_bwd<true, false, false>)
                       : (culled ? k_render_bwd<false, true, false> : k_render_bwd<false, false, false>));
    hipLaunchKernelGGL(k, grid, dim3(64), 0, s, vs, geom, lists, rec, vis, cnt);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (vs.total_gauss == 0) return hipSuccess;
  StageScope scope(PVG_STAGE_GRAD_GATHER, s);
  hipLaunchKernelGGL(ch ? (culled ? k_grad_gather<true, true> : k_grad_gather<false, true>)
                        : (culled ? k_grad_gather<true, false> : k_grad_gather<false, false>),
                     dim3(static_cast<unsigned>((vs.total_gauss + 255) / 256)), dim3(256), 0, s, vs, geom, lists, rec,
                     vis, g2d);
  return hipGetLastError();
}

}  // namespace pvg
