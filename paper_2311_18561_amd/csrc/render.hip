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
// Tiles reach the eight XCDs in row-sized chunks dealt round-robin
// (xcd_tile), which balances the XCDs' work and keeps a chunk's shared
// Gaussians in one L2.
#include "blend.hpp"

namespace pvg {


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
  const int64_t tile = xcd_tile(blockIdx.x, vs.total_tiles);
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
    const int cnt = __popcll(km);
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
    if (lane >= cnt && lane < pad_to(cnt)) {
      // padding up to a whole group (the lane may also have filled a slot
      // below cnt): opacity 0 gives alpha = 0, which no pixel uses, and
      // finite values keep the blends' products at 0
      s_xy[lane] = make_float2(0.0f, 0.0f);
      s_co[lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      s_rgb[lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (kCh) {
        s_z[lane] = 0.0f;
        s_fv[lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
    }
    __syncthreads();
    // Pairs go in groups of kGroup with one test for a finished wave per
    // group, so the pixels' active flags stay in scalar lane masks through a
    // group instead of being carried in vector registers from pair to pair.
    for (int j0 = 0; j0 < cnt; j0 += kGroup) {
      if (!__any(act[0] || act[1] || act[2] || act[3])) break;
#pragma unroll
      for (int u = 0; u < kGroup; ++u) {
        const int j = j0 + u;
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
          if (kCount) evaluated += (act[k] && j < cnt) ? 1 : 0;
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
  __shared__ float2 s_xy[64];
  __shared__ float4 s_co[64];   // -A, -B, -C and 1 / o
  __shared__ float4 s_q[64];    // pair_coefs of the conic and the opacity
  __shared__ float4 s_rgb[64];  // rgb and the 0-based list position (as int bits)
  __shared__ uint32_t s_g[64];
  __shared__ float s_acc[64][kRecFloats];
  __shared__ float s_z[kCh ? 64 : 1];
  __shared__ float4 s_fv[kCh ? 64 : 1];
  __shared__ int s_any[64];
  constexpr int kSums = kCh ? 14 : 9;  // also the record stride
  const int64_t ntiles = live_tiles(vs);
  const int64_t tile = xcd_tile(blockIdx.x, vs.total_tiles);
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
      // the negated conic and 1 / o for the record sums (one reciprocal per
      // Gaussian and batch rather than per pair)
      s_co[slot] = make_float4(-co.x, -co.y, -co.z, co.w > 0.0f ? __builtin_amdgcn_rcpf(co.w) : 0.0f);
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
        const float d = cg - rr[k];
        const float dal = T[k] * d;
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
        rr[k] = fmaf(au, d, rr[k]);  // alpha c + (1 - alpha) rr
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
        a[0] = gc.x * sx + gc.y * s1;  // gc holds -A, -B, -C
        a[1] = gc.y * sx + gc.z * s1;
        a[2] = -0.5f * (dx * sx);
        a[3] = -(dx * s1);
        a[4] = -0.5f * s2;
        a[5] = s0 * gc.w;  // gc.w = 1 / o (0 for o = 0)
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
      const uint32_t e = record_index<kCulled>(lists, geom, v, g, m, tx, ty);
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
  __shared__ uint32_t s_queue[256][3];  // wave-gathered Gaussians from the front, block-gathered from the back
  __shared__ uint32_t s_idx[4][1024];   // per wave: flagged pair indices of one round
  __shared__ float s_part[4][16];       // per wave: its share of a block-gathered Gaussian's sums
  __shared__ int s_qn, s_hn;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) { s_qn = 0; s_hn = 0; }
  __syncthreads();
  const int64_t gi = static_cast<int64_t>(blockIdx.x) * 256 + tid;
  const bool visible = gi < live_gauss(vs) && geom.radius[gi] > 0;
  uint32_t e0 = 0, cnt = 0;
  if (visible) record_range<kCulled>(vs, geom, lists, gi, e0, cnt);
  if (visible && cnt <= kShortRange) {
    float acc[16];
    gather_range<kSums>(e0, cnt, rec, vis, acc);
    float* dst = g2d + kG2DStride * gi;
#pragma unroll
    for (int c = 0; c < 14; ++c) dst[c] = acc[c];
  } else if (visible) {
    const int q = cnt > kHugeRange ? 255 - atomicAdd(&s_hn, 1) : atomicAdd(&s_qn, 1);
    s_queue[q][0] = static_cast<uint32_t>(gi);
    s_queue[q][1] = e0;
    s_queue[q][2] = cnt;
  }
  __syncthreads();
  const int qn = s_qn, hn = s_hn;
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
  // block-gathered Gaussians, one at a time: wave w sums rounds w, w + 4, ...
  // and the four shares are added in wave order
  for (int h = 0; h < hn; ++h) {
    const uint32_t g = s_queue[255 - h][0], he0 = s_queue[255 - h][1], hcnt = s_queue[255 - h][2];
    float acc[16], red[4];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = 0.0f;
    for (uint32_t r0 = 1024u * static_cast<uint32_t>(wid); r0 < hcnt; r0 += 4096u) {
      float part[16];
      gather_range_wave<kSums>(he0 + r0, min(1024u, hcnt - r0), lane, rec, vis, s_idx[wid], part);
#pragma unroll
      for (int c = 0; c < 16; ++c) acc[c] += part[c];
    }
    wave_sum16(acc, red);
    if ((lane & 15) == 0) {
      const int r = lane >> 4;
#pragma unroll
      for (int k = 0; k < 4; ++k) s_part[wid][4 * k + 2 * (r & 1) + (r >> 1)] = red[k];
    }
    __syncthreads();
    if (tid < 14) g2d[kG2DStride * static_cast<int64_t>(g) + tid] = ((s_part[0][tid] + s_part[1][tid]) + s_part[2][tid]) + s_part[3][tid];
    __syncthreads();
  }
}

hipError_t launch_render_fwd(const ViewSet& vs, const Geom& geom, const uint32_t* vals, const uint32_t* ranges,
                             bool culled, hipStream_t s) {
  if (vs.total_tiles == 0) return hipSuccess;
  StageScope scope(PVG_STAGE_RENDER_FWD, s);
  const dim3 grid(static_cast<unsigned>(render_grid(vs.total_tiles)));
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
    const dim3 grid(static_cast<unsigned>(render_grid(vs.total_tiles)));
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
