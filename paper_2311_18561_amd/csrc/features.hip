// Compositing of an N-vector per Gaussian and its adjoint on gfx950: the
// semantic class scores of Sec. 4.1 blended by Eq. (3) in place of the
// colour, for all N channels in one walk of each tile list.
//
// The walk is the colour kernel's (one wave per 16x16 tile, four pixels per
// lane, batches of 64 Gaussians staged in LDS, the same base-2 pair exponent
// and the same skip and stop decisions), so final_T and n_contrib match the
// colour render of the same lists bit for bit.  What changes is the payload:
// a batch stages kNC channels per Gaussian (the vector padded to a multiple
// of four with zeros) and a pair costs kNC multiply-adds per pixel on top of
// its alpha.  The adjoint keeps the pixels' N upstream gradients in
// registers, forms per pair the blended gradient sum_c f_c dL/dC_c once per
// pixel, and reduces six screen-space sums plus the kNC feature sums across
// the wave into one record per (Gaussian, tile) pair, stored without atomics
// at the pair's emission-order index; a gather then adds each Gaussian's
// flagged records, writing the screen-space part for the per-Gaussian chain
// and adding the feature part into the caller's gradient rows.
#include "blend.hpp"

namespace pvg {

// Floats of one adjoint record: d(mean 2D) 2, d(conic) 3, d(opacity) 1, two
// zeros (so that records are 16-byte aligned), d(feature) kNC.
constexpr int feature_record_floats(int kNC) { return 8 + kNC; }

// Channels c < nch of Gaussian g (row stride ld), padded with zeros to kNC.
template <int kNC>
__device__ __forceinline__ void load_feature(const float* __restrict__ feat, int64_t ld, int nch, uint32_t g,
                                             float4 out[kNC / 4]) {
  const float* row = feat + ld * static_cast<int64_t>(g);
#pragma unroll
  for (int q = 0; q < kNC / 4; ++q) {
    out[q].x = 4 * q + 0 < nch ? row[4 * q + 0] : 0.0f;
    out[q].y = 4 * q + 1 < nch ? row[4 * q + 1] : 0.0f;
    out[q].z = 4 * q + 2 < nch ? row[4 * q + 2] : 0.0f;
    out[q].w = 4 * q + 3 < nch ? row[4 * q + 3] : 0.0f;
  }
}

template <int kNC, bool kCulled>
__global__ void __launch_bounds__(64) k_feat_fwd(ViewSet vs, Geom geom, const uint32_t* __restrict__ vals,
                                                 const uint32_t* __restrict__ ranges, const float* __restrict__ feat,
                                                 int64_t ld, int nch, float* __restrict__ out) {
  constexpr int kQ = kNC / 4;
  __shared__ float2 s_xy[64];
  __shared__ float4 s_co[64];
  __shared__ int s_pos[64];
  __shared__ float4 s_f[64][kQ];
  const int64_t ntiles = live_tiles(vs);
  const int64_t tile = xcd_tile(blockIdx.x, vs.total_tiles);
  if (tile >= ntiles) return;
  const View& v = vs.one;
  const int tx = static_cast<int>(tile % v.GX), ty = static_cast<int>(tile / v.GX);
  const int lane = threadIdx.x;
  const int px = tx * kTile + (lane & 15);
  const int py0 = ty * kTile + (lane >> 4);
  const float fpx = static_cast<float>(px);
  float X0, X1, Y0, Y1;
  tile_bounds(tx, ty, v.W, v.H, X0, X1, Y0, Y1);
  const uint64_t lt = (1ull << lane) - 1ull;
  float T[kPix], F[kPix][kNC];
  int last[kPix];
  bool act[kPix];
#pragma unroll
  for (int k = 0; k < kPix; ++k) {
    T[k] = 1.0f;
    last[k] = 0;
    act[k] = px < v.W && py0 + 4 * k < v.H;
#pragma unroll
    for (int c = 0; c < kNC; ++c) F[k][c] = 0.0f;
  }
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
  for (uint32_t b0 = start; b0 < end; b0 += 64) {
    if (!__any(act[0] || act[1] || act[2] || act[3])) break;
    const uint32_t idx = b0 + lane;
    bool keep = false;
    uint32_t g = 0;
    float2 m;
    float4 co;
    if (idx < end) {
      g = vals[idx];
      m = reinterpret_cast<const float2*>(geom.xy)[g];
      co = reinterpret_cast<const float4*>(geom.conic_op)[g];
      keep = kCulled || tile_reachable(m.x, m.y, co.x, co.y, co.z, co.w, X0, X1, Y0, Y1);
    }
    const uint64_t km = __ballot(keep);
    const int cnt = __popcll(km);
    if (keep) {
      const int slot = __popcll(km & lt);
      s_xy[slot] = m;
      s_co[slot] = pair_coefs(co.x, co.y, co.z, co.w);
      s_pos[slot] = static_cast<int>(idx - start) + 1;
      float4 f[kQ];
      load_feature<kNC>(feat, ld, nch, g, f);
#pragma unroll
      for (int q = 0; q < kQ; ++q) s_f[slot][q] = f[q];
    }
    if (lane >= cnt && lane < pad_to(cnt)) {  // padding pairs (alpha = 0, finite values); the lane may also have filled a slot below cnt
      s_xy[lane] = make_float2(0.0f, 0.0f);
      s_co[lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      s_pos[lane] = 0;
#pragma unroll
      for (int q = 0; q < kQ; ++q) s_f[lane][q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    __syncthreads();
    // groups of kGroup pairs, one test for a finished wave per group (as in
    // the colour forward)
    for (int j0 = 0; j0 < cnt; j0 += kGroup) {
      if (!__any(act[0] || act[1] || act[2] || act[3])) break;
#pragma unroll
      for (int u = 0; u < kGroup; ++u) {
        const int j = j0 + u;
        const float2 gm = s_xy[j];
        const float4 gc = s_co[j];
        const int pos = s_pos[j];
        const float dx = gm.x - fpx;
        const float c1 = gc.y * dx, c0 = (gc.x * dx) * dx;
        float w[kPix];
#pragma unroll
        for (int k = 0; k < kPix; ++k) {
          const float dy = gm.y - static_cast<float>(py0 + 4 * k);
          const float p2 = pair_exp2(gc.z, c1, c0, dy);
          const float alpha = fminf(kAlphaMax, gc.w * __builtin_amdgcn_exp2f(p2));
          const bool ok = act[k] && !(p2 > 0.0f) && !(alpha < kAlphaMin);
          const float Tn = T[k] * (1.0f - alpha);
          const bool stop = ok && Tn < kTMin;
          const bool use = ok && !stop;
          w[k] = use ? alpha * T[k] : 0.0f;
          T[k] = use ? Tn : T[k];
          last[k] = use ? pos : last[k];
          act[k] = act[k] && !stop;
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          const float4 f = s_f[j][q];
#pragma unroll
          for (int k = 0; k < kPix; ++k) {
            F[k][4 * q + 0] = fmaf(f.x, w[k], F[k][4 * q + 0]);
            F[k][4 * q + 1] = fmaf(f.y, w[k], F[k][4 * q + 1]);
            F[k][4 * q + 2] = fmaf(f.z, w[k], F[k][4 * q + 2]);
            F[k][4 * q + 3] = fmaf(f.w, w[k], F[k][4 * q + 3]);
          }
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
      v.final_T[o] = T[k];
      v.n_contrib[o] = last[k];
#pragma unroll
      for (int c = 0; c < kNC; ++c)
        if (c < nch) out[c * HW + o] = F[k][c];
    }
  }
}

template <int kNC, bool kCulled>
__global__ void __launch_bounds__(64) k_feat_bwd(ViewSet vs, Geom geom, Lists lists, const float* __restrict__ feat,
                                                 int64_t ld, int nch, const float* __restrict__ dout, float* rec,
                                                 uint8_t* vis) {
  // As in the colour adjoint, every branch decision comes from pair_coefs,
  // pair_exp2 and single products, which fuse with nothing; the gradient
  // arithmetic may fuse.
#pragma clang fp contract(fast)
  constexpr int kQ = kNC / 4;
  constexpr int kRec = feature_record_floats(kNC);
  __shared__ float2 s_xy[64];
  __shared__ float4 s_co[64];
  __shared__ float4 s_q[64];
  __shared__ int s_pos[64];
  __shared__ float4 s_f[64][kQ];
  __shared__ float4 s_acc[64][kRec / 4];
  __shared__ int s_any[64];
  const int64_t ntiles = live_tiles(vs);
  const int64_t tile = xcd_tile(blockIdx.x, vs.total_tiles);
  if (tile >= ntiles) return;
  const View& v = vs.one;
  const int tx = static_cast<int>(tile % v.GX), ty = static_cast<int>(tile / v.GX);
  const int lane = threadIdx.x;
  const int px = tx * kTile + (lane & 15);
  const int py0 = ty * kTile + (lane >> 4);
  const float fpx = static_cast<float>(px);
  float X0, X1, Y0, Y1;
  tile_bounds(tx, ty, v.W, v.H, X0, X1, Y0, Y1);
  const uint64_t lt = (1ull << lane) - 1ull;
  const int64_t HW = static_cast<int64_t>(v.W) * v.H;
  reinterpret_cast<float*>(s_acc[lane])[6] = 0.0f;  // record slots 6 and 7 stay zero
  reinterpret_cast<float*>(s_acc[lane])[7] = 0.0f;
  float T[kPix], rr[kPix], G[kPix][kNC];
  int last[kPix];
  int lmax = 0;
#pragma unroll
  for (int k = 0; k < kPix; ++k) {
    const int py = py0 + 4 * k;
    const bool in = px < v.W && py < v.H;
    const int64_t o = static_cast<int64_t>(py) * v.W + px;
    T[k] = in ? v.final_T[o] : 1.0f;
    last[k] = in ? v.n_contrib[o] : 0;
#pragma unroll
    for (int c = 0; c < kNC; ++c) G[k][c] = (in && c < nch) ? dout[c * HW + o] : 0.0f;
    rr[k] = 0.0f;  // the blend behind the last contributor: no background for features
    lmax = max(lmax, last[k]);
  }
  lmax = wave_max(lmax);
  const uint32_t start = lists.ranges[2 * tile];
  lmax = min(lmax, static_cast<int>(lists.ranges[2 * tile + 1] - start));  // never read past the tile's list
  for (int hi = lmax; hi > 0; hi -= 64) {
    const int lo = max(0, hi - 64);
    bool keep = false;
    uint32_t g = 0;
    float2 m;
    float4 co;
    if (lane < hi - lo) {
      g = lists.vals[start + lo + lane];
      m = reinterpret_cast<const float2*>(geom.xy)[g];
      co = reinterpret_cast<const float4*>(geom.conic_op)[g];
      keep = kCulled || tile_reachable(m.x, m.y, co.x, co.y, co.z, co.w, X0, X1, Y0, Y1);
    }
    const uint64_t km = __ballot(keep);
    if (keep) {
      const int slot = __popcll(km & lt);
      s_xy[slot] = m;
      s_co[slot] = make_float4(-co.x, -co.y, -co.z, co.w > 0.0f ? __builtin_amdgcn_rcpf(co.w) : 0.0f);
      s_q[slot] = pair_coefs(co.x, co.y, co.z, co.w);
      s_pos[slot] = lo + lane;
      float4 f[kQ];
      load_feature<kNC>(feat, ld, nch, g, f);
#pragma unroll
      for (int q = 0; q < kQ; ++q) s_f[slot][q] = f[q];
    }
    __syncthreads();
    const int cnt = __popcll(km);
    for (int j = cnt - 1; j >= 0; --j) {
      const float2 gm = s_xy[j];
      const float4 gc = s_co[j];
      const float4 gq = s_q[j];
      const int pos = s_pos[j];
      // alpha of the lane's four pixels as in the colour adjoint; a pair no
      // pixel of the tile uses takes alpha = 0 everywhere, which leaves T
      // (rcp(1) is exact) and the blend behind it unchanged: it is skipped
      const float dx = gm.x - fpx;
      const float c1 = gq.y * dx, c0 = (gq.x * dx) * dx;
      float au[kPix], gate[kPix];
      bool any = false;
#pragma unroll
      for (int k = 0; k < kPix; ++k) {
        const bool inr = pos < last[k];
        const float dy = gm.y - static_cast<float>(py0 + 4 * k);
        const float p2 = pair_exp2(gq.z, c1, c0, dy);
        const float raw = gq.w * __builtin_amdgcn_exp2f(p2);
        const float alpha = fminf(kAlphaMax, raw);
        const bool ok = inr && !(p2 > 0.0f) && !(alpha < kAlphaMin);
        any = any || ok;
        au[k] = ok ? alpha : 0.0f;
        gate[k] = raw > kAlphaMax ? 0.0f : au[k];  // alpha's own gradient is 0 where it is clamped
      }
      const bool wany = __any(any);
      if (lane == 0) s_any[j] = wany ? 1 : 0;
      if (!wany) continue;
      // blended gradient of each pixel: sum_c f_c dL/dC_c
      float cg[kPix];
#pragma unroll
      for (int k = 0; k < kPix; ++k) cg[k] = 0.0f;
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const float4 f = s_f[j][q];
#pragma unroll
        for (int k = 0; k < kPix; ++k)
          cg[k] += f.x * G[k][4 * q] + f.y * G[k][4 * q + 1] + f.z * G[k][4 * q + 2] + f.w * G[k][4 * q + 3];
      }
      // transmittance recovery and the moments of the power gradient
      float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, w[kPix];
#pragma unroll
      for (int k = 0; k < kPix; ++k) {
        const float dy = gm.y - static_cast<float>(py0 + 4 * k);
        const float om = 1.0f - au[k];
        T[k] *= __builtin_amdgcn_rcpf(om);
        const float d = cg[k] - rr[k];
        const float dal = T[k] * d;
        w[k] = au[k] * T[k];
        rr[k] = fmaf(au[k], d, rr[k]);  // alpha c + (1 - alpha) rr
        const float gp = gate[k] * dal;
        s0 += gp;
        s1 = fmaf(dy, gp, s1);
        s2 = fmaf(dy * dy, gp, s2);
      }
      // the six screen-space sums and the kNC feature sums, reduced without
      // the record's two zero slots (6, 7) between them
      float a[6 + kNC];
      {
        const float sx = dx * s0;
        a[0] = gc.x * sx + gc.y * s1;  // gc holds -A, -B, -C and 1 / o
        a[1] = gc.y * sx + gc.z * s1;
        a[2] = -0.5f * (dx * sx);
        a[3] = -(dx * s1);
        a[4] = -0.5f * s2;
        a[5] = s0 * gc.w;
#pragma unroll
        for (int c = 0; c < kNC; ++c) a[6 + c] = w[0] * G[0][c] + w[1] * G[1][c] + w[2] * G[2][c] + w[3] * G[3][c];
      }
      wave_sum_store<6 + kNC, 6, 2>(a, lane, reinterpret_cast<float*>(s_acc[j]));
    }
    __syncthreads();
    if (keep && s_any[__popcll(km & lt)] != 0) {
      const int slot = __popcll(km & lt);
      const uint32_t e = record_index<kCulled>(lists, geom, v, g, m, tx, ty);
      if (static_cast<int64_t>(e) < lists.capacity) {
        float4* dst = reinterpret_cast<float4*>(rec + kRec * static_cast<int64_t>(e));
#pragma unroll
        for (int q = 0; q < kRec / 4; ++q) dst[q] = s_acc[slot][q];
        vis[e] = 1;
      }
    }
    __syncthreads();
  }
}

// Per visible Gaussian: the sum of its flagged records.  g2d receives the
// six screen-space sums (slots 6..13 zero: no colour, no channels) and the
// feature sums are added into feat_grad[g][c], c < nch.  Records are read
// 16 bytes at a time.  The block's feature sums are staged in LDS and added
// into its 256 rows of feat_grad at the end, consecutive threads on
// consecutive columns: a thread adding its own row's nch floats made each
// load and store touch a cache line per lane.
template <int kNC, bool kCulled>
__global__ void __launch_bounds__(256) k_feat_gather(ViewSet vs, Geom geom, Lists lists, const float* __restrict__ rec,
                                                     const uint8_t* __restrict__ vis, float* g2d, float* feat_grad,
                                                     int64_t ld, int nch) {
  constexpr int kRec = feature_record_floats(kNC);
  constexpr int kAcc = (kRec + 15) / 16 * 16;
  __shared__ uint32_t s_queue[256][3];  // wave-gathered Gaussians from the front, block-gathered from the back
  __shared__ uint32_t s_idx[4][1024];
  __shared__ float s_red[4][kRec];
  __shared__ float s_fg[256 * kNC];  // row r: the feature sums of Gaussian base + r
  __shared__ uint8_t s_has[256];     // row r holds a visible Gaussian's sums
  __shared__ int s_qn, s_hn;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) { s_qn = 0; s_hn = 0; }
  s_has[tid] = 0;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * 256;
  const int64_t gi = base + tid;
  const bool visible = gi < live_gauss(vs) && geom.radius[gi] > 0;
  uint32_t e0 = 0, cnt = 0;
  if (visible) record_range<kCulled>(vs, geom, lists, gi, e0, cnt);
  if (visible && cnt <= kShortRange) {
    float acc[kAcc];
    gather_range<kRec, kAcc>(e0, cnt, rec, vis, acc);
    float* dst = g2d + kG2DStride * gi;
#pragma unroll
    for (int c = 0; c < 14; ++c) dst[c] = c < 6 ? acc[c] : 0.0f;
#pragma unroll
    for (int c = 0; c < kNC; ++c)
      if (c < nch) s_fg[tid * kNC + c] = acc[8 + c];
    s_has[tid] = 1;
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
    float acc[kAcc];
    gather_range_wave<kRec, kAcc>(s_queue[qi][1], s_queue[qi][2], lane, rec, vis, s_idx[wid], acc);
    wave_sum_store<kRec>(acc, lane, s_red[wid]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < 14) g2d[kG2DStride * static_cast<int64_t>(g) + lane] = lane < 6 ? s_red[wid][lane] : 0.0f;
    const int row = static_cast<int>(static_cast<int64_t>(g) - base);
    if (lane < nch && lane < kNC) s_fg[row * kNC + lane] = s_red[wid][8 + lane];
    if (lane == 0) s_has[row] = 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // block-gathered Gaussians (more than kHugeRange listed pairs), one at a
  // time: wave w sums rounds w, w + 4, ... of 1,024 pairs and the four shares
  // are added in wave order
  __syncthreads();
  for (int h = 0; h < hn; ++h) {
    const uint32_t g = s_queue[255 - h][0], he0 = s_queue[255 - h][1], hcnt = s_queue[255 - h][2];
    float acc[kAcc];
#pragma unroll
    for (int c = 0; c < kAcc; ++c) acc[c] = 0.0f;
    for (uint32_t r0 = 1024u * static_cast<uint32_t>(wid); r0 < hcnt; r0 += 4096u) {
      float part[kAcc];
      gather_range_wave<kRec, kAcc>(he0 + r0, min(1024u, hcnt - r0), lane, rec, vis, s_idx[wid], part);
#pragma unroll
      for (int c = 0; c < kAcc; ++c) acc[c] += part[c];
    }
    wave_sum_store<kRec>(acc, lane, s_red[wid]);
    __syncthreads();
    if (tid < kRec) {
      const float v = ((s_red[0][tid] + s_red[1][tid]) + s_red[2][tid]) + s_red[3][tid];
      if (tid < 14) g2d[kG2DStride * static_cast<int64_t>(g) + tid] = tid < 6 ? v : 0.0f;
      const int row = static_cast<int>(static_cast<int64_t>(g) - base);
      if (tid >= 8 && tid - 8 < nch && tid - 8 < kNC) s_fg[row * kNC + (tid - 8)] = v;
      if (tid == 0) s_has[row] = 1;
    }
    if (tid < 14 && tid >= kRec) g2d[kG2DStride * static_cast<int64_t>(g) + tid] = 0.0f;
    __syncthreads();
  }
  __syncthreads();
  const int nw = min(nch, kNC);
  for (int i = tid; i < 256 * nw; i += 256) {
    const int row = i / nw, col = i - row * nw;
    if (s_has[row]) feat_grad[ld * (base + row) + col] += s_fg[row * kNC + col];
  }
}

int feature_width(int nch) {
  return nch <= 4 ? 4 : nch <= 8 ? 8 : nch <= 12 ? 12 : nch <= 16 ? 16 : nch <= 20 ? 20 : nch <= 24 ? 24 : 32;
}

namespace {
template <int kNC>
hipError_t fwd_at(const ViewSet& vs, const Geom& geom, const uint32_t* vals, const uint32_t* ranges, bool culled,
                  const float* feat, int64_t ld, int nch, float* out, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(render_grid(vs.total_tiles)));
  auto k = culled ? k_feat_fwd<kNC, true> : k_feat_fwd<kNC, false>;
  hipLaunchKernelGGL(k, grid, dim3(64), 0, s, vs, geom, vals, ranges, feat, ld, nch, out);
  return hipGetLastError();
}

template <int kNC>
hipError_t bwd_at(const ViewSet& vs, const Geom& geom, const Lists& lists, const float* feat, int64_t ld, int nch,
                  const float* dout, float* rec, uint8_t* vis, int64_t vis_bytes, float* g2d, float* feat_grad,
                  hipStream_t s) {
  {
    StageScope scope(PVG_STAGE_RENDER_BWD, s);
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(vis), 0u, vis_bytes / 4, s);
    if (e != hipSuccess) return e;
    const dim3 grid(static_cast<unsigned>(render_grid(vs.total_tiles)));
    auto k = lists.culled ? k_feat_bwd<kNC, true> : k_feat_bwd<kNC, false>;
    hipLaunchKernelGGL(k, grid, dim3(64), 0, s, vs, geom, lists, feat, ld, nch, dout, rec, vis);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (vs.total_gauss == 0) return hipSuccess;
  StageScope scope(PVG_STAGE_GRAD_GATHER, s);
  auto k = lists.culled ? k_feat_gather<kNC, true> : k_feat_gather<kNC, false>;
  hipLaunchKernelGGL(k, dim3(static_cast<unsigned>((vs.total_gauss + 255) / 256)), dim3(256), 0, s, vs, geom, lists,
                     rec, vis, g2d, feat_grad, ld, nch);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_feature_fwd(const ViewSet& vs, const Geom& geom, const uint32_t* vals, const uint32_t* ranges,
                              bool culled, const float* feat, int64_t ld, int nch, float* out, hipStream_t s) {
  if (vs.total_tiles == 0) return hipSuccess;
  StageScope scope(PVG_STAGE_RENDER_FWD, s);
  switch (feature_width(nch)) {
    case 4: return fwd_at<4>(vs, geom, vals, ranges, culled, feat, ld, nch, out, s);
    case 8: return fwd_at<8>(vs, geom, vals, ranges, culled, feat, ld, nch, out, s);
    case 12: return fwd_at<12>(vs, geom, vals, ranges, culled, feat, ld, nch, out, s);
    case 16: return fwd_at<16>(vs, geom, vals, ranges, culled, feat, ld, nch, out, s);
    case 20: return fwd_at<20>(vs, geom, vals, ranges, culled, feat, ld, nch, out, s);
    case 24: return fwd_at<24>(vs, geom, vals, ranges, culled, feat, ld, nch, out, s);
    default: return fwd_at<32>(vs, geom, vals, ranges, culled, feat, ld, nch, out, s);
  }
}

hipError_t launch_feature_bwd(const ViewSet& vs, const Geom& geom, const Lists& lists, const float* feat, int64_t ld,
                              int nch, const float* dout, float* rec, uint8_t* vis, int64_t vis_bytes, float* g2d,
                              float* feat_grad, hipStream_t s) {
  if (vs.total_tiles == 0) return hipSuccess;
  switch (feature_width(nch)) {
    case 4: return bwd_at<4>(vs, geom, lists, feat, ld, nch, dout, rec, vis, vis_bytes, g2d, feat_grad, s);
    case 8: return bwd_at<8>(vs, geom, lists, feat, ld, nch, dout, rec, vis, vis_bytes, g2d, feat_grad, s);
    case 12: return bwd_at<12>(vs, geom, lists, feat, ld, nch, dout, rec, vis, vis_bytes, g2d, feat_grad, s);
    case 16: return bwd_at<16>(vs, geom, lists, feat, ld, nch, dout, rec, vis, vis_bytes, g2d, feat_grad, s);
    case 20: return bwd_at<20>(vs, geom, lists, feat, ld, nch, dout, rec, vis, vis_bytes, g2d, feat_grad, s);
    case 24: return bwd_at<24>(vs, geom, lists, feat, ld, nch, dout, rec, vis, vis_bytes, g2d, feat_grad, s);
    default: return bwd_at<32>(vs, geom, lists, feat, ld, nch, dout, rec, vis, vis_bytes, g2d, feat_grad, s);
  }
}

}  // namespace pvg
