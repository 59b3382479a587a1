// Sky composite of the sky refinement (Sec. 3.4): C_f = C + (1 - O) f_sky(d),
// where f_sky is a learnable cube map looked up in the pixel's world-frame
// viewing direction, optionally jittered inside the pixel.  One thread per
// pixel; the adjoint writes dL/dO and adds each pixel's bilinear weights
// times (1 - O) dL/dC_f into the cube map's gradient.  Neighbouring pixels
// share texels (a high-resolution image has several pixels per texel), so the
// adjoint has two forms.  When a texel spans no more than a few pixels (the
// usual case: fine maps), it gathers: each workgroup owns a 16 x 16 texel
// block of one face, finds the pixel rectangle that can reach it (the block's
// bilinear footprint projected into the image, with the jitter's half pixel
// and a rounding margin around it), recomputes those pixels' taps, sums the
// ones that land in the block in LDS and writes each texel once, with no
// device-memory atomics; the block holding a pixel's first tap writes its
// dL/dO.  Pixels whose jitter is beyond half a pixel (outside what the
// rectangles assume) are left to a per-pixel pass that adds them atomically.
// Coarse maps (many pixels per texel) keep the scatter form on 16 x 16 pixel
// tiles: each tile sums its contributions to the texel box it covers on its
// first pixel's face in LDS and adds the box to global memory once per texel
// and channel; pixels on another face, or a box beyond kSkyBox texels, add to
// global memory directly.
//
// Conventions: d_cam = ((px + 1/2 + jx - cx) / fx, (py + 1/2 + jy - cy) / fy,
// 1), d = R^T d_cam; faces +X, -X, +Y, -Y, +Z, -Z (0..5) by the largest |d_i|
// (ties to the lower axis); face coordinates as in OpenGL cube maps; texel
// (u R - 1/2, v R - 1/2), bilinear inside the face with the coordinates
// clamped to [0, R - 1]; cube [6][3][R][R].  The geometry is FP32 without
// contraction, so the face and texel decisions are the oracle's.
#include <climits>
#include <cmath>

#include "blend.hpp"
#include "pvg_math.hpp"

namespace pvg {

struct SkyView {
  float R[9];
  float fx, fy, cx, cy;
  int32_t W, H;
};

// Face, the four taps' texel columns tx[k & 1] and rows ty[k >> 1], their
// flat indices inside the face, and the bilinear weights.
__device__ __forceinline__ void sky_taps(const SkyView& c, int px, int py, const float* __restrict__ jitter,
                                         int64_t HW, int64_t o, int Rn, int& face, int tx[2], int ty[2], int idx[4],
                                         float w[4]) {
  const float jx = jitter ? jitter[o] : 0.0f, jy = jitter ? jitter[HW + o] : 0.0f;
  const float c0 = ((static_cast<float>(px) + 0.5f) + jx - c.cx) / c.fx;
  const float c1 = ((static_cast<float>(py) + 0.5f) + jy - c.cy) / c.fy;
  float d[3];
  for (int k = 0; k < 3; ++k) d[k] = (c.R[k] * c0 + c.R[3 + k] * c1) + c.R[6 + k] * 1.0f;
  const float ax = fabsf(d[0]), ay = fabsf(d[1]), az = fabsf(d[2]);
  float sc, tc, ma;
  if (ax >= ay && ax >= az) {
    ma = ax;
    if (d[0] >= 0.0f) { face = 0; sc = -d[2]; tc = -d[1]; } else { face = 1; sc = d[2]; tc = -d[1]; }
  } else if (ay >= az) {
    ma = ay;
    if (d[1] >= 0.0f) { face = 2; sc = d[0]; tc = d[2]; } else { face = 3; sc = d[0]; tc = -d[2]; }
  } else {
    ma = az;
    if (d[2] >= 0.0f) { face = 4; sc = d[0]; tc = -d[1]; } else { face = 5; sc = -d[0]; tc = -d[1]; }
  }
  const float u = 0.5f * (sc / ma + 1.0f), v = 0.5f * (tc / ma + 1.0f);
  const float rm = static_cast<float>(Rn - 1);
  // fminf / fmaxf also send a NaN coordinate into the face
  const float x = fminf(fmaxf(u * static_cast<float>(Rn) - 0.5f, 0.0f), rm);
  const float y = fminf(fmaxf(v * static_cast<float>(Rn) - 0.5f, 0.0f), rm);
  const int x0 = min(max(static_cast<int>(floorf(x)), 0), Rn - 1), y0 = min(max(static_cast<int>(floorf(y)), 0), Rn - 1);
  const int x1 = min(x0 + 1, Rn - 1), y1 = min(y0 + 1, Rn - 1);
  tx[0] = x0; tx[1] = x1; ty[0] = y0; ty[1] = y1;
  const float fx = x - static_cast<float>(x0), fy = y - static_cast<float>(y0);
  idx[0] = y0 * Rn + x0; w[0] = (1.0f - fx) * (1.0f - fy);
  idx[1] = y0 * Rn + x1; w[1] = fx * (1.0f - fy);
  idx[2] = y1 * Rn + x0; w[2] = (1.0f - fx) * fy;
  idx[3] = y1 * Rn + x1; w[3] = fx * fy;
}

__global__ void __launch_bounds__(256) k_sky_fwd(SkyView c, const float* __restrict__ img,
                                                 const float* __restrict__ opac, const float* __restrict__ cube,
                                                 int Rn, const float* __restrict__ jitter, float* out) {
  const int64_t HW = static_cast<int64_t>(c.W) * c.H;
  const int64_t o = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (o >= HW) return;
  const int px = static_cast<int>(o % c.W), py = static_cast<int>(o / c.W);
  int face, tx[2], ty[2], idx[4];
  float w[4];
  sky_taps(c, px, py, jitter, HW, o, Rn, face, tx, ty, idx, w);
  const int64_t F = static_cast<int64_t>(Rn) * Rn;
  const float t = 1.0f - opac[o];
  for (int ch = 0; ch < 3; ++ch) {
    const float* cf = cube + (face * 3 + ch) * F;
    const float s = ((w[0] * cf[idx[0]] + w[1] * cf[idx[1]]) + w[2] * cf[idx[2]]) + w[3] * cf[idx[3]];
    out[ch * HW + o] = img[ch * HW + o] + t * s;
  }
}

__device__ __forceinline__ float sky_wave_max(float x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmaxf(x, __shfl_xor(x, off, 64));
  return x;
}

// v 2^k as a 64-bit two's-complement integer, for |v| 2^k < 2^62, from two
// 32-bit conversions: hi = floor(V / 2^32) and lo = V - hi 2^32 in [0, 2^32)
// with V = v 2^k (the fused multiply-add is exact whenever |V| >= 2^32, where
// lo is a multiple of V's last place; below, lo = V + 2^32 may round by 2^8
// at most, 2^-40 of the largest term the scale allows).
__device__ __forceinline__ unsigned long long sky_fixed(float v, int k) {
  const float V = ldexpf(v, k);
  const float h = floorf(V * 0x1p-32f);
  const float l = fmaf(h, -0x1p32f, V);
  return (static_cast<unsigned long long>(static_cast<unsigned>(__float2int_rz(h))) << 32) |
         static_cast<unsigned long long>(__float2uint_rz(l));
}

constexpr int kSkyBox = 512;  // texels of a tile's LDS box (3 channels of 64-bit sums: 12 KiB)

// One workgroup per 16 x 16 pixel tile (GX tiles per image row).  The box
// sums in 64-bit fixed point, as the gather's blocks do: every term is at
// most m = max|(1 - O) g| over the tile and a texel takes at most 256 of
// them, so terms scaled by 2^k with 256 m 2^k < 2^62 cannot overflow.
__global__ void __launch_bounds__(256) k_sky_bwd(SkyView c, const float* __restrict__ g,
                                                 const float* __restrict__ opac, const float* __restrict__ cube,
                                                 int Rn, const float* __restrict__ jitter, float* dopac, float* dcube,
                                                 int GX) {
  __shared__ unsigned long long s_acc[3 * kSkyBox];
  __shared__ int s_box[5];  // the tile's face, then min x, min y, max x, max y of its texels there
  __shared__ unsigned s_bound[2];  // max|(1 - O) g| (float bits) and a NaN flag
  const int64_t HW = static_cast<int64_t>(c.W) * c.H;
  const int64_t F = static_cast<int64_t>(Rn) * Rn;
  const int tile_x = static_cast<int>(blockIdx.x % GX), tile_y = static_cast<int>(blockIdx.x / GX);
  const int px = tile_x * 16 + static_cast<int>(threadIdx.x & 15);
  const int py = tile_y * 16 + static_cast<int>(threadIdx.x >> 4);
  const bool in = px < c.W && py < c.H;  // always true for thread 0: a tile starts inside the image
  const int64_t o = static_cast<int64_t>(py) * c.W + px;
  int face = -1, tx[2] = {0, 0}, ty[2] = {0, 0}, idx[4] = {0, 0, 0, 0};
  float w[4] = {0.0f, 0.0f, 0.0f, 0.0f}, tg[3] = {0.0f, 0.0f, 0.0f};
  if (in) {
    sky_taps(c, px, py, jitter, HW, o, Rn, face, tx, ty, idx, w);
    const float t = 1.0f - opac[o];
    float dO = 0.0f;
    for (int ch = 0; ch < 3; ++ch) {
      const float* cf = cube + (face * 3 + ch) * F;
      const float gc = g[ch * HW + o];
      const float s = ((w[0] * cf[idx[0]] + w[1] * cf[idx[1]]) + w[2] * cf[idx[2]]) + w[3] * cf[idx[3]];
      dO -= s * gc;
      tg[ch] = t * gc;
    }
    dopac[o] = dO;
  }
  if (threadIdx.x == 0) {
    s_box[0] = face;
    s_box[1] = INT_MAX; s_box[2] = INT_MAX; s_box[3] = -1; s_box[4] = -1;
    s_bound[0] = s_bound[1] = 0u;
  }
  __syncthreads();
  const int f0 = s_box[0];
  const bool mine = in && face == f0;
  {  // the taps span [tx[0], tx[1]] x [ty[0], ty[1]]; reduced over the wave
     // first (LDS atomics of all lanes on one address compile to a loop over
     // the lanes, which cost this kernel 65 of its 110 us)
    int x0 = mine ? tx[0] : INT_MAX, y0 = mine ? ty[0] : INT_MAX, x1 = mine ? tx[1] : -1, y1 = mine ? ty[1] : -1;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      x0 = min(x0, __shfl_xor(x0, off, 64));
      y0 = min(y0, __shfl_xor(y0, off, 64));
      x1 = max(x1, __shfl_xor(x1, off, 64));
      y1 = max(y1, __shfl_xor(y1, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      atomicMin(&s_box[1], x0);
      atomicMin(&s_box[2], y0);
      atomicMax(&s_box[3], x1);
      atomicMax(&s_box[4], y1);
    }
  }
  {
    const float a0 = fabsf(tg[0]), a1 = fabsf(tg[1]), a2 = fabsf(tg[2]);
    const bool nan = __any(mine && (a0 != a0 || a1 != a1 || a2 != a2));
    const float m = sky_wave_max(mine ? fmaxf(a0, fmaxf(a1, a2)) : 0.0f);
    if ((threadIdx.x & 63) == 0) {
      atomicMax(&s_bound[0], __float_as_uint(m));
      if (nan) s_bound[1] = 1u;
    }
  }
  __syncthreads();
  const int bx = s_box[1], by = s_box[2];
  const int bw = s_box[3] - bx + 1, bh = s_box[4] - by + 1;  // >= 1: thread 0 is in the box
  const int area = bw * bh;
  const float bound = __uint_as_float(s_bound[0]);
  const bool lds = area <= kSkyBox && s_bound[1] == 0u && bound <= 3.0e38f;  // uniform over the workgroup
  int eb;
  (void)frexpf(bound, &eb);  // every term < 2^eb
  const int ks = 62 - 9 - eb;
  if (lds) {
    for (int i = threadIdx.x; i < 3 * area; i += 256) s_acc[i] = 0ull;
    __syncthreads();
  }
  // A box of at most nine texels (a coarse map: a texel spans more than the
  // tile) takes the wave's sum per texel and channel, one LDS add per wave:
  // per-lane adds there put every lane of the wave on the same few addresses.
  // A wave's 64 terms are at most 64 m, so the four waves stay within the
  // fixed point's bound.
  const bool few = lds && area <= 9;  // uniform
  if (few) {
    for (int r = 0; r < area; ++r) {
      const int xr = bx + r % bw, yr = by + r / bw;
      float v[3] = {0.0f, 0.0f, 0.0f};
      if (mine)
        for (int k = 0; k < 4; ++k)
          if (w[k] != 0.0f && tx[k & 1] == xr && ty[k >> 1] == yr)
            for (int ch = 0; ch < 3; ++ch) v[ch] += w[k] * tg[ch];
      for (int ch = 0; ch < 3; ++ch) {
        const float sum = wave_sum(v[ch]);
        if ((threadIdx.x & 63) == 0 && sum != 0.0f) atomicAdd(&s_acc[ch * area + r], sky_fixed(sum, ks));
      }
    }
  }
  if (in) {
    for (int ch = 0; ch < 3; ++ch)
      for (int k = 0; k < 4; ++k) {
        if (w[k] == 0.0f) continue;
        const float val = w[k] * tg[ch];
        if (lds && mine) {
          if (!few) atomicAdd(&s_acc[ch * area + (ty[k >> 1] - by) * bw + (tx[k & 1] - bx)], sky_fixed(val, ks));
        } else {
          atomicAdd(&dcube[(face * 3 + ch) * F + idx[k]], val);
        }
      }
  }
  if (lds) {
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * area; i += 256) {
      const long long a = static_cast<long long>(s_acc[i]);
      if (a == 0) continue;
      const float val = static_cast<float>(ldexp(static_cast<double>(a), -ks));
      const int ch = i / area, r = i - ch * area;
      const int yy = by + r / bw, xx = bx + r % bw;
      atomicAdd(&dcube[(f0 * 3 + ch) * F + static_cast<int64_t>(yy) * Rn + xx], val);
    }
  }
}

// ---- the gather form ----

constexpr int kSkyTB = 16;               // largest texel block side (the LDS sums' size)
constexpr float kSkyJitter = 0.5f;       // the |jitter| the pixel rectangles allow for
constexpr int kSkyMaxSuper = 6 * 8 * 8;  // superblocks of a cube map
constexpr int kSkyGatherThreads = 512;   // threads of a texel block's workgroup

struct SkyGather {
  float M[9];    // camera direction from a face point: c = M q, M the inverse of R^T (row-major)
  float delta;   // the face points kept have c.z >= delta (the rest project beyond the image margin)
  int32_t tb;    // texel block side: 16, or less for coarse maps (1 to 16)
  int32_t nb;    // texel blocks per face side
  int32_t sbs;   // blocks per superblock side (at most 8 superblocks per face side)
  int32_t nsb;   // superblocks per face side
  int32_t count;                // superblocks that the view can reach, listed in `sb`
  uint16_t sb[kSkyMaxSuper];    // face * nsb^2 + row * nsb + column
};

__device__ __forceinline__ bool sky_in_contract(const float* __restrict__ jitter, int64_t HW, int64_t o) {
  if (!jitter) return true;
  return fabsf(jitter[o]) <= kSkyJitter && fabsf(jitter[HW + o]) <= kSkyJitter;  // false for NaN
}

// The point of face f at face coordinates s = 2u - 1, t = 2v - 1 (the
// direction d / max|d_i| of the face convention above).
__device__ __forceinline__ void sky_face_point(int f, float s, float t, float q[3]) {
  switch (f) {
    case 0: q[0] = 1.0f; q[1] = -t; q[2] = -s; break;
    case 1: q[0] = -1.0f; q[1] = -t; q[2] = s; break;
    case 2: q[0] = s; q[1] = 1.0f; q[2] = t; break;
    case 3: q[0] = s; q[1] = -1.0f; q[2] = -t; break;
    case 4: q[0] = s; q[1] = -t; q[2] = 1.0f; break;
    default: q[0] = -s; q[1] = -t; q[2] = -1.0f; break;
  }
}

// Inclusive pixel rectangle r = (x0, y0, x1, y1) that holds every pixel with
// |jitter| <= kSkyJitter whose taps can fall in texels [X0, X1] x [Y0, Y1] of
// face f: those pixels' texel coordinates lie in [X0 - 1, X1 + 1) x [Y0 - 1,
// Y1 + 1), a rectangle of the face plane; its corners go to the camera frame,
// the polygon is cut at c.z = delta, and the bounding box of the projected
// vertices, widened by the jitter and two pixels, is clipped to the image.
// False when no part of the block is in front of the camera.
__device__ bool sky_block_rect(const SkyView& c, const SkyGather& G, int Rn, int f, int X0, int X1, int Y0, int Y1,
                               int r[4]) {
  const float inv = 1.0f / static_cast<float>(Rn);
  const float s0 = 2.0f * (static_cast<float>(X0) - 0.5f) * inv - 1.0f;
  const float s1 = 2.0f * (static_cast<float>(X1) + 1.5f) * inv - 1.0f;
  const float t0 = 2.0f * (static_cast<float>(Y0) - 0.5f) * inv - 1.0f;
  const float t1 = 2.0f * (static_cast<float>(Y1) + 1.5f) * inv - 1.0f;
  const float ss[4] = {s0, s1, s1, s0}, ts[4] = {t0, t0, t1, t1};
  float cc[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    float q[3];
    sky_face_point(f, ss[k], ts[k], q);
#pragma unroll
    for (int i = 0; i < 3; ++i) cc[k][i] = G.M[3 * i] * q[0] + G.M[3 * i + 1] * q[1] + G.M[3 * i + 2] * q[2];
  }
  float xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
  auto take = [&](float x, float y, float z) {
    const float X = c.cx + c.fx * (x / z), Y = c.cy + c.fy * (y / z);
    xmin = fminf(xmin, X); xmax = fmaxf(xmax, X);
    ymin = fminf(ymin, Y); ymax = fmaxf(ymax, Y);
  };
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float* a = cc[k];
    const float* b = cc[(k + 1) & 3];
    const bool ia = a[2] >= G.delta, ib = b[2] >= G.delta;
    if (ia) take(a[0], a[1], a[2]);
    if (ia != ib) {
      const float u = (G.delta - a[2]) / (b[2] - a[2]);
      take(a[0] + u * (b[0] - a[0]), a[1] + u * (b[1] - a[1]), G.delta);
    }
  }
  if (!(xmin <= xmax) || !(ymin <= ymax)) return false;
  // pixel px sees X = px + 1/2 + jx, so px lies in [X - 1/2 - 0.5, X - 1/2 + 0.5]
  constexpr float lim = 1.0e7f;
  const float m = 0.5f + kSkyJitter;
  r[0] = max(static_cast<int>(floorf(fmaxf(xmin - m, -lim))) - 2, 0);
  r[1] = max(static_cast<int>(floorf(fmaxf(ymin - m, -lim))) - 2, 0);
  r[2] = min(static_cast<int>(ceilf(fminf(xmax - 0.5f + kSkyJitter, lim))) + 2, c.W - 1);
  r[3] = min(static_cast<int>(ceilf(fminf(ymax - 0.5f + kSkyJitter, lim))) + 2, c.H - 1);
  return r[0] <= r[2] && r[1] <= r[3];
}

// Pixels outside the rectangles' jitter bound: the whole adjoint of each,
// with device-memory atomics.  Runs before the gather, whose plain
// read-add-writes of the cube gradient then follow these adds.
__global__ void __launch_bounds__(256) k_sky_bwd_stray(SkyView c, const float* __restrict__ g,
                                                       const float* __restrict__ opac,
                                                       const float* __restrict__ cube, int Rn,
                                                       const float* __restrict__ jitter, float* dopac,
                                                       float* dcube) {
  const int64_t HW = static_cast<int64_t>(c.W) * c.H;
  const int64_t o = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (o >= HW || sky_in_contract(jitter, HW, o)) return;
  const int px = static_cast<int>(o % c.W), py = static_cast<int>(o / c.W);
  int face, tx[2], ty[2], idx[4];
  float w[4];
  sky_taps(c, px, py, jitter, HW, o, Rn, face, tx, ty, idx, w);
  const int64_t F = static_cast<int64_t>(Rn) * Rn;
  const float t = 1.0f - opac[o];
  float dO = 0.0f;
  for (int ch = 0; ch < 3; ++ch) {
    const float* cf = cube + (face * 3 + ch) * F;
    const float gc = g[ch * HW + o];
    const float s = ((w[0] * cf[idx[0]] + w[1] * cf[idx[1]]) + w[2] * cf[idx[2]]) + w[3] * cf[idx[3]];
    dO -= s * gc;
    const float tg = t * gc;
    for (int k = 0; k < 4; ++k)
      if (w[k] != 0.0f) atomicAdd(&dcube[(face * 3 + ch) * F + idx[k]], w[k] * tg);
  }
  dopac[o] = dO;
}

// One workgroup per texel block of the superblocks the host found within
// reach of the view (a square of sbs x sbs blocks each), in the XCD chunk
// order of the renderer's tiles so that neighbouring blocks, whose pixel
// rectangles overlap, share an L2.  The block's texels sum in LDS
// in 64-bit fixed point (integer LDS atomics run at the rate of plain LDS
// writes; float ones serialize lane by lane): a first pass over the
// rectangle bounds every term by m = max|1 - O| max|g| (w <= 1), the terms
// are scaled by 2^k with n m 2^k < 2^62 for the rectangle's n pixels, so no
// sum overflows and each term keeps about 2^-40 of m, and the sums leave LDS
// through FP64.  Integer sums do not depend on the order of the additions:
// the cube gradient of a view is the same from run to run.  A non-finite
// bound (NaN or infinity among the inputs) sums in float instead.
__global__ void __launch_bounds__(kSkyGatherThreads) k_sky_bwd_gather(SkyView c, SkyGather G, const float* __restrict__ g,
                                                        const float* __restrict__ opac,
                                                        const float* __restrict__ cube, int Rn,
                                                        const float* __restrict__ jitter, float* dopac,
                                                        float* dcube) {
  constexpr int kT = kSkyTB * kSkyTB;
  __shared__ unsigned long long s_acc[3 * kT];
  __shared__ int s_rect[5];
  __shared__ unsigned s_bound[3];  // max|1 - O| and max|g| (float bits), a NaN flag
  const int per_super = G.sbs * G.sbs;
  const int64_t total = static_cast<int64_t>(G.count) * per_super;
  const int64_t b = xcd_tile(blockIdx.x, total);
  if (b >= total) return;  // uniform over the workgroup
  const int sb = G.sb[b / per_super], in_sb = static_cast<int>(b % per_super);
  const int f = sb / (G.nsb * G.nsb), sr = sb % (G.nsb * G.nsb);
  const int bx = (sr % G.nsb) * G.sbs + in_sb % G.sbs, by = (sr / G.nsb) * G.sbs + in_sb / G.sbs;
  if (bx >= G.nb || by >= G.nb) return;
  const int tb = G.tb;
  const int X0 = bx * tb, Y0 = by * tb;
  const int X1 = min(X0 + tb - 1, Rn - 1), Y1 = min(Y0 + tb - 1, Rn - 1);
  if (threadIdx.x == 0) {
    int r[4];
    s_rect[4] = sky_block_rect(c, G, Rn, f, X0, X1, Y0, Y1, r) ? 1 : 0;
    for (int k = 0; k < 4; ++k) s_rect[k] = r[k];
    s_bound[0] = s_bound[1] = s_bound[2] = 0u;
  }
  for (int i = threadIdx.x; i < 3 * kT; i += kSkyGatherThreads) s_acc[i] = 0ull;
  __syncthreads();
  if (!s_rect[4]) return;  // uniform
  // the rectangle's pixels, a workgroup's worth at a time in raster order:
  // each thread steps its column and row by the workgroup size (no division
  // in the loop)
  const int rx = s_rect[0], ry = s_rect[1], rw = s_rect[2] - s_rect[0] + 1, rh = s_rect[3] - s_rect[1] + 1;
  const int step_r = kSkyGatherThreads / rw, step_c = kSkyGatherThreads % rw;
  const int col0 = static_cast<int>(threadIdx.x) % rw, row0 = static_cast<int>(threadIdx.x) / rw;
  const int64_t HW = static_cast<int64_t>(c.W) * c.H;
  const int64_t F = static_cast<int64_t>(Rn) * Rn;
  {  // the bound
    float mo = 0.0f, mg = 0.0f;
    bool nan = false;
    for (int col = col0, row = row0; row < rh;) {
      const int64_t o = static_cast<int64_t>(ry + row) * c.W + (rx + col);
      const float a = fabsf(1.0f - opac[o]);
      const float g0 = fabsf(g[o]), g1 = fabsf(g[HW + o]), g2 = fabsf(g[2 * HW + o]);
      nan |= a != a || g0 != g0 || g1 != g1 || g2 != g2;
      mo = a > mo ? a : mo;
      mg = fmaxf(mg, fmaxf(g0, fmaxf(g1, g2)));
      col += step_c;
      row += step_r;
      if (col >= rw) { col -= rw; ++row; }
    }
    mo = sky_wave_max(mo);
    mg = sky_wave_max(mg);
    nan = __any(nan);
    if ((threadIdx.x & 63) == 0) {  // non-negative floats order as their bits
      atomicMax(&s_bound[0], __float_as_uint(mo));
      atomicMax(&s_bound[1], __float_as_uint(mg));
      if (nan) s_bound[2] = 1u;
    }
  }
  __syncthreads();
  const float mo = __uint_as_float(s_bound[0]), mg = __uint_as_float(s_bound[1]);
  const bool fixed = s_bound[2] == 0u && mo <= 3.0e38f && mg <= 3.0e38f;  // uniform
  int eo, eg;
  (void)frexpf(mo, &eo);
  (void)frexpf(mg, &eg);  // m < 2^(eo + eg)
  const int en = 64 - __clzll(static_cast<unsigned long long>(rw) * static_cast<unsigned long long>(rh));
  const int k = 62 - eo - eg - en;  // n m 2^k < 2^62 for the rectangle's n < 2^en pixels
  float* facc = reinterpret_cast<float*>(s_acc);  // the float sums of a non-finite bound
  for (int col = col0, row = row0; row < rh;) {
    const int px = rx + col, py = ry + row;
    col += step_c;
    row += step_r;
    if (col >= rw) { col -= rw; ++row; }
    const int64_t o = static_cast<int64_t>(py) * c.W + px;
    if (!sky_in_contract(jitter, HW, o)) continue;
    int face, tx[2], ty[2], idx[4];
    float w[4];
    sky_taps(c, px, py, jitter, HW, o, Rn, face, tx, ty, idx, w);
    if (face != f) continue;
    const bool cin0 = tx[0] >= X0 && tx[0] <= X1, cin1 = tx[1] >= X0 && tx[1] <= X1;
    const bool rin0 = ty[0] >= Y0 && ty[0] <= Y1, rin1 = ty[1] >= Y0 && ty[1] <= Y1;
    const bool own = cin0 && rin0;  // the pixel's first tap is in this block
    // a tap of non-zero weight sits one column and/or one row past the first
    // (a clamped tap repeats the first with weight 0)
    const bool hit[4] = {own && w[0] != 0.0f, cin1 && rin0 && w[1] != 0.0f, cin0 && rin1 && w[2] != 0.0f,
                         cin1 && rin1 && w[3] != 0.0f};
    if (!(own || hit[1] || hit[2] || hit[3])) continue;
    const int slot = (ty[0] - Y0) * tb + (tx[0] - X0);
    const int off[4] = {0, 1, tb, tb + 1};
    const float t = 1.0f - opac[o];
    float dO = 0.0f;
    for (int ch = 0; ch < 3; ++ch) {
      const float gc = g[ch * HW + o];
      if (own) {
        const float* cf = cube + (face * 3 + ch) * F;
        const float sv = ((w[0] * cf[idx[0]] + w[1] * cf[idx[1]]) + w[2] * cf[idx[2]]) + w[3] * cf[idx[3]];
        dO -= sv * gc;
      }
      const float tg = t * gc;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (!hit[q]) continue;
        if (fixed)
          atomicAdd(&s_acc[ch * kT + slot + off[q]], sky_fixed(w[q] * tg, k));
        else
          atomicAdd(&facc[ch * kT + slot + off[q]], w[q] * tg);
      }
    }
    if (own) dopac[o] = dO;
  }
  __syncthreads();
  // each texel of the block is this workgroup's alone: plain read-add-write
  for (int i = threadIdx.x; i < 3 * kT; i += kSkyGatherThreads) {
    const int ch = i / kT, rr = i % kT;
    if (rr >= tb * tb) continue;
    float* p = dcube + (f * 3 + ch) * F + static_cast<int64_t>(Y0 + rr / tb) * Rn + (X0 + rr % tb);
    if (fixed) {
      const long long a = static_cast<long long>(s_acc[i]);
      if (a != 0) *p = static_cast<float>(static_cast<double>(*p) + ldexp(static_cast<double>(a), -k));
    } else {
      const float v = facc[i];
      if (v != 0.0f) *p += v;  // also every slot past the face's last row or column
    }
  }
}

// The gather's set-up, or false for the scatter: a rotation that is not
// orthonormal to 1e-3 (the clip plane's bound assumes |M q| >= about |q|).
static bool sky_gather_setup(const pvg_camera* cam, int Rn, SkyGather& G) {
  double A[3][3];  // R^T
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[i][j] = cam->R[3 * j + i];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double d = 0.0;
      for (int k = 0; k < 3; ++k) d += A[i][k] * A[j][k];
      if (!(std::fabs(d - (i == j ? 1.0 : 0.0)) <= 1e-3)) return false;
    }
  const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                     A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                     A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  double A_inv[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {  // inverse = adjugate / det: entry (i, j) is cofactor (j, i) / det
      const int j1 = (j + 1) % 3, j2 = (j + 2) % 3, i1 = (i + 1) % 3, i2 = (i + 2) % 3;
      A_inv[i][j] = (A[j1][i1] * A[j2][i2] - A[j1][i2] * A[j2][i1]) / det;
      G.M[3 * i + j] = static_cast<float>(A_inv[i][j]);
    }
  // A face point q with c = M q, |c| >= 0.998 and c.z < delta has max(|c.x|, |c.y|)
  // >= 0.61, so it projects more than fx 0.61 / delta > D pixels from the
  // principal point, beyond the widened image.
  const double m = kSkyJitter + 4.0;
  const double D = std::max(std::max(cam->cx + m, cam->width + m - cam->cx),
                            std::max(cam->cy + m, cam->height + m - cam->cy));
  G.delta = static_cast<float>(std::min(0.5, 0.5 * std::min(cam->fx, cam->fy) / D));
  // the rays of the widened image lie within `cone` of the optical axis
  double cone = 0.0;
  for (int k = 0; k < 4; ++k) {
    const double X = (k & 1) ? cam->width + m : -m, Y = (k & 2) ? cam->height + m : -m;
    cone = std::max(cone, std::atan(std::hypot((X - cam->cx) / cam->fx, (Y - cam->cy) / cam->fy)));
  }
  cone += 0.02;  // far above the rounding of the test below
  const double cc = std::cos(cone), sc = std::sin(cone);
  // Blocks of about 48 pixels a side: 16 texels up to three pixels per texel,
  // fewer texels for coarser maps (a 16-texel block of a 128 map seen at
  // fx = 1500 spans 370 pixels, and its workgroup alone walked 0.14M of them)
  const double px_per_texel = 2.0 * std::max(cam->fx, cam->fy) / Rn;
  G.tb = kSkyTB;
  while (G.tb > 1 && G.tb * px_per_texel > 48.0) G.tb >>= 1;
  G.nb = (Rn + G.tb - 1) / G.tb;
  G.sbs = std::max(8, (G.nb + 7) / 8);
  G.nsb = (G.nb + G.sbs - 1) / G.sbs;
  G.count = 0;
  // A superblock's footprint (its texels widened by one) can meet a ray of
  // the view only if the angle between the optical axis and the footprint's
  // centre, less the footprint's angular radius (largest at a corner: the
  // footprint is a convex quad inside a hemisphere), is within `cone`:
  // cos(angle to axis) >= cos(cone + radius).
  const double span = static_cast<double>(G.sbs) * G.tb;
  for (int f = 0; f < 6; ++f)
    for (int r = 0; r < G.nsb; ++r)
      for (int q = 0; q < G.nsb; ++q) {
        const double x0 = q * span - 1.0, x1 = std::min((q + 1) * span, static_cast<double>(Rn)) + 1.0;
        const double y0 = r * span - 1.0, y1 = std::min((r + 1) * span, static_cast<double>(Rn)) + 1.0;
        const double ss[5] = {(x0 + x1) / Rn - 1.0, 2.0 * x0 / Rn - 1.0, 2.0 * x1 / Rn - 1.0,
                              2.0 * x1 / Rn - 1.0, 2.0 * x0 / Rn - 1.0};
        const double ts[5] = {(y0 + y1) / Rn - 1.0, 2.0 * y0 / Rn - 1.0, 2.0 * y0 / Rn - 1.0,
                              2.0 * y1 / Rn - 1.0, 2.0 * y1 / Rn - 1.0};
        double u[5][3];
        for (int k = 0; k < 5; ++k) {
          const double sv = ss[k], tv = ts[k];
          double qd[3];
          switch (f) {
            case 0: qd[0] = 1.0; qd[1] = -tv; qd[2] = -sv; break;
            case 1: qd[0] = -1.0; qd[1] = -tv; qd[2] = sv; break;
            case 2: qd[0] = sv; qd[1] = 1.0; qd[2] = tv; break;
            case 3: qd[0] = sv; qd[1] = -1.0; qd[2] = -tv; break;
            case 4: qd[0] = sv; qd[1] = -tv; qd[2] = 1.0; break;
            default: qd[0] = -sv; qd[1] = -tv; qd[2] = -1.0; break;
          }
          double n2 = 0.0;
          for (int i = 0; i < 3; ++i) {
            u[k][i] = A_inv[i][0] * qd[0] + A_inv[i][1] * qd[1] + A_inv[i][2] * qd[2];
            n2 += u[k][i] * u[k][i];
          }
          for (int i = 0; i < 3; ++i) u[k][i] /= std::sqrt(n2);
        }
        double cb = 1.0;  // cos of the angular radius
        for (int k = 1; k < 5; ++k) cb = std::min(cb, u[0][0] * u[k][0] + u[0][1] * u[k][1] + u[0][2] * u[k][2]);
        const double sb = std::sqrt(std::max(0.0, 1.0 - cb * cb));
        const bool reach = cb < -cc || u[0][2] >= cc * cb - sc * sb;  // cone + radius beyond pi, or within
        if (reach) G.sb[G.count++] = static_cast<uint16_t>((f * G.nsb + r) * G.nsb + q);
      }
  // every ray lands in some superblock, so at least one passes; the scatter
  // takes over should rounding ever say otherwise
  if (G.count == 0) return false;
  return true;
}

static SkyView sky_view(const pvg_camera* cam) {
  SkyView v;
  for (int k = 0; k < 9; ++k) v.R[k] = cam->R[k];
  v.fx = cam->fx; v.fy = cam->fy; v.cx = cam->cx; v.cy = cam->cy;
  v.W = cam->width; v.H = cam->height;
  return v;
}

hipError_t launch_sky(const pvg_camera* cam, const float* img, const float* opac, const float* cube, int Rn,
                      const float* jitter, float* out, hipStream_t s) {
  const int64_t HW = static_cast<int64_t>(cam->width) * cam->height;
  if (HW == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sky_fwd, dim3(static_cast<unsigned>((HW + 255) / 256)), dim3(256), 0, s, sky_view(cam), img,
                     opac, cube, Rn, jitter, out);
  return hipGetLastError();
}

hipError_t launch_sky_bwd(const pvg_camera* cam, const float* g, const float* opac, const float* cube, int Rn,
                          const float* jitter, float* dopac, float* dcube, bool deterministic, hipStream_t s) {
  const int64_t HW = static_cast<int64_t>(cam->width) * cam->height;
  if (HW == 0) return hipSuccess;
  SkyGather G;
  if (deterministic && sky_gather_setup(cam, Rn, G)) {
    const SkyView v = sky_view(cam);
    if (jitter)
      hipLaunchKernelGGL(k_sky_bwd_stray, dim3(static_cast<unsigned>((HW + 255) / 256)), dim3(256), 0, s, v, g, opac,
                         cube, Rn, jitter, dopac, dcube);
    const int64_t total = static_cast<int64_t>(G.count) * G.sbs * G.sbs;
    hipLaunchKernelGGL(k_sky_bwd_gather, dim3(static_cast<unsigned>(render_grid(total))), dim3(kSkyGatherThreads), 0, s, v, G, g,
                       opac, cube, Rn, jitter, dopac, dcube);
    return hipGetLastError();
  }
  const int GX = (cam->width + 15) / 16, GY = (cam->height + 15) / 16;
  hipLaunchKernelGGL(k_sky_bwd, dim3(static_cast<unsigned>(GX) * static_cast<unsigned>(GY)), dim3(256), 0, s,
                     sky_view(cam), g, opac, cube, Rn, jitter, dopac, dcube, GX);
  return hipGetLastError();
}

}  // namespace pvg
