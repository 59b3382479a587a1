// Sky composite of the sky refinement (Sec. 3.4): C_f = C + (1 - O) f_sky(d),
// where f_sky is a learnable cube map looked up in the pixel's world-frame
// viewing direction, optionally jittered inside the pixel.  One thread per
// pixel; the adjoint writes dL/dO and adds each pixel's bilinear weights
// times (1 - O) dL/dC_f into the cube map's gradient.  Neighbouring pixels
// share texels (a high-resolution image has several pixels per texel), so the
// adjoint runs on 16 x 16 pixel tiles: each tile sums its contributions to
// the texel box it covers on its first pixel's face in LDS and adds the box
// to global memory once per texel and channel; pixels on another face, or a
// box beyond kSkyBox texels (a tile across a face edge or a coarse map seen
// at a grazing angle), add to global memory directly.
//
// Conventions: d_cam = ((px + 1/2 + jx - cx) / fx, (py + 1/2 + jy - cy) / fy,
// 1), d = R^T d_cam; faces +X, -X, +Y, -Y, +Z, -Z (0..5) by the largest |d_i|
// (ties to the lower axis); face coordinates as in OpenGL cube maps; texel
// (u R - 1/2, v R - 1/2), bilinear inside the face with the coordinates
// clamped to [0, R - 1]; cube [6][3][R][R].  The geometry is FP32 without
// contraction, so the face and texel decisions are the oracle's.
#include <climits>

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

constexpr int kSkyBox = 1024;  // texels of a tile's LDS box (3 channels: 12 KiB)

// One workgroup per 16 x 16 pixel tile (GX tiles per image row).
__global__ void __launch_bounds__(256) k_sky_bwd(SkyView c, const float* __restrict__ g,
                                                 const float* __restrict__ opac, const float* __restrict__ cube,
                                                 int Rn, const float* __restrict__ jitter, float* dopac, float* dcube,
                                                 int GX) {
  __shared__ float s_acc[3 * kSkyBox];
  __shared__ int s_box[5];  // the tile's face, then min x, min y, max x, max y of its texels there
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
  }
  __syncthreads();
  const int f0 = s_box[0];
  const bool mine = in && face == f0;
  if (mine) {  // the taps span [tx[0], tx[1]] x [ty[0], ty[1]]
    atomicMin(&s_box[1], tx[0]);
    atomicMin(&s_box[2], ty[0]);
    atomicMax(&s_box[3], tx[1]);
    atomicMax(&s_box[4], ty[1]);
  }
  __syncthreads();
  const int bx = s_box[1], by = s_box[2];
  const int bw = s_box[3] - bx + 1, bh = s_box[4] - by + 1;  // >= 1: thread 0 is in the box
  const int area = bw * bh;
  const bool lds = area <= kSkyBox;  // uniform over the workgroup
  if (lds) {
    for (int i = threadIdx.x; i < 3 * area; i += 256) s_acc[i] = 0.0f;
    __syncthreads();
  }
  if (in) {
    for (int ch = 0; ch < 3; ++ch)
      for (int k = 0; k < 4; ++k) {
        if (w[k] == 0.0f) continue;
        const float val = w[k] * tg[ch];
        if (lds && mine)
          atomicAdd(&s_acc[ch * area + (ty[k >> 1] - by) * bw + (tx[k & 1] - bx)], val);
        else
          atomicAdd(&dcube[(face * 3 + ch) * F + idx[k]], val);
      }
  }
  if (lds) {
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * area; i += 256) {
      const float val = s_acc[i];
      if (val == 0.0f) continue;
      const int ch = i / area, r = i - ch * area;
      const int yy = by + r / bw, xx = bx + r % bw;
      atomicAdd(&dcube[(f0 * 3 + ch) * F + static_cast<int64_t>(yy) * Rn + xx], val);
    }
  }
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
                          const float* jitter, float* dopac, float* dcube, hipStream_t s) {
  const int64_t HW = static_cast<int64_t>(cam->width) * cam->height;
  if (HW == 0) return hipSuccess;
  const int GX = (cam->width + 15) / 16, GY = (cam->height + 15) / 16;
  hipLaunchKernelGGL(k_sky_bwd, dim3(static_cast<unsigned>(GX) * static_cast<unsigned>(GY)), dim3(256), 0, s,
                     sky_view(cam), g, opac, cube, Rn, jitter, dopac, dcube, GX);
  return hipGetLastError();
}

}  // namespace pvg
