// Device-side per-Gaussian mathematics of the PVG rasterizer (gfx950).
//
// The evaluation order of every floating-point expression of the
// per-Gaussian stage is fixed (left to right, as written) and the file is
// compiled without FMA contraction, so that the discrete structure (screen
// radius, tile rectangle, depth key) is reproducible bit for bit by any other
// IEEE FP32 implementation that follows the same order.  The sine and
// exponential of the temporal model are correctly rounded FP32 values:
// evaluated in FP64 and rounded once.
#pragma once

#include "pvg_internal.hpp"

namespace pvg {

__device__ __forceinline__ float sin_cr(float x) { return static_cast<float>(sin(static_cast<double>(x))); }
__device__ __forceinline__ float exp_cr(float x) { return static_cast<float>(exp(static_cast<double>(x))); }

enum : uint32_t {
  kGuardXLo = 1u << 0, kGuardXHi = 1u << 1, kGuardYLo = 1u << 2, kGuardYHi = 1u << 3,
  kClampR = 1u << 4, kClampG = 1u << 5, kClampB = 1u << 6,
};

// Real spherical harmonics of degree <= 3 (no Condon-Shortley phase) at the
// unit vector (x, y, z), index l*l + l + m, as Cartesian polynomials.
namespace shc {
constexpr float c0 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
constexpr float c1 = 0.48860251190291992f;   // sqrt(3 / (4 pi))
constexpr float c2a = 1.09254843059207907f;  // sqrt(15 / pi) / 2
constexpr float c2b = 0.31539156525252001f;  // sqrt(5 / pi) / 4
constexpr float c2c = 0.54627421529603954f;  // sqrt(15 / pi) / 4
constexpr float c3a = 0.59004358992664352f;  // sqrt(35 / (2 pi)) / 4
constexpr float c3b = 2.89061144264055405f;  // sqrt(105 / pi) / 2
constexpr float c3c = 0.45704579946446573f;  // sqrt(21 / (2 pi)) / 4
constexpr float c3d = 0.37317633259011540f;  // sqrt(7 / pi) / 4
constexpr float c3e = 1.44530572132027702f;  // sqrt(105 / pi) / 4
}  // namespace shc

__device__ __forceinline__ void sh_eval_basis(int degree, float x, float y, float z, float Y[16]) {
  Y[0] = shc::c0;
  if (degree < 1) return;
  Y[1] = shc::c1 * y;
  Y[2] = shc::c1 * z;
  Y[3] = shc::c1 * x;
  if (degree < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = shc::c2a * (x * y);
  Y[5] = shc::c2a * (y * z);
  Y[6] = shc::c2b * ((2.0f * zz - xx) - yy);
  Y[7] = shc::c2a * (x * z);
  Y[8] = shc::c2c * (xx - yy);
  if (degree < 3) return;
  Y[9] = shc::c3a * (y * (3.0f * xx - yy));
  Y[10] = shc::c3b * (x * y * z);
  Y[11] = shc::c3c * (y * ((4.0f * zz - xx) - yy));
  Y[12] = shc::c3d * (z * ((2.0f * zz - 3.0f * xx) - 3.0f * yy));
  Y[13] = shc::c3c * (x * ((4.0f * zz - xx) - yy));
  Y[14] = shc::c3e * (z * (xx - yy));
  Y[15] = shc::c3a * (x * (xx - 3.0f * yy));
}

// Gradient of sum_k w[k] Y_k(x, y, z) with respect to (x, y, z) of the
// polynomials above (only its component tangent to the sphere is used).
__device__ __forceinline__ void sh_grad_basis(int degree, float x, float y, float z, const float w[16],
                                              float g[3]) {
  g[0] = 0.0f; g[1] = 0.0f; g[2] = 0.0f;
  if (degree < 1) return;
  g[1] += shc::c1 * w[1];
  g[2] += shc::c1 * w[2];
  g[0] += shc::c1 * w[3];
  if (degree < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  g[0] += shc::c2a * (y * w[4] + z * w[7]) + shc::c2b * (-2.0f * x) * w[6] + shc::c2c * (2.0f * x) * w[8];
  g[1] += shc::c2a * (x * w[4] + z * w[5]) + shc::c2b * (-2.0f * y) * w[6] + shc::c2c * (-2.0f * y) * w[8];
  g[2] += shc::c2a * (y * w[5] + x * w[7]) + shc::c2b * (4.0f * z) * w[6];
  if (degree < 3) return;
  // Y9 = a y (3xx - yy)
  g[0] += shc::c3a * (6.0f * x * y) * w[9];
  g[1] += shc::c3a * (3.0f * xx - 3.0f * yy) * w[9];
  // Y10 = b x y z
  g[0] += shc::c3b * (y * z) * w[10];
  g[1] += shc::c3b * (x * z) * w[10];
  g[2] += shc::c3b * (x * y) * w[10];
  // Y11 = c y (4zz - xx - yy)
  g[0] += shc::c3c * (-2.0f * x * y) * w[11];
  g[1] += shc::c3c * ((4.0f * zz - xx) - 3.0f * yy) * w[11];
  g[2] += shc::c3c * (8.0f * y * z) * w[11];
  // Y12 = d z (2zz - 3xx - 3yy)
  g[0] += shc::c3d * (-6.0f * x * z) * w[12];
  g[1] += shc::c3d * (-6.0f * y * z) * w[12];
  g[2] += shc::c3d * ((6.0f * zz - 3.0f * xx) - 3.0f * yy) * w[12];
  // Y13 = c x (4zz - xx - yy)
  g[0] += shc::c3c * ((4.0f * zz - 3.0f * xx) - yy) * w[13];
  g[1] += shc::c3c * (-2.0f * x * y) * w[13];
  g[2] += shc::c3c * (8.0f * x * z) * w[13];
  // Y14 = e z (xx - yy)
  g[0] += shc::c3e * (2.0f * x * z) * w[14];
  g[1] += shc::c3e * (-2.0f * y * z) * w[14];
  g[2] += shc::c3e * (xx - yy) * w[14];
  // Y15 = a x (xx - 3yy)
  g[0] += shc::c3a * (3.0f * xx - 3.0f * yy) * w[15];
  g[1] += shc::c3a * (-6.0f * x * y) * w[15];
}

// Forward state of one Gaussian in one view.
struct Proj {
  float mr[3];      // translated mean (Eq. (12)) or mu~(t) (Eq. (6))
  float op;         // o~(t) (Eq. (7))
  float p[3];       // camera-space point
  float tx, ty, J00, J02, J11, J12, T2[6];
  float ca, cb, cc, det;  // dilated 2D covariance
  float A, B, C, x, y;
  int32_t radius;
  int32_t rect[4];
  uint32_t flags;
  float dir[3], ulen;
  float rgb[3];
};

__device__ __forceinline__ int32_t clamp_tile(float v, int32_t hi) {
  const float f = floorf(v);
  if (f < 0.0f) return 0;
  if (f > static_cast<float>(hi)) return hi;
  return static_cast<int32_t>(f);
}

// Tile rectangle [x0, x1) x [y0, y1) of a splat at (x, y) with radius r.
__device__ __forceinline__ void tile_rect(float x, float y, int32_t r, int32_t GX, int32_t GY, int32_t rect[4]) {
  const float rr = static_cast<float>(r);
  rect[0] = clamp_tile((x - rr) / 16.0f, GX);
  rect[1] = clamp_tile((y - rr) / 16.0f, GY);
  rect[2] = clamp_tile(((x + rr) + 15.0f) / 16.0f, GX);
  rect[3] = clamp_tile(((y + rr) + 15.0f) / 16.0f, GY);
}

// Can a Gaussian reach alpha >= 1/255 at any pixel of the tile?  alpha =
// min(0.99, o~ G) >= 1/255 needs power >= ln(1 / (255 o~)); power = -q/2 with
// q the conic's quadratic form, whose minimum over the tile's sample
// rectangle is exact (interior: 0; else the best of the four edges).  The test
// keeps a wide margin, and never drops a Gaussian with non-finite values, so a
// dropped Gaussian is one every pixel of the tile would skip.
__device__ __forceinline__ bool tile_reachable(float gx, float gy, float A, float B, float C, float op, float X0,
                                               float X1, float Y0, float Y1) {
  if (!(isfinite(gx) && isfinite(gy) && isfinite(A) && isfinite(B) && isfinite(C) && isfinite(op))) return true;
  if (op < kAlphaMin) return false;
  if (!(A > 0.0f && C > 0.0f)) return true;
  const float dxl = gx - X1, dxh = gx - X0, dyl = gy - Y1, dyh = gy - Y0;
  float qmin;
  if (dxl <= 0.0f && dxh >= 0.0f && dyl <= 0.0f && dyh >= 0.0f) {
    qmin = 0.0f;
  } else {
    auto q = [&](float dx, float dy) { return A * dx * dx + 2.0f * B * dx * dy + C * dy * dy; };
    auto best_dy = [&](float dx) { return fminf(fmaxf(-B * dx / C, dyl), dyh); };
    auto best_dx = [&](float dy) { return fminf(fmaxf(-B * dy / A, dxl), dxh); };
    qmin = fminf(fminf(q(dxl, best_dy(dxl)), q(dxh, best_dy(dxh))), fminf(q(best_dx(dyl), dyl), q(best_dx(dyh), dyh)));
  }
  const float need = -logf(kAlphaMin / op);  // -power must stay below this
  return !(0.5f * qmin * 0.999f > need + 0.01f);
}

// Reachable tiles as one column interval per tile row.  A pixel can take
// alpha >= 1/255 only where o~ exp(-q/2) >= 1/255, q = d^T Q d the conic's
// quadratic form at d = mean - pixel, i.e. inside the ellipse q <= 2 ln(255 o~).
// The ellipse is widened for rounding: the bound gets a 0.1% and an additive
// margin, and Q is shrunk by k I with k far above the FP32 error of
// evaluating q (a few ulp of |A| dx^2 + 2 |B dx dy| + |C| dy^2); a conic too
// close to singular for that keeps its whole rectangle.  Within tile row ty
// the ellipse's x-extent over the row's sample band is exact: each horizontal
// slice is an interval, whose right end is a concave function of dy
// (maximal at the ellipse's rightmost point) and whose left end is convex.
struct ReachRows {
  float gx, gy;
  float ex, ey;    // largest |dx|, |dy| on the ellipse
  float dyr;       // dy of the rightmost point (the leftmost is at -dyr)
  float bA;        // B / A: a horizontal slice at dy is centred at -bA dy
  float c1, c2;    // its half-width is sqrt(c1 - c2 dy^2)
  float slack;     // pixels added on both sides for rounding
  int mode;        // 0: ellipse, 1: every tile of the rectangle, 2: no tile
};

__device__ __forceinline__ ReachRows reach_rows_init(float gx, float gy, float A, float B, float C, float op) {
  ReachRows r;
  r.gx = gx; r.gy = gy;
  r.ex = r.ey = r.dyr = r.bA = r.c1 = r.c2 = r.slack = 0.0f;
  r.mode = 0;
  if (!(isfinite(gx) && isfinite(gy) && isfinite(A) && isfinite(B) && isfinite(C) && isfinite(op))) {
    r.mode = 1;
    return r;
  }
  if (op < kAlphaMin) {  // alpha <= o~ < 1/255 everywhere
    r.mode = 2;
    return r;
  }
  const float k = 1e-5f * (fabsf(A) + fabsf(C) + 2.0f * fabsf(B));
  const float a = A - k, c = C - k;
  const float det = a * c - B * B;
  if (!(a > 0.0f && c > 0.0f && det > 0.0f)) {
    r.mode = 1;
    return r;
  }
  const float need = -logf(kAlphaMin / op);  // alpha >= 1/255 needs q / 2 <= need
  const float lim = 2.0f * (need + 0.01f) * 1.001f;
  r.ex = sqrtf(lim * c / det);
  r.ey = sqrtf(lim * a / det);
  r.dyr = -B * r.ex / c;
  r.bA = B / a;
  r.c1 = lim / a;
  r.c2 = det / (a * a);
  r.slack = 0.05f + 2e-5f * (r.ex + fabsf(gx));
  if (!(isfinite(r.ex) && isfinite(r.ey) && isfinite(r.c1) && isfinite(r.c2))) r.mode = 1;
  return r;
}

// Columns [lo, hi] of tile row ty, within the rectangle columns [x0, x1), that
// the ellipse reaches (lo > hi: none).  H is the image height.
__device__ __forceinline__ void reach_row(const ReachRows& r, int ty, int H, int x0, int x1, int& lo, int& hi) {
  lo = x0;
  hi = x1 - 1;
  if (r.mode == 1) return;
  hi = x0 - 1;
  if (r.mode == 2) return;
  const float Y0 = static_cast<float>(ty * kTile);
  const float Y1 = static_cast<float>(min(H, (ty + 1) * kTile) - 1);
  const float a = fmaxf(r.gy - Y1, -r.ey), b = fminf(r.gy - Y0, r.ey);  // dy band on the ellipse
  if (!(a <= b)) return;
  const float ha = __builtin_amdgcn_sqrtf(fmaxf(0.0f, r.c1 - r.c2 * (a * a)));
  const float hb = __builtin_amdgcn_sqrtf(fmaxf(0.0f, r.c1 - r.c2 * (b * b)));
  const float ca = -r.bA * a, cb = -r.bA * b;  // slice centres
  const float dmax = (r.dyr >= a && r.dyr <= b) ? r.ex : fmaxf(ca + ha, cb + hb);
  const float dmin = (-r.dyr >= a && -r.dyr <= b) ? -r.ex : fminf(ca - ha, cb - hb);
  const float xl = (r.gx - dmax) - r.slack, xh = (r.gx - dmin) + r.slack;  // sample columns reached
  // tiles whose sample columns [16 tx, 16 tx + 15] meet [xl, xh]
  float tl = ceilf((xl - 15.0f) * 0.0625f), th = floorf(xh * 0.0625f);
  if (!(tl >= static_cast<float>(x0))) tl = static_cast<float>(x0);
  if (!(th <= static_cast<float>(x1 - 1))) th = static_cast<float>(x1 - 1);
  if (tl > th) return;
  lo = static_cast<int>(tl);
  hi = static_cast<int>(th);
}

// Sample rectangle [X0, X1] x [Y0, Y1] of tile (tx, ty) in a W x H image.
__device__ __forceinline__ void tile_bounds(int tx, int ty, int W, int H, float& X0, float& X1, float& Y0, float& Y1) {
  X0 = static_cast<float>(tx * kTile);
  Y0 = static_cast<float>(ty * kTile);
  X1 = static_cast<float>(min(W, (tx + 1) * kTile) - 1);
  Y1 = static_cast<float>(min(H, (ty + 1) * kTile) - 1);
}

// The part of the per-Gaussian stage that depends on the time t but not on
// the camera: the vibrating mean mu~(t) (Eq. (6)) and the decayed opacity
// o~(t) (Eq. (7)), with the velocity and the flow factor exp(-beta / (2 l))
// of Eq. (10) (evaluated on first use).  Views of one training step share t,
// so a kernel that handles several views of a Gaussian forms this once.
// SH evaluation with the coefficient loads batched: K is a template
// parameter, so no run-time bound separates the loads (one made each row of
// three a separate round trip to memory).  They go kShGroup rows at a time
// (a smaller group holds fewer registers; all 16 rows at once measured
// fastest for the adjoint at degree 3).
constexpr int kShGroup = 16;

// sum_k sh_k,ch Y_k for the three channels, k ascending.
template <int K>
__device__ __forceinline__ void sh_colour_k(const Scene& s, int64_t i, const float Y[16], float out[3]) {
  const float* __restrict__ sh = s.sh;
  float acc[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += kShGroup) {
    float c[3 * kShGroup];
#pragma unroll
    for (int j = 0; j < 3 * kShGroup; ++j)
      if (k0 * 3 + j < 3 * K) c[j] = sh[(k0 * 3 + j) * s.n + i];
#pragma unroll
    for (int k = 0; k < kShGroup; ++k)
      if (k0 + k < K)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) acc[ch] += c[3 * k + ch] * Y[k0 + k];
  }
  for (int ch = 0; ch < 3; ++ch) out[ch] = acc[ch];
}
__device__ __forceinline__ void sh_colour(const Scene& s, int64_t i, const float Y[16], float out[3]) {
  switch (s.degree) {
    case 0: sh_colour_k<1>(s, i, Y, out); break;
    case 1: sh_colour_k<4>(s, i, Y, out); break;
    case 2: sh_colour_k<9>(s, i, Y, out); break;
    default: sh_colour_k<16>(s, i, Y, out); break;
  }
}

// w_k = sum_ch sh_k,ch d_ch (ch ascending) for k < K, 0 above.
template <int K>
__device__ __forceinline__ void sh_weights_k(const Scene& s, int64_t i, const float d[3], float w[16]) {
  const float* __restrict__ sh = s.sh;
#pragma unroll
  for (int k = 0; k < 16; ++k) w[k] = 0.0f;
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += kShGroup) {
    float c[3 * kShGroup];
#pragma unroll
    for (int j = 0; j < 3 * kShGroup; ++j)
      if (k0 * 3 + j < 3 * K) c[j] = sh[(k0 * 3 + j) * s.n + i];
#pragma unroll
    for (int k = 0; k < kShGroup; ++k)
      if (k0 + k < K) w[k0 + k] = (c[3 * k] * d[0] + c[3 * k + 1] * d[1]) + c[3 * k + 2] * d[2];
  }
}
__device__ __forceinline__ void sh_weights(const Scene& s, int64_t i, const float d[3], float w[16]) {
  switch (s.degree) {
    case 0: sh_weights_k<1>(s, i, d, w); break;
    case 1: sh_weights_k<4>(s, i, d, w); break;
    case 2: sh_weights_k<9>(s, i, d, w); break;
    default: sh_weights_k<16>(s, i, d, w); break;
  }
}

struct GaussTime {
  float t;        // the time it was formed for
  float mt[3];    // mu~(t)
  float vel[3];
  float op;       // o~(t)
  float beta, l;
  float ev;       // exp(-beta / (2 l)), or a negative value before its first use
};

__device__ __forceinline__ void gauss_time(const Scene& s, int64_t i, float t, GaussTime& G) {
  const int64_t n = s.n;
  const float l = s.period[i], tau = s.tau[i], beta = s.beta[i], o = s.opacity[i];
  const float d = t - tau;
  const float phi = (kTwoPi * d) / l;
  const float k = (l / kTwoPi) * sin_cr(phi);
  const float q = d / beta;
  G.t = t;
  G.op = o * exp_cr(-0.5f * (q * q));
  for (int c = 0; c < 3; ++c) {
    G.vel[c] = s.vel[c * n + i];
    G.mt[c] = s.mu[c * n + i] + k * G.vel[c];
  }
  G.beta = beta;
  G.l = l;
  G.ev = -1.0f;
}

// Temporal state of one view (Eqs. (6), (7)) with its flow translation
// (Eqs. (10), (12)): mr = mu~(t) + v_bar dt.
__device__ __forceinline__ void view_mean(const View& v, GaussTime& G, float mr[3]) {
  for (int c = 0; c < 3; ++c) mr[c] = G.mt[c];
  if (v.dt != 0.0f) {
    float ev = 1.0f;
    if (v.mode == 0) {
      if (G.ev < 0.0f) G.ev = exp_cr(-0.5f * (G.beta / G.l));
      ev = G.ev;
    }
    for (int c = 0; c < 3; ++c) mr[c] = mr[c] + (G.vel[c] * ev) * v.dt;
  }
}

// The camera-independent 3D covariance Sigma = R(q) S S^T R(q)^T of
// Gaussian i, with the intermediate values the adjoint reuses.
struct GaussCov {
  float qn[4], qnorm, Rq[9], sc[3], M[9];
  float Sig[9];  // row-major, symmetric
  bool ready;    // formed (a view that culls the Gaussian at the near plane does not need it)
};

__device__ __forceinline__ void gauss_cov(const Scene& s, int64_t i, GaussCov& G) {
  const int64_t n = s.n;
  G.ready = true;
  float q[4];
  for (int c = 0; c < 4; ++c) q[c] = s.rot[c * n + i];
  const float n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
  G.qnorm = sqrtf(n2);
  for (int c = 0; c < 4; ++c) G.qn[c] = q[c] / G.qnorm;
  {
    const float w = G.qn[0], x = G.qn[1], y = G.qn[2], z = G.qn[3];
    G.Rq[0] = 1.0f - 2.0f * (y * y + z * z);
    G.Rq[1] = 2.0f * (x * y - w * z);
    G.Rq[2] = 2.0f * (x * z + w * y);
    G.Rq[3] = 2.0f * (x * y + w * z);
    G.Rq[4] = 1.0f - 2.0f * (x * x + z * z);
    G.Rq[5] = 2.0f * (y * z - w * x);
    G.Rq[6] = 2.0f * (x * z - w * y);
    G.Rq[7] = 2.0f * (y * z + w * x);
    G.Rq[8] = 1.0f - 2.0f * (x * x + y * y);
  }
  for (int c = 0; c < 3; ++c) G.sc[c] = s.scale[c * n + i];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) G.M[3 * r + c] = G.Rq[3 * r + c] * G.sc[c];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      G.Sig[3 * r + c] = (G.M[3 * r] * G.M[3 * c] + G.M[3 * r + 1] * G.M[3 * c + 1]) + G.M[3 * r + 2] * G.M[3 * c + 2];
}

// Unit direction from the camera centre -R^T T to the (translated) mean.
__device__ __forceinline__ void view_direction(const View& v, Proj& P) {
  const float* W = v.R;
  float cp[3], u[3];
  for (int c = 0; c < 3; ++c) cp[c] = -((W[c] * v.T[0] + W[3 + c] * v.T[1]) + W[6 + c] * v.T[2]);
  for (int c = 0; c < 3; ++c) u[c] = P.mr[c] - cp[c];
  P.ulen = sqrtf((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
  for (int c = 0; c < 3; ++c) P.dir[c] = u[c] / P.ulen;
}

// The camera-dependent rest of the per-Gaussian stage, from the time state
// and the covariance: view transform and near cull, EWA projection, conic,
// radius and tile rectangle; returns false for an invisible Gaussian.  With
// `color` it also evaluates the clamped SH colour.  P's covariance fields are
// not filled (the caller holds them in C).
__device__ __forceinline__ bool project_view(const View& v, int64_t i, GaussTime& G, GaussCov& C, Proj& P,
                                             bool color) {
  const Scene& s = v.s;
  const int64_t n = s.n;
  view_mean(v, G, P.mr);
  P.op = G.op;
  const float* W = v.R;
  for (int r = 0; r < 3; ++r)
    P.p[r] = ((W[3 * r] * P.mr[0] + W[3 * r + 1] * P.mr[1]) + W[3 * r + 2] * P.mr[2]) + v.T[r];
  P.radius = 0;
  P.flags = 0;
  if (!(P.p[2] > v.znear)) return false;
  if (!C.ready) gauss_cov(s, i, C);
  const float* Sig = C.Sig;

  // EWA (Eq. (2)) with the Jacobian at the guarded point
  const float px = P.p[0], py = P.p[1], pz = P.p[2];
  const float limx = kGuard * ((0.5f * static_cast<float>(v.W)) / v.fx);
  const float limy = kGuard * ((0.5f * static_cast<float>(v.H)) / v.fy);
  const float txz = px / pz, tyz = py / pz;
  uint32_t fl = 0;
  if (txz < -limx) fl |= kGuardXLo;
  if (txz > limx) fl |= kGuardXHi;
  if (tyz < -limy) fl |= kGuardYLo;
  if (tyz > limy) fl |= kGuardYHi;
  P.tx = (fl & kGuardXLo) ? (-limx) * pz : (fl & kGuardXHi) ? limx * pz : px;
  P.ty = (fl & kGuardYLo) ? (-limy) * pz : (fl & kGuardYHi) ? limy * pz : py;
  P.J00 = v.fx / pz;
  P.J02 = -(v.fx * P.tx) / (pz * pz);
  P.J11 = v.fy / pz;
  P.J12 = -(v.fy * P.ty) / (pz * pz);
  for (int c = 0; c < 3; ++c) {
    P.T2[c] = P.J00 * W[c] + P.J02 * W[6 + c];
    P.T2[3 + c] = P.J11 * W[3 + c] + P.J12 * W[6 + c];
  }
  float U[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c)
      U[3 * r + c] = (P.T2[3 * r] * Sig[c] + P.T2[3 * r + 1] * Sig[3 + c]) + P.T2[3 * r + 2] * Sig[6 + c];
  const float s00 = (U[0] * P.T2[0] + U[1] * P.T2[1]) + U[2] * P.T2[2];
  const float s01 = (U[0] * P.T2[3] + U[1] * P.T2[4]) + U[2] * P.T2[5];
  const float s11 = (U[3] * P.T2[3] + U[4] * P.T2[4]) + U[5] * P.T2[5];
  P.ca = s00 + kDilation;
  P.cb = s01;
  P.cc = s11 + kDilation;
  P.det = P.ca * P.cc - P.cb * P.cb;
  P.flags = fl;
  if (!(P.det > 0.0f)) return false;
  P.A = P.cc / P.det;
  P.B = -P.cb / P.det;
  P.C = P.ca / P.det;
  P.x = (v.fx * txz + v.cx) - 0.5f;
  P.y = (v.fy * tyz + v.cy) - 0.5f;
  const float mid = 0.5f * (P.ca + P.cc);
  const float lam = mid + sqrtf(fmaxf(kLambdaFloor, mid * mid - P.det));
  const int32_t rad = static_cast<int32_t>(ceilf(3.0f * sqrtf(lam)));
  tile_rect(P.x, P.y, rad, v.GX, v.GY, P.rect);
  if ((P.rect[2] - P.rect[0]) * (P.rect[3] - P.rect[1]) == 0) return false;
  P.radius = rad;

  if (color) {
    view_direction(v, P);
    float Y[16];
    sh_eval_basis(s.degree, P.dir[0], P.dir[1], P.dir[2], Y);
    float sum[3];
    sh_colour(s, i, Y, sum);
    for (int ch = 0; ch < 3; ++ch) {
      const float raw = sum[ch] + 0.5f;
      if (raw < 0.0f) {  // clamped: stored as -0, which composites like +0 and marks the clamp
        P.flags |= (kClampR << ch);
        P.rgb[ch] = -0.0f;
      } else {
        P.rgb[ch] = raw;
      }
    }
  }
  return true;
}

// The whole per-Gaussian stage of Gaussian i in one view.
__device__ __forceinline__ bool project(const View& v, int64_t i, Proj& P, bool color) {
  GaussTime G;
  GaussCov C;
  C.ready = false;
  gauss_time(v.s, i, v.t, G);
  return project_view(v, i, G, C, P, color);
}

}  // namespace pvg
