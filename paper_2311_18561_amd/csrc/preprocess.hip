// Per-Gaussian stage (forward and adjoint) of the PVG rasterizer on gfx950.
//
// Forward: one thread per (view, Gaussian): temporal state (Sec. 3.2,
// Eqs. (6)-(7)), flow translation (Sec. 3.4, Eqs. (10), (12)), EWA projection
// (Sec. 3.1, Eq. (2)), radius, tile rectangle and SH colour.  Parameter reads
// are structure-of-arrays, so a wave reads 256 contiguous bytes per field; the
// SH coefficients (up to 192 B per Gaussian) are only read for visible ones.
//
// Adjoint: one thread per Gaussian recomputes the forward state of each view
// (bit-identical, so every branch decision is the forward's), applies the
// chain rule from that view's screen-space gradient (2D mean, conic,
// opacity, colour) back to {mu, q, s, o, c, tau, beta, v} and l, sums over
// the views in registers and writes each gradient entry once.
#include "pvg_math.hpp"

namespace pvg {

// The projected record of Gaussian i of view v at slot gi of geom.
__device__ __forceinline__ void preprocess_one(const View& v, int64_t i, const Geom& geom, int64_t gi) {
  Proj P;
  const bool vis = project(v, i, P, true);
  geom.depth[gi] = P.p[2];
  if (vis) {
    reinterpret_cast<float2*>(geom.xy)[gi] = make_float2(P.x, P.y);
    reinterpret_cast<float4*>(geom.conic_op)[gi] = make_float4(P.A, P.B, P.C, P.op);
    geom.rgb[3 * gi] = P.rgb[0];
    geom.rgb[3 * gi + 1] = P.rgb[1];
    geom.rgb[3 * gi + 2] = P.rgb[2];
    geom.radius[gi] = P.radius;
    geom.tiles[gi] = static_cast<uint32_t>((P.rect[2] - P.rect[0]) * (P.rect[3] - P.rect[1]));
  } else {
    reinterpret_cast<float2*>(geom.xy)[gi] = make_float2(0.0f, 0.0f);
    reinterpret_cast<float4*>(geom.conic_op)[gi] = make_float4(0.0f, 0.0f, 0.0f, P.op);
    geom.rgb[3 * gi] = 0.0f;
    geom.rgb[3 * gi + 1] = 0.0f;
    geom.rgb[3 * gi + 2] = 0.0f;
    geom.radius[gi] = 0;
    geom.tiles[gi] = 0u;
  }
  if (geom.feat) {  // mean velocity v~ = v exp(-beta / (2 l)) and staticness rho = beta / l
    const Scene& sc = v.s;
    const float l = sc.period[i], beta = sc.beta[i];
    const float e = exp_cr(-0.5f * (beta / l));
    reinterpret_cast<float4*>(geom.feat)[gi] =
        make_float4(sc.vel[i] * e, sc.vel[sc.n + i] * e, sc.vel[2 * sc.n + i] * e, beta / l);
  }
}

__global__ void __launch_bounds__(256) k_preprocess(ViewSet vs, Geom geom, unsigned long long* dummy) {
  const int64_t gi = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (gi >= live_gauss(vs)) return;
  const View& v = view_at(vs, view_of_gauss(vs, gi));
  preprocess_one(v, gi - v.geom_off, geom, gi);
  (void)dummy;
}

// Several views of one set of Gaussians: block b projects the 256 Gaussians
// of chunk b / nv into view b % nv, so the views of a chunk are dispatched
// back to back and its parameters come from HBM once (the other views' reads
// hit the caches); each view's record is the single-view one.
__global__ void __launch_bounds__(256) k_preprocess_views(PreViews pk) {
  const int32_t k = static_cast<int32_t>(blockIdx.x % static_cast<uint32_t>(pk.nv));
  const int64_t i = static_cast<int64_t>(blockIdx.x / static_cast<uint32_t>(pk.nv)) * 256 + threadIdx.x;
  if (i >= pk.views[0].s.n) return;
  preprocess_one(pk.views[k], i, pk.geoms[k], i);
}

// Gradient entries of one Gaussian other than its SH coefficients.
struct GeoGrad {
  float mu[3], scale[3], rot[4], vel[3], op, l, tau, beta;
};

// One view's chain rule for everything but dL/dsh, added into acc.  g is the
// view's screen-space gradient of the Gaussian: d(mean x, y), d(conic A, B, C),
// d(opacity), d(rgb), d(depth); on return g[6..8] holds d(rgb) with clamped channels
// zeroed and g[9..11] the view direction, which is all dL/dsh needs.  rgb is
// the forward's colour of the Gaussian, where a clamped channel is -0.
__device__ __forceinline__ void adjoint_geometry(const View& v, int64_t i, const Proj& P, const float* rgb, float* g,
                                                 GeoGrad& acc, bool feature) {
  const Scene& s = v.s;
  const int64_t n = s.n;
  const int K = (s.degree + 1) * (s.degree + 1);
  const float dmx = g[0], dmy = g[1], dA = g[2], dB = g[3], dC = g[4], dop = g[5];
  // the blended channels' gradients (0 without them), read before slots 9.. are reused:
  // camera depth z, mean velocity v~ and staticness rho
  const float dz = g[9], dvb0 = g[10], dvb1 = g[11], dvb2 = g[12], drho = g[13];
  float dmr[3] = {0.0f, 0.0f, 0.0f};

  // colour: rgb = max(0, sum_k sh_k Y_k(dir) + 1/2), dir = u / |u|; its
  // dependence on the direction moves the mean.  A feature view's "colour"
  // is a per-Gaussian value: no clamp, no direction term, g[6..8] kept.
  if (!feature) {
    float draw[3];
    for (int ch = 0; ch < 3; ++ch) draw[ch] = signbit(rgb[ch]) ? 0.0f : g[6 + ch];
    float wk[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      float w = 0.0f;
      if (k < K)
        for (int ch = 0; ch < 3; ++ch) w += s.sh[(3 * k + ch) * n + i] * draw[ch];
      wk[k] = w;
      // read the coefficients four at a time rather than all 48 at once
      if ((k & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    float dd[3];
    sh_grad_basis(s.degree, P.dir[0], P.dir[1], P.dir[2], wk, dd);
    const float proj = P.dir[0] * dd[0] + P.dir[1] * dd[1] + P.dir[2] * dd[2];
    for (int c = 0; c < 3; ++c) dmr[c] += (dd[c] - P.dir[c] * proj) / P.ulen;
    for (int c = 0; c < 3; ++c) {
      g[6 + c] = draw[c];
      g[9 + c] = P.dir[c];
    }
  }

  // conic (A, B, C) = inverse of the dilated covariance [[a, b], [b, c]]
  const float a = P.ca, b = P.cb, c = P.cc;
  const float id2 = 1.0f / (P.det * P.det);
  const float da = (-(c * c) * dA + (b * c) * dB - (b * b) * dC) * id2;
  const float db = ((2.0f * b * c) * dA - (a * c + b * b) * dB + (2.0f * a * b) * dC) * id2;
  const float dc = (-(b * b) * dA + (a * b) * dB - (a * a) * dC) * id2;
  // Sigma' = T2 Sigma T2^T (the +0.3 dilation is constant)
  const float hb = 0.5f * db;
  const float* T0 = P.T2;
  const float* T1 = P.T2 + 3;
  float dSig[9];
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q)
      dSig[3 * r + q] = da * T0[r] * T0[q] + hb * (T0[r] * T1[q] + T1[r] * T0[q]) + dc * T1[r] * T1[q];
  float V0[3], V1[3], dT0[3], dT1[3];
  for (int q = 0; q < 3; ++q) {
    V0[q] = da * T0[q] + hb * T1[q];
    V1[q] = hb * T0[q] + dc * T1[q];
  }
  for (int q = 0; q < 3; ++q) {
    dT0[q] = 2.0f * (V0[0] * P.Sig[q] + V0[1] * P.Sig[3 + q] + V0[2] * P.Sig[6 + q]);
    dT1[q] = 2.0f * (V1[0] * P.Sig[q] + V1[1] * P.Sig[3 + q] + V1[2] * P.Sig[6 + q]);
  }
  const float* W = v.R;
  float dJ00 = 0.0f, dJ02 = 0.0f, dJ11 = 0.0f, dJ12 = 0.0f;
  for (int q = 0; q < 3; ++q) {
    dJ00 += dT0[q] * W[q];
    dJ02 += dT0[q] * W[6 + q];
    dJ11 += dT1[q] * W[3 + q];
    dJ12 += dT1[q] * W[6 + q];
  }
  // J(p) at the guarded point, 2D mean m(p)
  const float px = P.p[0], py = P.p[1], pz = P.p[2];
  const float iz = 1.0f / pz, iz2 = iz * iz;
  float dp[3] = {0.0f, 0.0f, 0.0f};
  dp[2] += -v.fx * iz2 * dJ00 - v.fy * iz2 * dJ11;
  if (P.flags & (kGuardXLo | kGuardXHi)) {
    dp[2] += v.fx * (P.tx * iz) * iz2 * dJ02;
  } else {
    dp[0] += -v.fx * iz2 * dJ02;
    dp[2] += 2.0f * v.fx * px * iz2 * iz * dJ02;
  }
  if (P.flags & (kGuardYLo | kGuardYHi)) {
    dp[2] += v.fy * (P.ty * iz) * iz2 * dJ12;
  } else {
    dp[1] += -v.fy * iz2 * dJ12;
    dp[2] += 2.0f * v.fy * py * iz2 * iz * dJ12;
  }
  dp[2] += dz;  // the depth channel blends the camera-space z
  dp[0] += v.fx * iz * dmx;
  dp[1] += v.fy * iz * dmy;
  dp[2] += -v.fx * px * iz2 * dmx - v.fy * py * iz2 * dmy;
  for (int q = 0; q < 3; ++q) dmr[q] += W[q] * dp[0] + W[3 + q] * dp[1] + W[6 + q] * dp[2];

  // Sigma = M M^T, M = R(q^) diag(s)
  float dR[9];
  for (int q = 0; q < 3; ++q) {
    float ds = 0.0f;
    for (int r = 0; r < 3; ++r) {
      const float dM = 2.0f * (dSig[3 * r] * P.M[q] + dSig[3 * r + 1] * P.M[3 + q] + dSig[3 * r + 2] * P.M[6 + q]);
      ds += dM * P.Rq[3 * r + q];
      dR[3 * r + q] = dM * P.sc[q];
    }
    acc.scale[q] += ds;
  }
  {
    const float w = P.qn[0], x = P.qn[1], y = P.qn[2], z = P.qn[3];
    float dq[4];
    dq[0] = 2.0f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2.0f * (y * dR[1] + z * dR[2] + y * dR[3] - w * dR[5] + z * dR[6] + w * dR[7]) -
            4.0f * x * (dR[4] + dR[8]);
    dq[2] = 2.0f * (x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7]) -
            4.0f * y * (dR[0] + dR[8]);
    dq[3] = 2.0f * (-w * dR[1] + x * dR[2] + w * dR[3] + y * dR[5] + x * dR[6] + y * dR[7]) -
            4.0f * z * (dR[0] + dR[4]);
    const float qd = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
    for (int q = 0; q < 4; ++q) acc.rot[q] += (dq[q] - P.qn[q] * qd) / P.qnorm;
  }

  // temporal model
  const float l = s.period[i], tau = s.tau[i], beta = s.beta[i];
  float vel[3];
  for (int q = 0; q < 3; ++q) vel[q] = s.vel[q * n + i];
  const float vg = vel[0] * dmr[0] + vel[1] * dmr[1] + vel[2] * dmr[2];
  float dv[3] = {0.0f, 0.0f, 0.0f};
  float dl = 0.0f, dtau = 0.0f, dbeta = 0.0f;
  if (v.dt != 0.0f) {
    if (v.mode == 0) {
      const float e = expf(-0.5f * (beta / l));
      for (int q = 0; q < 3; ++q) dv[q] += e * v.dt * dmr[q];
      dbeta += vg * v.dt * e * (-0.5f / l);
      dl += vg * v.dt * e * (0.5f * beta / (l * l));
    } else {
      for (int q = 0; q < 3; ++q) dv[q] += v.dt * dmr[q];
    }
  }
  const float d = v.t - tau;
  const float phi = (kTwoPi * d) / l;
  float sphi, cphi;
  sincosf(phi, &sphi, &cphi);
  const float k = (l / kTwoPi) * sphi;
  for (int q = 0; q < 3; ++q) {
    acc.mu[q] += dmr[q];
    acc.vel[q] += dv[q] + k * dmr[q];
  }
  dtau += -cphi * vg;
  dl += (sphi / kTwoPi - (d / l) * cphi) * vg;
  {  // v~ = v e with e = exp(-beta / (2 l)), rho = beta / l
    const float e = expf(-0.5f * (beta / l));
    const float vdot = vel[0] * dvb0 + vel[1] * dvb1 + vel[2] * dvb2;
    acc.vel[0] += e * dvb0;
    acc.vel[1] += e * dvb1;
    acc.vel[2] += e * dvb2;
    dbeta += vdot * e * (-0.5f / l) + drho / l;
    dl += vdot * e * (0.5f * beta / (l * l)) - drho * beta / (l * l);
  }
  const float qb = d / beta;
  const float eo = expf(-0.5f * (qb * qb));
  acc.op += eo * dop;
  dtau += dop * P.op * d / (beta * beta);
  dbeta += dop * P.op * d * d / (beta * beta * beta);
  acc.l += dl;
  acc.tau += dtau;
  acc.beta += dbeta;
}

// Adjoint of the per-Gaussian stage for up to kMaxBwdViews views of one set
// of Gaussians: each Gaussian's gradient is summed over the views in
// registers (the SH part in a second loop over the views, to bound register
// use) and written, or added, once.  A Gaussian no view sees gets zeros
// (accumulate = 0) or is left alone.
// 3 waves per SIMD: the compiler fits the view loop in 168 registers without spilling
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_preprocess_bwd(BwdViews pk, pvg_gaussians_grad grad, int accumulate) {
  const Scene& s = pk.views[0].s;
  const int64_t n = s.n;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const int K = (s.degree + 1) * (s.degree + 1);
  bool any = false;
  for (int v = 0; v < pk.nv; ++v) any = any || pk.radius[v][i] > 0;
  if (!any) {
    if (!accumulate) {
      for (int c = 0; c < 3; ++c) {
        grad.mu[c * n + i] = 0.0f; grad.scale[c * n + i] = 0.0f; grad.vel[c * n + i] = 0.0f;
      }
      for (int c = 0; c < 4; ++c) grad.rot[c * n + i] = 0.0f;
      for (int c = 0; c < 3 * K; ++c) grad.sh[c * n + i] = 0.0f;
      grad.opacity[i] = 0.0f; grad.period[i] = 0.0f; grad.tau[i] = 0.0f; grad.beta[i] = 0.0f;
    }
    return;
  }
  GeoGrad acc = {};
  if (accumulate) {  // start from the previous values
    for (int q = 0; q < 3; ++q) {
      acc.mu[q] = grad.mu[q * n + i];
      acc.vel[q] = grad.vel[q * n + i];
      acc.scale[q] = grad.scale[q * n + i];
    }
    for (int q = 0; q < 4; ++q) acc.rot[q] = grad.rot[q * n + i];
    acc.op = grad.opacity[i];
    acc.l = grad.period[i];
    acc.tau = grad.tau[i];
    acc.beta = grad.beta[i];
  }
  float dnorm = 0.0f, dcount = 0.0f;  // view-space gradient statistics of the adaptive control
  for (int v = 0; v < pk.nv; ++v) {
    if (pk.radius[v][i] <= 0) continue;
    if (grad.densify_grad) {  // |dL / d(mean in NDC)|, NDC = 2 (pixel / size) - 1
      const float* g = pk.g2d[v] + kG2DStride * i;
      const float gx = g[0] * (0.5f * static_cast<float>(pk.views[v].W));
      const float gy = g[1] * (0.5f * static_cast<float>(pk.views[v].H));
      dnorm += sqrtf(gx * gx + gy * gy);
      dcount += 1.0f;
    }
    Proj P;
    project(pk.views[v], i, P, false);
    view_direction(pk.views[v], P);
    adjoint_geometry(pk.views[v], i, P, pk.rgb[v] + 3 * i, pk.g2d[v] + kG2DStride * i, acc,
                     pk.feat_grad[v] != nullptr);
  }
  if (grad.densify_grad) {
    grad.densify_grad[i] += dnorm;
    grad.densify_count[i] += dcount;
  }
  for (int q = 0; q < 3; ++q) {
    grad.mu[q * n + i] = acc.mu[q];
    grad.vel[q * n + i] = acc.vel[q];
    grad.scale[q * n + i] = acc.scale[q];
  }
  for (int q = 0; q < 4; ++q) grad.rot[q * n + i] = acc.rot[q];
  grad.opacity[i] = acc.op;
  grad.period[i] = acc.l;
  grad.tau[i] = acc.tau;
  grad.beta[i] = acc.beta;

  // dL/dsh_k = Y_k(dir) d(rgb), where the colour is not clamped
  float gsh[48];
#pragma unroll
  for (int j = 0; j < 48; ++j) gsh[j] = (j < 3 * K && accumulate) ? grad.sh[j * n + i] : 0.0f;
  for (int v = 0; v < pk.nv; ++v) {
    if (pk.radius[v][i] <= 0) continue;
    const float* g = pk.g2d[v] + kG2DStride * i;  // d(rgb) unclamped part and direction, from the first loop
    if (pk.feat_grad[v]) {  // a feature view: its gradient goes to the feature rows, not to the SH
      for (int c = 0; c < 3; ++c) pk.feat_grad[v][c * n + i] += g[6 + c];
      continue;
    }
    const float draw[3] = {g[6], g[7], g[8]};
    float Y[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) Y[k] = 0.0f;
    sh_eval_basis(s.degree, g[9], g[10], g[11], Y);
#pragma unroll
    for (int j = 0; j < 48; ++j) gsh[j] += Y[j / 3] * draw[j % 3];
  }
#pragma unroll
  for (int j = 0; j < 48; ++j)
    if (j < 3 * K) grad.sh[j * n + i] = gsh[j];
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f32(float* p, float v, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static unsigned grid_for(int64_t n, int block) { return static_cast<unsigned>((n + block - 1) / block); }

hipError_t launch_preprocess(const ViewSet& vs, const Geom& geom, hipStream_t s) {
  if (vs.total_gauss == 0) return hipSuccess;
  StageScope scope(PVG_STAGE_PREPROCESS, s);
  hipLaunchKernelGGL(k_preprocess, dim3(grid_for(vs.total_gauss, 256)), dim3(256), 0, s, vs, geom, nullptr);
  return hipGetLastError();
}

hipError_t launch_preprocess_views(const PreViews& pk, hipStream_t s) {
  const int64_t n = pk.views[0].s.n;
  if (n == 0 || pk.nv <= 0) return hipSuccess;
  StageScope scope(PVG_STAGE_PREPROCESS, s);
  hipLaunchKernelGGL(k_preprocess_views, dim3(grid_for(n, 256) * static_cast<unsigned>(pk.nv)), dim3(256), 0, s, pk);
  return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const BwdViews& pk, const pvg_gaussians_grad& grad, int accumulate,
                                 hipStream_t s) {
  const int64_t n = pk.views[0].s.n;
  if (n == 0 || pk.nv <= 0) return hipSuccess;
  StageScope scope(PVG_STAGE_PREPROCESS_BWD, s);
  hipLaunchKernelGGL(k_preprocess_bwd, dim3(grid_for(n, 256)), dim3(256), 0, s, pk, grad, accumulate);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace pvg
