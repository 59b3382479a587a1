// Per-Gaussian stage (forward and adjoint) of the PVG rasterizer on gfx950.
//
// Forward: temporal state (Sec. 3.2, Eqs. (6)-(7)), flow translation
// (Sec. 3.4, Eqs. (10), (12)), EWA projection (Sec. 3.1, Eq. (2)), radius,
// tile rectangle and SH colour.  Parameter reads are structure-of-arrays, so
// a wave reads 256 contiguous bytes per field; the SH coefficients (up to
// 192 B per Gaussian) are only read for visible ones.  For several views of
// one set of Gaussians a thread takes one Gaussian through every view: the
// time state (two double-precision transcendentals) is formed once per
// distinct render time and the 3D covariance once, then each view's
// projection.
//
// Adjoint: one thread per Gaussian recomputes the forward state of each view
// (bit-identical, so every branch decision is the forward's) and applies the
// chain rule from that view's screen-space gradient (2D mean, conic,
// opacity, colour) to the view's translated mean, covariance and opacity.
// Those are summed over the views in registers; the covariance's chain to
// (s, q) is then taken once, and the temporal chain to {mu, v, tau, beta, l}
// and o once per distinct render time, since each is linear in the sums.
#include "pvg_math.hpp"

namespace pvg {

// The projected record of Gaussian i of view v at slot gi of geom, from its
// time state and covariance.  With `dir` the colour is left to the caller:
// for a visible Gaussian the view direction goes to dir and the function
// returns true (the rgb slots are written only for an invisible one).
template <bool kDir = false>
__device__ __forceinline__ bool preprocess_view(const View& v, int64_t i, GaussTime& G, GaussCov& C,
                                                const Geom& geom, int64_t gi, float3* dir = nullptr) {
  Proj P;
  const bool vis = project_view(v, i, G, C, P, !kDir);
  geom.depth[gi] = P.p[2];
  if (vis) {
    reinterpret_cast<float2*>(geom.xy)[gi] = make_float2(P.x, P.y);
    reinterpret_cast<float4*>(geom.conic_op)[gi] = make_float4(P.A, P.B, P.C, P.op);
    if (kDir) {
      view_direction(v, P);
      *dir = make_float3(P.dir[0], P.dir[1], P.dir[2]);
    } else {
      geom.rgb[3 * gi] = P.rgb[0];
      geom.rgb[3 * gi + 1] = P.rgb[1];
      geom.rgb[3 * gi + 2] = P.rgb[2];
    }
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
  return vis;
}

__global__ void __launch_bounds__(256) k_preprocess(ViewSet vs, Geom geom, unsigned long long* dummy) {
  const int64_t gi = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (gi >= live_gauss(vs)) return;
  const View& v = view_at(vs, view_of_gauss(vs, gi));
  const int64_t i = gi - v.geom_off;
  GaussTime G;
  GaussCov C;
  C.ready = false;
  gauss_time(v.s, i, v.t, G);
  preprocess_view(v, i, G, C, geom, gi);
  (void)dummy;
}

// The clamped SH colours of Gaussian i in the views whose bit is set in
// `vis` (view directions in dir), its 3K coefficients loaded once for all of
// them; per view the operations of project_view's colour, in its order.
template <int K>
__device__ __forceinline__ void view_colours(const PreViews& pk, int64_t i, const float3 (&dir)[kMaxBwdViews],
                                             uint32_t vis) {
  const Scene& s = pk.views[0].s;
  float c[3 * K];
#pragma unroll
  for (int j = 0; j < 3 * K; ++j) c[j] = s.sh[j * s.n + i];
#pragma unroll
  for (int k = 0; k < kMaxBwdViews; ++k) {
    if (!((vis >> k) & 1u)) continue;
    float Y[16];
    sh_eval_basis(s.degree, dir[k].x, dir[k].y, dir[k].z, Y);
    float* rgb = pk.geoms[k].rgb + 3 * i;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float acc = 0.0f;
#pragma unroll
      for (int q = 0; q < K; ++q) acc += c[3 * q + ch] * Y[q];
      const float raw = acc + 0.5f;
      rgb[ch] = raw < 0.0f ? -0.0f : raw;  // clamped: -0 marks the clamp
    }
  }
}

// Several views of one set of Gaussians: thread i takes Gaussian i through
// every view of the pass, forming its time state once per distinct render
// time and its covariance once; then, if any view sees it, its SH
// coefficients are read once and its colour formed in each such view.  Each
// view's record is the single-view one (the same operations on the same
// values).
__global__ void __launch_bounds__(256) k_preprocess_views(PreViews pk) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const Scene& s = pk.views[0].s;
  if (i >= s.n) return;
  GaussTime G;
  GaussCov C;
  C.ready = false;
  gauss_time(s, i, pk.views[0].t, G);
  float3 dir[kMaxBwdViews];
  uint32_t vis = 0;
#pragma unroll
  for (int k = 0; k < kMaxBwdViews; ++k) {
    dir[k] = make_float3(0.0f, 0.0f, 1.0f);
    if (k < pk.nv) {
      if (pk.views[k].t != G.t) gauss_time(s, i, pk.views[k].t, G);
      if (preprocess_view<true>(pk.views[k], i, G, C, pk.geoms[k], i, &dir[k])) vis |= 1u << k;
    }
  }
  if (vis == 0) return;
  switch (s.degree) {
    case 0: view_colours<1>(pk, i, dir, vis); break;
    case 1: view_colours<4>(pk, i, dir, vis); break;
    case 2: view_colours<9>(pk, i, dir, vis); break;
    default: view_colours<16>(pk, i, dir, vis); break;
  }
}

// Gradient entries of one Gaussian other than its SH coefficients.
struct GeoGrad {
  float mu[3], scale[3], rot[4], vel[3], op, l, tau, beta;
};

// Per-Gaussian sums of the views' gradients with respect to the quantities
// the views share: the covariance Sigma, and per render time the translated
// means (split by flow mode: plain, translated by v_bar dt, translated by
// v dt) and the decayed opacity; plus the blended velocity and staticness.
struct ViewSums {
  float dSig[6];        // d Sigma, upper triangle (00, 01, 02, 11, 12, 22)
  float dmr[3];         // sum over the views of dL/d(translated mean)
  float dmr_dt_bar[3];  // sum of dt dL/d(mean) over the views translated by v_bar dt
  float dmr_dt_raw[3];  // the same over the views translated by v dt
  float dop;            // sum of dL/d o~(t)
  float dvb[3], drho;   // blended v~ = v exp(-beta / (2 l)) and rho = beta / l
};

__device__ __forceinline__ void clear_time_sums(ViewSums& S) {
  for (int c = 0; c < 3; ++c) { S.dmr[c] = 0.0f; S.dmr_dt_bar[c] = 0.0f; S.dmr_dt_raw[c] = 0.0f; }
  S.dop = 0.0f;
}

// One view's chain rule from its screen-space gradient g of the Gaussian:
// d(mean x, y), d(conic A, B, C), d(opacity), d(rgb), and the blended
// channels' d(z, v~, rho), to the view's translated mean, covariance and
// opacity, added into S.  On return g[6..8] holds d(rgb) with clamped
// channels zeroed and g[9..11] the view direction, which is all dL/dsh
// needs.  rgb is the forward's colour of the Gaussian, where a clamped
// channel is -0.
__device__ __forceinline__ void adjoint_view(const View& v, int64_t i, const Proj& P, const GaussCov& C,
                                             const float* rgb, float* g, ViewSums& S, bool feature) {
  const Scene& s = v.s;
  const int64_t n = s.n;
  const int K = (s.degree + 1) * (s.degree + 1);
  const float dmx = g[0], dmy = g[1], dA = g[2], dB = g[3], dC = g[4], dop = g[5];
  // the blended channels' gradients (0 without them), read before slots 9.. are reused:
  // camera depth z, mean velocity v~ and staticness rho
  const float dz = g[9];
  S.dvb[0] += g[10];
  S.dvb[1] += g[11];
  S.dvb[2] += g[12];
  S.drho += g[13];
  float dmr[3] = {0.0f, 0.0f, 0.0f};

  // colour: rgb = max(0, sum_k sh_k Y_k(dir) + 1/2), dir = u / |u|; its
  // dependence on the direction moves the mean.  A feature view's "colour"
  // is a per-Gaussian value: no clamp, no direction term, g[6..8] kept.
  if (!feature) {
    float draw[3];
    for (int ch = 0; ch < 3; ++ch) draw[ch] = signbit(rgb[ch]) ? 0.0f : g[6 + ch];
    float wk[16];
    sh_weights(s, i, draw, wk);
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
  {
    constexpr int kr[6] = {0, 0, 0, 1, 1, 2}, kq[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int r = kr[e], q = kq[e];
      S.dSig[e] += da * T0[r] * T0[q] + hb * (T0[r] * T1[q] + T1[r] * T0[q]) + dc * T1[r] * T1[q];
    }
  }
  float V0[3], V1[3], dT0[3], dT1[3];
  for (int q = 0; q < 3; ++q) {
    V0[q] = da * T0[q] + hb * T1[q];
    V1[q] = hb * T0[q] + dc * T1[q];
  }
  for (int q = 0; q < 3; ++q) {
    dT0[q] = 2.0f * (V0[0] * C.Sig[q] + V0[1] * C.Sig[3 + q] + V0[2] * C.Sig[6 + q]);
    dT1[q] = 2.0f * (V1[0] * C.Sig[q] + V1[1] * C.Sig[3 + q] + V1[2] * C.Sig[6 + q]);
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

  // the translated mean mr = mu~(t) + v_bar dt (mode 0) or + v dt (mode 1)
  for (int q = 0; q < 3; ++q) S.dmr[q] += dmr[q];
  if (v.dt != 0.0f) {
    float* dst = v.mode == 0 ? S.dmr_dt_bar : S.dmr_dt_raw;
    for (int q = 0; q < 3; ++q) dst[q] += v.dt * dmr[q];
  }
  S.dop += dop;
}

// Sigma = M M^T, M = R(q^) diag(s): the summed d Sigma to d s and d q.
__device__ __forceinline__ void adjoint_cov(const GaussCov& C, const float dS[6], GeoGrad& acc) {
  const float dSig[9] = {dS[0], dS[1], dS[2], dS[1], dS[3], dS[4], dS[2], dS[4], dS[5]};
  float dR[9];
  for (int q = 0; q < 3; ++q) {
    float ds = 0.0f;
    for (int r = 0; r < 3; ++r) {
      const float dM = 2.0f * (dSig[3 * r] * C.M[q] + dSig[3 * r + 1] * C.M[3 + q] + dSig[3 * r + 2] * C.M[6 + q]);
      ds += dM * C.Rq[3 * r + q];
      dR[3 * r + q] = dM * C.sc[q];
    }
    acc.scale[q] += ds;
  }
  const float w = C.qn[0], x = C.qn[1], y = C.qn[2], z = C.qn[3];
  float dq[4];
  dq[0] = 2.0f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  dq[1] = 2.0f * (y * dR[1] + z * dR[2] + y * dR[3] - w * dR[5] + z * dR[6] + w * dR[7]) -
          4.0f * x * (dR[4] + dR[8]);
  dq[2] = 2.0f * (x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7]) -
          4.0f * y * (dR[0] + dR[8]);
  dq[3] = 2.0f * (-w * dR[1] + x * dR[2] + w * dR[3] + y * dR[5] + x * dR[6] + y * dR[7]) -
          4.0f * z * (dR[0] + dR[4]);
  const float qd = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
  for (int q = 0; q < 4; ++q) acc.rot[q] += (dq[q] - C.qn[q] * qd) / C.qnorm;
}

// The temporal chain of the views at one render time t (Eqs. (6), (7), (10),
// (12)), from the time sums of S, into acc.
__device__ __forceinline__ void adjoint_time(const Scene& s, int64_t i, const GaussTime& G, const ViewSums& S,
                                             GeoGrad& acc) {
  const float l = G.l, beta = G.beta, tau = s.tau[i];
  const float* vel = G.vel;
  float dl = 0.0f, dtau = 0.0f, dbeta = 0.0f;
  // flow translation: mr = mu~ + v e dt (mode 0, e = exp(-beta / (2 l))) or + v dt
  {
    const float e = expf(-0.5f * (beta / l));
    const float vg = vel[0] * S.dmr_dt_bar[0] + vel[1] * S.dmr_dt_bar[1] + vel[2] * S.dmr_dt_bar[2];
    for (int q = 0; q < 3; ++q) acc.vel[q] += e * S.dmr_dt_bar[q] + S.dmr_dt_raw[q];
    dbeta += vg * e * (-0.5f / l);
    dl += vg * e * (0.5f * beta / (l * l));
  }
  // vibration: mu~ = mu + (l / 2 pi) sin(phi) v, phi = 2 pi (t - tau) / l
  const float vg = vel[0] * S.dmr[0] + vel[1] * S.dmr[1] + vel[2] * S.dmr[2];
  const float d = G.t - tau;
  const float phi = (kTwoPi * d) / l;
  float sphi, cphi;
  sincosf(phi, &sphi, &cphi);
  const float k = (l / kTwoPi) * sphi;
  for (int q = 0; q < 3; ++q) {
    acc.mu[q] += S.dmr[q];
    acc.vel[q] += k * S.dmr[q];
  }
  dtau += -cphi * vg;
  dl += (sphi / kTwoPi - (d / l) * cphi) * vg;
  // opacity decay: o~ = o exp(-(t - tau)^2 / (2 beta^2))
  const float qb = d / beta;
  const float eo = expf(-0.5f * (qb * qb));
  acc.op += eo * S.dop;
  dtau += S.dop * G.op * d / (beta * beta);
  dbeta += S.dop * G.op * d * d / (beta * beta * beta);
  acc.l += dl;
  acc.tau += dtau;
  acc.beta += dbeta;
}

// The blended velocity and staticness maps' chain (time-independent):
// v~ = v e, e = exp(-beta / (2 l)); rho = beta / l.
__device__ __forceinline__ void adjoint_features(const GaussTime& G, const ViewSums& S, GeoGrad& acc) {
  const float l = G.l, beta = G.beta;
  const float e = expf(-0.5f * (beta / l));
  const float vdot = G.vel[0] * S.dvb[0] + G.vel[1] * S.dvb[1] + G.vel[2] * S.dvb[2];
  for (int q = 0; q < 3; ++q) acc.vel[q] += e * S.dvb[q];
  acc.beta += vdot * e * (-0.5f / l) + S.drho / l;
  acc.l += vdot * e * (0.5f * beta / (l * l)) - S.drho * beta / (l * l);
}

// Adjoint of the per-Gaussian stage for up to kMaxBwdViews views of one set
// of Gaussians at one render time (the host splits passes where t changes):
// each Gaussian's gradient is summed over the views in registers (the SH part
// in a second loop over the views, to bound register use) and written, or
// added, once.  A Gaussian no view sees gets zeros (accumulate = 0) or is
// left alone.
// 3 waves per SIMD: the view loop fits in 168 registers without spilling
__global__ void __launch_bounds__(256) k_preprocess_bwd(BwdViews pk, pvg_gaussians_grad grad,
                                                                                             int accumulate) {
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
  GaussTime G;
  gauss_time(s, i, pk.views[0].t, G);
  GaussCov C;
  C.ready = false;
  ViewSums S;
  for (int e = 0; e < 6; ++e) S.dSig[e] = 0.0f;
  for (int c = 0; c < 3; ++c) S.dvb[c] = 0.0f;
  S.drho = 0.0f;
  clear_time_sums(S);
  float dnorm = 0.0f, dcount = 0.0f;  // view-space gradient statistics of the adaptive control
  for (int v = 0; v < pk.nv; ++v) {
    if (pk.radius[v][i] <= 0) continue;
    const View& vw = pk.views[v];
    float* g = pk.g2d[v] + kG2DStride * i;
    if (grad.densify_grad) {  // |dL / d(mean in NDC)|, NDC = 2 (pixel / size) - 1
      const float gx = g[0] * (0.5f * static_cast<float>(vw.W));
      const float gy = g[1] * (0.5f * static_cast<float>(vw.H));
      dnorm += sqrtf(gx * gx + gy * gy);
      dcount += 1.0f;
    }
    Proj P;
    project_view(vw, i, G, C, P, false);
    view_direction(vw, P);
    adjoint_view(vw, i, P, C, pk.rgb[v] + 3 * i, g, S, pk.feat_grad[v] != nullptr || pk.no_colour[v]);
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
  adjoint_time(s, i, G, S, acc);
  gauss_cov(s, i, C);  // formed again rather than held through the view loop
  adjoint_cov(C, S.dSig, acc);
  adjoint_features(G, S, acc);
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
    if (pk.no_colour[v]) continue;
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
  hipLaunchKernelGGL(k_preprocess_views, dim3(grid_for(n, 256)), dim3(256), 0, s, pk);
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
