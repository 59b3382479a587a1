// Plain CPU oracle for the PVG splatting rasterizer.  TEST INFRASTRUCTURE ONLY:
// only the test suite, the smoke check and the CPU-baseline leg of the
// benchmark load this library.  It shares no code with the GPU path.
//
// It computes, slowly and directly, what the tiled GPU renderer computes:
//   * the PVG temporal state (Sec. 3.2, Eqs. (5)-(7)): vibrating mean and
//     decaying opacity; the flow translation of the temporal-smoothing render
//     (Sec. 3.4, Eqs. (10) and (12));
//   * the 3D Gaussian from scale and unit quaternion (Sec. 3.1, after Eq. (3)),
//     its EWA projection Sigma' = J W Sigma W^T J^T (Sec. 3.1, Eq. (2));
//   * depth ordering per 16x16 tile and front-to-back alpha blending
//     C = sum_i T_i alpha_i c_i (Sec. 3.1, Eq. (3)), with alpha = opacity x the
//     projected 2D Gaussian at the pixel (Sec. 3.1, text after Eq. (3));
//   * the exact derivative of that image with respect to every per-point
//     parameter {mu, q, s, o, c, tau, beta, v} and the cycle length l
//     (Sec. 3.2 parameter list), for a fixed discrete structure.
//
// Conventions the paper leaves open (same constants as the GPU path, each
// side defines them on its own):
//   pinhole camera looking down +z, x right, y down; pixel (i,j) is sampled at
//   its integer coordinates after shifting the principal point by -0.5;
//   near plane z <= znear culls; J is evaluated at the point clamped to 1.3x
//   the half field of view; 0.3 px^2 is added to the 2D covariance; a
//   Gaussian with det <= 0 is invisible; radius = ceil(3 sqrt(lambda_max))
//   with lambda_max = mid + sqrt(max(0.1, mid^2 - det)); alpha =
//   min(0.99, o~ * G) and a pair with G-exponent > 0 or alpha < 1/255 is
//   skipped; a pixel stops before the Gaussian that would take T below 1e-4;
//   the colour is real spherical harmonics (no Condon-Shortley phase) of the
//   view direction plus 0.5, clamped at 0; order within a tile is
//   (depth bits, index).
//   sin and exp of the per-Gaussian temporal stage are the correctly rounded
//   FP32 values (evaluated in FP64 and rounded once), so that the discrete
//   structure is reproducible across implementations; the per-pixel exp of the
//   FP32 image is the C library's expf.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

constexpr int kTile = 16;
constexpr double kPi = 3.14159265358979323846;

struct Params {
  int64_t n;
  int degree;
  const void* mu; const void* scale; const void* rot; const void* sh;
  const void* opacity; const void* vel; const void* period; const void* tau; const void* beta;
};

template <class R> struct P {  // typed accessor over SoA parameter arrays
  const Params& p;
  R get(const void* base, int64_t row, int64_t i) const {
    return static_cast<const R*>(base)[row * p.n + i];
  }
};

struct Camera {  // world->camera x_c = R x_w + T, row-major R
  float R[9], T[3], fx, fy, cx, cy, znear;
  int W, H;
};

struct Frame {
  float t, dt;
  int mode;  // 0: advect by the average velocity v*exp(-rho/2); 1: by v
  float bg[3];
};

// flag bits of the discrete per-Gaussian decisions
enum : uint32_t {
  kGuardXLo = 1u << 0, kGuardXHi = 1u << 1, kGuardYLo = 1u << 2, kGuardYHi = 1u << 3,
  kShClampR = 1u << 4, kShClampG = 1u << 5, kShClampB = 1u << 6,
};

template <class R> R sin_cr(R x) { return static_cast<R>(std::sin(static_cast<double>(x))); }
template <class R> R cos_cr(R x) { return static_cast<R>(std::cos(static_cast<double>(x))); }
template <class R> R exp_cr(R x) { return static_cast<R>(std::exp(static_cast<double>(x))); }

// ---------------------------------------------------------------------------
// Real spherical harmonics, degree <= 3, index k = l*l + l + m.
// Y_l^m = N_l^|m| * Q_l^|m|(z) * {Re (x+iy)^m  (m>0) ; 1 (m=0) ; Im (x+iy)^|m| (m<0)}
// with N_l^m = sqrt((2l+1)/(4pi) (l-m)!/(l+m)!) * (sqrt 2 if m != 0) and
// Q_l^m(z) = d^m/dz^m P_l(z), the associated Legendre function without the
// (1-z^2)^{m/2} factor and without the Condon-Shortley phase, from the
// standard three-term recurrence.  Gradients are with respect to (x,y,z) of
// this polynomial extension.
template <class R>
void sh_basis(int degree, const R d[3], R Y[16], R dY[16][3]) {
  const R x = d[0], y = d[1], z = d[2];
  // powers of (x + i y): re[m], im[m]
  R re[4], im[4];
  re[0] = R(1); im[0] = R(0);
  for (int m = 1; m < 4; ++m) {
    re[m] = re[m - 1] * x - im[m - 1] * y;
    im[m] = re[m - 1] * y + im[m - 1] * x;
  }
  for (int l = 0; l <= degree; ++l) {
    for (int m = -l; m <= l; ++m) {
      const int am = m < 0 ? -m : m;
      // Q_l^am(z) and its z-derivative by recurrence in l
      R dfact = R(1);
      for (int k = 1; k <= 2 * am - 1; k += 2) dfact *= R(k);
      R q_prev2 = R(0), dq_prev2 = R(0);
      R q_prev = dfact, dq_prev = R(0);  // Q_am^am
      R q = q_prev, dq = dq_prev;
      if (l > am) {
        R q1 = z * R(2 * am + 1) * dfact;
        R dq1 = R(2 * am + 1) * dfact;
        q_prev2 = q_prev; dq_prev2 = dq_prev;
        q_prev = q1; dq_prev = dq1;
        q = q1; dq = dq1;
        for (int ll = am + 2; ll <= l; ++ll) {
          R qn = (R(2 * ll - 1) * z * q_prev - R(ll + am - 1) * q_prev2) / R(ll - am);
          R dqn = (R(2 * ll - 1) * (q_prev + z * dq_prev) - R(ll + am - 1) * dq_prev2) / R(ll - am);
          q_prev2 = q_prev; dq_prev2 = dq_prev;
          q_prev = qn; dq_prev = dqn;
          q = qn; dq = dqn;
        }
      }
      double fr = 1.0;  // (l-am)!/(l+am)!
      for (int k = l - am + 1; k <= l + am; ++k) fr /= k;
      double nrm = std::sqrt((2.0 * l + 1.0) / (4.0 * kPi) * fr);
      if (m != 0) nrm *= std::sqrt(2.0);
      const R N = static_cast<R>(nrm);
      R ang, dax, day;  // angular factor and its x, y derivatives
      if (m > 0) {
        ang = re[am];
        dax = R(am) * re[am - 1];
        day = -R(am) * im[am - 1];
      } else if (m < 0) {
        ang = im[am];
        dax = R(am) * im[am - 1];
        day = R(am) * re[am - 1];
      } else {
        ang = R(1); dax = R(0); day = R(0);
      }
      const int k = l * l + l + m;
      Y[k] = N * q * ang;
      dY[k][0] = N * q * dax;
      dY[k][1] = N * q * day;
      dY[k][2] = N * dq * ang;
    }
  }
}

// ---------------------------------------------------------------------------
// Per-Gaussian state.
template <class R> struct Splat {
  bool visible;
  R x, y;        // 2D mean in pixel coordinates (shifted by -0.5)
  R A, B, C;     // conic = inverse of the dilated 2D covariance
  R op;          // opacity at time t
  R rgb[3];
  R depth;       // camera-space z
  R feat[4];     // mean velocity v~ = v exp(-beta / (2 l)) (Sec. 3.4) and staticness rho = beta / l
  int radius;
  int rect[4];   // tile rectangle x0, y0, x1, y1 (half-open)
  uint32_t flags;
};

struct Fixed {  // discrete decisions imposed on an evaluation
  bool visible;
  uint32_t flags;
};

// The temporal stage: mean at time t (Eq. (6)), opacity at time t (Eq. (7)),
// and the flow-translated render mean (Eqs. (10), (12)).
template <class R>
void temporal(const R mu[3], const R v[3], R l, R tau, R beta, R o, R t, R dt, int mode,
              R mu_r[3], R& op) {
  const R two_pi = static_cast<R>(2.0 * kPi);
  const R d = t - tau;
  const R phi = (two_pi * d) / l;
  const R k = (l / two_pi) * sin_cr(phi);
  const R q = d / beta;
  op = o * exp_cr(R(-0.5) * (q * q));
  R mt[3];
  for (int c = 0; c < 3; ++c) mt[c] = mu[c] + k * v[c];
  if (dt != R(0)) {
    const R ev = mode == 0 ? exp_cr(R(-0.5) * (beta / l)) : R(1);
    for (int c = 0; c < 3; ++c) mu_r[c] = mt[c] + (v[c] * ev) * dt;
  } else {
    for (int c = 0; c < 3; ++c) mu_r[c] = mt[c];
  }
}

template <class R>
void quat_to_rot(const R qr[4], R Rq[9], R qn[4], R& norm) {
  const R n2 = ((qr[0] * qr[0] + qr[1] * qr[1]) + qr[2] * qr[2]) + qr[3] * qr[3];
  norm = std::sqrt(n2);
  for (int c = 0; c < 4; ++c) qn[c] = qr[c] / norm;
  const R w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  Rq[0] = R(1) - R(2) * (y * y + z * z);
  Rq[1] = R(2) * (x * y - w * z);
  Rq[2] = R(2) * (x * z + w * y);
  Rq[3] = R(2) * (x * y + w * z);
  Rq[4] = R(1) - R(2) * (x * x + z * z);
  Rq[5] = R(2) * (y * z - w * x);
  Rq[6] = R(2) * (x * z - w * y);
  Rq[7] = R(2) * (y * z + w * x);
  Rq[8] = R(1) - R(2) * (x * x + y * y);
}

// Intermediates of one Gaussian's projection, kept for the adjoint.
template <class R> struct Inter {
  R mu[3], v[3], l, tau, beta, o, s[3], q[4], qn[4], qnorm;
  R mu_r[3], p[3], Rq[9], M[9], Sig[9];
  R tx, ty, J00, J02, J11, J12, T2[6], S2[3];  // S2: dilated a, b, c
  R det, dir[3], ulen, Y[16], dY[16][3], raw[3];
};

// One Gaussian through O1 (temporal state, view transform, covariance, EWA,
// conic, radius, tile rectangle, colour).  With `fixed`, the discrete
// decisions (visibility, Jacobian guard, colour clamp) are taken from it
// instead of being decided here.
template <class R>
void preprocess_one(const Params& prm, int64_t i, const Camera& cam, const Frame& fr,
                    const Fixed* fixed, Splat<R>& s, Inter<R>* it_out) {
  P<R> a{prm};
  Inter<R> it;
  s.visible = false;
  s.radius = 0;
  s.flags = 0;
  for (int c = 0; c < 4; ++c) s.rect[c] = 0;
  for (int c = 0; c < 3; ++c) {
    it.mu[c] = a.get(prm.mu, c, i);
    it.v[c] = a.get(prm.vel, c, i);
    it.s[c] = a.get(prm.scale, c, i);
  }
  for (int c = 0; c < 4; ++c) it.q[c] = a.get(prm.rot, c, i);
  it.l = a.get(prm.period, 0, i);
  it.tau = a.get(prm.tau, 0, i);
  it.beta = a.get(prm.beta, 0, i);
  it.o = a.get(prm.opacity, 0, i);

  temporal<R>(it.mu, it.v, it.l, it.tau, it.beta, it.o, R(fr.t), R(fr.dt), fr.mode, it.mu_r, s.op);

  R W[9], T[3];
  for (int c = 0; c < 9; ++c) W[c] = R(cam.R[c]);
  for (int c = 0; c < 3; ++c) T[c] = R(cam.T[c]);
  for (int r = 0; r < 3; ++r)
    it.p[r] = ((W[3 * r] * it.mu_r[0] + W[3 * r + 1] * it.mu_r[1]) + W[3 * r + 2] * it.mu_r[2]) + T[r];
  s.depth = it.p[2];
  {  // the per-Gaussian quantities of the velocity and staticness maps
    const R e = exp_cr(R(-0.5) * (it.beta / it.l));
    for (int c = 0; c < 3; ++c) s.feat[c] = it.v[c] * e;
    s.feat[3] = it.beta / it.l;
  }
  if (fixed) {
    if (!fixed->visible) return;
  } else if (!(it.p[2] > R(cam.znear))) {
    return;
  }

  // Sigma = R(q) S S^T R(q)^T
  quat_to_rot<R>(it.q, it.Rq, it.qn, it.qnorm);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) it.M[3 * r + c] = it.Rq[3 * r + c] * it.s[c];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      it.Sig[3 * r + c] = (it.M[3 * r] * it.M[3 * c] + it.M[3 * r + 1] * it.M[3 * c + 1]) +
                          it.M[3 * r + 2] * it.M[3 * c + 2];

  // EWA: J at the point clamped to the guard band, Sigma' = (J W) Sigma (J W)^T
  const R fx = R(cam.fx), fy = R(cam.fy), cx = R(cam.cx), cy = R(cam.cy);
  const R px = it.p[0], py = it.p[1], pz = it.p[2];
  const R limx = R(1.3f) * ((R(0.5f) * R(cam.W)) / fx);
  const R limy = R(1.3f) * ((R(0.5f) * R(cam.H)) / fy);
  const R txz = px / pz, tyz = py / pz;
  uint32_t gflags = 0;
  if (fixed) {
    gflags = fixed->flags & (kGuardXLo | kGuardXHi | kGuardYLo | kGuardYHi);
  } else {
    if (txz < -limx) gflags |= kGuardXLo;
    if (txz > limx) gflags |= kGuardXHi;
    if (tyz < -limy) gflags |= kGuardYLo;
    if (tyz > limy) gflags |= kGuardYHi;
  }
  const R cxz = (gflags & kGuardXLo) ? -limx : (gflags & kGuardXHi) ? limx : txz;
  const R cyz = (gflags & kGuardYLo) ? -limy : (gflags & kGuardYHi) ? limy : tyz;
  it.tx = (gflags & (kGuardXLo | kGuardXHi)) ? cxz * pz : px;
  it.ty = (gflags & (kGuardYLo | kGuardYHi)) ? cyz * pz : py;
  it.J00 = fx / pz;
  it.J02 = -(fx * it.tx) / (pz * pz);
  it.J11 = fy / pz;
  it.J12 = -(fy * it.ty) / (pz * pz);
  for (int c = 0; c < 3; ++c) {
    it.T2[c] = it.J00 * W[c] + it.J02 * W[6 + c];
    it.T2[3 + c] = it.J11 * W[3 + c] + it.J12 * W[6 + c];
  }
  R U[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c)
      U[3 * r + c] = (it.T2[3 * r] * it.Sig[c] + it.T2[3 * r + 1] * it.Sig[3 + c]) +
                     it.T2[3 * r + 2] * it.Sig[6 + c];
  auto cov2 = [&](int r, int c) {
    return (U[3 * r] * it.T2[3 * c] + U[3 * r + 1] * it.T2[3 * c + 1]) + U[3 * r + 2] * it.T2[3 * c + 2];
  };
  const R ca = cov2(0, 0) + R(0.3f);
  const R cb = cov2(0, 1);
  const R cc = cov2(1, 1) + R(0.3f);
  it.S2[0] = ca; it.S2[1] = cb; it.S2[2] = cc;
  it.det = ca * cc - cb * cb;
  if (!fixed && !(it.det > R(0))) return;
  s.A = cc / it.det;
  s.B = -cb / it.det;
  s.C = ca / it.det;
  s.x = (fx * txz + cx) - R(0.5f);
  s.y = (fy * tyz + cy) - R(0.5f);

  if (!fixed) {
    const R mid = R(0.5f) * (ca + cc);
    const R lam = mid + std::sqrt(std::max(R(0.1f), mid * mid - it.det));
    const int rad = static_cast<int>(std::ceil(R(3) * std::sqrt(lam)));
    const int GX = (cam.W + kTile - 1) / kTile, GY = (cam.H + kTile - 1) / kTile;
    const R rr = R(rad);
    auto cl = [](R v, int hi) {
      const R f = std::floor(v);
      if (f < R(0)) return 0;
      if (f > R(hi)) return hi;
      return static_cast<int>(f);
    };
    s.rect[0] = cl((s.x - rr) / R(kTile), GX);
    s.rect[1] = cl((s.y - rr) / R(kTile), GY);
    s.rect[2] = cl(((s.x + rr) + R(kTile - 1)) / R(kTile), GX);
    s.rect[3] = cl(((s.y + rr) + R(kTile - 1)) / R(kTile), GY);
    if ((s.rect[2] - s.rect[0]) * (s.rect[3] - s.rect[1]) == 0) return;
    s.radius = rad;
  }

  // colour from spherical harmonics of the direction camera centre -> mean
  R cpos[3];
  for (int c = 0; c < 3; ++c)
    cpos[c] = -((W[c] * T[0] + W[3 + c] * T[1]) + W[6 + c] * T[2]);
  R u[3];
  for (int c = 0; c < 3; ++c) u[c] = it.mu_r[c] - cpos[c];
  it.ulen = std::sqrt((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
  for (int c = 0; c < 3; ++c) it.dir[c] = u[c] / it.ulen;
  sh_basis<R>(prm.degree, it.dir, it.Y, it.dY);
  const int K = (prm.degree + 1) * (prm.degree + 1);
  uint32_t cflags = 0;
  for (int ch = 0; ch < 3; ++ch) {
    R acc = R(0);
    for (int k = 0; k < K; ++k) acc += a.get(prm.sh, 3 * k + ch, i) * it.Y[k];
    it.raw[ch] = acc + R(0.5f);
    bool clamp;
    if (fixed) clamp = (fixed->flags & (kShClampR << ch)) != 0;
    else clamp = it.raw[ch] < R(0);
    if (clamp) cflags |= (kShClampR << ch);
    s.rgb[ch] = clamp ? R(0) : it.raw[ch];
  }
  s.flags = gflags | cflags;
  s.visible = true;
  if (it_out) *it_out = it;
}

// ---------------------------------------------------------------------------
// Per-pixel compositing (Eq. (3)).  `dec` holds the FP32 splats that take
// every discrete decision; `val` the splats whose values are blended (the
// same array for the FP32 image).  `rec` optionally receives the contributors.
template <class R> struct Contrib {
  uint32_t g;
  R alpha, T, G, dx, dy;
  bool clamped;
};

template <class R>
void composite_pixel(int px, int py, const uint32_t* list, int64_t len, const Splat<float>* dec,
                     const Splat<R>* val, const float bg[3], R out[3], R& Tfin, R Fout[5], int& ncontrib,
                     std::vector<Contrib<R>>* rec) {
  float T32 = 1.0f;
  R T = R(1);
  R C[3] = {R(0), R(0), R(0)};
  // "flexible rendering" (Sec. 3.1): the Gaussians' camera depths, mean
  // velocities and staticness blended like colour (no background term)
  R F[5] = {R(0), R(0), R(0), R(0), R(0)};
  ncontrib = 0;
  const float fpx = static_cast<float>(px), fpy = static_cast<float>(py);
  for (int64_t k = 0; k < len; ++k) {
    const uint32_t g = list[k];
    const Splat<float>& d = dec[g];
    const float dx = d.x - fpx, dy = d.y - fpy;
    const float power = -0.5f * (d.A * (dx * dx) + d.C * (dy * dy)) - d.B * (dx * dy);
    if (power > 0.0f) continue;
    const float raw = d.op * std::exp(power);
    const float a32 = std::min(0.99f, raw);
    if (a32 < 1.0f / 255.0f) continue;
    const float Tn = T32 * (1.0f - a32);
    if (Tn < 0.0001f) break;
    const bool clamped = raw > 0.99f;
    const Splat<R>& v = val[g];
    const R vdx = v.x - R(fpx), vdy = v.y - R(fpy);
    const R vpow = R(-0.5f) * (v.A * (vdx * vdx) + v.C * (vdy * vdy)) - v.B * (vdx * vdy);
    const R G = std::exp(vpow);
    const R alpha = clamped ? R(0.99f) : v.op * G;
    if (rec) rec->push_back({g, alpha, T, G, vdx, vdy, clamped});
    for (int c = 0; c < 3; ++c) C[c] = C[c] + v.rgb[c] * (alpha * T);
    F[0] = F[0] + v.depth * (alpha * T);
    for (int f = 0; f < 4; ++f) F[1 + f] = F[1 + f] + v.feat[f] * (alpha * T);
    T = T * (R(1) - alpha);
    T32 = Tn;
    ncontrib = static_cast<int>(k + 1);
  }
  for (int c = 0; c < 3; ++c) out[c] = C[c] + T * R(bg[c]);
  Tfin = T;
  for (int f = 0; f < 5; ++f) Fout[f] = F[f];
}

// FP32 image path specialisation: values and decisions are one array.
// Decision margin of a pixel's walk (margin != nullptr): the walk of Eq. (3)
// takes three discrete decisions per pair (skip when the exponent is
// positive, skip when alpha < 1/255, stop when T would fall below 1e-4).  A
// renderer whose FP32 exponent or exponential rounds differently by a few
// ulps may take the other branch where the exact value sits at a threshold.
// *margin receives the smallest, over the walked pairs, of each decision's
// distance to its threshold in units of the rounding it can absorb:
// |power| / (1e-5 S) with S the sum of the exponent's term magnitudes;
// |255 alpha - 1| / 1e-5 (alpha known to ~1e-6 relative); and
// |ln(T_new / 1e-4)| / U with U = 1e-5 sum alpha_i / (1 - alpha_i) + 1e-6 over
// the contributors so far (the relative uncertainty of T that the alphas'
// carry through the products 1 - alpha).  Below 1 a decision is ambiguous.
// With clamp_margin the adjoint's branch at the alpha clamp counts as well
// (the clamped pair passes no gradient): |raw / 0.99 - 1| / 1e-5 over the
// contributors, raw = o~ exp(power) before the clamp.
void composite_pixel_f32(int px, int py, const uint32_t* list, int64_t len, const Splat<float>* sp,
                         const float bg[3], float out[3], float& Tfin, float Fout[5], int& ncontrib,
                         float* margin = nullptr, bool clamp_margin = false) {
  float T = 1.0f;
  float C[3] = {0.0f, 0.0f, 0.0f};
  float F[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  ncontrib = 0;
  const float fpx = static_cast<float>(px), fpy = static_cast<float>(py);
  double m = 1e30, u = 1e-6;
  for (int64_t k = 0; k < len; ++k) {
    const Splat<float>& d = sp[list[k]];
    const float dx = d.x - fpx, dy = d.y - fpy;
    const float power = -0.5f * (d.A * (dx * dx) + d.C * (dy * dy)) - d.B * (dx * dy);
    if (margin) {
      const double S = 0.5 * (std::fabs(static_cast<double>(d.A)) * dx * dx +
                              std::fabs(static_cast<double>(d.C)) * dy * dy) +
                       std::fabs(static_cast<double>(d.B) * dx * dy);
      if (S > 0.0) m = std::min(m, std::fabs(static_cast<double>(power)) / (1e-5 * S));
    }
    if (power > 0.0f) continue;
    const float alpha = std::min(0.99f, d.op * std::exp(power));
    if (margin) m = std::min(m, std::fabs(255.0 * alpha - 1.0) / 1e-5);
    if (alpha < 1.0f / 255.0f) continue;
    const float Tn = T * (1.0f - alpha);
    if (margin) {
      u += 1e-5 * alpha / (1.0 - alpha);
      if (Tn > 0.0f) m = std::min(m, std::fabs(std::log(static_cast<double>(Tn) / 1e-4)) / u);
      else m = 0.0;
    }
    if (Tn < 0.0001f) break;
    if (margin && clamp_margin) {
      const double raw = static_cast<double>(d.op * std::exp(power));
      m = std::min(m, std::fabs(raw / 0.99 - 1.0) / 1e-5);
    }
    for (int c = 0; c < 3; ++c) C[c] = C[c] + d.rgb[c] * (alpha * T);
    F[0] = F[0] + d.depth * (alpha * T);
    for (int f = 0; f < 4; ++f) F[1 + f] = F[1 + f] + d.feat[f] * (alpha * T);
    T = Tn;
    ncontrib = static_cast<int>(k + 1);
  }
  for (int c = 0; c < 3; ++c) out[c] = C[c] + T * bg[c];
  Tfin = T;
  for (int f = 0; f < 5; ++f) Fout[f] = F[f];
  if (margin) *margin = static_cast<float>(std::min(m, 1e30));
}

Camera make_cam(const float* c, int W, int H) {
  Camera cam;
  std::memcpy(cam.R, c, 9 * sizeof(float));
  std::memcpy(cam.T, c + 9, 3 * sizeof(float));
  cam.fx = c[12]; cam.fy = c[13]; cam.cx = c[14]; cam.cy = c[15]; cam.znear = c[16];
  cam.W = W; cam.H = H;
  return cam;
}

Frame make_frame(const float* f) {
  Frame fr;
  fr.t = f[0]; fr.dt = f[1]; fr.mode = static_cast<int>(f[2]);
  fr.bg[0] = f[3]; fr.bg[1] = f[4]; fr.bg[2] = f[5];
  return fr;
}

Params make_params(int64_t n, int degree, const void* const* arr) {
  return Params{n, degree, arr[0], arr[1], arr[2], arr[3], arr[4], arr[5], arr[6], arr[7], arr[8]};
}

// Rebuild FP32 splats (the decision side) from the arrays the FP32 stage wrote.
std::vector<Splat<float>> load_splats(int64_t n, const float* xy, const float* conic_op,
                                      const float* rgb, const int32_t* radius, const uint32_t* flags,
                                      const float* depth = nullptr, const float* feat = nullptr) {
  std::vector<Splat<float>> sp(n);
  for (int64_t i = 0; i < n; ++i) {
    Splat<float>& s = sp[i];
    s.visible = radius[i] > 0;
    s.x = xy[2 * i]; s.y = xy[2 * i + 1];
    s.A = conic_op[4 * i]; s.B = conic_op[4 * i + 1]; s.C = conic_op[4 * i + 2];
    s.op = conic_op[4 * i + 3];
    for (int c = 0; c < 3; ++c) s.rgb[c] = rgb ? rgb[3 * i + c] : 0.0f;
    s.depth = depth ? depth[i] : 0.0f;
    for (int f = 0; f < 4; ++f) s.feat[f] = feat ? feat[4 * i + f] : 0.0f;
    s.flags = flags ? flags[i] : 0;
    s.radius = radius[i];
  }
  return sp;
}

struct Inst { uint32_t tile, dbits, g; };

constexpr int kG2D = 14;  // per-Gaussian screen-space gradient entries of the adjoint

}  // namespace

extern "C" {

// O1 in FP32 for all n Gaussians.  `arr` = 9 float* in the order mu, scale,
// rot, sh, opacity, vel, period, tau, beta (SoA, [rows][n]).  cam = R[9],
// T[3], fx, fy, cx, cy, znear; frame = t, dt, mode, bg[3].
// Outputs: xy[n][2], depth[n], conic_op[n][4], rgb[n][3], radius[n] (0 =
// invisible), rect[n][4], tiles[n], flags[n], and (optional) feat[n][4] = mean
// velocity v~ and staticness rho.
void orc_preprocess_f32(int64_t n, int degree, const void* const* arr, const float* camv, int W, int H,
                        const float* framev, float* xy, float* depth, float* conic_op, float* rgb,
                        int32_t* radius, int32_t* rect, uint32_t* tiles, uint32_t* flags, float* feat) {
  const Params prm = make_params(n, degree, arr);
  const Camera cam = make_cam(camv, W, H);
  const Frame fr = make_frame(framev);
  for (int64_t i = 0; i < n; ++i) {
    Splat<float> s;
    preprocess_one<float>(prm, i, cam, fr, nullptr, s, nullptr);
    xy[2 * i] = s.visible ? s.x : 0.0f;
    xy[2 * i + 1] = s.visible ? s.y : 0.0f;
    depth[i] = s.depth;
    if (feat)
      for (int f = 0; f < 4; ++f) feat[4 * i + f] = s.feat[f];
    conic_op[4 * i] = s.visible ? s.A : 0.0f;
    conic_op[4 * i + 1] = s.visible ? s.B : 0.0f;
    conic_op[4 * i + 2] = s.visible ? s.C : 0.0f;
    conic_op[4 * i + 3] = s.op;
    for (int c = 0; c < 3; ++c) rgb[3 * i + c] = s.visible ? s.rgb[c] : 0.0f;
    radius[i] = s.visible ? s.radius : 0;
    for (int c = 0; c < 4; ++c) rect[4 * i + c] = s.visible ? s.rect[c] : 0;
    tiles[i] = s.visible ? static_cast<uint32_t>((s.rect[2] - s.rect[0]) * (s.rect[3] - s.rect[1])) : 0u;
    flags[i] = s.visible ? s.flags : 0u;
  }
}

// O2 + O3: instances (tile, depth bits, index) of every visible Gaussian,
// sorted lexicographically.  Returns M, or -M-1 if M > cap (nothing written).
// ranges[tile] = [first, last+1) into the sorted list.
int64_t orc_bin_sort(int64_t n, const float* depth, const int32_t* rect, const int32_t* radius,
                     int GX, int GY, int64_t cap, uint32_t* inst_tile, uint32_t* inst_gauss,
                     uint32_t* ranges) {
  std::vector<Inst> inst;
  for (int64_t i = 0; i < n; ++i) {
    if (radius[i] <= 0) continue;
    uint32_t bits;
    std::memcpy(&bits, &depth[i], 4);
    for (int ty = rect[4 * i + 1]; ty < rect[4 * i + 3]; ++ty)
      for (int tx = rect[4 * i]; tx < rect[4 * i + 2]; ++tx)
        inst.push_back({static_cast<uint32_t>(ty * GX + tx), bits, static_cast<uint32_t>(i)});
  }
  const int64_t M = static_cast<int64_t>(inst.size());
  if (M > cap) return -M - 1;
  std::sort(inst.begin(), inst.end(), [](const Inst& a, const Inst& b) {
    if (a.tile != b.tile) return a.tile < b.tile;
    if (a.dbits != b.dbits) return a.dbits < b.dbits;
    return a.g < b.g;
  });
  for (int64_t t = 0; t < static_cast<int64_t>(GX) * GY; ++t) {
    ranges[2 * t] = 0;
    ranges[2 * t + 1] = 0;
  }
  for (int64_t k = 0; k < M; ++k) {
    inst_tile[k] = inst[k].tile;
    inst_gauss[k] = inst[k].g;
    const uint32_t t = inst[k].tile;
    if (k == 0 || inst[k - 1].tile != t) ranges[2 * t] = static_cast<uint32_t>(k);
    if (k == M - 1 || inst[k + 1].tile != t) ranges[2 * t + 1] = static_cast<uint32_t>(k + 1);
  }
  return M;
}

// O4 in FP32 over the tiles [tile_lo, tile_hi) (all tiles: 0, GX*GY).
// img[3][H][W], final_T[H][W], n_contrib[H][W]; untouched outside those tiles.
// depth (optional, per Gaussian) and depth_img (optional output): the blended
// depth channel sum T alpha z of each pixel.
void orc_render_f32(int64_t n, const float* xy, const float* conic_op, const float* rgb,
                    const int32_t* radius, const float* camv, int W, int H, const float* framev,
                    const uint32_t* ranges, const uint32_t* inst_gauss, int64_t tile_lo,
                    int64_t tile_hi, float* img, float* final_T, int32_t* n_contrib, const float* depth,
                    float* depth_img, const float* feat, float* feat_img) {
  const Frame fr = make_frame(framev);
  (void)camv;
  const std::vector<Splat<float>> sp = load_splats(n, xy, conic_op, rgb, radius, nullptr, depth, feat);
  const int GX = (W + kTile - 1) / kTile;
  const int64_t HW = static_cast<int64_t>(H) * W;
  for (int64_t t = tile_lo; t < tile_hi; ++t) {
    const int tx = static_cast<int>(t % GX), ty = static_cast<int>(t / GX);
    const uint32_t* list = inst_gauss + ranges[2 * t];
    const int64_t len = static_cast<int64_t>(ranges[2 * t + 1]) - ranges[2 * t];
    for (int py = ty * kTile; py < std::min(H, (ty + 1) * kTile); ++py)
      for (int px = tx * kTile; px < std::min(W, (tx + 1) * kTile); ++px) {
        float out[3], Tf, Fo[5];
        int nc;
        composite_pixel_f32(px, py, list, len, sp.data(), fr.bg, out, Tf, Fo, nc);
        const int64_t o = static_cast<int64_t>(py) * W + px;
        for (int c = 0; c < 3; ++c) img[c * HW + o] = out[c];
        final_T[o] = Tf;
        n_contrib[o] = nc;
        if (depth_img) depth_img[o] = Fo[0];
        if (feat_img)
          for (int f = 0; f < 4; ++f) feat_img[f * HW + o] = Fo[1 + f];
      }
  }
}

// The decision margin (see composite_pixel_f32) of every pixel of the tiles
// [tile_lo, tile_hi): margin[H][W], untouched outside those tiles.
void orc_render_margin_f32(int64_t n, const float* xy, const float* conic_op, const float* rgb,
                           const int32_t* radius, int W, int H, const float* framev, const uint32_t* ranges,
                           const uint32_t* inst_gauss, int64_t tile_lo, int64_t tile_hi, float* margin,
                           int clamp_margin) {
  const Frame fr = make_frame(framev);
  const std::vector<Splat<float>> sp = load_splats(n, xy, conic_op, rgb, radius, nullptr);
  const int GX = (W + kTile - 1) / kTile;
  for (int64_t t = tile_lo; t < tile_hi; ++t) {
    const int tx = static_cast<int>(t % GX), ty = static_cast<int>(t / GX);
    const uint32_t* list = inst_gauss + ranges[2 * t];
    const int64_t len = static_cast<int64_t>(ranges[2 * t + 1]) - ranges[2 * t];
    for (int py = ty * kTile; py < std::min(H, (ty + 1) * kTile); ++py)
      for (int px = tx * kTile; px < std::min(W, (tx + 1) * kTile); ++px) {
        float out[3], Tf, Fo[5];
        int nc;
        composite_pixel_f32(px, py, list, len, sp.data(), fr.bg, out, Tf, Fo, nc,
                            &margin[static_cast<int64_t>(py) * W + px], clamp_margin != 0);
      }
  }
}

// Brute force (no tiles, no global sort): every visible Gaussian whose tile
// rectangle holds the pixel's tile, ordered by (depth bits, index).
void orc_render_bruteforce_f32(int64_t n, const float* xy, const float* depth, const float* conic_op,
                               const float* rgb, const int32_t* radius, const int32_t* rect, int W,
                               int H, const float* framev, float* img, float* final_T,
                               int32_t* n_contrib) {
  const Frame fr = make_frame(framev);
  const std::vector<Splat<float>> sp = load_splats(n, xy, conic_op, rgb, radius, nullptr);
  const int64_t HW = static_cast<int64_t>(H) * W;
  std::vector<std::pair<uint32_t, uint32_t>> cand;
  std::vector<uint32_t> list;
  for (int py = 0; py < H; ++py)
    for (int px = 0; px < W; ++px) {
      const int tx = px / kTile, ty = py / kTile;
      cand.clear();
      for (int64_t i = 0; i < n; ++i) {
        if (radius[i] <= 0) continue;
        if (tx < rect[4 * i] || tx >= rect[4 * i + 2] || ty < rect[4 * i + 1] || ty >= rect[4 * i + 3])
          continue;
        uint32_t bits;
        std::memcpy(&bits, &depth[i], 4);
        cand.push_back({bits, static_cast<uint32_t>(i)});
      }
      std::sort(cand.begin(), cand.end());
      list.clear();
      for (auto& c : cand) list.push_back(c.second);
      float out[3], Tf, Fo[5];
      int nc;
      composite_pixel_f32(px, py, list.data(), static_cast<int64_t>(list.size()), sp.data(), fr.bg, out,
                          Tf, Fo, nc);
      const int64_t o = static_cast<int64_t>(py) * W + px;
      for (int c = 0; c < 3; ++c) img[c * HW + o] = out[c];
      final_T[o] = Tf;
      n_contrib[o] = nc;
    }
}

// FP64 image with the discrete structure of the FP32 stage (radius, flags,
// sorted lists, per-pair skip/clamp/stop decisions from the FP32 splats).
// `arr` holds double* parameter arrays.  Returns sum over the rendered pixels
// of w[c][y][x] * img[c][y][x] (w may be null: returns 0); writes img/final_T
// if non-null.  tile_mask (GX*GY bytes) selects tiles; null = all.  wD and wT
// (optional, [H][W]) add sum wD * depth + sum wT * final_T to the returned
// value, wF (optional, [4][H][W]) sum wF * (velocity map, staticness map);
// depth_img / feat_img (optional) receive those channels.
double orc_render_f64(int64_t n, int degree, const void* const* arr, const float* camv, int W, int H,
                      const float* framev, const float* xy32, const float* conic_op32,
                      const int32_t* radius32, const uint32_t* flags32, const uint32_t* ranges,
                      const uint32_t* inst_gauss, const uint8_t* tile_mask, const double* w,
                      double* img, double* final_T, const double* wD, const double* wT, double* depth_img,
                      const double* wF, double* feat_img, const double* colour) {
  // colour (optional, [n][3]): per-Gaussian values composited in place of
  // the SH colour (a feature vector three channels at a time, Sec. 4.1)
  const Params prm = make_params(n, degree, arr);
  const Camera cam = make_cam(camv, W, H);
  const Frame fr = make_frame(framev);
  const std::vector<Splat<float>> dec = load_splats(n, xy32, conic_op32, nullptr, radius32, flags32);
  std::vector<Splat<double>> val(n);
  for (int64_t i = 0; i < n; ++i) {
    if (radius32[i] <= 0) { val[i].visible = false; continue; }
    Fixed fx{true, flags32[i]};
    preprocess_one<double>(prm, i, cam, fr, &fx, val[i], nullptr);
    if (colour)
      for (int c = 0; c < 3; ++c) val[i].rgb[c] = colour[3 * i + c];
  }
  const int GX = (W + kTile - 1) / kTile, GY = (H + kTile - 1) / kTile;
  const int64_t HW = static_cast<int64_t>(H) * W;
  double L = 0.0;
  for (int64_t t = 0; t < static_cast<int64_t>(GX) * GY; ++t) {
    if (tile_mask && !tile_mask[t]) continue;
    const int tx = static_cast<int>(t % GX), ty = static_cast<int>(t / GX);
    const uint32_t* list = inst_gauss + ranges[2 * t];
    const int64_t len = static_cast<int64_t>(ranges[2 * t + 1]) - ranges[2 * t];
    for (int py = ty * kTile; py < std::min(H, (ty + 1) * kTile); ++py)
      for (int px = tx * kTile; px < std::min(W, (tx + 1) * kTile); ++px) {
        double out[3], Tf, Fo[5];
        int nc;
        composite_pixel<double>(px, py, list, len, dec.data(), val.data(), fr.bg, out, Tf, Fo, nc, nullptr);
        const double Df = Fo[0];
        const int64_t o = static_cast<int64_t>(py) * W + px;
        for (int c = 0; c < 3; ++c) {
          if (img) img[c * HW + o] = out[c];
          if (w) L += w[c * HW + o] * out[c];
        }
        if (final_T) final_T[o] = Tf;
        if (depth_img) depth_img[o] = Df;
        if (wD) L += wD[o] * Df;
        if (wT) L += wT[o] * Tf;
        for (int f = 0; f < 4; ++f) {
          if (feat_img) feat_img[f * HW + o] = Fo[1 + f];
          if (wF) L += wF[f * HW + o] * Fo[1 + f];
        }
      }
  }
  return L;
}

// FP64 adjoint (O6, O7) of the image of orc_render_f64 for the upstream
// gradient dimg[3][H][W], plus (optional, [H][W]) dD for the blended depth
// channel and dT for final_T (the rendered opacity is 1 - final_T).  Writes
// the gradient of every parameter array into `garr` (9 double* in parameter
// layout, overwritten) and, if non-null, the per-Gaussian screen-space
// gradient g2d[n][14] = (d x, d y, d A, d B, d C, d o~, d r, d g, d b, d z,
// d v~ (3), d rho).  dF (optional, [4][H][W]): upstream gradient of the
// velocity and staticness maps.
void orc_backward_f64(int64_t n, int degree, const void* const* arr, const float* camv, int W, int H,
                      const float* framev, const float* xy32, const float* conic_op32,
                      const int32_t* radius32, const uint32_t* flags32, const uint32_t* ranges,
                      const uint32_t* inst_gauss, const double* dimg, void* const* garr, double* g2d_out,
                      const uint8_t* tile_mask, const double* dD, const double* dT, const double* dF,
                      const double* colour, const double* g2d_in, double* g2d_abs_out, void* const* mag_arr) {
  // colour (optional, [n][3]): as in orc_render_f64; the colour is then a
  // plain per-Gaussian value, so nothing flows into the SH or, through the
  // view direction, into the mean, and g2d[6..8] is its gradient.
  // g2d_in (optional, [n][14]): skip the compositing adjoint and apply the
  // chain rule to these screen-space gradients (the chain is linear in them).
  // g2d_abs_out (optional, [n][14]): the sum over the pixels of the absolute
  // value of every term added into each screen-space entry (with the
  // alpha-gradient's own terms taken in absolute value): the scale that the
  // rounding of a sum of those terms is relative to.  mag_arr (optional, with
  // g2d_abs_out; nine arrays shaped like garr): per parameter entry, that
  // scale carried through the chain rule in absolute value.
  const Params prm = make_params(n, degree, arr);
  const Camera cam = make_cam(camv, W, H);
  const Frame fr = make_frame(framev);
  const std::vector<Splat<float>> dec = load_splats(n, xy32, conic_op32, nullptr, radius32, flags32);
  std::vector<Splat<double>> val(n);
  std::vector<Inter<double>> inter(n);
  for (int64_t i = 0; i < n; ++i) {
    if (radius32[i] <= 0) { val[i].visible = false; continue; }
    Fixed fx{true, flags32[i]};
    preprocess_one<double>(prm, i, cam, fr, &fx, val[i], &inter[i]);
    if (colour)
      for (int c = 0; c < 3; ++c) val[i].rgb[c] = colour[3 * i + c];
  }
  const int GX = (W + kTile - 1) / kTile, GY = (H + kTile - 1) / kTile;
  const int64_t HW = static_cast<int64_t>(H) * W;
  std::vector<double> g2d(static_cast<size_t>(n) * kG2D, 0.0);
  std::vector<double> g2a(g2d_abs_out ? static_cast<size_t>(n) * kG2D : 0, 0.0);
  std::vector<Contrib<double>> rec;
  if (g2d_in) std::memcpy(g2d.data(), g2d_in, g2d.size() * sizeof(double));

  // O6: per pixel, the derivative of Eq. (3) with respect to each
  // contributor's alpha, colour, and through alpha its opacity, conic and mean.
  for (int64_t t = 0; !g2d_in && t < static_cast<int64_t>(GX) * GY; ++t) {
    // tile_mask (optional): tiles left out must carry a zero dimg, so they add nothing
    if (tile_mask && !tile_mask[t]) continue;
    const int tx = static_cast<int>(t % GX), ty = static_cast<int>(t / GX);
    const uint32_t* list = inst_gauss + ranges[2 * t];
    const int64_t len = static_cast<int64_t>(ranges[2 * t + 1]) - ranges[2 * t];
    for (int py = ty * kTile; py < std::min(H, (ty + 1) * kTile); ++py)
      for (int px = tx * kTile; px < std::min(W, (tx + 1) * kTile); ++px) {
        rec.clear();
        double out[3], Tf, Fo[5];
        int nc;
        composite_pixel<double>(px, py, list, len, dec.data(), val.data(), fr.bg, out, Tf, Fo, nc, &rec);
        const int64_t o = static_cast<int64_t>(py) * W + px;
        const double g[3] = {dimg[o], dimg[HW + o], dimg[2 * HW + o]};
        const double gD = dD ? dD[o] : 0.0, gT = dT ? dT[o] : 0.0;
        // S = colour accumulated behind the current contributor, incl. background;
        // SD the same for depth (no background term); final_T = prod (1 - alpha)
        double S[3] = {Tf * fr.bg[0], Tf * fr.bg[1], Tf * fr.bg[2]};
        double SD = 0.0;
        double gF[4], SF[4] = {0.0, 0.0, 0.0, 0.0};
        for (int f = 0; f < 4; ++f) gF[f] = dF ? dF[f * HW + o] : 0.0;
        for (int64_t k = static_cast<int64_t>(rec.size()) - 1; k >= 0; --k) {
          const Contrib<double>& c = rec[k];
          const Splat<double>& v = val[c.g];
          double* gg = &g2d[kG2D * static_cast<size_t>(c.g)];
          double dalpha = 0.0, dabs = 0.0;
          for (int ch = 0; ch < 3; ++ch) {
            gg[6 + ch] += c.T * c.alpha * g[ch];
            dalpha += g[ch] * (c.T * v.rgb[ch] - S[ch] / (1.0 - c.alpha));
            dabs += std::fabs(g[ch]) * (std::fabs(c.T * v.rgb[ch]) + std::fabs(S[ch] / (1.0 - c.alpha)));
          }
          gg[9] += c.T * c.alpha * gD;
          dalpha += gD * (c.T * v.depth - SD / (1.0 - c.alpha));
          dalpha += gT * (-Tf / (1.0 - c.alpha));
          dabs += std::fabs(gD) * (std::fabs(c.T * v.depth) + std::fabs(SD / (1.0 - c.alpha))) +
                  std::fabs(gT * Tf / (1.0 - c.alpha));
          for (int f = 0; f < 4; ++f) {
            gg[10 + f] += c.T * c.alpha * gF[f];
            dalpha += gF[f] * (c.T * v.feat[f] - SF[f] / (1.0 - c.alpha));
            dabs += std::fabs(gF[f]) * (std::fabs(c.T * v.feat[f]) + std::fabs(SF[f] / (1.0 - c.alpha)));
          }
          if (g2d_abs_out) {
            double* ga = &g2a[kG2D * static_cast<size_t>(c.g)];
            for (int ch = 0; ch < 3; ++ch) ga[6 + ch] += std::fabs(c.T * c.alpha * g[ch]);
            ga[9] += std::fabs(c.T * c.alpha * gD);
            for (int f = 0; f < 4; ++f) ga[10 + f] += std::fabs(c.T * c.alpha * gF[f]);
            if (!c.clamped) {
              const double ap = c.alpha * dabs;
              ga[5] += c.G * dabs;
              ga[2] += 0.5 * c.dx * c.dx * ap;
              ga[3] += std::fabs(c.dx * c.dy) * ap;
              ga[4] += 0.5 * c.dy * c.dy * ap;
              ga[0] += (std::fabs(v.A * c.dx) + std::fabs(v.B * c.dy)) * ap;
              ga[1] += (std::fabs(v.B * c.dx) + std::fabs(v.C * c.dy)) * ap;
            }
          }
          for (int ch = 0; ch < 3; ++ch) S[ch] += c.T * c.alpha * v.rgb[ch];
          SD += c.T * c.alpha * v.depth;
          for (int f = 0; f < 4; ++f) SF[f] += c.T * c.alpha * v.feat[f];
          if (c.clamped) continue;
          gg[5] += c.G * dalpha;
          const double gp = c.alpha * dalpha;  // d alpha / d power = alpha
          gg[2] += -0.5 * c.dx * c.dx * gp;
          gg[3] += -c.dx * c.dy * gp;
          gg[4] += -0.5 * c.dy * c.dy * gp;
          gg[0] += -(v.A * c.dx + v.B * c.dy) * gp;
          gg[1] += -(v.B * c.dx + v.C * c.dy) * gp;
        }
      }
  }
  if (g2d_out) std::memcpy(g2d_out, g2d.data(), g2d.size() * sizeof(double));
  if (g2d_abs_out) std::memcpy(g2d_abs_out, g2a.data(), g2a.size() * sizeof(double));

  // O7: chain rule back to the per-point parameters.
  const int K = (degree + 1) * (degree + 1);
  double* gmu = static_cast<double*>(garr[0]);
  double* gs = static_cast<double*>(garr[1]);
  double* gq = static_cast<double*>(garr[2]);
  double* gsh = static_cast<double*>(garr[3]);
  double* go = static_cast<double*>(garr[4]);
  double* gv = static_cast<double*>(garr[5]);
  double* gl = static_cast<double*>(garr[6]);
  double* gtau = static_cast<double*>(garr[7]);
  double* gbeta = static_cast<double*>(garr[8]);
  for (int r = 0; r < 3; ++r)
    for (int64_t i = 0; i < n; ++i) { gmu[r * n + i] = 0; gs[r * n + i] = 0; gv[r * n + i] = 0; }
  for (int r = 0; r < 4; ++r) for (int64_t i = 0; i < n; ++i) gq[r * n + i] = 0;
  for (int r = 0; r < 3 * K; ++r) for (int64_t i = 0; i < n; ++i) gsh[r * n + i] = 0;
  for (int64_t i = 0; i < n; ++i) { go[i] = 0; gl[i] = 0; gtau[i] = 0; gbeta[i] = 0; }

  double Wm[9];
  for (int c = 0; c < 9; ++c) Wm[c] = cam.R[c];
  const double fx = cam.fx, fy = cam.fy;
  // the chain rule of Gaussian i from its screen-space gradient gg; put(field,
  // row, value) receives each parameter-gradient entry (fields in the order
  // mu, scale, rot, sh, opacity, vel, period, tau, beta)
  auto chain = [&](int64_t i, const double* gg, auto&& put) {
    const Inter<double>& it = inter[i];
    const Splat<double>& v = val[i];
    double dmur[3] = {0, 0, 0};

    // colour: rgb = max(0, sum_k sh_k Y_k(dir) + 1/2)
    double ddir[3] = {0, 0, 0};
    for (int ch = 0; ch < 3 && !colour; ++ch) {
      const bool clamp = (v.flags & (kShClampR << ch)) != 0;
      const double draw = clamp ? 0.0 : gg[6 + ch];
      for (int k = 0; k < K; ++k) {
        put(3, 3 * k + ch, it.Y[k] * draw);
        const double shv = static_cast<const double*>(prm.sh)[(3 * k + ch) * n + i];
        for (int c = 0; c < 3; ++c) ddir[c] += shv * draw * it.dY[k][c];
      }
    }
    const double dd = it.dir[0] * ddir[0] + it.dir[1] * ddir[1] + it.dir[2] * ddir[2];
    for (int c = 0; c < 3; ++c) dmur[c] += (ddir[c] - it.dir[c] * dd) / it.ulen;

    // conic (A,B,C) = inverse of S = [[a,b],[b,c]]: dL/dS = -Q G Q with
    // G = [[dA, dB/2], [dB/2, dC]] (B sits in both off-diagonal slots)
    const double Q[4] = {v.A, v.B, v.B, v.C};
    const double G[4] = {gg[2], 0.5 * gg[3], 0.5 * gg[3], gg[4]};
    double QG[4], dS[4];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) QG[2 * r + c] = Q[2 * r] * G[c] + Q[2 * r + 1] * G[2 + c];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) dS[2 * r + c] = -(QG[2 * r] * Q[c] + QG[2 * r + 1] * Q[2 + c]);
    // the 0.3 dilation passes the gradient through unchanged.
    // Sigma' = T2 Sigma T2^T  ->  dSigma = T2^T dS T2,  dT2 = 2 dS T2 Sigma
    double dSig[9], dT2[6], dST[6];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) dST[3 * r + c] = dS[2 * r] * it.T2[c] + dS[2 * r + 1] * it.T2[3 + c];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) dSig[3 * r + c] = it.T2[r] * dST[c] + it.T2[3 + r] * dST[3 + c];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0;
        for (int k = 0; k < 3; ++k) acc += dST[3 * r + k] * it.Sig[3 * k + c];
        dT2[3 * r + c] = 2.0 * acc;
      }
    // T2 = J W: dJ = dT2 W^T (only J00, J02, J11, J12 are variables)
    double dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
    for (int c = 0; c < 3; ++c) {
      dJ00 += dT2[c] * Wm[c];
      dJ02 += dT2[c] * Wm[6 + c];
      dJ11 += dT2[3 + c] * Wm[3 + c];
      dJ12 += dT2[3 + c] * Wm[6 + c];
    }
    const double px = it.p[0], py = it.p[1], pz = it.p[2];
    double dp[3] = {0, 0, 0};
    dp[2] += -fx / (pz * pz) * dJ00 - fy / (pz * pz) * dJ11;
    if (v.flags & (kGuardXLo | kGuardXHi)) {
      const double cl = it.tx / pz;  // J02 = -fx cl / pz
      dp[2] += fx * cl / (pz * pz) * dJ02;
    } else {
      dp[0] += -fx / (pz * pz) * dJ02;
      dp[2] += 2.0 * fx * px / (pz * pz * pz) * dJ02;
    }
    if (v.flags & (kGuardYLo | kGuardYHi)) {
      const double cl = it.ty / pz;
      dp[2] += fy * cl / (pz * pz) * dJ12;
    } else {
      dp[1] += -fy / (pz * pz) * dJ12;
      dp[2] += 2.0 * fy * py / (pz * pz * pz) * dJ12;
    }
    // the depth channel's z is the camera-space pz
    dp[2] += gg[9];
    // 2D mean m = (fx px/pz + cx - 1/2, fy py/pz + cy - 1/2)
    dp[0] += fx / pz * gg[0];
    dp[1] += fy / pz * gg[1];
    dp[2] += -fx * px / (pz * pz) * gg[0] - fy * py / (pz * pz) * gg[1];
    for (int c = 0; c < 3; ++c) dmur[c] += Wm[c] * dp[0] + Wm[3 + c] * dp[1] + Wm[6 + c] * dp[2];

    // Sigma = M M^T, M = R(q^) diag(s)
    double dM[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0;
        for (int k = 0; k < 3; ++k) acc += dSig[3 * r + k] * it.M[3 * k + c];
        dM[3 * r + c] = 2.0 * acc;
      }
    double dR[9];
    for (int c = 0; c < 3; ++c) {
      double acc = 0;
      for (int r = 0; r < 3; ++r) acc += dM[3 * r + c] * it.Rq[3 * r + c];
      put(1, c, acc);
      for (int r = 0; r < 3; ++r) dR[3 * r + c] = dM[3 * r + c] * it.s[c];
    }
    // R(q^) -> q^
    const double w = it.qn[0], x = it.qn[1], y = it.qn[2], z = it.qn[3];
    // partial derivatives of the nine entries, columns (w, x, y, z)
    const double dRdq[9][4] = {
        {0, 0, -4 * y, -4 * z},    {-2 * z, 2 * y, 2 * x, -2 * w}, {2 * y, 2 * z, 2 * w, 2 * x},
        {2 * z, 2 * y, 2 * x, 2 * w}, {0, -4 * x, 0, -4 * z},      {-2 * x, -2 * w, 2 * z, 2 * y},
        {-2 * y, 2 * z, -2 * w, 2 * x}, {2 * x, 2 * w, 2 * z, 2 * y}, {0, -4 * x, -4 * y, 0}};
    double dqn[4] = {0, 0, 0, 0};
    for (int e = 0; e < 9; ++e)
      for (int c = 0; c < 4; ++c) dqn[c] += dR[e] * dRdq[e][c];
    const double qd = w * dqn[0] + x * dqn[1] + y * dqn[2] + z * dqn[3];
    for (int c = 0; c < 4; ++c) put(2, c, (dqn[c] - it.qn[c] * qd) / it.qnorm);

    // flow translation (Eqs. (10), (12)): mu_r = mu~ + v e dt, e = exp(-beta/(2l))
    double dl = 0, dtau = 0, dbeta = 0;
    double dv[3] = {0, 0, 0};
    const double dt = fr.dt;
    if (dt != 0.0) {
      const double vd = it.v[0] * dmur[0] + it.v[1] * dmur[1] + it.v[2] * dmur[2];
      if (fr.mode == 0) {
        const double e = std::exp(-0.5 * it.beta / it.l);
        for (int c = 0; c < 3; ++c) dv[c] += e * dt * dmur[c];
        dbeta += vd * dt * e * (-0.5 / it.l);
        dl += vd * dt * e * (0.5 * it.beta / (it.l * it.l));
      } else {
        for (int c = 0; c < 3; ++c) dv[c] += dt * dmur[c];
      }
    }
    // vibration (Eq. (6)): mu~ = mu + k v, k = (l / 2pi) sin(2pi (t - tau) / l)
    const double del = static_cast<double>(fr.t) - it.tau;
    const double phi = 2.0 * kPi * del / it.l;
    const double k = it.l / (2.0 * kPi) * std::sin(phi);
    const double vg = it.v[0] * dmur[0] + it.v[1] * dmur[1] + it.v[2] * dmur[2];
    for (int c = 0; c < 3; ++c) {
      put(0, c, dmur[c]);
      dv[c] += k * dmur[c];
    }
    dtau += -std::cos(phi) * vg;
    dl += (std::sin(phi) / (2.0 * kPi) - del / it.l * std::cos(phi)) * vg;
    // velocity map: v~ = v e, e = exp(-beta/(2l)); staticness rho = beta / l
    {
      const double e = std::exp(-0.5 * it.beta / it.l);
      double vdot = 0.0;
      for (int c = 0; c < 3; ++c) {
        dv[c] += e * gg[10 + c];
        vdot += it.v[c] * gg[10 + c];
      }
      dbeta += vdot * e * (-0.5 / it.l) + gg[13] / it.l;
      dl += vdot * e * (0.5 * it.beta / (it.l * it.l)) - gg[13] * it.beta / (it.l * it.l);
      for (int c = 0; c < 3; ++c) put(5, c, dv[c]);
    }
    // opacity decay (Eq. (7)): o~ = o exp(-(t - tau)^2 / (2 beta^2))
    const double eo = std::exp(-0.5 * (del / it.beta) * (del / it.beta));
    const double dop = gg[5];
    put(4, 0, eo * dop);
    dtau += dop * v.op * del / (it.beta * it.beta);
    dbeta += dop * v.op * del * del / (it.beta * it.beta * it.beta);
    put(6, 0, dl);
    put(7, 0, dtau);
    put(8, 0, dbeta);
  };
  for (int64_t i = 0; i < n; ++i) {
    if (!val[i].visible) continue;
    chain(i, &g2d[kG2D * static_cast<size_t>(i)],
          [&](int f, int r, double x) { static_cast<double*>(garr[f])[r * n + i] = x; });
  }
  // the magnitude of each entry's terms: the chain's Jacobian column of every
  // screen-space entry, in absolute value, times that entry's absolute sum
  if (mag_arr && g2d_abs_out) {
    for (int f = 0; f < 9; ++f) {
      const int rows = f == 3 ? 3 * K : (f == 2 ? 4 : (f == 0 || f == 1 || f == 5) ? 3 : 1);
      std::fill(static_cast<double*>(mag_arr[f]), static_cast<double*>(mag_arr[f]) + rows * n, 0.0);
    }
    for (int64_t i = 0; i < n; ++i) {
      if (!val[i].visible) continue;
      const double* ga = &g2a[kG2D * static_cast<size_t>(i)];
      for (int k = 0; k < kG2D; ++k) {
        if (!(ga[k] > 0.0)) continue;
        double e[kG2D] = {};
        e[k] = 1.0;
        chain(i, e, [&](int f, int r, double x) {
          static_cast<double*>(mag_arr[f])[r * n + i] += std::fabs(x) * ga[k];
        });
      }
    }
  }
}

// Small pieces exposed for the closed-form pins.
void orc_temporal_f64(const double* mu, const double* v, double l, double tau, double beta, double o,
                      double t, double dt, int mode, double* mu_r, double* op) {
  temporal<double>(mu, v, l, tau, beta, o, t, dt, mode, mu_r, *op);
}

void orc_sh_basis_f64(int degree, const double* dir, double* Y, double* dY) {
  double y[16], dy[16][3];
  sh_basis<double>(degree, dir, y, dy);
  const int K = (degree + 1) * (degree + 1);
  for (int k = 0; k < K; ++k) {
    Y[k] = y[k];
    if (dY)
      for (int c = 0; c < 3; ++c) dY[3 * k + c] = dy[k][c];
  }
}

// Projection of one FP64 Gaussian (for the EWA Jacobian pin): returns the
// 2D mean m, the Jacobian entries (J00, J02, J11, J12) and the dilated 2D
// covariance (a, b, c) of the point mu with scale s and rotation q seen by cam.
int orc_project_f64(const double* mu, const double* s, const double* q, const float* camv, int W, int H,
                    double* m, double* J, double* cov) {
  // degree 0: the SH array holds one coefficient per colour channel
  double zero3[3] = {0, 0, 0}, one = 1.0, tau = 0.0, beta = 1.0, l = 1.0, o = 1.0, sh[3] = {0, 0, 0};
  const void* arr[9] = {mu, s, q, sh, &o, zero3, &l, &tau, &beta};
  const Params prm = make_params(1, 0, arr);
  (void)one;
  const Camera cam = make_cam(camv, W, H);
  const float fv[6] = {0, 0, 0, 0, 0, 0};
  const Frame fr = make_frame(fv);
  Splat<double> sp;
  Inter<double> it;
  Fixed fx{true, 0};
  preprocess_one<double>(prm, 0, cam, fr, &fx, sp, &it);
  m[0] = sp.x; m[1] = sp.y;
  J[0] = it.J00; J[1] = it.J02; J[2] = it.J11; J[3] = it.J12;
  cov[0] = it.S2[0]; cov[1] = it.S2[1]; cov[2] = it.S2[2];
  return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Sky (Sec. 3.4, sky refinement): C_f = C + (1 - O) f_sky(d), with f_sky a
// learnable cube map looked up in the pixel's viewing direction d, here taken
// through the pixel centre moved by an optional jitter (the paper perturbs d
// within the unit pixel while training); the lookup geometry in FP32, the
// blend in FP64.  Conventions taken here (the
// paper fixes none): d_cam = ((px + 0.5 + jx - cx) / fx, (py + 0.5 + jy - cy)
// / fy, 1), d = R^T d_cam in the world frame; faces +X, -X, +Y, -Y, +Z, -Z
// (0..5) chosen by the largest |d_i| (ties to the lower axis); face
// coordinates as in OpenGL cube maps; texel (x, y) = (u R - 1/2, v R - 1/2)
// sampled bilinearly with the coordinates clamped to [0, R - 1] inside the
// face; cube layout [6][3][R][R] (face, channel, row v, column u).
namespace sky {
// The lookup geometry (direction, face, face coordinates, texel taps) is
// evaluated in FP32, the precision in which the renderer takes the face and
// texel decisions; only the blend is accumulated in FP64.
template <class R>
void face_uv(const R d[3], int& face, R& u, R& v) {
  const R ax = std::fabs(d[0]), ay = std::fabs(d[1]), az = std::fabs(d[2]);
  R sc, tc, ma;
  if (ax >= ay && ax >= az) {
    ma = ax;
    if (d[0] >= 0) { face = 0; sc = -d[2]; tc = -d[1]; } else { face = 1; sc = d[2]; tc = -d[1]; }
  } else if (ay >= az) {
    ma = ay;
    if (d[1] >= 0) { face = 2; sc = d[0]; tc = d[2]; } else { face = 3; sc = d[0]; tc = -d[2]; }
  } else {
    ma = az;
    if (d[2] >= 0) { face = 4; sc = d[0]; tc = -d[1]; } else { face = 5; sc = -d[0]; tc = -d[1]; }
  }
  u = R(0.5) * (sc / ma + R(1));
  v = R(0.5) * (tc / ma + R(1));
}

// the four texels (face-local flat indices) and weights of the bilinear lookup
void taps(int Rn, float u, float v, int idx[4], double w[4]) {
  float x = u * static_cast<float>(Rn) - 0.5f, y = v * static_cast<float>(Rn) - 0.5f;
  x = std::min(std::max(x, 0.0f), static_cast<float>(Rn - 1));
  y = std::min(std::max(y, 0.0f), static_cast<float>(Rn - 1));
  const int x0 = static_cast<int>(std::floor(x)), y0 = static_cast<int>(std::floor(y));
  const int x1 = std::min(x0 + 1, Rn - 1), y1 = std::min(y0 + 1, Rn - 1);
  const float fx = x - static_cast<float>(x0), fy = y - static_cast<float>(y0);
  idx[0] = y0 * Rn + x0; w[0] = (1.0f - fx) * (1.0f - fy);
  idx[1] = y0 * Rn + x1; w[1] = fx * (1.0f - fy);
  idx[2] = y1 * Rn + x0; w[2] = (1.0f - fx) * fy;
  idx[3] = y1 * Rn + x1; w[3] = fx * fy;
}

void direction(const Camera& cam, int px, int py, const float* jitter, int64_t HW, int64_t o, float d[3]) {
  const float jx = jitter ? jitter[o] : 0.0f, jy = jitter ? jitter[HW + o] : 0.0f;
  const float c[3] = {((static_cast<float>(px) + 0.5f) + jx - cam.cx) / cam.fx,
                      ((static_cast<float>(py) + 0.5f) + jy - cam.cy) / cam.fy, 1.0f};
  for (int k = 0; k < 3; ++k) d[k] = (cam.R[k] * c[0] + cam.R[3 + k] * c[1]) + cam.R[6 + k] * c[2];
}
}  // namespace sky

extern "C" {
// out[3][H][W] = img + (1 - opac) * f_sky(d) in FP64; inputs [3][H][W], [H][W].
void orc_sky_f64(const double* img, const double* opac, const double* cube, int R, const float* camv, int W, int H,
                 const float* jitter, double* out) {
  const Camera cam = make_cam(camv, W, H);
  const int64_t HW = static_cast<int64_t>(H) * W, F = static_cast<int64_t>(R) * R;
  for (int py = 0; py < H; ++py)
    for (int px = 0; px < W; ++px) {
      const int64_t o = static_cast<int64_t>(py) * W + px;
      float d[3], u, v;
      double w[4];
      int face, idx[4];
      sky::direction(cam, px, py, jitter, HW, o, d);
      sky::face_uv<float>(d, face, u, v);
      sky::taps(R, u, v, idx, w);
      for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s += w[k] * cube[(face * 3 + c) * F + idx[k]];
        out[c * HW + o] = img[c * HW + o] + (1.0 - opac[o]) * s;
      }
    }
}

// Adjoint of orc_sky_f64 for dL/dout = g: dL/dopac [H][W] (overwritten) and
// dL/dcube [6][3][R][R] (overwritten); dL/dimg is g itself.
void orc_sky_bwd_f64(const double* g, const double* opac, const double* cube, int R, const float* camv, int W, int H,
                     const float* jitter, double* dopac, double* dcube) {
  const Camera cam = make_cam(camv, W, H);
  const int64_t HW = static_cast<int64_t>(H) * W, F = static_cast<int64_t>(R) * R;
  for (int64_t k = 0; k < 6 * 3 * F; ++k) dcube[k] = 0.0;
  for (int py = 0; py < H; ++py)
    for (int px = 0; px < W; ++px) {
      const int64_t o = static_cast<int64_t>(py) * W + px;
      float d[3], u, v;
      double w[4];
      int face, idx[4];
      sky::direction(cam, px, py, jitter, HW, o, d);
      sky::face_uv<float>(d, face, u, v);
      sky::taps(R, u, v, idx, w);
      double dO = 0.0;
      for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) {
          s += w[k] * cube[(face * 3 + c) * F + idx[k]];
          dcube[(face * 3 + c) * F + idx[k]] += w[k] * (1.0 - opac[o]) * g[c * HW + o];
        }
        dO -= s * g[c * HW + o];
      }
      dopac[o] = dO;
    }
}

// The face and face coordinates of a world direction, in FP32 as the
// composite takes them (for the pins).
void orc_sky_face_uv(const double* d, int* face, double* uv) {
  const float df[3] = {static_cast<float>(d[0]), static_cast<float>(d[1]), static_cast<float>(d[2])};
  float u, v;
  sky::face_uv<float>(df, *face, u, v);
  uv[0] = u;
  uv[1] = v;
}
}
