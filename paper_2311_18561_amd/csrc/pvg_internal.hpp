// Internal declarations shared by the HIP kernels and the host code of libpvg.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "pvg.h"

namespace pvg {

constexpr int kTile = 16;
constexpr int kTilePixels = kTile * kTile;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kDilation = 0.3f;        // low-pass added to the 2D covariance (px^2)
constexpr float kLambdaFloor = 0.1f;     // floor under the eigenvalue discriminant
constexpr float kGuard = 1.3f;           // Jacobian guard band, in half fields of view
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 0.0001f;
constexpr int kRecFloats = 14;  // floats per adjoint record slot: 9 screen-space sums + 5 channel sums
constexpr int kG2DStride = 16;           // floats per Gaussian in the screen-space gradient buffer

// Parameters of one scene (device pointers).
struct Scene {
  const float* mu; const float* scale; const float* rot; const float* sh; const float* opacity;
  const float* vel; const float* period; const float* tau; const float* beta;
  int64_t n;
  int32_t degree;
};

// One rendered view: scene, camera, frame, its tile grid and its place in a batch.
struct View {
  Scene s;
  float R[9], T[3];
  float fx, fy, cx, cy, znear;
  int32_t W, H, GX, GY;
  float t, dt;
  int32_t mode;
  float bg[3];
  int64_t geom_off;  // first slot of this view's Gaussians in the batch's geom arrays
  int64_t tile_off;  // first global tile id of this view
  float* img;        // [3][H][W]
  float* final_T;    // [H][W]
  int32_t* n_contrib;// [H][W]
  const float* dL_dimg;  // [3][H][W] upstream gradient (adjoint only)
  // flexible rendering channels (Sec. 3.1), each optional: the blended camera
  // depth sum T alpha z (forward output) and the upstream gradients of it and
  // of final_T (adjoint inputs; the rendered opacity is 1 - final_T)
  float* depth_img;          // [H][W]
  const float* dL_ddepth;    // [H][W]
  const float* dL_dT;        // [H][W]
  float* vbar_img;           // [3][H][W] velocity map
  float* rho_img;            // [H][W] staticness map
  const float* dL_dvbar;     // [3][H][W]
  const float* dL_drho;      // [H][W]
  // depth_img holds sum T alpha z / sum T alpha (forward output; the adjoint
  // reads it back to take the quotient's gradient)
  int32_t depth_norm;
  // the rendered opacity O = sum T alpha = 1 - final_T (forward output) and
  // its upstream gradient (adjoint input), each optional
  float* opacity_img;        // [H][W]
  const float* dL_dO;        // [H][W]
};

struct Geom {
  float* xy; float* depth; float* conic_op; float* rgb; int32_t* radius; uint32_t* tiles;
  float* feat;  // [n][4] optional: mean velocity v~ and staticness rho
};

// Views of a launch: either one view passed by value or a device table.
// Batched launches read their live totals from device memory (`live`:
// Gaussians, tiles, views), so one captured graph serves any batch that fits
// its grid bounds total_gauss / total_tiles.
struct ViewSet {
  const View* table;    // device table of views (batched launches), or null
  const int64_t* live;  // device [3]: live Gaussians, tiles, views (batched), or null
  View one;             // the view when table is null
  int32_t nviews;       // views (single: 1; batched: table capacity)
  int64_t total_gauss;  // sum of the views' n (batched: grid bound)
  int64_t total_tiles;  // sum of the views' GX * GY (batched: grid bound)
};

#ifdef __HIPCC__
__device__ __forceinline__ int64_t live_gauss(const ViewSet& vs) { return vs.live ? vs.live[0] : vs.total_gauss; }
__device__ __forceinline__ int64_t live_tiles(const ViewSet& vs) { return vs.live ? vs.live[1] : vs.total_tiles; }
__device__ __forceinline__ int32_t live_views(const ViewSet& vs) {
  return vs.live ? static_cast<int32_t>(vs.live[2]) : vs.nviews;
}
__device__ __forceinline__ const View& view_at(const ViewSet& vs, int32_t v) { return vs.table ? vs.table[v] : vs.one; }
// the view holding global Gaussian slot g (views are laid out back to back)
__device__ __forceinline__ int32_t view_of_gauss(const ViewSet& vs, int64_t g) {
  if (!vs.table) return 0;
  int32_t lo = 0, hi = live_views(vs) - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (vs.table[mid].geom_off <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}
__device__ __forceinline__ int32_t view_of_tile(const ViewSet& vs, int64_t tile) {
  if (!vs.table) return 0;
  int32_t lo = 0, hi = live_views(vs) - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (vs.table[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}
#endif

// ---------------------------------------------------------------- host side
// error handling (thread-local message)
void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
#define PVG_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return ::pvg::hip_fail(e_, #call); \
  } while (0)

// validation and view construction (api.cpp)
bool check_gaussians(const pvg_gaussians* g);
bool check_camera(const pvg_camera* c);
View make_view(const pvg_gaussians* g, const pvg_camera* c, const pvg_frame* f);

// stage profiler
struct StageScope {
  StageScope(int stage, hipStream_t s);
  ~StageScope();
  int stage_;
  hipStream_t s_;
  bool on_;
};
bool profiling();
unsigned long long* profile_work_counter(int stage);  // device counter, or null when off

// kernel launchers (stream-ordered, no host sync)
hipError_t launch_preprocess(const ViewSet& vs, const Geom& geom, hipStream_t s);
// Views of one set of Gaussians for the per-Gaussian adjoint (same scene and
// the same render time t in every view): each view's camera and frame, its
// radii (visibility) and its screen-space gradient g2d [n][kG2DStride].
constexpr int kMaxBwdViews = 8;
struct BwdViews {
  int32_t nv;
  View views[kMaxBwdViews];
  const int32_t* radius[kMaxBwdViews];
  const float* rgb[kMaxBwdViews];  // the forward's colours (clamped channels are -0)
  float* g2d[kMaxBwdViews];  // the adjoint also leaves per-view scratch values in slots 6..11
  // non-null: the view composited three channels of a per-Gaussian feature
  // in place of the colour; their gradient is added here ([3][n]) and the
  // colour's SH and view-direction chain is skipped
  float* feat_grad[kMaxBwdViews];
  // true: the view composited a feature vector and no colour at all (g2d
  // slots 6..11 unused); the colour's SH and view-direction chain is skipped
  bool no_colour[kMaxBwdViews];
};
hipError_t launch_preprocess_bwd(const BwdViews& pk, const pvg_gaussians_grad& grad, int accumulate,
                                 hipStream_t s);
// Forward records of up to kMaxBwdViews views of one set of Gaussians (each
// view's geom holds slots 0..n-1).
struct PreViews {
  int32_t nv;
  View views[kMaxBwdViews];
  Geom geoms[kMaxBwdViews];
};
hipError_t launch_preprocess_views(const PreViews& pk, hipStream_t s);
// sky composite (Sec. 3.4): out = img + (1 - opac) f_sky(d) and its adjoint
hipError_t launch_sky(const pvg_camera* cam, const float* img, const float* opac, const float* cube, int Rn,
                      const float* jitter, float* out, hipStream_t s);
// deterministic: the texel-block gather (the same cube gradient on every run)
// instead of the pixel-tile scatter, whose float atomics add in any order
hipError_t launch_sky_bwd(const pvg_camera* cam, const float* g, const float* opac, const float* cube, int Rn,
                          const float* jitter, float* dopac, float* dcube, bool deterministic, hipStream_t s);
// culled: the lists hold only tiles that pass tile_reachable (the render skips the test)
hipError_t launch_render_fwd(const ViewSet& vs, const Geom& geom, const uint32_t* vals,
                             const uint32_t* ranges, bool culled, hipStream_t s);
// The sorted lists as the adjoint reads them.  Rectangle lists: a pair's
// record is first[g] + its tile's row-major index in the rectangle.  Culled
// lists: rows[row_base[g] + ty].x + (tx - first reached column).
struct Lists {
  const uint32_t* vals;
  const uint32_t* ranges;
  const uint32_t* first;
  bool culled;
  const uint2* rows;
  const uint32_t* row_base;
  int64_t capacity;  // record slots; indices outside are never read or written
};
// adjoint of compositing: per-(Gaussian, tile) records, then their per-Gaussian sums into g2d
hipError_t launch_render_bwd(const ViewSet& vs, const Geom& geom, const Lists& lists, float* rec, uint8_t* vis,
                             int64_t vis_bytes, float* g2d, hipStream_t s);
// N-channel feature compositing (Sec. 4.1's per-Gaussian vectors through
// Eq. (3)) of one view: out [nch][H][W] and the view's final_T / n_contrib;
// feat [n][ld], channels c < nch used (1 <= nch <= kMaxFeatureChannels)
constexpr int kMaxFeatureChannels = 32;
int feature_width(int nch);  // channels a record carries: nch rounded up to a kernel width
hipError_t launch_feature_fwd(const ViewSet& vs, const Geom& geom, const uint32_t* vals, const uint32_t* ranges,
                              bool culled, const float* feat, int64_t ld, int nch, float* out, hipStream_t s);
// its adjoint for one view: records [capacity][8 + feature_width(nch)], then per
// visible Gaussian the screen-space sums into g2d and the feature sums added
// into feat_grad [n][ld]
hipError_t launch_feature_bwd(const ViewSet& vs, const Geom& geom, const Lists& lists, const float* feat, int64_t ld,
                              int nch, const float* dout, float* rec, uint8_t* vis, int64_t vis_bytes, float* g2d,
                              float* feat_grad, hipStream_t s);
// scratch of the adjoint: g2d [views][n][12] | regions x (rec [capacity][9] | vis [capacity] bytes, padded);
// one region per view adjoint that runs concurrently (at most kBwdStreams)
constexpr int kBwdStreams = 3;
size_t bwd_scratch_bytes(int64_t n, int32_t views, int32_t regions, int64_t capacity, size_t* off_rec,
                         size_t* off_vis, size_t* vis_bytes, size_t* slot_bytes, size_t* region_bytes);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
// Adaptive control (Sec. 3.3): thresholds of one densify/prune pass.
struct DensifyCfg {
  float grad_threshold, radius, clone_scale, prune_scale, min_opacity, scale_decay, beta_decay;
};
// Writable parameter arrays of the pass's output (n = its Gaussian count).
struct SceneOut {
  float* mu; float* scale; float* rot; float* sh; float* opacity;
  float* vel; float* period; float* tau; float* beta;
  int64_t n;
  int32_t degree;
};
size_t densify_tmp_bytes(int64_t n);
// Adam over the parameter rows (learning rates: mu, scale, rot, SH degree 0,
// SH higher degrees, opacity, vel, period, tau, beta); bc1 = 1 - beta1^t,
// bc2 = 1 - beta2^t.
struct AdamCfg {
  float lr[10];
  float beta1, beta2, eps, bc1, bc2;
};
hipError_t launch_adam_dense(float* p, const float* g, float* m, float* v, int64_t count, float lr, const AdamCfg& c,
                             hipStream_t st);
hipError_t launch_adam(const SceneOut& s, const pvg_gaussians_grad& g, float* m, float* v, const AdamCfg& c,
                       hipStream_t st);
hipError_t launch_opacity_reset(float* o, float* m_row, float* v_row, int64_t n, float cap, hipStream_t st);
// SSIM (11 x 11 Gaussian window, sigma 1.5): map and saved partials [3][C][H][W]; adjoint into dx
// L1 loss scale * sum |a - b| over n floats and its gradient scale * sign(a - b)
// (grad may be null); partials: kL1Blocks floats of scratch
constexpr int kL1Blocks = 1024;
hipError_t launch_l1(const float* a, const float* b, int64_t n, float scale, float* loss, float* grad,
                     float* partials, hipStream_t s);
hipError_t launch_ssim_fwd(const float* x, const float* y, int C, int H, int W, float* smap, float* part,
                           hipStream_t st);
hipError_t launch_ssim_bwd(const float* g, const float* x, const float* y, const float* part, int C, int H, int W,
                           float* dx, hipStream_t st);
hipError_t launch_densify_plan(const Scene& s, const float* gacc, const float* gcnt, const float* noise,
                               const DensifyCfg& c, void* tmp, hipStream_t st);
unsigned long long* densify_total_ptr(void* tmp, int64_t n);
// static / dynamic split by staticness (same workspace as densify)
hipError_t launch_static_plan(const Scene& s, float thr, void* tmp, hipStream_t st);
hipError_t launch_static_apply(const Scene& s, float thr, const void* tmp, const SceneOut& os, const SceneOut& od,
                               hipStream_t st);
hipError_t launch_densify_apply(const Scene& s, const float* noise, const DensifyCfg& c, const void* tmp,
                                const SceneOut& out, const float* extra_in, float* extra_out, int32_t n_extra,
                                hipStream_t st);
hipError_t launch_fill_f32(float* p, float v, int64_t n, hipStream_t s);

// binning: scratch layout and the sort pipeline
struct BinPlan {
  int64_t n;             // Gaussians in the batch
  int64_t tiles;         // total tiles
  int64_t capacity;      // instance capacity
  int tile_bits;         // bits of the global tile id
  int tile_passes;       // radix passes over the tile key
  // scratch carve-up (bytes offsets into tmp)
  size_t off_vis_keys, off_vis_vals, off_offsets, off_partials, off_hist, off_rowtot, off_partials2, off_rows,
      off_num_rows, total;
  int64_t hist_cols;       // blocks per radix row of the tile passes
  int64_t hist_cols_depth; // blocks per radix row of the depth passes
};
BinPlan plan_bins(int64_t n, int64_t tiles, int64_t capacity);
int run_bin_sort(const ViewSet& vs, const Geom& geom, pvg_bins* bins, void* tmp, const BinPlan& plan,
                 int sync_count, hipStream_t s);
// device address of the library-held bin_sort scratch (PVG_NOALLOC_SCRATCH_BYTES)
// on the current device, looked up on the first call per device
hipError_t noalloc_scratch(void** out);
// with a NoProfile in scope the calling thread's launches record no stage
// events (event creation may allocate)
struct NoProfile {
  NoProfile();
  ~NoProfile();
  bool prev_;
};
// batched forward of a device view table (no host synchronisation, capturable)
int run_batch_forward(const ViewSet& vs, const Geom& geom, pvg_bins* bins, void* tmp, const BinPlan& plan,
                      hipStream_t s);

}  // namespace pvg
