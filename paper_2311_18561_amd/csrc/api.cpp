// C ABI of libpvg: argument validation, view construction and the stage
// profiler.  Kernels live in preprocess.hip, binsort.hip and render.hip.
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pvg_internal.hpp"

namespace pvg {

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

int hip_fail(hipError_t e, const char* what) {
  set_error("%s failed: %s", what, hipGetErrorString(e));
  return PVG_ERR_HIP;
}

// ------------------------------------------------------------------ profiler
namespace {
struct EventPair { int stage; hipEvent_t a, b; };
std::mutex g_prof_mu;
bool g_prof_on = false;
bool g_count_work = false;
std::vector<EventPair> g_pending;
std::vector<hipEvent_t> g_pool;
double g_ms[PVG_STAGE_COUNT];
int64_t g_calls[PVG_STAGE_COUNT];
int64_t g_work[PVG_STAGE_COUNT];
unsigned long long* g_work_dev = nullptr;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

namespace {
thread_local bool t_no_profile = false;
}

NoProfile::NoProfile() : prev_(t_no_profile) { t_no_profile = true; }
NoProfile::~NoProfile() { t_no_profile = prev_; }

bool profiling() { return g_prof_on && !t_no_profile; }

unsigned long long* profile_work_counter(int stage) {
  if (!g_prof_on || !g_count_work || !g_work_dev) return nullptr;
  return g_work_dev + stage;
}

StageScope::StageScope(int stage, hipStream_t s) : stage_(stage), s_(s), on_(false) {
  if (!g_prof_on || t_no_profile) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  EventPair p{stage, take_event(), take_event()};
  if (!p.a || !p.b) return;
  if (hipEventRecord(p.a, s) != hipSuccess) return;
  g_pending.push_back(p);
  on_ = true;
}

StageScope::~StageScope() {
  if (!on_) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto it = g_pending.rbegin(); it != g_pending.rend(); ++it) {
    if (it->stage == stage_) {
      (void)hipEventRecord(it->b, s_);
      break;
    }
  }
}

// ------------------------------------------------------------------ validation
bool check_gaussians(const pvg_gaussians* g) {
  if (!g) { set_error("gaussians is null"); return false; }
  if (g->n < 0) { set_error("n = %lld < 0", static_cast<long long>(g->n)); return false; }
  if (g->n > 0xffffffffll) { set_error("n = %lld exceeds 2^32 - 1", static_cast<long long>(g->n)); return false; }
  if (g->sh_degree < 0 || g->sh_degree > 3) { set_error("sh_degree %d outside 0..3", g->sh_degree); return false; }
  if (g->n > 0 && (!g->mu || !g->scale || !g->rot || !g->sh || !g->opacity || !g->vel || !g->period || !g->tau ||
                   !g->beta)) {
    set_error("a parameter array is null");
    return false;
  }
  return true;
}

bool check_camera(const pvg_camera* c) {
  if (!c) { set_error("camera is null"); return false; }
  if (c->width <= 0 || c->height <= 0) { set_error("image size %d x %d is not positive", c->width, c->height); return false; }
  if (c->width > 65535 || c->height > 65535) { set_error("image size above 65535 pixels"); return false; }
  if (!(c->fx > 0.0f) || !(c->fy > 0.0f)) { set_error("focal length must be positive"); return false; }
  if (!(c->znear > 0.0f) || !std::isfinite(c->znear)) {
    set_error("znear must be positive and finite (depth keys are the bits of a positive float)");
    return false;
  }
  return true;
}

static bool check_frame(const pvg_frame* f) {
  if (!f) { set_error("frame is null"); return false; }
  if (f->advect_mode != 0 && f->advect_mode != 1) { set_error("advect_mode must be 0 or 1"); return false; }
  return true;
}

static bool check_geom(const pvg_geom* g, int64_t n) {
  if (!g) { set_error("geom is null"); return false; }
  if (g->n != n) { set_error("geom.n = %lld differs from n = %lld", static_cast<long long>(g->n), static_cast<long long>(n)); return false; }
  if (n > 0 && (!g->xy || !g->depth || !g->conic_op || !g->rgb || !g->radius || !g->tiles)) {
    set_error("a geom array is null");
    return false;
  }
  return true;
}

static bool check_bins(const pvg_bins* b) {
  if (!b) { set_error("bins is null"); return false; }
  if (b->capacity < 0 || b->capacity > 0xffffffffll) { set_error("capacity outside 0..2^32-1"); return false; }
  if (!b->ranges || !b->counters || (b->capacity > 0 && (!b->keys || !b->vals))) {
    set_error("a bins array is null");
    return false;
  }
  if (b->tile_cull != 0 && b->tile_cull != 1) { set_error("tile_cull must be 0 or 1"); return false; }
  return true;
}

static int64_t tiles_of(const pvg_camera* c) {
  return static_cast<int64_t>((c->width + kTile - 1) / kTile) * ((c->height + kTile - 1) / kTile);
}

View make_view(const pvg_gaussians* g, const pvg_camera* c, const pvg_frame* f) {
  View v;
  std::memset(&v, 0, sizeof(v));
  if (g) v.s = Scene{g->mu, g->scale, g->rot, g->sh, g->opacity, g->vel, g->period, g->tau, g->beta, g->n, g->sh_degree};
  std::memcpy(v.R, c->R, sizeof(v.R));
  std::memcpy(v.T, c->T, sizeof(v.T));
  v.fx = c->fx; v.fy = c->fy; v.cx = c->cx; v.cy = c->cy; v.znear = c->znear;
  v.W = c->width; v.H = c->height;
  v.GX = (c->width + kTile - 1) / kTile;
  v.GY = (c->height + kTile - 1) / kTile;
  if (f) {
    v.t = f->t; v.dt = f->dt; v.mode = f->advect_mode;
    v.bg[0] = f->bg[0]; v.bg[1] = f->bg[1]; v.bg[2] = f->bg[2];
  }
  return v;
}

static ViewSet single(const View& v, int64_t n) {
  ViewSet vs;
  std::memset(&vs, 0, sizeof(vs));
  vs.table = nullptr;
  vs.one = v;
  vs.nviews = 1;
  vs.total_gauss = n;
  vs.total_tiles = static_cast<int64_t>(v.GX) * v.GY;
  return vs;
}

// scratch of the feature adjoint: g2d [views][n][kG2DStride] | rec [capacity][8 + feature_width(n_ch)] |
// vis [capacity] bytes (padded for the 16-byte flag reads)
static size_t feature_scratch_bytes(int64_t n, int32_t views, int32_t n_ch, int64_t capacity, size_t* off_rec,
                                    size_t* off_vis, size_t* vis_bytes, size_t* slot_bytes) {
  auto al = [](size_t x) { return (x + 255) & ~static_cast<size_t>(255); };
  const size_t slot = al(sizeof(float) * kG2DStride * static_cast<size_t>(std::max<int64_t>(n, 1)));
  const size_t g2d = slot * static_cast<size_t>(std::max(views, 1));
  const size_t cap = static_cast<size_t>(std::max<int64_t>(capacity, 1));
  const size_t rec = al(sizeof(float) * static_cast<size_t>(8 + feature_width(n_ch)) * cap);
  const size_t vis = al((cap + 31) & ~static_cast<size_t>(15));
  if (off_rec) *off_rec = g2d;
  if (off_vis) *off_vis = g2d + rec;
  if (vis_bytes) *vis_bytes = vis;
  if (slot_bytes) *slot_bytes = slot;
  return g2d + rec + vis;
}

size_t bwd_scratch_bytes(int64_t n, int32_t views, int32_t regions, int64_t capacity, size_t* off_rec,
                         size_t* off_vis, size_t* vis_bytes, size_t* slot_bytes, size_t* region_bytes) {
  auto al = [](size_t x) { return (x + 255) & ~static_cast<size_t>(255); };
  const size_t slot = al(sizeof(float) * kG2DStride * static_cast<size_t>(std::max<int64_t>(n, 1)));
  const size_t g2d = slot * static_cast<size_t>(std::max(views, 1));
  const size_t rec = al(sizeof(float) * kRecFloats * static_cast<size_t>(std::max<int64_t>(capacity, 1)));
  // one flag byte per instance, padded so 16-byte reads past the last one stay inside
  const size_t vis = al((static_cast<size_t>(std::max<int64_t>(capacity, 1)) + 31) & ~static_cast<size_t>(15));
  if (off_rec) *off_rec = g2d;
  if (off_vis) *off_vis = g2d + rec;
  if (vis_bytes) *vis_bytes = vis;
  if (slot_bytes) *slot_bytes = slot;
  if (region_bytes) *region_bytes = rec + vis;
  return g2d + (rec + vis) * static_cast<size_t>(std::max(regions, 1));
}

// Side streams (default priority, non-blocking) on which the multi-view
// adjoint runs views concurrently; created once per device.
namespace {
std::mutex g_side_mu;
std::vector<std::vector<hipStream_t>> g_side;
thread_local std::vector<hipEvent_t> t_events;

int side_streams(std::vector<hipStream_t>& out) {
  int dev = 0;
  PVG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_side_mu);
  if (static_cast<int>(g_side.size()) <= dev) g_side.resize(dev + 1);
  if (g_side[dev].empty()) {
    for (int k = 0; k < kBwdStreams; ++k) {
      hipStream_t st = nullptr;
      PVG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      g_side[dev].push_back(st);
    }
  }
  out = g_side[dev];
  return PVG_OK;
}

// The i-th event of this thread's pool (events are only recorded and waited
// on within one call, so reuse across calls is safe).
hipEvent_t pool_event(size_t i) {
  while (t_events.size() <= i) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    t_events.push_back(e);
  }
  return t_events[i];
}
}  // namespace

static Geom to_geom(const pvg_geom* g) {
  return Geom{g->xy, g->depth, g->conic_op, g->rgb, g->radius, g->tiles, g->feat};
}

}  // namespace pvg

using namespace pvg;

extern "C" {

int pvg_workspace_query(int64_t n, int32_t width, int32_t height, int64_t capacity, pvg_ws_sizes* out) {
  if (!out || n < 0 || width <= 0 || height <= 0 || capacity < 0 || capacity > 0xffffffffll) {
    set_error("invalid workspace query");
    return PVG_ERR_INVALID;
  }
  const int64_t tiles = static_cast<int64_t>((width + kTile - 1) / kTile) * ((height + kTile - 1) / kTile);
  out->bin_tmp_bytes = plan_bins(n, tiles, capacity).total;
  out->bwd_tmp_bytes = bwd_scratch_bytes(n, 1, 1, capacity, nullptr, nullptr, nullptr, nullptr, nullptr);
  out->num_tiles = tiles;
  return PVG_OK;
}

int pvg_preprocess(const pvg_gaussians* g, const pvg_camera* cam, const pvg_frame* frame, pvg_geom* out,
                   void* stream) {
  if (!check_gaussians(g) || !check_camera(cam) || !check_frame(frame) || !check_geom(out, g ? g->n : 0))
    return PVG_ERR_INVALID;
  const View v = make_view(g, cam, frame);
  PVG_HIP(launch_preprocess(single(v, g->n), to_geom(out), static_cast<hipStream_t>(stream)));
  return PVG_OK;
}

int pvg_preprocess_views(const pvg_gaussians* g, int32_t n_views, const pvg_camera* cams, const pvg_frame* frames,
                         pvg_geom* outs, void* stream) {
  if (!check_gaussians(g)) return PVG_ERR_INVALID;
  if (n_views < 1 || !cams || !frames || !outs) {
    set_error("n_views < 1 or a per-view array is null");
    return PVG_ERR_INVALID;
  }
  for (int32_t k = 0; k < n_views; ++k)
    if (!check_camera(&cams[k]) || !check_frame(&frames[k]) || !check_geom(&outs[k], g->n)) return PVG_ERR_INVALID;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  PreViews pk;
  std::memset(&pk, 0, sizeof(pk));
  for (int32_t k0 = 0; k0 < n_views; k0 += kMaxBwdViews) {  // up to eight views per pass over the parameters
    pk.nv = std::min(n_views - k0, kMaxBwdViews);
    for (int32_t k = 0; k < pk.nv; ++k) {
      pk.views[k] = make_view(g, &cams[k0 + k], &frames[k0 + k]);
      pk.geoms[k] = to_geom(&outs[k0 + k]);
    }
    PVG_HIP(launch_preprocess_views(pk, s));
  }
  return PVG_OK;
}

// A caller's workspace is cut into 256-byte aligned parts read 16 bytes at a time.
static bool scratch_aligned(const void* tmp, const char* what) {
  if (reinterpret_cast<uintptr_t>(tmp) % 256 == 0) return true;
  set_error("%s scratch at %p does not start on a 256-byte boundary", what, tmp);
  return false;
}

int pvg_bin_sort(const pvg_geom* geom, const pvg_camera* cam, pvg_bins* bins, void* tmp, size_t tmp_bytes,
                 int32_t sync_count, void* stream) {
  if (!geom || !check_geom(geom, geom->n) || !check_camera(cam) || !check_bins(bins)) return PVG_ERR_INVALID;
  if (geom->n > 0xffffffffll) { set_error("n too large"); return PVG_ERR_INVALID; }
  const BinPlan plan = plan_bins(geom->n, tiles_of(cam), bins->capacity);
  if (!tmp || tmp_bytes < plan.total) {
    set_error("bin_sort scratch of %zu bytes is smaller than the %zu required", tmp_bytes, plan.total);
    return PVG_ERR_NOMEM;
  }
  if (!scratch_aligned(tmp, "bin_sort")) return PVG_ERR_INVALID;
  const View v = make_view(nullptr, cam, nullptr);
  bins->num_instances = -1;
  bins->num_visible = -1;
  return run_bin_sort(single(v, geom->n), to_geom(geom), bins, tmp, plan, sync_count,
                      static_cast<hipStream_t>(stream));
}

int pvg_bin_sort_noalloc(const pvg_geom* geom, const pvg_camera* cam, pvg_bins* bins, int32_t sync_count,
                         void* stream) {
  if (!geom || !check_geom(geom, geom->n) || !check_camera(cam) || !check_bins(bins)) return PVG_ERR_INVALID;
  if (geom->n > 0xffffffffll) { set_error("n too large"); return PVG_ERR_INVALID; }
  const BinPlan plan = plan_bins(geom->n, tiles_of(cam), bins->capacity);
  if (plan.total > PVG_NOALLOC_SCRATCH_BYTES) {
    set_error("bin_sort of %lld Gaussians on %lld tiles with capacity %lld needs %zu bytes of scratch; the "
              "library-held scratch holds %zu (use pvg_bin_sort with a workspace)",
              static_cast<long long>(geom->n), static_cast<long long>(tiles_of(cam)),
              static_cast<long long>(bins->capacity), plan.total, static_cast<size_t>(PVG_NOALLOC_SCRATCH_BYTES));
    return PVG_ERR_NOMEM;
  }
  void* tmp = nullptr;
  PVG_HIP(noalloc_scratch(&tmp));
  const NoProfile quiet;
  const View v = make_view(nullptr, cam, nullptr);
  bins->num_instances = -1;
  bins->num_visible = -1;
  return run_bin_sort(single(v, geom->n), to_geom(geom), bins, tmp, plan, sync_count,
                      static_cast<hipStream_t>(stream));
}

int pvg_render_fwd(const pvg_geom* geom, const pvg_bins* bins, const pvg_camera* cam, const pvg_frame* frame,
                   float* img, float* final_T, int32_t* n_contrib, void* stream) {
  return pvg_render_fwd_channels(geom, bins, cam, frame, img, final_T, n_contrib, nullptr, stream);
}

int pvg_render_fwd_channels(const pvg_geom* geom, const pvg_bins* bins, const pvg_camera* cam,
                            const pvg_frame* frame, float* img, float* final_T, int32_t* n_contrib,
                            const pvg_channels* channels, void* stream) {
  if (!geom || !check_geom(geom, geom->n) || !check_bins(bins) || !check_camera(cam) || !check_frame(frame))
    return PVG_ERR_INVALID;
  if (!img || !final_T || !n_contrib) { set_error("an output array is null"); return PVG_ERR_INVALID; }
  View v = make_view(nullptr, cam, frame);
  v.img = img;
  v.final_T = final_T;
  v.n_contrib = n_contrib;
  if (channels) {
    v.depth_img = channels->depth;
    v.depth_norm = channels->depth_normalized != 0;
    v.vbar_img = channels->vbar;
    v.rho_img = channels->rho;
    v.opacity_img = channels->opacity;
    if ((v.vbar_img || v.rho_img) && geom->n > 0 && !geom->feat) {
      set_error("the velocity and staticness channels need geom.feat");
      return PVG_ERR_INVALID;
    }
  }
  PVG_HIP(launch_render_fwd(single(v, geom->n), to_geom(geom), bins->vals, bins->ranges, bins->tile_cull != 0,
                            static_cast<hipStream_t>(stream)));
  return PVG_OK;
}

int pvg_render_features(const pvg_geom* geom, const pvg_bins* bins, const pvg_camera* cam, const float* feat,
                        int64_t ld, int32_t n_ch, float* out, float* final_T, int32_t* n_contrib, void* stream) {
  if (!geom || !check_geom(geom, geom->n) || !check_bins(bins) || !check_camera(cam)) return PVG_ERR_INVALID;
  if (n_ch < 1 || n_ch > kMaxFeatureChannels || ld < n_ch) {
    set_error("n_ch outside [1, %d] or ld < n_ch", kMaxFeatureChannels);
    return PVG_ERR_INVALID;
  }
  if (!out || !final_T || !n_contrib || (geom->n > 0 && !feat)) {
    set_error("feat or an output array is null");
    return PVG_ERR_INVALID;
  }
  View v = make_view(nullptr, cam, nullptr);
  v.final_T = final_T;
  v.n_contrib = n_contrib;
  PVG_HIP(launch_feature_fwd(single(v, geom->n), to_geom(geom), bins->vals, bins->ranges, bins->tile_cull != 0, feat,
                             ld, n_ch, out, static_cast<hipStream_t>(stream)));
  return PVG_OK;
}

int pvg_render_bwd(const pvg_gaussians* g, const pvg_camera* cam, const pvg_frame* frame, const pvg_geom* geom,
                   const pvg_bins* bins, const float* final_T, const int32_t* n_contrib, const float* dL_dimg,
                   pvg_gaussians_grad* grad, int32_t accumulate, void* tmp, size_t tmp_bytes, void* stream) {
  if (!final_T || !n_contrib || !dL_dimg) { set_error("an input array is null"); return PVG_ERR_INVALID; }
  return pvg_render_bwd_views(g, 1, cam, frame, geom, bins, &final_T, &n_contrib, &dL_dimg, grad, accumulate, tmp,
                              tmp_bytes, stream);
}

int pvg_sky_composite(const pvg_camera* cam, const float* img, const float* opacity, const float* cube,
                      int32_t cube_res, const float* jitter, float* out, void* stream) {
  if (!check_camera(cam)) return PVG_ERR_INVALID;
  if (!img || !opacity || !cube || !out) { set_error("a sky composite array is null"); return PVG_ERR_INVALID; }
  if (cube_res < 1 || cube_res > 16384) { set_error("cube_res = %d out of [1, 16384]", cube_res); return PVG_ERR_INVALID; }
  PVG_HIP(launch_sky(cam, img, opacity, cube, cube_res, jitter, out, static_cast<hipStream_t>(stream)));
  return PVG_OK;
}

static int sky_bwd(const pvg_camera* cam, const float* dL_dout, const float* opacity, const float* cube,
                   int32_t cube_res, const float* jitter, float* dL_dopacity, float* dL_dcube, bool deterministic,
                   void* stream) {
  if (!check_camera(cam)) return PVG_ERR_INVALID;
  if (!dL_dout || !opacity || !cube || !dL_dopacity || !dL_dcube) {
    set_error("a sky composite array is null");
    return PVG_ERR_INVALID;
  }
  if (cube_res < 1 || cube_res > 16384) { set_error("cube_res = %d out of [1, 16384]", cube_res); return PVG_ERR_INVALID; }
  PVG_HIP(launch_sky_bwd(cam, dL_dout, opacity, cube, cube_res, jitter, dL_dopacity, dL_dcube, deterministic,
                         static_cast<hipStream_t>(stream)));
  return PVG_OK;
}

int pvg_sky_composite_bwd(const pvg_camera* cam, const float* dL_dout, const float* opacity, const float* cube,
                          int32_t cube_res, const float* jitter, float* dL_dopacity, float* dL_dcube, void* stream) {
  return sky_bwd(cam, dL_dout, opacity, cube, cube_res, jitter, dL_dopacity, dL_dcube, false, stream);
}

int pvg_sky_composite_bwd_deterministic(const pvg_camera* cam, const float* dL_dout, const float* opacity,
                                        const float* cube, int32_t cube_res, const float* jitter, float* dL_dopacity,
                                        float* dL_dcube, void* stream) {
  return sky_bwd(cam, dL_dout, opacity, cube, cube_res, jitter, dL_dopacity, dL_dcube, true, stream);
}

int pvg_bwd_views_tmp_bytes(int64_t n, int32_t n_views, int32_t max_width, int32_t max_height, int64_t max_capacity,
                            size_t* bytes) {
  if (!bytes || n < 0 || n_views < 1 || max_width <= 0 || max_height <= 0 || max_capacity < 0 ||
      max_capacity > 0xffffffffll) {
    set_error("invalid scratch query");
    return PVG_ERR_INVALID;
  }
  const int64_t tiles = static_cast<int64_t>((max_width + kTile - 1) / kTile) * ((max_height + kTile - 1) / kTile);
  (void)tiles;
  *bytes = bwd_scratch_bytes(n, std::min(n_views, kMaxBwdViews), std::min(n_views, kBwdStreams), max_capacity,
                             nullptr, nullptr, nullptr, nullptr, nullptr);
  return PVG_OK;
}

int pvg_render_bwd_views(const pvg_gaussians* g, int32_t n_views, const pvg_camera* cams, const pvg_frame* frames,
                         const pvg_geom* geoms, const pvg_bins* bins, const float* const* final_T,
                         const int32_t* const* n_contrib, const float* const* dL_dimg, pvg_gaussians_grad* grad,
                         int32_t accumulate, void* tmp, size_t tmp_bytes, void* stream) {
  return pvg_render_bwd_views_channels(g, n_views, cams, frames, geoms, bins, final_T, n_contrib, dL_dimg, nullptr,
                                       grad, accumulate, tmp, tmp_bytes, stream);
}

// Zeros into every parameter gradient array (an overwriting adjoint that no
// view fed still writes its result).
static int zero_param_grads(const pvg_gaussians* g, const pvg_gaussians_grad* grad, hipStream_t s) {
  const int64_t n = g->n, K = (g->sh_degree + 1) * (g->sh_degree + 1);
  PVG_HIP(launch_fill_f32(grad->mu, 0.0f, 3 * n, s));
  PVG_HIP(launch_fill_f32(grad->scale, 0.0f, 3 * n, s));
  PVG_HIP(launch_fill_f32(grad->rot, 0.0f, 4 * n, s));
  PVG_HIP(launch_fill_f32(grad->sh, 0.0f, 3 * K * n, s));
  PVG_HIP(launch_fill_f32(grad->opacity, 0.0f, n, s));
  PVG_HIP(launch_fill_f32(grad->vel, 0.0f, 3 * n, s));
  PVG_HIP(launch_fill_f32(grad->period, 0.0f, n, s));
  PVG_HIP(launch_fill_f32(grad->tau, 0.0f, n, s));
  PVG_HIP(launch_fill_f32(grad->beta, 0.0f, n, s));
  return PVG_OK;
}

int pvg_render_bwd_views_channels(const pvg_gaussians* g, int32_t n_views, const pvg_camera* cams,
                                  const pvg_frame* frames, const pvg_geom* geoms, const pvg_bins* bins,
                                  const float* const* final_T, const int32_t* const* n_contrib,
                                  const float* const* dL_dimg, const pvg_channels* channels,
                                  pvg_gaussians_grad* grad, int32_t accumulate, void* tmp, size_t tmp_bytes,
                                  void* stream) {
  if (!check_gaussians(g)) return PVG_ERR_INVALID;
  if (n_views < 1 || !cams || !frames || !geoms || !bins || !final_T || !n_contrib || !dL_dimg) {
    set_error("n_views < 1 or a per-view array is null");
    return PVG_ERR_INVALID;
  }
  if (!grad || (g->n > 0 && (!grad->mu || !grad->scale || !grad->rot || !grad->sh || !grad->opacity ||
                             !grad->vel || !grad->period || !grad->tau || !grad->beta))) {
    set_error("a gradient array is null");
    return PVG_ERR_INVALID;
  }
  if ((grad->densify_grad == nullptr) != (grad->densify_count == nullptr)) {
    set_error("densify_grad and densify_count go together");
    return PVG_ERR_INVALID;
  }
  int64_t max_tiles = 1, max_cap = 0;
  for (int32_t k = 0; k < n_views; ++k) {
    if (!check_camera(&cams[k]) || !check_frame(&frames[k]) || !check_geom(&geoms[k], g->n) ||
        !check_bins(&bins[k]))
      return PVG_ERR_INVALID;
    if (!dL_dimg[k]) continue;  // no gradient flows into this view
    if (!final_T[k] || !n_contrib[k]) { set_error("view %d: final_T or n_contrib is null", k); return PVG_ERR_INVALID; }
    if (g->n > 0 && !bins[k].first) {
      set_error("view %d: bins.first is null: the adjoint needs each Gaussian's first instance index", k);
      return PVG_ERR_INVALID;
    }
    if (g->n > 0 && bins[k].tile_cull && (!bins[k].rows || !bins[k].row_base)) {
      set_error("view %d: bins.rows / bins.row_base are null: the adjoint of culled lists needs them", k);
      return PVG_ERR_INVALID;
    }
    max_tiles = std::max(max_tiles, tiles_of(&cams[k]));
    max_cap = std::max(max_cap, bins[k].capacity);
  }
  const int32_t slots = std::min(n_views, kMaxBwdViews);
  (void)max_tiles;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // views run concurrently on side streams, each with its own record region;
  // under stream capture everything stays on the caller's stream
  hipStreamCaptureStatus cap_status = hipStreamCaptureStatusNone;
  PVG_HIP(hipStreamIsCapturing(s, &cap_status));
  int32_t with_grad = 0;
  for (int32_t k = 0; k < n_views; ++k) with_grad += dL_dimg[k] ? 1 : 0;
  const bool serial = cap_status != hipStreamCaptureStatusNone || with_grad <= 1;
  const int32_t regions = serial ? 1 : std::min(with_grad, kBwdStreams);
  size_t off_rec = 0, off_vis = 0, vis_bytes = 0, slot_bytes = 0, region_bytes = 0;
  const size_t need = bwd_scratch_bytes(g->n, slots, regions, max_cap, &off_rec, &off_vis, &vis_bytes, &slot_bytes,
                                        &region_bytes);
  if (!tmp || tmp_bytes < need) {
    set_error("render_bwd scratch of %zu bytes is smaller than the %zu required", tmp_bytes, need);
    return PVG_ERR_NOMEM;
  }
  if (!scratch_aligned(tmp, "render_bwd")) return PVG_ERR_INVALID;
  std::vector<hipStream_t> side;
  if (!serial) {
    const int st = side_streams(side);
    if (st != PVG_OK) return st;
  }
  size_t nev = 0;
  auto fork = [&]() -> int {  // side streams wait for the caller's stream
    if (serial) return PVG_OK;
    hipEvent_t e = pool_event(nev++);
    if (!e) { set_error("hipEventCreate failed"); return PVG_ERR_HIP; }
    PVG_HIP(hipEventRecord(e, s));
    for (int32_t r = 0; r < regions; ++r) PVG_HIP(hipStreamWaitEvent(side[r], e, 0));
    return PVG_OK;
  };
  auto join = [&]() -> int {  // the caller's stream waits for the side streams
    if (serial) return PVG_OK;
    for (int32_t r = 0; r < regions; ++r) {
      hipEvent_t e = pool_event(nev++);
      if (!e) { set_error("hipEventCreate failed"); return PVG_ERR_HIP; }
      PVG_HIP(hipEventRecord(e, side[r]));
      PVG_HIP(hipStreamWaitEvent(s, e, 0));
    }
    return PVG_OK;
  };
  char* base = static_cast<char*>(tmp);
  BwdViews pk;
  std::memset(&pk, 0, sizeof(pk));
  bool first_group = true;
  // Views go to g2d slots in turn.  The per-Gaussian pass runs per group of
  // `group` views: concurrently, one view per side stream, so the pass over
  // a finished group overlaps the next group's compositing adjoints; the
  // side streams wait for the caller's stream only when slots are reused.
  const int32_t group = serial ? kMaxBwdViews : regions;
  int32_t used_slots = 0;
  auto flush = [&]() -> int {
    if (pk.nv == 0) return PVG_OK;
    int st = join();
    if (st != PVG_OK) return st;
    PVG_HIP(launch_preprocess_bwd(pk, *grad, first_group ? accumulate : 1, s));
    first_group = false;
    pk.nv = 0;
    if (used_slots == kMaxBwdViews) {  // the next views reuse the slots this pass read
      used_slots = 0;
      return fork();
    }
    return PVG_OK;
  };
  {
    const int st = fork();
    if (st != PVG_OK) return st;
  }
  int32_t launched = 0;
  for (int32_t k = 0; k < n_views; ++k) {
    if (!dL_dimg[k]) continue;
    View v = make_view(g, &cams[k], &frames[k]);
    v.final_T = const_cast<float*>(final_T[k]);
    v.n_contrib = const_cast<int32_t*>(n_contrib[k]);
    v.dL_dimg = dL_dimg[k];
    if (channels) {
      v.dL_ddepth = channels[k].dL_ddepth;
      v.dL_dT = channels[k].dL_dT;
      v.dL_dO = channels[k].dL_dopacity;
      v.dL_dvbar = channels[k].dL_dvbar;
      v.dL_drho = channels[k].dL_drho;
      if (channels[k].depth_normalized && v.dL_ddepth) {
        if (!channels[k].depth) {
          set_error("the normalized depth gradient of view %d needs the forward's normalized depth", k);
          return PVG_ERR_INVALID;
        }
        v.depth_norm = 1;
        v.depth_img = channels[k].depth;
      }
      if ((v.dL_dvbar || v.dL_drho) && g->n > 0 && !geoms[k].feat) {
        set_error("the velocity and staticness gradients need geom.feat of view %d", k);
        return PVG_ERR_INVALID;
      }
    }
    float* g2d = reinterpret_cast<float*>(base + slot_bytes * static_cast<size_t>(used_slots));
    ++used_slots;
    const int32_t r = launched % regions;
    char* region = base + off_rec + region_bytes * static_cast<size_t>(r);
    float* rec = reinterpret_cast<float*>(region);
    uint8_t* vis = reinterpret_cast<uint8_t*>(region + (off_vis - off_rec));
    const Lists lists{bins[k].vals, bins[k].ranges, bins[k].first, bins[k].tile_cull != 0,
                      reinterpret_cast<const uint2*>(bins[k].rows), bins[k].row_base, bins[k].capacity};
    PVG_HIP(launch_render_bwd(single(v, g->n), to_geom(&geoms[k]), lists, rec, vis,
                              static_cast<int64_t>(vis_bytes), g2d, serial ? s : side[r]));
    ++launched;
    if (pk.nv > 0 && !(v.t == pk.views[0].t)) {  // a pass shares one render time
      const int st = flush();
      if (st != PVG_OK) return st;
    }
    pk.views[pk.nv] = v;
    pk.radius[pk.nv] = geoms[k].radius;
    pk.rgb[pk.nv] = geoms[k].rgb;
    pk.g2d[pk.nv] = g2d;
    pk.feat_grad[pk.nv] = channels ? channels[k].feature_grad : nullptr;
    ++pk.nv;
    if (pk.nv == group || used_slots == kMaxBwdViews) {
      const int st = flush();
      if (st != PVG_OK) return st;
    }
  }
  const int st = flush();
  if (st != PVG_OK) return st;
  if (first_group && !accumulate && g->n > 0) return zero_param_grads(g, grad, s);
  return PVG_OK;
}

// The adjoint of feature compositing.  The views run in order on the
// caller's stream with one record region (a view's gather adds into the
// caller's feature gradient, so views must not overlap); the per-Gaussian
// pass runs per group of up to kMaxBwdViews views of one render time.
int pvg_features_bwd_tmp_bytes(int64_t n, int32_t n_views, int32_t n_ch, int64_t max_capacity, size_t* bytes) {
  if (!bytes || n < 0 || n_views < 1 || n_ch < 1 || n_ch > kMaxFeatureChannels || max_capacity < 0 ||
      max_capacity > 0xffffffffll) {
    set_error("n < 0, n_views < 1, n_ch outside [1, %d], capacity outside [0, 2^32) or null output",
              kMaxFeatureChannels);
    return PVG_ERR_INVALID;
  }
  *bytes = feature_scratch_bytes(n, std::min(n_views, kMaxBwdViews), n_ch, max_capacity, nullptr, nullptr, nullptr,
                                 nullptr);
  return PVG_OK;
}

int pvg_render_features_bwd(const pvg_gaussians* g, int32_t n_views, const pvg_camera* cams,
                            const pvg_frame* frames, const pvg_geom* geoms, const pvg_bins* bins,
                            const float* const* final_T, const int32_t* const* n_contrib, const float* feat,
                            int64_t ld, int32_t n_ch, const float* const* dL_dout, float* feat_grad,
                            pvg_gaussians_grad* grad, int32_t accumulate, void* tmp, size_t tmp_bytes,
                            void* stream) {
  if (!check_gaussians(g)) return PVG_ERR_INVALID;
  if (n_views < 1 || !cams || !frames || !geoms || !bins || !final_T || !n_contrib || !dL_dout) {
    set_error("n_views < 1 or a per-view array is null");
    return PVG_ERR_INVALID;
  }
  if (n_ch < 1 || n_ch > kMaxFeatureChannels || ld < n_ch) {
    set_error("n_ch outside [1, %d] or ld < n_ch", kMaxFeatureChannels);
    return PVG_ERR_INVALID;
  }
  if (g->n > 0 && (!feat || !feat_grad)) { set_error("feat or feat_grad is null"); return PVG_ERR_INVALID; }
  if (!grad || (g->n > 0 && (!grad->mu || !grad->scale || !grad->rot || !grad->sh || !grad->opacity ||
                             !grad->vel || !grad->period || !grad->tau || !grad->beta))) {
    set_error("a gradient array is null");
    return PVG_ERR_INVALID;
  }
  if ((grad->densify_grad == nullptr) != (grad->densify_count == nullptr)) {
    set_error("densify_grad and densify_count go together");
    return PVG_ERR_INVALID;
  }
  int64_t max_cap = 0;
  for (int32_t k = 0; k < n_views; ++k) {
    if (!check_camera(&cams[k]) || !check_frame(&frames[k]) || !check_geom(&geoms[k], g->n) ||
        !check_bins(&bins[k]))
      return PVG_ERR_INVALID;
    if (!dL_dout[k]) continue;
    if (!final_T[k] || !n_contrib[k]) { set_error("view %d: final_T or n_contrib is null", k); return PVG_ERR_INVALID; }
    if (g->n > 0 && !bins[k].first) {
      set_error("view %d: bins.first is null: the adjoint needs each Gaussian's first instance index", k);
      return PVG_ERR_INVALID;
    }
    if (g->n > 0 && bins[k].tile_cull && (!bins[k].rows || !bins[k].row_base)) {
      set_error("view %d: bins.rows / bins.row_base are null: the adjoint of culled lists needs them", k);
      return PVG_ERR_INVALID;
    }
    max_cap = std::max(max_cap, bins[k].capacity);
  }
  const int32_t slots = std::min(n_views, kMaxBwdViews);
  size_t off_rec = 0, off_vis = 0, vis_bytes = 0, slot_bytes = 0;
  const size_t need = feature_scratch_bytes(g->n, slots, n_ch, max_cap, &off_rec, &off_vis, &vis_bytes, &slot_bytes);
  if (!tmp || tmp_bytes < need) {
    set_error("feature adjoint scratch of %zu bytes is smaller than the %zu required", tmp_bytes, need);
    return PVG_ERR_NOMEM;
  }
  if (!scratch_aligned(tmp, "feature adjoint")) return PVG_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(tmp);
  float* rec = reinterpret_cast<float*>(base + off_rec);
  uint8_t* vis = reinterpret_cast<uint8_t*>(base + off_vis);
  BwdViews pk;
  std::memset(&pk, 0, sizeof(pk));
  bool first_group = true;
  auto flush = [&]() -> int {
    if (pk.nv == 0) return PVG_OK;
    PVG_HIP(launch_preprocess_bwd(pk, *grad, first_group ? accumulate : 1, s));
    first_group = false;
    pk.nv = 0;
    return PVG_OK;
  };
  for (int32_t k = 0; k < n_views; ++k) {
    if (!dL_dout[k]) continue;
    View v = make_view(g, &cams[k], &frames[k]);
    v.final_T = const_cast<float*>(final_T[k]);
    v.n_contrib = const_cast<int32_t*>(n_contrib[k]);
    if (pk.nv > 0 && !(v.t == pk.views[0].t)) {  // a pass shares one render time
      const int st = flush();
      if (st != PVG_OK) return st;
    }
    float* g2d = reinterpret_cast<float*>(base + slot_bytes * static_cast<size_t>(pk.nv));
    const Lists lists{bins[k].vals, bins[k].ranges, bins[k].first, bins[k].tile_cull != 0,
                      reinterpret_cast<const uint2*>(bins[k].rows), bins[k].row_base, bins[k].capacity};
    PVG_HIP(launch_feature_bwd(single(v, g->n), to_geom(&geoms[k]), lists, feat, ld, n_ch, dL_dout[k], rec, vis,
                               static_cast<int64_t>(vis_bytes), g2d, feat_grad, s));
    pk.views[pk.nv] = v;
    pk.radius[pk.nv] = geoms[k].radius;
    pk.rgb[pk.nv] = geoms[k].rgb;
    pk.g2d[pk.nv] = g2d;
    pk.feat_grad[pk.nv] = nullptr;
    pk.no_colour[pk.nv] = true;
    ++pk.nv;
    if (pk.nv == kMaxBwdViews) {
      const int st = flush();
      if (st != PVG_OK) return st;
    }
  }
  const int st = flush();
  if (st != PVG_OK) return st;
  if (first_group && !accumulate && g->n > 0) return zero_param_grads(g, grad, s);
  return PVG_OK;
}

namespace {
bool check_densify(const pvg_densify_config* c) {
  if (!c) { set_error("config is null"); return false; }
  const float v[7] = {c->grad_threshold, c->scene_radius, c->clone_scale, c->prune_scale, c->min_opacity,
                      c->split_scale_decay, c->split_beta_decay};
  for (float x : v)
    if (!std::isfinite(x)) { set_error("a densify threshold is not finite"); return false; }
  if (!(c->scene_radius > 0.0f)) { set_error("scene_radius must be > 0"); return false; }
  return true;
}
pvg::DensifyCfg densify_cfg(const pvg_densify_config* c) {
  return pvg::DensifyCfg{c->grad_threshold, c->scene_radius, c->clone_scale, c->prune_scale, c->min_opacity,
                         c->split_scale_decay, c->split_beta_decay};
}
pvg::Scene scene_of(const pvg_gaussians* g) {
  return pvg::Scene{g->mu, g->scale, g->rot, g->sh, g->opacity, g->vel, g->period, g->tau, g->beta, g->n,
                    g->sh_degree};
}
constexpr int64_t kMaxDensifyN = int64_t(1) << 30;  // outputs (at most 2 n) keep 32-bit offsets
}  // namespace

int pvg_densify_tmp_bytes(int64_t n, size_t* bytes) {
  if (!bytes || n < 0 || n > kMaxDensifyN) { set_error("n outside [0, 2^30] or null output"); return PVG_ERR_INVALID; }
  *bytes = pvg::densify_tmp_bytes(n);
  return PVG_OK;
}

int pvg_densify_plan(const pvg_gaussians* g, const float* grad_accum, const float* grad_count, const float* noise,
                     const pvg_densify_config* cfg, void* tmp, size_t tmp_bytes, int64_t* n_out, void* stream) {
  if (!check_gaussians(g) || !check_densify(cfg)) return PVG_ERR_INVALID;
  if (g->n > kMaxDensifyN) { set_error("n exceeds 2^30"); return PVG_ERR_INVALID; }
  if (!n_out || !tmp || (g->n > 0 && (!grad_accum || !grad_count || !noise))) {
    set_error("a statistics, noise, workspace or output pointer is null");
    return PVG_ERR_INVALID;
  }
  if (tmp_bytes < pvg::densify_tmp_bytes(g->n)) { set_error("tmp_bytes too small"); return PVG_ERR_NOMEM; }
  if (!scratch_aligned(tmp, "densify")) return PVG_ERR_INVALID;
  auto s = static_cast<hipStream_t>(stream);
  PVG_HIP(pvg::launch_densify_plan(scene_of(g), grad_accum, grad_count, noise, densify_cfg(cfg), tmp, s));
  unsigned long long total = 0;
  PVG_HIP(hipMemcpyAsync(&total, pvg::densify_total_ptr(tmp, g->n), sizeof(total), hipMemcpyDeviceToHost, s));
  PVG_HIP(hipStreamSynchronize(s));
  *n_out = static_cast<int64_t>(total);
  return PVG_OK;
}

int pvg_densify_apply(const pvg_gaussians* g, const float* noise, const pvg_densify_config* cfg, const void* tmp,
                      size_t tmp_bytes, const pvg_gaussians* out, int32_t n_extra, const float* extra_in,
                      float* extra_out, void* stream) {
  if (!check_gaussians(g) || !check_gaussians(out) || !check_densify(cfg)) return PVG_ERR_INVALID;
  if (g->n > kMaxDensifyN) { set_error("n exceeds 2^30"); return PVG_ERR_INVALID; }
  if (out->sh_degree != g->sh_degree) { set_error("out.sh_degree differs from the input's"); return PVG_ERR_INVALID; }
  if (!tmp || (g->n > 0 && !noise) || n_extra < 0 ||
      (n_extra > 0 && ((g->n > 0 && !extra_in) || (out->n > 0 && !extra_out)))) {
    set_error("noise, workspace or extra rows missing, or n_extra < 0");
    return PVG_ERR_INVALID;
  }
  if (tmp_bytes < pvg::densify_tmp_bytes(g->n)) { set_error("tmp_bytes too small"); return PVG_ERR_NOMEM; }
  if (!scratch_aligned(tmp, "densify")) return PVG_ERR_INVALID;
  auto s = static_cast<hipStream_t>(stream);
  unsigned long long total = 0;
  PVG_HIP(hipMemcpyAsync(&total, pvg::densify_total_ptr(const_cast<void*>(tmp), g->n), sizeof(total),
                         hipMemcpyDeviceToHost, s));
  PVG_HIP(hipStreamSynchronize(s));
  if (static_cast<int64_t>(total) != out->n) {
    set_error("out.n = %lld but the plan produces %llu Gaussians", static_cast<long long>(out->n), total);
    return PVG_ERR_INVALID;
  }
  const pvg::SceneOut so{const_cast<float*>(out->mu), const_cast<float*>(out->scale), const_cast<float*>(out->rot),
                         const_cast<float*>(out->sh), const_cast<float*>(out->opacity), const_cast<float*>(out->vel),
                         const_cast<float*>(out->period), const_cast<float*>(out->tau), const_cast<float*>(out->beta),
                         out->n, out->sh_degree};
  PVG_HIP(pvg::launch_densify_apply(scene_of(g), noise, densify_cfg(cfg), tmp, so, extra_in, extra_out, n_extra, s));
  return PVG_OK;
}

int pvg_adam_step(const pvg_gaussians* params, const pvg_gaussians_grad* grad, float* m, float* v,
                  const pvg_adam_config* cfg, void* stream) {
  if (!check_gaussians(params)) return PVG_ERR_INVALID;
  if (!cfg || cfg->step < 1 || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) ||
      !(cfg->eps > 0.0f)) {
    set_error("config: step >= 1, beta1 and beta2 in [0, 1), eps > 0");
    return PVG_ERR_INVALID;
  }
  for (float lr : cfg->lr)
    if (!(lr >= 0.0f) || !std::isfinite(lr)) { set_error("learning rates must be finite and >= 0"); return PVG_ERR_INVALID; }
  if (params->n > 0 && (!grad || !m || !v || !grad->mu || !grad->scale || !grad->rot || !grad->sh ||
                        !grad->opacity || !grad->vel || !grad->period || !grad->tau || !grad->beta)) {
    set_error("a gradient or moment array is null");
    return PVG_ERR_INVALID;
  }
  pvg::AdamCfg c;
  for (int k = 0; k < 10; ++k) c.lr[k] = cfg->lr[k];
  c.beta1 = cfg->beta1; c.beta2 = cfg->beta2; c.eps = cfg->eps;
  c.bc1 = static_cast<float>(1.0 - std::pow(static_cast<double>(cfg->beta1), cfg->step));
  c.bc2 = static_cast<float>(1.0 - std::pow(static_cast<double>(cfg->beta2), cfg->step));
  const pvg::SceneOut so{const_cast<float*>(params->mu), const_cast<float*>(params->scale),
                         const_cast<float*>(params->rot), const_cast<float*>(params->sh),
                         const_cast<float*>(params->opacity), const_cast<float*>(params->vel),
                         const_cast<float*>(params->period), const_cast<float*>(params->tau),
                         const_cast<float*>(params->beta), params->n, params->sh_degree};
  PVG_HIP(pvg::launch_adam(so, params->n > 0 ? *grad : pvg_gaussians_grad{}, m, v, c,
                           static_cast<hipStream_t>(stream)));
  return PVG_OK;
}

int pvg_adam_dense(float* p, const float* grad, float* m, float* v, int64_t count, float lr, float beta1,
                   float beta2, float eps, int32_t step, void* stream) {
  if (count < 0 || count > (int64_t{1} << 40)) { set_error("count outside 0..2^40"); return PVG_ERR_INVALID; }
  if (step < 1 || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) ||
      !(lr >= 0.0f) || !std::isfinite(lr)) {
    set_error("step >= 1, beta1 and beta2 in [0, 1), eps > 0 and a finite lr >= 0 are required");
    return PVG_ERR_INVALID;
  }
  if (count > 0 && (!p || !grad || !m || !v)) { set_error("an array is null"); return PVG_ERR_INVALID; }
  pvg::AdamCfg c;
  for (int k = 0; k < 10; ++k) c.lr[k] = lr;
  c.beta1 = beta1; c.beta2 = beta2; c.eps = eps;
  c.bc1 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta1), step));
  c.bc2 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta2), step));
  PVG_HIP(pvg::launch_adam_dense(p, grad, m, v, count, lr, c, static_cast<hipStream_t>(stream)));
  return PVG_OK;
}

int pvg_opacity_reset(const pvg_gaussians* params, float* m, float* v, float cap, void* stream) {
  if (!check_gaussians(params)) return PVG_ERR_INVALID;
  if (!std::isfinite(cap) || (params->n > 0 && (!m || !v))) { set_error("cap not finite or moments null"); return PVG_ERR_INVALID; }
  const int64_t n = params->n, K = (params->sh_degree + 1) * (params->sh_degree + 1);
  const int64_t row = 3 + 3 + 4 + 3 * K;  // the opacity row of the moments
  PVG_HIP(pvg::launch_opacity_reset(const_cast<float*>(params->opacity), m + row * n, v + row * n, n, cap,
                                    static_cast<hipStream_t>(stream)));
  return PVG_OK;
}

namespace {
pvg::SceneOut scene_out(const pvg_gaussians* o) {
  return pvg::SceneOut{const_cast<float*>(o->mu), const_cast<float*>(o->scale), const_cast<float*>(o->rot),
                       const_cast<float*>(o->sh), const_cast<float*>(o->opacity), const_cast<float*>(o->vel),
                       const_cast<float*>(o->period), const_cast<float*>(o->tau), const_cast<float*>(o->beta),
                       o->n, o->sh_degree};
}
}  // namespace

int pvg_staticness_split_plan(const pvg_gaussians* g, float rho_threshold, void* tmp, size_t tmp_bytes,
                              int64_t* n_static, void* stream) {
  if (!check_gaussians(g)) return PVG_ERR_INVALID;
  if (g->n > kMaxDensifyN || !n_static || !tmp || !std::isfinite(rho_threshold)) {
    set_error("n above 2^30, a null pointer or a non-finite threshold");
    return PVG_ERR_INVALID;
  }
  if (tmp_bytes < pvg::densify_tmp_bytes(g->n)) { set_error("tmp_bytes too small"); return PVG_ERR_NOMEM; }
  if (!scratch_aligned(tmp, "staticness split")) return PVG_ERR_INVALID;
  auto s = static_cast<hipStream_t>(stream);
  PVG_HIP(pvg::launch_static_plan(scene_of(g), rho_threshold, tmp, s));
  unsigned long long total = 0;
  PVG_HIP(hipMemcpyAsync(&total, pvg::densify_total_ptr(tmp, g->n), sizeof(total), hipMemcpyDeviceToHost, s));
  PVG_HIP(hipStreamSynchronize(s));
  *n_static = static_cast<int64_t>(total);
  return PVG_OK;
}

int pvg_staticness_split_apply(const pvg_gaussians* g, float rho_threshold, const void* tmp, size_t tmp_bytes,
                               const pvg_gaussians* out_static, const pvg_gaussians* out_dynamic, void* stream) {
  if (!check_gaussians(g) || !check_gaussians(out_static) || !check_gaussians(out_dynamic)) return PVG_ERR_INVALID;
  if (g->n > kMaxDensifyN || !tmp || !std::isfinite(rho_threshold)) {
    set_error("n above 2^30, a null workspace or a non-finite threshold");
    return PVG_ERR_INVALID;
  }
  if (out_static->sh_degree != g->sh_degree || out_dynamic->sh_degree != g->sh_degree) {
    set_error("outputs must have the input's sh_degree");
    return PVG_ERR_INVALID;
  }
  if (tmp_bytes < pvg::densify_tmp_bytes(g->n)) { set_error("tmp_bytes too small"); return PVG_ERR_NOMEM; }
  if (!scratch_aligned(tmp, "staticness split")) return PVG_ERR_INVALID;
  auto s = static_cast<hipStream_t>(stream);
  unsigned long long total = 0;
  PVG_HIP(hipMemcpyAsync(&total, pvg::densify_total_ptr(const_cast<void*>(tmp), g->n), sizeof(total),
                         hipMemcpyDeviceToHost, s));
  PVG_HIP(hipStreamSynchronize(s));
  if (static_cast<int64_t>(total) != out_static->n || g->n - static_cast<int64_t>(total) != out_dynamic->n) {
    set_error("outputs hold %lld and %lld Gaussians but the plan splits %lld into %llu static",
              static_cast<long long>(out_static->n), static_cast<long long>(out_dynamic->n),
              static_cast<long long>(g->n), total);
    return PVG_ERR_INVALID;
  }
  PVG_HIP(pvg::launch_static_apply(scene_of(g), rho_threshold, tmp, scene_out(out_static), scene_out(out_dynamic),
                                   s));
  return PVG_OK;
}

int pvg_ssim_fwd(const float* x, const float* y, int32_t channels, int32_t height, int32_t width, float* ssim_map,
                 float* partials, void* stream) {
  if (channels < 1 || channels > 65535 || height < 1 || height > 65535 || width < 1 || width > 65535) {
    set_error("channels, height and width must be in 1..65535");
    return PVG_ERR_INVALID;
  }
  if (!x || !y || !partials) { set_error("x, y or partials is null"); return PVG_ERR_INVALID; }
  PVG_HIP(pvg::launch_ssim_fwd(x, y, channels, height, width, ssim_map, partials, static_cast<hipStream_t>(stream)));
  return PVG_OK;
}

int pvg_ssim_bwd(const float* dL_dssim, const float* x, const float* y, const float* partials, int32_t channels,
                 int32_t height, int32_t width, float* dL_dx, void* stream) {
  if (channels < 1 || channels > 65535 || height < 1 || height > 65535 || width < 1 || width > 65535) {
    set_error("channels, height and width must be in 1..65535");
    return PVG_ERR_INVALID;
  }
  if (!dL_dssim || !x || !y || !partials || !dL_dx) { set_error("an array is null"); return PVG_ERR_INVALID; }
  PVG_HIP(pvg::launch_ssim_bwd(dL_dssim, x, y, partials, channels, height, width, dL_dx,
                               static_cast<hipStream_t>(stream)));
  return PVG_OK;
}

int pvg_l1_loss(const float* a, const float* b, int64_t n, float scale, float* loss, float* grad_a, float* partials,
                void* stream) {
  if (n < 0 || !a || !b || !loss || !partials) {
    set_error("n < 0, or a, b, loss or partials is null");
    return PVG_ERR_INVALID;
  }
  static_assert(PVG_L1_PARTIALS == pvg::kL1Blocks, "the header's scratch size is the kernel's block count");
  PVG_HIP(pvg::launch_l1(a, b, n, scale, loss, grad_a, partials, static_cast<hipStream_t>(stream)));
  return PVG_OK;
}

int pvg_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (on && !g_work_dev) {
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&g_work_dev), sizeof(unsigned long long) * PVG_STAGE_COUNT);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(profile counters)");
    e = hipMemset(g_work_dev, 0, sizeof(unsigned long long) * PVG_STAGE_COUNT);
    if (e != hipSuccess) return hip_fail(e, "hipMemset(profile counters)");
  }
  g_prof_on = on != 0;
  g_count_work = on >= 2;
  return PVG_OK;
}

int pvg_profile_collect(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& p : g_pending) {
    hipError_t e = hipEventSynchronize(p.b);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, p.a, p.b);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    g_ms[p.stage] += ms;
    g_calls[p.stage] += 1;
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pending.clear();
  if (g_work_dev) {
    unsigned long long w[PVG_STAGE_COUNT];
    hipError_t e = hipMemcpy(w, g_work_dev, sizeof(w), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(profile counters)");
    for (int i = 0; i < PVG_STAGE_COUNT; ++i) g_work[i] += static_cast<int64_t>(w[i]);
    e = hipMemset(g_work_dev, 0, sizeof(w));
    if (e != hipSuccess) return hip_fail(e, "hipMemset(profile counters)");
  }
  return PVG_OK;
}

int pvg_profile_read(int32_t stage, double* total_ms, int64_t* invocations, int64_t* work) {
  if (stage < 0 || stage >= PVG_STAGE_COUNT) { set_error("unknown stage %d", stage); return PVG_ERR_INVALID; }
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (total_ms) *total_ms = g_ms[stage];
  if (invocations) *invocations = g_calls[stage];
  if (work) *work = g_work[stage];
  return PVG_OK;
}

int pvg_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (int i = 0; i < PVG_STAGE_COUNT; ++i) { g_ms[i] = 0.0; g_calls[i] = 0; g_work[i] = 0; }
  return PVG_OK;
}

const char* pvg_stage_name(int32_t stage) {
  static const char* names[PVG_STAGE_COUNT] = {"preprocess", "compact", "depth_sort", "scan_emit", "tile_sort",
                                                "ranges", "render_fwd", "render_bwd", "preprocess_bwd", "grad_gather"};
  if (stage < 0 || stage >= PVG_STAGE_COUNT) return "unknown";
  return names[stage];
}

const char* pvg_status_str(int status) {
  switch (status) {
    case PVG_OK: return "ok";
    case PVG_ERR_INVALID: return "invalid argument";
    case PVG_ERR_CAPACITY: return "instance capacity exceeded";
    case PVG_ERR_NOMEM: return "insufficient memory or workspace";
    case PVG_ERR_BUSY: return "busy";
    case PVG_ERR_HIP: return "HIP runtime error";
    case PVG_ERR_NOT_FOUND: return "not found";
    case PVG_ERR_TIMEOUT: return "timeout";
    default: return "unknown status";
  }
}

int pvg_last_error(char* buf, size_t len) {
  const std::string& s = g_last_error;
  if (buf && len > 0) {
    const size_t k = std::min(len - 1, s.size());
    std::memcpy(buf, s.data(), k);
    buf[k] = '\0';
  }
  return static_cast<int>(s.size());
}

}  // extern "C"
