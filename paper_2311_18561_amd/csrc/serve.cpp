// Continuous-batching render server (pvg_serve.h).
//
// Host side: a request queue, an admission rule (FIFO; a batch takes queued
// requests while their Gaussians, pixels and tiles fit the batch workspace),
// a scheduler thread that launches batches into free "lanes" (workspace +
// stream + event), and a completion thread that retires finished lanes.
// Device side: one lane's batch is a single preprocess / bin-sort / composite
// sequence over a device view table (views laid out back to back, global tile
// ids), with every count kept on the device so that the sequence can be
// captured once per (Gaussian, tile) grid bucket and replayed as a hipGraph
// whose first node copies the batch's view table from pinned host memory.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <cstdlib>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pvg_internal.hpp"
#include "pvg_serve.h"

namespace pvg {
namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

int64_t next_pow2(int64_t x, int64_t lo) {
  int64_t p = lo;
  while (p < x) p <<= 1;
  return p;
}

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct SceneRec {
  int32_t id = 0;
  pvg_gaussians g{};      // device pointers into buf
  void* buf = nullptr;
  size_t bytes = 0;
  int64_t pending = 0;    // queued or running requests
  bool unload = false;
};

struct Ticket {
  uint64_t id = 0;
  pvg_request req{};
  pvg_gaussians g{};      // its scene (server-owned copy; kept alive by the scene's pending count)
  int64_t n = 0;          // Gaussians of its scene
  int64_t pixels = 0;
  int64_t tiles = 0;
  bool solo = false;      // rerun alone after a batch overflow
  bool launched = false;
  bool done = false;
  pvg_result res{};
};

struct Header {           // device-side batch header: live totals, then the view table
  int64_t live[4];
};

struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void* dev = nullptr;    // one allocation for the whole workspace
  size_t dev_bytes = 0;
  Geom geom{};
  pvg_bins bins{};
  void* tmp = nullptr;
  float* final_T = nullptr;
  int32_t* n_contrib = nullptr;
  Header* d_hdr = nullptr;
  View* d_views = nullptr;
  void* h_stage = nullptr;      // pinned: Header + views
  uint32_t* h_counters = nullptr;  // pinned: copy of bins.counters after the batch
  std::map<std::pair<int64_t, int64_t>, hipGraphExec_t> graphs;
  std::vector<Ticket*> batch;
  bool busy = false;
  int64_t t_launch = 0;
  int64_t live_g = 0, live_t = 0;
};

}  // namespace
}  // namespace pvg

struct pvg_server {
  pvg_serve_config cfg{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_poll;
  std::deque<pvg::Ticket*> pending;
  std::unordered_map<uint64_t, pvg::Ticket*> tickets;
  std::map<int32_t, pvg::SceneRec> scenes;
  std::vector<pvg::Lane> lanes;
  std::deque<pvg::Lane*> inflight;
  std::thread th_sched, th_poll;
  bool stop = false;
  uint64_t next_ticket = 1;
  int32_t next_scene = 1;
  int64_t mem_used = 0;
  int64_t max_tiles = 0;
  size_t hdr_bytes = 0;
  // statistics since the last reset
  std::vector<double> lat_ms;
  int64_t completed = 0, failed = 0, batches = 0, batch_reqs = 0, retries = 0, graph_launches = 0, graph_builds = 0;
  double pixels = 0.0;
  int64_t t_first = 0, t_last = 0;
  // fault injection for tests of failure handling: with PVG_FAULT_INJECT=k
  // in the environment at creation, every k-th batch launch fails before
  // touching the device (its tickets get PVG_ERR_HIP); 0: off
  int64_t fault_every = 0;
  int64_t launches = 0;  // scheduler thread only
};

namespace pvg {
namespace {

bool stub(const pvg_server* s) { return s->cfg.stub_launch_us > 0; }

// Device workspace of one lane, carved from one allocation.
int lane_init(pvg_server* s, Lane& L) {
  const auto& c = s->cfg;
  const int64_t G = c.max_batch_gaussians, P = c.max_batch_pixels, cap = c.instance_capacity;
  const BinPlan plan = plan_bins(G, s->max_tiles, cap);
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + bytes); return o; };
  const size_t o_xy = take(8 * G), o_depth = take(4 * G), o_co = take(16 * G), o_rgb = take(12 * G),
               o_rad = take(4 * G), o_tiles = take(4 * G);
  const size_t o_keys = take(8 * std::max<int64_t>(cap, 1)), o_vals = take(8 * std::max<int64_t>(cap, 1));
  const size_t o_ranges = take(8 * s->max_tiles), o_counters = take(16);
  const size_t o_tmp = take(plan.total);
  const size_t o_T = take(4 * P), o_nc = take(4 * P);
  const size_t o_hdr = take(s->hdr_bytes);
  L.dev_bytes = off;
  if (stub(s)) return PVG_OK;
  PVG_HIP(hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking));
  PVG_HIP(hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
  PVG_HIP(hipMalloc(&L.dev, off));
  char* b = static_cast<char*>(L.dev);
  L.geom = Geom{reinterpret_cast<float*>(b + o_xy), reinterpret_cast<float*>(b + o_depth),
                reinterpret_cast<float*>(b + o_co), reinterpret_cast<float*>(b + o_rgb),
                reinterpret_cast<int32_t*>(b + o_rad), reinterpret_cast<uint32_t*>(b + o_tiles)};
  L.bins.capacity = cap;
  L.bins.keys = reinterpret_cast<uint32_t*>(b + o_keys);
  L.bins.vals = reinterpret_cast<uint32_t*>(b + o_vals);
  L.bins.ranges = reinterpret_cast<uint32_t*>(b + o_ranges);
  L.bins.counters = reinterpret_cast<uint32_t*>(b + o_counters);
  L.bins.tile_cull = 1;
  L.tmp = b + o_tmp;
  L.final_T = reinterpret_cast<float*>(b + o_T);
  L.n_contrib = reinterpret_cast<int32_t*>(b + o_nc);
  L.d_hdr = reinterpret_cast<Header*>(b + o_hdr);
  L.d_views = reinterpret_cast<View*>(b + o_hdr + sizeof(Header));
  PVG_HIP(hipHostMalloc(&L.h_stage, s->hdr_bytes, hipHostMallocDefault));
  PVG_HIP(hipHostMalloc(reinterpret_cast<void**>(&L.h_counters), 16, hipHostMallocDefault));
  std::memset(L.h_stage, 0, s->hdr_bytes);
  std::memset(L.h_counters, 0, 16);
  return PVG_OK;
}

void lane_free(Lane& L) {
  for (auto& kv : L.graphs) (void)hipGraphExecDestroy(kv.second);
  L.graphs.clear();
  if (L.h_stage) (void)hipHostFree(L.h_stage);
  if (L.h_counters) (void)hipHostFree(L.h_counters);
  if (L.dev) (void)hipFree(L.dev);
  if (L.done) (void)hipEventDestroy(L.done);
  if (L.stream) (void)hipStreamDestroy(L.stream);
  L = Lane();
}

// The batch's device work, in stream order; capturable (no host sync, no
// memset, no allocation).
int enqueue_batch(pvg_server* s, Lane& L, const ViewSet& vs, const BinPlan& plan) {
  PVG_HIP(hipMemcpyAsync(L.d_hdr, L.h_stage, s->hdr_bytes, hipMemcpyHostToDevice, L.stream));
  const int st = run_batch_forward(vs, L.geom, &L.bins, L.tmp, plan, L.stream);
  if (st != PVG_OK) return st;
  PVG_HIP(hipMemcpyAsync(L.h_counters, L.bins.counters, 16, hipMemcpyDeviceToHost, L.stream));
  return PVG_OK;
}

// Writes the lane's view table for `batch` and launches it.
int launch_batch(pvg_server* s, Lane& L) {
  L.t_launch = now_ns();
  if (s->fault_every > 0 && ++s->launches % s->fault_every == 0) {
    set_error("injected launch fault (PVG_FAULT_INJECT)");
    return PVG_ERR_HIP;
  }
  if (stub(s)) return PVG_OK;
  Header* h = static_cast<Header*>(L.h_stage);
  View* views = reinterpret_cast<View*>(static_cast<char*>(L.h_stage) + sizeof(Header));
  int64_t og = 0, ot = 0, op = 0;
  for (size_t k = 0; k < L.batch.size(); ++k) {
    const Ticket* t = L.batch[k];
    pvg_frame fr{};
    fr.t = t->req.t;
    fr.bg[0] = t->req.bg[0]; fr.bg[1] = t->req.bg[1]; fr.bg[2] = t->req.bg[2];
    View v = make_view(&t->g, &t->req.camera, &fr);
    v.geom_off = og;
    v.tile_off = ot;
    v.img = t->req.dst;
    v.final_T = L.final_T + op;
    v.n_contrib = L.n_contrib + op;
    views[k] = v;
    og += t->n;
    ot += t->tiles;
    op += t->pixels;
  }
  h->live[0] = og;
  h->live[1] = ot;
  h->live[2] = static_cast<int64_t>(L.batch.size());
  h->live[3] = 0;
  L.live_g = og;
  L.live_t = ot;
  // grid buckets: powers of two, clamped to the workspace
  const int64_t gb = std::min(next_pow2(std::max<int64_t>(og, 1), 1 << 16), s->cfg.max_batch_gaussians);
  const int64_t tb = std::min(next_pow2(std::max<int64_t>(ot, 1), 1 << 8), s->max_tiles);
  ViewSet vs;
  std::memset(&vs, 0, sizeof(vs));
  vs.table = L.d_views;
  vs.live = L.d_hdr->live;
  vs.nviews = s->cfg.max_batch;
  vs.total_gauss = gb;
  vs.total_tiles = tb;
  const BinPlan plan = plan_bins(gb, tb, s->cfg.instance_capacity);
  if (!s->cfg.use_graphs) return enqueue_batch(s, L, vs, plan);
  const auto key = std::make_pair(gb, tb);
  auto it = L.graphs.find(key);
  if (it == L.graphs.end()) {
    PVG_HIP(hipStreamBeginCapture(L.stream, hipStreamCaptureModeThreadLocal));
    const int st = enqueue_batch(s, L, vs, plan);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(L.stream, &g);
    if (st != PVG_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) return hip_fail(e2, "hipGraphInstantiate");
    it = L.graphs.emplace(key, ex).first;
    std::lock_guard<std::mutex> lk(s->mu);
    s->graph_builds++;
  }
  PVG_HIP(hipGraphLaunch(it->second, L.stream));
  std::lock_guard<std::mutex> lk(s->mu);
  s->graph_launches++;
  return PVG_OK;
}

void release_scene_ref(pvg_server* s, int32_t scene_id) {
  auto it = s->scenes.find(scene_id);
  if (it == s->scenes.end()) return;
  if (--it->second.pending <= 0 && it->second.unload) {
    if (it->second.buf) (void)hipFree(it->second.buf);
    s->mem_used -= static_cast<int64_t>(it->second.bytes);
    s->scenes.erase(it);
  }
}

void finish(pvg_server* s, Ticket* t, int status, int batch_size, int64_t launch_ns, int64_t instances) {
  t->done = true;
  t->res.status = status;
  t->res.batch_size = batch_size;
  t->res.t_submit_ns = t->res.t_submit_ns ? t->res.t_submit_ns : now_ns();
  t->res.t_launch_ns = launch_ns;
  t->res.t_done_ns = now_ns();
  t->res.num_instances = instances;
  t->res.user_tag = t->req.user_tag;
  if (status == PVG_OK) {
    s->completed++;
    s->lat_ms.push_back((t->res.t_done_ns - t->res.t_submit_ns) * 1e-6);
    s->pixels += static_cast<double>(t->pixels);
    s->t_last = std::max(s->t_last, t->res.t_done_ns);
  } else {
    s->failed++;
  }
  release_scene_ref(s, t->req.scene_id);
}

// FIFO admission into one batch (caller holds the lock).
std::vector<Ticket*> form_batch(pvg_server* s) {
  std::vector<Ticket*> b;
  int64_t g = 0, p = 0, tl = 0;
  while (!s->pending.empty() && static_cast<int32_t>(b.size()) < s->cfg.max_batch) {
    Ticket* t = s->pending.front();
    const bool too_big = t->n > s->cfg.max_batch_gaussians || t->pixels > s->cfg.max_batch_pixels ||
                         t->tiles > s->max_tiles;
    if (too_big) {
      s->pending.pop_front();
      finish(s, t, PVG_ERR_NOMEM, 0, 0, 0);
      continue;
    }
    if (!b.empty() && (t->solo || g + t->n > s->cfg.max_batch_gaussians || p + t->pixels > s->cfg.max_batch_pixels ||
                       tl + t->tiles > s->max_tiles))
      break;
    s->pending.pop_front();
    t->launched = true;
    b.push_back(t);
    g += t->n;
    p += t->pixels;
    tl += t->tiles;
    if (t->solo) break;
  }
  return b;
}

void scheduler_loop(pvg_server* s) {
  if (!stub(s)) (void)hipSetDevice(s->cfg.device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    Lane* free_lane = nullptr;
    s->cv_work.wait(lk, [&] {
      free_lane = nullptr;
      bool busy = false;
      for (auto& L : s->lanes) {
        if (!L.busy && !free_lane) free_lane = &L;
        busy |= L.busy;
      }
      // exit only when nothing is queued or running: a running batch may
      // still requeue its requests (overflow retry)
      return (!s->pending.empty() && free_lane) || (s->stop && s->pending.empty() && !busy);
    });
    if (s->pending.empty()) break;
    std::vector<Ticket*> b = form_batch(s);
    if (b.empty()) {
      s->cv_done.notify_all();
      continue;
    }
    Lane& L = *free_lane;
    L.busy = true;
    L.batch = std::move(b);
    s->batches++;
    s->batch_reqs += static_cast<int64_t>(L.batch.size());
    lk.unlock();
    const int st = launch_batch(s, L);
    if (st == PVG_OK && !stub(s)) (void)hipEventRecord(L.done, L.stream);
    lk.lock();
    if (st != PVG_OK) {
      for (Ticket* t : L.batch) finish(s, t, st, static_cast<int>(L.batch.size()), L.t_launch, 0);
      L.batch.clear();
      L.busy = false;
      s->cv_done.notify_all();
      continue;
    }
    s->inflight.push_back(&L);
    s->cv_poll.notify_all();
  }
  s->cv_poll.notify_all();
}

void retire(pvg_server* s, Lane& L) {
  // caller holds the lock
  const uint32_t over = stub(s) ? 0u : L.h_counters[2];
  const int64_t inst = stub(s) ? 0 : static_cast<int64_t>(L.h_counters[3]);
  const int bs = static_cast<int>(L.batch.size());
  if (over) {
    if (bs > 1) {
      for (auto it = L.batch.rbegin(); it != L.batch.rend(); ++it) {
        (*it)->solo = true;
        (*it)->launched = false;
        s->pending.push_front(*it);
      }
      s->retries += bs;
    } else {
      set_error("a request needs %lld tile instances, more than the capacity %lld", static_cast<long long>(inst),
                static_cast<long long>(s->cfg.instance_capacity));
      finish(s, L.batch[0], PVG_ERR_CAPACITY, 1, L.t_launch, inst);
    }
  } else {
    for (Ticket* t : L.batch) finish(s, t, PVG_OK, bs, L.t_launch, inst);
  }
  L.batch.clear();
  L.busy = false;
}

void poll_loop(pvg_server* s) {
  if (!stub(s)) (void)hipSetDevice(s->cfg.device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_poll.wait(lk, [&] { return !s->inflight.empty() || s->stop; });
    if (s->inflight.empty()) {
      bool busy = false;
      for (auto& L : s->lanes) busy |= L.busy;
      if (s->pending.empty() && !busy) break;
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(50));
      lk.lock();
      continue;
    }
    bool progressed = false;
    for (auto it = s->inflight.begin(); it != s->inflight.end();) {
      Lane& L = **it;
      bool done;
      if (stub(s)) {
        done = now_ns() - L.t_launch >= s->cfg.stub_launch_us * 1000;
      } else {
        const hipError_t e = hipEventQuery(L.done);
        done = e != hipErrorNotReady;
        if (done && e != hipSuccess) {
          set_error("batch failed on the device: %s", hipGetErrorString(e));
          for (Ticket* t : L.batch) finish(s, t, PVG_ERR_HIP, static_cast<int>(L.batch.size()), L.t_launch, 0);
          L.batch.clear();
          L.busy = false;
          it = s->inflight.erase(it);
          progressed = true;
          continue;
        }
      }
      if (done) {
        retire(s, L);
        it = s->inflight.erase(it);
        progressed = true;
      } else {
        ++it;
      }
    }
    if (progressed) {
      s->cv_work.notify_all();
      s->cv_done.notify_all();
    } else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    }
  }
}

}  // namespace

int run_batch_forward(const ViewSet& vs, const Geom& geom, pvg_bins* bins, void* tmp, const BinPlan& plan,
                      hipStream_t s) {
  PVG_HIP(launch_preprocess(vs, geom, s));
  const int st = run_bin_sort(vs, geom, bins, tmp, plan, 0, s);
  if (st != PVG_OK) return st;
  PVG_HIP(launch_render_fwd(vs, geom, bins->vals, bins->ranges, bins->tile_cull != 0, s));
  return PVG_OK;
}

}  // namespace pvg

using namespace pvg;

extern "C" {

int pvg_serve_create(const pvg_serve_config* cfg, pvg_server** out) {
  if (!cfg || !out) { set_error("null argument"); return PVG_ERR_INVALID; }
  if (cfg->max_batch < 1 || cfg->max_batch > 64 || cfg->max_inflight < 1 || cfg->max_inflight > 8 ||
      cfg->max_batch_gaussians < 1 || cfg->max_batch_gaussians > 0xffffffffll || cfg->max_batch_pixels < 1 ||
      cfg->instance_capacity < 1 || cfg->instance_capacity > 0xffffffffll || cfg->mem_budget_bytes < 0) {
    set_error("invalid server configuration");
    return PVG_ERR_INVALID;
  }
  auto* s = new pvg_server();
  s->cfg = *cfg;
  if (const char* fi = std::getenv("PVG_FAULT_INJECT")) s->fault_every = std::max(0ll, std::atoll(fi));
  // tiles of a batch: pixels / 256 plus the partial tiles of up to max_batch views
  s->max_tiles = s->cfg.max_batch_pixels / 256 + static_cast<int64_t>(s->cfg.max_batch) * 512;
  s->hdr_bytes = align256(sizeof(Header) + sizeof(View) * static_cast<size_t>(s->cfg.max_batch));
  if (!stub(s)) {
    const hipError_t e = hipSetDevice(cfg->device);
    if (e != hipSuccess) { delete s; return hip_fail(e, "hipSetDevice"); }
  }
  s->lanes.resize(static_cast<size_t>(cfg->max_inflight));
  int64_t need = 0;
  for (auto& L : s->lanes) {
    const int st = lane_init(s, L);
    need += static_cast<int64_t>(L.dev_bytes);
    if (st != PVG_OK) {
      for (auto& M : s->lanes) lane_free(M);
      delete s;
      return st;
    }
  }
  if (cfg->mem_budget_bytes > 0 && need > cfg->mem_budget_bytes) {
    set_error("batch workspaces need %lld bytes, more than the budget %lld", static_cast<long long>(need),
              static_cast<long long>(cfg->mem_budget_bytes));
    for (auto& L : s->lanes) lane_free(L);
    delete s;
    return PVG_ERR_NOMEM;
  }
  s->mem_used = need;
  s->th_sched = std::thread(scheduler_loop, s);
  s->th_poll = std::thread(poll_loop, s);
  *out = s;
  return PVG_OK;
}

int pvg_serve_load_scene(pvg_server* s, const pvg_gaussians* g, int32_t* scene_id) {
  if (!s || !scene_id || !check_gaussians(g)) {
    if (!g || !s) set_error("null argument");
    return PVG_ERR_INVALID;
  }
  const int64_t n = g->n;
  const int K = (g->sh_degree + 1) * (g->sh_degree + 1);
  const size_t rows[9] = {3, 3, 4, static_cast<size_t>(3 * K), 1, 3, 1, 1, 1};
  size_t bytes = 0;
  for (size_t r : rows) bytes += align256(sizeof(float) * r * static_cast<size_t>(n));
  SceneRec rec;
  rec.bytes = bytes;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->cfg.mem_budget_bytes > 0 && s->mem_used + static_cast<int64_t>(bytes) > s->cfg.mem_budget_bytes) {
      set_error("scene of %zu bytes exceeds the remaining memory budget", bytes);
      return PVG_ERR_NOMEM;
    }
    s->mem_used += static_cast<int64_t>(bytes);
  }
  rec.g = *g;
  if (!stub(s) && n > 0) {
    hipError_t e = hipSetDevice(s->cfg.device);
    if (e == hipSuccess) e = hipMalloc(&rec.buf, bytes);
    if (e != hipSuccess) {
      std::lock_guard<std::mutex> lk(s->mu);
      s->mem_used -= static_cast<int64_t>(bytes);
      return hip_fail(e, "hipMalloc(scene)");
    }
    const float* src[9] = {g->mu, g->scale, g->rot, g->sh, g->opacity, g->vel, g->period, g->tau, g->beta};
    const float** dst[9] = {&rec.g.mu, &rec.g.scale, &rec.g.rot, &rec.g.sh, &rec.g.opacity,
                            &rec.g.vel, &rec.g.period, &rec.g.tau, &rec.g.beta};
    char* p = static_cast<char*>(rec.buf);
    for (int k = 0; k < 9; ++k) {
      const size_t b = sizeof(float) * rows[k] * static_cast<size_t>(n);
      if (e == hipSuccess) e = hipMemcpy(p, src[k], b, hipMemcpyDeviceToDevice);
      *dst[k] = reinterpret_cast<const float*>(p);
      p += align256(b);
    }
    if (e != hipSuccess) {
      (void)hipFree(rec.buf);
      std::lock_guard<std::mutex> lk(s->mu);
      s->mem_used -= static_cast<int64_t>(bytes);
      return hip_fail(e, "hipMemcpy(scene)");
    }
  }
  std::lock_guard<std::mutex> lk(s->mu);
  rec.id = s->next_scene++;
  s->scenes[rec.id] = rec;
  *scene_id = rec.id;
  return PVG_OK;
}

int pvg_serve_unload_scene(pvg_server* s, int32_t scene_id) {
  if (!s) { set_error("null server"); return PVG_ERR_INVALID; }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->scenes.find(scene_id);
  if (it == s->scenes.end() || it->second.unload) { set_error("unknown scene %d", scene_id); return PVG_ERR_NOT_FOUND; }
  it->second.unload = true;
  if (it->second.pending <= 0) {
    if (it->second.buf) (void)hipFree(it->second.buf);
    s->mem_used -= static_cast<int64_t>(it->second.bytes);
    s->scenes.erase(it);
  }
  return PVG_OK;
}

int pvg_serve_submit(pvg_server* s, const pvg_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) { set_error("null argument"); return PVG_ERR_INVALID; }
  if (!check_camera(&req->camera)) return PVG_ERR_INVALID;
  if (!req->dst && !stub(s)) { set_error("request dst is null"); return PVG_ERR_INVALID; }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) { set_error("server is shutting down"); return PVG_ERR_BUSY; }
  auto it = s->scenes.find(req->scene_id);
  if (it == s->scenes.end() || it->second.unload) { set_error("unknown scene %d", req->scene_id); return PVG_ERR_NOT_FOUND; }
  auto* t = new Ticket();
  t->id = s->next_ticket++;
  t->req = *req;
  t->g = it->second.g;
  t->n = it->second.g.n;
  t->pixels = static_cast<int64_t>(req->camera.width) * req->camera.height;
  t->tiles = static_cast<int64_t>((req->camera.width + kTile - 1) / kTile) * ((req->camera.height + kTile - 1) / kTile);
  t->res.t_submit_ns = now_ns();
  if (s->t_first == 0) s->t_first = t->res.t_submit_ns;
  it->second.pending++;
  s->tickets[t->id] = t;
  s->pending.push_back(t);
  *ticket = t->id;
  s->cv_work.notify_all();
  return PVG_OK;
}

int pvg_serve_wait(pvg_server* s, uint64_t ticket, int64_t timeout_us, pvg_result* out) {
  if (!s) { set_error("null server"); return PVG_ERR_INVALID; }
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) { set_error("unknown ticket"); return PVG_ERR_NOT_FOUND; }
  Ticket* t = it->second;
  if (timeout_us < 0) {
    s->cv_done.wait(lk, [&] { return t->done; });
  } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return t->done; })) {
    return PVG_ERR_TIMEOUT;
  }
  if (out) *out = t->res;
  return PVG_OK;
}

int pvg_serve_poll(pvg_server* s, uint64_t ticket, int32_t* done) {
  if (!s || !done) { set_error("null argument"); return PVG_ERR_INVALID; }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) { set_error("unknown ticket"); return PVG_ERR_NOT_FOUND; }
  *done = it->second->done ? 1 : 0;
  return PVG_OK;
}

int pvg_serve_release(pvg_server* s, uint64_t ticket) {
  if (!s) { set_error("null server"); return PVG_ERR_INVALID; }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) { set_error("unknown ticket"); return PVG_ERR_NOT_FOUND; }
  Ticket* t = it->second;
  if (!t->done) {
    if (t->launched) { set_error("ticket already launched"); return PVG_ERR_BUSY; }
    s->pending.erase(std::remove(s->pending.begin(), s->pending.end(), t), s->pending.end());
    release_scene_ref(s, t->req.scene_id);
  }
  s->tickets.erase(it);
  delete t;
  return PVG_OK;
}

int pvg_serve_stats(pvg_server* s, pvg_serve_report* out) {
  if (!s || !out) { set_error("null argument"); return PVG_ERR_INVALID; }
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->completed = s->completed;
  out->failed = s->failed;
  out->batches = s->batches;
  out->retries = s->retries;
  out->graph_launches = s->graph_launches;
  out->graph_builds = s->graph_builds;
  out->mean_batch = s->batches ? static_cast<double>(s->batch_reqs) / static_cast<double>(s->batches) : 0.0;
  if (!s->lat_ms.empty()) {
    std::vector<double> v = s->lat_ms;
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
      const size_t k = std::min(v.size() - 1, static_cast<size_t>(q * static_cast<double>(v.size() - 1) + 0.5));
      return v[k];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
  }
  out->span_s = s->t_last > s->t_first ? (s->t_last - s->t_first) * 1e-9 : 0.0;
  out->mpix_per_s = out->span_s > 0 ? s->pixels / out->span_s / 1e6 : 0.0;
  return PVG_OK;
}

int pvg_serve_reset_stats(pvg_server* s) {
  if (!s) { set_error("null server"); return PVG_ERR_INVALID; }
  std::lock_guard<std::mutex> lk(s->mu);
  s->lat_ms.clear();
  s->completed = s->failed = s->batches = s->batch_reqs = s->retries = s->graph_launches = s->graph_builds = 0;
  s->pixels = 0.0;
  s->t_first = s->t_last = 0;
  return PVG_OK;
}

int pvg_serve_destroy(pvg_server* s) {
  if (!s) { set_error("null server"); return PVG_ERR_INVALID; }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
    s->cv_poll.notify_all();
  }
  if (s->th_sched.joinable()) s->th_sched.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->cv_poll.notify_all();
  }
  if (s->th_poll.joinable()) s->th_poll.join();
  for (auto& L : s->lanes) {
    if (L.stream) (void)hipStreamSynchronize(L.stream);
    lane_free(L);
  }
  for (auto& kv : s->scenes)
    if (kv.second.buf) (void)hipFree(kv.second.buf);
  for (auto& kv : s->tickets) delete kv.second;
  delete s;
  return PVG_OK;
}

}  // extern "C"
