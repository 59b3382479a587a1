/*
 * pvg_serve.h - continuous-batching render server of libpvg.
 *
 * Serves the paper's inference path, a single I^ = Render({H_i(t)}; E, I)
 * per request (Sec. 3.2, Eq. (8)), for several scenes kept resident in HBM.
 * A server thread admits queued requests (mixed resolution, time stamp and
 * scene) into batches that fit the per-batch workspace, writes the batch's
 * view table, and launches one preprocess / bin-sort / composite sequence for
 * the whole batch (replayed from a captured hipGraph when enabled).  Up to
 * max_inflight batches run at once, each on its own stream, so requests that
 * arrive while a batch is on the GPU are admitted as soon as a slot frees and
 * their work overlaps the running batch.  A batch whose tile instances exceed
 * the capacity is split and its requests are rerun one by one; a request that
 * alone exceeds it fails with PVG_ERR_CAPACITY.
 *
 * A request's image is bit-for-bit the image pvg_preprocess + pvg_bin_sort +
 * pvg_render_fwd give for the same scene, camera, time and background,
 * whichever batch it shares.
 *
 * Threading: every pvg_serve_* call is thread safe.  Status codes and error
 * messages are those of pvg.h.
 */
#ifndef PVG_SERVE_H
#define PVG_SERVE_H

#include "pvg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pvg_server pvg_server;

typedef struct pvg_serve_config {
  int32_t device;              /* HIP device ordinal */
  int32_t max_batch;           /* requests per batch, 1..64 (1 = one request per launch) */
  int32_t max_inflight;        /* batches on the GPU at once, 1..8, each on its own stream */
  int32_t use_graphs;          /* 1: replay each batch shape as a captured hipGraph */
  int64_t mem_budget_bytes;    /* device memory for scene copies and batch workspaces */
  int64_t max_batch_gaussians; /* sum of the scenes' n over one batch */
  int64_t max_batch_pixels;    /* sum of width * height over one batch */
  int64_t instance_capacity;   /* tile instances per batch (< 2^32) */
  int64_t stub_launch_us;      /* > 0: no GPU work at all; a batch "completes" after this many
                                  microseconds (scheduling tests on hosts without a GPU) */
} pvg_serve_config;

typedef struct pvg_request {
  int32_t scene_id;
  int32_t reserved;
  pvg_camera camera;           /* any resolution up to the batch pixel budget */
  float t;                     /* render time */
  float bg[3];                 /* background */
  float* dst;                  /* device [3][height][width] image, caller-owned; must stay valid
                                  until the request completes */
  int64_t user_tag;            /* returned unchanged in the result */
} pvg_request;

typedef struct pvg_result {
  int32_t status;              /* PVG_OK or the request's error */
  int32_t batch_size;          /* requests in the batch that rendered it */
  int64_t t_submit_ns;         /* steady-clock times: submission, launch, completion seen */
  int64_t t_launch_ns;
  int64_t t_done_ns;
  int64_t num_instances;       /* tile instances of the request's batch */
  int64_t user_tag;
} pvg_result;

typedef struct pvg_serve_report {
  int64_t completed;           /* requests finished with PVG_OK since the last reset */
  int64_t failed;
  int64_t batches;
  int64_t retries;             /* requests rerun alone after a batch overflowed */
  int64_t graph_launches;
  int64_t graph_builds;
  double mean_batch;           /* requests per batch */
  double p50_ms, p99_ms;       /* latency percentiles, submission -> completion seen */
  double mpix_per_s;           /* rendered pixels / (last completion - first submission) */
  double span_s;
} pvg_serve_report;

/* Creates a server and its batch workspaces (counted against the budget).
 * Test hook: with PVG_FAULT_INJECT=k (k >= 1) in the environment when the
 * server is created, every k-th batch launch fails before any device work;
 * its tickets finish with PVG_ERR_HIP and the server carries on. */
int pvg_serve_create(const pvg_serve_config* cfg, pvg_server** out);
/* Copies a scene (device arrays) into server-owned HBM; fails with
 * PVG_ERR_NOMEM beyond the memory budget. */
int pvg_serve_load_scene(pvg_server* s, const pvg_gaussians* g, int32_t* scene_id);
/* Frees a scene; deferred until its pending requests are done. */
int pvg_serve_unload_scene(pvg_server* s, int32_t scene_id);
/* Queues a request; never blocks on the GPU. */
int pvg_serve_submit(pvg_server* s, const pvg_request* req, uint64_t* ticket);
/* Waits up to timeout_us (< 0: forever) for a ticket; PVG_ERR_TIMEOUT if not done. */
int pvg_serve_wait(pvg_server* s, uint64_t ticket, int64_t timeout_us, pvg_result* out);
int pvg_serve_poll(pvg_server* s, uint64_t ticket, int32_t* done);
/* Forgets a finished ticket, or cancels a queued one (PVG_ERR_BUSY once launched). */
int pvg_serve_release(pvg_server* s, uint64_t ticket);
int pvg_serve_stats(pvg_server* s, pvg_serve_report* out);
int pvg_serve_reset_stats(pvg_server* s);
/* Drains queued and in-flight work, then frees everything. */
int pvg_serve_destroy(pvg_server* s);

#ifdef __cplusplus
}
#endif
#endif /* PVG_SERVE_H */
