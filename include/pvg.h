/*
 * pvg.h - C ABI of the MI355X (gfx950) PVG splatting rasterizer.
 *
 * The library renders the image of a set of Periodic Vibration Gaussians
 * (PVG, arXiv 2311.18561) at a time t seen by a camera (E, I), and
 * differentiates it: I^ = Render({H_i(t)}; E, I) (Sec. 3.2, Eq. (8)), where
 * H(t) = {mu~(t), q, s, o~(t), c} (Eq. (5)),
 *   mu~(t) = mu + (l / 2pi) sin(2pi (t - tau) / l) v      (Eq. (6)),
 *   o~(t)  = o exp(-(t - tau)^2 / (2 beta^2))              (Eq. (7)),
 * projected with Sigma' = J W Sigma W^T J^T (Sec. 3.1, Eq. (2)) and
 * alpha-blended front to back in depth order, C = sum_i T_i alpha_i c_i
 * (Sec. 3.1, Eq. (3)), over 16x16 pixel tiles.  The temporal-smoothing render
 * of Sec. 3.4 (Eq. (12)) is the same call with frame.dt != 0: the Gaussians are
 * evaluated at t and moved by the flow translation v_bar * dt, with
 * v_bar = v exp(-rho / 2), rho = beta / l (Eq. (10)).
 *
 * Conventions.
 *   - Every array is FP32 (or the stated integer type), contiguous, on the
 *     device unless stated otherwise.  Parameter arrays are structure-of-arrays:
 *     "[3][n]" means element (c, i) is at c * n + i.
 *   - The caller owns every input, output and workspace buffer.  The library
 *     never frees caller memory and allocates none in the rendering calls.
 *     A workspace (`tmp`) starts on a 256-byte boundary (hipMalloc's and
 *     torch's allocations do): the library cuts it into 256-byte aligned
 *     parts that its kernels read 16 bytes at a time; a misaligned one is
 *     PVG_ERR_INVALID.
 *   - Every call is asynchronous on the caller's HIP stream (a hipStream_t
 *     passed as void*, NULL = the null stream) and returns an int status:
 *     0 = PVG_OK, negative = error.  Arguments are validated on the host
 *     (null pointers, n < 0, degree outside 0..3, non-positive image size or
 *     focal length, capacity < 0); a failed validation launches nothing.
 *     No C++ exception crosses the ABI and the library never aborts.
 *     pvg_last_error() returns the thread's last error message.
 *   - NaN parameters propagate: a Gaussian whose camera depth, covariance or
 *     tile rectangle is NaN is treated as invisible; NaN colours propagate.
 *   - Camera: x_cam = R x_world + T (R row-major), pinhole (fx, fy, cx, cy),
 *     looking down +z, x right, y down.  Pixel (i, j) is sampled at the point
 *     whose projected coordinates minus (0.5, 0.5) equal (i, j).
 *   - The fixed constants of the rasterizer (the paper leaves them open):
 *     16x16 tiles, near plane at camera.znear, Jacobian evaluated at the point
 *     clamped to 1.3x the half field of view, +0.3 px^2 on the 2D covariance,
 *     radius ceil(3 sqrt(lambda_max)) with a 0.1 floor under the eigenvalue
 *     discriminant, alpha = min(0.99, o~ G), pairs with alpha < 1/255 or a
 *     positive exponent skipped, a pixel stops before the Gaussian that would
 *     take its transmittance below 1e-4.  Colour: real spherical harmonics of
 *     degree <= 3 (index l*l + l + m, no Condon-Shortley phase) of the unit
 *     direction from the camera centre to the (translated) mean, plus 0.5,
 *     clamped at 0.  Order within a tile: camera depth, then Gaussian index.
 */
#ifndef PVG_H
#define PVG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum pvg_status {
  PVG_OK = 0,
  PVG_ERR_INVALID = -1,   /* bad argument */
  PVG_ERR_CAPACITY = -2,  /* instance buffers too small; bins->num_instances holds the need */
  PVG_ERR_NOMEM = -3,     /* a workspace or memory budget is too small */
  PVG_ERR_BUSY = -4,      /* the resource is in use (e.g. a scene with pending requests) */
  PVG_ERR_HIP = -5,       /* a HIP runtime call failed; pvg_last_error() has its message */
  PVG_ERR_NOT_FOUND = -6, /* unknown scene id or ticket */
  PVG_ERR_TIMEOUT = -7    /* a wait timed out */
};

/* The per-point parameter set {mu, q, s, o, c, tau, beta, v} of Sec. 3.2,
 * plus the cycle length l per point (a constant array reproduces the paper's
 * scene-wide l).  All device pointers, read only. */
typedef struct pvg_gaussians {
  int64_t n;           /* number of Gaussians, >= 0 */
  int32_t sh_degree;   /* 0..3; K = (sh_degree + 1)^2 coefficients per channel */
  int32_t reserved;
  const float* mu;      /* [3][n] mean position (world) */
  const float* scale;   /* [3][n] scale s > 0 (linear, not log) */
  const float* rot;     /* [4][n] quaternion (w, x, y, z), any nonzero norm */
  const float* sh;      /* [K][3][n] colour coefficients, element (k, ch, i) */
  const float* opacity; /* [n] peak opacity o in (0, 1] (already activated) */
  const float* vel;     /* [3][n] velocity v = d mu~ / dt at t = tau */
  const float* period;  /* [n] cycle length l > 0 */
  const float* tau;     /* [n] life peak tau */
  const float* beta;    /* [n] lifespan beta > 0 */
} pvg_gaussians;

/* Gradients in the layout of pvg_gaussians (device, written or accumulated).
 * densify_grad and densify_count (optional, both or neither, device [n]):
 * the statistics of the adaptive control (Sec. 3.3).  For every view of the
 * call in which Gaussian i is visible, the adjoint adds the norm of the
 * gradient of the loss with respect to its 2D mean in normalized device
 * coordinates, |(W/2 dL/dx, H/2 dL/dy)| with (x, y) in pixels, to
 * densify_grad[i] and 1 to densify_count[i]; they are never cleared. */
typedef struct pvg_gaussians_grad {
  float* mu; float* scale; float* rot; float* sh; float* opacity;
  float* vel; float* period; float* tau; float* beta;
  float* densify_grad; float* densify_count;
} pvg_gaussians_grad;

typedef struct pvg_camera { /* host struct, passed by pointer */
  float R[9];               /* world -> camera rotation, row-major */
  float T[3];               /* world -> camera translation */
  float fx, fy, cx, cy;     /* pinhole intrinsics in pixels, fx, fy > 0 */
  int32_t width, height;    /* image size in pixels, 1 .. 65535 (partial tiles allowed) */
  float znear;              /* > 0: Gaussians with camera z <= znear are culled */
} pvg_camera;

typedef struct pvg_frame {  /* host struct */
  float t;                  /* render time */
  float dt;                 /* flow-translation interval of Eq. (12); 0 = plain render */
  int32_t advect_mode;      /* 0: translate by v_bar = v exp(-beta / (2 l)) (Eq. (10)); 1: by v */
  float bg[3];              /* constant background added as T_final * bg */
} pvg_frame;

/* Per-Gaussian projected record (pvg_preprocess output; caller-allocated, length n). */
typedef struct pvg_geom {
  int64_t n;
  float* xy;          /* [n][2] pixel-space 2D mean */
  float* depth;       /* [n] camera-space z (the sort key) */
  float* conic_op;    /* [n][4] inverse 2D covariance (A, B, C) and opacity o~(t) */
  float* rgb;         /* [n][3] colour; a channel clamped at zero is stored as -0 (the adjoint reads the clamp from the sign) */
  int32_t* radius;    /* [n] screen radius in pixels; 0 = invisible */
  uint32_t* tiles;    /* [n] number of tiles the Gaussian's rectangle touches */
  float* feat;        /* [n][4] optional (may be NULL): mean velocity v~ = v exp(-beta / (2 l))
                         (Sec. 3.4) and staticness rho = beta / l, written by the preprocess and
                         read by the velocity and staticness channels */
} pvg_geom;

/* Tile instances: one (tile, Gaussian) pair per tile a visible Gaussian's
 * rectangle touches, sorted by (tile, depth, index). */
typedef struct pvg_bins {
  int64_t capacity;     /* instance capacity of each half of keys / vals, >= 0 */
  uint32_t* keys;       /* [2][capacity] tile id per instance (double buffer) */
  uint32_t* vals;       /* [2][capacity] Gaussian index; sorted result in vals[0 .. M) */
  uint32_t* ranges;     /* [tiles][2] [first, last + 1) of each tile in vals */
  uint32_t* counters;   /* [4] device: listed instances, visible count, overflow flag,
                           the count checked against the capacity (saturated to 2^32 - 1) */
  uint32_t* first;      /* [n] optional (may be NULL): index, in emission order, of each visible
                           Gaussian's first instance; pvg_render_bwd needs it */
  int64_t num_instances;/* host output of a synchronous count (sync_count = 1): listed instances */
  int64_t num_visible;  /* host output of a synchronous count */
  int32_t tile_cull;    /* 0: one instance per tile of each rectangle (Sec. 3.1 as in 3D Gaussian
                           splatting); 1: only the tiles where the Gaussian can reach alpha >= 1/255
                           at some pixel (per tile row, the columns meeting the x-extent of the
                           alpha = 1/255 ellipse, widened for rounding), which leaves every image
                           and gradient unchanged and shortens the lists; n_contrib then counts
                           positions in the shorter lists and `first` indexes listed instances.
                           The capacity bounds the listed instances and, with culling, also the
                           rectangle rows (16 bytes of bin_sort scratch each). */
  int32_t reserved;
  uint32_t* rows;       /* [capacity][2] optional (tile_cull = 1): per rectangle row of each
                           visible Gaussian, (emission index of the row's first listed instance,
                           first reached column | count << 16); pvg_render_bwd needs it with
                           tile_cull = 1 */
  uint32_t* row_base;   /* [n] optional (tile_cull = 1): index into rows of grid row 0 of each
                           visible Gaussian, modulo 2^32; pvg_render_bwd needs it with tile_cull = 1 */
} pvg_bins;

typedef struct pvg_ws_sizes {
  size_t bin_tmp_bytes;    /* scratch of pvg_bin_sort */
  size_t bwd_tmp_bytes;    /* scratch of pvg_render_bwd (grows with n, the tiles and the capacity) */
  int64_t num_tiles;       /* ceil(width / 16) * ceil(height / 16) */
} pvg_ws_sizes;

/* Scratch sizes for n Gaussians, one width x height image and an instance
 * capacity.  Host only; does not touch the device. */
int pvg_workspace_query(int64_t n, int32_t width, int32_t height, int64_t capacity, pvg_ws_sizes* out);

/* Per-Gaussian stage (Eqs. (6), (7), (10), (12), Eq. (2), colour): temporal
 * state at frame->t (translated by frame->dt), view transform and near cull,
 * 3D covariance R(q) S S^T R(q)^T, EWA 2D covariance and its inverse, screen
 * radius, tile rectangle and count, colour.  Writes every field of `out`
 * (out->n must equal g->n). */
int pvg_preprocess(const pvg_gaussians* g, const pvg_camera* cam, const pvg_frame* frame,
                   pvg_geom* out, void* stream);

/* pvg_preprocess for n_views views of the same Gaussians (a training step's
 * cameras and times, Sec. 3.4: H(t) and the translated H^(t + dt)): outs[k]
 * receives exactly what pvg_preprocess(g, &cams[k], &frames[k], &outs[k])
 * would write.  The views are processed eight at a time in one pass over the
 * parameters, so each Gaussian's parameters are read from HBM once per pass.
 * cams, frames and outs are host arrays of n_views entries (the geom arrays
 * in them are device memory, outs[k].n must equal g->n, and no two outs may
 * share memory).  PVG_ERR_INVALID on null arrays, n_views < 1 or an invalid
 * camera, frame or geom; asynchronous on `stream`. */
int pvg_preprocess_views(const pvg_gaussians* g, int32_t n_views, const pvg_camera* cams,
                         const pvg_frame* frames, pvg_geom* outs, void* stream);

/* Depth ordering per tile (Sec. 3.1): emits one instance per (visible
 * Gaussian, touched tile) and sorts them by (tile, camera depth, index)
 * with an LDS-histogram LSD radix sort; writes the per-tile ranges.
 * tmp: bin_tmp_bytes of scratch from pvg_workspace_query (same n, image and
 * capacity).  sync_count = 1: the instance count is read back to the host
 * (bins->num_instances, num_visible); if it exceeds bins->capacity the call
 * returns PVG_ERR_CAPACITY and sorts nothing.  sync_count = 0: nothing is
 * read back; on overflow counters[2] is set, every tile range is empty and
 * the render shows only the background. */
int pvg_bin_sort(const pvg_geom* geom, const pvg_camera* cam, pvg_bins* bins, void* tmp,
                 size_t tmp_bytes, int32_t sync_count, void* stream);

/* pvg_bin_sort without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP stream capture, tight serving loops, hosts
 * that forbid allocation): the scratch is a library-held device array of
 * PVG_NOALLOC_SCRATCH_BYTES, one per device, held until the process ends.
 * Same arguments, outputs, sync_count semantics and errors as pvg_bin_sort,
 * with identical results; PVG_ERR_NOMEM (nothing launched) when the scratch
 * that n, the camera's tile count and bins->capacity need (the
 * bin_tmp_bytes of pvg_workspace_query) exceeds PVG_NOALLOC_SCRATCH_BYTES.
 * Calls no device allocation or free; the stage profiler records no events
 * for it.  Every call on a device shares that device's array, which keeps
 * the last call's contents: calls ordered on one stream are safe, calls
 * that overlap on one device (other streams, other threads) race. */
#define PVG_NOALLOC_SCRATCH_BYTES (256ull << 20)
int pvg_bin_sort_noalloc(const pvg_geom* geom, const pvg_camera* cam, pvg_bins* bins, int32_t sync_count,
                         void* stream);

/* Front-to-back alpha blending of each pixel's tile list (Eq. (3)).
 * img [3][height][width] = C + T_final * bg; final_T [height][width];
 * n_contrib [height][width] = list position of the last contributor + 1. */
int pvg_render_fwd(const pvg_geom* geom, const pvg_bins* bins, const pvg_camera* cam,
                   const pvg_frame* frame, float* img, float* final_T, int32_t* n_contrib,
                   void* stream);

/* Extra render channels of the flexible rendering in Sec. 3.1, where a
 * Gaussian's camera depth z takes the place of its colour in Eq. (3).  Every
 * pointer is optional (NULL: not rendered / no gradient), device memory of
 * [height][width] floats, owned by the caller:
 *   depth      forward output: sum over contributors of T_i alpha_i z_i, or
 *              with depth_normalized the normalized depth of Sec. 3.1,
 *              sum T_i alpha_i z_i / sum T_i alpha_i (0 on pixels that no
 *              Gaussian reaches); for the adjoint with depth_normalized and
 *              dL_ddepth, the forward's normalized depth (read only);
 *   dL_ddepth  adjoint input: upstream gradient of `depth`;
 *   dL_dT      adjoint input: upstream gradient of final_T;
 *   opacity    forward output: the rendered opacity O = sum T_i alpha_i =
 *              1 - final_T (the opacity of the sky composite and the opacity
 *              loss of Sec. 3.4);
 *   dL_dopacity adjoint input: upstream gradient of `opacity` (it adds to
 *              dL_dT with the opposite sign);
 *   vbar, rho  the velocity map and the staticness map (Sec. 3.4 and the
 *              dynamic element analysis), blending each Gaussian's v~ and
 *              rho from geom->feat, which must then be non-NULL (the preprocess
 *              fills it); dL_dvbar and dL_drho their upstream gradients, which
 *              reach v, beta and l.
 * depth_normalized (0 or 1) selects the depth above; the adjoint must be
 * given the forward's choice.
 * feature_grad (adjoint only, optional): the view composited three channels
 * of a per-Gaussian feature vector in place of the colour (its geom->rgb
 * points at them, [n][3]; the semantic vectors of Sec. 4.1 go through such
 * views three channels at a time).  Their gradient is added into
 * feature_grad ([3][n] device, never cleared), no channel counts as
 * clamped, and the colour's SH and view-direction chain is skipped, so the
 * parameters receive only the compositing's gradient. */
typedef struct pvg_channels {
  float* depth;
  const float* dL_ddepth;
  const float* dL_dT;
  float* vbar;             /* forward output [3][height][width]: sum T_i alpha_i v~_i (world frame) */
  float* rho;              /* forward output [height][width]: sum T_i alpha_i rho_i */
  const float* dL_dvbar;   /* adjoint input [3][height][width] */
  const float* dL_drho;    /* adjoint input [height][width] */
  int32_t depth_normalized;
  float* feature_grad;
  float* opacity;            /* forward output [height][width]: 1 - final_T */
  const float* dL_dopacity;  /* adjoint input [height][width] */
} pvg_channels;

/* pvg_render_fwd that also writes the channels requested in `channels`
 * (NULL: exactly pvg_render_fwd).  Images, final_T and n_contrib are those
 * of pvg_render_fwd bit for bit. */
int pvg_render_fwd_channels(const pvg_geom* geom, const pvg_bins* bins, const pvg_camera* cam,
                            const pvg_frame* frame, float* img, float* final_T, int32_t* n_contrib,
                            const pvg_channels* channels, void* stream);

/* Adjoint of pvg_render_fwd and pvg_preprocess: given dL/dimg [3][H][W] and
 * the forward's final_T and n_contrib, writes (accumulate = 0) or adds
 * (accumulate = 1) dL/d(every array of g) into grad.  geom and bins must be
 * the forward's, or a deterministic recomputation of them (same inputs give
 * bit-identical geom and bins), and bins->first must have been filled.
 * tmp: bwd_tmp_bytes of scratch for the same n, image and capacity.  The
 * per-Gaussian sums are formed without atomics, so the result is bitwise
 * reproducible. */
int pvg_render_bwd(const pvg_gaussians* g, const pvg_camera* cam, const pvg_frame* frame,
                   const pvg_geom* geom, const pvg_bins* bins, const float* final_T,
                   const int32_t* n_contrib, const float* dL_dimg, pvg_gaussians_grad* grad,
                   int32_t accumulate, void* tmp, size_t tmp_bytes, void* stream);

/* Adjoint of several renders of one set of Gaussians (several cameras, and
 * H(t) with the flow-translated H(t + dt) of Sec. 3.4), summed into one
 * gradient: for each view the compositing adjoint as in pvg_render_bwd, then
 * one pass over the Gaussians that applies every view's per-Gaussian chain
 * rule and writes (accumulate = 0) or adds (accumulate = 1) the sum once, so
 * the parameters are read and the gradient written once rather than per view.
 * Host arrays of n_views entries: cams, frames, geoms, bins (as for
 * pvg_render_bwd, all for the same g), and device pointers final_T[v],
 * n_contrib[v], dL_dimg[v]; dL_dimg[v] = NULL skips view v.  tmp: at least
 * pvg_bwd_views_tmp_bytes(n, n_views, largest width and height, largest
 * bins capacity) bytes.  The views' compositing adjoints run concurrently on
 * library-owned side streams (default priority) forked from and joined back
 * into `stream`; under stream capture they run on `stream` alone.  Bitwise
 * reproducible (no atomics). */
int pvg_render_bwd_views(const pvg_gaussians* g, int32_t n_views, const pvg_camera* cams,
                         const pvg_frame* frames, const pvg_geom* geoms, const pvg_bins* bins,
                         const float* const* final_T, const int32_t* const* n_contrib,
                         const float* const* dL_dimg, pvg_gaussians_grad* grad, int32_t accumulate,
                         void* tmp, size_t tmp_bytes, void* stream);
/* pvg_render_bwd_views with the channels' upstream gradients: `channels`
 * (host array of n_views entries, or NULL: exactly pvg_render_bwd_views)
 * gives view k's dL_ddepth and dL_dT (either may be NULL; `depth` is
 * ignored).  The gradient of the depth channel reaches the mean, the flow
 * offset and the temporal parameters through z; that of final_T reaches
 * every parameter alpha depends on.  A view whose dL_dimg is NULL is skipped
 * with its channel gradients (pass zeros to use only the channels).  Same
 * scratch (pvg_bwd_views_tmp_bytes), streams and errors. */
int pvg_render_bwd_views_channels(const pvg_gaussians* g, int32_t n_views, const pvg_camera* cams,
                                  const pvg_frame* frames, const pvg_geom* geoms, const pvg_bins* bins,
                                  const float* const* final_T, const int32_t* const* n_contrib,
                                  const float* const* dL_dimg, const pvg_channels* channels,
                                  pvg_gaussians_grad* grad, int32_t accumulate, void* tmp,
                                  size_t tmp_bytes, void* stream);
/* Feature compositing (Sec. 4.1, Eq. (3)): every Gaussian carries an
 * N-vector (the semantic class scores), blended in place of the colour with
 * no background term, out[c] = sum_i T_i alpha_i f_i,c, all N channels in
 * one walk of each tile list.  feat: device [n][ld] floats, row stride ld >=
 * n_ch, channels 0 .. n_ch - 1 of each row used, read only; 1 <= n_ch <=
 * PVG_MAX_FEATURE_CHANNELS (split wider vectors into column groups: the
 * adjoint is linear in the upstream gradient).  out: device [n_ch][height]
 * [width]; final_T and n_contrib as in pvg_render_fwd, bit-identical to a
 * colour render of the same geom and bins, and what the adjoint needs.
 * PVG_ERR_INVALID on an invalid geom, bins or camera, a null pointer, n_ch
 * out of range or ld < n_ch; asynchronous on `stream`. */
#define PVG_MAX_FEATURE_CHANNELS 32
int pvg_render_features(const pvg_geom* geom, const pvg_bins* bins, const pvg_camera* cam, const float* feat,
                        int64_t ld, int32_t n_ch, float* out, float* final_T, int32_t* n_contrib, void* stream);

/* Scratch bytes of pvg_render_features_bwd for n Gaussians, n_views views,
 * n_ch channels and the largest bins capacity among the views.
 * PVG_ERR_INVALID on negative or out-of-range sizes or a null output. */
int pvg_features_bwd_tmp_bytes(int64_t n, int32_t n_views, int32_t n_ch, int64_t max_capacity, size_t* bytes);

/* Adjoint of pvg_render_features over several views of one set of Gaussians
 * (cameras, and H(t) with the flow-translated H(t + dt) of Sec. 3.4), given
 * dL_dout[k] (device [n_ch][height][width]; NULL skips view k) and the
 * forward's final_T[k] and n_contrib[k].  geoms and bins as for
 * pvg_render_bwd_views.  The vectors' gradient is added into feat_grad
 * (device [n][ld], never cleared); the parameters' gradient, which reaches
 * them through alpha only, is written (accumulate = 0) or added (1) into
 * grad: the SH arrays receive zeros, or are left as they are.  The views
 * run in order on `stream` (each adds into feat_grad).  tmp: at least
 * pvg_features_bwd_tmp_bytes bytes.  Without atomics: bitwise reproducible.
 * Errors as for pvg_render_bwd_views, and PVG_ERR_INVALID on n_ch out of
 * range, ld < n_ch, or a null feat or feat_grad with n > 0. */
int pvg_render_features_bwd(const pvg_gaussians* g, int32_t n_views, const pvg_camera* cams,
                            const pvg_frame* frames, const pvg_geom* geoms, const pvg_bins* bins,
                            const float* const* final_T, const int32_t* const* n_contrib, const float* feat,
                            int64_t ld, int32_t n_ch, const float* const* dL_dout, float* feat_grad,
                            pvg_gaussians_grad* grad, int32_t accumulate, void* tmp, size_t tmp_bytes,
                            void* stream);

/* Position-aware adaptive control (Sec. 3.3, Eq. (9), and the split rules
 * of the implementation details in the appendix).  gamma(mu) = 1 if |mu| <
 * 2 r, else |mu| / r - 1.  A Gaussian whose mean view-space gradient
 * densify_grad / densify_count (0 when the count is 0; see
 * pvg_gaussians_grad) is at least grad_threshold is cloned when max(s) <=
 * clone_scale * gamma(mu) and split otherwise.  Any Gaussian, new ones
 * included, is pruned when max(s) > prune_scale * gamma(mu) or o <
 * min_opacity.  A clone copies every parameter.  A split replaces the
 * Gaussian by two children k = 0, 1: scale split_scale_decay * s, tau + dtau,
 * beta split_beta_decay * beta, mean mu + R(q) (s * eps_k) + dtau v~, with
 * dtau = beta eps_k3 and v~ = v exp(-beta / (2 l)).  All decisions are FP32. */
typedef struct pvg_densify_config {
  float grad_threshold;     /* view-space gradient threshold (1.7e-4 in the paper) */
  float scene_radius;       /* r of Eq. (9), > 0 */
  float clone_scale;        /* g */
  float prune_scale;        /* b */
  float min_opacity;        /* also prune o < min_opacity; 0 disables */
  float split_scale_decay;  /* 0.8 in the paper */
  float split_beta_decay;   /* 1, or 0.8 in the later part of training */
} pvg_densify_config;

/* Workspace of a densify pass over n Gaussians (n <= 2^30). */
int pvg_densify_tmp_bytes(int64_t n, size_t* bytes);

/* Decide every Gaussian's outputs and count them: writes the plan into tmp
 * and the number of Gaussians after the pass into *n_out (host), then
 * returns; synchronizes `stream` to read the count.  noise: device [8][n]
 * standard normal draws (rows 4k .. 4k+2: child k's position offset in
 * units of s along the Gaussian's axes; row 4k+3: its dtau / beta), read
 * only for split Gaussians.  grad_accum / grad_count: device [n] statistics.
 * PVG_ERR_INVALID on null pointers, a non-finite threshold or r <= 0;
 * PVG_ERR_NOMEM when tmp_bytes is short. */
int pvg_densify_plan(const pvg_gaussians* g, const float* grad_accum, const float* grad_count, const float* noise,
                     const pvg_densify_config* cfg, void* tmp, size_t tmp_bytes, int64_t* n_out, void* stream);

/* Write the pass planned in tmp (same g, noise and cfg) into `out`, whose
 * arrays (device, caller-owned, written) hold out->n = *n_out Gaussians of
 * the same sh_degree.  Order: by parent index; within a parent the kept
 * original, its clone, then its split children.  extra_in [n_extra][n] ->
 * extra_out [n_extra][n_out] carry further per-Gaussian rows (optimizer
 * state): copied for a kept original, zero for every new Gaussian.
 * PVG_ERR_INVALID when out->n differs from the plan's count (checked before
 * any write; synchronizes `stream`). */
int pvg_densify_apply(const pvg_gaussians* g, const float* noise, const pvg_densify_config* cfg, const void* tmp,
                      size_t tmp_bytes, const pvg_gaussians* out, int32_t n_extra, const float* extra_in,
                      float* extra_out, void* stream);

/* Adam (Sec. 4: Adam with per-parameter learning rates) over every
 * parameter array of `params` (device, updated in place) with the gradients
 * `grad` of the activated values.  The step is taken in the unconstrained
 * space of each array: log s, logit o, log l, log beta, and the values
 * themselves for mu, q, SH, v and tau (the gradient chained there: s dL/ds,
 * o (1 - o) dL/do, ...).  m, v: device [17 + 3K][n] moments in the order mu
 * (3 rows), scale (3), rot (4), sh (3K), opacity, vel (3), period, tau, beta;
 * zero before the first step.  lr: mu, scale, rot, SH degree 0, SH higher
 * degrees, opacity, vel, period, tau, beta; a zero rate still updates the
 * moments.  step t >= 1 sets the bias corrections 1 - beta1^t, 1 - beta2^t. */
typedef struct pvg_adam_config {
  float lr[10];
  float beta1, beta2, eps;
  int32_t step;
} pvg_adam_config;
int pvg_adam_step(const pvg_gaussians* params, const pvg_gaussians_grad* grad, float* m, float* v,
                  const pvg_adam_config* cfg, void* stream);

/* Adam (Sec. 4) on a dense learnable array of `count` floats: the sky cube
 * map of Sec. 3.4 ([6][3][R][R], its texels taken as they are).  p (updated in
 * place), grad, and the moments m, v (zero before the first step) are device
 * arrays of `count` floats; the update is pvg_adam_step's on the identity
 * space with the single rate lr (a zero rate still updates the moments, a
 * zero step leaves p bit for bit).  step t >= 1 sets the bias corrections.
 * PVG_ERR_INVALID on null arrays, count < 0 or a bad rate or beta. */
int pvg_adam_dense(float* p, const float* grad, float* m, float* v, int64_t count, float lr, float beta1,
                   float beta2, float eps, int32_t step, void* stream);

/* Opacity reset (Sec. 4): o = min(o, cap) and the opacity row of the Adam
 * moments cleared. */
int pvg_opacity_reset(const pvg_gaussians* params, float* m, float* v, float cap, void* stream);

/* Static / dynamic split (Sec. 3.2: the staticness rho = beta / l with a
 * threshold separates static from dynamic points).  A Gaussian is static
 * when rho >= rho_threshold (FP32).  The plan (workspace of
 * pvg_densify_tmp_bytes(n)) writes the number of static Gaussians into
 * *n_static (host; synchronizes `stream`); the apply copies each Gaussian
 * into out_static (n = *n_static) or out_dynamic (n = g->n - *n_static),
 * both in index order, device arrays owned by the caller.  PVG_ERR_INVALID
 * when the outputs' sizes or degrees differ from the plan's (checked before
 * any write). */
int pvg_staticness_split_plan(const pvg_gaussians* g, float rho_threshold, void* tmp, size_t tmp_bytes,
                              int64_t* n_static, void* stream);
int pvg_staticness_split_apply(const pvg_gaussians* g, float rho_threshold, const void* tmp, size_t tmp_bytes,
                               const pvg_gaussians* out_static, const pvg_gaussians* out_dynamic, void* stream);

/* SSIM term of the training loss (Sec. 3.4 objective, weight lambda_r):
 * the structural similarity of Wang et al. per channel and pixel, with an 11
 * x 11 Gaussian window (sigma 1.5, normalised), zero padding outside the
 * image and C1 = 0.01^2, C2 = 0.03^2 (values in [0, 1]):
 *   S = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sxx + syy + C2)).
 * x (the render) and y (the target): device [channels][height][width].
 * ssim_map (optional, may be NULL): S, same layout.  partials: device
 * [3][channels][height][width] written for pvg_ssim_bwd (dS/dmx,
 * dS/d(G*x^2), dS/d(G*xy)).  PVG_ERR_INVALID on sizes outside 1..65535 or
 * null arrays. */
int pvg_ssim_fwd(const float* x, const float* y, int32_t channels, int32_t height, int32_t width, float* ssim_map,
                 float* partials, void* stream);

/* Adjoint of pvg_ssim_fwd with respect to x: dL_dx [C][H][W] (written) from
 * dL_dssim [C][H][W] and the forward's x, y and partials. */
int pvg_ssim_bwd(const float* dL_dssim, const float* x, const float* y, const float* partials, int32_t channels,
                 int32_t height, int32_t width, float* dL_dx, void* stream);

/* L1 term of the training loss (Sec. 3.4 objective; the photometric L1 of
 * Sec. 4): loss[0] = scale * sum_i |a_i - b_i| over n floats and, when
 * grad_a is not NULL, grad_a[i] = scale * sign(a_i - b_i) (0 where they are
 * equal, NaN where the difference is NaN), in one pass over a and b.
 * partials: device scratch of PVG_L1_PARTIALS floats, caller-owned.  The sum
 * is formed in a fixed order (per-workgroup partial sums, then their FP64
 * sum), so the loss is the same on every run.  All arrays are device memory;
 * PVG_ERR_INVALID on n < 0 or a null a, b, loss or partials; asynchronous on
 * `stream`. */
#define PVG_L1_PARTIALS 1024
int pvg_l1_loss(const float* a, const float* b, int64_t n, float scale, float* loss, float* grad_a, float* partials,
                void* stream);

/* Sky refinement (Sec. 3.4): out = img + (1 - opacity) * f_sky(d), with f_sky
 * a learnable cube map `cube` [6][3][cube_res][cube_res] (faces +X, -X, +Y,
 * -Y, +Z, -Z; channel; row v; column u) looked up bilinearly, inside the face,
 * in the world-frame direction d = R^T ((px + 1/2 + jx - cx) / fx, (py + 1/2
 * + jy - cy) / fy, 1) of pixel (px, py).  img [3][H][W] is the render with a
 * black background; opacity [H][W] is 1 - final_T; jitter (optional, may be
 * NULL) [2][H][W] moves each direction inside its pixel (the paper perturbs it
 * within the unit pixel while training).  The face is the axis of the largest
 * |d_i| (ties to the lower axis) with OpenGL face coordinates; texel (u R -
 * 1/2, v R - 1/2), clamped to [0, R - 1].  Device memory, caller-owned;
 * PVG_ERR_INVALID on a bad camera, null arrays or cube_res outside
 * [1, 16384]; asynchronous on `stream`. */
int pvg_sky_composite(const pvg_camera* cam, const float* img, const float* opacity, const float* cube,
                      int32_t cube_res, const float* jitter, float* out, void* stream);
/* Adjoint of pvg_sky_composite for dL_dout [3][H][W]: writes dL_dopacity
 * [H][W] (= -sum_c f_sky,c(d) dL_dout_c) and adds (1 - opacity) dL_dout times
 * the bilinear weights into dL_dcube [6][3][R][R] (zero it first for a fresh
 * gradient; calls on one device add into it in stream order).  dL/dimg is
 * dL_dout itself.  Each 16 x 16 pixel tile sums its texels in LDS in 64-bit
 * fixed point and adds them to dL_dcube with float atomics, so the order of
 * those additions, and the last bits of the result, vary from run to run.
 * Same arguments and errors as pvg_sky_composite. */
int pvg_sky_composite_bwd(const pvg_camera* cam, const float* dL_dout, const float* opacity, const float* cube,
                          int32_t cube_res, const float* jitter, float* dL_dopacity, float* dL_dcube,
                          void* stream);
/* pvg_sky_composite_bwd with a result that is the same on every run: each
 * 16 x 16 texel block of the cube map is summed by one workgroup over the
 * pixels that can reach it, in 64-bit fixed point, and written once, with no
 * device-memory atomics.  Slower (about 1.5 - 2.5x at 1920 x 1280 with
 * R = 1024).  Pixels whose jitter exceeds half a pixel, and cameras whose R
 * is not a rotation to 1e-3, fall back to float atomics and lose the
 * guarantee. */
int pvg_sky_composite_bwd_deterministic(const pvg_camera* cam, const float* dL_dout, const float* opacity,
                                        const float* cube, int32_t cube_res, const float* jitter,
                                        float* dL_dopacity, float* dL_dcube, void* stream);

/* Scratch bytes of pvg_render_bwd_views.  Host only. */
int pvg_bwd_views_tmp_bytes(int64_t n, int32_t n_views, int32_t max_width, int32_t max_height,
                            int64_t max_capacity, size_t* bytes);

/* ---- stage timing (HIP events recorded on the launch stream) ------------ */
enum pvg_stage {
  PVG_STAGE_PREPROCESS = 0, PVG_STAGE_COMPACT, PVG_STAGE_DEPTH_SORT, PVG_STAGE_SCAN_EMIT,
  PVG_STAGE_TILE_SORT, PVG_STAGE_RANGES, PVG_STAGE_RENDER_FWD, PVG_STAGE_RENDER_BWD,
  PVG_STAGE_PREPROCESS_BWD, PVG_STAGE_GRAD_GATHER, PVG_STAGE_COUNT
};
/* on = 1: every later launch is bracketed by a pair of hipEvents on its
 * stream.  on = 2: in addition the render stages count the (pixel, Gaussian)
 * pairs they evaluate (a slower variant of their kernels).  on = 0: off. */
int pvg_profile_enable(int32_t on);
/* Waits for the recorded events and adds their durations to the totals. */
int pvg_profile_collect(void);
/* Totals since the last reset: milliseconds, number of stage invocations and
 * work units (evaluated pairs for the render stages, 0 otherwise). */
int pvg_profile_read(int32_t stage, double* total_ms, int64_t* invocations, int64_t* work);
int pvg_profile_reset(void);
const char* pvg_stage_name(int32_t stage);

const char* pvg_status_str(int status);
/* Copies the calling thread's last error message (NUL-terminated); returns its length. */
int pvg_last_error(char* buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* PVG_H */
