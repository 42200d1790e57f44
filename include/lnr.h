/*
 * lnr.h - C ABI of the MI355X (gfx950) per-frame rendering path of
 * "Real-time Neural Rendering of LiDAR Point Clouds" (arXiv 2502.11618).
 *
 * The path (Fig. 1 of the paper): a coloured point cloud, partitioned once
 * into a uniform grid, is frustum-culled per cell and projected as 1x1-pixel
 * points into an RGB + depth + fill-mask image (RGBDA); a hierarchical
 * min-pool depth filter removes background points that leak between
 * foreground points (Fig. 2); a fully convolutional U-Net reconstructs the
 * final RGB image.  Every stage runs in hand-written HIP kernels.
 *
 * Conventions for every entry point:
 *   - Every call returns lnr_status; on failure lnr_last_error() holds a
 *     message.  Nothing crosses the ABI as an exception, abort or exit.
 *   - Argument checks are synchronous: when a call fails them nothing is
 *     enqueued and caller buffers are untouched.
 *   - Device work is enqueued on the caller's HIP stream (`hip_stream`, a
 *     hipStream_t passed as void*; NULL = the default stream) and returns
 *     before it completes.  Kernel faults surface as LNR_E_DEVICE from a later
 *     call or from lnr_sync().
 *   - Pointers documented as DEVICE point to device memory the caller owns
 *     and keeps alive until its stream work completes; HOST pointers are read
 *     or written before the call returns.  The library never frees caller
 *     memory.
 *   - A context owns device scratch that every call on it reuses; a context is
 *     externally synchronised and its calls must not overlap on different
 *     streams (use one context per concurrent stream).  Clouds and networks
 *     are read-only after loading and may be shared by contexts of the same
 *     device.
 */
#ifndef LNR_H
#define LNR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LNR_OK = 0,
  LNR_E_INVALID_ARG = -1,   /* a pointer, size or value is out of range        */
  LNR_E_OUT_OF_MEMORY = -2, /* hipMalloc failed                                  */
  LNR_E_BUDGET = -3,        /* the allocation would exceed the context's budget  */
  LNR_E_DEVICE = -4,        /* a HIP runtime call or kernel failed               */
  LNR_E_UNSUPPORTED = -5,   /* a valid request this build does not handle        */
  LNR_E_FORMAT = -6         /* a malformed weight blob                           */
} lnr_status;

typedef struct lnr_context lnr_context; /* device scratch, budget, last error       */
typedef struct lnr_cloud lnr_cloud;     /* partitioned cloud, device-resident         */
typedef struct lnr_unet lnr_unet;       /* U-Net weights repacked for one precision   */

/* Pinhole camera.  P is the row-major 3x4 projection: for a world point X,
 * (a, b, w) = P [X; 1]; w is the camera-space depth and (u, v) = (a/w, b/w)
 * the image position, pixel (px, py) covering [px, px+1) x [py, py+1).
 * A point is drawn iff z_near <= w <= z_far, 0 <= u < width, 0 <= v < height.
 * Requires 1 <= width, height <= 16384, finite P, 0 < z_near < z_far. */
typedef struct {
  float P[12];
  int32_t width, height;
  float z_near, z_far;
} lnr_camera;

/* An RGBDA image: caller-owned DEVICE buffers, row-major, tightly packed.
 *   key   : uint64[width*height]  z-buffer key (depth bits << 32 | point index);
 *           0xFFFFFFFFFFFFFFFF = empty.  May be NULL for lnr_depth_filter and
 *           lnr_reconstruct.
 *   depth : float[width*height]   camera-space depth, 0 where empty.
 *   rgba  : uint8[4*width*height] colour + fill mask A in {0, 1}; (0,0,0,0) where empty. */
typedef struct {
  uint64_t *key;
  float *depth;
  uint8_t *rgba;
  int32_t width, height;
} lnr_image;

/* U-Net arithmetic (the paper fixes none; Method, "U-Net Reconstruction").
 *   LNR_FP32     : float32 activations, float32 matrix-core products.
 *   LNR_BF16     : bfloat16 activations and weights, float32 accumulation.
 *   LNR_FP8_E4M3 : OCP e4m3 matrix-core operands, float32 accumulation:
 *                  float16 activations rounded to e4m3 (to nearest even,
 *                  saturating at 448) as they are multiplied, e4m3 weights
 *                  with one scale per output channel (its largest weight maps
 *                  to 448).
 *   LNR_FP8_E4M3X3 : as LNR_FP8_E4M3 with each operand split into e4m3 high
 *                  + low parts (low = e4m3 of the remainder), multiplied as
 *                  lo*hi + hi*lo + hi*hi.
 *   LNR_BF16X3   : float32 activations; each operand split into bfloat16
 *                  high + low parts and multiplied as hi*hi + hi*lo + lo*hi
 *                  with float32 accumulation (near-float32 accuracy on
 *                  bfloat16 matrix cores).
 *   LNR_FP16     : IEEE binary16 activations and weights, float32
 *                  accumulation: the data movement and matrix rate of
 *                  LNR_BF16 with a 10- instead of a 7-bit fraction.
 * Every precision computes the same network; only the rounding differs. */
typedef enum {
  LNR_FP32 = 0,
  LNR_BF16 = 1,
  LNR_FP8_E4M3 = 2,
  LNR_BF16X3 = 3,
  LNR_FP16 = 4,
  LNR_FP8_E4M3X3 = 5
} lnr_precision;

/* lnr_render flags.  The image is the same under every combination.
 *   LNR_RENDER_NO_CULL       visit every non-empty cell (no frustum test), to
 *                            check that culling is a pure speed-up.
 *   LNR_RENDER_ATOMIC_SPLAT  keep the z-buffer in device memory and lower it
 *                            with 64-bit atomicMin (after a per-work-item
 *                            on-chip z-buffer keeps the nearest point of each
 *                            pixel), instead of the default screen-tiled
 *                            splat (points binned per 32 x 32 tile, each
 *                            tile's z-buffer on chip, no atomic per point or
 *                            pixel in device memory); for comparison.
 *   LNR_RENDER_COUNT_ATOMICS the atomic splat, also counting the z-buffer
 *                            atomics it issues (lnr_render_atomic_count). */
#define LNR_RENDER_NO_CULL 1u
#define LNR_RENDER_COUNT_ATOMICS 2u
#define LNR_RENDER_ATOMIC_SPLAT 4u

/* Create a context on HIP device `hip_device`.  `hbm_budget_bytes` caps the
 * device memory the context, and the clouds and networks loaded through it,
 * may allocate (0 = no cap). */
lnr_status lnr_context_create(int hip_device, uint64_t hbm_budget_bytes, lnr_context **out);
/* Release a context.  NULL-safe.  Clouds, networks and servers created
 * through it stay valid: the context and its scratch are freed when it has
 * been destroyed and the last of them has been destroyed, so objects may be
 * destroyed in any order (garbage-collected bindings need this).  Passing the
 * context to any other call after this one is an error of the caller's. */
void lnr_context_destroy(lnr_context *ctx);
/* Message of the last failure on ctx (valid until the next call on ctx);
 * with ctx == NULL, the last failure of lnr_context_create. */
const char *lnr_last_error(const lnr_context *ctx);
/* Device bytes currently allocated through ctx (scratch, clouds, networks). */
uint64_t lnr_allocated_bytes(const lnr_context *ctx);

/* Load and partition a cloud (Method, "Point Cloud Projection": a uniform
 * grid is the only preprocessing and enables view-frustum culling).
 *   xyz_host : HOST float[n*3], interleaved x, y, z; must be finite.
 *   rgb_host : HOST uint8[n*3].
 *   1 <= n < 2^32; cell_size finite and > 0; at most 2^31 cells.
 * The grid origin is the componentwise minimum of the points; per axis
 * n_a = max(1, ceil((max_a - min_a) / cell_size)) cells, and a point's cell
 * index is min(n_a - 1, floor((x_a - min_a) / cell_size)) evaluated in double.
 * Points are stably sorted by cell id (z-major, then y, then x); a point's
 * position in that order is its index in z-buffer keys.  Synchronous: the
 * call returns after the device copy is built. */
lnr_status lnr_cloud_load(lnr_context *ctx, const float *xyz_host, const uint8_t *rgb_host, uint64_t n,
                          float cell_size, lnr_cloud **out);
/* Grid geometry of a loaded cloud (any output pointer may be NULL). */
lnr_status lnr_cloud_info(const lnr_cloud *c, uint64_t *n, int32_t dims[3], float origin[3], float *cell_size);
/* HOST uint32[n]: sorted position -> input index. */
lnr_status lnr_cloud_permutation(const lnr_cloud *c, uint32_t *perm_host);
/* HOST uint32[n_cells + 1]: exclusive prefix of the per-cell point counts. */
lnr_status lnr_cloud_cell_start(const lnr_cloud *c, uint32_t *cell_start_host);
void lnr_cloud_destroy(lnr_cloud *c);

/* Render one view into `out` (Fig. 1, projection stage): cull grid cells
 * against the frustum, project each point of the surviving cells to one pixel
 * and keep, per pixel, the point with the smallest key
 * (float32 depth bits << 32 | sorted index): the nearest point, ties to the
 * lowest index.  Then write depth and rgba = (r, g, b, 1) of the winner, or
 * 0 / (0,0,0,0) for empty pixels.  Per point, in float32 without fused
 * multiply-add: a = ((P0 x + P1 y) + P2 z) + P3, b and w likewise,
 * u = a / w, v = b / w (correctly rounded).  A cell is skipped only if no
 * point in it can pass the per-point test (float64 bound with slack), so
 * culling never changes the image.  out->key, depth and rgba must all be
 * non-NULL with out->width/height equal to the camera's.  flags: 0 or any of
 * LNR_RENDER_NO_CULL, LNR_RENDER_ATOMIC_SPLAT, LNR_RENDER_COUNT_ATOMICS (see
 * above; the image is the same).  The tiled splat takes 28 bytes of context
 * scratch per point of the cloud. */
lnr_status lnr_render(lnr_context *ctx, const lnr_cloud *c, const lnr_camera *cam, lnr_image *out, uint32_t flags,
                      void *hip_stream);
/* Render with the soft z-buffer of Method, "Point Cloud Projection" (colours of
 * points that arrive at similar depths are averaged, given a small depth
 * threshold).  As lnr_render, except that a filled pixel's rgb is, per
 * channel, the integer sum over every point landing on it whose float32 depth
 * w satisfies w <= zmin * (1 + soft_eps) (zmin = depth of its nearest point,
 * which still gives key and depth), divided by their count and rounded half
 * up.  soft_eps >= 0 and finite.  Uses 16 bytes of context scratch per pixel;
 * a pixel may collect at most 2^24 points. */
lnr_status lnr_render_soft(lnr_context *ctx, const lnr_cloud *c, const lnr_camera *cam, lnr_image *out,
                           float soft_eps, uint32_t flags, void *hip_stream);
/* Render several views of one cloud (a batch of cameras, e.g. the views of
 * one serving step), reading each point from device memory once per pass
 * instead of once per view (Method, "Point Cloud Projection", applied to
 * every camera of the batch).  outs[v] receives exactly what lnr_render of
 * cams[v] alone writes, bit for bit, for every v.
 *   cams, outs : HOST arrays of n_views cameras and images (the images'
 *                buffers are device buffers, as for lnr_render); no two
 *                of the views' buffers (key, depth and rgba of every view)
 *                may overlap (LNR_E_INVALID_ARG).
 *   n_views    : 1..1024.  The views go in passes of up to 8: a pass culls
 *                every grid cell against each of its views' frustums, and
 *                the points of a cell visible in any of them are loaded once
 *                and drawn into each view whose frustum the cell meets.
 *   flags      : 0 or LNR_RENDER_NO_CULL.  The z-buffers are the images' key
 *                buffers, lowered with 64-bit atomicMin after an on-chip
 *                z-buffer per work item (LNR_RENDER_ATOMIC_SPLAT's method):
 *                the screen-tiled splat would need its per-point scratch
 *                once per view.
 * Uses 16 bytes of context scratch per work item and depth bucket.
 * lnr_render_stats then reports the last pass: cells visible in at least one
 * of its views, and the points of those cells, each read once.  Errors as
 * lnr_render, checked for every view before anything is enqueued. */
lnr_status lnr_render_views(lnr_context *ctx, const lnr_cloud *c, const lnr_camera *cams, lnr_image *outs,
                            int32_t n_views, uint32_t flags, void *hip_stream);
/* Statistics of the last lnr_render on ctx; waits for ctx's last stream.
 * visible_cells: cells that passed the frustum test; processed_points:
 * points in those cells.  cull_flags_host (may be NULL): HOST uint8[n_cells]
 * of the cloud last rendered, 1 = visible. */
lnr_status lnr_render_stats(lnr_context *ctx, uint64_t *visible_cells, uint64_t *processed_points,
                            uint8_t *cull_flags_host);
/* Number of z-buffer atomicMin operations issued by the last render on ctx,
 * which must have been issued with LNR_RENDER_COUNT_ATOMICS (else
 * LNR_E_INVALID_ARG); waits for ctx's last stream.  One is issued when a key
 * (a point's, or with the on-chip z-buffer the nearest of a work item's
 * points on that pixel) is below the pixel's key as last read (Method, "Point
 * Cloud Projection": the z-buffer keeps the nearest point). */
lnr_status lnr_render_atomic_count(lnr_context *ctx, uint64_t *atomics);
/* Roofline denominator of the projection step: the device's throughput of
 * 64-bit atomicMin, the z-buffer's operation.  Allocates n_slots u64 words
 * (charged to the context's budget; freed before returning), sets them to
 * all ones, runs one untimed pass and one timed pass of n_ops operations
 * (rounded up to a multiple of 16384; *ops_done, if not NULL, receives the
 * count) on hip_stream, and waits for it.  pattern 0: every operation hits a
 * pseudo-random word (many points spread over an image); pattern 1: the 64
 * lanes of a wave hit one word (contention).  *ops_per_s = operations / time
 * between HIP events around the timed pass.  Errors: LNR_E_INVALID_ARG for
 * n_slots outside [1, 2^32), pattern not 0 or 1, n_ops outside
 * [1, 16384 (2^31 - 1)] or NULL ops_per_s; allocation and device errors as
 * elsewhere. */
lnr_status lnr_measure_atomic_min(lnr_context *ctx, uint64_t n_slots, int32_t pattern, uint64_t n_ops,
                                  void *hip_stream, double *ops_per_s, uint64_t *ops_done);

/* Depth filter, in place (Method, "Depth filtering" and Fig. 2): min-pool the
 * depth n_levels times (2x2, stride 2, empty = +inf), then upsample level by
 * level: a 4-neighbour Laplacian on the coarser min-pooled level marks edges;
 * each child is kept iff its depth <= ref * (1 + filter_strength), where ref
 * is the parent's upsampled depth, or at edges the maximum over the parent's
 * 3x3 neighbourhood; rejected pixels of non-final levels are refilled by
 * bilinear interpolation of the coarser level.  Removed pixels become depth
 * 0, rgba (0,0,0,0); kept pixels are unchanged; `key` is not read or written.
 * 0 <= n_levels <= floor(log2(min(width, height))); filter_strength >= 0 and
 * not NaN (+inf keeps everything). */
lnr_status lnr_depth_filter(lnr_context *ctx, lnr_image *inout, int32_t n_levels, float filter_strength,
                            void *hip_stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * filter, arguments, checks and result as lnr_depth_filter, without any device
 * allocation.  The min-pooled levels 1..n (each padded to 256 bytes) go to a
 * fixed 16 MiB array in device memory that the library holds, one per device,
 * until the process ends; every image up to 3840 x 2160 fits at every
 * n_levels, and a larger image whose levels do not fit is refused with
 * LNR_E_INVALID_ARG before anything is enqueued.  Calls on one device share
 * that array: calls that overlap on the device (different streams or contexts
 * of one device) race and give undefined results; calls ordered on one stream
 * are safe.  Nothing in the array has to start at any value (each call writes
 * every level before reading it).  Not timed by lnr_profile_enable.
 * LNR_E_DEVICE if the array's address could not be found when ctx was
 * created. */
lnr_status lnr_depth_filter_noalloc(lnr_context *ctx, lnr_image *inout, int32_t n_levels, float filter_strength,
                                    void *hip_stream);

/* Load U-Net weights (Fig. 1; Method, "U-Net Reconstruction") from a HOST
 * blob (layout: magic "LNRU", u32 version 1|2, u32 levels L, in_channels (5),
 * out_channels (3), widths[L], then 4L-1 conv records enc0a, enc0b, ...,
 * dec0b, head, each u32 c_out, c_in, k, [u32 has_bn if version 2], f32 OIHW
 * weights, f32 bias, [f32 gamma, beta, mean, var per channel and f32 eps if
 * has_bn]).  Batch norm is folded into its convolution.  Supported: 1 <= L
 * <= 6, widths multiples of 16 up to 512, 3x3 convs and a 1x1 head.
 * Synchronous. */
lnr_status lnr_unet_load(lnr_context *ctx, const void *blob_host, uint64_t bytes, lnr_precision prec,
                         lnr_unet **out);
void lnr_unet_destroy(lnr_unet *u);
/* Forward pass on an RGBDA image.  Input x = (r/255, g/255, b/255,
 * A ? D/16 : 0, A); per level two 3x3 conv + bias + ReLU, 2x2 max-pool
 * between encoder levels, nearest x2 upsample and concatenation
 * [skip, upsampled] in the decoder, 1x1 head without activation.
 * rgb_out: DEVICE float[3*H*W], planar.  Requires H and W divisible by
 * 2^(L-1). */
lnr_status lnr_reconstruct(lnr_context *ctx, const lnr_unet *u, const lnr_image *in, float *rgb_out,
                           void *hip_stream);

/* Wait for `hip_stream` and report any pending device error. */
lnr_status lnr_sync(lnr_context *ctx, void *hip_stream);

/* Kernel timing.  While enabled, every kernel a call on ctx enqueues is
 * bracketed by HIP events on the same stream, and lnr_profile_read returns
 * (and forgets) the launches recorded since the last read, oldest first:
 * name (static string, e.g. "splat", "conv/dec0a"), duration in ms.  It waits
 * for the recorded work.  At most `max` records are copied; *count receives
 * the number recorded (records past `max` are dropped).  Disabled by default;
 * enabling adds two event records per launch. */
typedef struct {
  const char *name;
  float ms;
} lnr_kernel_time;
lnr_status lnr_profile_enable(lnr_context *ctx, int enable);
/* Failure injection for tests of the error paths: after `after` further
 * device allocations through ctx succeed, the next one fails exactly as a
 * failed hipMalloc does (LNR_E_OUT_OF_MEMORY; no device memory is taken), and
 * injection then switches itself off.  after < 0 switches it off.  Every
 * entry point must then return that status, free what it allocated and leave
 * caller buffers untouched. */
lnr_status lnr_debug_fail_allocation(lnr_context *ctx, int64_t after);
lnr_status lnr_profile_read(lnr_context *ctx, lnr_kernel_time *out, int32_t max, int32_t *count);

/* ---------------------------------------------------------------------------
 * Serving: many viewer sessions rendering the same resident cloud.
 *
 * Sessions are opened with their resolution; a session's two output planes
 * are allocated from the context's budget when it opens, so a session that
 * does not fit is refused with LNR_E_BUDGET (admission by HBM budget).
 * Each submitted camera becomes a request.  lnr_server_step takes a free lane
 * (a HIP stream with its own scratch and an RGBDA image per batch slot) and
 * the oldest pending request, joins it with up to max_batch - 1 other pending
 * requests of the same resolution, and enqueues for them: render (or soft
 * render), depth filter and input pack per request, and one batched U-Net
 * over all of them (each convolution processes the whole batch in one
 * launch).  With use_graphs, the whole launch sequence of every (resolution,
 * batch size) is captured once as a HIP graph and replayed: the kernels read
 * the batch's cameras and output pointers from device arrays that each step
 * writes before the replay.  Lanes run concurrently, so batches
 * overlap on the device.  A session has at most one request in flight; a
 * newer camera submitted while the older one is still pending replaces it
 * (the older is reported as superseded).  Every image is computed exactly as
 * lnr_render + lnr_depth_filter + lnr_reconstruct would compute it alone.
 * The server and its sessions are externally synchronised (one host thread).
 * ------------------------------------------------------------------------- */
typedef struct lnr_server lnr_server;
typedef struct {
  int32_t max_batch;        /* 1..16 requests of one resolution per batch          */
  int32_t lanes;            /* 1..8 concurrent HIP streams                          */
  int32_t n_levels;         /* depth filter levels (0 = unfiltered input)           */
  float filter_strength;    /* depth filter strength                                */
  int32_t soft;             /* non-zero: soft z-buffer with soft_eps                */
  float soft_eps;
  int32_t use_graphs;       /* non-zero: replay a captured HIP graph per batch      */
  int32_t max_width, max_height; /* largest session resolution (sizes lane scratch) */
} lnr_server_config;
typedef struct {
  int32_t session;
  uint64_t tag;             /* the caller's tag of the request                      */
  int32_t superseded;       /* 1: replaced by a newer camera before it ran          */
  int32_t batch;            /* requests in the batch that computed it               */
  float batch_gpu_ms;       /* device time of that whole batch                      */
  const float *rgb;         /* DEVICE float[3*H*W]; the session's two output planes */
                            /* alternate, so this stays valid until lnr_server_step */
                            /* launches the session's request after next            */
  int32_t width, height;
} lnr_server_result;
/* The U-Net must have widths[0] <= 64 (its head is fused into the last
 * convolution, which lets one launch write every session's output).
 * lnr_server_open_session refuses (LNR_E_INVALID_ARG) a size whose
 * floor(log2(min(width, height))) is below cfg->n_levels. */
lnr_status lnr_server_create(lnr_context *ctx, const lnr_cloud *c, const lnr_unet *u, const lnr_server_config *cfg,
                             lnr_server **out);
void lnr_server_destroy(lnr_server *srv); /* waits for its lanes; NULL-safe */
lnr_status lnr_server_open_session(lnr_server *srv, int32_t width, int32_t height, int32_t *session);
lnr_status lnr_server_close_session(lnr_server *srv, int32_t session); /* waits for its request */
lnr_status lnr_server_submit(lnr_server *srv, int32_t session, const lnr_camera *cam, uint64_t tag);
/* Enqueue at most one batch on a free lane; *launched = requests enqueued (0 if
 * no lane is free or nothing is pending).  Never waits for the device. */
lnr_status lnr_server_step(lnr_server *srv, int32_t *launched);
/* Finished and superseded requests since the last poll (non-blocking). */
lnr_status lnr_server_poll(lnr_server *srv, lnr_server_result *out, int32_t max, int32_t *count);
/* Requests pending (not yet launched) and in flight. */
lnr_status lnr_server_pending(const lnr_server *srv, int32_t *pending, int32_t *in_flight);

#ifdef __cplusplus
}
#endif

#endif /* LNR_H */
