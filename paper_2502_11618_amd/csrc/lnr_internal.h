// Internal declarations shared by the host runtime (api.cpp) and the HIP
// kernel files of liblnr.  Not part of the public ABI (see include/lnr.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "lnr.h"

namespace lnr {

// ----------------------------------------------------------------------------
// geometry of a partitioned cloud (device-resident)
// ----------------------------------------------------------------------------
struct CloudDev {
  uint32_t n = 0;
  uint32_t n_cells = 0;
  int32_t dims[3] = {0, 0, 0};
  float origin[3] = {0, 0, 0};
  float cell_size = 0;
  uint32_t max_chunks = 0;    // sum over cells of ceil(count / kSplatChunk)
  float *x = nullptr, *y = nullptr, *z = nullptr;  // sorted SoA coordinates
  uint32_t *rgbx = nullptr;   // sorted colours, bytes r, g, b, 0
  uint32_t *perm = nullptr;   // sorted position -> input index
  uint32_t *cell_start = nullptr;  // [n_cells + 1]
  float *aabb = nullptr;      // [n_cells][6] = lo xyz, hi xyz
};

constexpr uint32_t kSplatChunk = 4096;   // points per splat work item
constexpr int kSplatThreads = 256;

// frustum-cull parameters, formed on the host in double precision
struct CullParams {
  double hs[6][4];     // half-spaces h(X) = c0 x + c1 y + c2 z + c3 >= 0
  double absP[3][4];   // |P| for the rounding slack
  double wh1;          // W + H + 1
  double wrow[4];      // third row of P: camera depth w of a point
  double z_near;
  int no_cull;
};

// Splat work items are queued per depth bucket of their cell (kBucketsPerOctave
// buckets per octave of camera depth above z_near, the last one open-ended),
// nearest bucket first, so nearer surfaces tend to reach the z-buffer before
// the points they hide and those fail the early-out test instead of costing
// an atomic (finer buckets, 32 or 64, measured the same).  Queue b holds up to
// max_chunks items at chunks[b * max_chunks].
constexpr int kDepthBuckets = 16;
constexpr float kBucketsPerOctave = 2.f;

struct SplatCam {
  float P[12];
  float Wf, Hf, z_near, z_far;
  uint32_t W;
};

// A camera in device memory (serving: one per batch slot, rewritten before
// each replay of a captured frame graph).
struct DevCam {
  CullParams cull;
  SplatCam splat;
};

// Multi-view render: views per pass over the cloud.  The per-view cameras
// travel as kernel arguments (a pass's culling parameters take 2.8 KB).
constexpr int kViewsPerPass = 8;
constexpr int kMaxRenderViews = 1024;  // views per lnr_render_views call
struct ViewsCull {
  CullParams v[kViewsPerPass];
  int n;
};
struct ViewsSplat {
  SplatCam cam[kViewsPerPass];
  uint64_t *key[kViewsPerPass];
  int n;
};
static_assert(sizeof(ViewsCull) + 64 <= 4096, "kernel arguments stay within 4 KB");

// counters written by the render kernels: [0] chunks, [1] visible cells,
// [2..3] processed points (u64), [4 + b] chunks queued in depth bucket b,
// [kAtomicWord] z-buffer atomics issued (counting renders only)
constexpr int kAtomicWord = 4 + kDepthBuckets;
// tiled splat: segments written so far, and units of work of its tile kernel
constexpr int kSegTopWord = kAtomicWord + 1;
constexpr int kUnitsWord = kSegTopWord + 1;
constexpr int kCounterWords = kUnitsWord + 1;

// ----------------------------------------------------------------------------
// kernel launchers (each returns hipGetLastError() of its launches)
// ----------------------------------------------------------------------------
// grid.hip
hipError_t launch_bbox(const float *xyz, uint32_t n, float *partial /* [nb][7] */, uint32_t nb, hipStream_t s);
uint32_t bbox_blocks(uint32_t n);
hipError_t launch_cell_ids(const float *xyz, uint32_t n, const double lo[3], double s, const int32_t dims[3],
                           uint32_t *cell, hipStream_t st);
hipError_t launch_cell_bounds(const uint32_t *sorted_cell, uint32_t n, uint32_t n_cells, uint32_t *cell_start,
                              hipStream_t s);
hipError_t launch_iota(uint32_t *v, uint32_t n, hipStream_t s);
// stable LSD radix sort of (key, val) pairs by the low `bits` bits of key; uses two ping-pong buffers.
// On return the sorted data are in (*keys, *vals); tmp buffers are swapped in as needed.
size_t radix_sort_scratch_bytes(uint32_t n);
hipError_t radix_sort_pairs(uint32_t **keys, uint32_t **vals, uint32_t **keys_alt, uint32_t **vals_alt, uint32_t n,
                            int bits, void *scratch, hipStream_t s);
size_t scan_scratch_bytes(uint32_t n);
hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, uint32_t n, void *scratch, hipStream_t s);
hipError_t launch_gather_points(const float *xyz, const uint8_t *rgb, const uint32_t *perm, uint32_t n, float *x,
                                float *y, float *z, uint32_t *rgbx, hipStream_t s);
hipError_t launch_cell_aabb(const float *x, const float *y, const float *z, const uint32_t *cell_start,
                            uint32_t n_cells, float *aabb, hipStream_t s);
hipError_t launch_chunk_count(const uint32_t *cell_start, uint32_t n_cells, uint32_t *total, hipStream_t s);

// render.hip
// per-frame reset of the key buffer (npix words), the counters and the tiled
// splat's per-tile segment counts (n_tiles words)
hipError_t launch_clear(uint64_t *key, uint32_t npix, uint32_t *counters, uint32_t *tile_nseg, uint32_t n_tiles,
                        hipStream_t s);
// Screen-tiled splat (32 x 32 pixel tiles), in up to five launches (stage
// 0..4: bin, tilescan, segsort, tile, tileres; stage 1 launches nothing when
// tiled_scan_merged(), the segment sort then taking the scan).  Scratch per
// render for a cloud of n points: recs u64[n] (a work item's records at its
// points' positions), segs uint4[n] and sorted u32[n] (at most one segment
// per record), tile_nseg u32[2 n_tiles] (the counts, then the merged sort's
// fill counters), tile_units u32[n_tiles], tile_off u32[n_tiles + 1], units
// uint2[unit_cap].
struct TiledSplatGrid {
  uint32_t tiles_x = 0, tiles_y = 0, n_tiles = 0;
  uint64_t unit_cap = 0;
};
TiledSplatGrid tiled_splat_grid(uint32_t W, uint32_t H, uint32_t n_points);
// true when the per-tile scan runs inside the segment sort (stage 1 then
// launches nothing); tile_nseg then holds 2 n_tiles words: the counts, then
// the fill counters of the sort, both zeroed by launch_clear
bool tiled_scan_merged(const TiledSplatGrid &g);
struct TiledSplatBufs {
  uint64_t *recs;
  uint4 *segs;
  uint32_t *sorted;
  uint32_t *tile_nseg;
  uint32_t *tile_off;
  uint32_t *tile_units;
  uint2 *units;
};
// cam_dev / prm_dev (may be nullptr): the same camera in device memory, read by
// the kernels instead of the by-value copy (graph replays with new cameras)
hipError_t launch_tiled_splat(const CloudDev &c, const uint2 *chunks, uint32_t *counters, const SplatCam &cam,
                              const SplatCam *cam_dev, uint32_t H, const TiledSplatBufs &b, uint64_t *key,
                              float *depth, uint32_t *rgba, int stage, hipStream_t s);
hipError_t launch_cull(const CloudDev &c, const CullParams &prm, const CullParams *prm_dev, uint8_t *flags,
                       uint2 *chunks, uint32_t *counters, hipStream_t s);
// the atomic splat (global z-buffer); count_atomics: also add the number of
// z-buffer atomics issued to counters[kAtomicWord]
hipError_t launch_splat(const CloudDev &c, const uint2 *chunks, uint32_t *counters, const SplatCam &cam,
                        uint64_t *key, bool count_atomics, hipStream_t s);
// several views in one pass: work items (start, count, view mask, 0) queued
// as launch_cull queues its chunks, then one splat that reads each work
// item's points once for all the views of its mask
hipError_t launch_cull_views(const CloudDev &c, const ViewsCull &prm, uint8_t *flags, uint4 *items, uint32_t *counters,
                             hipStream_t s);
hipError_t launch_splat_views(const CloudDev &c, const uint4 *items, const uint32_t *counters, const ViewsSplat &vs,
                              hipStream_t s);
// throughput probe: grid x 256 threads x iters 64-bit atomicMin on buf[n_slots]
// (pattern 0: pseudo-random words; 1: one word per wave, consecutive waves
// consecutive words)
constexpr uint32_t kProbeIters = 64;
hipError_t launch_atomic_probe(uint64_t *buf, uint32_t n_slots, int pattern, uint32_t grid, uint32_t seed,
                               hipStream_t s);
hipError_t launch_resolve(const uint64_t *key, const uint32_t *rgbx, float *depth, uint32_t *rgba, uint32_t npix,
                          hipStream_t s);
// soft z-buffer: clear the colour sums, accumulate, resolve (acc = 4 x u32 per pixel)
hipError_t launch_soft(const CloudDev &c, const uint2 *chunks, const uint32_t *counters, const SplatCam &cam,
                       const SplatCam *cam_dev, const uint64_t *key, float one_plus_eps, uint32_t *acc, float *depth,
                       uint32_t *rgba, uint32_t npix, hipStream_t s);

// filter.hip
hipError_t launch_pyramid(const float *depth, const uint32_t *rgba, int H, int W, int n, float *const *levels,
                          hipStream_t s);
// allocation-free filter: floats in the per-device scratch array (16 MiB), and
// its device address on the current device
constexpr size_t kNoAllocScratchFloats = size_t(4) << 20;
hipError_t noalloc_scratch_address(float **ptr);
// every upsampling level in one launch (1 <= n <= 15); D[1..n] min-pooled levels,
// Hs/Ws[0..n] level sizes; removes the rejected pixels of depth/rgba in place
hipError_t launch_upsample_fused(int n, const float *const *D, const int *Hs, const int *Ws, float *depth,
                                 uint32_t *rgba, float fs, float one_plus_fs, hipStream_t s);

// unet.hip
// values equal the public lnr_precision ones
enum class Prec { F32 = 0, BF16 = 1, FP8 = 2, BF16X3 = 3, FP16 = 4, FP8X3 = 5 };
// 16-bit activations in HBM (the e4m3 modes keep float16 activations)
inline bool prec_half(Prec p) { return p == Prec::BF16 || p == Prec::FP16 || p == Prec::FP8 || p == Prec::FP8X3; }

struct ConvLayer {
  int cout = 0, cin = 0, k = 3;  // logical sizes
  int cout_pad = 0;              // multiple of 32 (MFMA block rows)
  int cin_pad = 0;               // multiple of 8 (fp32) / 16 (bf16)
  void *w = nullptr;             // packed weights [cout_pad][k*k][cin_pad] (f32 or bf16 hi)
  void *w_lo = nullptr;          // bf16 low parts (BF16X3)
  float *bias = nullptr;         // [cout_pad]
  void *wu = nullptr;            // float32 only: Winograd F(2x2,3x3) weights G g G^T [cout_pad][16][cin_pad]
  float *wscale = nullptr;       // e4m3 modes: weight scale per output channel [cout_pad]
};

struct ConvCall {
  const void *in0;   // NHWC, C0 channels, H x W
  const void *in1;   // NHWC, C1 channels, (H/2) x (W/2), read nearest-upsampled (decoder), or null
  int C0, C1;
  int H, W;
  const ConvLayer *layer;
  void *out;         // NHWC, layer->cout channels
  void *out_pool;    // NHWC, (H/2) x (W/2), 2x2 max of out, or null
  // optional fused 1x1 head (c_out <= 64): when head_out is set, the ReLU output
  // is not stored; head_out[o][y][x] = head_b[o] + sum_c head_w[o][c] * out[c]
  const float *head_w = nullptr;  // [3][cout]
  const float *head_b = nullptr;  // [3]
  float *head_out = nullptr;      // planar float [3][H][W]
  // batch of same-shape images (per-image element strides; head_outs: device
  // array of per-image head outputs, or null for head_out + image * 3*H*W)
  int batch = 1;
  size_t in0_bs = 0, in1_bs = 0, out_bs = 0, pool_bs = 0;
  float *const *head_outs = nullptr;
  // first layer of a single image only: stage the network input straight from
  // the RGBDA image (the same values the input pack writes) instead of in0
  const float *rgbda_depth = nullptr;
  const uint32_t *rgbda_rgba = nullptr;
};

hipError_t launch_pack_input(const float *depth, const uint32_t *rgba, int H, int W, int cpad, Prec p, void *x,
                             hipStream_t s);
// the first two convolutions in one launch (bf16 and fp16, first level of 16 or
// 32 channels, at least two levels): the same outputs as two launch_conv3x3
// calls, without the first one's output in HBM
bool enc0_fusable(const ConvLayer &l0, const ConvLayer &l1, Prec p);
hipError_t launch_enc0_fused(const ConvCall &c0, const ConvCall &c1, Prec p, hipStream_t s);
hipError_t launch_conv3x3(const ConvCall &c, Prec p, hipStream_t s);
hipError_t launch_head(const void *x, int C, int H, int W, const ConvLayer &head, Prec p, float *out, hipStream_t s);

}  // namespace lnr
