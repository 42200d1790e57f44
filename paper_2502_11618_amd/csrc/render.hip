// Per-frame projection: grid-cell frustum culling, 1x1-pixel splat into a
// 64-bit z-buffer, and RGBDA resolve.
//
// Method, "Point Cloud Projection" and Fig. 1: the space-partitioned cloud is
// culled against the view frustum per grid cell; every surviving point is
// rasterised to a single pixel; a z-buffer resolves collisions; the result is
// RGB, depth D and a binary fill mask A.
//
// Exactness: the per-point arithmetic is float32 in a fixed order with no
// fused multiply-add (the library is built with -ffp-contract=off) and a
// correctly rounded division; the z-buffer keeps min(depth bits << 32 | index),
// which is order independent, so the image does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lnr_internal.h"

#pragma clang fp contract(off)

namespace lnr {
namespace {

constexpr int kThreads = 256;

// Per-frame reset: the key buffer (npix words), the render counters and the
// tiled splat's per-tile segment counts (n_tiles words, may be 0).
__global__ __launch_bounds__(kThreads) void clear_kernel(uint64_t *__restrict__ key, uint32_t npix,
                                                         uint32_t *__restrict__ counters,
                                                         uint32_t *__restrict__ tile_nseg, uint32_t n_tiles) {
  const uint32_t stride = gridDim.x * kThreads;
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < npix; i += stride) key[i] = ~0ull;
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < n_tiles; i += stride) tile_nseg[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x < kCounterWords) counters[threadIdx.x] = 0;
}

// Conservative visibility of a cell's box [lo, hi] for one camera: the box is
// visible unless some half-space's maximum over it is below -slack (all in
// double, in the order below).  If visible, *bucket is the depth bucket of the
// box centre.
__device__ __attribute__((always_inline)) inline bool cell_visible(const CullParams &prm, double lo0, double lo1, double lo2, double hi0,
                                    double hi1, double hi2, int *bucket) {
  bool vis = true;
  if (!prm.no_cull) {
    const double mx0 = fmax(fabs(lo0), fabs(hi0));
    const double mx1 = fmax(fabs(lo1), fabs(hi1));
    const double mx2 = fmax(fabs(lo2), fabs(hi2));
    double S[3];
    for (int r = 0; r < 3; ++r)
      S[r] = ((prm.absP[r][0] * mx0 + prm.absP[r][1] * mx1) + prm.absP[r][2] * mx2) + prm.absP[r][3];
    const double slack = 0x1p-20 * ((S[0] + S[1]) + prm.wh1 * S[2]);
    for (int h = 0; h < 6; ++h) {
      const double *k = prm.hs[h];
      const double m =
          ((fmax(k[0] * lo0, k[0] * hi0) + fmax(k[1] * lo1, k[1] * hi1)) + fmax(k[2] * lo2, k[2] * hi2)) + k[3];
      if (m < -slack) vis = false;
    }
  }
  if (vis) {
    // camera depth of the box centre -> bucket
    const double cw = ((prm.wrow[0] * (0.5 * (lo0 + hi0)) + prm.wrow[1] * (0.5 * (lo1 + hi1))) +
                       prm.wrow[2] * (0.5 * (lo2 + hi2))) + prm.wrow[3];
    const float q = cw > prm.z_near ? kBucketsPerOctave * __log2f((float)(cw / prm.z_near)) : 0.f;
    *bucket = q >= (float)(kDepthBuckets - 1) ? kDepthBuckets - 1 : (int)q;
  }
  return vis;
}

// Queue places for this lane's nch work items in queue `bucket`: the first
// one's place within that queue.  Compaction without LDS atomics: per depth
// bucket present in the wave, a wave-wide exclusive prefix of the lanes'
// work-item counts (a ballot and a count of the set lanes below when every
// cell has at most one work item, else a shuffle scan) places each cell
// within the wave's run; the
// runs of the block's waves follow each other in wave order through LDS, and
// one global atomic per bucket and block reserves the block's run.  Every
// thread of the block calls it (block barriers).
__device__ __attribute__((always_inline)) inline uint32_t reserve_places(uint32_t nch, int bucket, uint32_t *__restrict__ counters) {
  constexpr int kWaves = kThreads / 64;
  __shared__ uint32_t s_wave[kWaves][kDepthBuckets], s_base[kDepthBuckets];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t present = nch ? (1u << bucket) : 0u;  // buckets of this wave's visible cells
  for (int off = 32; off > 0; off >>= 1) present |= __shfl_xor(present, off, 64);
  // lanes whose cell has more than one work item: with none in the wave (the
  // common case), a bucket's prefix is a ballot and a count of the lanes below
  const bool multi = __ballot(nch > 1) != 0;
  const uint64_t below = (1ull << lane) - 1ull;
  uint32_t local = 0;
  if (lane < kDepthBuckets) s_wave[wave][lane] = 0u;  // buckets absent from the wave
  // one pass per bucket present in the wave (the set is the same for every
  // lane; the loop stays rolled, which keeps this short-lived kernel small)
#pragma unroll 1
  for (uint32_t m = __builtin_amdgcn_readfirstlane(present); m; m &= m - 1) {
    const int b = __builtin_ctz(m);
    const uint32_t v = bucket == b ? nch : 0u;
    uint32_t tot;
    if (!multi) {
      const uint64_t bal = __ballot(v != 0);
      if (v) local = (uint32_t)__popcll(bal & below);
      tot = (uint32_t)__popcll(bal);
    } else {
      uint32_t incl = v;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
      }
      if (v) local = incl - v;
      tot = __shfl(incl, 63, 64);
    }
    if (lane == 0) s_wave[wave][b] = tot;
  }
  __syncthreads();
  if (threadIdx.x < kDepthBuckets) {
    uint32_t sum = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) sum += s_wave[w][threadIdx.x];
    s_base[threadIdx.x] = sum ? atomicAdd(&counters[4 + threadIdx.x], sum) : 0u;
  }
  __syncthreads();
  uint32_t pos = 0;
  if (nch) {
    pos = s_base[bucket] + local;
    for (int w = 0; w < wave; ++w) pos += s_wave[w][bucket];
  }
  return pos;
}

// Frame totals: work items, visible cells and their points, reduced per wave
// with one atomic per wave.
__device__ __attribute__((always_inline)) inline void add_totals(bool vis, uint32_t nch, uint32_t cnt, uint32_t *__restrict__ counters) {
  uint32_t wave_chunks = nch;
  for (int off = 32; off > 0; off >>= 1) wave_chunks += __shfl_xor(wave_chunks, off, 64);
  const uint64_t vis_mask = __ballot(vis);
  uint32_t pts = vis ? cnt : 0u;
  for (int off = 32; off > 0; off >>= 1) pts += __shfl_xor(pts, off, 64);
  if ((threadIdx.x & 63) == 0 && wave_chunks) {
    atomicAdd(&counters[0], wave_chunks);
    atomicAdd(&counters[1], (uint32_t)__popcll(vis_mask));
    atomicAdd(reinterpret_cast<unsigned long long *>(&counters[2]), (unsigned long long)pts);
  }
}

// One lane per cell.  A visible non-empty cell is cut into splat work items
// of at most kSplatChunk points, queued in the depth bucket of the cell's
// centre.  DEV: the camera's parameters are read from device memory (prm_dev)
// instead of the kernel arguments, so that a captured graph can be replayed
// for new cameras.
template <bool DEV>
__global__ __launch_bounds__(kThreads) void cull_kernel(const float *__restrict__ aabb,
                                                        const uint32_t *__restrict__ cell_start, uint32_t n_cells,
                                                        CullParams prm_val, const CullParams *__restrict__ prm_dev,
                                                        uint8_t *__restrict__ flags, uint2 *__restrict__ chunks,
                                                        uint32_t cap, uint32_t *__restrict__ counters) {
  const CullParams &prm = DEV ? *prm_dev : prm_val;
  const uint32_t c = blockIdx.x * kThreads + threadIdx.x;
  uint32_t start = 0, cnt = 0;
  bool vis = false;
  int bucket = 0;
  if (c < n_cells) {
    start = cell_start[c];
    cnt = cell_start[c + 1] - start;
    if (cnt > 0)
      vis = cell_visible(prm, aabb[6ull * c + 0], aabb[6ull * c + 1], aabb[6ull * c + 2], aabb[6ull * c + 3],
                         aabb[6ull * c + 4], aabb[6ull * c + 5], &bucket);
    flags[c] = vis ? 1 : 0;
  }
  const uint32_t nch = vis ? (cnt + kSplatChunk - 1) / kSplatChunk : 0u;
  const uint32_t pos = reserve_places(nch, bucket, counters);
  for (uint32_t k = 0; k < nch; ++k) {
    const uint32_t off = k * kSplatChunk;
    chunks[(size_t)bucket * cap + pos + k] = make_uint2(start + off, min(kSplatChunk, cnt - off));
  }
  add_totals(vis, nch, cnt, counters);
}

// Several views at once: a cell is tested against every view's frustum, and
// its work items carry the mask of the views that see it (bit v = view v) and
// go to the queue of the nearest of those views' depth buckets.
__global__ __launch_bounds__(kThreads) void cull_views_kernel(const float *__restrict__ aabb,
                                                              const uint32_t *__restrict__ cell_start,
                                                              uint32_t n_cells, ViewsCull prm,
                                                              uint8_t *__restrict__ flags, uint4 *__restrict__ items,
                                                              uint32_t cap, uint32_t *__restrict__ counters) {
  const uint32_t c = blockIdx.x * kThreads + threadIdx.x;
  uint32_t start = 0, cnt = 0, mask = 0;
  int bucket = kDepthBuckets - 1;
  if (c < n_cells) {
    start = cell_start[c];
    cnt = cell_start[c + 1] - start;
    if (cnt > 0) {
      const double lo0 = aabb[6ull * c + 0], lo1 = aabb[6ull * c + 1], lo2 = aabb[6ull * c + 2];
      const double hi0 = aabb[6ull * c + 3], hi1 = aabb[6ull * c + 4], hi2 = aabb[6ull * c + 5];
      for (int v = 0; v < prm.n; ++v) {
        int b = 0;
        if (cell_visible(prm.v[v], lo0, lo1, lo2, hi0, hi1, hi2, &b)) {
          mask |= 1u << v;
          bucket = min(bucket, b);
        }
      }
    }
    flags[c] = mask ? 1 : 0;
  }
  const bool vis = mask != 0;
  const uint32_t nch = vis ? (cnt + kSplatChunk - 1) / kSplatChunk : 0u;
  const uint32_t pos = reserve_places(nch, bucket, counters);
  for (uint32_t k = 0; k < nch; ++k) {
    const uint32_t off = k * kSplatChunk;
    items[(size_t)bucket * cap + pos + k] = make_uint4(start + off, min(kSplatChunk, cnt - off), mask, 0u);
  }
  add_totals(vis, nch, cnt, counters);
}

// Work item `i` of the frame, walking the depth-bucket queues nearest first
// (counters[4 + b] items in bucket b); false past the last item.
template <typename Item>
__device__ inline bool work_item(uint32_t i, const uint32_t *__restrict__ counters, const Item *__restrict__ chunks,
                                 uint32_t cap, Item *ch) {
  if (i >= counters[0]) return false;
  for (int b = 0; b < kDepthBuckets; ++b) {
    const uint32_t nb = counters[4 + b];
    if (i < nb) {
      *ch = chunks[(size_t)b * cap + i];
      return true;
    }
    i -= nb;
  }
  return false;
}

// One block per work item.  Keys only ever decrease, so a (possibly stale)
// relaxed read of the pixel's key is an upper bound of its current value and
// the atomic can be skipped when the new key is not smaller.
//
// When the work item's points fall in a screen rectangle of at most
// kDedupPx pixels, they first meet in an LDS z-buffer over that rectangle
// (LDS 64-bit atomicMin), and only the nearest point of each pixel goes on to
// the global z-buffer, in row order: dense surfaces (many points per pixel)
// then cost one coalesced early-out read, and at most one atomic, per pixel
// instead of per point.  A work item spread over a larger rectangle (a near
// surface, few points per pixel) takes the per-point path.  The minimum is the
// same either way.
//
// COUNT adds the number of global atomics issued to counters[kAtomicWord]
// (one add per wave), for measurement; the keys written are the same.
constexpr int kDedupPx = 4096;
constexpr int kPtsPerThread = kSplatChunk / kThreads;
static_assert(kSplatChunk % kThreads == 0, "work items must split evenly over the threads");

template <bool COUNT>
__device__ inline void global_min(uint64_t *dst, uint64_t k, uint32_t &issued) {
  // relaxed atomic read: other blocks lower the word concurrently
  if (k < __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
    atomicMin(reinterpret_cast<unsigned long long *>(dst), (unsigned long long)k);
    if constexpr (COUNT) ++issued;
  }
}

// floor(p / w) for 0 <= p < 4096 and 1 <= w <= 4096, by a float reciprocal:
// the quotient of p + 1/2 is at least 1/(2w) from an integer, and the two
// float roundings move it by at most (4096/w) 2^-23, which is less, so the
// truncation lands on the same integer.  inv_w = 1.0f / w.
__device__ inline uint32_t small_div(uint32_t p, float inv_w) {
  return (uint32_t)(((float)p + 0.5f) * inv_w);
}

// Point j at (x, y, z) through the camera: true if drawn, with its key
// (depth bits << 32 | j) and pixel.
__device__ __attribute__((always_inline)) inline bool project_point(float x, float y, float z, uint32_t j, const SplatCam &cam, uint64_t &k,
                                     uint32_t &px, uint32_t &py) {
  const float *P = cam.P;
  const float a = ((P[0] * x + P[1] * y) + P[2] * z) + P[3];
  const float b = ((P[4] * x + P[5] * y) + P[6] * z) + P[7];
  const float w = ((P[8] * x + P[9] * y) + P[10] * z) + P[11];
  if (w >= cam.z_near && w <= cam.z_far) {
    const float u = a / w;
    const float v = b / w;
    if (u >= 0.f && u < cam.Wf && v >= 0.f && v < cam.Hf) {
      px = (uint32_t)u;
      py = (uint32_t)v;
      k = ((uint64_t)__float_as_uint(w) << 32) | j;
      return true;
    }
  }
  return false;
}

// The block-wide rectangle of the lanes' rectangles [x0, x1] x [y0, y1]
// (x0 > x1 if none).  Contains block barriers.
__device__ __attribute__((always_inline)) inline void block_rect(uint32_t x0, uint32_t y0, uint32_t x1, uint32_t y1, uint32_t *s_bb, uint32_t *rx0,
                                  uint32_t *ry0, uint32_t *rx1, uint32_t *ry1) {
  for (int off = 32; off > 0; off >>= 1) {
    x0 = min(x0, (uint32_t)__shfl_xor(x0, off, 64));
    y0 = min(y0, (uint32_t)__shfl_xor(y0, off, 64));
    x1 = max(x1, (uint32_t)__shfl_xor(x1, off, 64));
    y1 = max(y1, (uint32_t)__shfl_xor(y1, off, 64));
  }
  if (threadIdx.x == 0) {
    s_bb[0] = ~0u;
    s_bb[1] = ~0u;
    s_bb[2] = 0;
    s_bb[3] = 0;
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&s_bb[0], x0);
    atomicMin(&s_bb[1], y0);
    atomicMax(&s_bb[2], x1);
    atomicMax(&s_bb[3], y1);
  }
  __syncthreads();
  *rx0 = s_bb[0];
  *ry0 = s_bb[1];
  *rx1 = s_bb[2];
  *ry1 = s_bb[3];
}

// Project the work item's points (thread t takes points t, t + 256, ...):
// kk = key, (px, py) = pixel, px = ~0u if the point is not drawn; and the
// screen rectangle [x0, x1] x [y0, y1] of the drawn points over the whole
// block (x0 > x1 if none).  Contains block barriers.
__device__ inline void project_work_item(const float *__restrict__ xs, const float *__restrict__ ys,
                                         const float *__restrict__ zs, uint2 ch, const SplatCam &cam,
                                         uint64_t (&kk)[kPtsPerThread], uint32_t (&px)[kPtsPerThread],
                                         uint32_t (&py)[kPtsPerThread], uint32_t *s_bb, uint32_t *rx0, uint32_t *ry0,
                                         uint32_t *rx1, uint32_t *ry1) {
  const int tid = threadIdx.x;
  uint32_t x0 = ~0u, y0 = ~0u, x1 = 0, y1 = 0;
#pragma unroll
  for (int q = 0; q < kPtsPerThread; ++q) {
    const uint32_t i = tid + q * kThreads;
    uint64_t k = 0;
    uint32_t ux = ~0u, uy = 0;
    if (i < ch.y) {
      const uint32_t j = ch.x + i;
      if (project_point(xs[j], ys[j], zs[j], j, cam, k, ux, uy)) {
        x0 = min(x0, ux);
        x1 = max(x1, ux);
        y0 = min(y0, uy);
        y1 = max(y1, uy);
      } else {
        ux = ~0u;
      }
    }
    kk[q] = k;
    px[q] = ux;
    py[q] = uy;
  }
  block_rect(x0, y0, x1, y1, s_bb, rx0, ry0, rx1, ry1);
}

// Lower the global z-buffer (row length W) by the block's projected points,
// whose rectangle [x0, x1] x [y0, y1] is not empty: through the LDS z-buffer
// zb over the rectangle when it has at most kDedupPx pixels, else point by
// point.  Contains block barriers.
template <bool COUNT>
__device__ __attribute__((always_inline)) inline void splat_block(const uint64_t (&kk)[kPtsPerThread], const uint32_t (&px)[kPtsPerThread],
                                   const uint32_t (&py)[kPtsPerThread], uint32_t x0, uint32_t y0, uint32_t x1,
                                   uint32_t y1, uint32_t W, uint64_t *__restrict__ key, unsigned long long *zb,
                                   uint32_t &issued) {
  const int tid = threadIdx.x;
  const uint32_t bw = x1 - x0 + 1;
  const uint64_t a64 = (uint64_t)bw * (uint64_t)(y1 - y0 + 1);
  if (a64 <= (uint64_t)kDedupPx) {
    const uint32_t area = (uint32_t)a64;
    for (uint32_t p = tid; p < area; p += kThreads) zb[p] = ~0ull;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPtsPerThread; ++q)
      if (px[q] != ~0u) atomicMin(&zb[(py[q] - y0) * bw + (px[q] - x0)], (unsigned long long)kk[q]);
    __syncthreads();
    const float inv_bw = 1.0f / (float)bw;
    for (uint32_t p = tid; p < area; p += kThreads) {
      const uint64_t k = zb[p];
      if (k == ~0ull) continue;
      const uint32_t ry = small_div(p, inv_bw), rx = p - ry * bw;
      global_min<COUNT>(key + (size_t)(y0 + ry) * W + (x0 + rx), k, issued);
    }
  } else {
#pragma unroll
    for (int q = 0; q < kPtsPerThread; ++q)
      if (px[q] != ~0u) global_min<COUNT>(key + (size_t)py[q] * W + px[q], kk[q], issued);
  }
}

template <bool COUNT>
__global__ __launch_bounds__(kThreads) void splat_kernel(const float *__restrict__ xs, const float *__restrict__ ys,
                                                         const float *__restrict__ zs, const uint2 *__restrict__ chunks,
                                                         uint32_t cap, uint32_t *__restrict__ counters,
                                                         SplatCam cam, uint64_t *__restrict__ key) {
  __shared__ unsigned long long zb[kDedupPx];
  __shared__ uint32_t s_bb[4];
  uint2 ch;
  if (!work_item(blockIdx.x, counters, chunks, cap, &ch)) return;
  uint32_t issued = 0;
  uint64_t kk[kPtsPerThread];
  uint32_t px[kPtsPerThread], py[kPtsPerThread];
  uint32_t x0, y0, x1, y1;
  project_work_item(xs, ys, zs, ch, cam, kk, px, py, s_bb, &x0, &y0, &x1, &y1);
  if (x0 > x1) return;  // nothing drawn (the same for the whole block)
  splat_block<COUNT>(kk, px, py, x0, y0, x1, y1, cam.W, key, zb, issued);
  if constexpr (COUNT) {
    for (int off = 32; off > 0; off >>= 1) issued += __shfl_xor(issued, off, 64);
    if ((threadIdx.x & 63) == 0 && issued) atomicAdd(&counters[kAtomicWord], issued);
  }
}

// Several views at once: the work item's points are read from memory once,
// kept in registers, and projected and splatted into each view of its mask
// in turn, as splat_kernel does for one view.
__global__ __launch_bounds__(kThreads) void splat_views_kernel(const float *__restrict__ xs,
                                                               const float *__restrict__ ys,
                                                               const float *__restrict__ zs,
                                                               const uint4 *__restrict__ items, uint32_t cap,
                                                               const uint32_t *__restrict__ counters, ViewsSplat vs) {
  __shared__ unsigned long long zb[kDedupPx];
  __shared__ uint32_t s_bb[4];
  uint4 it;
  if (!work_item(blockIdx.x, counters, items, cap, &it)) return;
  const int tid = threadIdx.x;
  float x[kPtsPerThread], y[kPtsPerThread], z[kPtsPerThread];
#pragma unroll
  for (int q = 0; q < kPtsPerThread; ++q) {
    const uint32_t i = tid + q * kThreads;
    x[q] = y[q] = z[q] = 0.f;
    if (i < it.y) {
      x[q] = xs[it.x + i];
      y[q] = ys[it.x + i];
      z[q] = zs[it.x + i];
    }
  }
  uint32_t issued = 0;
  // the mask is the same for every lane: keep it (and the view index) scalar
  for (uint32_t m = __builtin_amdgcn_readfirstlane(it.z); m; m &= m - 1) {
    const int v = __builtin_ctz(m);
    const SplatCam &cam = vs.cam[v];
    uint64_t kk[kPtsPerThread];
    uint32_t px[kPtsPerThread], py[kPtsPerThread];
    uint32_t x0 = ~0u, y0 = ~0u, x1 = 0, y1 = 0;
#pragma unroll
    for (int q = 0; q < kPtsPerThread; ++q) {
      const uint32_t i = tid + q * kThreads;
      uint64_t k = 0;
      uint32_t ux = ~0u, uy = 0;
      if (i < it.y && project_point(x[q], y[q], z[q], it.x + i, cam, k, ux, uy)) {
        x0 = min(x0, ux);
        x1 = max(x1, ux);
        y0 = min(y0, uy);
        y1 = max(y1, uy);
      } else {
        ux = ~0u;
      }
      kk[q] = k;
      px[q] = ux;
      py[q] = uy;
    }
    block_rect(x0, y0, x1, y1, s_bb, &x0, &y0, &x1, &y1);
    if (x0 <= x1) splat_block<false>(kk, px, py, x0, y0, x1, y1, cam.W, vs.key[v], zb, issued);
    __syncthreads();  // s_bb and zb are reused by the next view
  }
}

// ---------------------------------------------------------------------------
// Screen-tiled splat (the default): no global atomic per point or pixel.
//
//   bin       one workgroup per work item: project the points; if they fall
//             in a screen rectangle of at most kDedupPx pixels, keep only the
//             nearest of each pixel (LDS z-buffer); counting-sort the rest by
//             32 x 32 screen tile in LDS and write them, grouped by tile, as
//             8-byte records at the work item's own place in the record
//             array.  Each (work item, tile) group is a segment.
//   tilescan  one workgroup: per-tile segment offsets, and the units of work
//             of the tile kernel: up to kSegsPerUnit segments of one tile.
//   segsort   groups the segment ids by tile, and empties the keys of the
//             tiles of more than one unit (the only keys not written whole).
//             Up to kMaxScanTiles tiles, segscan_kernel does both in one
//             launch (every workgroup repeats the scan in LDS).
//   tile      one workgroup per unit: LDS z-buffer of the tile over the
//             unit's records.  A tile of one unit owns its pixels and writes
//             key, depth and rgba (the resolve) with plain stores; the units
//             of a busier tile merge their minima into the key buffer with
//             atomicMin (one per pixel and unit), and
//   tileres   resolves those tiles afterwards.
//
// A record is (float32 depth bits << 32) | (pixel within the tile << 12) |
// (point index - work item start); the tile kernel rebuilds the key
// (depth bits << 32) | sorted index, so the image equals the atomic splat's.
// ---------------------------------------------------------------------------
constexpr int kTileShift = 5;  // 32 x 32 pixel tiles
constexpr int kTileSide = 1 << kTileShift;
constexpr int kTilePx = kTileSide * kTileSide;
constexpr int kHistBins = 1024;  // tiles one binning pass can address
constexpr int kSegsPerUnit = 32;
static_assert(kSplatChunk <= 4096, "a record keeps 12 bits of point offset");

// exclusive prefix over the block (blockDim.x = NT): each thread passes its
// value and gets the sum of the values of lower threads; *total receives the
// sum over the block
template <int NT>
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_tmp /* [NT / 64] */, uint32_t *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  if (lane == 63) s_tmp[wave] = incl;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const uint32_t x = s_tmp[w];
    if (w < wave) wbase += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return wbase + incl - v;
}

struct TileGrid {
  uint32_t tiles_x, tiles_y, n_tiles;
};

template <bool DEV>  // DEV: the camera comes from device memory (cam_dev), as in cull_kernel
__global__ __launch_bounds__(kThreads) void bin_kernel(const float *__restrict__ xs, const float *__restrict__ ys,
                                                       const float *__restrict__ zs, const uint2 *__restrict__ chunks,
                                                       uint32_t cap, uint32_t *__restrict__ counters, SplatCam cam_val,
                                                       const SplatCam *__restrict__ cam_dev, TileGrid tg,
                                                       uint64_t *__restrict__ recs, uint4 *__restrict__ segs,
                                                       uint32_t *__restrict__ tile_nseg) {
  const SplatCam &cam = DEV ? *cam_dev : cam_val;
  // The work item's entries live in LDS, one u64 per slot (~0 = none).  With
  // the on-chip z-buffer, slot = pixel of the rectangle (row order) and the
  // entry its nearest key (depth bits << 32 | point index); otherwise slot =
  // point (index - work item start) and the entry (depth bits << 32 |
  // py << 16 | px).
  __shared__ unsigned long long s_ent[kDedupPx];
  __shared__ uint32_t s_hist[kHistBins];
  __shared__ uint32_t s_tmp[kThreads / 64];
  __shared__ uint32_t s_bb[4];
  __shared__ uint32_t s_seg_base;
  uint2 ch;
  if (!work_item(blockIdx.x, counters, chunks, cap, &ch)) return;
  const int tid = threadIdx.x;
  uint32_t x0, y0, x1, y1, bw, nslots;
  bool dedup;
  {
    uint64_t kk[kPtsPerThread];
    uint32_t px[kPtsPerThread], py[kPtsPerThread];
    project_work_item(xs, ys, zs, ch, cam, kk, px, py, s_bb, &x0, &y0, &x1, &y1);
    if (x0 > x1) return;  // nothing drawn (the same for the whole block)
    bw = x1 - x0 + 1;
    const uint64_t a64 = (uint64_t)bw * (uint64_t)(y1 - y0 + 1);
    dedup = a64 <= (uint64_t)kDedupPx;
    if (dedup) {
      nslots = (uint32_t)a64;
      for (uint32_t p = tid; p < nslots; p += kThreads) s_ent[p] = ~0ull;
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kPtsPerThread; ++q)
        if (px[q] != ~0u) atomicMin(&s_ent[(py[q] - y0) * bw + (px[q] - x0)], (unsigned long long)kk[q]);
    } else {
      nslots = ch.y;
#pragma unroll
      for (int q = 0; q < kPtsPerThread; ++q) {
        const uint32_t i = tid + q * kThreads;
        if (i < ch.y)
          s_ent[i] = px[q] == ~0u ? ~0ull : ((kk[q] & 0xFFFFFFFF00000000ull) | (py[q] << 16) | px[q]);
      }
    }
  }
  __syncthreads();
  // pixel and key of an entry in slot p
  const float inv_bw = 1.0f / (float)bw;
  auto decode = [&](uint32_t p, uint64_t e, uint32_t *gx, uint32_t *gy) -> uint64_t {
    if (dedup) {
      const uint32_t ry = small_div(p, inv_bw);
      *gy = y0 + ry;
      *gx = x0 + (p - ry * bw);
      return e;
    }
    *gy = ((uint32_t)e >> 16) & 0xFFFFu;
    *gx = (uint32_t)e & 0xFFFFu;
    return (e & 0xFFFFFFFF00000000ull) | (uint64_t)(ch.x + p);
  };
  // counting sort of the entries by tile, in rounds of tile rows so that one
  // round addresses at most kHistBins tiles
  const uint32_t tx0 = x0 >> kTileShift, ty0 = y0 >> kTileShift;
  const uint32_t tbw = (x1 >> kTileShift) - tx0 + 1, ty1 = y1 >> kTileShift;
  const uint32_t rows_per_round = max(1u, (uint32_t)kHistBins / tbw);
  uint32_t rec_next = 0;  // records written by earlier rounds
  for (uint32_t r0 = ty0; r0 <= ty1; r0 += rows_per_round) {
    const uint32_t r1 = min(ty1 + 1, r0 + rows_per_round);
    const uint32_t tbins = (r1 - r0) * tbw;
    // a row wider than the histogram is split into column ranges
    for (uint32_t c0 = 0; c0 < tbins; c0 += kHistBins) {
      const uint32_t nbins = min((uint32_t)kHistBins, tbins - c0);
      for (uint32_t b = tid; b < nbins; b += kThreads) s_hist[b] = 0;
      __syncthreads();
      for (uint32_t p = tid; p < nslots; p += kThreads) {
        const uint64_t e = s_ent[p];
        if (e == ~0ull) continue;
        uint32_t gx, gy;
        decode(p, e, &gx, &gy);
        const uint32_t ty = gy >> kTileShift;
        const uint32_t bin = (ty - r0) * tbw + ((gx >> kTileShift) - tx0) - c0;
        if (ty >= r0 && ty < r1 && bin < nbins) atomicAdd(&s_hist[bin], 1u);
      }
      __syncthreads();
      // exclusive prefix over the bins of record counts and non-empty flags
      // at once (16-bit halves: at most 4096 of each); a thread owns kPer bins
      constexpr int kPer = kHistBins / kThreads;
      uint32_t sum = 0;
      for (int q = 0; q < kPer; ++q) {
        const uint32_t b = tid * kPer + q;
        const uint32_t c = b < nbins ? s_hist[b] : 0u;
        sum += (c << 16) | (c ? 1u : 0u);
      }
      uint32_t total;
      uint32_t run = block_exclusive_scan<kThreads>(sum, s_tmp, &total);
      const uint32_t n_rec = total >> 16, n_seg = total & 0xFFFFu;
      if (n_rec == 0) continue;  // uniform: nothing in these bins
      if (tid == 0) s_seg_base = atomicAdd(&counters[kSegTopWord], n_seg);
      __syncthreads();
      const uint32_t seg_base = s_seg_base;
      for (int q = 0; q < kPer; ++q) {
        const uint32_t b = tid * kPer + q;
        if (b >= nbins) break;
        const uint32_t c = s_hist[b];
        const uint32_t first = rec_next + (run >> 16);
        if (c) {
          const uint32_t tb = c0 + b;
          const uint32_t tile = (r0 + tb / tbw) * tg.tiles_x + (tx0 + tb % tbw);
          segs[seg_base + (run & 0xFFFFu)] = make_uint4(tile, ch.x + first, c, ch.x);
          atomicAdd(&tile_nseg[tile], 1u);
        }
        s_hist[b] = first;  // bin -> cursor at its first record
        run += (c << 16) | (c ? 1u : 0u);
      }
      __syncthreads();
      for (uint32_t p = tid; p < nslots; p += kThreads) {
        const uint64_t e = s_ent[p];
        if (e == ~0ull) continue;
        uint32_t gx, gy;
        const uint64_t k = decode(p, e, &gx, &gy);
        const uint32_t ty = gy >> kTileShift;
        const uint32_t bin = (ty - r0) * tbw + ((gx >> kTileShift) - tx0) - c0;
        if (ty < r0 || ty >= r1 || bin >= nbins) continue;
        const uint32_t pos = atomicAdd(&s_hist[bin], 1u);
        const uint32_t local = ((gy & (kTileSide - 1)) << kTileShift) | (gx & (kTileSide - 1));
        recs[ch.x + pos] = (k & 0xFFFFFFFF00000000ull) | ((uint64_t)local << 12) | (uint64_t)((uint32_t)k - ch.x);
      }
      rec_next += n_rec;
      __syncthreads();
    }
  }
}

// One workgroup: per-tile segment offsets (tile_off[n_tiles + 1]) and the
// units of the tile kernel: a tile with s segments gets max(1, ceil(s /
// kSegsPerUnit)) units (tile_units[t]); units[u] = (tile, first segment of
// the unit within the tile); counters[kUnitsWord] = number of units.
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void tilescan_kernel(const uint32_t *__restrict__ tile_nseg, TileGrid tg,
                                                                uint32_t *__restrict__ tile_off,
                                                                uint32_t *__restrict__ tile_units,
                                                                uint2 *__restrict__ units, uint32_t unit_cap,
                                                                uint32_t *__restrict__ counters) {
  __shared__ uint32_t s_tmp[kScanThreads / 64];
  const int tid = threadIdx.x;
  uint32_t seg_base = 0, unit_base = 0;
  for (uint32_t t0 = 0; t0 < tg.n_tiles; t0 += kScanThreads) {
    const uint32_t t = t0 + tid;
    const uint32_t ns = t < tg.n_tiles ? tile_nseg[t] : 0u;
    const uint32_t nu = t < tg.n_tiles ? max(1u, (ns + kSegsPerUnit - 1) / kSegsPerUnit) : 0u;
    uint32_t tot_s, tot_u;
    const uint32_t es = block_exclusive_scan<kScanThreads>(ns, s_tmp, &tot_s);
    const uint32_t eu = block_exclusive_scan<kScanThreads>(nu, s_tmp, &tot_u);
    if (t < tg.n_tiles) {
      tile_off[t] = seg_base + es;
      tile_units[t] = nu;
      for (uint32_t k = 0; k < nu; ++k)
        if (unit_base + eu + k < unit_cap) units[unit_base + eu + k] = make_uint2(t, k * kSegsPerUnit);
    }
    seg_base += tot_s;
    unit_base += tot_u;
  }
  if (tid == 0) {
    tile_off[tg.n_tiles] = seg_base;
    counters[kUnitsWord] = min(unit_base, unit_cap);
  }
}

// Segment ids grouped by tile: segment i of tile t goes to one of the places
// [tile_off[t], tile_off[t + 1]) (their order is irrelevant: the tile kernel
// takes a minimum).  Counts tile_nseg back down to zero.  Also empties the
// key buffer over the tiles of more than one unit, whose units merge into it
// with atomicMin (the tile kernel writes every other tile's keys whole).
__global__ __launch_bounds__(kThreads) void segsort_kernel(const uint4 *__restrict__ segs,
                                                           const uint32_t *__restrict__ counters,
                                                           const uint32_t *__restrict__ tile_off,
                                                           uint32_t *__restrict__ tile_nseg,
                                                           uint32_t *__restrict__ sorted,
                                                           const uint32_t *__restrict__ tile_units, TileGrid tg,
                                                           uint32_t W, uint32_t H, uint64_t *__restrict__ key) {
  const uint32_t n = counters[kSegTopWord];
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    const uint32_t t = segs[i].x;
    sorted[tile_off[t] + atomicSub(&tile_nseg[t], 1u) - 1u] = i;
  }
  for (uint32_t t = blockIdx.x; t < tg.n_tiles; t += gridDim.x) {
    if (tile_units[t] <= 1) continue;  // (the same for the whole block)
    const uint32_t tx = t % tg.tiles_x, ty = t / tg.tiles_x;
    for (int p = threadIdx.x; p < kTilePx; p += kThreads) {
      const uint32_t gx = (tx << kTileShift) + (p & (kTileSide - 1));
      const uint32_t gy = (ty << kTileShift) + (p >> kTileShift);
      if (gx < W && gy < H) key[(size_t)gy * W + gx] = ~0ull;
    }
  }
}

// The scan and the segment sort in one launch, for images of at most
// kMaxScanTiles tiles: every workgroup takes the exclusive prefix of the
// per-tile segment counts itself, into LDS (a few thousand words, read from
// L2; each thread sums a run of consecutive tiles, one block scan of the
// sums, then each thread walks its run), so no workgroup waits for another; workgroup 0 also writes tile_off,
// tile_units, units and counters[kUnitsWord] for the tile kernel, as
// tilescan_kernel does.  The places within a tile come from a second counter
// array (tile_fill, zeroed with tile_nseg), since tile_nseg is read by every
// workgroup's scan.  Then, as segsort_kernel: the segment ids grouped by tile,
// and the keys of the tiles of more than one unit emptied.
constexpr uint32_t kMaxScanTiles = 8192;
__global__ __launch_bounds__(kThreads) void segscan_kernel(const uint4 *__restrict__ segs,
                                                           uint32_t *__restrict__ counters,
                                                           const uint32_t *__restrict__ tile_nseg,
                                                           uint32_t *__restrict__ tile_fill,
                                                           uint32_t *__restrict__ tile_off,
                                                           uint32_t *__restrict__ tile_units,
                                                           uint2 *__restrict__ units, uint32_t unit_cap,
                                                           uint32_t *__restrict__ sorted, TileGrid tg, uint32_t W,
                                                           uint32_t H, uint64_t *__restrict__ key) {
  __shared__ uint32_t s_off[kMaxScanTiles + 1];
  __shared__ uint32_t s_tmp[kThreads / 64];
  const int tid = threadIdx.x;
  const bool first = blockIdx.x == 0;
  // thread tid owns tiles [tid per, (tid + 1) per): its own sums, one block
  // scan of them, then its tiles' offsets in order
  const uint32_t per = (tg.n_tiles + kThreads - 1) / kThreads;
  const uint32_t t_lo = min(tg.n_tiles, tid * per), t_hi = min(tg.n_tiles, t_lo + per);
  uint32_t my_s = 0, my_u = 0;
  for (uint32_t t = t_lo; t < t_hi; ++t) {
    const uint32_t ns = tile_nseg[t];
    my_s += ns;
    my_u += max(1u, (ns + kSegsPerUnit - 1) / kSegsPerUnit);
  }
  uint32_t tot_s, tot_u;
  uint32_t seg = block_exclusive_scan<kThreads>(my_s, s_tmp, &tot_s);
  uint32_t unit = block_exclusive_scan<kThreads>(my_u, s_tmp, &tot_u);
  for (uint32_t t = t_lo; t < t_hi; ++t) {
    const uint32_t ns = tile_nseg[t];
    const uint32_t nu = max(1u, (ns + kSegsPerUnit - 1) / kSegsPerUnit);
    s_off[t] = seg;
    if (first) {
      tile_off[t] = seg;
      tile_units[t] = nu;
      for (uint32_t k = 0; k < nu; ++k)
        if (unit + k < unit_cap) units[unit + k] = make_uint2(t, k * kSegsPerUnit);
    }
    seg += ns;
    unit += nu;
  }
  if (tid == 0) {
    s_off[tg.n_tiles] = tot_s;
    if (first) {
      tile_off[tg.n_tiles] = tot_s;
      counters[kUnitsWord] = min(tot_u, unit_cap);
    }
  }
  __syncthreads();
  const uint32_t n = counters[kSegTopWord];
  for (uint32_t i = blockIdx.x * kThreads + tid; i < n; i += gridDim.x * kThreads) {
    const uint32_t t = segs[i].x;
    sorted[s_off[t] + atomicAdd(&tile_fill[t], 1u)] = i;
  }
  for (uint32_t t = blockIdx.x; t < tg.n_tiles; t += gridDim.x) {
    if (s_off[t + 1] - s_off[t] <= (uint32_t)kSegsPerUnit) continue;  // one unit (the same for the whole block)
    const uint32_t tx = t % tg.tiles_x, ty = t / tg.tiles_x;
    for (int p = tid; p < kTilePx; p += kThreads) {
      const uint32_t gx = (tx << kTileShift) + (p & (kTileSide - 1));
      const uint32_t gy = (ty << kTileShift) + (p >> kTileShift);
      if (gx < W && gy < H) key[(size_t)gy * W + gx] = ~0ull;
    }
  }
}

__device__ inline void resolve_px(uint64_t k, const uint32_t *__restrict__ rgbx, size_t i, float *__restrict__ depth,
                                  uint32_t *__restrict__ rgba) {
  if (k == ~0ull) {
    depth[i] = 0.f;
    rgba[i] = 0u;
  } else {
    depth[i] = __uint_as_float((uint32_t)(k >> 32));
    rgba[i] = (rgbx[(uint32_t)k] & 0x00FFFFFFu) | (1u << 24);
  }
}

// Units of work, grid-stride: the LDS z-buffer of one tile over the records
// of up to kSegsPerUnit of its segments.
__global__ __launch_bounds__(kThreads) void tile_kernel(const uint64_t *__restrict__ recs,
                                                        const uint4 *__restrict__ segs,
                                                        const uint32_t *__restrict__ sorted,
                                                        const uint32_t *__restrict__ tile_off,
                                                        const uint32_t *__restrict__ tile_units,
                                                        const uint2 *__restrict__ units,
                                                        const uint32_t *__restrict__ counters, TileGrid tg,
                                                        const uint32_t *__restrict__ rgbx, uint32_t W, uint32_t H,
                                                        uint64_t *__restrict__ key, float *__restrict__ depth,
                                                        uint32_t *__restrict__ rgba) {
  __shared__ unsigned long long zb[kTilePx];
  __shared__ uint32_t s_pref[kSegsPerUnit + 1];
  __shared__ uint2 s_seg[kSegsPerUnit];  // first record, work item start
  const int tid = threadIdx.x;
  const uint32_t n_units = counters[kUnitsWord];
  for (uint32_t u = blockIdx.x; u < n_units; u += gridDim.x) {
    const uint2 un = units[u];
    const uint32_t t = un.x;
    const uint32_t beg = tile_off[t] + un.y, end = min(tile_off[t + 1], beg + kSegsPerUnit);
    const uint32_t nb = end > beg ? end - beg : 0u;
    for (int p = tid; p < kTilePx; p += kThreads) zb[p] = ~0ull;
    if (tid < 64) {  // the unit's segments and the prefix of their record counts (one wave)
      uint32_t c = 0;
      if ((uint32_t)tid < nb) {
        const uint4 sg = segs[sorted[beg + tid]];
        s_seg[tid] = make_uint2(sg.y, sg.w);
        c = sg.z;
      }
      uint32_t incl = c;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(incl, off, 64);
        if (tid >= off) incl += o;
      }
      if (tid <= kSegsPerUnit) s_pref[tid] = incl - c;  // s_pref[nb] = total
    }
    __syncthreads();
    const uint32_t total = s_pref[nb];
    // kInFlight records per thread: their loads are issued before the first
    // LDS atomic, so their latencies overlap
    constexpr int kInFlight = 4;
    for (uint32_t r0 = tid; r0 < total; r0 += kInFlight * kThreads) {
      uint64_t rc[kInFlight];
      uint32_t base[kInFlight];
#pragma unroll
      for (int m = 0; m < kInFlight; ++m) {
        const uint32_t r = r0 + m * kThreads;
        rc[m] = ~0ull;
        base[m] = 0;
        if (r < total) {
          uint32_t lo = 0, hi = nb;  // the last segment whose prefix is <= r
          while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_pref[mid] <= r) lo = mid;
            else hi = mid;
          }
          const uint2 sg = s_seg[lo];
          rc[m] = recs[sg.x + (r - s_pref[lo])];
          base[m] = sg.y;
        }
      }
#pragma unroll
      for (int m = 0; m < kInFlight; ++m) {
        if (rc[m] == ~0ull) continue;
        const uint64_t k = (rc[m] & 0xFFFFFFFF00000000ull) | (uint64_t)(base[m] + (uint32_t)(rc[m] & 0xFFFu));
        atomicMin(&zb[(rc[m] >> 12) & (kTilePx - 1)], (unsigned long long)k);
      }
    }
    __syncthreads();
    const bool alone = tile_units[t] == 1;
    const uint32_t tx = t % tg.tiles_x, ty = t / tg.tiles_x;
    for (int p = tid; p < kTilePx; p += kThreads) {
      const uint32_t gx = (tx << kTileShift) + (p & (kTileSide - 1));
      const uint32_t gy = (ty << kTileShift) + (p >> kTileShift);
      if (gx >= W || gy >= H) continue;
      const size_t i = (size_t)gy * W + gx;
      const uint64_t k = zb[p];
      if (alone) {
        key[i] = k;
        resolve_px(k, rgbx, i, depth, rgba);
      } else if (k != ~0ull) {
        atomicMin(reinterpret_cast<unsigned long long *>(key + i), (unsigned long long)k);
      }
    }
    __syncthreads();
  }
}

// Resolve of the tiles whose units merged through the key buffer.
__global__ __launch_bounds__(kThreads) void tileres_kernel(const uint32_t *__restrict__ tile_units, TileGrid tg,
                                                           const uint32_t *__restrict__ rgbx, uint32_t W, uint32_t H,
                                                           const uint64_t *__restrict__ key, float *__restrict__ depth,
                                                           uint32_t *__restrict__ rgba) {
  const uint32_t t = blockIdx.x;
  if (tile_units[t] == 1) return;
  const uint32_t tx = t % tg.tiles_x, ty = t / tg.tiles_x;
  for (int p = threadIdx.x; p < kTilePx; p += kThreads) {
    const uint32_t gx = (tx << kTileShift) + (p & (kTileSide - 1));
    const uint32_t gy = (ty << kTileShift) + (p >> kTileShift);
    if (gx >= W || gy >= H) continue;
    const size_t i = (size_t)gy * W + gx;
    resolve_px(key[i], rgbx, i, depth, rgba);
  }
}

// Throughput probe for the z-buffer's operation: each thread issues
// kProbeIters 64-bit atomicMin.  Pattern 0 draws the word of each from a
// per-thread xorshift32 sequence (Marsaglia's 13/17/5 shifts), so the
// operations spread over the buffer as a splat's do over the image; pattern 1
// sends the 64 lanes of a wave to one word.  Values decrease along each
// thread's sequence, so most operations lower the word.
__global__ __launch_bounds__(kThreads) void atomic_probe_kernel(uint64_t *__restrict__ buf, uint32_t n_slots,
                                                                int pattern, uint32_t seed) {
  const uint32_t gid = blockIdx.x * kThreads + threadIdx.x;
  uint32_t x = (gid + 1u) * 0x9E3779B9u ^ seed;
  if (x == 0) x = 1u;
  const uint32_t wave = gid >> 6, nwaves = gridDim.x * (kThreads / 64);
  for (uint32_t i = 0; i < kProbeIters; ++i) {
    uint32_t slot;
    if (pattern == 0) {
      x ^= x << 13;
      x ^= x >> 17;
      x ^= x << 5;
      slot = x % n_slots;
    } else {
      slot = (i * nwaves + wave) % n_slots;
    }
    const uint64_t v = ((uint64_t)(kProbeIters - i) << 32) | gid;
    atomicMin(reinterpret_cast<unsigned long long *>(buf + slot), (unsigned long long)v);
  }
}

// Soft z-buffer (Method, "Point Cloud Projection": colours of points at similar
// depths are averaged).  A second pass over the same work items adds the colour
// of every point whose depth is within (1 + eps) of its pixel's nearest depth
// into integer sums; integer atomics make the result order independent.
template <bool DEV>  // DEV: the camera comes from device memory (cam_dev), as in cull_kernel
__global__ __launch_bounds__(kThreads) void soft_accum_kernel(const float *__restrict__ xs, const float *__restrict__ ys,
                                                              const float *__restrict__ zs,
                                                              const uint32_t *__restrict__ rgbx,
                                                              const uint2 *__restrict__ chunks, uint32_t cap,
                                                              const uint32_t *__restrict__ counters, SplatCam cam_val,
                                                              const SplatCam *__restrict__ cam_dev,
                                                              const uint64_t *__restrict__ key, float one_plus_eps,
                                                              uint32_t *__restrict__ acc) {
  const SplatCam &cam = DEV ? *cam_dev : cam_val;
  uint2 ch;
  if (!work_item(blockIdx.x, counters, chunks, cap, &ch)) return;
  const float *P = cam.P;
  for (uint32_t i = threadIdx.x; i < ch.y; i += kThreads) {
    const uint32_t j = ch.x + i;
    const float x = xs[j], y = ys[j], z = zs[j];
    const float a = ((P[0] * x + P[1] * y) + P[2] * z) + P[3];
    const float b = ((P[4] * x + P[5] * y) + P[6] * z) + P[7];
    const float w = ((P[8] * x + P[9] * y) + P[10] * z) + P[11];
    if (!(w >= cam.z_near && w <= cam.z_far)) continue;
    const float u = a / w;
    const float v = b / w;
    if (!(u >= 0.f && u < cam.Wf && v >= 0.f && v < cam.Hf)) continue;
    const size_t p = (size_t)(uint32_t)v * cam.W + (uint32_t)u;
    const float zmin = __uint_as_float((uint32_t)(key[p] >> 32));
    if (!(w <= zmin * one_plus_eps)) continue;
    const uint32_t c = rgbx[j];
    atomicAdd(&acc[4 * p + 0], c & 255u);
    atomicAdd(&acc[4 * p + 1], (c >> 8) & 255u);
    atomicAdd(&acc[4 * p + 2], (c >> 16) & 255u);
    atomicAdd(&acc[4 * p + 3], 1u);
  }
}

__global__ __launch_bounds__(kThreads) void resolve_soft_kernel(const uint64_t *__restrict__ key,
                                                                const uint32_t *__restrict__ acc,
                                                                float *__restrict__ depth, uint32_t *__restrict__ rgba,
                                                                uint32_t npix) {
  const uint32_t stride = gridDim.x * kThreads;
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < npix; i += stride) {
    const uint64_t k = key[i];
    if (k == ~0ull) {
      depth[i] = 0.f;
      rgba[i] = 0u;
    } else {
      depth[i] = __uint_as_float((uint32_t)(k >> 32));
      const uint4 s = *reinterpret_cast<const uint4 *>(acc + 4ull * i);
      const uint64_t n2 = 2ull * s.w;
      const uint32_t r = (uint32_t)((2ull * s.x + s.w) / n2);
      const uint32_t g = (uint32_t)((2ull * s.y + s.w) / n2);
      const uint32_t b = (uint32_t)((2ull * s.z + s.w) / n2);
      rgba[i] = r | (g << 8) | (b << 16) | (1u << 24);
    }
  }
}

__global__ __launch_bounds__(kThreads) void clear_acc_kernel(uint4 *__restrict__ acc, uint32_t npix) {
  const uint32_t stride = gridDim.x * kThreads;
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < npix; i += stride) acc[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ __launch_bounds__(kThreads) void resolve_kernel(const uint64_t *__restrict__ key,
                                                           const uint32_t *__restrict__ rgbx, float *__restrict__ depth,
                                                           uint32_t *__restrict__ rgba, uint32_t npix) {
  const uint32_t stride = gridDim.x * kThreads;
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < npix; i += stride) {
    const uint64_t k = key[i];
    if (k == ~0ull) {
      depth[i] = 0.f;
      rgba[i] = 0u;
    } else {
      depth[i] = __uint_as_float((uint32_t)(k >> 32));
      rgba[i] = (rgbx[(uint32_t)k] & 0x00FFFFFFu) | (1u << 24);
    }
  }
}

inline uint32_t grid_for(uint32_t n) {
  uint32_t b = (n + kThreads - 1) / kThreads;
  return b < 1 ? 1 : (b > 8192 ? 8192 : b);
}

}  // namespace

hipError_t launch_clear(uint64_t *key, uint32_t npix, uint32_t *counters, uint32_t *tile_nseg, uint32_t n_tiles,
                        hipStream_t s) {
  clear_kernel<<<grid_for(npix > n_tiles ? npix : n_tiles), kThreads, 0, s>>>(key, npix, counters, tile_nseg,
                                                                             n_tiles);
  return hipGetLastError();
}

bool tiled_scan_merged(const TiledSplatGrid &g) { return g.n_tiles <= kMaxScanTiles; }

TiledSplatGrid tiled_splat_grid(uint32_t W, uint32_t H, uint32_t n_points) {
  TiledSplatGrid g;
  g.tiles_x = (W + kTileSide - 1) >> kTileShift;
  g.tiles_y = (H + kTileSide - 1) >> kTileShift;
  g.n_tiles = g.tiles_x * g.tiles_y;
  // a tile has max(1, ceil(s / kSegsPerUnit)) units, and there are at most
  // n_points segments (one record at least each)
  g.unit_cap = 2ull * g.n_tiles + n_points / kSegsPerUnit + 1;
  return g;
}

hipError_t launch_tiled_splat(const CloudDev &c, const uint2 *chunks, uint32_t *counters, const SplatCam &cam,
                              const SplatCam *cam_dev, uint32_t H, const TiledSplatBufs &b, uint64_t *key,
                              float *depth, uint32_t *rgba, int stage, hipStream_t s) {
  if (c.max_chunks == 0) return hipErrorInvalidValue;  // a loaded cloud has at least one point
  const TiledSplatGrid g = tiled_splat_grid(cam.W, H, c.n);
  const TileGrid tg{g.tiles_x, g.tiles_y, g.n_tiles};
  switch (stage) {
    case 0:
      if (cam_dev)
        bin_kernel<true><<<c.max_chunks, kThreads, 0, s>>>(c.x, c.y, c.z, chunks, c.max_chunks, counters, cam, cam_dev,
                                                          tg, b.recs, b.segs, b.tile_nseg);
      else
        bin_kernel<false><<<c.max_chunks, kThreads, 0, s>>>(c.x, c.y, c.z, chunks, c.max_chunks, counters, cam,
                                                           nullptr, tg, b.recs, b.segs, b.tile_nseg);
      break;
    case 1:
      if (tiled_scan_merged(g)) return hipSuccess;  // taken by the segment sort
      tilescan_kernel<<<1, kScanThreads, 0, s>>>(b.tile_nseg, tg, b.tile_off, b.tile_units, b.units,
                                                 (uint32_t)g.unit_cap, counters);
      break;
    case 2:
      if (tiled_scan_merged(g))
        segscan_kernel<<<256, kThreads, 0, s>>>(b.segs, counters, b.tile_nseg, b.tile_nseg + g.n_tiles, b.tile_off,
                                                b.tile_units, b.units, (uint32_t)g.unit_cap, b.sorted, tg, cam.W, H,
                                                key);
      else
        segsort_kernel<<<1024, kThreads, 0, s>>>(b.segs, counters, b.tile_off, b.tile_nseg, b.sorted, b.tile_units,
                                                  tg, cam.W, H, key);
      break;
    case 3: {
      const uint64_t grid = std::min<uint64_t>(g.unit_cap, std::max<uint64_t>(2ull * g.n_tiles, 4096));
      tile_kernel<<<(uint32_t)grid, kThreads, 0, s>>>(b.recs, b.segs, b.sorted, b.tile_off, b.tile_units, b.units,
                                                      counters, tg, c.rgbx, cam.W, H, key, depth, rgba);
      break;
    }
    case 4:
      tileres_kernel<<<g.n_tiles, kThreads, 0, s>>>(b.tile_units, tg, c.rgbx, cam.W, H, key, depth, rgba);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cull(const CloudDev &c, const CullParams &prm, const CullParams *prm_dev, uint8_t *flags,
                       uint2 *chunks, uint32_t *counters, hipStream_t s) {
  const uint32_t nb = (c.n_cells + kThreads - 1) / kThreads;
  if (prm_dev)
    cull_kernel<true><<<nb, kThreads, 0, s>>>(c.aabb, c.cell_start, c.n_cells, prm, prm_dev, flags, chunks,
                                              c.max_chunks, counters);
  else
    cull_kernel<false><<<nb, kThreads, 0, s>>>(c.aabb, c.cell_start, c.n_cells, prm, nullptr, flags, chunks,
                                               c.max_chunks, counters);
  return hipGetLastError();
}

hipError_t launch_splat(const CloudDev &c, const uint2 *chunks, uint32_t *counters, const SplatCam &cam,
                        uint64_t *key, bool count_atomics, hipStream_t s) {
  if (c.max_chunks == 0) return hipSuccess;
  const uint32_t g = c.max_chunks, cap = c.max_chunks;
  if (count_atomics)
    splat_kernel<true><<<g, kThreads, 0, s>>>(c.x, c.y, c.z, chunks, cap, counters, cam, key);
  else
    splat_kernel<false><<<g, kThreads, 0, s>>>(c.x, c.y, c.z, chunks, cap, counters, cam, key);
  return hipGetLastError();
}

hipError_t launch_cull_views(const CloudDev &c, const ViewsCull &prm, uint8_t *flags, uint4 *items, uint32_t *counters,
                             hipStream_t s) {
  if (prm.n < 1 || prm.n > kViewsPerPass) return hipErrorInvalidValue;
  const uint32_t nb = (c.n_cells + kThreads - 1) / kThreads;
  cull_views_kernel<<<nb, kThreads, 0, s>>>(c.aabb, c.cell_start, c.n_cells, prm, flags, items, c.max_chunks,
                                            counters);
  return hipGetLastError();
}

hipError_t launch_splat_views(const CloudDev &c, const uint4 *items, const uint32_t *counters, const ViewsSplat &vs,
                              hipStream_t s) {
  if (vs.n < 1 || vs.n > kViewsPerPass) return hipErrorInvalidValue;
  if (c.max_chunks == 0) return hipSuccess;
  splat_views_kernel<<<c.max_chunks, kThreads, 0, s>>>(c.x, c.y, c.z, items, c.max_chunks, counters, vs);
  return hipGetLastError();
}

hipError_t launch_atomic_probe(uint64_t *buf, uint32_t n_slots, int pattern, uint32_t grid, uint32_t seed,
                               hipStream_t s) {
  if (n_slots == 0 || grid == 0) return hipErrorInvalidValue;
  atomic_probe_kernel<<<grid, kThreads, 0, s>>>(buf, n_slots, pattern, seed);
  return hipGetLastError();
}

hipError_t launch_resolve(const uint64_t *key, const uint32_t *rgbx, float *depth, uint32_t *rgba, uint32_t npix,
                          hipStream_t s) {
  resolve_kernel<<<grid_for(npix), kThreads, 0, s>>>(key, rgbx, depth, rgba, npix);
  return hipGetLastError();
}

hipError_t launch_soft(const CloudDev &c, const uint2 *chunks, const uint32_t *counters, const SplatCam &cam,
                       const SplatCam *cam_dev, const uint64_t *key, float one_plus_eps, uint32_t *acc, float *depth,
                       uint32_t *rgba, uint32_t npix, hipStream_t s) {
  clear_acc_kernel<<<grid_for(npix), kThreads, 0, s>>>(reinterpret_cast<uint4 *>(acc), npix);
  if (c.max_chunks)
  {
    if (cam_dev)
      soft_accum_kernel<true><<<c.max_chunks, kThreads, 0, s>>>(c.x, c.y, c.z, c.rgbx, chunks, c.max_chunks, counters,
                                                               cam, cam_dev, key, one_plus_eps, acc);
    else
      soft_accum_kernel<false><<<c.max_chunks, kThreads, 0, s>>>(c.x, c.y, c.z, c.rgbx, chunks, c.max_chunks,
                                                                counters, cam, nullptr, key, one_plus_eps, acc);
  }
  resolve_soft_kernel<<<grid_for(npix), kThreads, 0, s>>>(key, acc, depth, rgba, npix);
  return hipGetLastError();
}

}  // namespace lnr
