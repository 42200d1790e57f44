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

#include "lnr_internal.h"

#pragma clang fp contract(off)

namespace lnr {
namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void clear_kernel(uint64_t *__restrict__ key, uint32_t npix,
                                                         uint32_t *__restrict__ counters) {
  const uint32_t stride = gridDim.x * kThreads;
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < npix; i += stride) key[i] = ~0ull;
  if (blockIdx.x == 0 && threadIdx.x < kCounterWords) counters[threadIdx.x] = 0;
}

// One lane per cell.  A non-empty cell is visible unless some half-space's
// maximum over the cell's box is below -slack (all in double, in the order
// below).  Visible cells are cut into splat work items of at most kSplatChunk
// points, queued in the depth bucket of the cell's centre; the totals are
// reduced per wave with one atomic per wave.
__global__ __launch_bounds__(kThreads) void cull_kernel(const float *__restrict__ aabb,
                                                        const uint32_t *__restrict__ cell_start, uint32_t n_cells,
                                                        CullParams prm, uint8_t *__restrict__ flags,
                                                        uint2 *__restrict__ chunks, uint32_t cap,
                                                        uint32_t *__restrict__ counters) {
  const uint32_t c = blockIdx.x * kThreads + threadIdx.x;
  const int lane = threadIdx.x & 63;
  uint32_t start = 0, cnt = 0;
  bool vis = false;
  int bucket = 0;
  if (c < n_cells) {
    start = cell_start[c];
    cnt = cell_start[c + 1] - start;
    if (cnt > 0) {
      const double lo0 = aabb[6ull * c + 0], lo1 = aabb[6ull * c + 1], lo2 = aabb[6ull * c + 2];
      const double hi0 = aabb[6ull * c + 3], hi1 = aabb[6ull * c + 4], hi2 = aabb[6ull * c + 5];
      if (prm.no_cull) {
        vis = true;
      } else {
        const double mx0 = fmax(fabs(lo0), fabs(hi0));
        const double mx1 = fmax(fabs(lo1), fabs(hi1));
        const double mx2 = fmax(fabs(lo2), fabs(hi2));
        double S[3];
        for (int r = 0; r < 3; ++r)
          S[r] = ((prm.absP[r][0] * mx0 + prm.absP[r][1] * mx1) + prm.absP[r][2] * mx2) + prm.absP[r][3];
        const double slack = 0x1p-20 * ((S[0] + S[1]) + prm.wh1 * S[2]);
        vis = true;
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
        bucket = q >= (float)(kDepthBuckets - 1) ? kDepthBuckets - 1 : (int)q;
      }
    }
    flags[c] = vis ? 1 : 0;
  }
  // this cell's work items go to its bucket's queue: places are reserved per
  // block in LDS, then with one global atomic per bucket
  __shared__ uint32_t s_n[kDepthBuckets], s_base[kDepthBuckets];
  if (threadIdx.x < kDepthBuckets) s_n[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t nch = vis ? (cnt + kSplatChunk - 1) / kSplatChunk : 0u;
  const uint32_t local = nch ? atomicAdd(&s_n[bucket], nch) : 0u;
  __syncthreads();
  if (threadIdx.x < kDepthBuckets && s_n[threadIdx.x])
    s_base[threadIdx.x] = atomicAdd(&counters[4 + threadIdx.x], s_n[threadIdx.x]);
  __syncthreads();
  if (nch) {
    const uint32_t pos = s_base[bucket] + local;
    for (uint32_t k = 0; k < nch; ++k) {
      const uint32_t off = k * kSplatChunk;
      chunks[(size_t)bucket * cap + pos + k] = make_uint2(start + off, min(kSplatChunk, cnt - off));
    }
  }
  uint32_t wave_chunks = nch;
  for (int off = 32; off > 0; off >>= 1) wave_chunks += __shfl_xor(wave_chunks, off, 64);
  const uint64_t vis_mask = __ballot(vis);
  uint32_t pts = vis ? cnt : 0u;
  for (int off = 32; off > 0; off >>= 1) pts += __shfl_xor(pts, off, 64);
  if (lane == 0 && wave_chunks) {
    atomicAdd(&counters[0], wave_chunks);
    atomicAdd(&counters[1], (uint32_t)__popcll(vis_mask));
    atomicAdd(reinterpret_cast<unsigned long long *>(&counters[2]), (unsigned long long)pts);
  }
}

// Work item `i` of the frame, walking the depth-bucket queues nearest first
// (counters[4 + b] items in bucket b); false past the last item.
__device__ inline bool work_item(uint32_t i, const uint32_t *__restrict__ counters, const uint2 *__restrict__ chunks,
                                 uint32_t cap, uint2 *ch) {
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
// the atomic can be skipped when the new key is not smaller.  COUNT adds the
// number of atomics issued to counters[kAtomicWord] (one add per wave), for
// measurement; the keys written are the same.
template <bool COUNT>
__global__ __launch_bounds__(kThreads) void splat_kernel(const float *__restrict__ xs, const float *__restrict__ ys,
                                                         const float *__restrict__ zs, const uint2 *__restrict__ chunks,
                                                         uint32_t cap, uint32_t *__restrict__ counters,
                                                         SplatCam cam, uint64_t *__restrict__ key) {
  uint2 ch;
  if (!work_item(blockIdx.x, counters, chunks, cap, &ch)) return;
  uint32_t issued = 0;
  const float *P = cam.P;
  // (keeping several points per thread in flight was measured slower: the
  // kernel is bound by the z-buffer atomics, not by load latency)
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
    const uint64_t k = ((uint64_t)__float_as_uint(w) << 32) | j;
    uint64_t *dst = key + (size_t)(uint32_t)v * cam.W + (uint32_t)u;
    // relaxed atomic read: other lanes lower the word concurrently
    if (k < __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      atomicMin(reinterpret_cast<unsigned long long *>(dst), (unsigned long long)k);
      if constexpr (COUNT) ++issued;
    }
  }
  if constexpr (COUNT) {
    for (int off = 32; off > 0; off >>= 1) issued += __shfl_xor(issued, off, 64);
    if ((threadIdx.x & 63) == 0 && issued) atomicAdd(&counters[kAtomicWord], issued);
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
__global__ __launch_bounds__(kThreads) void soft_accum_kernel(const float *__restrict__ xs, const float *__restrict__ ys,
                                                              const float *__restrict__ zs,
                                                              const uint32_t *__restrict__ rgbx,
                                                              const uint2 *__restrict__ chunks, uint32_t cap,
                                                              const uint32_t *__restrict__ counters, SplatCam cam,
                                                              const uint64_t *__restrict__ key, float one_plus_eps,
                                                              uint32_t *__restrict__ acc) {
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

hipError_t launch_clear(uint64_t *key, uint32_t npix, uint32_t *counters, hipStream_t s) {
  clear_kernel<<<grid_for(npix), kThreads, 0, s>>>(key, npix, counters);
  return hipGetLastError();
}

hipError_t launch_cull(const CloudDev &c, const CullParams &prm, uint8_t *flags, uint2 *chunks, uint32_t *counters,
                       hipStream_t s) {
  const uint32_t nb = (c.n_cells + kThreads - 1) / kThreads;
  cull_kernel<<<nb, kThreads, 0, s>>>(c.aabb, c.cell_start, c.n_cells, prm, flags, chunks, c.max_chunks, counters);
  return hipGetLastError();
}

hipError_t launch_splat(const CloudDev &c, const uint2 *chunks, uint32_t *counters, const SplatCam &cam,
                        uint64_t *key, bool count_atomics, hipStream_t s) {
  if (c.max_chunks == 0) return hipSuccess;
  if (count_atomics)
    splat_kernel<true><<<c.max_chunks, kThreads, 0, s>>>(c.x, c.y, c.z, chunks, c.max_chunks, counters, cam, key);
  else
    splat_kernel<false><<<c.max_chunks, kThreads, 0, s>>>(c.x, c.y, c.z, chunks, c.max_chunks, counters, cam, key);
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
                       const uint64_t *key, float one_plus_eps, uint32_t *acc, float *depth, uint32_t *rgba,
                       uint32_t npix, hipStream_t s) {
  clear_acc_kernel<<<grid_for(npix), kThreads, 0, s>>>(reinterpret_cast<uint4 *>(acc), npix);
  if (c.max_chunks)
    soft_accum_kernel<<<c.max_chunks, kThreads, 0, s>>>(c.x, c.y, c.z, c.rgbx, chunks, c.max_chunks, counters, cam,
                                                         key, one_plus_eps, acc);
  resolve_soft_kernel<<<grid_for(npix), kThreads, 0, s>>>(key, acc, depth, rgba, npix);
  return hipGetLastError();
}

}  // namespace lnr
