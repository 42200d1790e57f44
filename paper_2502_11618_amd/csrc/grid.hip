// Uniform-grid partition of a point cloud on the GPU (load time).
//
// Method, "Point Cloud Projection": a uniform grid is the only preprocessing;
// it lets each frame cull whole cells against the view frustum.  Here the grid
// is built on the device: bounding box -> cell id per point (float64 index
// formula) -> stable LSD radix sort of (cell id, input index) -> CSR cell
// offsets -> gathered SoA coordinates and packed colours -> tight per-cell
// bounding boxes.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "lnr_internal.h"

namespace lnr {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr uint32_t kTile = kThreads * kItems;  // 4096 elements per block

__device__ inline uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// ---------------------------------------------------------------------------
// bounding box and finiteness
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void bbox_kernel(const float *__restrict__ xyz, uint32_t n,
                                                        float *__restrict__ partial) {
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  float bad = 0.f;
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    for (int a = 0; a < 3; ++a) {
      const float v = xyz[3ull * i + a];
      if (!isfinite(v)) bad = 1.f;
      lo[a] = fminf(lo[a], v);
      hi[a] = fmaxf(hi[a], v);
    }
  }
  __shared__ float red[7][kThreads];
  for (int a = 0; a < 3; ++a) {
    red[a][threadIdx.x] = lo[a];
    red[3 + a][threadIdx.x] = hi[a];
  }
  red[6][threadIdx.x] = bad;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + s]);
        red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + s]);
      }
      red[6][threadIdx.x] = fmaxf(red[6][threadIdx.x], red[6][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 7) partial[blockIdx.x * 7 + threadIdx.x] = red[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// cell id: i_a = min(n_a - 1, floor((x_a - lo_a) / s)) in double; c = (iz*ny + iy)*nx + ix
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void cell_id_kernel(const float *__restrict__ xyz, uint32_t n, double lo0,
                                                           double lo1, double lo2, double s, int32_t nx, int32_t ny,
                                                           int32_t nz, uint32_t *__restrict__ cell) {
  const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const double rx = (double)xyz[3ull * i + 0] - lo0;
  const double ry = (double)xyz[3ull * i + 1] - lo1;
  const double rz = (double)xyz[3ull * i + 2] - lo2;
  const int64_t ix = min((int64_t)floor(rx / s), (int64_t)nx - 1);
  const int64_t iy = min((int64_t)floor(ry / s), (int64_t)ny - 1);
  const int64_t iz = min((int64_t)floor(rz / s), (int64_t)nz - 1);
  cell[i] = (uint32_t)((iz * ny + iy) * nx + ix);
}

__global__ void iota_kernel(uint32_t *v, uint32_t n) {
  const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i < n) v[i] = i;
}

// ---------------------------------------------------------------------------
// exclusive scan of uint32 (block reduce -> recursive scan of block sums -> downsweep)
// ---------------------------------------------------------------------------
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *total) {
  __shared__ uint32_t wsum[kThreads / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(x, off, 64);
    if (lane >= off) x += t;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int i = 0; i < kThreads / 64; ++i) {
    if (i < w) before += wsum[i];
    all += wsum[i];
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const uint32_t *__restrict__ in, uint32_t n,
                                                               uint32_t *__restrict__ sums) {
  const uint32_t base = blockIdx.x * kTile + threadIdx.x * kItems;
  uint32_t s = 0;
  for (int k = 0; k < kItems; ++k)
    if (base + k < n) s += in[base + k];
  uint32_t total;
  block_exclusive_scan(s, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void scan_down_kernel(const uint32_t *__restrict__ in, uint32_t n,
                                                             const uint32_t *__restrict__ block_off,
                                                             uint32_t *__restrict__ out) {
  const uint32_t base = blockIdx.x * kTile + threadIdx.x * kItems;
  uint32_t v[kItems];
  uint32_t s = 0;
  for (int k = 0; k < kItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(s, &total) + (block_off ? block_off[blockIdx.x] : 0u);
  for (int k = 0; k < kItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void radix_hist_kernel(const uint32_t *__restrict__ keys, uint32_t n, int shift,
                                                              uint32_t nb, uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kTile;
  for (int r = 0; r < kItems; ++r) {
    const uint32_t i = base + r * kThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Each block re-reads its tile in order (round r, thread t holds element r*256 + t)
// and places every element at (offset of its digit for this block) + (number of
// equal digits before it in the tile): the order of equal digits is preserved.
__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(const uint32_t *__restrict__ keys,
                                                                 const uint32_t *__restrict__ vals, uint32_t n,
                                                                 int shift, uint32_t nb,
                                                                 const uint32_t *__restrict__ offs,
                                                                 uint32_t *__restrict__ keys_out,
                                                                 uint32_t *__restrict__ vals_out) {
  __shared__ uint32_t s_off[256];
  __shared__ uint32_t s_wcnt[kThreads / 64][256];
  const int t = threadIdx.x, w = t >> 6;
  s_off[t] = offs[t * nb + blockIdx.x];
  for (int i = 0; i < kThreads / 64; ++i) s_wcnt[i][t] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kTile;
  const uint64_t lt = lanemask_lt();
  for (int r = 0; r < kItems; ++r) {
    const uint32_t i = base + r * kThreads + t;
    const bool valid = i < n;
    const uint32_t key = valid ? keys[i] : 0u;
    const uint32_t d = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      const uint64_t m = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? m : ~m;
    }
    const uint32_t rank = __popcll(peers & lt);
    if (valid && rank == 0) s_wcnt[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = s_off[d] + rank;
      for (int j = 0; j < w; ++j) pos += s_wcnt[j][d];
      keys_out[pos] = key;
      vals_out[pos] = vals[i];
    }
    __syncthreads();
    uint32_t add = 0;
    for (int j = 0; j < kThreads / 64; ++j) {
      add += s_wcnt[j][t];
      s_wcnt[j][t] = 0;
    }
    s_off[t] += add;
    __syncthreads();
  }
}

// cell_start[c] = first sorted position whose cell id is >= c
__global__ __launch_bounds__(kThreads) void cell_bounds_kernel(const uint32_t *__restrict__ sorted_cell, uint32_t n,
                                                               uint32_t n_cells, uint32_t *__restrict__ cell_start) {
  const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
  if (j > n) return;
  const int64_t prev = (j == 0) ? -1 : (int64_t)sorted_cell[j - 1];
  const int64_t cur = (j == n) ? (int64_t)n_cells : (int64_t)sorted_cell[j];
  for (int64_t c = prev + 1; c <= cur; ++c) cell_start[c] = j;
}

__global__ __launch_bounds__(kThreads) void gather_kernel(const float *__restrict__ xyz, const uint8_t *__restrict__ rgb,
                                                          const uint32_t *__restrict__ perm, uint32_t n,
                                                          float *__restrict__ x, float *__restrict__ y,
                                                          float *__restrict__ z, uint32_t *__restrict__ rgbx) {
  const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
  if (j >= n) return;
  const uint64_t p = perm[j];
  x[j] = xyz[3 * p + 0];
  y[j] = xyz[3 * p + 1];
  z[j] = xyz[3 * p + 2];
  rgbx[j] = (uint32_t)rgb[3 * p] | ((uint32_t)rgb[3 * p + 1] << 8) | ((uint32_t)rgb[3 * p + 2] << 16);
}

// one wave per cell: exact float min / max of its points
__global__ __launch_bounds__(kThreads) void cell_aabb_kernel(const float *__restrict__ x, const float *__restrict__ y,
                                                             const float *__restrict__ z,
                                                             const uint32_t *__restrict__ cell_start,
                                                             uint32_t n_cells, float *__restrict__ aabb) {
  const uint32_t c = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= n_cells) return;
  const uint32_t a = cell_start[c], b = cell_start[c + 1];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (uint32_t j = a + lane; j < b; j += 64) {
    const float v[3] = {x[j], y[j], z[j]};
    for (int k = 0; k < 3; ++k) {
      lo[k] = fminf(lo[k], v[k]);
      hi[k] = fmaxf(hi[k], v[k]);
    }
  }
  for (int off = 32; off > 0; off >>= 1)
    for (int k = 0; k < 3; ++k) {
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], off, 64));
      hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off, 64));
    }
  if (lane < 6) aabb[6ull * c + lane] = lane < 3 ? lo[lane] : hi[lane - 3];
}

__global__ __launch_bounds__(kThreads) void chunk_count_kernel(const uint32_t *__restrict__ cell_start,
                                                               uint32_t n_cells, uint32_t *__restrict__ total) {
  const uint32_t c = blockIdx.x * kThreads + threadIdx.x;
  uint32_t v = 0;
  if (c < n_cells) v = (cell_start[c + 1] - cell_start[c] + kSplatChunk - 1) / kSplatChunk;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(total, v);
}

inline uint32_t div_up(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

}  // namespace

uint32_t bbox_blocks(uint32_t n) {
  uint32_t nb = div_up(n, kThreads * 8);
  return nb < 1 ? 1 : (nb > 2048 ? 2048 : nb);
}

hipError_t launch_bbox(const float *xyz, uint32_t n, float *partial, uint32_t nb, hipStream_t s) {
  bbox_kernel<<<nb, kThreads, 0, s>>>(xyz, n, partial);
  return hipGetLastError();
}

hipError_t launch_cell_ids(const float *xyz, uint32_t n, const double lo[3], double s, const int32_t dims[3],
                           uint32_t *cell, hipStream_t st) {
  cell_id_kernel<<<div_up(n, kThreads), kThreads, 0, st>>>(xyz, n, lo[0], lo[1], lo[2], s, dims[0], dims[1], dims[2],
                                                            cell);
  return hipGetLastError();
}

hipError_t launch_iota(uint32_t *v, uint32_t n, hipStream_t s) {
  iota_kernel<<<div_up(n, kThreads), kThreads, 0, s>>>(v, n);
  return hipGetLastError();
}

size_t scan_scratch_bytes(uint32_t n) {
  size_t bytes = 0;
  uint64_t m = n;
  while (m > kTile) {
    m = div_up(m, kTile);
    bytes += 2 * ((m * 4 + 255) / 256 * 256);
  }
  return bytes + 256;
}

hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, uint32_t n, void *scratch, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t nb = div_up(n, kTile);
  if (nb == 1) {
    scan_down_kernel<<<1, kThreads, 0, s>>>(in, n, nullptr, out);
    return hipGetLastError();
  }
  uint32_t *sums = static_cast<uint32_t *>(scratch);
  const size_t chunk = ((uint64_t)nb * 4 + 255) / 256 * 256;
  uint32_t *sums_scan = reinterpret_cast<uint32_t *>(static_cast<char *>(scratch) + chunk);
  void *next = static_cast<char *>(scratch) + 2 * chunk;
  scan_reduce_kernel<<<nb, kThreads, 0, s>>>(in, n, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = exclusive_scan_u32(sums, sums_scan, nb, next, s);
  if (e != hipSuccess) return e;
  scan_down_kernel<<<nb, kThreads, 0, s>>>(in, n, sums_scan, out);
  return hipGetLastError();
}

size_t radix_sort_scratch_bytes(uint32_t n) {
  const uint64_t nb = div_up(n, kTile);
  const uint64_t h = 256 * nb;
  return 2 * ((h * 4 + 255) / 256 * 256) + scan_scratch_bytes((uint32_t)h);
}

hipError_t radix_sort_pairs(uint32_t **keys, uint32_t **vals, uint32_t **keys_alt, uint32_t **vals_alt, uint32_t n,
                            int bits, void *scratch, hipStream_t s) {
  const uint32_t nb = div_up(n, kTile);
  const uint64_t h = 256ull * nb;
  const size_t hb = (h * 4 + 255) / 256 * 256;
  uint32_t *hist = static_cast<uint32_t *>(scratch);
  uint32_t *offs = reinterpret_cast<uint32_t *>(static_cast<char *>(scratch) + hb);
  void *scan_scratch = static_cast<char *>(scratch) + 2 * hb;
  for (int shift = 0; shift < bits; shift += 8) {
    radix_hist_kernel<<<nb, kThreads, 0, s>>>(*keys, n, shift, nb, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = exclusive_scan_u32(hist, offs, (uint32_t)h, scan_scratch, s);
    if (e != hipSuccess) return e;
    radix_scatter_kernel<<<nb, kThreads, 0, s>>>(*keys, *vals, n, shift, nb, offs, *keys_alt, *vals_alt);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t *t = *keys;
    *keys = *keys_alt;
    *keys_alt = t;
    t = *vals;
    *vals = *vals_alt;
    *vals_alt = t;
  }
  return hipSuccess;
}

hipError_t launch_cell_bounds(const uint32_t *sorted_cell, uint32_t n, uint32_t n_cells, uint32_t *cell_start,
                              hipStream_t s) {
  cell_bounds_kernel<<<div_up((uint64_t)n + 1, kThreads), kThreads, 0, s>>>(sorted_cell, n, n_cells, cell_start);
  return hipGetLastError();
}

hipError_t launch_gather_points(const float *xyz, const uint8_t *rgb, const uint32_t *perm, uint32_t n, float *x,
                                float *y, float *z, uint32_t *rgbx, hipStream_t s) {
  gather_kernel<<<div_up(n, kThreads), kThreads, 0, s>>>(xyz, rgb, perm, n, x, y, z, rgbx);
  return hipGetLastError();
}

hipError_t launch_cell_aabb(const float *x, const float *y, const float *z, const uint32_t *cell_start,
                            uint32_t n_cells, float *aabb, hipStream_t s) {
  cell_aabb_kernel<<<div_up(n_cells, kThreads / 64), kThreads, 0, s>>>(x, y, z, cell_start, n_cells, aabb);
  return hipGetLastError();
}

hipError_t launch_chunk_count(const uint32_t *cell_start, uint32_t n_cells, uint32_t *total, hipStream_t s) {
  chunk_count_kernel<<<div_up(n_cells, kThreads), kThreads, 0, s>>>(cell_start, n_cells, total);
  return hipGetLastError();
}

}  // namespace lnr
