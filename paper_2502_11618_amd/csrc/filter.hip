// Hierarchical min-pool depth filter.
//
// Method, "Depth filtering", and Fig. 2: min-pool the depth image (2x2,
// stride 2) n times, then upsample back level by level.  At each step a
// Laplacian on the coarser min-pooled level marks edge pixels; the four
// children of each coarse pixel are kept if their depth is within
// filter_strength of the parent's upsampled depth (at edges: of the largest
// depth in the parent's 3x3 neighbourhood); rejected children of non-final
// levels are refilled by bilinear interpolation from the coarser level.
//
// Readings fixed here (the paper defers details to unavailable supplementary
// material): empty = +inf; ceil sizes for odd levels; clamped 4-neighbour
// Laplacian, an empty tap or |lap| > fs * D marks an edge; keep iff
// d <= ref * (1 + fs); half-pixel-centre bilinear weights 0.75 / 0.25.
// All arithmetic is float32 in the written order, no fused multiply-add.
#include <hip/hip_runtime.h>

#include "lnr_internal.h"

#pragma clang fp contract(off)

namespace lnr {
namespace {

__device__ inline float d0_at(const float *__restrict__ depth, const uint32_t *__restrict__ rgba, size_t i) {
  return (rgba[i] >> 24) ? depth[i] : INFINITY;
}

// One block turns a 32x32 tile of level k0 into up to 5 coarser levels.
// Level k0 = 0 is read from the RGBDA image (empty -> +inf).  Pixels of a level
// that fall outside the image evaluate to +inf, as the children outside the
// image do in the definition.
template <bool FROM_IMAGE>
__global__ __launch_bounds__(256) void pyramid_kernel(const float *__restrict__ src, const float *__restrict__ depth,
                                                      const uint32_t *__restrict__ rgba, int sH, int sW, int nl,
                                                      float *o1, float *o2, float *o3, float *o4, float *o5) {
  __shared__ float t[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  int H = (sH + 1) >> 1, W = (sW + 1) >> 1;
  int X = blockIdx.x * 16 + tx, Y = blockIdx.y * 16 + ty;
  float m = INFINITY;
#pragma unroll
  for (int dy = 0; dy < 2; ++dy)
#pragma unroll
    for (int dx = 0; dx < 2; ++dx) {
      const int sy = 2 * Y + dy, sx = 2 * X + dx;
      if (sy < sH && sx < sW) {
        const size_t i = (size_t)sy * sW + sx;
        m = fminf(m, FROM_IMAGE ? d0_at(depth, rgba, i) : src[i]);
      }
    }
  if (Y < H && X < W) o1[(size_t)Y * W + X] = m;
  t[ty][tx] = m;
  float *outs[4] = {o2, o3, o4, o5};
  int side = 16;
  for (int l = 1; l < nl; ++l) {
    __syncthreads();
    side >>= 1;
    const int pH = H, pW = W;
    H = (pH + 1) >> 1;
    W = (pW + 1) >> 1;
    float v = INFINITY;
    if (ty < side && tx < side) {
      v = fminf(fminf(t[2 * ty][2 * tx], t[2 * ty][2 * tx + 1]), fminf(t[2 * ty + 1][2 * tx], t[2 * ty + 1][2 * tx + 1]));
      X = blockIdx.x * side + tx;
      Y = blockIdx.y * side + ty;
      if (Y < H && X < W) outs[l - 1][(size_t)Y * W + X] = v;
    }
    __syncthreads();
    if (ty < side && tx < side) t[ty][tx] = v;
  }
}

// Edge-aware upsampling of every level in one launch.  A workgroup owns a
// kTile x kTile tile of level 0.  Level 0 needs the upsampled level 1 at the
// tile's parents and their neighbours (3x3 reference, bilinear taps); that
// region of level 1 needs a slightly larger region of level 2, and so on up to
// level n (U_n = D_n).  The workgroup loads the min-pooled levels over this
// chain of small regions into LDS in one go (one memory latency, not one per
// level), holds its level-0 pixels in registers, and recomputes the upsampled
// regions coarsest first in LDS, so no upsampled level is written to HBM and
// one launch replaces one per level.  Neighbouring tiles recompute the same
// coarse pixels with the same arithmetic, so every copy holds the same value.
// 1024 threads (4 level-0 pixels each): a 1080p image gives about two such
// workgroups per CU, and 16 waves each keep more loads in flight than 4
// (the upsample ran in 19.4 instead of 24.6 us with 256 threads).
constexpr int kTile = 64;
constexpr int kTileThreads = 1024;
constexpr int kPxPerThread = kTile * kTile / kTileThreads;
// Largest region side per level: a 64-pixel tile needs at most 34 pixels of
// level 1, 20 of level 2, 12, 8, and then at most 6 (a side L gives at most
// ceil((L + 1) / 2) + 2 at the next level).  Level k's region is stored with
// row stride kSide[k] at offset kOff[k] of each LDS pool.
constexpr int kMaxLevels = 15;
__constant__ const int kSide[kMaxLevels + 1] = {64, 34, 20, 12, 8, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6, 6};
constexpr int kPool = 34 * 34 + 20 * 20 + 12 * 12 + 8 * 8 + 11 * 6 * 6;

struct Region {
  int r0, r1, c0, c1;  // rows [r0, r1), columns [c0, c1) of one level, inside the image
};

__device__ inline Region parent_region(const Region &c, int Hp, int Wp) {
  // parents of c, widened by one pixel (3x3 reference and bilinear taps), clamped
  return {max(0, (c.r0 >> 1) - 1), min(Hp, ((c.r1 - 1) >> 1) + 2), max(0, (c.c0 >> 1) - 1),
          min(Wp, ((c.c1 - 1) >> 1) + 2)};
}

// Threshold depth of the children of coarse pixel (py, px): the Laplacian edge
// test on the min-pooled coarse level Dc, then the reference depth from the
// upsampled coarse level Uc (the centre, or at edges the maximum over the
// clamped 3x3), times (1 + fs).  Dc and Uc hold region R of the coarse level
// with row stride st.
__device__ inline float child_threshold(const float *Dc, const float *Uc, int st, const Region &R, int Hc, int Wc,
                                        int py, int px, float fs, float one_plus_fs) {
  const int ym = max(py - 1, 0), yp = min(py + 1, Hc - 1);
  const int xm = max(px - 1, 0), xp = min(px + 1, Wc - 1);
  const int r[3] = {(ym - R.r0) * st, (py - R.r0) * st, (yp - R.r0) * st};
  const int c[3] = {xm - R.c0, px - R.c0, xp - R.c0};
  const float ctr = Dc[r[1] + c[1]];
  const float up = Dc[r[0] + c[1]], down = Dc[r[2] + c[1]];
  const float left = Dc[r[1] + c[0]], right = Dc[r[1] + c[2]];
  bool edge = isinf(ctr) || isinf(up) || isinf(down) || isinf(left) || isinf(right);
  if (!edge) {
    const float lap = (((up + down) + left) + right) - 4.0f * ctr;
    edge = fabsf(lap) > fs * ctr;
  }
  // clamped taps repeat in-bounds ones, so their maximum is the maximum over
  // the in-bounds neighbourhood
  float ref = Uc[r[1] + c[1]];
  if (edge) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) ref = fmaxf(ref, Uc[r[i] + c[j]]);
  }
  return ref * one_plus_fs;
}

struct LevelPtrs {
  const float *D[kMaxLevels + 1];  // D[k], k = 1..n: min-pooled levels
  int H[kMaxLevels + 1], W[kMaxLevels + 1];  // sizes, level 0 included
};

__global__ __launch_bounds__(kTileThreads) void upsample_fused_kernel(LevelPtrs lv, int n, float *__restrict__ depth,
                                                                      uint32_t *__restrict__ rgba, float fs,
                                                                      float one_plus_fs) {
  __shared__ float sD[kPool], sU[kPool];
  // the chain of regions and their LDS offsets (in LDS: a private array
  // indexed by the level would live in scratch memory)
  __shared__ Region R[kMaxLevels + 1];
  __shared__ int off[kMaxLevels + 1];
  const int t = threadIdx.x;
  if (t == 0) {
    Region r = {(int)blockIdx.y * kTile, min(lv.H[0], (int)blockIdx.y * kTile + kTile), (int)blockIdx.x * kTile,
                min(lv.W[0], (int)blockIdx.x * kTile + kTile)};
    R[0] = r;
    int o = 0;
    for (int k = 1; k <= n; ++k) {
      r = parent_region(r, lv.H[k], lv.W[k]);
      R[k] = r;
      off[k] = o;
      o += kSide[k] * kSide[k];
    }
  }
  __syncthreads();
  // level-0 pixels of the tile into registers (their loads overlap the rest)
  const int rw0 = R[0].c1 - R[0].c0, cnt0 = (R[0].r1 - R[0].r0) * rw0;
  uint32_t q0[kPxPerThread];
  float d0[kPxPerThread];
#pragma unroll
  for (int m = 0; m < kPxPerThread; ++m) {
    const int i = t + m * kTileThreads;
    q0[m] = 0u;
    d0[m] = 0.f;
    if (i < cnt0) {
      const int y = i / rw0, x = i - y * rw0;
      const size_t p = (size_t)(R[0].r0 + y) * lv.W[0] + R[0].c0 + x;
      q0[m] = rgba[p];
      d0[m] = depth[p];
    }
  }
  // the min-pooled levels over their regions, all at once
  for (int k = 1; k <= n; ++k) {
    const Region &g = R[k];
    const int rw = g.c1 - g.c0, cnt = (g.r1 - g.r0) * rw, st = kSide[k];
    for (int i = t; i < cnt; i += kTileThreads) {
      const int y = i / rw, x = i - y * rw;
      sD[off[k] + y * st + x] = lv.D[k][(size_t)(g.r0 + y) * lv.W[k] + g.c0 + x];
    }
  }
  __syncthreads();
  // levels n-1 .. 1: U_k over R[k] from U_{k+1} over R[k+1] (U_n = D_n)
  for (int k = n - 1; k >= 1; --k) {
    const Region &g = R[k], &gc = R[k + 1];
    const int rw = g.c1 - g.c0, cnt = (g.r1 - g.r0) * rw, st = kSide[k], stc = kSide[k + 1];
    const float *Dc = sD + off[k + 1];
    const float *Uc = (k + 1 == n ? sD : sU) + off[k + 1];
    const float *Dk = sD + off[k];
    float *Uk = sU + off[k];
    for (int i = t; i < cnt; i += kTileThreads) {
      const int y = i / rw, x = i - y * rw;
      const int gy = g.r0 + y, gx = g.c0 + x;
      const int py = gy >> 1, px = gx >> 1;
      const float thr = child_threshold(Dc, Uc, stc, gc, lv.H[k + 1], lv.W[k + 1], py, px, fs, one_plus_fs);
      const float d = Dk[y * st + x];
      float val = d;
      if (!(!isinf(d) && d <= thr)) {
        // bilinear with half-pixel centres: the parent, and its neighbour on
        // the child's side in each direction (clamped at the border)
        const int y1 = (gy & 1) ? min(py + 1, lv.H[k + 1] - 1) : max(py - 1, 0);
        const int x1 = (gx & 1) ? min(px + 1, lv.W[k + 1] - 1) : max(px - 1, 0);
        const int ry0 = (py - gc.r0) * stc, ry1 = (y1 - gc.r0) * stc, rx0 = px - gc.c0, rx1 = x1 - gc.c0;
        const float U00 = Uc[ry0 + rx0], U01 = Uc[ry0 + rx1];
        const float U10 = Uc[ry1 + rx0], U11 = Uc[ry1 + rx1];
        val = 0.75f * (0.75f * U00 + 0.25f * U01) + 0.25f * (0.75f * U10 + 0.25f * U11);
      }
      Uk[y * st + x] = val;
    }
    __syncthreads();
  }
  // level 0: keep or remove each pixel of the tile
  const Region &gc = R[1];
  const float *D1 = sD + off[1];
  const float *U1 = (n == 1 ? sD : sU) + off[1];
#pragma unroll
  for (int m = 0; m < kPxPerThread; ++m) {
    const int i = t + m * kTileThreads;
    if (i >= cnt0 || !(q0[m] >> 24)) continue;  // empty pixels stay empty
    const int y = i / rw0, x = i - y * rw0;
    const int gy = R[0].r0 + y, gx = R[0].c0 + x;
    const float thr = child_threshold(D1, U1, kSide[1], gc, lv.H[1], lv.W[1], gy >> 1, gx >> 1, fs, one_plus_fs);
    if (!(!isinf(d0[m]) && d0[m] <= thr)) {
      const size_t p = (size_t)gy * lv.W[0] + gx;
      depth[p] = 0.f;
      rgba[p] = 0u;
    }
  }
}

}  // namespace

hipError_t launch_pyramid(const float *depth, const uint32_t *rgba, int H, int W, int n, float *const *levels,
                          hipStream_t s) {
  // levels[k] for k = 1..n are the min-pooled images; levels[0] is unused
  int sH = H, sW = W, k0 = 0;
  while (k0 < n) {
    const int nl = (n - k0) < 5 ? (n - k0) : 5;
    const int H1 = (sH + 1) >> 1, W1 = (sW + 1) >> 1;
    dim3 grid((W1 + 15) / 16, (H1 + 15) / 16);
    float *o[5];
    for (int l = 0; l < 5; ++l) o[l] = (l < nl) ? levels[k0 + 1 + l] : nullptr;
    if (k0 == 0)
      pyramid_kernel<true><<<grid, 256, 0, s>>>(nullptr, depth, rgba, sH, sW, nl, o[0], o[1], o[2], o[3], o[4]);
    else
      pyramid_kernel<false><<<grid, 256, 0, s>>>(levels[k0], nullptr, nullptr, sH, sW, nl, o[0], o[1], o[2], o[3],
                                                 o[4]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int l = 0; l < nl; ++l) {
      sH = (sH + 1) >> 1;
      sW = (sW + 1) >> 1;
    }
    k0 += nl;
  }
  return hipSuccess;
}

hipError_t launch_upsample_fused(int n, const float *const *D, const int *Hs, const int *Ws, float *depth,
                                 uint32_t *rgba, float fs, float one_plus_fs, hipStream_t s) {
  if (n < 1 || n > kMaxLevels) return hipErrorInvalidValue;
  LevelPtrs lv{};
  for (int k = 0; k <= n; ++k) {
    lv.D[k] = k ? D[k] : nullptr;
    lv.H[k] = Hs[k];
    lv.W[k] = Ws[k];
  }
  dim3 grid((Ws[0] + kTile - 1) / kTile, (Hs[0] + kTile - 1) / kTile);
  upsample_fused_kernel<<<grid, kTileThreads, 0, s>>>(lv, n, depth, rgba, fs, one_plus_fs);
  return hipGetLastError();
}

// Scratch of the allocation-free filter entry point: the min-pooled levels
// D_1..D_n of one image, each level starting on a 256-byte boundary.  The
// array exists once per device for the lifetime of the process.  Host code
// must not pass `scratch` itself to a kernel (on the host it names a stand-in,
// not device memory): it takes the device address from
// noalloc_scratch_address() once per device and uses that.
static __device__ __align__(256) float scratch[kNoAllocScratchFloats];

hipError_t noalloc_scratch_address(float **ptr) {
  *ptr = nullptr;
  return hipGetSymbolAddress(reinterpret_cast<void **>(ptr), HIP_SYMBOL(scratch));
}

}  // namespace lnr
