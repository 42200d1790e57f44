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

// One thread per coarse pixel p of level k+1 handles its 2x2 children at level k.
template <bool FINAL>
__global__ __launch_bounds__(256) void upsample_kernel(const float *__restrict__ Dk, int Hk, int Wk,
                                                       const float *__restrict__ Dc, const float *__restrict__ Uc,
                                                       int Hc, int Wc, float *__restrict__ Uk,
                                                       float *__restrict__ depth, uint32_t *__restrict__ rgba, float fs,
                                                       float one_plus_fs) {
  const int px = blockIdx.x * 16 + (threadIdx.x & 15);
  const int py = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (px >= Wc || py >= Hc) return;
  const int ym = max(py - 1, 0), yp = min(py + 1, Hc - 1);
  const int xm = max(px - 1, 0), xp = min(px + 1, Wc - 1);
  // edge test on the min-pooled coarse level
  const float c = Dc[(size_t)py * Wc + px];
  const float up = Dc[(size_t)ym * Wc + px], down = Dc[(size_t)yp * Wc + px];
  const float left = Dc[(size_t)py * Wc + xm], right = Dc[(size_t)py * Wc + xp];
  bool edge = isinf(c) || isinf(up) || isinf(down) || isinf(left) || isinf(right);
  if (!edge) {
    const float lap = (((up + down) + left) + right) - 4.0f * c;
    edge = fabsf(lap) > fs * c;
  }
  // upsampled coarse level, clamped 3x3 around p (clamped taps repeat in-bounds
  // ones, so their maximum is the maximum over the in-bounds neighbourhood)
  const int rows[3] = {ym, py, yp}, cols[3] = {xm, px, xp};
  float u[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) u[i][j] = Uc[(size_t)rows[i] * Wc + cols[j]];
  float ref = u[1][1];
  if (edge) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) ref = fmaxf(ref, u[i][j]);
  }
  const float thr = ref * one_plus_fs;
#pragma unroll
  for (int cy = 0; cy < 2; ++cy) {
    const int y = 2 * py + cy;
    if (y >= Hk) continue;
#pragma unroll
    for (int cx = 0; cx < 2; ++cx) {
      const int x = 2 * px + cx;
      if (x >= Wk) continue;
      const size_t i = (size_t)y * Wk + x;
      if (FINAL) {
        const uint32_t q = rgba[i];
        const float d = (q >> 24) ? depth[i] : INFINITY;
        const bool keep = !isinf(d) && d <= thr;
        if (!keep && (q >> 24)) {
          depth[i] = 0.f;
          rgba[i] = 0u;
        }
      } else {
        const float d = Dk[i];
        const bool keep = !isinf(d) && d <= thr;
        float val = d;
        if (!keep) {
          const float U00 = u[1][1], U01 = u[1][cx ? 2 : 0], U10 = u[cy ? 2 : 0][1], U11 = u[cy ? 2 : 0][cx ? 2 : 0];
          val = 0.75f * (0.75f * U00 + 0.25f * U01) + 0.25f * (0.75f * U10 + 0.25f * U11);
        }
        Uk[i] = val;
      }
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

hipError_t launch_upsample(int k, int n, const float *const *D, float *const *U, const int *Hs, const int *Ws,
                           float *depth, uint32_t *rgba, float fs, float one_plus_fs, hipStream_t s) {
  // coarse level k+1: D[k+1] min-pooled, U[k+1] upsampled (U[n] == D[n])
  const int Hc = Hs[k + 1], Wc = Ws[k + 1];
  dim3 grid((Wc + 15) / 16, (Hc + 15) / 16);
  const float *Uc = (k + 1 == n) ? D[n] : U[k + 1];
  if (k == 0)
    upsample_kernel<true><<<grid, 256, 0, s>>>(nullptr, Hs[0], Ws[0], D[1], Uc, Hc, Wc, nullptr, depth, rgba, fs,
                                               one_plus_fs);
  else
    upsample_kernel<false><<<grid, 256, 0, s>>>(D[k], Hs[k], Ws[k], D[k + 1], Uc, Hc, Wc, U[k], nullptr, nullptr, fs,
                                                one_plus_fs);
  return hipGetLastError();
}

}  // namespace lnr
