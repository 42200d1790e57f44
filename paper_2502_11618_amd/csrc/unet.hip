// U-Net forward pass on the gfx950 matrix cores.
//
// Fig. 1 and Method, "U-Net Reconstruction": a fully convolutional U-Net maps
// the depth-filtered RGBDA image to RGB.  Each 3x3 convolution is an implicit
// GEMM (M = output channels, N = output pixels, K = 9 taps x input channels):
// a workgroup stages an input tile with a one-pixel halo in LDS and runs the
// K loop on 32x32 MFMA blocks.  The decoder's nearest-neighbour upsample and
// channel concatenation are folded into the tile load (channels past the skip
// tensor are read from the coarser tensor at (y/2, x/2)), and the encoder's
// 2x2 max-pool is folded into the epilogue of the convolution that feeds it.
//
// Arithmetic modes:
//   F32    float32 activations, v_mfma_f32_32x32x2_f32.
//   BF16   bfloat16 activations and weights, v_mfma_f32_32x32x16_bf16,
//          float32 accumulation, round-to-nearest-even to bfloat16 on store.
//   BF16X3 float32 activations; operands split into bfloat16 hi + lo in LDS,
//          hi*hi + hi*lo + lo*hi on the bf16 MFMA with float32 accumulation.
#include <hip/hip_runtime.h>

#include "lnr_internal.h"

namespace lnr {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kTH = 8;    // output tile rows (4 waves x 2 rows)
// output tile columns = 16 x NB: each wave owns NB blocks of 2 rows x 16 pixels

__device__ inline uint16_t f2bf(float f) {  // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

struct ConvArgs {
  const void *in0;
  const void *in1;
  int C0, C1, H, W;
  const void *w;
  const void *w_lo;
  const float *bias;
  int cout, cin_pad;
  void *out;
  void *out_pool;
  const float *head_w;
  const float *head_b;
  float *head_out;
  // batch of same-shape images: blockIdx.z = image * (cout_pad / BM) + channel tile;
  // per-image element strides of the tensors above; head_outs (device array) gives
  // each image's planar head output when set
  int batch;
  size_t in0_bs, in1_bs, out_bs, pool_bs;
  float *const *head_outs;
};

// LDS layout: per tile pixel, CK channels plus padding that staggers pixels
// across banks (16-byte lane reads).
template <int MODE, int CK>
struct Lds {
  static constexpr int kStride = (MODE == 0) ? (CK + 4) : (CK + 8);  // elements per pixel
  using T = typename std::conditional<MODE == 0, float, uint16_t>::type;
  static constexpr int kArrays = (MODE == 2) ? 2 : 1;
};

template <int MODE, int BM, int CK, int NB>
__global__ __launch_bounds__(256) void conv3x3_kernel(ConvArgs a) {
  using L = Lds<MODE, CK>;
  using T = typename L::T;
  constexpr int S = L::kStride;
  constexpr int MB = BM / 32;
  constexpr int kTW = 16 * NB;
  constexpr int kLW = kTW + 2, kLPix = (kTH + 2) * kLW;
  __shared__ __attribute__((aligned(16))) T s_in[L::kArrays][kLPix * S];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = lane & 31, h = lane >> 5;
  const int ty0 = blockIdx.y * kTH, tx0 = blockIdx.x * kTW;
  const int nzc = gridDim.z / a.batch;
  const int bimg = blockIdx.z / nzc;
  const int co0 = (blockIdx.z - bimg * nzc) * BM;
  const int H = a.H, W = a.W;
  const int Cin = a.C0 + a.C1;
  // this image's tensors (element type in HBM: bf16 bits for BF16, float otherwise)
  using E = typename std::conditional<MODE == 1, uint16_t, float>::type;
  const E *in0 = static_cast<const E *>(a.in0) + (size_t)bimg * a.in0_bs;
  const E *in1 = a.in1 ? static_cast<const E *>(a.in1) + (size_t)bimg * a.in1_bs : nullptr;
  E *out = a.out ? static_cast<E *>(a.out) + (size_t)bimg * a.out_bs : nullptr;
  E *out_pool = a.out_pool ? static_cast<E *>(a.out_pool) + (size_t)bimg * a.pool_bs : nullptr;
  float *head_out = a.head_outs ? a.head_outs[bimg] : (a.head_out ? a.head_out + (size_t)bimg * 3 * H * W : nullptr);

  floatx16 acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mb][nb][r] = 0.f;

  // pixel of this lane in each N block (2 rows x 16 columns), tile coordinates
  const int pr = 2 * wv + (n >> 4);
  const int pc = n & 15;

  for (int ci = 0; ci < Cin; ci += CK) {
    // ---- stage the input tile (with halo) for channels [ci, ci + CK) ----
    const bool from0 = ci < a.C0;
    const int csrc = from0 ? a.C0 : a.C1;
    const int coff = from0 ? ci : ci - a.C0;
    constexpr int VEC = (MODE == 1) ? 8 : 4;  // channels per 16-byte global load
    constexpr int NV = CK / VEC;
    for (int e = tid; e < kLPix * NV; e += 256) {
      const int pix = e / NV, q = e - pix * NV;
      const int gy = ty0 - 1 + pix / kLW, gx = tx0 - 1 + pix % kLW;
      const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
      size_t gi = 0;
      if (inside) {
        gi = from0 ? ((size_t)gy * W + gx) * csrc + coff + q * VEC
                   : ((size_t)(gy >> 1) * (W >> 1) + (gx >> 1)) * csrc + coff + q * VEC;
      }
      const void *src = from0 ? (const void *)in0 : (const void *)in1;
      if (MODE == 0) {
        float4 v = inside ? *reinterpret_cast<const float4 *>(static_cast<const float *>(src) + gi)
                          : make_float4(0.f, 0.f, 0.f, 0.f);
        *reinterpret_cast<float4 *>(&s_in[0][pix * S + q * 4]) = v;
      } else if (MODE == 1) {
        uint4 v = inside ? *reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(src) + gi)
                         : make_uint4(0u, 0u, 0u, 0u);
        *reinterpret_cast<uint4 *>(&s_in[0][pix * S + q * 8]) = v;
      } else {
        float4 v = inside ? *reinterpret_cast<const float4 *>(static_cast<const float *>(src) + gi)
                          : make_float4(0.f, 0.f, 0.f, 0.f);
        const float f[4] = {v.x, v.y, v.z, v.w};
        uint16_t hi[4], lo[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          hi[i] = f2bf(f[i]);
          lo[i] = f2bf(f[i] - bf2f(hi[i]));
        }
        *reinterpret_cast<uint2 *>(&s_in[0][pix * S + q * 4]) =
            make_uint2(hi[0] | ((uint32_t)hi[1] << 16), hi[2] | ((uint32_t)hi[3] << 16));
        *reinterpret_cast<uint2 *>(&s_in[MODE == 2 ? 1 : 0][pix * S + q * 4]) =
            make_uint2(lo[0] | ((uint32_t)lo[1] << 16), lo[2] | ((uint32_t)lo[3] << 16));
      }
    }
    __syncthreads();

    // ---- K loop over the 9 taps and the staged channels ----
    if (MODE == 0) {
      // float32: steps it = (tap, 8-channel group); the operands of step it + 1
      // are loaded (weights from global/L1, activations from LDS) while the
      // MFMAs of step it run
      constexpr int G = CK / 8;
      constexpr int NIT = 9 * G;
      const float *wp = static_cast<const float *>(a.w);
      const float *sp = reinterpret_cast<const float *>(&s_in[0][0]);
      const float *wrow[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) wrow[mb] = wp + (size_t)(co0 + mb * 32 + n) * 9 * a.cin_pad + ci + 4 * h;
      auto load = [&](int it, float4 *av, float4 *bv) {
        const int tap = it / G, g = it - tap * G;
        const int dy = tap / 3, dx = tap - 3 * dy;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
          av[mb] = *reinterpret_cast<const float4 *>(wrow[mb] + tap * a.cin_pad + g * 8);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          bv[nb] = *reinterpret_cast<const float4 *>(sp + ((pr + dy) * kLW + (nb * 16 + pc + dx)) * S + g * 8 + 4 * h);
      };
      auto mma = [&](const float4 *av, const float4 *bv) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[mb][i], bv[nb][i], acc[mb][nb], 0, 0, 0);
      };
      float4 a0[MB], b0[NB], a1[MB], b1[NB];
      load(0, a0, b0);
#pragma unroll 1
      for (int it = 0; it < NIT; it += 2) {
        if (it + 1 < NIT) load(it + 1, a1, b1);
        mma(a0, b0);
        if (it + 1 < NIT) {
          if (it + 2 < NIT) load(it + 2, a0, b0);
          mma(a1, b1);
        }
      }
    } else {
#pragma unroll 1
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap - 3 * (tap / 3);
      int boff[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) boff[nb] = ((pr + dy) * kLW + (nb * 16 + pc + dx)) * S;
      {
        const uint16_t *wp = static_cast<const uint16_t *>(a.w);
        const uint16_t *wl = static_cast<const uint16_t *>(a.w_lo);
#pragma unroll
        for (int g = 0; g < CK / 16; ++g) {
          uint4 ah[MB], al[MB], bh[NB], bl[NB];
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
            const size_t wi = ((size_t)(co0 + mb * 32 + n) * 9 + tap) * a.cin_pad + ci + g * 16 + 8 * h;
            ah[mb] = *reinterpret_cast<const uint4 *>(wp + wi);
            if (MODE == 2) al[mb] = *reinterpret_cast<const uint4 *>(wl + wi);
          }
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            bh[nb] = *reinterpret_cast<const uint4 *>(&s_in[0][boff[nb] + g * 16 + 8 * h]);
            if (MODE == 2) bl[nb] = *reinterpret_cast<const uint4 *>(&s_in[MODE == 2 ? 1 : 0][boff[nb] + g * 16 + 8 * h]);
          }
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
              if (MODE == 2) {
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(al[mb]), as_bf16x8(bh[nb]),
                                                                      acc[mb][nb], 0, 0, 0);
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(ah[mb]), as_bf16x8(bl[nb]),
                                                                      acc[mb][nb], 0, 0, 0);
              }
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(ah[mb]), as_bf16x8(bh[nb]),
                                                                    acc[mb][nb], 0, 0, 0);
            }
        }
      }
    }
    }
    __syncthreads();
  }

  // ---- epilogue ----
  // accumulator register r = 4j + i holds output channel 8j + 4h + i of the block
  if (head_out) {
    // fused 1x1 head: this block holds every output channel of its pixels; each
    // lane sums its 16 channels per M block, the other half-wave adds the rest
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int gy = ty0 + pr, gx = tx0 + nb * 16 + pc;
      float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int c = co0 + mb * 32 + 8 * j + 4 * h + i;
            if (c < a.cout) {
              const float v = fmaxf(acc[mb][nb][4 * j + i] + a.bias[c], 0.f);
              s0 = fmaf(a.head_w[c], v, s0);
              s1 = fmaf(a.head_w[a.cout + c], v, s1);
              s2 = fmaf(a.head_w[2 * a.cout + c], v, s2);
            }
          }
      s0 += __shfl_xor(s0, 32, 64);
      s1 += __shfl_xor(s1, 32, 64);
      s2 += __shfl_xor(s2, 32, 64);
      if (h == 0 && gy < H && gx < W) {
        const size_t HW = (size_t)H * W, p = (size_t)gy * W + gx;
        head_out[p] = s0 + a.head_b[0];
        head_out[HW + p] = s1 + a.head_b[1];
        head_out[2 * HW + p] = s2 + a.head_b[2];
      }
    }
    return;
  }
  // bias + ReLU, store NHWC, optional fused 2x2 max-pool
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int gy = ty0 + pr, gx = tx0 + nb * 16 + pc;
      const bool inside = gy < H && gx < W;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = co0 + mb * 32 + 8 * j + 4 * h;
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = fmaxf(acc[mb][nb][4 * j + i] + a.bias[c + i], 0.f);
        const bool store = inside && c < a.cout;
        if (MODE == 1) {
          uint16_t b16[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) b16[i] = f2bf(v[i]);
          if (store)
            *reinterpret_cast<uint2 *>(reinterpret_cast<uint16_t *>(out) + ((size_t)gy * W + gx) * a.cout + c) =
                make_uint2(b16[0] | ((uint32_t)b16[1] << 16), b16[2] | ((uint32_t)b16[3] << 16));
        } else {
          if (store)
            *reinterpret_cast<float4 *>(reinterpret_cast<float *>(out) + ((size_t)gy * W + gx) * a.cout + c) =
                make_float4(v[0], v[1], v[2], v[3]);
        }
        if (out_pool) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            v[i] = fmaxf(v[i], __shfl_xor(v[i], 1, 64));
            v[i] = fmaxf(v[i], __shfl_xor(v[i], 16, 64));
          }
          if (store && (pc & 1) == 0 && (pr & 1) == 0) {
            const size_t pi = ((size_t)(gy >> 1) * (W >> 1) + (gx >> 1)) * a.cout + c;
            if (MODE == 1) {
              uint16_t b16[4];
#pragma unroll
              for (int i = 0; i < 4; ++i) b16[i] = f2bf(v[i]);
              *reinterpret_cast<uint2 *>(reinterpret_cast<uint16_t *>(out_pool) + pi) =
                  make_uint2(b16[0] | ((uint32_t)b16[1] << 16), b16[2] | ((uint32_t)b16[3] << 16));
            } else {
              *reinterpret_cast<float4 *>(reinterpret_cast<float *>(out_pool) + pi) = make_float4(v[0], v[1], v[2], v[3]);
            }
          }
        }
      }
    }
  }
}

// bfloat16 3x3 convolution with row reuse.  Each wave owns R output rows of a
// 32-pixel-wide column strip and BM output channels.  For one horizontal tap
// offset dx and one 16-channel group it reads the R + 2 input-row fragments it
// needs once and feeds each of them to the up-to-three vertical taps that use
// it, so the activation operand is read from LDS (R + 2) times per 3R MFMAs
// instead of 3R times.  N block = 32 consecutive pixels of one row; the
// accumulator layout, pooling and head epilogues follow the generic kernel
// (the 2x2 pool partner is the next row's accumulator of the same lane).
template <int BM, int CK, int R>
__global__ __launch_bounds__(256) void conv3x3_rows_bf16_kernel(ConvArgs a) {
  constexpr int S = CK + 8;               // bf16 elements per staged pixel
  constexpr int MB = BM / 32;
  constexpr int TH = 4 * R, TW = 32;       // output tile
  constexpr int LW = TW + 2, LPix = (TH + 2) * LW;
  __shared__ __attribute__((aligned(16))) uint16_t s_in[LPix * S];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = lane & 31, h = lane >> 5;
  const int ty0 = blockIdx.y * TH, tx0 = blockIdx.x * TW;
  const int nzc = gridDim.z / a.batch;
  const int bimg = blockIdx.z / nzc;
  const int co0 = (blockIdx.z - bimg * nzc) * BM;
  const int H = a.H, W = a.W;
  const int Cin = a.C0 + a.C1;
  const uint16_t *in0 = static_cast<const uint16_t *>(a.in0) + (size_t)bimg * a.in0_bs;
  const uint16_t *in1 = a.in1 ? static_cast<const uint16_t *>(a.in1) + (size_t)bimg * a.in1_bs : nullptr;
  uint16_t *out = a.out ? static_cast<uint16_t *>(a.out) + (size_t)bimg * a.out_bs : nullptr;
  uint16_t *out_pool = a.out_pool ? static_cast<uint16_t *>(a.out_pool) + (size_t)bimg * a.pool_bs : nullptr;
  float *head_out = a.head_outs ? a.head_outs[bimg] : (a.head_out ? a.head_out + (size_t)bimg * 3 * H * W : nullptr);
  const uint16_t *wp = static_cast<const uint16_t *>(a.w);

  floatx16 acc[MB][R];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[mb][r][q] = 0.f;

  const int row0 = wv * R;  // first output row of this wave within the tile
  for (int ci = 0; ci < Cin; ci += CK) {
    const bool from0 = ci < a.C0;
    const int csrc = from0 ? a.C0 : a.C1;
    const int coff = from0 ? ci : ci - a.C0;
    const uint16_t *src = from0 ? in0 : in1;
    constexpr int NV = CK / 8;
    for (int e = tid; e < LPix * NV; e += 256) {
      const int pix = e / NV, q = e - pix * NV;
      const int gy = ty0 - 1 + pix / LW, gx = tx0 - 1 + pix % LW;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
        const size_t gi = from0 ? ((size_t)gy * W + gx) * csrc + coff + q * 8
                                : ((size_t)(gy >> 1) * (W >> 1) + (gx >> 1)) * csrc + coff + q * 8;
        v = *reinterpret_cast<const uint4 *>(src + gi);
      }
      *reinterpret_cast<uint4 *>(&s_in[pix * S + q * 8]) = v;
    }
    __syncthreads();
#pragma unroll 1
    for (int g = 0; g < CK / 16; ++g) {
#pragma unroll 1
      for (int dx = 0; dx < 3; ++dx) {
        uint4 av[MB][3], bv[R + 2];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int dy = 0; dy < 3; ++dy)
            av[mb][dy] = *reinterpret_cast<const uint4 *>(
                wp + ((size_t)(co0 + mb * 32 + n) * 9 + dy * 3 + dx) * a.cin_pad + ci + g * 16 + 8 * h);
#pragma unroll
        for (int i = 0; i < R + 2; ++i)
          bv[i] = *reinterpret_cast<const uint4 *>(&s_in[((row0 + i) * LW + n + dx) * S + g * 16 + 8 * h]);
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
              acc[mb][r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(av[mb][dy]), as_bf16x8(bv[r + dy]),
                                                                   acc[mb][r], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  const int gx = tx0 + n;
  if (head_out) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int gy = ty0 + row0 + r;
      float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int c = co0 + mb * 32 + 8 * j + 4 * h + i;
            if (c < a.cout) {
              const float v = fmaxf(acc[mb][r][4 * j + i] + a.bias[c], 0.f);
              s0 = fmaf(a.head_w[c], v, s0);
              s1 = fmaf(a.head_w[a.cout + c], v, s1);
              s2 = fmaf(a.head_w[2 * a.cout + c], v, s2);
            }
          }
      s0 += __shfl_xor(s0, 32, 64);
      s1 += __shfl_xor(s1, 32, 64);
      s2 += __shfl_xor(s2, 32, 64);
      if (h == 0 && gy < H && gx < W) {
        const size_t HW = (size_t)H * W, p = (size_t)gy * W + gx;
        head_out[p] = s0 + a.head_b[0];
        head_out[HW + p] = s1 + a.head_b[1];
        head_out[2 * HW + p] = s2 + a.head_b[2];
      }
    }
    return;
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = co0 + mb * 32 + 8 * j + 4 * h;
      float v[R][4];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) v[r][i] = fmaxf(acc[mb][r][4 * j + i] + a.bias[c + i], 0.f);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int gy = ty0 + row0 + r;
        if (gy < H && gx < W && c < a.cout) {
          uint16_t b16[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) b16[i] = f2bf(v[r][i]);
          *reinterpret_cast<uint2 *>(out + ((size_t)gy * W + gx) * a.cout + c) =
              make_uint2(b16[0] | ((uint32_t)b16[1] << 16), b16[2] | ((uint32_t)b16[3] << 16));
        }
      }
      if (out_pool) {
#pragma unroll
        for (int r = 0; r < R; r += 2) {
          float m[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            m[i] = fmaxf(v[r][i], v[r + 1][i]);
            m[i] = fmaxf(m[i], __shfl_xor(m[i], 1, 64));
          }
          const int gy = ty0 + row0 + r;
          if ((n & 1) == 0 && gy < H && gx < W && c < a.cout) {
            uint16_t b16[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) b16[i] = f2bf(m[i]);
            *reinterpret_cast<uint2 *>(out_pool + ((size_t)(gy >> 1) * (W >> 1) + (gx >> 1)) * a.cout + c) =
                make_uint2(b16[0] | ((uint32_t)b16[1] << 16), b16[2] | ((uint32_t)b16[3] << 16));
          }
        }
      }
    }
  }
}

// RGBDA -> network input x = (r/255, g/255, b/255, A ? D/16 : 0, A, 0...), cpad channels
template <int MODE>
__global__ __launch_bounds__(256) void pack_kernel(const float *__restrict__ depth, const uint32_t *__restrict__ rgba,
                                                   int npix, int cpad, void *__restrict__ x) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= npix) return;
  const uint32_t q = rgba[p];
  const bool A = (q >> 24) != 0;
  float v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = 0.f;
  v[0] = (float)(q & 255u) / 255.0f;
  v[1] = (float)((q >> 8) & 255u) / 255.0f;
  v[2] = (float)((q >> 16) & 255u) / 255.0f;
  v[3] = A ? depth[p] * 0.0625f : 0.f;
  v[4] = A ? 1.f : 0.f;
  if (MODE == 1) {
    uint16_t *o = static_cast<uint16_t *>(x) + (size_t)p * cpad;
    for (int i = 0; i < cpad; i += 2) *reinterpret_cast<uint32_t *>(o + i) = f2bf(v[i]) | ((uint32_t)f2bf(v[i + 1]) << 16);
  } else {
    float *o = static_cast<float *>(x) + (size_t)p * cpad;
    for (int i = 0; i < cpad; i += 4) *reinterpret_cast<float4 *>(o + i) = make_float4(v[i], v[i + 1], v[i + 2], v[i + 3]);
  }
}

// 1x1 head, float32 weights [3][C], one thread per pixel, planar float32 output
template <int MODE>
__global__ __launch_bounds__(256) void head_kernel(const void *__restrict__ x, int C, int npix,
                                                   const float *__restrict__ w, const float *__restrict__ b,
                                                   float *__restrict__ out) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= npix) return;
  float y0 = b[0], y1 = b[1], y2 = b[2];
  for (int c = 0; c < C; c += 4) {
    float v[4];
    if (MODE == 1) {
      const uint2 q = *reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(x) + (size_t)p * C + c);
      v[0] = __uint_as_float(q.x << 16);
      v[1] = __uint_as_float(q.x & 0xFFFF0000u);
      v[2] = __uint_as_float(q.y << 16);
      v[3] = __uint_as_float(q.y & 0xFFFF0000u);
    } else {
      const float4 q = *reinterpret_cast<const float4 *>(static_cast<const float *>(x) + (size_t)p * C + c);
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      y0 = fmaf(w[c + i], v[i], y0);
      y1 = fmaf(w[C + c + i], v[i], y1);
      y2 = fmaf(w[2 * C + c + i], v[i], y2);
    }
  }
  out[p] = y0;
  out[(size_t)npix + p] = y1;
  out[2 * (size_t)npix + p] = y2;
}

template <int MODE, int BM, int CK, int NB>
hipError_t conv_launch(const ConvArgs &a, int cout_pad, hipStream_t s) {
  constexpr int kTW = 16 * NB;
  dim3 grid((a.W + kTW - 1) / kTW, (a.H + kTH - 1) / kTH, (cout_pad / BM) * a.batch);
  conv3x3_kernel<MODE, BM, CK, NB><<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

template <int MODE, int BM, int NB>
hipError_t conv_dispatch_ck(const ConvArgs &a, int ck, int cout_pad, hipStream_t s) {
  if constexpr (NB == 2 || MODE == 1)
    if (ck == 32) return conv_launch<MODE, BM, 32, NB>(a, cout_pad, s);
  if (ck == 16) return conv_launch<MODE, BM, 16, NB>(a, cout_pad, s);
  if constexpr (MODE == 0)
    if (ck == 8) return conv_launch<0, BM, 8, NB>(a, cout_pad, s);
  return hipErrorInvalidValue;
}

// Tile choice.  Layers with 64+ output channels use 64-channel workgroups with
// waves of 2 x 32 pixels, unless that grid would leave the chip under-filled
// (fewer than kSmallGridWgs workgroups per image): then 32-channel workgroups double the
// grid.  32-channel layers in float32 and split bf16 use waves of 2 x 64 pixels
// (more reuse of each weight fragment) with at most 16 staged channels so the
// wider LDS tile stays within 64 KB; plain bf16 measured faster with 2 x 32.
#ifndef LNR_CONV_SMALL_GRID_WGS
#define LNR_CONV_SMALL_GRID_WGS 768
#endif
#ifndef LNR_CONV_F32_MAX_CK
#define LNR_CONV_F32_MAX_CK 32
#endif
constexpr long kSmallGridWgs = LNR_CONV_SMALL_GRID_WGS;
#ifndef LNR_CONV_BF16_ROW_REUSE
#define LNR_CONV_BF16_ROW_REUSE 1
#endif
constexpr bool kBf16RowReuse = LNR_CONV_BF16_ROW_REUSE != 0;

template <int BM, int CK>
hipError_t conv_rows_launch(const ConvArgs &a, int cout_pad, hipStream_t s) {
  constexpr int R = 4;
  dim3 grid((a.W + 31) / 32, (a.H + 4 * R - 1) / (4 * R), (cout_pad / BM) * a.batch);
  conv3x3_rows_bf16_kernel<BM, CK, R><<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

template <int BM>
hipError_t conv_rows_dispatch_ck(const ConvArgs &a, int ck, int cout_pad, hipStream_t s) {
  if (ck == 32) return conv_rows_launch<BM, 32>(a, cout_pad, s);
  if (ck == 16) return conv_rows_launch<BM, 16>(a, cout_pad, s);
  return hipErrorInvalidValue;
}

template <int MODE>
hipError_t conv_dispatch(const ConvArgs &a, int ck, int cout_pad, hipStream_t s) {
  if constexpr (MODE == 1) {
    // row reuse measured faster at 128 output channels and 270x480 pixels
    // (510 workgroups), slower at 256 channels on 135x240 (288 workgroups)
    // and mixed at 32 and 64 channels: keep it to wide layers with enough
    // 32x16 tiles to occupy the chip.  Like the small-grid switch below, the
    // choice looks at one image only, so a frame's output does not depend on
    // the batch it was served in.
    const long rows_wgs = (long)((a.W + 31) / 32) * ((a.H + 15) / 16) * (cout_pad / 64);
    if (kBf16RowReuse && cout_pad >= 128 && cout_pad % 64 == 0 && rows_wgs >= 384)
      return conv_rows_dispatch_ck<64>(a, ck, cout_pad, s);
  }
  const long tiles = (long)((a.W + 31) / 32) * ((a.H + kTH - 1) / kTH);
  const bool small = kSmallGridWgs > 0 && tiles * (cout_pad / 64) < kSmallGridWgs;
  if (cout_pad % 64 == 0 && !small) {
    const int ck64 = (MODE == 0 && ck > LNR_CONV_F32_MAX_CK) ? LNR_CONV_F32_MAX_CK : ck;
    return conv_dispatch_ck<MODE, 64, 2>(a, ck64, cout_pad, s);
  }
  if constexpr (MODE == 1) {
    return conv_dispatch_ck<MODE, 32, 2>(a, ck, cout_pad, s);
  } else {
    if (cout_pad > 32) return conv_dispatch_ck<MODE, 32, 2>(a, ck, cout_pad, s);
    return conv_dispatch_ck<MODE, 32, 4>(a, ck < 16 ? ck : 16, cout_pad, s);
  }
}

}  // namespace

hipError_t launch_pack_input(const float *depth, const uint32_t *rgba, int H, int W, int cpad, Prec p, void *x,
                             hipStream_t s) {
  const int npix = H * W;
  const int nb = (npix + 255) / 256;
  if (p == Prec::BF16)
    pack_kernel<1><<<nb, 256, 0, s>>>(depth, rgba, npix, cpad, x);
  else
    pack_kernel<0><<<nb, 256, 0, s>>>(depth, rgba, npix, cpad, x);
  return hipGetLastError();
}

hipError_t launch_conv3x3(const ConvCall &c, Prec p, hipStream_t s) {
  const ConvLayer &L = *c.layer;
  ConvArgs a{c.in0, c.in1, c.C0, c.C1, c.H, c.W, L.w, L.w_lo, L.bias, L.cout, L.cin_pad, c.out, c.out_pool,
             c.head_w, c.head_b, c.head_out, c.batch < 1 ? 1 : c.batch, c.in0_bs, c.in1_bs, c.out_bs, c.pool_bs,
             c.head_outs};
  if (c.head_out && (L.cout_pad > 64 || c.out_pool)) return hipErrorInvalidValue;
  const int step = (p == Prec::F32) ? 8 : 16;
  int ck = 32;
  while (ck > step && ((c.C0 % ck) != 0 || (c.C1 % ck) != 0)) ck >>= 1;
  if ((c.C0 % ck) != 0 || (c.C1 % ck) != 0 || (c.C0 + c.C1) != L.cin_pad) return hipErrorInvalidValue;
  switch (p) {
    case Prec::F32: return conv_dispatch<0>(a, ck, L.cout_pad, s);
    case Prec::BF16: return conv_dispatch<1>(a, ck, L.cout_pad, s);
    case Prec::BF16X3: return conv_dispatch<2>(a, ck, L.cout_pad, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_head(const void *x, int C, int H, int W, const ConvLayer &head, Prec p, float *out, hipStream_t s) {
  const int npix = H * W;
  const int nb = (npix + 255) / 256;
  const float *w = static_cast<const float *>(head.w);
  if (p == Prec::BF16)
    head_kernel<1><<<nb, 256, 0, s>>>(x, C, npix, w, head.bias, out);
  else
    head_kernel<0><<<nb, 256, 0, s>>>(x, C, npix, w, head.bias, out);
  return hipGetLastError();
}

}  // namespace lnr
