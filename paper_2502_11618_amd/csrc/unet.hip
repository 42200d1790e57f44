// U-Net forward pass on the gfx950 matrix cores.
//
// Fig. 1 and Method, "U-Net Reconstruction": a fully convolutional U-Net maps
// the depth-filtered RGBDA image to RGB.  Each 3x3 convolution is an implicit
// GEMM (M = output channels, N = output pixels, K = 9 taps x input channels)
// on 32x32 MFMA blocks.  The decoder's nearest-neighbour upsample and channel
// concatenation are folded into the input staging (channels past the skip
// tensor are read from the coarser tensor at (y/2, x/2)), the encoder's 2x2
// max-pool into the epilogue of the convolution that feeds it, and the 1x1
// head into the epilogue of the last convolution.
//
// Arithmetic modes:
//   F32    float32 activations, v_mfma_f32_32x32x2_f32.
//   BF16   bfloat16 activations and weights, v_mfma_f32_32x32x16_bf16,
//          float32 accumulation, round-to-nearest-even to bfloat16 on store.
//   BF16X3 float32 activations; operands split into bfloat16 hi + lo in LDS,
//          hi*hi + hi*lo + lo*hi on the bf16 MFMA with float32 accumulation.
//   FP16   float16 activations and weights, v_mfma_f32_32x32x16_f16, float32
//          accumulation, round-to-nearest-even to float16 on store (the same
//          data movement as BF16, with a 10- instead of a 7-bit fraction).
//   FP8    float16 activations in HBM, rounded to OCP e4m3 (to nearest even,
//          saturating at 448) as they are staged into LDS; e4m3 weights with
//          one scale per output channel (its largest weight maps to 448);
//          v_mfma_f32_32x32x16_fp8_fp8 with float32 accumulation; the
//          epilogue multiplies by the channel's scale.
//   FP8X3  as FP8, with every operand split into e4m3 hi + lo (lo = e4m3 of
//          the remainder) and the product taken as lo*hi + hi*lo + hi*hi.
#include <hip/hip_runtime.h>

#include <atomic>

#include "lnr_internal.h"

namespace lnr {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

__device__ inline bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ inline long as_i64(uint2 v) { return __builtin_bit_cast(long, v); }
__device__ inline f16x8 as_f16x8(uint4 v) { return __builtin_bit_cast(f16x8, v); }

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
  const float *rgbda_depth;
  const uint32_t *rgbda_rgba;
  const float *wu;  // float32 Winograd-domain weights [cout_pad][16][cin_pad], or null
  const float *wscale;  // e4m3 modes: per-output-channel weight scale [cout_pad]
};

// 3x3 convolution as implicit GEMM (M = output channels, N = pixels, K = 9 taps
// x input channels), one kernel for every precision:
//   MODE 0  float32 activations and weights, v_mfma_f32_32x32x2_f32;
//   MODE 1  bf16 activations and weights, v_mfma_f32_32x32x16_bf16;
//   MODE 2  float32 activations, each operand split into bf16 hi + lo in LDS
//           (weights are stored split), product hi*hi + hi*lo + lo*hi;
//   MODE 3  fp16 activations and weights, v_mfma_f32_32x32x16_f16;
//   MODE 4  fp16 activations rounded to e4m3 as they are staged, e4m3 weights
//           scaled per output channel, v_mfma_f32_32x32x16_fp8_fp8;
//   MODE 5  as MODE 4 with hi + lo e4m3 planes of both operands (weights are
//           stored split), product lo*hi + hi*lo + hi*hi.
// Workgroup tile: 4R rows x 32 columns of output pixels x BM output channels;
// wave w owns rows [wR, wR + R).  Per staged chunk of CK input channels the
// input tile with its halo and the chunk's weights ([co][tap][CK], one copy per
// workgroup) sit in LDS.  For one horizontal tap offset dx and one channel
// group a wave reads R + 2 input-row fragments and 3 MB weight fragments and
// feeds every input row to the up-to-three vertical taps that use it.  Every
// LDS read is a per-lane base plus a compile-time offset, the staging offsets
// are computed once per thread, and the next chunk is fetched into registers
// while the current one is multiplied, so the vector ALU work per MFMA stays
// small.  The decoder's nearest upsample + concatenation is folded into the
// staging (channels past C0 come from the half-resolution input), 2x2 max-pool
// and the fused 1x1 head into the epilogue.
__device__ inline uint32_t pack_bf16x2(float lo, float hi) {
  typedef float floatx2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  const floatx2 v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));  // round to nearest even
}
__device__ inline uint32_t pack_f16x2(float lo, float hi) {
  typedef float floatx2 __attribute__((ext_vector_type(2)));
  typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
  const floatx2 v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));  // round to nearest even
}
// two float32 values -> the 16-bit storage format of MODE 1 (bf16) or MODE 3 (fp16)
// activations stored as float16 (the fp16 and both e4m3 modes) or bfloat16
constexpr bool f16_store(int mode) { return mode == 3 || mode == 4 || mode == 5; }
template <int MODE>
__device__ inline uint32_t pack16x2(float lo, float hi) {
  if constexpr (f16_store(MODE)) return pack_f16x2(lo, hi);
  else return pack_bf16x2(lo, hi);
}
template <int MODE>
__device__ inline float unpack16(uint32_t bits16) {
  if constexpr (f16_store(MODE)) return (float)__builtin_bit_cast(_Float16, (uint16_t)bits16);
  else return __uint_as_float(bits16 << 16);
}
// eight float16 values (a 16-byte vector) -> eight OCP e4m3 bytes, rounded to
// nearest even, saturating at +-448; with LO, the e4m3 of what the first
// rounding left (x - e4m3(x)) instead
template <bool LO>
__device__ inline int f16x2_to_e4m3(uint32_t w, int old, bool high_word) {
  float f0 = (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xFFFFu));
  float f1 = (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
  f0 = fminf(fmaxf(f0, -448.f), 448.f);
  f1 = fminf(fmaxf(f1, -448.f), 448.f);
  if constexpr (LO) {
    const int h = __builtin_amdgcn_cvt_pk_fp8_f32(f0, f1, 0, false);
    f0 = f0 - __builtin_amdgcn_cvt_f32_fp8(h, 0);
    f1 = f1 - __builtin_amdgcn_cvt_f32_fp8(h, 1);
  }
  return high_word ? __builtin_amdgcn_cvt_pk_fp8_f32(f0, f1, old, true)
                   : __builtin_amdgcn_cvt_pk_fp8_f32(f0, f1, old, false);
}
template <bool LO>
__device__ inline uint2 f16x8_to_e4m3(uint4 v) {
  const int a = f16x2_to_e4m3<LO>(v.y, f16x2_to_e4m3<LO>(v.x, 0, false), true);
  const int b = f16x2_to_e4m3<LO>(v.w, f16x2_to_e4m3<LO>(v.z, 0, false), true);
  return make_uint2((uint32_t)a, (uint32_t)b);
}

template <int MODE>
struct ConvTraits;
template <>
struct ConvTraits<0> {  // float32
  using In = float;       // activations in HBM
  using W = float;        // weights in HBM
  using L = float;        // LDS element
  using Frag = uint4;     // one lane's operand fragment in LDS
  static constexpr int kInVec = 4, kWVec = 4;    // elements per 16-byte HBM vector
  static constexpr int kPad = 4, kPlanes = 1, kGroup = 8;
};
template <>
struct ConvTraits<1> {  // bf16
  using In = uint16_t;
  using W = uint16_t;
  using L = uint16_t;
  using Frag = uint4;
  static constexpr int kInVec = 8, kWVec = 8;
  static constexpr int kPad = 8, kPlanes = 1, kGroup = 16;
};
template <>
struct ConvTraits<2> {  // float32 activations, split bf16 operands
  using In = float;
  using W = uint16_t;
  using L = uint16_t;
  using Frag = uint4;
  static constexpr int kInVec = 4, kWVec = 8;
  static constexpr int kPad = 8, kPlanes = 2, kGroup = 16;
};
template <>
struct ConvTraits<3> : ConvTraits<1> {};  // fp16: bf16's data movement
template <>
struct ConvTraits<4> {  // float16 activations in HBM, e4m3 bytes in LDS
  using In = uint16_t;
  using W = uint8_t;
  using L = uint8_t;
  using Frag = uint2;  // 8 e4m3 per lane and MFMA
  static constexpr int kInVec = 8, kWVec = 16;
  static constexpr int kPad = 16, kPlanes = 1, kGroup = 16;
};
template <>
struct ConvTraits<5> : ConvTraits<4> {  // e4m3 hi + lo planes
  static constexpr int kPlanes = 2;
};

// 16-bit activations in HBM (bf16 or fp16, also behind the e4m3 modes)
constexpr bool half_store(int mode) { return mode == 1 || mode == 3 || mode == 4 || mode == 5; }

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// accumulator -> layer sum: the e4m3 modes multiply by the output channel's weight scale
template <int MODE>
__device__ inline float scaled(float acc, float ws) {
  if constexpr (MODE == 4 || MODE == 5) return acc * ws;
  else return acc;
}

template <int MODE, int BM, int CK, int R, bool RGBDA>
__global__ __launch_bounds__(256) void conv3x3_kernel(ConvArgs a) {
  using T = ConvTraits<MODE>;
  using LT = typename T::L;
  using InT = typename T::In;
  using WT = typename T::W;
  static_assert(CK % T::kGroup == 0, "CK must be a multiple of the channel group");
  constexpr int S = CK + T::kPad;            // LDS elements per staged pixel / weight row (16-byte multiple)
  constexpr int MB = BM / 32;
  constexpr int TH = 4 * R, TW = 32;
  constexpr int LW = TW + 2, LPix = (TH + 2) * LW;
  constexpr int NVI = CK / T::kInVec, NVW = CK / T::kWVec;   // 16-byte vectors per pixel / weight row
  constexpr int PPI = 256 / NVI, PPW = 256 / NVW;            // pixels / weight rows per workgroup pass
  constexpr int NIN = (LPix + PPI - 1) / PPI;
  constexpr int WROWS = 9 * BM;
  constexpr int NWR = (WROWS + PPW - 1) / PPW;
  constexpr int INP = LPix * S, WP = WROWS * S;              // elements per LDS plane
  __shared__ __attribute__((aligned(16))) LT s_in[T::kPlanes * INP];
  __shared__ __attribute__((aligned(16))) LT s_w[T::kPlanes * WP];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = lane & 31, h = lane >> 5;
  const int ty0 = blockIdx.y * TH, tx0 = blockIdx.x * TW;
  const int nzc = gridDim.z / a.batch;
  const int bimg = blockIdx.z / nzc;
  const int co0 = (blockIdx.z - bimg * nzc) * BM;
  const int H = a.H, W = a.W;
  const int Cin = a.C0 + a.C1;
  const InT *in0 = static_cast<const InT *>(a.in0) + (size_t)bimg * a.in0_bs;
  const InT *in1 = a.in1 ? static_cast<const InT *>(a.in1) + (size_t)bimg * a.in1_bs : nullptr;
  InT *out = a.out ? static_cast<InT *>(a.out) + (size_t)bimg * a.out_bs : nullptr;
  InT *out_pool = a.out_pool ? static_cast<InT *>(a.out_pool) + (size_t)bimg * a.pool_bs : nullptr;
  float *head_out = a.head_outs ? a.head_outs[bimg] : (a.head_out ? a.head_out + (size_t)bimg * 3 * H * W : nullptr);

  // staging plan: this thread moves 16-byte vector qi of pixels pi0, pi0 + PPI,
  // ... (offsets in the full- and the half-resolution source, -1 outside the
  // image) and vector qw of weight rows pw0, pw0 + PPW, ...
  const int qi = (tid & (NVI - 1)) * T::kInVec, pi0 = tid >> ilog2(NVI);
  const int qw = (tid & (NVW - 1)) * T::kWVec, pw0 = tid >> ilog2(NVW);
  int off0[NIN], off1[NIN];
#pragma unroll
  for (int k = 0; k < NIN; ++k) {
    const int pix = pi0 + k * PPI;
    const int gy = ty0 - 1 + pix / LW, gx = tx0 - 1 + pix % LW;
    const bool inside = pix < LPix && gy >= 0 && gy < H && gx >= 0 && gx < W;
    off0[k] = inside ? gy * W + gx : -1;
    off1[k] = inside ? (gy >> 1) * (W >> 1) + (gx >> 1) : -1;
  }
  // weights [cout_pad][9][cin_pad]; staged row r = co * 9 + tap of this workgroup's channels
  const size_t wrow0 = ((size_t)co0 * 9 + pw0) * a.cin_pad + qw;
  const size_t wstep = (size_t)PPW * a.cin_pad;
  const WT *wsrc = static_cast<const WT *>(a.w) + wrow0;
  const WT *wsrc_lo = T::kPlanes == 2 ? static_cast<const WT *>(a.w_lo) + wrow0 : nullptr;
  constexpr int NWV = NWR * T::kPlanes;

  auto fetch = [&](int ci, uint4 (&pin)[NIN], uint4 (&pw)[NWV]) {
    const bool from0 = ci < a.C0;
    const size_t csrc = from0 ? a.C0 : a.C1;
    const InT *src = (from0 ? in0 + ci : in1 + (ci - a.C0)) + qi;
    // a pixel outside the image loads the image's first pixel and is replaced by zero
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
      const int o = from0 ? off0[k] : off1[k];
      if constexpr (RGBDA) {
        // network input x = (r/255, g/255, b/255, A ? D/16 : 0, A, 0, ...),
        // computed as the input pack computes it; this thread's vector holds
        // channels [qi, qi + kInVec)
        const size_t oc = (size_t)(o < 0 ? 0 : o);
        const uint32_t q = a.rgbda_rgba[oc];
        const float d = a.rgbda_depth[oc];
        const bool A = (q >> 24) != 0;
        const float x0 = (float)(q & 255u) / 255.0f, x1 = (float)((q >> 8) & 255u) / 255.0f;
        const float x2 = (float)((q >> 16) & 255u) / 255.0f, x3 = A ? d * 0.0625f : 0.f, x4 = A ? 1.f : 0.f;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if constexpr (half_store(MODE)) {
          if (qi == 0) v = make_uint4(pack16x2<MODE>(x0, x1), pack16x2<MODE>(x2, x3), pack16x2<MODE>(x4, 0.f), 0u);
        } else if constexpr (MODE == 0) {
          // channels (x0, x1, x2, 0 | x3, x4, 0, 0): k-steps pair channel s
          // with channel 4 + s, so the fourth pair is zero and skipped
          if (qi == 0) v = make_uint4(__float_as_uint(x0), __float_as_uint(x1), __float_as_uint(x2), 0u);
          if (qi == 4) v = make_uint4(__float_as_uint(x3), __float_as_uint(x4), 0u, 0u);
        } else {
          if (qi == 0) v = make_uint4(__float_as_uint(x0), __float_as_uint(x1), __float_as_uint(x2), __float_as_uint(x3));
          if (qi == 4) v = make_uint4(__float_as_uint(x4), 0u, 0u, 0u);
        }
        pin[k] = o < 0 ? make_uint4(0u, 0u, 0u, 0u) : v;
      } else {
        const uint4 v = *reinterpret_cast<const uint4 *>(src + (size_t)(o < 0 ? 0 : o) * csrc);
        pin[k] = o < 0 ? make_uint4(0u, 0u, 0u, 0u) : v;
      }
    }
#pragma unroll
    for (int k = 0; k < NWR; ++k) {
      const bool ok = (k + 1) * PPW <= WROWS || pw0 + k * PPW < WROWS;
      pw[k] = ok ? *reinterpret_cast<const uint4 *>(wsrc + k * wstep + ci) : make_uint4(0u, 0u, 0u, 0u);
      if constexpr (T::kPlanes == 2)
        pw[NWR + k] = ok ? *reinterpret_cast<const uint4 *>(wsrc_lo + k * wstep + ci) : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto store = [&](const uint4 (&pin)[NIN], const uint4 (&pw)[NWV]) {
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
      if (!((k + 1) * PPI <= LPix || pi0 + k * PPI < LPix)) continue;
      const int li = (pi0 + k * PPI) * S + qi;
      if constexpr (MODE == 2) {
        // 4 float32 channels -> 4 bf16 hi (plane 0) + 4 bf16 lo (plane 1)
        const float f[4] = {__uint_as_float(pin[k].x), __uint_as_float(pin[k].y), __uint_as_float(pin[k].z),
                            __uint_as_float(pin[k].w)};
        const uint32_t h01 = pack_bf16x2(f[0], f[1]), h23 = pack_bf16x2(f[2], f[3]);
        const uint32_t l01 = pack_bf16x2(f[0] - __uint_as_float(h01 << 16), f[1] - __uint_as_float(h01 & 0xFFFF0000u));
        const uint32_t l23 = pack_bf16x2(f[2] - __uint_as_float(h23 << 16), f[3] - __uint_as_float(h23 & 0xFFFF0000u));
        *reinterpret_cast<uint2 *>(&s_in[li]) = make_uint2(h01, h23);
        *reinterpret_cast<uint2 *>(&s_in[INP + li]) = make_uint2(l01, l23);
      } else if constexpr (MODE == 4 || MODE == 5) {
        // 8 float16 channels -> 8 e4m3 bytes (plane 0) [+ 8 e4m3 remainders (plane 1)]
        *reinterpret_cast<uint2 *>(&s_in[li]) = f16x8_to_e4m3<false>(pin[k]);
        if constexpr (MODE == 5) *reinterpret_cast<uint2 *>(&s_in[INP + li]) = f16x8_to_e4m3<true>(pin[k]);
      } else {
        *reinterpret_cast<uint4 *>(&s_in[li]) = pin[k];
      }
    }
#pragma unroll
    for (int k = 0; k < NWR; ++k) {
      if (!((k + 1) * PPW <= WROWS || pw0 + k * PPW < WROWS)) continue;
      const int li = (pw0 + k * PPW) * S + qw;
      *reinterpret_cast<uint4 *>(&s_w[li]) = pw[k];
      if constexpr (T::kPlanes == 2) *reinterpret_cast<uint4 *>(&s_w[WP + li]) = pw[NWR + k];
    }
  };

  floatx16 acc[MB][R];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[mb][r][q] = 0.f;

  // lane (n, h) reads channels [G g + (G/2) h, + G/2) of a group: input pixel
  // column n + dx of its rows, weight row (32 mb + n) * 9 + tap
  constexpr int G = T::kGroup, HG = G / 2;
  const LT *bbase = s_in + (wv * R * LW + n) * S + HG * h;
  const LT *abase = s_w + n * 9 * S + HG * h;
  // one step = one horizontal tap offset dx of one channel group: the
  // fragments of step s + 1 are read from LDS while the MFMAs of step s run
  constexpr int NSTEP = (CK / G) * 3;
  using FragT = typename T::Frag;
  struct Frags {
    FragT a[T::kPlanes][MB][3], b[T::kPlanes][R + 2];
  };
  auto load_frags = [&](int st, Frags &f) {
    const int g = st / 3, dx = st - 3 * g;
    const LT *ag = abase + g * G, *bg = bbase + g * G;
#pragma unroll
    for (int p = 0; p < T::kPlanes; ++p) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
          f.a[p][mb][dy] = *reinterpret_cast<const FragT *>(ag + p * WP + (mb * 32 * 9 + dy * 3 + dx) * S);
#pragma unroll
      for (int i = 0; i < R + 2; ++i) f.b[p][i] = *reinterpret_cast<const FragT *>(bg + p * INP + (i * LW + dx) * S);
    }
  };
  auto mma = [&](const Frags &f) {
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          if constexpr (MODE == 0) {
            const float4 av4 = __builtin_bit_cast(float4, f.a[0][mb][dy]);
            const float4 bv4 = __builtin_bit_cast(float4, f.b[0][r + dy]);
            acc[mb][r] = __builtin_amdgcn_mfma_f32_32x32x2f32(av4.x, bv4.x, acc[mb][r], 0, 0, 0);
            acc[mb][r] = __builtin_amdgcn_mfma_f32_32x32x2f32(av4.y, bv4.y, acc[mb][r], 0, 0, 0);
            acc[mb][r] = __builtin_amdgcn_mfma_f32_32x32x2f32(av4.z, bv4.z, acc[mb][r], 0, 0, 0);
            // the staged network input has zeros in channels 3 and 7
            if constexpr (!RGBDA)
              acc[mb][r] = __builtin_amdgcn_mfma_f32_32x32x2f32(av4.w, bv4.w, acc[mb][r], 0, 0, 0);
          } else if constexpr (MODE == 1) {
            acc[mb][r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(f.a[0][mb][dy]), as_bf16x8(f.b[0][r + dy]),
                                                                 acc[mb][r], 0, 0, 0);
          } else if constexpr (MODE == 3) {
            acc[mb][r] = __builtin_amdgcn_mfma_f32_32x32x16_f16(as_f16x8(f.a[0][mb][dy]), as_f16x8(f.b[0][r + dy]),
                                                                acc[mb][r], 0, 0, 0);
          } else if constexpr (MODE == 4) {
            acc[mb][r] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(as_i64(f.a[0][mb][dy]), as_i64(f.b[0][r + dy]),
                                                                    acc[mb][r], 0, 0, 0);
          } else if constexpr (MODE == 5) {
            acc[mb][r] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(as_i64(f.a[1][mb][dy]), as_i64(f.b[0][r + dy]),
                                                                    acc[mb][r], 0, 0, 0);
            acc[mb][r] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(as_i64(f.a[0][mb][dy]), as_i64(f.b[1][r + dy]),
                                                                    acc[mb][r], 0, 0, 0);
            acc[mb][r] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(as_i64(f.a[0][mb][dy]), as_i64(f.b[0][r + dy]),
                                                                    acc[mb][r], 0, 0, 0);
          } else {
            const int P1 = T::kPlanes - 1;  // lo plane
            acc[mb][r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(f.a[P1][mb][dy]), as_bf16x8(f.b[0][r + dy]),
                                                                 acc[mb][r], 0, 0, 0);
            acc[mb][r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(f.a[0][mb][dy]), as_bf16x8(f.b[P1][r + dy]),
                                                                 acc[mb][r], 0, 0, 0);
            acc[mb][r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(f.a[0][mb][dy]), as_bf16x8(f.b[0][r + dy]),
                                                                 acc[mb][r], 0, 0, 0);
          }
        }
  };
  auto compute = [&]() {
    if constexpr (MODE == 0) {
      // float32 MFMAs are long (64 cycles each, 4 per fragment pair): no need
      // to hold two steps of fragments
#pragma unroll 1
      for (int g = 0; g < CK / G; ++g) {
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          Frags f;
          load_frags(3 * g + dx, f);
          mma(f);
        }
      }
    } else {
      Frags f0, f1;
      load_frags(0, f0);
#pragma unroll
      for (int st = 0; st < NSTEP; st += 2) {
        if (st + 1 < NSTEP) load_frags(st + 1, f1);
        mma(f0);
        if (st + 1 < NSTEP) {
          if (st + 2 < NSTEP) load_frags(st + 2, f0);
          mma(f1);
        }
      }
      // scheduler strategy for MFMA / LDS-read interleaving (measured: 1 for
      // bf16, 0 for the three-pass split mode)
      if constexpr (MODE == 1 || MODE == 3 || MODE == 4) __builtin_amdgcn_iglp_opt(1);
      else __builtin_amdgcn_iglp_opt(0);
    }
  };
  {
    uint4 pin[NIN], pw[NWV];
    fetch(0, pin, pw);
    store(pin, pw);
  }
  __syncthreads();
  // every chunk but the last: fetch the next one while multiplying this one
  for (int ci = CK; ci < Cin; ci += CK) {
    uint4 pin[NIN], pw[NWV];
    fetch(ci, pin, pw);
    compute();
    __syncthreads();
    store(pin, pw);
    __syncthreads();
  }
  compute();

  // ---- epilogue: accumulator register 4j + i of block (mb, r) holds output
  // channel co0 + 32 mb + 8j + 4h + i of pixel (ty0 + wR + r, tx0 + n)
  const int gx = tx0 + n;
  const int row0 = wv * R;
  if (head_out) {
    // per row, the sums run over (mb, j, i) in the same order; the bias and
    // head weights of a group of 4 channels are read once for all rows
    float hs[R][3];
#pragma unroll
    for (int r = 0; r < R; ++r) hs[r][0] = hs[r][1] = hs[r][2] = 0.f;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = co0 + mb * 32 + 8 * j + 4 * h;
        if (c < a.cout) {
          const float4 b = *reinterpret_cast<const float4 *>(a.bias + c);
          const float bb[4] = {b.x, b.y, b.z, b.w};
          float ws[4] = {1.f, 1.f, 1.f, 1.f};
          if constexpr (MODE == 4 || MODE == 5) {
            const float4 w4 = *reinterpret_cast<const float4 *>(a.wscale + c);
            ws[0] = w4.x; ws[1] = w4.y; ws[2] = w4.z; ws[3] = w4.w;
          }
          float hw[3][4];  // head weights [output][channel c + i] (rows of cout floats, 16-byte aligned)
#pragma unroll
          for (int o = 0; o < 3; ++o) {
            const float4 w = *reinterpret_cast<const float4 *>(a.head_w + o * a.cout + c);
            hw[o][0] = w.x; hw[o][1] = w.y; hw[o][2] = w.z; hw[o][3] = w.w;
          }
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float v = fmaxf(scaled<MODE>(acc[mb][r][4 * j + i], ws[i]) + bb[i], 0.f);
              hs[r][0] = fmaf(hw[0][i], v, hs[r][0]);
              hs[r][1] = fmaf(hw[1][i], v, hs[r][1]);
              hs[r][2] = fmaf(hw[2][i], v, hs[r][2]);
            }
        }
      }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int gy = ty0 + row0 + r;
      const float s0 = hs[r][0] + __shfl_xor(hs[r][0], 32, 64);
      const float s1 = hs[r][1] + __shfl_xor(hs[r][1], 32, 64);
      const float s2 = hs[r][2] + __shfl_xor(hs[r][2], 32, 64);
      if (h == 0 && gy < H && gx < W) {
        const size_t HW = (size_t)H * W, p = (size_t)gy * W + gx;
        head_out[p] = s0 + a.head_b[0];
        head_out[HW + p] = s1 + a.head_b[1];
        head_out[2 * HW + p] = s2 + a.head_b[2];
      }
    }
    return;
  }
  auto put4 = [&](InT *dst, const float (&v)[4]) {
    if constexpr (half_store(MODE))
      *reinterpret_cast<uint2 *>(dst) = make_uint2(pack16x2<MODE>(v[0], v[1]), pack16x2<MODE>(v[2], v[3]));
    else
      *reinterpret_cast<float4 *>(dst) = make_float4(v[0], v[1], v[2], v[3]);
  };
  // bf16: a lane holds 8 bytes of each of 32 pixels' channel runs, so direct
  // stores write 16-byte pieces 2 BM bytes apart.  Where LDS allows, each wave
  // stages its R x 32 pixels x BM channels in LDS ([pixel][channel], 16-byte
  // pad per pixel) and writes them back as whole 16-byte runs of consecutive
  // channels, consecutive lanes covering consecutive memory.
  constexpr int PSTR = BM * 2 + 16;                              // staged bytes per pixel
  constexpr int STAGE = 4 * R * 32 * PSTR;                       // all waves
  constexpr bool kStage = half_store(MODE) && (STAGE <= (int)sizeof(s_in) || STAGE <= (int)sizeof(s_w));
  char *stage = nullptr;
  if constexpr (kStage) {
    __syncthreads();  // every wave is done with the K loop's LDS
    char *base = STAGE <= (int)sizeof(s_in) ? reinterpret_cast<char *>(s_in) : reinterpret_cast<char *>(s_w);
    stage = base + wv * R * 32 * PSTR;
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = co0 + mb * 32 + 8 * j + 4 * h;
      if (c >= a.cout) continue;
      const float4 b = *reinterpret_cast<const float4 *>(a.bias + c);
      const float bb[4] = {b.x, b.y, b.z, b.w};
      float ws[4] = {1.f, 1.f, 1.f, 1.f};
      if constexpr (MODE == 4 || MODE == 5) {
        const float4 w4 = *reinterpret_cast<const float4 *>(a.wscale + c);
        ws[0] = w4.x; ws[1] = w4.y; ws[2] = w4.z; ws[3] = w4.w;
      }
      float v[R][4];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) v[r][i] = fmaxf(scaled<MODE>(acc[mb][r][4 * j + i], ws[i]) + bb[i], 0.f);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (kStage) {
          *reinterpret_cast<uint2 *>(stage + (r * 32 + n) * PSTR + (mb * 32 + 8 * j + 4 * h) * 2) =
              make_uint2(pack16x2<MODE>(v[r][0], v[r][1]), pack16x2<MODE>(v[r][2], v[r][3]));
        } else {
          const int gy = ty0 + row0 + r;
          if (gy < H && gx < W) put4(out + ((size_t)gy * W + gx) * a.cout + c, v[r]);
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
          if ((n & 1) == 0 && gy < H && gx < W)
            put4(out_pool + ((size_t)(gy >> 1) * (W >> 1) + (gx >> 1)) * a.cout + c, m);
        }
      }
    }
  }
  if constexpr (kStage) {
    // the wave reads back its own rows (its LDS writes above come first in
    // order): 16-byte run s of pixel p of row r is item (r 32 + p) BM / 8 + s
    constexpr int RUNS = BM / 8, ITEMS = R * 32 * RUNS;
    static_assert(ITEMS % 64 == 0, "whole wave passes");
#pragma unroll
    for (int it = 0; it < ITEMS / 64; ++it) {
      const int item = it * 64 + lane, rp = item / RUNS, run = item - rp * RUNS;
      const int r = rp >> 5, p = rp & 31;
      const int gy = ty0 + row0 + r, gxx = tx0 + p, c = co0 + 8 * run;
      const uint4 x = *reinterpret_cast<const uint4 *>(stage + rp * PSTR + run * 16);
      if (gy < H && gxx < W && c < a.cout)
        *reinterpret_cast<uint4 *>(out + ((size_t)gy * W + gxx) * a.cout + c) = x;
    }
  }
}

// The network's first two convolutions in one kernel, for the 16-bit modes
// (MODE 1 bf16, MODE 3 fp16) when the first level has at most 32 channels.
// An output tile of 8 rows x 32 columns x 32 channels of the second
// convolution needs the first convolution's output on a 10 x 34 pixel region
// (its halo), which needs the network input on 12 x 36 pixels.  Phase 1 stages
// that input and the first layer's weights in LDS and computes the first
// convolution on the 340 region pixels (eleven 32-pixel MFMA blocks: ten region
// rows of 32 columns and one block of the 20 pixels of the two right-hand
// columns), with bias, ReLU and the same 16-bit rounding the unfused layer's
// store applies, and zero where a region pixel lies outside the image (the
// second layer's padding).  The result stays in LDS as the second layer's
// staged input; phase 2 is the generic kernel's single-chunk K loop and
// epilogue (ReLU output for the skip connection and its 2x2 max-pool) on it.
// Both layers take their sums in the generic kernel's order, so the outputs
// are bit-identical to the two unfused launches; the first layer's output
// never goes to HBM.  CK1 = channels of the first level (16 or 32); RGBDA:
// the input comes from the RGBDA image (a single image) instead of the
// packed 16-channel input tensor.
template <int MODE, int CK1, bool RGBDA>
__global__ __launch_bounds__(256) void enc0_fused_kernel(ConvArgs a0, ConvArgs a1) {
  static_assert(MODE == 1 || MODE == 3, "16-bit modes only");
  using T = ConvTraits<MODE>;
  using LT = typename T::L;
  using InT = typename T::In;
  constexpr int R = 2, TH = 4 * R, TW = 32;
  constexpr int XW = TW + 4, XPix = (TH + 4) * XW;  // network input region
  constexpr int MW = TW + 2, MPix = (TH + 2) * MW;  // first layer's output region
  constexpr int C0 = 16, S0 = C0 + T::kPad, S1 = CK1 + T::kPad;
  constexpr int WROWS = 9 * 32;
  // LDS: [ input region | first-layer weights ] (phase 1), reused for the
  // second layer's weights and then the output staging; [ region ] throughout
  constexpr int A_ELEMS = XPix * S0 + WROWS * S0;
  static_assert(WROWS * S1 <= A_ELEMS, "second-layer weights fit where phase 1 was");
  __shared__ __attribute__((aligned(16))) LT s_a[A_ELEMS];
  __shared__ __attribute__((aligned(16))) LT s_mid[MPix * S1];
  LT *s_x = s_a, *s_w0 = s_a + XPix * S0, *s_w1 = s_a;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = lane & 31, h = lane >> 5;
  const int ty0 = blockIdx.y * TH, tx0 = blockIdx.x * TW;
  const int bimg = blockIdx.z;
  const int H = a1.H, W = a1.W;
  const InT *in0 = static_cast<const InT *>(a0.in0) + (size_t)bimg * a0.in0_bs;
  InT *out = static_cast<InT *>(a1.out) + (size_t)bimg * a1.out_bs;
  InT *out_pool = static_cast<InT *>(a1.out_pool) + (size_t)bimg * a1.pool_bs;

  // ---- phase 1 staging: network input (16 channels per pixel), first-layer
  // weights [32][9][16]; second-layer weights [32][9][CK1] go to registers now
  // and to LDS after phase 1.  Every load is issued before the first use.
  constexpr int NXP = (XPix + 255) / 256;               // input pixels per thread
  constexpr int NV0 = WROWS * 2, NW0 = (NV0 + 255) / 256;  // first-layer weight vectors
  constexpr int NV1 = WROWS * (CK1 / 8), NW1 = (NV1 + 255) / 256;
  const uint16_t *w0 = static_cast<const uint16_t *>(a0.w);
  const uint16_t *w1 = static_cast<const uint16_t *>(a1.w);
  uint4 w0r[NW0], w1r[NW1];
#pragma unroll
  for (int k = 0; k < NW0; ++k) {
    const int it = tid + 256 * k;
    w0r[k] = it < NV0 ? *reinterpret_cast<const uint4 *>(w0 + (size_t)it * 8) : make_uint4(0u, 0u, 0u, 0u);
  }
#pragma unroll
  for (int k = 0; k < NW1; ++k) {
    const int it = tid + 256 * k;
    w1r[k] = it < NV1 ? *reinterpret_cast<const uint4 *>(w1 + (size_t)it * 8) : make_uint4(0u, 0u, 0u, 0u);
  }
  bool xin[NXP];
  size_t xo[NXP];
#pragma unroll
  for (int k = 0; k < NXP; ++k) {
    const int pix = tid + 256 * k;
    const int gy = ty0 - 2 + pix / XW, gx = tx0 - 2 + pix % XW;
    xin[k] = pix < XPix && gy >= 0 && gy < H && gx >= 0 && gx < W;
    xo[k] = xin[k] ? (size_t)gy * W + gx : 0;
  }
  if constexpr (RGBDA) {
    uint32_t xc[NXP];
    float xd[NXP];
#pragma unroll
    for (int k = 0; k < NXP; ++k) {
      xc[k] = a0.rgbda_rgba[xo[k]];
      xd[k] = a0.rgbda_depth[xo[k]];
    }
#pragma unroll
    for (int k = 0; k < NXP; ++k) {
      const int pix = tid + 256 * k;
      if (pix >= XPix) continue;
      // network input x = (r/255, g/255, b/255, A ? D/16 : 0, A, 0, ...), as the input pack computes it
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (xin[k]) {
        const uint32_t c = xc[k];
        const bool A = (c >> 24) != 0;
        const float x0 = (float)(c & 255u) / 255.0f, x1 = (float)((c >> 8) & 255u) / 255.0f;
        const float x2 = (float)((c >> 16) & 255u) / 255.0f, x3 = A ? xd[k] * 0.0625f : 0.f, x4 = A ? 1.f : 0.f;
        v = make_uint4(pack16x2<MODE>(x0, x1), pack16x2<MODE>(x2, x3), pack16x2<MODE>(x4, 0.f), 0u);
      }
      *reinterpret_cast<uint4 *>(&s_x[pix * S0]) = v;
      *reinterpret_cast<uint4 *>(&s_x[pix * S0 + 8]) = make_uint4(0u, 0u, 0u, 0u);
    }
  } else {
    uint4 xa[NXP], xb[NXP];
#pragma unroll
    for (int k = 0; k < NXP; ++k) {
      const uint4 *src = reinterpret_cast<const uint4 *>(in0 + xo[k] * C0);
      xa[k] = src[0];
      xb[k] = src[1];
    }
#pragma unroll
    for (int k = 0; k < NXP; ++k) {
      const int pix = tid + 256 * k;
      const uint32_t m = xin[k] ? ~0u : 0u;  // a pixel outside the image is zero
      if (pix < XPix) {
        *reinterpret_cast<uint4 *>(&s_x[pix * S0]) = make_uint4(xa[k].x & m, xa[k].y & m, xa[k].z & m, xa[k].w & m);
        *reinterpret_cast<uint4 *>(&s_x[pix * S0 + 8]) = make_uint4(xb[k].x & m, xb[k].y & m, xb[k].z & m, xb[k].w & m);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NW0; ++k) {
    const int it = tid + 256 * k;
    if (it < NV0) *reinterpret_cast<uint4 *>(&s_w0[(it >> 1) * S0 + (it & 1) * 8]) = w0r[k];
  }
  __syncthreads();

  // ---- phase 1: first convolution on the region, wave w takes blocks w, w + 4, w + 8
  for (int blk = wv; blk < 11; blk += 4) {
    // this lane's region pixel (mr, mc); lanes 20..31 of block 10 compute a
    // copy of pixel (0, 32) and store nothing
    const bool extra = blk == 10;
    const bool live = !extra || n < 20;
    const int mr = extra ? (live ? n >> 1 : 0) : blk;
    const int mc = extra ? 32 + (n & 1) : n;
    floatx16 acc;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.f;
    const LT *bb = s_x + (mr * XW + mc) * S0 + 8 * h;
    const LT *ab = s_w0 + n * 9 * S0 + 8 * h;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const uint4 av = *reinterpret_cast<const uint4 *>(ab + (dy * 3 + dx) * S0);
        const uint4 bv = *reinterpret_cast<const uint4 *>(bb + (dy * XW + dx) * S0);
        if constexpr (MODE == 1)
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(av), as_bf16x8(bv), acc, 0, 0, 0);
        else
          acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(as_f16x8(av), as_f16x8(bv), acc, 0, 0, 0);
      }
    // register 4j + i holds channel 8j + 4h + i of the lane's pixel
    const int gy = ty0 - 1 + mr, gx = tx0 - 1 + mc;
    const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
    if (live) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = 8 * j + 4 * h;
        if (c >= CK1) continue;
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        if (inside && c < a0.cout) {
          const float4 b = *reinterpret_cast<const float4 *>(a0.bias + c);
          v[0] = fmaxf(acc[4 * j + 0] + b.x, 0.f);
          v[1] = fmaxf(acc[4 * j + 1] + b.y, 0.f);
          v[2] = fmaxf(acc[4 * j + 2] + b.z, 0.f);
          v[3] = fmaxf(acc[4 * j + 3] + b.w, 0.f);
        }
        *reinterpret_cast<uint2 *>(&s_mid[(mr * MW + mc) * S1 + c]) =
            make_uint2(pack16x2<MODE>(v[0], v[1]), pack16x2<MODE>(v[2], v[3]));
      }
    }
  }
  __syncthreads();  // phase 1's LDS reads are done: its space takes the second layer's weights
#pragma unroll
  for (int k = 0; k < NW1; ++k) {
    const int it = tid + 256 * k;
    if (it < NV1) {
      const int row = it / (CK1 / 8), q = (it - row * (CK1 / 8)) * 8;
      *reinterpret_cast<uint4 *>(&s_w1[row * S1 + q]) = w1r[k];
    }
  }
  __syncthreads();

  // ---- phase 2: second convolution, the generic kernel's K loop for one chunk
  floatx16 acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[r][q] = 0.f;
  {
    constexpr int G = T::kGroup, HG = G / 2, NSTEP = (CK1 / G) * 3;
    const LT *bbase = s_mid + (wv * R * MW + n) * S1 + HG * h;
    const LT *abase = s_w1 + n * 9 * S1 + HG * h;
#pragma unroll
    for (int st = 0; st < NSTEP; ++st) {
      const int g = st / 3, dx = st - 3 * g;
      uint4 fa[3], fb[R + 2];
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) fa[dy] = *reinterpret_cast<const uint4 *>(abase + g * G + (dy * 3 + dx) * S1);
#pragma unroll
      for (int i = 0; i < R + 2; ++i) fb[i] = *reinterpret_cast<const uint4 *>(bbase + g * G + (i * MW + dx) * S1);
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if constexpr (MODE == 1)
            acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(fa[dy]), as_bf16x8(fb[r + dy]), acc[r], 0, 0, 0);
          else
            acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_f16(as_f16x8(fa[dy]), as_f16x8(fb[r + dy]), acc[r], 0, 0, 0);
        }
    }
  }

  // ---- epilogue (as the generic kernel's, one 32-channel block): ReLU output
  // staged per wave in LDS and written as 16-byte runs, and its 2x2 max-pool
  constexpr int BM = 32, PSTR = BM * 2 + 16, STAGE = 4 * R * 32 * PSTR;
  static_assert(STAGE <= (int)sizeof(s_a), "output staging fits");
  __syncthreads();  // every wave is done with the second layer's weights
  char *stage = reinterpret_cast<char *>(s_a) + wv * R * 32 * PSTR;
  const int gx = tx0 + n, row0 = wv * R;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = 8 * j + 4 * h;
    if (c >= a1.cout) continue;
    const float4 b = *reinterpret_cast<const float4 *>(a1.bias + c);
    const float bb[4] = {b.x, b.y, b.z, b.w};
    float v[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) v[r][i] = fmaxf(acc[r][4 * j + i] + bb[i], 0.f);
#pragma unroll
    for (int r = 0; r < R; ++r)
      *reinterpret_cast<uint2 *>(stage + (r * 32 + n) * PSTR + c * 2) =
          make_uint2(pack16x2<MODE>(v[r][0], v[r][1]), pack16x2<MODE>(v[r][2], v[r][3]));
    // R = 2: rows 0 and 1 of the wave form one pooled row
    float m[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      m[i] = fmaxf(v[0][i], v[1][i]);
      m[i] = fmaxf(m[i], __shfl_xor(m[i], 1, 64));
    }
    const int gy = ty0 + row0;
    if ((n & 1) == 0 && gy < H && gx < W)
      *reinterpret_cast<uint2 *>(out_pool + ((size_t)(gy >> 1) * (W >> 1) + (gx >> 1)) * a1.cout + c) =
          make_uint2(pack16x2<MODE>(m[0], m[1]), pack16x2<MODE>(m[2], m[3]));
  }
  {
    // the wave reads back its own rows: 16-byte run s of pixel p of row r is
    // item (r 32 + p) RUNS + s
    constexpr int RUNS = BM / 8, ITEMS = R * 32 * RUNS;
#pragma unroll
    for (int it = 0; it < ITEMS / 64; ++it) {
      const int item = it * 64 + lane, rp = item / RUNS, run = item - rp * RUNS;
      const int r = rp >> 5, p = rp & 31;
      const int gy = ty0 + row0 + r, gxx = tx0 + p, c = 8 * run;
      const uint4 x = *reinterpret_cast<const uint4 *>(stage + rp * PSTR + run * 16);
      if (gy < H && gxx < W && c < a1.cout)
        *reinterpret_cast<uint4 *>(out + ((size_t)gy * W + gxx) * a1.cout + c) = x;
    }
  }
}

// 3x3 convolution in float32 by Winograd's minimal filtering F(2x2, 3x3): each
// 2x2 block of output pixels is Y = A^T [sum_c U_c (.) V_c] A with
// V_c = B^T d_c B the transform of the block's 4x4 input patch d_c of channel
// c and U_c = G g_c G^T the transform of the 3x3 filter (computed on the host);
//   B^T = [1 0 -1 0; 0 1 1 0; 0 -1 1 0; 0 1 0 -1],
//   G   = [1 0 0; 1/2 1/2 1/2; 1/2 -1/2 1/2; 0 0 1],
//   A^T = [1 1 1 0; 0 1 -1 -1].
// The channel sum is, for each of the 16 transform positions (xi, nu), a GEMM
// (output channels x blocks, K = input channels) on v_mfma_f32_32x32x2_f32:
// 16 multiplies per block and channel pair instead of 36 for the direct form.
// A tile is 8 rows x 32 columns of output pixels (4 x 16 blocks) x 32 MB output
// channels.  A workgroup has 8 waves; wave w owns transform row xi = w & 3 of
// block rows 2 (w >> 2) and 2 (w >> 2) + 1 (32 blocks, one per lane column)
// and holds the accumulators (xi, nu = 0..3) of MB blocks of 32 channels, so
// with MB = 2 its input fragments feed two MFMA blocks.  Row xi of B^T d
// combines two patch rows, so a wave reads 8 of the 16 patch pixels and
// transforms in registers.  Workgroups are persistent (one per CU) and stream
// the CK-channel chunks of their tiles through two LDS buffers, one barrier
// per chunk.  Epilogue: each wave reduces its row by A (2 values per block and
// channel) into LDS, and every thread then finishes 4 channels of one block:
// the A^T row reduction, bias, ReLU, the 2x2 output block (which is also the
// max-pool window) and the fused 1x1 head.
template <bool HEAD, int MB, int CK>
__global__ __launch_bounds__(512) void wino3x3_kernel(ConvArgs a, int ntx, int nty, int nzc, int ntiles) {
  constexpr int NT = 512, TB = 2;                    // threads; tile blocks of 2 tile rows
  constexpr int NCO = 32 * MB;                       // output channels per workgroup tile
  constexpr int NV = CK / 4;                         // staged channels CK: 16-byte vectors per pixel
  constexpr int TH = 4 * TB, TW = 32, LW = TW + 2, LPix = (TH + 2) * LW;
  // input tile in LDS, in 16-byte units (4 channels): unit of (row, col, vector v)
  // = v PX + (col & 1) PY + row HZ + (col >> 1).  Lanes read the pixels of 16
  // consecutive blocks, 2 columns apart: with even and odd columns in separate
  // planes those are 16 consecutive units, one per bank group.
  constexpr int HZ = LW / 2, PY = (TH + 2) * HZ, PX = 2 * PY;
  constexpr int CS = 16 * CK + 4;                    // LDS floats per output channel of U (+4: bank spread)
  constexpr int INP = NV * PX * 4, BUF = INP + NCO * CS;
  constexpr int PP = NT / NV;                        // pixels / U rows per staging pass
  constexpr int NIN = (LPix + PP - 1) / PP, NWR = NCO * 16 / PP;
  constexpr int ES = 2 * 32 + 4;                     // epilogue floats per tile: 2 columns x 32 channels (+4)
  constexpr int EPL = TB * 4 * 32 * ES;
  // LDS: [buffer 0][GAP][buffer 1]; the epilogue's EPL floats start at the
  // buffer just finished (0 or BUF) and may run into the gap
  constexpr int GAP = EPL > BUF ? EPL - BUF : 0, B1 = BUF + GAP;
  static_assert(NCO * 16 % PP == 0, "U rows must fill whole staging passes");
  __shared__ __attribute__((aligned(16))) float smem[2 * BUF + GAP];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = lane & 31, h = lane >> 5;
  const int xi = wv & 3, tb = wv >> 2;
  const int H = a.H, W = a.W;
  const int Cin = a.C0 + a.C1;

  // Persistent workgroups walk a list of tiles (an 8 x 32 pixel block of one
  // image and one block of NCO output channels).  Tile order: output-channel
  // blocks of one pixel block are consecutive, then pixel blocks, then images;
  // with a grid of 8k workgroups, workgroup w (on XCD w mod 8) walks every
  // k-th tile of the w mod 8 -th eighth of the list, so tiles that share input
  // pixels run on the same XCD at about the same time.
  const int G = gridDim.x;
  int t_first, t_end, t_step;
  if (G % 8 == 0 && G < ntiles) {
    const int x = blockIdx.x & 7, per = G >> 3;
    t_first = (int)((long)x * ntiles / 8) + (blockIdx.x >> 3);
    t_end = (int)((long)(x + 1) * ntiles / 8);
    t_step = per;
  } else {
    t_first = blockIdx.x;
    t_end = ntiles;
    t_step = G;
  }
  struct TileId { int ty0, tx0, co0, bimg; };
  auto decode = [&](int T) {
    TileId d;
    const int cz = T % nzc, sp = T / nzc;
    const int nsp = ntx * nty;
    d.bimg = sp / nsp;
    const int r = sp - d.bimg * nsp;
    d.ty0 = (r / ntx) * TH;
    d.tx0 = (r % ntx) * TW;
    d.co0 = cz * NCO;
    return d;
  };

  // staging plan: this thread moves float4 qv of pixels p0, p0 + PP, ... and of
  // U rows p0, p0 + PP, ... (row r = 16 co + position)
  const int qv = (tid % NV) * 4, p0 = tid / NV;
  int lofs[NIN];
#pragma unroll
  for (int k = 0; k < NIN; ++k) {
    const int pix = p0 + k * PP, row = pix / LW, col = pix % LW;
    lofs[k] = 4 * ((qv / 4) * PX + (col & 1) * PY + row * HZ + (col >> 1));
  }
  // fetch state: the tile whose chunks are being fetched
  int off0[NIN], off1[NIN];
  const float *fin0 = nullptr, *fin1 = nullptr, *wsrc = nullptr;
  auto set_fetch_tile = [&](const TileId &d) {
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
      const int pix = p0 + k * PP, row = pix / LW, col = pix % LW;
      const int gy = d.ty0 - 1 + row, gx = d.tx0 - 1 + col;
      const bool inside = pix < LPix && gy >= 0 && gy < H && gx >= 0 && gx < W;
      off0[k] = inside ? gy * W + gx : -1;
      off1[k] = inside ? (gy >> 1) * (W >> 1) + (gx >> 1) : -1;
    }
    fin0 = static_cast<const float *>(a.in0) + (size_t)d.bimg * a.in0_bs;
    fin1 = a.in1 ? static_cast<const float *>(a.in1) + (size_t)d.bimg * a.in1_bs : nullptr;
    wsrc = a.wu + ((size_t)d.co0 * 16 + p0) * a.cin_pad + qv;
  };
  const size_t wstep = (size_t)PP * a.cin_pad;
  auto fetch_in = [&](int ci, uint4 (&v)[NIN]) {
    const bool from0 = ci < a.C0;
    const size_t csrc = from0 ? a.C0 : a.C1;
    const float *src = (from0 ? fin0 + ci : fin1 + (ci - a.C0)) + qv;
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
      const int o = from0 ? off0[k] : off1[k];
      const uint4 x = *reinterpret_cast<const uint4 *>(src + (size_t)(o < 0 ? 0 : o) * csrc);
      v[k] = o < 0 ? make_uint4(0u, 0u, 0u, 0u) : x;
    }
  };
  auto fetch_w = [&](int ci, uint4 (&v)[NWR]) {
#pragma unroll
    for (int k = 0; k < NWR; ++k) v[k] = *reinterpret_cast<const uint4 *>(wsrc + k * wstep + ci);
  };
  auto store_in = [&](int buf, const uint4 (&v)[NIN]) {
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
      if (!((k + 1) * PP <= LPix || p0 + k * PP < LPix)) continue;
      *reinterpret_cast<uint4 *>(&smem[buf + lofs[k]]) = v[k];
    }
  };
  auto store_w = [&](int buf, const uint4 (&v)[NWR]) {
#pragma unroll
    for (int k = 0; k < NWR; ++k) {
      const int r = p0 + k * PP;
      *reinterpret_cast<uint4 *>(&smem[buf + INP + (r >> 4) * CS + (r & 15) * CK + qv]) = v[k];
    }
  };

  // lane (n, h): block (tr, tc) of the tile, channels 8g + 4h + s of
  // chunk group g at k-step s.  Row xi of B^T d is patch row ra + sg * patch row rb.
  const int tr = 2 * tb + (n >> 4), tc = n & 15;
  const int ra = xi == 0 ? 0 : (xi == 2 ? 2 : 1);
  const int rb = xi == 0 ? 2 : (xi == 1 ? 2 : (xi == 2 ? 1 : 3));
  const float sg = xi == 1 ? 1.f : -1.f;
  const int ioa = 4 * (h * PX + (2 * tr + ra) * HZ + tc);
  const int iob = 4 * (h * PX + (2 * tr + rb) * HZ + tc);
  const int iow = INP + n * CS + 4 * xi * CK + 4 * h;
  // acc[mb][nu]: positions (xi, nu) of output channels co0 + 32 mb + ... of 32 blocks
  floatx16 acc[MB][4];
  auto zero_acc = [&]() {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[mb][v][q] = 0.f;
  };
  auto compute = [&](int buf) {
    const float *pa = smem + buf + ioa, *pb = smem + buf + iob, *pu = smem + buf + iow;
#pragma unroll 1
    for (int g = 0; g < CK / 8; ++g) {
      float4 da[4], db[4], u[MB][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        // column 2 tc + j of vector 2 g + h
        const int o = 4 * (2 * g * PX + (j & 1) * PY + (j >> 1));
        da[j] = *reinterpret_cast<const float4 *>(pa + o);
        db[j] = *reinterpret_cast<const float4 *>(pb + o);
      }
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int v = 0; v < 4; ++v) u[mb][v] = *reinterpret_cast<const float4 *>(pu + mb * 32 * CS + v * CK + 8 * g);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        auto comp = [s](const float4 &f) { return s == 0 ? f.x : (s == 1 ? f.y : (s == 2 ? f.z : f.w)); };
        float r[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) r[j] = fmaf(sg, comp(db[j]), comp(da[j]));
        const float t[4] = {r[0] - r[2], r[1] + r[2], r[2] - r[1], r[1] - r[3]};
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            acc[mb][v] = __builtin_amdgcn_mfma_f32_32x32x2f32(comp(u[mb][v]), t[v], acc[mb][v], 0, 0, 0);
      }
    }
  };

  // ---- epilogue of one tile into E (EPL floats of LDS nobody reads any
  // more), one block of 32 output channels at a time.  Accumulator register
  // 4j + i of acc[mb][nu] holds position (xi, nu) of channel co0 + 32 mb +
  // 8j + 4h + i for block n; each wave reduces nu by A into E, then thread
  // (block et, quad q) reduces xi by A^T for channels c .. c + 3.
  const int q = tid & 7, et = tid >> 3, etb = et >> 5, en = et & 31;
  auto epilogue = [&](float *E, const TileId &d) {
    const int gy0 = d.ty0 + 2 * (2 * etb + (en >> 4)), gx0 = d.tx0 + 2 * (en & 15);
    float *out = a.out ? static_cast<float *>(a.out) + (size_t)d.bimg * a.out_bs : nullptr;
    float *out_pool = a.out_pool ? static_cast<float *>(a.out_pool) + (size_t)d.bimg * a.pool_bs : nullptr;
    float hs[2][2][3];  // head partial sums of this thread's channels
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int col = 0; col < 2; ++col) hs[r][col][0] = hs[r][col][1] = hs[r][col][2] = 0.f;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      if (mb > 0) __syncthreads();  // the previous block's readers are done with E
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float4 p0v, p1v;
        p0v.x = acc[mb][0][4 * j + 0] + acc[mb][1][4 * j + 0] + acc[mb][2][4 * j + 0];
        p0v.y = acc[mb][0][4 * j + 1] + acc[mb][1][4 * j + 1] + acc[mb][2][4 * j + 1];
        p0v.z = acc[mb][0][4 * j + 2] + acc[mb][1][4 * j + 2] + acc[mb][2][4 * j + 2];
        p0v.w = acc[mb][0][4 * j + 3] + acc[mb][1][4 * j + 3] + acc[mb][2][4 * j + 3];
        p1v.x = acc[mb][1][4 * j + 0] - acc[mb][2][4 * j + 0] - acc[mb][3][4 * j + 0];
        p1v.y = acc[mb][1][4 * j + 1] - acc[mb][2][4 * j + 1] - acc[mb][3][4 * j + 1];
        p1v.z = acc[mb][1][4 * j + 2] - acc[mb][2][4 * j + 2] - acc[mb][3][4 * j + 2];
        p1v.w = acc[mb][1][4 * j + 3] - acc[mb][2][4 * j + 3] - acc[mb][3][4 * j + 3];
        float *e = E + ((tb * 4 + xi) * 32 + n) * ES + 8 * j + 4 * h;
        *reinterpret_cast<float4 *>(e) = p0v;
        *reinterpret_cast<float4 *>(e + 32) = p1v;
      }
      __syncthreads();
      const int c = d.co0 + 32 * mb + 4 * q;
      float y[2][2][4];  // [row][column][channel]
#pragma unroll
      for (int col = 0; col < 2; ++col) {
        float4 P[4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
          P[x] = *reinterpret_cast<const float4 *>(E + ((etb * 4 + x) * 32 + en) * ES + col * 32 + 4 * q);
        y[0][col][0] = P[0].x + P[1].x + P[2].x;
        y[0][col][1] = P[0].y + P[1].y + P[2].y;
        y[0][col][2] = P[0].z + P[1].z + P[2].z;
        y[0][col][3] = P[0].w + P[1].w + P[2].w;
        y[1][col][0] = P[1].x - P[2].x - P[3].x;
        y[1][col][1] = P[1].y - P[2].y - P[3].y;
        y[1][col][2] = P[1].z - P[2].z - P[3].z;
        y[1][col][3] = P[1].w - P[2].w - P[3].w;
      }
      const bool live = c < a.cout;
      float4 b = make_float4(0.f, 0.f, 0.f, 0.f);
      if (live) b = *reinterpret_cast<const float4 *>(a.bias + c);
      const float bb[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int col = 0; col < 2; ++col)
#pragma unroll
          for (int i = 0; i < 4; ++i) y[r][col][i] = fmaxf(y[r][col][i] + bb[i], 0.f);
      if constexpr (HEAD) {
        if (live) {
#pragma unroll
          for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int col = 0; col < 2; ++col)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                hs[r][col][0] = fmaf(a.head_w[c + i], y[r][col][i], hs[r][col][0]);
                hs[r][col][1] = fmaf(a.head_w[a.cout + c + i], y[r][col][i], hs[r][col][1]);
                hs[r][col][2] = fmaf(a.head_w[2 * a.cout + c + i], y[r][col][i], hs[r][col][2]);
              }
        }
      } else if (live) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int col = 0; col < 2; ++col) {
            const int gy = gy0 + r, gx = gx0 + col;
            if (gy < H && gx < W)
              *reinterpret_cast<float4 *>(out + ((size_t)gy * W + gx) * a.cout + c) =
                  make_float4(y[r][col][0], y[r][col][1], y[r][col][2], y[r][col][3]);
          }
        if (out_pool && gy0 < H && gx0 < W) {
          float m[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) m[i] = fmaxf(fmaxf(y[0][0][i], y[0][1][i]), fmaxf(y[1][0][i], y[1][1][i]));
          *reinterpret_cast<float4 *>(out_pool + ((size_t)(gy0 >> 1) * (W >> 1) + (gx0 >> 1)) * a.cout + c) =
              make_float4(m[0], m[1], m[2], m[3]);
        }
      }
    }
    if constexpr (HEAD) {
      // the tile holds every output channel (cout <= NCO): sum the head over
      // the block's 8 threads; thread q < 4 writes pixel (q >> 1, q & 1)
      float *head_out =
          a.head_outs ? a.head_outs[d.bimg] : (a.head_out ? a.head_out + (size_t)d.bimg * 3 * H * W : nullptr);
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int col = 0; col < 2; ++col)
#pragma unroll
          for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int m = 1; m < 8; m <<= 1) hs[r][col][k] += __shfl_xor(hs[r][col][k], m, 64);
      if (q < 4) {
        const int r = q >> 1, col = q & 1, gy = gy0 + r, gx = gx0 + col;
        float o0 = hs[0][0][0], o1 = hs[0][0][1], o2 = hs[0][0][2];
#pragma unroll
        for (int rr = 0; rr < 2; ++rr)
#pragma unroll
          for (int cc = 0; cc < 2; ++cc)
            if (rr == r && cc == col) {
              o0 = hs[rr][cc][0];
              o1 = hs[rr][cc][1];
              o2 = hs[rr][cc][2];
            }
        if (gy < H && gx < W) {
          const size_t HW = (size_t)H * W, p = (size_t)gy * W + gx;
          head_out[p] = o0 + a.head_b[0];
          head_out[HW + p] = o1 + a.head_b[1];
          head_out[2 * HW + p] = o2 + a.head_b[2];
        }
      }
    }
  };

  // The chunks of this workgroup's tiles form one stream: chunk step t is
  // multiplied from LDS buffer t & 1 while step t + 1 (the next chunk of the
  // tile, or the first chunk of the next tile) is fetched into registers; it
  // is then written to the other buffer, which every wave finished reading
  // before the previous barrier.  After a tile's last chunk the epilogue runs
  // on the buffer just finished, so the next tile's first chunk is already
  // staged when its multiplications start.
  if (t_first >= t_end) return;
  const int nch = Cin / CK;
  TileId cur = decode(t_first);
  set_fetch_tile(cur);
  {
    uint4 v[NIN], w[NWR];
    fetch_in(0, v);
    fetch_w(0, w);
    store_in(0, v);
    store_w(0, w);
  }
  __syncthreads();
  zero_acc();
  uint4 v[NIN], w[NWR];
  int T = t_first, c = 0, buf = 0;
  for (;;) {
    const bool last = c + 1 == nch;
    const int Tn = last ? T + t_step : T;
    const bool more = Tn < t_end;
    TileId nxt = cur;
    if (more) {
      if (last) {
        nxt = decode(Tn);
        set_fetch_tile(nxt);
      }
      const int cn = last ? 0 : (c + 1) * CK;
      fetch_w(cn, w);
      fetch_in(cn, v);
    } else {
      // (defined values on every path keep the arrays in registers)
#pragma unroll
      for (int k = 0; k < NWR; ++k) w[k] = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
      for (int k = 0; k < NIN; ++k) v[k] = make_uint4(0u, 0u, 0u, 0u);
    }
    compute(buf);  // one call site: the accumulators stay in place
    const int other = buf == 0 ? B1 : 0;
    if (more) {
      store_in(other, v);
      store_w(other, w);
    }
    __syncthreads();
    if (last) {
      epilogue(smem + (buf == 0 ? 0 : BUF), cur);
      if (!more) break;
      __syncthreads();  // E is read before the buffer is staged again
      zero_acc();
      cur = nxt;
      T = Tn;
      c = 0;
    } else {
      ++c;
    }
    buf = other;
  }
}

// RGBDA -> network input x = (r/255, g/255, b/255, A ? D/16 : 0, A, 0...), cpad channels
// GAP: the float32 network's channel order (x0, x1, x2, 0, x3, x4, 0, 0), the
// one its first convolution stages; otherwise (x0, ..., x4, 0, ...)
template <int MODE, bool GAP>
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
  v[GAP ? 4 : 3] = A ? depth[p] * 0.0625f : 0.f;
  v[GAP ? 5 : 4] = A ? 1.f : 0.f;
  if (half_store(MODE)) {  // cpad is 16: two 16-byte stores
    uint4 *o = reinterpret_cast<uint4 *>(static_cast<uint16_t *>(x) + (size_t)p * cpad);
    o[0] = make_uint4(pack16x2<MODE>(v[0], v[1]), pack16x2<MODE>(v[2], v[3]), pack16x2<MODE>(v[4], v[5]),
                      pack16x2<MODE>(v[6], v[7]));
    o[1] = make_uint4(0u, 0u, 0u, 0u);
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
    if (half_store(MODE)) {
      const uint2 q = *reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(x) + (size_t)p * C + c);
      v[0] = unpack16<MODE>(q.x & 0xFFFFu);
      v[1] = unpack16<MODE>(q.x >> 16);
      v[2] = unpack16<MODE>(q.y & 0xFFFFu);
      v[3] = unpack16<MODE>(q.y >> 16);
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

// Tile choice per layer (measured on the 1080p workload).  64-channel
// workgroups with 2 rows per wave where the layer has a multiple of 64 output
// channels; in float32 and bf16, when one image gives fewer than kSmallGrid
// such workgroups (the 135x240 level of a 1080p frame), 32-channel workgroups
// with 2 rows per wave double the grid so the last round of workgroups is not
// nearly empty (split bf16 measured no gain from it; a layer with the fused
// head keeps all its channels in one workgroup).  32-channel layers (the first level)
// use 2 rows per wave, except deep (more than 32 input channels) bf16 layers,
// where 4 rows measured faster.  Float32 stages 16 channels at a time (32
// would not leave room for two workgroups per CU), the bf16 modes up to 32;
// ck is the largest of 32 / 16 / 8 that divides both concatenated inputs.
// The choice depends on one image's shape only, so a frame's output does not
// depend on the batch it is computed in.
constexpr long kSmallGrid = 768;
template <int MODE, int BM, int CK, int R>
hipError_t conv_launch(const ConvArgs &a, int cout_pad, hipStream_t s) {
  dim3 grid((a.W + 31) / 32, (a.H + 4 * R - 1) / (4 * R), (cout_pad / BM) * a.batch);
  if (a.rgbda_depth) {
    // only the network's first layer (one staged chunk of cin0_pad channels)
    if constexpr (CK == ConvTraits<MODE>::kGroup)
      conv3x3_kernel<MODE, BM, CK, R, true><<<grid, 256, 0, s>>>(a);
    else
      return hipErrorInvalidValue;
  } else {
    conv3x3_kernel<MODE, BM, CK, R, false><<<grid, 256, 0, s>>>(a);
  }
  return hipGetLastError();
}

// Float32 layers whose inputs come in chunks of 16 channels (all but the
// first) run as Winograd F(2x2, 3x3) in persistent workgroups, one resident
// per CU (LDS), each walking its share of the 8 x 32 pixel tiles.
template <int MB, int CK>
hipError_t wino_launch_mc(const ConvArgs &a, int cout_pad, bool head, hipStream_t s) {
  const int ntx = (a.W + 31) / 32, nty = (a.H + 7) / 8;
  const int nzc = cout_pad / (32 * MB), ntiles = ntx * nty * nzc * a.batch;
  static std::atomic<int> cus[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  int n = cus[dev].load(std::memory_order_relaxed);
  if (n == 0) {
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      return hipErrorInvalidDevice;
    cus[dev].store(n, std::memory_order_relaxed);
  }
  const int grid = ntiles < n ? ntiles : n;
  if (head)
    wino3x3_kernel<true, MB, CK><<<grid, 512, 0, s>>>(a, ntx, nty, nzc, ntiles);
  else
    wino3x3_kernel<false, MB, CK><<<grid, 512, 0, s>>>(a, ntx, nty, nzc, ntiles);
  return hipGetLastError();
}
// Layers with a multiple of 64 output channels: tiles of 64 channels (each
// wave reuses its input fragments for two MFMA blocks), staged 8 input
// channels at a time (two LDS buffers of U for 64 channels must fit), unless
// one image gives fewer than kSmallGrid such tiles (the 135x240 level of a
// 1080p frame), where 32-channel tiles keep every CU busy; a layer with the
// fused head needs all its channels (at most 64) in one tile.  Others: 32
// channels, 16 input channels at a time.  Both take the same sums in the same
// order, so the choice does not change results.
hipError_t wino_launch(const ConvArgs &a, int cout_pad, bool head, hipStream_t s) {
  const long tiles64 = (long)((a.W + 31) / 32) * ((a.H + 7) / 8) * (cout_pad / 64);
  if (cout_pad % 64 == 0 && (tiles64 >= kSmallGrid || head)) return wino_launch_mc<2, 8>(a, cout_pad, head, s);
  return wino_launch_mc<1, 16>(a, cout_pad, head, s);
}

template <int MODE>
hipError_t conv_dispatch(const ConvArgs &a, int ck, int cout_pad, hipStream_t s) {
  const bool wide = cout_pad % 64 == 0;
  // a fused head sums over every output channel in one workgroup: no 32-channel
  // split of a 64-channel layer then
  const bool head = a.head_out || a.head_outs;
  const bool small = !head && (long)((a.W + 31) / 32) * ((a.H + 7) / 8) * (cout_pad / 64) < kSmallGrid;
  if constexpr (MODE == 0) {
    if (ck == 8) return wide ? conv_launch<0, 64, 8, 2>(a, cout_pad, s) : conv_launch<0, 32, 8, 2>(a, cout_pad, s);
    return (wide && !small) ? conv_launch<0, 64, 16, 2>(a, cout_pad, s) : conv_launch<0, 32, 16, 2>(a, cout_pad, s);
  } else if constexpr (MODE == 2 || MODE == 5) {
    if (ck < 16) return hipErrorInvalidValue;
    if (wide) return conv_launch<MODE, 64, 16, 2>(a, cout_pad, s);
    return conv_launch<MODE, 32, 16, 2>(a, cout_pad, s);
  } else {
    if (ck < 16) return hipErrorInvalidValue;
    if (wide && !small)
      return ck == 32 ? conv_launch<MODE, 64, 32, 2>(a, cout_pad, s) : conv_launch<MODE, 64, 16, 2>(a, cout_pad, s);
    if (wide)  // small grid: 32-channel workgroups, 2 rows per wave
      return ck == 32 ? conv_launch<MODE, 32, 32, 2>(a, cout_pad, s) : conv_launch<MODE, 32, 16, 2>(a, cout_pad, s);
    if (a.C0 + a.C1 > 32)
      return ck == 32 ? conv_launch<MODE, 32, 32, 4>(a, cout_pad, s) : conv_launch<MODE, 32, 16, 4>(a, cout_pad, s);
    // the layer with the fused head: 16-channel chunks measured faster (the same sums in the same order)
    return ck == 32 && !head ? conv_launch<MODE, 32, 32, 2>(a, cout_pad, s)
                             : conv_launch<MODE, 32, 16, 2>(a, cout_pad, s);
  }
}

}  // namespace

hipError_t launch_pack_input(const float *depth, const uint32_t *rgba, int H, int W, int cpad, Prec p, void *x,
                             hipStream_t s) {
  const int npix = H * W;
  const int nb = (npix + 255) / 256;
  if (p == Prec::BF16)
    pack_kernel<1, false><<<nb, 256, 0, s>>>(depth, rgba, npix, cpad, x);
  else if (p == Prec::FP16 || p == Prec::FP8 || p == Prec::FP8X3)  // float16 activations
    pack_kernel<3, false><<<nb, 256, 0, s>>>(depth, rgba, npix, cpad, x);
  else if (p == Prec::F32)
    pack_kernel<0, true><<<nb, 256, 0, s>>>(depth, rgba, npix, cpad, x);
  else
    pack_kernel<0, false><<<nb, 256, 0, s>>>(depth, rgba, npix, cpad, x);
  return hipGetLastError();
}

hipError_t launch_conv3x3(const ConvCall &c, Prec p, hipStream_t s) {
  const ConvLayer &L = *c.layer;
  ConvArgs a{c.in0, c.in1, c.C0, c.C1, c.H, c.W, L.w, L.w_lo, L.bias, L.cout, L.cin_pad, c.out, c.out_pool,
             c.head_w, c.head_b, c.head_out, c.batch < 1 ? 1 : c.batch, c.in0_bs, c.in1_bs, c.out_bs, c.pool_bs,
             c.head_outs, c.rgbda_depth, c.rgbda_rgba, static_cast<const float *>(L.wu), L.wscale};
  const bool head = c.head_out || c.head_outs;
  if (head && (L.cout_pad > 64 || c.out_pool)) return hipErrorInvalidValue;
  if (c.rgbda_depth && (!c.rgbda_rgba || c.C1 != 0 || c.batch > 1)) return hipErrorInvalidValue;
  const int step = (p == Prec::F32) ? 8 : 16;
  int ck = 32;
  while (ck > step && ((c.C0 % ck) != 0 || (c.C1 % ck) != 0)) ck >>= 1;
  if ((c.C0 % ck) != 0 || (c.C1 % ck) != 0 || (c.C0 + c.C1) != L.cin_pad) return hipErrorInvalidValue;
  if (p == Prec::F32 && L.wu && !c.rgbda_depth && c.C0 % 16 == 0 && c.C1 % 16 == 0 &&
      (!head || L.cout_pad <= 64))
    return wino_launch(a, L.cout_pad, head, s);
  switch (p) {
    case Prec::F32: return conv_dispatch<0>(a, ck, L.cout_pad, s);
    case Prec::BF16: return conv_dispatch<1>(a, ck, L.cout_pad, s);
    case Prec::BF16X3: return conv_dispatch<2>(a, ck, L.cout_pad, s);
    case Prec::FP16: return conv_dispatch<3>(a, ck, L.cout_pad, s);
    case Prec::FP8: return L.wscale ? conv_dispatch<4>(a, ck, L.cout_pad, s) : hipErrorInvalidValue;
    case Prec::FP8X3: return L.wscale && L.w_lo ? conv_dispatch<5>(a, ck, L.cout_pad, s) : hipErrorInvalidValue;
    default: break;
  }
  return hipErrorInvalidValue;
}

bool enc0_fusable(const ConvLayer &l0, const ConvLayer &l1, Prec p) {
  return (p == Prec::BF16 || p == Prec::FP16) && l0.cin_pad == 16 && l0.cout_pad == 32 && l1.cout_pad == 32 &&
         l1.cin == l0.cout && l1.cin_pad == l1.cin && (l1.cin_pad == 16 || l1.cin_pad == 32);
}

hipError_t launch_enc0_fused(const ConvCall &c0, const ConvCall &c1, Prec p, hipStream_t s) {
  const ConvLayer &L0 = *c0.layer, &L1 = *c1.layer;
  if (!enc0_fusable(L0, L1, p) || !c1.out || !c1.out_pool || c1.head_out || c1.head_outs || c0.C1 || c1.C1 ||
      c0.H != c1.H || c0.W != c1.W || c0.batch != c1.batch || (c0.rgbda_depth && (!c0.rgbda_rgba || c0.batch > 1)) ||
      (!c0.rgbda_depth && c0.C0 != 16) || c1.C0 != L1.cin_pad)
    return hipErrorInvalidValue;
  const int batch = c0.batch < 1 ? 1 : c0.batch;
  ConvArgs a0{c0.in0, nullptr, c0.C0, 0, c0.H, c0.W, L0.w, nullptr, L0.bias, L0.cout, L0.cin_pad, nullptr, nullptr,
              nullptr, nullptr, nullptr, batch, c0.in0_bs, 0, 0, 0, nullptr, c0.rgbda_depth, c0.rgbda_rgba,
              nullptr, nullptr};
  ConvArgs a1{nullptr, nullptr, c1.C0, 0, c1.H, c1.W, L1.w, nullptr, L1.bias, L1.cout, L1.cin_pad, c1.out,
              c1.out_pool, nullptr, nullptr, nullptr, batch, 0, 0, c1.out_bs, c1.pool_bs, nullptr, nullptr, nullptr,
              nullptr, nullptr};
  const dim3 grid((c1.W + 31) / 32, (c1.H + 7) / 8, batch);
  const bool rgbda = c0.rgbda_depth != nullptr;
#define LNR_ENC0(M, CK, RG) enc0_fused_kernel<M, CK, RG><<<grid, 256, 0, s>>>(a0, a1)
  if (p == Prec::FP16) {
    if (L1.cin_pad == 32) { if (rgbda) LNR_ENC0(3, 32, true); else LNR_ENC0(3, 32, false); }
    else { if (rgbda) LNR_ENC0(3, 16, true); else LNR_ENC0(3, 16, false); }
  } else {
    if (L1.cin_pad == 32) { if (rgbda) LNR_ENC0(1, 32, true); else LNR_ENC0(1, 32, false); }
    else { if (rgbda) LNR_ENC0(1, 16, true); else LNR_ENC0(1, 16, false); }
  }
#undef LNR_ENC0
  return hipGetLastError();
}

hipError_t launch_head(const void *x, int C, int H, int W, const ConvLayer &head, Prec p, float *out, hipStream_t s) {
  const int npix = H * W;
  const int nb = (npix + 255) / 256;
  const float *w = static_cast<const float *>(head.w);
  if (p == Prec::BF16)
    head_kernel<1><<<nb, 256, 0, s>>>(x, C, npix, w, head.bias, out);
  else if (p == Prec::FP16 || p == Prec::FP8 || p == Prec::FP8X3)  // float16 activations
    head_kernel<3><<<nb, 256, 0, s>>>(x, C, npix, w, head.bias, out);
  else
    head_kernel<0><<<nb, 256, 0, s>>>(x, C, npix, w, head.bias, out);
  return hipGetLastError();
}

}  // namespace lnr
