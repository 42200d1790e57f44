// Host runtime behind the C ABI declared in include/lnr.h: argument checks,
// device memory and budget accounting, weight repacking, and the enqueueing
// of the HIP kernels that make up each stage.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <deque>
#include <map>
#include <tuple>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "lnr_internal.h"

using namespace lnr;

namespace {

struct Buf {
  void *p = nullptr;
  size_t cap = 0;
};

thread_local std::string g_create_error;

// device scratch reused by consecutive calls on one stream
struct Scratch {
  Buf flags, chunks, counters, pyramid, act, soft_acc;
  Buf recs, segs, sorted, tile_nseg, tile_off, tile_units, units;  // tiled splat
  Buf views;                                                         // multi-view work items
};

}  // namespace

struct lnr_context {
  int device = 0;
  uint64_t budget = 0;
  uint64_t allocated = 0;
  std::string err;
  hipStream_t last_stream = nullptr;
  bool rendered = false;
  bool counted = false;  // the last render counted its z-buffer atomics
  uint32_t last_cells = 0;
  Scratch sc;
  // kernel timing
  struct Rec {
    const char *name;
    hipEvent_t a, b;
  };
  bool profiling = false;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> event_pool;
  // clouds, networks and servers created through this context; the context
  // is freed when it has been destroyed and the last of them is gone, so the
  // caller may destroy objects in any order
  int children = 0;
  bool closed = false;
  // lnr_debug_fail_allocation: device allocations left before one fails (-1: none)
  int64_t fail_alloc_after = -1;
  // device address of this device's allocation-free filter scratch (null if
  // the lookup failed; noalloc_error then says why)
  float *noalloc_scratch = nullptr;
  std::string noalloc_error;
};

struct lnr_cloud {
  lnr_context *ctx = nullptr;
  CloudDev d;
  std::vector<std::pair<void *, size_t>> allocs;
};

struct lnr_unet {
  lnr_context *ctx = nullptr;
  Prec prec = Prec::F32;
  int L = 0;
  int widths[6] = {0, 0, 0, 0, 0, 0};
  int cin0_pad = 8;
  std::vector<ConvLayer> convs;  // 4L - 2 3x3 convolutions in network order
  ConvLayer head;
  std::vector<std::pair<void *, size_t>> allocs;
};

namespace {

lnr_status fail(lnr_context *ctx, lnr_status st, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return st;
}

lnr_status hip_fail(lnr_context *ctx, hipError_t e, const char *what) {
  return fail(ctx, LNR_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define LNR_HIP(ctx, expr)                                 \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
  } while (0)

hipEvent_t get_event(lnr_context *ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Enqueue one launcher; with timing enabled, bracket it by events on the same stream.
// The runtime's last-error slot is cleared first: launchers report it after
// their launches, and an error left there by an unrelated earlier runtime call
// on this thread must not be blamed on this kernel.
#define LNR_LAUNCH(ctx, nm, s, expr)                                            \
  do {                                                                          \
    (void)hipGetLastError();                                                    \
    hipEvent_t a_ = nullptr, b_ = nullptr;                                      \
    if ((ctx)->profiling) {                                                     \
      a_ = get_event(ctx);                                                      \
      b_ = get_event(ctx);                                                      \
      if (a_) (void)hipEventRecord(a_, s);                                      \
    }                                                                           \
    hipError_t e_ = (expr);                                                     \
    if (a_ && b_) {                                                             \
      (void)hipEventRecord(b_, s);                                              \
      (ctx)->recs.push_back({nm, a_, b_});                                      \
    }                                                                           \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, nm);                         \
  } while (0)

const char *const kConvNames[2][6][2] = {
    {{"conv/enc0a", "conv/enc0b"}, {"conv/enc1a", "conv/enc1b"}, {"conv/enc2a", "conv/enc2b"},
     {"conv/enc3a", "conv/enc3b"}, {"conv/enc4a", "conv/enc4b"}, {"conv/enc5a", "conv/enc5b"}},
    {{"conv/dec0a", "conv/dec0b"}, {"conv/dec1a", "conv/dec1b"}, {"conv/dec2a", "conv/dec2b"},
     {"conv/dec3a", "conv/dec3b"}, {"conv/dec4a", "conv/dec4b"}, {"conv/dec5a", "conv/dec5b"}}};

lnr_status dalloc(lnr_context *ctx, void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  if (ctx->fail_alloc_after >= 0 && ctx->fail_alloc_after-- == 0)
    return fail(ctx, LNR_E_OUT_OF_MEMORY, "hipMalloc(" + std::to_string(bytes) + ") failed: injected failure");
  if (ctx->budget && ctx->allocated + bytes > ctx->budget)
    return fail(ctx, LNR_E_BUDGET,
                "allocation of " + std::to_string(bytes) + " bytes exceeds the context budget of " +
                    std::to_string(ctx->budget) + " bytes (" + std::to_string(ctx->allocated) + " in use)");
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(ctx, LNR_E_OUT_OF_MEMORY, "hipMalloc(" + std::to_string(bytes) + ") failed: " + hipGetErrorString(e));
  }
  ctx->allocated += bytes;
  return LNR_OK;
}

void dfree(lnr_context *ctx, void *p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  if (bytes == 0) bytes = 256;
  ctx->allocated -= std::min<uint64_t>(ctx->allocated, bytes);
}

// grow-only scratch; an old buffer is released only after the device is idle
lnr_status ensure(lnr_context *ctx, Buf &b, size_t bytes) {
  if (b.cap >= bytes && b.p) return LNR_OK;
  if (b.p) {
    LNR_HIP(ctx, hipDeviceSynchronize());
    dfree(ctx, b.p, b.cap);
    b.p = nullptr;
    b.cap = 0;
  }
  lnr_status st = dalloc(ctx, &b.p, bytes);
  if (st == LNR_OK) b.cap = bytes;
  return st;
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

lnr_status use_device(lnr_context *ctx) {
  LNR_HIP(ctx, hipSetDevice(ctx->device));
  return LNR_OK;
}

template <typename T>
lnr_status cloud_alloc(lnr_cloud *c, T **p, size_t count) {
  void *v = nullptr;
  lnr_status st = dalloc(c->ctx, &v, count * sizeof(T));
  if (st != LNR_OK) return st;
  c->allocs.emplace_back(v, count * sizeof(T) ? count * sizeof(T) : 256);
  *p = static_cast<T *>(v);
  return LNR_OK;
}

void cloud_free(lnr_cloud *c) {
  for (auto &a : c->allocs) dfree(c->ctx, a.first, a.second);
  c->allocs.clear();
}

struct TempAllocs {
  lnr_context *ctx;
  std::vector<std::pair<void *, size_t>> v;
  explicit TempAllocs(lnr_context *c) : ctx(c) {}
  ~TempAllocs() {
    for (auto &a : v) dfree(ctx, a.first, a.second);
  }
  template <typename T>
  lnr_status get(T **p, size_t bytes) {
    void *q = nullptr;
    lnr_status st = dalloc(ctx, &q, bytes);
    if (st != LNR_OK) return st;
    v.emplace_back(q, bytes ? bytes : 256);
    *p = static_cast<T *>(q);
    return LNR_OK;
  }
};

bool camera_ok(const lnr_camera *cam, std::string *why) {
  for (int i = 0; i < 12; ++i)
    if (!std::isfinite(cam->P[i])) {
      *why = "camera P must be finite";
      return false;
    }
  if (cam->width < 1 || cam->height < 1 || cam->width > 16384 || cam->height > 16384) {
    *why = "camera width/height must be in [1, 16384]";
    return false;
  }
  if (!(std::isfinite(cam->z_near) && std::isfinite(cam->z_far) && cam->z_near > 0.f && cam->z_near < cam->z_far)) {
    *why = "camera needs finite 0 < z_near < z_far";
    return false;
  }
  return true;
}

// Frustum half-spaces of the per-point test, in double, in a fixed order of
// operations (the order defines the exact cull decision).
CullParams make_cull_params(const lnr_camera *cam, bool no_cull) {
  CullParams p{};
  double P[3][4];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 4; ++k) P[r][k] = (double)cam->P[4 * r + k];
  const double *a = P[0], *b = P[1], *w = P[2];
  const double n64 = (double)cam->z_near, f64 = (double)cam->z_far;
  const double Wd = (double)cam->width, Hd = (double)cam->height;
  const double hs[6][4] = {
      {w[0], w[1], w[2], w[3] - n64},
      {-w[0], -w[1], -w[2], f64 - w[3]},
      {a[0], a[1], a[2], a[3]},
      {Wd * w[0] - a[0], Wd * w[1] - a[1], Wd * w[2] - a[2], Wd * w[3] - a[3]},
      {b[0], b[1], b[2], b[3]},
      {Hd * w[0] - b[0], Hd * w[1] - b[1], Hd * w[2] - b[2], Hd * w[3] - b[3]},
  };
  std::memcpy(p.hs, hs, sizeof(hs));
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 4; ++k) p.absP[r][k] = std::fabs(P[r][k]);
  p.wh1 = (Wd + Hd) + 1.0;
  for (int k = 0; k < 4; ++k) p.wrow[k] = w[k];
  p.z_near = n64;
  p.no_cull = no_cull ? 1 : 0;
  return p;
}

uint16_t host_f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float host_bf2f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
// float32 -> IEEE binary16, round to nearest even (the compiler's conversion)
uint16_t host_f2h(float f) {
  const _Float16 h = (_Float16)f;
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}

// OCP 8-bit e4m3 (sign, 4 exponent bits with bias 7, 3 fraction bits; no
// infinities; the largest finite value 448 = 1.75 * 2^8; subnormals m * 2^-9):
// round to nearest, ties to even, saturating at +-448 (the device's
// v_cvt_pk_fp8_f32 rounds the same way)
uint8_t host_e4m3(double x) {
  const uint8_t sgn = std::signbit(x) ? 0x80 : 0x00;
  const double a = std::fabs(x);
  if (!(a < 464.0)) return sgn | 0x7E;  // beyond the half-way point above 448 (and NaN) saturate
  if (a < 0x1p-6) return sgn | (uint8_t)std::nearbyint(a * 512.0);  // 8 = the smallest normal, 0x08
  int e = std::ilogb(a);
  double m = std::nearbyint((std::ldexp(a, -e) - 1.0) * 8.0);
  if (m == 8.0) {
    m = 0.0;
    ++e;
  }
  if (e + 7 > 15 || (e + 7 == 15 && m > 6.0)) return sgn | 0x7E;
  return sgn | (uint8_t)((e + 7) << 3) | (uint8_t)m;
}
double host_e4m3_value(uint8_t v) {
  const int E = (v >> 3) & 15, m = v & 7;
  const double a = E == 0 ? m * 0x1p-9 : (1.0 + m / 8.0) * std::ldexp(1.0, E - 7);
  return (v & 0x80) ? -a : a;
}


// ---------------------------------------------------------------------------
// U-Net activation layout for a batch of B same-shape images, and its launches
// ---------------------------------------------------------------------------
struct UNetLayout {
  int H = 0, W = 0, B = 1;
  size_t es = 4;  // bytes per activation element
  size_t x0_off = 0, x0_bs = 0;
  size_t t_off[6] = {}, s_off[6] = {}, p_off[6] = {}, d_off[6] = {};
  size_t act_bs[6] = {}, pool_bs[6] = {};  // per-image elements at level l (w_l and w_{l-1} channels)
  size_t bytes = 0;
};

UNetLayout unet_layout(const lnr_unet *u, int H, int W, int B) {
  UNetLayout y;
  y.H = H;
  y.W = W;
  y.B = B;
  y.es = prec_half(u->prec) ? 2 : 4;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  size_t off = 0;
  y.x0_bs = (size_t)H * W * u->cin0_pad;
  y.x0_off = off;
  off += al(y.x0_bs * B * y.es);
  for (int l = 0; l < u->L; ++l) {
    const size_t px = (size_t)(H >> l) * (W >> l);
    y.act_bs[l] = px * u->widths[l];
    y.pool_bs[l] = (l > 0) ? px * u->widths[l - 1] : 0;
    y.t_off[l] = off;
    off += al(y.act_bs[l] * B * y.es);
    y.s_off[l] = off;
    off += al(y.act_bs[l] * B * y.es);
    y.d_off[l] = off;
    off += al(y.act_bs[l] * B * y.es);
    y.p_off[l] = off;
    off += al(y.pool_bs[l] * B * y.es);
  }
  y.bytes = off;
  return y;
}

lnr_status unet_pack(lnr_context *ctx, Scratch &sc, const lnr_unet *u, const UNetLayout &y, int b, const float *depth,
                     const uint32_t *rgba, hipStream_t s) {
  char *x0 = static_cast<char *>(sc.act.p) + y.x0_off + (size_t)b * y.x0_bs * y.es;
  LNR_LAUNCH(ctx, "pack", s, launch_pack_input(depth, rgba, y.H, y.W, u->cin0_pad, u->prec, x0, s));
  return LNR_OK;
}

// All 3x3 convolutions of the network over the batch; the 1x1 head is fused
// into the last one when widths[0] <= 64 (outputs: head_outs_dev[b] if given,
// else rgb_out + b * 3*H*W), otherwise it runs as its own kernel per image.
lnr_status unet_convs(lnr_context *ctx, Scratch &sc, const lnr_unet *u, const UNetLayout &y, float *rgb_out,
                      float *const *head_outs_dev, hipStream_t s, const float *rgbda_depth = nullptr,
                      const uint32_t *rgbda_rgba = nullptr) {
  char *base = static_cast<char *>(sc.act.p);
  const int L = u->L, B = y.B;
  const bool fuse_head = u->widths[0] <= 64;
  if (!fuse_head && head_outs_dev) return fail(ctx, LNR_E_UNSUPPORTED, "batched outputs need widths[0] <= 64");
  int li = 0;
  for (int l = 0; l < L; ++l) {
    const int Hl = y.H >> l, Wl = y.W >> l;
    ConvCall a{};
    a.in0 = (l == 0) ? (const void *)(base + y.x0_off) : (const void *)(base + y.p_off[l]);
    a.C0 = (l == 0) ? u->cin0_pad : u->widths[l - 1];
    a.in0_bs = (l == 0) ? y.x0_bs : y.pool_bs[l];
    a.in1 = nullptr;
    a.C1 = 0;
    a.H = Hl;
    a.W = Wl;
    a.layer = &u->convs[li];
    a.out = base + y.t_off[l];
    a.out_bs = y.act_bs[l];
    a.batch = B;
    if (l == 0 && rgbda_depth) {
      a.rgbda_depth = rgbda_depth;
      a.rgbda_rgba = rgbda_rgba;
    }
    ConvCall c{};
    c.in0 = base + y.t_off[l];
    c.C0 = u->widths[l];
    c.in0_bs = y.act_bs[l];
    c.H = Hl;
    c.W = Wl;
    c.layer = &u->convs[li + 1];
    c.out = base + y.s_off[l];
    c.out_bs = y.act_bs[l];
    c.out_pool = (l < L - 1) ? (void *)(base + y.p_off[l + 1]) : nullptr;
    c.pool_bs = (l < L - 1) ? y.pool_bs[l + 1] : 0;
    c.batch = B;
    if (L == 1 && fuse_head) {
      c.head_w = static_cast<const float *>(u->head.w);
      c.head_b = u->head.bias;
      c.head_out = rgb_out;
      c.head_outs = head_outs_dev;
    }
    li += 2;
    if (l == 0 && L > 1 && enc0_fusable(*a.layer, *c.layer, u->prec)) {
      // both first-level convolutions in one launch; its time is reported as conv/enc0
      LNR_LAUNCH(ctx, "conv/enc0", s, launch_enc0_fused(a, c, u->prec, s));
      continue;
    }
    LNR_LAUNCH(ctx, kConvNames[0][l][0], s, launch_conv3x3(a, u->prec, s));
    LNR_LAUNCH(ctx, kConvNames[0][l][1], s, launch_conv3x3(c, u->prec, s));
  }
  for (int l = L - 2; l >= 0; --l) {
    const int Hl = y.H >> l, Wl = y.W >> l;
    ConvCall a{};
    a.in0 = base + y.s_off[l];
    a.C0 = u->widths[l];
    a.in0_bs = y.act_bs[l];
    a.in1 = (l == L - 2) ? (const void *)(base + y.s_off[L - 1]) : (const void *)(base + y.d_off[l + 1]);
    a.C1 = u->widths[l + 1];
    a.in1_bs = y.act_bs[l + 1];
    a.H = Hl;
    a.W = Wl;
    a.layer = &u->convs[li++];
    a.out = base + y.t_off[l];
    a.out_bs = y.act_bs[l];
    a.batch = B;
    LNR_LAUNCH(ctx, kConvNames[1][l][0], s, launch_conv3x3(a, u->prec, s));
    ConvCall c{};
    c.in0 = base + y.t_off[l];
    c.C0 = u->widths[l];
    c.in0_bs = y.act_bs[l];
    c.H = Hl;
    c.W = Wl;
    c.layer = &u->convs[li++];
    c.out = base + y.d_off[l];
    c.out_bs = y.act_bs[l];
    c.batch = B;
    if (l == 0 && fuse_head) {
      c.head_w = static_cast<const float *>(u->head.w);
      c.head_b = u->head.bias;
      c.head_out = rgb_out;
      c.head_outs = head_outs_dev;
    }
    LNR_LAUNCH(ctx, kConvNames[1][l][1], s, launch_conv3x3(c, u->prec, s));
  }
  if (!fuse_head) {
    const size_t off = (L == 1) ? y.s_off[0] : y.d_off[0];
    for (int b = 0; b < B; ++b)
      LNR_LAUNCH(ctx, "head", s,
                 launch_head(base + off + (size_t)b * y.act_bs[0] * y.es, u->widths[0], y.H, y.W, u->head, u->prec,
                             rgb_out + (size_t)b * 3 * y.H * y.W, s));
  }
  return LNR_OK;
}

}  // namespace

extern "C" {

lnr_status lnr_context_create(int hip_device, uint64_t hbm_budget_bytes, lnr_context **out) {
  if (!out) {
    g_create_error = "out is NULL";
    return LNR_E_INVALID_ARG;
  }
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0) {
    g_create_error = std::string("no HIP device available: ") + hipGetErrorString(e);
    return LNR_E_DEVICE;
  }
  if (hip_device < 0 || hip_device >= count) {
    g_create_error = "hip_device out of range";
    return LNR_E_INVALID_ARG;
  }
  e = hipSetDevice(hip_device);
  if (e != hipSuccess) {
    g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
    return LNR_E_DEVICE;
  }
  auto *ctx = new (std::nothrow) lnr_context;
  if (!ctx) {
    g_create_error = "out of host memory";
    return LNR_E_OUT_OF_MEMORY;
  }
  ctx->device = hip_device;
  ctx->budget = hbm_budget_bytes;
  // the allocation-free filter's scratch: look its address up once per
  // device, with that device current, and keep it
  {
    static std::mutex mu;
    static std::map<int, std::pair<float *, hipError_t>> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(hip_device);
    if (it == addr.end()) {
      float *ptr = nullptr;
      hipError_t ge = noalloc_scratch_address(&ptr);
      if (ge != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
      }
      it = addr.emplace(hip_device, std::make_pair(ptr, ge)).first;
    }
    ctx->noalloc_scratch = it->second.first;
    if (it->second.second != hipSuccess)
      ctx->noalloc_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(it->second.second);
  }
  *out = ctx;
  return LNR_OK;
}

namespace {
void context_free(lnr_context *ctx) {
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (Buf *b : {&ctx->sc.flags, &ctx->sc.chunks, &ctx->sc.counters, &ctx->sc.pyramid, &ctx->sc.act, &ctx->sc.soft_acc,
                 &ctx->sc.recs, &ctx->sc.segs, &ctx->sc.sorted, &ctx->sc.tile_nseg, &ctx->sc.tile_off,
                 &ctx->sc.tile_units, &ctx->sc.units, &ctx->sc.views})
    dfree(ctx, b->p, b->cap);
  for (auto &r : ctx->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  delete ctx;
  (void)hipGetLastError();  // nothing above may leave an error pending for the caller's next call
}

void context_release(lnr_context *ctx) {
  if (--ctx->children == 0 && ctx->closed) context_free(ctx);
}
}  // namespace

void lnr_context_destroy(lnr_context *ctx) {
  if (!ctx) return;
  ctx->closed = true;
  if (ctx->children == 0) context_free(ctx);
}

const char *lnr_last_error(const lnr_context *ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

uint64_t lnr_allocated_bytes(const lnr_context *ctx) { return ctx ? ctx->allocated : 0; }

// ---------------------------------------------------------------------------
// cloud
// ---------------------------------------------------------------------------
static lnr_status cloud_build(lnr_context *ctx, lnr_cloud *c, const float *xyz_host, const uint8_t *rgb_host,
                              uint32_t N, float cell_size);

lnr_status lnr_cloud_load(lnr_context *ctx, const float *xyz_host, const uint8_t *rgb_host, uint64_t n,
                          float cell_size, lnr_cloud **out) {
  if (!ctx) return LNR_E_INVALID_ARG;
  if (!xyz_host || !rgb_host || !out) return fail(ctx, LNR_E_INVALID_ARG, "NULL pointer argument");
  *out = nullptr;
  if (n < 1 || n >= (1ull << 32)) return fail(ctx, LNR_E_INVALID_ARG, "n must be in [1, 2^32)");
  if (!(std::isfinite(cell_size) && cell_size > 0.f))
    return fail(ctx, LNR_E_INVALID_ARG, "cell_size must be finite and > 0");
  lnr_status st = use_device(ctx);
  if (st != LNR_OK) return st;
  std::unique_ptr<lnr_cloud> c(new lnr_cloud);
  c->ctx = ctx;
  st = cloud_build(ctx, c.get(), xyz_host, rgb_host, (uint32_t)n, cell_size);
  if (st != LNR_OK) {
    (void)hipDeviceSynchronize();
    cloud_free(c.get());
    return st;
  }
  ++ctx->children;
  *out = c.release();
  return LNR_OK;
}

static lnr_status cloud_build(lnr_context *ctx, lnr_cloud *cl, const float *xyz_host, const uint8_t *rgb_host,
                              uint32_t N, float cell_size) {
  lnr_cloud *c = cl;
  lnr_status st;
  hipStream_t s = nullptr;
  TempAllocs tmp(ctx);
  float *d_xyz;
  uint8_t *d_rgb;
  if ((st = tmp.get(&d_xyz, 12ull * N)) != LNR_OK) return st;
  if ((st = tmp.get(&d_rgb, 3ull * N)) != LNR_OK) return st;
  LNR_HIP(ctx, hipMemcpy(d_xyz, xyz_host, 12ull * N, hipMemcpyHostToDevice));
  LNR_HIP(ctx, hipMemcpy(d_rgb, rgb_host, 3ull * N, hipMemcpyHostToDevice));

  // bounding box + finiteness
  const uint32_t nb = bbox_blocks(N);
  float *d_part;
  if ((st = tmp.get(&d_part, 7ull * nb * 4)) != LNR_OK) return st;
  (void)hipGetLastError();  // a pending error from an unrelated earlier call is not ours
  LNR_HIP(ctx, launch_bbox(d_xyz, N, d_part, nb, s));
  std::vector<float> part(7ull * nb);
  LNR_HIP(ctx, hipMemcpy(part.data(), d_part, part.size() * 4, hipMemcpyDeviceToHost));
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (uint32_t b = 0; b < nb; ++b) {
    if (part[7 * b + 6] != 0.f) return fail(ctx, LNR_E_INVALID_ARG, "xyz contains non-finite values");
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], part[7 * b + a]);
      hi[a] = std::max(hi[a], part[7 * b + 3 + a]);
    }
  }
  const double s64 = (double)cell_size;
  uint64_t C = 1;
  for (int a = 0; a < 3; ++a) {
    const double ext = (double)hi[a] - (double)lo[a];
    const double na = std::max(1.0, std::ceil(ext / s64));
    if (na > 2147483648.0) return fail(ctx, LNR_E_INVALID_ARG, "grid has more than 2^31 cells");
    c->d.dims[a] = (int32_t)na;
    C *= (uint64_t)na;
    if (C > (1ull << 31)) return fail(ctx, LNR_E_INVALID_ARG, "grid has more than 2^31 cells");
    c->d.origin[a] = lo[a];
  }
  c->d.n = N;
  c->d.n_cells = (uint32_t)C;
  c->d.cell_size = cell_size;

  // cell ids, stable sort by cell
  uint32_t *keys, *vals, *keys_alt, *vals_alt;
  void *sort_scratch;
  if ((st = tmp.get(&keys, 4ull * N)) != LNR_OK) return st;
  if ((st = tmp.get(&keys_alt, 4ull * N)) != LNR_OK) return st;
  if ((st = tmp.get(&vals_alt, 4ull * N)) != LNR_OK) return st;
  if ((st = tmp.get(&sort_scratch, radix_sort_scratch_bytes(N))) != LNR_OK) return st;
  if ((st = cloud_alloc(c, &vals, N)) != LNR_OK) return st;  // becomes perm (may swap below)
  const double lo64[3] = {(double)lo[0], (double)lo[1], (double)lo[2]};
  LNR_HIP(ctx, launch_cell_ids(d_xyz, N, lo64, s64, c->d.dims, keys, s));
  LNR_HIP(ctx, launch_iota(vals, N, s));
  int bits = 0;
  while (bits < 32 && ((uint64_t)(C - 1) >> bits) != 0) ++bits;
  uint32_t *k_sorted = keys, *v_sorted = vals, *k_alt = keys_alt, *v_alt = vals_alt;
  LNR_HIP(ctx, radix_sort_pairs(&k_sorted, &v_sorted, &k_alt, &v_alt, N, bits, sort_scratch, s));
  if (v_sorted != vals) {
    // the sorted permutation ended in the temporary buffer: copy it into the cloud's buffer
    LNR_HIP(ctx, hipMemcpyAsync(vals, v_sorted, 4ull * N, hipMemcpyDeviceToDevice, s));
  }
  c->d.perm = vals;

  if ((st = cloud_alloc(c, &c->d.cell_start, (size_t)C + 1)) != LNR_OK) return st;
  LNR_HIP(ctx, launch_cell_bounds(k_sorted, N, (uint32_t)C, c->d.cell_start, s));
  if ((st = cloud_alloc(c, &c->d.x, N)) != LNR_OK) return st;
  if ((st = cloud_alloc(c, &c->d.y, N)) != LNR_OK) return st;
  if ((st = cloud_alloc(c, &c->d.z, N)) != LNR_OK) return st;
  if ((st = cloud_alloc(c, &c->d.rgbx, N)) != LNR_OK) return st;
  LNR_HIP(ctx, launch_gather_points(d_xyz, d_rgb, c->d.perm, N, c->d.x, c->d.y, c->d.z, c->d.rgbx, s));
  if ((st = cloud_alloc(c, &c->d.aabb, 6 * (size_t)C)) != LNR_OK) return st;
  LNR_HIP(ctx, launch_cell_aabb(c->d.x, c->d.y, c->d.z, c->d.cell_start, (uint32_t)C, c->d.aabb, s));
  uint32_t *d_total;
  if ((st = tmp.get(&d_total, 256)) != LNR_OK) return st;
  LNR_HIP(ctx, hipMemsetAsync(d_total, 0, 4, s));
  LNR_HIP(ctx, launch_chunk_count(c->d.cell_start, (uint32_t)C, d_total, s));
  uint32_t total = 0;
  LNR_HIP(ctx, hipMemcpy(&total, d_total, 4, hipMemcpyDeviceToHost));
  LNR_HIP(ctx, hipDeviceSynchronize());
  c->d.max_chunks = total;
  return LNR_OK;
}

lnr_status lnr_cloud_info(const lnr_cloud *c, uint64_t *n, int32_t dims[3], float origin[3], float *cell_size) {
  if (!c) return LNR_E_INVALID_ARG;
  if (n) *n = c->d.n;
  if (dims)
    for (int a = 0; a < 3; ++a) dims[a] = c->d.dims[a];
  if (origin)
    for (int a = 0; a < 3; ++a) origin[a] = c->d.origin[a];
  if (cell_size) *cell_size = c->d.cell_size;
  return LNR_OK;
}

lnr_status lnr_cloud_permutation(const lnr_cloud *c, uint32_t *perm_host) {
  if (!c || !perm_host) return LNR_E_INVALID_ARG;
  lnr_context *ctx = c->ctx;
  lnr_status st = use_device(ctx);
  if (st != LNR_OK) return st;
  LNR_HIP(ctx, hipMemcpy(perm_host, c->d.perm, 4ull * c->d.n, hipMemcpyDeviceToHost));
  return LNR_OK;
}

lnr_status lnr_cloud_cell_start(const lnr_cloud *c, uint32_t *cell_start_host) {
  if (!c || !cell_start_host) return LNR_E_INVALID_ARG;
  lnr_context *ctx = c->ctx;
  lnr_status st = use_device(ctx);
  if (st != LNR_OK) return st;
  LNR_HIP(ctx, hipMemcpy(cell_start_host, c->d.cell_start, 4ull * (c->d.n_cells + 1ull), hipMemcpyDeviceToHost));
  return LNR_OK;
}

void lnr_cloud_destroy(lnr_cloud *c) {
  if (!c) return;
  lnr_context *ctx = c->ctx;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  cloud_free(c);
  delete c;
  (void)hipGetLastError();
  context_release(ctx);
}

// ---------------------------------------------------------------------------
// render
// ---------------------------------------------------------------------------
// scratch of the tiled splat for a cloud of n_points points and grid g (see TiledSplatGrid)
static lnr_status ensure_tiled(lnr_context *ctx, Scratch &scr, const TiledSplatGrid &g, uint32_t n_points) {
  const size_t n = std::max<uint32_t>(1, n_points);
  lnr_status st;
  if ((st = ensure(ctx, scr.recs, 8 * n)) != LNR_OK || (st = ensure(ctx, scr.segs, 16 * n)) != LNR_OK ||
      (st = ensure(ctx, scr.sorted, 4 * n)) != LNR_OK || (st = ensure(ctx, scr.tile_nseg, 8ull * g.n_tiles)) != LNR_OK ||
      (st = ensure(ctx, scr.tile_off, 4ull * g.n_tiles + 4)) != LNR_OK ||
      (st = ensure(ctx, scr.tile_units, 4ull * g.n_tiles)) != LNR_OK ||
      (st = ensure(ctx, scr.units, 8ull * g.unit_cap)) != LNR_OK)
    return st;
  return LNR_OK;
}

static TiledSplatBufs tiled_bufs(Scratch &scr) {
  return TiledSplatBufs{static_cast<uint64_t *>(scr.recs.p),       static_cast<uint4 *>(scr.segs.p),
                        static_cast<uint32_t *>(scr.sorted.p),     static_cast<uint32_t *>(scr.tile_nseg.p),
                        static_cast<uint32_t *>(scr.tile_off.p),   static_cast<uint32_t *>(scr.tile_units.p),
                        static_cast<uint2 *>(scr.units.p)};
}

static SplatCam make_splat_cam(const lnr_camera *cam) {
  SplatCam sc{};
  std::memcpy(sc.P, cam->P, sizeof(sc.P));
  sc.Wf = (float)cam->width;
  sc.Hf = (float)cam->height;
  sc.z_near = cam->z_near;
  sc.z_far = cam->z_far;
  sc.W = (uint32_t)cam->width;
  return sc;
}

// checks of one render target against its camera
static lnr_status check_target(lnr_context *ctx, const lnr_camera *cam, const lnr_image *out) {
  std::string why;
  if (!camera_ok(cam, &why)) return fail(ctx, LNR_E_INVALID_ARG, why);
  if (!out->key || !out->depth || !out->rgba) return fail(ctx, LNR_E_INVALID_ARG, "image buffers must be non-NULL");
  if (out->width != cam->width || out->height != cam->height)
    return fail(ctx, LNR_E_INVALID_ARG, "image size differs from the camera's");
  if (!aligned(out->key, 8) || !aligned(out->depth, 4) || !aligned(out->rgba, 4))
    return fail(ctx, LNR_E_INVALID_ARG, "image buffers are misaligned");
  return LNR_OK;
}

// dev (may be nullptr): the same camera in device memory; the culling and
// projection kernels then read it there (the tiled and soft splats only), so
// the launches can be captured once and replayed for other cameras of the
// same size
static lnr_status render_impl(lnr_context *ctx, Scratch &scr, const lnr_cloud *c, const lnr_camera *cam,
                              lnr_image *out, uint32_t flags, bool soft, float soft_eps, void *hip_stream,
                              const DevCam *dev = nullptr) {
  if (!ctx) return LNR_E_INVALID_ARG;
  if (soft && !(std::isfinite(soft_eps) && soft_eps >= 0.f))
    return fail(ctx, LNR_E_INVALID_ARG, "soft_eps must be finite and >= 0");
  if (!c || !cam || !out) return fail(ctx, LNR_E_INVALID_ARG, "NULL pointer argument");
  if (flags & ~(LNR_RENDER_NO_CULL | LNR_RENDER_COUNT_ATOMICS | LNR_RENDER_ATOMIC_SPLAT))
    return fail(ctx, LNR_E_INVALID_ARG, "unknown render flags");
  lnr_status st = check_target(ctx, cam, out);
  if (st != LNR_OK) return st;
  if (c->ctx->device != ctx->device) return fail(ctx, LNR_E_INVALID_ARG, "cloud lives on another device");
  st = use_device(ctx);
  if (st != LNR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((st = ensure(ctx, scr.flags, c->d.n_cells)) != LNR_OK) return st;
  if ((st = ensure(ctx, scr.chunks, 8ull * kDepthBuckets * std::max<uint32_t>(1, c->d.max_chunks))) != LNR_OK)
    return st;
  if ((st = ensure(ctx, scr.counters, 4 * kCounterWords)) != LNR_OK) return st;
  const uint32_t npix = (uint32_t)cam->width * (uint32_t)cam->height;
  uint32_t *counters = static_cast<uint32_t *>(scr.counters.p);
  const CullParams prm = make_cull_params(cam, (flags & LNR_RENDER_NO_CULL) != 0);
  const SplatCam sc = make_splat_cam(cam);
  const bool count = (flags & LNR_RENDER_COUNT_ATOMICS) != 0;
  const bool atomic = count || (flags & LNR_RENDER_ATOMIC_SPLAT) != 0;
  const TiledSplatGrid tg = tiled_splat_grid((uint32_t)cam->width, (uint32_t)cam->height, c->d.n);
  // every allocation comes before the first launch: a failure leaves the image untouched
  if (!atomic && (st = ensure_tiled(ctx, scr, tg, c->d.n)) != LNR_OK) return st;
  if (soft && (st = ensure(ctx, scr.soft_acc, 16ull * npix)) != LNR_OK) return st;
  const TiledSplatBufs tb = tiled_bufs(scr);
  if (dev && atomic) return fail(ctx, LNR_E_INVALID_ARG, "a camera in device memory needs the tiled splat");
  // (the tiled splat writes every key itself: its segment sort empties the
  // keys of the tiles that merge through atomics, so only the counters here)
  LNR_LAUNCH(ctx, "clear", s,
             launch_clear(out->key, atomic ? npix : 0u, counters, tb.tile_nseg, atomic ? 0u : 2 * tg.n_tiles, s));
  LNR_LAUNCH(ctx, "cull", s,
             launch_cull(c->d, prm, dev ? &dev->cull : nullptr, static_cast<uint8_t *>(scr.flags.p),
                         static_cast<uint2 *>(scr.chunks.p), counters, s));
  const uint2 *chunks = static_cast<const uint2 *>(scr.chunks.p);
  uint32_t *rgba32 = reinterpret_cast<uint32_t *>(out->rgba);
  if (atomic) {
    LNR_LAUNCH(ctx, "splat", s, launch_splat(c->d, chunks, counters, sc, out->key, count, s));
    if (!soft) LNR_LAUNCH(ctx, "resolve", s, launch_resolve(out->key, c->d.rgbx, out->depth, rgba32, npix, s));
  } else {
    static const char *const names[5] = {"bin", "tilescan", "segsort", "tile", "tileres"};
    const bool merged = tiled_scan_merged(tg);  // the scan runs inside the segment sort
    for (int stage = 0; stage < 5; ++stage)
      if (!(merged && stage == 1))
        LNR_LAUNCH(ctx, names[stage], s,
                 launch_tiled_splat(c->d, chunks, counters, sc, dev ? &dev->splat : nullptr, (uint32_t)cam->height,
                                    tb, out->key, out->depth, rgba32, stage, s));
  }
  if (soft)
    LNR_LAUNCH(ctx, "soft", s,
               launch_soft(c->d, chunks, counters, sc, dev ? &dev->splat : nullptr, out->key, 1.0f + soft_eps,
                           static_cast<uint32_t *>(scr.soft_acc.p), out->depth, rgba32, npix, s));
  ctx->last_stream = s;
  ctx->rendered = true;
  ctx->counted = count;
  ctx->last_cells = c->d.n_cells;
  return LNR_OK;
}

lnr_status lnr_render(lnr_context *ctx, const lnr_cloud *c, const lnr_camera *cam, lnr_image *out, uint32_t flags,
                      void *hip_stream) {
  if (!ctx) return LNR_E_INVALID_ARG;
  return render_impl(ctx, ctx->sc, c, cam, out, flags, false, 0.f, hip_stream);
}

lnr_status lnr_render_soft(lnr_context *ctx, const lnr_cloud *c, const lnr_camera *cam, lnr_image *out,
                           float soft_eps, uint32_t flags, void *hip_stream) {
  if (!ctx) return LNR_E_INVALID_ARG;
  return render_impl(ctx, ctx->sc, c, cam, out, flags, true, soft_eps, hip_stream);
}

lnr_status lnr_render_views(lnr_context *ctx, const lnr_cloud *c, const lnr_camera *cams, lnr_image *outs,
                            int32_t n_views, uint32_t flags, void *hip_stream) {
  if (!ctx) return LNR_E_INVALID_ARG;
  if (!c || !cams || !outs) return fail(ctx, LNR_E_INVALID_ARG, "NULL pointer argument");
  if (n_views < 1 || n_views > kMaxRenderViews)
    return fail(ctx, LNR_E_INVALID_ARG, "n_views must be in [1, " + std::to_string(kMaxRenderViews) + "]");
  if (flags & ~LNR_RENDER_NO_CULL) return fail(ctx, LNR_E_INVALID_ARG, "unknown or unsupported render flags");
  lnr_status st;
  for (int v = 0; v < n_views; ++v)
    if ((st = check_target(ctx, &cams[v], &outs[v])) != LNR_OK) return st;
  // the views are drawn together: no two of their buffers (key, depth, rgba
  // of every view) may overlap
  {
    std::vector<std::pair<uintptr_t, uintptr_t>> r;
    r.reserve(3 * (size_t)n_views);
    for (int v = 0; v < n_views; ++v) {
      const uint64_t np = (uint64_t)outs[v].width * (uint64_t)outs[v].height;
      const uintptr_t k = reinterpret_cast<uintptr_t>(outs[v].key), d = reinterpret_cast<uintptr_t>(outs[v].depth),
                      c = reinterpret_cast<uintptr_t>(outs[v].rgba);
      r.emplace_back(k, k + 8 * np);
      r.emplace_back(d, d + 4 * np);
      r.emplace_back(c, c + 4 * np);
    }
    std::sort(r.begin(), r.end());
    for (size_t i = 1; i < r.size(); ++i)
      if (r[i].first < r[i - 1].second) return fail(ctx, LNR_E_INVALID_ARG, "the views' image buffers overlap");
  }
  if (c->ctx->device != ctx->device) return fail(ctx, LNR_E_INVALID_ARG, "cloud lives on another device");
  if ((st = use_device(ctx)) != LNR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Scratch &scr = ctx->sc;
  if ((st = ensure(ctx, scr.flags, c->d.n_cells)) != LNR_OK) return st;
  if ((st = ensure(ctx, scr.views, 16ull * kDepthBuckets * std::max<uint32_t>(1, c->d.max_chunks))) != LNR_OK)
    return st;
  if ((st = ensure(ctx, scr.counters, 4 * kCounterWords)) != LNR_OK) return st;
  uint32_t *counters = static_cast<uint32_t *>(scr.counters.p);
  uint4 *items = static_cast<uint4 *>(scr.views.p);
  const bool no_cull = (flags & LNR_RENDER_NO_CULL) != 0;
  for (int g = 0; g < n_views; g += kViewsPerPass) {
    const int n = std::min(kViewsPerPass, n_views - g);
    ViewsCull vc{};
    ViewsSplat vs{};
    vc.n = vs.n = n;
    for (int v = 0; v < n; ++v) {
      const lnr_camera *cam = &cams[g + v];
      const lnr_image &o = outs[g + v];
      vc.v[v] = make_cull_params(cam, no_cull);
      vs.cam[v] = make_splat_cam(cam);
      vs.key[v] = o.key;
      LNR_LAUNCH(ctx, "clear", s,
                 launch_clear(o.key, (uint32_t)o.width * (uint32_t)o.height, counters, nullptr, 0u, s));
    }
    LNR_LAUNCH(ctx, "cull_views", s,
               launch_cull_views(c->d, vc, static_cast<uint8_t *>(scr.flags.p), items, counters, s));
    LNR_LAUNCH(ctx, "splat_views", s, launch_splat_views(c->d, items, counters, vs, s));
    for (int v = 0; v < n; ++v) {
      const lnr_image &o = outs[g + v];
      LNR_LAUNCH(ctx, "resolve", s,
                 launch_resolve(o.key, c->d.rgbx, o.depth, reinterpret_cast<uint32_t *>(o.rgba),
                                (uint32_t)o.width * (uint32_t)o.height, s));
    }
  }
  ctx->last_stream = s;
  ctx->rendered = true;
  ctx->counted = false;
  ctx->last_cells = c->d.n_cells;
  return LNR_OK;
}

lnr_status lnr_render_stats(lnr_context *ctx, uint64_t *visible_cells, uint64_t *processed_points,
                            uint8_t *cull_flags_host) {
  if (!ctx) return LNR_E_INVALID_ARG;
  if (!ctx->rendered) return fail(ctx, LNR_E_INVALID_ARG, "no render on this context yet");
  lnr_status st = use_device(ctx);
  if (st != LNR_OK) return st;
  LNR_HIP(ctx, hipStreamSynchronize(ctx->last_stream));
  uint32_t cnt[kCounterWords];
  LNR_HIP(ctx, hipMemcpy(cnt, ctx->sc.counters.p, sizeof(cnt), hipMemcpyDeviceToHost));
  if (visible_cells) *visible_cells = cnt[1];
  if (processed_points) *processed_points = (uint64_t)cnt[2] | ((uint64_t)cnt[3] << 32);
  if (cull_flags_host)
    LNR_HIP(ctx, hipMemcpy(cull_flags_host, ctx->sc.flags.p, ctx->last_cells, hipMemcpyDeviceToHost));
  return LNR_OK;
}

lnr_status lnr_render_atomic_count(lnr_context *ctx, uint64_t *atomics) {
  if (!ctx) return LNR_E_INVALID_ARG;
  if (!atomics) return fail(ctx, LNR_E_INVALID_ARG, "NULL pointer argument");
  if (!ctx->rendered || !ctx->counted)
    return fail(ctx, LNR_E_INVALID_ARG, "the last render on this context did not count its atomics");
  lnr_status st = use_device(ctx);
  if (st != LNR_OK) return st;
  LNR_HIP(ctx, hipStreamSynchronize(ctx->last_stream));
  uint32_t cnt[kCounterWords];
  LNR_HIP(ctx, hipMemcpy(cnt, ctx->sc.counters.p, sizeof(cnt), hipMemcpyDeviceToHost));
  *atomics = cnt[kAtomicWord];
  return LNR_OK;
}

lnr_status lnr_measure_atomic_min(lnr_context *ctx, uint64_t n_slots, int32_t pattern, uint64_t n_ops,
                                  void *hip_stream, double *ops_per_s, uint64_t *ops_done) {
  if (!ctx) return LNR_E_INVALID_ARG;
  if (!ops_per_s) return fail(ctx, LNR_E_INVALID_ARG, "NULL pointer argument");
  if (n_slots < 1 || n_slots > 0xffffffffull) return fail(ctx, LNR_E_INVALID_ARG, "n_slots must be in [1, 2^32)");
  if (pattern != 0 && pattern != 1) return fail(ctx, LNR_E_INVALID_ARG, "pattern must be 0 or 1");
  constexpr uint64_t per_block = 256ull * kProbeIters;
  if (n_ops < 1 || n_ops > per_block * 0x7fffffffull) return fail(ctx, LNR_E_INVALID_ARG, "n_ops out of range");
  lnr_status st = use_device(ctx);
  if (st != LNR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const uint32_t grid = (uint32_t)((n_ops + per_block - 1) / per_block);
  TempAllocs tmp(ctx);
  uint64_t *buf;
  if ((st = tmp.get(&buf, 8ull * n_slots)) != LNR_OK) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  LNR_HIP(ctx, hipEventCreate(&e0));
  hipError_t he = hipEventCreate(&e1);
  float ms = 0.f;
  if (he == hipSuccess) he = hipMemsetAsync(buf, 0xff, 8ull * n_slots, s);
  if (he == hipSuccess) he = launch_atomic_probe(buf, (uint32_t)n_slots, pattern, grid, 1u, s);  // warm-up
  if (he == hipSuccess) he = hipMemsetAsync(buf, 0xff, 8ull * n_slots, s);
  if (he == hipSuccess) he = hipEventRecord(e0, s);
  if (he == hipSuccess) he = launch_atomic_probe(buf, (uint32_t)n_slots, pattern, grid, 2u, s);
  if (he == hipSuccess) he = hipEventRecord(e1, s);
  if (he == hipSuccess) he = hipEventSynchronize(e1);
  if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  LNR_HIP(ctx, he);
  const uint64_t done = (uint64_t)grid * per_block;
  *ops_per_s = ms > 0.f ? (double)done / (ms * 1e-3) : 0.0;
  if (ops_done) *ops_done = done;
  return LNR_OK;
}

// ---------------------------------------------------------------------------
// depth filter
// ---------------------------------------------------------------------------
// fixed: the allocation-free entry point's per-device array (nullptr: the
// context's grow-only scratch)
static lnr_status depth_filter_impl(lnr_context *ctx, Scratch &scr, lnr_image *io, int32_t n_levels,
                                    float filter_strength, void *hip_stream, float *fixed = nullptr);

lnr_status lnr_depth_filter(lnr_context *ctx, lnr_image *io, int32_t n_levels, float filter_strength,
                            void *hip_stream) {
  if (!ctx) return LNR_E_INVALID_ARG;
  return depth_filter_impl(ctx, ctx->sc, io, n_levels, filter_strength, hip_stream);
}

lnr_status lnr_depth_filter_noalloc(lnr_context *ctx, lnr_image *io, int32_t n_levels, float filter_strength,
                                    void *hip_stream) {
  if (!ctx) return LNR_E_INVALID_ARG;
  if (!ctx->noalloc_scratch)
    return fail(ctx, LNR_E_DEVICE, "allocation-free scratch unavailable: " + ctx->noalloc_error);
  return depth_filter_impl(ctx, ctx->sc, io, n_levels, filter_strength, hip_stream, ctx->noalloc_scratch);
}

static lnr_status depth_filter_impl(lnr_context *ctx, Scratch &scr, lnr_image *io, int32_t n_levels,
                                    float filter_strength, void *hip_stream, float *fixed) {
  if (!ctx) return LNR_E_INVALID_ARG;
  if (!io || !io->depth || !io->rgba) return fail(ctx, LNR_E_INVALID_ARG, "NULL pointer argument");
  if (io->width < 1 || io->height < 1 || io->width > 16384 || io->height > 16384)
    return fail(ctx, LNR_E_INVALID_ARG, "image width/height must be in [1, 16384]");
  if (!aligned(io->depth, 4) || !aligned(io->rgba, 4)) return fail(ctx, LNR_E_INVALID_ARG, "misaligned buffers");
  int maxn = 0;
  while ((2 << maxn) <= std::min(io->width, io->height)) ++maxn;
  if (n_levels < 0 || n_levels > maxn)
    return fail(ctx, LNR_E_INVALID_ARG, "n_levels must be in [0, floor(log2(min(W, H)))]");
  if (std::isnan(filter_strength) || filter_strength < 0.f)
    return fail(ctx, LNR_E_INVALID_ARG, "filter_strength must be >= 0 and not NaN");
  if (n_levels == 0) return LNR_OK;
  lnr_status st = use_device(ctx);
  if (st != LNR_OK) return st;
  int Hs[32], Ws[32];
  Hs[0] = io->height;
  Ws[0] = io->width;
  size_t total = 0, offs[32];
  for (int k = 1; k <= n_levels; ++k) {
    Hs[k] = (Hs[k - 1] + 1) / 2;
    Ws[k] = (Ws[k - 1] + 1) / 2;
  }
  // D[1..n], each 256-byte aligned
  for (int k = 1; k <= n_levels; ++k) {
    offs[k] = total;
    total += ((size_t)Hs[k] * Ws[k] * 4 + 255) / 256 * 256;
  }
  char *base;
  if (fixed) {
    if (total > kNoAllocScratchFloats * sizeof(float))
      return fail(ctx, LNR_E_INVALID_ARG,
                  "the min-pooled levels need " + std::to_string(total) + " bytes, more than the " +
                      std::to_string(kNoAllocScratchFloats * sizeof(float)) +
                      " bytes of the allocation-free filter's scratch");
    base = reinterpret_cast<char *>(fixed);
  } else {
    if ((st = ensure(ctx, scr.pyramid, total)) != LNR_OK) return st;
    base = static_cast<char *>(scr.pyramid.p);
  }
  float *D[32] = {nullptr};
  for (int k = 1; k <= n_levels; ++k) D[k] = reinterpret_cast<float *>(base + offs[k]);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  uint32_t *rgba = reinterpret_cast<uint32_t *>(io->rgba);
  if (fixed) {
    // no timing events either: nothing is created or allocated on this path
    (void)hipGetLastError();
    LNR_HIP(ctx, launch_pyramid(io->depth, rgba, io->height, io->width, n_levels, D, s));
    LNR_HIP(ctx, launch_upsample_fused(n_levels, D, Hs, Ws, io->depth, rgba, filter_strength,
                                       1.0f + filter_strength, s));
  } else {
    LNR_LAUNCH(ctx, "pyramid", s, launch_pyramid(io->depth, rgba, io->height, io->width, n_levels, D, s));
    LNR_LAUNCH(ctx, "upsample", s,
               launch_upsample_fused(n_levels, D, Hs, Ws, io->depth, rgba, filter_strength, 1.0f + filter_strength,
                                     s));
  }
  ctx->last_stream = s;
  return LNR_OK;
}

// ---------------------------------------------------------------------------
// U-Net
// ---------------------------------------------------------------------------
lnr_status lnr_unet_load(lnr_context *ctx, const void *blob_host, uint64_t bytes, lnr_precision prec,
                         lnr_unet **out) {
  if (!ctx) return LNR_E_INVALID_ARG;
  if (!blob_host || !out) return fail(ctx, LNR_E_INVALID_ARG, "NULL pointer argument");
  *out = nullptr;
  if (prec != LNR_FP32 && prec != LNR_BF16 && prec != LNR_BF16X3 && prec != LNR_FP16 && prec != LNR_FP8_E4M3 &&
      prec != LNR_FP8_E4M3X3)
    return fail(ctx, LNR_E_INVALID_ARG, "unknown precision");
  const uint8_t *p = static_cast<const uint8_t *>(blob_host);
  size_t off = 0;
  auto rd_u32 = [&](uint32_t *v) -> bool {
    if (off + 4 > bytes) return false;
    std::memcpy(v, p + off, 4);
    off += 4;
    return true;
  };
  if (bytes < 20 || std::memcmp(p, "LNRU", 4) != 0) return fail(ctx, LNR_E_FORMAT, "bad magic");
  off = 4;
  uint32_t version, L, in_ch, out_ch;
  rd_u32(&version);
  rd_u32(&L);
  rd_u32(&in_ch);
  rd_u32(&out_ch);
  if (version != 1 && version != 2) return fail(ctx, LNR_E_FORMAT, "unknown version");
  if (L < 1 || L > 6) return fail(ctx, LNR_E_UNSUPPORTED, "levels must be in [1, 6]");
  if (in_ch != 5 || out_ch != 3) return fail(ctx, LNR_E_UNSUPPORTED, "network must map 5 to 3 channels");
  std::unique_ptr<lnr_unet> u(new lnr_unet);
  u->ctx = ctx;
  u->L = (int)L;
  u->prec = static_cast<Prec>(prec);
  for (uint32_t l = 0; l < L; ++l) {
    uint32_t w;
    if (!rd_u32(&w)) return fail(ctx, LNR_E_FORMAT, "truncated header");
    if (w < 16 || w > 512 || w % 16) return fail(ctx, LNR_E_UNSUPPORTED, "widths must be multiples of 16 in [16, 512]");
    u->widths[l] = (int)w;
  }
  u->cin0_pad = (u->prec == Prec::F32) ? 8 : 16;
  // expected (c_out, c_in, k) in blob order
  std::vector<int> exp;
  for (int l = 0; l < (int)L; ++l) {
    const int ci = l == 0 ? 5 : u->widths[l - 1];
    exp.insert(exp.end(), {u->widths[l], ci, 3, u->widths[l], u->widths[l], 3});
  }
  for (int l = (int)L - 2; l >= 0; --l)
    exp.insert(exp.end(), {u->widths[l], u->widths[l] + u->widths[l + 1], 3, u->widths[l], u->widths[l], 3});
  exp.insert(exp.end(), {3, u->widths[0], 1});
  const int nconv = 4 * (int)L - 1;
  lnr_status st = use_device(ctx);
  if (st != LNR_OK) return st;
  auto free_all = [&]() {
    for (auto &a : u->allocs) dfree(ctx, a.first, a.second);
    u->allocs.clear();
  };
  auto upload = [&](const void *src, size_t nbytes, void **dst) -> lnr_status {
    lnr_status s2 = dalloc(ctx, dst, nbytes);
    if (s2 != LNR_OK) return s2;
    u->allocs.emplace_back(*dst, nbytes);
    hipError_t e = hipMemcpy(*dst, src, nbytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(weights)");
    return LNR_OK;
  };
  for (int li = 0; li < nconv; ++li) {
    uint32_t co, ci, k, has_bn = 0;
    if (!rd_u32(&co) || !rd_u32(&ci) || !rd_u32(&k) || (version == 2 && !rd_u32(&has_bn))) {
      free_all();
      return fail(ctx, LNR_E_FORMAT, "truncated record header");
    }
    if ((int)co != exp[3 * li] || (int)ci != exp[3 * li + 1] || (int)k != exp[3 * li + 2]) {
      free_all();
      return fail(ctx, LNR_E_FORMAT, "conv record " + std::to_string(li) + " has an unexpected shape");
    }
    const size_t nw = (size_t)co * ci * k * k;
    size_t need = 4 * (nw + co) + (has_bn ? 16ull * co + 4 : 0);
    if (off + need > bytes) {
      free_all();
      return fail(ctx, LNR_E_FORMAT, "truncated weights");
    }
    std::vector<float> W(nw), b(co);
    std::memcpy(W.data(), p + off, 4 * nw);
    off += 4 * nw;
    std::memcpy(b.data(), p + off, 4 * co);
    off += 4 * co;
    std::vector<double> Wd(W.begin(), W.end()), bd(b.begin(), b.end());
    if (has_bn) {
      std::vector<float> g(co), beta(co), mean(co), var(co);
      std::memcpy(g.data(), p + off, 4 * co);
      std::memcpy(beta.data(), p + off + 4 * co, 4 * co);
      std::memcpy(mean.data(), p + off + 8 * co, 4 * co);
      std::memcpy(var.data(), p + off + 12 * co, 4 * co);
      float eps;
      std::memcpy(&eps, p + off + 16 * co, 4);
      off += 16 * co + 4;
      for (uint32_t o = 0; o < co; ++o) {
        const double sc = (double)g[o] / std::sqrt((double)var[o] + (double)eps);
        for (size_t i = 0; i < (size_t)ci * k * k; ++i) Wd[o * ci * k * k + i] *= sc;
        bd[o] = (bd[o] - (double)mean[o]) * sc + (double)beta[o];
      }
    }
    ConvLayer cl;
    cl.cout = (int)co;
    cl.cin = (int)ci;
    cl.k = (int)k;
    if (li == nconv - 1) {
      // head: float32 [3][c_in] for every precision
      std::vector<float> hw((size_t)co * ci), hb(co);
      for (size_t i = 0; i < hw.size(); ++i) hw[i] = (float)Wd[i];
      for (uint32_t o = 0; o < co; ++o) hb[o] = (float)bd[o];
      cl.cout_pad = (int)co;
      cl.cin_pad = (int)ci;
      if ((st = upload(hw.data(), 4 * hw.size(), &cl.w)) != LNR_OK) return free_all(), st;
      void *bp;
      if ((st = upload(hb.data(), 4 * hb.size(), &bp)) != LNR_OK) return free_all(), st;
      cl.bias = static_cast<float *>(bp);
      u->head = cl;
      continue;
    }
    cl.cout_pad = ((int)co + 31) / 32 * 32;
    cl.cin_pad = (li == 0) ? u->cin0_pad : (int)ci;
    const size_t np = (size_t)cl.cout_pad * 9 * cl.cin_pad;
    std::vector<float> packed(np, 0.f);
    // the float32 network input is staged as (x0, x1, x2, 0, x3, x4, 0, 0)
    const bool gap = li == 0 && u->prec == Prec::F32;
    for (int o = 0; o < (int)co; ++o)
      for (int i = 0; i < (int)ci; ++i)
        for (int t = 0; t < 9; ++t)
          packed[((size_t)o * 9 + t) * cl.cin_pad + (gap && i >= 3 ? i + 1 : i)] =
              (float)Wd[((size_t)o * ci + i) * 9 + t];
    std::vector<float> bias(cl.cout_pad, 0.f);
    for (int o = 0; o < (int)co; ++o) bias[o] = (float)bd[o];
    void *bp;
    if ((st = upload(bias.data(), 4 * bias.size(), &bp)) != LNR_OK) return free_all(), st;
    cl.bias = static_cast<float *>(bp);
    if (u->prec == Prec::F32) {
      if ((st = upload(packed.data(), 4 * np, &cl.w)) != LNR_OK) return free_all(), st;
      if (cl.cin_pad % 16 == 0) {
        // Winograd F(2x2, 3x3) filter transform U = G g G^T, rounded once from
        // the float64 weights; U[o][4 xi + nu][i]
        static const double G[4][3] = {{1, 0, 0}, {0.5, 0.5, 0.5}, {0.5, -0.5, 0.5}, {0, 0, 1}};
        std::vector<float> wu((size_t)cl.cout_pad * 16 * cl.cin_pad, 0.f);
        for (int o = 0; o < (int)co; ++o)
          for (int i = 0; i < (int)ci; ++i) {
            const double *g = &Wd[((size_t)o * ci + i) * 9];
            for (int xi = 0; xi < 4; ++xi)
              for (int nu = 0; nu < 4; ++nu) {
                double acc = 0;
                for (int dy = 0; dy < 3; ++dy)
                  for (int dx = 0; dx < 3; ++dx) acc += G[xi][dy] * g[dy * 3 + dx] * G[nu][dx];
                wu[((size_t)o * 16 + 4 * xi + nu) * cl.cin_pad + i] = (float)acc;
              }
          }
        if ((st = upload(wu.data(), 4 * wu.size(), &cl.wu)) != LNR_OK) return free_all(), st;
      }
    } else if (u->prec == Prec::FP16) {
      std::vector<uint16_t> h(np);
      for (size_t i = 0; i < np; ++i) h[i] = host_f2h(packed[i]);
      if ((st = upload(h.data(), 2 * np, &cl.w)) != LNR_OK) return free_all(), st;
    } else if (u->prec == Prec::FP8 || u->prec == Prec::FP8X3) {
      // one scale per output channel: its largest weight (of the float64,
      // batch-norm-folded weights) maps to 448; the lo plane holds the e4m3 of
      // what rounding the scaled weight to e4m3 left
      std::vector<uint8_t> hi(np, 0), lo(np, 0);
      std::vector<float> scale(cl.cout_pad, 1.f);
      const size_t row = (size_t)9 * cl.cin_pad;
      for (int o = 0; o < (int)co; ++o) {
        double amax = 0;
        for (int i = 0; i < (int)ci; ++i)
          for (int t = 0; t < 9; ++t) amax = std::max(amax, std::fabs(Wd[((size_t)o * ci + i) * 9 + t]));
        const double sc = amax > 0 ? amax / 448.0 : 1.0;
        scale[o] = (float)sc;
        for (int i = 0; i < (int)ci; ++i)
          for (int t = 0; t < 9; ++t) {
            const size_t q = (size_t)o * row + (size_t)t * cl.cin_pad + i;
            const double v = Wd[((size_t)o * ci + i) * 9 + t] / (double)scale[o];
            hi[q] = host_e4m3(v);
            lo[q] = host_e4m3(v - host_e4m3_value(hi[q]));
          }
      }
      if ((st = upload(hi.data(), np, &cl.w)) != LNR_OK) return free_all(), st;
      if (u->prec == Prec::FP8X3 && (st = upload(lo.data(), np, &cl.w_lo)) != LNR_OK) return free_all(), st;
      void *sp;
      if ((st = upload(scale.data(), 4 * scale.size(), &sp)) != LNR_OK) return free_all(), st;
      cl.wscale = static_cast<float *>(sp);
    } else {
      std::vector<uint16_t> hi(np), lo(np);
      for (size_t i = 0; i < np; ++i) {
        hi[i] = host_f2bf(packed[i]);
        lo[i] = host_f2bf(packed[i] - host_bf2f(hi[i]));
      }
      if ((st = upload(hi.data(), 2 * np, &cl.w)) != LNR_OK) return free_all(), st;
      if (u->prec == Prec::BF16X3)
        if ((st = upload(lo.data(), 2 * np, &cl.w_lo)) != LNR_OK) return free_all(), st;
    }
    u->convs.push_back(cl);
  }
  if (off != bytes) {
    free_all();
    return fail(ctx, LNR_E_FORMAT, "trailing bytes after the last record");
  }
  ++ctx->children;
  *out = u.release();
  return LNR_OK;
}

void lnr_unet_destroy(lnr_unet *u) {
  if (!u) return;
  lnr_context *ctx = u->ctx;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto &a : u->allocs) dfree(ctx, a.first, a.second);
  delete u;
  (void)hipGetLastError();
  context_release(ctx);
}

lnr_status lnr_reconstruct(lnr_context *ctx, const lnr_unet *u, const lnr_image *in, float *rgb_out,
                           void *hip_stream) {
  if (!ctx) return LNR_E_INVALID_ARG;
  if (!u || !in || !in->depth || !in->rgba || !rgb_out) return fail(ctx, LNR_E_INVALID_ARG, "NULL pointer argument");
  const int H = in->height, W = in->width, L = u->L;
  if (H < 1 || W < 1 || H > 16384 || W > 16384) return fail(ctx, LNR_E_INVALID_ARG, "bad image size");
  if (H % (1 << (L - 1)) || W % (1 << (L - 1)))
    return fail(ctx, LNR_E_INVALID_ARG, "H and W must be divisible by 2^(levels-1)");
  if (!aligned(in->depth, 4) || !aligned(in->rgba, 4) || !aligned(rgb_out, 4))
    return fail(ctx, LNR_E_INVALID_ARG, "misaligned buffers");
  lnr_status st = use_device(ctx);
  if (st != LNR_OK) return st;
  const UNetLayout lay = unet_layout(u, H, W, 1);
  if ((st = ensure(ctx, ctx->sc.act, lay.bytes)) != LNR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // one image: the first convolution reads the RGBDA image itself (batches
  // from the serving loop go through the input pack into one batched tensor)
  if ((st = unet_convs(ctx, ctx->sc, u, lay, rgb_out, nullptr, s, in->depth,
                       reinterpret_cast<const uint32_t *>(in->rgba))) != LNR_OK)
    return st;
  ctx->last_stream = s;
  return LNR_OK;
}

lnr_status lnr_sync(lnr_context *ctx, void *hip_stream) {
  if (!ctx) return LNR_E_INVALID_ARG;
  lnr_status st = use_device(ctx);
  if (st != LNR_OK) return st;
  LNR_HIP(ctx, hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)));
  LNR_HIP(ctx, hipGetLastError());
  return LNR_OK;
}

lnr_status lnr_debug_fail_allocation(lnr_context *ctx, int64_t after) {
  if (!ctx) return LNR_E_INVALID_ARG;
  ctx->fail_alloc_after = after < 0 ? -1 : after;
  return LNR_OK;
}

lnr_status lnr_profile_enable(lnr_context *ctx, int enable) {
  if (!ctx) return LNR_E_INVALID_ARG;
  ctx->profiling = enable != 0;
  return LNR_OK;
}

lnr_status lnr_profile_read(lnr_context *ctx, lnr_kernel_time *out, int32_t max, int32_t *count) {
  if (!ctx || !count || (max > 0 && !out)) return ctx ? fail(ctx, LNR_E_INVALID_ARG, "bad arguments") : LNR_E_INVALID_ARG;
  lnr_status st = use_device(ctx);
  if (st != LNR_OK) return st;
  *count = (int32_t)ctx->recs.size();
  hipError_t err = hipSuccess;
  if (!ctx->recs.empty()) err = hipEventSynchronize(ctx->recs.back().b);
  for (size_t i = 0; i < ctx->recs.size(); ++i) {
    auto &r = ctx->recs[i];
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, r.a, r.b);
    if ((int32_t)i < max) out[i] = lnr_kernel_time{r.name, ms};
    ctx->event_pool.push_back(r.a);
    ctx->event_pool.push_back(r.b);
  }
  ctx->recs.clear();
  if (err != hipSuccess) return hip_fail(ctx, err, "hipEventElapsedTime");
  return LNR_OK;
}

// ---------------------------------------------------------------------------
// serving
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

struct ServerSession {
  bool open = false;
  int W = 0, H = 0;
  void *buf = nullptr;
  size_t bytes = 0;
  float *out[2] = {nullptr, nullptr};
  int next_out = 0;
  bool pending = false;
  bool in_flight = false;
  lnr_camera cam{};
  uint64_t tag = 0;
  uint64_t seq = 0;  // submission order of the pending request
};

struct ServerLane {
  hipStream_t stream = nullptr;
  Scratch sc;
  hipEvent_t ev_start = nullptr, ev_done = nullptr;
  bool busy = false;
  std::vector<int> sess;
  std::vector<uint64_t> tags;
  std::vector<const float *> outs;
  float **head_outs_dev = nullptr;   // device array [max_batch]
  float **head_outs_host = nullptr;  // pinned host staging of the same
  DevCam *cams_dev = nullptr;        // the batch's cameras, device array [max_batch]
  DevCam *cams_host = nullptr;       // pinned host staging of the same
  // the RGBDA image of each batch slot (rendered, filtered, packed), at the
  // largest session size: a key plane, a depth plane and an rgba plane of
  // max_batch slots each, slot b at pixel b * slot_px of every plane
  void *slot_buf = nullptr;
  size_t slot_bytes = 0, slot_px = 0;
  // one graph per (height, width, batch): every launch of a whole batch
  std::map<std::tuple<int, int, int>, hipGraphExec_t> graphs;
  std::vector<hipGraph_t> graph_defs;
};

}  // namespace

struct lnr_server {
  lnr_context *ctx = nullptr;
  const lnr_cloud *cloud = nullptr;
  const lnr_unet *unet = nullptr;
  lnr_server_config cfg{};
  std::vector<ServerSession> sessions;
  std::vector<ServerLane> lanes;
  std::deque<lnr_server_result> done;
  uint64_t seq = 0;
};

namespace {

void server_release(lnr_server *srv) {
  lnr_context *ctx = srv->ctx;
  for (auto &l : srv->lanes) {
    if (l.stream) (void)hipStreamSynchronize(l.stream);
    for (auto &g : l.graphs) (void)hipGraphExecDestroy(g.second);
    for (auto g : l.graph_defs) (void)hipGraphDestroy(g);
    for (Buf *b : {&l.sc.flags, &l.sc.chunks, &l.sc.counters, &l.sc.pyramid, &l.sc.act, &l.sc.soft_acc, &l.sc.recs,
                   &l.sc.segs, &l.sc.sorted, &l.sc.tile_nseg, &l.sc.tile_off, &l.sc.tile_units, &l.sc.units,
                   &l.sc.views})
      dfree(ctx, b->p, b->cap);
    if (l.head_outs_dev) dfree(ctx, l.head_outs_dev, 8ull * 16);
    if (l.head_outs_host) (void)hipHostFree(l.head_outs_host);
    if (l.cams_dev) dfree(ctx, l.cams_dev, sizeof(DevCam) * 16);
    if (l.cams_host) (void)hipHostFree(l.cams_host);
    if (l.slot_buf) dfree(ctx, l.slot_buf, l.slot_bytes);
    if (l.ev_start) (void)hipEventDestroy(l.ev_start);
    if (l.ev_done) (void)hipEventDestroy(l.ev_done);
    if (l.stream) (void)hipStreamDestroy(l.stream);
  }
  srv->lanes.clear();
  for (auto &ss : srv->sessions)
    if (ss.buf) dfree(ctx, ss.buf, ss.bytes);
  srv->sessions.clear();
}

// move a finished lane's requests to the done list
void server_collect(lnr_server *srv, ServerLane &l) {
  if (!l.busy || hipEventQuery(l.ev_done) != hipSuccess) return;
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, l.ev_start, l.ev_done);
  for (size_t i = 0; i < l.sess.size(); ++i) {
    ServerSession &ss = srv->sessions[l.sess[i]];
    ss.in_flight = false;
    lnr_server_result r{};
    r.session = l.sess[i];
    r.tag = l.tags[i];
    r.superseded = 0;
    r.batch = (int32_t)l.sess.size();
    r.batch_gpu_ms = ms;
    r.rgb = l.outs[i];
    r.width = ss.W;
    r.height = ss.H;
    srv->done.push_back(r);
  }
  l.sess.clear();
  l.tags.clear();
  l.outs.clear();
  l.busy = false;
}

}  // namespace

extern "C" {

lnr_status lnr_server_create(lnr_context *ctx, const lnr_cloud *c, const lnr_unet *u, const lnr_server_config *cfg,
                             lnr_server **out) {
  if (!ctx) return LNR_E_INVALID_ARG;
  if (!c || !u || !cfg || !out) return fail(ctx, LNR_E_INVALID_ARG, "NULL pointer argument");
  *out = nullptr;
  if (cfg->max_batch < 1 || cfg->max_batch > 16) return fail(ctx, LNR_E_INVALID_ARG, "max_batch must be in [1, 16]");
  if (cfg->lanes < 1 || cfg->lanes > 8) return fail(ctx, LNR_E_INVALID_ARG, "lanes must be in [1, 8]");
  if (cfg->max_width < 1 || cfg->max_height < 1 || cfg->max_width > 16384 || cfg->max_height > 16384)
    return fail(ctx, LNR_E_INVALID_ARG, "bad max resolution");
  if (cfg->soft && !(std::isfinite(cfg->soft_eps) && cfg->soft_eps >= 0.f))
    return fail(ctx, LNR_E_INVALID_ARG, "soft_eps must be finite and >= 0");
  if (std::isnan(cfg->filter_strength) || cfg->filter_strength < 0.f || cfg->n_levels < 0)
    return fail(ctx, LNR_E_INVALID_ARG, "bad depth filter parameters");
  if (u->widths[0] > 64) return fail(ctx, LNR_E_UNSUPPORTED, "serving needs a U-Net with widths[0] <= 64");
  const int a = 1 << (u->L - 1);
  const int mW = (cfg->max_width + a - 1) / a * a, mH = (cfg->max_height + a - 1) / a * a;
  lnr_status st = use_device(ctx);
  if (st != LNR_OK) return st;
  std::unique_ptr<lnr_server> srv(new lnr_server);
  srv->ctx = ctx;
  srv->cloud = c;
  srv->unet = u;
  srv->cfg = *cfg;
  srv->lanes.resize(cfg->lanes);
  // every lane's scratch is sized for the largest resolution and batch up front,
  // so captured graphs keep pointing at live buffers
  const size_t npix = (size_t)mW * mH;
  size_t pyr = 0;
  {
    int h = mH, w = mW;
    for (int k = 1; k <= std::max(cfg->n_levels, 1); ++k) {
      h = (h + 1) / 2;
      w = (w + 1) / 2;
      pyr += ((size_t)h * w * 4 + 255) / 256 * 256;
    }
  }
  const size_t act = unet_layout(u, mH, mW, cfg->max_batch).bytes;
  // per batch slot: key (8 B), depth (4 B) and rgba (4 B) per pixel, each
  // plane of every slot 256-byte aligned
  const size_t slot_px = (npix + 31) / 32 * 32;
  const size_t slot_bytes = 16 * slot_px * (size_t)cfg->max_batch;
  for (auto &l : srv->lanes) {
    hipError_t e = hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&l.ev_start);
    if (e == hipSuccess) e = hipEventCreate(&l.ev_done);
    if (e == hipSuccess) e = hipHostMalloc((void **)&l.head_outs_host, 8ull * 16, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&l.cams_host, sizeof(DevCam) * 16, hipHostMallocDefault);
    if (e != hipSuccess) {
      server_release(srv.get());
      return hip_fail(ctx, e, "server lane setup");
    }
    if ((st = ensure(ctx, l.sc.flags, c->d.n_cells)) != LNR_OK ||
        (st = ensure(ctx, l.sc.chunks, 8ull * kDepthBuckets * std::max<uint32_t>(1, c->d.max_chunks))) != LNR_OK ||
        (st = ensure(ctx, l.sc.counters, 4 * kCounterWords)) != LNR_OK || (st = ensure(ctx, l.sc.pyramid, pyr)) != LNR_OK ||
        (st = ensure(ctx, l.sc.act, act)) != LNR_OK ||
        (st = ensure_tiled(ctx, l.sc, tiled_splat_grid((uint32_t)mW, (uint32_t)mH, c->d.n), c->d.n)) != LNR_OK ||
        (cfg->soft && (st = ensure(ctx, l.sc.soft_acc, 16 * npix)) != LNR_OK) ||
        (st = dalloc(ctx, (void **)&l.head_outs_dev, 8ull * 16)) != LNR_OK ||
        (st = dalloc(ctx, (void **)&l.cams_dev, sizeof(DevCam) * 16)) != LNR_OK ||
        (st = dalloc(ctx, &l.slot_buf, slot_bytes)) != LNR_OK) {
      server_release(srv.get());
      return st;
    }
    l.slot_bytes = slot_bytes;
    l.slot_px = slot_px;
  }
  ++ctx->children;
  *out = srv.release();
  return LNR_OK;
}

void lnr_server_destroy(lnr_server *srv) {
  if (!srv) return;
  lnr_context *ctx = srv->ctx;
  (void)hipSetDevice(ctx->device);
  server_release(srv);
  delete srv;
  (void)hipGetLastError();
  context_release(ctx);
}

lnr_status lnr_server_open_session(lnr_server *srv, int32_t width, int32_t height, int32_t *session) {
  if (!srv || !session) return srv ? fail(srv->ctx, LNR_E_INVALID_ARG, "NULL pointer argument") : LNR_E_INVALID_ARG;
  lnr_context *ctx = srv->ctx;
  const int a = 1 << (srv->unet->L - 1);
  if (width < 1 || height < 1 || width > srv->cfg.max_width || height > srv->cfg.max_height || width % a ||
      height % a)
    return fail(ctx, LNR_E_INVALID_ARG, "session size must be within the server's maximum and divisible by 2^(L-1)");
  if (srv->cfg.n_levels > 0) {
    int maxn = 0;
    while ((2 << maxn) <= std::min(width, height)) ++maxn;
    if (srv->cfg.n_levels > maxn)
      return fail(ctx, LNR_E_INVALID_ARG,
                  "the server's n_levels exceeds floor(log2(min(width, height))) of this session size");
  }
  lnr_status st = use_device(ctx);
  if (st != LNR_OK) return st;
  const size_t np = (size_t)width * height;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t bytes = 2 * al(12 * np);  // two output planes; the images live in the lanes' slots
  ServerSession ss;
  if ((st = dalloc(ctx, &ss.buf, bytes)) != LNR_OK) return st;  // LNR_E_BUDGET: not admitted
  ss.bytes = bytes;
  char *p = static_cast<char *>(ss.buf);
  ss.out[0] = reinterpret_cast<float *>(p);
  p += al(12 * np);
  ss.out[1] = reinterpret_cast<float *>(p);
  ss.open = true;
  ss.W = width;
  ss.H = height;
  for (size_t i = 0; i < srv->sessions.size(); ++i)
    if (!srv->sessions[i].open && !srv->sessions[i].buf) {
      srv->sessions[i] = ss;
      *session = (int32_t)i;
      return LNR_OK;
    }
  srv->sessions.push_back(ss);
  *session = (int32_t)srv->sessions.size() - 1;
  return LNR_OK;
}

lnr_status lnr_server_close_session(lnr_server *srv, int32_t session) {
  if (!srv) return LNR_E_INVALID_ARG;
  lnr_context *ctx = srv->ctx;
  if (session < 0 || session >= (int32_t)srv->sessions.size() || !srv->sessions[session].open)
    return fail(ctx, LNR_E_INVALID_ARG, "no such session");
  lnr_status st = use_device(ctx);
  if (st != LNR_OK) return st;
  for (auto &l : srv->lanes)
    if (l.busy && std::find(l.sess.begin(), l.sess.end(), session) != l.sess.end()) {
      LNR_HIP(ctx, hipEventSynchronize(l.ev_done));
      server_collect(srv, l);
    }
  ServerSession &ss = srv->sessions[session];
  dfree(ctx, ss.buf, ss.bytes);
  ss = ServerSession();
  return LNR_OK;
}

lnr_status lnr_server_submit(lnr_server *srv, int32_t session, const lnr_camera *cam, uint64_t tag) {
  if (!srv) return LNR_E_INVALID_ARG;
  lnr_context *ctx = srv->ctx;
  if (!cam) return fail(ctx, LNR_E_INVALID_ARG, "NULL camera");
  if (session < 0 || session >= (int32_t)srv->sessions.size() || !srv->sessions[session].open)
    return fail(ctx, LNR_E_INVALID_ARG, "no such session");
  ServerSession &ss = srv->sessions[session];
  std::string why;
  if (!camera_ok(cam, &why)) return fail(ctx, LNR_E_INVALID_ARG, why);
  if (cam->width != ss.W || cam->height != ss.H) return fail(ctx, LNR_E_INVALID_ARG, "camera size differs from the session's");
  if (ss.pending) {
    lnr_server_result r{};
    r.session = session;
    r.tag = ss.tag;
    r.superseded = 1;
    r.width = ss.W;
    r.height = ss.H;
    srv->done.push_back(r);
  }
  ss.pending = true;
  ss.cam = *cam;
  ss.tag = tag;
  ss.seq = srv->seq++;
  return LNR_OK;
}

lnr_status lnr_server_step(lnr_server *srv, int32_t *launched) {
  if (!srv || !launched) return srv ? fail(srv->ctx, LNR_E_INVALID_ARG, "NULL pointer argument") : LNR_E_INVALID_ARG;
  lnr_context *ctx = srv->ctx;
  *launched = 0;
  lnr_status st = use_device(ctx);
  if (st != LNR_OK) return st;
  ServerLane *lane = nullptr;
  for (auto &l : srv->lanes) {
    server_collect(srv, l);
    if (!l.busy && !lane) lane = &l;
  }
  if (!lane) return LNR_OK;
  // the oldest runnable request decides the resolution of the batch
  int first = -1;
  for (size_t i = 0; i < srv->sessions.size(); ++i) {
    const ServerSession &ss = srv->sessions[i];
    if (ss.open && ss.pending && !ss.in_flight && (first < 0 || ss.seq < srv->sessions[first].seq)) first = (int)i;
  }
  if (first < 0) return LNR_OK;
  const int W = srv->sessions[first].W, H = srv->sessions[first].H;
  std::vector<int> batch;
  {
    std::vector<std::pair<uint64_t, int>> cand;
    for (size_t i = 0; i < srv->sessions.size(); ++i) {
      const ServerSession &ss = srv->sessions[i];
      if (ss.open && ss.pending && !ss.in_flight && ss.W == W && ss.H == H) cand.emplace_back(ss.seq, (int)i);
    }
    std::sort(cand.begin(), cand.end());
    for (size_t i = 0; i < cand.size() && (int)batch.size() < srv->cfg.max_batch; ++i) batch.push_back(cand[i].second);
  }
  const int B = (int)batch.size();
  hipStream_t s = lane->stream;
  // On any failure below, undo what this step changed: the lane's output list,
  // the sessions' output-plane toggles and the context's timing switch (no
  // request is marked in flight before the end, so the batch stays pending).
  struct Rollback {
    lnr_server *srv;
    ServerLane *lane;
    const std::vector<int> &batch;
    bool was_profiling;
    std::vector<int> toggled;
    bool armed = true;
    ~Rollback() {
      srv->ctx->profiling = was_profiling;
      if (!armed) return;
      lane->outs.clear();
      for (int i : toggled) srv->sessions[i].next_out ^= 1;
    }
  } rb{srv, lane, batch, ctx->profiling, {}};
  ctx->profiling = false;
  const UNetLayout lay = unet_layout(srv->unet, H, W, B);
  for (int b = 0; b < B; ++b) {
    ServerSession &ss = srv->sessions[batch[b]];
    lane->cams_host[b].cull = make_cull_params(&ss.cam, false);
    lane->cams_host[b].splat = make_splat_cam(&ss.cam);
    float *o = ss.out[ss.next_out];
    ss.next_out ^= 1;
    rb.toggled.push_back(batch[b]);
    lane->head_outs_host[b] = o;
    lane->outs.push_back(o);
  }
  // Every launch of the batch: per slot render (camera read from cams_dev),
  // depth filter and input pack, then the batched U-Net writing through
  // head_outs_dev.  Nothing in it depends on the batch's cameras or sessions
  // beyond those two device arrays, so one capture per (size, batch) serves
  // every later batch of that shape.
  char *slots = static_cast<char *>(lane->slot_buf);
  const size_t sp = lane->slot_px, mb = (size_t)srv->cfg.max_batch;
  auto enqueue = [&]() -> lnr_status {
    for (int b = 0; b < B; ++b) {
      const ServerSession &ss = srv->sessions[batch[b]];
      lnr_image img{reinterpret_cast<uint64_t *>(slots) + (size_t)b * sp,
                    reinterpret_cast<float *>(slots + 8 * sp * mb) + (size_t)b * sp,
                    reinterpret_cast<uint8_t *>(slots + 12 * sp * mb) + 4 * (size_t)b * sp, W, H};
      lnr_status r = render_impl(ctx, lane->sc, srv->cloud, &ss.cam, &img, 0, srv->cfg.soft != 0,
                                 srv->cfg.soft_eps, s, lane->cams_dev + b);
      if (r == LNR_OK && srv->cfg.n_levels > 0)
        r = depth_filter_impl(ctx, lane->sc, &img, srv->cfg.n_levels, srv->cfg.filter_strength, s);
      if (r == LNR_OK)
        r = unet_pack(ctx, lane->sc, srv->unet, lay, b, img.depth, reinterpret_cast<const uint32_t *>(img.rgba), s);
      if (r != LNR_OK) return r;
    }
    return unet_convs(ctx, lane->sc, srv->unet, lay, nullptr, lane->head_outs_dev, s);
  };
  LNR_HIP(ctx, hipEventRecord(lane->ev_start, s));
  LNR_HIP(ctx, hipMemcpyAsync(lane->head_outs_dev, lane->head_outs_host, 8ull * B, hipMemcpyHostToDevice, s));
  LNR_HIP(ctx, hipMemcpyAsync(lane->cams_dev, lane->cams_host, sizeof(DevCam) * B, hipMemcpyHostToDevice, s));
  if (srv->cfg.use_graphs) {
    const auto key = std::make_tuple(H, W, B);
    auto it = lane->graphs.find(key);
    if (it == lane->graphs.end()) {
      hipGraph_t g = nullptr;
      hipGraphExec_t ge = nullptr;
      LNR_HIP(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      st = enqueue();
      hipError_t e = hipStreamEndCapture(s, &g);
      if (st != LNR_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
      e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(ctx, e, "hipGraphInstantiate");
      }
      lane->graph_defs.push_back(g);
      it = lane->graphs.emplace(key, ge).first;
    }
    LNR_HIP(ctx, hipGraphLaunch(it->second, s));
  } else {
    if ((st = enqueue()) != LNR_OK) return st;
  }
  LNR_HIP(ctx, hipEventRecord(lane->ev_done, s));
  rb.armed = false;
  for (int b = 0; b < B; ++b) {
    ServerSession &ss = srv->sessions[batch[b]];
    ss.pending = false;
    ss.in_flight = true;
    lane->sess.push_back(batch[b]);
    lane->tags.push_back(ss.tag);
  }
  lane->busy = true;
  *launched = B;
  return LNR_OK;
}

lnr_status lnr_server_poll(lnr_server *srv, lnr_server_result *out, int32_t max, int32_t *count) {
  if (!srv || !count || (max > 0 && !out)) return srv ? fail(srv->ctx, LNR_E_INVALID_ARG, "bad arguments") : LNR_E_INVALID_ARG;
  lnr_status st = use_device(srv->ctx);
  if (st != LNR_OK) return st;
  for (auto &l : srv->lanes) server_collect(srv, l);
  int32_t n = 0;
  while (n < max && !srv->done.empty()) {
    out[n++] = srv->done.front();
    srv->done.pop_front();
  }
  *count = n;
  return LNR_OK;
}

lnr_status lnr_server_pending(const lnr_server *srv, int32_t *pending, int32_t *in_flight) {
  if (!srv) return LNR_E_INVALID_ARG;
  int32_t p = 0, f = 0;
  for (const auto &ss : srv->sessions) {
    p += (ss.open && ss.pending) ? 1 : 0;
    f += (ss.open && ss.in_flight) ? 1 : 0;
  }
  if (pending) *pending = p;
  if (in_flight) *in_flight = f;
  return LNR_OK;
}

}  // extern "C"

