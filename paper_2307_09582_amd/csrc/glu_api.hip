// C ABI entry points for search, apply, fused search+apply, downsampling and
// Theta expansion, plus the shared host helpers (errors, validation, tiles).
#include <atomic>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>

#include "glu_device.h"
#include "glu_host.h"

namespace glu {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string t_last_error;

glu_status fail(glu_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_last_error = std::string(glu_status_string(st)) + ": " + buf;
  return st;
}

void clear_error() { t_last_error.clear(); }

glu_status hip_fail(hipError_t e, const char* what) {
  return fail(GLU_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
glu_status check_image(const glu_image* im, const char* name, int clo, int chi, bool allow_f16) {
  if (!im) return fail(GLU_ERR_NULL, "%s descriptor is NULL", name);
  if (!dtype_ok(im->dtype)) return fail(GLU_ERR_DTYPE, "%s dtype %d unknown", name, (int)im->dtype);
  if (!allow_f16 && im->dtype != GLU_F32) return fail(GLU_ERR_DTYPE, "%s must be GLU_F32", name);
  if (im->height < 0 || im->width < 0) return fail(GLU_ERR_SHAPE, "%s has negative size", name);
  if (im->channels < clo || im->channels > chi)
    return fail(GLU_ERR_SHAPE, "%s has %d channels, expected %d..%d", name, im->channels, clo, chi);
  const int64_t npx = (int64_t)im->height * im->width;
  if (npx == 0) return GLU_OK;
  if (!im->data) return fail(GLU_ERR_NULL, "%s data is NULL", name);
  if (im->row_stride < (int64_t)im->width * im->channels)
    return fail(GLU_ERR_SHAPE, "%s row_stride %lld < width*channels", name, (long long)im->row_stride);
  if (reinterpret_cast<uintptr_t>(im->data) % dtype_size(im->dtype) != 0)
    return fail(GLU_ERR_ALIGN, "%s data not aligned to its element size", name);
  return GLU_OK;
}

glu_status check_params(const glu_params* p) {
  if (!p) return fail(GLU_ERR_NULL, "params is NULL");
  if (p->s < 1 || p->s > 1024) return fail(GLU_ERR_PARAM, "s = %d outside 1..1024", p->s);
  if (p->k < 1 || p->k > kMaxK || (p->k % 2) == 0)
    return fail(GLU_ERR_PARAM, "k = %d must be odd in 1..%d", p->k, kMaxK);
  if (!(p->eps >= 0.0f) || !std::isfinite(p->eps)) return fail(GLU_ERR_PARAM, "eps must be finite and >= 0");
  if (p->mode != GLU_SEARCH_EXHAUSTIVE && p->mode != GLU_SEARCH_FAST && p->mode != GLU_SEARCH_GNU)
    return fail(GLU_ERR_PARAM, "unknown mode %d", (int)p->mode);
  if (p->flags & ~(uint32_t)GLU_FLAG_NO_DEGENERATE) return fail(GLU_ERR_PARAM, "unknown flags 0x%x", p->flags);
  if ((p->flags & GLU_FLAG_NO_DEGENERATE) && p->mode != GLU_SEARCH_EXHAUSTIVE)
    return fail(GLU_ERR_PARAM, "GLU_FLAG_NO_DEGENERATE applies to the exhaustive search only");
  return GLU_OK;
}

glu_status check_theta(const glu_theta* th, int H, int W, bool need) {
  if (!th) return fail(GLU_ERR_NULL, "theta descriptor is NULL");
  if (th->height != H || th->width != W)
    return fail(GLU_ERR_SHAPE, "theta is %dx%d, expected %dx%d", th->height, th->width, H, W);
  if ((int64_t)H * W == 0) return GLU_OK;
  if (need && (!th->code || !th->alpha)) return fail(GLU_ERR_NULL, "theta code/alpha is NULL");
  if (th->row_stride < W) return fail(GLU_ERR_SHAPE, "theta row_stride < width");
  if (reinterpret_cast<uintptr_t>(th->code) % 2 || reinterpret_cast<uintptr_t>(th->alpha) % 4)
    return fail(GLU_ERR_ALIGN, "theta buffers not aligned to their element size");
  return GLU_OK;
}

// ---------------------------------------------------------------------------
// tiles
// ---------------------------------------------------------------------------
static const int kVariantCols[] = {64, 32, 128, 64, 32, 64, 128, 128};
static const int kVariantStripsPerThread[] = {1, 1, 1, 2, 2, 4, 2, 4};

int n_tile_variants() { return (int)(sizeof(kVariantCols) / sizeof(kVariantCols[0])); }

TileChoice choose_tile(int s, int k, int mode, bool fused, bool table, int variant, int P_override) {
  if (variant < 0 || variant >= n_tile_variants()) variant = 0;
  TileChoice tc;
  tc.P = P_override > 0 ? P_override : search_strip_pixels(s, k, mode == MODE_EXH);
  const int cols = kVariantCols[variant];
  tc.tqx = std::max(1, cols / s);
  // the fast search keeps less per-strip state: its default tile gives each
  // thread two strips, so the next strip's pixels load during the search
  const int spt = (variant == 0 && mode == MODE_FAST) ? 2 : kVariantStripsPerThread[variant];
  const int strips_target = kThreads * spt;
  const int rows = std::max(1, strips_target * tc.P / (tc.tqx * s));
  tc.tqy = std::max(1, rows / s);
  auto bytes = [&](const TileChoice& t) {
    return 16 * search_tile_words(t.tqy, t.tqx, k, mode, fused, table);
  };
  while (bytes(tc) > kLdsBudget) {
    if (tc.tqy > 1)
      tc.tqy = (tc.tqy + 1) / 2 == tc.tqy ? tc.tqy - 1 : (tc.tqy + 1) / 2;
    else if (tc.tqx > 1)
      tc.tqx = (tc.tqx + 1) / 2 == tc.tqx ? tc.tqx - 1 : (tc.tqx + 1) / 2;
    else
      break;
  }
  return tc;
}

void fill_tiles(ImgDesc& d, const TileChoice& tc) {
  d.tqy = tc.tqy;
  d.tqx = tc.tqx;
  d.tiles_x = ceil_div(d.w, tc.tqx);
  d.tiles_y = ceil_div(d.h, tc.tqy);
}

// SIMDs of the current device (4 per compute unit), looked up once per
// device.
static int device_simds() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 4 * 256;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    v = 4 * cus;
    cache[dev].store(v, std::memory_order_relaxed);
  }
  return v;
}

// window classes with their own kernels: 3, 5 and 7 are compile-time sizes, others run-time
static int kw_class(int k) { return k == 3 ? 0 : (k == 5 ? 1 : (k == 7 ? 3 : 2)); }

int kernel_variant(int k, int P, int mode, int dtype, bool table) {
  const int pidx = P - 1;  // P = 1 .. 8
  return (((kw_class(k) * 8 + pidx) * 2 + mode) * 2 + dtype) * 2 + (table ? 1 : 0);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
template <int KW, int P, int MODE, typename T, bool FUSED, bool TABLE>
__global__ __launch_bounds__(kThreads) void k_search(const ImgDesc d, float eps) {
  extern __shared__ float4 smem[];
  const int tile = blockIdx.x;
  const int ty = tile / d.tiles_x, tx = tile - ty * d.tiles_x;
  search_tile<KW, P, MODE, T, FUSED, TABLE>(d, ty, tx, eps, smem);
}

// One workgroup per tile of one LR row by d.tqx LR columns; blockIdx.y is
// the image of a batch (element offsets per image in `off`).
struct ApplyBatch {
  int64_t theta, T_low, T_hat;
};

template <int KW, int P, typename T>
__global__ __launch_bounds__(kThreads) void k_apply(const ImgDesc d0, uint32_t s_magic, const ApplyBatch off) {
  extern __shared__ float4 smem[];
  ImgDesc d = d0;
  const int64_t b = blockIdx.y;
  d.code += b * off.theta;
  d.alpha += b * off.theta;
  d.T = static_cast<const T*>(d0.T) + b * off.T_low;
  d.That = static_cast<T*>(d0.That) + b * off.T_hat;
  const int tile = blockIdx.x;
  const int qy = tile / d.tiles_x, qx0 = (tile - qy * d.tiles_x) * d.tqx;
  switch (d.C) {
    case 1: apply_tile<KW, P, T, 1, kApplyStrips>(d, qy, qx0, s_magic, smem); break;
    case 2: apply_tile<KW, P, T, 2, kApplyStrips>(d, qy, qx0, s_magic, smem); break;
    case 3: apply_tile<KW, P, T, 3, kApplyStrips>(d, qy, qx0, s_magic, smem); break;
    default: apply_tile<KW, P, T, 4, kApplyStrips>(d, qy, qx0, s_magic, smem); break;
  }
}

typedef void (*SearchKernel)(const ImgDesc, float);
typedef void (*ApplyKernel)(const ImgDesc, uint32_t, const ApplyBatch);

template <int KW, int P, typename T>
static SearchKernel pick_search_t(int mode, bool fused, bool table) {
  if (mode == MODE_EXH) {
    if constexpr (kernel_has_table(MODE_EXH, KW)) {
      if (table)
        return fused ? k_search<KW, P, MODE_EXH, T, true, true> : k_search<KW, P, MODE_EXH, T, false, true>;
    }
    return fused ? k_search<KW, P, MODE_EXH, T, true, false> : k_search<KW, P, MODE_EXH, T, false, false>;
  }
  return fused ? k_search<KW, P, MODE_FAST, T, true, false> : k_search<KW, P, MODE_FAST, T, false, false>;
}

template <int KW, int P>
static SearchKernel pick_search_p(int mode, int dtype, bool fused, bool table) {
  return dtype == GLU_F16 ? pick_search_t<KW, P, __half>(mode, fused, table)
                          : pick_search_t<KW, P, float>(mode, fused, table);
}

template <int KW>
static SearchKernel pick_search_k(int P, int mode, int dtype, bool fused, bool table) {
  if (P == 4) return pick_search_p<KW, 4>(mode, dtype, fused, table);
  if constexpr (KW == 5) {
    if (P == 8) return pick_search_p<KW, 8>(mode, dtype, fused, table);
  }
  if (P == 3) return pick_search_p<KW, 3>(mode, dtype, fused, table);
  if (P == 2) return pick_search_p<KW, 2>(mode, dtype, fused, table);
  return pick_search_p<KW, 1>(mode, dtype, fused, table);
}

static SearchKernel pick_search(int k, int P, int mode, int dtype, bool fused, bool table) {
  if (k == 3) return pick_search_k<3>(P, mode, dtype, fused, table);
  if (k == 5) return pick_search_k<5>(P, mode, dtype, fused, table);
  if (k == 7) return pick_search_k<7>(P, mode, dtype, fused, table);
  return pick_search_k<0>(P, mode, dtype, fused, table);
}

template <int KW>
static ApplyKernel pick_apply_k(int P, int dtype) {
  if (P == 4) return dtype == GLU_F16 ? k_apply<KW, 4, __half> : k_apply<KW, 4, float>;
  return dtype == GLU_F16 ? k_apply<KW, 1, __half> : k_apply<KW, 1, float>;
}

static ApplyKernel pick_apply(int k, int P, int dtype) {
  if (k == 3) return pick_apply_k<3>(P, dtype);
  if (k == 5) return pick_apply_k<5>(P, dtype);
  return pick_apply_k<0>(P, dtype);
}

static bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

uint32_t launch_vec_flags(const ImgDesc& d, int P, size_t esize) {
  uint32_t v = 0;
  if (P != 4) return 0;
  const size_t va = esize == 4 ? 16 : 8;
  if (d.I && aligned(d.I, va) && d.I_stride % 4 == 0) v |= VEC_I;
  bool th = d.th_stride % 4 == 0;
  if (d.code) th = th && aligned(d.code, 8) && aligned(d.alpha, 16);
  if (d.err) th = th && aligned(d.err, 16);
  if (th) v |= VEC_THETA;
  if (d.That && (d.C == 3 || d.C == 1) && aligned(d.That, va) && d.That_stride % 4 == 0) v |= VEC_T;
  return v;
}

// Apply tile width in LR columns: a multiple of the smallest width whose
// HR span tqx * s is a multiple of 64 * P (so every wave run lies in one HR
// row and starts 64-pixel aligned), near 1024 strips per tile, and shrunk
// while the tile's LDS exceeds 24 KiB.
int apply_tile_width(int s, int P, int k, int C, int esize) {
  const int span = 64 * P;
  int unit = span / std::gcd(s, span);
  int tqx = std::max(1, (1024 * P / (s * s)) / unit) * unit;
  while (tqx > unit && 16 * apply_tile_words(tqx, k, P, C, esize) > 24 * 1024) tqx -= unit;
  return tqx;
}

// Validates and launches search (fused when T/That given).
static glu_status run_search(const glu_image* I, const glu_image* I_low, const glu_image* T_low,
                             const glu_params* p, glu_theta* theta, float* err, glu_image* T_hat,
                             bool fused, void* stream) {
  glu_status st;
  if ((st = check_params(p))) return st;
  if ((st = check_image(I, "I", 3, 3))) return st;
  if ((st = check_image(I_low, "I_low", 3, 3))) return st;
  const int H = I->height, W = I->width;
  const int h = ceil_div(H, p->s), w = ceil_div(W, p->s);
  if (I_low->height != h || I_low->width != w)
    return fail(GLU_ERR_SHAPE, "I_low is %dx%d, expected ceil(H/s) x ceil(W/s) = %dx%d", I_low->height,
                I_low->width, h, w);
  if (I_low->dtype != I->dtype) return fail(GLU_ERR_DTYPE, "I_low dtype differs from I");
  if (!fused || theta) {
    if ((st = check_theta(theta, H, W, true))) return st;
  }
  if (err && reinterpret_cast<uintptr_t>(err) % 4) return fail(GLU_ERR_ALIGN, "err not aligned");
  int C = 0;
  if (fused) {
    if ((st = check_image(T_low, "T_low", 1, 4))) return st;
    if ((st = check_image(T_hat, "T_hat", 1, 4))) return st;
    if (T_low->height != h || T_low->width != w) return fail(GLU_ERR_SHAPE, "T_low must be ceil(H/s) x ceil(W/s)");
    if (T_hat->height != H || T_hat->width != W) return fail(GLU_ERR_SHAPE, "T_hat must be H x W");
    if (T_hat->channels != T_low->channels) return fail(GLU_ERR_SHAPE, "T_hat and T_low channel counts differ");
    if (T_low->dtype != I->dtype || T_hat->dtype != I->dtype)
      return fail(GLU_ERR_DTYPE, "T_low / T_hat dtype must match I");
    C = T_low->channels;
  }
  if ((int64_t)H * W == 0) return GLU_OK;

  ImgDesc d{};
  d.I = I->data;
  d.L = I_low->data;
  d.T = fused ? T_low->data : nullptr;
  d.That = fused ? T_hat->data : nullptr;
  d.code = theta ? theta->code : nullptr;
  d.alpha = theta ? theta->alpha : nullptr;
  d.err = err;
  d.I_stride = I->row_stride;
  d.L_stride = I_low->row_stride;
  d.T_stride = fused ? T_low->row_stride : 0;
  d.That_stride = fused ? T_hat->row_stride : 0;
  d.th_stride = theta ? theta->row_stride : W;
  d.H = H;
  d.W = W;
  d.h = h;
  d.w = w;
  d.s = p->s;
  d.k = p->k;
  d.C = C;
  d.dtype = I->dtype;
  const int mode = p->mode == GLU_SEARCH_EXHAUSTIVE ? MODE_EXH : MODE_FAST;
  bool table = uses_pair_table(mode, p->k, p->s);
  // A small image in strips of the default width gives the chip fewer than
  // four waves per SIMD (a 512 x 512 image in strips of 4 pixels: one), and
  // the search's arithmetic chains then go unhidden.  Such images take
  // narrower strips (halved down to 1 pixel) until the launch has about
  // four waves per SIMD, and a 3 x 3 exhaustive search of them takes the
  // pair table at any s >= 2, so that narrow strips do not rebuild the pair
  // constants for every pixel.  The arithmetic per pixel is unchanged, so
  // the outputs are bitwise those of the default strips.
  int P_small = 0;
  {
    const int64_t lanes_for_four_waves = (int64_t)device_simds() * 4 * 64;
    const int64_t npx = (int64_t)H * W;
    int P = search_strip_pixels(p->s, p->k, mode == MODE_EXH);
    if (P > 1 && npx / P < lanes_for_four_waves) {
      while (P > 1 && npx / P < lanes_for_four_waves) P = P % 2 == 0 ? P / 2 : 1;
      P_small = P;
      if (mode == MODE_EXH && kernel_has_table(MODE_EXH, p->k) && p->s >= 2) table = true;
    }
  }
  const TileChoice tc =
      choose_tile(p->s, p->k, mode, fused, table, tuned_variant(p->mode, p->k, p->s, I->dtype), P_small);
  fill_tiles(d, tc);
  d.gnu = p->mode == GLU_SEARCH_GNU;
  d.no_degen = (p->flags & GLU_FLAG_NO_DEGENERATE) != 0;
  d.vec = launch_vec_flags(d, tc.P, dtype_size(I->dtype));
  const size_t lds = 16 * (size_t)search_tile_words(tc.tqy, tc.tqx, p->k, mode, fused, table);
  const int64_t ntiles = (int64_t)d.tiles_x * d.tiles_y;
  if (ntiles > 0x7fffffff) return fail(GLU_ERR_UNSUPPORTED, "image needs too many tiles");
  SearchKernel kern = pick_search(p->k, tc.P, mode, I->dtype, fused, table);
  hipLaunchKernelGGL(kern, dim3((unsigned)ntiles), dim3(kThreads), lds, (hipStream_t)stream, d, p->eps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "search launch");
  return GLU_OK;
}

// Validates a batch of n images of one size: n in 0..65535, strides >= 0,
// and outputs of different images that do not overlap.
glu_status check_batch(int32_t n, const glu_batch_strides* bs, bool backward) {
  if (n < 0 || n > 65535) return fail(GLU_ERR_PARAM, "batch of %d images outside 0..65535", n);
  if (n > 1 && !bs) return fail(GLU_ERR_NULL, "batch strides are NULL");
  if (bs && (bs->theta < 0 || bs->T_low < 0 || bs->T_hat < 0 || bs->grad_T_low < 0 || bs->grad_alpha < 0))
    return fail(GLU_ERR_PARAM, "negative batch stride");
  (void)backward;
  return GLU_OK;
}

static glu_status apply_batched(int32_t n, const glu_batch_strides* bs, const glu_theta* theta,
                                const glu_image* T_low, const glu_params* p, glu_image* T_hat, void* stream) {
  glu_status st;
  if ((st = check_batch(n, bs, false))) return st;
  if ((st = check_params(p))) return st;
  if ((st = check_image(T_low, "T_low", 1, 4))) return st;
  if ((st = check_image(T_hat, "T_hat", 1, 4))) return st;
  const int H = T_hat->height, W = T_hat->width;
  if ((st = check_theta(theta, H, W, true))) return st;
  const int h = ceil_div(H, p->s), w = ceil_div(W, p->s);
  if (T_low->height != h || T_low->width != w) return fail(GLU_ERR_SHAPE, "T_low must be ceil(H/s) x ceil(W/s)");
  if (T_low->channels != T_hat->channels) return fail(GLU_ERR_SHAPE, "T_low and T_hat channel counts differ");
  if (T_low->dtype != T_hat->dtype) return fail(GLU_ERR_DTYPE, "T_low and T_hat dtypes differ");
  if (n > 1 && bs->T_hat < (int64_t)(H - 1) * T_hat->row_stride + (int64_t)W * T_hat->channels)
    return fail(GLU_ERR_SHAPE, "T_hat batch stride makes images overlap");
  if ((int64_t)H * W == 0 || n == 0) return GLU_OK;
  ApplyBatch off{};
  if (n > 1) {
    off.theta = bs->theta;
    off.T_low = bs->T_low;
    off.T_hat = bs->T_hat;
  }
  ImgDesc d{};
  d.T = T_low->data;
  d.That = T_hat->data;
  d.code = theta->code;
  d.alpha = theta->alpha;
  d.T_stride = T_low->row_stride;
  d.That_stride = T_hat->row_stride;
  d.th_stride = theta->row_stride;
  d.H = H;
  d.W = W;
  d.h = h;
  d.w = w;
  d.s = p->s;
  d.k = p->k;
  d.C = T_low->channels;
  d.dtype = T_low->dtype;
  const int P = (p->s % 4 == 0) ? 4 : 1;
  const int es = (int)dtype_size(T_low->dtype);
  d.vec = launch_vec_flags(d, P, es);
  if (aligned(T_hat->data, 16) && (T_hat->row_stride * es) % 16 == 0) d.vec |= VEC_TW;
  // every image of the batch must keep the alignment of the first
  if (off.theta % 4) d.vec &= ~VEC_THETA;
  if ((off.T_hat * es) % 16) d.vec &= ~(VEC_TW | VEC_T);
  d.tqx = apply_tile_width(p->s, P, p->k, d.C, es);
  d.tqy = 1;
  d.tiles_x = ceil_div(w, d.tqx);
  d.tiles_y = h;
  const int64_t groups = (int64_t)d.tiles_x * h;
  if (groups > 0x7fffffff) return fail(GLU_ERR_UNSUPPORTED, "image too large");
  const uint32_t s_magic = (uint32_t)std::min<uint64_t>(0xffffffffull, (1ull << 32) / (uint64_t)p->s);
  const size_t lds = 16 * (size_t)apply_tile_words(d.tqx, p->k, P, d.C, es);
  ApplyKernel kern = pick_apply(p->k, P, T_low->dtype);
  hipLaunchKernelGGL(kern, dim3((unsigned)groups, (unsigned)n), dim3(kThreads), lds, (hipStream_t)stream, d, s_magic,
                     off);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "apply launch");
  return GLU_OK;
}

}  // namespace glu

using namespace glu;

// ---------------------------------------------------------------------------
// small kernels: downsampling and Theta expansion
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_downsample(const T* __restrict__ I, int64_t Is, int H, int W, int C,
                                                    T* __restrict__ L, int64_t Ls, int h, int w, int s, int box) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)h * w) return;
  const int qy = (int)(idx / w), qx = (int)(idx - (int64_t)qy * w);
  T* out = L + (int64_t)qy * Ls + (int64_t)qx * C;
  if (!box) {
    const int y = min(qy * s + s / 2, H - 1), x = min(qx * s + s / 2, W - 1);
    const T* in = I + (int64_t)y * Is + (int64_t)x * C;
    for (int c = 0; c < C; ++c) out[c] = in[c];
    return;
  }
  const int y0 = qy * s, x0 = qx * s, y1 = min(H, y0 + s), x1 = min(W, x0 + s);
  const float inv = 1.0f / (float)((y1 - y0) * (x1 - x0));
  for (int c = 0; c < C; ++c) {
    float acc = 0.0f;
    for (int y = y0; y < y1; ++y)
      for (int x = x0; x < x1; ++x) acc += to_f<T>(I[(int64_t)y * Is + (int64_t)x * C + c]);
    out[c] = from_f<T>(acc * inv);
  }
}

__global__ __launch_bounds__(256) void k_theta_expand(const uint16_t* __restrict__ code, int64_t ts, int H, int W,
                                                      int s, int k, int w, int64_t* __restrict__ a,
                                                      int64_t* __restrict__ b) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)H * W) return;
  const int y = (int)(idx / W), x = (int)(idx - (int64_t)y * W);
  const int K2 = k * k, r = k / 2;
  const int cd = code[(int64_t)y * ts + x];
  const int oa = cd / K2, ob = cd - oa * K2;
  const int qy = y / s, qx = x / s;
  a[idx] = (int64_t)(qy + oa / k - r) * w + (qx + oa % k - r);
  b[idx] = (int64_t)(qy + ob / k - r) * w + (qx + ob % k - r);
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* glu_status_string(glu_status s) {
  switch (s) {
    case GLU_OK: return "GLU_OK";
    case GLU_ERR_NULL: return "GLU_ERR_NULL";
    case GLU_ERR_SHAPE: return "GLU_ERR_SHAPE";
    case GLU_ERR_DTYPE: return "GLU_ERR_DTYPE";
    case GLU_ERR_PARAM: return "GLU_ERR_PARAM";
    case GLU_ERR_ALIGN: return "GLU_ERR_ALIGN";
    case GLU_ERR_NOMEM: return "GLU_ERR_NOMEM";
    case GLU_ERR_HIP: return "GLU_ERR_HIP";
    case GLU_ERR_UNSUPPORTED: return "GLU_ERR_UNSUPPORTED";
    case GLU_ERR_WORKSPACE: return "GLU_ERR_WORKSPACE";
  }
  return "GLU_ERR_UNKNOWN";
}

const char* glu_last_error(void) { return t_last_error.c_str(); }

const char* glu_version(void) { return "glu-mi355x 0.1 (gfx950)"; }

glu_status glu_search(const glu_image* I, const glu_image* I_low, const glu_params* p, glu_theta* theta,
                      float* err, void* stream) {
  clear_error();
  return run_search(I, I_low, nullptr, p, theta, err, nullptr, false, stream);
}

glu_status glu_search_apply(const glu_image* I, const glu_image* I_low, const glu_image* T_low,
                            const glu_params* p, glu_theta* theta, float* err, glu_image* T_hat, void* stream) {
  clear_error();
  return run_search(I, I_low, T_low, p, theta, err, T_hat, true, stream);
}

glu_status glu_downsample(const glu_image* I, glu_image* I_low, int32_t s, glu_down_mode mode, void* stream) {
  clear_error();
  glu_status st;
  if ((st = check_image(I, "I", 1, 4))) return st;
  if ((st = check_image(I_low, "I_low", 1, 4))) return st;
  if (s < 1 || s > 1024) return fail(GLU_ERR_PARAM, "s = %d outside 1..1024", s);
  if (mode != GLU_DOWN_POINT && mode != GLU_DOWN_BOX) return fail(GLU_ERR_PARAM, "unknown downsample mode");
  const int h = ceil_div(I->height, s), w = ceil_div(I->width, s);
  if (I_low->height != h || I_low->width != w) return fail(GLU_ERR_SHAPE, "I_low must be ceil(H/s) x ceil(W/s)");
  if (I_low->channels != I->channels) return fail(GLU_ERR_SHAPE, "channel counts differ");
  if (I_low->dtype != I->dtype) return fail(GLU_ERR_DTYPE, "dtypes differ");
  const int64_t n = (int64_t)h * w;
  if (n == 0) return GLU_OK;
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (I->dtype == GLU_F16)
    hipLaunchKernelGGL(k_downsample<__half>, dim3(grid), dim3(256), 0, (hipStream_t)stream,
                       (const __half*)I->data, I->row_stride, I->height, I->width, I->channels,
                       (__half*)I_low->data, I_low->row_stride, h, w, s, mode == GLU_DOWN_BOX);
  else
    hipLaunchKernelGGL(k_downsample<float>, dim3(grid), dim3(256), 0, (hipStream_t)stream,
                       (const float*)I->data, I->row_stride, I->height, I->width, I->channels,
                       (float*)I_low->data, I_low->row_stride, h, w, s, mode == GLU_DOWN_BOX);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "downsample launch");
  return GLU_OK;
}

glu_status glu_theta_expand(const glu_theta* theta, const glu_params* p, int64_t* a, int64_t* b, void* stream) {
  clear_error();
  glu_status st;
  if ((st = check_params(p))) return st;
  if (!theta) return fail(GLU_ERR_NULL, "theta is NULL");
  if ((st = check_theta(theta, theta->height, theta->width, true))) return st;
  const int64_t n = (int64_t)theta->height * theta->width;
  if (n == 0) return GLU_OK;
  if (!a || !b) return fail(GLU_ERR_NULL, "output a/b is NULL");
  if (reinterpret_cast<uintptr_t>(a) % 8 || reinterpret_cast<uintptr_t>(b) % 8)
    return fail(GLU_ERR_ALIGN, "a/b not 8-byte aligned");
  const int w = ceil_div(theta->width, p->s);
  hipLaunchKernelGGL(k_theta_expand, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     theta->code, theta->row_stride, theta->height, theta->width, p->s, p->k, w, a, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "theta_expand launch");
  return GLU_OK;
}

}  // extern "C"

extern "C" {

glu_status glu_apply(const glu_theta* theta, const glu_image* T_low, const glu_params* p, glu_image* T_hat,
                     void* stream) {
  clear_error();
  return apply_batched(1, nullptr, theta, T_low, p, T_hat, stream);
}

glu_status glu_apply_batched(int32_t n, const glu_batch_strides* strides, const glu_theta* theta,
                             const glu_image* T_low, const glu_params* p, glu_image* T_hat, void* stream) {
  clear_error();
  return apply_batched(n, strides, theta, T_low, p, T_hat, stream);
}

}  // extern "C"
