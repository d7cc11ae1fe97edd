// Batched execution (one launch per kernel variant) and the tile autotuner.
//
// A plan holds a device table of image descriptors (any mix of sizes,
// ratios s, windows k and storage types), grouped by kernel variant (window
// class, pixels per strip, storage type, pair table or none), each group
// with the prefix sum of
// its tile counts.  One launch of a kernel specialised for the group's
// variant runs fused search + apply over all of the group's images, one
// workgroup per tile: workgroup g finds the image of tile g by binary search
// over the prefix sums and runs the same per-tile device code as the
// single-image path, so every pixel gets bitwise the same result as a
// single-image launch with the same tile shape.  A batch of one variant
// (frames of a video) is one launch; a mixed batch is one launch per
// variant, enqueued back to back.  One kernel holding every variant would
// carry the register allocation of the largest one, and a persistent loop
// over tiles keeps values live across iterations; both cost occupancy.
// Launching does no allocation, copy or memset, so it can be captured into
// a hipGraph and replayed.
//
// The autotuner times the candidate tile shapes of one (mode, k, s, dtype)
// configuration on a real workload and records the fastest in a
// process-wide cache that plans (and the single-image entry points) consult.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "glu_device.h"
#include "glu_host.h"

namespace glu {

// ---------------------------------------------------------------------------
// autotune cache
// ---------------------------------------------------------------------------
typedef std::tuple<int, int, int, int> TuneKey;  // mode, k, s, dtype
static std::mutex g_tune_mu;
static std::map<TuneKey, int> g_tune;

int tuned_variant(int mode, int k, int s, int dtype) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(TuneKey(mode, k, s, dtype));
  return it == g_tune.end() ? 0 : it->second;
}

static void set_tuned_variant(int mode, int k, int s, int dtype, int v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[TuneKey(mode, k, s, dtype)] = v;
}

// ---------------------------------------------------------------------------
// batch kernel: one workgroup per tile of a variant group
// ---------------------------------------------------------------------------
struct BatchTable {
  const ImgDesc* items;
  int32_t n_items;
  int64_t n_tiles;
  int64_t tile0;  // first tile of this launch (launches of at most kMaxGrid tiles)
  float eps;
};

constexpr int64_t kMaxGrid = int64_t(1) << 30;

__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <int MODE, int KW, int P, typename T, bool TABLE>
__global__ __launch_bounds__(kThreads) void k_batch(const BatchTable tab) {
  extern __shared__ float4 smem[];
  {
    const int64_t t = tab.tile0 + blockIdx.x;
    if (t >= tab.n_tiles) return;
    // image of tile t: last item with tile_begin <= t
    int lo = 0, hi = tab.n_items - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (uniform_i64(tab.items[mid].tile_begin) <= t) lo = mid;
      else hi = mid - 1;
    }
    // the descriptor is the same for the whole workgroup: read it through
    // readfirstlane so that it lives in scalar registers, as kernel
    // arguments do in the single-image launch
    ImgDesc d;
    {
      constexpr int NW = (int)(sizeof(ImgDesc) / 4);
      const uint32_t* src = reinterpret_cast<const uint32_t*>(tab.items + lo);
      uint32_t w[NW];
#pragma unroll
      for (int i = 0; i < NW; ++i) w[i] = (uint32_t)__builtin_amdgcn_readfirstlane((int)src[i]);
      __builtin_memcpy(&d, w, sizeof(ImgDesc));
    }
    const int64_t local = t - d.tile_begin;
    const int ty = (int)(local / d.tiles_x), tx = (int)(local - (int64_t)ty * d.tiles_x);
    search_tile<KW, P, MODE, T, true, TABLE>(d, ty, tx, tab.eps, smem);
  }
}

typedef void (*BatchKernel)(const BatchTable);

template <int MODE, int KW, bool TABLE>
static BatchKernel pick_batch_kwt(int P, int dtype) {
  if (P == 4) return dtype == GLU_F16 ? k_batch<MODE, KW, 4, __half, TABLE> : k_batch<MODE, KW, 4, float, TABLE>;
  if constexpr (KW == 5) {
    if (P == 8) return dtype == GLU_F16 ? k_batch<MODE, KW, 8, __half, TABLE> : k_batch<MODE, KW, 8, float, TABLE>;
  }
  if (P == 3) return dtype == GLU_F16 ? k_batch<MODE, KW, 3, __half, TABLE> : k_batch<MODE, KW, 3, float, TABLE>;
  if (P == 2) return dtype == GLU_F16 ? k_batch<MODE, KW, 2, __half, TABLE> : k_batch<MODE, KW, 2, float, TABLE>;
  return dtype == GLU_F16 ? k_batch<MODE, KW, 1, __half, TABLE> : k_batch<MODE, KW, 1, float, TABLE>;
}

template <int MODE, int KW>
static BatchKernel pick_batch_kw(int P, int dtype, bool table) {
  if constexpr (kernel_has_table(MODE, KW)) {
    if (table) return pick_batch_kwt<MODE, KW, true>(P, dtype);
  }
  return pick_batch_kwt<MODE, KW, false>(P, dtype);
}

template <int MODE>
static BatchKernel pick_batch_m(int k, int P, int dtype, bool table) {
  if (k == 3) return pick_batch_kw<MODE, 3>(P, dtype, table);
  if (k == 5) return pick_batch_kw<MODE, 5>(P, dtype, table);
  if (k == 7) return pick_batch_kw<MODE, 7>(P, dtype, table);
  return pick_batch_kw<MODE, 0>(P, dtype, table);
}

static BatchKernel pick_batch(int mode, int k, int P, int dtype, bool table) {
  return mode == MODE_EXH ? pick_batch_m<MODE_EXH>(k, P, dtype, table) : pick_batch_m<MODE_FAST>(k, P, dtype, table);
}

// One launch of a plan: the images of one kernel variant.
struct BatchGroup {
  BatchKernel kern;
  int32_t first;    // first descriptor of the group in the device table
  int32_t n_items;
  int64_t n_tiles;
  int32_t n_wgs;    // workgroups of the group (one per tile, capped at kMaxGrid)
  size_t lds;       // dynamic LDS bytes (largest tile of the group)
};

}  // namespace glu

using namespace glu;

struct glu_batch_plan {
  ImgDesc* d_items = nullptr;
  int32_t n_items = 0;
  int64_t n_tiles = 0;
  int32_t n_groups = 0;  // workgroups over all launches
  std::vector<glu::BatchGroup> groups;
  int mode = 0;
  float eps = 0.f;
};

namespace glu {

// Builds the descriptor of one item (validated like glu_search_apply).
static glu_status make_item(const glu_batch_item& it, const glu_params& p, int mode, int variant_override,
                            ImgDesc& d, size_t& lds) {
  glu_params ip = p;
  ip.s = it.s;
  ip.k = it.k;
  glu_status st;
  if ((st = check_params(&ip))) return st;
  if ((st = check_image(&it.I, "item I", 3, 3))) return st;
  if ((st = check_image(&it.I_low, "item I_low", 3, 3))) return st;
  if ((st = check_image(&it.T_low, "item T_low", 1, 4))) return st;
  if ((st = check_image(&it.T_hat, "item T_hat", 1, 4))) return st;
  const int H = it.I.height, W = it.I.width;
  const int h = ceil_div(H, it.s), w = ceil_div(W, it.s);
  if (it.I_low.height != h || it.I_low.width != w) return fail(GLU_ERR_SHAPE, "item I_low must be ceil(H/s) x ceil(W/s)");
  if (it.T_low.height != h || it.T_low.width != w) return fail(GLU_ERR_SHAPE, "item T_low must be ceil(H/s) x ceil(W/s)");
  if (it.T_hat.height != H || it.T_hat.width != W) return fail(GLU_ERR_SHAPE, "item T_hat must be H x W");
  if (it.T_hat.channels != it.T_low.channels) return fail(GLU_ERR_SHAPE, "item channel counts differ");
  if (it.I_low.dtype != it.I.dtype || it.T_low.dtype != it.I.dtype || it.T_hat.dtype != it.I.dtype)
    return fail(GLU_ERR_DTYPE, "item dtypes differ");
  const bool store_theta = it.theta.code != nullptr;
  if (store_theta && (st = check_theta(&it.theta, H, W, true))) return st;
  std::memset(&d, 0, sizeof(d));
  d.I = it.I.data;
  d.L = it.I_low.data;
  d.T = it.T_low.data;
  d.That = it.T_hat.data;
  d.code = store_theta ? it.theta.code : nullptr;
  d.alpha = store_theta ? it.theta.alpha : nullptr;
  d.err = nullptr;
  d.I_stride = it.I.row_stride;
  d.L_stride = it.I_low.row_stride;
  d.T_stride = it.T_low.row_stride;
  d.That_stride = it.T_hat.row_stride;
  d.th_stride = store_theta ? it.theta.row_stride : W;
  d.H = H;
  d.W = W;
  d.h = h;
  d.w = w;
  d.s = it.s;
  d.k = it.k;
  d.C = it.T_low.channels;
  d.dtype = it.I.dtype;
  const bool table = uses_pair_table(mode, it.k, it.s);
  const int var = variant_override >= 0 ? variant_override : tuned_variant(p.mode, it.k, it.s, it.I.dtype);
  const TileChoice tc = choose_tile(it.s, it.k, mode, true, table, var);
  fill_tiles(d, tc);
  d.gnu = p.mode == GLU_SEARCH_GNU;
  d.no_degen = (p.flags & GLU_FLAG_NO_DEGENERATE) != 0;
  d.vec = launch_vec_flags(d, tc.P, dtype_size((glu_dtype)it.I.dtype));
  d.variant = kernel_variant(it.k, tc.P, mode, it.I.dtype, table);
  lds = 16 * (size_t)search_tile_words(tc.tqy, tc.tqx, it.k, mode, true, table);
  return GLU_OK;
}

static glu_status plan_build(const glu_batch_item* items, int32_t n, const glu_params* p, int variant_override,
                             glu_batch_plan** out) {
  glu_status st;
  if (!out) return fail(GLU_ERR_NULL, "out is NULL");
  *out = nullptr;
  if (!items && n > 0) return fail(GLU_ERR_NULL, "items is NULL");
  if (n < 0) return fail(GLU_ERR_PARAM, "n < 0");
  if (!p) return fail(GLU_ERR_NULL, "params is NULL");
  glu_params base = *p;
  base.s = 1;
  base.k = 3;
  if ((st = check_params(&base))) return st;
  const int mode = p->mode == GLU_SEARCH_EXHAUSTIVE ? MODE_EXH : MODE_FAST;
  std::vector<ImgDesc> all;
  std::vector<size_t> all_lds;
  all.reserve(n);
  for (int i = 0; i < n; ++i) {
    ImgDesc d;
    size_t l;
    if ((st = make_item(items[i], *p, mode, variant_override, d, l))) {
      return fail(st, "item %d: %s", i, glu_last_error());
    }
    if ((int64_t)d.H * d.W == 0) continue;
    all.push_back(d);
    all_lds.push_back(l);
  }
  // group by kernel variant, keeping the items' order inside a group
  std::vector<int> order(all.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return all[a].variant < all[b].variant; });
  std::vector<ImgDesc> host;
  host.reserve(all.size());
  std::vector<BatchGroup> groups;
  int64_t tiles_total = 0;
  for (size_t j = 0; j < order.size(); ++j) {
    ImgDesc d = all[order[j]];
    if (groups.empty() || host.back().variant != d.variant) {
      BatchGroup g{};
      g.kern = pick_batch(mode, d.k, search_strip_pixels(d.s, d.k, mode == MODE_EXH), d.dtype,
                          uses_pair_table(mode, d.k, d.s));
      g.first = (int32_t)host.size();
      g.lds = 16;
      groups.push_back(g);
    }
    BatchGroup& g = groups.back();
    d.tile_begin = g.n_tiles;
    g.n_tiles += (int64_t)d.tiles_x * d.tiles_y;
    g.n_items += 1;
    g.lds = std::max(g.lds, all_lds[order[j]]);
    tiles_total += (int64_t)d.tiles_x * d.tiles_y;
    host.push_back(d);
  }
  glu_batch_plan* plan = new (std::nothrow) glu_batch_plan();
  if (!plan) return fail(GLU_ERR_NOMEM, "plan");
  plan->n_items = (int32_t)host.size();
  plan->n_tiles = tiles_total;
  plan->mode = mode;
  plan->eps = p->eps;
  if (!host.empty()) {
    hipError_t e = hipMalloc(&plan->d_items, sizeof(ImgDesc) * host.size());
    if (e != hipSuccess) {
      delete plan;
      return fail(GLU_ERR_NOMEM, "descriptor table: %s", hipGetErrorString(e));
    }
    e = hipMemcpy(plan->d_items, host.data(), sizeof(ImgDesc) * host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      hipFree(plan->d_items);
      delete plan;
      return hip_fail(e, "descriptor upload");
    }
    int64_t wgs = 0;
    for (BatchGroup& g : groups) {
      g.n_wgs = (int32_t)std::min<int64_t>(g.n_tiles, kMaxGrid);
      wgs += g.n_tiles;
    }
    plan->n_groups = (int32_t)std::min<int64_t>(wgs, 0x7fffffff);
  }
  plan->groups = std::move(groups);
  *out = plan;
  return GLU_OK;
}

static glu_status plan_launch(const glu_batch_plan* plan, void* stream) {
  if (!plan) return fail(GLU_ERR_NULL, "plan is NULL");
  for (const BatchGroup& g : plan->groups) {
    for (int64_t t0 = 0; t0 < g.n_tiles; t0 += kMaxGrid) {
      BatchTable t;
      t.items = plan->d_items + g.first;
      t.n_items = g.n_items;
      t.n_tiles = g.n_tiles;
      t.tile0 = t0;
      t.eps = plan->eps;
      const unsigned grid = (unsigned)std::min<int64_t>(g.n_tiles - t0, kMaxGrid);
      hipLaunchKernelGGL(g.kern, dim3(grid), dim3(kThreads), g.lds, (hipStream_t)stream, t);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "batch launch");
    }
  }
  return GLU_OK;
}

}  // namespace glu

extern "C" {

glu_status glu_batch_plan_create(const glu_batch_item* items, int32_t n, const glu_params* p,
                                 glu_batch_plan** out) {
  clear_error();
  return plan_build(items, n, p, -1, out);
}

glu_status glu_batch_plan_launch(const glu_batch_plan* plan, void* stream) {
  clear_error();
  return plan_launch(plan, stream);
}

void glu_batch_plan_destroy(glu_batch_plan* plan) {
  if (!plan) return;
  if (plan->d_items) hipFree(plan->d_items);
  delete plan;
}

glu_status glu_batch_plan_info(const glu_batch_plan* plan, int64_t* n_tiles, int32_t* n_groups) {
  clear_error();
  if (!plan) return fail(GLU_ERR_NULL, "plan is NULL");
  if (n_tiles) *n_tiles = plan->n_tiles;
  if (n_groups) *n_groups = plan->n_groups;
  return GLU_OK;
}

glu_status glu_autotune(const glu_batch_item* item, const glu_params* p, int32_t* chosen, void* stream) {
  clear_error();
  if (!item || !p) return fail(GLU_ERR_NULL, "item/params is NULL");
  const int mode = p->mode == GLU_SEARCH_EXHAUSTIVE ? MODE_EXH : MODE_FAST;
  hipStream_t sm = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(GLU_ERR_HIP, "event create");
  float best_ms = 1e30f;
  int best = 0;
  glu_status st = GLU_OK;
  for (int v = 0; v < n_tile_variants() && st == GLU_OK; ++v) {
    glu_batch_plan* plan = nullptr;
    if ((st = plan_build(item, 1, p, v, &plan))) break;
    for (int i = 0; i < 2 && st == GLU_OK; ++i) st = plan_launch(plan, stream);  // warm-up
    const int reps = 5;
    hipEventRecord(e0, sm);
    for (int i = 0; i < reps && st == GLU_OK; ++i) st = plan_launch(plan, stream);
    hipEventRecord(e1, sm);
    hipError_t e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    glu_batch_plan_destroy(plan);
    if (e != hipSuccess) st = hip_fail(e, "autotune timing");
    if (st == GLU_OK && ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st) return st;
  set_tuned_variant(p->mode, item->k, item->s, item->I.dtype, best);
  if (chosen) *chosen = best;
  return GLU_OK;
}

glu_status glu_autotune_save(const char* path) {
  clear_error();
  if (!path) return fail(GLU_ERR_NULL, "path is NULL");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(GLU_ERR_PARAM, "cannot write %s", path);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::fprintf(f, "{\"arch\": \"gfx950\", \"entries\": [");
  bool first = true;
  for (const auto& kv : g_tune) {
    std::fprintf(f, "%s{\"mode\": %d, \"k\": %d, \"s\": %d, \"dtype\": %d, \"variant\": %d}", first ? "" : ", ",
                 std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
                 kv.second);
    first = false;
  }
  std::fprintf(f, "]}\n");
  std::fclose(f);
  return GLU_OK;
}

glu_status glu_autotune_load(const char* path) {
  clear_error();
  if (!path) return fail(GLU_ERR_NULL, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(GLU_ERR_PARAM, "cannot read %s", path);
  std::string s;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, n);
  std::fclose(f);
  // entries are flat objects with five integer fields
  size_t pos = 0;
  int loaded = 0;
  while ((pos = s.find("{\"mode\"", pos)) != std::string::npos) {
    int m, k, sv, dt, v;
    if (std::sscanf(s.c_str() + pos, "{\"mode\": %d, \"k\": %d, \"s\": %d, \"dtype\": %d, \"variant\": %d}", &m, &k,
                    &sv, &dt, &v) == 5) {
      if (v >= 0 && v < n_tile_variants()) {
        set_tuned_variant(m, k, sv, dt, v);
        ++loaded;
      }
    }
    pos += 7;
  }
  if (loaded == 0 && s.find("\"entries\"") == std::string::npos) return fail(GLU_ERR_PARAM, "not a tune file");
  return GLU_OK;
}

}  // extern "C"
