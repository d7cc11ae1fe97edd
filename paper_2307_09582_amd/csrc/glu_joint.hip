// Joint optimisation of down- and upsampling (Sec. 3.3, Algorithm 2).
//
// Each round:
//   1. search the whole image with the current I_low (the product search
//      kernel) -> Theta, E;
//   2. large-error set {p : E_p > tau}: marked and compacted in raster order
//      (per-tile counts, one exclusive scan, ordered scatter);
//   3. its 8-connected components by a lock-free union-find over the
//      compacted pixels (atomicMin links a larger root under a smaller one,
//      so every component ends with its smallest pixel index, i.e. its first
//      pixel in raster order, as root);
//   4. on the host: the component table (pixels, LR cells Q, the pixels of
//      each block of Q) and a conflict-free schedule.  Two components
//      interact only if some cells of their Q lie within 2r of each other
//      (the trial of one reads I_low within 2r of its Q and rewrites Theta /
//      E within r of it).  A component's level is one more than the largest
//      level of the earlier components it interacts with, so running the
//      levels in order, components of one level side by side, gives exactly
//      the sequential order of the algorithm;
//   5. one trial workgroup per component: e0 over the affected set A (pixels
//      whose window contains a cell of Q), replace I_low[q] by I[p*] with p*
//      the largest-error pixel of the component in q's block, re-search A
//      into a staging buffer, e1, keep (e1 <= e0) or roll back.  Sums are
//      float64 in a fixed order.
// After the last round the whole image is searched once more, so the
// returned Theta / E are exactly the search of I against the final I_low.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "glu_device.h"
#include "glu_host.h"

namespace glu {

constexpr int kTilePx = 1024;  // pixels per marking tile (4 per thread)

struct JdBuffers {
  float* E;          // H*W current error
  int* parent;       // H*W union-find parents (-1: not large)
  int* list;         // compacted large-error pixels, raster order
  int* list_root;    // root per list entry
  int* tile_count;   // per marking tile
  int* tile_off;     // exclusive scan of tile_count
  int* total;        // [0] = |large set|
  uint16_t* st_code;  // H*W staged Theta of trials
  float* st_alpha;
  float* st_err;
  float* oldL;       // h*w*3 saved colours
  int* flag;         // h*w cells of the affected set being enumerated
  int* comp;         // component table (8 ints each)
  int* qtab;         // (q, pixel offset, pixel count) per component cell
  int* pix;          // component pixels grouped by component, cell, raster
  int* pstar;        // chosen pixel per qtab entry
  double* dec;       // per component: accepted, e0, e1
  double* partial;   // per tile sums for the error total
};

// ---------------------------------------------------------------------------
// marking, compaction, union-find
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_jd_mark(const float* __restrict__ E, int64_t n, float tau,
                                                 int* __restrict__ parent, int* __restrict__ tile_count) {
  __shared__ int wcount[4];
  const int64_t base = (int64_t)blockIdx.x * kTilePx;
  int c = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t p = base + u * 256 + threadIdx.x;
    if (p < n) {
      const bool m = E[p] > tau;
      parent[p] = m ? (int)p : -1;
      c += m;
    }
  }
  // deterministic block sum
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  if ((threadIdx.x & 63) == 0) wcount[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) tile_count[blockIdx.x] = wcount[0] + wcount[1] + wcount[2] + wcount[3];
}

// exclusive scan of the tile counts by one workgroup: each thread sums a
// contiguous run of tiles, the 256 run totals are scanned with wave
// shuffles (inclusive scan per wave, then the wave totals), and each
// thread writes its run's offsets
__global__ __launch_bounds__(256) void k_jd_scan(const int* __restrict__ cnt, int ntiles, int* __restrict__ off,
                                                 int* __restrict__ total) {
  __shared__ int wave_sum[4];
  const int per = (ntiles + 255) / 256;
  const int t0 = min(ntiles, (int)threadIdx.x * per), t1 = min(ntiles, t0 + per);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int v = 0;
  for (int i = t0; i < t1; ++i) v += cnt[i];
  int inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(inc, d, 64);
    inc += lane >= d ? u : 0;
  }
  if (lane == 63) wave_sum[wave] = inc;
  __syncthreads();
  int base = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) base += w < wave ? wave_sum[w] : 0;
  if (threadIdx.x == 255) total[0] = base + inc;
  int acc = base + inc - v;
  for (int i = t0; i < t1; ++i) {
    const int c = cnt[i];
    off[i] = acc;
    acc += c;
  }
}

// ordered scatter: pixel u*256 + tid of the tile goes after every marked
// pixel of lower index in the tile (ranks from wave ballots)
__global__ __launch_bounds__(256) void k_jd_scatter(const int* __restrict__ parent, int64_t n,
                                                    const int* __restrict__ tile_off, int* __restrict__ list) {
  __shared__ int wtot[2][4];
  const int64_t base = (int64_t)blockIdx.x * kTilePx;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  int run = tile_off[blockIdx.x];
  for (int u = 0; u < 4; ++u) {
    const int64_t p = base + u * 256 + threadIdx.x;
    const bool m = p < n && parent[p] >= 0;
    const unsigned long long bal = __ballot(m);
    if (lane == 0) wtot[u & 1][wave] = __popcll(bal);
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int c = wtot[u & 1][w];
      before += w < wave ? c : 0;
      tot += c;
    }
    if (m) list[run + before + __popcll(bal & below)] = (int)p;
    run += tot;
  }
}

__device__ __forceinline__ int uf_find(int* parent, int x) {
  int p = __atomic_load_n(&parent[x], __ATOMIC_RELAXED);
  while (p != x) {
    x = p;
    p = __atomic_load_n(&parent[x], __ATOMIC_RELAXED);
  }
  return x;
}

__device__ __forceinline__ void uf_unite(int* parent, int a, int b) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicMin(&parent[a], b);
    if (old == a) return;
    a = old;
  }
}

// union and flatten read the list length from the device and stride over
// the list, so the host can launch them before it knows the length
__global__ __launch_bounds__(256) void k_jd_union(int* __restrict__ parent, const int* __restrict__ list,
                                                  const int* __restrict__ total, int H, int W) {
  const int nl = total[0];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nl; i += gridDim.x * 256) {
  const int p = list[i];
  const int y = p / W, x = p - y * W;
  // the four neighbours that precede p in raster order
  if (x > 0 && __atomic_load_n(&parent[p - 1], __ATOMIC_RELAXED) >= 0) uf_unite(parent, p, p - 1);
  if (y > 0) {
    const int up = p - W;
    if (x > 0 && __atomic_load_n(&parent[up - 1], __ATOMIC_RELAXED) >= 0) uf_unite(parent, p, up - 1);
    if (__atomic_load_n(&parent[up], __ATOMIC_RELAXED) >= 0) uf_unite(parent, p, up);
    if (x + 1 < W && __atomic_load_n(&parent[up + 1], __ATOMIC_RELAXED) >= 0) uf_unite(parent, p, up + 1);
  }
  }
}

__global__ __launch_bounds__(256) void k_jd_flatten(int* __restrict__ parent, const int* __restrict__ list,
                                                    const int* __restrict__ total, int* __restrict__ root) {
  const int nl = total[0];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nl; i += gridDim.x * 256) root[i] = uf_find(parent, list[i]);
}

// float64 sum of E in a fixed order: per tile, then one workgroup over
// tiles; each reduces with wave shuffles (a fixed tree per wave) and adds
// the four wave sums in order
__device__ __forceinline__ double block_sum256(double v) {
  __shared__ double wsum[4];
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_down(v, d, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
  __syncthreads();  // wsum may be written again by a later call
  return r;
}

// exclusive scan of one int per thread over a workgroup of 256 (wave
// shuffles, then the wave totals); *total gets the sum
__device__ __forceinline__ int block_exclusive_scan256(int v, int* total) {
  __shared__ int wtot[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(inc, d, 64);
    inc += lane >= d ? u : 0;
  }
  if (lane == 63) wtot[wave] = inc;
  __syncthreads();
  int base = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) base += w < wave ? wtot[w] : 0;
  *total = wtot[0] + wtot[1] + wtot[2] + wtot[3];
  __syncthreads();
  return base + inc - v;
}

__global__ __launch_bounds__(256) void k_jd_sum_tiles(const float* __restrict__ E, int64_t n,
                                                      double* __restrict__ partial) {
  const int64_t base = (int64_t)blockIdx.x * kTilePx;
  double v = 0.0;
  for (int u = 0; u < 4; ++u) {
    const int64_t p = base + u * 256 + threadIdx.x;
    if (p < n) v += (double)E[p];
  }
  v = block_sum256(v);
  if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

__global__ __launch_bounds__(256) void k_jd_sum_final(double* __restrict__ partial, int ntiles,
                                                      double* __restrict__ out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < ntiles; i += 256) v += partial[i];
  v = block_sum256(v);
  if (threadIdx.x == 0) out[0] = v;
}

// ---------------------------------------------------------------------------
// trial of one component
// ---------------------------------------------------------------------------
struct JdTrialArgs {
  const float* I;
  float* L;
  int64_t I_stride, L_stride;
  uint16_t* code;
  float* alpha;
  int64_t th_stride;
  JdBuffers b;
  int H, W, h, w, s, k, mode;
  int gnu;  // GNU: fast-mode anchor only
  float eps;
  int comp_begin;  // first component (in schedule order) of this launch
};

// comp[8 * c + ...]: 0 px_off, 1 n_px, 2 q_off, 3 n_q, 4 slot (sequential
// index), 5 bbox y0, 6 bbox x0, 7 bbox packed (y1 << 16 | x1) of the
// affected cells (inclusive, clamped to the LR image).

// One pixel's search against the current LR guide.  For 3 x 3 windows the
// nine cells are read once into registers; other windows read them from
// global memory as the candidate loops need them.
template <int KW>
__device__ __forceinline__ void search_one(const JdTrialArgs& a, int y, int x, int& code, float& al, float& e) {
  const float* ipp = a.I + (int64_t)y * a.I_stride + (int64_t)x * 3;
  const float ip[1][3] = {{ipp[0], ipp[1], ipp[2]}};
  const int r = a.k / 2;
  const GlobalWin gw{a.L, a.L_stride, y / a.s, x / a.s, a.h, a.w, a.k, r};
  float best[1], alp[1];
  int cd[1];
  auto run = [&](const auto& win) {
    if (a.mode == MODE_EXH) {
      exh_strip<KW, 1, true, false>(ip, win, nullptr, a.eps, a.k, false, best, cd);
      alp[0] = exh_alpha<KW, false>(ip[0], win, nullptr, a.eps, a.k, cd[0]);
    } else {
      fast_strip<KW, 1, true>(ip, win, a.eps, a.k, a.gnu != 0, best, cd, alp);
    }
  };
  if constexpr (KW == 3)
    run(RegWin<3>(gw));
  else
    run(gw);
  code = cd[0];
  al = alp[0];
  e = __builtin_amdgcn_sqrtf(best[0]);
}

// affected cells of one trial listed in LDS (more fall back to the box walk)
constexpr int kTrialCells = 4096;

template <int KW>
__global__ __launch_bounds__(256) void k_jd_trial(const JdTrialArgs a) {
  __shared__ int s_cells[kTrialCells];
  const int* cm = a.b.comp + 8 * (a.comp_begin + blockIdx.x);
  const int q_off = cm[2], n_q = cm[3], slot = cm[4];
  const int by0 = cm[5], bx0 = cm[6], by1 = cm[7] >> 16, bx1 = cm[7] & 0xffff;
  const int s = a.s, r = a.k / 2;
  const int bw = bx1 - bx0 + 1, bh = by1 - by0 + 1;
  // components of one launch have disjoint affected cells but their boxes
  // may overlap, so a cell is tagged with the component's own mark
  const int mark = slot + 1;

  // mark the affected cells (within r of a cell of Q)
  for (int i = threadIdx.x; i < n_q; i += 256) {
    const int q = a.b.qtab[3 * (q_off + i)];
    const int qy = q / a.w, qx = q - qy * a.w;
    for (int dy = -r; dy <= r; ++dy)
      for (int dx = -r; dx <= r; ++dx) {
        const int cy = qy + dy, cx = qx + dx;
        if (cy >= 0 && cy < a.h && cx >= 0 && cx < a.w) a.b.flag[cy * a.w + cx] = mark;
      }
  }
  __threadfence_block();
  __syncthreads();

  // affected pixels are enumerated as: cells of the box in raster order,
  // flagged ones only, and each block's pixels in raster order.  The
  // flagged cells are first compacted into an LDS list (each thread takes a
  // contiguous run of the box); a component with more affected cells than
  // the list holds walks the whole box instead.
  const int ss = s * s;
  const int nbox = bw * bh;
  int naff;  // affected cells (the same in every thread)
  {
    const int per = (nbox + 255) / 256;
    const int c0 = min(nbox, (int)threadIdx.x * per), c1 = min(nbox, c0 + per);
    int cnt = 0;
    for (int c = c0; c < c1; ++c) {
      const int cy = by0 + c / bw, cx = bx0 + c % bw;
      cnt += __atomic_load_n(&a.b.flag[cy * a.w + cx], __ATOMIC_RELAXED) == mark;
    }
    int o = block_exclusive_scan256(cnt, &naff);
    if (naff <= kTrialCells) {
      for (int c = c0; c < c1; ++c) {
        const int cy = by0 + c / bw, cx = bx0 + c % bw;
        if (__atomic_load_n(&a.b.flag[cy * a.w + cx], __ATOMIC_RELAXED) == mark) s_cells[o++] = c;
      }
    }
    __syncthreads();
  }
  const bool listed = naff <= kTrialCells;
  const int64_t nslots = (int64_t)(listed ? naff : nbox) * ss;
  // pixel (y, x) of slot t; false for a slot outside the affected set
  auto slot_pixel = [&](int64_t t, int& y, int& x) -> bool {
    const int k = (int)(t / ss), within = (int)(t - (int64_t)k * ss);
    const int cell = listed ? s_cells[k] : k;
    const int cy = by0 + cell / bw, cx = bx0 + cell % bw;
    if (!listed && __atomic_load_n(&a.b.flag[cy * a.w + cx], __ATOMIC_RELAXED) != mark) return false;
    y = cy * s + within / s;
    x = cx * s + within % s;
    return y < a.H && x < a.W;
  };

  double e0 = 0.0;
  for (int64_t t = threadIdx.x; t < nslots; t += 256) {
    int y, x;
    if (!slot_pixel(t, y, x)) continue;
    e0 += (double)a.b.E[(int64_t)y * a.W + x];
  }
  e0 = block_sum256(e0);

  // p* per cell of Q (first largest E in raster order), save and replace
  for (int i = threadIdx.x; i < n_q; i += 256) {
    const int* qt = a.b.qtab + 3 * (q_off + i);
    const int q = qt[0], po = qt[1], pn = qt[2];
    int best = a.b.pix[po];
    float be = a.b.E[best];
    for (int j = 1; j < pn; ++j) {
      const int p = a.b.pix[po + j];
      const float e = a.b.E[p];
      if (e > be) {
        be = e;
        best = p;
      }
    }
    a.b.pstar[q_off + i] = best;
    const int qy = q / a.w, qx = q - qy * a.w;
    float* Lq = a.L + (int64_t)qy * a.L_stride + (int64_t)qx * 3;
    const int py = best / a.W, px = best - py * a.W;
    const float* Ip = a.I + (int64_t)py * a.I_stride + (int64_t)px * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a.b.oldL[(int64_t)q * 3 + c] = Lq[c];
      Lq[c] = Ip[c];
    }
  }
  __threadfence();
  __syncthreads();

  // re-search the affected set into the staging buffers
  double e1 = 0.0;
  for (int64_t t = threadIdx.x; t < nslots; t += 256) {
    int y, x;
    if (!slot_pixel(t, y, x)) continue;
    int cd;
    float al, e;
    search_one<KW>(a, y, x, cd, al, e);
    const int64_t p = (int64_t)y * a.W + x;
    a.b.st_code[p] = (uint16_t)cd;
    a.b.st_alpha[p] = al;
    a.b.st_err[p] = e;
    e1 += (double)e;
  }
  e1 = block_sum256(e1);
  const bool accept = !(e1 > e0);

  // commit or roll back; clear the flags
  if (accept) {
    for (int64_t t = threadIdx.x; t < nslots; t += 256) {
      int y, x;
      if (!slot_pixel(t, y, x)) continue;
      const int64_t p = (int64_t)y * a.W + x;
      const int64_t to = (int64_t)y * a.th_stride + x;
      a.code[to] = a.b.st_code[p];
      a.alpha[to] = a.b.st_alpha[p];
      a.b.E[p] = a.b.st_err[p];
    }
  } else {
    for (int i = threadIdx.x; i < n_q; i += 256) {
      const int q = a.b.qtab[3 * (q_off + i)];
      const int qy = q / a.w, qx = q - qy * a.w;
      float* Lq = a.L + (int64_t)qy * a.L_stride + (int64_t)qx * 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) Lq[c] = a.b.oldL[(int64_t)q * 3 + c];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n_q; i += 256) {
    const int q = a.b.qtab[3 * (q_off + i)];
    const int qy = q / a.w, qx = q - qy * a.w;
    for (int dy = -r; dy <= r; ++dy)
      for (int dx = -r; dx <= r; ++dx) {
        const int cy = qy + dy, cx = qx + dx;
        if (cy >= 0 && cy < a.h && cx >= 0 && cx < a.w) a.b.flag[cy * a.w + cx] = 0;
      }
  }
  if (threadIdx.x == 0) {
    a.b.dec[3 * slot + 0] = accept ? 1.0 : 0.0;
    a.b.dec[3 * slot + 1] = e0;
    a.b.dec[3 * slot + 2] = e1;
  }
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
struct JdLayout {
  size_t E, parent, list, list_root, tile_count, tile_off, total, st_code, st_alpha, st_err, oldL, flag, comp, qtab,
      pix, pstar, dec, partial, sums, end;
};

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

static JdLayout jd_layout(int64_t H, int64_t W, int s) {
  const int64_t n = H * W, h = (H + s - 1) / s, w = (W + s - 1) / s, nl = h * w;
  const int64_t ntiles = (n + kTilePx - 1) / kTilePx;
  const int64_t max_comp = ((H + 1) / 2) * ((W + 1) / 2);
  JdLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.E = take(4 * n);
  L.parent = take(4 * n);
  L.list = take(4 * n);
  L.list_root = take(4 * n);
  L.tile_count = take(4 * ntiles);
  L.tile_off = take(4 * ntiles);
  L.total = take(16);
  L.st_code = take(2 * n);
  L.st_alpha = take(4 * n);
  L.st_err = take(4 * n);
  L.oldL = take(12 * nl);
  L.flag = take(4 * nl);
  L.comp = take(32 * max_comp);
  L.qtab = take(12 * n);
  L.pix = take(4 * n);
  L.pstar = take(4 * n);
  L.dec = take(24 * max_comp);
  L.partial = take(8 * ntiles);
  L.sums = take(16);
  L.end = o;
  return L;
}

enum { PIN_SUM, PIN_SUM0, PIN_TOTAL, PIN_LIST, PIN_ROOT, PIN_UP, PIN_DEC, PIN_PSTAR, PIN_N };
static thread_local PinnedBuf tl_pin[PIN_N];

static glu_status jd_sum(const float* E, int64_t n, double* partial, double* sums, hipStream_t st, double* out) {
  const int64_t ntiles = (n + kTilePx - 1) / kTilePx;
  hipLaunchKernelGGL(k_jd_sum_tiles, dim3((unsigned)ntiles), dim3(256), 0, st, E, n, partial);
  hipLaunchKernelGGL(k_jd_sum_final, dim3(1), dim3(256), 0, st, partial, (int)ntiles, sums);
  PinnedBuf& pb = tl_pin[PIN_SUM];
  hipError_t e = pb.reserve(sizeof(double));
  if (e == hipSuccess) e = hipMemcpyAsync(pb.p, sums, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "joint: error sum");
  *out = *pb.as<double>();
  return GLU_OK;
}

}  // namespace glu

using namespace glu;

extern "C" {

size_t glu_joint_downsample_workspace(int32_t H, int32_t W, const glu_params* p) {
  if (!p || p->s < 1 || H < 0 || W < 0) return 0;
  return jd_layout(H, W, p->s).end;
}

glu_status glu_joint_downsample(const glu_image* I, glu_image* I_low, const glu_params* p, float tau,
                                int32_t max_iter, glu_theta* theta, float* err, void* workspace, size_t ws_bytes,
                                glu_jd_stats* stats, glu_jd_log* log, void* stream) {
  clear_error();
  glu_status st;
  if ((st = check_params(p))) return st;
  if (p->flags) return fail(GLU_ERR_UNSUPPORTED, "joint downsampling takes no flags");
  if ((st = check_image(I, "I", 3, 3, false))) return st;
  if ((st = check_image(I_low, "I_low", 3, 3, false))) return st;
  if (!(tau >= 0.0f) || !std::isfinite(tau)) return fail(GLU_ERR_PARAM, "tau must be finite and >= 0");
  if (max_iter < 0 || max_iter > 64) return fail(GLU_ERR_PARAM, "max_iter must be in 0..64");
  const int H = I->height, W = I->width, s = p->s;
  const int h = ceil_div(H, s), w = ceil_div(W, s);
  if (I_low->height != h || I_low->width != w) return fail(GLU_ERR_SHAPE, "I_low must be ceil(H/s) x ceil(W/s)");
  if (w > 0xffff || h > 0xffff) return fail(GLU_ERR_UNSUPPORTED, "LR image wider or taller than 65535");
  if ((st = check_theta(theta, H, W, true))) return st;
  if ((int64_t)H * W > 0 && theta->row_stride != W)
    return fail(GLU_ERR_UNSUPPORTED, "joint downsampling needs a dense theta (row_stride == W)");
  if (err && reinterpret_cast<uintptr_t>(err) % 4) return fail(GLU_ERR_ALIGN, "err not aligned");
  if ((int64_t)H * W >= (int64_t)1 << 31) return fail(GLU_ERR_UNSUPPORTED, "image has 2^31 pixels or more");
  const JdLayout lay = jd_layout(H, W, s);
  if ((int64_t)H * W > 0 && (!workspace || ws_bytes < lay.end))
    return fail(GLU_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", lay.end, ws_bytes);
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(GLU_ERR_ALIGN, "workspace must be 256-byte aligned");
  if (log && log->capacity > 0 &&
      (!log->round || !log->first_pixel || !log->accepted || !log->e0 || !log->e1 || !log->n_q))
    return fail(GLU_ERR_NULL, "log arrays are NULL");
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (log) {
    log->count = 0;
    log->truncated = 0;
  }
  if ((int64_t)H * W == 0) return GLU_OK;

  hipStream_t sm = (hipStream_t)stream;
  char* ws = static_cast<char*>(workspace);
  JdBuffers b{};
  b.E = reinterpret_cast<float*>(ws + lay.E);
  b.parent = reinterpret_cast<int*>(ws + lay.parent);
  b.list = reinterpret_cast<int*>(ws + lay.list);
  b.list_root = reinterpret_cast<int*>(ws + lay.list_root);
  b.tile_count = reinterpret_cast<int*>(ws + lay.tile_count);
  b.tile_off = reinterpret_cast<int*>(ws + lay.tile_off);
  b.total = reinterpret_cast<int*>(ws + lay.total);
  b.st_code = reinterpret_cast<uint16_t*>(ws + lay.st_code);
  b.st_alpha = reinterpret_cast<float*>(ws + lay.st_alpha);
  b.st_err = reinterpret_cast<float*>(ws + lay.st_err);
  b.oldL = reinterpret_cast<float*>(ws + lay.oldL);
  b.flag = reinterpret_cast<int*>(ws + lay.flag);
  b.comp = reinterpret_cast<int*>(ws + lay.comp);
  b.qtab = reinterpret_cast<int*>(ws + lay.qtab);
  b.pix = reinterpret_cast<int*>(ws + lay.pix);
  b.pstar = reinterpret_cast<int*>(ws + lay.pstar);
  b.dec = reinterpret_cast<double*>(ws + lay.dec);
  b.partial = reinterpret_cast<double*>(ws + lay.partial);
  double* sums = reinterpret_cast<double*>(ws + lay.sums);

  const int64_t n = (int64_t)H * W;
  const int64_t ntiles = (n + kTilePx - 1) / kTilePx;
  const int r = p->k / 2;
  hipError_t e = hipMemsetAsync(b.flag, 0, sizeof(int) * (size_t)h * w, sm);
  if (e != hipSuccess) return hip_fail(e, "joint: clear flags");

  // The one full search.  After it, Theta and E stay those of a full search
  // against the current I_low: a trial re-searches every pixel whose window
  // holds a replaced cell (its affected set) with the same arithmetic as the
  // search kernels (pair constants from pair_consts, the same candidate
  // order, the same fast-search steps), and commits exactly those pixels'
  // Theta and E when it keeps the update; a trial that rolls back restores
  // its cells and leaves Theta and E untouched.  So no round starts with a
  // search, and none follows the last one.
  {
    glu_theta th = *theta;
    if ((st = glu_search(I, I_low, p, &th, b.E, stream))) return st;
  }
  // the initial error sum: copied with the first round's data (one
  // synchronisation per round; rounds_run = 0 reads it at the end)
  hipLaunchKernelGGL(k_jd_sum_tiles, dim3((unsigned)ntiles), dim3(256), 0, sm, b.E, n, b.partial);
  hipLaunchKernelGGL(k_jd_sum_final, dim3(1), dim3(256), 0, sm, b.partial, (int)ntiles, sums + 1);
  e = tl_pin[PIN_SUM0].reserve(sizeof(double));
  if (e == hipSuccess) e = hipMemcpyAsync(tl_pin[PIN_SUM0].p, sums + 1, sizeof(double), hipMemcpyDeviceToHost, sm);
  if (e != hipSuccess) return hip_fail(e, "joint: initial error sum");
  bool have_initial = false;
  auto take_initial = [&]() {
    if (!have_initial && stats) stats->err_sum_initial = *tl_pin[PIN_SUM0].as<double>();
    have_initial = true;
  };

  // A round's decisions (accept flags, e0, e1, p*) are copied back after its
  // trials without waiting; the host reads them at the next round's
  // synchronisation (or after the loop), together with what it kept of the
  // round's component table.
  int64_t log_q_used = 0;
  struct Pending {
    int round = 0, total = 0, M = 0, levels = 0;
    std::vector<int> first_pixel, cq_n, cq_off, qs;
  } pend;
  // stats and log entries of the pending round's decisions, reported as
  // round `as_round`; returns the number of kept trials
  auto emit_round = [&](int as_round) -> int {
    const int M = pend.M;
    const double* dec = tl_pin[PIN_DEC].as<double>();
    const int* pstar = tl_pin[PIN_PSTAR].as<int>();
    int accepted = 0;
    for (int c = 0; c < M; ++c) accepted += dec[3 * c] != 0.0;
    if (stats) {
      stats->rounds_run = as_round;
      stats->n_large[as_round - 1] = pend.total;
      stats->n_components[as_round - 1] = M;
      stats->n_accepted[as_round - 1] = accepted;
      stats->n_waves[as_round - 1] = pend.levels;
    }
    if (log) {
      for (int c = 0; c < M; ++c) {
        if (log->count >= log->capacity) {
          log->truncated = 1;
          break;
        }
        const int i = log->count;
        log->round[i] = as_round;
        log->first_pixel[i] = pend.first_pixel[c];
        log->accepted[i] = dec[3 * c] != 0.0;
        log->e0[i] = dec[3 * c + 1];
        log->e1[i] = dec[3 * c + 2];
        log->n_q[i] = pend.cq_n[c];
        // q, p* pairs appended after the previous entries'
        if (log->q_and_pstar && log_q_used + pend.cq_n[c] <= log->q_capacity) {
          for (int j = 0; j < pend.cq_n[c]; ++j) {
            log->q_and_pstar[2 * (log_q_used + j)] = pend.qs[pend.cq_off[c] + j];
            log->q_and_pstar[2 * (log_q_used + j) + 1] = pstar[pend.cq_off[c] + j];
          }
        } else {
          log->truncated = 1;
        }
        log->count = i + 1;
        log_q_used += pend.cq_n[c];
      }
    }
    return accepted;
  };
  // Reads the pending round.  A round that keeps no trial leaves I_low as
  // it found it, so the next round's search, large-error set, components
  // and trials are the same and decide the same: every later round repeats
  // it decision for decision.  Those rounds are reported here without
  // being run again; true means the loop is done.
  auto take_pending = [&]() -> bool {
    if (pend.round == 0) return false;
    const int r0 = pend.round;
    pend.round = 0;
    if (emit_round(r0) != 0) return false;
    for (int r = r0 + 1; r <= max_iter; ++r) emit_round(r);
    return true;
  };

  std::vector<int> list, root, comp, qtab, pix, grid;
  // list entries copied with the count before the count is known: enough
  // for the previous round's set twice over (a larger set takes a second copy)
  int list_guess = 4096;
  // union and flatten stride over the list with a small fixed grid
  const unsigned ugrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, (n + 255) / 256));
  for (int round = 1; round <= max_iter; ++round) {
    hipLaunchKernelGGL(k_jd_mark, dim3((unsigned)ntiles), dim3(256), 0, sm, b.E, n, tau, b.parent, b.tile_count);
    hipLaunchKernelGGL(k_jd_scan, dim3(1), dim3(256), 0, sm, b.tile_count, (int)ntiles, b.tile_off, b.total);
    hipLaunchKernelGGL(k_jd_scatter, dim3((unsigned)ntiles), dim3(256), 0, sm, b.parent, n, b.tile_off, b.list);
    hipLaunchKernelGGL(k_jd_union, dim3(ugrid), dim3(256), 0, sm, b.parent, b.list, b.total, H, W);
    hipLaunchKernelGGL(k_jd_flatten, dim3(ugrid), dim3(256), 0, sm, b.parent, b.list, b.total, b.list_root);
    const int guess = (int)std::min<int64_t>(n, list_guess);
    e = tl_pin[PIN_TOTAL].reserve(sizeof(int));
    if (e == hipSuccess) e = tl_pin[PIN_LIST].reserve(sizeof(int) * guess);
    if (e == hipSuccess) e = tl_pin[PIN_ROOT].reserve(sizeof(int) * guess);
    if (e == hipSuccess) e = hipMemcpyAsync(tl_pin[PIN_TOTAL].p, b.total, sizeof(int), hipMemcpyDeviceToHost, sm);
    if (e == hipSuccess) e = hipMemcpyAsync(tl_pin[PIN_LIST].p, b.list, sizeof(int) * guess, hipMemcpyDeviceToHost, sm);
    if (e == hipSuccess)
      e = hipMemcpyAsync(tl_pin[PIN_ROOT].p, b.list_root, sizeof(int) * guess, hipMemcpyDeviceToHost, sm);
    if (e == hipSuccess) e = hipStreamSynchronize(sm);
    if (e != hipSuccess) return hip_fail(e, "joint: large-error set");
    take_initial();
    if (take_pending()) break;  // the previous round kept nothing: the rest repeat it
    const int total = *tl_pin[PIN_TOTAL].as<int>();
    if (total == 0) break;
    list.resize(total);
    root.resize(total);
    std::memcpy(list.data(), tl_pin[PIN_LIST].p, sizeof(int) * std::min(total, guess));
    std::memcpy(root.data(), tl_pin[PIN_ROOT].p, sizeof(int) * std::min(total, guess));
    if (total > guess) {
      const int rest = total - guess;
      e = tl_pin[PIN_LIST].reserve(sizeof(int) * rest);
      if (e == hipSuccess) e = tl_pin[PIN_ROOT].reserve(sizeof(int) * rest);
      if (e == hipSuccess)
        e = hipMemcpyAsync(tl_pin[PIN_LIST].p, b.list + guess, sizeof(int) * rest, hipMemcpyDeviceToHost, sm);
      if (e == hipSuccess)
        e = hipMemcpyAsync(tl_pin[PIN_ROOT].p, b.list_root + guess, sizeof(int) * rest, hipMemcpyDeviceToHost, sm);
      if (e == hipSuccess) e = hipStreamSynchronize(sm);
      if (e != hipSuccess) return hip_fail(e, "joint: large-error set");
      std::memcpy(list.data() + guess, tl_pin[PIN_LIST].p, sizeof(int) * rest);
      std::memcpy(root.data() + guess, tl_pin[PIN_ROOT].p, sizeof(int) * rest);
    }
    list_guess = std::max(4096, 2 * total);

    // components in the order of their first pixel (= root, the smallest index)
    std::vector<int> order(total);
    for (int i = 0; i < total; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return root[x] < root[y]; });
    // group: [start, end) per component over `order` (raster order inside)
    std::vector<int> cstart;
    for (int i = 0; i < total; ++i)
      if (i == 0 || root[order[i]] != root[order[i - 1]]) cstart.push_back(i);
    const int M = (int)cstart.size();
    cstart.push_back(total);

    // per component: cells Q (ascending) with their pixels; conflict level
    grid.assign((size_t)h * w, 0);
    std::vector<int> level(M), cq_off(M), cq_n(M), cpx_off(M);
    std::vector<int> bbox(4 * M);
    qtab.clear();
    pix.clear();
    std::vector<std::pair<int, int>> cellpix;
    int max_level = 0;
    for (int c = 0; c < M; ++c) {
      cellpix.clear();
      for (int i = cstart[c]; i < cstart[c + 1]; ++i) {
        const int px = list[order[i]];
        const int y = px / W, x = px - y * W;
        cellpix.push_back({(y / s) * w + x / s, px});
      }
      std::stable_sort(cellpix.begin(), cellpix.end(),
                       [](const std::pair<int, int>& u, const std::pair<int, int>& v) { return u.first < v.first; });
      cq_off[c] = (int)qtab.size() / 3;
      cpx_off[c] = (int)pix.size();
      int lv = 0;
      int y0 = h, x0 = w, y1 = -1, x1 = -1;
      for (size_t i = 0; i < cellpix.size();) {
        const int q = cellpix[i].first;
        const int po = (int)pix.size();
        size_t j = i;
        while (j < cellpix.size() && cellpix[j].first == q) pix.push_back(cellpix[j++].second);
        qtab.push_back(q);
        qtab.push_back(po);
        qtab.push_back((int)(j - i));
        i = j;
        const int qy = q / w, qx = q - qy * w;
        for (int cy = std::max(0, qy - 2 * r); cy <= std::min(h - 1, qy + 2 * r); ++cy)
          for (int cx = std::max(0, qx - 2 * r); cx <= std::min(w - 1, qx + 2 * r); ++cx)
            lv = std::max(lv, grid[(size_t)cy * w + cx]);
        y0 = std::min(y0, std::max(0, qy - r));
        x0 = std::min(x0, std::max(0, qx - r));
        y1 = std::max(y1, std::min(h - 1, qy + r));
        x1 = std::max(x1, std::min(w - 1, qx + r));
      }
      cq_n[c] = (int)qtab.size() / 3 - cq_off[c];
      level[c] = lv + 1;
      max_level = std::max(max_level, lv + 1);
      for (int i = 0; i < cq_n[c]; ++i) {
        const int q = qtab[3 * (cq_off[c] + i)];
        grid[q] = std::max(grid[q], lv + 1);
      }
      bbox[4 * c] = y0;
      bbox[4 * c + 1] = x0;
      bbox[4 * c + 2] = y1;
      bbox[4 * c + 3] = x1;
    }
    // schedule: by level, sequential order inside a level
    std::vector<int> sched(M);
    for (int c = 0; c < M; ++c) sched[c] = c;
    std::stable_sort(sched.begin(), sched.end(), [&](int x, int y) { return level[x] < level[y]; });
    comp.assign(8 * (size_t)M, 0);
    std::vector<int> lvl_start(max_level + 2, M);
    for (int i = M - 1; i >= 0; --i) lvl_start[level[sched[i]]] = i;
    lvl_start[max_level + 1] = M;
    for (int i = 0; i < M; ++i) {
      const int c = sched[i];
      int* cm = &comp[8 * (size_t)i];
      cm[0] = cpx_off[c];
      cm[1] = cstart[c + 1] - cstart[c];
      cm[2] = cq_off[c];
      cm[3] = cq_n[c];
      cm[4] = c;
      cm[5] = bbox[4 * c];
      cm[6] = bbox[4 * c + 1];
      cm[7] = (bbox[4 * c + 2] << 16) | bbox[4 * c + 3];
    }
    {
      // one pinned staging buffer holds the three tables back to back
      const size_t nc = comp.size(), nqt = qtab.size(), npx = pix.size();
      e = tl_pin[PIN_UP].reserve(sizeof(int) * (nc + nqt + npx));
      if (e == hipSuccess) {
        int* up = tl_pin[PIN_UP].as<int>();
        std::memcpy(up, comp.data(), sizeof(int) * nc);
        std::memcpy(up + nc, qtab.data(), sizeof(int) * nqt);
        std::memcpy(up + nc + nqt, pix.data(), sizeof(int) * npx);
        e = hipMemcpyAsync(b.comp, up, sizeof(int) * nc, hipMemcpyHostToDevice, sm);
        if (e == hipSuccess) e = hipMemcpyAsync(b.qtab, up + nc, sizeof(int) * nqt, hipMemcpyHostToDevice, sm);
        if (e == hipSuccess) e = hipMemcpyAsync(b.pix, up + nc + nqt, sizeof(int) * npx, hipMemcpyHostToDevice, sm);
      }
      if (e != hipSuccess) return hip_fail(e, "joint: component table upload");
    }

    JdTrialArgs ta{};
    ta.I = static_cast<const float*>(I->data);
    ta.L = static_cast<float*>(I_low->data);
    ta.I_stride = I->row_stride;
    ta.L_stride = I_low->row_stride;
    ta.code = theta->code;
    ta.alpha = theta->alpha;
    ta.th_stride = theta->row_stride;
    ta.b = b;
    ta.H = H;
    ta.W = W;
    ta.h = h;
    ta.w = w;
    ta.s = s;
    ta.k = p->k;
    ta.mode = p->mode == GLU_SEARCH_EXHAUSTIVE ? MODE_EXH : MODE_FAST;
    ta.gnu = p->mode == GLU_SEARCH_GNU;
    ta.eps = p->eps;
    for (int lv = 1; lv <= max_level; ++lv) {
      const int a0 = lvl_start[lv], a1 = lvl_start[lv + 1];
      if (a1 <= a0) continue;
      ta.comp_begin = a0;
      hipLaunchKernelGGL(p->k == 3 ? k_jd_trial<3> : k_jd_trial<0>, dim3((unsigned)(a1 - a0)), dim3(256), 0, sm, ta);
      e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "joint: trial launch");
    }
    // decisions: copied back now, read at the next synchronisation
    e = tl_pin[PIN_DEC].reserve(sizeof(double) * 3 * (size_t)M);
    if (e == hipSuccess) e = tl_pin[PIN_PSTAR].reserve(sizeof(int) * (qtab.size() / 3));
    if (e == hipSuccess)
      e = hipMemcpyAsync(tl_pin[PIN_DEC].p, b.dec, sizeof(double) * 3 * (size_t)M, hipMemcpyDeviceToHost, sm);
    if (e == hipSuccess)
      e = hipMemcpyAsync(tl_pin[PIN_PSTAR].p, b.pstar, sizeof(int) * (qtab.size() / 3), hipMemcpyDeviceToHost, sm);
    if (e != hipSuccess) return hip_fail(e, "joint: decisions");
    pend.round = round;
    pend.total = total;
    pend.M = M;
    pend.levels = max_level;
    pend.first_pixel.resize(M);
    pend.cq_n.assign(cq_n.begin(), cq_n.end());
    pend.cq_off.assign(cq_off.begin(), cq_off.end());
    pend.qs.resize(qtab.size() / 3);
    for (int c = 0; c < M; ++c) pend.first_pixel[c] = list[order[cstart[c]]];
    for (size_t i = 0; i < pend.qs.size(); ++i) pend.qs[i] = qtab[3 * i];
  }
  // the last round's decisions (and the initial sum when no round ran)
  e = hipStreamSynchronize(sm);
  if (e != hipSuccess) return hip_fail(e, "joint: decisions");
  take_initial();
  take_pending();
  // the returned Theta / E: those of the search against the final I_low
  {
    if (err) {
      e = hipMemcpyAsync(err, b.E, sizeof(float) * (size_t)n, hipMemcpyDeviceToDevice, sm);
      if (e != hipSuccess) return hip_fail(e, "joint: copy err");
    }
  }
  if (stats) {
    double fin = 0.0;
    if ((st = jd_sum(b.E, n, b.partial, sums, sm, &fin))) return st;
    stats->err_sum_final = fin;
  }
  return GLU_OK;
}

}  // extern "C"
