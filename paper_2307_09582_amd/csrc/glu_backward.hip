// Backward of the apply step (Eq. 1 with the indices a, b held fixed):
//
//   dL/dalpha_p  = sum_c G_p,c (T_low[a_p],c - T_low[b_p],c)
//   dL/dT_low_q  = sum_{p: a_p = q} alpha_p G_p + sum_{p: b_p = q} (1 - alpha_p) G_p
//
// Deterministic and free of atomics.  Every HR pixel p sends its two
// contributions to cells of its own window, so the referrers of an LR cell q
// are the pixels whose cell c = p_down lies within r of q.  The gather is
// done in two passes over a caller-provided workspace S:
//
//   pass 1 (HR stream, one read of G and Theta): for every LR cell c and
//     every window offset o, S[o][c] = sum over the pixels of c's s x s
//     block of the part of their contribution aimed at the cell
//     c + offset(o).  dL/dalpha is computed from LR target cells staged in
//     LDS and written on the way.  Two forms, both with fixed orders:
//     * registers (3 x 3 windows with a strip width of 4, 3 or 2 pixels,
//       5 x 5 windows with 4): a lane owns a column of P pixels of a cell's
//       block and every RW-th HR row of it, and keeps k^2 C sums (window
//       offset, channel) in registers; the lanes of a cell, then the row
//       groups, add theirs in a fixed order.
//     * scan (every other shape): a workgroup owns nb consecutive cells of
//       one LR row (nb * k^2 <= 256), streams chunks of its HR rows into
//       LDS, and one lane per (cell, offset) scans the chunk's pixels of
//       its cell in raster order without branches.
//   pass 2 (LR): dT_low[q] = sum over o in ascending order of
//     S[o][q - offset(o)].  S is offset-major, so for each o neighbouring
//     lanes read neighbouring cells.
//
// Both passes use fixed summation orders, so results are bitwise
// reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "glu_device.h"
#include "glu_host.h"

namespace glu {

struct BwdArgs {
  const uint16_t* code;
  const float* alpha;
  const void* T;        // T_low (C channels, f32 or f16)
  const float* G;       // grad_T_hat (C channels, f32)
  float* dalpha;        // nullable
  float* S;             // workspace, nullable when dT is not wanted
  float* dT;            // grad_T_low (C channels), nullable
  int64_t th_stride, T_stride, G_stride, dT_stride;
  int32_t H, W, h, w, s, k, C;
  int32_t nb;           // LR cells per workgroup (one LR row), nb * k^2 <= 256
  int32_t rows_chunk;   // HR rows staged per chunk
  int32_t groups_x;     // workgroups per LR row
  int32_t ring_blocks;  // pass 2: workgroups of border cells (the rest take the interior)
  uint32_t s_magic;     // floor(2^32 / s) for udiv_rt
  uint32_t vec;         // VEC_THETA | VEC_G | VEC_T(dalpha rows)
  // element offsets between the images of a batch (blockIdx.y)
  int64_t b_th, b_T, b_G, b_da, b_S, b_dT;
};

// The arguments of image blockIdx.y of a batch.
template <typename T>
__device__ __forceinline__ BwdArgs batch_image(const BwdArgs& a0) {
  BwdArgs a = a0;
  const int64_t b = blockIdx.y;
  a.code += b * a0.b_th;
  a.alpha += b * a0.b_th;
  a.T = static_cast<const T*>(a0.T) + b * a0.b_T;
  a.G += b * a0.b_G;
  if (a.dalpha) a.dalpha += b * a0.b_da;
  if (a.S) a.S += b * a0.b_S;
  if (a.dT) a.dT += b * a0.b_dT;
  return a;
}

// Loads C <= 4 gradient channels of pixels x .. x+P-1 (vector path for
// P = 4, C = 3 or 1 on aligned rows).
template <int P>
__device__ __forceinline__ void load_grad(const float* __restrict__ row, int x, int W, int C, bool vec, bool full,
                                          float (&g)[P][4]) {
  const float* p = row + (int64_t)x * C;
  bool done = false;
  f32x4 v0 = {0.f, 0.f, 0.f, 0.f}, v1 = v0, v2 = v0;
  if constexpr (P == 4) {
    if (vec && full && C == 3) {
      const f32x4* q = reinterpret_cast<const f32x4*>(p);
      v0 = __builtin_nontemporal_load(q);
      v1 = __builtin_nontemporal_load(q + 1);
      v2 = __builtin_nontemporal_load(q + 2);
      done = true;
    } else if (vec && full && C == 1) {
      const f32x4 a = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
      // spread as C == 3 rows would be, channel 0 only
      v0 = f32x4{a.x, 0.f, 0.f, a.y};
      v1 = f32x4{0.f, 0.f, a.z, 0.f};
      v2 = f32x4{0.f, a.w, 0.f, 0.f};
      done = true;
    }
  }
  if (done) {
    if constexpr (P == 4) {
      g[0][0] = v0.x; g[0][1] = v0.y; g[0][2] = v0.z;
      g[1][0] = v0.w; g[1][1] = v1.x; g[1][2] = v1.y;
      g[2][0] = v1.z; g[2][1] = v1.w; g[2][2] = v2.x;
      g[3][0] = v2.y; g[3][1] = v2.z; g[3][2] = v2.w;
#pragma unroll
      for (int i = 0; i < 4; ++i) g[i][3] = 0.f;
    }
  } else {
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const bool ok = full || (x + i < W);
#pragma unroll
      for (int c = 0; c < 4; ++c) g[i][c] = (ok && c < C) ? p[i * C + c] : 0.f;
    }
  }
}

// LDS float4 words of pass 1: staged LR target cells, then per pixel slot of
// a chunk a float4 (gradients, with alpha in .w when C <= 3), a float alpha
// (C == 4) and a uint16 code pair, then (k = 3) the code decoding table.
__host__ __device__ inline int bwd_lds_words(int k, int nb, int s, int rows_chunk) {
  const int n = rows_chunk * nb * s;
  return k * (nb + k - 1) + n + (n + 3) / 4 + (n + 7) / 8 + (k == 3 ? (81 + 3) / 4 : 0);
}

template <typename T, int P, int KW, int C>
__device__ __forceinline__ void bwd_block(const BwdArgs& a, float4* smem) {
  const int k = KW > 0 ? KW : a.k;
  const int r = k / 2, K2 = k * k, s = a.s;
  const int qy = blockIdx.x / a.groups_x;
  const int qx0 = (blockIdx.x - qy * a.groups_x) * a.nb;
  const int nb = min(a.nb, a.w - qx0);
  const int pitch = a.nb * s;                  // slots per staged HR row
  const int nslot = a.rows_chunk * pitch;
  const int lx = a.nb + k - 1;
  float4* sT = smem;
  float4* sG = smem + k * lx;
  float* sA = reinterpret_cast<float*>(sG + nslot);
  uint16_t* sC = reinterpret_cast<uint16_t*>(sA + ((nslot + 3) & ~3));
  // k = 3: code -> LDS offset of cell a | of cell b << 8 | (o_a | o_b << 8) << 16
  // (offsets (o / 3) * lx + o % 3 < 256 because nb <= 28)
  uint32_t* sDec = reinterpret_cast<uint32_t*>(sC + ((nslot + 7) & ~7));
  const T* __restrict__ TL = static_cast<const T*>(a.T);
  const bool vecTh = (a.vec & VEC_THETA) != 0, vecG = (a.vec & VEC_G) != 0, vecA = (a.vec & VEC_T) != 0;

  const int y0 = qy * s, y1 = min(a.H, y0 + s);
  const int x0 = qx0 * s, x1 = min(a.W, x0 + nb * s);
  const int seg = x1 - x0;             // pixels per HR row of the group
  const int spr = (seg + P - 1) / P;   // strips per HR row of the group

  if constexpr (KW == 3) {
    for (int c = (int)threadIdx.x; c < 81; c += kThreads) {
      const int oa = c / 9, ob = c - oa * 9;
      sDec[c] = (uint32_t)((oa / 3) * lx + oa % 3) | ((uint32_t)((ob / 3) * lx + ob % 3) << 8) |
                ((uint32_t)(oa | (ob << 8)) << 16);
    }
  }
  if (a.dalpha) {
    // LR target cells rows qy - r .. qy + r, columns qx0 - r .. qx0 + a.nb - 1 + r,
    // clamped to the LR image (codes from the search never leave it)
    for (int i = (int)threadIdx.x; i < k * lx; i += kThreads) {
      const int rr = i / lx, c = i - rr * lx;
      const int cy = min(max(qy - r + rr, 0), a.h - 1);
      const int cx = min(max(qx0 - r + c, 0), a.w - 1);
      sT[i] = load_cell<T>(TL + (int64_t)cy * a.T_stride + (int64_t)cx * C, C);
    }
  }
  if (KW == 3 || a.dalpha) __syncthreads();

  // scan lane: one (cell, offset) pair of the group
  const int lane_cell = (int)threadIdx.x / K2;
  const int lane_o = (int)threadIdx.x - lane_cell * K2;
  const bool scanner = a.S && lane_cell < nb;
  const int cx0 = lane_cell * s, cx1 = min(seg, cx0 + s);  // pixel columns of the cell
  float acc[C];
#pragma unroll
  for (int ch = 0; ch < C; ++ch) acc[ch] = 0.f;

  for (int yc = y0; yc < y1; yc += a.rows_chunk) {
    const int nrow = min(y1, yc + a.rows_chunk) - yc;
    const int nstrips = nrow * spr;
    for (int t = (int)threadIdx.x; t < nstrips; t += kThreads) {
      const int ry = t / spr;
      const int rx = (t - ry * spr) * P;
      const int y = yc + ry, x = x0 + rx;
      const bool full = rx + P <= seg;
      const int64_t to = (int64_t)y * a.th_stride + x;
      int cd[P];
      float al[P];
      bool done = false;
      if constexpr (P == 4) {
        if (vecTh && full) {
          const u32x2 c = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(a.code + to));
          const f32x4 a4 = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(a.alpha + to));
          cd[0] = c.x & 0xffff;
          cd[1] = c.x >> 16;
          cd[2] = c.y & 0xffff;
          cd[3] = c.y >> 16;
          al[0] = a4.x;
          al[1] = a4.y;
          al[2] = a4.z;
          al[3] = a4.w;
          done = true;
        }
      }
      if (!done) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
          const bool ok = full || (rx + q < seg);
          cd[q] = ok ? a.code[to + q] : 0;
          al[q] = ok ? a.alpha[to + q] : 0.f;
        }
      }
      float g[P][4];
      load_grad<P>(a.G + (int64_t)y * a.G_stride, x, a.W, C, vecG, full, g);
      // cell of the strip inside the group (all P pixels share it)
      const int cl = udiv_rt(rx, s, a.s_magic);
      float da[P];
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const int cdc = min(cd[q], K2 * K2 - 1);
        int offa, offb, pair;
        if constexpr (KW == 3) {
          const uint32_t e = sDec[cdc];
          offa = e & 0xff;
          offb = (e >> 8) & 0xff;
          pair = e >> 16;
        } else {
          const int oa = cdc / K2, ob = cdc - oa * K2;
          offa = (oa / k) * lx + oa % k;
          offb = (ob / k) * lx + ob % k;
          pair = oa | (ob << 8);
        }
        const int i = ry * pitch + rx + q;
        if (a.S && (full || rx + q < seg)) {
          if constexpr (C <= 3) {
            sG[i] = make_float4(g[q][0], g[q][1], g[q][2], al[q]);
          } else {
            sG[i] = make_float4(g[q][0], g[q][1], g[q][2], g[q][3]);
            sA[i] = al[q];
          }
          sC[i] = (uint16_t)pair;
        }
        da[q] = 0.f;
        if (a.dalpha) {
          const float4 Ta = sT[cl + offa];
          const float4 Tb = sT[cl + offb];
          const float dv[4] = {Ta.x - Tb.x, Ta.y - Tb.y, Ta.z - Tb.z, Ta.w - Tb.w};
          float v = g[q][0] * dv[0];
#pragma unroll
          for (int ch = 1; ch < C; ++ch) v = fmaf(g[q][ch], dv[ch], v);
          da[q] = v;
        }
      }
      if (a.dalpha) {
        bool st = false;
        if constexpr (P == 4) {
          if (vecA && full) {
            __builtin_nontemporal_store(f32x4{da[0], da[1], da[2], da[3]},
                                        reinterpret_cast<f32x4*>(a.dalpha + to));
            st = true;
          }
        }
        if (!st) {
#pragma unroll
          for (int q = 0; q < P; ++q)
            if (full || rx + q < seg) a.dalpha[to + q] = da[q];
        }
      }
    }
    if (!a.S) continue;
    __syncthreads();
    if (scanner) {
      // pixels of the cell in raster order; weight alpha for o_a == o,
      // 1 - alpha for o_b == o (both when o_a == o_b == o)
      for (int ry = 0; ry < nrow; ++ry) {
        const int base = ry * pitch;
#pragma unroll 4
        for (int rx = cx0; rx < cx1; ++rx) {
          const int i = base + rx;
          const int pk = sC[i];
          const float4 g = sG[i];
          const float al = C <= 3 ? g.w : sA[i];
          const float wa = ((pk & 0xff) == lane_o) ? al : 0.0f;
          const float wb = ((pk >> 8) == lane_o) ? 1.0f - al : 0.0f;
          const float wt = wa + wb;
          const float gv[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
          for (int ch = 0; ch < C; ++ch) acc[ch] = fmaf(wt, gv[ch], acc[ch]);
        }
      }
    }
    __syncthreads();
  }
  if (scanner) {
    const int64_t hw = (int64_t)a.h * a.w;
    float* out = a.S + ((int64_t)lane_o * hw + (int64_t)qy * a.w + qx0 + lane_cell) * C;
#pragma unroll
    for (int ch = 0; ch < C; ++ch) out[ch] = acc[ch];
  }
}

template <typename T, int P, int KW, int C>
__global__ __launch_bounds__(kThreads) void k_bwd_block(const BwdArgs a0) {
  extern __shared__ float4 smem[];
  const BwdArgs a = batch_image<T>(a0);
  bwd_block<T, P, KW, C>(a, smem);
}

typedef void (*BwdKernel)(const BwdArgs);

template <typename T, int P, int KW>
static BwdKernel pick_bwd_c(int C) {
  switch (C) {
    case 1: return k_bwd_block<T, P, KW, 1>;
    case 2: return k_bwd_block<T, P, KW, 2>;
    case 3: return k_bwd_block<T, P, KW, 3>;
    default: return k_bwd_block<T, P, KW, 4>;
  }
}

template <typename T, int P>
static BwdKernel pick_bwd_k(int k, int C) {
  return k == 3 ? pick_bwd_c<T, P, 3>(C) : pick_bwd_c<T, P, 0>(C);
}

static BwdKernel pick_bwd(bool f16, int P, int k, int C) {
  if (f16) return P == 4 ? pick_bwd_k<__half, 4>(k, C) : pick_bwd_k<__half, 1>(k, C);
  return P == 4 ? pick_bwd_k<float, 4>(k, C) : pick_bwd_k<float, 1>(k, C);
}

// Register form of pass 1 (k = 3 with strips of P = 4, 3 or 2 pixels, P
// the largest of them that divides s; k = 5 with P = 4; cps = s / P lanes
// per cell row, at most 64).  The four waves of a workgroup form RW row
// groups times SG = 4 / RW column segments: RW = min(4, s) (for s = 3 the
// fourth wave idles), except RW = 1 for k = 5 with s < 16.  A segment holds nbs = floor(64 / cps)
// cells of LR row qy, and the workgroup nb = SG nbs of them.  Wave v takes
// segment v / RW and the HR rows y0 + (v mod RW) + RW i; lane l the pixels
// P l .. P l + P - 1 of the segment, all in the segment's cell l / cps.
// Each lane keeps k^2 C sums in registers, one per window offset and
// channel: a pixel adds alpha G where o_a = o and (1 - alpha) G where
// o_b = o.  The first lane of a cell adds up the sums of its cps lanes
// (cross-lane reads in a fixed order).  With one row group it writes S
// itself; otherwise the row groups' sums meet in LDS, and one lane per
// (offset, cell) adds them in row-group order and writes S.
constexpr int kRegWaves = kThreads / 64;

struct RegGeom {
  int cps, rw, sg, nbs, nb;
};

__host__ __device__ inline RegGeom reg_geom(int s, int P, int k) {
  RegGeom g;
  g.cps = s / P;
  // k = 5: one row group up to s = 8 (its 25 C sums per lane in four row
  // groups would need too much LDS there), four from s = 16 on
  g.rw = (k == 3 || s >= 16) ? (s < kRegWaves ? s : kRegWaves) : 1;
  g.sg = kRegWaves / g.rw;
  g.nbs = 64 / g.cps;
  g.nb = g.sg * g.nbs;
  return g;
}

// LDS float4 words of the register form: LR target cells (k rows of
// nb + k - 1), the code table (k^4 uint2), then, with several row groups,
// their sums (RW x nb cells x k^2 C floats).
__host__ __device__ inline int reg_lds_words(const RegGeom& g, int k, int C) {
  const int K2 = k * k;
  return k * (g.nb + k - 1) + (K2 * K2 * 2 + 3) / 4 + (g.rw > 1 ? (g.rw * g.nb * K2 * C + 3) / 4 : 0);
}

// SELF: self-upsampling gradient.  G then holds the HR guide I and T the LR
// guide, and each pixel's gradient is formed here as
// 2 (alpha T[a] + (1 - alpha) T[b] - I).
template <typename T, int C, int P, int KW, bool SELF = false>
__global__ __launch_bounds__(kThreads) void k_bwd_reg(const BwdArgs a0) {
  extern __shared__ float4 smem[];
  constexpr int K2 = KW * KW, R = KW / 2;
  const BwdArgs a = batch_image<T>(a0);
  const int s = a.s;
  const RegGeom gm = reg_geom(s, P, KW);
  const int cps = gm.cps, nb = gm.nb, nbs = gm.nbs, RW = gm.rw;
  const int qy = blockIdx.x / a.groups_x;
  const int qx0 = (blockIdx.x - qy * a.groups_x) * nb;
  const int lx = nb + KW - 1;
  float4* sT = smem;
  uint2* sDec = reinterpret_cast<uint2*>(sT + KW * lx);
  float* sSum = reinterpret_cast<float*>(sT + KW * lx + (K2 * K2 * 2 + 3) / 4);
  const int tid = (int)threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int seg = wave / RW, rg = wave - seg * RW;
  const T* __restrict__ TL = static_cast<const T*>(a.T);

  // code -> (LDS offsets of the cells a and b relative to the pixel's
  // window corner, window offsets o_a and o_b)
  for (int c = tid; c < K2 * K2; c += kThreads) {
    const int oa = c / K2, ob = c - oa * K2;
    sDec[c] = make_uint2((uint32_t)((oa / KW) * lx + oa % KW) | ((uint32_t)((ob / KW) * lx + ob % KW) << 16),
                         (uint32_t)oa | ((uint32_t)ob << 16));
  }
  if (a.dalpha || SELF) {
    // rows qy - R .. qy + R, columns qx0 - R .. qx0 + nb - 1 + R, clamped to
    // the LR image (codes from the search never leave it)
    for (int i = tid; i < KW * lx; i += kThreads) {
      const int rr = i / lx, c = i - rr * lx;
      const int cy = min(max(qy - R + rr, 0), a.h - 1);
      const int cx = min(max(qx0 - R + c, 0), a.w - 1);
      sT[i] = load_cell<T>(TL + (int64_t)cy * a.T_stride + (int64_t)cx * C, C);
    }
  }
  __syncthreads();

  const bool vecTh = P == 4 && (a.vec & VEC_THETA) != 0, vecG = P == 4 && (a.vec & VEC_G) != 0,
             vecA = P == 4 && (a.vec & VEC_T) != 0;
  const int cls = lane / cps;            // cell in the segment
  const int cl = seg * nbs + cls;        // cell in the workgroup
  const int x = (qx0 + seg * nbs) * s + P * lane;
  const bool mine = seg < gm.sg && lane < nbs * cps;  // the lane owns a column of a cell
  const bool active = mine && x < a.W;               // x < W also keeps the cell inside the image
  const bool full = x + P <= a.W;
  float acc[K2][C];
#pragma unroll
  for (int o = 0; o < K2; ++o)
#pragma unroll
    for (int ch = 0; ch < C; ++ch) acc[o][ch] = 0.f;

  if (active) {
    const int y1 = min(a.H, (qy + 1) * s);
    for (int y = qy * s + rg; y < y1; y += RW) {
      const int64_t to = (int64_t)y * a.th_stride + x;
      int cd[P];
      float al[P];
      bool done = false;
      if constexpr (P == 4) {
        if (vecTh && full) {
          const u32x2 c = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(a.code + to));
          const f32x4 a4 = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(a.alpha + to));
          cd[0] = c.x & 0xffff;
          cd[1] = c.x >> 16;
          cd[2] = c.y & 0xffff;
          cd[3] = c.y >> 16;
          al[0] = a4.x;
          al[1] = a4.y;
          al[2] = a4.z;
          al[3] = a4.w;
          done = true;
        }
      }
      if (!done) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
          const bool ok = full || (x + q < a.W);
          cd[q] = ok ? a.code[to + q] : 0;
          al[q] = ok ? a.alpha[to + q] : 0.f;
        }
      }
      float g[P][4];
      load_grad<P>(a.G + (int64_t)y * a.G_stride, x, a.W, C, vecG, full, g);  // zero past the image
      float da[P];
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const uint2 e = sDec[min(cd[q], K2 * K2 - 1)];
        da[q] = 0.f;
        if constexpr (SELF) {
          // G = 2 (alpha T[a] + (1 - alpha) T[b] - I); zero past the image
          const float4 Ta = sT[cl + (e.x & 0xffff)];
          const float4 Tb = sT[cl + (e.x >> 16)];
          const float ta[4] = {Ta.x, Ta.y, Ta.z, Ta.w}, tb[4] = {Tb.x, Tb.y, Tb.z, Tb.w};
          const bool ok = full || (x + q < a.W);
#pragma unroll
          for (int ch = 0; ch < C; ++ch)
            g[q][ch] = ok ? 2.0f * (fmaf(al[q], ta[ch] - tb[ch], tb[ch]) - g[q][ch]) : 0.0f;
        }
        if (a.dalpha) {
          const float4 Ta = sT[cl + (e.x & 0xffff)];
          const float4 Tb = sT[cl + (e.x >> 16)];
          const float dv[4] = {Ta.x - Tb.x, Ta.y - Tb.y, Ta.z - Tb.z, Ta.w - Tb.w};
          float v = g[q][0] * dv[0];
#pragma unroll
          for (int ch = 1; ch < C; ++ch) v = fmaf(g[q][ch], dv[ch], v);
          da[q] = v;
        }
        if (a.S) {
          const int oa = (int)(e.y & 0xffff), ob = (int)(e.y >> 16);
          // o_a and o_b differ except in a (j, j) code, where the one weight
          // is alpha + (1 - alpha), summed in float like the two terms
          const float wb = 1.0f - al[q];
          const float wa = oa == ob ? al[q] + wb : al[q];
#pragma unroll
          for (int o = 0; o < K2; ++o) {
            const float wt = oa == o ? wa : (ob == o ? wb : 0.0f);
#pragma unroll
            for (int ch = 0; ch < C; ++ch) acc[o][ch] = fmaf(wt, g[q][ch], acc[o][ch]);
          }
        }
      }
      if (a.dalpha) {
        bool st = false;
        if constexpr (P == 4) {
          if (vecA && full) {
            __builtin_nontemporal_store(f32x4{da[0], da[1], da[2], da[3]}, reinterpret_cast<f32x4*>(a.dalpha + to));
            st = true;
          }
        }
        if (!st) {
#pragma unroll
          for (int q = 0; q < P; ++q)
            if (full || x + q < a.W) a.dalpha[to + q] = da[q];
        }
      }
    }
  }
  if (!a.S) return;
  // the first lane of each cell adds up its cps lanes (every lane takes part
  // in the cross-lane reads): a butterfly when cps is a power of two, else
  // in lane order
  if ((cps & (cps - 1)) == 0) {
    for (int m = 1; m < cps; m <<= 1) {
#pragma unroll
      for (int o = 0; o < K2; ++o)
#pragma unroll
        for (int ch = 0; ch < C; ++ch) acc[o][ch] += __shfl_xor(acc[o][ch], m, 64);
    }
  } else {
    const int first = min(cls, nbs - 1) * cps;
#pragma unroll
    for (int o = 0; o < K2; ++o)
#pragma unroll
      for (int ch = 0; ch < C; ++ch) {
        float v = __shfl(acc[o][ch], first, 64);
        for (int j = 1; j < cps; ++j) v += __shfl(acc[o][ch], first + j, 64);
        acc[o][ch] = v;
      }
  }
  const int64_t hw = (int64_t)a.h * a.w;
  if (RW == 1) {
    // one row group: the cell's first lane holds the whole sum
    if (active && lane % cps == 0) {
      float* out = a.S + ((int64_t)qy * a.w + qx0 + cl) * C;
#pragma unroll
      for (int o = 0; o < K2; ++o)
#pragma unroll
        for (int ch = 0; ch < C; ++ch) out[(int64_t)o * hw * C + ch] = acc[o][ch];
    }
    return;
  }
  if (mine && lane % cps == 0) {
    float* dst = sSum + ((rg * nb + cl) * K2) * C;
#pragma unroll
    for (int o = 0; o < K2; ++o)
#pragma unroll
      for (int ch = 0; ch < C; ++ch) dst[o * C + ch] = acc[o][ch];
  }
  __syncthreads();
  const int nbv = min(nb, a.w - qx0);
  for (int i = tid; i < K2 * nbv; i += kThreads) {
    const int o = i / nbv, c = i - o * nbv;
    float v[C];
#pragma unroll
    for (int ch = 0; ch < C; ++ch) v[ch] = 0.f;
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int ch = 0; ch < C; ++ch) v[ch] += sSum[((r * nb + c) * K2 + o) * C + ch];
    float* out = a.S + ((int64_t)o * hw + (int64_t)qy * a.w + qx0 + c) * C;
#pragma unroll
    for (int ch = 0; ch < C; ++ch) out[ch] = v[ch];
  }
}

template <int P, int KW>
static BwdKernel pick_reg_p(bool f16, int C) {
  switch (C) {
    case 1: return f16 ? k_bwd_reg<__half, 1, P, KW> : k_bwd_reg<float, 1, P, KW>;
    case 2: return f16 ? k_bwd_reg<__half, 2, P, KW> : k_bwd_reg<float, 2, P, KW>;
    case 3: return f16 ? k_bwd_reg<__half, 3, P, KW> : k_bwd_reg<float, 3, P, KW>;
    default: return f16 ? k_bwd_reg<__half, 4, P, KW> : k_bwd_reg<float, 4, P, KW>;
  }
}

static BwdKernel pick_reg(bool f16, int C, int P, int k, bool self_grad) {
  if (self_grad) {
    // float32 guides with 3 channels only
    if (k == 5) return k_bwd_reg<float, 3, 4, 5, true>;
    if (P == 4) return k_bwd_reg<float, 3, 4, 3, true>;
    if (P == 3) return k_bwd_reg<float, 3, 3, 3, true>;
    return k_bwd_reg<float, 3, 2, 3, true>;
  }
  if (k == 5) return pick_reg_p<4, 5>(f16, C);
  if (P == 4) return pick_reg_p<4, 3>(f16, C);
  if (P == 3) return pick_reg_p<3, 3>(f16, C);
  return pick_reg_p<2, 3>(f16, C);
}

// The register form covers 3 x 3 windows whose s has a strip width P of 4,
// 3 or 2 pixels, and 5 x 5 windows with P = 4; s / P <= 64 lanes per cell
// row.
static bool reg_geometry(int s, int k, int C, int& P) {
  P = strip_pixels(s);
  if (s / P > 64) return false;
  if (!((k == 3 && P >= 2) || (k == 5 && P == 4))) return false;
  return 16 * reg_lds_words(reg_geom(s, P, k), k, C) <= 64 * 1024;
}

// Pass 2: dL/dT_low[q] = sum over window offsets o = (dy, dx) of S[o][c]
// for the cells c whose offset o points at q.  The apply reads a window
// position outside the LR image as the nearest in-image cell, so such a
// position's gradient goes to that cell too.
// * Border cells (the ring of cells on the first or last row or column), in
//   the first ring_blocks workgroups: per offset every c with
//   clamp(c + d) = q, in ascending order.  One thread per (cell, offset)
//   sums that offset's sources (at most (r + 1)^2, loaded together), then
//   one thread per cell adds the k^2 partial sums in offset order: every
//   load of the ring is in flight at once, so the few ring workgroups finish
//   within the interior's time.  Codes from the search never point outside
//   the image, and then every extra source holds zero sums.
// * Interior cells, one thread each, in the remaining workgroups: the source
//   of offset o is c = q - (dy, dx) alone, in the image for every offset
//   when k = 3.
__device__ __forceinline__ void ring_cell(int64_t i, int h, int w, int& qy, int& qx) {
  // row 0, row h - 1 (h > 1), then columns 0 and w - 1 (w > 1) of rows
  // 1 .. h - 2
  const int rows2 = h > 1 ? 2 : 1, per = w > 1 ? 2 : 1;
  if (i < (int64_t)rows2 * w) {
    const int j = (int)i;
    qy = j < w ? 0 : h - 1;
    qx = j < w ? j : j - w;
  } else {
    const int j = (int)(i - (int64_t)rows2 * w);
    qy = 1 + j / per;
    qx = (j % per) ? w - 1 : 0;
  }
}

// source rows (or columns) lo .. hi of offset component dd at q in an axis
// of n cells: every c with clamp(c + dd) = q, at most r + 1 of them
__device__ __forceinline__ void clamp_sources(int q, int dd, int n, int& lo, int& hi) {
  if (n == 1) {
    lo = 0;
    hi = 0;
  } else if (q == 0 && dd <= 0) {
    lo = 0;
    hi = min(n - 1, -dd);
  } else if (q == n - 1 && dd >= 0) {
    lo = max(0, n - 1 - dd);
    hi = n - 1;
  } else {
    lo = hi = q - dd;  // empty when outside [0, n)
    if (lo < 0 || lo >= n) hi = lo - 1;
  }
}

template <int KW, int C>
__global__ __launch_bounds__(256) void k_bwd_lr(const BwdArgs a0) {
  const BwdArgs a = batch_image<float>(a0);  // T is not read here
  const int h = a.h, w = a.w;
  const int64_t hw = (int64_t)h * w;
  const int k = KW > 0 ? KW : a.k;
  const int r = k / 2, K2 = k * k;
  if ((int)blockIdx.x < a.ring_blocks) {
    __shared__ float part[256 * C];
    const int cpb = 256 / K2;  // ring cells per workgroup
    const int t = (int)threadIdx.x;
    const int cl = t / K2, o = t - cl * K2;
    const int64_t inner = (h > 2 && w > 2) ? (int64_t)(h - 2) * (w - 2) : 0;
    const int64_t ci = (int64_t)blockIdx.x * cpb + cl;
    const bool live = cl < cpb && ci < hw - inner;
    int qy = 0, qx = 0;
    float p[C];
#pragma unroll
    for (int ch = 0; ch < C; ++ch) p[ch] = 0.f;
    if (live) {
      ring_cell(ci, h, w, qy, qx);
      int y0, y1, x0, x1;
      clamp_sources(qy, o / k - r, h, y0, y1);
      clamp_sources(qx, o % k - r, w, x0, x1);
      if constexpr (KW > 0) {
        constexpr int NS = KW / 2 + 1;
#pragma unroll
        for (int iy = 0; iy < NS; ++iy)
#pragma unroll
          for (int ix = 0; ix < NS; ++ix) {
            const int cy = y0 + iy, cx = x0 + ix;
            const bool v = cy <= y1 && cx <= x1;
            const float* src = a.S + ((int64_t)o * hw + (v ? (int64_t)cy * w + cx : 0)) * C;
#pragma unroll
            for (int ch = 0; ch < C; ++ch) p[ch] += v ? src[ch] : 0.0f;
          }
      } else {
        for (int cy = y0; cy <= y1; ++cy)
          for (int cx = x0; cx <= x1; ++cx) {
            const float* src = a.S + ((int64_t)o * hw + (int64_t)cy * w + cx) * C;
#pragma unroll
            for (int ch = 0; ch < C; ++ch) p[ch] += src[ch];
          }
      }
    }
#pragma unroll
    for (int ch = 0; ch < C; ++ch) part[t * C + ch] = p[ch];
    __syncthreads();
    if (live && o == 0) {
      float acc[C];
#pragma unroll
      for (int ch = 0; ch < C; ++ch) acc[ch] = 0.f;
      for (int oo = 0; oo < K2; ++oo)
#pragma unroll
        for (int ch = 0; ch < C; ++ch) acc[ch] += part[(t + oo) * C + ch];
      float* out = a.dT + (int64_t)qy * a.dT_stride + (int64_t)qx * C;
#pragma unroll
      for (int ch = 0; ch < C; ++ch) out[ch] = acc[ch];
    }
    return;
  }
  const int64_t i = (int64_t)(blockIdx.x - a.ring_blocks) * 256 + threadIdx.x;
  const int wi = w - 2;
  if (i >= (int64_t)(h - 2) * wi) return;
  const int64_t ry = hw < 0x7fffffff ? (int64_t)((uint32_t)i / (uint32_t)wi) : i / wi;
  const int qy = 1 + (int)ry, qx = 1 + (int)(i - ry * wi);
  float acc[C];
#pragma unroll
  for (int ch = 0; ch < C; ++ch) acc[ch] = 0.f;
  // every offset unrolled for k = 3, one row of offsets for k = 5 and 7
  constexpr int kUnroll = KW == 3 ? 9 : (KW > 0 ? KW : 1);
#pragma unroll kUnroll
  for (int o = 0; o < K2; ++o) {
    const int cy = qy - (o / k - r), cx = qx - (o % k - r);
    if constexpr (KW == 3) {
      const float* src = a.S + ((int64_t)o * hw + (int64_t)cy * w + cx) * C;
#pragma unroll
      for (int ch = 0; ch < C; ++ch) acc[ch] += src[ch];
    } else {
      const bool in = cy >= 0 && cy < h && cx >= 0 && cx < w;
      const float* src = a.S + ((int64_t)o * hw + (in ? (int64_t)cy * w + cx : 0)) * C;
#pragma unroll
      for (int ch = 0; ch < C; ++ch) acc[ch] += in ? src[ch] : 0.0f;
    }
  }
  float* out = a.dT + (int64_t)qy * a.dT_stride + (int64_t)qx * C;
#pragma unroll
  for (int ch = 0; ch < C; ++ch) out[ch] = acc[ch];
}

template <int KW>
static BwdKernel pick_lr_c(int C) {
  switch (C) {
    case 1: return k_bwd_lr<KW, 1>;
    case 2: return k_bwd_lr<KW, 2>;
    case 3: return k_bwd_lr<KW, 3>;
    default: return k_bwd_lr<KW, 4>;
  }
}

// Cells per workgroup (one scan lane per (cell, offset)) and HR rows per
// chunk, chunks shrunk until the LDS of a workgroup is at most 32 KiB.
static void bwd_geometry(int s, int k, int w, int& nb, int& rows_chunk) {
  const int K2 = k * k;
  nb = std::max(1, std::min(kThreads / K2, w));
  rows_chunk = s;
  while (rows_chunk > 1 && 16 * bwd_lds_words(k, nb, s, rows_chunk) > 32 * 1024) rows_chunk = (rows_chunk + 1) / 2;
  while (nb > 1 && 16 * bwd_lds_words(k, nb, s, rows_chunk) > 32 * 1024) nb = (nb + 1) / 2;
}

// The workspace of glu_apply_backward_static: one array per device (each GPU
// holds its own copy at its own address).  Host code uses only the address
// hipGetSymbolAddress returns for the current device, never the array's
// name, which on the host is a stand-in, not a device address.
static __device__ __align__(256) char scratch[GLU_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Device address of the current device's array, looked up on the first
// call with that device current.
static glu_status static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "static scratch: current device");
  if (dev < 0 || dev >= kMaxDevices) return fail(GLU_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "static scratch address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return GLU_OK;
}

}  // namespace glu

using namespace glu;

extern "C" {

size_t glu_apply_backward_workspace(int32_t H, int32_t W, int32_t C, const glu_params* p) {
  if (!p || p->s < 1 || p->k < 1 || H < 0 || W < 0 || C < 1 || C > 4) return 0;
  const int64_t h = ceil_div(H, p->s), w = ceil_div(W, p->s);
  return (size_t)(h * w * p->k * p->k * C) * sizeof(float);
}

size_t glu_apply_backward_batched_workspace(int32_t n, int32_t H, int32_t W, int32_t C, const glu_params* p) {
  if (n < 0) return 0;
  return (size_t)n * glu_apply_backward_workspace(H, W, C, p);
}

static glu_status backward_batched(int32_t n, const glu_batch_strides* bs, const glu_theta* theta,
                                   const glu_image* T_low, const glu_params* p, const glu_image* grad_T_hat,
                                   glu_image* grad_T_low, float* grad_alpha, void* workspace, size_t ws_bytes,
                                   void* stream, bool self_grad = false) {
  glu_status st;
  if ((st = check_batch(n, bs, true))) return st;
  if ((st = check_params(p))) return st;
  if ((st = check_image(T_low, "T_low", 1, 4))) return st;
  if ((st = check_image(grad_T_hat, "grad_T_hat", 1, 4, false))) return st;
  const int H = grad_T_hat->height, W = grad_T_hat->width, C = T_low->channels;
  if ((st = check_theta(theta, H, W, true))) return st;
  const int h = ceil_div(H, p->s), w = ceil_div(W, p->s);
  if (T_low->height != h || T_low->width != w) return fail(GLU_ERR_SHAPE, "T_low must be ceil(H/s) x ceil(W/s)");
  if (grad_T_hat->channels != C) return fail(GLU_ERR_SHAPE, "grad_T_hat channels differ from T_low");
  if (grad_T_low) {
    if ((st = check_image(grad_T_low, "grad_T_low", 1, 4, false))) return st;
    if (grad_T_low->height != h || grad_T_low->width != w || grad_T_low->channels != C)
      return fail(GLU_ERR_SHAPE, "grad_T_low must match T_low");
  }
  if (grad_alpha && reinterpret_cast<uintptr_t>(grad_alpha) % 4) return fail(GLU_ERR_ALIGN, "grad_alpha not aligned");
  if (n > 1) {
    if (grad_T_low && bs->grad_T_low < (int64_t)(h - 1) * grad_T_low->row_stride + (int64_t)w * C)
      return fail(GLU_ERR_SHAPE, "grad_T_low batch stride makes images overlap");
    if (grad_alpha && bs->grad_alpha < (int64_t)(H - 1) * theta->row_stride + W)
      return fail(GLU_ERR_SHAPE, "grad_alpha batch stride makes images overlap");
  }
  if (grad_T_low && (int64_t)H * W > 0 && n > 0) {
    const size_t need = glu_apply_backward_batched_workspace(n, H, W, C, p);
    if (!workspace || ws_bytes < need)
      return fail(GLU_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    if (reinterpret_cast<uintptr_t>(workspace) % 4) return fail(GLU_ERR_ALIGN, "workspace not aligned");
  }
  if ((int64_t)H * W == 0 || n == 0) return GLU_OK;
  if (!grad_T_low && !grad_alpha) return GLU_OK;
  BwdArgs a{};
  a.code = theta->code;
  a.alpha = theta->alpha;
  a.T = T_low->data;
  a.G = static_cast<const float*>(grad_T_hat->data);
  a.dalpha = grad_alpha;
  a.S = grad_T_low ? static_cast<float*>(workspace) : nullptr;
  a.dT = grad_T_low ? static_cast<float*>(grad_T_low->data) : nullptr;
  a.th_stride = theta->row_stride;
  a.T_stride = T_low->row_stride;
  a.G_stride = grad_T_hat->row_stride;
  a.dT_stride = grad_T_low ? grad_T_low->row_stride : 0;
  a.H = H;
  a.W = W;
  a.h = h;
  a.w = w;
  a.s = p->s;
  a.k = p->k;
  a.C = C;
  if (n > 1) {
    a.b_th = bs->theta;
    a.b_T = bs->T_low;
    a.b_G = bs->T_hat;
    a.b_da = bs->grad_alpha;
    a.b_dT = bs->grad_T_low;
    a.b_S = (int64_t)(glu_apply_backward_workspace(H, W, C, p) / sizeof(float));
  }
  int regP = 0;
  const bool reg = reg_geometry(p->s, p->k, C, regP);
  if (self_grad && (!reg || C != 3 || grad_alpha || T_low->dtype != GLU_F32))
    return fail(GLU_ERR_UNSUPPORTED,
                "self-upsampling gradient needs the register form, a 3-channel float32 guide and no dalpha");
  if (reg)
    a.nb = reg_geom(p->s, regP, p->k).nb;
  else
    bwd_geometry(p->s, p->k, w, a.nb, a.rows_chunk);
  a.groups_x = ceil_div(w, a.nb);
  a.s_magic = (uint32_t)std::min<uint64_t>(0xffffffffull, (1ull << 32) / (uint64_t)p->s);
  const int P = reg ? regP : ((p->s % 4 == 0) ? 4 : 1);
  {
    // alignment of the vector paths (all with x a multiple of 4), for every
    // image of the batch
    auto al = [](const void* q, size_t m) { return (reinterpret_cast<uintptr_t>(q) % m) == 0; };
    uint32_t v = 0;
    if (P == 4 && theta->row_stride % 4 == 0 && al(theta->code, 8) && al(theta->alpha, 16) &&
        (!grad_alpha || al(grad_alpha, 16)) && a.b_th % 4 == 0 && a.b_da % 4 == 0)
      v |= VEC_THETA | VEC_T;
    if (P == 4 && (C == 3 || C == 1) && grad_T_hat->row_stride % 4 == 0 && al(grad_T_hat->data, 16) &&
        a.b_G % 4 == 0)
      v |= VEC_G;
    a.vec = v;
  }
  const size_t lds = (size_t)16 * (reg ? reg_lds_words(reg_geom(p->s, regP, p->k), p->k, C) : bwd_lds_words(p->k, a.nb, p->s, a.rows_chunk));
  const int64_t groups = (int64_t)h * a.groups_x;
  if (groups > 0x7fffffff) return fail(GLU_ERR_UNSUPPORTED, "image too large");
  hipStream_t sm = (hipStream_t)stream;
  BwdKernel kern = reg ? pick_reg(T_low->dtype == GLU_F16, C, regP, p->k, self_grad) : pick_bwd(T_low->dtype == GLU_F16, P, p->k, C);
  hipLaunchKernelGGL(kern, dim3((unsigned)groups, (unsigned)n), dim3(kThreads), lds, sm, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "backward pass 1 launch");
  if (grad_T_low) {
    // the ring of border cells first, then the interior cells (k_bwd_lr)
    const int64_t inner = (h > 2 && w > 2) ? (int64_t)(h - 2) * (w - 2) : 0;
    const int64_t ring = (int64_t)h * w - inner;
    const int64_t cells_per_ring_block = 256 / ((int64_t)p->k * p->k);
    const int64_t blocks_ring = (ring + cells_per_ring_block - 1) / cells_per_ring_block;
    const int64_t blocks = blocks_ring + (inner + 255) / 256;
    if (blocks > 0x7fffffff) return fail(GLU_ERR_UNSUPPORTED, "image too large");
    a.ring_blocks = (int32_t)blocks_ring;
    BwdKernel lr = p->k == 3 ? pick_lr_c<3>(C) : p->k == 5 ? pick_lr_c<5>(C) : p->k == 7 ? pick_lr_c<7>(C) : pick_lr_c<0>(C);
    hipLaunchKernelGGL(lr, dim3((unsigned)blocks, (unsigned)n), dim3(256), 0, sm, a);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "backward pass 2 launch");
  }
  return GLU_OK;
}

glu_status glu_apply_backward(const glu_theta* theta, const glu_image* T_low, const glu_params* p,
                              const glu_image* grad_T_hat, glu_image* grad_T_low, float* grad_alpha, void* workspace,
                              size_t ws_bytes, void* stream) {
  clear_error();
  return backward_batched(1, nullptr, theta, T_low, p, grad_T_hat, grad_T_low, grad_alpha, workspace, ws_bytes,
                          stream);
}

glu_status glu_apply_backward_batched(int32_t n, const glu_batch_strides* strides, const glu_theta* theta,
                                      const glu_image* T_low, const glu_params* p, const glu_image* grad_T_hat,
                                      glu_image* grad_T_low, float* grad_alpha, void* workspace, size_t ws_bytes,
                                      void* stream) {
  clear_error();
  return backward_batched(n, strides, theta, T_low, p, grad_T_hat, grad_T_low, grad_alpha, workspace, ws_bytes,
                          stream);
}

glu_status glu_apply_backward_static(const glu_theta* theta, const glu_image* T_low, const glu_params* p,
                                     const glu_image* grad_T_hat, glu_image* grad_T_low, float* grad_alpha,
                                     void* stream) {
  clear_error();
  void* ws = nullptr;
  if (grad_T_low) {
    if (!p) return fail(GLU_ERR_NULL, "params is NULL");
    if (!grad_T_hat || !T_low) return fail(GLU_ERR_NULL, "image descriptor is NULL");
    const size_t need = glu_apply_backward_workspace(grad_T_hat->height, grad_T_hat->width, T_low->channels, p);
    if (need > GLU_STATIC_SCRATCH_BYTES)
      return fail(GLU_ERR_WORKSPACE, "workspace of %zu bytes needed, the static array holds %zu", need,
                  (size_t)GLU_STATIC_SCRATCH_BYTES);
    glu_status st = static_scratch(&ws);
    if (st) return st;
  }
  return backward_batched(1, nullptr, theta, T_low, p, grad_T_hat, grad_T_low, grad_alpha, ws,
                          GLU_STATIC_SCRATCH_BYTES, stream);
}

}  // extern "C"

namespace glu {

glu_status apply_backward_selfgrad(const glu_theta* theta, const glu_image* I_low, const glu_params* p,
                                   const glu_image* I, glu_image* grad_I_low, void* workspace, size_t ws_bytes,
                                   void* stream) {
  return backward_batched(1, nullptr, theta, I_low, p, I, grad_I_low, nullptr, workspace, ws_bytes, stream, true);
}

}  // namespace glu
