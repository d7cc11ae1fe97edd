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
//     every window offset o, S[c][o] = sum over the pixels of c's s x s
//     block, in raster order, of the part of their contribution aimed at the
//     cell c + offset(o).  A workgroup owns nb consecutive cells of one LR
//     row: it streams their s HR rows (vector loads, dL/dalpha written on
//     the way) into LDS, then one thread per (cell, o) scans the block's
//     pixels in raster order.
//   pass 2 (LR): dT_low[q] = sum over o in ascending order of
//     S[q - offset(o)][o].
//
// Both passes use fixed summation orders, so results are bitwise
// reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>

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
  int32_t nb;           // LR cells per workgroup (one LR row)
  int32_t rows_chunk;   // HR rows staged per chunk
  int32_t groups_x;     // workgroups per LR row
  uint32_t s_magic;     // floor(2^32 / s) for udiv_rt
  uint32_t vec;         // VEC_THETA | VEC_G | VEC_T(dalpha rows)
};

// Loads C <= 4 gradient channels of pixels x .. x+P-1 (vector path for
// P = 4, C = 3 or 1 on aligned rows).
template <int P>
__device__ __forceinline__ void load_grad(const float* __restrict__ row, int x, int W, int C, bool vec, bool full,
                                          float (&g)[P][4]) {
  const float* p = row + (int64_t)x * C;
  if constexpr (P == 4) {
    if (vec && full && C == 3) {
      const float4* q = reinterpret_cast<const float4*>(p);
      const float4 a = q[0], b = q[1], c = q[2];
      g[0][0] = a.x; g[0][1] = a.y; g[0][2] = a.z;
      g[1][0] = a.w; g[1][1] = b.x; g[1][2] = b.y;
      g[2][0] = b.z; g[2][1] = b.w; g[2][2] = c.x;
      g[3][0] = c.y; g[3][1] = c.z; g[3][2] = c.w;
#pragma unroll
      for (int i = 0; i < 4; ++i) g[i][3] = 0.f;
      return;
    }
    if (vec && full && C == 1) {
      const float4 a = *reinterpret_cast<const float4*>(p);
      g[0][0] = a.x; g[1][0] = a.y; g[2][0] = a.z; g[3][0] = a.w;
#pragma unroll
      for (int i = 0; i < 4; ++i) g[i][1] = g[i][2] = g[i][3] = 0.f;
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const bool ok = full || (x + i < W);
#pragma unroll
    for (int c = 0; c < 4; ++c) g[i][c] = (ok && c < C) ? p[i * C + c] : 0.f;
  }
}

// LDS layout of pass 1 for one chunk of HR rows of the group: per pixel slot
// a packed code word (o_a | o_b << 8), alpha, and C gradient values (SoA).
template <typename T, int P>
__global__ __launch_bounds__(kThreads) void k_bwd_block(const BwdArgs a) {
  extern __shared__ float4 smem[];
  const int k = a.k, r = k / 2, K2 = k * k, s = a.s, C = a.C;
  const int qy = blockIdx.x / a.groups_x;
  const int qx0 = (blockIdx.x - qy * a.groups_x) * a.nb;
  const int nb = min(a.nb, a.w - qx0);
  const int chunk_px = a.rows_chunk * a.nb * s;  // pixel slots per chunk
  int* sCode = reinterpret_cast<int*>(smem);
  float* sAl = reinterpret_cast<float*>(sCode + chunk_px);
  float* sG = sAl + chunk_px;  // C * chunk_px
  const T* __restrict__ TL = static_cast<const T*>(a.T);
  const bool vecTh = (a.vec & VEC_THETA) != 0, vecG = (a.vec & VEC_G) != 0, vecA = (a.vec & VEC_T) != 0;

  const int y0 = qy * s, y1 = min(a.H, y0 + s);
  const int x0 = qx0 * s, x1 = min(a.W, x0 + nb * s);
  const int seg = x1 - x0;             // pixels per HR row of the group
  const int spr = (seg + P - 1) / P;   // strips per HR row of the group
  const int n_pairs_grp = nb * K2;
  float acc[2][4];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) acc[u][ch] = 0.f;

  for (int yc = y0; yc < y1; yc += a.rows_chunk) {
    const int yce = min(y1, yc + a.rows_chunk);
    const int nstrips = (yce - yc) * spr;
    for (int t = threadIdx.x; t < nstrips; t += kThreads) {
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
      const int qx = udiv_rt(x, s, a.s_magic);  // all P pixels share it
      float da[P];
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const int cdc = min(cd[q], K2 * K2 - 1);
        const int oa = cdc / K2, ob = cdc - oa * K2;
        const int i = ry * seg + rx + q;
        if (full || rx + q < seg) {
          sCode[i] = oa | (ob << 8);
          sAl[i] = al[q];
#pragma unroll
          for (int ch = 0; ch < 4; ++ch)
            if (ch < C) sG[ch * chunk_px + i] = g[q][ch];
        }
        da[q] = 0.f;
        if (a.dalpha && (full || rx + q < seg)) {
          const int ay = min(max(qy + oa / k - r, 0), a.h - 1), ax = min(max(qx + oa % k - r, 0), a.w - 1);
          const int by = min(max(qy + ob / k - r, 0), a.h - 1), bx = min(max(qx + ob % k - r, 0), a.w - 1);
          const float4 Ta = load_cell<T>(TL + (int64_t)ay * a.T_stride + (int64_t)ax * C, C);
          const float4 Tb = load_cell<T>(TL + (int64_t)by * a.T_stride + (int64_t)bx * C, C);
          float v = g[q][0] * (Ta.x - Tb.x);
          if (C > 1) v = fmaf(g[q][1], Ta.y - Tb.y, v);
          if (C > 2) v = fmaf(g[q][2], Ta.z - Tb.z, v);
          if (C > 3) v = fmaf(g[q][3], Ta.w - Tb.w, v);
          da[q] = v;
        }
      }
      if (a.dalpha) {
        bool st = false;
        if constexpr (P == 4) {
          if (vecA && full) {
            *reinterpret_cast<float4*>(a.dalpha + to) = make_float4(da[0], da[1], da[2], da[3]);
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
    __syncthreads();
    if (a.S) {
      // each thread owns up to two (cell, offset) pairs of the group
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int pr = threadIdx.x + u * kThreads;
        if (pr >= n_pairs_grp) continue;
        const int cell = pr / K2, o = pr - cell * K2;
        const int cx0 = cell * s, cx1 = min(seg, cx0 + s);  // pixel columns of this cell
        for (int ry = 0; ry < yce - yc; ++ry) {
          for (int rx = cx0; rx < cx1; ++rx) {
            const int i = ry * seg + rx;
            const int pk = sCode[i];
            const int oa = pk & 0xff, ob = pk >> 8;
            if (oa == o || ob == o) {
              const float al = sAl[i];
              float wgt = (oa == o) ? al : 0.0f;
              wgt = (ob == o) ? wgt + (1.0f - al) : wgt;
#pragma unroll
              for (int ch = 0; ch < 4; ++ch)
                if (ch < C) acc[u][ch] = fmaf(wgt, sG[ch * chunk_px + i], acc[u][ch]);
            }
          }
        }
      }
    }
    __syncthreads();
  }
  if (a.S) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int pr = threadIdx.x + u * kThreads;
      if (pr >= n_pairs_grp) continue;
      const int cell = pr / K2, o = pr - cell * K2;
      float* out = a.S + (((int64_t)qy * a.w + qx0 + cell) * K2 + o) * C;
#pragma unroll
      for (int ch = 0; ch < 4; ++ch)
        if (ch < C) out[ch] = acc[u][ch];
    }
  }
}

__global__ __launch_bounds__(256) void k_bwd_lr(const BwdArgs a) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)a.h * a.w) return;
  const int qy = (int)(q / a.w), qx = (int)(q - (int64_t)qy * a.w);
  const int k = a.k, r = k / 2, K2 = k * k, C = a.C;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int o = 0; o < K2; ++o) {
    // the cell c whose window offset o points at q: c = q - (o / k - r, o % k - r)
    const int cy = qy - (o / k - r), cx = qx - (o % k - r);
    if (cy < 0 || cy >= a.h || cx < 0 || cx >= a.w) continue;
    const float* src = a.S + (((int64_t)cy * a.w + cx) * K2 + o) * C;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch)
      if (ch < C) acc[ch] += src[ch];
  }
  float* out = a.dT + (int64_t)qy * a.dT_stride + (int64_t)qx * C;
#pragma unroll
  for (int ch = 0; ch < 4; ++ch)
    if (ch < C) out[ch] = acc[ch];
}

static void bwd_geometry(int s, int k, int C, int w, int& nb, int& rows_chunk) {
  const int K2 = k * k;
  nb = std::max(1, std::min(2 * kThreads / K2, w));
  // limit the cells of a group so one HR row of it stays within a few strips
  nb = std::min(nb, std::max(1, 512 / s));
  const int bytes_per_px = 4 * (2 + C);
  auto lds = [&](int n, int rc) { return bytes_per_px * rc * n * s; };
  rows_chunk = s;
  while (rows_chunk > 1 && lds(nb, rows_chunk) > kLdsBudget) rows_chunk = (rows_chunk + 1) / 2;
  while (nb > 1 && lds(nb, rows_chunk) > kLdsBudget) nb = (nb + 1) / 2;
}

}  // namespace glu

using namespace glu;

extern "C" {

size_t glu_apply_backward_workspace(int32_t H, int32_t W, int32_t C, const glu_params* p) {
  if (!p || p->s < 1 || p->k < 1 || H < 0 || W < 0 || C < 1 || C > 4) return 0;
  const int64_t h = ceil_div(H, p->s), w = ceil_div(W, p->s);
  return (size_t)(h * w * p->k * p->k * C) * sizeof(float);
}

glu_status glu_apply_backward(const glu_theta* theta, const glu_image* T_low, const glu_params* p,
                              const glu_image* grad_T_hat, glu_image* grad_T_low, float* grad_alpha, void* workspace,
                              size_t ws_bytes, void* stream) {
  clear_error();
  glu_status st;
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
  if (grad_T_low && (int64_t)H * W > 0) {
    const size_t need = glu_apply_backward_workspace(H, W, C, p);
    if (!workspace || ws_bytes < need)
      return fail(GLU_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    if (reinterpret_cast<uintptr_t>(workspace) % 4) return fail(GLU_ERR_ALIGN, "workspace not aligned");
  }
  if ((int64_t)H * W == 0) return GLU_OK;
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
  bwd_geometry(p->s, p->k, C, w, a.nb, a.rows_chunk);
  a.groups_x = ceil_div(w, a.nb);
  a.s_magic = (uint32_t)std::min<uint64_t>(0xffffffffull, (1ull << 32) / (uint64_t)p->s);
  const int P = (p->s % 4 == 0) ? 4 : 1;
  {
    // alignment of the vector paths (all with x a multiple of 4)
    auto al = [](const void* q, size_t n) { return (reinterpret_cast<uintptr_t>(q) % n) == 0; };
    uint32_t v = 0;
    if (P == 4 && theta->row_stride % 4 == 0 && al(theta->code, 8) && al(theta->alpha, 16) &&
        (!grad_alpha || al(grad_alpha, 16)))
      v |= VEC_THETA | VEC_T;
    if (P == 4 && (C == 3 || C == 1) && grad_T_hat->row_stride % 4 == 0 && al(grad_T_hat->data, 16)) v |= VEC_G;
    a.vec = v;
  }
  const size_t lds = (size_t)4 * (2 + C) * a.rows_chunk * a.nb * p->s;
  const int64_t groups = (int64_t)h * a.groups_x;
  if (groups > 0x7fffffff) return fail(GLU_ERR_UNSUPPORTED, "image too large");
  hipStream_t sm = (hipStream_t)stream;
  if (T_low->dtype == GLU_F16) {
    if (P == 4)
      hipLaunchKernelGGL((k_bwd_block<__half, 4>), dim3((unsigned)groups), dim3(kThreads), lds, sm, a);
    else
      hipLaunchKernelGGL((k_bwd_block<__half, 1>), dim3((unsigned)groups), dim3(kThreads), lds, sm, a);
  } else {
    if (P == 4)
      hipLaunchKernelGGL((k_bwd_block<float, 4>), dim3((unsigned)groups), dim3(kThreads), lds, sm, a);
    else
      hipLaunchKernelGGL((k_bwd_block<float, 1>), dim3((unsigned)groups), dim3(kThreads), lds, sm, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "backward pass 1 launch");
  if (grad_T_low) {
    const int64_t n = (int64_t)h * w;
    hipLaunchKernelGGL(k_bwd_lr, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, sm, a);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "backward pass 2 launch");
  }
  return GLU_OK;
}

}  // extern "C"
