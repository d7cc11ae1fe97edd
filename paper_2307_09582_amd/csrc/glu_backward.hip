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
//     cell c + offset(o).  One thread owns one (c, o) pair and scans the
//     block's pixels from LDS in a fixed order.  The same pass writes
//     dL/dalpha.
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
};

// LDS layout of pass 1: staged T_low cells (float4), then per staged pixel a
// packed code word, alpha, and C gradient values (SoA).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bwd_block(const BwdArgs a) {
  extern __shared__ float4 smem[];
  const int k = a.k, r = k / 2, K2 = k * k, s = a.s, C = a.C;
  const int groups_x = (a.w + a.nb - 1) / a.nb;
  const int qy = blockIdx.x / groups_x;
  const int qx0 = (blockIdx.x - qy * groups_x) * a.nb;
  const int nb = min(a.nb, a.w - qx0);
  const int ly = 1 + 2 * r, lx = nb + 2 * r;
  float4* sT = smem;                                       // ly * lx cells
  const int chunk_px = a.rows_chunk * a.nb * s;            // pixel slots per chunk
  int* sCode = reinterpret_cast<int*>(sT + ly * lx);       // chunk_px
  float* sAl = reinterpret_cast<float*>(sCode + chunk_px);  // chunk_px
  float* sG = sAl + chunk_px;                              // C * chunk_px

  // stage the T_low cells the chunk's pixels can reach (for dalpha)
  if (a.dalpha) {
    const T* TL = static_cast<const T*>(a.T);
    for (int c = threadIdx.x; c < ly * lx; c += kThreads) {
      const int oy = c / lx;
      const int cy = qy - r + oy, cx = qx0 - r + (c - oy * lx);
      float tt[4] = {0.f, 0.f, 0.f, 0.f};
      if (cy >= 0 && cy < a.h && cx >= 0 && cx < a.w) {
        const T* q = TL + (int64_t)cy * a.T_stride + (int64_t)cx * C;
#pragma unroll
        for (int ch = 0; ch < 4; ++ch)
          if (ch < C) tt[ch] = to_f<T>(q[ch]);
      }
      sT[c] = make_float4(tt[0], tt[1], tt[2], tt[3]);
    }
    __syncthreads();
  }

  const int y0 = qy * s, y1 = min(a.H, y0 + s);
  const int x0 = qx0 * s, x1 = min(a.W, x0 + nb * s);
  const int seg = x1 - x0;  // pixels per HR row of the group
  // phase-2 ownership: thread -> (cell, offset)
  const int n_pairs_grp = nb * K2;
  float acc[2][4];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) acc[u][ch] = 0.f;

  for (int yc = y0; yc < y1; yc += a.rows_chunk) {
    const int yce = min(y1, yc + a.rows_chunk);
    const int npx = (yce - yc) * seg;
    // load the chunk: code, alpha, G; write dalpha
    for (int i = threadIdx.x; i < npx; i += kThreads) {
      const int ry = i / seg, rx = i - ry * seg;
      const int y = yc + ry, x = x0 + rx;
      const int64_t to = (int64_t)y * a.th_stride + x;
      const int cd = a.code[to];
      const float al = a.alpha[to];
      const float* g = a.G + (int64_t)y * a.G_stride + (int64_t)x * C;
      float gv[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ch = 0; ch < 4; ++ch)
        if (ch < C) gv[ch] = g[ch];
      const int cdc = min(cd, K2 * K2 - 1);
      const int oa = cdc / K2, ob = cdc - oa * K2;
      // slot in the chunk: row-major over (row, x)
      sCode[i] = oa | (ob << 8);
      sAl[i] = al;
#pragma unroll
      for (int ch = 0; ch < 4; ++ch)
        if (ch < C) sG[ch * chunk_px + i] = gv[ch];
      if (a.dalpha) {
        const int cx = x / s - qx0;  // cell within the group
        const float4 Ta = sT[(oa / k) * lx + cx + oa % k];
        const float4 Tb = sT[(ob / k) * lx + cx + ob % k];
        float da = gv[0] * (Ta.x - Tb.x);
        if (C > 1) da = fmaf(gv[1], Ta.y - Tb.y, da);
        if (C > 2) da = fmaf(gv[2], Ta.z - Tb.z, da);
        if (C > 3) da = fmaf(gv[3], Ta.w - Tb.w, da);
        a.dalpha[to] = da;
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
            const float al = sAl[i];
            if (oa == o || ob == o) {
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
  const int r = k / 2;
  auto lds = [&](int n, int rc) { return 16 * (1 + 2 * r) * (n + 2 * r) + bytes_per_px * rc * n * s; };
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
  if ((int64_t)H * W == 0) {
    return GLU_OK;
  }
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
  const int r = p->k / 2;
  const size_t lds = 16 * (size_t)(1 + 2 * r) * (a.nb + 2 * r) + (size_t)4 * (2 + C) * a.rows_chunk * a.nb * p->s;
  const int64_t groups = (int64_t)h * ceil_div(w, a.nb);
  if (groups > 0x7fffffff) return fail(GLU_ERR_UNSUPPORTED, "image too large");
  hipStream_t sm = (hipStream_t)stream;
  if (T_low->dtype == GLU_F16)
    hipLaunchKernelGGL(k_bwd_block<__half>, dim3((unsigned)groups), dim3(kThreads), lds, sm, a);
  else
    hipLaunchKernelGGL(k_bwd_block<float>, dim3((unsigned)groups), dim3(kThreads), lds, sm, a);
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
