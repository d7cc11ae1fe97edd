// Gradient-driven joint downsampling (defined by this library, not by the
// paper): the LR guide alternates with the pair search, moving along the
// gradient of the self-upsampling error and snapping back to HR pixels.
//
// Per step, with Theta = (a, b, alpha) from the search on the current L:
//   1. G = 2 (I_hat - I), I_hat = Eq. 1 applied to L itself (Sec. 3.3's
//      self-upsampling) -- k_selfgrad;
//   2. D = dL/dL of sum_p ||I_hat_p - I_p||^2 with Theta fixed: the gradient
//      of Eq. 1 with respect to its LR target (the apply backward);
//   3. every L_q becomes the HR pixel of its own block nearest to
//      L_q - eta D_q (ties: smallest HR index), so each LR pixel stays a copy
//      of one HR pixel of its block (Sec. 3.3) -- k_snap;
//   4. the search on the new L, and the sum of E in a fixed order.
// The host keeps the L with the least sum of E (one synchronisation per
// step) and returns it, or the last L, with its Theta and E.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "glu_device.h"
#include "glu_host.h"

namespace glu {

// G = 2 (alpha L[a] + (1 - alpha) L[b] - I), one thread per pixel.
__global__ __launch_bounds__(256) void k_selfgrad(const float* __restrict__ I, int64_t I_stride,
                                                  const float* __restrict__ L, int64_t L_stride,
                                                  const uint16_t* __restrict__ code, const float* __restrict__ alpha,
                                                  int64_t th_stride, float* __restrict__ G, int H, int W, int h, int w,
                                                  int s, int k) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)H * W) return;
  const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
  const int r = k / 2, K2 = k * k;
  const int cd = min((int)code[(int64_t)y * th_stride + x], K2 * K2 - 1);
  const float al = alpha[(int64_t)y * th_stride + x];
  const int oa = cd / K2, ob = cd - oa * K2;
  const int qy = y / s, qx = x / s;
  // codes from the search point inside the LR image; others read the nearest cell
  const int ay = min(max(qy + oa / k - r, 0), h - 1), ax = min(max(qx + oa % k - r, 0), w - 1);
  const int by = min(max(qy + ob / k - r, 0), h - 1), bx = min(max(qx + ob % k - r, 0), w - 1);
  const float* La = L + (int64_t)ay * L_stride + (int64_t)ax * 3;
  const float* Lb = L + (int64_t)by * L_stride + (int64_t)bx * 3;
  const float* Ip = I + (int64_t)y * I_stride + (int64_t)x * 3;
  float* g = G + i * 3;
#pragma unroll
  for (int c = 0; c < 3; ++c) g[c] = 2.0f * (fmaf(al, La[c] - Lb[c], Lb[c]) - Ip[c]);
}

// Eight lanes per LR cell, eight cells per wave: Z = L_q - eta D_q, then
// the pixel of the cell's block nearest to Z (squared distance, ties to the
// smallest HR index); L_q becomes that pixel's colour.  A cell's lanes read
// and write only its own L_q.
constexpr int kSnapLanes = 8;

__global__ __launch_bounds__(256) void k_snap(const float* __restrict__ I, int64_t I_stride, float* __restrict__ L,
                                              int64_t L_stride, const float* __restrict__ D, float eta, int H, int W,
                                              int h, int w, int s) {
  // kSnapLanes lanes per LR cell, 64 / kSnapLanes cells per wave
  const int lane = (int)threadIdx.x & 63;
  const int sub = lane % kSnapLanes;
  const int64_t q = ((int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6)) * (64 / kSnapLanes) +
                    lane / kSnapLanes;
  const bool live = q < (int64_t)h * w;
  float best = __builtin_inff();
  int arg = INT32_MAX;  // raster index inside the block
  int qy = 0, qx = 0, nbx = 1;
  if (live) {
    qy = (int)(q / w);
    qx = (int)(q - (int64_t)qy * w);
    const float* Lq = L + (int64_t)qy * L_stride + (int64_t)qx * 3;
    const float* Dq = D + q * 3;
    const float z0 = fmaf(-eta, Dq[0], Lq[0]), z1 = fmaf(-eta, Dq[1], Lq[1]), z2 = fmaf(-eta, Dq[2], Lq[2]);
    const int y0 = qy * s, x0 = qx * s;
    const int nby = min(H, y0 + s) - y0;
    nbx = min(W, x0 + s) - x0;
    const int n = nby * nbx;
    // each lane visits its pixels in raster order of the block, keeping the first minimum
    for (int j = sub; j < n; j += kSnapLanes) {
      const int by = j / nbx, bx = j - by * nbx;
      const float* p = I + (int64_t)(y0 + by) * I_stride + (int64_t)(x0 + bx) * 3;
      const float d0 = p[0] - z0, d1 = p[1] - z1, d2 = p[2] - z2;
      const float dd = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
      if (dd < best) {
        best = dd;
        arg = j;
      }
    }
  }
  // lexicographic (distance, raster index) minimum over the cell's lanes, in
  // a fixed order; the raster index inside the block orders the pixels as
  // their HR indices do
#pragma unroll
  for (int m = kSnapLanes / 2; m >= 1; m >>= 1) {
    const float ob = __shfl_xor(best, m, 64);
    const int oa = __shfl_xor(arg, m, 64);
    if (ob < best || (ob == best && oa < arg)) {
      best = ob;
      arg = oa;
    }
  }
  if (live && sub == 0) {
    const int py = qy * s + arg / nbx, px = qx * s + arg % nbx;
    const float* p = I + (int64_t)py * I_stride + (int64_t)px * 3;
    float* Lq = L + (int64_t)qy * L_stride + (int64_t)qx * 3;
    Lq[0] = p[0];
    Lq[1] = p[1];
    Lq[2] = p[2];
  }
}

// Sum of E over the image in a fixed order: kernel 1 sums rows
// [blockIdx.x * rows, ...) per workgroup (per-thread strided partial sums in
// double, then a fixed tree in LDS); kernel 2 sums the partials in order.
// One row per workgroup keeps a few thousand workgroups in flight.
constexpr int kSumRows = 1;

__global__ __launch_bounds__(256) void k_esum_part(const float* __restrict__ E, int64_t stride, int H, int W,
                                                   double* __restrict__ part) {
  __shared__ double red[256];
  const int y0 = blockIdx.x * kSumRows, y1 = min(H, y0 + kSumRows);
  double acc = 0.0;
  for (int y = y0; y < y1; ++y)
    for (int x = (int)threadIdx.x; x < W; x += 256) acc += (double)E[(int64_t)y * stride + x];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int m = 128; m >= 1; m >>= 1) {
    if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_esum_final(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = (int)threadIdx.x; i < n; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int m = 128; m >= 1; m >>= 1) {
    if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// Best-step bookkeeping on the device, so that the steps need no host
// synchronisation: *best is the step of least error sum so far (the first
// on ties); step t's sum is sums[t].
__global__ void k_best_step(const double* __restrict__ sums, int t, int* __restrict__ best) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (t == 0 || sums[t] < sums[*best]) *best = t;
  }
}

// Copies the h x w x 3 LR image src into dst when step t is the best so far.
__global__ __launch_bounds__(256) void k_copy_lr_if_best(const int* __restrict__ best, int t, float* __restrict__ dst,
                                                         int64_t dst_stride, const float* __restrict__ src,
                                                         int64_t src_stride, int h, int w) {
  if (*best != t) return;
  const int64_t n = (int64_t)h * w * 3;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int64_t row = i / ((int64_t)w * 3), col = i - row * w * 3;
    dst[row * dst_stride + col] = src[row * src_stride + col];
  }
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

constexpr int kMaxSteps = 64;

static thread_local PinnedBuf tl_sum_pin;

// Workspace layout (256-byte aligned pieces).
struct JdgLayout {
  size_t G, S, D, Lbest, E, part, sum, total;
};

static JdgLayout jdg_layout(int H, int W, const glu_params* p) {
  const int64_t h = ceil_div(H, p->s), w = ceil_div(W, p->s);
  JdgLayout l{};
  size_t off = 0;
  l.G = off;
  off += align256((size_t)H * W * 3 * sizeof(float));
  l.S = off;
  off += align256(glu_apply_backward_workspace(H, W, 3, p));
  l.D = off;
  off += align256((size_t)h * w * 3 * sizeof(float));
  l.Lbest = off;
  off += align256((size_t)h * w * 3 * sizeof(float));
  l.E = off;
  off += align256((size_t)H * W * sizeof(float));
  l.part = off;
  off += align256((size_t)ceil_div(std::max(H, 1), kSumRows) * sizeof(double));
  l.sum = off;  // the error sums of steps 0 .. kMaxSteps, then the best step (int)
  off += align256((kMaxSteps + 1) * sizeof(double) + sizeof(int));
  l.total = off;
  return l;
}

}  // namespace glu

using namespace glu;

extern "C" {

size_t glu_joint_downsample_grad_workspace(int32_t H, int32_t W, const glu_params* p) {
  if (!p || p->s < 1 || p->k < 1 || H < 0 || W < 0) return 0;
  return jdg_layout(H, W, p).total;
}

glu_status glu_joint_downsample_grad(const glu_image* I, glu_image* I_low, const glu_params* p, float eta,
                                     int32_t n_steps, int32_t keep_best, glu_theta* theta, float* err,
                                     void* workspace, size_t ws_bytes, double* err_sums, int32_t* best_step,
                                     void* stream) {
  clear_error();
  glu_status st;
  if ((st = check_params(p))) return st;
  if (p->flags) return fail(GLU_ERR_UNSUPPORTED, "joint downsampling takes no flags");
  if ((st = check_image(I, "I", 3, 3, false))) return st;
  if ((st = check_image(I_low, "I_low", 3, 3, false))) return st;
  const int H = I->height, W = I->width;
  const int h = ceil_div(H, p->s), w = ceil_div(W, p->s);
  if (I_low->height != h || I_low->width != w) return fail(GLU_ERR_SHAPE, "I_low must be ceil(H/s) x ceil(W/s)");
  if ((st = check_theta(theta, H, W, true))) return st;
  if (!(eta >= 0.0f) || !std::isfinite(eta)) return fail(GLU_ERR_PARAM, "eta must be finite and >= 0");
  if (n_steps < 0 || n_steps > kMaxSteps) return fail(GLU_ERR_PARAM, "n_steps = %d outside 0..%d", n_steps, kMaxSteps);
  if (err && reinterpret_cast<uintptr_t>(err) % 4) return fail(GLU_ERR_ALIGN, "err not aligned");
  if (!err && theta->row_stride != W && (int64_t)H * W > 0)
    return fail(GLU_ERR_SHAPE, "theta must be dense (row_stride == W) when err is NULL");
  const JdgLayout lay = jdg_layout(H, W, p);
  if ((int64_t)H * W > 0 && (!workspace || ws_bytes < lay.total))
    return fail(GLU_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", lay.total, ws_bytes);
  if (workspace && reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(GLU_ERR_ALIGN, "workspace must be 256-byte aligned");
  if ((int64_t)H * W == 0) {
    if (err_sums)
      for (int t = 0; t <= n_steps; ++t) err_sums[t] = 0.0;
    if (best_step) *best_step = 0;
    return GLU_OK;
  }
  hipStream_t sm = (hipStream_t)stream;
  char* ws = static_cast<char*>(workspace);
  float* G = reinterpret_cast<float*>(ws + lay.G);
  float* D = reinterpret_cast<float*>(ws + lay.D);
  float* Lbest = reinterpret_cast<float*>(ws + lay.Lbest);
  float* E = err ? err : reinterpret_cast<float*>(ws + lay.E);
  double* part = reinterpret_cast<double*>(ws + lay.part);
  double* dsum = reinterpret_cast<double*>(ws + lay.sum);
  const int nparts = ceil_div(H, kSumRows);
  float* L = static_cast<float*>(I_low->data);
  const int64_t Ls = I_low->row_stride;
  const size_t Lrow_bytes = (size_t)w * 3 * sizeof(float);

  glu_image Gimg{G, H, W, 3, (int64_t)W * 3, GLU_F32};
  glu_image Dimg{D, h, w, 3, (int64_t)w * 3, GLU_F32};

  auto search = [&]() -> glu_status { return glu_search(I, I_low, p, theta, E, stream); };
  int* best_dev = reinterpret_cast<int*>(dsum + kMaxSteps + 1);
  // step t's error sum into dsum[t], then the best-step update (and, with
  // keep_best, the copy of the LR guide when step t is the best so far)
  auto esum = [&](int t) -> glu_status {
    hipLaunchKernelGGL(k_esum_part, dim3((unsigned)nparts), dim3(256), 0, sm, E, theta->row_stride, H, W, part);
    hipLaunchKernelGGL(k_esum_final, dim3(1), dim3(256), 0, sm, part, nparts, dsum + t);
    hipLaunchKernelGGL(k_best_step, dim3(1), dim3(64), 0, sm, dsum, t, best_dev);
    if (keep_best) {
      const int64_t n3 = (int64_t)h * w * 3;
      const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (n3 + 255) / 256));
      hipLaunchKernelGGL(k_copy_lr_if_best, dim3(grid), dim3(256), 0, sm, best_dev, t, Lbest, (int64_t)w * 3, L, Ls,
                         h, w);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "error sum");
    return GLU_OK;
  };
  auto copy_L = [&](float* dst, int64_t dst_stride, const float* src, int64_t src_stride) -> glu_status {
    hipError_t e = hipMemcpy2DAsync(dst, (size_t)dst_stride * sizeof(float), src, (size_t)src_stride * sizeof(float),
                                    Lrow_bytes, (size_t)h, hipMemcpyDeviceToDevice, sm);
    if (e != hipSuccess) return hip_fail(e, "I_low copy");
    return GLU_OK;
  };

  if ((st = search())) return st;
  if ((st = esum(0))) return st;
  bool fused_grad = true;
  for (int t = 1; t <= n_steps; ++t) {
    // the backward forms the self-upsampling gradient itself where it can
    // (register form); otherwise G is written first
    if (fused_grad) {
      st = apply_backward_selfgrad(theta, I_low, p, I, &Dimg, ws + lay.S, ws_bytes - lay.S, stream);
      if (st == GLU_ERR_UNSUPPORTED) {
        clear_error();
        fused_grad = false;
      } else if (st) {
        return st;
      }
    }
    if (!fused_grad) {
      const int64_t npx = (int64_t)H * W;
      hipLaunchKernelGGL(k_selfgrad, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, sm,
                         static_cast<const float*>(I->data), I->row_stride, static_cast<const float*>(I_low->data), Ls,
                         theta->code, theta->alpha, theta->row_stride, G, H, W, h, w, p->s, p->k);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "self-gradient launch");
      if ((st = glu_apply_backward(theta, I_low, p, &Gimg, &Dimg, nullptr, ws + lay.S, ws_bytes - lay.S, stream)))
        return st;
    }
    hipError_t e;
    const int64_t cells = (int64_t)h * w;
    hipLaunchKernelGGL(k_snap, dim3((unsigned)((cells + 4 * (64 / kSnapLanes) - 1) / (4 * (64 / kSnapLanes)))), dim3(256), 0, sm,
                       static_cast<const float*>(I->data), I->row_stride, L, Ls, D, eta, H, W, h, w, p->s);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "snap launch");
    if ((st = search())) return st;
    if ((st = esum(t))) return st;
  }
  // one synchronisation: the sums and the best step
  {
    PinnedBuf& pb = tl_sum_pin;
    const size_t bytes = (kMaxSteps + 1) * sizeof(double) + sizeof(int);
    hipError_t e = pb.reserve(bytes);
    if (e == hipSuccess) e = hipMemcpyAsync(pb.p, dsum, bytes, hipMemcpyDeviceToHost, sm);
    if (e == hipSuccess) e = hipStreamSynchronize(sm);
    if (e != hipSuccess) return hip_fail(e, "error sums");
  }
  const double* sums_h = tl_sum_pin.as<double>();
  const int best_t = keep_best ? *reinterpret_cast<const int*>(sums_h + kMaxSteps + 1) : n_steps;
  if (err_sums)
    for (int t = 0; t <= n_steps; ++t) err_sums[t] = sums_h[t];
  if (keep_best && best_t != n_steps) {
    if ((st = copy_L(L, Ls, Lbest, (int64_t)w * 3))) return st;
    if ((st = search())) return st;
  }
  if (best_step) *best_step = best_t;
  hipError_t e = hipStreamSynchronize(sm);
  if (e != hipSuccess) return hip_fail(e, "gradient joint downsampling");
  return GLU_OK;
}

}  // extern "C"
