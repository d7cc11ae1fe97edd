// Internal definitions shared by the host and device code of libglu.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <type_traits>

#include "glu.h"

namespace glu {

constexpr int kThreads = 256;       // threads per workgroup (4 wave64)
constexpr int kMaxK = 15;           // largest window (code fits uint16)
constexpr int kLdsBudget = 60 * 1024;  // dynamic LDS per workgroup we allow
constexpr int kApplyStrips = 4;     // strips per thread and pass in the apply kernel

// Alignment flags of one launch (all pixels of a launch share them).
enum : uint32_t {
  VEC_I = 1u << 0,      // HR guide rows allow 16/8-byte vector loads
  VEC_THETA = 1u << 1,  // theta / err rows allow vector stores
  VEC_T = 1u << 2,      // T_hat rows allow vector stores (C == 1 or 3)
  VEC_G = 1u << 3,      // gradient rows allow vector loads
  VEC_TW = 1u << 4,     // T_hat base and rows 16-byte aligned (apply stores a
                        // wave's 64 strips as one run of 16-byte words)
};

// One image of a search / apply launch.  The plain entry points launch one
// of these; the batch kernel looks its tile's image up in a table of them.
struct ImgDesc {
  const void* I;        // HR guide (3 channels)
  const void* L;        // LR guide (3 channels)
  const void* T;        // LR target (C channels), fused / apply
  void* That;           // HR output (C channels)
  uint16_t* code;       // Theta codes (nullable in fused mode)
  float* alpha;         // Theta weights (nullable in fused mode)
  float* err;           // E (nullable)
  int64_t I_stride, L_stride, T_stride, That_stride, th_stride;  // elements
  int32_t H, W, h, w, s, k, C;
  int32_t tqy, tqx;     // tile in LR centres
  int32_t tiles_x, tiles_y;
  uint32_t vec;         // VEC_* flags
  int32_t dtype;        // glu_dtype of I, L, T, That
  int32_t variant;      // kernel variant index (batched dispatch)
  int32_t gnu;          // fast-mode kernels: stop after the anchor (GNU)
  int32_t no_degen;     // exhaustive: pairs i < j only (GLU_FLAG_NO_DEGENERATE)
  int64_t tile_begin;   // first global tile index of this image (batched)
};

// Colexicographic index of the unordered pair (i, j), i < j.
__host__ __device__ constexpr int pair_index(int i, int j) { return j * (j - 1) / 2 + i; }
__host__ __device__ constexpr int n_pairs(int K2) { return K2 * (K2 - 1) / 2; }

// LDS words (float4) used by one tile of the search.
inline int search_lds_cells(int tqy, int tqx, int k) {
  const int r = k / 2;
  return (tqy + 2 * r) * (tqx + 2 * r);
}

}  // namespace glu
