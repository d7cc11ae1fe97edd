// Host-side helpers of libglu: error reporting, argument validation and the
// tile-shape choice shared by every entry point.
#pragma once

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "glu_internal.h"

namespace glu {

// Records a failure for glu_last_error() and returns the status.
glu_status fail(glu_status st, const char* fmt, ...);
// Clears the calling thread's last error.
void clear_error();

// Maps a HIP error to GLU_ERR_HIP with context.
glu_status hip_fail(hipError_t e, const char* what);

// Page-locked host staging (hipHostMalloc) for small copies between the
// iterations of the joint downsampling calls: copies to or from pageable
// memory are staged by the runtime and stall the host.  Callers keep one
// buffer per thread and purpose (thread_local), grown on demand and kept
// until the process ends; every use ends with a stream synchronisation
// before the buffer is touched again.
struct PinnedBuf {
  void* p = nullptr;
  size_t cap = 0;
  hipError_t reserve(size_t bytes) {
    if (bytes <= cap) return hipSuccess;
    if (p) {
      hipHostFree(p);
      p = nullptr;
      cap = 0;
    }
    const size_t c = std::max<size_t>(bytes, 4096);
    hipError_t e = hipHostMalloc(&p, c, hipHostMallocDefault);
    if (e == hipSuccess) cap = c;
    return e;
  }
  template <typename V>
  V* as() const {
    return static_cast<V*>(p);
  }
};
// The backward of Eq. 1 with T_low = I_low for the self-upsampling loss
// sum_p ||I_hat_p - I_p||^2: grad_I_low of that loss with Theta fixed, with
// the per-pixel gradient 2 (I_hat - I) formed inside the backward's first
// pass.  GLU_ERR_UNSUPPORTED for shapes outside its register form; the
// caller then forms the gradient image itself.
glu_status apply_backward_selfgrad(const glu_theta* theta, const glu_image* I_low, const glu_params* p,
                                   const glu_image* I, glu_image* grad_I_low, void* workspace, size_t ws_bytes,
                                   void* stream);

inline size_t dtype_size(glu_dtype t) { return t == GLU_F16 ? 2 : 4; }
inline bool dtype_ok(int t) { return t == GLU_F32 || t == GLU_F16; }

// Validation of one image descriptor: non-NULL (unless empty), channel
// count, stride, dtype and element alignment.
glu_status check_image(const glu_image* im, const char* name, int channels_lo, int channels_hi,
                       bool allow_f16 = true);
glu_status check_params(const glu_params* p);
glu_status check_theta(const glu_theta* th, int H, int W, bool need_buffers);

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Tile shape of a search / apply launch.
struct TileChoice {
  int P;    // pixels per strip (4 when 4 divides s, else 1)
  int tqy;  // tile height in LR centres
  int tqx;  // tile width in LR centres
};

// Pixels per search strip: consecutive pixels of one HR row that share a
// centre, so P divides s (4, else 3, else 2, else 1).
inline int strip_pixels(int s) { return s % 4 == 0 ? 4 : (s % 3 == 0 ? 3 : (s % 2 == 0 ? 2 : 1)); }

// Pixels per strip of a search launch: the exhaustive 5 x 5 search builds
// the constants of its 300 pairs per strip, so it shares them over 8 pixels
// when 8 divides s (strips of 8 did not pay for 7 x 7 windows, whose
// runtime-k kernel loses more to register pressure).
inline int search_strip_pixels(int s, int k, bool exhaustive) {
  return (exhaustive && k == 5 && s % 8 == 0) ? 8 : strip_pixels(s);
}

// Default tile: about 64 HR columns by enough rows for 256 strips, shrunk
// until the LDS of the tile fits.  `variant` selects alternatives for the
// autotuner (0 = default).
// P_override > 0 replaces the default strip width (it must divide s).
TileChoice choose_tile(int s, int k, int mode, bool fused, bool table, int variant, int P_override = 0);
int n_tile_variants();

// Fills the image descriptor fields common to search / apply launches.
void fill_tiles(ImgDesc& d, const TileChoice& tc);

// Kernel variant index used by the batched dispatcher.
int kernel_variant(int k, int P, int mode, int dtype, bool table);

// VEC_* alignment flags of a launch (vector loads / stores allowed).
uint32_t launch_vec_flags(const ImgDesc& d, int P, size_t esize);

// Batch of n images of one size (glu_*_batched): n and stride checks.
glu_status check_batch(int32_t n, const glu_batch_strides* bs, bool backward);

// Apply tile width in LR columns (see apply_tile).
int apply_tile_width(int s, int P, int k, int C, int esize);

// Tile variant recorded by the autotuner for (mode, k, s, dtype), 0 if none.
int tuned_variant(int mode, int k, int s, int dtype);

}  // namespace glu
