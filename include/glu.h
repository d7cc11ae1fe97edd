/*
 * glu.h - C ABI of the guided linear upsampling (GLU) library for AMD MI355X
 * (gfx950).
 *
 * Method: S. Song, F. Zhong, T. Wang, X. Qin, C. Tu, "Guided Linear
 * Upsampling", ACM Transactions on Graphics 42(4), 2023.
 *
 * Every high-resolution (HR) pixel p is represented as the interpolation of
 * two low-resolution (LR) pixels a, b taken from a k x k window around its LR
 * location (Sec. 3.1, Eq. 1):
 *
 *     T_hat_p = alpha T_low[a] + (1 - alpha) T_low[b]
 *
 * Theta = (a, b, alpha) is solved on the guide alone (Eq. 2-4, Algorithm 1)
 * and then transferred to any LR operator output T_low = f(I_low).  The LR
 * guide I_low can itself be optimised jointly (Sec. 3.3, Algorithm 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Buffers are DEVICE pointers owned by the caller unless a comment says
 *    HOST.  The library never frees a caller buffer.
 *  - Images are HWC interleaved ("glu_image"): element (y, x, c) sits at
 *    data[y * row_stride + x * channels + c]; row_stride is in elements and
 *    must be >= width * channels.
 *  - HR pixel p = (y, x); its LR cell is p_down = (y / s, x / s) (integer
 *    division).  The LR guide must be ceil(H/s) x ceil(W/s) (every HR pixel
 *    has a cell).  The window is the k x k block of LR cells centred on
 *    p_down, truncated at the LR border (no clamped duplicates).
 *  - Theta is stored compactly ("glu_theta", 6 bytes per pixel):
 *      code  (uint16) = o_a * k*k + o_b, where o = (dy + r) * k + (dx + r) is
 *                       the offset of a cell in the untruncated window,
 *                       r = (k - 1) / 2, (dy, dx) = cell - p_down;
 *      alpha (float)  = the weight on a.
 *    code(y, x) is code[y * row_stride + x], the same for alpha.
 *    Exhaustive mode returns o_a <= o_b (a is the lower LR index) and
 *    alpha = 1 when o_a == o_b; fast mode returns a = the anchor (the window
 *    cell of most similar colour, Algorithm 1).
 *  - Every call is asynchronous on `stream` (a hipStream_t passed as void*;
 *    NULL is the default stream) unless its comment says it synchronises.
 *  - Arguments are validated before anything is enqueued.  On an error
 *    nothing runs, outputs are untouched, and glu_last_error() gives the
 *    reason.  Faults of enqueued work surface at the caller's next
 *    synchronisation.  No C++ exception crosses this ABI.
 *  - Identical inputs give bitwise identical outputs (no floating-point
 *    atomics anywhere).
 *  - Calls are re-entrant; calls that share output buffers must not
 *    overlap.
 */
#ifndef GLU_H
#define GLU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GLU_OK = 0,
  GLU_ERR_NULL = 1,        /* a required pointer is NULL                        */
  GLU_ERR_SHAPE = 2,       /* sizes or channel counts do not fit together      */
  GLU_ERR_DTYPE = 3,       /* unsupported or mismatched element type           */
  GLU_ERR_PARAM = 4,       /* s, k, eps, tau, max_iter or mode out of range    */
  GLU_ERR_ALIGN = 5,       /* a pointer is not aligned to its element size     */
  GLU_ERR_NOMEM = 6,       /* host or device allocation failed                 */
  GLU_ERR_HIP = 7,         /* a HIP runtime call or kernel launch failed       */
  GLU_ERR_UNSUPPORTED = 8, /* valid request the library does not implement     */
  GLU_ERR_WORKSPACE = 9    /* workspace missing or smaller than required       */
} glu_status;

typedef enum { GLU_F32 = 0, GLU_F16 = 1 } glu_dtype;

/* GLU_SEARCH_EXHAUSTIVE: every pair of the window with the projection weight
 * of Eq. 4 clamped to [0, 1] (Sec. 3.1); GLU_SEARCH_FAST: Algorithm 1 with
 * the weight of Eq. 5 (Sec. 3.2); GLU_SEARCH_GNU: guided nearest-neighbour
 * upsampling, the weight-1 special case of Sec. 3.2 (a = b = the window cell
 * of nearest colour, first in LR index on ties; E = that distance). */
typedef enum { GLU_SEARCH_EXHAUSTIVE = 0, GLU_SEARCH_FAST = 1, GLU_SEARCH_GNU = 2 } glu_mode;

/* glu_params.flags.  GLU_FLAG_NO_DEGENERATE (exhaustive mode only): the
 * candidates are the unordered pairs i < j of the window alone (36 for 3 x 3,
 * Sec. 3.2), without the single-cell candidates (i, i) with weight 1 that the
 * default search adds; a window with a single cell (k = 1, or a 1 x 1 LR
 * image) falls back to that cell.  With eps > 0 a pixel equal to a window
 * colour then keeps a small error, since Eq. 4's weight never reaches 1.
 * Taken by glu_search, glu_search_apply and batch plans; the joint
 * downsampling calls return GLU_ERR_UNSUPPORTED for it, and the fast and GNU
 * modes GLU_ERR_PARAM. */
enum { GLU_FLAG_NO_DEGENERATE = 1u };

/* Regular-grid downsampling keeps one HR pixel per LR pixel (Sec. 3.1,
 * Sec. 3.3); BOX averages the in-image pixels of each s x s block. */
typedef enum { GLU_DOWN_POINT = 0, GLU_DOWN_BOX = 1 } glu_down_mode;

typedef struct {
  void* data;          /* device pointer, HWC interleaved              */
  int32_t height;
  int32_t width;
  int32_t channels;
  int64_t row_stride;  /* elements between consecutive rows            */
  glu_dtype dtype;
} glu_image;

typedef struct {
  uint16_t* code;      /* device, height rows of row_stride entries     */
  float* alpha;        /* device, same layout as code                   */
  int32_t height;
  int32_t width;
  int64_t row_stride;  /* elements between consecutive rows             */
} glu_theta;

typedef struct {
  int32_t s;           /* integer downsampling ratio, >= 1              */
  int32_t k;           /* odd window size, 1 <= k <= 15 (paper: 3)      */
  float eps;           /* Eq. 4 / Eq. 5 regulariser, >= 0 (paper: 1e-3) */
  glu_mode mode;
  uint32_t flags;      /* GLU_FLAG_* bits, 0 for the paper's search      */
} glu_params;

/* Per-round statistics of glu_joint_downsample (HOST struct). */
typedef struct {
  int32_t rounds_run;
  int32_t n_large[64];       /* |{p : E_p > tau}| at the start of each round */
  int32_t n_components[64];  /* 8-connected components of that set           */
  int32_t n_accepted[64];    /* trials kept (e1 <= e0)                       */
  int32_t n_waves[64];       /* conflict-free launch waves used              */
  double err_sum_initial;    /* sum_p E_p after the initial search           */
  double err_sum_final;      /* sum_p E_p at return                          */
} glu_jd_stats;

/* Decision log of glu_joint_downsample (HOST arrays allocated by the caller).
 * One entry per trial, in the order the sequential algorithm takes them:
 * round, first pixel of the component (raster order), accept flag, e0, e1,
 * number of replaced LR cells n_q, and n_q pairs (q, p_star) appended to
 * q_and_pstar.  count is set to the number of entries written; if capacity
 * or q_capacity is too small the log is truncated and `truncated` is set. */
typedef struct {
  int32_t capacity;
  int32_t count;
  int32_t* round;
  int32_t* first_pixel;
  uint8_t* accepted;
  double* e0;
  double* e1;
  int32_t* n_q;
  int64_t q_capacity;        /* capacity of q_and_pstar in pairs             */
  int64_t* q_and_pstar;      /* 2 * sum(n_q) entries: q, p_star, q, ...     */
  int32_t truncated;
} glu_jd_log;

/* ---------------------------------------------------------------------------
 * glu_search - per-pixel parameter search (Sec. 3.1 Eq. 3 with Eq. 4, or
 * Sec. 3.2 Algorithm 1 with Eq. 5).
 *
 *   I      HR guide, H x W x 3, GLU_F32 or GLU_F16.
 *   I_low  LR guide, ceil(H/s) x ceil(W/s) x 3, same dtype as I.
 *   p      s, k, eps, mode.
 *   theta  output, H x W (code, alpha).
 *   err    nullable output, E_p = ||I_p - I_hat_p|| (Euclidean, not squared,
 *          Sec. 3.3) as float, laid out like theta (theta->row_stride).
 *
 * Exhaustive mode visits the candidates of the window in colexicographic
 * order of (i, j), i <= j in LR index, and keeps the first of least error;
 * the degenerate pairs (i, i) carry alpha = 1.
 * ------------------------------------------------------------------------- */
glu_status glu_search(const glu_image* I, const glu_image* I_low, const glu_params* p,
                      glu_theta* theta, float* err, void* stream);

/* ---------------------------------------------------------------------------
 * glu_apply - Eq. 1: T_hat_p = alpha_p T_low[a_p] + (1 - alpha_p) T_low[b_p].
 *
 *   theta  H x W, as written by glu_search (s, k in p must match).
 *   T_low  ceil(H/s) x ceil(W/s) x C, 1 <= C <= 4, GLU_F32 or GLU_F16.
 *   T_hat  output, H x W x C, same dtype as T_low.
 * Codes that glu_search never writes have one defined meaning, shared with
 * glu_apply_backward: a code above k^4 - 1 counts as k^4 - 1, and a window
 * position outside the LR image reads the nearest in-image cell (its row
 * and column clamped to the image).
 * ------------------------------------------------------------------------- */
glu_status glu_apply(const glu_theta* theta, const glu_image* T_low, const glu_params* p,
                     glu_image* T_hat, void* stream);

/* ---------------------------------------------------------------------------
 * Batches of n images of one size (H, W, C, dtype, s, k shared) in one
 * launch: image b of each buffer starts at the descriptor's pointer plus b
 * times the buffer's batch stride, in elements of that buffer.  Row strides
 * are the descriptors'.  Output images of a batch must not overlap.
 * ------------------------------------------------------------------------- */
typedef struct {
  int64_t theta;       /* code and alpha planes                              */
  int64_t T_low;
  int64_t T_hat;       /* T_hat (glu_apply_batched) or grad_T_hat (backward) */
  int64_t grad_T_low;
  int64_t grad_alpha;
} glu_batch_strides;

/* glu_apply over n images in one launch (n in 0..65535; strides may be
 * NULL when n <= 1).  Results are bitwise those of n glu_apply calls. */
glu_status glu_apply_batched(int32_t n, const glu_batch_strides* strides, const glu_theta* theta,
                             const glu_image* T_low, const glu_params* p, glu_image* T_hat, void* stream);

/* ---------------------------------------------------------------------------
 * glu_search_apply - glu_search followed by glu_apply in one pass over the
 * HR image (Algorithm 1 computes T_hat_p right after Theta_p).
 *
 *   theta  nullable: when NULL Theta is not stored.
 *   err    nullable, as in glu_search (needs theta for its row stride; when
 *          theta is NULL the stride is W).
 * Results are bitwise identical to the two separate calls.
 * ------------------------------------------------------------------------- */
glu_status glu_search_apply(const glu_image* I, const glu_image* I_low, const glu_image* T_low,
                            const glu_params* p, glu_theta* theta, float* err, glu_image* T_hat,
                            void* stream);

/* ---------------------------------------------------------------------------
 * glu_apply_backward - gradients of Eq. 1 (Sec. 3.1) with the indices (a, b)
 * held fixed (the indices are piecewise constant in the inputs):
 *
 *   grad_alpha_p = sum_c G_p,c (T_low[a_p],c - T_low[b_p],c)
 *   grad_T_low_q = sum_{p: a_p = q} alpha_p G_p + sum_{p: b_p = q} (1 - alpha_p) G_p
 *
 *   theta       H x W, as written by glu_search (s, k in p must match).
 *   T_low       ceil(H/s) x ceil(W/s) x C, 1 <= C <= 4, GLU_F32 or GLU_F16.
 *   grad_T_hat  G, H x W x C, GLU_F32.
 *   grad_T_low  nullable output, ceil(H/s) x ceil(W/s) x C, GLU_F32 (written,
 *               not accumulated).
 *   grad_alpha  nullable output, float, theta layout.
 *   workspace   device scratch of glu_apply_backward_workspace() bytes,
 *               needed only when grad_T_low is requested (contents on entry
 *               ignored; caller-owned).
 * grad_T_low is a gather over the inverted index map: each LR cell sums the
 * contributions of the HR pixels whose window can reach it in a fixed order
 * (per source block, then per window offset), without atomics, so the
 * result is bitwise reproducible.  Codes glu_search never writes follow
 * glu_apply's rule: the gradient of a window position outside the LR image
 * goes to the clamped cell the apply reads, so the result is the gradient
 * of what glu_apply computes.
 * ------------------------------------------------------------------------- */
size_t glu_apply_backward_workspace(int32_t H, int32_t W, int32_t C, const glu_params* p);
glu_status glu_apply_backward(const glu_theta* theta, const glu_image* T_low, const glu_params* p,
                              const glu_image* grad_T_hat, glu_image* grad_T_low,
                              float* grad_alpha, void* workspace, size_t ws_bytes, void* stream);

/* glu_apply_backward over n images of one size in one launch per pass
 * (strides as for glu_apply_batched, with strides->T_hat the batch stride of
 * grad_T_hat; may be NULL when n <= 1).  The workspace holds one image's
 * workspace per image.  Results are bitwise those of n separate calls. */
size_t glu_apply_backward_batched_workspace(int32_t n, int32_t H, int32_t W, int32_t C, const glu_params* p);
glu_status glu_apply_backward_batched(int32_t n, const glu_batch_strides* strides, const glu_theta* theta,
                                      const glu_image* T_low, const glu_params* p,
                                      const glu_image* grad_T_hat, glu_image* grad_T_low,
                                      float* grad_alpha, void* workspace, size_t ws_bytes, void* stream);

/* glu_apply_backward_static - glu_apply_backward without a workspace
 * argument and without any allocation, for callers that cannot allocate
 * device memory (code under hipGraph capture, tight serving loops, hosts
 * that forbid it).  The workspace is a library-owned device array of
 * GLU_STATIC_SCRATCH_BYTES on each GPU the library runs on (held until the
 * process ends); its address is looked up once per device, on the first
 * call with that device current.  Arguments, layouts, results (bitwise)
 * and errors are those of glu_apply_backward on the current device, plus
 * GLU_ERR_WORKSPACE when glu_apply_backward_workspace() of the call exceeds
 * GLU_STATIC_SCRATCH_BYTES (e.g. 3840 x 2160 at s = 8, k = 3, C = 3 needs
 * 14.0 MiB).  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (two streams, two threads) race and must be ordered
 * by the caller.  Nothing in the array needs clearing between calls. */
#define GLU_STATIC_SCRATCH_BYTES ((size_t)16 << 20)
glu_status glu_apply_backward_static(const glu_theta* theta, const glu_image* T_low, const glu_params* p,
                                     const glu_image* grad_T_hat, glu_image* grad_T_low, float* grad_alpha,
                                     void* stream);

/* ---------------------------------------------------------------------------
 * glu_downsample - initial LR guide (not on the timed path).
 *   POINT: I_low[q] = I[min(qy s + s/2, H-1), min(qx s + s/2, W-1)] (a copy
 *          of one HR pixel per LR pixel, Sec. 3.3).
 *   BOX:   mean of the in-image pixels of the s x s block.
 * I_low must be ceil(H/s) x ceil(W/s) with I's channels and dtype.
 * ------------------------------------------------------------------------- */
glu_status glu_downsample(const glu_image* I, glu_image* I_low, int32_t s, glu_down_mode mode,
                          void* stream);

/* ---------------------------------------------------------------------------
 * glu_theta_expand - the paper's 3 x H x W form of Theta (Sec. 5.4): absolute
 * LR linear indices a, b (int64, qy * w + qx) decoded from the codes.
 * a, b are device arrays of H * W entries, row-major, dense.
 * ------------------------------------------------------------------------- */
glu_status glu_theta_expand(const glu_theta* theta, const glu_params* p, int64_t* a, int64_t* b,
                            void* stream);

/* ---------------------------------------------------------------------------
 * glu_joint_downsample - Algorithm 2 (Sec. 3.3): alternate the search with
 * trial replacements of I_low by large-error HR pixels, keeping a trial only
 * when the summed error does not increase.
 *
 *   I          HR guide, H x W x 3, GLU_F32.
 *   I_low      in: initial LR guide (regular grid by default); out: optimised.
 *   p          search parameters (mode used for every search).
 *   tau        error threshold (paper: 30/255), >= 0.
 *   max_iter   N, 0..64 (paper: 3).
 *   theta, err outputs: the search of I against the final I_low.
 *   workspace  device buffer of at least glu_joint_downsample_workspace()
 *              bytes (caller-owned, contents on entry ignored).
 *   stats, log nullable HOST outputs.
 * Reading of Algorithm 2: components are 8-connected and taken in the raster
 * order of their first pixel, one after another; each trial re-searches and
 * sums over the affected set A = {p : window(p) contains a replaced cell};
 * rollback when e1 > e0.  Components whose affected sets cannot interact are
 * run side by side, which gives the sequential result exactly.
 * Synchronises `stream` a few times per round (component counts and the
 * component table are read on the host to schedule the trials).
 * ------------------------------------------------------------------------- */
size_t glu_joint_downsample_workspace(int32_t H, int32_t W, const glu_params* p);
glu_status glu_joint_downsample(const glu_image* I, glu_image* I_low, const glu_params* p,
                                float tau, int32_t max_iter, glu_theta* theta, float* err,
                                void* workspace, size_t ws_bytes, glu_jd_stats* stats,
                                glu_jd_log* log, void* stream);

/* ---------------------------------------------------------------------------
 * glu_joint_downsample_grad - gradient-driven joint downsampling.  Defined
 * by this library (not in the paper) as an alternative to the trial
 * replacements of Algorithm 2; it keeps Sec. 3.3's rule that every LR guide
 * pixel is a copy of one HR pixel of its own block.  From Theta, E =
 * search(I, I_low), each of n_steps steps:
 *   D   = d/dI_low of sum_p ||I_hat_p - I_p||^2, I_hat = Eq. 1 applied to
 *         I_low itself, Theta held fixed (G = 2 (I_hat - I) through the
 *         gradient of Eq. 1, as in glu_apply_backward);
 *   I_low[q] = I[p*], p* the pixel of q's s x s block nearest (squared RGB
 *         distance) to I_low[q] - eta D[q], ties to the smallest HR index;
 *   Theta, E = search(I, I_low).
 *
 *   I          H x W x 3, GLU_F32.
 *   I_low      in: initial guide, out: the result, ceil(H/s) x ceil(W/s) x 3,
 *              GLU_F32.
 *   eta        step size, finite, >= 0.
 *   n_steps    0..64.
 *   keep_best  non-zero: return the I_low of least sum of E seen (the first
 *              on equality), with its Theta and E; zero: the last one.
 *   theta      output, H x W (required).
 *   err        nullable output, E with theta's row stride; when NULL, theta
 *              must be dense (row_stride == W).
 *   workspace  device, glu_joint_downsample_grad_workspace() bytes, 256-byte
 *              aligned, caller-owned.
 *   err_sums   nullable HOST array of n_steps + 1 doubles: sum of E after 0,
 *              1, ... steps (fixed summation order).
 *   best_step  nullable HOST int: the step whose I_low is returned.
 * Synchronises the stream once per step.
 * ------------------------------------------------------------------------- */
size_t glu_joint_downsample_grad_workspace(int32_t H, int32_t W, const glu_params* p);
glu_status glu_joint_downsample_grad(const glu_image* I, glu_image* I_low, const glu_params* p, float eta,
                                     int32_t n_steps, int32_t keep_best, glu_theta* theta, float* err,
                                     void* workspace, size_t ws_bytes, double* err_sums /* HOST */,
                                     int32_t* best_step /* HOST */, void* stream);

/* ---------------------------------------------------------------------------
 * Batched execution: search + apply of many images or frames of any mix of
 * sizes, ratios s, windows k and storage types.  The items are grouped by
 * kernel variant (window 3, 5, 7 or other; pixels per strip; float32 or
 * float16; LDS table or none): each group runs as ONE launch of a kernel
 * specialised for it, with one workgroup per tile of the group's images, so
 * a batch of one variant (the frames of a video) is a single launch and a
 * mixed batch one launch per variant present, enqueued back to back on the
 * stream.
 *
 * glu_batch_plan_create validates every item (same rules as
 * glu_search_apply, with the item's own s and k; eps and mode from p),
 * picks a tile shape per item (from the autotune cache when present, see
 * glu_autotune), builds a device descriptor table and copies it once.  It
 * allocates that table and synchronises.  The plan owns its device memory.
 * glu_batch_plan_launch enqueues the plan's launches; it performs no
 * allocation, copy or memset, so it can be captured into a hipGraph.
 * Item buffers must stay valid for every launch of the plan.
 * ------------------------------------------------------------------------- */
typedef struct {
  glu_image I;
  glu_image I_low;
  glu_image T_low;
  glu_image T_hat;
  glu_theta theta;   /* theta.code == NULL: Theta not stored              */
  int32_t s;
  int32_t k;
} glu_batch_item;

typedef struct glu_batch_plan glu_batch_plan;

glu_status glu_batch_plan_create(const glu_batch_item* items /* HOST */, int32_t n,
                                 const glu_params* p, glu_batch_plan** out /* HOST */);
glu_status glu_batch_plan_launch(const glu_batch_plan* plan, void* stream);
void glu_batch_plan_destroy(glu_batch_plan* plan);
/* Number of tiles and of workgroups over all launches of a plan (HOST ints,
 * nullable). */
glu_status glu_batch_plan_info(const glu_batch_plan* plan, int64_t* n_tiles, int32_t* n_groups);

/* ---------------------------------------------------------------------------
 * glu_autotune - time the candidate tile shapes for (mode, k, s, dtype) on
 * the current device with the given item as workload, and record the
 * fastest in the process-wide cache (guarded by a mutex).  Synchronises.
 * The cache can be saved to / loaded from a JSON file.
 * ------------------------------------------------------------------------- */
glu_status glu_autotune(const glu_batch_item* item /* HOST */, const glu_params* p,
                        int32_t* chosen_tile /* HOST, nullable */, void* stream);
glu_status glu_autotune_save(const char* path);
glu_status glu_autotune_load(const char* path);

const char* glu_status_string(glu_status s);
/* Detail of the last failure on the calling thread ("" if none). */
const char* glu_last_error(void);
/* Library version string. */
const char* glu_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GLU_H */
