// Device code of the GLU hot path: per-pixel pair search (Sec. 3.1 Eq. 3-4,
// Sec. 3.2 Algorithm 1 / Eq. 5) and the apply step (Sec. 3.1 Eq. 1), written
// for gfx950 (wave64, LDS-staged LR windows, VALU fp32 arithmetic).
//
// Work decomposition.  A workgroup of 256 threads owns a tile of
// tqy x tqx LR cells ("centres") and every HR pixel whose LR cell is one of
// them (tqy*s rows by tqx*s columns).  It stages the LR cells of the tile
// plus an r-cell halo in LDS once; in exhaustive mode it also precomputes,
// per centre and per unordered window pair (i, j), the constants
// e = L_i - L_j and 1 / (|e|^2 + eps) shared by the s*s pixels of that centre.
// Each thread then takes strips of P consecutive pixels of one row, all with
// the same centre (P divides s), loads them with vector loads and runs the
// candidate loop with the pair constants read from LDS.
#pragma once

#include "glu_internal.h"

namespace glu {

// ---------------------------------------------------------------------------
// element conversion
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ float to_f(T v);
template <>
__device__ __forceinline__ float to_f<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f<__half>(__half v) { return __half2float(v); }

template <typename T>
__device__ __forceinline__ T from_f(float v);
template <>
__device__ __forceinline__ float from_f<float>(float v) { return v; }
template <>
__device__ __forceinline__ __half from_f<__half>(float v) { return __float2half_rn(v); }

__device__ __forceinline__ float clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }

// Clang vector types for the non-temporal load/store builtins.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// HR strip loads and stores (P consecutive pixels of one row)
// ---------------------------------------------------------------------------
// Loads the 3 guide channels of pixels x .. x+P-1 of `row`.  `vec` says the
// row base allows P-pixel vector loads (P = 4: 16 bytes for float, 8 bytes for
// half, x a multiple of 4); `full` that all P pixels lie inside the image.
template <typename T, int P>
__device__ __forceinline__ void load_strip3(const T* __restrict__ row, int x, int W, bool vec,
                                            bool full, float (&ip)[P][3]) {
  const T* p = row + (int64_t)x * 3;
  if constexpr (P == 4 && sizeof(T) == 4) {
    if (vec && full) {
      const float4* q = reinterpret_cast<const float4*>(p);
      float4 a = q[0], b = q[1], c = q[2];
      ip[0][0] = a.x; ip[0][1] = a.y; ip[0][2] = a.z;
      ip[1][0] = a.w; ip[1][1] = b.x; ip[1][2] = b.y;
      ip[2][0] = b.z; ip[2][1] = b.w; ip[2][2] = c.x;
      ip[3][0] = c.y; ip[3][1] = c.z; ip[3][2] = c.w;
      return;
    }
  }
  if constexpr (P == 4 && sizeof(T) == 2) {
    if (vec && full) {
      const uint2* q = reinterpret_cast<const uint2*>(p);
      uint2 u0 = q[0], u1 = q[1], u2 = q[2];
      const __half* h0 = reinterpret_cast<const __half*>(&u0);
      const __half* h1 = reinterpret_cast<const __half*>(&u1);
      const __half* h2 = reinterpret_cast<const __half*>(&u2);
      float f[12];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        f[i] = __half2float(h0[i]);
        f[4 + i] = __half2float(h1[i]);
        f[8 + i] = __half2float(h2[i]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ip[i][0] = f[3 * i];
        ip[i][1] = f[3 * i + 1];
        ip[i][2] = f[3 * i + 2];
      }
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const bool ok = full || (x + i < W);
#pragma unroll
    for (int c = 0; c < 3; ++c) ip[i][c] = ok ? to_f<T>(p[3 * i + c]) : 0.0f;
  }
}

template <int P>
__device__ __forceinline__ void store_theta(uint16_t* __restrict__ code_row, float* __restrict__ alpha_row,
                                            float* __restrict__ err_row, int x, int W, bool vec, bool full,
                                            const int (&code)[P], const float (&al)[P], const float (&e)[P]) {
  if constexpr (P == 4) {
    if (vec && full) {
      if (code_row) {
        uint2 c;
        c.x = (uint32_t)code[0] | ((uint32_t)code[1] << 16);
        c.y = (uint32_t)code[2] | ((uint32_t)code[3] << 16);
        *reinterpret_cast<uint2*>(code_row + x) = c;
        *reinterpret_cast<float4*>(alpha_row + x) = make_float4(al[0], al[1], al[2], al[3]);
      }
      if (err_row) *reinterpret_cast<float4*>(err_row + x) = make_float4(e[0], e[1], e[2], e[3]);
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < P; ++i) {
    if (full || x + i < W) {
      if (code_row) {
        code_row[x + i] = (uint16_t)code[i];
        alpha_row[x + i] = al[i];
      }
      if (err_row) err_row[x + i] = e[i];
    }
  }
}

// Stores C channels (C <= 4) of pixels x .. x+P-1.
template <typename T, int P>
__device__ __forceinline__ void store_out(T* __restrict__ row, int x, int W, int C, bool vec, bool full,
                                          const float (&o)[P][4]) {
  T* p = row + (int64_t)x * C;
  if constexpr (P == 4 && sizeof(T) == 4) {
    if (vec && full && C == 3) {
      float4* q = reinterpret_cast<float4*>(p);
      q[0] = make_float4(o[0][0], o[0][1], o[0][2], o[1][0]);
      q[1] = make_float4(o[1][1], o[1][2], o[2][0], o[2][1]);
      q[2] = make_float4(o[2][2], o[3][0], o[3][1], o[3][2]);
      return;
    }
    if (vec && full && C == 1) {
      *reinterpret_cast<float4*>(p) = make_float4(o[0][0], o[1][0], o[2][0], o[3][0]);
      return;
    }
  }
  if constexpr (P == 4 && sizeof(T) == 2) {
    if (vec && full && C == 3) {
      __half h[12];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) h[3 * i + c] = __float2half_rn(o[i][c]);
      uint2* q = reinterpret_cast<uint2*>(p);
      const uint2* hv = reinterpret_cast<const uint2*>(h);
      q[0] = hv[0];
      q[1] = hv[1];
      q[2] = hv[2];
      return;
    }
    if (vec && full && C == 1) {
      __half h[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) h[i] = __float2half_rn(o[i][0]);
      *reinterpret_cast<uint2*>(p) = *reinterpret_cast<const uint2*>(h);
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < P; ++i) {
    if (full || x + i < W) {
      for (int c = 0; c < C; ++c) p[i * C + c] = from_f<T>(o[i][c]);
    }
  }
}

// ---------------------------------------------------------------------------
// Pair constants and weights
// ---------------------------------------------------------------------------
// For the window pair (i, j): e = L_i - L_j, inv = 1 / (|e|^2 + eps) and the
// scaled direction e * inv (Eq. 4), so that the weight is one clamped dot
// product.  inv = 0 marks a zero denominator (eps = 0 and L_i == L_j), whose
// weight is 1.
struct PairK {
  float4 e;   // e.x, e.y, e.z, unused
  float4 ei;  // e * inv (x, y, z), inv
};

__device__ __forceinline__ PairK pair_consts(float4 Li, float4 Lj, float eps) {
  const float ex = Li.x - Lj.x, ey = Li.y - Lj.y, ez = Li.z - Lj.z;
  const float n = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
  const float den = n + eps;
  // hardware reciprocal (1 ulp): the weight stays well inside the parity
  // tolerance, and every path of the search uses this same function
  const float inv = den > 0.0f ? __builtin_amdgcn_rcpf(den) : 0.0f;
  PairK k;
  k.e = make_float4(ex, ey, ez, 0.0f);
  k.ei = make_float4(ex * inv, ey * inv, ez * inv, inv);
  return k;
}

// One record of the exhaustive search's pair table: e (x, y, z) and inv in
// one 16-byte LDS word.  The scaled direction e * inv is formed when the
// record is read, with the same products pair_consts forms, so a record
// gives bitwise the constants pair_consts returns.
__device__ __forceinline__ float4 pair_rec(const PairK& k) { return make_float4(k.e.x, k.e.y, k.e.z, k.ei.w); }

__device__ __forceinline__ PairK pair_from_rec(float4 r) {
  PairK k;
  k.e = make_float4(r.x, r.y, r.z, 0.0f);
  k.ei = make_float4(r.x * r.w, r.y * r.w, r.z * r.w, r.w);
  return k;
}

// Eq. 4 weight on i for the pixel offset d = I_p - L_j, clamped to [0, 1]
// (the clamp folds into the last multiply-add).
__device__ __forceinline__ float pair_alpha(float dx, float dy, float dz, const PairK& t) {
  return clamp01(fmaf(dz, t.ei.z, fmaf(dy, t.ei.y, dx * t.ei.x)));
}

// Residual |d - alpha e|^2 computed from the residual itself (no expansion,
// so no cancellation when the error is small next to |d|).
__device__ __forceinline__ float pair_err2(float dx, float dy, float dz, float al, const PairK& t) {
  const float rx = fmaf(-al, t.e.x, dx);
  const float ry = fmaf(-al, t.e.y, dy);
  const float rz = fmaf(-al, t.e.z, dz);
  return fmaf(rz, rz, fmaf(ry, ry, rx * rx));
}

// Window accessors: win(o) is the LR guide colour of window offset o
// (o = (dy + r) * k + (dx + r)) with .w = 1 for a cell inside the LR image
// and .w = 0 outside.
//   LdsWin     - the tile's staged copy in LDS (window top-left at p, row
//                pitch lx);
//   GlobalWin  - straight from the LR guide in global memory, with coherent
//                (L1-bypassing) loads so that colours another thread of the
//                same workgroup just rewrote are seen (joint downsampling);
//   RegWin     - a k x k window (compile-time k) read once from a GlobalWin
//                into registers.
template <int KW>
struct LdsWin {
  const float4* __restrict__ p;
  int lx;
  int kw_rt;
  __device__ __forceinline__ float4 operator()(int o) const {
    const int kw = KW > 0 ? KW : kw_rt;
    return p[(o / kw) * lx + (o % kw)];
  }
};

struct GlobalWin {
  const float* L;
  int64_t Ls;
  int qy, qx, h, w, kw, r;
  __device__ __forceinline__ float4 operator()(int o) const {
    const int cy = qy + o / kw - r, cx = qx + o % kw - r;
    if (cy < 0 || cy >= h || cx < 0 || cx >= w) return make_float4(0.f, 0.f, 0.f, 0.f);
    const float* q = L + (int64_t)cy * Ls + (int64_t)cx * 3;
    // relaxed agent-scope atomic loads: coherent, yet free to be issued
    // together (volatile ones would each wait for the previous)
    return make_float4(__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                       __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                       __hip_atomic_load(q + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), 1.0f);
  }
};

template <int KW>
struct RegWin {
  float4 c[KW * KW];
  __device__ __forceinline__ explicit RegWin(const GlobalWin& g) {
#pragma unroll
    for (int o = 0; o < KW * KW; ++o) c[o] = g(o);
  }
  __device__ __forceinline__ float4 operator()(int o) const { return c[o]; }
};

// ---------------------------------------------------------------------------
// Exhaustive search of one strip (Eq. 3 with Eq. 4 over all pairs)
// ---------------------------------------------------------------------------
// Candidates in colexicographic order of window offsets (j outer, i < j
// inner, then (j, j)); the first strict minimum of |residual|^2 wins.
//
// Interior windows (all k*k cells present): the degenerate candidate (j, j)
// with j > 0 never beats (0, j), which precedes it and whose error is at
// most |I_p - L_j| (alpha >= 0 moves the point along the segment towards
// the pixel), so only (0, 0) is evaluated.  Border windows evaluate every
// valid candidate.
// With the pairs i < j as the only candidates, a window with a single valid
// cell (k = 1, or a 1 x 1 LR image) has none: its pixels take that cell
// (code j k^2 + j, weight 1).  Pixels with a finite best are left alone.
template <int P, typename Win>
__device__ __forceinline__ void exh_lone_cell(const float (&ip)[P][3], const Win& win, int K2, float (&best)[P],
                                              int (&code)[P]) {
  bool any = false;
#pragma unroll
  for (int q = 0; q < P; ++q) any |= !(best[q] < __builtin_inff());
  if (!any) return;
  for (int j = 0; j < K2; ++j) {
    const float4 Lj = win(j);
    if (Lj.w == 0.0f) continue;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      if (best[q] < __builtin_inff()) continue;
      const float dx = ip[q][0] - Lj.x, dy = ip[q][1] - Lj.y, dz = ip[q][2] - Lj.z;
      best[q] = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      code[q] = j * K2 + j;
    }
    break;
  }
}

template <int KW, int P, bool BORDER, bool TABLE, typename Win>
__device__ __forceinline__ void exh_strip(const float (&ip)[P][3], const Win& win,
                                          const float4* __restrict__ tab, float eps, int kw_rt, bool no_degen,
                                          float (&best)[P], int (&code)[P]) {
  constexpr int kUnrollJ = KW == 3 ? 9 : 1;
  constexpr int kUnrollI = KW == 3 ? 8 : 2;
  const int kw = KW > 0 ? KW : kw_rt;
  const int K2 = kw * kw;
#pragma unroll
  for (int q = 0; q < P; ++q) {
    best[q] = __builtin_inff();
    code[q] = 0;
  }
  if (!BORDER && !no_degen) {
    const float4 L0 = win(0);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const float dx = ip[q][0] - L0.x, dy = ip[q][1] - L0.y, dz = ip[q][2] - L0.z;
      best[q] = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    }
  }
#pragma unroll kUnrollJ
  for (int j = (BORDER ? 0 : 1); j < K2; ++j) {
    const float4 Lj = win(j);
    if (BORDER && Lj.w == 0.0f) continue;
    float d[P][3];
#pragma unroll
    for (int q = 0; q < P; ++q) {
      d[q][0] = ip[q][0] - Lj.x;
      d[q][1] = ip[q][1] - Lj.y;
      d[q][2] = ip[q][2] - Lj.z;
    }
#pragma unroll kUnrollI
    for (int i = 0; i < j; ++i) {
      PairK t;
      if (TABLE) {
        t = pair_from_rec(tab[pair_index(i, j)]);
      } else {
        const float4 Li = win(i);
        if (BORDER && Li.w == 0.0f) continue;
        t = pair_consts(Li, Lj, eps);
      }
      const int cc = i * K2 + j;
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const float al = pair_alpha(d[q][0], d[q][1], d[q][2], t);
        const float e2 = pair_err2(d[q][0], d[q][1], d[q][2], al, t);
        const bool lt = e2 < best[q];
        best[q] = lt ? e2 : best[q];
        code[q] = lt ? cc : code[q];
      }
    }
    if (BORDER && !no_degen) {
      const int cc = j * K2 + j;
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const float e2 = fmaf(d[q][2], d[q][2], fmaf(d[q][1], d[q][1], d[q][0] * d[q][0]));
        const bool lt = e2 < best[q];
        best[q] = lt ? e2 : best[q];
        code[q] = lt ? cc : code[q];
      }
    }
  }
  if (no_degen) exh_lone_cell<P>(ip, win, K2, best, code);
}

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

constexpr int colex_j(int p) {
  int j = 1;
  while ((j + 1) * j / 2 <= p) ++j;
  return j;
}
constexpr int colex_i(int p) { return p - colex_j(p) * (colex_j(p) - 1) / 2; }

// Exhaustive search of one strip for a full (interior) 3 x 3 window with the
// pair table: the 36 pairs are visited in colexicographic order with their
// indices known at compile time; the table record of the next pair is read
// from LDS while the current one is evaluated, and a scheduling barrier per
// pair keeps only two records live (instead of all 36).
template <int P, typename Win>
__device__ __forceinline__ void exh_interior3(const float (&ip)[P][3], const Win& win,
                                              const float4* __restrict__ tab, bool no_degen, float (&best)[P],
                                              int (&code)[P]) {
  constexpr int K2 = 9;
  constexpr int NP = 36;
  {
    // (0, 0) first, unless the pairs i < j are the only candidates
    const float4 L0 = win(0);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const float dx = ip[q][0] - L0.x, dy = ip[q][1] - L0.y, dz = ip[q][2] - L0.z;
      best[q] = no_degen ? __builtin_inff() : fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      code[q] = 0;
    }
  }
  float d[P][3];
  float4 nxt = tab[0];
  float4 Ln = win(1);
  static_for<0, NP>([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    constexpr int j = colex_j(p), i = colex_i(p);
    const PairK t = pair_from_rec(nxt);
    if constexpr (p + 1 < NP) nxt = tab[p + 1];
    if constexpr (i == 0) {
      const float4 Lj = Ln;
      if constexpr (j + 1 < K2) Ln = win(j + 1);
#pragma unroll
      for (int q = 0; q < P; ++q) {
        d[q][0] = ip[q][0] - Lj.x;
        d[q][1] = ip[q][1] - Lj.y;
        d[q][2] = ip[q][2] - Lj.z;
      }
    }
    constexpr int cc = i * K2 + j;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const float al = pair_alpha(d[q][0], d[q][1], d[q][2], t);
      const float e2 = pair_err2(d[q][0], d[q][1], d[q][2], al, t);
      const bool lt = e2 < best[q];
      best[q] = lt ? e2 : best[q];
      code[q] = lt ? cc : code[q];
    }
    __builtin_amdgcn_sched_barrier(0);
  });
}

// exh_interior3 without the table: the window's nine colours are read into
// registers once per strip and each pair's constants are built from them
// with pair_consts, as the table is; same pairs, same order, so the results
// are bitwise those of exh_strip.  The scheduling barrier per pair keeps
// one pair's constants live at a time.
template <int P, typename Win>
__device__ __forceinline__ void exh_interior3_rw(const float (&ip)[P][3], const Win& win, float eps, bool no_degen,
                                                 float (&best)[P], int (&code)[P]) {
  constexpr int K2 = 9;
  constexpr int NP = 36;
  float4 Lw[K2];
#pragma unroll
  for (int o = 0; o < K2; ++o) {
    const float4 L = win(o);
    Lw[o] = make_float4(L.x, L.y, L.z, 0.0f);
  }
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const float dx = ip[q][0] - Lw[0].x, dy = ip[q][1] - Lw[0].y, dz = ip[q][2] - Lw[0].z;
    best[q] = no_degen ? __builtin_inff() : fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    code[q] = 0;
  }
  float d[P][3];
  static_for<0, NP>([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    constexpr int j = colex_j(p), i = colex_i(p);
    if constexpr (i == 0) {
#pragma unroll
      for (int q = 0; q < P; ++q) {
        d[q][0] = ip[q][0] - Lw[j].x;
        d[q][1] = ip[q][1] - Lw[j].y;
        d[q][2] = ip[q][2] - Lw[j].z;
      }
    }
    const PairK t = pair_consts(Lw[i], Lw[j], eps);
    constexpr int cc = i * K2 + j;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const float al = pair_alpha(d[q][0], d[q][1], d[q][2], t);
      const float e2 = pair_err2(d[q][0], d[q][1], d[q][2], al, t);
      const bool lt = e2 < best[q];
      best[q] = lt ? e2 : best[q];
      code[q] = lt ? cc : code[q];
    }
    __builtin_amdgcn_sched_barrier(0);
  });
  if (no_degen) exh_lone_cell<P>(ip, win, K2, best, code);
}

// Weight of the winning exhaustive pair, recomputed with the same arithmetic
// the loop used.
template <int KW, bool TABLE, typename Win>
__device__ __forceinline__ float exh_alpha(const float (&ip)[3], const Win& win,
                                           const float4* __restrict__ tab, float eps, int kw_rt, int code) {
  const int kw = KW > 0 ? KW : kw_rt;
  const int K2 = kw * kw;
  const int oi = code / K2, oj = code - oi * K2;
  const float4 Lj = win(oj);
  PairK t;
  if (TABLE) {
    // (oi, oi) maps to a valid table slot (the record after the last pair
    // of column oi); its value is not used
    t = pair_from_rec(tab[pair_index(oi, oj)]);
  } else {
    const float4 Li = win(oi);
    t = pair_consts(Li, Lj, eps);
  }
  const float al = pair_alpha(ip[0] - Lj.x, ip[1] - Lj.y, ip[2] - Lj.z, t);
  return (oi == oj || t.ei.w == 0.0f) ? 1.0f : al;
}

// ---------------------------------------------------------------------------
// Fast search of one strip (Algorithm 1 with Eq. 5)
// ---------------------------------------------------------------------------
// a = first window cell of least colour distance; then every b of the window
// (b = a included, weight 1) with w_b = |I-L_b| / (|I-L_a| + |I-L_b| + eps),
// keeping the first b of least error.
template <int KW, int P, bool BORDER, typename Win>
__device__ __forceinline__ void fast_strip(const float (&ip)[P][3], const Win& win,
                                           float eps, int kw_rt, bool gnu, float (&best)[P], int (&code)[P],
                                           float (&alpha)[P]) {
  constexpr int kUnrollJ = KW == 3 ? 9 : 1;
  const int kw = KW > 0 ? KW : kw_rt;
  const int K2 = kw * kw;
  constexpr bool kKeep = (KW > 0) && (KW * KW * P <= 36);
  float sd[kKeep ? P : 1][kKeep ? KW * KW : 1];
  float dmin[P];
  int ia[P];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    dmin[q] = __builtin_inff();
    ia[q] = 0;
  }
#pragma unroll kUnrollJ
  for (int j = 0; j < K2; ++j) {
    const float4 Lj = win(j);
    if (BORDER && Lj.w == 0.0f) continue;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const float dx = ip[q][0] - Lj.x, dy = ip[q][1] - Lj.y, dz = ip[q][2] - Lj.z;
      const float D = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      if constexpr (kKeep) sd[q][j] = __builtin_amdgcn_sqrtf(D);
      const bool lt = D < dmin[q];
      dmin[q] = lt ? D : dmin[q];
      ia[q] = lt ? j : ia[q];
    }
  }
  if (gnu) {
    // guided nearest neighbour: the anchor alone, weight 1 (uniform branch)
#pragma unroll
    for (int q = 0; q < P; ++q) {
      best[q] = dmin[q];
      code[q] = ia[q] * K2 + ia[q];
      alpha[q] = 1.0f;
    }
    return;
  }
  // sae: the anchor's distance plus eps, the part of the Eq. 5 denominator
  // fixed for the pixel; bsel: window offset of the best partner so far
  // (the code is formed once, after the loop)
  float La[P][3], sae[P], omb[P];
  int bsel[P];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const float4 A = win(ia[q]);
    La[q][0] = A.x;
    La[q][1] = A.y;
    La[q][2] = A.z;
    sae[q] = __builtin_amdgcn_sqrtf(dmin[q]) + eps;
    best[q] = dmin[q];
    bsel[q] = ia[q];
    omb[q] = 1.0f;
  }
#pragma unroll kUnrollJ
  for (int b = 0; b < K2; ++b) {
    const float4 Lb = win(b);
    if (BORDER && Lb.w == 0.0f) continue;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      float sb;
      if constexpr (kKeep) {
        sb = sd[q][b];
      } else {
        const float dx = ip[q][0] - Lb.x, dy = ip[q][1] - Lb.y, dz = ip[q][2] - Lb.z;
        sb = __builtin_amdgcn_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
      }
      const float den = sae[q] + sb;
      const float om = sb * __builtin_amdgcn_rcpf(den);
      const float om1 = 1.0f - om;
      // residual = om L_a + (1 - om) L_b - I, negated
      const float tx = fmaf(-om, La[q][0], ip[q][0]);
      const float ty = fmaf(-om, La[q][1], ip[q][1]);
      const float tz = fmaf(-om, La[q][2], ip[q][2]);
      const float rx = fmaf(-om1, Lb.x, tx);
      const float ry = fmaf(-om1, Lb.y, ty);
      const float rz = fmaf(-om1, Lb.z, tz);
      const float e2 = fmaf(rz, rz, fmaf(ry, ry, rx * rx));
      const bool lt = e2 < best[q];
      best[q] = lt ? e2 : best[q];
      bsel[q] = lt ? b : bsel[q];
      omb[q] = lt ? om : omb[q];
    }
  }
#pragma unroll
  for (int q = 0; q < P; ++q) {
    code[q] = ia[q] * K2 + bsel[q];
    alpha[q] = (bsel[q] == ia[q]) ? 1.0f : omb[q];
  }
}

// Fast search of a strip of a 3 x 3 window (Algorithm 1 with Eq. 5) with
// the window's nine colours held in registers and the strip's pixels
// searched one after another: one pixel's nine distances are live at a time
// instead of P x 9, so the fused kernel fits four waves per SIMD (114 VGPRs
// against 146).  Same arithmetic in the same order as fast_strip, so the
// outputs are bitwise the same; BORDER skips window cells outside the image.
template <int P, bool BORDER, typename Win>
__device__ __forceinline__ void fast_strip_rw(const float (&ip)[P][3], const Win& win, float eps, bool gnu,
                                              float (&best)[P], int (&code)[P], float (&alpha)[P]) {
  float Lw[9][3];
  bool in[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const float4 L = win(j);
    Lw[j][0] = L.x;
    Lw[j][1] = L.y;
    Lw[j][2] = L.z;
    in[j] = !BORDER || L.w != 0.0f;
  }
  static_for<0, P>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    // squared distances; their square roots are taken in the partner loop,
    // which GNU mode skips
    float Dj[9];
    float dmin = __builtin_inff();
    int ia = 0;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      const float dx = ip[q][0] - Lw[j][0], dy = ip[q][1] - Lw[j][1], dz = ip[q][2] - Lw[j][2];
      const float D = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      Dj[j] = D;
      const bool lt = in[j] && D < dmin;
      dmin = lt ? D : dmin;
      ia = lt ? j : ia;
    }
    if (gnu) {
      best[q] = dmin;
      code[q] = ia * 9 + ia;
      alpha[q] = 1.0f;
    } else {
      const float4 A = win(ia);
      const float sae = __builtin_amdgcn_sqrtf(dmin) + eps;
      float bq = dmin, omb = 1.0f;
      int bsel = ia;
#pragma unroll
      for (int b = 0; b < 9; ++b) {
        const float sb = __builtin_amdgcn_sqrtf(Dj[b]);
        const float den = sae + sb;
        const float om = sb * __builtin_amdgcn_rcpf(den);
        const float om1 = 1.0f - om;
        const float tx = fmaf(-om, A.x, ip[q][0]);
        const float ty = fmaf(-om, A.y, ip[q][1]);
        const float tz = fmaf(-om, A.z, ip[q][2]);
        const float rx = fmaf(-om1, Lw[b][0], tx);
        const float ry = fmaf(-om1, Lw[b][1], ty);
        const float rz = fmaf(-om1, Lw[b][2], tz);
        const float e2 = fmaf(rz, rz, fmaf(ry, ry, rx * rx));
        const bool lt = in[b] && e2 < bq;
        bq = lt ? e2 : bq;
        bsel = lt ? b : bsel;
        omb = lt ? om : omb;
      }
      best[q] = bq;
      code[q] = ia * 9 + bsel;
      alpha[q] = (bsel == ia) ? 1.0f : omb;
    }
    __builtin_amdgcn_sched_barrier(0);
  });
}

// ---------------------------------------------------------------------------
// Staged output stores of the fused search
// ---------------------------------------------------------------------------
// A strip of 4 pixels of C = 3 (or 1) channels is 3 (or 1) words of 4
// elements (16 bytes in float32, 8 in float16).  Lane l writes the words
// of its strip to slots 3l .. 3l+2 (or l) of its wave's LDS buffer.
template <typename T, int P>
__device__ __forceinline__ void stage_strip(float4* buf, int lane, int C, const float (&o)[P][4]) {
  if constexpr (P == 4) {
    if constexpr (sizeof(T) == 4) {
      if (C == 3) {
        buf[3 * lane + 0] = make_float4(o[0][0], o[0][1], o[0][2], o[1][0]);
        buf[3 * lane + 1] = make_float4(o[1][1], o[1][2], o[2][0], o[2][1]);
        buf[3 * lane + 2] = make_float4(o[2][2], o[3][0], o[3][1], o[3][2]);
      } else {
        buf[lane] = make_float4(o[0][0], o[1][0], o[2][0], o[3][0]);
      }
    } else {
      uint2* b2 = reinterpret_cast<uint2*>(buf);
      auto pk = [](float a, float b) {
        return (uint32_t)__half_as_ushort(__float2half_rn(a)) | ((uint32_t)__half_as_ushort(__float2half_rn(b)) << 16);
      };
      if (C == 3) {
        b2[3 * lane + 0] = make_uint2(pk(o[0][0], o[0][1]), pk(o[0][2], o[1][0]));
        b2[3 * lane + 1] = make_uint2(pk(o[1][1], o[1][2]), pk(o[2][0], o[2][1]));
        b2[3 * lane + 2] = make_uint2(pk(o[2][2], o[3][0]), pk(o[3][1], o[3][2]));
      } else {
        b2[lane] = make_uint2(pk(o[0][0], o[1][0]), pk(o[2][0], o[3][0]));
      }
    }
  }
}

// Stores the staged strips of the calling wave.  off = element offset of
// the lane's own strip from `out` (the tile's first element), or -1 when the
// lane staged nothing; every lane of the wave must call this together.
template <typename T>
__device__ __forceinline__ void store_staged(float4* buf, int lane, int C, int off, T* __restrict__ out) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int nw = C == 3 ? 3 : 1;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k >= nw) break;
    const int idx = lane + 64 * k;
    const int st = nw == 3 ? idx / 3 : idx;  // strip (owner lane) of the word
    const int part = idx - st * nw;
    const int o = __shfl(off, st, 64);
    if (o >= 0) {
      T* dst = out + o + 4 * part;
      if constexpr (sizeof(T) == 4)
        __builtin_nontemporal_store(reinterpret_cast<const f32x4*>(buf)[idx], reinterpret_cast<f32x4*>(dst));
      else
        __builtin_nontemporal_store(reinterpret_cast<const u32x2*>(buf)[idx], reinterpret_cast<u32x2*>(dst));
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Strips of 2 or 3 float32 pixels are not whole 16-byte words, so their
// staging is per pixel: lane l writes its strip's P pixels (C floats each)
// to pixels P*l .. P*l + P-1 of its wave's buffer, and in store round k lane
// l stores pixel 64 k + l, so that neighbouring lanes write neighbouring
// pixels (one contiguous run of 64 pixels per round when the wave's strips
// are consecutive in a row).
template <int P>
__device__ __forceinline__ void stage_strip_px(float* buf, int lane, int C, const float (&o)[P][4]) {
#pragma unroll
  for (int q = 0; q < P; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < C) buf[(lane * P + q) * C + c] = o[q][c];
}

template <int P>
__device__ __forceinline__ void store_staged_px(const float* buf, int lane, int C, int off, float* __restrict__ out) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int m = lane + 64 * k;
    const int st = m / P;  // owner lane of the pixel
    const int q = m - st * P;
    const int o = __shfl(off, st, 64);
    if (o >= 0) {
      float* dst = out + o + q * C;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c < C) __builtin_nontemporal_store(buf[m * C + c], dst + c);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Unsigned division by a runtime divisor 1 <= d < 2^16 for 0 <= n < 2^30,
// with m = min(2^32 - 1, floor(2^32 / d)) or m = floor((2^32 - 1) / d):
// either is floor(2^32 / d) or one less, so the estimate q = umulhi(n, m)
// is floor(n / d) or one less (2n / 2^32 < 1), and one correction step
// makes it exact.
__device__ __forceinline__ int udiv_rt(int n, int d, uint32_t m) {
  int q = (int)__umulhi((uint32_t)n, m);
  if ((q + 1) * d <= n) ++q;
  return q;
}

// ---------------------------------------------------------------------------
// One tile of search (+ apply when FUSED)
// ---------------------------------------------------------------------------
enum { MODE_EXH = 0, MODE_FAST = 1 };

// The exhaustive search reads per-cell pair constants from an LDS table for
// 3 x 3 windows (36 pairs, 592 bytes per LR cell), shared by the s^2 pixels
// of the cell.  Larger windows (300 pairs for 5 x 5) would shrink the tiles
// below one strip per thread, so they build the constants of each pair once
// per strip instead; so do 3 x 3 windows with s < 5, whose cells are too
// small to pay for their table (the tile that fits the LDS budget then
// leaves threads idle).  Both forms use pair_consts, so they give bitwise
// the same results.
constexpr int kMinTableS = 5;
__host__ __device__ constexpr bool kernel_has_table(int mode, int k) { return mode == MODE_EXH && k == 3; }
__host__ __device__ constexpr bool uses_pair_table(int mode, int k, int s) {
  return kernel_has_table(mode, k) && s >= kMinTableS;
}

// Output staging of the fused search: per wave, 64 strips of 4 pixels of 3
// float channels (48 bytes each).
constexpr int kStageWords = (kThreads / 64) * 64 * 3;
// Fused tiles of windows up to this size map a Theta code to the LDS
// offsets of its two cells with a table of k^4 entries.
constexpr int kMaxOffTableK = 5;

// LDS float4 words one search tile needs.
__host__ __device__ inline int search_tile_words(int tqy, int tqx, int k, int mode, bool fused, bool table) {
  const int r = k / 2;
  const int ncell = (tqy + 2 * r) * (tqx + 2 * r);
  int words = ncell * (fused ? 2 : 1);
  if (mode == MODE_EXH && table) words += tqy * tqx * (n_pairs(k * k) + 1);
  if (fused) words += kStageWords;
  if (fused && k <= kMaxOffTableK) words += (k * k * k * k + 3) / 4;
  return words;
}

// One LR cell of a tile's staging: the guide (with the inside-image flag in
// .w) and, when sT is wanted, the target; zeros outside the image.
template <typename T>
__device__ __forceinline__ void load_lr_cell(const ImgDesc& d, int qy0, int qx0, int R, int lx, int c, bool want_t,
                                             float4& v, float4& tv) {
  const T* __restrict__ L = static_cast<const T*>(d.L);
  const T* __restrict__ TL = static_cast<const T*>(d.T);
  const int oy = c / lx;
  const int cy = qy0 - R + oy, cx = qx0 - R + (c - oy * lx);
  v = make_float4(0.f, 0.f, 0.f, 0.f);
  tv = v;
  if (cy >= 0 && cy < d.h && cx >= 0 && cx < d.w) {
    const T* q = L + (int64_t)cy * d.L_stride + (int64_t)cx * 3;
    v = make_float4(to_f<T>(q[0]), to_f<T>(q[1]), to_f<T>(q[2]), 1.0f);
    if (want_t) {
      const T* t = TL + (int64_t)cy * d.T_stride + (int64_t)cx * d.C;
      float tt[4];
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) tt[ch] = ch < d.C ? to_f<T>(t[ch]) : 0.f;
      tv = make_float4(tt[0], tt[1], tt[2], tt[3]);
    }
  }
}

template <int KW, int P, int MODE, typename T, bool FUSED, bool TABLE>
__device__ __forceinline__ void search_tile(const ImgDesc& d, int ty, int tx, float eps, float4* smem) {
  const int kw = KW > 0 ? KW : d.k;
  const int R = kw / 2;
  const int K2 = kw * kw;
  const int s = d.s;
  const int tqy = d.tqy, tqx = d.tqx;
  const int qy0 = ty * tqy, qx0 = tx * tqx;
  const int ly = tqy + 2 * R, lx = tqx + 2 * R;
  const int ncell = ly * lx;
  float4* sL = smem;
  float4* sT = FUSED ? smem + ncell : nullptr;
  float4* sTab = smem + (FUSED ? 2 : 1) * ncell;
  const int tstride = n_pairs(K2) + 1;
  const int lane = (int)threadIdx.x & 63;
  // per-wave output staging (fused): after the pair table
  float4* sStageAll = smem + (FUSED ? 2 : 1) * ncell + ((MODE == MODE_EXH && TABLE) ? tqy * tqx * tstride : 0);
  float4* sStage = sStageAll + ((int)threadIdx.x >> 6) * 64 * 3;
  // code -> (offset of cell a) | (offset of cell b) << 16, relative to the
  // pixel's centre at window offset 0 (fused, k <= kMaxOffTableK)
  constexpr bool kOffTab = FUSED && KW > 0 && KW <= kMaxOffTableK;
  uint32_t* sOff = reinterpret_cast<uint32_t*>(sStageAll + kStageWords);

  const int rows = tqy * s, cols = tqx * s;
  const int spr = cols / P;
  const int nstrips = rows * spr;
  const bool interior = (qy0 - R >= 0) && (qy0 + tqy + R <= d.h) && (qx0 - R >= 0) &&
                        (qx0 + tqx + R <= d.w) && ((qy0 + tqy) * s <= d.H) && ((qx0 + tqx) * s <= d.W);
  const bool vecI = (d.vec & VEC_I) != 0, vecTh = (d.vec & VEC_THETA) != 0, vecT = (d.vec & VEC_T) != 0;
  const T* __restrict__ Ig = static_cast<const T*>(d.I);

  // The HR pixels of a thread's next strip are loaded one strip ahead: the
  // first strip's loads are in flight while the tile is staged, later ones
  // while the current strip is searched.
  // strip -> (row, column) and pixel -> LR cell without integer division
  // instructions: spr <= 1024 and s <= 1024, strip and pixel indices of a
  // tile far below 2^30
  const uint32_t m_spr = 0xffffffffu / (uint32_t)spr, m_s = 0xffffffffu / (uint32_t)s;
  float ipn[P][3];
  auto prefetch = [&](int t) {
    if (t >= nstrips) return;
    const int ry = udiv_rt(t, spr, m_spr);
    const int rx = (t - ry * spr) * P;
    const int y = qy0 * s + ry, x = qx0 * s + rx;
    if (y >= d.H || x >= d.W) return;
    load_strip3<T, P>(Ig + (int64_t)y * d.I_stride, x, d.W, vecI, interior || (x + P <= d.W), ipn);
  };
  // The tile's first round of LR cells is loaded into registers, then the
  // first strip's pixels, and only then are the cells written to LDS: the
  // two sets of loads are in flight together (a staging loop ahead of the
  // prefetch would wait for it at its head).
  float4 lv, ltv;
  const bool lr_first = (int)threadIdx.x < ncell;
  if (lr_first) load_lr_cell<T>(d, qy0, qx0, R, lx, threadIdx.x, FUSED, lv, ltv);
  prefetch(threadIdx.x);
  if (lr_first) {
    sL[threadIdx.x] = lv;
    if (FUSED) sT[threadIdx.x] = ltv;
  }
  for (int c = threadIdx.x + kThreads; c < ncell; c += kThreads) {
    load_lr_cell<T>(d, qy0, qx0, R, lx, c, FUSED, lv, ltv);
    sL[c] = lv;
    if (FUSED) sT[c] = ltv;
  }
  if constexpr (kOffTab) {
    for (int c = threadIdx.x; c < K2 * K2; c += kThreads) {
      const int oa = c / K2, ob = c - oa * K2;
      sOff[c] = (uint32_t)((oa / kw) * lx + oa % kw) | ((uint32_t)((ob / kw) * lx + ob % kw) << 16);
    }
  }
  __syncthreads();
  if constexpr (MODE == MODE_EXH && TABLE) {
    // the table exists for 3 x 3 windows: 36 pairs per centre
    static_assert(KW == 3, "the pair table is built for 3 x 3 windows");
    constexpr int NP = 36;
    constexpr int kBuild = (kThreads / NP) * NP;  // 252 threads: each keeps one pair index
    const int ncent = tqy * tqx;
    const int tid = (int)threadIdx.x;
    if (tid < kBuild) {
      const int pr = tid % NP;
      // colexicographic pair pr = j (j - 1) / 2 + i, i < j
      const int j = 1 + (pr >= 1) + (pr >= 3) + (pr >= 6) + (pr >= 10) + (pr >= 15) + (pr >= 21) + (pr >= 28);
      const int i = pr - ((j * (j - 1)) >> 1);
      // window offset o -> (o / 3, o % 3) for o < 9, as LDS offsets
      const int iy = (i * 11) >> 5, jy = (j * 11) >> 5;
      const int offi = iy * lx + i - 3 * iy, offj = jy * lx + j - 3 * jy;
      const float inv_tqx = __builtin_amdgcn_rcpf((float)tqx);
      for (int c = tid / NP; c < ncent; c += kBuild / NP) {
        // centre (cy, cx) of the tile: c / tqx, exact for c < 2^16
        const int cy = (int)(((float)c + 0.5f) * inv_tqx), cx = c - cy * tqx;
        const float4 Li = sL[cy * lx + cx + offi];
        const float4 Lj = sL[cy * lx + cx + offj];
        sTab[c * tstride + pr] = pair_rec(pair_consts(Li, Lj, eps));
      }
    }
    __syncthreads();
  }

  // Fused tiles whose T_hat rows allow vector stores hand the full strips of
  // a wave to one staged store: the strips' values go to LDS and every lane
  // then stores 4-element words of consecutive strips, so neighbouring
  // lanes write neighbouring words of a row.  The loop is uniform over a
  // wave for that; lanes past the tile or the image only take part in it.
  const bool staged = FUSED && P == 4 && vecT && (d.C == 3 || d.C == 1) &&
                      (int64_t)rows * d.That_stride < 0x7fffffff;  // tile offsets fit 32 bits
  // float32 strips of 2 or 3 pixels of the fast search: staged per pixel
  // (the exhaustive kernels keep direct stores: the staging's registers
  // cost them a wave per SIMD, more than the stores gain)
  constexpr bool kStagePx = FUSED && MODE == MODE_FAST && (P == 2 || P == 3) && sizeof(T) == 4;
  const bool staged_px = kStagePx && (int64_t)rows * d.That_stride < 0x7fffffff;
  for (int t = threadIdx.x; t - lane < nstrips; t += kThreads) {
    const int ry = udiv_rt(t, spr, m_spr);
    const int rx = (t - ry * spr) * P;
    const int y = qy0 * s + ry, x = qx0 * s + rx;
    float ip[P][3];
#pragma unroll
    for (int q = 0; q < P; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) ip[q][c] = ipn[q][c];
    prefetch(t + kThreads);
    const bool live = t < nstrips && y < d.H && x < d.W;
    const bool full = interior || (x + P <= d.W);
    int stage_off = -1;  // element offset of a staged strip from the tile's first T_hat element
    if (live) {
    const int cy = udiv_rt(ry, s, m_s), cx = udiv_rt(rx, s, m_s);
    const LdsWin<KW> win{sL + cy * lx + cx, lx, kw};
    const float4* tab = sTab + (cy * tqx + cx) * tstride;
    float best[P], al[P];
    int code[P];
    if (MODE == MODE_EXH) {
      if (interior) {
        if constexpr (KW == 3 && TABLE)
          exh_interior3<P>(ip, win, tab, d.no_degen != 0, best, code);
        else if constexpr (KW == 3 && P >= 2)
          exh_interior3_rw<P>(ip, win, eps, d.no_degen != 0, best, code);
        else
          exh_strip<KW, P, false, TABLE>(ip, win, tab, eps, kw, d.no_degen != 0, best, code);
#pragma unroll
        for (int q = 0; q < P; ++q) al[q] = exh_alpha<KW, TABLE>(ip[q], win, tab, eps, kw, code[q]);
      } else {
        exh_strip<KW, P, true, false>(ip, win, tab, eps, kw, d.no_degen != 0, best, code);
#pragma unroll
        for (int q = 0; q < P; ++q) al[q] = exh_alpha<KW, false>(ip[q], win, tab, eps, kw, code[q]);
      }
    } else {
      if constexpr (KW == 3 && P >= 2) {
        if (interior)
          fast_strip_rw<P, false>(ip, win, eps, d.gnu != 0, best, code, al);
        else
          fast_strip_rw<P, true>(ip, win, eps, d.gnu != 0, best, code, al);
      } else {
        if (interior)
          fast_strip<KW, P, false>(ip, win, eps, kw, d.gnu != 0, best, code, al);
        else
          fast_strip<KW, P, true>(ip, win, eps, kw, d.gnu != 0, best, code, al);
      }
    }
    float e[P];
#pragma unroll
    for (int q = 0; q < P; ++q) e[q] = __builtin_amdgcn_sqrtf(best[q]);
    const int64_t to = (int64_t)y * d.th_stride;
    store_theta<P>(d.code ? d.code + to : nullptr, d.alpha ? d.alpha + to : nullptr, d.err ? d.err + to : nullptr,
                   x, d.W, vecTh, full, code, al, e);
    if (FUSED) {
      float o[P][4];
#pragma unroll
      for (int q = 0; q < P; ++q) {
        float4 Ta, Tb;
        if constexpr (kOffTab) {
          const uint32_t pk = sOff[code[q]];
          const float4* base = sT + cy * lx + cx;
          Ta = base[pk & 0xffff];
          Tb = base[pk >> 16];
        } else {
          const int oa = code[q] / K2, ob = code[q] - oa * K2;
          Ta = sT[(cy + oa / kw) * lx + cx + oa % kw];
          Tb = sT[(cy + ob / kw) * lx + cx + ob % kw];
        }
        o[q][0] = fmaf(al[q], Ta.x - Tb.x, Tb.x);
        o[q][1] = fmaf(al[q], Ta.y - Tb.y, Tb.y);
        o[q][2] = fmaf(al[q], Ta.z - Tb.z, Tb.z);
        o[q][3] = fmaf(al[q], Ta.w - Tb.w, Tb.w);
      }
      if (staged && full) {
        stage_strip<T, P>(sStage, lane, d.C, o);
        stage_off = (int)((int64_t)ry * d.That_stride + (int64_t)rx * d.C);
      } else if (kStagePx && staged_px && full) {
        stage_strip_px<P>(reinterpret_cast<float*>(sStage), lane, d.C, o);
        stage_off = (int)((int64_t)ry * d.That_stride + (int64_t)rx * d.C);
      } else {
        store_out<T, P>(static_cast<T*>(d.That) + (int64_t)y * d.That_stride, x, d.W, d.C, vecT, full, o);
      }
    }
    }  // live
    if (staged)
      store_staged<T>(sStage, lane, d.C, stage_off,
                      static_cast<T*>(d.That) + (int64_t)qy0 * s * d.That_stride + (int64_t)qx0 * s * d.C);
    if constexpr (kStagePx) {
      if (staged_px)
        store_staged_px<P>(reinterpret_cast<const float*>(sStage), lane, d.C, stage_off,
                           static_cast<float*>(d.That) + (int64_t)qy0 * s * d.That_stride + (int64_t)qx0 * s * d.C);
    }
  }
}

// ---------------------------------------------------------------------------
// Apply (Eq. 1) over tiles of one LR row
// ---------------------------------------------------------------------------
// Apply is a pure stream: 6 bytes of Theta in and C * sizeof(T) bytes of
// T_hat out per pixel.  A workgroup owns the s HR rows of one LR row over
// tqx LR columns.  It issues the Theta loads of its first strips, stages
// the k rows of LR target cells the tile can reach in LDS (one float4 per
// cell), and gathers from LDS.  tqx * s is a multiple of 64 * P, so the 64
// strips of a wave are consecutive pixels of one HR row: the wave writes
// its results to an LDS buffer and stores them as one contiguous run of
// 16-byte words (non-temporal, the output is not read again here).
//
// Divisions by s use udiv_rt (defined with the search tile).

template <typename T>
__device__ __forceinline__ float4 load_cell(const T* __restrict__ p, int C) {
  float v[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (c < C) v[c] = to_f<T>(p[c]);
  return make_float4(v[0], v[1], v[2], v[3]);
}

// Writes N values of T to LDS at dst (aligned to the widest power of two,
// up to 16, that divides N * sizeof(T)) with the widest such accesses.
template <typename T, int N>
__device__ __forceinline__ void lds_put(char* dst, const T (&v)[N]) {
  constexpr int B = N * (int)sizeof(T);
  if constexpr (B % 16 == 0) {
    uint4 w[B / 16];
    __builtin_memcpy(w, v, B);
#pragma unroll
    for (int i = 0; i < B / 16; ++i) reinterpret_cast<uint4*>(dst)[i] = w[i];
  } else if constexpr (B % 8 == 0) {
    uint2 w[B / 8];
    __builtin_memcpy(w, v, B);
#pragma unroll
    for (int i = 0; i < B / 8; ++i) reinterpret_cast<uint2*>(dst)[i] = w[i];
  } else if constexpr (B % 4 == 0) {
    uint32_t w[B / 4];
    __builtin_memcpy(w, v, B);
#pragma unroll
    for (int i = 0; i < B / 4; ++i) reinterpret_cast<uint32_t*>(dst)[i] = w[i];
  } else {
    uint16_t w[B / 2];
    __builtin_memcpy(w, v, B);
#pragma unroll
    for (int i = 0; i < B / 2; ++i) reinterpret_cast<uint16_t*>(dst)[i] = w[i];
  }
}

// LDS float4 words of one apply tile: the staged LR cells plus one output
// buffer per wave.
__host__ __device__ inline int apply_tile_words(int tqx, int k, int P, int C, int esize) {
  return k * (tqx + k - 1) + (kThreads / 64) * 4 * P * C * esize;
}

template <int KW, int P, typename T, int C, int NS>
__device__ __forceinline__ void apply_tile(const ImgDesc& d, int qy, int qx0, uint32_t s_magic, float4* smem) {
  constexpr int B = P * C * (int)sizeof(T);  // bytes of one strip of T_hat
  constexpr int kWords = 4 * B;              // 16-byte words of a wave's 64 strips
  constexpr int kWaves = kThreads / 64;
  const int kw = KW > 0 ? KW : d.k;
  const int R = kw / 2;
  const int K2 = kw * kw;
  const int maxcode = K2 * K2 - 1;
  const int s = d.s, tqx = d.tqx, lx = tqx + kw - 1;
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int wpr = tqx * s / (64 * P);  // wave runs per HR row
  const int nrun = s * wpr;             // wave runs of the tile
  const int xt = qx0 * s;               // first HR column of the tile
  float4* sT = smem;
  char* sx = reinterpret_cast<char*>(smem + kw * lx) + wave * kWords * 16;
  const bool vecTh = P == 4 && (d.vec & VEC_THETA) != 0;
  const bool vecTW = (d.vec & VEC_TW) != 0;
  const T* __restrict__ TL = static_cast<const T*>(d.T);

  int cd[NS][P];
  float al[NS][P];
  int ys[NS], x0s[NS];
  // Theta of the strips of wave runs g0 + n * kWaves + wave, n < NS
  auto load = [&](int g0) {
#pragma unroll
    for (int n = 0; n < NS; ++n) {
      const int g = g0 + n * kWaves + wave;  // uniform over the wave
      const int row = g / wpr;
      const int y = qy * s + row;
      const int x0 = xt + (g - row * wpr) * 64 * P;
      const int x = x0 + lane * P;
      ys[n] = (g < nrun && y < d.H) ? y : -1;
      x0s[n] = x0;
      const bool live = ys[n] >= 0 && x < d.W;
      const int64_t to = (int64_t)y * d.th_stride + x;
      bool done = false;
      if constexpr (P == 4) {
        if (live && vecTh && x + P <= d.W) {
          const u32x2 c = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(d.code + to));
          const f32x4 a4 = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(d.alpha + to));
          cd[n][0] = c.x & 0xffff;
          cd[n][1] = c.x >> 16;
          cd[n][2] = c.y & 0xffff;
          cd[n][3] = c.y >> 16;
          al[n][0] = a4.x;
          al[n][1] = a4.y;
          al[n][2] = a4.z;
          al[n][3] = a4.w;
          done = true;
        }
      }
      if (!done) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
          const bool ok = live && x + q < d.W;
          cd[n][q] = ok ? (int)d.code[to + q] : 0;
          al[n][q] = ok ? d.alpha[to + q] : 0.0f;
        }
      }
    }
  };

  load(0);
  // LR target cells rows qy - R .. qy + R, columns qx0 - R .. qx0 + tqx - 1 + R,
  // clamped to the LR image (codes from the search never leave it; other
  // codes read the nearest cell instead of leaving the buffer)
  for (int i = (int)threadIdx.x; i < kw * lx; i += kThreads) {
    const int r = i / lx, c = i - r * lx;
    const int cy = min(max(qy - R + r, 0), d.h - 1);
    const int cx = min(max(qx0 - R + c, 0), d.w - 1);
    sT[i] = load_cell<T>(TL + (int64_t)cy * d.T_stride + (int64_t)cx * C, C);
  }
  __syncthreads();

  for (int g0 = 0;;) {
#pragma unroll
    for (int n = 0; n < NS; ++n) {
      const int y = ys[n];
      if (y < 0) continue;  // uniform over the wave
      const int x0 = x0s[n];
      const int x = x0 + lane * P;
      // all P pixels of a strip share their LR cell (P divides s); cells
      // of lanes past the right edge stay inside the tile
      const int cx = udiv_rt(x - xt, s, s_magic);
      float o[P][C];
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const int c = min(cd[n][q], maxcode);
        const int oa = c / K2, ob = c - oa * K2;
        const float4 ta = sT[(oa / kw) * lx + cx + oa % kw];
        const float4 tb = sT[(ob / kw) * lx + cx + ob % kw];
        const float va[4] = {ta.x, ta.y, ta.z, ta.w};
        const float vb[4] = {tb.x, tb.y, tb.z, tb.w};
#pragma unroll
        for (int ch = 0; ch < C; ++ch) o[q][ch] = fmaf(al[n][q], va[ch] - vb[ch], vb[ch]);
      }
      T* __restrict__ orow = static_cast<T*>(d.That) + (int64_t)y * d.That_stride;
      if (vecTW && x0 + 64 * P <= d.W) {
        T v[P * C];
#pragma unroll
        for (int q = 0; q < P; ++q)
#pragma unroll
          for (int ch = 0; ch < C; ++ch) v[q * C + ch] = from_f<T>(o[q][ch]);
        lds_put<T, P * C>(sx + lane * B, v);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        f32x4* dst = reinterpret_cast<f32x4*>(orow + (int64_t)x0 * C);
        const f32x4* src = reinterpret_cast<const f32x4*>(sx);
#pragma unroll
        for (int k16 = 0; k16 < (kWords + 63) / 64; ++k16) {
          const int idx = lane + 64 * k16;
          if (idx < kWords) __builtin_nontemporal_store(src[idx], dst + idx);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      } else {
#pragma unroll
        for (int q = 0; q < P; ++q)
          if (x + q < d.W)
#pragma unroll
            for (int ch = 0; ch < C; ++ch) orow[(int64_t)(x + q) * C + ch] = from_f<T>(o[q][ch]);
      }
    }
    g0 += NS * kWaves;
    if (g0 >= nrun) break;
    load(g0);
  }
}

}  // namespace glu
