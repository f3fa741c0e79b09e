// Device-side helpers of the gfx950 tetrahedron rasterizer.
//
// The library is compiled with -ffp-contract=off: every fused multiply-add
// is written out with fmaf(), so the binning quantities (projected
// vertices, pixel rectangles, depth keys, face determinants, coverage
// signs) come from a fixed IEEE operation sequence.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ts_internal.h"

namespace ts {

__device__ __forceinline__ int find_view_by_tile(const DevView* views, int nv, int tile) {
  int lo = 0, hi = nv - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Eq. 1 in the stable form alpha = -expm1(-s d) / (1 + exp(s f_next)),
// d = f_prev - f_next; zero unless d > 0 (the max(., 0) of Eq. 1).
__device__ __forceinline__ float alpha_eq1(float fprev, float fnext, float s) {
  float d = fprev - fnext;
  if (!(d > 0.0f)) return 0.0f;
  return -expm1f(-(s * d)) / (1.0f + expf(s * fnext));
}

// face vertex table: (0,1,2) (0,1,3) (0,2,3) (1,2,3)
__host__ __device__ constexpr int face_vertex(int F, int k) {
  return F == 0 ? (k == 0 ? 0 : k == 1 ? 1 : 2)
       : F == 1 ? (k == 0 ? 0 : k == 1 ? 1 : 3)
       : F == 2 ? (k == 0 ? 0 : k == 1 ? 2 : 3)
                : (k == 0 ? 1 : k == 1 ? 2 : 3);
}

// rD: 1 / D, or 0 where D == 0 (it has D's sign).  Written without branches
// (bitwise on the comparisons), so the four faces' tests are plain compares
// rather than divergent blocks that each wait for their own LDS operands.
__device__ __forceinline__ bool face_inside(float N0, float N1, float N2, float rD) {
  const bool up = (N0 >= 0.0f) & (N1 >= 0.0f) & (N2 >= 0.0f);
  const bool down = (N0 <= 0.0f) & (N1 <= 0.0f) & (N2 <= 0.0f);
  return ((rD > 0.0f) & up) | ((rD < 0.0f) & down);
}

// One pixel centre against one record.  For a projected face (A,B,C) the
// rows of the inverse barycentric system times [p;1] (App. A.1) are
// N = (cross(B',C'), cross(C',A'), cross(A',B')) over D, with X' = X - p;
// the pixel is inside iff the three N have the sign of D (D == 0: never).
// The six edge cross products e_ij = cross(P_i - p, P_j - p) give every N
// exactly (a swapped pair is an exact negation).  Along the ray, with
// w_k = 1/Z_k (App. A.2):  f = sum N_k w_k f_k / sum N_k w_k,
// 1/z = sum N_k w_k / D.  Entry = nearest hit face, exit = farthest; the
// interpolated f is divided out for those two faces only.
struct PixEval {
  float ax[4], ay[4];
  float N[4][3];
  float S[4];
  float fin, fout; // f at the entry / exit face
  int fe, fx;      // entry / exit face
  float zin_inv;   // 1 / depth where the ray enters (entry face); larger is nearer
  float alpha;     // Eq. 1 (unclamped)
  float e1, e2;    // expm1(-s d), exp(s f_next) (for the derivative)
};

// Image planes and scene arrays are reached through pointers read from a
// descriptor, which the compiler treats as generic (flat) addresses.  A flat load also
// counts against the LDS wait counter, so every LDS wait after it waits for
// the load too; through a global-space pointer it does not.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// A tet's four vertex ids through a global-space pointer.
__device__ __forceinline__ int4 load_tet(const int32_t* tets, size_t k) {
  const auto* t = gmem(tets) + 4 * k;
  return make_int4(t[0], t[1], t[2], t[3]);
}

// Float atomic add to device memory through a global-space pointer (for a
// pointer read from a descriptor; see gmem).
__device__ __forceinline__ void gatomic_add(float* p, float v) {
  __hip_atomic_fetch_add(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A wave-uniform float moved into a scalar register: its load is waited for
// here, once, and not at its first use inside a loop, where the wait would
// also cover every load the loop's prefetch has in flight.
__device__ __forceinline__ float uniform_f(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// exp(x) from the hardware base-2 exponential
__device__ __forceinline__ float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }

// expm1(x) for x <= 0: Taylor series through x^7/5040 on [-0.25, 0] (truncation
// below 1e-9 relative), exp(x) - 1 below (no cancellation there).
__device__ __forceinline__ float fast_expm1_neg(float x) {
  float p = fmaf(x, 1.0f / 5040.0f, 1.0f / 720.0f);
  p = fmaf(x, p, 1.0f / 120.0f);
  p = fmaf(x, p, 1.0f / 24.0f);
  p = fmaf(x, p, 1.0f / 6.0f);
  p = fmaf(x, p, 0.5f);
  p = fmaf(x, p, 1.0f);
  const float small = x * p;
  const float big = fast_exp(x) - 1.0f;
  return x > -0.25f ? small : big;
}

__device__ __forceinline__ bool pixel_eval(const ViewRec& r, float qx, float qy, float s, PixEval& h) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    h.ax[k] = r.px[k] - qx;
    h.ay[k] = r.py[k] - qy;
  }
  const float e01 = h.ax[0] * h.ay[1] - h.ay[0] * h.ax[1];
  const float e02 = h.ax[0] * h.ay[2] - h.ay[0] * h.ax[2];
  const float e03 = h.ax[0] * h.ay[3] - h.ay[0] * h.ax[3];
  const float e12 = h.ax[1] * h.ay[2] - h.ay[1] * h.ax[2];
  const float e13 = h.ax[1] * h.ay[3] - h.ay[1] * h.ax[3];
  const float e23 = h.ax[2] * h.ay[3] - h.ay[2] * h.ax[3];
  h.N[0][0] = e12; h.N[0][1] = -e02; h.N[0][2] = e01;
  h.N[1][0] = e13; h.N[1][1] = -e03; h.N[1][2] = e01;
  h.N[2][0] = e23; h.N[2][1] = -e03; h.N[2][2] = e02;
  h.N[3][0] = e23; h.N[3][1] = -e13; h.N[3][2] = e12;
  // every face is evaluated (no branches); only inside faces are selected
  int nh = 0;
  float best_in = -INFINITY, best_out = INFINITY;
  float num_in = 0.0f, S_in = 1.0f, num_out = 0.0f, S_out = 1.0f;
  h.fe = 0;
  h.fx = 0;
#pragma unroll
  for (int F = 0; F < 4; ++F) {
    const bool in = face_inside(h.N[F][0], h.N[F][1], h.N[F][2], r.rD[F]);
    const int A = face_vertex(F, 0), B = face_vertex(F, 1), C = face_vertex(F, 2);
    const float qa = h.N[F][0] * r.iz[A], qb = h.N[F][1] * r.iz[B], qc = h.N[F][2] * r.iz[C];
    const float S = (qa + qb) + qc;
    const float num = fmaf(qa, r.f[A], fmaf(qb, r.f[B], qc * r.f[C]));
    const float invz = S * r.rD[F];  // 1 / depth at the hit: larger is nearer
    h.S[F] = S;
    nh += in ? 1 : 0;
    const bool bi = in && invz > best_in, bo = in && invz < best_out;
    best_in = bi ? invz : best_in;
    num_in = bi ? num : num_in;
    S_in = bi ? S : S_in;
    h.fe = bi ? F : h.fe;
    best_out = bo ? invz : best_out;
    num_out = bo ? num : num_out;
    S_out = bo ? S : S_out;
    h.fx = bo ? F : h.fx;
  }
  const float fin = num_in * rcp(S_in), fout = num_out * rcp(S_out);
  h.fin = fin;
  h.fout = fout;
  h.zin_inv = best_in;
  // Eq. 1, stable form, with the hardware exponential
  const float d = fin - fout;
  const bool pos = d > 0.0f;
  const float x = pos ? -(s * d) : 0.0f;
  h.e1 = fast_expm1_neg(x);
  h.e2 = pos ? fast_exp(s * fout) : 0.0f;
  h.alpha = pos ? -h.e1 * rcp(1.0f + h.e2) : 0.0f;
  return nh >= 2;
}

__device__ __forceinline__ void unpack_rect(const ViewRec& r, int& i0, int& i1, int& j0, int& j1) {
  i0 = (int)(r.rx & 0xffffu);
  i1 = (int)(r.rx >> 16);
  j0 = (int)(r.ry & 0xffffu);
  j1 = (int)(r.ry >> 16);
}

// Dispatch-order bucket of a list length: 0 for an empty list, then four
// buckets per power of two.
__device__ __forceinline__ int len_bucket(uint32_t len) {
  if (len == 0) return 0;
  const int b = 31 - __clz(len);  // floor(log2 len)
  const int sub = b >= 2 ? (int)((len >> (b - 2)) & 3u) : (b == 1 ? (int)((len & 1u) << 1) : 0);
  return 1 + 4 * b + sub;
}

// ---------------------------------------------------------------------------
// Reverse mode of one (pixel, record) pair: the pixel's blend weight w and
// dL/dalpha are chained to the record's 23 screen-space parameters.
// ---------------------------------------------------------------------------
// d f(face F) / d(record parameters) times df, added to g.  F is a
// compile-time constant, so every index is static; the face's values (S, f)
// are recomputed from its cross products N.
// f = sum N_k w_k f_k / S, S = sum N_k w_k.
template <int F, bool ZERO_SAFE = false>
__device__ __forceinline__ void face_geom_grad(const ViewRec& R, const float (&ax)[4], const float (&ay)[4],
                                               float N0, float N1, float N2, float df, float (&g)[32]) {
  constexpr int A = face_vertex(F, 0), B = face_vertex(F, 1), C = face_vertex(F, 2);
  constexpr int I[3] = {A, B, C};
  const float N[3] = {N0, N1, N2};
  const float qa = N0 * R.iz[A], qb = N1 * R.iz[B], qc = N2 * R.iz[C];
  const float S = (qa + qb) + qc;
  const float invS = ZERO_SAFE ? (df != 0.0f ? rcp(S) : 0.0f) : rcp(S);
  const float fF = fmaf(qa, R.f[A], fmaf(qb, R.f[B], qc * R.f[C])) * invS;
  float a[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int v = I[k];
    const float wk = R.iz[v];
    const float diff = (R.f[v] - fF) * invS * df;
    g[G_F + v] = fmaf(N[k] * wk * invS, df, g[G_F + v]);   // d/df_k
    g[G_IZ + v] = fmaf(N[k], diff, g[G_IZ + v]);            // d/dw_k
    a[k] = wk * diff;                                       // d/dN_k
  }
  const float Ax = ax[A], Ay = ay[A], Bx = ax[B], By = ay[B], Cx = ax[C], Cy = ay[C];
  // N0 = cross(B', C'), N1 = cross(C', A'), N2 = cross(A', B')
  g[G_PX + A] += a[2] * By - a[1] * Cy;
  g[G_PY + A] += a[1] * Cx - a[2] * Bx;
  g[G_PX + B] += a[0] * Cy - a[2] * Ay;
  g[G_PY + B] += a[2] * Ax - a[0] * Cx;
  g[G_PX + C] += a[1] * Ay - a[0] * By;
  g[G_PY + C] += a[0] * Bx - a[1] * Ax;
}

// dL/dalpha of a pair chained through Eq. 1 (stable form) to its entry and
// exit SDF values: alpha = A / B, A = -expm1(-s d), B = 1 + exp(s f_next),
// d = f_prev - f_next; e2 = exp(s f_next).  Zero when alpha is zero (the
// max(., 0) of Eq. 1).
__device__ __forceinline__ void eq1_chain(float da, float alpha, float e2, float s, float& dd, float& dfn) {
  const bool on = da != 0.0f && alpha > 0.0f;
  const float B = 1.0f + e2;
  const float invB = rcp(B);
  const float e1p1 = 1.0f - alpha * B;                   // exp(-s d) = 1 + expm1(-s d)
  const float dA = da * invB;
  const float dB = -da * alpha * invB;
  const float ddv = dA * s * e1p1;                       // d/df_prev
  dd = on ? ddv : 0.0f;
  dfn = on ? dB * s * e2 - ddv : 0.0f;                   // d/df_next
}

// g <- the pair's gradient with respect to the record's 23 screen-space
// parameters, given the blend weight w = T alpha (colour, depth and normal
// enter linearly), dL/df_prev = dd and dL/df_next = dfn, and the entry/exit
// faces fs = fe | fx << 2.  Without branches: all four faces are chained, a
// face whose weight is zero contributes exactly zero (its 1/S is taken as 0),
// so g is updated in place and a lane with w = dd = dfn = 0 returns zeros.
// With ACC the pair's gradient is added to g instead.
template <bool ACC = false>
__device__ __forceinline__ void pair_grad_all(const ViewRec& R, float qx, float qy, const float (&gr)[8], float dd,
                                              float dfn, float w, int fs, float (&g)[32]) {
  if (!ACC) {
#pragma unroll
    for (int q = 0; q < 32; ++q) g[q] = 0.0f;
  }
  g[G_C + 0] = fmaf(w, gr[0], g[G_C + 0]);
  g[G_C + 1] = fmaf(w, gr[1], g[G_C + 1]);
  g[G_C + 2] = fmaf(w, gr[2], g[G_C + 2]);
  g[G_ZT] = fmaf(w, gr[4], g[G_ZT]);
  g[G_N + 0] = fmaf(w, gr[5], g[G_N + 0]);
  g[G_N + 1] = fmaf(w, gr[6], g[G_N + 1]);
  g[G_N + 2] = fmaf(w, gr[7], g[G_N + 2]);
  const int fe = fs & 3, fx = fs >> 2;
  float ax[4], ay[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    ax[k] = R.px[k] - qx;
    ay[k] = R.py[k] - qy;
  }
  const float e01 = ax[0] * ay[1] - ay[0] * ax[1];
  const float e02 = ax[0] * ay[2] - ay[0] * ax[2];
  const float e03 = ax[0] * ay[3] - ay[0] * ax[3];
  const float e12 = ax[1] * ay[2] - ay[1] * ax[2];
  const float e13 = ax[1] * ay[3] - ay[1] * ax[3];
  const float e23 = ax[2] * ay[3] - ay[2] * ax[3];
  const float w0 = (fe == 0 ? dd : 0.0f) + (fx == 0 ? dfn : 0.0f);
  const float w1 = (fe == 1 ? dd : 0.0f) + (fx == 1 ? dfn : 0.0f);
  const float w2 = (fe == 2 ? dd : 0.0f) + (fx == 2 ? dfn : 0.0f);
  const float w3 = (fe == 3 ? dd : 0.0f) + (fx == 3 ? dfn : 0.0f);
  face_geom_grad<0, true>(R, ax, ay, e12, -e02, e01, w0, g);
  face_geom_grad<1, true>(R, ax, ay, e13, -e03, e01, w1, g);
  face_geom_grad<2, true>(R, ax, ay, e23, -e03, e02, w2, g);
  face_geom_grad<3, true>(R, ax, ay, e23, -e13, e12, w3, g);
}

// ---------------------------------------------------------------------------
// Transpose of the 64 x 64 bit matrix whose row r is lane r's word: bit c of
// lane r becomes bit r of lane c.  Six butterfly steps; at step j, lanes r
// and r ^ j exchange the j-wide column blocks that the transpose swaps.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t x) {
  constexpr uint64_t M[6] = {0x00000000ffffffffull, 0x0000ffff0000ffffull, 0x00ff00ff00ff00ffull,
                             0x0f0f0f0f0f0f0f0full, 0x3333333333333333ull, 0x5555555555555555ull};
  const unsigned lane = __lane_id();
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int j = 32 >> s;
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, j, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), j, 64);
    const uint64_t y = ((uint64_t)hi << 32) | lo;
    x = (lane & (unsigned)j) ? (x & ~M[s]) | ((y & ~M[s]) >> j) : (x & M[s]) | ((y & M[s]) << j);
  }
  return x;
}

// ---------------------------------------------------------------------------
// wave-wide transposed sum of 32 per-lane values (gfx950 permlane swaps and
// DPP): afterwards lane L holds the sum over all 64 lanes of v[L >> 1].
// Each step halves the values per lane while pairing lanes across a 32-,
// 16-, 8-, 4-, 2- and 1-lane distance: 16+8 swaps, 4+2+1 DPP-fused adds.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}

__device__ __forceinline__ float wave_transpose_sum32(const float (&v)[32]) {
  float u[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[k]), __float_as_uint(v[k + 16]), false, false);
    u[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  float w[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(u[k]), __float_as_uint(u[k + 8]), false, false);
    w[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  const unsigned lane = __lane_id();
  const bool b3 = lane & 8u, b2 = lane & 4u, b1 = lane & 2u;
  float x[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float send = b3 ? w[k] : w[k + 4];
    const float keep = b3 ? w[k + 4] : w[k];
    x[k] = keep + dpp<0x128>(send);   // row_ror:8  (lane j <-> j ^ 8)
  }
  float y[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float send = b2 ? x[k] : x[k + 2];
    const float keep = b2 ? x[k + 2] : x[k];
    y[k] = keep + dpp<0x141>(send);   // row_half_mirror (j <-> 7 - j)
  }
  const float send = b1 ? y[0] : y[1];
  const float keep = b1 ? y[1] : y[0];
  float z = keep + dpp<0x4E>(send);   // quad_perm [2,3,0,1]
  z = z + dpp<0xB1>(z);               // quad_perm [1,0,3,2]
  return z;
}


// Per 8-lane group (half of a DPP row): afterwards lane L of a group holds,
// in .x .. .w, the sums over the group's 8 lanes of v[4 (L & 7)] ..
// v[4 (L & 7) + 3].  Each step halves the values per lane while pairing
// lanes mirrored in the half-row, 2 apart and 1 apart.  Every lane must be
// active.
__device__ __forceinline__ float4 row8_transpose_sum32(const float (&v)[32]) {
  const unsigned lane = __lane_id();
  const bool b2 = lane & 4u, b1 = lane & 2u, b0 = lane & 1u;
  float x[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float send = b2 ? v[k] : v[k + 16];
    const float keep = b2 ? v[k + 16] : v[k];
    x[k] = keep + dpp<0x141>(send);   // row_half_mirror (j <-> 7 - j in each half-row)
  }
  float y[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float send = b1 ? x[k] : x[k + 8];
    const float keep = b1 ? x[k + 8] : x[k];
    y[k] = keep + dpp<0x4E>(send);    // quad_perm [2,3,0,1] (j <-> j ^ 2)
  }
  float z[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float send = b0 ? y[k] : y[k + 4];
    const float keep = b0 ? y[k + 4] : y[k];
    z[k] = keep + dpp<0xB1>(send);    // quad_perm [1,0,3,2] (j <-> j ^ 1)
  }
  return make_float4(z[0], z[1], z[2], z[3]);
}

// Per 4-lane group (a quad): afterwards lane L of a group holds in r[0..7]
// the sums over the quad's lanes of v[8 (L & 3)] .. v[8 (L & 3) + 7].  Each
// step halves the values per lane while pairing lanes 2 apart, then 1 apart.
// Every lane must be active.
__device__ __forceinline__ void quad_transpose_sum32(const float (&v)[32], float (&r)[8]) {
  const unsigned lane = __lane_id();
  const bool b1 = lane & 2u, b0 = lane & 1u;
  float x[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float send = b1 ? v[k] : v[k + 16];
    const float keep = b1 ? v[k + 16] : v[k];
    x[k] = keep + dpp<0x4E>(send);    // quad_perm [2,3,0,1] (j <-> j ^ 2)
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float send = b0 ? x[k] : x[k + 8];
    const float keep = b0 ? x[k + 8] : x[k];
    r[k] = keep + dpp<0xB1>(send);    // quad_perm [1,0,3,2] (j <-> j ^ 1)
  }
}

}  // namespace ts
