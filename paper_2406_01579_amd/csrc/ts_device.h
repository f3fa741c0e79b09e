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

// Eq. 1 in the stable form alpha = -expm1(-s d) / (1 + exp(s f_next)),
// d = f_prev - f_next; zero unless d > 0 (the max(., 0) of Eq. 1).
__device__ __forceinline__ float alpha_eq1(float fprev, float fnext, float s) {
  float d = fprev - fnext;
  if (!(d > 0.0f)) return 0.0f;
  return -expm1f(-(s * d)) / (1.0f + expf(s * fnext));
}

// Coverage and entry/exit of one pixel centre (qx, qy) against one record.
// The inside test of each projected face uses the sign of the three 2D
// cross products N_k (rows of the inverse barycentric system times [p;1],
// App. A.1) against the sign of the face determinant D; a face with D == 0
// never contains the pixel.  Values along the ray use the perspective-
// correct barycentrics of App. A.2: with w_k = 1/Z_k,
//   f = sum N_k w_k f_k / sum N_k w_k,   1/z = sum N_k w_k / D.
struct FaceSel {
  int face;        // 0..3
  float N[3];
  float S;         // sum N_k w_k
  float f;         // SDF at the hit point
};

// face vertex table: (0,1,2) (0,1,3) (0,2,3) (1,2,3)
__device__ __forceinline__ int face_vertex(int F, int k) {
  // packed 2 bits per entry
  const uint32_t tbl = (0u << 0) | (1u << 2) | (2u << 4) |     // face 0
                       (0u << 6) | (1u << 8) | (3u << 10) |    // face 1
                       (0u << 12) | (2u << 14) | (3u << 16) |  // face 2
                       (1u << 18) | (2u << 20) | (3u << 22);   // face 3
  return (tbl >> (2 * (3 * F + k))) & 3u;
}

struct PixHit {
  FaceSel in, out;
  float alpha;
  float ax[4], ay[4];  // projected vertex minus pixel centre
};

__device__ __forceinline__ bool face_inside(float N0, float N1, float N2, float D) {
  if (D > 0.0f) return N0 >= 0.0f && N1 >= 0.0f && N2 >= 0.0f;
  if (D < 0.0f) return N0 <= 0.0f && N1 <= 0.0f && N2 <= 0.0f;
  return false;
}

// Returns true if at least two faces contain the pixel centre; fills h.
__device__ __forceinline__ bool pixel_hit(const ViewRec& r, float qx, float qy, float s, PixHit& h) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    h.ax[k] = r.px[k] - qx;
    h.ay[k] = r.py[k] - qy;
  }
  // e_ij = cross(P_i - q, P_j - q)
  const float e01 = h.ax[0] * h.ay[1] - h.ay[0] * h.ax[1];
  const float e02 = h.ax[0] * h.ay[2] - h.ay[0] * h.ax[2];
  const float e03 = h.ax[0] * h.ay[3] - h.ay[0] * h.ax[3];
  const float e12 = h.ax[1] * h.ay[2] - h.ay[1] * h.ax[2];
  const float e13 = h.ax[1] * h.ay[3] - h.ay[1] * h.ax[3];
  const float e23 = h.ax[2] * h.ay[3] - h.ay[2] * h.ax[3];
  // (N0, N1, N2) of face (A,B,C) = (cross(B',C'), cross(C',A'), cross(A',B'))
  float N[4][3] = {{e12, -e02, e01}, {e13, -e03, e01}, {e23, -e03, e02}, {e23, -e13, e12}};
  int nh = 0;
  float best_in = -INFINITY, best_out = INFINITY;
#pragma unroll
  for (int F = 0; F < 4; ++F) {
    if (!face_inside(N[F][0], N[F][1], N[F][2], r.D[F])) continue;
    ++nh;
    const int A = face_vertex(F, 0), B = face_vertex(F, 1), C = face_vertex(F, 2);
    const float qa = N[F][0] * r.iz[A], qb = N[F][1] * r.iz[B], qc = N[F][2] * r.iz[C];
    const float S = (qa + qb) + qc;
    const float num = fmaf(qa, r.f[A], fmaf(qb, r.f[B], qc * r.f[C]));
    const float f = num / S;
    const float invz = S / r.D[F];  // 1 / depth at the hit: larger is nearer
    if (invz > best_in) {
      best_in = invz;
      h.in.face = F; h.in.N[0] = N[F][0]; h.in.N[1] = N[F][1]; h.in.N[2] = N[F][2]; h.in.S = S; h.in.f = f;
    }
    if (invz < best_out) {
      best_out = invz;
      h.out.face = F; h.out.N[0] = N[F][0]; h.out.N[1] = N[F][1]; h.out.N[2] = N[F][2]; h.out.S = S; h.out.f = f;
    }
  }
  if (nh < 2) return false;
  h.alpha = alpha_eq1(h.in.f, h.out.f, s);
  return true;
}

__device__ __forceinline__ void unpack_rect(const ViewRec& r, int& i0, int& i1, int& j0, int& j1) {
  i0 = (int)(r.rx & 0xffffu);
  i1 = (int)(r.rx >> 16);
  j0 = (int)(r.ry & 0xffffu);
  j1 = (int)(r.ry >> 16);
}

}  // namespace ts
