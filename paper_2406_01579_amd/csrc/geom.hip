// Geometry regularisers of Sec. 4.2 on the deformable tet grid, for gfx950.
//
//  * eikonal term  L_eik = sum_k (|g_k| - 1)^2 over the tets, g_k the SDF
//    gradient inside tet k (App. A.3, as the 3x3 edge system g = E^-1 df);
//  * normal-consistency term  L_nc = sum_e (1 - cos(m_a, m_b)) over the
//    unique edges (a, b), m_v = sum of the unit normals g_k/|g_k| of the tets
//    around vertex v.
//
// Three grid-stride passes: per tet (g, the eikonal partial sums, scatter of
// n_k into m), per edge (the consistency term and dL/dm), per tet again
// (g recomputed; dL/dg from both terms chained to the four SDF values and
// vertex positions).  1 - cos is evaluated as |u_a - u_b|^2 / 2 on the unit
// vectors, which has no cancellation for nearly parallel normals.  Loss
// partial sums are per block in a fixed order and summed in double by one
// block, so the losses do not depend on scheduling except through the float
// atomics that build m.
//
// The unique-edge list is built once per topology: the six (a < b) pairs of
// every tet are sorted by b and then stably by a with the LSD radix sort, and
// a flag/scan/scatter pass keeps the first of each run.
//
// Marching Tetrahedra (the mesh extraction of Sec. 4.1): a flag/scan/scatter
// pass over the edges places one surface vertex on every edge whose ends
// differ in the inside test (f < 0), numbered in edge order; a second one
// over the tets writes one triangle (one or three inside vertices) or two
// (two inside) in tet order, looking the crossed edges up in the sorted edge
// list by binary search.  The winding is fixed by a 16-entry case table built
// at compile time (outward normals, flipped for negatively oriented tets).
#include <algorithm>

#include "ts_device.h"

namespace ts {
namespace {

constexpr int RT = 256;
constexpr int RBLOCKS = 1024;
constexpr int EDGE_ITEMS = 8;
constexpr int EDGE_TILE = RT * EDGE_ITEMS;

__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t* lds /*[RT/64]*/, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wave] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < RT / 64; ++w) {
    const uint32_t t = lds[w];
    if (w < wave) base += t;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

__device__ __forceinline__ float block_sum(float v, float* lds /*[RT/64]*/) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  float s = 0.0f;
#pragma unroll
  for (int w = 0; w < RT / 64; ++w) s += lds[w];
  __syncthreads();
  return s;
}

__device__ __forceinline__ bool load_tet(const int32_t* tets, uint32_t k, int32_t V, int32_t (&v)[4]) {
  const int4 t = reinterpret_cast<const int4*>(tets)[k];
  v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  return (uint32_t)t.x < (uint32_t)V && (uint32_t)t.y < (uint32_t)V && (uint32_t)t.z < (uint32_t)V &&
         (uint32_t)t.w < (uint32_t)V;
}

// the (a < b) vertex pair of local edge e of tet k; (V, V) for a tet with an
// index outside [0, V)
__device__ __forceinline__ void pair_of(const int32_t* tets, uint32_t i, int32_t V, uint32_t& a, uint32_t& b) {
  const uint32_t k = i / 6, e = i - 6 * k;
  int32_t v[4];
  if (!load_tet(tets, k, V, v)) {
    a = b = (uint32_t)V;
    return;
  }
  // local pairs (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
  const int32_t p = e < 3 ? v[0] : (e < 5 ? v[1] : v[2]);
  const int32_t q = e == 0 ? v[1] : (e == 1 || e == 3) ? v[2] : v[3];
  a = (uint32_t)min(p, q);
  b = (uint32_t)max(p, q);
}

// SDF gradient of the linear interpolant over the tet: E g = df with rows
// e_a = x_{a+1} - x_0, df_a = f_{a+1} - f_0; cr[a] is column a of det * E^-1
struct TetGrad {
  float x[4][3], f[4];
  float cr[3][3];
  float det;
  float g[3];
};

__device__ __forceinline__ void tet_grad(const float* verts, const float* sdf, const int32_t (&v)[4], TetGrad& T) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int m = 0; m < 3; ++m) T.x[a][m] = verts[3 * (size_t)v[a] + m];
    T.f[a] = sdf[v[a]];
  }
  float e[3][3], df[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int m = 0; m < 3; ++m) e[a][m] = T.x[a + 1][m] - T.x[0][m];
    df[a] = T.f[a + 1] - T.f[0];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    T.cr[a][0] = e[b][1] * e[c][2] - e[b][2] * e[c][1];
    T.cr[a][1] = e[b][2] * e[c][0] - e[b][0] * e[c][2];
    T.cr[a][2] = e[b][0] * e[c][1] - e[b][1] * e[c][0];
  }
  T.det = e[0][0] * T.cr[0][0] + e[0][1] * T.cr[0][1] + e[0][2] * T.cr[0][2];
#pragma unroll
  for (int m = 0; m < 3; ++m)
    T.g[m] = T.det != 0.0f ? (T.cr[0][m] * df[0] + T.cr[1][m] * df[1] + T.cr[2][m] * df[2]) / T.det : 0.0f;
}

// ---------------------------------------------------------------------------
// unique edges
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RT) void k_edge_keys_b(const int32_t* tets, uint32_t n, int32_t V, uint32_t* keyb,
                                                    uint32_t* n_dev) {
  if (blockIdx.x == 0 && threadIdx.x == 0) n_dev[0] = n;
  for (uint32_t i = blockIdx.x * RT + threadIdx.x; i < n; i += gridDim.x * RT) {
    uint32_t a, b;
    pair_of(tets, i, V, a, b);
    keyb[i] = b;
  }
}

__global__ __launch_bounds__(RT) void k_edge_keys_a(const int32_t* tets, uint32_t n, int32_t V, const uint32_t* idx,
                                                    uint32_t* keya) {
  for (uint32_t j = blockIdx.x * RT + threadIdx.x; j < n; j += gridDim.x * RT) {
    uint32_t a, b;
    pair_of(tets, idx[j], V, a, b);
    keya[j] = a;
  }
}

// flag = first of its run of equal pairs, and a real edge
__device__ __forceinline__ uint32_t edge_flags(const int32_t* tets, uint32_t n, int32_t V, const uint32_t* idx,
                                               uint32_t j0, uint32_t (&ab)[EDGE_ITEMS][2]) {
  uint32_t bits = 0;
  uint32_t pa = 0xffffffffu, pb = 0xffffffffu;
  if (j0 > 0 && j0 - 1 < n) pair_of(tets, idx[j0 - 1], V, pa, pb);
#pragma unroll
  for (int t = 0; t < EDGE_ITEMS; ++t) {
    const uint32_t j = j0 + t;
    uint32_t a = (uint32_t)V, b = (uint32_t)V;
    if (j < n) pair_of(tets, idx[j], V, a, b);
    ab[t][0] = a;
    ab[t][1] = b;
    if (j < n && a < (uint32_t)V && (a != pa || b != pb)) bits |= 1u << t;
    pa = a;
    pb = b;
  }
  return bits;
}

__global__ __launch_bounds__(RT) void k_edge_count(const int32_t* tets, uint32_t n, int32_t V, const uint32_t* idx,
                                                   uint32_t* bsum) {
  __shared__ uint32_t lds[RT / 64];
  uint32_t ab[EDGE_ITEMS][2];
  const uint32_t j0 = blockIdx.x * EDGE_TILE + threadIdx.x * EDGE_ITEMS;
  const uint32_t c = __popc(edge_flags(tets, n, V, idx, j0, ab));
  uint32_t tot;
  block_scan_excl(c, lds, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_edge_spine(uint32_t* bsum, uint32_t nb, int32_t* n_edges) {
  __shared__ uint32_t part[16];
  const uint32_t t = threadIdx.x;
  const uint32_t per = (nb + 1023) / 1024;
  const uint32_t lo = min(nb, t * per), hi = min(nb, (t + 1) * per);
  uint32_t s = 0;
  for (uint32_t i = lo; i < hi; ++i) s += bsum[i];
  const int lane = t & 63, wave = t >> 6;
  uint32_t x = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) part[wave] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int w = 0; w < 16; ++w) {
    if (w < wave) base += part[w];
    tot += part[w];
  }
  uint32_t run = base + x - s;
  for (uint32_t i = lo; i < hi; ++i) {
    const uint32_t c = bsum[i];
    bsum[i] = run;
    run += c;
  }
  if (t == 0) n_edges[0] = (int32_t)tot;
}

__global__ __launch_bounds__(RT) void k_edge_write(const int32_t* tets, uint32_t n, int32_t V, const uint32_t* idx,
                                                   const uint32_t* bsum, int32_t* edges) {
  __shared__ uint32_t lds[RT / 64];
  uint32_t ab[EDGE_ITEMS][2];
  const uint32_t j0 = blockIdx.x * EDGE_TILE + threadIdx.x * EDGE_ITEMS;
  const uint32_t bits = edge_flags(tets, n, V, idx, j0, ab);
  uint32_t tot;
  uint32_t o = bsum[blockIdx.x] + block_scan_excl(__popc(bits), lds, &tot);
#pragma unroll
  for (int t = 0; t < EDGE_ITEMS; ++t) {
    if (bits & (1u << t)) {
      reinterpret_cast<int2*>(edges)[o] = make_int2((int32_t)ab[t][0], (int32_t)ab[t][1]);
      ++o;
    }
  }
}

// ---------------------------------------------------------------------------
// regularisers
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RT) void k_fill_f32(float* p, size_t n, float v) {
  for (size_t i = blockIdx.x * (size_t)RT + threadIdx.x; i < n; i += (size_t)gridDim.x * RT) p[i] = v;
}

__global__ __launch_bounds__(RT) void k_reg_tet_fwd(const float* verts, const int32_t* tets, const float* sdf,
                                                    int32_t V, uint32_t K, float* m, float* part) {
  __shared__ float lds[RT / 64];
  float eik = 0.0f;
  for (uint32_t k = blockIdx.x * RT + threadIdx.x; k < K; k += gridDim.x * RT) {
    int32_t v[4];
    if (!load_tet(tets, k, V, v)) continue;
    TetGrad T;
    tet_grad(verts, sdf, v, T);
    if (T.det == 0.0f) continue;
    const float gn = sqrtf(T.g[0] * T.g[0] + T.g[1] * T.g[1] + T.g[2] * T.g[2]);
    eik += (gn - 1.0f) * (gn - 1.0f);
    if (gn > 0.0f && m) {
      const float ig = 1.0f / gn;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) unsafeAtomicAdd(&m[3 * (size_t)v[a] + c], T.g[c] * ig);
    }
  }
  const float s = block_sum(eik, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(RT) void k_reg_edge(const int32_t* edges, const int32_t* n_edges, uint32_t cap,
                                                 int32_t V, const float* m, float* dm, const float* w, float* part) {
  __shared__ float lds[RT / 64];
  const uint32_t ne = min((uint32_t)max(n_edges[0], 0), cap);
  const float wnc = dm ? w[1] : 0.0f;
  float nc = 0.0f;
  for (uint32_t e = blockIdx.x * RT + threadIdx.x; e < ne; e += gridDim.x * RT) {
    const int2 ab = reinterpret_cast<const int2*>(edges)[e];
    if ((uint32_t)ab.x >= (uint32_t)V || (uint32_t)ab.y >= (uint32_t)V) continue;
    float ma[3], mb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ma[c] = m[3 * (size_t)ab.x + c];
      mb[c] = m[3 * (size_t)ab.y + c];
    }
    const float la = sqrtf(ma[0] * ma[0] + ma[1] * ma[1] + ma[2] * ma[2]);
    const float lb = sqrtf(mb[0] * mb[0] + mb[1] * mb[1] + mb[2] * mb[2]);
    if (!(la > 0.0f && lb > 0.0f)) continue;
    const float ia = 1.0f / la, ib = 1.0f / lb;
    float ua[3], ub[3], d[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ua[c] = ma[c] * ia;
      ub[c] = mb[c] * ib;
      d[c] = ub[c] - ua[c];
    }
    // 1 - cos = |u_b - u_a|^2 / 2
    const float t = 0.5f * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    nc += t;
    if (dm) {
      // d(1 - ua.ub)/dm_a = -(ub - cos ua)/|m_a| = -(d + t ua)/|m_a|, and symmetrically for b
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        unsafeAtomicAdd(&dm[3 * (size_t)ab.x + c], -wnc * (d[c] + t * ua[c]) * ia);
        unsafeAtomicAdd(&dm[3 * (size_t)ab.y + c], -wnc * (-d[c] + t * ub[c]) * ib);
      }
    }
  }
  const float s = block_sum(nc, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(RT) void k_reg_tet_bwd(const float* verts, const int32_t* tets, const float* sdf,
                                                    int32_t V, uint32_t K, const float* dm, const float* w,
                                                    float* dverts, float* dsdf) {
  const float weik = w[0];
  for (uint32_t k = blockIdx.x * RT + threadIdx.x; k < K; k += gridDim.x * RT) {
    int32_t v[4];
    if (!load_tet(tets, k, V, v)) continue;
    TetGrad T;
    tet_grad(verts, sdf, v, T);
    if (T.det == 0.0f) continue;
    const float gn = sqrtf(T.g[0] * T.g[0] + T.g[1] * T.g[1] + T.g[2] * T.g[2]);
    if (!(gn > 0.0f)) continue;
    const float ig = 1.0f / gn;
    float n[3], dn[3] = {0.0f, 0.0f, 0.0f}, dg[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) n[c] = T.g[c] * ig;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) dn[c] += dm[3 * (size_t)v[a] + c];
    const float nd = n[0] * dn[0] + n[1] * dn[1] + n[2] * dn[2];
    const float ke = weik * 2.0f * (gn - 1.0f);
#pragma unroll
    for (int c = 0; c < 3; ++c) dg[c] = ke * n[c] + (dn[c] - n[c] * nd) * ig;
    // g = E^-1 df: dL/ddf = E^-T dg = mu; dL/dE = -mu g^T
    float mu[3], msum = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      mu[a] = (T.cr[a][0] * dg[0] + T.cr[a][1] * dg[1] + T.cr[a][2] * dg[2]) / T.det;
      msum += mu[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      unsafeAtomicAdd(&dsdf[v[a + 1]], mu[a]);
#pragma unroll
      for (int c = 0; c < 3; ++c) unsafeAtomicAdd(&dverts[3 * (size_t)v[a + 1] + c], -mu[a] * T.g[c]);
    }
    unsafeAtomicAdd(&dsdf[v[0]], -msum);
#pragma unroll
    for (int c = 0; c < 3; ++c) unsafeAtomicAdd(&dverts[3 * (size_t)v[0] + c], msum * T.g[c]);
  }
}


// ---------------------------------------------------------------------------
// Marching Tetrahedra
// ---------------------------------------------------------------------------
struct MTCase {
  uint8_t ntri;   // 0, 1 or 2
  uint8_t o[4];   // local vertex order (i, j, k, l), an even permutation
  uint8_t rev;    // reverse the winding (lone outside vertex)
};
struct MTTable {
  MTCase c[16];
};

constexpr MTTable make_mt_table() {
  MTTable T{};
  for (int m = 0; m < 16; ++m) {
    const int cnt = (m & 1) + ((m >> 1) & 1) + ((m >> 2) & 1) + ((m >> 3) & 1);
    MTCase c{};
    int o[4] = {0, 1, 2, 3};
    int n = 0;
    if (cnt == 1 || cnt == 3) {
      const int want = cnt == 1 ? 1 : 0;
      for (int q = 0; q < 4; ++q)
        if (((m >> q) & 1) == want) o[n++] = q;
      for (int q = 0; q < 4; ++q)
        if (((m >> q) & 1) != want) o[n++] = q;
      c.ntri = 1;
      c.rev = cnt == 3;
    } else if (cnt == 2) {
      for (int q = 0; q < 4; ++q)
        if ((m >> q) & 1) o[n++] = q;
      for (int q = 0; q < 4; ++q)
        if (!((m >> q) & 1)) o[n++] = q;
      c.ntri = 2;
    }
    int inv = 0;
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b) inv += o[a] > o[b];
    if (inv & 1) {
      const int t = o[2];
      o[2] = o[3];
      o[3] = t;
    }
    for (int q = 0; q < 4; ++q) c.o[q] = (uint8_t)o[q];
    T.c[m] = c;
  }
  return T;
}
__constant__ MTTable c_mt = make_mt_table();

__global__ __launch_bounds__(RT) void k_mt_edge_pass(const float* verts, const float* sdf, int32_t V,
                                                     const int32_t* edges, const int32_t* n_edges, uint32_t cap,
                                                     uint32_t* bsum, int32_t* vid, float* out, uint32_t vcap,
                                                     int write) {
  __shared__ uint32_t lds[RT / 64];
  const uint32_t ne = min((uint32_t)max(n_edges[0], 0), cap);
  const uint32_t j0 = blockIdx.x * EDGE_TILE + threadIdx.x * EDGE_ITEMS;
  uint32_t bits = 0;
  int2 ab[EDGE_ITEMS];
#pragma unroll
  for (int t = 0; t < EDGE_ITEMS; ++t) {
    const uint32_t j = j0 + t;
    ab[t] = make_int2(-1, -1);
    if (j < ne) {
      const int2 e = reinterpret_cast<const int2*>(edges)[j];
      if ((uint32_t)e.x < (uint32_t)V && (uint32_t)e.y < (uint32_t)V) {
        ab[t] = e;
        if ((sdf[e.x] < 0.0f) != (sdf[e.y] < 0.0f)) bits |= 1u << t;
      }
    }
  }
  uint32_t tot;
  const uint32_t base = block_scan_excl(__popc(bits), lds, &tot);
  if (!write) {
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
    return;
  }
  uint32_t o = bsum[blockIdx.x] + base;
#pragma unroll
  for (int t = 0; t < EDGE_ITEMS; ++t) {
    const uint32_t j = j0 + t;
    if (j >= ne) continue;
    if (!(bits & (1u << t))) {
      vid[j] = -1;
      continue;
    }
    vid[j] = (int32_t)o;
    if (o < vcap) {
      const float fa = sdf[ab[t].x], fb = sdf[ab[t].y];
      const float tt = fa / (fa - fb);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float xa = verts[3 * (size_t)ab[t].x + c], xb = verts[3 * (size_t)ab[t].y + c];
        out[3 * (size_t)o + c] = xa + tt * (xb - xa);
      }
    }
    ++o;
  }
}

// index of edge (a, b) in the sorted list, -1 if absent
__device__ __forceinline__ int32_t find_edge(const int32_t* edges, uint32_t ne, int32_t a, int32_t b) {
  const int2* E = reinterpret_cast<const int2*>(edges);
  uint32_t lo = 0, hi = ne;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    const int2 e = E[mid];
    if (e.x < a || (e.x == a && e.y < b))
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < ne && E[lo].x == a && E[lo].y == b) ? (int32_t)lo : -1;
}

__device__ __forceinline__ int32_t surf_vertex(const int32_t* edges, uint32_t ne, const int32_t* vid, int32_t u,
                                               int32_t w) {
  const int32_t e = find_edge(edges, ne, min(u, w), max(u, w));
  return e < 0 ? -1 : vid[e];
}

__global__ __launch_bounds__(RT) void k_mt_tet_pass(const float* verts, const int32_t* tets, const float* sdf,
                                                    int32_t V, uint32_t K, const int32_t* edges,
                                                    const int32_t* n_edges, uint32_t cap, const int32_t* vid,
                                                    uint32_t* bsum, int32_t* tris, uint32_t tcap, int write) {
  __shared__ uint32_t lds[RT / 64];
  const uint32_t k0 = blockIdx.x * EDGE_TILE + threadIdx.x * EDGE_ITEMS;
  uint32_t mask[EDGE_ITEMS];
  uint32_t cnt = 0;
#pragma unroll
  for (int t = 0; t < EDGE_ITEMS; ++t) {
    const uint32_t k = k0 + t;
    mask[t] = 0;
    if (k < K) {
      int32_t v[4];
      if (load_tet(tets, k, V, v))
        mask[t] = (sdf[v[0]] < 0.0f ? 1u : 0u) | (sdf[v[1]] < 0.0f ? 2u : 0u) | (sdf[v[2]] < 0.0f ? 4u : 0u) |
                  (sdf[v[3]] < 0.0f ? 8u : 0u);
    }
    cnt += c_mt.c[mask[t]].ntri;
  }
  uint32_t tot;
  const uint32_t base = block_scan_excl(cnt, lds, &tot);
  if (!write) {
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
    return;
  }
  const uint32_t ne = min((uint32_t)max(n_edges[0], 0), cap);
  uint32_t o = bsum[blockIdx.x] + base;
#pragma unroll 1
  for (int t = 0; t < EDGE_ITEMS; ++t) {
    const MTCase c = c_mt.c[mask[t]];
    if (c.ntri == 0) continue;
    int32_t v[4];
    load_tet(tets, k0 + t, V, v);
    // orientation of the tet: sign of det[x1 - x0, x2 - x0, x3 - x0]
    float e[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int m = 0; m < 3; ++m) e[a][m] = verts[3 * (size_t)v[a + 1] + m] - verts[3 * (size_t)v[0] + m];
    const float det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) +
                      e[0][1] * (e[1][2] * e[2][0] - e[1][0] * e[2][2]) +
                      e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
    const bool flip = det < 0.0f;
    const int32_t i = v[c.o[0]], j = v[c.o[1]], kk = v[c.o[2]], l = v[c.o[3]];
    int32_t tri[2][3];
    if (c.ntri == 1) {
      tri[0][0] = surf_vertex(edges, ne, vid, i, j);
      tri[0][1] = surf_vertex(edges, ne, vid, i, kk);
      tri[0][2] = surf_vertex(edges, ne, vid, i, l);
    } else {
      const int32_t ik = surf_vertex(edges, ne, vid, i, kk), il = surf_vertex(edges, ne, vid, i, l);
      const int32_t jl = surf_vertex(edges, ne, vid, j, l), jk = surf_vertex(edges, ne, vid, j, kk);
      tri[0][0] = ik; tri[0][1] = il; tri[0][2] = jl;
      tri[1][0] = ik; tri[1][1] = jl; tri[1][2] = jk;
    }
    const bool rev = flip != (c.rev != 0);
    for (int q = 0; q < c.ntri; ++q, ++o) {
      if (o >= tcap) continue;
      tris[3 * (size_t)o + 0] = tri[q][0];
      tris[3 * (size_t)o + 1] = rev ? tri[q][2] : tri[q][1];
      tris[3 * (size_t)o + 2] = rev ? tri[q][1] : tri[q][2];
    }
  }
}

__global__ __launch_bounds__(RT) void k_reg_losses(const float* part, int nb, double* losses) {
  __shared__ double lds[2][RT / 64];
  double s0 = 0.0, s1 = 0.0;
  for (int i = threadIdx.x; i < nb; i += RT) {
    s0 += (double)part[i];
    s1 += (double)part[nb + i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o, 64);
    s1 += __shfl_xor(s1, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    lds[0][threadIdx.x >> 6] = s0;
    lds[1][threadIdx.x >> 6] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < RT / 64; ++w) {
      a += lds[0][w];
      b += lds[1][w];
    }
    losses[0] = a;
    losses[1] = b;
  }
}

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }
inline int bit_length(uint32_t x) { return x ? 32 - __builtin_clz(x) : 0; }

}  // namespace

// --- host side ------------------------------------------------------------------
EdgeLayout edge_layout(int32_t K) {
  EdgeLayout E{};
  const uint64_t n = 6ull * (uint64_t)K;
  E.n = n;
  E.sort_blocks = (n + SORT_TILE - 1) / SORT_TILE;
  E.edge_blocks = (n + EDGE_TILE - 1) / EDGE_TILE;
  size_t o = 0;
  E.o_n = o; o += al(16);
  E.o_ka = o; o += al(4 * n);
  E.o_va = o; o += al(4 * n);
  E.o_kb = o; o += al(4 * n);
  E.o_vb = o; o += al(4 * n);
  E.o_hist = o; o += al(4 * (256 * (size_t)E.sort_blocks + 256));
  E.o_bsum = o; o += al(4 * ((size_t)E.edge_blocks + 1));
  E.bytes = o;
  return E;
}

hipError_t launch_mesh_edges(const int32_t* tets, int32_t K, int32_t V, int32_t* edges, int32_t* n_edges, void* ws,
                             const EdgeLayout& E, hipStream_t st) {
  char* w = static_cast<char*>(ws);
  uint32_t* n_dev = reinterpret_cast<uint32_t*>(w + E.o_n);
  uint32_t* ka = reinterpret_cast<uint32_t*>(w + E.o_ka);
  uint32_t* va = reinterpret_cast<uint32_t*>(w + E.o_va);
  uint32_t* kb = reinterpret_cast<uint32_t*>(w + E.o_kb);
  uint32_t* vb = reinterpret_cast<uint32_t*>(w + E.o_vb);
  uint32_t* hist = reinterpret_cast<uint32_t*>(w + E.o_hist);
  uint32_t* bsum = reinterpret_cast<uint32_t*>(w + E.o_bsum);
  const uint32_t n = (uint32_t)E.n;
  const unsigned g = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + RT - 1) / RT, 4096));
  k_edge_keys_b<<<g, RT, 0, st>>>(tets, n, V, ka, n_dev);
  const int bits = std::max(1, bit_length((uint32_t)V));
  uint32_t *ko = nullptr, *vo = nullptr;
  hipError_t e = radix_sort_pairs(ka, va, kb, vb, true, n_dev, (int64_t)n, bits, hist, (int64_t)E.sort_blocks, st,
                                  &ko, &vo);
  if (e != hipSuccess) return e;
  // second pass keyed by a, carrying the pair indices sorted by b
  k_edge_keys_a<<<g, RT, 0, st>>>(tets, n, V, vo, ko);
  uint32_t* k2 = (ko == ka) ? kb : ka;
  uint32_t* v2 = (vo == va) ? vb : va;
  e = radix_sort_pairs(ko, vo, k2, v2, false, n_dev, (int64_t)n, bits, hist, (int64_t)E.sort_blocks, st, &ko, &vo);
  if (e != hipSuccess) return e;
  const unsigned nb = (unsigned)E.edge_blocks;
  if (nb > 0) k_edge_count<<<nb, RT, 0, st>>>(tets, n, V, vo, bsum);
  k_edge_spine<<<1, 1024, 0, st>>>(bsum, nb, n_edges);
  if (nb > 0) k_edge_write<<<nb, RT, 0, st>>>(tets, n, V, vo, bsum, edges);
  return hipGetLastError();
}

RegLayout reg_layout(int32_t V) {
  RegLayout R{};
  size_t o = 0;
  R.o_m = o; o += al(4 * 3 * (size_t)V);
  R.o_dm = o; o += al(4 * 3 * (size_t)V);
  R.o_part = o; o += al(4 * 2 * (size_t)RBLOCKS);
  R.bytes = o;
  R.blocks = RBLOCKS;
  return R;
}

hipError_t launch_regularizers(const float* verts, const int32_t* tets, const float* sdf, int32_t V, int32_t K,
                               const int32_t* edges, const int32_t* n_edges, int64_t edge_cap, const float* weights,
                               double* losses, float* dverts, float* dsdf, void* ws, const RegLayout& R,
                               hipStream_t st) {
  char* w = static_cast<char*>(ws);
  float* m = reinterpret_cast<float*>(w + R.o_m);
  float* dm = reinterpret_cast<float*>(w + R.o_dm);
  float* part = reinterpret_cast<float*>(w + R.o_part);
  const bool bwd = dverts != nullptr;
  const size_t nv3 = 3 * (size_t)V;
  const unsigned gf = (unsigned)std::max<size_t>(1, std::min<size_t>((nv3 + RT - 1) / RT, 2048));
  k_fill_f32<<<gf, RT, 0, st>>>(m, nv3, 0.0f);
  if (bwd) k_fill_f32<<<gf, RT, 0, st>>>(dm, nv3, 0.0f);
  k_reg_tet_fwd<<<R.blocks, RT, 0, st>>>(verts, tets, sdf, V, (uint32_t)K, m, part);
  k_reg_edge<<<R.blocks, RT, 0, st>>>(edges, n_edges, (uint32_t)edge_cap, V, m, bwd ? dm : nullptr, weights,
                                      part + R.blocks);
  if (bwd) k_reg_tet_bwd<<<R.blocks, RT, 0, st>>>(verts, tets, sdf, V, (uint32_t)K, dm, weights, dverts, dsdf);
  if (losses) k_reg_losses<<<1, RT, 0, st>>>(part, R.blocks, losses);
  return hipGetLastError();
}

MTLayout mt_layout(int32_t K, int64_t edge_cap) {
  MTLayout M{};
  M.edge_blocks = ((uint64_t)edge_cap + EDGE_TILE - 1) / EDGE_TILE;
  M.tet_blocks = ((uint64_t)K + EDGE_TILE - 1) / EDGE_TILE;
  size_t o = 0;
  M.o_vid = o; o += al(4 * (size_t)edge_cap);
  M.o_bsum_e = o; o += al(4 * ((size_t)M.edge_blocks + 1));
  M.o_bsum_t = o; o += al(4 * ((size_t)M.tet_blocks + 1));
  M.bytes = o;
  return M;
}

hipError_t launch_marching_tets(const float* verts, const int32_t* tets, const float* sdf, int32_t V, int32_t K,
                                const int32_t* edges, const int32_t* n_edges, int64_t edge_cap, float* out_verts,
                                int64_t vert_cap, int32_t* out_tris, int64_t tri_cap, int32_t* counts, void* ws,
                                const MTLayout& M, hipStream_t st) {
  char* w = static_cast<char*>(ws);
  int32_t* vid = reinterpret_cast<int32_t*>(w + M.o_vid);
  uint32_t* be = reinterpret_cast<uint32_t*>(w + M.o_bsum_e);
  uint32_t* bt = reinterpret_cast<uint32_t*>(w + M.o_bsum_t);
  const unsigned ne = (unsigned)M.edge_blocks, nt = (unsigned)M.tet_blocks;
  const uint32_t vc = (uint32_t)std::min<int64_t>(vert_cap, 0xffffffffll);
  const uint32_t tc = (uint32_t)std::min<int64_t>(tri_cap, 0xffffffffll);
  if (ne > 0)
    k_mt_edge_pass<<<ne, RT, 0, st>>>(verts, sdf, V, edges, n_edges, (uint32_t)edge_cap, be, vid, out_verts, vc, 0);
  k_edge_spine<<<1, 1024, 0, st>>>(be, ne, counts);
  if (ne > 0)
    k_mt_edge_pass<<<ne, RT, 0, st>>>(verts, sdf, V, edges, n_edges, (uint32_t)edge_cap, be, vid, out_verts, vc, 1);
  if (nt > 0)
    k_mt_tet_pass<<<nt, RT, 0, st>>>(verts, tets, sdf, V, (uint32_t)K, edges, n_edges, (uint32_t)edge_cap, vid, bt,
                                     out_tris, tc, 0);
  k_edge_spine<<<1, 1024, 0, st>>>(bt, nt, counts + 1);
  if (nt > 0)
    k_mt_tet_pass<<<nt, RT, 0, st>>>(verts, tets, sdf, V, (uint32_t)K, edges, n_edges, (uint32_t)edge_cap, vid, bt,
                                     out_tris, tc, 1);
  return hipGetLastError();
}

}  // namespace ts
