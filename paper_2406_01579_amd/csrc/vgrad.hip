// Per-tet backward of the gfx950 tetrahedron rasterizer.  A group of P
// adjacent lanes (P a power of two covering the largest view count of a
// scene) owns one kept tet; lane q takes the tet's records in views q, q + P,
// ...: it sums each record's per-entry screen-space gradients over the tiles
// the record was binned to (the entries the compositing backward reached are
// flagged) and chains them through the projection and the mean depth to the
// vertex positions.  The group then sums over its lanes, and its first lane
// chains the view-independent parts -- the SDF values, the tet normal
// n = g/|g| (App. A.3, as the equivalent 3x3 edge system g = E^-1 (f_k - f_0))
// and the mean colour -- and adds the result to the per-vertex gradients
// (combined per block in LDS, then float atomics).  A record's loads form
// short dependent rounds (its compact box with the first entry, then its
// entry flags, then the flagged entries; 1/Z is recomputed from the tet's
// vertices with the projection's operations), and the views of a tet are in
// flight together.
#include "ts_device.h"

namespace ts {

// Scene of a kept slot: scenes own consecutive slot ranges starting at
// kbase[s] (non-decreasing; an empty scene shares its base with the next),
// so the slot's scene is the last one whose base is at or below it.  Found
// from the slot alone, so the record loads need not wait for the tet's own.
__device__ __forceinline__ int scene_of_kept(const int32_t* kbase, int ns, uint32_t k) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((uint32_t)kbase[mid] <= k) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// sum over aligned groups of P lanes (P a power of two <= 64)
template <int P>
__device__ __forceinline__ float group_sum(float x) {
#pragma unroll
  for (int o = 1; o < P; o <<= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Per-block combine of the vertex gradients: tets that share a vertex
// (every vertex of a tetrahedral grid belongs to many tets, and neighbouring
// kept slots are neighbouring tets) add into one LDS slot, keyed by vertex
// id, and each slot is added to HBM once per block.  Open addressing with a
// bounded probe; a vertex that finds no slot, or a tet of another scene than
// the block's first, adds to HBM directly.
constexpr int VB_HASH = 512;
constexpr int VB_PROBES = 16;
static_assert(VB_HASH == 1 << 9, "the slot hash keeps 9 bits");

// With DET the per-vertex terms of every kept tet's four corners are written
// out (with the corner's global vertex id as a sort key) instead of being
// combined, and k_vertex_gather adds them in a fixed order.
// A 4-waves-per-SIMD target (at most 128 VGPRs): at 5 the kernel fits 96
// VGPRs only by spilling a dozen values to scratch inside its loops, and
// took 61 us against 52 us at the training shape.
template <int P, bool DET>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_vertex_bwd(void* ws, Layout L) {
  __shared__ uint32_t hkey[DET ? 1 : VB_HASH];   // vertex id + 1; 0: empty
  __shared__ float hval[7][DET ? 1 : VB_HASH];   // dverts xyz, dsdf, dcolors xyz
  __shared__ int bscene;
  DevHeader* hdr = at<DevHeader>(ws, L.o_hdr);
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const DevScene* sc = at<const DevScene>(ws, L.o_scene);
  const int32_t* scene_views = at<const int32_t>(ws, L.o_scene_views);
  const int32_t* kbase = at<const int32_t>(ws, L.o_scene_kept_base);
  const int32_t* rbase = at<const int32_t>(ws, L.o_view_rec_base);
  const uint32_t* rfirst = at<const uint32_t>(ws, L.o_rfirst);
  const TetRec* trec = at<const TetRec>(ws, L.o_trec);
  const uint32_t* count1 = at<const uint32_t>(ws, L.o_count1);
  const uint8_t* eflag = at<const uint8_t>(ws, L.o_eflag);
  const float* tgrad = at<const float>(ws, L.o_tgrad);
  const uint32_t nk = min(hdr->kept_total, (uint32_t)L.kept_cap);
  const uint32_t nrec = hdr->records_total;
  const bool per_record = record_grads(L);
  if (DET && blockIdx.x == 0 && threadIdx.x == 0) hdr->corners_total = 4u * nk;
  const uint64_t cap = (uint64_t)L.entry_cap;
  const int q0 = (int)(threadIdx.x % P);
  const uint32_t stride = gridDim.x * (blockDim.x / P);
  // the loop runs the same number of times in every lane of a group
  for (uint32_t k = (blockIdx.x * blockDim.x + threadIdx.x) / P; k < nk + (stride - nk % stride) % stride;
       k += stride) {
    const bool tet_ok = k < nk;
    const TetRec& T = trec[tet_ok ? k : 0u];
    const int ks = tet_ok ? scene_of_kept(kbase, L.ns, k) : 0;
    if constexpr (!DET) {
      for (int h = threadIdx.x; h < VB_HASH; h += blockDim.x) {
        hkey[h] = 0u;
#pragma unroll
        for (int m = 0; m < 7; ++m) hval[m][h] = 0.0f;
      }
      if (threadIdx.x == 0) bscene = tet_ok ? ks : -1;   // thread 0 holds the block's first tet
      __syncthreads();
    }
    float dv[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    float dfv[4] = {0, 0, 0, 0}, dn[3] = {0, 0, 0}, dc[3] = {0, 0, 0};
    bool any = false;
    if (tet_ok) {
      const DevScene& S = sc[ks];
      const uint32_t kl = k - (uint32_t)kbase[ks];
      for (int q = q0; q < S.view_count; q += P) {
        const int v = scene_views[S.view_first + q];
        const uint32_t r = (uint32_t)rbase[v] + kl;
        if (r >= nrec) continue;
        const uint32_t cnt = count1[r];
        if (cnt == 0) continue;
        float g[23];
        bool hit = false;
        if (per_record) {
          // the record's accumulator (zero if no tile reached it)
          const float4* src = reinterpret_cast<const float4*>(tgrad + (size_t)r * TGRAD_STRIDE);
#pragma unroll
          for (int z = 0; z < 6; ++z) {
            const float4 x = src[z];
            if (4 * z + 0 < 23) g[4 * z + 0] = x.x;
            if (4 * z + 1 < 23) g[4 * z + 1] = x.y;
            if (4 * z + 2 < 23) g[4 * z + 2] = x.z;
            if (4 * z + 3 < 23) g[4 * z + 3] = x.w;
          }
#pragma unroll
          for (int z = 0; z < 23; ++z) hit = hit || g[z] != 0.0f;
        } else {
        const uint32_t o = rfirst[r];   // the record's first entry
        const uint32_t n = (uint32_t)min((uint64_t)cnt, cap > o ? cap - o : 0ull);
        if (n == 0u) continue;  // entries past the capacity (an overflowed forward)
        // reached flags, bit j for entry o + j: the first eight from two
        // aligned 8-byte words (the flag array is padded for this), the rest
        // (records binned to more than eight tiles) byte by byte
        uint32_t fl = 0u;
        {
          const uint64_t* w8 = reinterpret_cast<const uint64_t*>(eflag + ((size_t)o & ~(size_t)7));
          const uint64_t a = w8[0], b = w8[1];
          const int sh = (int)(o & 7u) * 8;
          const uint64_t lo = sh ? (a >> sh) | (b << (64 - sh)) : a;
#pragma unroll
          for (int j = 0; j < 8; ++j) fl |= ((lo >> (8 * j)) & 0xffull) ? (1u << j) : 0u;
          for (uint32_t j = 8; j < n && j < 32u; ++j) fl |= eflag[o + j] ? (1u << j) : 0u;
          if (n < 32u) fl &= (1u << n) - 1u;
        }
#pragma unroll
        for (int z = 0; z < 23; ++z) g[z] = 0.0f;
        for (uint32_t t = fl; t != 0u; t &= t - 1u) {
          const uint64_t d = (uint64_t)o + (uint64_t)(__ffs(t) - 1);
          const float4* src = reinterpret_cast<const float4*>(tgrad + (size_t)d * TGRAD_STRIDE);
#pragma unroll
          for (int z = 0; z < 6; ++z) {
            const float4 x = src[z];
            if (4 * z + 0 < 23) g[4 * z + 0] += x.x;
            if (4 * z + 1 < 23) g[4 * z + 1] += x.y;
            if (4 * z + 2 < 23) g[4 * z + 2] += x.z;
            if (4 * z + 3 < 23) g[4 * z + 3] += x.w;
          }
          hit = true;
        }
        // a record binned to more than 32 tiles: the rest one by one
        for (uint32_t j = 32; j < n; ++j) {
          const uint64_t d = (uint64_t)o + j;
          if (!eflag[d]) continue;
          const float* src = tgrad + (size_t)d * TGRAD_STRIDE;
          for (int z = 0; z < 23; ++z) g[z] += src[z];
          hit = true;
        }
        }
        if (!hit) continue;
        any = true;
        const DevView& V = vw[v];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const float x = T.x[a][0], y = T.x[a][1], z = T.x[a][2];
          const float X = fmaf(V.R[0], x, fmaf(V.R[1], y, fmaf(V.R[2], z, V.t[0])));
          const float Y = fmaf(V.R[3], x, fmaf(V.R[4], y, fmaf(V.R[5], z, V.t[1])));
          // 1 / Z as the projection computed it (same operations)
          const float iz = 1.0f / fmaf(V.R[6], x, fmaf(V.R[7], y, fmaf(V.R[8], z, V.t[2])));
          // x' = fx X/Z + cx, y' = fy Y/Z + cy; w = 1/Z; z_t = mean Z
          const float dpx = g[G_PX + a] * V.fx, dpy = g[G_PY + a] * V.fy;
          const float dX = dpx * iz, dY = dpy * iz;
          float dZ = -(dpx * X + dpy * Y) * iz * iz;
          dZ += -g[G_IZ + a] * iz * iz;
          dZ += 0.25f * g[G_ZT];
#pragma unroll
          for (int m = 0; m < 3; ++m) dv[a][m] += V.R[m] * dX + V.R[3 + m] * dY + V.R[6 + m] * dZ;
          dfv[a] += g[G_F + a];
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          dn[m] += g[G_N + m];
          dc[m] += g[G_C + m];
        }
      }
    }
    // sum over the tet's lanes
    if (P > 1) {
      any = __ballot(any) & (((1ull << (P - 1)) << 1) - 1ull) << (threadIdx.x % 64 / P * P);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int m = 0; m < 3; ++m) dv[a][m] = group_sum<P>(dv[a][m]);
        dfv[a] = group_sum<P>(dfv[a]);
      }
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        dn[m] = group_sum<P>(dn[m]);
        dc[m] = group_sum<P>(dc[m]);
      }
    }
    // every lane of the group holds the same sums (a butterfly of commutative
    // adds) and chains the tet's view-independent parts alike; lane q then
    // adds the tet's corners a = q (mod min(P, 4)) to the vertex sums
    constexpr int PV = P < 4 ? P : 4;
    if (tet_ok && (any || DET)) {
    const DevScene& S = sc[ks];
    // normal: n = g/|g|, g = E^-1 df
    if (dn[0] != 0.0f || dn[1] != 0.0f || dn[2] != 0.0f) {
      float e[3][3], df[3];
      for (int a = 0; a < 3; ++a) {
        for (int m = 0; m < 3; ++m) e[a][m] = T.x[a + 1][m] - T.x[0][m];
        df[a] = T.f[a + 1] - T.f[0];
      }
      float cr[3][3] = {{e[1][1] * e[2][2] - e[1][2] * e[2][1], e[1][2] * e[2][0] - e[1][0] * e[2][2],
                         e[1][0] * e[2][1] - e[1][1] * e[2][0]},
                        {e[2][1] * e[0][2] - e[2][2] * e[0][1], e[2][2] * e[0][0] - e[2][0] * e[0][2],
                         e[2][0] * e[0][1] - e[2][1] * e[0][0]},
                        {e[0][1] * e[1][2] - e[0][2] * e[1][1], e[0][2] * e[1][0] - e[0][0] * e[1][2],
                         e[0][0] * e[1][1] - e[0][1] * e[1][0]}};
      const float det = e[0][0] * cr[0][0] + e[0][1] * cr[0][1] + e[0][2] * cr[0][2];
      if (det != 0.0f) {
        float gg[3];
        for (int m = 0; m < 3; ++m) gg[m] = (cr[0][m] * df[0] + cr[1][m] * df[1] + cr[2][m] * df[2]) / det;
        const float gn = sqrtf(gg[0] * gg[0] + gg[1] * gg[1] + gg[2] * gg[2]);
        if (gn > 0.0f) {
          const float nrm[3] = {gg[0] / gn, gg[1] / gn, gg[2] / gn};
          const float nd = nrm[0] * dn[0] + nrm[1] * dn[1] + nrm[2] * dn[2];
          float dg[3];
          for (int m = 0; m < 3; ++m) dg[m] = (dn[m] - nrm[m] * nd) / gn;
          // mu = E^-T dg ; d/df_a = mu_a (a=1..3), d/df_0 = -sum mu ; d/dx_a = -mu_a g, d/dx_0 = sum mu g
          float mu[3], msum = 0.0f;
          for (int a = 0; a < 3; ++a) {
            mu[a] = (cr[a][0] * dg[0] + cr[a][1] * dg[1] + cr[a][2] * dg[2]) / det;
            msum += mu[a];
          }
          for (int a = 0; a < 3; ++a) {
            dfv[a + 1] += mu[a];
            for (int m = 0; m < 3; ++m) dv[a + 1][m] -= mu[a] * gg[m];
          }
          dfv[0] -= msum;
          for (int m = 0; m < 3; ++m) dv[0][m] += msum * gg[m];
        }
      }
    }
    const int4 vi = load_tet(S.tets, T.tet);
    const int idx[4] = {vi.x, vi.y, vi.z, vi.w};
    if constexpr (DET) {
      // the four corners' terms and sort keys (corner id 4 k + a is the
      // sort's identity value)
      uint32_t* key = at<uint32_t>(ws, L.o_vkey_a);
      float4* term = at<float4>(ws, L.o_vterm);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (a % PV != q0) continue;
        const size_t cid = 4 * (size_t)k + (size_t)a;
        key[cid] = (uint32_t)S.vbase + (uint32_t)idx[a];
        term[2 * cid] = make_float4(dv[a][0], dv[a][1], dv[a][2], dfv[a]);
        term[2 * cid + 1] = make_float4(0.25f * dc[0], 0.25f * dc[1], 0.25f * dc[2], 0.0f);
      }
    } else
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (a % PV != q0) continue;
      const uint32_t vv = (uint32_t)idx[a];
      const float val[7] = {dv[a][0], dv[a][1], dv[a][2], dfv[a], 0.25f * dc[0], 0.25f * dc[1], 0.25f * dc[2]};
      bool put = false;
      if (ks == bscene) {
        uint32_t h = (vv * 2654435761u) >> 23;   // 9 bits: VB_HASH slots
        for (int probe = 0; probe < VB_PROBES; ++probe) {
          const uint32_t old = atomicCAS(&hkey[h], 0u, vv + 1u);
          if (old == 0u || old == vv + 1u) {
#pragma unroll
            for (int m = 0; m < 7; ++m)
              if (val[m] != 0.0f) atomicAdd(&hval[m][h], val[m]);
            put = true;
            break;
          }
          h = (h + 1u) & (VB_HASH - 1u);
        }
      }
      if (!put) {
        for (int m = 0; m < 3; ++m) {
          if (val[m] != 0.0f) gatomic_add(&S.dverts[3 * (size_t)vv + m], val[m]);
          if (val[4 + m] != 0.0f) gatomic_add(&S.dcolors[3 * (size_t)vv + m], val[4 + m]);
        }
        if (val[3] != 0.0f) gatomic_add(&S.dsdf[vv], val[3]);
      }
    }
    }
    if constexpr (DET) continue;
    __syncthreads();
    if (bscene >= 0) {
      const DevScene& S = sc[bscene];
      for (int h = threadIdx.x; h < VB_HASH; h += blockDim.x) {
        const uint32_t key = hkey[h];
        if (key == 0u) continue;
        const size_t vv = (size_t)(key - 1u);
        for (int m = 0; m < 3; ++m) {
          if (hval[m][h] != 0.0f) gatomic_add(&S.dverts[3 * vv + m], hval[m][h]);
          if (hval[4 + m][h] != 0.0f) gatomic_add(&S.dcolors[3 * vv + m], hval[4 + m][h]);
        }
        if (hval[3][h] != 0.0f) gatomic_add(&S.dsdf[vv], hval[3][h]);
      }
    }
    __syncthreads();
  }
}

template <bool DET>
static void launch_vbwd(void* ws, const Layout& L, unsigned blocks, int nvs, hipStream_t st) {
  if (nvs <= 1) k_vertex_bwd<1, DET><<<blocks, 256, 0, st>>>(ws, L);
  else if (nvs <= 2) k_vertex_bwd<2, DET><<<blocks, 256, 0, st>>>(ws, L);
  else if (nvs <= 4) k_vertex_bwd<4, DET><<<blocks, 256, 0, st>>>(ws, L);
  else k_vertex_bwd<8, DET><<<blocks, 256, 0, st>>>(ws, L);
}

hipError_t launch_vertex_backward(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  (void)p;
  // lanes per tet: the largest view count of a scene, rounded up to a power of two (at most 8)
  const int nvs = L.max_scene_views;
  const int64_t threads = L.kept_cap * (nvs <= 1 ? 1 : nvs <= 2 ? 2 : nvs <= 4 ? 4 : 8);
  const int64_t b = (threads + 255) / 256;
  const unsigned blocks = (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
  if (deterministic(L)) launch_vbwd<true>(ws, L, blocks, nvs, st);
  else launch_vbwd<false>(ws, L, blocks, nvs, st);
  return hipGetLastError();
}

// Deterministic vertex sums: the corners, sorted by vertex (stable, so a
// vertex's corners keep ascending corner id, i.e. kept-tet order), are
// walked from the first corner of each vertex and added in that order; one
// thread writes each vertex that some kept tet touches (the others stay as
// the gradient clear left them, zero).
__global__ __launch_bounds__(256) void k_vertex_gather(void* ws, Layout L, const uint32_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ cids) {
  const DevHeader* hdr = at<const DevHeader>(ws, L.o_hdr);
  const DevScene* sc = at<const DevScene>(ws, L.o_scene);
  const float4* term = at<const float4>(ws, L.o_vterm);
  const uint32_t n = min(hdr->corners_total, (uint32_t)(4 * L.kept_cap));
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t key = keys[i];
    if (i > 0 && keys[i - 1] == key) continue;
    float acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (uint32_t j = i; j < n && keys[j] == key; ++j) {
      const float4 a = term[2 * (size_t)cids[j]], b = term[2 * (size_t)cids[j] + 1];
      acc[0] += a.x;
      acc[1] += a.y;
      acc[2] += a.z;
      acc[3] += a.w;
      acc[4] += b.x;
      acc[5] += b.y;
      acc[6] += b.z;
    }
    // the scene: the last one whose first vertex is at or below the key
    int lo = 0, hi = L.ns - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((uint32_t)sc[mid].vbase <= key) lo = mid;
      else hi = mid - 1;
    }
    const DevScene& S = sc[lo];
    const size_t v = (size_t)(key - (uint32_t)S.vbase);
    S.dverts[3 * v] = acc[0];
    S.dverts[3 * v + 1] = acc[1];
    S.dverts[3 * v + 2] = acc[2];
    S.dsdf[v] = acc[3];
    S.dcolors[3 * v] = acc[4];
    S.dcolors[3 * v + 1] = acc[5];
    S.dcolors[3 * v + 2] = acc[6];
  }
}

hipError_t launch_vertex_gather(void* ws, const Layout& L, hipStream_t st) {
  uint32_t *ko, *vo;
  DevHeader* hdr = at<DevHeader>(ws, L.o_hdr);
  const int64_t nc = 4 * L.kept_cap;
  hipError_t e = radix_sort_pairs(at<uint32_t>(ws, L.o_vkey_a), at<uint32_t>(ws, L.o_vval_a),
                                  at<uint32_t>(ws, L.o_vkey_b), at<uint32_t>(ws, L.o_vval_b), true,
                                  &hdr->corners_total, nc, L.vkey_bits, at<uint32_t>(ws, L.o_hist),
                                  L.sort_blocks_max, st, &ko, &vo);
  if (e != hipSuccess) return e;
  const int64_t b = (nc + 255) / 256;
  const unsigned blocks = (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
  k_vertex_gather<<<blocks, 256, 0, st>>>(ws, L, ko, vo);
  return hipGetLastError();
}

}  // namespace ts
