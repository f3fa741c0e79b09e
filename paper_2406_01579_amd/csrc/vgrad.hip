// Per-tet backward of the gfx950 tetrahedron rasterizer.  One thread per
// kept tet: for every view of the tet's scene it sums the per-entry
// screen-space gradients of the (view, tet) record over the tiles the record
// was binned to and chains them through the projection and the mean depth to
// world-space vertex positions; the view-independent parts -- the SDF
// values, the per-tet normal n = g/|g| (App. A.3, as the equivalent 3x3 edge
// system g = E^-1 (f_k - f_0)) and the mean colour -- are chained once per
// tet.  The result is added to the per-vertex gradients (float atomics).
#include "ts_device.h"

namespace ts {

__global__ __launch_bounds__(256) void k_vertex_bwd(void* ws, Layout L) {
  const DevHeader* hdr = at<const DevHeader>(ws, L.o_hdr);
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const DevScene* sc = at<const DevScene>(ws, L.o_scene);
  const int32_t* scene_views = at<const int32_t>(ws, L.o_scene_views);
  const int32_t* kbase = at<const int32_t>(ws, L.o_scene_kept_base);
  const int32_t* rbase = at<const int32_t>(ws, L.o_view_rec_base);
  const ViewRec* vrec = at<const ViewRec>(ws, L.o_vrec);
  const TetRec* trec = at<const TetRec>(ws, L.o_trec);
  const uint32_t* count1 = at<const uint32_t>(ws, L.o_count1);
  const uint8_t* eflag = at<const uint8_t>(ws, L.o_eflag);
  const float* tgrad = at<const float>(ws, L.o_tgrad);
  const uint32_t nk = min(hdr->kept_total, (uint32_t)L.kept_cap);
  const uint32_t nrec = hdr->records_total;
  const uint64_t cap = (uint64_t)L.entry_cap;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nk; k += gridDim.x * blockDim.x) {
    const TetRec& T = trec[k];
    const DevScene& S = sc[T.scene];
    const uint32_t kl = k - (uint32_t)kbase[T.scene];
    float dv[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    float dfv[4] = {0, 0, 0, 0}, dn[3] = {0, 0, 0}, dc[3] = {0, 0, 0};
    bool any = false;
    for (int q = 0; q < S.view_count; ++q) {
      const int v = scene_views[S.view_first + q];
      const uint32_t r = (uint32_t)rbase[v] + kl;
      if (r >= nrec) continue;
      const uint32_t cnt = count1[r];
      if (cnt == 0) continue;
      const ViewRec& R = vrec[r];
      const DevView& V = vw[v];
      const uint32_t o = R.entry0;
      float g[23];
      for (int z = 0; z < 23; ++z) g[z] = 0.0f;
      bool hit = false;
      // the record's entries, one per tile it was binned to; the compositing
      // backward flags the ones it reached
      for (uint32_t j = 0; j < cnt; ++j) {
        const uint64_t d = (uint64_t)o + j;
        if (d >= cap) break;
        if (!eflag[d]) continue;
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
      if (!hit) continue;
      any = true;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const float x = T.x[a][0], y = T.x[a][1], z = T.x[a][2];
        const float X = fmaf(V.R[0], x, fmaf(V.R[1], y, fmaf(V.R[2], z, V.t[0])));
        const float Y = fmaf(V.R[3], x, fmaf(V.R[4], y, fmaf(V.R[5], z, V.t[1])));
        const float iz = R.iz[a];
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
    if (!any) continue;
    // normal: n = g/|g|, g = E^-1 df
    {
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
      if (det != 0.0f && (dn[0] != 0.0f || dn[1] != 0.0f || dn[2] != 0.0f)) {
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
    const int4 vi = reinterpret_cast<const int4*>(S.tets)[T.tet];
    const int idx[4] = {vi.x, vi.y, vi.z, vi.w};
    for (int a = 0; a < 4; ++a) {
      const size_t vv = (size_t)idx[a];
      for (int m = 0; m < 3; ++m) {
        if (dv[a][m] != 0.0f) unsafeAtomicAdd(&S.dverts[3 * vv + m], dv[a][m]);
        const float dcm = 0.25f * dc[m];
        if (dcm != 0.0f) unsafeAtomicAdd(&S.dcolors[3 * vv + m], dcm);
      }
      if (dfv[a] != 0.0f) unsafeAtomicAdd(&S.dsdf[vv], dfv[a]);
    }
  }
}

hipError_t launch_vertex_backward(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  (void)p;
  k_vertex_bwd<<<1024, 256, 0, st>>>(ws, L);
  return hipGetLastError();
}

}  // namespace ts
