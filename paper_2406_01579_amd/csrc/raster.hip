// Per-tile compositing kernels of the gfx950 tetrahedron rasterizer.
//
// One workgroup per screen tile; each 64-lane wave owns an 8x8 block of the
// tile (one pixel per lane).  The tile's depth-sorted record list is staged
// through LDS in chunks; with tiles larger than 8x8 every wave skips, with a
// wave-uniform test, records whose pixel rectangle misses its block.
//
// Forward (Eq. 1, Eq. 2, Sec. 3.3): front-to-back blending of colour, depth,
// normal and opacity with the 3DGS thresholds; stores per pixel the position
// of the last blended entry and the transmittance before it.
//
// Backward: reverse traversal from the tile's last blended entry.  With
// R = the colour seen behind the current entry (R starts as g_rgb . bg),
//   dL/dalpha_i = T_i (s_i - R),   R <- alpha_i s_i + (1 - alpha_i) R,
// where s_i = g . (c_i, 1, z_i, n_i) and T_i is recovered by
// T_i = T_{i+1} / (1 - alpha_i) starting from the stored T before the last
// blended entry (so an entry with alpha = 1 never needs a division).  Each
// lane's gradient of the record's screen-space parameters is summed over the
// wave with a transposed permlane/DPP reduction and over the waves of the
// tile in LDS, then stored per entry (deterministic order across tiles).
#include "ts_device.h"

namespace ts {

constexpr int CH = 64;  // records per LDS chunk

struct TileCtx {
  int view, tile, lt, tx, ty;
  uint32_t start, end;  // the tile's entry range
  int i, j;       // this lane's pixel
  bool inside;
  int wi0, wj0;   // this wave's 8x8 block origin
};

template <int TW, int TH>
__device__ __forceinline__ TileCtx tile_ctx(const DevView* vw, const TileSlot* slots) {
  TileCtx c;
  const TileSlot sl = slots[blockIdx.x];
  c.tile = (int)sl.tile;
  c.view = (int)sl.view;
  c.start = sl.start;
  c.end = sl.end;
  const DevView& V = vw[c.view];
  c.lt = c.tile - V.tile_base;
  c.tx = c.lt % V.tiles_x;
  c.ty = c.lt / V.tiles_x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int WX = TW / 8;
  c.wi0 = c.tx * TW + (wave % WX) * 8;
  c.wj0 = c.ty * TH + (wave / WX) * 8;
  c.i = c.wi0 + (lane & 7);
  c.j = c.wj0 + (lane >> 3);
  c.inside = c.i < V.W && c.j < V.H;
  return c;
}

// The records of sorted entries [base, base + n) into LDS, eight threads per
// 128-byte record.  With rfirst, the copy's first-entry field comes from the
// records' first entries, where the placement kernel writes them.
__device__ __forceinline__ void load_chunk(ViewRec* recs, const ViewRec* __restrict__ vrec,
                                           const uint32_t* __restrict__ srec, uint32_t base, int n, int nthreads,
                                           const uint32_t* __restrict__ rfirst = nullptr) {
  for (int q = threadIdx.x; q < n * 8; q += nthreads) {
    const int e = q >> 3, part = q & 7;
    const uint32_t r = srec[base + e];
    float4 t = reinterpret_cast<const float4*>(&vrec[r])[part];
    if (rfirst && part == 7) t.w = __uint_as_float(rfirst[r]);   // entry0 is the last word of the record
    reinterpret_cast<float4*>(&recs[e])[part] = t;
  }
}

template <int TW, int TH>
__device__ __forceinline__ bool rect_hits_block(const ViewRec& R, int wi0, int wj0) {
  if (TW == 8 && TH == 8) return true;  // a tile's list only holds records that overlap it
  int i0, i1, j0, j1;
  unpack_rect(R, i0, i1, j0, j1);
  return !(i1 < wi0 || i0 > wi0 + 7 || j1 < wj0 || j0 > wj0 + 7);
}

__device__ __forceinline__ bool rect_has_pixel(const ViewRec& R, int i, int j) {
  int i0, i1, j0, j1;
  unpack_rect(R, i0, i1, j0, j1);
  return i >= i0 && i <= i1 && j >= j0 && j <= j1;
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_composite(void* ws, Layout L, float alpha_min, float alpha_clamp,
                                                      float t_min) {
  constexpr int NT = TW * TH;
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const uint32_t* srec = at<const uint32_t>(ws, sorted_entry_records(L));
  const ViewRec* vrec = at<const ViewRec>(ws, L.o_vrec);
  int32_t* last_out = at<int32_t>(ws, L.o_last);
  float* tlast_out = at<float>(ws, L.o_tlast);
  __shared__ ViewRec recs[CH];

  const TileCtx c = tile_ctx<TW, TH>(vw, at<const TileSlot>(ws, L.o_tile_order));
  const DevView& V = vw[c.view];
  const float s = uniform_f(V.s);
  const uint32_t start = c.start, end = c.end;
  const float qx = (float)c.i + 0.5f, qy = (float)c.j + 0.5f;

  float T = 1.0f, Tb = 1.0f, O = 0.0f;
  float acc[7] = {0, 0, 0, 0, 0, 0, 0};
  int last = -1;
  bool done = !c.inside;

  for (uint32_t base = start; base < end; base += CH) {
    if (__syncthreads_count(done ? 0 : 1) == 0) break;
    const int n = (int)min((uint32_t)CH, end - base);
    load_chunk(recs, vrec, srec, base, n, NT);
    __syncthreads();
    if (__ballot(!done) != 0ull) {
      for (int e = 0; e < n; ++e) {
        const ViewRec& R = recs[e];
        if (!rect_hits_block<TW, TH>(R, c.wi0, c.wj0)) continue;
        if (done || !rect_has_pixel(R, c.i, c.j)) continue;
        PixEval h;
        if (!pixel_eval(R, qx, qy, s, h)) continue;
        float a = h.alpha;
        if (a < alpha_min) continue;
        a = fminf(a, alpha_clamp);
        const float Tn = T * (1.0f - a);
        if (Tn < t_min) { done = true; continue; }
        const float w = T * a;
        acc[0] = fmaf(w, R.c[0], acc[0]);
        acc[1] = fmaf(w, R.c[1], acc[1]);
        acc[2] = fmaf(w, R.c[2], acc[2]);
        acc[3] = fmaf(w, R.zt, acc[3]);
        acc[4] = fmaf(w, R.n[0], acc[4]);
        acc[5] = fmaf(w, R.n[1], acc[5]);
        acc[6] = fmaf(w, R.n[2], acc[6]);
        O += w;
        Tb = T;
        T = Tn;
        last = (int)(base + e);
        if (T == 0.0f) done = true;
      }
    }
    __syncthreads();
  }
  if (c.inside) {
    const size_t plane = (size_t)V.W * V.H;
    const size_t px = (size_t)c.j * V.W + c.i;
    auto* out = gmem(V.out);
    out[0 * plane + px] = fmaf(T, V.bg[0], acc[0]);
    out[1 * plane + px] = fmaf(T, V.bg[1], acc[1]);
    out[2 * plane + px] = fmaf(T, V.bg[2], acc[2]);
    out[3 * plane + px] = O;
    out[4 * plane + px] = acc[3];
    out[5 * plane + px] = acc[4];
    out[6 * plane + px] = acc[5];
    out[7 * plane + px] = acc[6];
    if (keeps_pixel_state(L)) {
      const size_t g = (size_t)V.pix_base + px;
      last_out[g] = last;
      tlast_out[g] = Tb;
    }
  }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// d f(face F) / d(record parameters) times df, added to g.  F is a
// compile-time constant, so every index below is static.
// f = sum N_k w_k f_k / S, S = sum N_k w_k, N the face's cross products.
template <int F>
__device__ __forceinline__ void face_grad(const ViewRec& R, const PixEval& h, float df, float (&g)[32]) {
  constexpr int A = face_vertex(F, 0), B = face_vertex(F, 1), C = face_vertex(F, 2);
  constexpr int I[3] = {A, B, C};
  const float invS = rcp(h.S[F]);
  const float fF = F == h.fe ? h.fin : h.fout;   // F is the entry or the exit face
  float a[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int v = I[k];
    const float wk = R.iz[v];
    const float diff = (R.f[v] - fF) * invS * df;
    g[G_F + v] = fmaf(h.N[F][k] * wk * invS, df, g[G_F + v]);   // d/df_k
    g[G_IZ + v] = fmaf(h.N[F][k], diff, g[G_IZ + v]);            // d/dw_k
    a[k] = wk * diff;                                             // d/dN_k
  }
  const float Ax = h.ax[A], Ay = h.ay[A], Bx = h.ax[B], By = h.ay[B], Cx = h.ax[C], Cy = h.ay[C];
  // N0 = cross(B', C'), N1 = cross(C', A'), N2 = cross(A', B')
  g[G_PX + A] += a[2] * By - a[1] * Cy;
  g[G_PY + A] += a[1] * Cx - a[2] * Bx;
  g[G_PX + B] += a[0] * Cy - a[2] * Ay;
  g[G_PY + B] += a[2] * Ax - a[0] * Cx;
  g[G_PX + C] += a[1] * Ay - a[0] * By;
  g[G_PY + C] += a[0] * Bx - a[1] * Ax;
}

// DET (tiles of more than one wave): each wave's sum of an entry goes to its
// own LDS slot and the slots are added in wave order, instead of LDS float
// atomics in arrival order.
template <int TW, int TH, bool DET>
__global__ __launch_bounds__(TW* TH) void k_composite_bwd(void* ws, Layout L, float alpha_min, float alpha_clamp,
                                                          float t_min, int recompute) {
  constexpr int NT = TW * TH;
  constexpr int NW = NT / 64;
  constexpr bool WSLOT = DET && NW > 1;
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const uint32_t* srec = at<const uint32_t>(ws, sorted_entry_records(L));
  const ViewRec* vrec = at<const ViewRec>(ws, L.o_vrec);
  const int32_t* last_in = at<const int32_t>(ws, L.o_last);
  const float* tlast_in = at<const float>(ws, L.o_tlast);
  float* tgrad = at<float>(ws, L.o_tgrad);
  uint8_t* eflag = at<uint8_t>(ws, L.o_eflag);
  __shared__ ViewRec recs[CH];
  __shared__ float gacc[CH][TGRAD_STRIDE];
  __shared__ float gaccw[WSLOT ? NW : 1][WSLOT ? CH : 1][TGRAD_STRIDE];
  __shared__ int smax[NW];

  const TileCtx c = tile_ctx<TW, TH>(vw, at<const TileSlot>(ws, L.o_tile_order));
  const DevView& V = vw[c.view];
  const float s = uniform_f(V.s);
  const uint32_t start = c.start, end = c.end;
  const float qx = (float)c.i + 0.5f, qy = (float)c.j + 0.5f;
  const size_t plane = (size_t)V.W * V.H;
  const size_t px = c.inside ? (size_t)c.j * V.W + c.i : 0;
  const unsigned lane = threadIdx.x & 63u;

  int last = -1;
  float Tb = 1.0f;
  if (recompute) {
    // replay the forward sweep for this pixel to find its last blended entry
    float T = 1.0f;
    bool done = !c.inside;
    for (uint32_t base = start; base < end; base += CH) {
      if (__syncthreads_count(done ? 0 : 1) == 0) break;
      const int n = (int)min((uint32_t)CH, end - base);
      load_chunk(recs, vrec, srec, base, n, NT);
      __syncthreads();
      for (int e = 0; e < n; ++e) {
        const ViewRec& R = recs[e];
        if (!rect_hits_block<TW, TH>(R, c.wi0, c.wj0)) continue;
        if (done || !rect_has_pixel(R, c.i, c.j)) continue;
        PixEval h;
        if (!pixel_eval(R, qx, qy, s, h)) continue;
        float a = h.alpha;
        if (a < alpha_min) continue;
        a = fminf(a, alpha_clamp);
        const float Tn = T * (1.0f - a);
        if (Tn < t_min) { done = true; continue; }
        Tb = T;
        T = Tn;
        last = (int)(base + e);
        if (T == 0.0f) done = true;
      }
      __syncthreads();
    }
  } else if (c.inside) {
    const size_t gi = (size_t)V.pix_base + px;
    last = last_in[gi];
    Tb = tlast_in[gi];
  }

  // upstream gradient
  float gr[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) gr[q] = c.inside ? gmem(V.dout)[q * plane + px] : 0.0f;
  float Rbehind = gr[0] * V.bg[0] + gr[1] * V.bg[1] + gr[2] * V.bg[2];

  // the tile is processed from its largest last-blended position down
  int wmax = last;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) wmax = max(wmax, __shfl_xor(wmax, o, 64));
  if (NW > 1) {
    if (lane == 0) smax[threadIdx.x >> 6] = wmax;
    __syncthreads();
    for (int w = 0; w < NW; ++w) wmax = max(wmax, smax[w]);
  }
  const int tmax = wmax;
  const uint32_t pend = (tmax >= (int)start) ? (uint32_t)tmax + 1u : start;

  bool first = true;
  float Tnext = 1.0f;
  for (int64_t cb = (int64_t)start + (((int64_t)pend - 1 - (int64_t)start) / CH) * CH;
       cb >= (int64_t)start && pend > start; cb -= CH) {
    const uint32_t base = (uint32_t)cb;
    const int n = (int)min((uint32_t)CH, pend - base);
    load_chunk(recs, vrec, srec, base, n, NT, at<const uint32_t>(ws, L.o_rfirst));
    if (WSLOT)
      for (int q = threadIdx.x; q < NW * CH * TGRAD_STRIDE; q += NT) (&gaccw[0][0][0])[q] = 0.0f;
    else if (NW > 1)
      for (int q = threadIdx.x; q < CH * TGRAD_STRIDE; q += NT) (&gacc[0][0])[q] = 0.0f;
    __syncthreads();
    for (int e = n - 1; e >= 0; --e) {
      const ViewRec& R = recs[e];
      if (!rect_hits_block<TW, TH>(R, c.wi0, c.wj0)) continue;
      const int p = (int)(base + e);
      float g[32];
#pragma unroll
      for (int q = 0; q < 32; ++q) g[q] = 0.0f;
      bool contrib = false;
      if (c.inside && p <= last && rect_has_pixel(R, c.i, c.j)) {
        PixEval h;
        if (pixel_eval(R, qx, qy, s, h) && h.alpha >= alpha_min) {
          const float a = fminf(h.alpha, alpha_clamp);
          const bool clamped = h.alpha > alpha_clamp;
          float T;
          if (first) { T = Tb; first = false; }
          else T = Tnext * rcp(1.0f - a);
          Tnext = T;
          const float w = T * a;
          const float sdot = gr[0] * R.c[0] + gr[1] * R.c[1] + gr[2] * R.c[2] + gr[3] + gr[4] * R.zt +
                             gr[5] * R.n[0] + gr[6] * R.n[1] + gr[7] * R.n[2];
          const float da = T * (sdot - Rbehind);
          Rbehind = a * sdot + (1.0f - a) * Rbehind;
          g[G_C + 0] = w * gr[0];
          g[G_C + 1] = w * gr[1];
          g[G_C + 2] = w * gr[2];
          g[G_ZT] = w * gr[4];
          g[G_N + 0] = w * gr[5];
          g[G_N + 1] = w * gr[6];
          g[G_N + 2] = w * gr[7];
          if (!clamped && h.alpha > 0.0f) {
            // alpha = A / B, A = -expm1(-s d), B = 1 + exp(s f_next)
            const float invB = rcp(1.0f + h.e2);
            const float dA = da * invB;
            const float dB = -da * h.alpha * invB;
            const float dd = dA * s * (h.e1 + 1.0f);     // d/df_prev
            const float dfn = dB * s * h.e2 - dd;         // d/df_next
#pragma unroll
            for (int F = 0; F < 4; ++F) {
              const float wF = (h.fe == F ? dd : 0.0f) + (h.fx == F ? dfn : 0.0f);
              if (wF != 0.0f) {
                if (F == 0) face_grad<0>(R, h, wF, g);
                if (F == 1) face_grad<1>(R, h, wF, g);
                if (F == 2) face_grad<2>(R, h, wF, g);
                if (F == 3) face_grad<3>(R, h, wF, g);
              }
            }
          }
          contrib = true;
        }
      }
      if (__ballot(contrib) == 0ull) {
        if (NW == 1 && lane < TGRAD_STRIDE) gacc[e][lane] = 0.0f;
        continue;
      }
      const float tot = wave_transpose_sum32(g);   // lane L: sum of g[L >> 1]
      const unsigned q = lane >> 1;
      if ((lane & 1u) == 0u && q < (unsigned)TGRAD_STRIDE) {
        if (NW == 1) gacc[e][q] = tot;
        else if (WSLOT) gaccw[threadIdx.x >> 6][e][q] = tot;
        else atomicAdd(&gacc[e][q], tot);
      }
    }
    __syncthreads();
    if (WSLOT) {
      for (int q = threadIdx.x; q < n * TGRAD_STRIDE; q += NT) {
        const int e = q / TGRAD_STRIDE, k = q - e * TGRAD_STRIDE;
        float acc = 0.0f;
#pragma unroll
        for (int w = 0; w < NW; ++w) acc += gaccw[w][e][k];
        gacc[e][k] = acc;
      }
      __syncthreads();
    }
    if (record_grads(L)) {
      for (int q = threadIdx.x; q < n * (TGRAD_STRIDE - 1); q += NT) {
        const int e = q / (TGRAD_STRIDE - 1), k = q - e * (TGRAD_STRIDE - 1);
        const float v = gacc[e][k];
        if (v != 0.0f) unsafeAtomicAdd(&tgrad[(size_t)srec[base + e] * TGRAD_STRIDE + k], v);
      }
      __syncthreads();
      continue;
    }
    // each entry's gradient goes to its pre-sort slot: the record's first
    // entry plus this tile's row-major index inside the record's tile rectangle
    for (int q = threadIdx.x; q < n * TGRAD_STRIDE; q += NT) {
      const int e = q / TGRAD_STRIDE, k = q - e * TGRAD_STRIDE;
      const ViewRec& R = recs[e];
      int i0, i1, j0, j1;
      unpack_rect(R, i0, i1, j0, j1);
      const int tx0 = i0 / TW, ty0 = j0 / TH, nx = i1 / TW - tx0 + 1;
      const size_t d = (size_t)R.entry0 + (size_t)((c.ty - ty0) * nx + (c.tx - tx0));
      if (d >= (size_t)L.entry_cap) continue;   // an overflowed forward's entry
      tgrad[d * TGRAD_STRIDE + k] = gacc[e][k];
      if (k == 0) eflag[d] = 1;
    }
    __syncthreads();
  }
}

template <int TW, int TH>
static void launch_fwd(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  k_composite<TW, TH><<<(unsigned)L.total_tiles, TW * TH, 0, st>>>(ws, L, p.alpha_min, p.alpha_clamp, p.t_min);
}
template <int TW, int TH>
static void launch_bwd(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  const int rc = (p.flags & RENDER_RECOMPUTE_STATE) ? 1 : 0;
  if (deterministic(L))
    k_composite_bwd<TW, TH, true><<<(unsigned)L.total_tiles, TW * TH, 0, st>>>(ws, L, p.alpha_min, p.alpha_clamp,
                                                                               p.t_min, rc);
  else
    k_composite_bwd<TW, TH, false><<<(unsigned)L.total_tiles, TW * TH, 0, st>>>(ws, L, p.alpha_min, p.alpha_clamp,
                                                                                p.t_min, rc);
}

#define TS_TILE_SWITCH(FN)                                          \
  switch (p.tile_w * 1000 + p.tile_h) {                             \
    case 8008: FN<8, 8>(ws, L, p, st); break;                       \
    case 16008: FN<16, 8>(ws, L, p, st); break;                     \
    case 8016: FN<8, 16>(ws, L, p, st); break;                      \
    case 16016: FN<16, 16>(ws, L, p, st); break;                    \
    case 32008: FN<32, 8>(ws, L, p, st); break;                     \
    default: return hipErrorInvalidValue;                           \
  }

hipError_t launch_composite(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  if (L.total_tiles == 0) return hipSuccess;
  TS_TILE_SWITCH(launch_fwd)
  return hipGetLastError();
}

hipError_t launch_composite_backward(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  if (L.total_tiles == 0) return hipSuccess;
  TS_TILE_SWITCH(launch_bwd)
  return hipGetLastError();
}

}  // namespace ts
