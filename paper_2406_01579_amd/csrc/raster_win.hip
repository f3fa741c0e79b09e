// Compositing with the per-pixel resort window of Sec. 3.3, on 8x8 tiles.
//
// The per-tile order (mean vertex depth, then tet id) is only close to each
// pixel's own front-to-back order.  With a window of N_w entries every pixel
// passes its candidates, in the per-tile order, through a buffer of at most
// N_w entries ordered by the depth at which the pixel's ray enters the tet:
// when an arrival makes the buffer overflow, its nearest entry leaves and is
// blended; at the end of the list the rest leave nearest first.  Only
// candidates with alpha >= alpha_min enter the buffer.  Equal depths leave in
// arrival order.
//
// Forward: as in the multi-wave kernels, all waves evaluate the chunk's packed
// (entry, pixel) pairs -- pixel live and inside the entry's rectangle -- into
// LDS (alpha and the entry depth) and mark each pixel's candidates; wave 0
// runs the window over each pixel's candidates and the blend.  A lane's
// window keys live in registers with static slot indices; each slot's payload
// (alpha and the seven blended features) lives in LDS, where a per-lane slot
// index is cheap.
//
// Backward: a pixel's blend order is no longer the tile order, so the
// reverse-order walk of the plain backward does not apply.  Sweep 1 replays
// the window front to back and records, for every blended (entry, pixel)
// pair, the transmittance before the blend, the raw alpha, the dot product of
// the pixel's upstream gradient with the entry's features, and the pixel's
// previously blended entry: a per-pixel list in blend order, kept in a
// workspace array indexed by (entry, lane).  Sweep 2 walks every pixel's list
// from its last blend back (the reverse mode of Eq. 2) and leaves
// (dL/dalpha, T alpha) in place.  Sweep 3 goes over the chunks again in tile
// order and chains every pair to the record's parameters, reduced over the
// tile into the per-entry gradient.  The backward keeps the dense per-entry
// evaluation (every wave owns interleaved entries for all 64 pixels).
#include "tile8.h"

namespace ts {

namespace {

constexpr int WSLOTS = RENDER_WINDOW_MAX + 1;  // an arrival overflows a full window by one
constexpr int CHW = 32;                        // entries per LDS chunk

// One lane's window.  key = 1 / entry depth (larger is nearer), -1 for a free
// slot (a hit's key is positive); idx = global entry index (arrival order).
struct Window {
  float key[WSLOTS];
  int idx[WSLOTS];
  int cnt;
};

__device__ __forceinline__ void win_init(Window& w) {
#pragma unroll
  for (int k = 0; k < WSLOTS; ++k) {
    w.key[k] = -1.0f;
    w.idx[k] = 0;
  }
  w.cnt = 0;
}

// Puts (key, idx) into the lowest free slot and returns that slot.
__device__ __forceinline__ int win_insert(Window& w, float key, int idx) {
  int slot = 0;
#pragma unroll
  for (int k = WSLOTS - 1; k >= 0; --k) slot = (w.key[k] < 0.0f) ? k : slot;
#pragma unroll
  for (int k = 0; k < WSLOTS; ++k) {
    const bool here = k == slot;
    w.key[k] = here ? key : w.key[k];
    w.idx[k] = here ? idx : w.idx[k];
  }
  ++w.cnt;
  return slot;
}

// Takes the nearest entry out (largest key; equal keys: earliest arrival) and
// returns its slot; *idx receives its entry index.  Needs cnt > 0.
__device__ __forceinline__ int win_pop(Window& w, int* idx) {
  int m = 0;
  float bk = w.key[0];
  int bi = w.idx[0];
#pragma unroll
  for (int k = 1; k < WSLOTS; ++k) {
    const bool better = w.key[k] > bk || (w.key[k] == bk && bk >= 0.0f && w.idx[k] < bi);
    m = better ? k : m;
    bk = better ? w.key[k] : bk;
    bi = better ? w.idx[k] : bi;
  }
#pragma unroll
  for (int k = 0; k < WSLOTS; ++k) w.key[k] = (k == m) ? -1.0f : w.key[k];
  --w.cnt;
  *idx = bi;
  return m;
}

// Phase A of a chunk: every wave evaluates its interleaved entries for its
// lane's pixel; alpha (-1: no hit or pixel finished) and entry key to LDS.
template <int NWV>
__device__ __forceinline__ void eval_chunk(const ViewRec* recs, int n, const Tile8& c, float qx, float qy, float s,
                                           bool mydone, float (*alds)[64], float (*zlds)[64]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int e = wave; e < n; e += NWV) {
    float a = -1.0f, z = 0.0f;
    const ViewRec& R = recs[e];
    if (!mydone && has_pixel(R, c.i, c.j)) {
      PixEval h;
      if (pixel_eval(R, qx, qy, s, h)) {
        a = h.alpha;
        z = h.zin_inv;
      }
    }
    alds[e][lane] = a;
    zlds[e][lane] = z;
  }
}

// Per chunk: the entries' blended features as a conflict-free table
// (feat[k][e]: c[3], zt, n[3]) and a cleared per-pixel candidate mask.
template <int CH>
__device__ __forceinline__ void load_chunk_tables(const ViewRec* recs, int n, float (*feat)[CH], uint32_t* hm,
                                                  int nthreads) {
  if (threadIdx.x < 64) hm[threadIdx.x] = 0u;
  for (int q = threadIdx.x; q < n * 7; q += nthreads) {
    const int e = q / 7, k = q - e * 7;
    feat[k][e] = k < 3 ? recs[e].c[k] : k == 3 ? recs[e].zt : recs[e].n[k - 4];
  }
}

}  // namespace

template <int NWV>
__global__ __launch_bounds__(64 * NWV) void k_composite_win(void* ws, Layout L, float alpha_min, float alpha_clamp,
                                                            float t_min, int nw) {
  constexpr int NT = 64 * NWV;
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const uint32_t* srec = at<const uint32_t>(ws, sorted_entry_records(L));
  const ViewRec* vrec = at<const ViewRec>(ws, L.o_vrec);
  int32_t* last_out = at<int32_t>(ws, L.o_last);
  float* tlast_out = at<float>(ws, L.o_tlast);
  __shared__ ViewRec recs[CHW];
  __shared__ float alds[CHW][64];
  __shared__ float zlds[CHW][64];
  __shared__ float feat[7][CHW];        // per entry: c[3], zt, n[3]
  __shared__ uint64_t pmask[CHW];
  __shared__ uint32_t poff[CHW + 1];
  __shared__ uint32_t hm[64];           // per pixel: the chunk's candidates (bit e)
  __shared__ float pay[WSLOTS][8][64];  // per slot: alpha, c[3], zt, n[3]
  __shared__ unsigned long long done_mask;

  const Tile8 c = tile8(vw, at<const TileSlot>(ws, L.o_tile_order));
  const DevView& V = vw[c.view];
  const float s = V.s;
  const uint32_t start = c.start, end = c.end;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float qx = (float)c.i + 0.5f, qy = (float)c.j + 0.5f;

  float T = 1.0f, Tb = 1.0f, O = 0.0f;
  float acc[7] = {0, 0, 0, 0, 0, 0, 0};
  int last = -1;
  bool done = !c.inside;
  Window win;
  win_init(win);

  // blend the entry that leaves the window from slot m
  auto blend = [&](int m, int idx) {
    const float a = fminf(pay[m][0][lane], alpha_clamp);
    const float Tn = T * (1.0f - a);
    if (Tn < t_min) {
      done = true;
      return;
    }
    const float w = T * a;
    acc[0] = fmaf(w, pay[m][1][lane], acc[0]);
    acc[1] = fmaf(w, pay[m][2][lane], acc[1]);
    acc[2] = fmaf(w, pay[m][3][lane], acc[2]);
    acc[3] = fmaf(w, pay[m][4][lane], acc[3]);
    acc[4] = fmaf(w, pay[m][5][lane], acc[4]);
    acc[5] = fmaf(w, pay[m][6][lane], acc[5]);
    acc[6] = fmaf(w, pay[m][7][lane], acc[6]);
    O += w;
    Tb = T;
    T = Tn;
    last = idx;
    if (T == 0.0f) done = true;
  };

  if (threadIdx.x == 0) done_mask = 0ull;
  __syncthreads();
  if (wave == 0) {
    const unsigned long long m = __ballot(done);
    if (lane == 0) done_mask = m;
  }
  RecPipe<CHW, NT> rp;
  if (start < end) {
    rp.fetch_idx(srec, start, (int)min((uint32_t)CHW, end - start));
    rp.fetch_rec(vrec);
    if (end - start > (uint32_t)CHW) rp.fetch_idx(srec, start + CHW, (int)min((uint32_t)CHW, end - start - CHW));
  }
  for (uint32_t base = start; base < end; base += CHW) {
    __syncthreads();
    if (done_mask == ~0ull) break;
    const int n = (int)min((uint32_t)CHW, end - base);
    rp.store(recs, n);
    if (end - base > (uint32_t)CHW) rp.fetch_rec(vrec);
    if (end - base > 2u * CHW) rp.fetch_idx(srec, base + 2 * CHW, (int)min((uint32_t)CHW, end - base - 2 * CHW));
    __syncthreads();
    load_chunk_tables(recs, n, feat, hm, NT);
    if (wave == 0) chunk_pairs<CHW>(recs, n, c, ~done_mask, pmask, poff);
    __syncthreads();
    for_each_pair<CHW>(n, pmask, poff, NT, [&](int e, int pix) {
      const float px_ = (float)(c.tx * 8 + (pix & 7)) + 0.5f, py_ = (float)(c.ty * 8 + (pix >> 3)) + 0.5f;
      PixEval h;
      if (pixel_eval(recs[e], px_, py_, s, h) && h.alpha >= alpha_min) {
        alds[e][pix] = h.alpha;
        zlds[e][pix] = h.zin_inv;
        atomicOr(&hm[pix], 1u << e);
      }
    });
    __syncthreads();
    if (wave == 0) {
      // each pixel's candidates in arrival order
      uint32_t cand = done ? 0u : hm[lane];
      while (__ballot(cand != 0u) != 0ull) {
        if (cand != 0u) {
          const int e = __ffs(cand) - 1;
          cand &= cand - 1u;
          const int slot = win_insert(win, zlds[e][lane], (int)(base + e));
          pay[slot][0][lane] = alds[e][lane];
#pragma unroll
          for (int k = 0; k < 7; ++k) pay[slot][1 + k][lane] = feat[k][e];
          if (win.cnt > nw) {
            int idx;
            const int m = win_pop(win, &idx);
            blend(m, idx);
          }
          if (done) cand = 0u;
        }
      }
      const unsigned long long m = __ballot(done);
      if (lane == 0) done_mask = m;
    }
  }
  if (wave == 0) {
    // end of the list: the rest of the window leaves nearest first
    while (__ballot(!done && win.cnt > 0) != 0ull) {
      if (!done && win.cnt > 0) {
        int idx;
        const int m = win_pop(win, &idx);
        blend(m, idx);
      }
    }
    if (c.inside) {
      const size_t plane = (size_t)V.W * V.H;
      const size_t px = (size_t)c.j * V.W + c.i;
      float* out = V.out;
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
}

// A 5-waves-per-SIMD target fits the backward in 96 VGPRs without spills:
// one more resident workgroup per CU.
template <int NWV>
__global__ __launch_bounds__(64 * NWV) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_composite_bwd_win(void* ws, Layout L, float alpha_min,
                                                                float alpha_clamp, float t_min, int nw) {
  constexpr int NT = 64 * NWV;
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const uint32_t* srec = at<const uint32_t>(ws, sorted_entry_records(L));
  const ViewRec* vrec = at<const ViewRec>(ws, L.o_vrec);
  float* tgrad = at<float>(ws, L.o_tgrad);
  uint8_t* eflag = at<uint8_t>(ws, L.o_eflag);
  // per (entry, lane): {T before the blend, raw alpha, g . features, previous
  // blended entry}; sweep 2 turns the first two into {dL/dalpha, T alpha}
  float4* pairs = at<float4>(ws, L.o_wpair);
  __shared__ ViewRec recs[CHW];
  __shared__ float alds[CHW][64];
  __shared__ float zlds[CHW][64];
  __shared__ float pay[WSLOTS][2][64];  // per slot: raw alpha, g . features
  __shared__ float gacc[CHW][TGRAD_STRIDE];
  __shared__ unsigned long long done_mask;

  const Tile8 c = tile8(vw, at<const TileSlot>(ws, L.o_tile_order));
  const DevView& V = vw[c.view];
  const float s = V.s;
  const uint32_t start = c.start, end = c.end;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float qx = (float)c.i + 0.5f, qy = (float)c.j + 0.5f;
  const size_t plane = (size_t)V.W * V.H;
  const size_t px = c.inside ? (size_t)c.j * V.W + c.i : 0;
  float gr[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) gr[q] = c.inside ? V.dout[q * plane + px] : 0.0f;

  // ---- sweep 1: the window front to back, recording every blend
  float T = 1.0f;
  int prev = -1;  // this pixel's last blended entry
  bool done = !c.inside;
  Window win;
  win_init(win);
  auto record = [&](int m, int idx) {
    const float araw = pay[m][0][lane], sdot = pay[m][1][lane];
    const float a = fminf(araw, alpha_clamp);
    const float Tn = T * (1.0f - a);
    if (Tn < t_min) {
      done = true;
      return;
    }
    pairs[(size_t)idx * 64 + lane] = make_float4(T, araw, sdot, __int_as_float(prev));
    prev = idx;
    T = Tn;
    if (T == 0.0f) done = true;
  };

  if (threadIdx.x == 0) done_mask = 0ull;
  __syncthreads();
  if (wave == 0) {
    const unsigned long long m = __ballot(done);
    if (lane == 0) done_mask = m;
  }
  uint32_t pend = start;  // end of the walked part of the list
  for (uint32_t base = start; base < end; base += CHW) {
    __syncthreads();
    if (done_mask == ~0ull) break;
    const int n = (int)min((uint32_t)CHW, end - base);
    pend = base + (uint32_t)n;
    load_recs(recs, vrec, srec, base, n, NT);
    __syncthreads();
    eval_chunk<NWV>(recs, n, c, qx, qy, s, (done_mask >> lane) & 1ull, alds, zlds);
    // every walked pair starts as "not blended"
    for (int e = wave; e < n; e += NWV) pairs[(size_t)(base + e) * 64 + lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    __syncthreads();
    if (wave == 0) {
      for (int e = 0; e < n; ++e) {
        const float a = alds[e][lane];
        if (done || a < 0.0f || a < alpha_min) continue;
        const int slot = win_insert(win, zlds[e][lane], (int)(base + e));
        const ViewRec& R = recs[e];
        const float sdot = gr[0] * R.c[0] + gr[1] * R.c[1] + gr[2] * R.c[2] + gr[3] + gr[4] * R.zt +
                           gr[5] * R.n[0] + gr[6] * R.n[1] + gr[7] * R.n[2];
        pay[slot][0][lane] = a;
        pay[slot][1][lane] = sdot;
        if (win.cnt > nw) {
          int idx;
          const int m = win_pop(win, &idx);
          record(m, idx);
        }
      }
      const unsigned long long m = __ballot(done);
      if (lane == 0) done_mask = m;
    }
  }
  if (wave == 0) {
    while (__ballot(!done && win.cnt > 0) != 0ull) {
      if (!done && win.cnt > 0) {
        int idx;
        const int m = win_pop(win, &idx);
        record(m, idx);
      }
    }
    // ---- sweep 2: each pixel's blends from the last one back; Rbehind is
    // the upstream gradient dotted with what lies behind, per unit of T
    float Rbehind = gr[0] * V.bg[0] + gr[1] * V.bg[1] + gr[2] * V.bg[2];
    int k = prev;
    while (__ballot(k >= 0) != 0ull) {
      if (k >= 0) {
        float4* p = &pairs[(size_t)k * 64 + lane];
        const float4 v = *p;
        const float Tk = v.x, araw = v.y, sdot = v.z;
        const float a = fminf(araw, alpha_clamp);
        float da = Tk * (sdot - Rbehind);
        Rbehind = a * sdot + (1.0f - a) * Rbehind;
        if (araw > alpha_clamp) da = 0.0f;
        *reinterpret_cast<float2*>(p) = make_float2(da, Tk * a);
        k = __float_as_int(v.w);
      }
    }
  }
  // ---- sweep 3: per-entry gradients in tile order, reduced over the tile
  for (uint32_t base = start; base < pend; base += CHW) {
    const int n = (int)min((uint32_t)CHW, pend - base);
    __syncthreads();
    load_recs(recs, vrec, srec, base, n, NT, at<const uint4>(ws, L.o_rbox));
    __syncthreads();
    for (int e = wave; e < n; e += NWV) {
      const float2 dw = *reinterpret_cast<const float2*>(&pairs[(size_t)(base + e) * 64 + lane]);
      const float da = dw.x, w = dw.y;
      const bool contrib = (da != 0.0f) || (w != 0.0f);
      if (__ballot(contrib) == 0ull) {
        if (lane < (unsigned)TGRAD_STRIDE) gacc[e][lane] = 0.0f;
        continue;
      }
      // branch-free: a lane that did not blend this entry chains zero
      // weights (zero gradient)
      float g[32];
      {
        const ViewRec& R = recs[e];
        PixEval h;
        pixel_eval(R, qx, qy, s, h);
        float dd, dfn;
        eq1_chain(da, h.alpha, h.e2, s, dd, dfn);
        pair_grad_all(R, qx, qy, gr, dd, dfn, w, h.fe | (h.fx << 2), g);
      }
      const float tot = wave_transpose_sum32(g);
      const unsigned q = lane >> 1;
      if ((lane & 1u) == 0u && q < (unsigned)TGRAD_STRIDE) gacc[e][q] = tot;
    }
    __syncthreads();
    store_entry_grads(recs, gacc, n, c, tgrad, eflag, NT, (uint64_t)L.entry_cap,
                      record_grads(L) ? srec + base : nullptr);
  }
}

template <int NWV>
static void launch_fwd_win(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  k_composite_win<NWV><<<(unsigned)L.total_tiles, 64 * NWV, 0, st>>>(ws, L, p.alpha_min, p.alpha_clamp, p.t_min,
                                                                      p.window);
}
template <int NWV>
static void launch_bwd_win(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  k_composite_bwd_win<NWV><<<(unsigned)L.total_tiles, 64 * NWV, 0, st>>>(ws, L, p.alpha_min, p.alpha_clamp,
                                                                          p.t_min, p.window);
}

hipError_t launch_composite_win(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  if (L.total_tiles == 0) return hipSuccess;
  if (p.window < 1 || p.window > RENDER_WINDOW_MAX || p.tile_w != 8 || p.tile_h != 8) return hipErrorInvalidValue;
  switch (p.waves) {
    case 1: launch_fwd_win<1>(ws, L, p, st); break;
    case 2: launch_fwd_win<2>(ws, L, p, st); break;
    case 4: launch_fwd_win<4>(ws, L, p, st); break;
    case 8: launch_fwd_win<8>(ws, L, p, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_composite_backward_win(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  if (L.total_tiles == 0) return hipSuccess;
  if (p.window < 1 || p.window > RENDER_WINDOW_MAX || p.tile_w != 8 || p.tile_h != 8 || L.o_wpair == 0)
    return hipErrorInvalidValue;
  switch (p.waves) {
    case 1: launch_bwd_win<1>(ws, L, p, st); break;
    case 2: launch_bwd_win<2>(ws, L, p, st); break;
    case 4: launch_bwd_win<4>(ws, L, p, st); break;
    case 8: launch_bwd_win<8>(ws, L, p, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ts
