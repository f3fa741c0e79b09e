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
// the window front to back and writes every blend, in the order the blends
// happen, to the tile's part of a blend buffer (a per-pixel list through
// each record's link to the pixel's previous blend), and marks the pixel in
// the entry's blend mask; the masks then give each entry's pairs their
// places, entry by entry in tile order and pixel by pixel inside an entry.
// Sweep 2 walks every pixel's list from its last blend back (the reverse mode
// of Eq. 2) and writes each pair, chained through Eq. 1, to its place; the
// flat pair-gradient kernel of the multi-wave path then sums each entry over
// the tile.  The forward counts each tile's blends so that the backward
// knows where its records and pairs go.
#include "tile8.h"

namespace ts {

namespace {

// A lane's window holds up to N_w entries, plus the arrival that overflows
// it: WS >= N_w + 1 slots (the kernels are built for WS in {2, 4, 6, 9}, the
// smallest that fits N_w, so the slot scans stay short).
constexpr int CHW = 32;       // entries per LDS chunk (forward)
// The backward's chunks are shorter: its per-(entry, pixel) arrays then fit
// four workgroups per CU.  Its replay makes the forward's decisions with any
// chunk length (they are per pixel and per candidate, in tile order), and it
// walks exactly the forward's walked range.
constexpr int CHW_BWD = 16;

// One lane's window.  key = 1 / entry depth (larger is nearer), -1 for a free
// slot (a hit's key is positive); idx = global entry index (arrival order).
template <int WS>
struct Window {
  float key[WS];
  int idx[WS];
  int cnt;
};

template <int WS>
__device__ __forceinline__ void win_init(Window<WS>& w) {
#pragma unroll
  for (int k = 0; k < WS; ++k) {
    w.key[k] = -1.0f;
    w.idx[k] = 0;
  }
  w.cnt = 0;
}

// Puts (key, idx) into the lowest free slot and returns that slot.
template <int WS>
__device__ __forceinline__ int win_insert(Window<WS>& w, float key, int idx) {
  int slot = 0;
#pragma unroll
  for (int k = WS - 1; k >= 0; --k) slot = (w.key[k] < 0.0f) ? k : slot;
#pragma unroll
  for (int k = 0; k < WS; ++k) {
    const bool here = k == slot;
    w.key[k] = here ? key : w.key[k];
    w.idx[k] = here ? idx : w.idx[k];
  }
  ++w.cnt;
  return slot;
}

// Takes the nearest entry out (largest key; equal keys: earliest arrival) and
// returns its slot; *idx receives its entry index.  Needs cnt > 0.
template <int WS>
__device__ __forceinline__ int win_pop(Window<WS>& w, int* idx) {
  int m = 0;
  float bk = w.key[0];
  int bi = w.idx[0];
#pragma unroll
  for (int k = 1; k < WS; ++k) {
    const bool better = w.key[k] > bk || (w.key[k] == bk && bk >= 0.0f && w.idx[k] < bi);
    m = better ? k : m;
    bk = better ? w.key[k] : bk;
    bi = better ? w.idx[k] : bi;
  }
#pragma unroll
  for (int k = 0; k < WS; ++k) w.key[k] = (k == m) ? -1.0f : w.key[k];
  --w.cnt;
  *idx = bi;
  return m;
}

// A blend mask, set by atomics (done in L2): read from L2 as well, past any
// copy of its line in this CU's L1 (one brought in by a neighbouring slot).
__device__ __forceinline__ unsigned long long mask_load(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

template <int NWV, int WS>
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
  __shared__ PairMap<CHW> pm;
  __shared__ uint32_t hm[64];           // per pixel: the chunk's candidates (bit e)
  __shared__ float pay[WS][8][64];      // per slot: alpha, c[3], zt, n[3]
  __shared__ unsigned long long done_mask;

  const Tile8 c = tile8(vw, at<const TileSlot>(ws, L.o_tile_order));
  const DevView& V = vw[c.view];
  const float s = uniform_f(V.s);
  const uint32_t start = c.start, end = c.end;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float qx = (float)c.i + 0.5f, qy = (float)c.j + 0.5f;

  float T = 1.0f, Tb = 1.0f, O = 0.0f;
  float acc[7] = {0, 0, 0, 0, 0, 0, 0};
  int last = -1;
  bool done = !c.inside;
  uint32_t nblend = 0;    // this pixel's blends
  uint32_t walked = start;  // end of the chunks walked
  Window<WS> win;
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
    ++nblend;
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
    rp.fetch_idx(srec, start, end - 1);
    rp.fetch_rec(vrec);
    rp.fetch_idx(srec, start + CHW, end - 1);
  }
  for (uint32_t base = start; base < end; base += CHW) {
    __syncthreads();
    if (done_mask == ~0ull) break;
    const int n = (int)min((uint32_t)CHW, end - base);
    walked = base + (uint32_t)n;
    rp.store(recs, n);
    rp.fetch_rec(vrec);
    rp.fetch_idx(srec, base + 2 * CHW, end - 1);
    __syncthreads();
    load_chunk_tables(recs, n, feat, hm, NT);
    if (wave == 0) chunk_pairs<CHW>(recs, n, c, ~done_mask, pm);
    __syncthreads();
    for_each_pair<CHW>(pm, NT, [&](int e, int pix) {
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
    // the tile's blends and walked length: where the backward puts its
    // records and pairs, and its dispatch order (a tile with no blend has
    // nothing to walk back)
    uint32_t nb = nblend;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nb += (uint32_t)__shfl_xor((int)nb, o, 64);
    if (lane == 0) {
      const uint32_t pend = nb > 0u ? walked : start;
      at<uint32_t>(ws, L.o_tile_pend)[blockIdx.x] = pend;
      at<uint32_t>(ws, L.o_slot_pairs)[blockIdx.x] = nb;
      if (pend > start) {
        uint32_t* bh = at<uint32_t>(ws, L.o_bwd_hist);
        const int b = len_bucket(pend - start);
        atomicAdd(bh + b, 1u);
        atomicAdd(bh + 2 * TILE_BUCKETS + b, nb);
      }
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
}

// Backward, with NWV waves per 8x8 tile, dispatched longest walk first (the
// tiles with no blend leave at once).
// Sweep 1 replays the window front to back exactly as the forward runs it
// (packed evaluation of the live (entry, pixel) pairs, then each pixel's
// candidates through its window, in wave 0) and writes every blend, in the
// order the blends happen, to the tile's part of the blend buffer: T before
// the blend, raw alpha, the upstream gradient dotted with the entry's
// features, exp(s f_next), the pixel's previous blend (a per-pixel list),
// faces and pixel, record and gradient slot; and sets the pixel's bit in the
// entry's blend mask.  Then the tile's walked entries, in tile order, get the
// places of their pairs: the exclusive sum of their masks' pixel counts.
// Sweep 2 (wave 0) walks every pixel's list from its last blend back (the
// reverse mode of Eq. 2), chains dL/dalpha through Eq. 1 and writes the pair
// to its place, in the pair format of the multi-wave backward: an entry's
// pairs consecutive in pixel order, so the flat pair-gradient kernel sums
// each entry over the tile in a fixed order.
template <int NWV, int WS>
__global__ __launch_bounds__(64 * NWV) void k_composite_bwd_win(void* ws, Layout L, float alpha_min,
                                                                float alpha_clamp, float t_min, int nw) {
  constexpr int NT = 64 * NWV;
  constexpr int CHB = CHW_BWD;
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const uint32_t* srec = at<const uint32_t>(ws, sorted_entry_records(L));
  const ViewRec* vrec = at<const ViewRec>(ws, L.o_vrec);
  const uint4* rbox = at<const uint4>(ws, L.o_rbox);
  const uint32_t* rfirst = at<const uint32_t>(ws, L.o_rfirst);
  uint4* blends = at<uint4>(ws, L.o_wblend);
  unsigned long long* emask = at<unsigned long long>(ws, L.o_wmask);
  uint32_t* ebase = at<uint32_t>(ws, L.o_wbase);
  uint4* pairs = at<uint4>(ws, L.o_pairs);
  const uint64_t cap = (uint64_t)L.entry_cap;
  __shared__ ViewRec recs[CHB];
  __shared__ float alds[CHB][64];       // raw alpha
  __shared__ float zlds[CHB][64];       // window key: 1 / entry depth
  __shared__ float e2lds[CHB][64];      // exp(s f_next)
  __shared__ uint8_t sel[CHB][64];      // entry face | exit face << 2
  __shared__ float feat[7][CHB];        // per entry: c[3], zt, n[3]
  __shared__ uint32_t erec[CHB], eslot[CHB];   // per entry: record, gradient slot
  __shared__ PairMap<CHB> pm;
  __shared__ uint32_t hm[64];           // per pixel: the chunk's candidates (bit e)
  __shared__ uint32_t pay[WS][6][64];   // per slot: raw alpha, g . features, e2, faces, record, slot
  __shared__ uint32_t wsum[NWV];
  __shared__ unsigned long long done_mask;

  const TileSlot* bslots = at<const TileSlot>(ws, L.o_bwd_order);
  if (blockIdx.x >= at<const DevHeader>(ws, L.o_hdr)->bwd_work) return;
  const uint32_t pend = at<const uint32_t>(ws, L.o_bwd_pend)[blockIdx.x];
  if (pend == bslots[blockIdx.x].start) return;
  const Tile8 c = tile8(vw, bslots);
  const DevView& V = vw[c.view];
  const float s = uniform_f(V.s);
  const uint32_t start = c.start, end = pend;   // the forward walked [start, pend)
  const unsigned lane = threadIdx.x & 63u;
  const int wave = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint32_t pair0 = at<const uint32_t>(ws, L.o_bwd_base)[blockIdx.x];   // the tile's first blend / pair
  const uint32_t tile_xy = (uint32_t)c.tx | ((uint32_t)c.ty << 16);
  const size_t plane = (size_t)V.W * V.H;
  const size_t px = c.inside ? (size_t)c.j * V.W + c.i : 0;
  float gr[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) gr[q] = c.inside ? gmem(V.dout)[q * plane + px] : 0.0f;

  // ---- sweep 1 (window and blend records in wave 0)
  float T = 1.0f;
  int prev = -1;          // this pixel's last blend (index into the blend buffer)
  uint32_t run = pair0;   // next blend's place (wave-uniform)
  bool done = !c.inside;
  Window<WS> win;
  win_init(win);
  // one step of every lane that pops slot m (pop set): blend or stop; the
  // blends of the step take consecutive places in lane order
  auto step = [&](bool pop, int m) {
    bool bl = false;
    float a = 0.0f, Tn = 0.0f;
    if (pop) {
      a = fminf(__uint_as_float(pay[m][0][lane]), alpha_clamp);
      Tn = T * (1.0f - a);
      if (Tn < t_min) done = true;
      else bl = true;
    }
    const uint64_t bm = __ballot(bl);
    if (bl) {
      const uint32_t k = run + (uint32_t)__popcll(bm & lt);
      const uint32_t d = pay[m][5][lane];
      if ((uint64_t)k < cap) {
        blends[2 * (size_t)k] = make_uint4(__float_as_uint(T), pay[m][0][lane], pay[m][1][lane], pay[m][2][lane]);
        blends[2 * (size_t)k + 1] = make_uint4((uint32_t)prev, pay[m][3][lane] | (lane << 8), pay[m][4][lane], d);
      }
      if ((uint64_t)d < cap) atomicOr(&emask[d], 1ull << lane);
      prev = (uint64_t)k < cap ? (int)k : -1;   // (past the capacity: an overflowed forward)
      T = Tn;
      if (T == 0.0f) done = true;
    }
    run += (uint32_t)__popcll(bm);
  };

  if (threadIdx.x == 0) done_mask = 0ull;
  __syncthreads();
  if (wave == 0) {
    const unsigned long long m = __ballot(done);
    if (lane == 0) done_mask = m;
  }
  RecPipe<CHB, NT, true> rp;
  if (start < end) {
    rp.fetch_idx(srec, start, end - 1);
    rp.fetch_rec(vrec, rfirst);
    rp.fetch_idx(srec, start + CHB, end - 1);
  }
  for (uint32_t base = start; base < end; base += CHB) {
    __syncthreads();
    if (done_mask == ~0ull) break;
    const int n = (int)min((uint32_t)CHB, end - base);
    rp.store(recs, n, erec);
    rp.fetch_rec(vrec, rfirst);
    rp.fetch_idx(srec, base + 2 * CHB, end - 1);
    __syncthreads();
    load_chunk_tables(recs, n, feat, hm, NT);
    if (threadIdx.x < (unsigned)n) {
      // the entry's gradient slot (its record came with the chunk's records);
      // its blend mask starts empty
      const ViewRec& R = recs[threadIdx.x];
      int i0, i1, j0, j1;
      unpack_rect(R, i0, i1, j0, j1);
      const int tx0 = i0 >> 3, ty0 = j0 >> 3, nx = (i1 >> 3) - tx0 + 1;
      const uint32_t d = R.entry0 + (uint32_t)((c.ty - ty0) * nx + (c.tx - tx0));
      eslot[threadIdx.x] = d;
      if ((uint64_t)d < cap) emask[d] = 0ull;
    }
    if (wave == 0) chunk_pairs<CHB>(recs, n, c, ~done_mask, pm);
    __syncthreads();
    for_each_pair<CHB>(pm, NT, [&](int e, int pix) {
      const float px_ = (float)(c.tx * 8 + (pix & 7)) + 0.5f, py_ = (float)(c.ty * 8 + (pix >> 3)) + 0.5f;
      PixEval h;
      if (pixel_eval(recs[e], px_, py_, s, h) && h.alpha >= alpha_min) {
        alds[e][pix] = h.alpha;
        zlds[e][pix] = h.zin_inv;
        e2lds[e][pix] = h.e2;
        sel[e][pix] = (uint8_t)(h.fe | (h.fx << 2));
        atomicOr(&hm[pix], 1u << e);
      }
    });
    __syncthreads();
    if (wave == 0) {
      // each pixel's candidates in arrival order
      uint32_t cand = done ? 0u : hm[lane];
      while (__ballot(cand != 0u) != 0ull) {
        bool pop = false;
        int m = 0;
        if (cand != 0u) {
          const int e = __ffs(cand) - 1;
          cand &= cand - 1u;
          const int slot = win_insert(win, zlds[e][lane], (int)(base + e));
          const float sdot = gr[0] * feat[0][e] + gr[1] * feat[1][e] + gr[2] * feat[2][e] + gr[3] +
                             gr[4] * feat[3][e] + gr[5] * feat[4][e] + gr[6] * feat[5][e] + gr[7] * feat[6][e];
          pay[slot][0][lane] = __float_as_uint(alds[e][lane]);
          pay[slot][1][lane] = __float_as_uint(sdot);
          pay[slot][2][lane] = __float_as_uint(e2lds[e][lane]);
          pay[slot][3][lane] = sel[e][lane];
          pay[slot][4][lane] = erec[e];
          pay[slot][5][lane] = eslot[e];
          if (win.cnt > nw) {
            int idx;
            m = win_pop(win, &idx);
            pop = true;
          }
        }
        step(pop, m);
        if (done) cand = 0u;
      }
      const unsigned long long dm = __ballot(done);
      if (lane == 0) done_mask = dm;
    }
  }
  if (wave == 0) {
    // end of the list: the rest of the window leaves nearest first
    while (__ballot(!done && win.cnt > 0) != 0ull) {
      bool pop = false;
      int m = 0;
      if (!done && win.cnt > 0) {
        int idx;
        m = win_pop(win, &idx);
        pop = true;
      }
      step(pop, m);
    }
  }
  __syncthreads();

  // ---- the places of the pairs: per walked entry, in tile order, the
  // exclusive sum of its blend counts (the masks are complete)
  uint32_t carry = pair0;
  for (uint32_t b0 = start; b0 < end; b0 += NT) {
    const uint32_t idx = b0 + threadIdx.x;
    uint32_t d = 0u, cnt = 0u;
    if (idx < end) {
      const uint32_t r = srec[idx];
      const uint4 bx = rbox[r];   // pixel rectangle, view
      const int i0 = (int)(bx.x & 0xffffu), i1 = (int)(bx.x >> 16), j0 = (int)(bx.y & 0xffffu),
                j1 = (int)(bx.y >> 16);
      const int tx0 = i0 >> 3, ty0 = j0 >> 3, nx = (i1 >> 3) - tx0 + 1;
      d = rfirst[r] + (uint32_t)((c.ty - ty0) * nx + (c.tx - tx0));
      (void)j1;
      cnt = (uint64_t)d < cap ? (uint32_t)__popcll(mask_load(emask + d)) : 0u;
    }
    uint32_t x = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      x += lane >= (unsigned)o ? y : 0u;
    }
    if (lane == 63u) wsum[wave] = x;
    __syncthreads();
    uint32_t before = carry;
    for (int q = 0; q < wave; ++q) before += wsum[q];
    if (cnt > 0u && (uint64_t)d < cap) ebase[d] = before + x - cnt;
    for (int q = 0; q < NWV; ++q) carry += wsum[q];
    __syncthreads();
  }

  // ---- sweep 2: each pixel's blends from the last one back; Rbehind is the
  // upstream gradient dotted with what lies behind, per unit of T
  if (wave == 0) {
    float Rbehind = gr[0] * V.bg[0] + gr[1] * V.bg[1] + gr[2] * V.bg[2];
    int k = prev;
    while (__ballot(k >= 0) != 0ull) {
      if (k >= 0) {
        const uint4 b0 = blends[2 * (size_t)k], b1 = blends[2 * (size_t)k + 1];
        const float Tk = __uint_as_float(b0.x), araw = __uint_as_float(b0.y), sdot = __uint_as_float(b0.z);
        const float e2 = __uint_as_float(b0.w);
        const float a = fminf(araw, alpha_clamp);
        float da = Tk * (sdot - Rbehind);
        Rbehind = a * sdot + (1.0f - a) * Rbehind;
        if (araw > alpha_clamp) da = 0.0f;
        float dd, dfn;
        eq1_chain(da, araw, e2, s, dd, dfn);
        const uint32_t d = b1.w;
        if ((uint64_t)d < cap) {
          const unsigned long long mk = mask_load(emask + d);
          const unsigned long long below = mk & lt;
          const uint32_t pos = ebase[d] + (uint32_t)__popcll(below);
          const uint32_t hw = below == 0ull ? PAIR_HEAD | ((uint32_t)__popcll(mk) << 11) : 0u;
          if ((uint64_t)pos < cap) {
            pairs[2 * (size_t)pos] = make_uint4(__float_as_uint(dd), __float_as_uint(dfn), __float_as_uint(Tk * a),
                                                lane | ((b1.y & 15u) << 6) | hw);
            pairs[2 * (size_t)pos + 1] = make_uint4(b1.z, (uint32_t)c.view, tile_xy, d);
          }
        }
        k = (int)b1.x;
      }
    }
  }
}

template <int NWV, int WS>
static void launch_fwd_win_ws(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  k_composite_win<NWV, WS><<<(unsigned)L.total_tiles, 64 * NWV, 0, st>>>(ws, L, p.alpha_min, p.alpha_clamp,
                                                                          p.t_min, p.window);
}
template <int NWV, int WS>
static void launch_bwd_win_ws(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  k_composite_bwd_win<NWV, WS><<<(unsigned)L.total_tiles, 64 * NWV, 0, st>>>(ws, L, p.alpha_min, p.alpha_clamp,
                                                                              p.t_min, p.window);
}
// the smallest slot count that holds N_w entries and one arrival
template <int NWV>
static void launch_fwd_win(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  if (p.window <= 1) launch_fwd_win_ws<NWV, 2>(ws, L, p, st);
  else if (p.window <= 3) launch_fwd_win_ws<NWV, 4>(ws, L, p, st);
  else if (p.window <= 5) launch_fwd_win_ws<NWV, 6>(ws, L, p, st);
  else launch_fwd_win_ws<NWV, RENDER_WINDOW_MAX + 1>(ws, L, p, st);
}
template <int NWV>
static void launch_bwd_win(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  if (p.window <= 1) launch_bwd_win_ws<NWV, 2>(ws, L, p, st);
  else if (p.window <= 3) launch_bwd_win_ws<NWV, 4>(ws, L, p, st);
  else if (p.window <= 5) launch_bwd_win_ws<NWV, 6>(ws, L, p, st);
  else launch_bwd_win_ws<NWV, RENDER_WINDOW_MAX + 1>(ws, L, p, st);
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
  if (p.window < 1 || p.window > RENDER_WINDOW_MAX || p.tile_w != 8 || p.tile_h != 8 || L.o_wblend == 0 ||
      L.o_pairs == 0)
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
