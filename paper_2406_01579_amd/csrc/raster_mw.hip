// Multi-wave compositing kernels for 8x8 tiles.
//
// A tile's entry list is walked front to back (forward) or back to front
// (backward) by one pixel per lane, and the per-pixel state along the list
// (transmittance, the colour behind) is a short sequential recurrence.  The
// expensive part of every (pixel, entry) pair -- coverage of the projected
// hull, entry/exit SDF values and Eq. 1 -- does not depend on that state.
// So NWV waves share one 8x8 tile: for each LDS chunk of entries they
// evaluate the (entry, pixel) pairs that can hit in parallel into LDS, and one
// wave runs the recurrence over the chunk.  The backward's recurrence leaves,
// per blended pair, dL/df_prev, dL/df_next and the blend weight in a pair
// buffer, grouped per (tile, entry) segment; a second, flat kernel chains
// every pair to its record's 23 screen-space parameters and sums each
// segment, with no per-tile sequence and no atomics.  The forward counts
// each tile's blended pairs and segments so that every backward workgroup
// knows where its pairs go.  Images are bit-identical to the one-wave kernels
// (the same per-pair arithmetic in the same order).
#include "tile8.h"

namespace ts {

namespace {


// Forward sweep over [start, end) with NWV waves; wave 0 ends with the
// pixel's blend state.  Used by the forward kernel and by the backward's
// state replay.
template <int NWV, int CHN>
__device__ __forceinline__ void forward_sweep(const ViewRec* __restrict__ vrec, const uint32_t* __restrict__ srec,
                                              uint32_t start, uint32_t end, const Tile8& c, float s, float alpha_min,
                                              float alpha_clamp, float t_min, ViewRec* recs, float (*alds)[64],
                                              PairMap<CHN>& pm, uint64_t* hm, float (*feat)[CHN],
                                              unsigned long long* done_mask,
                                              float& T, float& Tb, float& O, float (&acc)[7], int& last,
                                              bool want_acc, uint32_t& nblend,
                                              unsigned long long* bmask = nullptr) {
  constexpr int NT = 64 * NWV;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bool done = !c.inside;
  if (threadIdx.x == 0) *done_mask = 0ull;
  __syncthreads();
  if (wave == 0) {
    const unsigned long long m = __ballot(done);
    if (lane == 0) *done_mask = m;
  }
  RecPipe<CHN, NT> rp;
  if (start < end) {
    rp.fetch_idx(srec, start, end - 1);
    rp.fetch_rec(vrec);
    rp.fetch_idx(srec, start + CHN, end - 1);
  }
  for (uint32_t base = start; base < end; base += CHN) {
    __syncthreads();
    if (*done_mask == ~0ull) break;
    const int n = (int)min((uint32_t)CHN, end - base);
    rp.store(recs, n);
    rp.fetch_rec(vrec);
    rp.fetch_idx(srec, base + 2 * CHN, end - 1);
    __syncthreads();
    // phase A: coverage and Eq. 1 of the live (entry, pixel) pairs, packed;
    // hm[pixel] collects the chunk entries the pixel may blend
    if (threadIdx.x < 64) hm[threadIdx.x] = 0ull;
    for (int q = threadIdx.x; q < n * 7; q += NT) {
      const int e = q / 7, k = q - e * 7;
      feat[k][e] = k < 3 ? recs[e].c[k] : k == 3 ? recs[e].zt : recs[e].n[k - 4];
    }
    if (wave == 0) chunk_pairs<CHN>(recs, n, c, ~*done_mask, pm);
    __syncthreads();
    for_each_pair<CHN>(pm, NT, [&](int e, int pix) {
      const float qx = (float)(c.tx * 8 + (pix & 7)) + 0.5f, qy = (float)(c.ty * 8 + (pix >> 3)) + 0.5f;
      PixEval h;
      if (pixel_eval(recs[e], qx, qy, s, h) && h.alpha >= alpha_min) {
        alds[e][pix] = h.alpha;
        atomicOr(&hm[pix], 1ull << e);
      }
    });
    __syncthreads();
    if (wave == 0) {
      // each pixel visits only its candidate entries, front to back
      uint64_t cand = hm[lane];
      uint64_t blended = 0ull;   // this lane's blended entries of the chunk
      while (__ballot(cand != 0ull && !done) != 0ull) {
        if (cand != 0ull && !done) {
          const int e = __ffsll((unsigned long long)cand) - 1;
          cand &= cand - 1ull;
          const float a = fminf(alds[e][lane], alpha_clamp);
          const float Tn = T * (1.0f - a);
          if (Tn < t_min) {
            done = true;
          } else {
            const float w = T * a;
            if (want_acc) {
              acc[0] = fmaf(w, feat[0][e], acc[0]);
              acc[1] = fmaf(w, feat[1][e], acc[1]);
              acc[2] = fmaf(w, feat[2][e], acc[2]);
              acc[3] = fmaf(w, feat[3][e], acc[3]);
              acc[4] = fmaf(w, feat[4][e], acc[4]);
              acc[5] = fmaf(w, feat[5][e], acc[5]);
              acc[6] = fmaf(w, feat[6][e], acc[6]);
              O += w;
            }
            Tb = T;
            T = Tn;
            last = (int)(base + e);
            blended |= 1ull << e;
            if (T == 0.0f) done = true;
          }
        }
      }
      nblend += (uint32_t)__popcll(blended);   // the chunk's blended pairs (per lane)
      if (bmask) {
        // per entry of the chunk, the pixels that blended it (what the
        // backward's pairs are): lane e writes entry e's mask
        const uint64_t mine = wave_transpose64(blended);
        if (lane < n) bmask[base + lane] = mine;
      }
      const unsigned long long m = __ballot(done);
      if (lane == 0) *done_mask = m;
    }
  }
  __syncthreads();
}

// Background of `count` tiles with an empty list (the dispatch slots from
// `first`; a workgroup takes up to EMPTY_PER_WG of them): the outputs of a
// pixel no record reaches (T = 1), no blended entry, and the tile's end of
// blended prefix at its start.
constexpr uint32_t EMPTY_PER_WG = 16;
template <int NT>
__device__ __forceinline__ void background_tiles(void* ws, const Layout& L, const DevView* vw, uint32_t first,
                                                 uint32_t count) {
  const TileSlot* slots = at<const TileSlot>(ws, L.o_tile_order);
  uint32_t* tpend = at<uint32_t>(ws, L.o_tile_pend);
  int32_t* last_out = at<int32_t>(ws, L.o_last);
  float* tlast_out = at<float>(ws, L.o_tlast);
  for (uint32_t q = threadIdx.x; q < count * 64u; q += NT) {
    const uint32_t slot = first + (q >> 6);
    const int pix = (int)(q & 63u);
    const TileSlot sl = slots[slot];
    const DevView& V = vw[sl.view];
    if (pix == 0) tpend[slot] = sl.start;
    const int lt = (int)sl.tile - V.tile_base;
    const int i = (lt % V.tiles_x) * 8 + (pix & 7), j = (lt / V.tiles_x) * 8 + (pix >> 3);
    if (i >= V.W || j >= V.H) continue;
    const size_t plane = (size_t)V.W * V.H;
    const size_t px = (size_t)j * V.W + i;
    auto* out = gmem(V.out);
    out[0 * plane + px] = V.bg[0];
    out[1 * plane + px] = V.bg[1];
    out[2 * plane + px] = V.bg[2];
#pragma unroll
    for (int k = 3; k < 8; ++k) out[k * plane + px] = 0.0f;
    if (keeps_pixel_state(L)) {
      const size_t g = (size_t)V.pix_base + px;
      last_out[g] = -1;
      tlast_out[g] = 1.0f;
    }
  }
}

}  // namespace

template <int NWV, int CHN>
__global__ __launch_bounds__(64 * NWV) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_composite_mw(void* ws, Layout L, float alpha_min, float alpha_clamp,
                                                           float t_min) {
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const uint32_t* srec = at<const uint32_t>(ws, sorted_entry_records(L));
  const ViewRec* vrec = at<const ViewRec>(ws, L.o_vrec);
  int32_t* last_out = at<int32_t>(ws, L.o_last);
  float* tlast_out = at<float>(ws, L.o_tlast);
  __shared__ ViewRec recs[CHN];
  __shared__ float alds[CHN][64];
  __shared__ PairMap<CHN> pm;
  __shared__ uint64_t hm[64];
  __shared__ float feat[7][CHN];
  __shared__ unsigned long long done_mask;

  // the tiles with an empty list take the last slots (length bucket 0):
  // workgroups past the others write their background, EMPTY_PER_WG tiles
  // each, and the rest of the grid leaves at once
  {
    const uint32_t n_empty = at<const uint32_t>(ws, L.o_tile_hist)[0];
    const uint32_t n_work = (uint32_t)L.total_tiles - n_empty;
    if (blockIdx.x >= n_work) {
      const uint32_t first = n_work + (blockIdx.x - n_work) * EMPTY_PER_WG;
      if (first < (uint32_t)L.total_tiles)
        background_tiles<64 * NWV>(ws, L, vw, first, min(EMPTY_PER_WG, (uint32_t)L.total_tiles - first));
      return;
    }
  }
  const Tile8 c = tile8(vw, at<const TileSlot>(ws, L.o_tile_order));
  const DevView& V = vw[c.view];
  const float s = uniform_f(V.s);
  const uint32_t start = c.start, end = c.end;
  float T = 1.0f, Tb = 1.0f, O = 0.0f;
  float acc[7] = {0, 0, 0, 0, 0, 0, 0};
  int last = -1;
  uint32_t nblend = 0;
  const bool count = L.o_pairs != 0;
  forward_sweep<NWV, CHN>(vrec, srec, start, end, c, s, alpha_min, alpha_clamp, t_min, recs, alds, pm, hm,
                          feat, &done_mask, T, Tb, O, acc, last, true, nblend,
                          L.o_bmask ? at<unsigned long long>(ws, L.o_bmask) : nullptr);
  if ((threadIdx.x >> 6) == 0) {
    // end of the tile's blended prefix: where the backward starts its walk
    int wmax = last;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      wmax = max(wmax, __shfl_xor(wmax, o, 64));
      nblend += (uint32_t)__shfl_xor((int)nblend, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      const uint32_t pend = wmax >= (int)start ? (uint32_t)wmax + 1u : start;
      at<uint32_t>(ws, L.o_tile_pend)[blockIdx.x] = pend;
      if (count) at<uint32_t>(ws, L.o_slot_pairs)[blockIdx.x] = nblend;
      // the backward dispatch order's histograms of walked lengths and of
      // blended pairs (bucket 0, nothing walked, is not counted)
      if (pend > start) {
        uint32_t* bh = at<uint32_t>(ws, L.o_bwd_hist);
        const int b = len_bucket(pend - start);
        atomicAdd(bh + b, 1u);
        if (count) atomicAdd(bh + 2 * TILE_BUCKETS + b, nblend);
      }
    }
  }
  if ((threadIdx.x >> 6) == 0 && c.inside) {
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

// Backward, walk and recurrence: per chunk, coverage and Eq. 1 of every
// (entry, pixel) the pixel's walk reached, packed, then the reverse
// recurrence of Eq. 2 (one wave).  Every blended pair's dL/df_prev,
// dL/df_next and blend weight go to the pair buffer, entry-major inside the
// chunk, and every entry with a blended pixel gets a segment (its record, its
// per-(record, tile) gradient slot, its first pair and pair count); the
// tile's pairs and segments start at the bases the forward's counts gave
// this backward slot.
template <int NWV, int CHB>
__global__ __launch_bounds__(64 * NWV) void k_composite_bwd_mw(void* ws, Layout L, float alpha_min,
                                                               float alpha_clamp, float t_min, int recompute) {
  static_assert(CHB <= 32, "a pixel's chunk candidates are a 32-bit mask");
  constexpr int NT = 64 * NWV;
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const uint32_t* srec = at<const uint32_t>(ws, sorted_entry_records(L));
  const ViewRec* vrec = at<const ViewRec>(ws, L.o_vrec);
  const float* tlast_in = at<const float>(ws, L.o_tlast);
  const unsigned long long* bmask = at<const unsigned long long>(ws, L.o_bmask);
  uint4* pairs = at<uint4>(ws, L.o_pairs);
  __shared__ ViewRec recs[CHB];
  __shared__ uint4 eseg[CHB];        // per entry with a blended pixel: record, view, tile, gradient slot
  __shared__ uint32_t ridx[CHB];     // per entry: its record
  __shared__ float abuf[CHB][64];    // raw alpha
  __shared__ float e2buf[CHB][64];   // exp(s f_next)
  __shared__ uint8_t sel[CHB][64];   // entry face | exit face << 2
  __shared__ PairMap<CHB> pm;        // phase A's pairs
  __shared__ uint64_t pmask[CHB];    // phase B: per entry, the pixels that blended it
  __shared__ uint32_t poff[CHB + 1]; // and the places of its pairs
  __shared__ uint64_t hmask[64];     // per pixel: chunk entries it may have blended (bit e)
  __shared__ float feat[7][CHB];     // per entry: c[3], zt, n[3] (conflict-free gathers)
  __shared__ unsigned long long done_mask;
  __shared__ int smax;

  // dispatch order by the length the forward walked (longest first); the
  // tiles where nothing was blended come last and leave at once
  const TileSlot* bslots = at<const TileSlot>(ws, L.o_bwd_order);
  if (!recompute && blockIdx.x >= at<const DevHeader>(ws, L.o_hdr)->bwd_work) return;
  if (!recompute && at<const uint32_t>(ws, L.o_bwd_pend)[blockIdx.x] == bslots[blockIdx.x].start) return;
  const Tile8 c = tile8(vw, bslots);
  const DevView& V = vw[c.view];
  const float s = uniform_f(V.s);
  const uint32_t start = c.start, end = c.end;
  const size_t plane = (size_t)V.W * V.H;
  const size_t px = c.inside ? (size_t)c.j * V.W + c.i : 0;
  const unsigned lane = threadIdx.x & 63u;
  const int wave = threadIdx.x >> 6;
  const uint64_t cap = (uint64_t)L.entry_cap;

  // per-pixel state (wave 0): T before the last blend, upstream gradient;
  // pend: end of the tile's blended prefix (from the forward, or the replay)
  int last = -1;
  float Tb = 1.0f;
  uint32_t pend;
  if (recompute) {
    float T = 1.0f, O = 0.0f;
    float acc[7];
    uint32_t nb_unused = 0;
    forward_sweep<NWV, CHB>(vrec, srec, start, end, c, s, alpha_min, alpha_clamp, t_min, recs, abuf, pm,
                            hmask, feat, &done_mask, T, Tb, O, acc, last, false, nb_unused);
    if (wave == 0) {
      int wmax = last;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) wmax = max(wmax, __shfl_xor(wmax, o, 64));
      if (lane == 0) smax = wmax;
    }
    __syncthreads();
    pend = smax >= (int)start ? (uint32_t)smax + 1u : start;
  } else {
    pend = at<const uint32_t>(ws, L.o_bwd_pend)[blockIdx.x];
    if (wave == 0 && c.inside) Tb = tlast_in[(size_t)V.pix_base + px];
  }
  float gr[8];
  float Rbehind = 0.0f;
  if (wave == 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) gr[q] = c.inside ? gmem(V.dout)[q * plane + px] : 0.0f;
    Rbehind = gr[0] * V.bg[0] + gr[1] * V.bg[1] + gr[2] * V.bg[2];
  }
  // where this tile's pairs go
  uint32_t pair_run = at<const uint32_t>(ws, L.o_bwd_base)[blockIdx.x];
  const uint32_t tile_xy = (uint32_t)c.tx | ((uint32_t)c.ty << 16);

  bool first = true;
  float Tnext = 1.0f;
  // chunks from the one holding pend - 1 down to start; only the first is partial
  const int64_t cb0 = (int64_t)start + (((int64_t)pend - 1 - (int64_t)start) / CHB) * CHB;
  const uint32_t* rfirst = at<const uint32_t>(ws, L.o_rfirst);
  RecPipe<CHB, NT, true> rp;
  // wave 0, lane e: the blend mask of the current chunk's entry e, and of the
  // next chunk's (its load in flight across the current chunk)
  uint64_t bm_cur = 0ull, bm_next = 0ull;
  // the chunk starting at b, or below the list the entry pend - 1 again
  const auto below = [&](int64_t b) { return b >= (int64_t)start ? (uint32_t)b : pend - 1u; };
  if (pend > start) {
    rp.fetch_idx(srec, (uint32_t)cb0, pend - 1u);
    rp.fetch_rec(vrec, rfirst);
    rp.fetch_idx(srec, below(cb0 - CHB), pend - 1u);
    if (wave == 0 && lane < pend - (uint32_t)cb0 && lane < (unsigned)CHB) bm_next = bmask[(uint32_t)cb0 + lane];
  }
  for (int64_t cb = cb0; cb >= (int64_t)start && pend > start; cb -= CHB) {
    const uint32_t base = (uint32_t)cb;
    const int n = (int)min((uint32_t)CHB, pend - base);
    __syncthreads();
    // the next masks' load is issued before the next records', so taking
    // over the current masks (a wait for their load, a chunk old) does not
    // also wait for the record loads just issued
    bm_cur = bm_next;
    if (wave == 0 && cb - CHB >= (int64_t)start && lane < (unsigned)CHB) bm_next = bmask[base - CHB + lane];
    rp.store(recs, n, ridx);
    rp.fetch_rec(vrec, rfirst);
    rp.fetch_idx(srec, below(cb - 2 * CHB), pend - 1u);
    __syncthreads();
    // phase A: coverage, faces and Eq. 1 of every (entry, pixel) pair the
    // forward blended, packed
    if (threadIdx.x < 64) hmask[threadIdx.x] = 0ull;
    for (int q = threadIdx.x; q < n * 7; q += NT) {
      const int e = q / 7, k = q - e * 7;
      feat[k][e] = k < 3 ? recs[e].c[k] : k == 3 ? recs[e].zt : recs[e].n[k - 4];
    }
    if (wave == 0) {
      // lane e: the pixels that blended entry e (the forward's masks, loaded
      // a chunk ahead)
      const uint64_t live_e = bm_cur;
      chunk_pairs<CHB>(recs, n, c, live_e, pm);
    }
    __syncthreads();
    for_each_pair<CHB>(pm, NT, [&](int e, int pix) {
      const float px_ = (float)(c.tx * 8 + (pix & 7)) + 0.5f, py_ = (float)(c.ty * 8 + (pix >> 3)) + 0.5f;
      PixEval h;
      if (pixel_eval(recs[e], px_, py_, s, h)) {
        abuf[e][pix] = h.alpha;
        e2buf[e][pix] = h.e2;
        sel[e][pix] = (uint8_t)(h.fe | (h.fx << 2));
        if (h.alpha >= alpha_min) atomicOr(&hmask[pix], 1ull << e);
      }
    });
    __syncthreads();
    // phase B (wave 0): the chunk's pairs are the bits of hmask (every
    // candidate at or before the pixel's last blend was blended); their
    // places first, then the reverse recurrence writes each pair
    if (wave == 0) {
      const uint32_t m0 = (uint32_t)hmask[lane];   // CHB <= 32 entries
      const uint64_t lt = (1ull << lane) - 1ull;
      // lane e: the pixels that blended entry e
      const uint64_t cmask_e = wave_transpose64((uint64_t)m0);
      pair_offsets<CHB, 1>(n, cmask_e, pmask, poff);
      // the entries with a blended pixel: what every one of their pairs carries
      if ((int)lane < n && cmask_e != 0ull) {
        const ViewRec& R = recs[lane];
        int i0, i1, j0, j1;
        unpack_rect(R, i0, i1, j0, j1);
        const int tx0 = i0 >> 3, ty0 = j0 >> 3, nx = (i1 >> 3) - tx0 + 1;
        const uint32_t d = R.entry0 + (uint32_t)((c.ty - ty0) * nx + (c.tx - tx0));
        eseg[lane] = make_uint4(ridx[lane], (uint32_t)c.view, tile_xy, d);
      }
      // each pixel visits only the entries it blended, nearest-last first
      uint32_t m = m0;
      while (__ballot(m != 0u) != 0ull) {
        if (m != 0u) {
          const int e = 31 - __clz(m);
          m ^= 1u << e;
          const float araw = abuf[e][lane];
          const float e2 = e2buf[e][lane];
          const float a = fminf(araw, alpha_clamp);
          const float T = first ? Tb : Tnext * rcp(1.0f - a);
          first = false;
          Tnext = T;
          const float sdot = gr[0] * feat[0][e] + gr[1] * feat[1][e] + gr[2] * feat[2][e] + gr[3] +
                             gr[4] * feat[3][e] + gr[5] * feat[4][e] + gr[6] * feat[5][e] + gr[7] * feat[6][e];
          const float da = araw > alpha_clamp ? 0.0f : T * (sdot - Rbehind);
          Rbehind = a * sdot + (1.0f - a) * Rbehind;
          // dL/dalpha chained through Eq. 1 to the entry and exit SDF values
          float dd, dfn;
          eq1_chain(da, araw, e2, s, dd, dfn);
          const uint64_t below = pmask[e] & lt;
          const uint32_t pi = pair_run + poff[e] + (uint32_t)__popcll(below);
          if ((uint64_t)pi < cap) {
            // the segment's first pair carries its pair count
            const uint32_t hw = below == 0ull ? PAIR_HEAD | ((uint32_t)__popcll(pmask[e]) << 11) : 0u;
            pairs[2 * (size_t)pi] = make_uint4(__float_as_uint(dd), __float_as_uint(dfn), __float_as_uint(T * a),
                                               lane | ((uint32_t)sel[e][lane] << 6) | hw);
            pairs[2 * (size_t)pi + 1] = eseg[e];
          }
        }
      }
      pair_run += poff[n];
    }
  }
}

// Backward, per-pair gradients, flat over the pair buffer: each workgroup
// pass takes a window of PG_W consecutive pairs, one per lane.  A lane chains
// its pair to the record's 23 screen-space parameters (colour, depth and
// normal enter linearly with the blend weight; the entry and exit faces
// through App. A.1-A.2) and leaves them in an LDS row; everything it needs
// comes with the pair (one load) and then the record and the view's
// upstream gradient (a second).  The segments whose first pair lies in the
// window are then summed there in a fixed order, one (segment, parameter)
// per thread, into the segment's gradient slot (flagged as reached) or, with
// per-record gradients, added to the record's accumulator.  Only the
// window's last segment runs past it, by at most 63 pairs: the first wave
// also takes the pairs after the window up to the next segment's first pair
// (their loads in flight beside its own pair's), and skips the pairs before
// the window's first segment, which the previous window takes.  Fixed order
// throughout: reproducible bitwise.  (Earlier layouts: a 4-lane group per
// segment left most lanes idle behind a wave's longest segment, 47 us at the
// training shape; one workgroup per tile summing its segments through LDS in
// rounds, 68 us; pairs that reached their record and tile through a segment
// table, 55 us.)
constexpr int PG_W = 256;          // pairs per window (one per thread)
constexpr int PG_TAIL = 64;        // rows for the last segment's pairs past the window
constexpr int PG_G = TGRAD_STRIDE - 1;    // the 23 parameters (the slot's last float is padding)
constexpr int PG_LD = PG_G;               // LDS row stride (floats), odd: conflict-free column writes

struct PairIn {
  uint4 a, b;   // the pair's two halves
  bool ok;
};

// Loads of pair pidx; ok = in range (the buffers of an overflowed forward
// may be stale: the reads then stay in bounds and the result is discarded).
__device__ __forceinline__ PairIn pair_load(const uint4* __restrict__ pairs, uint32_t pidx, const Layout& L) {
  PairIn q;
  q.a = pairs[2 * (size_t)pidx];
  q.b = pairs[2 * (size_t)pidx + 1];
  q.ok = q.b.y < (uint32_t)L.nv && (int64_t)q.b.x < L.rec_cap;
  return q;
}

__device__ __forceinline__ void pair_row(const PairIn& q, const DevView* __restrict__ vw,
                                         const float4* __restrict__ vrec4, float* row) {
  // the record's projected vertices, inverse depths and SDF values (its first 64 bytes)
  ViewRec R;
  const float4* src = vrec4 + (size_t)q.b.x * 8;
  reinterpret_cast<float4*>(&R)[0] = src[0];
  reinterpret_cast<float4*>(&R)[1] = src[1];
  reinterpret_cast<float4*>(&R)[2] = src[2];
  reinterpret_cast<float4*>(&R)[3] = src[3];
  const DevView& V = vw[q.b.y];
  const auto* dout = gmem(V.dout);
  const int W = V.W, H = V.H;
  const int pix = (int)(q.a.w & 63u);
  const int i = (int)(q.b.z & 0xffffu) * 8 + (pix & 7), j = (int)(q.b.z >> 16) * 8 + (pix >> 3);
  // (clamped: a stale pair of an overflowed forward stays in bounds)
  const size_t plane = (size_t)W * H, p = (size_t)min(j, H - 1) * W + min(i, W - 1);
  float gr[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) gr[k] = dout[k * plane + p];
  float g[32];
  pair_grad_all(R, (float)i + 0.5f, (float)j + 0.5f, gr, __uint_as_float(q.a.x), __uint_as_float(q.a.y),
                __uint_as_float(q.a.z), (int)((q.a.w >> 6) & 15u), g);
#pragma unroll
  for (int k = 0; k < PG_G; ++k) row[k] = g[k];
}

__global__ __launch_bounds__(256) void k_pair_grads(void* ws, Layout L) {
  const DevHeader* hdr = at<const DevHeader>(ws, L.o_hdr);
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const float4* vrec4 = at<const float4>(ws, L.o_vrec);
  const uint4* pairs = at<const uint4>(ws, L.o_pairs);
  float* tgrad = at<float>(ws, L.o_tgrad);
  uint8_t* eflag = at<uint8_t>(ws, L.o_eflag);
  const uint64_t cap = (uint64_t)L.entry_cap;
  const uint32_t npair = (uint32_t)min((uint64_t)hdr->pairs_total, cap);
  const bool per_record = record_grads(L);
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  // (32 KB of LDS in all: five workgroups per CU)
  __shared__ float gs[PG_W + PG_TAIL][PG_LD];
  __shared__ uint32_t hrow[PG_W];   // the window's segments: their first row | pair count << 16
  __shared__ uint2 hseg[PG_W];      // ... record, gradient slot
  __shared__ uint32_t wheads[PG_W / 64];

  for (uint32_t w0 = blockIdx.x * PG_W; w0 < npair; w0 += gridDim.x * PG_W) {
    const uint32_t pidx = w0 + threadIdx.x;
    const bool have = pidx < npair;
    PairIn q;
    q.ok = false;
    if (have) q = pair_load(pairs, pidx, L);
    const bool head = q.ok && (q.a.w & PAIR_HEAD) != 0u;
    const uint64_t hb = __ballot(head);
    // the first wave: the pairs after the window up to the next first pair
    // (or the end) belong to the window's last segment
    PairIn t;
    t.ok = false;
    bool skip = false;
    if (wave == 0u) {
      const uint32_t tp = pidx + PG_W;
      if (tp < npair) t = pair_load(pairs, tp, L);
      const uint64_t tb = __ballot(tp >= npair || (t.a.w & PAIR_HEAD) != 0u);
      const uint32_t tn = tb ? (uint32_t)__ffsll((unsigned long long)tb) - 1u : 64u;
      t.ok = t.ok && lane < tn;
      // pairs before the window's first segment start belong to the previous window
      const uint32_t h0 = hb ? (uint32_t)__ffsll((unsigned long long)hb) - 1u : 64u;
      skip = lane < h0 && w0 > 0u;
    }
    if (q.ok && !skip) pair_row(q, vw, vrec4, gs[threadIdx.x]);
    if (t.ok) pair_row(t, vw, vrec4, gs[PG_W + threadIdx.x]);
    if (lane == 0u) wheads[wave] = (uint32_t)__popcll(hb);
    __syncthreads();
    if (head) {
      uint32_t h = (uint32_t)__popcll(hb & ((1ull << lane) - 1ull));
      for (uint32_t w = 0; w < wave; ++w) h += wheads[w];
      hrow[h] = threadIdx.x | (min((q.a.w >> 11) & 127u, 64u) << 16);
      hseg[h] = make_uint2(q.b.x, q.b.w);
    }
    uint32_t nh = 0u;
#pragma unroll
    for (int w = 0; w < PG_W / 64; ++w) nh += wheads[w];
    __syncthreads();
    for (uint32_t it = threadIdx.x; it < nh * TGRAD_STRIDE; it += PG_W) {
      const uint32_t h = it / TGRAD_STRIDE, k = it - h * TGRAD_STRIDE;
      const uint32_t r0 = hrow[h] & 0xffffu, cnt = k < (uint32_t)PG_G ? hrow[h] >> 16 : 0u;
      const uint2 hs = hseg[h];
      // eight rows per step, their reads in flight together (a fixed order)
      float sum = 0.0f;
      for (uint32_t m0 = 0; m0 < cnt; m0 += 8u) {
        float v[8];
#pragma unroll
        for (uint32_t u = 0; u < 8u; ++u) v[u] = m0 + u < cnt ? gs[r0 + m0 + u][k] : 0.0f;
        sum += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
      }
      if (per_record) {
        if (k < TGRAD_STRIDE - 1 && sum != 0.0f) unsafeAtomicAdd(&tgrad[(size_t)hs.x * TGRAD_STRIDE + k], sum);
      } else if ((uint64_t)hs.y < cap) {
        tgrad[(size_t)hs.y * TGRAD_STRIDE + k] = sum;
        if (k == 0u) eflag[hs.y] = 1;
      }
    }
    __syncthreads();
  }
}

hipError_t launch_pair_grads(void* ws, const Layout& L, hipStream_t st) {
  if (L.o_pairs == 0) return hipErrorInvalidValue;
  const int64_t b = (L.entry_cap + PG_W - 1) / PG_W;   // one window of pairs per block and pass
  const unsigned blocks = (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
  k_pair_grads<<<blocks, 256, 0, st>>>(ws, L);
  return hipGetLastError();
}

template <int NWV>
static void launch_fwd_mw(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  if (p.chunk_fwd == 32)
    k_composite_mw<NWV, 32><<<(unsigned)L.total_tiles, 64 * NWV, 0, st>>>(ws, L, p.alpha_min, p.alpha_clamp, p.t_min);
  else
    k_composite_mw<NWV, 64><<<(unsigned)L.total_tiles, 64 * NWV, 0, st>>>(ws, L, p.alpha_min, p.alpha_clamp, p.t_min);
}
template <int NWV>
static void launch_bwd_mw(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  const int rc = (p.flags & RENDER_RECOMPUTE_STATE) ? 1 : 0;
  if (p.chunk_bwd == 16)
    k_composite_bwd_mw<NWV, 16><<<(unsigned)L.total_tiles, 64 * NWV, 0, st>>>(ws, L, p.alpha_min, p.alpha_clamp,
                                                                               p.t_min, rc);
  else
    k_composite_bwd_mw<NWV, 32><<<(unsigned)L.total_tiles, 64 * NWV, 0, st>>>(ws, L, p.alpha_min, p.alpha_clamp,
                                                                               p.t_min, rc);
}

hipError_t launch_composite_mw(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  if (L.total_tiles == 0) return hipSuccess;
  switch (p.waves) {
    case 2: launch_fwd_mw<2>(ws, L, p, st); break;
    case 4: launch_fwd_mw<4>(ws, L, p, st); break;
    case 8: launch_fwd_mw<8>(ws, L, p, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_composite_backward_mw(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  if (L.total_tiles == 0) return hipSuccess;
  switch (p.waves) {
    case 2: launch_bwd_mw<2>(ws, L, p, st); break;
    case 4: launch_bwd_mw<4>(ws, L, p, st); break;
    case 8: launch_bwd_mw<8>(ws, L, p, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ts
