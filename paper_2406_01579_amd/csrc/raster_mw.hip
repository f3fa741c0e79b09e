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
                                              uint64_t* pmask, uint32_t* poff, uint64_t* hm, float (*feat)[CHN],
                                              unsigned long long* done_mask,
                                              float& T, float& Tb, float& O, float (&acc)[7], int& last,
                                              bool want_acc, uint32_t* nblend = nullptr,
                                              uint32_t* nseg = nullptr) {
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
    rp.fetch_idx(srec, start, (int)min((uint32_t)CHN, end - start));
    rp.fetch_rec(vrec);
    if (end - start > (uint32_t)CHN) rp.fetch_idx(srec, start + CHN, (int)min((uint32_t)CHN, end - start - CHN));
  }
  for (uint32_t base = start; base < end; base += CHN) {
    __syncthreads();
    if (*done_mask == ~0ull) break;
    const int n = (int)min((uint32_t)CHN, end - base);
    rp.store(recs, n);
    if (end - base > (uint32_t)CHN) rp.fetch_rec(vrec);
    if (end - base > 2u * CHN) rp.fetch_idx(srec, base + 2 * CHN, (int)min((uint32_t)CHN, end - base - 2 * CHN));
    __syncthreads();
    // phase A: coverage and Eq. 1 of the live (entry, pixel) pairs, packed;
    // hm[pixel] collects the chunk entries the pixel may blend
    if (threadIdx.x < 64) hm[threadIdx.x] = 0ull;
    for (int q = threadIdx.x; q < n * 7; q += NT) {
      const int e = q / 7, k = q - e * 7;
      feat[k][e] = k < 3 ? recs[e].c[k] : k == 3 ? recs[e].zt : recs[e].n[k - 4];
    }
    if (wave == 0) chunk_pairs<CHN>(recs, n, c, ~*done_mask, pmask, poff);
    __syncthreads();
    for_each_pair<CHN>(n, pmask, poff, NT, [&](int e, int pix) {
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
      if (nblend) {
        // the chunk's blended pairs (per lane) and its entries with a blended
        // pixel (the same in every lane)
        *nblend += (uint32_t)__popcll(blended);
        uint32_t lo = (uint32_t)blended, hi = (uint32_t)(blended >> 32);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          lo |= (uint32_t)__shfl_xor((int)lo, o, 64);
          hi |= (uint32_t)__shfl_xor((int)hi, o, 64);
        }
        *nseg += (uint32_t)(__popc(lo) + __popc(hi));
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
    float* out = V.out;
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

template <int NWV>
__global__ __launch_bounds__(64 * NWV) void k_composite_mw(void* ws, Layout L, float alpha_min, float alpha_clamp,
                                                           float t_min) {
  constexpr int CHN = 64;
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const uint32_t* srec = at<const uint32_t>(ws, sorted_entry_records(L));
  const ViewRec* vrec = at<const ViewRec>(ws, L.o_vrec);
  int32_t* last_out = at<int32_t>(ws, L.o_last);
  float* tlast_out = at<float>(ws, L.o_tlast);
  __shared__ ViewRec recs[CHN];
  __shared__ float alds[CHN][64];
  __shared__ uint64_t pmask[CHN];
  __shared__ uint32_t poff[CHN + 1];
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
  const float s = V.s;
  const uint32_t start = c.start, end = c.end;
  float T = 1.0f, Tb = 1.0f, O = 0.0f;
  float acc[7] = {0, 0, 0, 0, 0, 0, 0};
  int last = -1;
  uint32_t nblend = 0, nseg = 0;
  const bool count = L.o_pairs != 0;
  forward_sweep<NWV, CHN>(vrec, srec, start, end, c, s, alpha_min, alpha_clamp, t_min, recs, alds, pmask, poff, hm,
                          feat, &done_mask, T, Tb, O, acc, last, true, count ? &nblend : nullptr,
                          count ? &nseg : nullptr);
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
      if (count) at<uint2>(ws, L.o_slot_pairs)[blockIdx.x] = make_uint2(nblend, nseg);
      // the backward dispatch order's histograms of walked lengths, blended
      // pairs and segments (bucket 0, nothing walked, is not counted)
      if (pend > start) {
        uint32_t* bh = at<uint32_t>(ws, L.o_bwd_hist);
        const int b = len_bucket(pend - start);
        atomicAdd(bh + b, 1u);
        if (count) {
          atomicAdd(bh + 2 * TILE_BUCKETS + b, nblend);
          atomicAdd(bh + 4 * TILE_BUCKETS + b, nseg);
        }
      }
    }
  }
  if ((threadIdx.x >> 6) == 0 && c.inside) {
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

// Backward, walk and recurrence: per chunk, coverage and Eq. 1 of every
// (entry, pixel) the pixel's walk reached, packed, then the reverse
// recurrence of Eq. 2 (one wave).  Every blended pair's dL/df_prev,
// dL/df_next and blend weight go to the pair buffer, entry-major inside the
// chunk, and every entry with a blended pixel gets a segment (its record, its
// per-(record, tile) gradient slot, its first pair and pair count); the
// tile's pairs and segments start at the bases the forward's counts gave
// this backward slot.
template <int NWV>
__global__ __launch_bounds__(64 * NWV) void k_composite_bwd_mw(void* ws, Layout L, float alpha_min,
                                                               float alpha_clamp, float t_min, int recompute) {
  constexpr int NT = 64 * NWV;
  constexpr int CHB = 32;
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const uint32_t* srec = at<const uint32_t>(ws, sorted_entry_records(L));
  const ViewRec* vrec = at<const ViewRec>(ws, L.o_vrec);
  const int32_t* last_in = at<const int32_t>(ws, L.o_last);
  const float* tlast_in = at<const float>(ws, L.o_tlast);
  float4* pairs = at<float4>(ws, L.o_pairs);
  uint4* segs = at<uint4>(ws, L.o_segs);
  __shared__ ViewRec recs[CHB];
  __shared__ float abuf[CHB][64];    // raw alpha
  __shared__ float e2buf[CHB][64];   // exp(s f_next)
  __shared__ uint8_t sel[CHB][64];   // entry face | exit face << 2
  __shared__ uint64_t pmask[CHB];
  __shared__ uint32_t poff[CHB + 1];
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
  const float s = V.s;
  const uint32_t start = c.start, end = c.end;
  const size_t plane = (size_t)V.W * V.H;
  const size_t px = c.inside ? (size_t)c.j * V.W + c.i : 0;
  const unsigned lane = threadIdx.x & 63u;
  const int wave = threadIdx.x >> 6;
  const uint64_t cap = (uint64_t)L.entry_cap;

  // per-pixel state (wave 0): last blended entry, T before it, upstream gradient;
  // pend: end of the tile's blended prefix (from the forward, or the replay)
  int last = -1;
  float Tb = 1.0f;
  uint32_t pend;
  if (recompute) {
    float T = 1.0f, O = 0.0f;
    float acc[7];
    forward_sweep<NWV, CHB>(vrec, srec, start, end, c, s, alpha_min, alpha_clamp, t_min, recs, abuf, pmask, poff,
                            hmask, feat, &done_mask, T, Tb, O, acc, last, false);
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
    if (wave == 0 && c.inside) {
      const size_t gi = (size_t)V.pix_base + px;
      last = last_in[gi];
      Tb = tlast_in[gi];
    }
  }
  float gr[8];
  float Rbehind = 0.0f;
  if (wave == 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) gr[q] = c.inside ? V.dout[q * plane + px] : 0.0f;
    Rbehind = gr[0] * V.bg[0] + gr[1] * V.bg[1] + gr[2] * V.bg[2];
  }
  // this tile's pairs and segments
  const uint4 pb = at<const uint4>(ws, L.o_bwd_base)[blockIdx.x];
  uint32_t pair_run = pb.x, seg_run = pb.y;

  bool first = true;
  float Tnext = 1.0f;
  // chunks from the one holding pend - 1 down to start; only the first is partial
  const int64_t cb0 = (int64_t)start + (((int64_t)pend - 1 - (int64_t)start) / CHB) * CHB;
  const uint4* rbox = at<const uint4>(ws, L.o_rbox);
  RecPipe<CHB, NT, true> rp;
  if (pend > start) {
    rp.fetch_idx(srec, (uint32_t)cb0, (int)(pend - (uint32_t)cb0));
    rp.fetch_rec(vrec, rbox);
    if (cb0 - CHB >= (int64_t)start) rp.fetch_idx(srec, (uint32_t)(cb0 - CHB), CHB);
  }
  for (int64_t cb = cb0; cb >= (int64_t)start && pend > start; cb -= CHB) {
    const uint32_t base = (uint32_t)cb;
    const int n = (int)min((uint32_t)CHB, pend - base);
    __syncthreads();
    rp.store(recs, n);
    if (cb - CHB >= (int64_t)start) rp.fetch_rec(vrec, rbox);
    if (cb - 2 * CHB >= (int64_t)start) rp.fetch_idx(srec, (uint32_t)(cb - 2 * CHB), CHB);
    __syncthreads();
    // phase A: coverage, faces and Eq. 1 of every (entry, pixel) the pixel's
    // walk reached (entry at or before its last blend), packed
    if (threadIdx.x < 64) hmask[threadIdx.x] = 0ull;
    for (int q = threadIdx.x; q < n * 7; q += NT) {
      const int e = q / 7, k = q - e * 7;
      feat[k][e] = k < 3 ? recs[e].c[k] : k == 3 ? recs[e].zt : recs[e].n[k - 4];
    }
    if (wave == 0) {
      // lane e: the pixels whose walk reached entry e (last >= base + e).  A
      // pixel whose last blend lies past the chunk takes part in all of it;
      // only the pixels whose last blend lies inside the chunk need a test
      // per entry.
      const int rel = c.inside ? last - (int)base : -1;
      uint64_t live_e = __ballot(rel >= n - 1);
      uint64_t part = __ballot(rel >= 0 && rel < n - 1);
      if (__popcll(part) * 2 <= n) {
        for (; part != 0ull; part &= part - 1ull) {
          const int p = __ffsll((unsigned long long)part) - 1;
          const int lp = __shfl(rel, p, 64);
          live_e |= ((int)lane <= lp) ? (1ull << p) : 0ull;
        }
      } else {
        for (int e = 0; e < n - 1; ++e) {
          const uint64_t b = __ballot(rel >= e);
          live_e = ((int)lane == e) ? b : live_e;
        }
      }
      chunk_pairs<CHB>(recs, n, c, live_e, pmask, poff);
    }
    __syncthreads();
    for_each_pair<CHB>(n, pmask, poff, NT, [&](int e, int pix) {
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
      const uint32_t m0 = (uint32_t)hmask[lane];   // CHB = 32 entries
      const uint64_t lt = (1ull << lane) - 1ull;
      // lane e: the pixels that blended entry e
      uint32_t any = m0;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) any |= __shfl_xor(any, o, 64);
      any = __builtin_amdgcn_readfirstlane(any);
      uint64_t cmask_e = 0ull;
      for (uint32_t t = any; t != 0u; t &= t - 1u) {
        const int e = __ffs(t) - 1;
        const uint64_t b = __ballot((m0 >> e) & 1u);
        cmask_e = ((int)lane == e) ? b : cmask_e;
      }
      pair_offsets<CHB, 1>(n, cmask_e, pmask, poff);
      // segments: the entries with a blended pixel, in entry order
      const bool has = (int)lane < n && cmask_e != 0ull;
      const uint64_t sm = __ballot(has);
      if (has) {
        const uint32_t si = seg_run + (uint32_t)__popcll(sm & lt);
        const ViewRec& R = recs[lane];
        int i0, i1, j0, j1;
        unpack_rect(R, i0, i1, j0, j1);
        const int tx0 = i0 >> 3, ty0 = j0 >> 3, nx = (i1 >> 3) - tx0 + 1;
        const uint32_t d = R.entry0 + (uint32_t)((c.ty - ty0) * nx + (c.tx - tx0));
        if ((uint64_t)si < cap)
          segs[si] = make_uint4(srec[base + lane], d, pair_run + poff[lane],
                                (uint32_t)__popcll(cmask_e) | (blockIdx.x << 7));
      }
      seg_run += (uint32_t)__popcll(sm);
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
          const uint32_t pi = pair_run + poff[e] + (uint32_t)__popcll(pmask[e] & lt);
          if ((uint64_t)pi < cap)
            pairs[pi] = make_float4(dd, dfn, T * a, __uint_as_float(lane | ((uint32_t)sel[e][lane] << 6)));
        }
      }
      pair_run += poff[n];
    }
  }
}

// Backward, per-pair gradients: one 4-lane group per segment (a (tile,
// entry) pair with blended pixels) chains each of its pairs to the record's
// 23 screen-space parameters (colour, depth and normal enter linearly with
// the blend weight; the entry and exit faces through App. A.1-A.2) and sums
// them -- in registers over the group's pairs in order, then over the group
// in a fixed DPP pattern -- into the segment's gradient slot (flagged as
// reached), or, with per-record gradients, adds the sum to the record's
// accumulator.  Fixed order throughout: reproducible bitwise.  (A layout
// with one workgroup per tile, one pair per thread and the segments summed
// through LDS took 68 us against 49 us for this one at the training shape:
// its rounds are dependent load chains and its summation diverges.)
__global__ __launch_bounds__(256) void k_pair_grads(void* ws, Layout L) {
  const DevHeader* hdr = at<const DevHeader>(ws, L.o_hdr);
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const TileSlot* bslots = at<const TileSlot>(ws, L.o_bwd_order);
  const float4* vrec4 = at<const float4>(ws, L.o_vrec);
  const float4* pairs = at<const float4>(ws, L.o_pairs);
  const uint4* segs = at<const uint4>(ws, L.o_segs);
  float* tgrad = at<float>(ws, L.o_tgrad);
  uint8_t* eflag = at<uint8_t>(ws, L.o_eflag);
  const uint64_t cap = (uint64_t)L.entry_cap;
  const uint32_t nseg = (uint32_t)min((uint64_t)hdr->segs_total, cap);
  const bool per_record = record_grads(L);
  const uint32_t lg = threadIdx.x & 3u;
  const uint32_t groups = gridDim.x * (blockDim.x / 4);
  // the loop runs the same number of times in every lane of a wave (the
  // group sum needs them all)
  const uint32_t wave0 = (blockIdx.x * blockDim.x + (threadIdx.x & ~63u)) / 4;
  for (uint32_t sbase = wave0; sbase < nseg; sbase += groups) {
    const uint32_t si = sbase + ((threadIdx.x & 63u) >> 2);
    const bool sv = si < nseg;
    const uint4 sg = sv ? segs[si] : make_uint4(0u, 0u, 0u, 0u);
    const uint32_t cnt = sg.w & 127u;
    float g[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) g[q] = 0.0f;
    if (sv && cnt > 0u) {
      const TileSlot sl = bslots[sg.w >> 7];
      const DevView& V = vw[sl.view];
      const int lt = (int)sl.tile - V.tile_base;
      const int x0 = (lt % V.tiles_x) * 8, y0 = (lt / V.tiles_x) * 8;
      const size_t plane = (size_t)V.W * V.H;
      // the record's projected vertices, inverse depths and SDF values (its first 64 bytes)
      ViewRec R;
      const float4* src = vrec4 + (size_t)sg.x * 8;
      reinterpret_cast<float4*>(&R)[0] = src[0];
      reinterpret_cast<float4*>(&R)[1] = src[1];
      reinterpret_cast<float4*>(&R)[2] = src[2];
      reinterpret_cast<float4*>(&R)[3] = src[3];
      for (uint32_t k = lg; k < cnt; k += 4u) {
        const uint64_t pi = (uint64_t)sg.z + k;
        if (pi >= cap) break;
        const float4 pr = pairs[pi];
        const uint32_t pw = __float_as_uint(pr.w);
        const int pix = (int)(pw & 63u);
        const int i = x0 + (pix & 7), j = y0 + (pix >> 3);
        const size_t p = (size_t)j * V.W + i;
        float gr[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) gr[q] = V.dout[q * plane + p];
        pair_grad_all<true>(R, (float)i + 0.5f, (float)j + 0.5f, gr, pr.x, pr.y, pr.z, (int)((pw >> 6) & 15u), g);
      }
    }
    float r[8];
    quad_transpose_sum32(g, r);   // lane lg: the segment's sums of g[8 lg .. 8 lg + 7]
    if (sv && cnt > 0u && lg < 3u) {
      if (per_record) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (8 * lg + q < TGRAD_STRIDE - 1 && r[q] != 0.0f)
            unsafeAtomicAdd(&tgrad[(size_t)sg.x * TGRAD_STRIDE + 8 * lg + q], r[q]);
      } else if ((uint64_t)sg.y < cap) {
        float4* dst = reinterpret_cast<float4*>(tgrad + (size_t)sg.y * TGRAD_STRIDE + 8 * lg);
        dst[0] = make_float4(r[0], r[1], r[2], r[3]);
        dst[1] = make_float4(r[4], r[5], r[6], r[7]);
        if (lg == 0u) eflag[sg.y] = 1;
      }
    }
  }
}

hipError_t launch_pair_grads(void* ws, const Layout& L, hipStream_t st) {
  if (L.o_pairs == 0) return hipErrorInvalidValue;
  const int64_t b = (L.entry_cap + 63) / 64;   // 64 segments per block and pass
  const unsigned blocks = (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
  k_pair_grads<<<blocks, 256, 0, st>>>(ws, L);
  return hipGetLastError();
}

template <int NWV>
static void launch_fwd_mw(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  k_composite_mw<NWV><<<(unsigned)L.total_tiles, 64 * NWV, 0, st>>>(ws, L, p.alpha_min, p.alpha_clamp, p.t_min);
}
template <int NWV>
static void launch_bwd_mw(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  k_composite_bwd_mw<NWV><<<(unsigned)L.total_tiles, 64 * NWV, 0, st>>>(
      ws, L, p.alpha_min, p.alpha_clamp, p.t_min, (p.flags & RENDER_RECOMPUTE_STATE) ? 1 : 0);
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
