// Multi-wave compositing kernels for 8x8 tiles.
//
// A tile's entry list is walked front to back (forward) or back to front
// (backward) by one pixel per lane, and the per-pixel state along the list
// (transmittance, the colour behind) is a short sequential recurrence.  The
// expensive part of every (pixel, entry) pair -- coverage of the projected
// hull, entry/exit SDF values and Eq. 1, and in the backward the chain to the
// record's screen-space parameters and the wave reduction -- does not depend
// on that state.  So NWV waves share one 8x8 tile: for each LDS chunk of
// entries they evaluate interleaved entries in parallel into LDS, one wave
// runs the recurrence over the chunk, and (backward) the waves then build and
// reduce the per-entry gradients in parallel.  Images are bit-identical to
// the one-wave kernels (the same per-pair arithmetic in the same order);
// gradients agree to rounding (an entry's pixel groups are added in LDS in
// arrival order), bitwise with the deterministic variant.
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
                                              bool want_acc) {
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
            if (T == 0.0f) done = true;
          }
        }
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
  forward_sweep<NWV, CHN>(vrec, srec, start, end, c, s, alpha_min, alpha_clamp, t_min, recs, alds, pmask, poff, hm,
                          feat, &done_mask, T, Tb, O, acc, last, true);
  if ((threadIdx.x >> 6) == 0) {
    // end of the tile's blended prefix: where the backward starts its walk
    int wmax = last;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wmax = max(wmax, __shfl_xor(wmax, o, 64));
    if ((threadIdx.x & 63) == 0) {
      const uint32_t pend = wmax >= (int)start ? (uint32_t)wmax + 1u : start;
      at<uint32_t>(ws, L.o_tile_pend)[blockIdx.x] = pend;
      // the backward dispatch order's histogram of walked lengths (bucket 0,
      // nothing walked, is not counted)
      if (pend > start) atomicAdd(at<uint32_t>(ws, L.o_bwd_hist) + len_bucket(pend - start), 1u);
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

// DET: every entry's gradient is the sum of its 8-pixel groups in group
// order (group sums staged in LDS), not LDS float atomics in arrival order;
// the chunk is halved (16 entries) to make room.
template <int NWV, bool DET>
__global__ __launch_bounds__(64 * NWV) void k_composite_bwd_mw(void* ws, Layout L, float alpha_min,
                                                               float alpha_clamp, float t_min, int recompute) {
  constexpr int NT = 64 * NWV;
  constexpr int CHB = DET ? 16 : 32;
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const uint32_t* srec = at<const uint32_t>(ws, sorted_entry_records(L));
  const ViewRec* vrec = at<const ViewRec>(ws, L.o_vrec);
  const int32_t* last_in = at<const int32_t>(ws, L.o_last);
  const float* tlast_in = at<const float>(ws, L.o_tlast);
  float* tgrad = at<float>(ws, L.o_tgrad);
  uint8_t* eflag = at<uint8_t>(ws, L.o_eflag);
  __shared__ ViewRec recs[CHB];
  __shared__ float abuf[CHB][64];    // raw alpha (-1: no hit / not reached); phase B: dL/df_prev
  __shared__ float e2buf[CHB][64];   // exp(s f_next); phase B: dL/df_next
  __shared__ uint8_t sel[CHB][64];   // entry face | exit face << 2
  __shared__ float wbuf[CHB][64];    // blend weight T alpha
  __shared__ float gacc[CHB][TGRAD_STRIDE];
  __shared__ float grs[8][64];       // upstream gradient of each pixel
  __shared__ uint64_t pmask[CHB];
  __shared__ uint32_t poff[CHB + 1];
  __shared__ uint64_t hmask[64];     // per pixel: chunk entries it blended (bit e)
  __shared__ float feat[7][CHB];     // per entry: c[3], zt, n[3] (conflict-free gathers)
  __shared__ unsigned long long done_mask;
  __shared__ int smax;
  __shared__ __align__(16) float gsum[DET ? CHB * 8 : 1][TGRAD_STRIDE];  // DET: per 8-pixel group

  // dispatch order by the length the forward walked (longest first); the
  // tiles where nothing was blended come last and leave at once
  const TileSlot* bslots = at<const TileSlot>(ws, L.o_bwd_order);
  if (!recompute && blockIdx.x >= at<const DevHeader>(ws, L.o_hdr)->bwd_work) return;
  if (!recompute && at<const uint32_t>(ws, L.o_bwd_pend)[blockIdx.x] == bslots[blockIdx.x].start) return;
  const Tile8 c = tile8(vw, bslots);
  const DevView& V = vw[c.view];
  const float s = V.s;
  const uint32_t start = c.start, end = c.end;
  const float qx = (float)c.i + 0.5f, qy = (float)c.j + 0.5f;
  const size_t plane = (size_t)V.W * V.H;
  const size_t px = c.inside ? (size_t)c.j * V.W + c.i : 0;
  const unsigned lane = threadIdx.x & 63u;
  const int wave = threadIdx.x >> 6;

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
  float Rbehind = 0.0f;
  if (wave == 0) {
    float gr[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      gr[q] = c.inside ? V.dout[q * plane + px] : 0.0f;
      grs[q][lane] = gr[q];
    }
    Rbehind = gr[0] * V.bg[0] + gr[1] * V.bg[1] + gr[2] * V.bg[2];
  }

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
    // phase B: reverse recurrence (one wave); the others clear the chunk's sums
    for (int q = threadIdx.x; q < n * TGRAD_STRIDE; q += NT) (&gacc[0][0])[q] = 0.0f;
    if (wave == 0) {
      // each pixel visits only the entries it blended, nearest-last first
      const uint32_t m0 = (uint32_t)hmask[lane];   // CHB = 32 entries
      uint32_t m = m0;
      float gr[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) gr[q] = grs[q][lane];
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
          // chain dL/dalpha through Eq. 1 here, so phase C needs neither alpha nor e2
          float dd, dfn;
          eq1_chain(da, araw, e2, s, dd, dfn);
          abuf[e][lane] = dd;
          e2buf[e][lane] = dfn;
          wbuf[e][lane] = T * a;
        }
      }
      // lane e: the pixels that blended entry e (the pairs of phase C)
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
      pair_offsets<CHB, 8>(n, cmask_e, pmask, poff);
    }
    __syncthreads();
    // phase C: the gradient of every contributing (entry, pixel) pair.  Each
    // entry's pairs fill 8-lane groups (eight per wave); a group is summed
    // with DPP inside its half-row and added to the entry's sum (LDS float
    // add: an entry with more than 8 contributing pixels spans several
    // groups).
    {
      const uint32_t ngroups = poff[n];
      const int l8 = (int)(lane & 7u);
      for (uint32_t g0 = (uint32_t)wave * 8u; g0 < ngroups; g0 += 8u * NWV) {
        const uint32_t grp = g0 + (lane >> 3);
        // branch-free: a lane past the last group or the entry's last pair
        // chains zero weights
        const bool gv = grp < ngroups;
        const int e = entry_of<CHB>(n, poff, gv ? grp : ngroups - 1u);
        const uint64_t m = pmask[e];
        const uint32_t k = (grp - poff[e]) * 8u + (uint32_t)l8;
        const bool valid = gv && k < (uint32_t)__popcll(m);
        const int pix = valid ? select_bit(m, k) : 0;
        const float px_ = (float)(c.tx * 8 + (pix & 7)) + 0.5f, py_ = (float)(c.ty * 8 + (pix >> 3)) + 0.5f;
        float grp8[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) grp8[q] = grs[q][pix];
        const float dd = valid ? abuf[e][pix] : 0.0f, dfn = valid ? e2buf[e][pix] : 0.0f;
        const float w = valid ? wbuf[e][pix] : 0.0f;
        float g[32];
        pair_grad_all(recs[e], px_, py_, grp8, dd, dfn, w, sel[e][pix], g);
        const float4 r = row8_transpose_sum32(g);
        static_assert(TGRAD_STRIDE - 1 == 23, "23 gradient slots: lane 5 holds the last three");
        if constexpr (DET) {
          if (gv && 4 * l8 < TGRAD_STRIDE) *reinterpret_cast<float4*>(&gsum[grp][4 * l8]) = r;
        } else if (gv && 4 * l8 < TGRAD_STRIDE - 1) {
          atomicAdd(&gacc[e][4 * l8], r.x);
          atomicAdd(&gacc[e][4 * l8 + 1], r.y);
          atomicAdd(&gacc[e][4 * l8 + 2], r.z);
          if (4 * l8 + 3 < TGRAD_STRIDE - 1) atomicAdd(&gacc[e][4 * l8 + 3], r.w);
        }
      }
    }
    __syncthreads();
    if constexpr (DET) {
      // each entry: its groups' sums in group order
      for (int q = threadIdx.x; q < n * (TGRAD_STRIDE - 1); q += NT) {
        const int e = q / (TGRAD_STRIDE - 1), k = q - e * (TGRAD_STRIDE - 1);
        float acc = 0.0f;
        for (uint32_t gi = poff[e]; gi < poff[e + 1]; ++gi) acc += gsum[gi][k];
        gacc[e][k] = acc;
      }
      __syncthreads();
    }
    store_entry_grads(recs, gacc, n, c, tgrad, eflag, NT, (uint64_t)L.entry_cap,
                      record_grads(L) ? srec + base : nullptr);
  }
}

template <int NWV>
static void launch_fwd_mw(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  k_composite_mw<NWV><<<(unsigned)L.total_tiles, 64 * NWV, 0, st>>>(ws, L, p.alpha_min, p.alpha_clamp, p.t_min);
}
template <int NWV>
static void launch_bwd_mw(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  const int rc = (p.flags & RENDER_RECOMPUTE_STATE) ? 1 : 0;
  if (deterministic(L))
    k_composite_bwd_mw<NWV, true><<<(unsigned)L.total_tiles, 64 * NWV, 0, st>>>(ws, L, p.alpha_min, p.alpha_clamp,
                                                                                p.t_min, rc);
  else
    k_composite_bwd_mw<NWV, false><<<(unsigned)L.total_tiles, 64 * NWV, 0, st>>>(ws, L, p.alpha_min, p.alpha_clamp,
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
