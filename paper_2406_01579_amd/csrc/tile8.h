// Helpers shared by the compositing kernels that run one 8x8 pixel tile per
// workgroup (one pixel per lane of each 64-lane wave): the tile's pixel
// coordinates, the record-rectangle test, and the coalesced LDS staging of a
// chunk of sorted records (8 lanes per 128-byte record).
#pragma once

#include "ts_device.h"

namespace ts {
namespace {

// The records of sorted entries [base, base + n) into LDS, eight threads per
// 128-byte record.  With rfirst, the copy's first-entry field comes from the
// records' first entries, where the placement kernel writes them.
__device__ __forceinline__ void load_recs(ViewRec* recs, const ViewRec* __restrict__ vrec,
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

__device__ __forceinline__ bool has_pixel(const ViewRec& R, int i, int j) {
  int i0, i1, j0, j1;
  unpack_rect(R, i0, i1, j0, j1);
  return i >= i0 && i <= i1 && j >= j0 && j <= j1;
}

struct Tile8 {
  int view, tile;
  int tx, ty;            // tile coordinates inside the view
  int i, j;              // this lane's pixel
  bool inside;
  uint32_t start, end;   // the tile's entry range
};

__device__ __forceinline__ Tile8 tile8(const DevView* vw, const TileSlot* slots) {
  Tile8 c;
  const TileSlot sl = slots[blockIdx.x];
  c.tile = (int)sl.tile;
  c.view = (int)sl.view;
  c.start = sl.start;
  c.end = sl.end;
  const DevView& V = vw[c.view];
  const int lt = c.tile - V.tile_base;
  const int lane = threadIdx.x & 63;
  c.tx = lt % V.tiles_x;
  c.ty = lt / V.tiles_x;
  c.i = c.tx * 8 + (lane & 7);
  c.j = c.ty * 8 + (lane >> 3);
  c.inside = c.i < V.W && c.j < V.H;
  return c;
}

// The tile's reduced gradient of each chunk entry (gacc[e][0..TGRAD_STRIDE))
// goes to the entry's pre-sort slot: the record's first entry plus this
// tile's row-major index inside the record's tile rectangle; the slot is
// flagged as reached.  With chunk_rec (the chunk's record indices) it is
// added into its record's accumulator instead.
// (A slot past the entry capacity belongs to an overflowed forward, whose
// outputs are invalid anyway: it is skipped.)
__device__ __forceinline__ void store_entry_grads(const ViewRec* recs, const float (*gacc)[TGRAD_STRIDE], int n,
                                                  const Tile8& c, float* __restrict__ tgrad,
                                                  uint8_t* __restrict__ eflag, int nthreads, uint64_t cap,
                                                  const uint32_t* __restrict__ chunk_rec = nullptr) {
  if (chunk_rec) {
    for (int q = threadIdx.x; q < n * (TGRAD_STRIDE - 1); q += nthreads) {
      const int e = q / (TGRAD_STRIDE - 1), k = q - e * (TGRAD_STRIDE - 1);
      const float v = gacc[e][k];
      if (v != 0.0f) unsafeAtomicAdd(&tgrad[(size_t)chunk_rec[e] * TGRAD_STRIDE + k], v);
    }
    return;
  }
  for (int q = threadIdx.x; q < n * TGRAD_STRIDE; q += nthreads) {
    const int e = q / TGRAD_STRIDE, k = q - e * TGRAD_STRIDE;
    const ViewRec& R = recs[e];
    int i0, i1, j0, j1;
    unpack_rect(R, i0, i1, j0, j1);
    const int tx0 = i0 >> 3, ty0 = j0 >> 3, nx = (i1 >> 3) - tx0 + 1;
    const size_t d = (size_t)R.entry0 + (size_t)((c.ty - ty0) * nx + (c.tx - tx0));
    if (d >= cap) continue;
    tgrad[d * TGRAD_STRIDE + k] = gacc[e][k];
    if (k == 0) eflag[d] = 1;
  }
}

// ---------------------------------------------------------------------------
// Pair packing.  Of the 64 pixels of a tile, a record's pixel rectangle
// usually holds a handful; evaluating one record per wave would leave most
// lanes idle.  Instead each chunk lists the (entry, pixel) pairs whose pixel
// lies in the entry's rectangle and is still live, entry-major, and the
// workgroup's lanes take consecutive pairs.
// ---------------------------------------------------------------------------
// Pixels of the tile (bit = row-major local index) inside R's rectangle.
__device__ __forceinline__ uint64_t rect_mask(const ViewRec& R, const Tile8& c) {
  int i0, i1, j0, j1;
  unpack_rect(R, i0, i1, j0, j1);
  const int x0 = max(i0 - c.tx * 8, 0), x1 = min(i1 - c.tx * 8, 7);
  const int y0 = max(j0 - c.ty * 8, 0), y1 = min(j1 - c.ty * 8, 7);
  if (x0 > x1 || y0 > y1) return 0ull;
  const uint64_t row = (uint64_t)(((2u << x1) - (1u << x0)) & 0xffu);
  const uint64_t rows = (~0ull >> (8 * (7 - y1))) & (~0ull << (8 * y0));
  return (row * 0x0101010101010101ull) & rows;
}

// Position of the k-th (from 0) set bit of m; m has more than k set bits.
__device__ __forceinline__ int select_bit(uint64_t m, uint32_t k) {
  int pos = 0;
  uint32_t c = (uint32_t)__popc((uint32_t)m);
  const bool hi = k >= c;
  k = hi ? k - c : k;
  uint32_t x = hi ? (uint32_t)(m >> 32) : (uint32_t)m;
  pos = hi ? 32 : 0;
#pragma unroll
  for (int w = 16; w >= 1; w >>= 1) {
    c = (uint32_t)__popc(x & ((1u << w) - 1u));
    const bool up = k >= c;
    k = up ? k - c : k;
    x = up ? x >> w : x;
    pos = up ? pos + w : pos;
  }
  return pos;
}

// Wave 0, lane e < n: m_e is entry e's pair mask.  Writes pmask[0..CH) and
// the exclusive offsets poff[0..CH] of the entries' pairs counted in groups
// of GROUP (poff[n] = number of groups).
template <int CH, int GROUP = 1>
__device__ __forceinline__ void pair_offsets(int n, uint64_t m_e, uint64_t* pmask, uint32_t* poff) {
  const int lane = threadIdx.x & 63;
  const uint64_t m = lane < n ? m_e : 0ull;
  uint32_t x = ((uint32_t)__popcll(m) + (GROUP - 1)) / GROUP;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    x += lane >= d ? y : 0u;
  }
  if (lane < CH) {
    pmask[lane] = m;
    poff[lane + 1] = x;
  }
  if (lane == 0) poff[0] = 0u;
}

// A chunk's pair list, laid out so that a lane finds the entry of its pair
// with a popcount and one LDS read (a binary search over the entries'
// offsets was six dependent LDS reads per pair).  The entries with at least
// one pair are listed in order; per block of 64 consecutive pairs, bstart
// marks the pairs that begin a listed entry and bfirst counts the listed
// entries that begin before the block.  Pair p (block b = p / 64) then
// belongs to listed entry bfirst[b] + (starts in block b at or before p) - 1.
template <int CH>
struct PairMap {
  uint64_t bstart[CH];   // per block of 64 pairs: bit q set where a listed entry's pairs begin
  uint64_t lmask[CH];    // listed entry k: its pixel mask
  uint32_t bfirst[CH];   // per block: listed entries beginning before it
  uint32_t lent[CH];     // listed entry k: its chunk index | its first pair << 8
  uint32_t total;        // pairs in the chunk
};

// Wave 0, lane e < n: m_e is entry e's pixel mask.  Every lane of the wave
// must call it; the map is complete after the next barrier.
template <int CH>
__device__ __forceinline__ void pair_map(int n, uint64_t m_e, PairMap<CH>& M) {
  static_assert(CH <= 64, "one lane per entry");
  const int lane = threadIdx.x & 63;
  const uint64_t m = lane < n ? m_e : 0ull;
  const uint32_t cnt = (uint32_t)__popcll(m);
  uint32_t x = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    x += lane >= d ? y : 0u;
  }
  const uint32_t first = x - cnt;
  const uint32_t k = (uint32_t)__popcll(__ballot(m != 0ull) & ((1ull << lane) - 1ull));
  // the pairs fill at most CH blocks; this wave's own LDS operations take
  // effect in program order, so the clear lands before the marks
  if (lane < CH) M.bstart[lane] = 0ull;
  __builtin_amdgcn_wave_barrier();
  if (m != 0ull) {
    M.lmask[k] = m;
    M.lent[k] = (uint32_t)lane | (first << 8);
    atomicOr(&M.bstart[first >> 6], 1ull << (first & 63u));
  }
  __builtin_amdgcn_wave_barrier();
  const uint64_t bs = lane < CH ? M.bstart[lane] : 0ull;
  const uint32_t bc = (uint32_t)__popcll(bs);
  uint32_t y = bc;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t z = __shfl_up(y, d, 64);
    y += lane >= d ? z : 0u;
  }
  if (lane < CH) M.bfirst[lane] = y - bc;
  if (lane == 63) M.total = x;
}

// Wave 0, lane e < n: entry e's pairs are the pixels of its rectangle in
// live_e (the pixels that still take part for that entry).
template <int CH>
__device__ __forceinline__ void chunk_pairs(const ViewRec* recs, int n, const Tile8& c, uint64_t live_e,
                                            PairMap<CH>& M) {
  const int lane = threadIdx.x & 63;
  pair_map<CH>(n, lane < n ? rect_mask(recs[lane], c) & live_e : 0ull, M);
}

// All threads: f(e, pix) for every listed pair (entry e, local pixel pix),
// entry-major, pixels in ascending order inside an entry.
template <int CH, class F>
__device__ __forceinline__ void for_each_pair(const PairMap<CH>& M, int nthreads, F&& f) {
  const uint32_t total = M.total;
  for (uint32_t p = threadIdx.x; p < total; p += (uint32_t)nthreads) {
    const uint32_t b = p >> 6;
    // pair 0 begins the first listed entry, so at least one start lies at or before p
    const uint32_t k = M.bfirst[b] + (uint32_t)__popcll(M.bstart[b] & (~0ull >> (63u - (p & 63u)))) - 1u;
    const uint32_t le = M.lent[k];
    f((int)(le & 0xffu), select_bit(M.lmask[k], p - (le >> 8)));
  }
}

// Software pipeline of the chunk loads: while a chunk is processed, the next
// chunk's records are in flight into registers and the record indices of the
// one after it are in flight too, so a chunk's two dependent global loads
// overlap the previous chunk's work.  Each thread owns PQ of the chunk's
// 16-byte record parts.  With E0, the copy's first-entry field comes from
// the records' first entries (loaded beside the last part).
template <int CH, int NT, bool E0 = false>
struct RecPipe {
  static constexpr int PQ = (CH * 8 + NT - 1) / NT;
  uint32_t idx[PQ];
  uint32_t cur[PQ];                      // the record indices of the parts in flight
  float vx[PQ], vy[PQ], vz[PQ], vw[PQ];  // scalars, so the parts stay in registers
  // The chunk of entries from b, cut at hi (a valid entry): a part past hi
  // loads entry hi's index again.  Callers issue every load of the pipeline
  // unconditionally (past the list: its last entry, cached and never
  // stored), so no register is given a default while an older load into it
  // may be in flight, a wait that would also cover the loads just issued.
  __device__ __forceinline__ void fetch_idx(const uint32_t* __restrict__ srec, uint32_t b, uint32_t hi) {
#pragma unroll
    for (int j = 0; j < PQ; ++j) {
      const int q = (int)threadIdx.x + j * NT;
      idx[j] = srec[min(b + (uint32_t)(q >> 3), hi)];
    }
  }
  // every part (one past the chunk reads a record of the list, never stored)
  __device__ __forceinline__ void fetch_rec(const ViewRec* __restrict__ vrec,
                                            const uint32_t* __restrict__ rfirst = nullptr) {
#pragma unroll
    for (int j = 0; j < PQ; ++j) {
      const int q = (int)threadIdx.x + j * NT;
      cur[j] = idx[j];
      const float4 t = reinterpret_cast<const float4*>(vrec)[(size_t)idx[j] * 8 + (size_t)(q & 7)];
      vx[j] = t.x;
      vy[j] = t.y;
      vz[j] = t.z;
      vw[j] = t.w;
      if (E0 && (q & 7) == 7) vw[j] = __uint_as_float(rfirst[idx[j]]);   // entry0: the record's last word
    }
  }
  // With ridx, also each record's index (what a chunk needs of srec later
  // comes from LDS then, not from a global load on its critical path).
  __device__ __forceinline__ void store(ViewRec* recs, int n, uint32_t* ridx = nullptr) const {
#pragma unroll
    for (int j = 0; j < PQ; ++j) {
      const int q = (int)threadIdx.x + j * NT;
      if (q < n * 8) {
        reinterpret_cast<float4*>(&recs[q >> 3])[q & 7] = make_float4(vx[j], vy[j], vz[j], vw[j]);
        if (ridx && (q & 7) == 0) ridx[q >> 3] = cur[j];
      }
    }
  }
};

}  // namespace
}  // namespace ts
