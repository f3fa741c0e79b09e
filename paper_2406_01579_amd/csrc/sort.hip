// Stable LSD radix sort of (uint32 key, uint32 value) pairs for gfx950, in
// the reduce-then-scan form of Merrill & Grimshaw (2010), the GPU radix sort
// the paper cites (Sec. 3.3).  Per 8-bit digit pass:
//   upsweep   - per-block digit histogram (LDS atomics)
//   spine     - one block per digit: exclusive scan of that digit's block
//               counts and the digit total; (digit start + block prefix) is
//               every (digit, block)'s global output offset
//   downsweep - per block, in input order, the rank of every key among the
//               equal digits before it (wave ballots + wave-private LDS
//               counts); the block's pairs are then laid out in LDS in
//               digit order and written from there, so consecutive threads
//               write consecutive places of a digit's run.
// The element count lives on the device (it is produced by earlier kernels),
// so grids are sized for the capacity and idle blocks exit at once.
#include "ts_internal.h"

namespace ts {

namespace {
constexpr int RADIX = 1 << SORT_BITS;
constexpr int WAVES = SORT_THREADS / 64;
static_assert(RADIX == SORT_THREADS, "one thread per digit in the spine and downsweep prologue");

__device__ __forceinline__ uint32_t sort_n(const uint32_t* n_dev, int64_t cap) {
  uint32_t n = *n_dev;
  return (int64_t)n > cap ? (uint32_t)cap : n;
}

template <int ITEMS>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_up(const uint32_t* __restrict__ keys, const uint32_t* n_dev,
                                                           int64_t cap, int shift, int digit_bits,
                                                           uint32_t* __restrict__ hist) {
  constexpr uint32_t TILE_ = SORT_THREADS * ITEMS;
  __shared__ uint32_t h[RADIX];
  const uint32_t n = sort_n(n_dev, cap);
  const uint32_t nb = (n + TILE_ - 1) / TILE_;
  const uint32_t b = blockIdx.x;
  if (b >= nb) return;
  const uint32_t mask = (1u << digit_bits) - 1u;
  for (int d = threadIdx.x; d < RADIX; d += SORT_THREADS) h[d] = 0;
  __syncthreads();
  const uint32_t i0 = b * TILE_;
  for (int it = 0; it < ITEMS; ++it) {
    uint32_t i = i0 + it * SORT_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < RADIX; d += SORT_THREADS) hist[(size_t)d * nb + b] = h[d];
}

// one block per digit: exclusive scan of that digit's per-block counts (in
// place) and the digit total
template <int ITEMS>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_spine(uint32_t* hist, uint32_t* totals,
                                                              const uint32_t* n_dev, int64_t cap) {
  constexpr uint32_t TILE_ = SORT_THREADS * ITEMS;
  __shared__ uint32_t part[SORT_THREADS];
  const uint32_t n = sort_n(n_dev, cap);
  const uint32_t nb = (n + TILE_ - 1) / TILE_;
  const uint32_t d = blockIdx.x;
  uint32_t* row = hist + (size_t)d * nb;
  const uint32_t per = (nb + SORT_THREADS - 1) / SORT_THREADS;
  const uint32_t t = threadIdx.x;
  const uint32_t lo = min(nb, t * per), hi = min(nb, (t + 1) * per);
  uint32_t sum = 0;
  for (uint32_t i = lo; i < hi; ++i) sum += row[i];
  // block-wide exclusive scan of the per-thread sums (wave scan + wave totals)
  const int lane = t & 63, wave = t >> 6;
  uint32_t x = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) part[wave] = x;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
  for (int w = 0; w < WAVES; ++w) {
    if (w < wave) wbase += part[w];
    tot += part[w];
  }
  uint32_t run = wbase + x - sum;
  for (uint32_t i = lo; i < hi; ++i) {
    uint32_t c = row[i];
    row[i] = run;
    run += c;
  }
  if (t == 0) totals[d] = tot;
}

// Each wave ranks a contiguous quarter of the block's tile with ballot
// matching and wave-private running counts in LDS (no block barriers while
// ranking); one exclusive prefix across the waves then turns the ranks into
// output positions.  Input order is preserved for equal digits (stable).
template <int ITEMS>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_down(const uint32_t* __restrict__ kin,
                                                             const uint32_t* __restrict__ vin,
                                                             uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                             const uint32_t* n_dev, int64_t cap, int shift,
                                                             int digit_bits, const uint32_t* __restrict__ hist,
                                                             const uint32_t* __restrict__ totals) {
  constexpr uint32_t TILE_ = SORT_THREADS * ITEMS;
  __shared__ uint32_t base[RADIX];
  __shared__ uint32_t wrun[WAVES][RADIX];
  __shared__ uint32_t part[WAVES];
  __shared__ uint32_t lbase[RADIX];          // block-local start of each digit's run
  __shared__ uint32_t skey[TILE_], sval[TILE_];   // the block's pairs in digit order
  const uint32_t n = sort_n(n_dev, cap);
  const uint32_t nb = (n + TILE_ - 1) / TILE_;
  const uint32_t b = blockIdx.x;
  if (b >= nb) return;
  const uint32_t mask = (1u << digit_bits) - 1u;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  {
    // digit start = exclusive scan of the digit totals (RADIX == SORT_THREADS)
    const uint32_t tot = totals[threadIdx.x];
    uint32_t x = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) part[wave] = x;
    for (int w = 0; w < WAVES; ++w) wrun[w][threadIdx.x] = 0;
    __syncthreads();
    uint32_t wbase = 0;
    for (int w = 0; w < wave; ++w) wbase += part[w];
    base[threadIdx.x] = wbase + x - tot + hist[(size_t)threadIdx.x * nb + b];
  }
  // ranking: wave w owns items [b*TILE + w*SUB, b*TILE + (w+1)*SUB)
  constexpr int SUB = ITEMS * 64;
  const uint32_t i0 = b * TILE_ + wave * SUB + lane;
  uint32_t keys[ITEMS], vals[ITEMS], rank[ITEMS];
  // keys and values in flight together, before any ranking
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint32_t i = i0 + it * 64;
    keys[it] = i < n ? kin[i] : 0u;
    vals[it] = i < n ? (vin ? vin[i] : i) : 0u;
  }
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint32_t i = i0 + it * 64;
    const bool valid = i < n;
    const uint32_t digit = (keys[it] >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int bit = 0; bit < digit_bits; ++bit) {
      const bool set = (digit >> bit) & 1u;
      const uint64_t bb = __ballot(set);
      peers &= set ? bb : ~bb;
    }
    const uint32_t within = (uint32_t)__popcll(peers & lt);
    const uint32_t before = valid ? wrun[wave][digit] : 0u;   // every peer reads before the leader writes
    rank[it] = before + within;
    if (valid && within == 0) wrun[wave][digit] = before + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  {
    // digit d: the block's count, its block-local start (an exclusive scan
    // over the digits), and each wave's start inside the run
    const int d = threadIdx.x;
    uint32_t cnt = 0;
    for (int w = 0; w < WAVES; ++w) {
      const uint32_t c = wrun[w][d];
      wrun[w][d] = cnt;
      cnt += c;
    }
    uint32_t x = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) part[wave] = x;
    __syncthreads();
    uint32_t wb = 0;
    for (int w = 0; w < wave; ++w) wb += part[w];
    lbase[d] = wb + x - cnt;
  }
  __syncthreads();
  // the pairs into LDS in (digit, input) order ...
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const uint32_t i = i0 + it * 64;
    if (i < n) {
      const uint32_t digit = (keys[it] >> shift) & mask;
      const uint32_t li = lbase[digit] + wrun[wave][digit] + rank[it];
      skey[li] = keys[it];
      sval[li] = vals[it];
    }
  }
  __syncthreads();
  // ... and out in that order: consecutive threads write consecutive places
  // of a digit's run
  const uint32_t nloc = min((uint32_t)TILE_, n - b * TILE_);
  for (uint32_t li = threadIdx.x; li < nloc; li += SORT_THREADS) {
    const uint32_t k = skey[li];
    const uint32_t digit = (k >> shift) & mask;
    const uint32_t pos = base[digit] + (li - lbase[digit]);
    kout[pos] = k;
    vout[pos] = sval[li];
  }
}
}  // namespace

template <int ITEMS>
static hipError_t radix_sort_impl(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b,
                                  bool identity, const uint32_t* n_dev, int64_t cap, int bits, uint32_t* hist,
                                  int64_t hist_blocks, hipStream_t st, uint32_t** keys_out, uint32_t** vals_out) {
  constexpr int64_t TILE_ = (int64_t)SORT_THREADS * ITEMS;
  const unsigned nb = (unsigned)((cap + TILE_ - 1) / TILE_);
  // digit totals live after the (digit, block) table
  uint32_t* totals = hist + (size_t)RADIX * (size_t)hist_blocks;
  uint32_t *ki = keys_a, *vi = vals_a, *ko = keys_b, *vo = vals_b;
  bool first = true;
  for (int shift = 0; shift < bits; shift += SORT_BITS) {
    const int db = (bits - shift) < SORT_BITS ? (bits - shift) : SORT_BITS;
    if (nb > 0) {
      k_radix_up<ITEMS><<<nb, SORT_THREADS, 0, st>>>(ki, n_dev, cap, shift, db, hist);
      k_radix_spine<ITEMS><<<RADIX, SORT_THREADS, 0, st>>>(hist, totals, n_dev, cap);
      k_radix_down<ITEMS><<<nb, SORT_THREADS, 0, st>>>(ki, (first && identity) ? nullptr : vi, ko, vo, n_dev, cap,
                                                         shift, db, hist, totals);
    }
    first = false;
    uint32_t* t = ki; ki = ko; ko = t;
    t = vi; vi = vo; vo = t;
  }
  *keys_out = ki;
  *vals_out = vi;
  return hipGetLastError();
}

hipError_t radix_sort_pairs(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b, bool identity,
                            const uint32_t* n_dev, int64_t cap, int bits, uint32_t* hist, int64_t hist_blocks,
                            hipStream_t st, uint32_t** keys_out, uint32_t** vals_out, int items) {
  if (items == 8)
    return radix_sort_impl<8>(keys_a, vals_a, keys_b, vals_b, identity, n_dev, cap, bits, hist, hist_blocks, st,
                              keys_out, vals_out);
  if (items != SORT_ITEMS) return hipErrorInvalidValue;
  return radix_sort_impl<SORT_ITEMS>(keys_a, vals_a, keys_b, vals_b, identity, n_dev, cap, bits, hist, hist_blocks,
                                     st, keys_out, vals_out);
}

}  // namespace ts
