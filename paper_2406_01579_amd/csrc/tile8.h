// Helpers shared by the compositing kernels that run one 8x8 pixel tile per
// workgroup (one pixel per lane of each 64-lane wave): the tile's pixel
// coordinates, the record-rectangle test, and the coalesced LDS staging of a
// chunk of sorted records (8 lanes per 128-byte record).
#pragma once

#include "ts_device.h"

namespace ts {
namespace {

__device__ __forceinline__ void load_recs(ViewRec* recs, const ViewRec* __restrict__ vrec,
                                          const uint32_t* __restrict__ srec, uint32_t base, int n, int nthreads) {
  for (int q = threadIdx.x; q < n * 8; q += nthreads) {
    const int e = q >> 3, part = q & 7;
    const uint32_t r = srec[base + e];
    reinterpret_cast<float4*>(&recs[e])[part] = reinterpret_cast<const float4*>(&vrec[r])[part];
  }
}

__device__ __forceinline__ bool has_pixel(const ViewRec& R, int i, int j) {
  int i0, i1, j0, j1;
  unpack_rect(R, i0, i1, j0, j1);
  return i >= i0 && i <= i1 && j >= j0 && j <= j1;
}

struct Tile8 {
  int view, tile;
  int tx, ty;     // tile coordinates inside the view
  int i, j;
  bool inside;
};

__device__ __forceinline__ Tile8 tile8(const DevView* vw, int nv, const uint32_t* order) {
  Tile8 c;
  c.tile = (int)order[blockIdx.x];
  c.view = find_view_by_tile(vw, nv, c.tile);
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
// flagged as reached.
__device__ __forceinline__ void store_entry_grads(const ViewRec* recs, const float (*gacc)[TGRAD_STRIDE], int n,
                                                  const Tile8& c, float* __restrict__ tgrad,
                                                  uint8_t* __restrict__ eflag, int nthreads) {
  for (int q = threadIdx.x; q < n * TGRAD_STRIDE; q += nthreads) {
    const int e = q / TGRAD_STRIDE, k = q - e * TGRAD_STRIDE;
    const ViewRec& R = recs[e];
    int i0, i1, j0, j1;
    unpack_rect(R, i0, i1, j0, j1);
    const int tx0 = i0 >> 3, ty0 = j0 >> 3, nx = (i1 >> 3) - tx0 + 1;
    const size_t d = (size_t)R.entry0 + (size_t)((c.ty - ty0) * nx + (c.tx - tx0));
    tgrad[d * TGRAD_STRIDE + k] = gacc[e][k];
    if (k == 0) eflag[d] = 1;
  }
}

}  // namespace
}  // namespace ts
