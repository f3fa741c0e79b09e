// Internal declarations of the gfx950 tetrahedron rasterizer: device-side
// descriptors, the workspace layout, and the host-side launchers that the
// C ABI (api.cpp) strings together.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/tetsplat.h"

namespace ts {

// ---------------------------------------------------------------------------
// device descriptors (written into the workspace by k_write_desc)
// ---------------------------------------------------------------------------
struct DevScene {
  const float* verts;
  const int32_t* tets;
  const float* sdf;
  const float* colors;
  float* dverts;
  float* dsdf;
  float* dcolors;
  int32_t V, K;
  float s;
  int32_t block_base;   // first pre-filter block of this scene
  int32_t n_blocks;
  int32_t view_first;   // this scene's views: scene_views[view_first .. + view_count)
  int32_t view_count;
  int32_t vbase;        // first vertex of this scene in the concatenation of all scenes' vertices
};

struct DevView {
  float R[9], t[3];
  float fx, fy, cx, cy, znear;
  float bg[3];
  float* out;
  const float* dout;
  int32_t scene, W, H;
  int32_t tiles_x, tiles_y;
  int32_t tile_base;    // first global tile id of this view
  int32_t pix_base;     // first global pixel id of this view
  float s;              // steepness of Eq. 1 of the view's scene
};

// One compositing workgroup's tile, in dispatch order (longest list first),
// so that a workgroup finds its tile, view and entry range in one load.
struct TileSlot {
  uint32_t tile;        // global tile id
  uint32_t view;
  uint32_t start, end;  // the tile's entry range
};

// device-written counters at the start of the workspace
struct DevHeader {
  uint32_t kept_total;
  uint32_t records_total;
  uint32_t entries_total;
  uint32_t overflow;
  uint32_t invalid_index;
  uint32_t bwd_work;    // backward dispatch slots with a walked entry (they come first)
  uint32_t corners_total;  // deterministic backward: 4 x kept tets, the corners sorted by vertex
  uint32_t pad0;
  int64_t entry_capacity, kept_capacity;
  uint64_t entries_needed;  // entries the last forward wanted (exact, also on overflow)
  uint32_t pairs_total;     // (entry, pixel) pairs the forward blended (multi-wave 8x8 path)
  uint32_t pad1[49];
};
static_assert(sizeof(DevHeader) == 256, "header is 256 bytes");

// Per kept tet, view independent (96 B): vertex positions, SDF, normal,
// mean colour, tet id.
struct TetRec {
  float x[4][3];
  float f[4];
  float n[3];
  float c[3];
  int32_t tet;
  int32_t scene;
};
static_assert(sizeof(TetRec) == 96, "tet record is 96 bytes");

// Per (view, kept tet) record read by the compositing kernels (128 B, one
// cache line): projected vertices, inverse camera depths, SDF, reciprocal 2D
// face determinants, shading features, pixel rectangle.
struct ViewRec {
  float px[4], py[4];
  float iz[4];      // 1 / Z_k
  float f[4];
  float rD[4];      // 1 / the 2D determinant of each projected face (its sign: the
                    // face's orientation); 0 for a degenerate face
  float c[3];
  float zt;         // mean camera depth (blend depth, sort key)
  float n[3];
  uint32_t rx;      // i0 | i1 << 16 (inclusive pixel columns)
  uint32_t ry;      // j0 | j1 << 16
  int32_t kept;     // global kept slot
  int32_t view;
  uint32_t entry0;  // first tile-duplicated entry: filled into LDS copies from the records' first entries
};
static_assert(sizeof(ViewRec) == 128, "view record is 128 bytes");

constexpr int TGRAD_STRIDE = 24;  // floats per per-entry gradient
// A blended (entry, pixel) pair of the 8x8 multi-wave and resort-window
// backwards, 32 bytes: dL/df_prev, dL/df_next, the blend weight T alpha and a
// word (pixel | entry and exit faces << 6 | PAIR_HEAD on the first pair of
// its segment, which also holds the segment's pair count << 11); then the
// entry's record, view, tile (x | y << 16) and gradient slot.  A segment is a
// (tile, entry) with blended pixels: its pairs are consecutive, in pixel
// order, at most 64.
constexpr uint32_t PAIR_HEAD = 1u << 10;
// per-entry gradient layout (screen space of one record)
enum { G_PX = 0, G_PY = 4, G_IZ = 8, G_F = 12, G_C = 16, G_ZT = 19, G_N = 20 };

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
constexpr int PF_TILE = 1024;      // tets per pre-filter block
constexpr int SCAN_TILE = 256;     // records per scan block (the emit kernel's unit too)
constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 4;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;
constexpr int SORT_BITS = 8;

struct Layout {
  int ns, nv;
  int flags;            // render_params.flags of the call
  int64_t kept_cap, rec_cap, entry_cap;
  int64_t pf_blocks, scan_blocks_rec, sort_blocks_max, total_tiles, total_pixels;
  int64_t tile_blocks;   // blocks of 1024 tiles (the tile-list scan)
  int max_scene_views;  // largest number of views of one scene
  size_t o_hdr, o_scene, o_view, o_scene_views, o_view_rec_base, o_scene_kept_base, o_scene_kept_count;
  size_t o_pf_cnt, o_kept_tet, o_trec;
  size_t o_pf_keep;   // pre-filter decisions, one bit per tet (PF_TILE / 32 words per block)
  size_t o_vrec, o_count1, o_key1a, o_scan_part;   // key1a: depth float bits per record
  size_t o_rbox;   // per record: pixel rectangle (rx, ry), view (16 B; the last word unused)
  size_t o_rfirst; // per record: its first entry (4 B, dense: the placement kernel's writes coalesce)
  size_t o_hist;
  size_t o_key2a, o_key2b, o_val2a, o_val2b, o_eflag;
  size_t o_ranges, o_tile_hist, o_tile_order, o_tgrad, o_last, o_tlast;
  size_t o_tile_cnt, o_tile_bsum;   // entries per tile (then the emit cursor); per 1024-tile block, its start
  size_t o_tile_pend;    // per dispatch slot: end of the entries the forward blended (backward walk)
  size_t o_bwd_hist, o_bwd_order, o_bwd_pend;  // backward dispatch order (by walked length)
  // multi-wave 8x8 backward (0 otherwise): per forward slot its blended
  // pairs; per backward slot the base of its pairs; 32 bytes per blended
  // (entry, pixel) pair; per sorted entry the pixels of its tile that blended
  // it (64-bit mask, written for the walked entries; per-tile order only)
  size_t o_slot_pairs, o_bwd_base, o_pairs, o_bmask;
  // resort-window backward (0 when the window is off): per blend, in each
  // tile's blend order, 32 B (T before the blend, raw alpha, upstream
  // gradient . features, exp(s f_next); the pixel's previous blend, faces
  // and pixel, record, gradient slot); per entry slot the pixels of its tile
  // that blended it (64-bit mask) and the place of its first pair
  size_t o_wblend, o_wmask, o_wbase;
  // deterministic backward (0 otherwise): per kept-tet corner a vertex key and
  // corner id (double-buffered for the sort) and its 7 gradient terms (8 floats)
  size_t o_vkey_a, o_vkey_b, o_vval_a, o_vval_b, o_vterm;
  int vkey_bits;         // bit length of the total vertex count
  size_t bytes;
};

bool plan_layout(const render_scene* scenes, int ns, const render_view* views, int nv, const render_params* p,
                 int64_t kept_cap, int64_t entry_cap, Layout& L, const char** why);

// the tile lists: entries placed per tile by the emit kernel (tile keys and
// records), then put in depth order inside each tile; the other buffer pair
// is the depth sort's scratch
inline __host__ __device__ size_t sorted_tile_keys(const Layout& L) { return L.o_key2a; }
inline __host__ __device__ size_t sorted_entry_records(const Layout& L) { return L.o_val2a; }

template <class T>
__host__ __device__ inline T* at(void* ws, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(ws) + off); }

// ---------------------------------------------------------------------------
// launchers (each returns hipSuccess or the launch error)
// ---------------------------------------------------------------------------
hipError_t launch_prefilter(void* ws, const Layout& L, const render_params& p, hipStream_t st);
hipError_t launch_desc_prefilter(const DevScene* hs, int ns, const DevView* hv, int nv, const int32_t* scene_views,
                                 void* ws, const Layout& L, const render_params& p, hipStream_t st);
hipError_t launch_project(void* ws, const Layout& L, const render_params& p, hipStream_t st);
hipError_t launch_tile_depth_sort(void* ws, const Layout& L, hipStream_t st);
hipError_t launch_count_scan(void* ws, const Layout& L, const render_params& p, hipStream_t st);
hipError_t launch_emit(void* ws, const Layout& L, const render_params& p, hipStream_t st);
hipError_t launch_tile_order(void* ws, const Layout& L, hipStream_t st);
constexpr int TILE_BUCKETS = 129;  // tiles bucketed by list length, four buckets per power of two
// the backward-order histogram region: slot counts, slot cursors, pair totals
// and pair cursors (TILE_BUCKETS each)
constexpr int BWD_HIST_WORDS = 4 * TILE_BUCKETS;
hipError_t launch_bwd_order(void* ws, const Layout& L, hipStream_t st);
hipError_t launch_composite(void* ws, const Layout& L, const render_params& p, hipStream_t st);
hipError_t launch_composite_backward(void* ws, const Layout& L, const render_params& p, hipStream_t st);
hipError_t launch_composite_mw(void* ws, const Layout& L, const render_params& p, hipStream_t st);
hipError_t launch_composite_backward_mw(void* ws, const Layout& L, const render_params& p, hipStream_t st);
// the per-pair gradients of the multi-wave backward, reduced per (tile, entry)
hipError_t launch_pair_grads(void* ws, const Layout& L, hipStream_t st);
hipError_t launch_composite_win(void* ws, const Layout& L, const render_params& p, hipStream_t st);
hipError_t launch_composite_backward_win(void* ws, const Layout& L, const render_params& p, hipStream_t st);
hipError_t launch_vertex_backward(void* ws, const Layout& L, const render_params& p, hipStream_t st);
// deterministic backward: sort the kept tets' corners by vertex, sum each vertex's terms in corner order
hipError_t launch_vertex_gather(void* ws, const Layout& L, hipStream_t st);

// per-pixel compositing state is kept (not recomputed by the backward)
inline __host__ __device__ bool keeps_pixel_state(const Layout& L) { return L.o_last != 0; }
// one gradient accumulator per record instead of one gradient per entry
inline __host__ __device__ bool record_grads(const Layout& L) { return (L.flags & RENDER_RECORD_GRADS) != 0; }
inline __host__ __device__ bool deterministic(const Layout& L) { return (L.flags & RENDER_DETERMINISTIC) != 0; }
hipError_t launch_desc_zero_grads(const DevScene* hs, int ns, const DevView* hv, int nv, const int32_t* scene_views,
                                  void* ws, const Layout& L, hipStream_t st);

// radix sort of (uint32 key, uint32 value) pairs, stable, LSD over key bits
// [0, bits).  n is read on the device from *n_dev (clamped to cap).  The
// first pass takes vals_in == nullptr as the identity permutation.  On
// return the sorted data is in (*keys_out, *vals_out), which point at one of
// the two buffer pairs.  `items` (SORT_ITEMS or 8) is the keys per thread
// of a block; hist_blocks is sized for SORT_ITEMS, enough for 8.
hipError_t radix_sort_pairs(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b, bool identity,
                            const uint32_t* n_dev, int64_t cap, int bits, uint32_t* hist, int64_t hist_blocks,
                            hipStream_t st, uint32_t** keys_out, uint32_t** vals_out, int items = SORT_ITEMS);

// unique-edge build, the Sec. 4.2 regularisers and Marching Tetrahedra (geom.hip)
struct EdgeLayout {
  uint64_t n;            // 6 K candidate pairs
  uint64_t sort_blocks, edge_blocks;
  size_t o_n, o_ka, o_va, o_kb, o_vb, o_hist, o_bsum, bytes;
};
struct RegLayout {
  size_t o_m, o_dm, o_part, bytes;
  int blocks;
};
EdgeLayout edge_layout(int32_t K);
hipError_t launch_mesh_edges(const int32_t* tets, int32_t K, int32_t V, int32_t* edges, int32_t* n_edges, void* ws,
                             const EdgeLayout& E, hipStream_t st);
RegLayout reg_layout(int32_t V);
hipError_t launch_regularizers(const float* verts, const int32_t* tets, const float* sdf, int32_t V, int32_t K,
                               const int32_t* edges, const int32_t* n_edges, int64_t edge_cap, const float* weights,
                               double* losses, float* dverts, float* dsdf, void* ws, const RegLayout& R,
                               hipStream_t st);
hipError_t launch_prefilter_bounds(const DevScene& S, float tf, float* bounds, int64_t* kept, hipStream_t st);
hipError_t launch_refit_cube(const float* bounds, const float* cube_in, int R, float* cube_out, hipStream_t st);
hipError_t launch_cube_grid(int R, const float* cube, float* verts, int32_t* tets, hipStream_t st);

struct MTLayout {
  uint64_t edge_blocks, tet_blocks;
  size_t o_vid, o_bsum_e, o_bsum_t, bytes;
};
MTLayout mt_layout(int32_t K, int64_t edge_cap);
hipError_t launch_marching_tets(const float* verts, const int32_t* tets, const float* sdf, int32_t V, int32_t K,
                                const int32_t* edges, const int32_t* n_edges, int64_t edge_cap, float* out_verts,
                                int64_t vert_cap, int32_t* out_tris, int64_t tri_cap, int32_t* counts, void* ws,
                                const MTLayout& M, hipStream_t st);

}  // namespace ts
