/*
 * tetsplat.h -- C ABI of the MI355X (gfx950) tile-based differentiable
 * tetrahedron rasterizer of "Tetrahedron Splatting for 3D Generation"
 * (TeT-Splatting, arXiv 2406.01579).
 *
 * What the library computes (paper passages):
 *   - Scene: a tetrahedral grid (V_T, T) with one SDF value per vertex,
 *     linearly interpolated inside every tet (Sec. 3.1), and one RGB per
 *     vertex; a tet's colour is the mean of its four vertex colours (materials
 *     taken at the tet centre, App. B).
 *   - Pre-filter: tets whose opacity upper bound alpha_max (Eq. 1 at the max
 *     and min vertex SDF) is below prefilter_tf are dropped (Sec. 3.2).
 *   - Normal: n = g/|g| with g the constant SDF gradient of the tet
 *     (Sec. 3.2, App. A.3).
 *   - Per view: cull, project the four vertices, bin each tet to every screen
 *     tile its pixel rectangle touches, sort by (tile, mean vertex depth)
 *     (Sec. 3.3).
 *   - Per pixel: entry/exit SDF values from 2D barycentrics on the projected
 *     faces with perspective correction (App. A.1, A.2), opacity by Eq. 1,
 *     front-to-back alpha blending of colour, depth, normal and opacity
 *     (Eq. 2) with the 3DGS blending thresholds (Sec. 3.3).
 *   - Backward: reverse-order traversal of every tile, chained to the SDF
 *     values, the vertex colours and the vertex positions.
 *
 * Conventions.
 *   - Every pointer inside the structs below is a DEVICE pointer, float32 or
 *     int32, contiguous, row-major.  The struct arrays themselves are HOST
 *     memory and are read during the call only.
 *   - Cameras are OpenCV pinholes: world->camera x_c = R x_w + t with +x right,
 *     +y down, +z forward; pixel (i, j) has centre (i + 0.5, j + 0.5).
 *   - Output image layout: out[8][H][W] = R, G, B, O(opacity), D(depth),
 *     Nx, Ny, Nz.  The background colour is added to RGB as T_final * bg.
 *   - The caller owns every buffer, including the workspace.  The library
 *     never allocates or frees device memory.
 *   - Calls are asynchronous on the given HIP stream (hipStream_t, passed as
 *     void*; NULL is the null stream) unless stated otherwise.
 *   - Return value 0 on success, else one of the negative codes; the message
 *     of the last failure on the calling thread is in render_last_error().
 *     No call aborts or throws across this boundary.
 */
#ifndef TETSPLAT_H
#define TETSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RENDER_OK = 0,
  RENDER_EINVAL = -1,    /* bad argument: null pointer, size, unsupported tile shape or flag */
  RENDER_ENOSPC = -2,    /* workspace smaller than render_workspace_size() says */
  RENDER_EHIP = -3,      /* HIP runtime error; its name is in render_last_error() */
  RENDER_EOVERFLOW = -4  /* a capacity bound was exceeded; outputs are invalid, re-plan */
};

/* render_params.flags */
enum {
  RENDER_RECOMPUTE_STATE = 1, /* the workspace keeps no per-pixel compositing state (8 B per
                                 pixel less: each pixel's last blended entry and the
                                 transmittance before it); the backward recomputes it by a
                                 forward sweep over the tile */
  RENDER_VALIDATE = 2,        /* accepted for compatibility: tet indices are always checked
                                 against [0, V) on the device; a tet with an index outside it is
                                 dropped and counted in render_status.invalid_index */
  RENDER_DETERMINISTIC = 4,   /* bitwise-reproducible gradients: every sum runs in a fixed order
                                 (an entry's pixel groups in group order; a vertex's per-tet terms
                                 in kept-tet order, after a stable sort of the kept tets' corners
                                 by vertex).  Slower; needs 4 x 48 B more workspace per kept tet.
                                 Not with RENDER_RECORD_GRADS */
  RENDER_RECORD_GRADS = 8     /* the compositing backward adds each tile's gradient of a record
                                 into one 96 B accumulator per (view, kept tet) record (float
                                 atomics) instead of storing 96 B per (record, tile) entry: a
                                 smaller workspace, gradients reproducible to rounding only */
};

typedef struct {
  const float* verts;   /* [V,3] vertex positions */
  const int32_t* tets;  /* [K,4] vertex indices of each tet */
  const float* sdf;     /* [V]   signed distance per vertex */
  const float* colors;  /* [V,3] RGB per vertex */
  int32_t V, K;
  float s;              /* steepness of Eq. 1 (s of Phi_s) */
} render_scene;

typedef struct {
  int32_t scene;        /* index into the scene array */
  int32_t width, height;
  float R[9];           /* row-major world->camera rotation */
  float t[3];
  float fx, fy, cx, cy;
  float znear;          /* tets with any vertex depth below znear are culled */
  float bg[3];          /* background RGB */
  float* out;           /* [8,H,W] output image, written by render_forward */
} render_view;

typedef struct {
  int32_t tile_w, tile_h; /* screen tile; supported: 8x8, 16x8, 8x16, 16x16, 32x8 */
  int32_t flags;          /* RENDER_* flags above */
  int32_t waves;          /* 64-lane waves sharing one 8x8 tile (1, 2, 4, 8; 0: 4); larger
                             tiles use one wave per 8x8 block of pixels */
  float alpha_min;        /* skip a tet whose alpha is below this (3DGS: 1/255) */
  float alpha_clamp;      /* clamp alpha to at most this (3DGS: 0.99) */
  float t_min;            /* stop before a tet that takes T below this (3DGS: 1e-4) */
  float prefilter_tf;     /* pre-filter threshold T_f on alpha_max (paper: 1/255) */
  int32_t window;         /* per-pixel resort window N_w (Sec. 3.3), 0..RENDER_WINDOW_MAX; 0: off,
                             the blend order is the per-tile order.  With N_w > 0 each pixel passes
                             its candidates, in the per-tile order, through a buffer of N_w entries
                             ordered by the depth where its ray enters the tet; on overflow the
                             nearest leaves and is blended, at the end of the list the rest leave
                             nearest first (equal depths: arrival order); only candidates with
                             alpha >= alpha_min enter.  Needs 8x8 tiles; the workspace then holds
                             16 B per (entry, pixel of its tile) for the backward. */
  int32_t chunk_fwd;      /* entries staged in LDS per step of the forward's walk of a tile list:
                             32 or 64 (0: 64).  With chunk_bwd, only on the multi-wave 8x8 path
                             (8x8 tiles, waves > 1, no resort window).  A speed knob: images and
                             gradients do not depend on it. */
  int32_t chunk_bwd;      /* the same for the backward's walk: 16 or 32 (0: 32) */
} render_params;

#define RENDER_WINDOW_MAX 8

typedef struct {
  float* dverts;        /* [V,3] dL/dverts, overwritten */
  float* dsdf;          /* [V]   dL/dsdf, overwritten */
  float* dcolors;       /* [V,3] dL/dcolors, overwritten */
} render_grads;

typedef struct {
  int64_t entries;      /* tile-duplicated (tet, tile) entries of the last forward */
  int64_t kept;         /* tets kept by the pre-filter, summed over scenes */
  int64_t records;      /* (view, kept tet) records */
  int32_t overflow;     /* bit 0: kept capacity, bit 1: entry capacity exceeded (the forward's
                           outputs are invalid); bit 2: the (entry, pixel) pairs the forward
                           blended exceed the entry capacity (multi-wave 8x8 path): the outputs
                           stand, a backward of this forward would not */
  int32_t invalid_index;/* nonzero if some tet had a vertex index outside [0, V) */
  int64_t entry_capacity, kept_capacity;
  int64_t entries_needed; /* entry capacity the forward and its backward want (exact even on
                             overflow): its entries, or its blended pairs if more */
} render_status;

/*
 * Workspace size in bytes for a forward/backward pair on these scenes and
 * views.  kept_capacity bounds the total number of tets kept by the
 * pre-filter (0: the sum of K over scenes, always sufficient);
 * entry_capacity bounds the number of (tet, tile) entries over all views
 * (0: 8 per (view, kept tet) record).  Pure host computation; the views'
 * output pointers are not read and may be NULL.
 */
int render_workspace_size(const render_scene* scenes, int n_scenes, const render_view* views, int n_views,
                          const render_params* params, int64_t kept_capacity, int64_t entry_capacity,
                          size_t* bytes);

/*
 * Forward pass (Sec. 3.2-3.3, Eq. 1-2): writes every view's out[8,H,W] and
 * leaves the tiling, the sorted lists and the per-pixel state in the
 * workspace for render_backward.  The capacities are the ones the workspace
 * was sized for (same arguments as render_workspace_size).  Asynchronous: a
 * capacity overflow is reported by render_read_status(), not by the return
 * value.
 */
int render_forward(const render_scene* scenes, int n_scenes, const render_view* views, int n_views,
                   const render_params* params, int64_t kept_capacity, int64_t entry_capacity,
                   void* workspace, size_t workspace_bytes, void* stream);

/*
 * Backward pass: given dL/dout (dL_dout[v] is a device [8,H,W] array for view
 * v) and the workspace of the matching render_forward call (same scenes,
 * views, params and capacities, inputs unchanged), overwrites grads[s] for
 * every scene s.  Gradients flow through Eq. 1, the barycentric and
 * perspective interpolation, the projection, the normal and the colour mean;
 * clamped, skipped and unreached tets contribute zero.  Without
 * RENDER_DETERMINISTIC, sums over an entry's pixel groups and over a vertex's
 * tets use float atomics, so the result is reproducible to rounding, not
 * bitwise; with it, bitwise.
 */
int render_backward(const render_scene* scenes, int n_scenes, const render_view* views, int n_views,
                     const render_params* params, int64_t kept_capacity, int64_t entry_capacity,
                     void* workspace, size_t workspace_bytes, const float* const* dL_dout,
                     render_grads* grads, void* stream);

/* Synchronises the stream and reads the counters of the last forward. */
int render_read_status(const void* workspace, render_status* status, void* stream);

/*
 * render_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same forward, with the library's own static device workspace of
 * RENDER_STATIC_WORKSPACE_BYTES in place of a caller buffer.  The caller
 * still passes inputs and outputs (views[v].out).  The call allocates
 * nothing: the workspace is a file-scope device array that each GPU the
 * library runs on holds until the process ends; its address is looked up
 * once per device on the first call made with that device current.
 *   - A problem whose workspace (render_workspace_size with the same
 *     arguments) exceeds RENDER_STATIC_WORKSPACE_BYTES returns RENDER_ENOSPC
 *     before anything is launched.
 *   - header_copy (optional, may be NULL): device or pinned host memory of
 *     RENDER_STATUS_BYTES; the status header is copied there asynchronously
 *     on the stream after the forward (decode it with render_decode_status
 *     once the stream has reached it).
 *   - Every call on one GPU shares that GPU's array, which keeps the last
 *     call's contents (the forward initialises everything it reads): calls
 *     that overlap on one GPU race, and render_backward cannot follow this
 *     call (it needs the caller's workspace).
 */
#define RENDER_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int render_forward_static(const render_scene* scenes, int n_scenes, const render_view* views, int n_views,
                          const render_params* params, int64_t kept_capacity, int64_t entry_capacity,
                          void* header_copy, void* stream);

/*
 * For callers that do not want a synchronisation after every forward: copy
 * the first RENDER_STATUS_BYTES bytes of the workspace to host memory
 * asynchronously (e.g. into pinned memory on the same stream), wait for that
 * copy when convenient, and decode it here.  Pure host computation.
 */
#define RENDER_STATUS_BYTES 256
int render_decode_status(const void* header_copy, render_status* status);

/*
 * Device pointers into the workspace for inspection by tests (valid after a
 * render_forward on that workspace; pure host computation):
 *   tile_keys[E]        uint32 global tile id of each sorted entry
 *   entry_record[E]     int32 (view, kept tet) record of each sorted entry
 *   kept_tet[kept]      int32 tet id of each kept slot, ascending per scene
 *   view_rec_base[nv]   int32 first record of each view; record r of view v
 *                       holds kept slot scene_kept_base[scene] + r - base
 *   scene_kept_base[ns], scene_kept_count[ns]  int32
 *   ranges[tiles][2]    uint32 half-open entry range of each global tile
 *   last[pixels], t_last[pixels]  per-pixel compositing state (NULL with RENDER_RECOMPUTE_STATE)
 * Global tile ids concatenate the views' row-major tile grids; pixel ids
 * concatenate the views' row-major pixel grids.
 */
typedef struct {
  const uint32_t* tile_keys;
  const int32_t* entry_record;
  const int32_t* kept_tet;
  const int32_t* view_rec_base;
  const int32_t* scene_kept_base;
  const int32_t* scene_kept_count;
  const uint32_t* ranges;
  const int32_t* last;
  const float* t_last;
  int64_t total_tiles, total_pixels;
} render_debug_view;
int render_debug_pointers(const render_scene* scenes, int n_scenes, const render_view* views, int n_views,
                          const render_params* params, int64_t kept_capacity, int64_t entry_capacity,
                          const void* workspace, render_debug_view* out);

/*
 * Stage timing.  render_profile(1) resets the totals and, from then on,
 * brackets every pipeline stage of render_forward / render_backward with a
 * pair of HIP events recorded on the call's stream (the stream the stage's
 * kernels run on); render_profile(0) stops.  render_profile_read waits for
 * the recorded events and returns, per stage, the summed milliseconds and the
 * number of timed launches.  Not for use under stream capture.  Not thread
 * safe: profile from one host thread.
 */
enum {
  RENDER_STAGE_UPLOAD = 0,      /* descriptor upload (and header reset) */
  RENDER_STAGE_PREFILTER = 1,   /* alpha_max pre-filter, compaction, normals */
  RENDER_STAGE_PROJECT = 2,     /* per-view projection and tile counts */
  RENDER_STAGE_DEPTH_SORT = 3,  /* depth order inside every tile's list */
  RENDER_STAGE_SCAN = 4,        /* entry counts per record and per tile, their scans, tile lists */
  RENDER_STAGE_EMIT = 5,        /* entries placed into the tile lists */
  RENDER_STAGE_PAIR_GRADS = 6,  /* backward: per-(entry, pixel) gradients summed per (tile, entry) */
  RENDER_STAGE_RANGES = 7,      /* dispatch orders (forward and backward) */
  RENDER_STAGE_COMPOSITE = 8,   /* forward compositing */
  RENDER_STAGE_ZERO_GRADS = 9,  /* gradient buffer clear */
  RENDER_STAGE_COMPOSITE_BWD = 10, /* reverse-order compositing backward (walk and recurrence) */
  RENDER_STAGE_VERTEX_BWD = 11, /* per-record chain to vertices */
  RENDER_NSTAGES = 12
};
int render_profile(int enable);
int render_profile_read(double* ms /* [RENDER_NSTAGES] */, int64_t* counts /* [RENDER_NSTAGES] */);

/*
 * Geometry regularisers (Sec. 4.2).
 *
 * render_mesh_edges: the unique undirected edges of a tet mesh, each once as
 * (a, b) with a < b, in ascending (a, b) order -- the edge set of the
 * normal-consistency term.  tets: device int32 [K][4], 16-byte aligned;
 * a tet with an index outside [0, V) contributes no edge.  edges: device
 * int32 [6K][2] (6K pairs always suffice); n_edges: device int32, receives
 * the count.  Workspace from render_mesh_edges_workspace_size (device,
 * caller-owned).  Asynchronous on stream.  Built once per topology.
 */
int render_mesh_edges_workspace_size(int32_t K, size_t* bytes);
int render_mesh_edges(const int32_t* tets, int32_t K, int32_t V, int32_t* edges, int32_t* n_edges,
                      void* workspace, size_t workspace_bytes, void* stream);

/*
 * render_regularizers: the eikonal term L_eik = sum over tets of
 * (|g_k| - 1)^2, g_k the SDF gradient inside tet k (App. A.3), and the
 * normal-consistency term L_nc = sum over edges of 1 - cos(m_a, m_b), m_v the
 * sum of the unit normals g_k/|g_k| of the tets that contain vertex v.  Tets
 * with a zero determinant, or an index outside [0, V), are left out of both;
 * an edge with a zero vertex normal at either end is left out.
 *   verts [V][3], sdf [V], tets [K][4] (16-byte aligned): device inputs;
 *   edges / n_edges: as written by render_mesh_edges (edge_capacity bounds
 *     the count that is read);
 *   losses: device double[2] <- (L_eik, L_nc), unweighted; may be NULL;
 *   dverts [V][3], dsdf [V]: device; the gradient of
 *     weights[0] * L_eik + weights[1] * L_nc is ADDED to them (so it can
 *     follow render_backward); both NULL for the losses alone;
 *   weights: device float[2], read only when gradients are requested.
 * Gradients use float atomics (reproducible to rounding, not bitwise).
 * Asynchronous on stream; no host synchronisation, so it can be captured.
 */
int render_regularizers_workspace_size(int32_t V, int32_t K, size_t* bytes);
int render_regularizers(const float* verts, const int32_t* tets, const float* sdf, int32_t V, int32_t K,
                        const int32_t* edges, const int32_t* n_edges, int64_t edge_capacity, const float* weights,
                        double* losses, float* dverts, float* dsdf, void* workspace, size_t workspace_bytes,
                        void* stream);

/*
 * render_prefilter_bounds: coarse-to-fine pre-filtering (App. B).  The
 * bounding box of the vertices of the tets the pre-filter keeps (alpha_max of
 * Eq. 1 at the tet's largest and smallest SDF value >= params->prefilter_tf,
 * the rule render_forward applies), and their count.  A caller rebuilds its
 * grid over that box, samples the SDF there and pre-filters again.
 *   scene: one scene (device pointers; colors are not read and may be NULL);
 *   bounds: device float[6] <- (min x, min y, min z, max x, max y, max z),
 *     all NaN when no tet is kept;
 *   kept: device int64 <- the number of kept tets (may be NULL).
 * Exact and deterministic (min/max and integer counts).  Tets with an index
 * outside [0, V) are not kept.  Asynchronous on stream; no workspace.
 */
int render_prefilter_bounds(const render_scene* scene, const render_params* params, float* bounds, int64_t* kept,
                            void* stream);

/*
 * Coarse-to-fine grid rebuild (App. B: the second pre-filter pass runs on a
 * grid refitted around the tets the first pass keeps).  Grids are Kuhn cube
 * grids: R^3 cubic cells of size h with low corner (lx, ly, lz), given as a
 * DEVICE float[4] cube = (lx, ly, lz, h); vertex (x, y, z), 0 <= x, y, z <= R,
 * has index x + (R+1)(y + (R+1) z) and position low + (x, y, z) h (float32,
 * one product and one sum per coordinate); cell q = x + R(y + R z) is split
 * into tets 6q + p along the six axis orders (a, b, c), p in lexicographic
 * order, with vertices (v0, v0 + e_a, v0 + e_a + e_b, v0 + (1, 1, 1)).
 *
 * render_cube_grid writes verts: device float [(R+1)^3][3] and, unless tets
 * is NULL, tets: device int32 [6 R^3][4] (16-byte aligned).  1 <= R <= 1024.
 *
 * render_refit_cube: the second-pass cube from bounds (as written by
 * render_prefilter_bounds for the first pass) and the first-pass cube cube_in
 * (device float[4]); writes cube_out (device float[4]).  The new cube keeps R
 * and cubic cells: centred on the box, side = the box's largest extent plus
 * one first-pass cell on each side (extents in float32, the side rounded to
 * float32 from their double sum, centre and low corner in double rounded to
 * float32, h = side / R in float32).  A NaN box (nothing kept) copies
 * cube_in.  cube_out may not alias bounds.
 *
 * Both are asynchronous on stream, take no workspace and read nothing on the
 * host, so the two passes need no synchronisation.
 */
int render_cube_grid(int32_t R, const float* cube, float* verts, int32_t* tets, void* stream);
int render_refit_cube(const float* bounds, const float* cube_in, int32_t R, float* cube_out, void* stream);

/*
 * render_marching_tets: triangle mesh of the zero level set (Marching
 * Tetrahedra, the mesh extraction of Sec. 4.1).  A vertex is inside when
 * f < 0.  Every edge of `edges` (as written by render_mesh_edges for the
 * same tets) whose ends differ in that test carries one surface vertex at
 * the zero of the linear interpolant, p = x_a + t (x_b - x_a),
 * t = f_a / (f_a - f_b); vertices are numbered in edge order.  A tet with
 * one or three inside vertices gives one triangle, with two inside a quad
 * split into two triangles; triangles are in tet order and wind outward
 * (normal from the inside vertices to the outside ones).
 *   out_verts: device float [vert_capacity][3]; out_tris: device int32
 *   [tri_capacity][3] (indices into out_verts); counts: device int32[2] <-
 *   (vertices, triangles) -- the full counts, also when they exceed the
 *   capacities (then only the first `capacity` items are written);
 *   vert_capacity <= edge count and tri_capacity <= 2 K always suffice.
 * Tets with an index outside [0, V) give no triangle.  Asynchronous on
 * stream; workspace from render_marching_tets_workspace_size.
 */
int render_marching_tets_workspace_size(int32_t K, int64_t edge_capacity, size_t* bytes);
int render_marching_tets(const float* verts, const int32_t* tets, const float* sdf, int32_t V, int32_t K,
                         const int32_t* edges, const int32_t* n_edges, int64_t edge_capacity, float* out_verts,
                         int64_t vert_capacity, int32_t* out_tris, int64_t tri_capacity, int32_t* counts,
                         void* workspace, size_t workspace_bytes, void* stream);

/* Message of the last failed call on this thread ("" if none). */
const char* render_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TETSPLAT_H */
