// Host side of the C ABI declared in include/tetsplat.h: argument checks,
// workspace layout, and the forward/backward launch sequences.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ts_internal.h"

namespace ts {
namespace {

thread_local std::string g_err;

// Optional per-stage timing with HIP events recorded on the caller's stream.
struct StageEvent {
  int stage;
  hipEvent_t a, b;
};
struct Profiler {
  bool on = false;
  std::vector<StageEvent> pending;
  std::vector<hipEvent_t> pool;
  double ms[RENDER_NSTAGES] = {};
  int64_t count[RENDER_NSTAGES] = {};
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Profiler g_prof;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(RENDER_EHIP, "%s: %s (%s)", where, hipGetErrorName(e), hipGetErrorString(e));
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool tile_ok(int tw, int th) {
  const int k = tw * 1000 + th;
  return k == 8008 || k == 16008 || k == 8016 || k == 16016 || k == 32008;
}

int check_args(const render_scene* scenes, int ns, const render_view* views, int nv, const render_params* p,
               bool need_out = true) {
  if (!scenes || !views || !p) return fail(RENDER_EINVAL, "null scenes, views or params");
  if (ns <= 0 || nv <= 0) return fail(RENDER_EINVAL, "need at least one scene and one view (got %d, %d)", ns, nv);
  if (!tile_ok(p->tile_w, p->tile_h))
    return fail(RENDER_EINVAL, "unsupported tile %dx%d (8x8, 16x8, 8x16, 16x16, 32x8)", p->tile_w, p->tile_h);
  if (p->flags & ~(RENDER_RECOMPUTE_STATE | RENDER_VALIDATE | RENDER_DETERMINISTIC | RENDER_RECORD_GRADS))
    return fail(RENDER_EINVAL, "unknown flags 0x%x", p->flags);
  if ((p->flags & RENDER_DETERMINISTIC) && (p->flags & RENDER_RECORD_GRADS))
    return fail(RENDER_EINVAL, "RENDER_DETERMINISTIC and RENDER_RECORD_GRADS exclude each other");
  if (!(p->alpha_clamp > 0.0f && p->alpha_clamp <= 1.0f)) return fail(RENDER_EINVAL, "alpha_clamp must be in (0, 1]");
  if (!(p->waves == 0 || p->waves == 1 || p->waves == 2 || p->waves == 4 || p->waves == 8))
    return fail(RENDER_EINVAL, "waves must be 0, 1, 2, 4 or 8 (got %d)", p->waves);
  if (p->window < 0 || p->window > RENDER_WINDOW_MAX)
    return fail(RENDER_EINVAL, "window must be in [0, %d] (got %d)", RENDER_WINDOW_MAX, p->window);
  if (p->window > 0 && (p->tile_w != 8 || p->tile_h != 8))
    return fail(RENDER_EINVAL, "the resort window needs 8x8 tiles (got %dx%d)", p->tile_w, p->tile_h);
  if (!(p->chunk_fwd == 0 || p->chunk_fwd == 32 || p->chunk_fwd == 64))
    return fail(RENDER_EINVAL, "chunk_fwd must be 0, 32 or 64 (got %d)", p->chunk_fwd);
  if (!(p->chunk_bwd == 0 || p->chunk_bwd == 16 || p->chunk_bwd == 32))
    return fail(RENDER_EINVAL, "chunk_bwd must be 0, 16 or 32 (got %d)", p->chunk_bwd);
  if ((p->chunk_fwd | p->chunk_bwd) != 0 &&
      (p->tile_w != 8 || p->tile_h != 8 || p->waves == 1 || p->window > 0))
    return fail(RENDER_EINVAL, "chunk lengths apply to the multi-wave 8x8 path only (8x8 tiles, waves > 1, "
                "no resort window)");
  for (int s = 0; s < ns; ++s) {
    const render_scene& S = scenes[s];
    if (S.V < 0 || S.K < 0) return fail(RENDER_EINVAL, "scene %d: negative V or K", s);
    if (S.K > 0 && (!S.verts || !S.tets || !S.sdf || !S.colors))
      return fail(RENDER_EINVAL, "scene %d: null device pointer", s);
    if (((uintptr_t)S.tets & 15u) != 0) return fail(RENDER_EINVAL, "scene %d: tets must be 16-byte aligned", s);
    if (S.K > (1 << 30) || S.V > (1 << 30)) return fail(RENDER_EINVAL, "scene %d: too large", s);
  }
  for (int v = 0; v < nv; ++v) {
    const render_view& V = views[v];
    if (V.scene < 0 || V.scene >= ns) return fail(RENDER_EINVAL, "view %d: scene index %d out of range", v, V.scene);
    if (V.width <= 0 || V.height <= 0 || V.width > 16384 || V.height > 16384)
      return fail(RENDER_EINVAL, "view %d: image size %dx%d out of range", v, V.width, V.height);
    if (need_out && !V.out) return fail(RENDER_EINVAL, "view %d: null output", v);
  }
  return RENDER_OK;
}

void fill_desc(const render_scene* scenes, int ns, const render_view* views, int nv, const render_params* p,
               const Layout& L, std::vector<DevScene>& hs, std::vector<DevView>& hv, std::vector<int32_t>& sv) {
  hs.assign(ns, DevScene{});
  int blk = 0;
  int64_t vb = 0;
  for (int s = 0; s < ns; ++s) {
    hs[s].vbase = (int32_t)vb;
    vb += scenes[s].V;
    DevScene& d = hs[s];
    d.verts = scenes[s].verts;
    d.tets = scenes[s].tets;
    d.sdf = scenes[s].sdf;
    d.colors = scenes[s].colors;
    d.V = scenes[s].V;
    d.K = scenes[s].K;
    d.s = scenes[s].s;
    d.block_base = blk;
    d.n_blocks = (scenes[s].K + PF_TILE - 1) / PF_TILE;
    blk += d.n_blocks;
  }
  // views grouped by scene (stable): scene s owns sv[view_first .. + view_count)
  sv.clear();
  for (int s = 0; s < ns; ++s) {
    hs[s].view_first = (int32_t)sv.size();
    for (int v = 0; v < nv; ++v)
      if (views[v].scene == s) sv.push_back(v);
    hs[s].view_count = (int32_t)sv.size() - hs[s].view_first;
  }
  hv.assign(nv, DevView{});
  int64_t tb = 0, pb = 0;
  for (int v = 0; v < nv; ++v) {
    DevView& d = hv[v];
    const render_view& V = views[v];
    std::memcpy(d.R, V.R, sizeof d.R);
    std::memcpy(d.t, V.t, sizeof d.t);
    d.fx = V.fx; d.fy = V.fy; d.cx = V.cx; d.cy = V.cy; d.znear = V.znear;
    std::memcpy(d.bg, V.bg, sizeof d.bg);
    d.out = V.out;
    d.dout = nullptr;
    d.scene = V.scene;
    d.W = V.width;
    d.H = V.height;
    d.tiles_x = (V.width + p->tile_w - 1) / p->tile_w;
    d.tiles_y = (V.height + p->tile_h - 1) / p->tile_h;
    d.tile_base = (int32_t)tb;
    d.pix_base = (int32_t)pb;
    d.s = scenes[V.scene].s;
    tb += (int64_t)d.tiles_x * d.tiles_y;
    pb += (int64_t)V.width * V.height;
  }
  (void)L;
}

}  // namespace

bool plan_layout(const render_scene* scenes, int ns, const render_view* views, int nv, const render_params* p,
                 int64_t kept_cap, int64_t entry_cap, Layout& L, const char** why) {
  L = Layout{};
  L.ns = ns;
  L.nv = nv;
  L.flags = p->flags;
  int64_t sumK = 0, sumV = 0, pf_blocks = 0;
  for (int s = 0; s < ns; ++s) {
    sumK += scenes[s].K;
    sumV += scenes[s].V;
    pf_blocks += (scenes[s].K + PF_TILE - 1) / PF_TILE;
  }
  if (kept_cap <= 0 || kept_cap > sumK) kept_cap = sumK;
  int64_t rec_cap = 0, tiles = 0, pixels = 0;
  for (int v = 0; v < nv; ++v) {
    const int64_t Ks = scenes[views[v].scene].K;
    rec_cap += Ks < kept_cap ? Ks : kept_cap;
    tiles += (int64_t)((views[v].width + p->tile_w - 1) / p->tile_w) * ((views[v].height + p->tile_h - 1) / p->tile_h);
    pixels += (int64_t)views[v].width * views[v].height;
  }
  if (entry_cap <= 0) entry_cap = 8 * rec_cap;
  if (entry_cap < 1) entry_cap = 1;
  if (rec_cap < 1) rec_cap = 1;
  if (kept_cap < 1) kept_cap = 1;
  const int64_t lim = (int64_t)1 << 31;
  const bool det = (p->flags & RENDER_DETERMINISTIC) != 0;
  if (rec_cap >= lim || entry_cap >= lim || tiles >= lim || pixels >= lim || kept_cap >= lim || sumV >= lim ||
      (det && 4 * kept_cap >= lim)) {
    *why = "problem exceeds 2^31 records, entries, tiles, pixels, vertices or kept-tet corners";
    return false;
  }
  L.kept_cap = kept_cap;
  L.rec_cap = rec_cap;
  L.entry_cap = entry_cap;
  L.pf_blocks = pf_blocks;
  L.scan_blocks_rec = (rec_cap + SCAN_TILE - 1) / SCAN_TILE;
  // the radix sort is left for the deterministic backward's corner sort
  const int64_t smax = det ? 4 * kept_cap : 1;
  L.sort_blocks_max = (smax + SORT_TILE - 1) / SORT_TILE;
  L.total_tiles = tiles;
  L.total_pixels = pixels;
  L.tile_blocks = (tiles + 1023) / 1024;
  int vbits = 1;
  while (((int64_t)1 << vbits) < sumV) ++vbits;
  L.vkey_bits = vbits;
  {
    std::vector<int> vps(ns, 0);
    for (int v = 0; v < nv; ++v) ++vps[views[v].scene];
    L.max_scene_views = 0;
    for (int s = 0; s < ns; ++s) L.max_scene_views = vps[s] > L.max_scene_views ? vps[s] : L.max_scene_views;
  }

  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at_ = o; o = align_up(o + bytes, 256); return at_; };
  L.o_hdr = take(sizeof(DevHeader));
  L.o_scene = take(sizeof(DevScene) * ns);
  L.o_view = take(sizeof(DevView) * nv);
  L.o_scene_views = take(4 * (size_t)nv);
  L.o_view_rec_base = take(4 * (size_t)nv);
  L.o_scene_kept_base = take(4 * (size_t)ns);
  L.o_scene_kept_count = take(4 * (size_t)ns);
  L.o_pf_cnt = take(4 * (size_t)(pf_blocks + 1));
  L.o_pf_keep = take(4 * (size_t)(PF_TILE / 32) * (size_t)(pf_blocks + 1));
  L.o_kept_tet = take(4 * (size_t)kept_cap);
  L.o_trec = take(sizeof(TetRec) * (size_t)kept_cap);
  L.o_vrec = take(sizeof(ViewRec) * (size_t)rec_cap);
  L.o_rbox = take(16 * (size_t)rec_cap);
  L.o_rfirst = take(4 * (size_t)rec_cap);
  L.o_count1 = take(4 * (size_t)rec_cap);
  L.o_key1a = take(4 * (size_t)rec_cap);
  L.o_scan_part = take(4 * (size_t)(L.scan_blocks_rec + 1));
  L.o_hist = take(4 * (size_t)(256 * L.sort_blocks_max + 256));
  L.o_key2a = take(4 * (size_t)entry_cap);
  L.o_key2b = take(4 * (size_t)entry_cap);
  L.o_val2a = take(4 * (size_t)entry_cap);
  L.o_val2b = take(4 * (size_t)entry_cap);
  L.o_eflag = take((size_t)entry_cap + 16);  // padded: the vertex backward reads aligned 8-byte words
  L.o_tile_cnt = take(4 * (size_t)tiles);
  L.o_tile_bsum = take(4 * (size_t)(L.tile_blocks + 1));   // right after the counts: cleared together
  L.o_ranges = take(8 * (size_t)tiles);
  L.o_tile_hist = take(4 * 2 * (size_t)TILE_BUCKETS);  // right after the ranges: cleared together
  L.o_tile_order = take(sizeof(TileSlot) * (size_t)tiles);
  L.o_tile_pend = take(4 * (size_t)tiles);
  L.o_bwd_hist = take(4 * (size_t)BWD_HIST_WORDS);
  L.o_bwd_order = take(sizeof(TileSlot) * (size_t)tiles);
  L.o_bwd_pend = take(4 * (size_t)tiles);
  // screen-space gradients: one per entry, or one accumulator per record
  L.o_tgrad = take(4 * (size_t)TGRAD_STRIDE *
                   (size_t)((p->flags & RENDER_RECORD_GRADS) ? rec_cap : entry_cap));
  const bool keep_state = (p->flags & RENDER_RECOMPUTE_STATE) == 0;
  L.o_last = keep_state ? take(4 * (size_t)pixels) : 0;
  L.o_tlast = keep_state ? take(4 * (size_t)pixels) : 0;
  if (p->window > 0) {
    L.o_wblend = take(32 * (size_t)entry_cap);   // at most entry_capacity blends
    L.o_wmask = take(8 * (size_t)entry_cap);
    L.o_wbase = take(4 * (size_t)entry_cap);
  }
  // the 8x8 backwards that go through per-pair terms: multi-wave, and every
  // resort-window launch
  const bool pairs_path = p->tile_w == 8 && p->tile_h == 8 && (p->waves != 1 || p->window > 0);
  if (pairs_path) {
    L.o_slot_pairs = take(4 * (size_t)tiles);
    L.o_bwd_base = take(4 * (size_t)tiles);
    L.o_pairs = take(32 * (size_t)entry_cap);   // at most entry_capacity blended pairs
    if (p->window == 0) L.o_bmask = take(8 * (size_t)entry_cap);
  }
  if (det) {
    const size_t nc = 4 * (size_t)kept_cap;
    L.o_vkey_a = take(4 * nc);
    L.o_vkey_b = take(4 * nc);
    L.o_vval_a = take(4 * nc);
    L.o_vval_b = take(4 * nc);
    L.o_vterm = take(32 * nc);
  }
  L.bytes = o;
  return true;
}

namespace {

int prepare(const render_scene* scenes, int ns, const render_view* views, int nv, const render_params* p,
            int64_t kept_cap, int64_t entry_cap, void* ws, size_t ws_bytes, Layout& L) {
  int rc = check_args(scenes, ns, views, nv, p);
  if (rc) return rc;
  const char* why = nullptr;
  if (!plan_layout(scenes, ns, views, nv, p, kept_cap, entry_cap, L, &why)) return fail(RENDER_EINVAL, "%s", why);
  if (!ws) return fail(RENDER_EINVAL, "null workspace");
  if (((uintptr_t)ws & 255u) != 0) return fail(RENDER_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < L.bytes)
    return fail(RENDER_ENOSPC, "workspace has %zu bytes, needs %zu", ws_bytes, L.bytes);
  return RENDER_OK;
}

// 8x8 tiles with more than one wave use the multi-wave compositing kernels
int effective_waves(const render_params& p) { return p.waves == 0 ? 4 : p.waves; }
bool multiwave(const render_params& p) { return p.tile_w == 8 && p.tile_h == 8 && effective_waves(p) > 1; }
render_params with_waves(render_params p) {
  p.waves = effective_waves(p);
  if (p.chunk_fwd == 0) p.chunk_fwd = 64;
  if (p.chunk_bwd == 0) p.chunk_bwd = 32;
  return p;
}

#define TS_TRY(call, name)                        \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_fail(e_, name); \
  } while (0)

// run one pipeline stage, bracketed by events when profiling is on
#define TS_STAGE(stage, call, name)                                   \
  do {                                                                \
    hipEvent_t ea_ = nullptr, eb_ = nullptr;                          \
    if (g_prof.on) {                                                  \
      ea_ = g_prof.get();                                             \
      eb_ = g_prof.get();                                             \
      if (ea_) hipEventRecord(ea_, st);                               \
    }                                                                 \
    TS_TRY(call, name);                                               \
    if (ea_ && eb_) {                                                 \
      hipEventRecord(eb_, st);                                        \
      g_prof.pending.push_back(StageEvent{stage, ea_, eb_});          \
    }                                                                 \
  } while (0)

// The workspace of render_forward_static: one copy per device, reached only
// through the address hipGetSymbolAddress returns for the current device (the
// array's name is a host-side stand-in in host code).
__device__ __align__(256) unsigned char scratch[RENDER_STATIC_WORKSPACE_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

int static_workspace(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "get device");
  if (dev < 0 || dev >= MAX_DEVICES) return fail(RENDER_EINVAL, "device %d beyond the %d supported", dev, MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "static workspace address");
    if (!p) return fail(RENDER_EHIP, "static workspace address is null");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RENDER_OK;
}

}  // namespace
}  // namespace ts

using namespace ts;

extern "C" {

const char* render_last_error(void) { return g_err.c_str(); }

int render_mesh_edges_workspace_size(int32_t K, size_t* bytes) {
  if (!bytes) return fail(RENDER_EINVAL, "null bytes");
  if (K < 0 || K > 700000000) return fail(RENDER_EINVAL, "K out of range (%d)", K);
  *bytes = ts::edge_layout(K).bytes;
  return RENDER_OK;
}

int render_mesh_edges(const int32_t* tets, int32_t K, int32_t V, int32_t* edges, int32_t* n_edges, void* workspace,
                      size_t workspace_bytes, void* stream) {
  if (K < 0 || K > 700000000 || V < 0 || V > (1 << 30)) return fail(RENDER_EINVAL, "K or V out of range");
  if (!n_edges || !workspace || (K > 0 && (!tets || !edges))) return fail(RENDER_EINVAL, "null pointer");
  if (((uintptr_t)tets & 15u) != 0) return fail(RENDER_EINVAL, "tets must be 16-byte aligned");
  if (((uintptr_t)edges & 7u) != 0) return fail(RENDER_EINVAL, "edges must be 8-byte aligned");
  const ts::EdgeLayout E = ts::edge_layout(K);
  if (workspace_bytes < E.bytes) return fail(RENDER_ENOSPC, "workspace %zu < %zu bytes", workspace_bytes, E.bytes);
  hipError_t e = ts::launch_mesh_edges(tets, K, V, edges, n_edges, workspace, E, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RENDER_EHIP, "mesh edges: %s", hipGetErrorString(e));
  return RENDER_OK;
}

int render_prefilter_bounds(const render_scene* scene, const render_params* params, float* bounds, int64_t* kept,
                            void* stream) {
  if (!scene || !params || !bounds) return fail(RENDER_EINVAL, "null scene, params or bounds");
  const render_scene& S = *scene;
  if (S.V < 0 || S.K < 0 || S.K > (1 << 30) || S.V > (1 << 30)) return fail(RENDER_EINVAL, "V or K out of range");
  if (S.K > 0 && (!S.verts || !S.tets || !S.sdf)) return fail(RENDER_EINVAL, "null device pointer");
  if (((uintptr_t)S.tets & 15u) != 0) return fail(RENDER_EINVAL, "tets must be 16-byte aligned");
  if (((uintptr_t)bounds & 3u) != 0 || ((uintptr_t)kept & 7u) != 0) return fail(RENDER_EINVAL, "misaligned output");
  ts::DevScene d{};
  d.verts = S.verts;
  d.tets = S.tets;
  d.sdf = S.sdf;
  d.colors = S.colors;
  d.V = S.V;
  d.K = S.K;
  d.s = S.s;
  hipError_t e = ts::launch_prefilter_bounds(d, params->prefilter_tf, bounds, kept, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RENDER_EHIP, "prefilter bounds: %s", hipGetErrorString(e));
  return RENDER_OK;
}

int render_cube_grid(int32_t R, const float* cube, float* verts, int32_t* tets, void* stream) {
  if (R < 1 || R > 1024) return fail(RENDER_EINVAL, "R out of range (%d)", R);
  if (!cube || !verts) return fail(RENDER_EINVAL, "null cube or verts");
  if (((uintptr_t)cube & 3u) != 0 || ((uintptr_t)verts & 3u) != 0 || ((uintptr_t)tets & 15u) != 0)
    return fail(RENDER_EINVAL, "misaligned cube, verts or tets");
  hipError_t e = ts::launch_cube_grid(R, cube, verts, tets, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RENDER_EHIP, "cube grid: %s", hipGetErrorString(e));
  return RENDER_OK;
}

int render_refit_cube(const float* bounds, const float* cube_in, int32_t R, float* cube_out, void* stream) {
  if (R < 1 || R > 1024) return fail(RENDER_EINVAL, "R out of range (%d)", R);
  if (!bounds || !cube_in || !cube_out) return fail(RENDER_EINVAL, "null bounds or cube");
  if ((((uintptr_t)bounds | (uintptr_t)cube_in | (uintptr_t)cube_out) & 3u) != 0)
    return fail(RENDER_EINVAL, "misaligned bounds or cube");
  hipError_t e = ts::launch_refit_cube(bounds, cube_in, R, cube_out, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RENDER_EHIP, "refit cube: %s", hipGetErrorString(e));
  return RENDER_OK;
}

int render_marching_tets_workspace_size(int32_t K, int64_t edge_capacity, size_t* bytes) {
  if (!bytes) return fail(RENDER_EINVAL, "null bytes");
  if (K < 0 || K > (1 << 30) || edge_capacity < 0 || edge_capacity > 0x7fffffffll)
    return fail(RENDER_EINVAL, "K or edge_capacity out of range");
  *bytes = ts::mt_layout(K, edge_capacity).bytes;
  return RENDER_OK;
}

int render_marching_tets(const float* verts, const int32_t* tets, const float* sdf, int32_t V, int32_t K,
                         const int32_t* edges, const int32_t* n_edges, int64_t edge_capacity, float* out_verts,
                         int64_t vert_capacity, int32_t* out_tris, int64_t tri_capacity, int32_t* counts,
                         void* workspace, size_t workspace_bytes, void* stream) {
  if (K < 0 || V < 0 || V > (1 << 30) || K > (1 << 30)) return fail(RENDER_EINVAL, "K or V out of range");
  if (edge_capacity < 0 || edge_capacity > 0x7fffffffll || vert_capacity < 0 || tri_capacity < 0)
    return fail(RENDER_EINVAL, "capacity out of range");
  if (!counts || !n_edges || !workspace || (K > 0 && (!verts || !tets || !sdf)) || (edge_capacity > 0 && !edges) ||
      (vert_capacity > 0 && !out_verts) || (tri_capacity > 0 && !out_tris))
    return fail(RENDER_EINVAL, "null pointer");
  if (((uintptr_t)tets & 15u) != 0) return fail(RENDER_EINVAL, "tets must be 16-byte aligned");
  if (((uintptr_t)edges & 7u) != 0) return fail(RENDER_EINVAL, "edges must be 8-byte aligned");
  const ts::MTLayout M = ts::mt_layout(K, edge_capacity);
  if (workspace_bytes < M.bytes) return fail(RENDER_ENOSPC, "workspace %zu < %zu bytes", workspace_bytes, M.bytes);
  hipError_t e = ts::launch_marching_tets(verts, tets, sdf, V, K, edges, n_edges, edge_capacity, out_verts,
                                          vert_capacity, out_tris, tri_capacity, counts, workspace, M,
                                          (hipStream_t)stream);
  if (e != hipSuccess) return fail(RENDER_EHIP, "marching tets: %s", hipGetErrorString(e));
  return RENDER_OK;
}

int render_regularizers_workspace_size(int32_t V, int32_t K, size_t* bytes) {
  if (!bytes) return fail(RENDER_EINVAL, "null bytes");
  if (K < 0 || V < 0 || V > (1 << 30) || K > (1 << 30)) return fail(RENDER_EINVAL, "K or V out of range");
  *bytes = ts::reg_layout(V).bytes;
  return RENDER_OK;
}

int render_regularizers(const float* verts, const int32_t* tets, const float* sdf, int32_t V, int32_t K,
                        const int32_t* edges, const int32_t* n_edges, int64_t edge_capacity, const float* weights,
                        double* losses, float* dverts, float* dsdf, void* workspace, size_t workspace_bytes,
                        void* stream) {
  if (K < 0 || V < 0 || V > (1 << 30) || K > (1 << 30)) return fail(RENDER_EINVAL, "K or V out of range");
  if (edge_capacity < 0 || edge_capacity > 0xffffffffll) return fail(RENDER_EINVAL, "edge_capacity out of range");
  if (!workspace || !n_edges || (K > 0 && (!verts || !tets || !sdf)) || (edge_capacity > 0 && !edges))
    return fail(RENDER_EINVAL, "null pointer");
  if ((dverts == nullptr) != (dsdf == nullptr)) return fail(RENDER_EINVAL, "dverts and dsdf: both or neither");
  if (dverts && !weights) return fail(RENDER_EINVAL, "gradients need weights");
  if (((uintptr_t)tets & 15u) != 0) return fail(RENDER_EINVAL, "tets must be 16-byte aligned");
  if (((uintptr_t)edges & 7u) != 0) return fail(RENDER_EINVAL, "edges must be 8-byte aligned");
  const ts::RegLayout R = ts::reg_layout(V);
  if (workspace_bytes < R.bytes) return fail(RENDER_ENOSPC, "workspace %zu < %zu bytes", workspace_bytes, R.bytes);
  hipError_t e = ts::launch_regularizers(verts, tets, sdf, V, K, edges, n_edges, edge_capacity, weights, losses,
                                         dverts, dsdf, workspace, R, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RENDER_EHIP, "regularizers: %s", hipGetErrorString(e));
  return RENDER_OK;
}

int render_workspace_size(const render_scene* scenes, int n_scenes, const render_view* views, int n_views,
                          const render_params* params, int64_t kept_capacity, int64_t entry_capacity,
                          size_t* bytes) {
  int rc = check_args(scenes, n_scenes, views, n_views, params, false);
  if (rc) return rc;
  if (!bytes) return fail(RENDER_EINVAL, "null bytes");
  Layout L;
  const char* why = nullptr;
  if (!plan_layout(scenes, n_scenes, views, n_views, params, kept_capacity, entry_capacity, L, &why))
    return fail(RENDER_EINVAL, "%s", why);
  *bytes = L.bytes;
  return RENDER_OK;
}

int render_forward(const render_scene* scenes, int n_scenes, const render_view* views, int n_views,
                   const render_params* params, int64_t kept_capacity, int64_t entry_capacity, void* workspace,
                   size_t workspace_bytes, void* stream) {
  Layout L;
  int rc = prepare(scenes, n_scenes, views, n_views, params, kept_capacity, entry_capacity, workspace,
                   workspace_bytes, L);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<DevScene> hs;
  std::vector<DevView> hv;
  std::vector<int32_t> sv;
  fill_desc(scenes, n_scenes, views, n_views, params, L, hs, hv, sv);
  // (the descriptor upload rides on the pre-filter's first launch when it fits)
  TS_STAGE(RENDER_STAGE_PREFILTER,
           launch_desc_prefilter(hs.data(), n_scenes, hv.data(), n_views, sv.data(), workspace, L, *params, st),
           "descriptor upload and pre-filter");
  TS_STAGE(RENDER_STAGE_PROJECT, launch_project(workspace, L, *params, st), "project");
  TS_STAGE(RENDER_STAGE_SCAN, launch_count_scan(workspace, L, *params, st), "count scan and tile lists");
  TS_STAGE(RENDER_STAGE_EMIT, launch_emit(workspace, L, *params, st), "emit");
  TS_STAGE(RENDER_STAGE_RANGES, launch_tile_order(workspace, L, st), "tile order");
  TS_STAGE(RENDER_STAGE_DEPTH_SORT, launch_tile_depth_sort(workspace, L, st), "depth order in tiles");
  TS_STAGE(RENDER_STAGE_COMPOSITE,
           params->window > 0 ? launch_composite_win(workspace, L, with_waves(*params), st)
           : multiwave(*params) ? launch_composite_mw(workspace, L, with_waves(*params), st)
                                : launch_composite(workspace, L, *params, st),
           "composite");
  // the backward's dispatch order, and the places of its per-pair terms
  if (L.o_pairs != 0) TS_STAGE(RENDER_STAGE_RANGES, launch_bwd_order(workspace, L, st), "backward tile order");
  return RENDER_OK;
}

int render_backward(const render_scene* scenes, int n_scenes, const render_view* views, int n_views,
                    const render_params* params, int64_t kept_capacity, int64_t entry_capacity, void* workspace,
                    size_t workspace_bytes, const float* const* dL_dout, render_grads* grads, void* stream) {
  Layout L;
  int rc = prepare(scenes, n_scenes, views, n_views, params, kept_capacity, entry_capacity, workspace,
                   workspace_bytes, L);
  if (rc) return rc;
  if (!dL_dout || !grads) return fail(RENDER_EINVAL, "null dL_dout or grads");
  for (int v = 0; v < n_views; ++v)
    if (!dL_dout[v]) return fail(RENDER_EINVAL, "view %d: null dL_dout", v);
  for (int s = 0; s < n_scenes; ++s)
    if (scenes[s].V > 0 && (!grads[s].dverts || !grads[s].dsdf || !grads[s].dcolors))
      return fail(RENDER_EINVAL, "scene %d: null gradient buffer", s);
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<DevScene> hs;
  std::vector<DevView> hv;
  std::vector<int32_t> sv;
  fill_desc(scenes, n_scenes, views, n_views, params, L, hs, hv, sv);
  for (int s = 0; s < n_scenes; ++s) {
    hs[s].dverts = grads[s].dverts;
    hs[s].dsdf = grads[s].dsdf;
    hs[s].dcolors = grads[s].dcolors;
  }
  for (int v = 0; v < n_views; ++v) hv[v].dout = dL_dout[v];
  TS_STAGE(RENDER_STAGE_ZERO_GRADS,
           launch_desc_zero_grads(hs.data(), n_scenes, hv.data(), n_views, sv.data(), workspace, L, st),
           "upload descriptors and zero gradients");
  TS_STAGE(RENDER_STAGE_COMPOSITE_BWD,
           params->window > 0 ? launch_composite_backward_win(workspace, L, with_waves(*params), st)
           : multiwave(*params) ? launch_composite_backward_mw(workspace, L, with_waves(*params), st)
                                : launch_composite_backward(workspace, L, *params, st),
           "composite backward");
  if (L.o_pairs != 0) TS_STAGE(RENDER_STAGE_PAIR_GRADS, launch_pair_grads(workspace, L, st), "pair gradients");
  TS_STAGE(RENDER_STAGE_VERTEX_BWD, launch_vertex_backward(workspace, L, *params, st), "vertex backward");
  if (deterministic(L)) TS_STAGE(RENDER_STAGE_VERTEX_BWD, launch_vertex_gather(workspace, L, st), "vertex gather");
  return RENDER_OK;
}

int render_forward_static(const render_scene* scenes, int n_scenes, const render_view* views, int n_views,
                          const render_params* params, int64_t kept_capacity, int64_t entry_capacity,
                          void* header_copy, void* stream) {
  int rc = check_args(scenes, n_scenes, views, n_views, params);
  if (rc) return rc;
  Layout L;
  const char* why = nullptr;
  if (!plan_layout(scenes, n_scenes, views, n_views, params, kept_capacity, entry_capacity, L, &why))
    return fail(RENDER_EINVAL, "%s", why);
  if (L.bytes > RENDER_STATIC_WORKSPACE_BYTES)
    return fail(RENDER_ENOSPC, "the problem needs a %zu-byte workspace; the static workspace holds %zu", L.bytes,
                (size_t)RENDER_STATIC_WORKSPACE_BYTES);
  void* ws = nullptr;
  rc = static_workspace(&ws);
  if (rc) return rc;
  rc = render_forward(scenes, n_scenes, views, n_views, params, kept_capacity, entry_capacity, ws,
                      RENDER_STATIC_WORKSPACE_BYTES, stream);
  if (rc) return rc;
  if (header_copy) {
    hipError_t e = hipMemcpyAsync(header_copy, ws, RENDER_STATUS_BYTES, hipMemcpyDefault,
                                  static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "status header copy");
  }
  return RENDER_OK;
}

int render_decode_status(const void* header_copy, render_status* status) {
  if (!header_copy || !status) return fail(RENDER_EINVAL, "null header copy or status");
  DevHeader h;
  std::memcpy(&h, header_copy, sizeof h);
  status->entries = h.entries_total;
  status->kept = h.kept_total;
  status->records = h.records_total;
  status->overflow = (int32_t)h.overflow;
  status->invalid_index = (int32_t)h.invalid_index;
  status->entry_capacity = h.entry_capacity;
  status->kept_capacity = h.kept_capacity;
  status->entries_needed = (int64_t)h.entries_needed;
  return RENDER_OK;
}

int render_read_status(const void* workspace, render_status* status, void* stream) {
  if (!workspace || !status) return fail(RENDER_EINVAL, "null workspace or status");
  hipStream_t st = static_cast<hipStream_t>(stream);
  DevHeader h;
  hipError_t e = hipMemcpyAsync(&h, workspace, sizeof h, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "read status");
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  status->entries = h.entries_total;
  status->kept = h.kept_total;
  status->records = h.records_total;
  status->overflow = (int32_t)h.overflow;
  status->invalid_index = (int32_t)h.invalid_index;
  status->entry_capacity = h.entry_capacity;
  status->kept_capacity = h.kept_capacity;
  status->entries_needed = (int64_t)h.entries_needed;
  return RENDER_OK;
}

int render_debug_pointers(const render_scene* scenes, int n_scenes, const render_view* views, int n_views,
                          const render_params* params, int64_t kept_capacity, int64_t entry_capacity,
                          const void* workspace, render_debug_view* out) {
  int rc = check_args(scenes, n_scenes, views, n_views, params);
  if (rc) return rc;
  if (!workspace || !out) return fail(RENDER_EINVAL, "null workspace or output");
  Layout L;
  const char* why = nullptr;
  if (!plan_layout(scenes, n_scenes, views, n_views, params, kept_capacity, entry_capacity, L, &why))
    return fail(RENDER_EINVAL, "%s", why);
  void* ws = const_cast<void*>(workspace);
  out->tile_keys = at<const uint32_t>(ws, sorted_tile_keys(L));
  out->entry_record = at<const int32_t>(ws, sorted_entry_records(L));
  out->kept_tet = at<const int32_t>(ws, L.o_kept_tet);
  out->view_rec_base = at<const int32_t>(ws, L.o_view_rec_base);
  out->scene_kept_base = at<const int32_t>(ws, L.o_scene_kept_base);
  out->scene_kept_count = at<const int32_t>(ws, L.o_scene_kept_count);
  out->ranges = at<const uint32_t>(ws, L.o_ranges);
  out->last = L.o_last ? at<const int32_t>(ws, L.o_last) : nullptr;   // null: state not kept
  out->t_last = L.o_tlast ? at<const float>(ws, L.o_tlast) : nullptr;
  out->total_tiles = L.total_tiles;
  out->total_pixels = L.total_pixels;
  return RENDER_OK;
}

int render_profile(int enable) {
  // drop pending events and totals
  for (auto& p : g_prof.pending) {
    g_prof.pool.push_back(p.a);
    g_prof.pool.push_back(p.b);
  }
  g_prof.pending.clear();
  for (int i = 0; i < RENDER_NSTAGES; ++i) { g_prof.ms[i] = 0.0; g_prof.count[i] = 0; }
  g_prof.on = enable != 0;
  return RENDER_OK;
}

int render_profile_read(double* ms, int64_t* counts) {
  if (!ms || !counts) return fail(RENDER_EINVAL, "null output");
  for (auto& p : g_prof.pending) {
    hipError_t e = hipEventSynchronize(p.b);
    if (e != hipSuccess) return hip_fail(e, "event synchronize");
    float t = 0.0f;
    e = hipEventElapsedTime(&t, p.a, p.b);
    if (e != hipSuccess) return hip_fail(e, "event elapsed time");
    g_prof.ms[p.stage] += t;
    g_prof.count[p.stage] += 1;
    g_prof.pool.push_back(p.a);
    g_prof.pool.push_back(p.b);
  }
  g_prof.pending.clear();
  for (int i = 0; i < RENDER_NSTAGES; ++i) { ms[i] = g_prof.ms[i]; counts[i] = g_prof.count[i]; }
  return RENDER_OK;
}

}  // extern "C"
