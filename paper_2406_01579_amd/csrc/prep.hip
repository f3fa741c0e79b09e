// Per-scene and per-view preparation kernels of the gfx950 tetrahedron
// rasterizer: descriptor upload, the alpha_max pre-filter with order-
// preserving compaction and per-tet normal/colour (Sec. 3.2, App. A.3),
// projection and tile counting (Sec. 3.3), the device-wide scan of tile
// counts, tile-duplicated key emission, and tile ranges.
#include <algorithm>
#include <cstring>
#include <vector>

#include "ts_device.h"

namespace ts {

// ---------------------------------------------------------------------------
// descriptor upload through kernel arguments (no host-to-device copies, so
// the whole call sequence can be captured in a graph)
// ---------------------------------------------------------------------------
constexpr int BLOB_WORDS = 960;
struct alignas(16) Blob {
  uint32_t w[BLOB_WORDS];
};

__global__ void k_write_blob(Blob b, uint32_t* dst, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = b.w[i];
}

static hipError_t upload(const void* src, size_t bytes, void* dst, hipStream_t st) {
  const uint32_t* s = static_cast<const uint32_t*>(src);
  uint32_t* d = static_cast<uint32_t*>(dst);
  size_t words = bytes / 4;
  for (size_t o = 0; o < words; o += BLOB_WORDS) {
    Blob b;
    int n = (int)((words - o) < (size_t)BLOB_WORDS ? (words - o) : (size_t)BLOB_WORDS);
    for (int i = 0; i < n; ++i) b.w[i] = s[o + i];
    k_write_blob<<<1, 256, 0, st>>>(b, d + o, n);
  }
  return hipGetLastError();
}

// The header (forward only), scenes, views and scene-view lists occupy
// consecutive workspace regions: they go up as one image (alignment gaps
// zeroed).
static hipError_t desc_image(const DevScene* hs, int ns, const DevView* hv, int nv, const int32_t* scene_views,
                             const Layout& L, bool reset_header, std::vector<uint8_t>& img, size_t& first) {
  static_assert(sizeof(DevHeader) % 4 == 0 && sizeof(DevScene) % 4 == 0 && sizeof(DevView) % 4 == 0,
                "descriptors are whole words");
  first = reset_header ? L.o_hdr : L.o_scene;
  const size_t end = L.o_scene_views + 4 * (size_t)nv;
  if (L.o_hdr > L.o_scene || L.o_scene > L.o_view || L.o_view > L.o_scene_views) return hipErrorInvalidValue;
  img.assign(end - first, 0);
  if (reset_header) {
    // fresh counters for a forward pass (its kernels accumulate into them)
    DevHeader h{};
    h.entry_capacity = L.entry_cap;
    h.kept_capacity = L.kept_cap;
    std::memcpy(img.data() + (L.o_hdr - first), &h, sizeof h);
  }
  std::memcpy(img.data() + (L.o_scene - first), hs, sizeof(DevScene) * ns);
  std::memcpy(img.data() + (L.o_view - first), hv, sizeof(DevView) * nv);
  std::memcpy(img.data() + (L.o_scene_views - first), scene_views, sizeof(int32_t) * nv);
  return hipSuccess;
}


// ---------------------------------------------------------------------------
// a1: pre-filter.  alpha_max = Eq. 1 at (max f, min f) over the 4 vertices;
// keep iff alpha_max >= prefilter_tf.  Kept tets are compacted in ascending
// tet id per scene (block counts; each compaction block sums the counts of
// the blocks before it and rescans its own tets).
// ---------------------------------------------------------------------------
constexpr int PF_THREADS = 256;
constexpr int PF_PER_THREAD = PF_TILE / PF_THREADS;  // 4 consecutive tets per thread

__device__ __forceinline__ int find_scene_by_block(const DevScene* sc, int ns, int b) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (sc[mid].block_base <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Out-of-range vertex indices never reach a memory access: such a tet is
// dropped (and counted in the header when `invalid` is given).
__device__ __forceinline__ bool keep_tet(const DevScene& S, int k, float tf, uint32_t* invalid, int4* vi_out) {
  int4 vi = load_tet(S.tets, k);
  if (vi_out) *vi_out = vi;
  if ((unsigned)vi.x >= (unsigned)S.V || (unsigned)vi.y >= (unsigned)S.V || (unsigned)vi.z >= (unsigned)S.V ||
      (unsigned)vi.w >= (unsigned)S.V) {
    if (invalid) *invalid = 1u;
    return false;
  }
  const auto* sdf = gmem(S.sdf);
  float f0 = sdf[vi.x], f1 = sdf[vi.y], f2 = sdf[vi.z], f3 = sdf[vi.w];
  float fmax = fmaxf(fmaxf(f0, f1), fmaxf(f2, f3));
  float fmin = fminf(fminf(f0, f1), fminf(f2, f3));
  return alpha_eq1(fmax, fmin, S.s) >= tf;
}

__device__ __forceinline__ uint32_t block_exclusive_scan_256(uint32_t v, uint32_t* lds /*[8]*/, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wave] = x;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
  for (int w = 0; w < PF_THREADS / 64; ++w) {
    uint32_t t = lds[w];
    if (w < wave) wbase += t;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return wbase + x - v;
}

// A block's kept count, with PF_INVALID set when one of its tets had a
// vertex index out of range (the totals put it into the header).
constexpr uint32_t PF_INVALID = 1u << 31;

__device__ __forceinline__ void pf_count_body(void* ws, const Layout& L, float tf, const DevScene* sc) {
  uint32_t* cnt = at<uint32_t>(ws, L.o_pf_cnt);
  __shared__ uint32_t lds[8];
  const int b = blockIdx.x;
  const int s = find_scene_by_block(sc, L.ns, b);
  const DevScene S = sc[s];
  const int k0 = (b - S.block_base) * PF_TILE + threadIdx.x * PF_PER_THREAD;
  uint32_t c = 0, nib = 0, bad = 0;
  static_assert(PF_PER_THREAD == 4 && PF_THREADS % 8 == 0, "a thread's four decisions are a nibble of a word");
#pragma unroll
  for (int q = 0; q < PF_PER_THREAD; ++q) {
    int k = k0 + q;
    const bool kp = k < S.K && keep_tet(S, k, tf, &bad, nullptr);
    c += kp ? 1u : 0u;
    nib |= kp ? 1u << q : 0u;
  }
  const int any_bad = __syncthreads_or((int)bad);
  // the decisions, 4 bits per thread: eight threads fill a word
  const int lane = threadIdx.x & 63;
  uint32_t w = nib << (4 * (lane & 7));
  w |= __shfl_xor(w, 1, 64);
  w |= __shfl_xor(w, 2, 64);
  w |= __shfl_xor(w, 4, 64);
  if ((lane & 7) == 0) at<uint32_t>(ws, L.o_pf_keep)[(size_t)b * (PF_TILE / 32) + (threadIdx.x >> 3)] = w;
  uint32_t tot;
  block_exclusive_scan_256(c, lds, &tot);
  if (threadIdx.x == 0) cnt[b] = tot | (any_bad ? PF_INVALID : 0u);
}

__global__ __launch_bounds__(PF_THREADS) void k_pf_count(void* ws, Layout L, float tf) {
  pf_count_body(ws, L, tf, at<const DevScene>(ws, L.o_scene));
}

// The same, with the forward's descriptor image (header, scenes, views and
// scene-view lists) as the argument: block 0 writes it to the workspace for
// the kernels after this one (no block of this one reads the workspace's
// copy or the header), and every block reads its scene from the argument.
__global__ __launch_bounds__(PF_THREADS) void k_pf_count_desc(Blob d, int nwords, void* ws, Layout L, float tf) {
  if (blockIdx.x == 0) {
    uint32_t* dst = at<uint32_t>(ws, L.o_hdr);
    for (int i = threadIdx.x; i < nwords; i += PF_THREADS) dst[i] = d.w[i];
  }
  pf_count_body(ws, L, tf, reinterpret_cast<const DevScene*>(d.w + (L.o_scene - L.o_hdr) / 4));
}

// Per-scene kept ranges, per-view record bases, totals and capacity checks
// from the pre-filter blocks' counts (thread t sums a contiguous range of
// them; a scan of the range sums gives each range's start, and the scene
// whose first block lies in a range takes its base from there).  One block.
__device__ void prefilter_totals(void* ws, const Layout& L, uint32_t* lds /*[8]*/) {
  DevHeader* hdr = at<DevHeader>(ws, L.o_hdr);
  const DevScene* sc = at<const DevScene>(ws, L.o_scene);
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const uint32_t* cnt = at<const uint32_t>(ws, L.o_pf_cnt);
  int32_t* kbase = at<int32_t>(ws, L.o_scene_kept_base);
  int32_t* kcount = at<int32_t>(ws, L.o_scene_kept_count);
  int32_t* rbase = at<int32_t>(ws, L.o_view_rec_base);
  const int n = (int)L.pf_blocks;
  const int per = (n + PF_THREADS - 1) / PF_THREADS;
  const int j0 = min(n, (int)threadIdx.x * per), j1 = min(n, j0 + per);
  uint32_t sum = 0, bad = 0;
  for (int j = j0; j < j1; ++j) {
    sum += cnt[j] & ~PF_INVALID;
    bad |= cnt[j] & PF_INVALID;
  }
  const int any_bad = __syncthreads_or((int)(bad != 0u));
  uint32_t total;
  const uint32_t start = block_exclusive_scan_256(sum, lds, &total);
  const uint32_t cap = (uint32_t)L.kept_cap;
  // scene s starts at block block_base (a scene with no blocks shares the
  // next one's; past the last block: the total)
  for (int s = 0; s < L.ns; ++s) {
    const int bb = sc[s].block_base;
    const bool mine = (bb >= j0 && bb < j1) || (bb >= n && threadIdx.x == PF_THREADS - 1);
    if (mine) {
      uint32_t x = start;
      for (int j = j0; j < min(bb, j1); ++j) x += cnt[j] & ~PF_INVALID;
      kbase[s] = (int32_t)min(x, cap);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    hdr->kept_total = total;
    uint32_t ovf = total > cap ? 1u : 0u;
    for (int s = 0; s < L.ns; ++s) {
      const uint32_t b0 = (uint32_t)kbase[s];
      const uint32_t b1 = s + 1 < L.ns ? (uint32_t)kbase[s + 1] : min(total, cap);
      kcount[s] = (int32_t)(b1 - b0);
    }
    uint64_t r = 0;
    for (int v = 0; v < L.nv; ++v) {
      rbase[v] = (int32_t)r;
      r += (uint64_t)kcount[vw[v].scene];
    }
    if (r > (uint64_t)L.rec_cap) { ovf |= 1u; r = (uint64_t)L.rec_cap; }
    hdr->records_total = (uint32_t)r;
    hdr->overflow = ovf;
    hdr->entries_total = 0;
    if (any_bad) hdr->invalid_index = 1u;
  }
}

// rescan and write the kept tets' records: vertices, SDF, normal (App. A.3 via
// the equivalent 3x3 edge system), mean colour.  Each block finds the kept
// tets before it by summing the counts of the blocks before it (all threads
// at once); block 0 also writes the per-scene and per-view totals.
__global__ __launch_bounds__(PF_THREADS) void k_pf_scatter(void* ws, Layout L, float tf) {
  const DevScene* sc = at<const DevScene>(ws, L.o_scene);
  const uint32_t* cnt = at<const uint32_t>(ws, L.o_pf_cnt);
  TetRec* trec = at<TetRec>(ws, L.o_trec);
  int32_t* kept_tet = at<int32_t>(ws, L.o_kept_tet);
  __shared__ uint32_t lds[8];
  const int b = blockIdx.x;
  if (b == 0) prefilter_totals(ws, L, lds);
  if (b >= (int)L.pf_blocks) return;   // (no blocks of tets: block 0 only writes the totals)
  uint32_t part = 0;
  for (int j = threadIdx.x; j < b; j += PF_THREADS) part += cnt[j] & ~PF_INVALID;
  uint32_t before;
  block_exclusive_scan_256(part, lds, &before);
  const int s = find_scene_by_block(sc, L.ns, b);
  const DevScene S = sc[s];
  const int k0 = (b - S.block_base) * PF_TILE + threadIdx.x * PF_PER_THREAD;
  // the count kernel's decisions (this thread's nibble); only kept tets are read
  const uint32_t nib =
      (at<const uint32_t>(ws, L.o_pf_keep)[(size_t)b * (PF_TILE / 32) + (threadIdx.x >> 3)] >> (4 * (threadIdx.x & 7))) & 15u;
  bool kp[PF_PER_THREAD];
  int4 vi[PF_PER_THREAD];
  uint32_t c = 0;
#pragma unroll
  for (int q = 0; q < PF_PER_THREAD; ++q) {
    kp[q] = (nib >> q) & 1u;
    vi[q] = make_int4(0, 0, 0, 0);
    if (kp[q]) vi[q] = load_tet(S.tets, k0 + q);
    c += kp[q] ? 1u : 0u;
  }
  uint32_t tot;
  uint32_t slot = before + block_exclusive_scan_256(c, lds, &tot);
#pragma unroll
  for (int q = 0; q < PF_PER_THREAD; ++q) {
    if (!kp[q]) continue;
    const uint32_t my = slot++;
    if (my >= (uint32_t)L.kept_cap) continue;
    const int idx[4] = {vi[q].x, vi[q].y, vi[q].z, vi[q].w};
    TetRec r;
    for (int a = 0; a < 4; ++a) {
      r.x[a][0] = gmem(S.verts)[3 * (size_t)idx[a] + 0];
      r.x[a][1] = gmem(S.verts)[3 * (size_t)idx[a] + 1];
      r.x[a][2] = gmem(S.verts)[3 * (size_t)idx[a] + 2];
      r.f[a] = gmem(S.sdf)[idx[a]];
    }
    // g = E^-1 (f_k - f_0), E rows e_k = x_k - x_0 (k = 1..3)
    float e[3][3], df[3];
    for (int a = 0; a < 3; ++a) {
      for (int j = 0; j < 3; ++j) e[a][j] = r.x[a + 1][j] - r.x[0][j];
      df[a] = r.f[a + 1] - r.f[0];
    }
    float c23[3] = {e[1][1] * e[2][2] - e[1][2] * e[2][1], e[1][2] * e[2][0] - e[1][0] * e[2][2],
                    e[1][0] * e[2][1] - e[1][1] * e[2][0]};
    float c31[3] = {e[2][1] * e[0][2] - e[2][2] * e[0][1], e[2][2] * e[0][0] - e[2][0] * e[0][2],
                    e[2][0] * e[0][1] - e[2][1] * e[0][0]};
    float c12[3] = {e[0][1] * e[1][2] - e[0][2] * e[1][1], e[0][2] * e[1][0] - e[0][0] * e[1][2],
                    e[0][0] * e[1][1] - e[0][1] * e[1][0]};
    float det = e[0][0] * c23[0] + e[0][1] * c23[1] + e[0][2] * c23[2];
    float g[3];
    for (int j = 0; j < 3; ++j) g[j] = (det != 0.0f) ? (c23[j] * df[0] + c31[j] * df[1] + c12[j] * df[2]) / det : 0.0f;
    float gn = sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    for (int j = 0; j < 3; ++j) r.n[j] = (gn > 0.0f) ? g[j] / gn : 0.0f;
    for (int j = 0; j < 3; ++j) {
      const auto* C = gmem(S.colors);
      r.c[j] = ((C[3 * (size_t)idx[0] + j] + C[3 * (size_t)idx[1] + j]) +
                (C[3 * (size_t)idx[2] + j] + C[3 * (size_t)idx[3] + j])) * 0.25f;
    }
    r.tet = k0 + q;
    r.scene = s;
    trec[my] = r;
    kept_tet[my] = k0 + q;
  }
}

hipError_t launch_prefilter(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  if (L.pf_blocks > 0) k_pf_count<<<(unsigned)L.pf_blocks, PF_THREADS, 0, st>>>(ws, L, p.prefilter_tf);
  k_pf_scatter<<<(unsigned)std::max<int64_t>(L.pf_blocks, 1), PF_THREADS, 0, st>>>(ws, L, p.prefilter_tf);
  return hipGetLastError();
}

// The forward's descriptor upload and pre-filter: when the descriptor image
// fits one kernel argument, the pre-filter's counting launch carries it (one
// launch fewer); otherwise it goes up first.
hipError_t launch_desc_prefilter(const DevScene* hs, int ns, const DevView* hv, int nv, const int32_t* scene_views,
                                 void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  std::vector<uint8_t> img;
  size_t first;
  hipError_t e = desc_image(hs, ns, hv, nv, scene_views, L, true, img, first);
  if (e != hipSuccess) return e;
  const size_t words = img.size() / 4;
  if (words > (size_t)BLOB_WORDS || L.pf_blocks == 0 || first != L.o_hdr) {
    e = upload(img.data(), img.size(), at<void>(ws, first), st);
    if (e != hipSuccess) return e;
    return launch_prefilter(ws, L, p, st);
  }
  Blob b;
  std::memcpy(b.w, img.data(), img.size());
  k_pf_count_desc<<<(unsigned)L.pf_blocks, PF_THREADS, 0, st>>>(b, (int)words, ws, L, p.prefilter_tf);
  k_pf_scatter<<<(unsigned)L.pf_blocks, PF_THREADS, 0, st>>>(ws, L, p.prefilter_tf);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a2: per (view, kept tet) record: camera transform, near-plane cull,
// projection, pixel rectangle, tile count, depth key (float32, fixed op
// sequence), 2D face determinants, shading features.
// ---------------------------------------------------------------------------
// One block projects 256 consecutive kept tets of one view per step.  The
// 96-byte tet records come in and the 128-byte view records go out through
// LDS, so that every HBM access of the records is contiguous across the
// block.  A record takes 9 x 16 bytes in LDS: when each thread reads or
// writes its own record 16 bytes at a time, sixteen neighbouring threads
// touch 64 distinct banks.
constexpr int PROJ_STRIDE = 9;   // uint4 per record in LDS
static_assert(sizeof(TetRec) == 6 * 16 && sizeof(ViewRec) == 8 * 16, "record sizes in 16-byte units");

__global__ __launch_bounds__(256) void k_project(void* ws, Layout L, int tw_log2, int th_log2) {
  const DevHeader* hdr = at<const DevHeader>(ws, L.o_hdr);
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const int32_t* kbase = at<const int32_t>(ws, L.o_scene_kept_base);
  const int32_t* kcount = at<const int32_t>(ws, L.o_scene_kept_count);
  const int32_t* rbase = at<const int32_t>(ws, L.o_view_rec_base);
  const uint4* trec4 = at<const uint4>(ws, L.o_trec);
  uint4* vrec4 = at<uint4>(ws, L.o_vrec);
  uint32_t* count1 = at<uint32_t>(ws, L.o_count1);
  uint32_t* key1 = at<uint32_t>(ws, L.o_key1a);
  uint4* rbox = at<uint4>(ws, L.o_rbox);
  __shared__ uint4 sbuf[256 * PROJ_STRIDE];
  __shared__ uint32_t svalid[256];
  {
    // the per-tile entry counters and tile-block sums, the dispatch-order
    // histograms and cursors (forward and backward) start cleared for the
    // binning kernels that follow
    const uint64_t nb = (uint64_t)gridDim.x * gridDim.y, b = (uint64_t)blockIdx.y * gridDim.x + blockIdx.x;
    uint32_t* tcnt = at<uint32_t>(ws, L.o_tile_cnt);
    const uint64_t ncnt = (L.o_tile_bsum - L.o_tile_cnt) / 4 + (uint64_t)L.tile_blocks;
    for (uint64_t i = b * 256 + threadIdx.x; i < ncnt; i += nb * 256) tcnt[i] = 0u;
    if (b == 0) {
      uint32_t* th = at<uint32_t>(ws, L.o_tile_hist);
      for (int i = threadIdx.x; i < 2 * TILE_BUCKETS; i += 256) th[i] = 0u;
      uint32_t* bh = at<uint32_t>(ws, L.o_bwd_hist);
      for (int i = threadIdx.x; i < BWD_HIST_WORDS; i += 256) bh[i] = 0u;
    }
  }
  const int v = blockIdx.y;
  const DevView V = vw[v];
  const int n = kcount[V.scene];
  const int r0 = rbase[v];
  const int kb = kbase[V.scene];
  if ((uint64_t)r0 + (uint64_t)n > (uint64_t)hdr->records_total) return;  // capacity overflow guard
  const int t = threadIdx.x;
  for (int k0 = blockIdx.x * 256; k0 < n; k0 += gridDim.x * 256) {
    const int nloc = min(256, n - k0);
    // tet records in, contiguous
    const uint4* src = trec4 + (size_t)(kb + k0) * 6;
    for (int q = t; q < nloc * 6; q += 256) sbuf[(q / 6) * PROJ_STRIDE + (q % 6)] = src[q];
    __syncthreads();
    TetRec T;
    if (t < nloc) {
#pragma unroll
      for (int q = 0; q < 6; ++q) reinterpret_cast<uint4*>(&T)[q] = sbuf[t * PROJ_STRIDE + q];
    }
    __syncthreads();
    uint32_t valid = 0;
    if (t < nloc) {
      const int k = k0 + t;
      const int r = r0 + k;
      float X[4], Y[4], Z[4], px[4], py[4];
      bool culled = false;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const float x = T.x[a][0], y = T.x[a][1], z = T.x[a][2];
        X[a] = fmaf(V.R[0], x, fmaf(V.R[1], y, fmaf(V.R[2], z, V.t[0])));
        Y[a] = fmaf(V.R[3], x, fmaf(V.R[4], y, fmaf(V.R[5], z, V.t[1])));
        Z[a] = fmaf(V.R[6], x, fmaf(V.R[7], y, fmaf(V.R[8], z, V.t[2])));
        culled |= (Z[a] < V.znear);
      }
      uint32_t cnt = 0, key = 0xffffffffu;
      if (!culled) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          px[a] = fmaf(V.fx, X[a] / Z[a], V.cx);
          py[a] = fmaf(V.fy, Y[a] / Z[a], V.cy);
        }
        const float zt = ((Z[0] + Z[1]) + (Z[2] + Z[3])) * 0.25f;
        const float xmin = fminf(fminf(px[0], px[1]), fminf(px[2], px[3]));
        const float xmax = fmaxf(fmaxf(px[0], px[1]), fmaxf(px[2], px[3]));
        const float ymin = fminf(fminf(py[0], py[1]), fminf(py[2], py[3]));
        const float ymax = fmaxf(fmaxf(py[0], py[1]), fmaxf(py[2], py[3]));
        const int i0 = (int)fminf(fmaxf(ceilf(xmin - 0.5f), 0.0f), (float)V.W);
        const int i1 = (int)fmaxf(fminf(floorf(xmax - 0.5f), (float)(V.W - 1)), -1.0f);
        const int j0 = (int)fminf(fmaxf(ceilf(ymin - 0.5f), 0.0f), (float)V.H);
        const int j1 = (int)fmaxf(fminf(floorf(ymax - 0.5f), (float)(V.H - 1)), -1.0f);
        if (i0 <= i1 && j0 <= j1) {
          const int tx0 = i0 >> tw_log2, tx1 = i1 >> tw_log2, ty0 = j0 >> th_log2, ty1 = j1 >> th_log2;
          cnt = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
          key = __float_as_uint(zt);
          ViewRec R;
          for (int a = 0; a < 4; ++a) {
            R.px[a] = px[a];
            R.py[a] = py[a];
            R.iz[a] = 1.0f / Z[a];
            R.f[a] = T.f[a];
          }
          for (int F = 0; F < 4; ++F) {
            const int A = face_vertex(F, 0), B = face_vertex(F, 1), C = face_vertex(F, 2);
            const float D = (px[B] - px[A]) * (py[C] - py[A]) - (py[B] - py[A]) * (px[C] - px[A]);
            R.rD[F] = D != 0.0f ? rcp(D) : 0.0f;   // once per record, not per pixel
          }
          R.c[0] = T.c[0]; R.c[1] = T.c[1]; R.c[2] = T.c[2];
          R.zt = zt;
          R.n[0] = T.n[0]; R.n[1] = T.n[1]; R.n[2] = T.n[2];
          R.rx = (uint32_t)i0 | ((uint32_t)i1 << 16);
          R.ry = (uint32_t)j0 | ((uint32_t)j1 << 16);
          R.kept = kb + k;
          R.view = v;
          R.entry0 = 0;
#pragma unroll
          for (int q = 0; q < 8; ++q) sbuf[t * PROJ_STRIDE + q] = reinterpret_cast<const uint4*>(&R)[q];
          valid = 1;
          // the fields the emit and vertex-backward kernels need, compact
          rbox[r] = make_uint4(R.rx, R.ry, (uint32_t)v, 0u);
        }
      }
      count1[r] = cnt;
      key1[r] = key;
    }
    svalid[t] = valid;
    __syncthreads();
    // view records out, contiguous (records that cover no pixel are skipped)
    uint4* dst = vrec4 + (size_t)(r0 + k0) * 8;
    for (int q = t; q < nloc * 8; q += 256)
      if (svalid[q >> 3]) dst[q] = sbuf[(q >> 3) * PROJ_STRIDE + (q & 7)];
    __syncthreads();
  }
}

hipError_t launch_project(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  int twl = __builtin_ctz((unsigned)p.tile_w), thl = __builtin_ctz((unsigned)p.tile_h);
  dim3 grid(512, (unsigned)L.nv);
  k_project<<<grid, 256, 0, st>>>(ws, L, twl, thl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a3-a5a: binning.  Records are taken in record order (per view ascending
// kept slot, i.e. ascending tet id), SCAN_TILE at a time.  Two counts come
// out of one pass over every record's (record, tile) entries: the entries
// per record (their exclusive scan is each record's first entry: the slot of
// its per-(record, tile) gradient) and the entries per tile.  The tiles'
// exclusive scan is where each tile's list starts; the emit kernel then
// places every entry in its tile's list through a per-tile cursor.  The
// order inside a list is left to the atomics: the per-tile depth sort that
// follows imposes the final order.  Entries of one wave that share a tile
// (neighbouring records touch neighbouring tiles) are combined first, so
// each wave issues one global atomic per distinct tile, all at once.
// ---------------------------------------------------------------------------
// The wave's lanes with `active` set, grouped by tile: returns the lane's
// place in its group; *lead is the group's first lane and *cnt (in that lane
// only, else 0) the group's size.  Every lane of the wave must call it.
__device__ __forceinline__ uint32_t wave_group_by_tile(uint32_t tile, bool active, int* lead, uint32_t* cnt) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt = (1ull << lane) - 1ull;
  uint64_t pending = __ballot(active);
  uint32_t off = 0;
  *lead = lane;
  *cnt = 0u;
  while (pending != 0ull) {
    const int l0 = __ffsll((unsigned long long)pending) - 1;
    const uint32_t t0 = (uint32_t)__shfl((int)tile, l0, 64);
    const uint64_t m = __ballot(active && tile == t0) & pending;
    if ((m >> lane) & 1ull) {
      *lead = l0;
      off = (uint32_t)__popcll(m & lt);
    }
    if (lane == l0) *cnt = (uint32_t)__popcll(m);
    pending &= ~m;
  }
  return off;
}

// Round k of a block's entries: entry e = e0 + 256 k + threadIdx.x for every
// thread (active if e < ne) -- its record (binary search over the block's
// record offsets loff) and tile.
__device__ __forceinline__ void block_entry(const uint32_t* loff, uint32_t m, uint32_t q0, uint32_t e,
                                            const uint4* __restrict__ rbox, const DevView* __restrict__ vw,
                                            int tw_log2, int th_log2, uint32_t& r, uint32_t& tile) {
  int k = 0;
#pragma unroll
  for (int step = SCAN_TILE / 2; step > 0; step >>= 1) {
    const int k2 = k + step;
    k = (k2 < (int)m && loff[k2] <= e) ? k2 : k;
  }
  r = q0 + (uint32_t)k;
  const uint4 bx = rbox[r];   // rectangle and view
  const int i0 = (int)(bx.x & 0xffffu), i1 = (int)(bx.x >> 16), j0 = (int)(bx.y & 0xffffu);
  const DevView& V = vw[bx.z];
  const int tx0 = i0 >> tw_log2, tx1 = i1 >> tw_log2, ty0 = j0 >> th_log2;
  const int nx = tx1 - tx0 + 1;
  const uint32_t j = e - loff[k];
  const int ty = ty0 + (int)(j / (uint32_t)nx), tx = tx0 + (int)(j % (uint32_t)nx);
  tile = (uint32_t)(V.tile_base + ty * V.tiles_x + tx);
}

// records per thread of a 256-thread scan block (one, or none past the block's
// records, when a block holds fewer than 256)
constexpr int SCAN_PER = SCAN_TILE >= 256 ? SCAN_TILE / 256 : 1;
static_assert(SCAN_TILE % 256 == 0 || 256 % SCAN_TILE == 0, "scan blocks of whole thread rounds");

// The block's records: counts, their exclusive scan (loff) and the total.
__device__ __forceinline__ uint32_t block_record_offsets(const uint32_t* __restrict__ count1, uint32_t q0, uint32_t m,
                                                         uint32_t* loff, uint32_t* lds, uint32_t (&c)[SCAN_PER]) {
  constexpr int PER = SCAN_PER;
  const int t = threadIdx.x;
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const uint32_t k = (uint32_t)(t * PER + i);
    c[i] = k < m ? count1[q0 + k] : 0u;
    sum += c[i];
  }
  uint32_t tot;
  uint32_t run = block_exclusive_scan_256(sum, lds, &tot);
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    if (t * PER + i < SCAN_TILE) loff[t * PER + i] = run;
    run += c[i];
  }
  __syncthreads();
  return tot;
}

// per SCAN_TILE records: the block's entry total, and its entries counted per
// tile
__global__ __launch_bounds__(256) void k_scan_reduce(void* ws, Layout L, int tw_log2, int th_log2) {
  const DevHeader* hdr = at<const DevHeader>(ws, L.o_hdr);
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const uint32_t* count1 = at<const uint32_t>(ws, L.o_count1);
  const uint4* rbox = at<const uint4>(ws, L.o_rbox);
  uint32_t* part = at<uint32_t>(ws, L.o_scan_part);
  uint32_t* tcnt = at<uint32_t>(ws, L.o_tile_cnt);
  __shared__ uint32_t loff[SCAN_TILE];
  __shared__ uint32_t lds[8];
  const uint32_t n = hdr->records_total;
  const uint32_t q0 = blockIdx.x * SCAN_TILE;
  if (q0 >= n) return;
  const uint32_t m = min((uint32_t)SCAN_TILE, n - q0);
  uint32_t c[SCAN_PER];
  const uint32_t tot = block_record_offsets(count1, q0, m, loff, lds, c);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
  for (uint32_t e0 = 0; e0 < tot; e0 += 256u) {
    const uint32_t e = e0 + threadIdx.x;
    const bool active = e < tot;
    uint32_t r = 0, tile = 0;
    if (active) block_entry(loff, m, q0, e, rbox, vw, tw_log2, th_log2, r, tile);
    int lead;
    uint32_t cnt;
    wave_group_by_tile(tile, active, &lead, &cnt);
    if (cnt) atomicAdd(&tcnt[tile], cnt);
  }
}

// per 1024 tiles: the entry total of the block's tiles (for the spine)
__global__ __launch_bounds__(1024) void k_tile_block_sum(void* ws, Layout L) {
  const uint32_t* tcnt = at<const uint32_t>(ws, L.o_tile_cnt);
  uint32_t* tbsum = at<uint32_t>(ws, L.o_tile_bsum);
  __shared__ uint32_t lds[16];
  const uint32_t t = blockIdx.x * 1024u + threadIdx.x;
  uint32_t x = t < (uint32_t)L.total_tiles ? tcnt[t] : 0u;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t sum = 0;
    for (int w = 0; w < 16; ++w) sum += lds[w];
    tbsum[blockIdx.x] = sum;
  }
}

// one block: exclusive scans of the record-block entry totals (the blocks'
// first entries) and of the tile-block entry totals (the tile blocks' first
// list places), the entry total and the capacity check
__device__ __forceinline__ void spine_scan_1024(uint32_t* part, int nb, unsigned long long* lp,
                                                unsigned long long* total) {
  const int per = (nb + 1023) / 1024;
  const int t = threadIdx.x;
  unsigned long long sum = 0;
  for (int i = t * per; i < min(nb, (t + 1) * per); ++i) sum += part[i];
  lp[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    unsigned long long v = (t >= o) ? lp[t - o] : 0ull;
    __syncthreads();
    lp[t] += v;
    __syncthreads();
  }
  unsigned long long run = lp[t] - sum;
  for (int i = t * per; i < min(nb, (t + 1) * per); ++i) {
    uint32_t c = part[i];
    part[i] = (uint32_t)run;
    run += c;
  }
  *total = lp[1023];
  __syncthreads();
}

__global__ __launch_bounds__(1024) void k_scan_spine(void* ws, Layout L) {
  DevHeader* hdr = at<DevHeader>(ws, L.o_hdr);
  __shared__ unsigned long long lp[1024];
  const uint32_t n = hdr->records_total;
  unsigned long long total, ttotal;
  spine_scan_1024(at<uint32_t>(ws, L.o_scan_part), (int)((n + SCAN_TILE - 1) / SCAN_TILE), lp, &total);
  spine_scan_1024(at<uint32_t>(ws, L.o_tile_bsum), (int)L.tile_blocks, lp, &ttotal);
  if (threadIdx.x == 0) {
    uint32_t E = total > (unsigned long long)L.entry_cap ? (uint32_t)L.entry_cap : (uint32_t)total;
    if (total > (unsigned long long)L.entry_cap) hdr->overflow |= 2u;
    hdr->entries_total = E;
    hdr->entries_needed = total;
  }
}

// per 1024 tiles: each tile's list [start, end) (clamped to the entry
// capacity; (0, 0) when empty), its cursor (the list start, for the emit
// kernel), and the dispatch-order histogram of the list lengths
__device__ __forceinline__ uint32_t block_exclusive_scan_1024(uint32_t v, uint32_t* lds /*[16]*/) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wave] = x;
  __syncthreads();
  uint32_t wbase = 0;
  for (int w = 0; w < wave; ++w) wbase += lds[w];
  __syncthreads();
  return wbase + x - v;
}

__global__ __launch_bounds__(1024) void k_tile_lists(void* ws, Layout L) {
  uint32_t* tcnt = at<uint32_t>(ws, L.o_tile_cnt);
  const uint32_t* tbpre = at<const uint32_t>(ws, L.o_tile_bsum);
  uint32_t* ranges = at<uint32_t>(ws, L.o_ranges);
  uint32_t* hist = at<uint32_t>(ws, L.o_tile_hist);
  __shared__ uint32_t lds[16];
  __shared__ uint32_t hb[TILE_BUCKETS];
  if (threadIdx.x < TILE_BUCKETS) hb[threadIdx.x] = 0u;
  const uint64_t cap = (uint64_t)L.entry_cap;
  const uint32_t t = blockIdx.x * 1024u + threadIdx.x;
  const bool in = t < (uint32_t)L.total_tiles;
  const uint32_t c = in ? tcnt[t] : 0u;
  const uint64_t start = (uint64_t)tbpre[blockIdx.x] + block_exclusive_scan_1024(c, lds);
  if (in) {
    uint32_t s0 = (uint32_t)min(start, cap), s1 = (uint32_t)min(start + c, cap);
    if (s0 == s1) s0 = s1 = 0u;   // an empty list is (0, 0)
    ranges[2 * (size_t)t] = s0;
    ranges[2 * (size_t)t + 1] = s1;
    tcnt[t] = (uint32_t)min(start, (uint64_t)0xffffffffu);   // the emit kernel's cursor
    atomicAdd(&hb[len_bucket(s1 - s0)], 1u);
  }
  __syncthreads();
  if (threadIdx.x < TILE_BUCKETS && hb[threadIdx.x]) atomicAdd(&hist[threadIdx.x], hb[threadIdx.x]);
}

hipError_t launch_count_scan(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  int twl = __builtin_ctz((unsigned)p.tile_w), thl = __builtin_ctz((unsigned)p.tile_h);
  unsigned nb = (unsigned)L.scan_blocks_rec;
  // per-record offsets are finished inside the emit kernel
  k_scan_reduce<<<nb, 256, 0, st>>>(ws, L, twl, thl);
  if (L.total_tiles > 0) k_tile_block_sum<<<(unsigned)L.tile_blocks, 1024, 0, st>>>(ws, L);
  k_scan_spine<<<1, 1024, 0, st>>>(ws, L);
  if (L.total_tiles > 0) k_tile_lists<<<(unsigned)L.tile_blocks, 1024, 0, st>>>(ws, L);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a4: duplicate each record once per overlapped tile into the tile's list:
// per SCAN_TILE records, each record's first entry into its box, then the
// block's entries (records) placed through the per-tile cursors; places past
// the entry capacity are dropped (the overflow is flagged).  The lists' tile
// keys are written by the depth sort, contiguously per tile, not here, where
// every 4-byte place is a scattered write.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_emit(void* ws, Layout L, int tw_log2, int th_log2) {
  const DevHeader* hdr = at<const DevHeader>(ws, L.o_hdr);
  const DevView* vw = at<const DevView>(ws, L.o_view);
  const uint32_t* count1 = at<const uint32_t>(ws, L.o_count1);
  const uint4* rbox = at<const uint4>(ws, L.o_rbox);
  uint32_t* rfirst = at<uint32_t>(ws, L.o_rfirst);
  uint32_t* cursor = at<uint32_t>(ws, L.o_tile_cnt);
  uint32_t* val2 = at<uint32_t>(ws, sorted_entry_records(L));
  constexpr int PER = SCAN_PER;
  __shared__ uint32_t loff[SCAN_TILE];
  __shared__ uint32_t lds[8];
  const uint32_t* part = at<const uint32_t>(ws, L.o_scan_part);
  const uint32_t n = hdr->records_total;
  const uint64_t cap = (uint64_t)L.entry_cap;
  const uint32_t nblk = (n + SCAN_TILE - 1) / SCAN_TILE;
  const int t = threadIdx.x;
  for (uint32_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const uint32_t q0 = blk * SCAN_TILE;
    const uint32_t m = min((uint32_t)SCAN_TILE, n - q0);
    uint32_t c[PER];
    const uint32_t tot = block_record_offsets(count1, q0, m, loff, lds, c);
    const uint32_t base = part[blk];
#pragma unroll
    for (int i = 0; i < PER; ++i)
      if (c[i] != 0u) rfirst[q0 + (uint32_t)(t * PER + i)] = base + loff[t * PER + i];
    for (uint32_t e0 = 0; e0 < tot; e0 += 256u) {
      const uint32_t e = e0 + (uint32_t)t;
      const bool active = e < tot;
      uint32_t r = 0, tile = 0;
      if (active) block_entry(loff, m, q0, e, rbox, vw, tw_log2, th_log2, r, tile);
      int lead;
      uint32_t cnt;
      const uint32_t off = wave_group_by_tile(tile, active, &lead, &cnt);
      uint32_t gb = cnt ? atomicAdd(&cursor[tile], cnt) : 0u;
      gb = (uint32_t)__shfl((int)gb, lead, 64);
      const uint64_t pos = (uint64_t)gb + off;
      if (active && pos < cap) val2[pos] = r;
    }
    __syncthreads();
  }
}

hipError_t launch_emit(void* ws, const Layout& L, const render_params& p, hipStream_t st) {
  int twl = __builtin_ctz((unsigned)p.tile_w), thl = __builtin_ctz((unsigned)p.tile_h);
  // one block per SCAN_TILE records, up to 4096 (then several each)
  const int64_t nb = L.scan_blocks_rec;
  k_emit<<<(unsigned)(nb < 4096 ? (nb > 0 ? nb : 1) : 4096), 256, 0, st>>>(ws, L, twl, thl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dispatch order of the compositing workgroups: tiles with the longest lists
// first (bucketed by the list length: four buckets per power of two), so the
// longest sequential walks start in the first scheduling round.  The forward
// orders by list length; the backward by the length the forward actually
// walked before every pixel of the tile stopped.  The order inside a bucket is
// whatever the atomics give; results do not depend on it.
// ---------------------------------------------------------------------------

// Every scatter block: first[b] = the number of tiles in buckets above b
// (longest first), from the complete histogram; the block's tiles of bucket
// b then take consecutive places from first[b] + an atomic cursor.
static_assert(TILE_BUCKETS <= 256, "one thread per bucket");
// tiles per thread of the scatter kernels (4 -- a quarter of the blocks and
// of their per-bucket cursor atomics -- was 5 us slower per step: the
// per-block work grew more than the atomics shrank)
constexpr int SC_PER = 1;
__device__ __forceinline__ void bucket_first(const uint32_t* hist, uint32_t* first, uint32_t* lds /*[8]*/) {
  const int t = threadIdx.x;
  const uint32_t v = t < TILE_BUCKETS ? hist[TILE_BUCKETS - 1 - t] : 0u;
  uint32_t tot;
  const uint32_t ex = block_exclusive_scan_256(v, lds, &tot);
  if (t < TILE_BUCKETS) first[TILE_BUCKETS - 1 - t] = ex;
}

__global__ __launch_bounds__(256) void k_tile_scatter(void* ws, Layout L) {
  const uint32_t* ranges = at<const uint32_t>(ws, L.o_ranges);
  const uint32_t* hist = at<const uint32_t>(ws, L.o_tile_hist);
  uint32_t* cursor = at<uint32_t>(ws, L.o_tile_hist) + TILE_BUCKETS;
  TileSlot* order = at<TileSlot>(ws, L.o_tile_order);
  const DevView* vw = at<const DevView>(ws, L.o_view);
  __shared__ uint32_t cnt[TILE_BUCKETS], base[TILE_BUCKETS], first[TILE_BUCKETS], lds[8];
  if (threadIdx.x < TILE_BUCKETS) cnt[threadIdx.x] = 0;
  bucket_first(hist, first, lds);
  __syncthreads();
  int b[SC_PER];
  uint32_t rank[SC_PER];
#pragma unroll
  for (int i = 0; i < SC_PER; ++i) {
    const uint32_t t = (blockIdx.x * SC_PER + (uint32_t)i) * 256u + threadIdx.x;
    b[i] = 0;
    rank[i] = 0u;
    if (t < (uint32_t)L.total_tiles) {
      b[i] = len_bucket(ranges[2 * t + 1] - ranges[2 * t]);
      rank[i] = atomicAdd(&cnt[b[i]], 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x < TILE_BUCKETS && cnt[threadIdx.x])
    base[threadIdx.x] = first[threadIdx.x] + atomicAdd(&cursor[threadIdx.x], cnt[threadIdx.x]);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < SC_PER; ++i) {
    const uint32_t t = (blockIdx.x * SC_PER + (uint32_t)i) * 256u + threadIdx.x;
    if (t < (uint32_t)L.total_tiles) {
      TileSlot sl;
      sl.tile = t;
      sl.view = (uint32_t)find_view_by_tile(vw, L.nv, (int)t);
      sl.start = ranges[2 * t];
      sl.end = ranges[2 * t + 1];
      order[base[b[i]] + rank[i]] = sl;
    }
  }
}

hipError_t launch_tile_order(void* ws, const Layout& L, hipStream_t st) {
  if (L.total_tiles == 0) return hipSuccess;
  const unsigned nb = (unsigned)((L.total_tiles + 256 * SC_PER - 1) / (256 * SC_PER));
  // the length histogram was counted by k_tile_lists
  k_tile_scatter<<<nb, 256, 0, st>>>(ws, L);
  return hipGetLastError();
}

// backward order: forward slots re-bucketed by the walked length pend - start
// (the forward compositing kernel counted every slot with pend > start; the
// tiles with nothing walked form bucket 0, placed last, whose own count the
// offsets never need).  On the multi-wave 8x8 path every slot also gets the
// base of its blended pairs in the backward's pair buffer, by the same
// bucket scheme (the forward counted them per slot and per bucket), and the
// total is checked against the entry capacity, which bounds the pairs.
__global__ __launch_bounds__(256) void k_bwd_scatter(void* ws, Layout L) {
  const TileSlot* slots = at<const TileSlot>(ws, L.o_tile_order);
  const uint32_t* pend = at<const uint32_t>(ws, L.o_tile_pend);
  const uint32_t* hist = at<const uint32_t>(ws, L.o_bwd_hist);
  uint32_t* cursor = at<uint32_t>(ws, L.o_bwd_hist) + TILE_BUCKETS;
  TileSlot* bslots = at<TileSlot>(ws, L.o_bwd_order);
  uint32_t* bpend = at<uint32_t>(ws, L.o_bwd_pend);
  const bool pairs = L.o_pairs != 0;
  __shared__ uint32_t cnt[TILE_BUCKETS], base[TILE_BUCKETS], first[TILE_BUCKETS], lds[8];
  __shared__ uint32_t pcnt[TILE_BUCKETS], pbase[TILE_BUCKETS], pfirst[TILE_BUCKETS];
  if (threadIdx.x < TILE_BUCKETS) cnt[threadIdx.x] = pcnt[threadIdx.x] = 0;
  bucket_first(hist, first, lds);
  __syncthreads();
  if (pairs) {
    bucket_first(hist + 2 * TILE_BUCKETS, pfirst, lds);
    __syncthreads();
  }
  // the slots before bucket 0 are the tiles with something walked
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    DevHeader* hdr = at<DevHeader>(ws, L.o_hdr);
    hdr->bwd_work = first[0];
    if (pairs) {
      uint64_t np = 0;
      for (int b = 0; b < TILE_BUCKETS; ++b) np += hist[2 * TILE_BUCKETS + b];
      hdr->pairs_total = (uint32_t)min(np, (uint64_t)0xffffffffu);
      // the capacity a backward needs covers the pairs too
      if (np > hdr->entries_needed) hdr->entries_needed = np;
      if (np > (uint64_t)L.entry_cap) hdr->overflow |= 4u;   // the forward's outputs stand; its backward would not
    }
  }
  int b[SC_PER];
  uint32_t rank[SC_PER], prank[SC_PER], pe[SC_PER];
  TileSlot sl[SC_PER];
#pragma unroll
  for (int i = 0; i < SC_PER; ++i) {
    const uint32_t t = (blockIdx.x * SC_PER + (uint32_t)i) * 256u + threadIdx.x;
    b[i] = 0;
    rank[i] = prank[i] = pe[i] = 0u;
    if (t < (uint32_t)L.total_tiles) {
      sl[i] = slots[t];
      pe[i] = pend[t];
      b[i] = len_bucket(pe[i] - sl[i].start);
      rank[i] = atomicAdd(&cnt[b[i]], 1u);
      if (pairs && pe[i] > sl[i].start) prank[i] = atomicAdd(&pcnt[b[i]], at<const uint32_t>(ws, L.o_slot_pairs)[t]);
    }
  }
  __syncthreads();
  if (threadIdx.x < TILE_BUCKETS && cnt[threadIdx.x]) {
    base[threadIdx.x] = first[threadIdx.x] + atomicAdd(&cursor[threadIdx.x], cnt[threadIdx.x]);
    if (pairs)
      pbase[threadIdx.x] = pfirst[threadIdx.x] +
                           atomicAdd(at<uint32_t>(ws, L.o_bwd_hist) + 3 * TILE_BUCKETS + threadIdx.x, pcnt[threadIdx.x]);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < SC_PER; ++i) {
    const uint32_t t = (blockIdx.x * SC_PER + (uint32_t)i) * 256u + threadIdx.x;
    if (t < (uint32_t)L.total_tiles) {
      const uint32_t q = base[b[i]] + rank[i];
      bslots[q] = sl[i];
      bpend[q] = pe[i];
      if (pairs) at<uint32_t>(ws, L.o_bwd_base)[q] = pbase[b[i]] + prank[i];
    }
  }
}

hipError_t launch_bwd_order(void* ws, const Layout& L, hipStream_t st) {
  if (L.total_tiles == 0) return hipSuccess;
  const unsigned nb = (unsigned)((L.total_tiles + 256 * SC_PER - 1) / (256 * SC_PER));
  // histograms: counted by the forward compositing kernel; cursors: cleared
  // by the project kernel
  k_bwd_scatter<<<nb, 256, 0, st>>>(ws, L);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a5b: depth order inside each tile.  The tile sort leaves every tile's
// entries in record order (per view ascending kept slot, i.e. ascending tet
// id); each tile is then sorted by the key (depth float bits, record), which
// is unique and gives the (tile, depth, tet id) order of Sec. 3.3 with the
// tie broken by tet id.  One workgroup per tile with entries, longest lists
// first (the forward dispatch order).  The sort is a bottom-up merge sort in
// which every element goes straight to its place in the merged pair of runs:
// its index in its own run plus the number of keys below it in the other
// run (a binary search; the keys are distinct), one barrier per doubling of
// the run length.  A list of at most DS_CAP entries is sorted in LDS; a
// longer one sorts runs of DS_CAP in LDS and merges them the same way in
// HBM, ping-ponging between the other tile-sort buffer pair and the tile's
// own range of the result pair (whose tile keys are rewritten at the end).
// DS_CAP = 1024 keeps the workgroup at 16 KB of LDS (eight per CU): at the
// training shape the lists average about 400 entries and reach about 1,100,
// and the sort took 37 us against 43 us with 2048 (five per CU) and 45 us
// with 512 (more lists take the HBM merge).
// ---------------------------------------------------------------------------
constexpr int DS_CAP = 1024;

// Where element i (key `key`) of a run of length w goes when runs are merged
// pairwise: `get(j)` reads the key at index j of the current array of length n.
template <class Get>
__device__ __forceinline__ uint32_t merge_position(uint32_t i, unsigned long long key, uint32_t w, uint32_t n,
                                                   Get&& get) {
  const uint32_t lo = i - i % w;
  const bool left = ((i / w) & 1u) == 0u;
  uint32_t a = left ? min(lo + w, n) : lo - w;   // the other run [a, b)
  const uint32_t a0 = a;
  uint32_t b = left ? min(lo + 2 * w, n) : lo;
  while (a < b) {
    const uint32_t mid = (a + b) >> 1;
    if (get(mid) < key) a = mid + 1;
    else b = mid;
  }
  return (left ? lo : lo - w) + (i - lo) + (a - a0);
}

// Sort k[0, m) (m <= DS_CAP) in LDS, t as the second buffer; returns the
// buffer that holds the result.  (Measured at the training shape: this plain
// form, 42 us for the 3,450 lists, beat a bitonic network in LDS, 77 us, and
// one that first sorts runs of 64 per wave in registers and then searches
// several keys per thread together, 53 us: the sort is bound by the latency
// of its dependent LDS reads, and the wave-level network adds a chain of
// lane exchanges of its own.)
__device__ __forceinline__ unsigned long long* lds_merge_sort(unsigned long long* k, unsigned long long* t,
                                                              uint32_t m) {
  for (uint32_t w = 1; w < m; w <<= 1) {
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
      const unsigned long long key = k[i];
      t[merge_position(i, key, w, m, [&](uint32_t j) { return k[j]; })] = key;
    }
    __syncthreads();
    unsigned long long* x = k; k = t; t = x;
  }
  return k;
}

__global__ __launch_bounds__(256) void k_tile_depth_sort(void* ws, Layout L) {
  __shared__ unsigned long long kbuf[2][DS_CAP];
  const uint32_t n_empty = at<const uint32_t>(ws, L.o_tile_hist)[0];
  if (blockIdx.x >= (uint32_t)L.total_tiles - n_empty) return;
  const TileSlot sl = at<const TileSlot>(ws, L.o_tile_order)[blockIdx.x];
  const uint32_t s0 = sl.start, n = sl.end - sl.start;
  uint32_t* rk = at<uint32_t>(ws, sorted_tile_keys(L));       // result pair: tile keys, records
  uint32_t* rv = at<uint32_t>(ws, sorted_entry_records(L));
  // the list's tile keys (a list past DS_CAP uses them as merge scratch first
  // and writes them at the end)
  if (n <= (uint32_t)DS_CAP)
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) rk[s0 + i] = sl.tile;
  if (n < 2) return;
  const uint32_t* zkey = at<const uint32_t>(ws, L.o_key1a);   // depth bits per record
  const bool res_a = sorted_entry_records(L) == L.o_val2a;    // scratch pair: the other buffers
  uint32_t* xk = at<uint32_t>(ws, res_a ? L.o_key2b : L.o_key2a);
  uint32_t* xv = at<uint32_t>(ws, res_a ? L.o_val2b : L.o_val2a);
  // runs of DS_CAP (the whole list if it fits) sorted in LDS
  for (uint32_t r0 = 0; r0 < n; r0 += DS_CAP) {
    const uint32_t m = min((uint32_t)DS_CAP, n - r0);
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
      const uint32_t r = rv[s0 + r0 + i];
      kbuf[0][i] = ((unsigned long long)zkey[r] << 32) | r;
    }
    __syncthreads();
    const unsigned long long* srt = lds_merge_sort(kbuf[0], kbuf[1], m);
    if (n <= (uint32_t)DS_CAP) {
      for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) rv[s0 + i] = (uint32_t)srt[i];
      return;
    }
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
      xk[s0 + r0 + i] = (uint32_t)(srt[i] >> 32);
      xv[s0 + r0 + i] = (uint32_t)srt[i];
    }
    __syncthreads();
  }
  // pairwise merges of the runs in HBM: scratch -> result pair -> scratch ...
  uint32_t *ak = xk, *av = xv, *bk = rk, *bv = rv;
  for (uint32_t w = DS_CAP; w < n; w <<= 1) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
      const unsigned long long key = ((unsigned long long)ak[s0 + i] << 32) | av[s0 + i];
      const uint32_t pos = merge_position(i, key, w, n, [&](uint32_t j) {
        return ((unsigned long long)ak[s0 + j] << 32) | av[s0 + j];
      });
      bk[s0 + pos] = (uint32_t)(key >> 32);
      bv[s0 + pos] = (uint32_t)key;
    }
    __syncthreads();
    uint32_t* t = ak; ak = bk; bk = t;
    t = av; av = bv; bv = t;
  }
  // the sorted records into the result pair, whose tile keys are restored
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    if (av != rv) rv[s0 + i] = av[s0 + i];
    rk[s0 + i] = sl.tile;
  }
}

hipError_t launch_tile_depth_sort(void* ws, const Layout& L, hipStream_t st) {
  if (L.total_tiles == 0) return hipSuccess;
  k_tile_depth_sort<<<(unsigned)L.total_tiles, 256, 0, st>>>(ws, L);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// gradient buffers are overwritten: clear them first
// ---------------------------------------------------------------------------
// The scenes' gradients (row y: scene y); row 0 also clears the entry flags
// of the last forward's entries (the backward sets the ones it reaches) and
// the cursors of the backward dispatch order.
__device__ __forceinline__ void zero_grads_body(const DevScene& S, void* ws, const Layout& L) {
  const size_t n3 = 3 * (size_t)S.V;
  const size_t i0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = i0; i < n3; i += stride) {
    S.dverts[i] = 0.0f;
    S.dcolors[i] = 0.0f;
    if (i < (size_t)S.V) S.dsdf[i] = 0.0f;
  }
  if (blockIdx.y != 0) return;
  const DevHeader* hdr = at<const DevHeader>(ws, L.o_hdr);
  uint32_t* f = at<uint32_t>(ws, L.o_eflag);
  const uint32_t words = (hdr->entries_total + 3u) / 4u;
  for (size_t i = i0; i < words; i += stride) f[i] = 0u;
  if (record_grads(L)) {
    // the records' gradient accumulators
    float4* acc = at<float4>(ws, L.o_tgrad);
    const size_t n4 = (size_t)min(hdr->records_total, (uint32_t)L.rec_cap) * (TGRAD_STRIDE / 4);
    for (size_t i = i0; i < n4; i += stride) acc[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
}

__global__ void k_zero_grads(void* ws, Layout L) {
  zero_grads_body(at<const DevScene>(ws, L.o_scene)[blockIdx.y], ws, L);
}

// The same, taking the backward's descriptor image (scenes first) as the
// kernel argument: row 0 also writes it to the workspace for the kernels
// after this one, and every block reads its scene from the argument.
__global__ void k_zero_grads_desc(Blob b, int nwords, void* ws, Layout L) {
  if (blockIdx.y == 0) {
    uint32_t* dst = at<uint32_t>(ws, L.o_scene);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += gridDim.x * blockDim.x) dst[i] = b.w[i];
  }
  zero_grads_body(reinterpret_cast<const DevScene*>(b.w)[blockIdx.y], ws, L);
}

// Descriptor upload and gradient clearing of a backward pass: one launch when
// the descriptors fit in one kernel argument, else the upload launches and
// then the clearing kernel.
hipError_t launch_desc_zero_grads(const DevScene* hs, int ns, const DevView* hv, int nv, const int32_t* scene_views,
                                  void* ws, const Layout& L, hipStream_t st) {
  std::vector<uint8_t> img;
  size_t first;
  hipError_t e = desc_image(hs, ns, hv, nv, scene_views, L, false, img, first);
  if (e != hipSuccess) return e;
  dim3 grid(256, (unsigned)L.ns);
  const size_t words = img.size() / 4;
  if (words <= (size_t)BLOB_WORDS) {
    static_assert(alignof(DevScene) <= 16, "scenes start the image, which starts the argument");
    Blob b;
    std::memcpy(b.w, img.data(), img.size());
    k_zero_grads_desc<<<grid, 256, 0, st>>>(b, (int)words, ws, L);
  } else {
    e = upload(img.data(), img.size(), at<void>(ws, first), st);
    if (e != hipSuccess) return e;
    k_zero_grads<<<grid, 256, 0, st>>>(ws, L);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Coarse-to-fine pre-filtering (App. B): bounding box of the vertices of the
// kept tets.  Coordinates are reduced as order-preserving integer images of
// their float bits (min/max are exact and order-independent).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ord_bits(float x) {
  const uint32_t b = __float_as_uint(x);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ord_float(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__global__ void k_bounds_init(uint32_t* box, unsigned long long* kept) {
  const int t = threadIdx.x;
  if (t < 3) box[t] = 0xffffffffu;
  if (t >= 3 && t < 6) box[t] = 0u;
  if (t == 0 && kept) *kept = 0ull;
}

__global__ __launch_bounds__(256) void k_pf_bounds(DevScene S, float tf, uint32_t* box, unsigned long long* kept) {
  uint32_t mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, mx[3] = {0u, 0u, 0u};
  uint32_t cnt = 0;
  for (int k = blockIdx.x * 256 + threadIdx.x; k < S.K; k += gridDim.x * 256) {
    int4 vi;
    if (!keep_tet(S, k, tf, nullptr, &vi)) continue;
    ++cnt;
    const int idx[4] = {vi.x, vi.y, vi.z, vi.w};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const uint32_t u = ord_bits(S.verts[3 * (size_t)idx[a] + c]);
        mn[c] = min(mn[c], u);
        mx[c] = max(mx[c], u);
      }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      mn[c] = min(mn[c], (uint32_t)__shfl_xor((int)mn[c], o, 64));
      mx[c] = max(mx[c], (uint32_t)__shfl_xor((int)mx[c], o, 64));
    }
    cnt += (uint32_t)__shfl_xor((int)cnt, o, 64);
  }
  if ((threadIdx.x & 63) == 0 && cnt > 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      atomicMin(&box[c], mn[c]);
      atomicMax(&box[3 + c], mx[c]);
    }
    if (kept) atomicAdd(kept, (unsigned long long)cnt);
  }
}

// in place: integer images back to floats; NaN where nothing was kept
__global__ void k_bounds_final(uint32_t* box) {
  const int t = threadIdx.x;
  if (t < 6) {
    const uint32_t u = box[t];
    const bool empty = (t < 3) ? (u == 0xffffffffu) : (u == 0u);
    reinterpret_cast<float*>(box)[t] = empty ? __uint_as_float(0x7fc00000u) : ord_float(u);
  }
}

hipError_t launch_prefilter_bounds(const DevScene& S, float tf, float* bounds, int64_t* kept, hipStream_t st) {
  uint32_t* box = reinterpret_cast<uint32_t*>(bounds);
  unsigned long long* kp = reinterpret_cast<unsigned long long*>(kept);
  k_bounds_init<<<1, 64, 0, st>>>(box, kp);
  const unsigned g = (unsigned)std::max(1, std::min((S.K + 255) / 256, 2048));
  if (S.K > 0) k_pf_bounds<<<g, 256, 0, st>>>(S, tf, box, kp);
  k_bounds_final<<<1, 64, 0, st>>>(box);
  return hipGetLastError();
}



// ---------------------------------------------------------------------------
// Coarse-to-fine grid (App. B).  The second pass keeps the resolution R and
// cubic cells: a cube centred on the first pass's kept box, whose side is the
// box's largest extent plus one coarse cell on each side.  Arithmetic of the
// cube: extents in float32, side rounded to float32 from the double sum, the
// centre and low corner in double (rounded to float32 at the end), cell size
// side / R in float32.  An empty kept set (NaN box) keeps the input cube.
// ---------------------------------------------------------------------------
__global__ void k_refit_cube(const float* __restrict__ box, const float* __restrict__ cube_in, int R,
                             float* __restrict__ cube_out) {
  if (threadIdx.x != 0) return;
  float lo[3], hi[3];
  bool empty = false;
  for (int c = 0; c < 3; ++c) {
    lo[c] = box[c];
    hi[c] = box[3 + c];
    empty = empty || !(lo[c] == lo[c]) || !(hi[c] == hi[c]);
  }
  if (empty) {
    for (int c = 0; c < 4; ++c) cube_out[c] = cube_in[c];
    return;
  }
  float ext = hi[0] - lo[0];
  ext = fmaxf(ext, hi[1] - lo[1]);
  ext = fmaxf(ext, hi[2] - lo[2]);
  const double pad = 2.0 * (double)cube_in[3];
  const float side = (float)((double)ext + pad);
  const double half = (double)side * 0.5;
  for (int c = 0; c < 3; ++c) {
    const double mid = ((double)lo[c] + (double)hi[c]) * 0.5;
    cube_out[c] = (float)(mid - half);
  }
  cube_out[3] = side / (float)R;
}

// Vertex (x, y, z) = x + (R+1)(y + (R+1) z) at low + (x, y, z) h (float32:
// one product, one sum, no fused multiply-add); cell q = x + R(y + R z) holds
// tets 6q + p, p over the six axis orders (a, b, c) in lexicographic order,
// with vertices (v0, v0 + e_a, v0 + e_a + e_b, v0 + (1, 1, 1)).
__global__ __launch_bounds__(256) void k_cube_grid(int R, const float* __restrict__ cube, float* __restrict__ verts,
                                                   int4* __restrict__ tets) {
  const uint32_t n = (uint32_t)R + 1u;
  const uint64_t nv = (uint64_t)n * n * n, nc = (uint64_t)R * R * R;
  const float lx = cube[0], ly = cube[1], lz = cube[2], h = cube[3];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nv; t += stride) {
    const uint32_t x = (uint32_t)(t % n), y = (uint32_t)((t / n) % n), z = (uint32_t)(t / ((uint64_t)n * n));
    verts[3 * t + 0] = lx + (float)x * h;
    verts[3 * t + 1] = ly + (float)y * h;
    verts[3 * t + 2] = lz + (float)z * h;
  }
  if (!tets) return;
  const int st[3] = {1, (int)n, (int)(n * n)};
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nc; q += stride) {
    const uint32_t x = (uint32_t)(q % R), y = (uint32_t)((q / R) % R), z = (uint32_t)(q / ((uint64_t)R * R));
    const int v0 = (int)(x + n * (y + n * z));
    const int diag = v0 + 1 + (int)n + (int)(n * n);
    // axis orders (0,1,2) (0,2,1) (1,0,2) (1,2,0) (2,0,1) (2,1,0): first and second axis
    const int fa[6] = {0, 0, 1, 1, 2, 2}, fb[6] = {1, 2, 0, 2, 0, 1};
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const int a1 = v0 + st[fa[p]];
      tets[6 * q + p] = make_int4(v0, a1, a1 + st[fb[p]], diag);
    }
  }
}

hipError_t launch_refit_cube(const float* bounds, const float* cube_in, int R, float* cube_out, hipStream_t st) {
  k_refit_cube<<<1, 64, 0, st>>>(bounds, cube_in, R, cube_out);
  return hipGetLastError();
}

hipError_t launch_cube_grid(int R, const float* cube, float* verts, int32_t* tets, hipStream_t st) {
  const uint64_t nv = (uint64_t)(R + 1) * (R + 1) * (R + 1);
  const uint64_t blocks = std::min<uint64_t>((nv + 255) / 256, 8192);
  k_cube_grid<<<(unsigned)std::max<uint64_t>(blocks, 1), 256, 0, st>>>(R, cube, verts,
                                                                       reinterpret_cast<int4*>(tets));
  return hipGetLastError();
}

}  // namespace ts
