// Plain CPU oracle for the tile-based differentiable tetrahedron rasterizer of
// "Tetrahedron Splatting for 3D Generation" (TeT-Splatting, arXiv 2406.01579).
//
// TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark load or call this library.  The product path
// never does, and this file shares no code, header, table or helper with the
// HIP implementation.
//
// It is deliberately slow and literal: for every requested pixel it loops over
// every kept tetrahedron, tests whether the pixel lies in the tet's projected
// hull with the 2D barycentric coordinates of the four projected faces
// (Appendix A.1), takes the entry/exit SDF values with perspective correction
// (Appendix A.2), converts them to opacity with Eq. 1, sorts the hits by the
// tet's average vertex depth (Sec. 3.3) and alpha-blends front to back (Eq. 2).
// The gradient is the reverse mode of exactly that computation.
//
// Precision: every function is a template on the real type.  It is
// instantiated with float (the parity target), double (the error reference)
// and a forward-mode dual number (an independent derivative, used to pin the
// hand-written reverse mode).  Decisions that turn floating point into
// integers shared with the tiling stage -- which tets are kept by the
// pre-filter, near-plane culling, pixel/tile rectangles and the depth sort
// key -- are always taken in float32 with the fixed operation sequence written
// below, so all instantiations blend the same tets in the same order.
//
// Readings of the paper used here (where it is silent or ambiguous):
//  * inside test: all three barycentrics >= 0 (closed triangle); a face whose
//    2D determinant is exactly zero never contains the pixel (App. A.1 only
//    bounds u' and v').
//  * entry/exit: among the faces containing the pixel, the one with the
//    smallest perspective depth gives f_prev, the largest gives f_next; fewer
//    than two hit faces means the tet does not contribute (Sec. 3.2).
//  * Eq. 1 is evaluated in the algebraically identical form
//    alpha = -expm1(-s (f_prev - f_next)) / (1 + exp(s f_next)), which stays
//    finite where Phi_s(f_prev) underflows.
//  * pre-filter: alpha_max = Eq. 1 at (f_max, f_min) of the 4 vertices
//    (the text's "s_prev/s_next" are the SDF values).
//  * per-tet colour: mean of the four vertex colours (materials taken at the
//    tet centre, App. B).
//  * depth z_i of Eq. 2 and the sort key: mean of the 4 camera-space depths.
//  * normal: g/|g| in world space (Sec. 3.2, App. A.3), zero if the 4x4
//    system is singular or g = 0; blended N is not renormalised.
//  * blending thresholds follow the 3DGS rasterizer the paper builds on
//    (Sec. 3.3): skip alpha < alpha_min, clamp alpha to alpha_clamp, stop
//    before a tet that would take T below t_min; additionally stop once T is
//    exactly zero (nothing after it can contribute).  All are parameters.
//  * camera: OpenCV pinhole, pixel centres at (i+0.5, j+0.5), background
//    colour added as T_final * bg to RGB only.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// forward-mode dual number
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double x) : v(x), d(0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
inline bool operator==(Dual a, Dual b) { return a.v == b.v; }

// ---------------------------------------------------------------------------
// running error bound (Wilkinson's running error analysis; Higham, Accuracy
// and Stability of Numerical Algorithms, 2nd ed., Sec. 3.3): v is the value
// computed in float64 with exactly the double instantiation's operations, e a
// first-order bound on how far a float32 evaluation of the same operations
// can be from v.  Each float32 operation rounds with relative error at most
// u = 2^-24 plus an absolute error of at most 2^-150 below the normal range
// (Higham, Thm 2.3; the exponentials at most two units of u); inputs and
// constants are float32 values, exact.  A result past the float32 range is
// infinite there: its bound is infinite, and a finite value divided by it
// (zero in float32) is off by at most its own magnitude.
// ---------------------------------------------------------------------------
constexpr double U32 = 1.0 / 16777216.0;
constexpr double ETA32 = 0x1p-150;
constexpr double FLT32_MAX = 3.4028234663852886e38;
struct Rerr {
  double v, e;
  Rerr() : v(0), e(0) {}
  Rerr(double x) : v(x), e(0) {}
  Rerr(double x, double ex) : v(x), e(ex) {}
};
inline double rnd32(double v) {
  return std::fabs(v) > FLT32_MAX ? HUGE_VAL : U32 * std::fabs(v) + ETA32;
}
inline Rerr operator+(Rerr a, Rerr b) { double v = a.v + b.v; return {v, a.e + b.e + rnd32(v)}; }
inline Rerr operator-(Rerr a, Rerr b) { double v = a.v - b.v; return {v, a.e + b.e + rnd32(v)}; }
inline Rerr operator-(Rerr a) { return {-a.v, a.e}; }
inline Rerr operator*(Rerr a, Rerr b) {
  double v = a.v * b.v;
  return {v, std::fabs(b.v) * a.e + std::fabs(a.v) * b.e + rnd32(v)};
}
inline Rerr operator/(Rerr a, Rerr b) {
  double v = a.v / b.v;
  if (std::isinf(b.e) && !std::isinf(a.e)) return {v, std::fabs(v) + ETA32};
  return {v, (a.e + std::fabs(v) * b.e) / std::fabs(b.v) + rnd32(v)};
}
inline Rerr& operator+=(Rerr& a, Rerr b) { a = a + b; return a; }
inline Rerr& operator-=(Rerr& a, Rerr b) { a = a - b; return a; }
inline Rerr& operator*=(Rerr& a, Rerr b) { a = a * b; return a; }
inline bool operator<(Rerr a, Rerr b) { return a.v < b.v; }
inline bool operator>(Rerr a, Rerr b) { return a.v > b.v; }
inline bool operator<=(Rerr a, Rerr b) { return a.v <= b.v; }
inline bool operator>=(Rerr a, Rerr b) { return a.v >= b.v; }
inline bool operator==(Rerr a, Rerr b) { return a.v == b.v; }

inline float r_exp(float x) { return std::exp(x); }
inline double r_exp(double x) { return std::exp(x); }
inline Dual r_exp(Dual x) { double e = std::exp(x.v); return {e, e * x.d}; }
inline float r_expm1(float x) { return std::expm1(x); }
inline double r_expm1(double x) { return std::expm1(x); }
inline Dual r_expm1(Dual x) { return {std::expm1(x.v), std::exp(x.v) * x.d}; }
inline float r_sqrt(float x) { return std::sqrt(x); }
inline double r_sqrt(double x) { return std::sqrt(x); }
inline Dual r_sqrt(Dual x) { double r = std::sqrt(x.v); return {r, r > 0 ? x.d / (2 * r) : 0.0}; }
inline Rerr r_exp(Rerr x) { double v = std::exp(x.v); return {v, v * x.e + 2 * rnd32(v)}; }
inline Rerr r_expm1(Rerr x) {
  double v = std::expm1(x.v);
  return {v, std::exp(x.v) * x.e + 2 * rnd32(v)};
}
inline Rerr r_sqrt(Rerr x) {
  double r = std::sqrt(x.v);
  return {r, (r > 0 ? x.e / (2 * r) : std::sqrt(x.e)) + rnd32(r)};
}
inline float r_fma(float a, float b, float c) { return std::fma(a, b, c); }
inline double r_fma(double a, double b, double c) { return std::fma(a, b, c); }
inline Dual r_fma(Dual a, Dual b, Dual c) { return a * b + c; }
inline Rerr r_fma(Rerr a, Rerr b, Rerr c) {
  double v = std::fma(a.v, b.v, c.v);
  return {v, std::fabs(b.v) * a.e + std::fabs(a.v) * b.e + c.e + rnd32(v)};
}
inline double val(float x) { return x; }
inline double val(double x) { return x; }
inline double val(Dual x) { return x.v; }
inline double val(Rerr x) { return x.v; }
inline double tan_(float) { return 0; }
inline double tan_(double) { return 0; }
inline double tan_(Dual x) { return x.d; }
inline double tan_(Rerr x) { return x.e; }

// ---------------------------------------------------------------------------
// inputs
// ---------------------------------------------------------------------------
struct Cam {
  int W, H;
  float R[9], t[3], fx, fy, cx, cy, znear, bg[3];
};
Cam load_cam(const float* r) {
  Cam c;
  c.W = (int)r[0];
  c.H = (int)r[1];
  for (int i = 0; i < 9; ++i) c.R[i] = r[2 + i];
  for (int i = 0; i < 3; ++i) c.t[i] = r[11 + i];
  c.fx = r[14]; c.fy = r[15]; c.cx = r[16]; c.cy = r[17]; c.znear = r[18];
  for (int i = 0; i < 3; ++i) c.bg[i] = r[19 + i];
  return c;
}
struct Params {
  int tile_w, tile_h;
  float alpha_min, alpha_clamp, t_min, prefilter_tf, s;
  int window;  // per-pixel resort window N_w (Sec. 3.3); 0: off
};
Params load_params(const float* p) {
  return Params{(int)p[0], (int)p[1], p[2], p[3], p[4], p[5], p[6], (int)p[7]};
}

template <class R>
struct Scene {
  const R* verts;  // [V,3]
  const int* tets; // [K,4]
  const R* sdf;    // [V]
  const R* colors; // [V,3]
  int V, K;
};

// ---------------------------------------------------------------------------
// Eq. 1 (stable form), generic
// ---------------------------------------------------------------------------
template <class R>
R alpha_eq1(R fprev, R fnext, R s) {
  R d = fprev - fnext;
  if (!(d > R(0))) return R(0);
  return -r_expm1(-(s * d)) / (R(1) + r_exp(s * fnext));
}

// ---------------------------------------------------------------------------
// O1: per-tet view-independent data (Sec. 3.2 pre-filter and normal, App. A.3)
// ---------------------------------------------------------------------------
// Pre-filter decision in float32: alpha_max from the max and min vertex SDF.
bool keep_decision(float f0, float f1, float f2, float f3, float s, float tf, float* amax_out) {
  float fmax = std::max(std::max(f0, f1), std::max(f2, f3));
  float fmin = std::min(std::min(f0, f1), std::min(f2, f3));
  float a = alpha_eq1<float>(fmax, fmin, s);
  if (amax_out) *amax_out = a;
  return a >= tf;
}

// Gaussian elimination with partial pivoting; false if a pivot is exactly 0.
template <class R>
bool solve4(R A[4][4], R b[4], R x[4]) {
  int p[4] = {0, 1, 2, 3};
  R M[4][5];
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j < 4; ++j) M[i][j] = A[i][j];
    M[i][4] = b[i];
  }
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (std::fabs(val(M[r][c])) > std::fabs(val(M[piv][c]))) piv = r;
    if (val(M[piv][c]) == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < 5; ++j) std::swap(M[c][j], M[piv][j]);
    for (int r = c + 1; r < 4; ++r) {
      R m = M[r][c] / M[c][c];
      for (int j = c; j < 5; ++j) M[r][j] = M[r][j] - m * M[c][j];
    }
  }
  for (int i = 3; i >= 0; --i) {
    R acc = M[i][4];
    for (int j = i + 1; j < 4; ++j) acc = acc - M[i][j] * x[j];
    x[i] = acc / M[i][i];
  }
  (void)p;
  return true;
}

template <class R>
struct KTet {
  int id;
  int vi[4];
  R x[4][3];
  R f[4];
  R g[3], gnorm, n[3], c[3];
  bool gvalid;  // 4x4 system solvable and |g| > 0
};

// App. A.3: [g; *] = inverse([v_k^T 1]) f ; n = g/|g|.
template <class R>
void tet_normal(KTet<R>& t) {
  R M[4][4], b[4], y[4];
  for (int k = 0; k < 4; ++k) {
    for (int j = 0; j < 3; ++j) M[k][j] = t.x[k][j];
    M[k][3] = R(1);
    b[k] = t.f[k];
  }
  t.gvalid = solve4(M, b, y);
  for (int j = 0; j < 3; ++j) t.g[j] = t.gvalid ? y[j] : R(0);
  t.gnorm = r_sqrt(t.g[0] * t.g[0] + t.g[1] * t.g[1] + t.g[2] * t.g[2]);
  if (!(t.gnorm > R(0))) t.gvalid = false;
  for (int j = 0; j < 3; ++j) t.n[j] = t.gvalid ? t.g[j] / t.gnorm : R(0);
}

template <class R>
std::vector<KTet<R>> prefilter(const Scene<R>& sc, const Params& P) {
  std::vector<KTet<R>> out;
  for (int k = 0; k < sc.K; ++k) {
    const int* tv = sc.tets + 4 * (size_t)k;
    float ff[4];
    for (int i = 0; i < 4; ++i) ff[i] = (float)val(sc.sdf[tv[i]]);
    if (!keep_decision(ff[0], ff[1], ff[2], ff[3], P.s, P.prefilter_tf, nullptr)) continue;
    KTet<R> t;
    t.id = k;
    for (int i = 0; i < 4; ++i) {
      t.vi[i] = tv[i];
      for (int j = 0; j < 3; ++j) t.x[i][j] = sc.verts[3 * (size_t)tv[i] + j];
      t.f[i] = sc.sdf[tv[i]];
    }
    tet_normal(t);
    for (int j = 0; j < 3; ++j) {
      const R* c = sc.colors;
      t.c[j] = ((c[3 * (size_t)tv[0] + j] + c[3 * (size_t)tv[1] + j]) +
                (c[3 * (size_t)tv[2] + j] + c[3 * (size_t)tv[3] + j])) * R(0.25);
    }
    out.push_back(t);
  }
  return out;
}

// ---------------------------------------------------------------------------
// O2: per-view projection.  Binning quantities in float32 with a fixed op
// sequence; the same projection in R for the blended values.
// ---------------------------------------------------------------------------
template <class T>
void cam_xform(const Cam& c, T x, T y, T z, T& X, T& Y, T& Z) {
  X = r_fma(T(c.R[0]), x, r_fma(T(c.R[1]), y, r_fma(T(c.R[2]), z, T(c.t[0]))));
  Y = r_fma(T(c.R[3]), x, r_fma(T(c.R[4]), y, r_fma(T(c.R[5]), z, T(c.t[1]))));
  Z = r_fma(T(c.R[6]), x, r_fma(T(c.R[7]), y, r_fma(T(c.R[8]), z, T(c.t[2]))));
}

struct Bin {  // float32 tiling quantities of one tet in one view
  bool culled;
  int i0, i1, j0, j1;  // inclusive pixel rectangle
  float zt;
  uint32_t zbits;
};

template <class R>
Bin bin_tet(const KTet<R>& t, const Cam& c) {
  Bin b{};
  float px[4], py[4], Z[4];
  for (int k = 0; k < 4; ++k) {
    float X, Y;
    cam_xform<float>(c, (float)val(t.x[k][0]), (float)val(t.x[k][1]), (float)val(t.x[k][2]), X, Y, Z[k]);
    if (Z[k] < c.znear) { b.culled = true; return b; }
    px[k] = std::fma(c.fx, X / Z[k], c.cx);
    py[k] = std::fma(c.fy, Y / Z[k], c.cy);
  }
  b.zt = ((Z[0] + Z[1]) + (Z[2] + Z[3])) * 0.25f;
  std::memcpy(&b.zbits, &b.zt, 4);
  float xmin = std::min(std::min(px[0], px[1]), std::min(px[2], px[3]));
  float xmax = std::max(std::max(px[0], px[1]), std::max(px[2], px[3]));
  float ymin = std::min(std::min(py[0], py[1]), std::min(py[2], py[3]));
  float ymax = std::max(std::max(py[0], py[1]), std::max(py[2], py[3]));
  b.i0 = (int)std::min(std::max(std::ceil(xmin - 0.5f), 0.0f), (float)c.W);
  b.i1 = (int)std::max(std::min(std::floor(xmax - 0.5f), (float)(c.W - 1)), -1.0f);
  b.j0 = (int)std::min(std::max(std::ceil(ymin - 0.5f), 0.0f), (float)c.H);
  b.j1 = (int)std::max(std::min(std::floor(ymax - 0.5f), (float)(c.H - 1)), -1.0f);
  if (b.i0 > b.i1 || b.j0 > b.j1) b.culled = true;
  return b;
}

template <class R>
struct VTet {
  Bin b;
  R X[4], Y[4], Z[4], px[4], py[4], zt;
};

template <class R>
VTet<R> project_tet(const KTet<R>& t, const Cam& c) {
  VTet<R> v;
  v.b = bin_tet(t, c);
  if (v.b.culled) return v;
  for (int k = 0; k < 4; ++k) {
    cam_xform<R>(c, t.x[k][0], t.x[k][1], t.x[k][2], v.X[k], v.Y[k], v.Z[k]);
    v.px[k] = r_fma(R(c.fx), v.X[k] / v.Z[k], R(c.cx));
    v.py[k] = r_fma(R(c.fy), v.Y[k] / v.Z[k], R(c.cy));
  }
  v.zt = ((v.Z[0] + v.Z[1]) + (v.Z[2] + v.Z[3])) * R(0.25);
  return v;
}

// ---------------------------------------------------------------------------
// O3: one pixel against one tet (App. A.1 barycentrics, A.2 perspective)
// ---------------------------------------------------------------------------
const int FACE[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};

template <class R>
R cross2(R ax, R ay, R bx, R by) { return ax * by - ay * bx; }

template <class R>
struct FaceHit {
  int face;
  R D, N[3], l[3];  // l = (1-u'-v', u', v')
  R q[3], Sg;       // q_k = l_k / Z_k, Sg = sum q
  R u, v, f, z;
};

template <class R>
bool face_hit(const R px[4], const R py[4], const R Z[4], const R f[4], int F, R qx, R qy, FaceHit<R>& h) {
  int A = FACE[F][0], B = FACE[F][1], C = FACE[F][2];
  h.face = F;
  // 2D determinant of [v_a' v_b' v_c'; 1 1 1]
  h.D = cross2(px[B] - px[A], py[B] - py[A], px[C] - px[A], py[C] - py[A]);
  if (h.D == R(0)) return false;
  // rows of the inverse times [p; 1] (Cramer's rule)
  h.N[0] = cross2(px[B] - qx, py[B] - qy, px[C] - qx, py[C] - qy);
  h.N[1] = cross2(px[C] - qx, py[C] - qy, px[A] - qx, py[A] - qy);
  h.N[2] = cross2(px[A] - qx, py[A] - qy, px[B] - qx, py[B] - qy);
  for (int i = 0; i < 3; ++i) h.l[i] = h.N[i] / h.D;
  if (!(h.l[0] >= R(0) && h.l[1] >= R(0) && h.l[2] >= R(0))) return false;
  // perspective correction
  h.q[0] = h.l[0] / Z[A];
  h.q[1] = h.l[1] / Z[B];
  h.q[2] = h.l[2] / Z[C];
  h.Sg = h.q[0] + h.q[1] + h.q[2];
  h.u = h.q[1] / h.Sg;
  h.v = h.q[2] / h.Sg;
  h.f = (R(1) - h.u - h.v) * f[A] + h.u * f[B] + h.v * f[C];
  h.z = R(1) / h.Sg;
  return true;
}

template <class R>
struct TetHit {
  FaceHit<R> in, out;  // entry (f_prev) and exit (f_next) faces
  R alpha;
};

template <class R>
bool tet_pixel(const R px[4], const R py[4], const R Z[4], const R f[4], R qx, R qy, R s, TetHit<R>& th) {
  FaceHit<R> hits[4];
  int nh = 0;
  for (int F = 0; F < 4; ++F)
    if (face_hit(px, py, Z, f, F, qx, qy, hits[nh])) ++nh;
  if (nh < 2) return false;
  int ie = 0, ix = 0;
  for (int i = 1; i < nh; ++i) {
    if (hits[i].z < hits[ie].z) ie = i;
    if (hits[i].z > hits[ix].z) ix = i;
  }
  th.in = hits[ie];
  th.out = hits[ix];
  th.alpha = alpha_eq1<R>(th.in.f, th.out.f, s);
  return true;
}

// ---------------------------------------------------------------------------
// O5/O6: per-pixel depth sort and front-to-back compositing (Eq. 2)
// ---------------------------------------------------------------------------
template <class R>
struct Contrib {
  uint32_t zbits;
  int tet_id;
  int slot;  // index into the kept list
  TetHit<R> hit;
  R T;          // transmittance before this tet
  R a;          // blended (clamped) alpha
  bool clamped, blended;
};

template <class R>
struct PixelResult {
  R out[8];  // R,G,B,O,D,Nx,Ny,Nz
  R T_final;
  int n_blended;
  std::vector<Contrib<R>> list;  // in blend order
};

// Sec. 3.3 resort window.  The pixel's candidates, in the per-tile order
// (mean depth, tet id), pass through a buffer of at most N_w entries kept
// sorted by the pixel's own entry depth (ties keep arrival order); when the
// buffer overflows, its nearest entry leaves and is blended next.  At the end
// of the list the rest leaves nearest first.  Only candidates that can blend
// (alpha >= alpha_min) enter the buffer.
template <class R>
void resort_window(std::vector<Contrib<R>>& list, int nw, float alpha_min) {
  std::vector<Contrib<R>> out, buf;
  for (const auto& ct : list) {
    if (ct.hit.alpha < R(alpha_min)) continue;
    auto at = std::upper_bound(buf.begin(), buf.end(), ct, [](const Contrib<R>& a, const Contrib<R>& b) {
      return a.hit.in.z < b.hit.in.z;
    });
    buf.insert(at, ct);
    if ((int)buf.size() > nw) {
      out.push_back(buf.front());
      buf.erase(buf.begin());
    }
  }
  out.insert(out.end(), buf.begin(), buf.end());
  list.swap(out);
}

// One threshold decision of a pixel's walk: the quantity compared and the
// threshold it was compared with (kind 0: alpha vs alpha_min, 1: alpha vs
// alpha_clamp, 2: T (1 - alpha) vs t_min).
template <class R>
struct Decision {
  int kind;
  R value;
  float threshold;
};

template <class R>
void shade_pixel(const std::vector<KTet<R>>& kt, const std::vector<VTet<R>>& vt, const Cam& c,
                 const Params& P, int i, int j, PixelResult<R>& pr, bool keep_list,
                 std::vector<Decision<R>>* log = nullptr) {
  R qx = R(i + 0.5), qy = R(j + 0.5);
  std::vector<Contrib<R>> list;
  for (size_t k = 0; k < kt.size(); ++k) {
    const VTet<R>& v = vt[k];
    if (v.b.culled) continue;
    if (i < v.b.i0 || i > v.b.i1 || j < v.b.j0 || j > v.b.j1) continue;
    Contrib<R> ct;
    if (!tet_pixel(v.px, v.py, v.Z, kt[k].f, qx, qy, R(P.s), ct.hit)) continue;
    ct.zbits = v.b.zbits;
    ct.tet_id = kt[k].id;
    ct.slot = (int)k;
    list.push_back(ct);
  }
  std::sort(list.begin(), list.end(), [](const Contrib<R>& a, const Contrib<R>& b) {
    return a.zbits != b.zbits ? a.zbits < b.zbits : a.tet_id < b.tet_id;
  });
  if (log)
    for (const auto& ct : list) log->push_back({0, ct.hit.alpha, P.alpha_min});
  if (P.window > 0) resort_window(list, P.window, P.alpha_min);
  for (int q = 0; q < 8; ++q) pr.out[q] = R(0);
  R T = R(1);
  int nb = 0;
  std::vector<Contrib<R>> kept;
  for (auto& ct : list) {
    R a = ct.hit.alpha;
    ct.blended = false;
    ct.clamped = false;
    if (a < R(P.alpha_min)) continue;
    if (log) log->push_back({1, a, P.alpha_clamp});
    if (a > R(P.alpha_clamp)) { a = R(P.alpha_clamp); ct.clamped = true; }
    R Tn = T * (R(1) - a);
    if (log) log->push_back({2, Tn, P.t_min});
    if (Tn < R(P.t_min)) break;
    const KTet<R>& t = kt[ct.slot];
    R w = T * a;
    pr.out[0] += w * t.c[0];
    pr.out[1] += w * t.c[1];
    pr.out[2] += w * t.c[2];
    pr.out[3] += w;
    pr.out[4] += w * vt[ct.slot].zt;
    pr.out[5] += w * t.n[0];
    pr.out[6] += w * t.n[1];
    pr.out[7] += w * t.n[2];
    ct.T = T;
    ct.a = a;
    ct.blended = true;
    ++nb;
    if (keep_list) kept.push_back(ct);
    T = Tn;
    if (T == R(0)) break;
  }
  for (int q = 0; q < 3; ++q) pr.out[q] += T * R(c.bg[q]);
  pr.T_final = T;
  pr.n_blended = nb;
  if (keep_list) pr.list.swap(kept);
}

// ---------------------------------------------------------------------------
// O7: reverse mode
// ---------------------------------------------------------------------------
// Screen-space gradient of one tet in one view.
template <class R>
struct TGrad {
  R px[4], py[4], Z[4], f[4], c[3], zt, n[3];
  void zero() {
    for (int k = 0; k < 4; ++k) px[k] = py[k] = Z[k] = f[k] = R(0);
    c[0] = c[1] = c[2] = zt = n[0] = n[1] = n[2] = R(0);
  }
  void add(const TGrad& o) {
    for (int k = 0; k < 4; ++k) { px[k] += o.px[k]; py[k] += o.py[k]; Z[k] += o.Z[k]; f[k] += o.f[k]; }
    for (int q = 0; q < 3; ++q) { c[q] += o.c[q]; n[q] += o.n[q]; }
    zt += o.zt;
  }
};

// Reverse of face_hit's value path, given dL/d(f of this face).
template <class R>
void face_backward(const FaceHit<R>& h, const R px[4], const R py[4], const R Z[4], const R f[4],
                   R qx, R qy, R df, TGrad<R>& g) {
  int I[3] = {FACE[h.face][0], FACE[h.face][1], FACE[h.face][2]};
  // f = (1-u-v) fA + u fB + v fC
  g.f[I[0]] += (R(1) - h.u - h.v) * df;
  g.f[I[1]] += h.u * df;
  g.f[I[2]] += h.v * df;
  R du = (f[I[1]] - f[I[0]]) * df;
  R dv = (f[I[2]] - f[I[0]]) * df;
  // u = q1/Sg, v = q2/Sg
  R dq[3] = {R(0), du / h.Sg, dv / h.Sg};
  R dSg = -(du * h.u + dv * h.v) / h.Sg;
  for (int k = 0; k < 3; ++k) dq[k] += dSg;
  // q_k = l_k / Z_k
  R dl[3];
  for (int k = 0; k < 3; ++k) {
    dl[k] = dq[k] / Z[I[k]];
    g.Z[I[k]] -= dq[k] * h.q[k] / Z[I[k]];
  }
  // l_k = N_k / D
  R dN[3], dD = R(0);
  for (int k = 0; k < 3; ++k) {
    dN[k] = dl[k] / h.D;
    dD -= dl[k] * h.l[k] / h.D;
  }
  // D = cross(B-A, C-A)
  {
    R e1x = px[I[1]] - px[I[0]], e1y = py[I[1]] - py[I[0]];
    R e2x = px[I[2]] - px[I[0]], e2y = py[I[2]] - py[I[0]];
    R de1x = dD * e2y, de1y = -dD * e2x, de2x = -dD * e1y, de2y = dD * e1x;
    g.px[I[1]] += de1x; g.py[I[1]] += de1y;
    g.px[I[2]] += de2x; g.py[I[2]] += de2y;
    g.px[I[0]] -= de1x + de2x; g.py[I[0]] -= de1y + de2y;
  }
  // N_0 = cross(B-p, C-p), N_1 = cross(C-p, A-p), N_2 = cross(A-p, B-p)
  const int pr[3][2] = {{1, 2}, {2, 0}, {0, 1}};
  for (int k = 0; k < 3; ++k) {
    int a = I[pr[k][0]], b = I[pr[k][1]];
    R ax = px[a] - qx, ay = py[a] - qy, bx = px[b] - qx, by = py[b] - qy;
    g.px[a] += dN[k] * by;
    g.py[a] -= dN[k] * bx;
    g.px[b] -= dN[k] * ay;
    g.py[b] += dN[k] * ax;
  }
}

template <class R>
void pixel_backward(const std::vector<KTet<R>>& kt, const std::vector<VTet<R>>& vt, const Cam& c,
                    const Params& P, int i, int j, const double* dout,
                    std::vector<std::pair<int, TGrad<R>>>& contrib) {
  PixelResult<R> pr;
  shade_pixel(kt, vt, c, P, i, j, pr, true);
  R qx = R(i + 0.5), qy = R(j + 0.5);
  R grgb[3] = {R(dout[0]), R(dout[1]), R(dout[2])};
  R gO = R(dout[3]), gD = R(dout[4]);
  R gN[3] = {R(dout[5]), R(dout[6]), R(dout[7])};
  R Rb = grgb[0] * R(c.bg[0]) + grgb[1] * R(c.bg[1]) + grgb[2] * R(c.bg[2]);
  R s = R(P.s);
  for (int q = (int)pr.list.size() - 1; q >= 0; --q) {
    const Contrib<R>& ct = pr.list[q];
    const KTet<R>& t = kt[ct.slot];
    const VTet<R>& v = vt[ct.slot];
    R sc = grgb[0] * t.c[0] + grgb[1] * t.c[1] + grgb[2] * t.c[2] + gD * v.zt +
           gN[0] * t.n[0] + gN[1] * t.n[1] + gN[2] * t.n[2] + gO;
    R w = ct.T * ct.a;
    TGrad<R> g;
    g.zero();
    for (int k = 0; k < 3; ++k) { g.c[k] = w * grgb[k]; g.n[k] = w * gN[k]; }
    g.zt = w * gD;
    R da = ct.T * (sc - Rb);
    Rb = ct.a * sc + (R(1) - ct.a) * Rb;
    if (!ct.clamped) {
      // alpha = A / B, A = -expm1(-s d), B = 1 + exp(s f_next), d = f_prev - f_next
      R fp = ct.hit.in.f, fn = ct.hit.out.f;
      R d = fp - fn;
      if (d > R(0)) {
        R e1 = r_expm1(-(s * d));
        R e2 = r_exp(s * fn);
        R B = R(1) + e2;
        R al = -e1 / B;
        R dA = da / B;
        R dB = -da * al / B;
        R dfn = dB * s * e2;
        R de1 = -dA;
        R dd = -s * de1 * (e1 + R(1));
        R dfp = dd;
        dfn -= dd;
        face_backward(ct.hit.in, v.px, v.py, v.Z, t.f, qx, qy, dfp, g);
        face_backward(ct.hit.out, v.px, v.py, v.Z, t.f, qx, qy, dfn, g);
      }
    }
    contrib.emplace_back(ct.slot, g);
  }
}

// Chain one tet's screen-space gradient in one view to camera space and then
// world space; returns position gradients per vertex (plus the direct terms).
template <class R>
void tet_view_backward(const KTet<R>& t, const VTet<R>& v, const Cam& c, const TGrad<R>& g,
                       R dv[4][3]) {
  for (int k = 0; k < 4; ++k) {
    R dZ = g.Z[k] + g.zt * R(0.25);
    R rx = v.X[k] / v.Z[k], ry = v.Y[k] / v.Z[k];
    R drx = g.px[k] * R(c.fx), dry = g.py[k] * R(c.fy);
    R dX = drx / v.Z[k], dY = dry / v.Z[k];
    dZ -= drx * rx / v.Z[k] + dry * ry / v.Z[k];
    for (int j = 0; j < 3; ++j)
      dv[k][j] = R(c.R[j]) * dX + R(c.R[3 + j]) * dY + R(c.R[6 + j]) * dZ;
  }
  (void)t;
}

// normal n = g/|g| with [g;*] = M^-1 f, M rows [v_k^T 1]
template <class R>
void normal_backward(const KTet<R>& t, const R dn[3], R dv[4][3], R df[4]) {
  for (int k = 0; k < 4; ++k) { df[k] = R(0); for (int j = 0; j < 3; ++j) dv[k][j] = R(0); }
  if (!t.gvalid) return;
  R nd = t.n[0] * dn[0] + t.n[1] * dn[1] + t.n[2] * dn[2];
  R dg[3];
  for (int j = 0; j < 3; ++j) dg[j] = (dn[j] - t.n[j] * nd) / t.gnorm;
  R MT[4][4], b[4] = {dg[0], dg[1], dg[2], R(0)}, lam[4];
  for (int r = 0; r < 4; ++r) {
    for (int k = 0; k < 4; ++k) MT[r][k] = (r < 3) ? t.x[k][r] : R(1);
  }
  if (!solve4(MT, b, lam)) return;
  for (int k = 0; k < 4; ++k) {
    df[k] = lam[k];
    for (int j = 0; j < 3; ++j) dv[k][j] = -lam[k] * t.g[j];
  }
}

// ---------------------------------------------------------------------------
// drivers
// ---------------------------------------------------------------------------
template <class R>
struct Prepared {
  std::vector<KTet<R>> kt;
  std::vector<Cam> cams;
  std::vector<std::vector<VTet<R>>> vt;  // [view][kept]
};

template <class R>
void prepare(const Scene<R>& sc, const float* cams, int nv, const Params& P, Prepared<R>& pp) {
  pp.kt = prefilter(sc, P);
  pp.cams.resize(nv);
  pp.vt.assign(nv, {});
  for (int v = 0; v < nv; ++v) {
    pp.cams[v] = load_cam(cams + 22 * (size_t)v);
    pp.vt[v].resize(pp.kt.size());
  }
  long n = (long)pp.kt.size();
#pragma omp parallel for schedule(static)
  for (long k = 0; k < n; ++k)
    for (int v = 0; v < nv; ++v) pp.vt[v][k] = project_tet(pp.kt[k], pp.cams[v]);
}

template <class R>
struct Inputs {
  std::vector<R> verts, sdf, colors;
  Scene<R> sc;
};

template <class R>
void load_inputs(Inputs<R>& in, const double* verts, const int* tets, const double* sdf,
                 const double* colors, int V, int K, const double* tverts = nullptr,
                 const double* tsdf = nullptr, const double* tcolors = nullptr);

template <class R>
void load_inputs(Inputs<R>& in, const double* verts, const int* tets, const double* sdf,
                 const double* colors, int V, int K, const double*, const double*, const double*) {
  in.verts.resize(3 * (size_t)V);
  in.sdf.resize(V);
  in.colors.resize(3 * (size_t)V);
  for (size_t i = 0; i < 3 * (size_t)V; ++i) { in.verts[i] = R(verts[i]); in.colors[i] = R(colors[i]); }
  for (int i = 0; i < V; ++i) in.sdf[i] = R(sdf[i]);
  in.sc = Scene<R>{in.verts.data(), tets, in.sdf.data(), in.colors.data(), V, K};
}

template <>
void load_inputs<Dual>(Inputs<Dual>& in, const double* verts, const int* tets, const double* sdf,
                       const double* colors, int V, int K, const double* tv, const double* ts,
                       const double* tc) {
  in.verts.resize(3 * (size_t)V);
  in.sdf.resize(V);
  in.colors.resize(3 * (size_t)V);
  for (size_t i = 0; i < 3 * (size_t)V; ++i) {
    in.verts[i] = Dual(verts[i], tv ? tv[i] : 0.0);
    in.colors[i] = Dual(colors[i], tc ? tc[i] : 0.0);
  }
  for (int i = 0; i < V; ++i) in.sdf[i] = Dual(sdf[i], ts ? ts[i] : 0.0);
  in.sc = Scene<Dual>{in.verts.data(), tets, in.sdf.data(), in.colors.data(), V, K};
}

template <class R>
void render_impl(const Scene<R>& sc, const float* cams, int nv, const Params& P, const int* pix,
                 long npix, double* out, double* tout, int* nblend, double* tfinal) {
  Prepared<R> pp;
  prepare(sc, cams, nv, P, pp);
#pragma omp parallel for schedule(dynamic, 16)
  for (long q = 0; q < npix; ++q) {
    int v = pix[3 * q], i = pix[3 * q + 1], j = pix[3 * q + 2];
    PixelResult<R> pr;
    shade_pixel(pp.kt, pp.vt[v], pp.cams[v], P, i, j, pr, false);
    for (int c = 0; c < 8; ++c) {
      out[8 * q + c] = val(pr.out[c]);
      if (tout) tout[8 * q + c] = tan_(pr.out[c]);
    }
    if (nblend) nblend[q] = pr.n_blended;
    if (tfinal) tfinal[q] = val(pr.T_final);
  }
}

template <class R>
void backward_impl(const Scene<R>& sc, const float* cams, int nv, const Params& P, const int* pix,
                   long npix, const double* dout, double* dverts, double* dsdf, double* dcolors) {
  Prepared<R> pp;
  prepare(sc, cams, nv, P, pp);
  size_t nk = pp.kt.size();
  std::vector<std::vector<std::pair<int, TGrad<R>>>> per_pix(npix);
#pragma omp parallel for schedule(dynamic, 16)
  for (long q = 0; q < npix; ++q) {
    int v = pix[3 * q], i = pix[3 * q + 1], j = pix[3 * q + 2];
    pixel_backward(pp.kt, pp.vt[v], pp.cams[v], P, i, j, dout + 8 * q, per_pix[q]);
  }
  // serial reduction in pixel order (deterministic)
  std::vector<TGrad<R>> acc(nk * (size_t)nv);
  for (auto& g : acc) g.zero();
  for (long q = 0; q < npix; ++q) {
    int v = pix[3 * q];
    for (auto& pg : per_pix[q]) acc[(size_t)v * nk + pg.first].add(pg.second);
  }
  std::vector<R> gv(3 * (size_t)sc.V, R(0)), gs(sc.V, R(0)), gc(3 * (size_t)sc.V, R(0));
  for (size_t k = 0; k < nk; ++k) {
    const KTet<R>& t = pp.kt[k];
    R dn[3] = {R(0), R(0), R(0)}, dc[3] = {R(0), R(0), R(0)}, dfk[4] = {R(0), R(0), R(0), R(0)};
    R dvk[4][3];
    for (int a = 0; a < 4; ++a) for (int j = 0; j < 3; ++j) dvk[a][j] = R(0);
    for (int v = 0; v < nv; ++v) {
      const TGrad<R>& g = acc[(size_t)v * nk + k];
      if (pp.vt[v][k].b.culled) continue;
      R dvv[4][3];
      tet_view_backward(t, pp.vt[v][k], pp.cams[v], g, dvv);
      for (int a = 0; a < 4; ++a) {
        for (int j = 0; j < 3; ++j) dvk[a][j] += dvv[a][j];
        dfk[a] += g.f[a];
      }
      for (int j = 0; j < 3; ++j) { dn[j] += g.n[j]; dc[j] += g.c[j]; }
    }
    R nv_[4][3], nf[4];
    normal_backward(t, dn, nv_, nf);
    for (int a = 0; a < 4; ++a) {
      int vi = t.vi[a];
      for (int j = 0; j < 3; ++j) {
        gv[3 * (size_t)vi + j] += dvk[a][j] + nv_[a][j];
        gc[3 * (size_t)vi + j] += dc[j] * R(0.25);
      }
      gs[vi] += dfk[a] + nf[a];
    }
  }
  for (size_t i = 0; i < 3 * (size_t)sc.V; ++i) { dverts[i] = val(gv[i]); dcolors[i] = val(gc[i]); }
  for (int i = 0; i < sc.V; ++i) dsdf[i] = val(gs[i]);
}

// ---------------------------------------------------------------------------
// Error budget of a float32 backward.  Every gradient element x (the x, y, z
// of a vertex position, its SDF value, its r, g, b) is a sum of terms, one per
// (pixel, tet) pair the pixel blended: the pair's screen-space gradient g (the
// TGrad above) carried to the tet's four vertices by a chain J that is linear
// in g (projection, mean depth, normal, mean colour).  For these sums:
//   A[x] = sum over (view, tet) of |J| (sum over pixels of |g|), with |J| the
//          element-wise absolute chain.  Summing n terms in any order and
//          grouping moves the result by at most gamma_{n-1} times the sum of
//          the terms' magnitudes (Higham, Sec. 4.2); carried through J in
//          absolute value that is gamma times A[x].
//   E[x] = sum over (view, tet) of |J| (sum over pixels of the running error
//          bound of g): how far a float32 evaluation of each term, by the
//          operations written above, can be from its exact value.  A term
//          that the float32 and float64 walks do not both blend (a threshold
//          decision that rounding flips) counts with its full magnitude.
//   N[x] = the number of terms that reach x.
// Output arrays are [V, 7] (dverts xyz, dsdf, dcolors xyz).
// ---------------------------------------------------------------------------
double& tgrad_at(TGrad<double>& g, int k) {
  if (k < 4) return g.px[k];
  if (k < 8) return g.py[k - 4];
  if (k < 12) return g.Z[k - 8];
  if (k < 16) return g.f[k - 12];
  if (k < 19) return g.c[k - 16];
  if (k == 19) return g.zt;
  return g.n[k - 20];
}
template <class R>
R tgrad_get(const TGrad<R>& g, int k) {
  if (k < 4) return g.px[k];
  if (k < 8) return g.py[k - 4];
  if (k < 12) return g.Z[k - 8];
  if (k < 16) return g.f[k - 12];
  if (k < 19) return g.c[k - 16];
  if (k == 19) return g.zt;
  return g.n[k - 20];
}
constexpr int TGRAD_N = 23;

// J g for one tet in one view, per vertex: (dverts xyz, dsdf, dcolors xyz).
void chain_term(const KTet<double>& t, const VTet<double>& v, const Cam& c, const TGrad<double>& g,
                double out[4][7]) {
  double dv[4][3], nv_[4][3], nf[4];
  tet_view_backward(t, v, c, g, dv);
  normal_backward(t, g.n, nv_, nf);
  for (int a = 0; a < 4; ++a) {
    for (int j = 0; j < 3; ++j) {
      out[a][j] = dv[a][j] + nv_[a][j];
      out[a][4 + j] = g.c[j] * 0.25;
    }
    out[a][3] = g.f[a] + nf[a];
  }
}

struct BudgetTerm {
  int slot;
  TGrad<double> mag, err;  // |g| and the float32 error bound of g, per component
};

void budget_impl(const double* verts, const int* tets, const double* sdf, const double* colors, int V, int K,
                 const float* cams, int nv, const Params& P, const int* pix, long npix, const double* dout,
                 double* A, double* E, double* N) {
  Inputs<double> in64;
  Inputs<Rerr> inr;
  Inputs<float> in32;
  load_inputs(in64, verts, tets, sdf, colors, V, K);
  load_inputs(inr, verts, tets, sdf, colors, V, K);
  load_inputs(in32, verts, tets, sdf, colors, V, K);
  Prepared<double> p64;
  Prepared<Rerr> pr;
  Prepared<float> p32;
  prepare(in64.sc, cams, nv, P, p64);
  prepare(inr.sc, cams, nv, P, pr);
  prepare(in32.sc, cams, nv, P, p32);
  const size_t nk = p64.kt.size();  // the kept set is a float32 decision: the same in all three
  std::vector<std::vector<BudgetTerm>> per(npix);
#pragma omp parallel for schedule(dynamic, 16)
  for (long q = 0; q < npix; ++q) {
    const int v = pix[3 * q], i = pix[3 * q + 1], j = pix[3 * q + 2];
    std::vector<std::pair<int, TGrad<Rerr>>> cr;
    std::vector<std::pair<int, TGrad<float>>> c32;
    pixel_backward(pr.kt, pr.vt[v], pr.cams[v], P, i, j, dout + 8 * q, cr);
    pixel_backward(p32.kt, p32.vt[v], p32.cams[v], P, i, j, dout + 8 * q, c32);
    std::vector<int> slots;
    for (auto& x : cr) slots.push_back(x.first);
    for (auto& x : c32) slots.push_back(x.first);
    std::sort(slots.begin(), slots.end());
    slots.erase(std::unique(slots.begin(), slots.end()), slots.end());
    for (int sl : slots) {
      const TGrad<Rerr>* gr = nullptr;
      const TGrad<float>* g32 = nullptr;
      for (auto& x : cr)
        if (x.first == sl) gr = &x.second;
      for (auto& x : c32)
        if (x.first == sl) g32 = &x.second;
      BudgetTerm t;
      t.slot = sl;
      for (int k = 0; k < TGRAD_N; ++k) {
        const double m = gr ? std::fabs(tgrad_get(*gr, k).v) : 0.0;
        const double m32 = g32 ? std::fabs((double)tgrad_get(*g32, k)) : 0.0;
        tgrad_at(t.mag, k) = std::max(m, m32);
        // blended by both walks: the running bound; by one only: the whole term
        tgrad_at(t.err, k) = (gr && g32) ? tgrad_get(*gr, k).e : (gr ? m + tgrad_get(*gr, k).e : m32);
      }
      per[q].push_back(t);
    }
  }
  std::fill(A, A + 7 * (size_t)V, 0.0);
  std::fill(E, E + 7 * (size_t)V, 0.0);
  std::fill(N, N + 7 * (size_t)V, 0.0);
  std::vector<TGrad<double>> mag(nk * (size_t)nv), err(nk * (size_t)nv);
  for (auto& g : mag) g.zero();
  for (auto& g : err) g.zero();
  std::vector<long> cnt(nk * (size_t)nv, 0);
  for (long q = 0; q < npix; ++q) {
    const int v = pix[3 * q];
    for (const BudgetTerm& t : per[q]) {
      const size_t r = (size_t)v * nk + t.slot;
      mag[r].add(t.mag);
      err[r].add(t.err);
      ++cnt[r];
    }
  }
  for (int v = 0; v < nv; ++v)
    for (size_t k = 0; k < nk; ++k) {
      const size_t r = (size_t)v * nk + k;
      if (cnt[r] == 0) continue;
      const KTet<double>& t = p64.kt[k];
      for (int c = 0; c < TGRAD_N; ++c) {
        const double m = tgrad_at(mag[r], c), e = tgrad_at(err[r], c);
        if (m == 0.0 && e == 0.0) continue;
        TGrad<double> one;
        one.zero();
        tgrad_at(one, c) = 1.0;
        double col[4][7];
        chain_term(t, p64.vt[v][k], p64.cams[v], one, col);
        for (int a = 0; a < 4; ++a)
          for (int q = 0; q < 7; ++q) {
            if (col[a][q] == 0.0) continue;  // (an infinite bound times a zero chain entry adds nothing)
            A[7 * (size_t)t.vi[a] + q] += std::fabs(col[a][q]) * m;
            E[7 * (size_t)t.vi[a] + q] += std::fabs(col[a][q]) * e;
          }
      }
      for (int a = 0; a < 4; ++a)
        for (int q = 0; q < 7; ++q) N[7 * (size_t)t.vi[a] + q] += (double)cnt[r];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI for the test suite (ctypes).  prec: 32 -> float, 64 -> double.
// cams: float32 [n_views, 22]; params: float32 [7] =
// (tile_w, tile_h, alpha_min, alpha_clamp, t_min, prefilter_tf, s).
// pix: int32 [npix, 3] = (view, i, j).  out: float64 [npix, 8].
// ---------------------------------------------------------------------------
extern "C" {

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Threads of the oracle's parallel loops from now on (n >= 1).
int oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

int oracle_render(int prec, const double* verts, const int* tets, const double* sdf, const double* colors,
                  int V, int K, const float* cams, int nv, const float* params, const int* pix, long npix,
                  double* out, int* nblend, double* tfinal) {
  Params P = load_params(params);
  if (prec == 32) {
    Inputs<float> in;
    load_inputs(in, verts, tets, sdf, colors, V, K);
    render_impl(in.sc, cams, nv, P, pix, npix, out, nullptr, nblend, tfinal);
  } else if (prec == 64) {
    Inputs<double> in;
    load_inputs(in, verts, tets, sdf, colors, V, K);
    render_impl(in.sc, cams, nv, P, pix, npix, out, nullptr, nblend, tfinal);
  } else {
    return -1;
  }
  return 0;
}

// Running error bound of the forward: out = float64 value, bound = first-order
// bound on a float32 evaluation's distance from it (per channel).
int oracle_render_errbound(const double* verts, const int* tets, const double* sdf, const double* colors, int V,
                           int K, const float* cams, int nv, const float* params, const int* pix, long npix,
                           double* out, double* bound) {
  Params P = load_params(params);
  Inputs<Rerr> in;
  load_inputs(in, verts, tets, sdf, colors, V, K);
  render_impl(in.sc, cams, nv, P, pix, npix, out, bound, nullptr, nullptr);
  return 0;
}

// Eq. 1 (stable form) with its running error bound.
double oracle_alpha_errbound(double fprev, double fnext, double s, double* bound) {
  Rerr a = alpha_eq1<Rerr>(Rerr(fprev), Rerr(fnext), Rerr(s));
  *bound = a.e;
  return a.v;
}

// Forward-mode derivative: out = value, tout = directional derivative along
// (tverts, tsdf, tcolors).  Any tangent pointer may be null.
int oracle_render_dual(const double* verts, const int* tets, const double* sdf, const double* colors, int V,
                       int K, const double* tverts, const double* tsdf, const double* tcolors, const float* cams,
                       int nv, const float* params, const int* pix, long npix, double* out, double* tout) {
  Params P = load_params(params);
  Inputs<Dual> in;
  load_inputs<Dual>(in, verts, tets, sdf, colors, V, K, tverts, tsdf, tcolors);
  render_impl(in.sc, cams, nv, P, pix, npix, out, tout, nullptr, nullptr);
  return 0;
}

int oracle_backward(int prec, const double* verts, const int* tets, const double* sdf, const double* colors,
                    int V, int K, const float* cams, int nv, const float* params, const int* pix, long npix,
                    const double* dout, double* dverts, double* dsdf, double* dcolors) {
  Params P = load_params(params);
  if (prec == 32) {
    Inputs<float> in;
    load_inputs(in, verts, tets, sdf, colors, V, K);
    backward_impl(in.sc, cams, nv, P, pix, npix, dout, dverts, dsdf, dcolors);
  } else if (prec == 64) {
    Inputs<double> in;
    load_inputs(in, verts, tets, sdf, colors, V, K);
    backward_impl(in.sc, cams, nv, P, pix, npix, dout, dverts, dsdf, dcolors);
  } else {
    return -1;
  }
  return 0;
}

// Error budget of a float32 backward for the upstream gradient dout (see
// budget_impl): A, E, N are float64 [V, 7] = (dverts xyz, dsdf, dcolors xyz).
int oracle_backward_budget(const double* verts, const int* tets, const double* sdf, const double* colors, int V,
                           int K, const float* cams, int nv, const float* params, const int* pix, long npix,
                           const double* dout, double* A, double* E, double* N) {
  Params P = load_params(params);
  budget_impl(verts, tets, sdf, colors, V, K, cams, nv, P, pix, npix, dout, A, E, N);
  return 0;
}

// Per-tet view-independent data.  keep: uint8 [K]; amax32: float32 alpha_max
// used by the decision; normal/color/grad: float64 [K,3] (zero for dropped tets).
int oracle_prefilter(int prec, const double* verts, const int* tets, const double* sdf, const double* colors,
                     int V, int K, const float* params, uint8_t* keep, float* amax32, double* normal,
                     double* color, double* grad) {
  Params P = load_params(params);
  for (int k = 0; k < K; ++k) {
    float ff[4];
    for (int i = 0; i < 4; ++i) ff[i] = (float)sdf[tets[4 * (size_t)k + i]];
    keep[k] = keep_decision(ff[0], ff[1], ff[2], ff[3], P.s, P.prefilter_tf, amax32 ? amax32 + k : nullptr);
  }
  auto fill = [&](auto tag) {
    using R = decltype(tag);
    Inputs<R> in;
    load_inputs(in, verts, tets, sdf, colors, V, K);
    std::vector<KTet<R>> kt = prefilter(in.sc, P);
    std::memset(normal, 0, sizeof(double) * 3 * (size_t)K);
    std::memset(color, 0, sizeof(double) * 3 * (size_t)K);
    if (grad) std::memset(grad, 0, sizeof(double) * 3 * (size_t)K);
    for (auto& t : kt)
      for (int j = 0; j < 3; ++j) {
        normal[3 * (size_t)t.id + j] = val(t.n[j]);
        color[3 * (size_t)t.id + j] = val(t.c[j]);
        if (grad) grad[3 * (size_t)t.id + j] = val(t.g[j]);
      }
  };
  if (prec == 32) fill(0.0f);
  else if (prec == 64) fill(0.0);
  else return -1;
  (void)V;
  return 0;
}

// Binning reference (float32 decisions only): entries (view tile id, z bits,
// tet id) for every kept, unculled tet and every tile its pixel rectangle
// touches, emitted in ascending tet id and stably sorted by (tile, z bits).
// Global tile ids concatenate the views' row-major tile grids.  Returns the
// entry count E; arrays are written only if cap >= E.  ranges: int32
// [total_tiles, 2] half-open [start, end), (0,0) for empty tiles.
long oracle_binning(const double* verts, const int* tets, const double* sdf, int V, int K, const float* cams,
                    int nv, const float* params, long cap, int* tile, uint32_t* zbits, int* tet, int* ranges,
                    int* rect /* [nv, K, 4] or null: i0,i1,j0,j1 (-1 if dropped/culled) */) {
  Params P = load_params(params);
  std::vector<double> colors(3 * (size_t)V, 0.0);
  Inputs<float> in;
  load_inputs(in, verts, tets, sdf, colors.data(), V, K);
  std::vector<KTet<float>> kt = prefilter(in.sc, P);
  struct Ent { int tile; uint32_t z; int tet; };
  std::vector<Ent> ents;
  long tile_off = 0;
  if (rect) for (size_t q = 0; q < 4 * (size_t)nv * K; ++q) rect[q] = -1;
  for (int v = 0; v < nv; ++v) {
    Cam c = load_cam(cams + 22 * (size_t)v);
    int tx_n = (c.W + P.tile_w - 1) / P.tile_w, ty_n = (c.H + P.tile_h - 1) / P.tile_h;
    for (auto& t : kt) {
      Bin b = bin_tet(t, c);
      if (b.culled) continue;
      if (rect) {
        int* r = rect + 4 * ((size_t)v * K + t.id);
        r[0] = b.i0; r[1] = b.i1; r[2] = b.j0; r[3] = b.j1;
      }
      for (int ty = b.j0 / P.tile_h; ty <= b.j1 / P.tile_h; ++ty)
        for (int tx = b.i0 / P.tile_w; tx <= b.i1 / P.tile_w; ++tx)
          ents.push_back({(int)(tile_off + (long)ty * tx_n + tx), b.zbits, t.id});
    }
    tile_off += (long)tx_n * ty_n;
  }
  std::stable_sort(ents.begin(), ents.end(), [](const Ent& a, const Ent& b) {
    return a.tile != b.tile ? a.tile < b.tile : a.z < b.z;
  });
  long E = (long)ents.size();
  if (cap >= E) {
    for (long e = 0; e < E; ++e) { tile[e] = ents[e].tile; zbits[e] = ents[e].z; tet[e] = ents[e].tet; }
    if (ranges) {
      for (long t = 0; t < tile_off; ++t) ranges[2 * t] = ranges[2 * t + 1] = 0;
      for (long e = 0; e < E; ++e) {
        int t = ents[e].tile;
        if (e == 0 || ents[e - 1].tile != t) ranges[2 * t] = (int)e;
        ranges[2 * t + 1] = (int)e + 1;
      }
    }
  }
  return E;
}

// Trace of one pixel: the tets blended, in order, with their alpha (after the
// clamp), transmittance before them, raw alpha, entry/exit SDF values and
// entry depth.
int oracle_pixel_trace(int prec, const double* verts, const int* tets, const double* sdf, const double* colors,
                       int V, int K, const float* cams, int nv, const float* params, int view, int i, int j,
                       int cap, int* tet_id, double* alpha, double* T, double* alpha_raw, double* fprev,
                       double* fnext, double* zin) {
  Params P = load_params(params);
  auto run = [&](auto tag) -> int {
    using R = decltype(tag);
    Inputs<R> in;
    load_inputs(in, verts, tets, sdf, colors, V, K);
    Prepared<R> pp;
    prepare(in.sc, cams, nv, P, pp);
    PixelResult<R> pr;
    shade_pixel(pp.kt, pp.vt[view], pp.cams[view], P, i, j, pr, true);
    int n = (int)pr.list.size();
    for (int q = 0; q < n && q < cap; ++q) {
      tet_id[q] = pr.list[q].tet_id;
      alpha[q] = val(pr.list[q].a);
      T[q] = val(pr.list[q].T);
      alpha_raw[q] = val(pr.list[q].hit.alpha);
      fprev[q] = val(pr.list[q].hit.in.f);
      fnext[q] = val(pr.list[q].hit.out.f);
      zin[q] = val(pr.list[q].hit.in.z);
    }
    return n;
  };
  if (prec == 32) return run(0.0f);
  if (prec == 64) return run(0.0);
  return -1;
}

// Threshold decisions of one pixel's walk (the skip, clamp and stop tests of
// every candidate it reaches, the one that stops it included), each with the
// float64 value decided on and its running error bound (how far a float32
// evaluation of the same operations can be from it).  Returns the number of
// decisions; writes at most cap.
int oracle_pixel_decisions(const double* verts, const int* tets, const double* sdf, const double* colors, int V,
                           int K, const float* cams, int nv, const float* params, int view, int i, int j, int cap,
                           int* kind, double* value, double* bound, double* threshold) {
  Params P = load_params(params);
  Inputs<Rerr> in;
  load_inputs(in, verts, tets, sdf, colors, V, K);
  Prepared<Rerr> pp;
  prepare(in.sc, cams, nv, P, pp);
  PixelResult<Rerr> pr;
  std::vector<Decision<Rerr>> log;
  shade_pixel(pp.kt, pp.vt[view], pp.cams[view], P, i, j, pr, false, &log);
  int n = (int)log.size();
  for (int q = 0; q < n && q < cap; ++q) {
    kind[q] = log[q].kind;
    value[q] = log[q].value.v;
    bound[q] = log[q].value.e;
    threshold[q] = log[q].threshold;
  }
  return n;
}

// One tet against one pixel centre from already-projected data:
// px,py: projected vertices, Z: camera depths, f: SDF.  out[6] =
// (hit, f_prev, f_next, z_entry, z_exit, alpha).
int oracle_tet_pixel(const double* px, const double* py, const double* Z, const double* f, double qx, double qy,
                     double s, double* out) {
  TetHit<double> th;
  bool hit = tet_pixel<double>(px, py, Z, f, qx, qy, s, th);
  out[0] = hit ? 1.0 : 0.0;
  out[1] = hit ? th.in.f : 0.0;
  out[2] = hit ? th.out.f : 0.0;
  out[3] = hit ? th.in.z : 0.0;
  out[4] = hit ? th.out.z : 0.0;
  out[5] = hit ? th.alpha : 0.0;
  return 0;
}

// Eq. 1 in the stable form, float64 (for closed-form pins).
double oracle_alpha(double fprev, double fnext, double s) { return alpha_eq1<double>(fprev, fnext, s); }
float oracle_alpha_f32(float fprev, float fnext, float s) { return alpha_eq1<float>(fprev, fnext, s); }

}  // extern "C"
