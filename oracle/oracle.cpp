// Plain FP64 CPU oracle of the differentiable path tracer.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
// reference that the HIP library is checked against.  It shares no code,
// header, table or constant generator with the HIP library; only the seeded
// scene data (plain arrays) is common to both.  It may be used by the tests,
// by the smoke check and by the bench's CPU-baseline leg, never by the
// product path.
//
// What it computes (Dr.Jit paper, Sec. "Physically Based Differentiable
// Rendering" and Fig. "prb-structure"): a Monte Carlo path tracer (megakernel
// #1 of the PRB decomposition) producing a primal image with a box
// reconstruction filter, and the reverse-mode derivative of that estimator
// with respect to texel albedos and per-material GGX roughness, taken with
// detached sampling (Sec. "AD tape surgery": only the BSDF value f is attached,
// every sampling decision is held fixed).  The derivative is computed in the
// plain way -- each path is stored and swept backwards accumulating suffix
// radiance -- and, independently, by forward-mode sparse dual numbers.  Path
// replay (recovering the suffix by subtraction) is what the GPU does; the
// oracle does not replay.
//
// All arithmetic is double precision.  Scene data arrive as float32 and are
// widened exactly.  Conventions the paper leaves open (depth counting, RNG
// stream layout, BSDF formulas, emitters, MIS) follow the readings listed in
// the design notes; each function states which passage or definition it
// follows.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

namespace orc {

static const double kPi = 3.14159265358979323846;
static const double kInf = std::numeric_limits<double>::infinity();

// ---------------------------------------------------------------------------
// small vector type
// ---------------------------------------------------------------------------
struct V3 {
  double x, y, z;
  V3() : x(0), y(0), z(0) {}
  V3(double a, double b, double c) : x(a), y(b), z(c) {}
  double operator[](int i) const { return i == 0 ? x : (i == 1 ? y : z); }
};
static inline V3 operator+(V3 a, V3 b) { return V3(a.x + b.x, a.y + b.y, a.z + b.z); }
static inline V3 operator-(V3 a, V3 b) { return V3(a.x - b.x, a.y - b.y, a.z - b.z); }
static inline V3 operator*(V3 a, double s) { return V3(a.x * s, a.y * s, a.z * s); }
static inline V3 operator*(double s, V3 a) { return a * s; }
static inline V3 operator-(V3 a) { return V3(-a.x, -a.y, -a.z); }
static inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline V3 cross(V3 a, V3 b) {
  return V3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static inline double length(V3 a) { return std::sqrt(dot(a, a)); }
static inline V3 normalize(V3 a) { return a * (1.0 / length(a)); }

struct RGB {
  double c[3];
  RGB() { c[0] = c[1] = c[2] = 0; }
  RGB(double a, double b, double d) { c[0] = a; c[1] = b; c[2] = d; }
  double& operator[](int i) { return c[i]; }
  double operator[](int i) const { return c[i]; }
};
static inline RGB operator+(RGB a, RGB b) { return RGB(a[0] + b[0], a[1] + b[1], a[2] + b[2]); }
static inline RGB operator-(RGB a, RGB b) { return RGB(a[0] - b[0], a[1] - b[1], a[2] - b[2]); }
static inline RGB operator*(RGB a, RGB b) { return RGB(a[0] * b[0], a[1] * b[1], a[2] * b[2]); }
static inline RGB operator*(RGB a, double s) { return RGB(a[0] * s, a[1] * s, a[2] * s); }
static inline bool is_zero(RGB a) { return a[0] == 0 && a[1] == 0 && a[2] == 0; }

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).
// Ten rounds; each round multiplies words 0 and 2 by the two Philox
// multipliers, xors the high halves with the other words and the round key,
// and bumps the key by the two Weyl constants.
// ---------------------------------------------------------------------------
static inline void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                                 uint32_t out[4]) {
  const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = M0 * (uint64_t)c0;
    uint64_t p1 = M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0; k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Uniform in [0,1): the top 24 bits scaled by 2^-24 (exact in FP32 and FP64).
static inline double u01(uint32_t r) { return (double)(r >> 8) * (1.0 / 16777216.0); }
// Discrete choice in [0,n) from a raw 32-bit word (exact integer arithmetic).
static inline uint32_t pick(uint32_t r, uint32_t n) { return (uint32_t)(((uint64_t)r * n) >> 32); }

// Random-number stream of one sample: key = seed, counter = (g_lo, g_hi, b, dim).
struct Stream {
  uint32_t key[2];
  uint32_t g_lo, g_hi;
  void block(uint32_t b, uint32_t dim, uint32_t out[4]) const {
    uint32_t ctr[4] = {g_lo, g_hi, b, dim};
    philox4x32_10(ctr, key, out);
  }
};
static const uint32_t kCameraBlock = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// scene
// ---------------------------------------------------------------------------
enum { BSDF_NULL = 0, BSDF_DIFFUSE = 1, BSDF_DIFFUSE_TEXTURED = 2, BSDF_CONDUCTOR = 3,
       BSDF_DIELECTRIC = 4, BSDF_PLASTIC = 5, BSDF_TWOSIDED = 6, BSDF_MASK = 7 };
enum { EM_AREA = 0, EM_ENV = 1, EM_DIRECTIONAL = 2 };
enum { FLAG_NO_NEE = 1 };

struct Material {
  int type, texture, rough_slot;
  RGB albedo, f0;
  double alpha, eta, opacity;
};

struct Emitter {
  int type;
  V3 p0, e1, e2, n;  // area quad (n = unit normal of the front side); directional: p0 = direction
  double area;
  RGB radiance;
};

// Optional acceleration structure (see "Acceleration" below).
struct BvhNode {
  double lo[3], hi[3];
  int a, b;  // interior: the two children; leaf: a = first index into order, b = -count
};
struct Bvh {
  std::vector<BvhNode> nodes;
  std::vector<int> order;  // triangle ids, leaf by leaf
};

struct Scene {
  Bvh bvh;                 // empty: every query loops over all triangles
  std::vector<V3> pos;
  std::vector<double> uv;  // 2 per vertex
  std::vector<int> idx;    // 3 per triangle
  std::vector<int> tri_mat, tri_em;
  std::vector<Material> mats;
  std::vector<Emitter> ems;
  std::vector<int> tex_w, tex_h;
  int n_rough = 0;
  // environment map (latitude-longitude, row 0 = +y)
  int env_w = 0, env_h = 0;
  std::vector<double> env;       // [h][w][3]
  std::vector<double> env_cdf_row;   // [h+1]
  std::vector<double> env_cdf_col;   // [h][w+1]
  std::vector<double> env_weight;   // [h][w]
  double env_total = 0;
  int env_index = -1;
  double eps = 0;  // ray-spawn offset
  int n_tris() const { return (int)tri_mat.size(); }
};

struct Params {
  const float* const* tex;  // per texture [H][W][3]
  const float* rough;       // [n_rough]
};

// ---------------------------------------------------------------------------
// Decisions within FP32 reach.  A float32 implementation of the same
// estimator follows the same path as this double-precision one except where
// a discrete decision (texel index, environment cell, CDF bin, Russian
// roulette, lobe choice, which triangle a ray hits or grazes) is taken within
// float32 rounding of its threshold.  When a caller asks, such samples are
// flagged so comparisons can set them aside (and count them).
// ---------------------------------------------------------------------------
static thread_local bool* t_amb = nullptr;
static const double kTolUV = 3e-7;     // texture coordinate (uv units) to a texel edge
static const double kTolU = 2e-6;      // uniform vs a computed threshold
static const double kTolAngle = 2e-6;  // direction angle (radians) to an environment cell edge
static const double kTolBary = 2e-5;   // ray to a triangle edge (normalised barycentric)
static const double kTolT = 1e-6;      // relative distance between two hits
static inline void flag_if(bool c) {
  if (c && t_amb) *t_amb = true;
}
// distance of x to the nearest integer in [1, n-1] (the interior cell edges)
static inline double edge_dist(double x, int n) {
  double k = std::floor(x + 0.5);
  if (k < 1 || k > n - 1) return 1e300;
  return std::fabs(x - k);
}

// ---------------------------------------------------------------------------
// Intersection: watertight ray/triangle test of Woop, Benthin and Wald (JCGT
// 2013) evaluated in double precision, no culling, t in (tmin, tmax).  The
// closest hit is the minimum over ALL triangles (brute force); ties go to the
// lowest triangle id.
// ---------------------------------------------------------------------------
struct RayPre {
  int kx, ky, kz;
  double sx, sy, sz;
};
static RayPre ray_pre(V3 d) {
  RayPre r;
  double ax = std::fabs(d.x), ay = std::fabs(d.y), az = std::fabs(d.z);
  r.kz = 0;
  if (ay > ax) r.kz = 1;
  if (az > (r.kz == 0 ? ax : ay)) r.kz = 2;
  r.kx = (r.kz + 1) % 3;
  r.ky = (r.kx + 1) % 3;
  if (d[r.kz] < 0) std::swap(r.kx, r.ky);
  r.sx = d[r.kx] / d[r.kz];
  r.sy = d[r.ky] / d[r.kz];
  r.sz = 1.0 / d[r.kz];
  return r;
}

static bool tri_hit(const Scene& s, int prim, V3 o, const RayPre& rp, double tmin, double tmax,
                    double* t_out, double b_out[3]) {
  V3 A = s.pos[s.idx[3 * prim]] - o;
  V3 B = s.pos[s.idx[3 * prim + 1]] - o;
  V3 C = s.pos[s.idx[3 * prim + 2]] - o;
  double Ax = A[rp.kx] - rp.sx * A[rp.kz], Ay = A[rp.ky] - rp.sy * A[rp.kz];
  double Bx = B[rp.kx] - rp.sx * B[rp.kz], By = B[rp.ky] - rp.sy * B[rp.kz];
  double Cx = C[rp.kx] - rp.sx * C[rp.kz], Cy = C[rp.ky] - rp.sy * C[rp.kz];
  double U = Cx * By - Cy * Bx;
  double V = Ax * Cy - Ay * Cx;
  double W = Bx * Ay - By * Ax;
  if ((U < 0 || V < 0 || W < 0) && (U > 0 || V > 0 || W > 0)) return false;
  double det = U + V + W;
  if (det == 0) return false;
  double Az = rp.sz * A[rp.kz], Bz = rp.sz * B[rp.kz], Cz = rp.sz * C[rp.kz];
  double T = U * Az + V * Bz + W * Cz;
  double t = T / det;
  if (!(t > tmin && t < tmax)) return false;
  *t_out = t;
  b_out[0] = U / det;
  b_out[1] = V / det;
  b_out[2] = W / det;
  return true;
}

struct Hit {
  int prim = -1;
  double t = kInf;
  double b[3] = {0, 0, 0};
};

// ---------------------------------------------------------------------------
// Acceleration.  The definition of every ray query is the loop over all
// triangles; for the ~1M-triangle scenes a binary bounding-volume hierarchy
// may stand in for that loop without changing any answer.  Each triangle's
// box is padded by 1e-4 of its own extent plus 1e-9 of the scene's, so any
// point on the triangle, or within the ambiguity tolerances of it (which
// reach at most a few 1e-5 of its extent), lies inside every box on the way
// to it, well beyond the rounding of the slab test.  A query walks the boxes
// its ray meets within its (padded) distance interval and examines their
// triangles with exactly the per-triangle code of the loop; only triangles
// the ray cannot reach are left out, and ties are resolved by id as the loop
// resolves them, so the answers are the loop's bit for bit (the tests check
// this on scenes small enough to loop over).
// ---------------------------------------------------------------------------
static int bvh_build_range(Scene& s, const std::vector<double>& blo, const std::vector<double>& bhi,
                           const std::vector<double>& cen, int first, int count) {
  Bvh& B = s.bvh;
  const int id = (int)B.nodes.size();
  B.nodes.push_back(BvhNode());
  BvhNode nd;
  double clo[3] = {kInf, kInf, kInf}, chi[3] = {-kInf, -kInf, -kInf};
  for (int a = 0; a < 3; ++a) { nd.lo[a] = kInf; nd.hi[a] = -kInf; }
  for (int k = first; k < first + count; ++k) {
    const int t = B.order[k];
    for (int a = 0; a < 3; ++a) {
      nd.lo[a] = std::min(nd.lo[a], blo[3 * (size_t)t + a]);
      nd.hi[a] = std::max(nd.hi[a], bhi[3 * (size_t)t + a]);
      clo[a] = std::min(clo[a], cen[3 * (size_t)t + a]);
      chi[a] = std::max(chi[a], cen[3 * (size_t)t + a]);
    }
  }
  int axis = 0;
  for (int a = 1; a < 3; ++a)
    if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
  if (count <= 4 || !(chi[axis] > clo[axis])) {
    nd.a = first;
    nd.b = -count;
    B.nodes[id] = nd;
    return id;
  }
  // median split of the centroids along the widest axis
  const int half = count / 2;
  std::nth_element(B.order.begin() + first, B.order.begin() + first + half,
                   B.order.begin() + first + count, [&](int x, int y) {
                     return cen[3 * (size_t)x + axis] < cen[3 * (size_t)y + axis];
                   });
  nd.a = bvh_build_range(s, blo, bhi, cen, first, half);
  nd.b = bvh_build_range(s, blo, bhi, cen, first + half, count - half);
  B.nodes[id] = nd;
  return id;
}

static void bvh_build(Scene& s) {
  const int n = s.n_tris();
  s.bvh.nodes.clear();
  s.bvh.order.resize(n);
  if (n == 0) return;
  double slo[3] = {kInf, kInf, kInf}, shi[3] = {-kInf, -kInf, -kInf};
  for (const V3& p : s.pos)
    for (int a = 0; a < 3; ++a) { slo[a] = std::min(slo[a], p[a]); shi[a] = std::max(shi[a], p[a]); }
  const double sext = std::max(shi[0] - slo[0], std::max(shi[1] - slo[1], shi[2] - slo[2]));
  std::vector<double> blo(3 * (size_t)n), bhi(3 * (size_t)n), cen(3 * (size_t)n);
  for (int t = 0; t < n; ++t) {
    double lo[3] = {kInf, kInf, kInf}, hi[3] = {-kInf, -kInf, -kInf};
    for (int v = 0; v < 3; ++v) {
      const V3& p = s.pos[s.idx[3 * (size_t)t + v]];
      for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], p[a]); hi[a] = std::max(hi[a], p[a]); }
    }
    const double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    const double pad = 1e-4 * ext + 1e-9 * sext;
    for (int a = 0; a < 3; ++a) {
      blo[3 * (size_t)t + a] = lo[a] - pad;
      bhi[3 * (size_t)t + a] = hi[a] + pad;
      cen[3 * (size_t)t + a] = 0.5 * (lo[a] + hi[a]);
    }
    s.bvh.order[t] = t;
  }
  s.bvh.nodes.reserve((size_t)n + 2);
  bvh_build_range(s, blo, bhi, cen, 0, n);
}

// Whether the ray o + t d meets the node's box for some t in [t0, t1].
static bool box_meets(const BvhNode& N, V3 o, V3 d, double t0, double t1) {
  double tn = t0, tf = t1;
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0) {
      if (o[a] < N.lo[a] || o[a] > N.hi[a]) return false;
      continue;
    }
    double ta = (N.lo[a] - o[a]) / d[a], tb = (N.hi[a] - o[a]) / d[a];
    if (ta > tb) std::swap(ta, tb);
    tn = std::max(tn, ta);
    tf = std::min(tf, tb);
    if (tn > tf) return false;
  }
  return true;
}

// Calls f(triangle) for every triangle of every leaf whose box the ray
// meets within [t0, *t1]; *t1 may shrink while the walk goes on.  f returns
// true to stop the walk.  Without a hierarchy: every triangle, in id order.
template <class F>
static void for_reachable(const Scene& s, V3 o, V3 d, double t0, const double* t1, F f) {
  const Bvh& B = s.bvh;
  if (B.nodes.empty()) {
    for (int i = 0; i < s.n_tris(); ++i)
      if (f(i)) return;
    return;
  }
  int stack[128];  // median splits: depth <= log2(n / 4) + 2 < 64 for any int n
  int sp = 0;
  stack[sp++] = 0;
  while (sp > 0) {
    const BvhNode& N = B.nodes[stack[--sp]];
    if (!box_meets(N, o, d, t0, *t1)) continue;
    if (N.b < 0) {
      for (int k = 0; k < -N.b; ++k)
        if (f(B.order[N.a + k])) return;
      continue;
    }
    stack[sp++] = N.b;
    stack[sp++] = N.a;
  }
}

// The distance interval a query with tolerance 1e-6 x max(1, |t|) reaches:
// [lo, hi] widened by 1e-5 x max(1, |lo|, |hi|).
static inline void widen(double* lo, double* hi) {
  const double w = 1e-5 * std::max(1.0, std::max(std::fabs(*lo), std::fabs(*hi)));
  *lo -= w;
  *hi += w;
}

// Flag the ray if any triangle's edge passes within kTolBary of it in front
// of t_lim, or another triangle is hit within kTolT of t_hit.
static void scan_edges(const Scene& s, V3 o, V3 d, double tmin, double t_lim, int hit_prim,
                       bool skip_null) {
  double w0 = tmin, w1 = t_lim;
  widen(&w0, &w1);
  for_reachable(s, o, d, w0, &w1, [&](int j) -> bool {
    if (skip_null && s.mats[s.tri_mat[j]].type == 0) return false;
    V3 p0 = s.pos[s.idx[3 * j]], p1 = s.pos[s.idx[3 * j + 1]], p2 = s.pos[s.idx[3 * j + 2]];
    V3 e1 = p1 - p0, e2 = p2 - p0, pv = cross(d, e2);
    double det = dot(e1, pv);
    if (std::fabs(det) <= 1e-14 * length(e1) * length(e2)) return false;
    V3 tv = o - p0;
    double bu = dot(tv, pv) / det;
    V3 qv = cross(tv, e1);
    double bv = dot(d, qv) / det;
    double tt = dot(e2, qv) / det;
    double tol_t = kTolT * std::max(1.0, std::fabs(tt));
    if (!(tt > tmin - tol_t && tt < t_lim + tol_t)) return false;
    double bmin = std::min(std::min(bu, bv), 1.0 - bu - bv);
    bool flag = std::fabs(bmin) < kTolBary ||
                (bmin > 0 && j != hit_prim && std::fabs(tt - t_lim) <= tol_t) ||
                (bmin > 0 && std::fabs(tt - tmin) <= tol_t);
    if (flag) flag_if(true);
    return flag;
  });
}

// Closest hit: the minimum t over all triangles, ties to the lowest id.
static Hit closest_hit(const Scene& s, V3 o, V3 d, double tmin, double tmax) {
  RayPre rp = ray_pre(d);
  Hit h;
  double best = tmax;
  for_reachable(s, o, d, tmin, &best, [&](int i) -> bool {
    double t, b[3];
    if (tri_hit(s, i, o, rp, tmin, tmax, &t, b) && (t < best || (t == best && i < h.prim))) {
      h.prim = i; h.t = t; h.b[0] = b[0]; h.b[1] = b[1]; h.b[2] = b[2];
      best = t;
    }
    return false;
  });
  if (t_amb) scan_edges(s, o, d, tmin, h.prim >= 0 ? h.t : tmax, h.prim, false);
  return h;
}

// Any hit on a triangle whose material is not the pass-through (null) BSDF.
static bool occluded(const Scene& s, V3 o, V3 d, double tmax) {
  if (t_amb) scan_edges(s, o, d, 0.0, tmax, -1, true);
  RayPre rp = ray_pre(d);
  bool hit = false;
  const double t1 = tmax;
  for_reachable(s, o, d, 0.0, &t1, [&](int i) -> bool {
    if (s.mats[s.tri_mat[i]].type == BSDF_NULL) return false;
    double t, b[3];
    hit = tri_hit(s, i, o, rp, 0.0, tmax, &t, b);
    return hit;
  });
  return hit;
}

// Offset origin of a ray leaving point p along d: to the side of the
// geometric normal that d points into.
static inline V3 spawn(const Scene& s, V3 p, V3 n_g, V3 d) {
  double sg = dot(d, n_g) >= 0 ? 1.0 : -1.0;
  return p + n_g * (sg * s.eps);
}

// ---------------------------------------------------------------------------
// Orthonormal basis around a unit normal: the branchless construction of
// Duff, Burgess, Christensen, Hery, Kensler, Liani, Villemin (JCGT 2017).
// ---------------------------------------------------------------------------
struct Frame {
  V3 s, t, n;
  V3 to_local(V3 v) const { return V3(dot(v, s), dot(v, t), dot(v, n)); }
  V3 to_world(V3 v) const { return s * v.x + t * v.y + n * v.z; }
};
static Frame make_frame(V3 n) {
  double sign = std::copysign(1.0, n.z);
  double a = -1.0 / (sign + n.z);
  double b = n.x * n.y * a;
  Frame f;
  f.n = n;
  f.s = V3(1.0 + sign * n.x * n.x * a, sign * b, -sign * n.x);
  f.t = V3(b, sign + n.y * n.y * a, -n.y);
  return f;
}

// ---------------------------------------------------------------------------
// Microfacet terms: GGX distribution and separable Smith shadowing (Walter,
// Marschner, Li, Torrance, EGSR 2007), alpha = roughness (not squared).
// Templated on the scalar so the roughness derivative can be checked by
// complex-step differentiation.
// ---------------------------------------------------------------------------
template <class T>
static T ggx_D(T alpha, double cos_m) {
  if (cos_m <= 0) return T(0);
  double c2 = cos_m * cos_m;
  T a2 = alpha * alpha;
  T den = c2 * (a2 - 1.0) + 1.0;
  return a2 / (kPi * den * den);
}
template <class T>
static T ggx_G1(T alpha, double v_dot_m, double v_dot_n) {
  if (v_dot_m * v_dot_n <= 0) return T(0);
  double c2 = v_dot_n * v_dot_n;
  double tan2 = std::max(0.0, 1.0 - c2) / c2;
  return 2.0 / (1.0 + std::sqrt(1.0 + alpha * alpha * tan2));
}
// d ln D / d alpha and d ln G1 / d alpha, written out analytically.
static double ggx_dlnD(double alpha, double cos_m) {
  double c2 = cos_m * cos_m;
  double den = c2 * (alpha * alpha - 1.0) + 1.0;
  return 2.0 / alpha - 4.0 * alpha * c2 / den;
}
static double ggx_dlnG1(double alpha, double v_dot_n) {
  double c2 = v_dot_n * v_dot_n;
  double tan2 = std::max(0.0, 1.0 - c2) / c2;
  double r = std::sqrt(1.0 + alpha * alpha * tan2);
  return -(alpha * tan2 / r) / (1.0 + r);
}
// Visible-normal-free sampling of m proportional to D(m) cos(theta_m):
// tan^2 theta = alpha^2 u / (1-u), phi = 2 pi u'.
static V3 ggx_sample_m(double alpha, double u1, double u2) {
  double cos2 = (1.0 - u1) / (1.0 + (alpha * alpha - 1.0) * u1);
  double ct = std::sqrt(cos2);
  double st = std::sqrt(std::max(0.0, 1.0 - cos2));
  double ph = 2.0 * kPi * u2;
  return V3(st * std::cos(ph), st * std::sin(ph), ct);
}

// Exact unpolarised Fresnel reflectance at a dielectric interface; cos_i >= 0
// is measured on the incident side, eta = n_transmitted / n_incident.
static double fresnel_dielectric(double cos_i, double eta) {
  double sin2_t = (1.0 - cos_i * cos_i) / (eta * eta);
  if (sin2_t >= 1.0) return 1.0;
  double cos_t = std::sqrt(1.0 - sin2_t);
  double rs = (cos_i - eta * cos_t) / (cos_i + eta * cos_t);
  double rp = (eta * cos_i - cos_t) / (eta * cos_i + cos_t);
  return 0.5 * (rs * rs + rp * rp);
}

static double schlick(double f0, double c) {
  double m = 1.0 - c;
  double m2 = m * m;
  return f0 + (1.0 - f0) * m2 * m2 * m;
}

// ---------------------------------------------------------------------------
// BSDFs.  eval() returns f(wi,wo)*|cos(theta_o)| per channel and the density
// with which sample() would generate wo; it also returns the derivatives of
// that value with respect to the attached parameters: the albedo channels
// (d/d rho_c of channel c) and the roughness (d/d alpha of each channel).
// wi points back along the incoming ray, both in the local frame (z = n_g).
// ---------------------------------------------------------------------------
struct Shading {
  const Material* m;
  RGB albedo;     // texture or constant
  double alpha;   // roughness slot or constant
};

struct Eval {
  RGB f;        // f * |cos theta_o|
  double pdf = 0;
  RGB d_albedo;  // d f_c / d rho_c
  RGB d_alpha;   // d f_c / d alpha
};

static void eval_lambert(const RGB& albedo, V3 wi, V3 wo, Eval* e) {
  if (wi.z <= 0 || wo.z <= 0) return;
  double k = wo.z / kPi;
  e->f = albedo * k;
  e->d_albedo = RGB(k, k, k);
  e->pdf = wo.z / kPi;
}

static double ggx_reflect_pdf(double alpha, V3 wo, V3 h) {
  return ggx_D<double>(alpha, h.z) * h.z / (4.0 * std::fabs(dot(wo, h)));
}

static Eval bsdf_eval(const Shading& sh, V3 wi, V3 wo) {
  Eval e;
  const Material& m = *sh.m;
  double a = sh.alpha;
  switch (m.type) {
    case BSDF_DIFFUSE:
    case BSDF_DIFFUSE_TEXTURED:
    case BSDF_MASK:
      eval_lambert(sh.albedo, wi, wo, &e);
      break;
    case BSDF_TWOSIDED:
      if (wi.z < 0) { wi.z = -wi.z; wo.z = -wo.z; }
      eval_lambert(sh.albedo, wi, wo, &e);
      break;
    case BSDF_CONDUCTOR: {
      if (wi.z <= 0 || wo.z <= 0) break;
      V3 h = normalize(wi + wo);
      double D = ggx_D<double>(a, h.z);
      double G = ggx_G1<double>(a, dot(wi, h), wi.z) * ggx_G1<double>(a, dot(wo, h), wo.z);
      double base = D * G / (4.0 * wi.z);
      double dl = ggx_dlnD(a, h.z) + ggx_dlnG1(a, wi.z) + ggx_dlnG1(a, wo.z);
      for (int c = 0; c < 3; ++c) {
        e.f[c] = schlick(m.f0[c], dot(wi, h)) * base;
        e.d_alpha[c] = e.f[c] * dl;
      }
      e.pdf = ggx_reflect_pdf(a, wo, h);
      break;
    }
    case BSDF_PLASTIC: {
      if (wi.z <= 0 || wo.z <= 0) break;
      V3 h = normalize(wi + wo);
      double D = ggx_D<double>(a, h.z);
      double G = ggx_G1<double>(a, dot(wi, h), wi.z) * ggx_G1<double>(a, dot(wo, h), wo.z);
      double spec = fresnel_dielectric(dot(wi, h), m.eta) * D * G / (4.0 * wi.z);
      double dl = ggx_dlnD(a, h.z) + ggx_dlnG1(a, wi.z) + ggx_dlnG1(a, wo.z);
      double Fi = fresnel_dielectric(wi.z, m.eta), Fo = fresnel_dielectric(wo.z, m.eta);
      double kd = (1.0 - Fi) * (1.0 - Fo) * wo.z / kPi;
      for (int c = 0; c < 3; ++c) {
        e.f[c] = spec + kd * sh.albedo[c];
        e.d_albedo[c] = kd;
        e.d_alpha[c] = spec * dl;
      }
      double ps = std::min(std::max(Fi, 0.1), 0.9);
      e.pdf = ps * ggx_reflect_pdf(a, wo, h) + (1.0 - ps) * wo.z / kPi;
      break;
    }
    case BSDF_DIELECTRIC: {
      double ci = wi.z, co = wo.z;
      if (ci == 0 || co == 0) break;
      double eta = ci > 0 ? m.eta : 1.0 / m.eta;  // n_other / n_incident
      bool reflect = ci * co > 0;
      V3 h = reflect ? normalize(wi + wo) : normalize(wi + wo * eta);
      if (h.z < 0) h = -h;
      double D = ggx_D<double>(a, h.z);
      double G = ggx_G1<double>(a, dot(wi, h), ci) * ggx_G1<double>(a, dot(wo, h), co);
      if (D == 0 || G == 0) break;
      double F = fresnel_dielectric(std::fabs(dot(wi, h)), eta);
      double dl = ggx_dlnD(a, h.z) + ggx_dlnG1(a, ci) + ggx_dlnG1(a, co);
      double val, pdf;
      if (reflect) {
        val = F * D * G / (4.0 * std::fabs(ci));
        pdf = F * D * h.z / (4.0 * std::fabs(dot(wo, h)));
      } else {
        double ih = dot(wi, h), oh = dot(wo, h);
        if (ih * oh >= 0) break;  // both on one side of the microfacet
        double den = ih + eta * oh;
        den *= den;
        val = std::fabs(ih) * std::fabs(oh) * (1.0 - F) * D * G / (std::fabs(ci) * den);
        pdf = (1.0 - F) * D * h.z * eta * eta * std::fabs(oh) / den;
      }
      e.f = RGB(val, val, val);
      e.d_alpha = RGB(val * dl, val * dl, val * dl);
      e.pdf = pdf;
      break;
    }
    default:
      break;
  }
  return e;
}

struct Sample {
  bool ok = false;
  V3 wo;
  Eval e;  // value, density and derivatives at the sampled direction
};

// Cosine-weighted hemisphere sample (the paper's ambient-occlusion example):
// phi = 2 pi u_a, sin^2 theta = u_b.
static V3 cosine_hemisphere(double ua, double ub) {
  double ph = 2.0 * kPi * ua;
  double r = std::sqrt(ub);
  return V3(std::cos(ph) * r, std::sin(ph) * r, std::sqrt(1.0 - ub));
}

static V3 reflect_about(V3 wi, V3 m) { return m * (2.0 * dot(wi, m)) - wi; }

static Sample bsdf_sample(const Shading& sh, V3 wi, double u1, double u2, double ulobe) {
  Sample s;
  const Material& m = *sh.m;
  double a = sh.alpha;
  switch (m.type) {
    case BSDF_DIFFUSE:
    case BSDF_DIFFUSE_TEXTURED:
    case BSDF_MASK:
      if (wi.z <= 0) return s;
      s.wo = cosine_hemisphere(u1, u2);
      break;
    case BSDF_TWOSIDED:
      s.wo = cosine_hemisphere(u1, u2);
      if (wi.z < 0) s.wo.z = -s.wo.z;
      break;
    case BSDF_CONDUCTOR: {
      if (wi.z <= 0) return s;
      V3 mm = ggx_sample_m(a, u1, u2);
      if (dot(wi, mm) <= 0) return s;
      s.wo = reflect_about(wi, mm);
      if (s.wo.z <= 0) return s;
      break;
    }
    case BSDF_PLASTIC: {
      if (wi.z <= 0) return s;
      double ps = std::min(std::max(fresnel_dielectric(wi.z, m.eta), 0.1), 0.9);
      flag_if(std::fabs(ulobe - ps) < kTolU);
      if (ulobe < ps) {
        V3 mm = ggx_sample_m(a, u1, u2);
        if (dot(wi, mm) <= 0) return s;
        s.wo = reflect_about(wi, mm);
        if (s.wo.z <= 0) return s;
      } else {
        s.wo = cosine_hemisphere(u1, u2);
      }
      break;
    }
    case BSDF_DIELECTRIC: {
      if (wi.z == 0) return s;
      double sg = wi.z > 0 ? 1.0 : -1.0;
      double eta = wi.z > 0 ? m.eta : 1.0 / m.eta;
      V3 mm = ggx_sample_m(a, u1, u2) * sg;  // microfacet normal on wi's side
      double c = dot(wi, mm);
      if (c <= 0) return s;
      double F = fresnel_dielectric(c, eta);
      flag_if(std::fabs(ulobe - F) < kTolU);
      if (ulobe < F) {
        s.wo = reflect_about(wi, mm);
        if (s.wo.z * sg <= 0) return s;
      } else {
        double sin2_t = (1.0 - c * c) / (eta * eta);
        if (sin2_t >= 1.0) return s;  // unreachable: F = 1 under total reflection
        double cos_t = std::sqrt(1.0 - sin2_t);
        s.wo = wi * (-1.0 / eta) + mm * (c / eta - cos_t);
        if (s.wo.z * sg >= 0) return s;
      }
      break;
    }
    default:
      return s;
  }
  s.e = bsdf_eval(sh, wi, s.wo);
  s.ok = s.e.pdf > 0 && !is_zero(s.e.f);
  return s;
}

// ---------------------------------------------------------------------------
// Emitters: one-sided quad area lights (uniform area sampling), latitude-
// longitude environment map (piecewise-constant 2D sampling on luminance
// times sin(theta)), directional lights.  Selection is uniform over all
// emitters.
// ---------------------------------------------------------------------------
static void env_dir_to_cell(const Scene& s, V3 d, int* row, int* col, double* sin_t) {
  double ct = std::min(1.0, std::max(-1.0, d.y));
  double th = std::acos(ct);
  double ph = std::atan2(d.z, d.x);
  if (ph < 0) ph += 2.0 * kPi;
  int c = (int)std::floor(ph / (2.0 * kPi) * s.env_w);
  int r = (int)std::floor(th / kPi * s.env_h);
  if (t_amb) {
    double st = std::sin(th);
    flag_if(edge_dist(th / kPi * s.env_h, s.env_h) * kPi / s.env_h < kTolAngle);
    double dph = std::min(std::fabs(ph - c * 2.0 * kPi / s.env_w),
                          std::fabs(ph - (c + 1) * 2.0 * kPi / s.env_w));
    flag_if(dph * std::max(st, 1e-12) < kTolAngle);
  }
  *col = std::min(std::max(c, 0), s.env_w - 1);
  *row = std::min(std::max(r, 0), s.env_h - 1);
  *sin_t = std::sin(th);
}

static RGB env_lookup(const Scene& s, V3 d) {
  int r, c;
  double st;
  env_dir_to_cell(s, d, &r, &c, &st);
  const double* p = &s.env[3 * ((size_t)r * s.env_w + c)];
  return RGB(p[0], p[1], p[2]);
}

static double env_pdf(const Scene& s, V3 d) {
  if (s.env_total <= 0) return 0;
  int r, c;
  double st;
  env_dir_to_cell(s, d, &r, &c, &st);
  if (st <= 0) return 0;
  double p_uv = s.env_weight[(size_t)r * s.env_w + c] / s.env_total * s.env_w * s.env_h;
  return p_uv / (2.0 * kPi * kPi * st);
}

// Largest i in [0, n) with cdf[i] <= u  (cdf has n+1 entries, cdf[0]=0, cdf[n]=1).
static int cdf_find(const double* cdf, int n, double u) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (cdf[mid] <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

static bool env_sample(const Scene& s, double u1, double u2, V3* d) {
  if (s.env_total <= 0) return false;
  int r = cdf_find(s.env_cdf_row.data(), s.env_h, u1);
  double r0 = s.env_cdf_row[r], r1 = s.env_cdf_row[r + 1];
  flag_if(std::fabs(u1 - r0) < kTolU || std::fabs(u1 - r1) < kTolU);
  double v = (r + (u1 - r0) / (r1 - r0)) / s.env_h;
  const double* cc = &s.env_cdf_col[(size_t)r * (s.env_w + 1)];
  int c = cdf_find(cc, s.env_w, u2);
  flag_if(std::fabs(u2 - cc[c]) < kTolU || std::fabs(u2 - cc[c + 1]) < kTolU);
  double u = (c + (u2 - cc[c]) / (cc[c + 1] - cc[c])) / s.env_w;
  double th = v * kPi, ph = u * 2.0 * kPi;
  *d = V3(std::sin(th) * std::cos(ph), std::cos(th), std::sin(th) * std::sin(ph));
  return true;
}

static void build_env(Scene& s) {
  int W = s.env_w, H = s.env_h;
  s.env_weight.assign((size_t)W * H, 0.0);
  s.env_cdf_row.assign(H + 1, 0.0);
  s.env_cdf_col.assign((size_t)H * (W + 1), 0.0);
  std::vector<double> rowsum(H, 0.0);
  double total = 0;
  for (int r = 0; r < H; ++r) {
    double st = std::sin(kPi * (r + 0.5) / H);
    for (int c = 0; c < W; ++c) {
      const double* p = &s.env[3 * ((size_t)r * W + c)];
      double y = 0.2126 * p[0] + 0.7152 * p[1] + 0.0722 * p[2];
      double w = std::max(y, 0.0) * st;
      s.env_weight[(size_t)r * W + c] = w;
      rowsum[r] += w;
    }
    total += rowsum[r];
  }
  s.env_total = total;
  if (total <= 0) return;
  double acc = 0;
  for (int r = 0; r < H; ++r) {
    acc += rowsum[r];
    s.env_cdf_row[r + 1] = acc / total;
    double* cc = &s.env_cdf_col[(size_t)r * (W + 1)];
    double a2 = 0;
    for (int c = 0; c < W; ++c) {
      a2 += s.env_weight[(size_t)r * W + c];
      cc[c + 1] = rowsum[r] > 0 ? a2 / rowsum[r] : (double)(c + 1) / W;
    }
    cc[W] = 1.0;
  }
  s.env_cdf_row[H] = 1.0;
}

static inline double power_heuristic(double a, double b) {
  double a2 = a * a, b2 = b * b;
  return a2 / (a2 + b2);
}

// ---------------------------------------------------------------------------
// Derivative bookkeeping.  A parameter key identifies a texel (texture,
// texel index) -- whose three channels are three parameters, channel c of the
// radiance depending on channel c of the albedo only -- or a roughness slot.
// ---------------------------------------------------------------------------
typedef uint64_t Key;
static inline Key texel_key(int tex, int64_t texel) {
  return (1ull << 63) | ((uint64_t)tex << 40) | (uint64_t)texel;
}
static inline Key rough_key(int slot) { return (uint64_t)slot; }
static inline bool is_texel(Key k) { return (k >> 63) != 0; }

struct Tangent {  // sparse: key -> per-channel derivative
  std::vector<std::pair<Key, RGB>> e;
  void add(Key k, const RGB& v) {
    for (auto& p : e) if (p.first == k) { p.second = p.second + v; return; }
    e.push_back({k, v});
  }
};

// What a vertex contributes and how its attached BSDF value depends on the
// parameters: for the NEE term and for the sampled continuation.
struct VertexRec {
  RGB emit;            // emission collected at this vertex (beta, Le, MIS included)
  RGB nee;             // next-event contribution
  RGB nee_coef;        // nee / f_nee per channel, so d nee = nee_coef * d f_nee
  Eval nee_eval;       // f and derivatives at the light direction
  bool has_bsdf = false;
  Eval bsdf_eval;      // f and derivatives at the sampled direction
  Key k_tex = 0; bool has_tex = false;
  Key k_rough = 0; bool has_rough = false;
};

struct Opts {
  int spp, max_depth, rr_depth;
  uint32_t flags;
  uint64_t seed;
};

struct ShadeCtx {
  Shading sh;
  Key k_tex = 0; bool has_tex = false;
  Key k_rough = 0; bool has_rough = false;
};

static ShadeCtx fetch_shading(const Scene& s, const Params& P, int mat, double u, double v) {
  ShadeCtx c;
  const Material& m = s.mats[mat];
  c.sh.m = &m;
  c.sh.albedo = m.albedo;
  c.sh.alpha = m.alpha;
  if (m.texture >= 0) {
    // nearest texel: x = min(floor(u W), W-1), the paper's closure example
    int W = s.tex_w[m.texture], H = s.tex_h[m.texture];
    double fu = std::floor(std::max(u, 0.0) * W), fv = std::floor(std::max(v, 0.0) * H);
    int x = (int)std::min(fu, (double)(W - 1));
    int y = (int)std::min(fv, (double)(H - 1));
    int64_t texel = (int64_t)y * W + x;
    if (t_amb) {
      flag_if(edge_dist(std::max(u, 0.0) * W, W) / W < kTolUV);
      flag_if(edge_dist(std::max(v, 0.0) * H, H) / H < kTolUV);
    }
    const float* t = P.tex[m.texture] + 3 * texel;
    c.sh.albedo = RGB(t[0], t[1], t[2]);
    c.k_tex = texel_key(m.texture, texel);
    c.has_tex = true;
  }
  if (m.rough_slot >= 0) {
    c.sh.alpha = P.rough[m.rough_slot];
    c.k_rough = rough_key(m.rough_slot);
    c.has_rough = true;
  }
  return c;
}

// Perspective pinhole camera: pixel (x, y) with jitter (jx, jy), row 0 at the
// top, vertical field of view fov_y.
struct Cam {
  V3 o, fwd, right, up;
  double tan_half, aspect;
  int W, H;
};
static Cam make_cam(const double* c) {
  Cam k;
  k.o = V3(c[0], c[1], c[2]);
  V3 tgt(c[3], c[4], c[5]), up(c[6], c[7], c[8]);
  k.fwd = normalize(tgt - k.o);
  k.right = normalize(cross(k.fwd, up));
  k.up = cross(k.right, k.fwd);
  k.tan_half = std::tan(c[9] * kPi / 360.0);
  k.W = (int)c[10];
  k.H = (int)c[11];
  k.aspect = (double)k.W / k.H;
  return k;
}
static V3 cam_dir(const Cam& k, int x, int y, double jx, double jy) {
  double px = (x + jx) / k.W, py = (y + jy) / k.H;
  double sx = (2.0 * px - 1.0) * k.tan_half * k.aspect;
  double sy = (1.0 - 2.0 * py) * k.tan_half;
  return normalize(k.fwd + k.right * sx + k.up * sy);
}

// ---------------------------------------------------------------------------
// Radiance-cache hook.  At the first scattering vertex with index k >= K
// (and k < D), after that vertex's emission has been collected, the raw
// features of the vertex are recorded: position, the direction back along
// the incoming ray, the geometric normal turned towards that direction,
// roughness (1 for non-microfacet types) and albedo (rho, f0 for a
// conductor, 1 for a dielectric).  mode 0 (cached estimator): the path stops
// there and the caller adds beta * max(C(features), 0).  mode 1 (training
// record): the plain path continues; the target is the radiance collected
// after the record point divided by beta at it.  The hook also notes which
// scene parameter each of the last four features is (the roughness slot for
// a microfacet type, the albedo texel for a type whose albedo feature is its
// albedo), for the derivative through the network's inputs.
// ---------------------------------------------------------------------------
struct CacheHook {
  int K = 3;
  int mode = 0;
  bool has = false;
  double feat[13];   // p[3], w[3], n[3], alpha, albedo[3]
  RGB beta;          // throughput at the record vertex
  RGB L_at;          // radiance collected up to and including its emission
  bool tex_in = false, rough_in = false;  // features 10..12 / 9 are parameters
  Key k_tex = 0, k_rough = 0;
  // self-training (mode 0 only): every scattering vertex with index k < K
  // before the record vertex, with its features, beta and the radiance
  // collected up to and including its emission
  struct Visit {
    int k;
    double feat[13];
    RGB beta, L_at;
  };
  std::vector<Visit>* visits = nullptr;
};

// ---------------------------------------------------------------------------
// One path-traced sample (the estimator of the primal megakernel).
//
// Depth: D counts path segments including the camera ray; emission found at
// vertex k counts if k <= D; next-event estimation and BSDF sampling at vertex
// k only if k < D.  Russian roulette after BSDF sampling at vertex k >= rr_depth.
// Null surfaces, and mask surfaces whose stochastic opacity test fails, are
// passed through; they count as vertices.
//
// If `recs` is given the per-vertex contributions are recorded (reverse
// sweep).  If `tan` is given, forward-mode tangents of beta and of L are
// propagated (sparse dual numbers).
// ---------------------------------------------------------------------------
static RGB trace_sample(const Scene& s, const Params& P, const Opts& opt, const Stream& rs, V3 o,
                        V3 d, std::vector<VertexRec>* recs, Tangent* tanL,
                        CacheHook* ch = nullptr) {
  RGB L, beta(1, 1, 1);
  Tangent tbeta;  // d beta
  double prev_pdf = 0;  // 0: no MIS for the next emitter hit (camera / delta event)
  V3 prev_p = o;
  const int n_em = (int)s.ems.size();
  const double p_sel = n_em > 0 ? 1.0 / n_em : 0.0;
  const bool no_nee = (opt.flags & FLAG_NO_NEE) != 0;
  if (recs) recs->clear();
  auto add_emit = [&](const RGB& Le, double w) {
    RGB c = beta * Le * w;
    L = L + c;
    if (recs) {
      if (recs->empty()) recs->push_back(VertexRec());
      recs->back().emit = recs->back().emit + c;
    }
    if (tanL) for (auto& p : tbeta.e) tanL->add(p.first, p.second * Le * w);
  };
  for (int k = 1; k <= opt.max_depth; ++k) {
    Hit h = closest_hit(s, o, d, 0.0, kInf);
    if (recs) recs->push_back(VertexRec());
    if (h.prim < 0) {
      if (s.env_index >= 0) {
        double w = (prev_pdf == 0 || no_nee) ? 1.0 : power_heuristic(prev_pdf, p_sel * env_pdf(s, d));
        add_emit(env_lookup(s, d), w);
      }
      break;
    }
    int i0 = s.idx[3 * h.prim], i1 = s.idx[3 * h.prim + 1], i2 = s.idx[3 * h.prim + 2];
    V3 p = s.pos[i0] * h.b[0] + s.pos[i1] * h.b[1] + s.pos[i2] * h.b[2];
    V3 n_g = normalize(cross(s.pos[i1] - s.pos[i0], s.pos[i2] - s.pos[i0]));
    double u = s.uv[2 * i0] * h.b[0] + s.uv[2 * i1] * h.b[1] + s.uv[2 * i2] * h.b[2];
    double v = s.uv[2 * i0 + 1] * h.b[0] + s.uv[2 * i1 + 1] * h.b[1] + s.uv[2 * i2 + 1] * h.b[2];
    // emission from a one-sided area light
    int em = s.tri_em[h.prim];
    double cos_y = -dot(d, n_g);
    if (em >= 0 && cos_y > 0 && s.ems[em].type == EM_AREA) {
      const Emitter& E = s.ems[em];
      double w = 1.0;
      if (!(prev_pdf == 0 || no_nee)) {
        V3 dv = p - prev_p;
        double p_l = p_sel * dot(dv, dv) / (E.area * cos_y);
        w = power_heuristic(prev_pdf, p_l);
      }
      add_emit(E.radiance, w);
    }
    if (k == opt.max_depth) break;
    uint32_t r0[4], r1[4];
    rs.block((uint32_t)(k - 1), 0, r0);
    rs.block((uint32_t)(k - 1), 1, r1);
    const Material& mat = s.mats[s.tri_mat[h.prim]];
    bool pass = mat.type == BSDF_NULL || (mat.type == BSDF_MASK && u01(r1[3]) >= mat.opacity);
    if (pass) {
      if (mat.type == BSDF_MASK) prev_pdf = 0;
      o = spawn(s, p, n_g, d);
      continue;
    }
    Frame fr = make_frame(n_g);
    V3 wi = fr.to_local(-d);
    ShadeCtx sc = fetch_shading(s, P, s.tri_mat[h.prim], u, v);
    // features of a vertex for the cache: position, direction back along the
    // incoming ray, normal turned towards it, roughness, albedo
    const int t = mat.type;
    const bool ggx = t == BSDF_CONDUCTOR || t == BSDF_DIELECTRIC || t == BSDF_PLASTIC;
    auto features = [&](double f[13]) {
      V3 w = -d;
      V3 nn = dot(n_g, w) >= 0 ? n_g : -n_g;
      RGB alb = t == BSDF_CONDUCTOR ? mat.f0 : (t == BSDF_DIELECTRIC ? RGB(1, 1, 1) : sc.sh.albedo);
      double v[13] = {p.x, p.y, p.z, w.x, w.y, w.z, nn.x, nn.y, nn.z, ggx ? sc.sh.alpha : 1.0,
                      alb[0], alb[1], alb[2]};
      std::memcpy(f, v, sizeof(v));
    };
    if (ch && ch->visits && !ch->has && k < ch->K) {
      CacheHook::Visit vis;
      vis.k = k;
      features(vis.feat);
      vis.beta = beta;
      vis.L_at = L;
      ch->visits->push_back(vis);
    }
    if (ch && !ch->has && k >= ch->K) {
      features(ch->feat);
      ch->tex_in = sc.has_tex && t != BSDF_CONDUCTOR && t != BSDF_DIELECTRIC;
      ch->k_tex = sc.k_tex;
      ch->rough_in = sc.has_rough && ggx;
      ch->k_rough = sc.k_rough;
      ch->has = true;
      ch->beta = beta;
      ch->L_at = L;
      if (ch->mode == 0) break;
    }
    VertexRec* rec = recs ? &recs->back() : nullptr;
    if (rec) {
      rec->k_tex = sc.k_tex; rec->has_tex = sc.has_tex;
      rec->k_rough = sc.k_rough; rec->has_rough = sc.has_rough;
    }
    // next-event estimation
    if (!no_nee && n_em > 0) {
      const Emitter& E = s.ems[pick(r0[0], (uint32_t)n_em)];
      double lu = u01(r0[1]), lv = u01(r0[2]);
      bool valid = false, delta = false, finite = false;
      V3 wl, y;
      double pdf_l = 0;
      RGB Le;
      if (E.type == EM_AREA) {
        y = E.p0 + E.e1 * lu + E.e2 * lv;
        V3 dv = y - p;
        double dist2 = dot(dv, dv), dist = std::sqrt(dist2);
        wl = dv * (1.0 / dist);
        double cy = -dot(wl, E.n);
        if (cy > 0) {
          pdf_l = dist2 / (E.area * cy);
          Le = E.radiance;
          finite = true;
          valid = true;
        }
      } else if (E.type == EM_ENV) {
        if (env_sample(s, lu, lv, &wl)) {
          pdf_l = env_pdf(s, wl);
          if (pdf_l > 0) { Le = env_lookup(s, wl); valid = true; }
        }
      } else {  // directional
        wl = normalize(E.p0);
        Le = E.radiance;
        pdf_l = 1.0;
        delta = true;
        valid = true;
      }
      if (valid) {
        Eval fe = bsdf_eval(sc.sh, wi, fr.to_local(wl));
        // shadow ray from the offset origin; towards an area light it stops
        // short of the sampled point by 1e-4 of its length
        V3 so = spawn(s, p, n_g, wl), sd = wl;
        double tmax = kInf;
        if (finite) {
          V3 dv = y - so;
          double dl = length(dv);
          sd = dv * (1.0 / dl);
          tmax = (1.0 - 1e-4) * dl;
        }
        if (!is_zero(fe.f) && !occluded(s, so, sd, tmax)) {
          double w = delta ? 1.0 : power_heuristic(p_sel * pdf_l, fe.pdf);
          RGB coef = beta * Le * (w / (p_sel * pdf_l));
          RGB c = coef * fe.f;
          L = L + c;
          if (rec) { rec->nee = c; rec->nee_coef = coef; rec->nee_eval = fe; }
          if (tanL) {
            for (auto& pp : tbeta.e) tanL->add(pp.first, pp.second * (Le * (w / (p_sel * pdf_l))) * fe.f);
            if (sc.has_tex) tanL->add(sc.k_tex, coef * fe.d_albedo);
            if (sc.has_rough) tanL->add(sc.k_rough, coef * fe.d_alpha);
          }
        }
      }
    }
    // BSDF sampling
    Sample bs = bsdf_sample(sc.sh, wi, u01(r1[0]), u01(r1[1]), u01(r0[3]));
    if (!bs.ok) break;
    RGB wgt = bs.e.f * (1.0 / bs.e.pdf);
    if (rec) { rec->has_bsdf = true; rec->bsdf_eval = bs.e; }
    if (tanL) {
      // d(beta * f / pdf) = d beta * f/pdf + beta * d f / pdf
      Tangent nt;
      for (auto& pp : tbeta.e) nt.add(pp.first, pp.second * wgt);
      if (sc.has_tex) nt.add(sc.k_tex, beta * bs.e.d_albedo * (1.0 / bs.e.pdf));
      if (sc.has_rough) nt.add(sc.k_rough, beta * bs.e.d_alpha * (1.0 / bs.e.pdf));
      tbeta = nt;
    }
    beta = beta * wgt;
    prev_pdf = bs.e.pdf;
    prev_p = p;
    V3 wo = fr.to_world(bs.wo);
    o = spawn(s, p, n_g, wo);
    d = wo;
    if (k >= opt.rr_depth) {
      double q = std::min(std::max(beta[0], std::max(beta[1], beta[2])), 0.95);
      flag_if(std::fabs(u01(r1[2]) - q) < kTolU);
      if (u01(r1[2]) >= q) break;
      beta = beta * (1.0 / q);
      for (auto& pp : tbeta.e) pp.second = pp.second * (1.0 / q);
    }
  }
  return L;
}

static Stream make_stream(uint64_t seed, uint64_t g) {
  Stream st;
  st.key[0] = (uint32_t)seed;
  st.key[1] = (uint32_t)(seed >> 32);
  st.g_lo = (uint32_t)g;
  st.g_hi = (uint32_t)(g >> 32);
  return st;
}

// Camera ray of sample g of pixel (x, y).
static void camera_ray(const Cam& k, const Stream& st, int x, int y, V3* o, V3* d) {
  uint32_t r[4];
  st.block(kCameraBlock, 0, r);
  *o = k.o;
  *d = cam_dir(k, x, y, u01(r[0]), u01(r[1]));
}

// Sparse gradient accumulator (per thread).
struct GradAcc {
  std::unordered_map<Key, RGB> m;
  void add(Key k, const RGB& v) {
    auto it = m.find(k);
    if (it == m.end()) m.emplace(k, v); else it->second = it->second + v;
  }
};

// Reverse sweep over a stored path: S_k is everything collected after vertex
// k's sampled direction; the derivative of sample radiance (weighted by the
// adjoint dL) is sum_k [ d NEE_k + S_k * (d f_k)/f_k ], per channel.
static void reverse_sweep(const std::vector<VertexRec>& recs, const RGB& dL, GradAcc* acc) {
  RGB S;
  for (int k = (int)recs.size() - 1; k >= 0; --k) {
    const VertexRec& r = recs[k];
    if (r.has_bsdf) {
      RGB ga, gr;
      for (int c = 0; c < 3; ++c) {
        double f = r.bsdf_eval.f[c];
        if (f != 0) {
          ga[c] = dL[c] * S[c] * r.bsdf_eval.d_albedo[c] / f;
          gr[c] = dL[c] * S[c] * r.bsdf_eval.d_alpha[c] / f;
        }
      }
      if (r.has_tex) acc->add(r.k_tex, ga);
      if (r.has_rough) acc->add(r.k_rough, RGB(gr[0] + gr[1] + gr[2], 0, 0));
    }
    if (!is_zero(r.nee)) {
      RGB ga = dL * r.nee_coef * r.nee_eval.d_albedo;
      RGB gr = dL * r.nee_coef * r.nee_eval.d_alpha;
      if (r.has_tex) acc->add(r.k_tex, ga);
      if (r.has_rough) acc->add(r.k_rough, RGB(gr[0] + gr[1] + gr[2], 0, 0));
    }
    S = S + r.nee + r.emit;
  }
}

template <class F>
static void parallel_for(int64_t n, int n_threads, F fn) {
  if (n_threads <= 1 || n < 2) {
    for (int64_t i = 0; i < n; ++i) fn(0, i);
    return;
  }
  std::atomic<int64_t> next(0);
  std::vector<std::thread> th;
  for (int t = 0; t < n_threads; ++t) {
    th.emplace_back([&, t]() {
      for (;;) {
        int64_t i = next.fetch_add(1);
        if (i >= n) break;
        fn(t, i);
      }
    });
  }
  for (auto& x : th) x.join();
}

// ---------------------------------------------------------------------------
// Neural radiance cache: input encoding and network.
//
// Encoding of a record (80 inputs): a multiresolution hash grid over the
// position normalised to the scene box -- 16 levels of 2 features, 2^19
// entries per level, resolutions from 16 to 2048 in a geometric series,
// trilinear interpolation of the 8 corners, dense indexing while a level's
// (N+1)^3 corners fit the table and otherwise the spatial hash of Mueller et
// al. (Instant-NGP, 2022): xor of the corner coordinates times 1,
// 2654435761, 805459861, modulo the table size; then 16 real spherical
// harmonics (bands 0-3) of the direction, 16 of the normal, the roughness
// and the albedo (68 values), zero-padded to 80.
//
// Network: 80 -> 64 -> 64 -> 64 -> 64 -> 3, ReLU on the hidden layers, no
// biases; weights row-major [out][in], layers in order.  In the BF16 mode the
// values a BF16 implementation stores in BF16 are rounded to it (round to
// nearest even): the inputs, the weights, the hidden activations, and in the
// backward pass the output gradient and the hidden-layer gradients.
// ---------------------------------------------------------------------------
struct GridCfg {
  int L, F, log2T;
  double Nmin, Nmax;
  double lo[3], hi[3];
};
static const int kIn = 80, kHid = 64, kOut = 3;
static const int kNumWeights = kHid * kIn + 3 * kHid * kHid + kOut * kHid;

static int level_res(const GridCfg& g, int l) {
  double r = g.Nmin * std::exp(l * (std::log(g.Nmax) - std::log(g.Nmin)) / (g.L - 1));
  return (int)std::floor(r + 1e-6);
}

// the 8 corner indices and trilinear weights of one level
static void grid_corners(const GridCfg& g, int l, const double xn[3], uint32_t idx[8], double w[8]) {
  int N = level_res(g, l);
  uint64_t T = 1ull << g.log2T;
  int c0[3];
  double fr[3];
  for (int a = 0; a < 3; ++a) {
    double pos = xn[a] * N;
    int c = (int)std::floor(pos);
    c = std::min(std::max(c, 0), N - 1);
    c0[a] = c;
    fr[a] = pos - c;
  }
  bool dense = (uint64_t)(N + 1) * (N + 1) * (N + 1) <= T;
  for (int k = 0; k < 8; ++k) {
    uint32_t c[3];
    double wk = 1.0;
    for (int a = 0; a < 3; ++a) {
      int bit = (k >> a) & 1;
      c[a] = (uint32_t)(c0[a] + bit);
      wk *= bit ? fr[a] : 1.0 - fr[a];
    }
    uint32_t id;
    if (dense) {
      id = c[0] + c[1] * (uint32_t)(N + 1) + c[2] * (uint32_t)(N + 1) * (uint32_t)(N + 1);
    } else {
      id = (c[0] * 1u) ^ (c[1] * 2654435761u) ^ (c[2] * 805459861u);
      id &= (uint32_t)(T - 1);
    }
    idx[k] = id;
    w[k] = wk;
  }
}

static void normalise_pos(const GridCfg& g, const double p[3], double xn[3]) {
  for (int a = 0; a < 3; ++a) {
    double e = g.hi[a] - g.lo[a];
    double v = e > 0 ? (p[a] - g.lo[a]) / e : 0.0;
    xn[a] = std::min(std::max(v, 0.0), 1.0);
  }
}

// Real spherical harmonics, bands 0..3, orthonormal on the sphere.
static void sh16(const double d[3], double o[16]) {
  double x = d[0], y = d[1], z = d[2];
  const double c0 = 0.5 * std::sqrt(1.0 / kPi);
  const double c1 = std::sqrt(3.0 / (4.0 * kPi));
  const double c2a = 0.5 * std::sqrt(15.0 / kPi), c2b = 0.25 * std::sqrt(5.0 / kPi);
  const double c2c = 0.25 * std::sqrt(15.0 / kPi);
  const double c3a = 0.25 * std::sqrt(35.0 / (2.0 * kPi)), c3b = 0.5 * std::sqrt(105.0 / kPi);
  const double c3c = 0.25 * std::sqrt(21.0 / (2.0 * kPi)), c3d = 0.25 * std::sqrt(7.0 / kPi);
  const double c3e = 0.25 * std::sqrt(105.0 / kPi);
  o[0] = c0;
  o[1] = c1 * y;
  o[2] = c1 * z;
  o[3] = c1 * x;
  o[4] = c2a * x * y;
  o[5] = c2a * y * z;
  o[6] = c2b * (3.0 * z * z - 1.0);
  o[7] = c2a * x * z;
  o[8] = c2c * (x * x - y * y);
  o[9] = c3a * y * (3.0 * x * x - y * y);
  o[10] = c3b * x * y * z;
  o[11] = c3c * y * (5.0 * z * z - 1.0);
  o[12] = c3d * z * (5.0 * z * z - 3.0);
  o[13] = c3c * x * (5.0 * z * z - 1.0);
  o[14] = c3e * z * (x * x - y * y);
  o[15] = c3a * x * (x * x - 3.0 * y * y);
}

static void encode(const GridCfg& g, const float* grid, const double f[13], double out[80]) {
  for (int i = 0; i < 80; ++i) out[i] = 0.0;
  double xn[3];
  normalise_pos(g, f, xn);
  uint64_t T = 1ull << g.log2T;
  for (int l = 0; l < g.L; ++l) {
    uint32_t idx[8];
    double w[8];
    grid_corners(g, l, xn, idx, w);
    for (int ft = 0; ft < g.F; ++ft) {
      double acc = 0;
      for (int k = 0; k < 8; ++k) acc += w[k] * grid[((uint64_t)l * T + idx[k]) * g.F + ft];
      out[l * g.F + ft] = acc;
    }
  }
  sh16(f + 3, out + 32);
  sh16(f + 6, out + 48);
  out[64] = f[9];
  out[65] = f[10];
  out[66] = f[11];
  out[67] = f[12];
}

static double bf16_round(double v) {
  float fv = (float)v;
  uint32_t b;
  std::memcpy(&b, &fv, 4);
  if ((b & 0x7F800000u) != 0x7F800000u) b += 0x7FFFu + ((b >> 16) & 1u);
  b &= 0xFFFF0000u;
  float r;
  std::memcpy(&r, &b, 4);
  return r;
}

struct Mlp {
  // layer l: out x in, offset
  static int rows(int l) { return l == 4 ? kOut : kHid; }
  static int cols(int l) { return l == 0 ? kIn : kHid; }
  static int off(int l) { return l == 0 ? 0 : kHid * kIn + (l - 1) * kHid * kHid; }
};

// acts[l] holds the input of layer l (acts[0] = x), as the BF16 path would
// store it; y = output (not rounded).
static void mlp_forward(const double* W, const double* x, bool emu, std::vector<double>* acts,
                        double y[3]) {
  std::vector<double> a(x, x + kIn);
  if (emu) for (auto& v : a) v = bf16_round(v);
  if (acts) { acts->clear(); acts->insert(acts->end(), a.begin(), a.end()); }
  for (int l = 0; l < 5; ++l) {
    int R = Mlp::rows(l), C = Mlp::cols(l);
    const double* w = W + Mlp::off(l);
    std::vector<double> o(R, 0.0);
    for (int r = 0; r < R; ++r) {
      double acc = 0;
      for (int c = 0; c < C; ++c) {
        double wv = emu ? bf16_round(w[r * C + c]) : w[r * C + c];
        acc += wv * a[c];
      }
      o[r] = acc;
    }
    if (l < 4) {
      for (auto& v : o) {
        v = v > 0 ? v : 0.0;
        if (emu) v = bf16_round(v);
      }
      if (acts) acts->insert(acts->end(), o.begin(), o.end());
      a = o;
    } else {
      for (int r = 0; r < kOut; ++r) y[r] = o[r];
    }
  }
}

// dW += d(loss)/dW, dx = d(loss)/dx for one sample with output gradient dy.
static void mlp_backward(const double* W, const double* x, const double dy[3], bool emu,
                         double* dW, double* dx) {
  std::vector<double> acts;
  double y[3];
  mlp_forward(W, x, emu, &acts, y);
  auto act = [&](int l) { return acts.data() + (l == 0 ? 0 : kIn + (l - 1) * kHid); };
  std::vector<double> g(dy, dy + kOut);
  if (emu) for (auto& v : g) v = bf16_round(v);
  for (int l = 4; l >= 0; --l) {
    int R = Mlp::rows(l), C = Mlp::cols(l);
    const double* w = W + Mlp::off(l);
    const double* in = act(l);
    for (int r = 0; r < R; ++r)
      for (int c = 0; c < C; ++c) dW[Mlp::off(l) + r * C + c] += g[r] * in[c];
    std::vector<double> gi(C, 0.0);
    for (int c = 0; c < C; ++c) {
      double acc = 0;
      for (int r = 0; r < R; ++r) acc += (emu ? bf16_round(w[r * C + c]) : w[r * C + c]) * g[r];
      gi[c] = acc;
    }
    if (l > 0) {
      for (int c = 0; c < C; ++c) {
        gi[c] = in[c] > 0 ? gi[c] : 0.0;  // ReLU of layer l-1's output
        if (emu) gi[c] = bf16_round(gi[c]);
      }
      g = gi;
    } else {
      for (int c = 0; c < C; ++c) dx[c] = gi[c];
    }
  }
}

// Magnitude sums of the terms of every network output and gradient entry
// for one sample: ay[r] = sum_c |w_rc| |a_c| over the output layer's inputs,
// aW += |g_r| |in_c| per weight, adx[c] = sum_r |w_rc| |g_r| -- the scale of a
// floating-point sum's rounding error (sum over its terms of their
// magnitudes), with the forward activations and backpropagated signals of
// mlp_backward.  Test infrastructure: tolerance scales, not estimator work.
static void mlp_term_magnitudes(const double* W, const double* x, const double dy[3], bool emu,
                                double* aW, double* adx, double ay[3]) {
  std::vector<double> acts;
  double y[3];
  mlp_forward(W, x, emu, &acts, y);
  auto act = [&](int l) { return acts.data() + (l == 0 ? 0 : kIn + (l - 1) * kHid); };
  auto wt = [&](const double* w, int i) { return std::fabs(emu ? bf16_round(w[i]) : w[i]); };
  {
    const double* w = W + Mlp::off(4);
    const double* in = act(4);
    for (int r = 0; r < kOut; ++r) {
      double acc = 0;
      for (int c = 0; c < kHid; ++c) acc += wt(w, r * kHid + c) * std::fabs(in[c]);
      ay[r] = acc;
    }
  }
  std::vector<double> g(dy, dy + kOut);
  if (emu) for (auto& v : g) v = bf16_round(v);
  for (int l = 4; l >= 0; --l) {
    int R = Mlp::rows(l), C = Mlp::cols(l);
    const double* w = W + Mlp::off(l);
    const double* in = act(l);
    for (int r = 0; r < R; ++r)
      for (int c = 0; c < C; ++c) aW[Mlp::off(l) + r * C + c] += std::fabs(g[r] * in[c]);
    std::vector<double> gi(C, 0.0);
    for (int c = 0; c < C; ++c) {
      double acc = 0, mag = 0;
      for (int r = 0; r < R; ++r) {
        const double wv = emu ? bf16_round(w[r * C + c]) : w[r * C + c];
        acc += wv * g[r];
        mag += std::fabs(wv * g[r]);
      }
      gi[c] = acc;
      if (l == 0) adx[c] = mag;
    }
    if (l > 0) {
      for (int c = 0; c < C; ++c) {
        gi[c] = in[c] > 0 ? gi[c] : 0.0;
        if (emu) gi[c] = bf16_round(gi[c]);
      }
      g = gi;
    }
  }
}

// Relative L2 (Mueller et al., neural radiance caching, 2021): mean over
// samples and channels of (y - t)^2 / (sg(y)^2 + 0.01).
static double rel_l2(int64_t n, const double* y, const double* t, double* dy) {
  double acc = 0;
  double inv = 1.0 / (3.0 * n);
  for (int64_t i = 0; i < 3 * n; ++i) {
    double den = y[i] * y[i] + 0.01;
    double r = y[i] - t[i];
    acc += r * r / den;
    if (dy) dy[i] = 2.0 * r / den * inv;
  }
  return acc * inv;
}

}  // namespace orc

using namespace orc;

extern "C" {

// Build the oracle's scene from the shared scene arrays.  Returns an opaque
// handle (NULL on invalid input).
void* oracle_scene_new(int nv, const float* positions, const float* uvs, int nt,
                       const int* indices, const int* tri_material, const int* tri_emitter,
                       int nm, const int* mat_type, const int* mat_texture,
                       const int* mat_rough_slot, const float* mat_albedo, const float* mat_alpha,
                       const float* mat_f0, const float* mat_eta, const float* mat_opacity,
                       int ne, const int* em_type, const float* em_p0, const float* em_e1,
                       const float* em_e2, const float* em_radiance, int n_tex,
                       const int* tex_w, const int* tex_h, int n_rough, const float* env,
                       int env_w, int env_h) {
  Scene* s = new Scene();
  s->pos.resize(nv);
  V3 lo(kInf, kInf, kInf), hi(-kInf, -kInf, -kInf);
  for (int i = 0; i < nv; ++i) {
    V3 p(positions[3 * i], positions[3 * i + 1], positions[3 * i + 2]);
    s->pos[i] = p;
    lo = V3(std::min(lo.x, p.x), std::min(lo.y, p.y), std::min(lo.z, p.z));
    hi = V3(std::max(hi.x, p.x), std::max(hi.y, p.y), std::max(hi.z, p.z));
  }
  s->uv.assign(2 * (size_t)nv, 0.0);
  if (uvs) for (int i = 0; i < 2 * nv; ++i) s->uv[i] = uvs[i];
  s->idx.assign(indices, indices + 3 * (size_t)nt);
  s->tri_mat.assign(tri_material, tri_material + nt);
  s->tri_em.assign(tri_emitter, tri_emitter + nt);
  for (int i = 0; i < nm; ++i) {
    Material m;
    m.type = mat_type[i];
    m.texture = mat_texture[i];
    m.rough_slot = mat_rough_slot[i];
    m.albedo = RGB(mat_albedo[3 * i], mat_albedo[3 * i + 1], mat_albedo[3 * i + 2]);
    m.f0 = RGB(mat_f0[3 * i], mat_f0[3 * i + 1], mat_f0[3 * i + 2]);
    m.alpha = mat_alpha[i];
    m.eta = mat_eta[i];
    m.opacity = mat_opacity[i];
    s->mats.push_back(m);
  }
  for (int i = 0; i < ne; ++i) {
    Emitter e;
    e.type = em_type[i];
    e.p0 = V3(em_p0[3 * i], em_p0[3 * i + 1], em_p0[3 * i + 2]);
    e.e1 = V3(em_e1[3 * i], em_e1[3 * i + 1], em_e1[3 * i + 2]);
    e.e2 = V3(em_e2[3 * i], em_e2[3 * i + 1], em_e2[3 * i + 2]);
    e.radiance = RGB(em_radiance[3 * i], em_radiance[3 * i + 1], em_radiance[3 * i + 2]);
    V3 c = cross(e.e1, e.e2);
    e.area = length(c);
    e.n = e.area > 0 ? c * (1.0 / e.area) : V3(0, 0, 1);
    if (e.type == EM_ENV) s->env_index = i;
    s->ems.push_back(e);
  }
  s->tex_w.assign(tex_w, tex_w + n_tex);
  s->tex_h.assign(tex_h, tex_h + n_tex);
  s->n_rough = n_rough;
  double ext = std::max(hi.x - lo.x, std::max(hi.y - lo.y, hi.z - lo.z));
  s->eps = 1e-4 * ext;
  if (env && env_w > 0 && env_h > 0) {
    s->env_w = env_w;
    s->env_h = env_h;
    s->env.resize(3 * (size_t)env_w * env_h);
    for (size_t i = 0; i < s->env.size(); ++i) s->env[i] = env[i];
    build_env(*s);
  } else if (s->env_index >= 0) {
    delete s;
    return nullptr;
  }
  return s;
}

void oracle_scene_free(void* h) { delete (Scene*)h; }

// Builds (on != 0) or drops (on == 0) the bounding-volume hierarchy that
// stands in for the loop over all triangles in every ray query.
void oracle_scene_accel(void* h, int on) {
  Scene& s = *(Scene*)h;
  if (on) {
    if (s.bvh.nodes.empty()) bvh_build(s);
  } else {
    s.bvh = Bvh();
  }
}

double oracle_scene_eps(void* h) { return ((Scene*)h)->eps; }

// Philox4x32-10 on n (counter, key) pairs: ctr [n][4], key [n][2] -> out [n][4].
void oracle_philox(int64_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  for (int64_t i = 0; i < n; ++i) philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

// Brute-force ray queries.  any = 0: closest hit (prim id, t, barycentrics);
// any = 1: occlusion (prim = 1 if occluded else -1; null surfaces ignored).
// `ambiguous` flags rays whose answer is decided within FP32 reach: a
// runner-up hit or a near-miss within 1e-6 relative in t, a barycentric
// within 1e-6 of an edge, or a hit within 1e-6 of the interval ends.
void oracle_trace(void* h, int64_t n, const double* o, const double* d, const double* tmin,
                  const double* tmax, int any, int n_threads, int* prim, double* t_out,
                  double* b_out, int* ambiguous) {
  const Scene& s = *(Scene*)h;
  parallel_for(n, n_threads, [&](int, int64_t i) {
    V3 O(o[3 * i], o[3 * i + 1], o[3 * i + 2]), D(d[3 * i], d[3 * i + 1], d[3 * i + 2]);
    if (any) {
      prim[i] = occluded(s, O, D, tmax[i]) ? 1 : -1;
    } else {
      Hit hh = closest_hit(s, O, D, tmin[i], tmax[i]);
      prim[i] = hh.prim;
      t_out[i] = hh.t;
      for (int c = 0; c < 3; ++c) b_out[3 * i + c] = hh.b[c];
    }
    // ambiguity: examine every reachable triangle's plane hit with signed
    // barycentrics
    int amb = 0;
    double tb = any ? tmax[i] : (prim[i] >= 0 ? t_out[i] : tmax[i]);
    double w0 = tmin[i], w1 = tmax[i];
    widen(&w0, &w1);
    for_reachable(s, O, D, w0, &w1, [&](int j) -> bool {
      if (any && s.mats[s.tri_mat[j]].type == BSDF_NULL) return false;
      V3 p0 = s.pos[s.idx[3 * j]], p1 = s.pos[s.idx[3 * j + 1]], p2 = s.pos[s.idx[3 * j + 2]];
      V3 e1 = p1 - p0, e2 = p2 - p0, pv = cross(D, e2);
      double det = dot(e1, pv);
      double scale = length(e1) * length(e2);
      if (std::fabs(det) <= 1e-12 * scale) return false;
      V3 tv = O - p0;
      double bu = dot(tv, pv) / det;
      V3 qv = cross(tv, e1);
      double bv = dot(D, qv) / det;
      double tt = dot(e2, qv) / det;
      double bmin = std::min(std::min(bu, bv), 1.0 - bu - bv);
      double tol_t = 1e-6 * std::max(1.0, std::fabs(tt));
      bool near_range = tt > tmin[i] - tol_t && tt < tmax[i] + tol_t;
      if (!near_range) return false;
      bool near_edge = std::fabs(bmin) <= 1e-6;
      bool inside = bmin > 1e-6;
      if (near_edge && tt <= tb + tol_t) amb = 1;
      if (inside && (std::fabs(tt - tmin[i]) <= tol_t || std::fabs(tt - tmax[i]) <= tol_t)) amb = 1;
      if (!any && inside && j != prim[i] && prim[i] >= 0 && std::fabs(tt - tb) <= tol_t) amb = 1;
      return amb != 0;
    });
    ambiguous[i] = amb;
  });
}

// Pixel estimates I_p = (1/spp) sum_s L(g) for a list of pixels
// (id = (cam*H + y)*W + x), box filter of one-pixel support.
// cams: [n_cams][12] = origin, target, up, fov_y_deg, width, height.
void oracle_render(void* h, const float* const* textures, const float* roughness,
                   const double* cams, int n_cams, int spp, int max_depth, int rr_depth,
                   uint32_t flags, uint64_t seed, int64_t n_pix, const int64_t* pixel_ids,
                   int n_threads, double* out, int* ambiguous) {
  const Scene& s = *(Scene*)h;
  Params P{textures, roughness};
  Opts opt{spp, max_depth, rr_depth, flags, seed};
  std::vector<Cam> cs;
  for (int c = 0; c < n_cams; ++c) cs.push_back(make_cam(cams + 12 * c));
  const int W = cs[0].W, H = cs[0].H;
  parallel_for(n_pix, n_threads, [&](int, int64_t i) {
    int64_t pid = pixel_ids[i];
    int cam = (int)(pid / ((int64_t)W * H));
    int y = (int)((pid / W) % H), x = (int)(pid % W);
    RGB acc;
    int n_amb = 0;
    for (int sidx = 0; sidx < spp; ++sidx) {
      uint64_t g = (uint64_t)pid * spp + sidx;
      Stream st = make_stream(seed, g);
      V3 o, d;
      bool amb = false;
      t_amb = ambiguous ? &amb : nullptr;
      camera_ray(cs[cam], st, x, y, &o, &d);
      acc = acc + trace_sample(s, P, opt, st, o, d, nullptr, nullptr);
      t_amb = nullptr;
      n_amb += amb ? 1 : 0;
    }
    for (int c = 0; c < 3; ++c) out[3 * i + c] = acc[c] / spp;
    if (ambiguous) ambiguous[i] = n_amb;
  });
}

// Forward-mode derivative of the image along a parameter direction v:
// out_p = sum over parameters of (d I_p / d param) v_param, per channel, with
// the same attached/detached split as the reverse sweep (texel albedos and
// roughness attached through the BSDF values, sampling and MIS weights
// detached).  tex_tangent[t]: [H][W][3] per texture (may be NULL);
// rough_tangent: one value per roughness slot (may be NULL).
void oracle_jvp(void* h, const float* const* textures, const float* roughness,
                const double* cams, int n_cams, int spp, int max_depth, int rr_depth,
                uint32_t flags, uint64_t seed, const double* const* tex_tangent,
                const double* rough_tangent, int64_t n_pix, const int64_t* pixel_ids, int n_threads,
                double* out) {
  const Scene& s = *(Scene*)h;
  Params P{textures, roughness};
  Opts opt{spp, max_depth, rr_depth, flags, seed};
  std::vector<Cam> cs;
  for (int c = 0; c < n_cams; ++c) cs.push_back(make_cam(cams + 12 * c));
  const int W = cs[0].W, H = cs[0].H;
  parallel_for(n_pix, n_threads, [&](int, int64_t i) {
    int64_t pid = pixel_ids[i];
    int cam = (int)(pid / ((int64_t)W * H));
    int y = (int)((pid / W) % H), x = (int)(pid % W);
    RGB acc;
    for (int sidx = 0; sidx < spp; ++sidx) {
      uint64_t g = (uint64_t)pid * spp + sidx;
      Stream st = make_stream(seed, g);
      V3 o, d;
      camera_ray(cs[cam], st, x, y, &o, &d);
      Tangent tl;
      trace_sample(s, P, opt, st, o, d, nullptr, &tl);
      for (auto& e : tl.e) {
        Key k = e.first;
        if (is_texel(k)) {
          int tex = (int)((k >> 40) & 0x7FFFFF);
          int64_t texel = (int64_t)(k & ((1ull << 40) - 1));
          if (tex_tangent && tex_tangent[tex])
            for (int c = 0; c < 3; ++c) acc[c] += e.second[c] * tex_tangent[tex][3 * texel + c];
        } else if (rough_tangent) {
          for (int c = 0; c < 3; ++c) acc[c] += e.second[c] * rough_tangent[(int)k];
        }
      }
    }
    for (int c = 0; c < 3; ++c) out[3 * i + c] = acc[c] / spp;
  });
}

// Radiance estimates along explicit rays: ray i uses samples g = i*spp + s.
void oracle_radiance(void* h, const float* const* textures, const float* roughness, int64_t n,
                     const double* o, const double* d, int spp, int max_depth, int rr_depth,
                     uint32_t flags, uint64_t seed, int n_threads, double* out) {
  const Scene& s = *(Scene*)h;
  Params P{textures, roughness};
  Opts opt{spp, max_depth, rr_depth, flags, seed};
  parallel_for(n, n_threads, [&](int, int64_t i) {
    V3 O(o[3 * i], o[3 * i + 1], o[3 * i + 2]), D(d[3 * i], d[3 * i + 1], d[3 * i + 2]);
    RGB acc;
    for (int sidx = 0; sidx < spp; ++sidx) {
      Stream st = make_stream(seed, (uint64_t)i * spp + sidx);
      acc = acc + trace_sample(s, P, opt, st, O, D, nullptr, nullptr);
    }
    for (int c = 0; c < 3; ++c) out[3 * i + c] = acc[c] / spp;
  });
}

// Reverse-mode gradient of sum_p <adj_p, I_p> for the listed pixels, with
// the per-sample adjoint adj_p / spp (box filter).  mode 0: stored-path
// reverse sweep; mode 1: forward-mode sparse tangents.  Gradients are
// ACCUMULATED into grad_tex[t] ([H][W][3], may be NULL) and grad_rough.
void oracle_adjoint(void* h, const float* const* textures, const float* roughness,
                    const double* cams, int n_cams, int spp, int max_depth, int rr_depth,
                    uint32_t flags, uint64_t seed, int64_t n_pix, const int64_t* pixel_ids,
                    const double* adj, int mode, int n_threads, double* const* grad_tex,
                    double* grad_rough) {
  const Scene& s = *(Scene*)h;
  Params P{textures, roughness};
  Opts opt{spp, max_depth, rr_depth, flags, seed};
  std::vector<Cam> cs;
  for (int c = 0; c < n_cams; ++c) cs.push_back(make_cam(cams + 12 * c));
  const int W = cs[0].W, H = cs[0].H;
  int nth = std::max(1, n_threads);
  std::vector<GradAcc> accs(nth);
  parallel_for(n_pix, nth, [&](int t, int64_t i) {
    int64_t pid = pixel_ids[i];
    int cam = (int)(pid / ((int64_t)W * H));
    int y = (int)((pid / W) % H), x = (int)(pid % W);
    RGB dL(adj[3 * i] / spp, adj[3 * i + 1] / spp, adj[3 * i + 2] / spp);
    if (is_zero(dL)) return;
    std::vector<VertexRec> recs;
    for (int sidx = 0; sidx < spp; ++sidx) {
      uint64_t g = (uint64_t)pid * spp + sidx;
      Stream st = make_stream(seed, g);
      V3 o, d;
      camera_ray(cs[cam], st, x, y, &o, &d);
      if (mode == 0) {
        trace_sample(s, P, opt, st, o, d, &recs, nullptr);
        reverse_sweep(recs, dL, &accs[t]);
      } else {
        Tangent tl;
        trace_sample(s, P, opt, st, o, d, nullptr, &tl);
        for (auto& p : tl.e) {
          RGB g3 = dL * p.second;
          if (is_texel(p.first)) accs[t].add(p.first, g3);
          else accs[t].add(p.first, RGB(g3[0] + g3[1] + g3[2], 0, 0));
        }
      }
    }
  });
  for (auto& a : accs) {
    for (auto& kv : a.m) {
      Key k = kv.first;
      if (is_texel(k)) {
        int tex = (int)((k >> 40) & 0x7FFFFF);
        int64_t texel = (int64_t)(k & ((1ull << 40) - 1));
        if (grad_tex && grad_tex[tex])
          for (int c = 0; c < 3; ++c) grad_tex[tex][3 * texel + c] += kv.second[c];
      } else if (grad_rough) {
        grad_rough[(int)k] += kv.second[0];
      }
    }
  }
}

// Ambient occlusion of the paper's running example: for each primary ray that
// hits, the fraction of n_ao cosine-weighted rays of length 1 (spawned at the
// hit) that are unoccluded.  AO ray j of primary ray i uses Philox block
// (g = i, b = j, dim = 0).  Misses give -1.
void oracle_ao(void* h, int64_t n, const double* o, const double* d, int n_ao, uint64_t seed,
               int n_threads, double* out) {
  const Scene& s = *(Scene*)h;
  parallel_for(n, n_threads, [&](int, int64_t i) {
    V3 O(o[3 * i], o[3 * i + 1], o[3 * i + 2]), D(d[3 * i], d[3 * i + 1], d[3 * i + 2]);
    Hit hh = closest_hit(s, O, D, 0.0, kInf);
    if (hh.prim < 0) { out[i] = -1; return; }
    int i0 = s.idx[3 * hh.prim], i1 = s.idx[3 * hh.prim + 1], i2 = s.idx[3 * hh.prim + 2];
    V3 p = s.pos[i0] * hh.b[0] + s.pos[i1] * hh.b[1] + s.pos[i2] * hh.b[2];
    V3 n_g = normalize(cross(s.pos[i1] - s.pos[i0], s.pos[i2] - s.pos[i0]));
    if (dot(n_g, D) > 0) n_g = -n_g;  // shade the side the ray arrived on
    Frame fr = make_frame(n_g);
    Stream st = make_stream(seed, (uint64_t)i);
    int count = 0;
    for (int j = 0; j < n_ao; ++j) {
      uint32_t r[4];
      st.block((uint32_t)j, 0, r);
      V3 wl = fr.to_world(cosine_hemisphere(u01(r[0]), u01(r[1])));
      if (!occluded(s, spawn(s, p, n_g, wl), wl, 1.0)) ++count;
    }
    out[i] = (double)count / n_ao;
  });
}

// Single BSDF evaluation (local frame).  Outputs f*|cos| [3], pdf,
// d/d albedo [3], d/d alpha [3].
void oracle_bsdf_eval(int type, const double* albedo, double alpha, const double* f0, double eta,
                      const double* wi, const double* wo, double* f, double* pdf, double* dalb,
                      double* dalpha) {
  Material m;
  m.type = type; m.texture = -1; m.rough_slot = -1;
  m.albedo = RGB(albedo[0], albedo[1], albedo[2]);
  m.f0 = RGB(f0[0], f0[1], f0[2]);
  m.alpha = alpha; m.eta = eta; m.opacity = 1.0;
  Shading sh{&m, m.albedo, alpha};
  Eval e = bsdf_eval(sh, V3(wi[0], wi[1], wi[2]), V3(wo[0], wo[1], wo[2]));
  for (int c = 0; c < 3; ++c) { f[c] = e.f[c]; dalb[c] = e.d_albedo[c]; dalpha[c] = e.d_alpha[c]; }
  *pdf = e.pdf;
}

// Single BSDF sample (local frame).  Returns 1 on success; wo [3], f*|cos| [3], pdf.
int oracle_bsdf_sample(int type, const double* albedo, double alpha, const double* f0, double eta,
                       const double* wi, double u1, double u2, double ulobe, double* wo, double* f,
                       double* pdf) {
  Material m;
  m.type = type; m.texture = -1; m.rough_slot = -1;
  m.albedo = RGB(albedo[0], albedo[1], albedo[2]);
  m.f0 = RGB(f0[0], f0[1], f0[2]);
  m.alpha = alpha; m.eta = eta; m.opacity = 1.0;
  Shading sh{&m, m.albedo, alpha};
  Sample s = bsdf_sample(sh, V3(wi[0], wi[1], wi[2]), u1, u2, ulobe);
  wo[0] = s.wo.x; wo[1] = s.wo.y; wo[2] = s.wo.z;
  for (int c = 0; c < 3; ++c) f[c] = s.e.f[c];
  *pdf = s.e.pdf;
  return s.ok ? 1 : 0;
}

// GGX terms and their roughness log-derivatives: analytic and complex-step.
// out: D, dlnD, dlnD_cs, G1, dlnG1, dlnG1_cs
void oracle_ggx_terms(double alpha, double cos_m, double cos_v, double* out) {
  typedef std::complex<double> C;
  const double hstep = 1e-30;
  C ac(alpha, hstep);
  double D = ggx_D<double>(alpha, cos_m);
  C Dc = ggx_D<C>(ac, cos_m);
  double G = ggx_G1<double>(alpha, cos_v, cos_v);
  C Gc = ggx_G1<C>(ac, cos_v, cos_v);
  out[0] = D;
  out[1] = ggx_dlnD(alpha, cos_m);
  out[2] = D != 0 ? (Dc.imag() / hstep) / D : 0;
  out[3] = G;
  out[4] = ggx_dlnG1(alpha, cos_v);
  out[5] = G != 0 ? (Gc.imag() / hstep) / G : 0;
}

// GGX microfacet sample (for distribution tests).
void oracle_ggx_sample(double alpha, double u1, double u2, double* m) {
  V3 v = ggx_sample_m(alpha, u1, u2);
  m[0] = v.x; m[1] = v.y; m[2] = v.z;
}

double oracle_fresnel(double cos_i, double eta) { return fresnel_dielectric(cos_i, eta); }

// Orthonormal frame of a unit normal: s [3], t [3].
void oracle_frame(const double* n, double* s, double* t) {
  Frame f = make_frame(V3(n[0], n[1], n[2]));
  s[0] = f.s.x; s[1] = f.s.y; s[2] = f.s.z;
  t[0] = f.t.x; t[1] = f.t.y; t[2] = f.t.z;
}

// Environment map: density of direction d, and a sample for (u1, u2).
double oracle_env_pdf(void* h, const double* d) {
  return env_pdf(*(Scene*)h, V3(d[0], d[1], d[2]));
}
int oracle_env_sample(void* h, double u1, double u2, double* d) {
  V3 v;
  if (!env_sample(*(Scene*)h, u1, u2, &v)) return 0;
  d[0] = v.x; d[1] = v.y; d[2] = v.z;
  return 1;
}
void oracle_env_lookup(void* h, const double* d, double* rgb) {
  RGB c = env_lookup(*(Scene*)h, V3(d[0], d[1], d[2]));
  rgb[0] = c[0]; rgb[1] = c[1]; rgb[2] = c[2];
}

// Camera ray directions for given pixels and jitters (test hook).
void oracle_camera_dirs(const double* cam, int64_t n, const double* px, const double* py,
                        double* dirs) {
  Cam k = make_cam(cam);
  for (int64_t i = 0; i < n; ++i) {
    int x = (int)std::floor(px[i]), y = (int)std::floor(py[i]);
    V3 d = cam_dir(k, x, y, px[i] - x, py[i] - y);
    dirs[3 * i] = d.x; dirs[3 * i + 1] = d.y; dirs[3 * i + 2] = d.z;
  }
}

// Mean squared error loss over n values and its gradient 2 (I - T) / n.
double oracle_loss_l2(int64_t n, const double* img, const double* target, double* adj) {
  double acc = 0;
  for (int64_t i = 0; i < n; ++i) {
    double r = img[i] - target[i];
    acc += r * r;
    if (adj) adj[i] = 2.0 * r / n;
  }
  return acc / n;
}

// One Adam step (Kingma & Ba 2015) at step t >= 1 with bias correction, then
// clamping of the parameter to [lo, hi].
void oracle_adam(int64_t n, double* p, const double* g, double* m, double* v, double lr,
                 double b1, double b2, double eps, int t, double lo, double hi) {
  double c1 = 1.0 - std::pow(b1, t), c2 = 1.0 - std::pow(b2, t);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    double x = p[i] - lr * mh / (std::sqrt(vh) + eps);
    p[i] = std::min(std::max(x, lo), hi);
  }
}

// ---------------------------------------------------------------------------
// radiance cache
// cfg: [L, F, log2T, Nmin, Nmax, lo0, lo1, lo2, hi0, hi1, hi2] (doubles)
// ---------------------------------------------------------------------------
static GridCfg grid_cfg(const double* c) {
  GridCfg g;
  g.L = (int)c[0]; g.F = (int)c[1]; g.log2T = (int)c[2]; g.Nmin = c[3]; g.Nmax = c[4];
  for (int a = 0; a < 3; ++a) { g.lo[a] = c[5 + a]; g.hi[a] = c[8 + a]; }
  return g;
}

void oracle_sh16(const double* d, double* out) { sh16(d, out); }

int oracle_level_res(const double* cfg, int l) { return level_res(grid_cfg(cfg), l); }

void oracle_grid_corners(const double* cfg, int l, const double* xn, uint32_t* idx, double* w) {
  grid_corners(grid_cfg(cfg), l, xn, idx, w);
}

// feat [n][13] raw features -> out [n][80]; grid: float [L][T][F]
void oracle_nrc_encode(int64_t n, const double* feat, const double* cfg, const float* grid,
                       double* out) {
  GridCfg g = grid_cfg(cfg);
  for (int64_t i = 0; i < n; ++i) encode(g, grid, feat + 13 * i, out + 80 * i);
}

// grad [L][T][F] += sum_i trilinear-weight * dfeat[i][l*F + f]
void oracle_nrc_grid_backward(int64_t n, const double* feat, const double* cfg,
                              const double* dfeat, double* grad) {
  GridCfg g = grid_cfg(cfg);
  uint64_t T = 1ull << g.log2T;
  for (int64_t i = 0; i < n; ++i) {
    double xn[3];
    normalise_pos(g, feat + 13 * i, xn);
    for (int l = 0; l < g.L; ++l) {
      uint32_t idx[8];
      double w[8];
      grid_corners(g, l, xn, idx, w);
      for (int ft = 0; ft < g.F; ++ft)
        for (int k = 0; k < 8; ++k)
          grad[((uint64_t)l * T + idx[k]) * g.F + ft] += w[k] * dfeat[80 * i + l * g.F + ft];
    }
  }
}

int oracle_mlp_num_weights(void) { return kNumWeights; }

void oracle_mlp_forward(int64_t n, const double* x, const double* W, int emu, int n_threads,
                        double* y) {
  parallel_for(n, n_threads, [&](int, int64_t i) { mlp_forward(W, x + kIn * i, emu != 0, nullptr, y + 3 * i); });
}

// dW (accumulated) and dx [n][80] for output gradients dy [n][3]
void oracle_mlp_backward(int64_t n, const double* x, const double* W, const double* dy, int emu,
                         double* dW, double* dx) {
  for (int64_t i = 0; i < n; ++i) mlp_backward(W, x + kIn * i, dy + 3 * i, emu != 0, dW, dx + kIn * i);
}

// Term-magnitude sums (mlp_term_magnitudes) for n samples: aW accumulated
// over the samples, adx [n][80], ay [n][3].
void oracle_mlp_term_magnitudes(int64_t n, const double* x, const double* W, const double* dy,
                                int emu, double* aW, double* adx, double* ay) {
  for (int64_t i = 0; i < n; ++i)
    mlp_term_magnitudes(W, x + kIn * i, dy + 3 * i, emu != 0, aW, adx + kIn * i, ay + 3 * i);
}

double oracle_rel_l2(int64_t n, const double* y, const double* t, double* dy) {
  return rel_l2(n, y, t, dy);
}

// Cached estimator: each sample's path stops at its record vertex (first
// scattering vertex with index >= K) and adds beta * max(C, 0) with C the
// network's output on the encoded record.  Same pixel ids/layout as
// oracle_render.  W: network weights (double); grid: float [L][T][F].
void oracle_render_cached(void* h, const float* const* textures, const float* roughness,
                          const double* cams, int n_cams, int spp, int max_depth, int rr_depth,
                          uint32_t flags, uint64_t seed, int K, const double* cfg,
                          const float* grid, const double* W, int emu, int64_t n_pix,
                          const int64_t* pixel_ids, int n_threads, double* out, int* ambiguous) {
  const Scene& s = *(Scene*)h;
  Params P{textures, roughness};
  Opts opt{spp, max_depth, rr_depth, flags, seed};
  GridCfg g = grid_cfg(cfg);
  std::vector<Cam> cs;
  for (int c = 0; c < n_cams; ++c) cs.push_back(make_cam(cams + 12 * c));
  const int Wd = cs[0].W, Ht = cs[0].H;
  parallel_for(n_pix, n_threads, [&](int, int64_t i) {
    int64_t pid = pixel_ids[i];
    int cam = (int)(pid / ((int64_t)Wd * Ht));
    int y = (int)((pid / Wd) % Ht), x = (int)(pid % Wd);
    RGB acc;
    int n_amb = 0;
    for (int sidx = 0; sidx < spp; ++sidx) {
      uint64_t gi = (uint64_t)pid * spp + sidx;
      Stream st = make_stream(seed, gi);
      V3 o, d;
      bool amb = false;
      t_amb = ambiguous ? &amb : nullptr;
      camera_ray(cs[cam], st, x, y, &o, &d);
      CacheHook ch;
      ch.K = K;
      ch.mode = 0;
      RGB L = trace_sample(s, P, opt, st, o, d, nullptr, nullptr, &ch);
      t_amb = nullptr;
      if (ch.has) {
        double enc[80], yv[3];
        encode(g, grid, ch.feat, enc);
        mlp_forward(W, enc, emu != 0, nullptr, yv);
        for (int c = 0; c < 3; ++c) L[c] += ch.beta[c] * std::max(yv[c], 0.0);
      }
      acc = acc + L;
      n_amb += amb ? 1 : 0;
    }
    for (int c = 0; c < 3; ++c) out[3 * i + c] = acc[c] / spp;
    if (ambiguous) ambiguous[i] = n_amb;
  });
}

// Reverse-mode gradient of the cached estimator (same adjoint convention as
// oracle_adjoint, reverse sweep).  The term beta * max(C, 0) at the record
// vertex enters the sweep like emission found there, so it reaches earlier
// vertices' BSDF derivatives through beta.  input_grad = 0: that is all (the
// cache output is detached).  input_grad = 1: the network is differentiated
// too, through the inputs that are scene parameters -- the chain rule on
// dL . beta * max(C(x), 0): output gradient dy_c = dL_c beta_c [C_c > 0],
// back through the network to x, and d/dx of the albedo features (10..12)
// and the roughness feature (9) added to the texel / roughness slot they
// were read from.  With it the result is the derivative of the cached
// estimator itself, not of its detached form.
void oracle_adjoint_cached(void* h, const float* const* textures, const float* roughness,
                           const double* cams, int n_cams, int spp, int max_depth, int rr_depth,
                           uint32_t flags, uint64_t seed, int K, const double* cfg,
                           const float* grid, const double* W, int emu, int input_grad,
                           int64_t n_pix, const int64_t* pixel_ids, const double* adj,
                           int n_threads, double* const* grad_tex, double* grad_rough) {
  const Scene& s = *(Scene*)h;
  Params P{textures, roughness};
  Opts opt{spp, max_depth, rr_depth, flags, seed};
  GridCfg g = grid_cfg(cfg);
  std::vector<Cam> cs;
  for (int c = 0; c < n_cams; ++c) cs.push_back(make_cam(cams + 12 * c));
  const int Wd = cs[0].W, Ht = cs[0].H;
  int nth = std::max(1, n_threads);
  std::vector<GradAcc> accs(nth);
  std::vector<std::vector<double>> dWs(nth);  // weight gradient of mlp_backward, unused
  parallel_for(n_pix, nth, [&](int t, int64_t i) {
    int64_t pid = pixel_ids[i];
    int cam = (int)(pid / ((int64_t)Wd * Ht));
    int y = (int)((pid / Wd) % Ht), x = (int)(pid % Wd);
    RGB dL(adj[3 * i] / spp, adj[3 * i + 1] / spp, adj[3 * i + 2] / spp);
    if (is_zero(dL)) return;
    std::vector<VertexRec> recs;
    for (int sidx = 0; sidx < spp; ++sidx) {
      uint64_t gi = (uint64_t)pid * spp + sidx;
      Stream st = make_stream(seed, gi);
      V3 o, d;
      camera_ray(cs[cam], st, x, y, &o, &d);
      CacheHook ch;
      ch.K = K;
      ch.mode = 0;
      trace_sample(s, P, opt, st, o, d, &recs, nullptr, &ch);
      if (ch.has) {
        double enc[80], yv[3];
        encode(g, grid, ch.feat, enc);
        mlp_forward(W, enc, emu != 0, nullptr, yv);
        RGB c;
        for (int ci = 0; ci < 3; ++ci) c[ci] = ch.beta[ci] * std::max(yv[ci], 0.0);
        recs.back().emit = recs.back().emit + c;
        if (input_grad && (ch.tex_in || ch.rough_in)) {
          double dy[3], dx[80];
          for (int ci = 0; ci < 3; ++ci) dy[ci] = yv[ci] > 0 ? dL[ci] * ch.beta[ci] : 0.0;
          if (dy[0] != 0 || dy[1] != 0 || dy[2] != 0) {
            if (dWs[t].empty()) dWs[t].assign(kNumWeights, 0.0);
            mlp_backward(W, enc, dy, emu != 0, dWs[t].data(), dx);
            if (ch.tex_in) accs[t].add(ch.k_tex, RGB(dx[65], dx[66], dx[67]));
            if (ch.rough_in) accs[t].add(ch.k_rough, RGB(dx[64], 0, 0));
          }
        }
      }
      reverse_sweep(recs, dL, &accs[t]);
    }
  });
  for (auto& a : accs) {
    for (auto& kv : a.m) {
      Key k = kv.first;
      if (is_texel(k)) {
        int tex = (int)((k >> 40) & 0x7FFFFF);
        int64_t texel = (int64_t)(k & ((1ull << 40) - 1));
        if (grad_tex && grad_tex[tex])
          for (int c = 0; c < 3; ++c) grad_tex[tex][3 * texel + c] += kv.second[c];
      } else if (grad_rough) {
        grad_rough[(int)k] += kv.second[0];
      }
    }
  }
}

// Training records: path j (key = seed, g = j) starts at pixel
// floor(r n_pix / 2^32) with r the first word of block (camera, dim 2), runs a
// plain path, and, if it reaches a record vertex, returns its features and
// target = (radiance collected after the record point) / beta there
// (channels with beta = 0 get target 0).  valid[j] = 1 if recorded.
void oracle_train_records(void* h, const float* const* textures, const float* roughness,
                          const double* cams, int n_cams, int max_depth, int rr_depth,
                          uint32_t flags, uint64_t seed, int K, int64_t n_paths, int n_threads,
                          double* feat, double* target, int* valid, int* ambiguous,
                          double* beta_out, double* lat_out, double* ltot_out) {
  const Scene& s = *(Scene*)h;
  Params P{textures, roughness};
  Opts opt{1, max_depth, rr_depth, flags, seed};
  std::vector<Cam> cs;
  for (int c = 0; c < n_cams; ++c) cs.push_back(make_cam(cams + 12 * c));
  const int Wd = cs[0].W, Ht = cs[0].H;
  const uint32_t n_pix = (uint32_t)((int64_t)n_cams * Wd * Ht);
  parallel_for(n_paths, n_threads, [&](int, int64_t j) {
    Stream st = make_stream(seed, (uint64_t)j);
    uint32_t r[4];
    st.block(kCameraBlock, 2, r);
    uint32_t pid = pick(r[0], n_pix);
    int cam = (int)(pid / ((uint32_t)Wd * Ht));
    int y = (int)((pid / Wd) % Ht), x = (int)(pid % Wd);
    V3 o, d;
    bool amb = false;
    t_amb = ambiguous ? &amb : nullptr;
    camera_ray(cs[cam], st, x, y, &o, &d);
    CacheHook ch;
    ch.K = K;
    ch.mode = 1;
    RGB L = trace_sample(s, P, opt, st, o, d, nullptr, nullptr, &ch);
    t_amb = nullptr;
    valid[j] = ch.has ? 1 : 0;
    if (ambiguous) ambiguous[j] = amb ? 1 : 0;
    for (int c = 0; c < 13; ++c) feat[13 * j + c] = ch.has ? ch.feat[c] : 0.0;
    for (int c = 0; c < 3; ++c) {
      double b = ch.beta[c];
      target[3 * j + c] = (ch.has && b != 0) ? (L[c] - ch.L_at[c]) / b : 0.0;
      if (beta_out) beta_out[3 * j + c] = ch.has ? b : 0.0;
      if (lat_out) lat_out[3 * j + c] = ch.has ? ch.L_at[c] : L[c];
      if (ltot_out) ltot_out[3 * j + c] = L[c];
    }
  });
}

// Self-training records: path j (key = seed, g = j, pixel as in
// oracle_train_records) runs the cached estimator with record vertex K (the
// first scattering vertex with index >= K, max_depth as given), so its
// radiance beyond that vertex is the cache's own answer there.  Every
// scattering vertex v_k with k < K on the way gives record j (K - 1) + k - 1:
// its features and target = (L_end - L_k) / beta_k (0 for channels with
// beta_k = 0), with L_end the path's cached estimate (radiance up to the record
// vertex plus beta max(C, 0) there) and L_k the radiance collected up to and
// including v_k's emission -- the radiance scattered from v_k.  valid marks
// the records written; ambiguous[j] as in oracle_train_records.
void oracle_train_records_self(void* h, const float* const* textures, const float* roughness,
                               const double* cams, int n_cams, int max_depth, int rr_depth,
                               uint32_t flags, uint64_t seed, int K, const double* cfg,
                               const float* grid, const double* W, int emu, int64_t n_paths,
                               int n_threads, double* feat, double* target, int* valid,
                               int* ambiguous) {
  const Scene& s = *(Scene*)h;
  Params P{textures, roughness};
  Opts opt{1, max_depth, rr_depth, flags, seed};
  GridCfg g = grid_cfg(cfg);
  std::vector<Cam> cs;
  for (int c = 0; c < n_cams; ++c) cs.push_back(make_cam(cams + 12 * c));
  const int Wd = cs[0].W, Ht = cs[0].H;
  const uint32_t n_pix = (uint32_t)((int64_t)n_cams * Wd * Ht);
  const int R = K - 1;  // records per path
  parallel_for(n_paths, n_threads, [&](int, int64_t j) {
    Stream st = make_stream(seed, (uint64_t)j);
    uint32_t r[4];
    st.block(kCameraBlock, 2, r);
    uint32_t pid = pick(r[0], n_pix);
    int cam = (int)(pid / ((uint32_t)Wd * Ht));
    int y = (int)((pid / Wd) % Ht), x = (int)(pid % Wd);
    V3 o, d;
    bool amb = false;
    t_amb = ambiguous ? &amb : nullptr;
    camera_ray(cs[cam], st, x, y, &o, &d);
    std::vector<CacheHook::Visit> visits;
    CacheHook ch;
    ch.K = K;
    ch.mode = 0;
    ch.visits = &visits;
    RGB L = trace_sample(s, P, opt, st, o, d, nullptr, nullptr, &ch);
    t_amb = nullptr;
    if (ch.has) {
      double enc[80], yv[3];
      encode(g, grid, ch.feat, enc);
      mlp_forward(W, enc, emu != 0, nullptr, yv);
      for (int c = 0; c < 3; ++c) L[c] += ch.beta[c] * std::max(yv[c], 0.0);
    }
    if (ambiguous) ambiguous[j] = amb ? 1 : 0;
    for (int i = 0; i < R; ++i) {
      valid[j * R + i] = 0;
      for (int c = 0; c < 13; ++c) feat[13 * (j * R + i) + c] = 0.0;
      for (int c = 0; c < 3; ++c) target[3 * (j * R + i) + c] = 0.0;
    }
    for (const auto& v : visits) {
      const int64_t slot = j * R + (v.k - 1);
      valid[slot] = 1;
      for (int c = 0; c < 13; ++c) feat[13 * slot + c] = v.feat[c];
      for (int c = 0; c < 3; ++c)
        target[3 * slot + c] = v.beta[c] != 0 ? (L[c] - v.L_at[c]) / v.beta[c] : 0.0;
    }
  });
}

}  // extern "C"
