// Host runtime of the C ABI: argument validation, scene build (binned-SAH
// BVH, tables, environment sampling distributions), upload into the
// caller's device buffer, and the entry points that launch the kernels.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "drt_internal.h"

using namespace drt;

namespace {

thread_local std::string g_err;

drt_status fail(drt_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

drt_status ok() {
  g_err.clear();
  return DRT_OK;
}

drt_status hip_fail(hipError_t e, const char* what) {
  return fail(DRT_EHIP, "%s: %s", what, hipGetErrorString(e));
}

inline uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Limits of the rendering calls: samples per call (n_cams x W x H x spp),
// path segments, and paths of a wavefront or training workspace.
constexpr int64_t kMaxSamples = (int64_t)1 << 46;
constexpr int kMaxDepth = 1 << 16;

// a * b <= lim for non-negative a and b, decided without overflowing
inline bool prod_le(int64_t a, int64_t b, int64_t lim) { return b == 0 || a <= lim / b; }

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
drt_status validate(const drt_scene_desc* d) {
  if (!d) return fail(DRT_EINVAL, "scene desc is NULL");
  if (d->n_triangles <= 0) return fail(DRT_EINVAL, "scene has no triangles");
  if (d->n_vertices <= 0 || !d->positions || !d->indices || !d->tri_material || !d->tri_emitter)
    return fail(DRT_EINVAL, "scene arrays missing");
  if (d->n_materials <= 0 || !d->materials) return fail(DRT_EINVAL, "scene has no materials");
  if (d->n_emitters < 0 || (d->n_emitters > 0 && !d->emitters))
    return fail(DRT_EINVAL, "emitter array missing");
  if (d->n_textures < 0 || d->n_textures > DRT_MAX_TEXTURES)
    return fail(DRT_EINVAL, "n_textures must be in [0, %d]", DRT_MAX_TEXTURES);
  if (d->n_textures > 0 && !d->textures) return fail(DRT_EINVAL, "texture descs missing");
  for (int t = 0; t < d->n_textures; ++t)
    if (d->textures[t].width <= 0 || d->textures[t].height <= 0)
      return fail(DRT_EINVAL, "texture %d has an empty size", t);
  if (d->n_roughness < 0) return fail(DRT_EINVAL, "n_roughness < 0");
  if ((int64_t)d->n_triangles * 3 > INT32_MAX) return fail(DRT_EUNSUPPORTED, "too many triangles");
  for (int64_t i = 0; i < 3 * (int64_t)d->n_triangles; ++i)
    if (d->indices[i] < 0 || d->indices[i] >= d->n_vertices)
      return fail(DRT_EINVAL, "triangle %lld references vertex %d of %d", (long long)(i / 3),
                  d->indices[i], d->n_vertices);
  for (int i = 0; i < d->n_triangles; ++i) {
    if (d->tri_material[i] < 0 || d->tri_material[i] >= d->n_materials)
      return fail(DRT_EINVAL, "triangle %d has material %d", i, d->tri_material[i]);
    int e = d->tri_emitter[i];
    if (e < -1 || e >= d->n_emitters) return fail(DRT_EINVAL, "triangle %d has emitter %d", i, e);
    if (e >= 0 && d->emitters[e].type != DRT_EMITTER_AREA)
      return fail(DRT_EINVAL, "triangle %d references a non-area emitter", i);
  }
  for (int i = 0; i < 3 * d->n_vertices; ++i)
    if (!std::isfinite(d->positions[i])) return fail(DRT_EINVAL, "non-finite vertex position");
  for (int m = 0; m < d->n_materials; ++m) {
    const drt_material& mt = d->materials[m];
    if (mt.type < DRT_BSDF_NULL || mt.type > DRT_BSDF_MASK)
      return fail(DRT_EINVAL, "material %d has unknown type %d", m, mt.type);
    if (mt.texture >= d->n_textures || mt.texture < -1)
      return fail(DRT_EINVAL, "material %d texture %d out of range", m, mt.texture);
    if (mt.type == DRT_BSDF_DIFFUSE_TEXTURED && mt.texture < 0)
      return fail(DRT_EINVAL, "material %d: textured diffuse without a texture", m);
    if (mt.rough_slot >= d->n_roughness || mt.rough_slot < -1)
      return fail(DRT_EINVAL, "material %d roughness slot %d out of range", m, mt.rough_slot);
  }
  int n_env = 0;
  for (int e = 0; e < d->n_emitters; ++e) {
    int t = d->emitters[e].type;
    if (t < DRT_EMITTER_AREA || t > DRT_EMITTER_DIRECTIONAL)
      return fail(DRT_EINVAL, "emitter %d has unknown type %d", e, t);
    if (t == DRT_EMITTER_ENV) ++n_env;
  }
  if (n_env > 1) return fail(DRT_EINVAL, "at most one environment emitter");
  if (n_env == 1 && (!d->envmap || d->env_width <= 0 || d->env_height <= 0))
    return fail(DRT_EINVAL, "environment emitter without an environment map");
  return DRT_OK;
}

// ---------------------------------------------------------------------------
// BVH build: binned SAH over triangle centroids, two-child nodes.
// ---------------------------------------------------------------------------
struct Box {
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  void grow(const Box& b) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], b.lo[a]);
      hi[a] = std::max(hi[a], b.hi[a]);
    }
  }
  void grow(const float* p) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], p[a]);
      hi[a] = std::max(hi[a], p[a]);
    }
  }
  double area() const {
    double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    if (dx < 0 || dy < 0 || dz < 0) return 0;
    return 2.0 * (dx * dy + dy * dz + dz * dx);
  }
};

struct BuildNode {
  Box box;
  int begin, count;   // triangle range in the permutation
  int child[2];       // -1 for a leaf
  int depth;
};

struct Builder {
  const std::vector<Box>& tb;
  const std::vector<float>& cen;  // 3 per triangle
  std::vector<int> perm;
  std::vector<BuildNode> nodes;
  int max_depth = 0, forced = 0;
  static constexpr int kBins = 16;
  static constexpr int kMaxLeaf = 4;
  static constexpr double kTrav = 1.0, kIsect = 1.0;

  Builder(const std::vector<Box>& b, const std::vector<float>& c, int n) : tb(b), cen(c) {
    perm.resize(n);
    for (int i = 0; i < n; ++i) perm[i] = i;
  }

  int make(int begin, int count, int depth) {
    BuildNode nd;
    nd.begin = begin;
    nd.count = count;
    nd.child[0] = nd.child[1] = -1;
    nd.depth = depth;
    for (int i = begin; i < begin + count; ++i) nd.box.grow(tb[perm[i]]);
    nodes.push_back(nd);
    max_depth = std::max(max_depth, depth);
    return (int)nodes.size() - 1;
  }

  // Split node `id` if that pays (SAH) or is needed (count > kMaxLeaf), as
  // long as it stays within the interior-depth limit.
  void split(int id) {
    std::vector<int> todo{id};
    while (!todo.empty()) {
      int cur = todo.back();
      todo.pop_back();
      BuildNode nd = nodes[cur];
      if (nd.count <= 1) continue;
      if (nd.depth >= kMaxInteriorDepth) {
        if (nd.count > kMaxLeaf) ++forced;
        continue;
      }
      Box cb;
      for (int i = nd.begin; i < nd.begin + nd.count; ++i) cb.grow(&cen[3 * perm[i]]);
      int best_axis = -1, best_bin = -1;
      double best_cost = INFINITY;
      for (int a = 0; a < 3; ++a) {
        double ext = (double)cb.hi[a] - cb.lo[a];
        if (!(ext > 0)) continue;
        Box bb[kBins];
        int bc[kBins] = {0};
        double k = kBins / ext;
        for (int i = nd.begin; i < nd.begin + nd.count; ++i) {
          int t = perm[i];
          int b = std::min(kBins - 1, (int)((cen[3 * t + a] - cb.lo[a]) * k));
          bc[b]++;
          bb[b].grow(tb[t]);
        }
        double rarea[kBins];
        int rcnt[kBins];
        Box acc;
        int c = 0;
        for (int b = kBins - 1; b > 0; --b) {
          acc.grow(bb[b]);
          c += bc[b];
          rarea[b] = acc.area();
          rcnt[b] = c;
        }
        acc = Box();
        c = 0;
        for (int b = 0; b < kBins - 1; ++b) {
          acc.grow(bb[b]);
          c += bc[b];
          if (c == 0 || rcnt[b + 1] == 0) continue;
          double cost = acc.area() * c + rarea[b + 1] * rcnt[b + 1];
          if (cost < best_cost) {
            best_cost = cost;
            best_axis = a;
            best_bin = b;
          }
        }
      }
      double parea = nd.box.area();
      double leaf_cost = kIsect * nd.count;
      double split_cost = best_axis >= 0 && parea > 0 ? kTrav + kIsect * best_cost / parea : INFINITY;
      if (nd.count <= kMaxLeaf && split_cost >= leaf_cost) continue;
      int mid;
      if (best_axis < 0) {
        mid = nd.begin + nd.count / 2;  // all centroids coincide: split by index
      } else {
        double ext = (double)cb.hi[best_axis] - cb.lo[best_axis];
        double k = kBins / ext;
        auto it = std::partition(perm.begin() + nd.begin, perm.begin() + nd.begin + nd.count,
                                 [&](int t) {
                                   int b = std::min(kBins - 1,
                                                    (int)((cen[3 * t + best_axis] - cb.lo[best_axis]) * k));
                                   return b <= best_bin;
                                 });
        mid = (int)(it - perm.begin());
        if (mid == nd.begin || mid == nd.begin + nd.count) mid = nd.begin + nd.count / 2;
      }
      int l = make(nd.begin, mid - nd.begin, nd.depth + 1);
      int r = make(mid, nd.begin + nd.count - mid, nd.depth + 1);
      nodes[cur].child[0] = l;
      nodes[cur].child[1] = r;
      todo.push_back(r);
      todo.push_back(l);
    }
  }
};

void set_child_box(DNode& n, int slot, const Box& b) {
  for (int a = 0; a < 3; ++a) {
    n.box[a][slot] = b.lo[a];
    n.box[3 + a][slot] = b.hi[a];
  }
}

}  // namespace

struct drt_scene {
  DScene dev;                 // device pointers into the caller's buffer
  drt_scene_info info;
  bool on_device = false;
};

namespace {

// Everything the scene build produces, in host memory, laid out exactly as
// in the device buffer.
struct Packed {
  std::vector<unsigned char> bytes;
  uint64_t off_nodes, off_tris, off_shade, off_mats, off_ems, off_env, off_puv, off_crow, off_ccol;
  drt_scene_info info;
  DScene layout;  // pointers relative to the buffer start (offsets)
};

uint64_t plan_bytes(const drt_scene_desc* d, uint64_t* offs = nullptr) {
  uint64_t n_nodes = std::max<int64_t>(1, d->n_triangles);
  uint64_t o = 0, off[9];
  off[0] = o; o = align256(o + n_nodes * sizeof(DNode));
  off[1] = o; o = align256(o + (uint64_t)d->n_triangles * sizeof(DTri));
  off[2] = o; o = align256(o + (uint64_t)d->n_triangles * sizeof(DShade));
  off[3] = o; o = align256(o + (uint64_t)d->n_materials * sizeof(DMaterial));
  off[4] = o; o = align256(o + (uint64_t)std::max(1, d->n_emitters) * sizeof(DEmitter));
  uint64_t ew = d->envmap ? d->env_width : 0, eh = d->envmap ? d->env_height : 0;
  off[5] = o; o = align256(o + ew * eh * 3 * 4);
  off[6] = o; o = align256(o + ew * eh * 4);
  off[7] = o; o = align256(o + (eh + 1) * 4);
  off[8] = o; o = align256(o + eh * (ew + 1) * 4);
  if (offs) std::memcpy(offs, off, sizeof(off));
  return o;
}

drt_status build_packed(const drt_scene_desc* d, Packed* P) {
  drt_status st = validate(d);
  if (st != DRT_OK) return st;
  const int nt = d->n_triangles;
  uint64_t off[9];
  uint64_t total = plan_bytes(d, off);
  try {
    P->bytes.assign(total, 0);
  } catch (const std::bad_alloc&) {
    return fail(DRT_ENOMEM, "host allocation of %llu bytes failed", (unsigned long long)total);
  }
  P->off_nodes = off[0]; P->off_tris = off[1]; P->off_shade = off[2]; P->off_mats = off[3];
  P->off_ems = off[4]; P->off_env = off[5]; P->off_puv = off[6]; P->off_crow = off[7];
  P->off_ccol = off[8];

  // per-triangle bounds and centroids
  std::vector<Box> tb(nt);
  std::vector<float> cen(3 * (size_t)nt);
  Box scene_box;
  for (int i = 0; i < nt; ++i) {
    for (int k = 0; k < 3; ++k) tb[i].grow(&d->positions[3 * (size_t)d->indices[3 * (size_t)i + k]]);
    for (int a = 0; a < 3; ++a) cen[3 * (size_t)i + a] = 0.5f * (tb[i].lo[a] + tb[i].hi[a]);
    scene_box.grow(tb[i]);
  }
  Box vbox;
  for (int i = 0; i < d->n_vertices; ++i) vbox.grow(&d->positions[3 * (size_t)i]);

  Builder b(tb, cen, nt);
  b.nodes.reserve(2 * (size_t)nt);
  int root = b.make(0, nt, 0);
  b.split(root);
  if (b.nodes[root].child[0] < 0) {
    // the root must be a two-child node: split small scenes by index, and
    // let a single triangle appear in both children
    int l, r;
    if (nt >= 2) {
      l = b.make(0, nt / 2, 1);
      r = b.make(nt / 2, nt - nt / 2, 1);
    } else {
      l = b.make(0, 1, 1);
      r = b.make(0, 1, 1);
    }
    b.nodes[root].child[0] = l;
    b.nodes[root].child[1] = r;
  }

  // four-wide nodes: every binary interior node at even depth becomes one;
  // its children are its grandchildren, or a child itself where that child
  // is a leaf (pre-order numbering)
  auto slots_of = [&](int id, int out[4]) {
    int n = 0;
    for (int c : b.nodes[id].child) {
      const BuildNode& cn = b.nodes[c];
      if (cn.child[0] < 0) out[n++] = c;
      else { out[n++] = cn.child[0]; out[n++] = cn.child[1]; }
    }
    return n;
  };
  std::vector<int> dn_of(b.nodes.size(), -1);
  std::vector<int> order;
  std::vector<std::pair<int, int>> stack{{root, 0}};  // (binary node, four-wide level)
  int levels = 0;
  while (!stack.empty()) {
    const auto [id, level] = stack.back();
    stack.pop_back();
    levels = std::max(levels, level + 1);
    dn_of[id] = (int)order.size();
    order.push_back(id);
    int sl[4];
    int n = slots_of(id, sl);
    for (int k = n - 1; k >= 0; --k)
      if (b.nodes[sl[k]].child[0] >= 0) stack.push_back({sl[k], level + 1});
  }
  DNode* nodes = (DNode*)&P->bytes[off[0]];
  int n_leaves = 0;
  for (size_t k = 0; k < order.size(); ++k) {
    DNode& n = nodes[k];
    std::memset(&n, 0, sizeof(n));
    int sl[4];
    int ns = slots_of(order[k], sl);
    for (int s = 0; s < 4; ++s) {
      if (s >= ns) {
        n.child[s] = 0;
        n.count[s] = -1;
        continue;
      }
      const BuildNode& ch = b.nodes[sl[s]];
      set_child_box(n, s, ch.box);
      if (ch.child[0] < 0) {
        n.child[s] = ch.begin;
        n.count[s] = ch.count;
        ++n_leaves;
      } else {
        n.child[s] = dn_of[sl[s]];
        n.count[s] = 0;
      }
    }
  }
  // triangles in leaf order
  DTri* tris = (DTri*)&P->bytes[off[1]];
  for (int i = 0; i < nt; ++i) {
    int t = b.perm[i];
    const float* p0 = &d->positions[3 * (size_t)d->indices[3 * (size_t)t]];
    const float* p1 = &d->positions[3 * (size_t)d->indices[3 * (size_t)t + 1]];
    const float* p2 = &d->positions[3 * (size_t)d->indices[3 * (size_t)t + 2]];
    DTri& r = tris[i];
    r.p0x = p0[0]; r.p0y = p0[1]; r.p0z = p0[2];
    r.p1x = p1[0]; r.p1y = p1[1]; r.p1z = p1[2];
    r.p2x = p2[0]; r.p2y = p2[1]; r.p2z = p2[2];
    r.prim = t;
    r.flags = d->materials[d->tri_material[t]].type == DRT_BSDF_NULL ? 1 : 0;
    r.pad = 0;
  }
  DShade* sh = (DShade*)&P->bytes[off[2]];
  for (int t = 0; t < nt; ++t) {
    float uv[6] = {0, 0, 0, 0, 0, 0};
    if (d->uvs)
      for (int k = 0; k < 3; ++k) {
        int v = d->indices[3 * (size_t)t + k];
        uv[2 * k] = d->uvs[2 * (size_t)v];
        uv[2 * k + 1] = d->uvs[2 * (size_t)v + 1];
      }
    // the geometric normal, in double and rounded once (zero-area triangles,
    // which the watertight test never reports as hit, get +z)
    const float* q[3];
    for (int k = 0; k < 3; ++k) q[k] = &d->positions[3 * (size_t)d->indices[3 * (size_t)t + k]];
    const double e1[3] = {(double)q[1][0] - q[0][0], (double)q[1][1] - q[0][1], (double)q[1][2] - q[0][2]};
    const double e2[3] = {(double)q[2][0] - q[0][0], (double)q[2][1] - q[0][1], (double)q[2][2] - q[0][2]};
    const double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                         e1[0] * e2[1] - e1[1] * e2[0]};
    const double len = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    const float n[3] = {len > 0 ? (float)(c[0] / len) : 0.f, len > 0 ? (float)(c[1] / len) : 0.f,
                        len > 0 ? (float)(c[2] / len) : 1.f};
    sh[t] = DShade{uv[0], uv[1], uv[2], uv[3], uv[4], uv[5], d->tri_material[t], d->tri_emitter[t],
                   n[0], n[1], n[2], 0};
  }
  DMaterial* mats = (DMaterial*)&P->bytes[off[3]];
  for (int m = 0; m < d->n_materials; ++m) {
    const drt_material& s = d->materials[m];
    DMaterial& o = mats[m];
    std::memset(&o, 0, sizeof(o));
    o.type = s.type; o.texture = s.texture; o.rough_slot = s.rough_slot;
    for (int c = 0; c < 3; ++c) { o.albedo[c] = s.albedo[c]; o.f0[c] = s.f0[c]; }
    o.alpha = s.alpha; o.eta = s.eta; o.opacity = s.opacity;
  }
  DEmitter* ems = (DEmitter*)&P->bytes[off[4]];
  int env_emitter = -1;
  for (int e = 0; e < d->n_emitters; ++e) {
    const drt_emitter& s = d->emitters[e];
    DEmitter& o = ems[e];
    std::memset(&o, 0, sizeof(o));
    o.type = s.type;
    double e1[3], e2[3], c[3];
    for (int a = 0; a < 3; ++a) {
      o.p0[a] = s.p0[a]; o.e1[a] = s.e1[a]; o.e2[a] = s.e2[a]; o.radiance[a] = s.radiance[a];
      e1[a] = s.e1[a]; e2[a] = s.e2[a];
    }
    c[0] = e1[1] * e2[2] - e1[2] * e2[1];
    c[1] = e1[2] * e2[0] - e1[0] * e2[2];
    c[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double area = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    o.area = (float)area;
    for (int a = 0; a < 3; ++a) o.n[a] = area > 0 ? (float)(c[a] / area) : (a == 2 ? 1.f : 0.f);
    if (s.type == DRT_EMITTER_DIRECTIONAL) {
      double l = std::sqrt((double)s.p0[0] * s.p0[0] + (double)s.p0[1] * s.p0[1] +
                           (double)s.p0[2] * s.p0[2]);
      for (int a = 0; a < 3; ++a) o.p0[a] = l > 0 ? (float)(s.p0[a] / l) : 0.f;
    }
    if (s.type == DRT_EMITTER_ENV) env_emitter = e;
  }
  // environment: radiance, (u,v)-density and CDFs of luminance * sin(theta)
  int ew = d->envmap ? d->env_width : 0, eh = d->envmap ? d->env_height : 0;
  if (ew > 0 && eh > 0) {
    float* env = (float*)&P->bytes[off[5]];
    float* puv = (float*)&P->bytes[off[6]];
    float* crow = (float*)&P->bytes[off[7]];
    float* ccol = (float*)&P->bytes[off[8]];
    std::memcpy(env, d->envmap, (size_t)ew * eh * 3 * sizeof(float));
    std::vector<double> w((size_t)ew * eh), rs(eh, 0.0);
    double total = 0;
    for (int r = 0; r < eh; ++r) {
      double st_ = std::sin(M_PI * (r + 0.5) / eh);
      for (int c = 0; c < ew; ++c) {
        const float* p = &d->envmap[3 * ((size_t)r * ew + c)];
        double y = 0.2126 * p[0] + 0.7152 * p[1] + 0.0722 * p[2];
        w[(size_t)r * ew + c] = std::max(y, 0.0) * st_;
        rs[r] += w[(size_t)r * ew + c];
      }
      total += rs[r];
    }
    double acc = 0;
    crow[0] = 0.f;
    for (int r = 0; r < eh; ++r) {
      acc += rs[r];
      crow[r + 1] = total > 0 ? (float)(acc / total) : 0.f;
      float* cc = &ccol[(size_t)r * (ew + 1)];
      cc[0] = 0.f;
      double a2 = 0;
      for (int c = 0; c < ew; ++c) {
        a2 += w[(size_t)r * ew + c];
        cc[c + 1] = rs[r] > 0 ? (float)(a2 / rs[r]) : (float)(c + 1) / ew;
        puv[(size_t)r * ew + c] = total > 0 ? (float)(w[(size_t)r * ew + c] / total * ew * eh) : 0.f;
      }
      cc[ew] = 1.f;
    }
    if (total > 0) crow[eh] = 1.f;
  }

  float ext = 0;
  for (int a = 0; a < 3; ++a) ext = std::max(ext, vbox.hi[a] - vbox.lo[a]);
  drt_scene_info& info = P->info;
  std::memset(&info, 0, sizeof(info));
  info.n_nodes = (int32_t)order.size();
  info.n_leaves = n_leaves;
  info.max_depth = b.max_depth;
  info.forced_leaves = b.forced;
  info.n_triangles = nt;
  info.n_materials = d->n_materials;
  info.n_emitters = d->n_emitters;
  info.n_textures = d->n_textures;
  info.n_roughness = d->n_roughness;
  info.env_width = ew;
  info.env_height = eh;
  info.eps = (float)(1e-4 * (double)ext);
  for (int a = 0; a < 3; ++a) { info.bounds_lo[a] = vbox.lo[a]; info.bounds_hi[a] = vbox.hi[a]; }
  info.device_bytes = total;

  DScene& L = P->layout;
  std::memset(&L, 0, sizeof(L));
  L.n_ems = d->n_emitters;
  L.env_w = ew;
  L.env_h = eh;
  L.env_emitter = env_emitter;
  L.n_mats = d->n_materials;
  L.n_rough = d->n_roughness;
  L.n_tex = d->n_textures;
  L.eps = info.eps;
  // the megakernels' LDS copy of the tree and triangles: a traversal visits
  // at most 3 x levels stacked nodes (three of a node's four children wait
  // on the stack per level)
  L.n_nodes = info.n_nodes;
  L.n_tris = nt;
  const int64_t lds_bytes = (int64_t)info.n_nodes * (int64_t)sizeof(DNode) +
                            (int64_t)nt * (int64_t)(sizeof(DTri) + sizeof(DShade)) +
                            (int64_t)d->n_materials * (int64_t)sizeof(DMaterial) +
                            (int64_t)d->n_emitters * (int64_t)sizeof(DEmitter);
  L.lds_scene = 3 * levels <= kStackDepthSmall && lds_bytes <= kLdsSceneBytes;
  info.lds_copy = L.lds_scene;
  for (int t = 0; t < d->n_textures; ++t) {
    L.tex_w[t] = d->textures[t].width;
    L.tex_h[t] = d->textures[t].height;
  }
  return DRT_OK;
}

void bind(DScene& s, const Packed& P, unsigned char* base) {
  s = P.layout;
  s.nodes = (const DNode*)(base + P.off_nodes);
  s.tris = (const DTri*)(base + P.off_tris);
  s.shade = (const DShade*)(base + P.off_shade);
  s.mats = (const DMaterial*)(base + P.off_mats);
  s.ems = (const DEmitter*)(base + P.off_ems);
  s.env = (const float*)(base + P.off_env);
  s.env_puv = (const float*)(base + P.off_puv);
  s.env_cdf_row = (const float*)(base + P.off_crow);
  s.env_cdf_col = (const float*)(base + P.off_ccol);
}

drt_status check_params(const drt_scene* s, const drt_params* p, const drt_camera* cams,
                        int32_t n_cams, const drt_render_opts* o, DParams* dp, DCams* dc,
                        DRender* dr) {
  if (!s) return fail(DRT_EINVAL, "scene is NULL");
  if (!s->on_device) return fail(DRT_ESTATE, "scene was packed on the host, not uploaded");
  if (!p || !cams || !o) return fail(DRT_EINVAL, "params, cameras and opts are required");
  if (n_cams < 1 || n_cams > DRT_MAX_CAMERAS)
    return fail(DRT_EINVAL, "n_cams must be in [1, %d]", DRT_MAX_CAMERAS);
  if (o->spp < 1) return fail(DRT_EINVAL, "spp must be >= 1");
  if (o->max_depth < 1 || o->max_depth > kMaxDepth)
    return fail(DRT_EINVAL, "max_depth must be in [1, %d]", kMaxDepth);
  if (o->rr_depth < 1) return fail(DRT_EINVAL, "rr_depth must be >= 1");
  const int W = cams[0].width, H = cams[0].height;
  if (W <= 0 || H <= 0) return fail(DRT_EINVAL, "camera size must be positive");
  if (tiles_of(H) > kMaxTileRows)
    return fail(DRT_EUNSUPPORTED, "image height above %d pixels", kMaxTileRows * kTile);
  int64_t samples = n_cams;
  for (const int64_t f : {(int64_t)W, (int64_t)H, (int64_t)o->spp}) {
    if (!prod_le(samples, f, kMaxSamples)) return fail(DRT_EUNSUPPORTED, "sample count too large");
    samples *= f;
  }
  const DScene& sc = s->dev;
  for (int t = 0; t < sc.n_tex; ++t)
    if (!p->textures[t]) return fail(DRT_EINVAL, "texture %d pointer is NULL", t);
  if (sc.n_rough > 0 && !p->roughness) return fail(DRT_EINVAL, "roughness pointer is NULL");
  std::memset(dp, 0, sizeof(*dp));
  for (int t = 0; t < DRT_MAX_TEXTURES; ++t) dp->tex[t] = t < sc.n_tex ? p->textures[t] : nullptr;
  dp->rough = p->roughness;
  std::memset(dc, 0, sizeof(*dc));
  dc->n = n_cams;
  dc->width = W;
  dc->height = H;
  for (int c = 0; c < n_cams; ++c) {
    const drt_camera& k = cams[c];
    if (k.width != W || k.height != H) return fail(DRT_EINVAL, "cameras differ in size");
    if (!(k.fov_y_deg > 0 && k.fov_y_deg < 180)) return fail(DRT_EINVAL, "fov_y out of (0,180)");
    double o3[3] = {k.origin[0], k.origin[1], k.origin[2]};
    double f[3] = {k.target[0] - o3[0], k.target[1] - o3[1], k.target[2] - o3[2]};
    double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(fl > 0)) return fail(DRT_EINVAL, "camera %d: target equals origin", c);
    for (double& x : f) x /= fl;
    double u[3] = {k.up[0], k.up[1], k.up[2]};
    double r[3] = {f[1] * u[2] - f[2] * u[1], f[2] * u[0] - f[0] * u[2], f[0] * u[1] - f[1] * u[0]};
    double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rl > 0)) return fail(DRT_EINVAL, "camera %d: up is parallel to the view direction", c);
    for (double& x : r) x /= rl;
    double v[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    DCam& d = dc->cam[c];
    d.ox = (float)o3[0]; d.oy = (float)o3[1]; d.oz = (float)o3[2];
    d.fx = (float)f[0]; d.fy = (float)f[1]; d.fz = (float)f[2];
    d.rx = (float)r[0]; d.ry = (float)r[1]; d.rz = (float)r[2];
    d.ux = (float)v[0]; d.uy = (float)v[1]; d.uz = (float)v[2];
    d.tan_half = (float)std::tan(k.fov_y_deg * M_PI / 360.0);
    d.aspect = (float)((double)W / H);
  }
  dr->spp = o->spp;
  dr->max_depth = o->max_depth;
  dr->rr_depth = o->rr_depth;
  dr->flags = o->flags;
  dr->key0 = (uint32_t)o->seed;
  dr->key1 = (uint32_t)(o->seed >> 32);
  dr->stats = o->stats;
  dr->hits = nullptr;
  dr->items = nullptr;
  return DRT_OK;
}

// Query buffers of the cached calls: the int32 scratch (8-byte aligned)
// holds ids | order | spatial keys | parameter references (2 per query) |
// one padding entry when the capacity is odd | sort pairs (2 per query,
// 8-byte aligned) | histogram (drt_nrc_query_ints).  The references are
// written only when io.qref is set.
static int64_t query_pairs_offset(int64_t capacity) { return (5 * capacity + 1) & ~(int64_t)1; }
static DNrcIO query_io(const DNrcNet& net, const drt_nrc_config* cfg, float* queries,
                       int32_t* ints, int32_t* count, int64_t capacity) {
  DNrcIO io = {};
  io.rec = queries;
  io.qpix = ints;
  io.count = count;
  io.capacity = capacity;
  io.K = cfg->trunc_vertex;
  io.qbin = reinterpret_cast<uint32_t*>(ints + 2 * capacity);
  for (int a = 0; a < 3; ++a) {
    io.lo[a] = net.lo[a];
    io.inv_ext[a] = net.inv_ext[a];
  }
  return io;
}

// Sort the queries by spatial key, then let the network answer them.
static hipError_t answer_queries(const DNrcNet& net, const float* weights, const DNrcIO& io,
                                 int64_t need, float scale, float* out, hipStream_t st) {
  int* order = io.qpix + io.capacity;
  int* pairs = io.qpix + query_pairs_offset(io.capacity);
  uint32_t* hist = reinterpret_cast<uint32_t*>(pairs + 2 * io.capacity);
  hipError_t e = launch_query_sort(io.qbin, io.count, need, hist, pairs, order, st);
  if (e != hipSuccess) return e;
  return launch_nrc_infer(net, weights, io.rec, io.qpix, order, io.count, need, scale, out, st);
}

drt_status nrc_net(const drt_nrc_config* c, const uint16_t* grid, DNrcNet* net) {
  if (!c) return fail(DRT_EINVAL, "cache config is NULL");
  if (c->levels != DRT_NRC_LEVELS || c->features != 2)
    return fail(DRT_EUNSUPPORTED, "the cache has 16 levels of 2 features");
  if (c->log2_table < 10 || c->log2_table > 24) return fail(DRT_EINVAL, "log2_table must be in [10, 24]");
  if (c->base_res < 1 || c->max_res < c->base_res) return fail(DRT_EINVAL, "bad grid resolutions");
  if (c->trunc_vertex < 2) return fail(DRT_EINVAL, "trunc_vertex must be >= 2");
  std::memset(net, 0, sizeof(*net));
  net->grid = reinterpret_cast<const uint32_t*>(grid);
  net->log2_table = c->log2_table;
  const double T = std::ldexp(1.0, c->log2_table);
  for (int l = 0; l < DRT_NRC_LEVELS; ++l) {
    double r = c->base_res * std::exp(l * (std::log((double)c->max_res) - std::log((double)c->base_res)) /
                                      (DRT_NRC_LEVELS - 1));
    int N = (int)std::floor(r + 1e-6);
    net->res[l] = N;
    net->dense[l] = (double)(N + 1) * (N + 1) * (N + 1) <= T ? 1 : 0;
  }
  for (int a = 0; a < 3; ++a) {
    double e = (double)c->bbox_hi[a] - c->bbox_lo[a];
    net->lo[a] = c->bbox_lo[a];
    net->inv_ext[a] = e > 0 ? (float)(1.0 / e) : 0.f;
  }
  return DRT_OK;
}

}  // namespace

extern "C" {

const char* drt_last_error(void) { return g_err.c_str(); }

const char* drt_version(void) { return "drt 0.1 (gfx950)"; }

drt_status drt_scene_plan(const drt_scene_desc* desc, uint64_t* device_bytes) {
  if (!device_bytes) return fail(DRT_EINVAL, "device_bytes is NULL");
  drt_status st = validate(desc);
  if (st != DRT_OK) return st;
  *device_bytes = plan_bytes(desc);
  return ok();
}

drt_status drt_scene_pack(const drt_scene_desc* desc, void* host_buffer, uint64_t buffer_bytes,
                          drt_scene** out) {
  if (!out || !host_buffer) return fail(DRT_EINVAL, "host_buffer and out are required");
  *out = nullptr;
  Packed P;
  drt_status st = build_packed(desc, &P);
  if (st != DRT_OK) return st;
  if (buffer_bytes < P.bytes.size())
    return fail(DRT_EINVAL, "buffer too small: %llu < %llu", (unsigned long long)buffer_bytes,
                (unsigned long long)P.bytes.size());
  std::memcpy(host_buffer, P.bytes.data(), P.bytes.size());
  drt_scene* s = new (std::nothrow) drt_scene();
  if (!s) return fail(DRT_ENOMEM, "out of host memory");
  bind(s->dev, P, (unsigned char*)host_buffer);
  s->info = P.info;
  s->on_device = false;
  *out = s;
  return ok();
}

drt_status drt_scene_upload(const drt_scene_desc* desc, void* device_buffer, uint64_t buffer_bytes,
                            void* hip_stream, drt_scene** out) {
  if (!out || !device_buffer) return fail(DRT_EINVAL, "device_buffer and out are required");
  *out = nullptr;
  if (((uintptr_t)device_buffer & 255) != 0) return fail(DRT_EINVAL, "device_buffer not 256-byte aligned");
  Packed P;
  drt_status st = build_packed(desc, &P);
  if (st != DRT_OK) return st;
  if (buffer_bytes < P.bytes.size())
    return fail(DRT_EINVAL, "buffer too small: %llu < %llu", (unsigned long long)buffer_bytes,
                (unsigned long long)P.bytes.size());
  hipStream_t stream = (hipStream_t)hip_stream;
  hipError_t e = hipMemcpyAsync(device_buffer, P.bytes.data(), P.bytes.size(),
                                hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "scene upload copy");
  e = hipStreamSynchronize(stream);  // the staging bytes die with this call
  if (e != hipSuccess) return hip_fail(e, "scene upload sync");
  drt_scene* s = new (std::nothrow) drt_scene();
  if (!s) return fail(DRT_ENOMEM, "out of host memory");
  bind(s->dev, P, (unsigned char*)device_buffer);
  s->info = P.info;
  s->on_device = true;
  *out = s;
  return ok();
}

drt_status drt_scene_info_get(const drt_scene* scene, drt_scene_info* out) {
  if (!scene || !out) return fail(DRT_EINVAL, "scene and out are required");
  *out = scene->info;
  return ok();
}

drt_status drt_scene_destroy(drt_scene* scene) {
  delete scene;
  return ok();
}

drt_status drt_render_forward(const drt_scene* scene, const drt_params* params,
                              const drt_camera* cams, int32_t n_cams, const drt_render_opts* opts,
                              float* image, void* hip_stream) {
  DParams dp;
  DCams dc;
  DRender dr;
  drt_status st = check_params(scene, params, cams, n_cams, opts, &dp, &dc, &dr);
  if (st != DRT_OK) return st;
  if (!image) return fail(DRT_EINVAL, "image is NULL");
  hipError_t e = launch_render_forward(scene->dev, dp, dc, dr, image, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "render_forward launch");
  return ok();
}

drt_status drt_render_adjoint(const drt_scene* scene, const drt_params* params,
                              const drt_camera* cams, int32_t n_cams, const drt_render_opts* opts,
                              const float* adj_image, const drt_grads* grads, void* hip_stream) {
  DParams dp;
  DCams dc;
  DRender dr;
  drt_status st = check_params(scene, params, cams, n_cams, opts, &dp, &dc, &dr);
  if (st != DRT_OK) return st;
  if (!adj_image || !grads) return fail(DRT_EINVAL, "adj_image and grads are required");
  DGrads dg;
  std::memset(&dg, 0, sizeof(dg));
  for (int t = 0; t < scene->dev.n_tex; ++t) dg.tex[t] = grads->textures[t];
  dg.rough = scene->dev.n_rough > 0 ? grads->roughness : nullptr;
  hipError_t e = launch_render_adjoint(scene->dev, dp, dc, dr, adj_image, dg, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "render_adjoint launch");
  return ok();
}

// One record slot (max_depth x kBlock x 16 B) per workgroup of 8x8 pixels;
// 0 for invalid sizes.
static int64_t record_slot_bytes(int32_t n_cams, int32_t width, int32_t height, int32_t max_depth) {
  if (n_cams < 1 || n_cams > DRT_MAX_CAMERAS || width < 1 || height < 1 || max_depth < 1 ||
      max_depth > kMaxDepth)
    return 0;
  // < 2^5 x 2^28 x 2^28 tiles; their records must stay far from int64's end
  const int64_t groups = (int64_t)n_cams * tiles_of(width) * tiles_of(height);
  const int64_t per_group = (int64_t)max_depth * kBlock * (int64_t)sizeof(int4);
  if (!prod_le(groups, per_group, (int64_t)1 << 60)) return 0;
  return groups * per_group;
}

// Record buffer of the replayed adjoint: a 256-byte header (the persistent
// workgroups' work counter), then one slot per persistent workgroup -- as
// many as are resident on the current device, at most one per work unit
// (tile x sample range).
static constexpr int64_t kHitHeader = 256;
int64_t drt_render_adjoint_hit_bytes(int32_t n_cams, int32_t width, int32_t height, int32_t spp,
                                     int32_t max_depth) {
  if (spp < 1) return 0;
  const int64_t per_tile = record_slot_bytes(n_cams, width, height, max_depth);  // 0 when too large
  if (per_tile <= 0) return 0;
  const int64_t tiles = (int64_t)n_cams * tiles_of(width) * tiles_of(height);
  const int64_t units = tiles * adjoint_split(spp);
  const int resident = adjoint_resident_groups();
  const int64_t slots = resident > 0 && resident < units ? resident : units;
  return kHitHeader + per_tile / tiles * slots;
}

drt_status drt_render_adjoint_hits(const drt_scene* scene, const drt_params* params,
                                   const drt_camera* cams, int32_t n_cams,
                                   const drt_render_opts* opts, const float* adj_image,
                                   const drt_grads* grads, void* hit_records, int64_t hit_bytes,
                                   void* hip_stream) {
  DParams dp;
  DCams dc;
  DRender dr;
  drt_status st = check_params(scene, params, cams, n_cams, opts, &dp, &dc, &dr);
  if (st != DRT_OK) return st;
  if (!adj_image || !grads || !hit_records)
    return fail(DRT_EINVAL, "adj_image, grads and hit_records are required");
  // the persistent workgroups count work units in 32 bits
  const int64_t tiles = (int64_t)n_cams * tiles_of(cams[0].width) *
                        tiles_of(cams[0].height);
  if (tiles * adjoint_split(opts->spp) > ((int64_t)1 << 31))
    return fail(DRT_EUNSUPPORTED, "image too large for the persistent replay");
  const int64_t need = drt_render_adjoint_hit_bytes(n_cams, cams[0].width, cams[0].height,
                                                    opts->spp, opts->max_depth);
  if (need <= 0 || hit_bytes < need)
    return fail(DRT_EINVAL, "hit_records of %lld bytes < %lld", (long long)hit_bytes, (long long)need);
  if (((uintptr_t)hit_records & 15) != 0) return fail(DRT_EINVAL, "hit_records is not 16-byte aligned");
  DGrads dg;
  std::memset(&dg, 0, sizeof(dg));
  for (int t = 0; t < scene->dev.n_tex; ++t) dg.tex[t] = grads->textures[t];
  dg.rough = scene->dev.n_rough > 0 ? grads->roughness : nullptr;
  dr.items = static_cast<uint32_t*>(hit_records);
  dr.hits = reinterpret_cast<int4*>(static_cast<char*>(hit_records) + kHitHeader);
  hipError_t e = launch_render_adjoint(scene->dev, dp, dc, dr, adj_image, dg, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "render_adjoint launch");
  return ok();
}

drt_status drt_render_adjoint_noalloc(const drt_scene* scene, const drt_params* params,
                                      const drt_camera* cams, int32_t n_cams,
                                      const drt_render_opts* opts, const float* adj_image,
                                      const drt_grads* grads, void* hip_stream) {
  DParams dp;
  DCams dc;
  DRender dr;
  drt_status st = check_params(scene, params, cams, n_cams, opts, &dp, &dc, &dr);
  if (st != DRT_OK) return st;
  if (!adj_image || !grads) return fail(DRT_EINVAL, "adj_image and grads are required");
  const int64_t tiles = (int64_t)n_cams * tiles_of(cams[0].width) *
                        tiles_of(cams[0].height);
  if (tiles * adjoint_split(opts->spp) > ((int64_t)1 << 31))
    return fail(DRT_EUNSUPPORTED, "image too large for the persistent replay");
  const int64_t need = drt_render_adjoint_hit_bytes(n_cams, cams[0].width, cams[0].height,
                                                    opts->spp, opts->max_depth);
  if (need <= 0) return fail(DRT_EINVAL, "invalid sizes for the intersection records");
  if (need > kNoAllocScratchBytes)
    return fail(DRT_EUNSUPPORTED,
                "intersection records of %lld bytes exceed the library's scratch of %lld bytes "
                "(lower max_depth; 4096 resident workgroups allow max_depth <= 8)",
                (long long)need, (long long)kNoAllocScratchBytes);
  void* scratch = nullptr;
  hipError_t e = noalloc_scratch(&scratch);
  if (e != hipSuccess) return hip_fail(e, "scratch address (hipGetSymbolAddress)");
  DGrads dg;
  std::memset(&dg, 0, sizeof(dg));
  for (int t = 0; t < scene->dev.n_tex; ++t) dg.tex[t] = grads->textures[t];
  dg.rough = scene->dev.n_rough > 0 ? grads->roughness : nullptr;
  dr.items = static_cast<uint32_t*>(scratch);
  dr.hits = reinterpret_cast<int4*>(static_cast<char*>(scratch) + kHitHeader);
  e = launch_render_adjoint(scene->dev, dp, dc, dr, adj_image, dg, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "render_adjoint launch");
  return ok();
}

int64_t drt_render_wavefront_workspace_bytes(int64_t n_paths) {
  return n_paths < 0 || n_paths > kMaxSamples ? 0 : wavefront_workspace_bytes(n_paths);
}

drt_status drt_render_wavefront(const drt_scene* scene, const drt_params* params,
                                const drt_camera* cams, int32_t n_cams, const drt_render_opts* opts,
                                void* workspace, int64_t workspace_bytes, float* image,
                                void* hip_stream) {
  DParams dp;
  DCams dc;
  DRender dr;
  drt_status st = check_params(scene, params, cams, n_cams, opts, &dp, &dc, &dr);
  if (st != DRT_OK) return st;
  if (!image || !workspace) return fail(DRT_EINVAL, "image and workspace are required");
  const int64_t n = (int64_t)n_cams * cams[0].width * cams[0].height * opts->spp;
  if (workspace_bytes < wavefront_workspace_bytes(n))
    return fail(DRT_EINVAL, "workspace of %lld bytes < %lld", (long long)workspace_bytes,
                (long long)wavefront_workspace_bytes(n));
  if (((uintptr_t)workspace & 15) != 0) return fail(DRT_EINVAL, "workspace is not 16-byte aligned");
  dr.stats = nullptr;
  hipError_t e = launch_render_wavefront(scene->dev, dp, dc, dr, workspace, image, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "render_wavefront launch");
  return ok();
}

int64_t drt_render_adjoint_wavefront_workspace_bytes(int64_t n_paths) {
  return n_paths < 0 || n_paths > kMaxSamples ? 0 : wavefront_adjoint_workspace_bytes(n_paths);
}

drt_status drt_render_adjoint_wavefront(const drt_scene* scene, const drt_params* params,
                                        const drt_camera* cams, int32_t n_cams,
                                        const drt_render_opts* opts, const float* adj_image,
                                        const drt_grads* grads, void* workspace,
                                        int64_t workspace_bytes, void* hip_stream) {
  DParams dp;
  DCams dc;
  DRender dr;
  drt_status st = check_params(scene, params, cams, n_cams, opts, &dp, &dc, &dr);
  if (st != DRT_OK) return st;
  if (!adj_image || !grads || !workspace)
    return fail(DRT_EINVAL, "adj_image, grads and workspace are required");
  const int64_t n = (int64_t)n_cams * cams[0].width * cams[0].height * opts->spp;
  if (workspace_bytes < wavefront_adjoint_workspace_bytes(n))
    return fail(DRT_EINVAL, "workspace of %lld bytes < %lld", (long long)workspace_bytes,
                (long long)wavefront_adjoint_workspace_bytes(n));
  if (((uintptr_t)workspace & 15) != 0) return fail(DRT_EINVAL, "workspace is not 16-byte aligned");
  DGrads dg;
  std::memset(&dg, 0, sizeof(dg));
  for (int t = 0; t < scene->dev.n_tex; ++t) dg.tex[t] = grads->textures[t];
  dg.rough = scene->dev.n_rough > 0 ? grads->roughness : nullptr;
  dr.stats = nullptr;
  hipError_t e = launch_render_adjoint_wavefront(scene->dev, dp, dc, dr, adj_image, dg, workspace,
                                                 (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "render_adjoint_wavefront launch");
  return ok();
}

int64_t drt_render_checkpointed_workspace_bytes(int64_t n_paths, int32_t max_depth) {
  if (n_paths < 0 || n_paths > ((int64_t)1 << 40) || max_depth < 1 || max_depth > kMaxDepth) return 0;
  return checkpoint_workspace_bytes(n_paths, max_depth);
}

// Shared checks of the two checkpointed calls.
static drt_status checkpoint_args(const drt_scene* scene, const drt_params* params,
                                  const drt_camera* cams, int32_t n_cams,
                                  const drt_render_opts* opts, void* workspace,
                                  int64_t workspace_bytes, DParams* dp, DCams* dc, DRender* dr) {
  drt_status st = check_params(scene, params, cams, n_cams, opts, dp, dc, dr);
  if (st != DRT_OK) return st;
  if (!workspace) return fail(DRT_EINVAL, "workspace is required");
  const int64_t n = (int64_t)n_cams * cams[0].width * cams[0].height * opts->spp;
  const int64_t need = checkpoint_workspace_bytes(n, opts->max_depth);
  if (workspace_bytes < need)
    return fail(DRT_EINVAL, "workspace of %lld bytes < %lld", (long long)workspace_bytes,
                (long long)need);
  if (((uintptr_t)workspace & 15) != 0) return fail(DRT_EINVAL, "workspace is not 16-byte aligned");
  dr->stats = nullptr;
  return DRT_OK;
}

drt_status drt_render_checkpointed_forward(const drt_scene* scene, const drt_params* params,
                                           const drt_camera* cams, int32_t n_cams,
                                           const drt_render_opts* opts, void* workspace,
                                           int64_t workspace_bytes, float* image,
                                           void* hip_stream) {
  DParams dp;
  DCams dc;
  DRender dr;
  drt_status st = checkpoint_args(scene, params, cams, n_cams, opts, workspace, workspace_bytes,
                                  &dp, &dc, &dr);
  if (st != DRT_OK) return st;
  if (!image) return fail(DRT_EINVAL, "image is required");
  hipError_t e = launch_render_checkpoint_forward(scene->dev, dp, dc, dr, workspace, image,
                                                  (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "checkpointed forward launch");
  return ok();
}

drt_status drt_render_checkpointed_adjoint(const drt_scene* scene, const drt_params* params,
                                           const drt_camera* cams, int32_t n_cams,
                                           const drt_render_opts* opts, const float* adj_image,
                                           const drt_grads* grads, void* workspace,
                                           int64_t workspace_bytes, void* hip_stream) {
  DParams dp;
  DCams dc;
  DRender dr;
  drt_status st = checkpoint_args(scene, params, cams, n_cams, opts, workspace, workspace_bytes,
                                  &dp, &dc, &dr);
  if (st != DRT_OK) return st;
  if (!adj_image || !grads) return fail(DRT_EINVAL, "adj_image and grads are required");
  DGrads dg;
  std::memset(&dg, 0, sizeof(dg));
  for (int t = 0; t < scene->dev.n_tex; ++t) dg.tex[t] = grads->textures[t];
  dg.rough = scene->dev.n_rough > 0 ? grads->roughness : nullptr;
  hipError_t e = launch_render_checkpoint_adjoint(scene->dev, dp, dc, dr, adj_image, dg, workspace,
                                                  (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "checkpointed adjoint launch");
  return ok();
}

drt_status drt_render_jvp(const drt_scene* scene, const drt_params* params, const drt_camera* cams,
                          int32_t n_cams, const drt_render_opts* opts, const drt_grads* direction,
                          float* image_tangent, void* hip_stream) {
  DParams dp;
  DCams dc;
  DRender dr;
  drt_status st = check_params(scene, params, cams, n_cams, opts, &dp, &dc, &dr);
  if (st != DRT_OK) return st;
  if (!direction || !image_tangent) return fail(DRT_EINVAL, "direction and image_tangent are required");
  DGrads dt;
  std::memset(&dt, 0, sizeof(dt));
  for (int t = 0; t < scene->dev.n_tex; ++t) dt.tex[t] = direction->textures[t];
  dt.rough = scene->dev.n_rough > 0 ? direction->roughness : nullptr;
  hipError_t e = launch_render_jvp(scene->dev, dp, dc, dr, dt, image_tangent, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "render_jvp launch");
  return ok();
}

drt_status drt_trace(const drt_scene* scene, const float* rays, int64_t n, int32_t mode,
                     drt_hit* hits, void* hip_stream) {
  if (!scene) return fail(DRT_EINVAL, "scene is required");
  if (!scene->on_device) return fail(DRT_ESTATE, "scene was packed on the host, not uploaded");
  if (n < 0) return fail(DRT_EINVAL, "n < 0");
  if (mode != 0 && mode != 1) return fail(DRT_EINVAL, "mode must be 0 or 1");
  if (n == 0) return ok();
  if (!rays || !hits) return fail(DRT_EINVAL, "rays and hits are required");
  hipError_t e = launch_trace(scene->dev, rays, n, mode, hits, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "trace launch");
  return ok();
}

drt_status drt_philox(const uint32_t* counters, const uint32_t* keys, int64_t n, uint32_t* out,
                      void* hip_stream) {
  if (n < 0) return fail(DRT_EINVAL, "n < 0");
  if (n == 0) return ok();
  if (!counters || !keys || !out) return fail(DRT_EINVAL, "counters, keys and out are required");
  hipError_t e = launch_philox(counters, keys, n, out, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "philox launch");
  return ok();
}

int64_t drt_loss_workspace_floats(int64_t n) { return loss_workspace_floats(n); }

drt_status drt_loss_l2(const float* img, const float* target, int64_t n, float* adj, float* loss,
                       float* workspace, void* hip_stream) {
  if (!img || !target || !loss || !workspace) return fail(DRT_EINVAL, "null pointer argument");
  if (n <= 0) return fail(DRT_EINVAL, "n must be positive");
  hipError_t e = launch_loss_l2(img, target, n, adj, loss, workspace, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "loss launch");
  return ok();
}

drt_status drt_adam_step(float* param, float* grad, float* m, float* v, int64_t n,
                         const drt_adam_opts* opts, void* hip_stream) {
  if (!opts) return fail(DRT_EINVAL, "opts is required");
  if (n < 0) return fail(DRT_EINVAL, "n < 0");
  if (n > 0 && (!param || !grad || !m || !v)) return fail(DRT_EINVAL, "null pointer argument");
  if (opts->step < 1) return fail(DRT_EINVAL, "Adam step must be >= 1");
  if (!(opts->lr >= 0) || !(opts->beta1 >= 0 && opts->beta1 < 1) ||
      !(opts->beta2 >= 0 && opts->beta2 < 1) || !(opts->eps > 0))
    return fail(DRT_EINVAL, "invalid Adam hyper-parameters");
  if (n == 0) return ok();
  hipError_t e = launch_adam(param, grad, m, v, n, *opts, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "adam launch");
  return ok();
}

drt_status drt_nrc_encode(const drt_nrc_config* cfg, const uint16_t* grid, const float* records,
                          int64_t n, float* x, void* hip_stream) {
  DNrcNet net;
  drt_status st = nrc_net(cfg, grid, &net);
  if (st != DRT_OK) return st;
  if (n < 0) return fail(DRT_EINVAL, "n < 0");
  if (n == 0) return ok();
  if (!grid || !records || !x) return fail(DRT_EINVAL, "null pointer argument");
  hipError_t e = launch_nrc_encode(net, records, n, x, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "nrc_encode launch");
  return ok();
}

drt_status drt_nrc_grid_backward(const drt_nrc_config* cfg, const float* records, const float* dx,
                                 int64_t n, float* dgrid, void* hip_stream) {
  DNrcNet net;
  drt_status st = nrc_net(cfg, nullptr, &net);
  if (st != DRT_OK) return st;
  if (n < 0 || n > ((int64_t)1 << 32)) return fail(DRT_EINVAL, "n out of range");
  if (n == 0) return ok();
  if (!records || !dx || !dgrid) return fail(DRT_EINVAL, "null pointer argument");
  hipError_t e = launch_nrc_grid_backward(net, records, dx, n, dgrid, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "nrc_grid_backward launch");
  return ok();
}

drt_status drt_nrc_forward(const float* weights, const float* x, int64_t n, float* y,
                           void* hip_stream) {
  if (n < 0) return fail(DRT_EINVAL, "n < 0");
  if (n == 0) return ok();
  if (!weights || !x || !y) return fail(DRT_EINVAL, "null pointer argument");
  hipError_t e = launch_nrc_forward(weights, x, n, y, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "nrc_forward launch");
  return ok();
}

drt_status drt_nrc_backward(const float* weights, const float* x, const float* dy, int64_t n,
                            void* workspace, int64_t workspace_bytes, float* dW, float* dx,
                            void* hip_stream) {
  if (n < 0 || n > ((int64_t)1 << 31)) return fail(DRT_EINVAL, "n out of range");
  if (n == 0) return ok();
  if (!weights || !x || !dy || !dW || !workspace) return fail(DRT_EINVAL, "null pointer argument");
  if (workspace_bytes < nrc_train_workspace_bytes(n))
    return fail(DRT_EINVAL, "workspace of %lld bytes < %lld", (long long)workspace_bytes,
                (long long)nrc_train_workspace_bytes(n));
  if (((uintptr_t)workspace & 15) != 0) return fail(DRT_EINVAL, "workspace is not 16-byte aligned");
  hipError_t e = launch_nrc_backward(weights, x, dy, n, workspace, dW, dx, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "nrc_backward launch");
  return ok();
}

drt_status drt_nrc_collect(const drt_scene* scene, const drt_params* params,
                           const drt_camera* cams, int32_t n_cams, const drt_render_opts* opts,
                           const drt_nrc_config* cfg, int64_t n_paths, float* records,
                           int32_t* valid, int32_t* count, void* hip_stream) {
  DParams dp;
  DCams dc;
  DRender dr;
  drt_status st = check_params(scene, params, cams, n_cams, opts, &dp, &dc, &dr);
  if (st != DRT_OK) return st;
  if (!cfg || cfg->trunc_vertex < 2) return fail(DRT_EINVAL, "cache config with trunc_vertex >= 2 required");
  if (n_paths < 0 || n_paths > ((int64_t)1 << 32)) return fail(DRT_EINVAL, "n_paths out of range");
  if (!count) return fail(DRT_EINVAL, "count is NULL");
  hipStream_t stream = (hipStream_t)hip_stream;
  hipError_t e = launch_zero(count, 1, stream);
  if (e != hipSuccess) return hip_fail(e, "zero launch");
  if (n_paths == 0) return ok();
  if (!records || !valid) return fail(DRT_EINVAL, "records and valid are required");
  DNrcIO io = {};
  io.rec = records;
  io.valid = valid;
  io.count = count;
  io.K = cfg->trunc_vertex;
  e = launch_nrc_records(scene->dev, dp, dc, dr, n_paths, io, stream);
  if (e != hipSuccess) return hip_fail(e, "nrc_collect launch");
  return ok();
}

// Workspace of drt_nrc_collect_self, 256-byte aligned parts: tail queries
// [n][16] | query ints | query count | path estimates [n][3] | record
// throughputs [n (K - 1)][3].
static int64_t align256(int64_t b) { return (b + 255) & ~(int64_t)255; }
struct SelfWs {
  int64_t q, ints, qcount, lpath, tbeta, total;
};
static SelfWs self_ws(int64_t n, int K) {
  SelfWs w;
  w.q = 0;
  w.ints = w.q + align256(n * NRC_REC * 4);
  w.qcount = w.ints + align256(drt_nrc_query_ints(n) * 4);
  w.lpath = w.qcount + 256;
  w.tbeta = w.lpath + align256(n * 3 * 4);
  w.total = w.tbeta + align256(n * (K - 1) * 3 * 4);
  return w;
}

int64_t drt_nrc_collect_self_workspace_bytes(int64_t n_paths, int32_t tail_vertex) {
  if (n_paths < 0 || n_paths > INT32_MAX || tail_vertex < 2 || tail_vertex > 32) return 0;
  return self_ws(n_paths, tail_vertex).total;
}

drt_status drt_nrc_collect_self(const drt_scene* scene, const drt_params* params,
                                const drt_camera* cams, int32_t n_cams,
                                const drt_render_opts* opts, const drt_nrc_config* cfg,
                                const float* weights, const uint16_t* grid, int32_t tail_vertex,
                                int64_t n_paths, float* records, int32_t* valid, int32_t* count,
                                void* workspace, int64_t workspace_bytes, void* hip_stream) {
  DParams dp;
  DCams dc;
  DRender dr;
  drt_status st = check_params(scene, params, cams, n_cams, opts, &dp, &dc, &dr);
  if (st != DRT_OK) return st;
  DNrcNet net;
  st = nrc_net(cfg, grid, &net);
  if (st != DRT_OK) return st;
  if (tail_vertex < 2 || tail_vertex > 32) return fail(DRT_EINVAL, "tail_vertex must be in [2, 32]");
  if (n_paths < 0 || n_paths > INT32_MAX || n_paths * (tail_vertex - 1) > ((int64_t)1 << 31))
    return fail(DRT_EINVAL, "n_paths out of range");
  if (!weights || !grid || !count) return fail(DRT_EINVAL, "null pointer argument");
  hipStream_t stream = (hipStream_t)hip_stream;
  hipError_t e = launch_zero(count, 1, stream);
  if (e != hipSuccess) return hip_fail(e, "zero launch");
  if (n_paths == 0) return ok();
  if (!records || !valid) return fail(DRT_EINVAL, "records and valid are required");
  const SelfWs w = self_ws(n_paths, tail_vertex);
  if (!workspace || workspace_bytes < w.total)
    return fail(DRT_EINVAL, "workspace smaller than drt_nrc_collect_self_workspace_bytes");
  char* base = static_cast<char*>(workspace);
  int32_t* qcount = reinterpret_cast<int32_t*>(base + w.qcount);
  DNrcIO io = query_io(net, cfg, reinterpret_cast<float*>(base + w.q),
                       reinterpret_cast<int32_t*>(base + w.ints), qcount, n_paths);
  io.K = tail_vertex;
  io.lsamp = reinterpret_cast<float*>(base + w.lpath);
  io.trec = records;
  io.tbeta = reinterpret_cast<float*>(base + w.tbeta);
  io.valid = valid;
  io.rcount = count;
  e = launch_zero(qcount, 1, stream);
  if (e != hipSuccess) return hip_fail(e, "zero launch");
  e = launch_nrc_records_self(scene->dev, dp, dc, dr, n_paths, io, stream);
  if (e != hipSuccess) return hip_fail(e, "self-training paths launch");
  e = answer_queries(net, weights, io, n_paths, 1.0f, io.lsamp, stream);
  if (e != hipSuccess) return hip_fail(e, "cache query launch");
  e = launch_nrc_self_targets(io, n_paths, stream);
  if (e != hipSuccess) return hip_fail(e, "self-training targets launch");
  return ok();
}

int64_t drt_nrc_train_workspace_bytes(int64_t n) {
  return n < 0 || n > ((int64_t)1 << 31) ? 0 : nrc_train_workspace_bytes(n);
}

drt_status drt_nrc_train(const drt_nrc_config* cfg, const float* weights, const uint16_t* grid,
                         const float* records, const int32_t* valid, const int32_t* count,
                         int64_t n, void* workspace, int64_t workspace_bytes, float* dW,
                         float* dgrid, float* loss, void* hip_stream) {
  DNrcNet net;
  drt_status st = nrc_net(cfg, grid, &net);
  if (st != DRT_OK) return st;
  if (n < 0 || n > ((int64_t)1 << 31)) return fail(DRT_EINVAL, "n out of range");
  if (!weights || !grid || !count || !dW || !dgrid || !loss)
    return fail(DRT_EINVAL, "null pointer argument");
  if (n > 0 && (!records || !valid)) return fail(DRT_EINVAL, "records and valid are required");
  if (n > 0 && (!workspace || workspace_bytes < nrc_train_workspace_bytes(n)))
    return fail(DRT_EINVAL, "workspace of %lld bytes < %lld", (long long)workspace_bytes,
                (long long)nrc_train_workspace_bytes(n));
  if (((uintptr_t)workspace & 15) != 0) return fail(DRT_EINVAL, "workspace is not 16-byte aligned");
  hipStream_t stream = (hipStream_t)hip_stream;
  hipError_t e = launch_zero(loss, 1, stream);
  if (e != hipSuccess) return hip_fail(e, "zero launch");
  if (n == 0) return ok();
  e = launch_nrc_train(net, weights, records, valid, count, n, workspace, dW, dgrid, loss, stream);
  if (e != hipSuccess) return hip_fail(e, "nrc_train launch");
  return ok();
}

drt_status drt_nrc_train_frame(const drt_scene* scene, const drt_params* params,
                               const drt_camera* cams, int32_t n_cams, const drt_render_opts* opts,
                               const drt_nrc_config* cfg, const drt_nrc_frame_opts* frame,
                               const drt_nrc_state* S, void* hip_stream) {
  // every check first: nothing is enqueued on an argument error
  DParams dp;
  DCams dc;
  DRender dr;
  drt_status st = check_params(scene, params, cams, n_cams, opts, &dp, &dc, &dr);
  if (st != DRT_OK) return st;
  if (!frame || !S) return fail(DRT_EINVAL, "frame options and cache state are required");
  DNrcNet net;
  st = nrc_net(cfg, S->grid_half, &net);
  if (st != DRT_OK) return st;
  const int K = frame->self_training;
  if (K == 1 || K < 0 || K > 32) return fail(DRT_EINVAL, "self_training must be 0 or in [2, 32]");
  const int64_t n = frame->n_paths;
  if (n < 1 || n > INT32_MAX) return fail(DRT_EINVAL, "n_paths must be in [1, 2^31)");
  const int64_t n_rec = K ? n * (K - 1) : n;
  if (n_rec > ((int64_t)1 << 31)) return fail(DRT_EINVAL, "too many records");
  if (frame->step < 1) return fail(DRT_EINVAL, "Adam step must be >= 1");
  if (!(frame->lr >= 0) || !(frame->beta1 >= 0 && frame->beta1 < 1) ||
      !(frame->beta2 >= 0 && frame->beta2 < 1) || !(frame->eps > 0))
    return fail(DRT_EINVAL, "invalid Adam hyper-parameters");
  if (!S->weights || !S->weights_m || !S->weights_v || !S->weights_grad || !S->grid || !S->grid_m ||
      !S->grid_v || !S->grid_grad || !S->grid_half || !S->records || !S->valid || !S->count ||
      !S->loss)
    return fail(DRT_EINVAL, "cache state has a NULL buffer");
  if (!S->train_workspace || S->train_workspace_bytes < nrc_train_workspace_bytes(n_rec) ||
      ((uintptr_t)S->train_workspace & 15) != 0)
    return fail(DRT_EINVAL, "train workspace missing, misaligned or smaller than "
                "drt_nrc_train_workspace_bytes(%lld)", (long long)n_rec);
  if (K && (!S->self_workspace || S->self_workspace_bytes < self_ws(n, K).total))
    return fail(DRT_EINVAL, "self-training workspace smaller than drt_nrc_collect_self_workspace_bytes");
  const int64_t n_grid = (int64_t)DRT_NRC_LEVELS << cfg->log2_table << 1;
  drt_render_opts o = *opts;
  o.spp = 1;
  if (K)
    st = drt_nrc_collect_self(scene, params, cams, n_cams, &o, cfg, S->weights, S->grid_half, K, n,
                              S->records, S->valid, S->count, S->self_workspace,
                              S->self_workspace_bytes, hip_stream);
  else
    st = drt_nrc_collect(scene, params, cams, n_cams, &o, cfg, n, S->records, S->valid, S->count,
                         hip_stream);
  if (st != DRT_OK) return st;
  st = drt_nrc_train(cfg, S->weights, S->grid_half, S->records, S->valid, S->count, n_rec,
                     S->train_workspace, S->train_workspace_bytes, S->weights_grad, S->grid_grad,
                     S->loss, hip_stream);
  if (st != DRT_OK) return st;
  drt_adam_opts a = {};
  a.lr = frame->lr;
  a.beta1 = frame->beta1;
  a.beta2 = frame->beta2;
  a.eps = frame->eps;
  a.step = frame->step;
  a.lo = -INFINITY;
  a.hi = INFINITY;
  a.zero_grad = 1;
  st = drt_adam_step(S->weights, S->weights_grad, S->weights_m, S->weights_v, DRT_NRC_WEIGHTS, &a,
                     hip_stream);
  if (st != DRT_OK) return st;
  a.half_out = S->grid_half;
  st = drt_adam_step(S->grid, S->grid_grad, S->grid_m, S->grid_v, n_grid, &a, hip_stream);
  if (st != DRT_OK) return st;
  return ok();
}

int64_t drt_nrc_query_ints(int64_t capacity) {
  return capacity < 0 || capacity > ((int64_t)1 << 40) ? 0
                                                       : query_pairs_offset(capacity) + 2 * capacity + kQueryBins;
}

drt_status drt_render_forward_cached(const drt_scene* scene, const drt_params* params,
                                     const drt_camera* cams, int32_t n_cams,
                                     const drt_render_opts* opts, const drt_nrc_config* cfg,
                                     const float* weights, const uint16_t* grid, float* queries,
                                     int32_t* query_ints, int32_t* query_count,
                                     int64_t capacity, float* image, void* hip_stream) {
  DParams dp;
  DCams dc;
  DRender dr;
  drt_status st = check_params(scene, params, cams, n_cams, opts, &dp, &dc, &dr);
  if (st != DRT_OK) return st;
  DNrcNet net;
  st = nrc_net(cfg, grid, &net);
  if (st != DRT_OK) return st;
  if (!weights || !grid || !queries || !query_ints || !query_count || !image)
    return fail(DRT_EINVAL, "null pointer argument");
  int64_t need = (int64_t)n_cams * cams[0].width * cams[0].height * opts->spp;
  if (capacity < need || need > INT32_MAX)
    return fail(DRT_EINVAL, "query capacity %lld < %lld samples", (long long)capacity, (long long)need);
  if (drt_nrc_query_ints(capacity) == 0) return fail(DRT_EINVAL, "query capacity out of range");
  if ((uintptr_t)query_ints & 7) return fail(DRT_EINVAL, "query_ints must be 8-byte aligned");
  hipStream_t stream = (hipStream_t)hip_stream;
  DNrcIO io = query_io(net, cfg, queries, query_ints, query_count, capacity);
  hipError_t e = launch_zero(query_count, 1, stream);
  if (e != hipSuccess) return hip_fail(e, "zero launch");
  e = launch_render_cached(scene->dev, dp, dc, dr, image, io, stream);
  if (e != hipSuccess) return hip_fail(e, "render_cached launch");
  e = answer_queries(net, weights, io, need, 1.0f / (float)opts->spp, image, stream);
  if (e != hipSuccess) return hip_fail(e, "cache query launch");
  return ok();
}

int64_t drt_render_adjoint_cached_hit_bytes(int32_t n_cams, int32_t width, int32_t height,
                                            int32_t spp, int32_t max_depth) {
  if (spp < 1 || spp > (1 << 20)) return 0;
  const int64_t per_sample = record_slot_bytes(n_cams, width, height, max_depth);
  return prod_le(per_sample, spp, (int64_t)1 << 62) ? per_sample * spp : 0;
}

drt_status drt_render_adjoint_cached(const drt_scene* scene, const drt_params* params,
                                     const drt_camera* cams, int32_t n_cams,
                                     const drt_render_opts* opts, const drt_nrc_config* cfg,
                                     const float* weights, const uint16_t* grid, float* queries,
                                     int32_t* query_ints, int32_t* query_count, int64_t capacity,
                                     float* sample_radiance, const float* adj_image,
                                     const drt_grads* grads, void* hit_records, int64_t hit_bytes,
                                     void* hip_stream) {
  DParams dp;
  DCams dc;
  DRender dr;
  drt_status st = check_params(scene, params, cams, n_cams, opts, &dp, &dc, &dr);
  if (st != DRT_OK) return st;
  DNrcNet net;
  st = nrc_net(cfg, grid, &net);
  if (st != DRT_OK) return st;
  if (!weights || !grid || !queries || !query_ints || !query_count || !sample_radiance ||
      !adj_image || !grads)
    return fail(DRT_EINVAL, "null pointer argument");
  int64_t need = (int64_t)n_cams * cams[0].width * cams[0].height * opts->spp;
  if (capacity < need || need > INT32_MAX)
    return fail(DRT_EINVAL, "query capacity %lld < %lld samples", (long long)capacity, (long long)need);
  if (drt_nrc_query_ints(capacity) == 0) return fail(DRT_EINVAL, "query capacity out of range");
  if ((uintptr_t)query_ints & 7) return fail(DRT_EINVAL, "query_ints must be 8-byte aligned");
  if (hit_records) {
    const int64_t hneed = drt_render_adjoint_cached_hit_bytes(n_cams, cams[0].width, cams[0].height,
                                                              opts->spp, opts->max_depth);
    if (hneed <= 0 || hit_bytes < hneed)
      return fail(DRT_EINVAL, "hit_records of %lld bytes < %lld", (long long)hit_bytes, (long long)hneed);
    if (((uintptr_t)hit_records & 15) != 0) return fail(DRT_EINVAL, "hit_records is not 16-byte aligned");
    dr.hits = static_cast<int4*>(hit_records);
  }
  DGrads dg;
  std::memset(&dg, 0, sizeof(dg));
  for (int t = 0; t < scene->dev.n_tex; ++t) dg.tex[t] = grads->textures[t];
  dg.rough = scene->dev.n_rough > 0 ? grads->roughness : nullptr;
  hipStream_t stream = (hipStream_t)hip_stream;
  DNrcIO io = query_io(net, cfg, queries, query_ints, query_count, capacity);
  io.lsamp = sample_radiance;
  const bool input_grad = (opts->flags & DRT_FLAG_CACHE_INPUT_GRAD) != 0;
  if (input_grad) io.qref = query_ints + 3 * capacity;
  hipError_t e = launch_zero(query_count, 1, stream);
  if (e != hipSuccess) return hip_fail(e, "zero launch");
  e = launch_render_cached(scene->dev, dp, dc, dr, nullptr, io, stream);
  if (e != hipSuccess) return hip_fail(e, "render_cached launch");
  e = answer_queries(net, weights, io, need, 1.0f, sample_radiance, stream);
  if (e != hipSuccess) return hip_fail(e, "cache query launch");
  if (input_grad) {
    // the queries are in key order now (answer_queries sorted them)
    e = launch_nrc_input_grad(net, weights, io.rec, io.qpix, io.qref, io.qpix + capacity, io.count,
                              need, opts->spp, adj_image, dg, stream);
    if (e != hipSuccess) return hip_fail(e, "cache input-gradient launch");
  }
  e = launch_render_adjoint_cached(scene->dev, dp, dc, dr, adj_image, dg, io, stream);
  if (e != hipSuccess) return hip_fail(e, "render_adjoint_cached launch");
  return ok();
}

}  // extern "C"
