// Device functions of the path tracer shared by the megakernels and the
// wavefront kernels: float3 arithmetic, Philox4x32-10, the four-wide BVH
// traversal with the watertight triangle test (Woop et al. 2013), frames,
// GGX and the eight BSDFs (eval / sample / parameter derivatives), emitter
// sampling with the power heuristic, the pinhole camera, the LDS tables.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "drt_internal.h"

namespace drt {

#define DEV __device__ __forceinline__

constexpr float kPi = 3.14159265358979323846f;
constexpr float kInvPi = 0.318309886183790671538f;

// ---------------------------------------------------------------------------
// small vector type
// ---------------------------------------------------------------------------
struct f3 {
  float x, y, z;
};
DEV f3 mk(float x, float y, float z) { return f3{x, y, z}; }
DEV f3 operator+(f3 a, f3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
DEV f3 operator-(f3 a, f3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
DEV f3 operator*(f3 a, f3 b) { return mk(a.x * b.x, a.y * b.y, a.z * b.z); }
DEV f3 operator*(f3 a, float s) { return mk(a.x * s, a.y * s, a.z * s); }
DEV f3 operator-(f3 a) { return mk(-a.x, -a.y, -a.z); }
DEV float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
DEV f3 cross(f3 a, f3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
DEV f3 normalize(f3 a) { return a * __builtin_amdgcn_rsqf(dot(a, a)); }
// sin and cos of 2 pi u for u in [0, 1): the hardware takes revolutions
DEV void sincos_2pi(float u, float* s, float* c) {
  *s = __builtin_amdgcn_sinf(u);
  *c = __builtin_amdgcn_cosf(u);
}
DEV bool nonzero(f3 a) { return a.x != 0.f || a.y != 0.f || a.z != 0.f; }
DEV float maxc(f3 a) { return fmaxf(a.x, fmaxf(a.y, a.z)); }
DEV float comp(f3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// multiplies, cross-xor with the round key, key bumped by the Weyl constants.
// ---------------------------------------------------------------------------
DEV uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32 -> 64-bit product gives both halves
    uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}
// top 24 bits -> [0, 1), exact in float
DEV float u01(uint32_t r) { return (float)(r >> 8) * 5.9604644775390625e-8f; }
// exact discrete choice in [0, n): floor(r * n / 2^32)
DEV uint32_t pick(uint32_t r, uint32_t n) { return __umulhi(r, n); }

// ---------------------------------------------------------------------------
// per-lane counters (stats flag)
// ---------------------------------------------------------------------------
struct Counters {
  uint32_t rays, shadow, nodes, tris, verts, scatter, samples;
  float lrem_max;
  // texel scatter: lanes that scattered, and distinct texels among the
  // lanes of each wave-wide scatter (their ratio bounds what a wave-level
  // merge of equal keys could save)
  uint32_t tex_lanes, tex_keys;
  // SIMD utilisation by phase (stats kernels only): iterations of the
  // wave's node loop, triangle loop, vertex steps and shading blocks, each
  // counted once per wave, beside the per-lane counts (nodes, tris,
  // lane_steps, verts)
  uint32_t wave_nodes, wave_tris, wave_steps, lane_steps, wave_shade;
};

// true on one active lane of the wave (the lowest): counts an event once
// per wave
DEV bool first_active_lane() {
  return __lane_id() == __ffsll((unsigned long long)__ballot(1)) - 1;
}

// ---------------------------------------------------------------------------
// BVH traversal.  The per-lane stack lives in LDS at stk[i * kBlock], so the
// 64 lanes of a wave touch 64 consecutive words (conflict-free).
// ---------------------------------------------------------------------------
struct RayPre {
  f3 o, d;
  f3 idir, ooi;  // 1/d (finite) and o/d for the slab test
  int kx, ky, kz;
  float sx, sy, sz;
  float okx, oky, okz;  // o's components along kx, ky, kz
  int nx, ny, nz;       // per axis, the node float4 of the near bounds (lo; hi where d < 0)
};

DEV RayPre ray_pre(f3 o, f3 d) {
  RayPre r;
  r.o = o;
  r.d = d;
  float dx = fabsf(d.x) < 1e-20f ? copysignf(1e-20f, d.x) : d.x;
  float dy = fabsf(d.y) < 1e-20f ? copysignf(1e-20f, d.y) : d.y;
  float dz = fabsf(d.z) < 1e-20f ? copysignf(1e-20f, d.z) : d.z;
  r.idir = mk(1.0f / dx, 1.0f / dy, 1.0f / dz);
  r.ooi = o * r.idir;
  // watertight test set-up (Woop, Benthin, Wald, JCGT 2013): kz = dominant axis
  float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
  int kz = 0;
  if (ay > ax) kz = 1;
  if (az > (kz == 0 ? ax : ay)) kz = 2;
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  if (comp(d, kz) < 0.f) {
    int t = kx;
    kx = ky;
    ky = t;
  }
  r.kx = kx;
  r.ky = ky;
  r.kz = kz;
  float dkz = comp(d, kz);
  r.sx = comp(d, kx) / dkz;
  r.sy = comp(d, ky) / dkz;
  r.sz = 1.0f / dkz;
  r.okx = comp(o, kx);
  r.oky = comp(o, ky);
  r.okz = comp(o, kz);
  r.nx = r.idir.x < 0.f ? 3 : 0;
  r.ny = r.idir.y < 0.f ? 4 : 1;
  r.nz = r.idir.z < 0.f ? 5 : 2;
  return r;
}

// Slab distances of four children's bounds along one axis.  fma(c, 1/d, -o/d)
// is monotone in c, so the bound on the near side of the ray's direction
// gives the smaller distance: picking it per ray orders each slab pair with
// no min / max.
DEV float4 slab4(float4 c, float idir, float ooi) {
  return make_float4(fmaf(c.x, idir, -ooi), fmaf(c.y, idir, -ooi), fmaf(c.z, idir, -ooi),
                     fmaf(c.w, idir, -ooi));
}
DEV float4 max4(float4 a, float4 b) {
  return make_float4(fmaxf(a.x, b.x), fmaxf(a.y, b.y), fmaxf(a.z, b.z), fmaxf(a.w, b.w));
}
DEV float4 min4(float4 a, float4 b) {
  return make_float4(fminf(a.x, b.x), fminf(a.y, b.y), fminf(a.z, b.z), fminf(a.w, b.w));
}

struct Hit {
  float t, b1, b2;
  int tri;   // BVH-order index, -1 on a miss
  int prim;  // original id
};

// a b - c d with one rounding's worth of error (Kahan's fma-based
// difference of products; its relative error is at most 2 ulp, so its sign
// is exact and it is zero only when a b = c d exactly).
DEV float diff_of_products(float a, float b, float c, float d) {
  const float w = __fmul_rn(c, d);
  const float e = __builtin_fmaf(-c, d, w);  // w - c d, exactly
  const float f = __builtin_fmaf(a, b, -w);
  return f + e;
}

// Watertight ray/triangle test (no culling), t in (tmin, tmax] -- the caller
// decides about t == tmax -- on the vertices' components along the ray's
// permuted axes kx, ky, kz, relative to the origin.  Each edge function is
// Kahan's difference of products, whose sign is exact: two triangles
// sharing an edge evaluate the same two products in swapped roles, so they
// always agree on which side of the edge the ray passes (no cracks from the
// rounding of a fused multiply-add), and a value is zero only when the exact
// one is -- which is what the method's higher-precision fallback for zero
// edge functions secures, so none is needed.
DEV bool tri_test_k(const RayPre& r, float Akx, float Aky, float Akz, float Bkx, float Bky,
                    float Bkz, float Ckx, float Cky, float Ckz, float tmin, float tmax,
                    float& t_out, float& b1, float& b2) {
  const float Ax = Akx - r.sx * Akz, Ay = Aky - r.sy * Akz;
  const float Bx = Bkx - r.sx * Bkz, By = Bky - r.sy * Bkz;
  const float Cx = Ckx - r.sx * Ckz, Cy = Cky - r.sy * Ckz;
  const float U = diff_of_products(Cx, By, Cy, Bx);
  const float V = diff_of_products(Ax, Cy, Ay, Cx);
  const float W = diff_of_products(Bx, Ay, By, Ax);
  // the rest is computed whatever the edge functions say and the decision
  // taken at the end (fewer divergent branches in the triangle loop); with
  // det = 0 the quotients are not finite and the result is masked
  const bool mixed = (U < 0.f || V < 0.f || W < 0.f) && (U > 0.f || V > 0.f || W > 0.f);
  const float det = U + V + W;
  const float T_ = U * (r.sz * Akz) + V * (r.sz * Bkz) + W * (r.sz * Ckz);
  const float inv = 1.0f / det;
  const float t = T_ * inv;
  t_out = t;
  b1 = V * inv;
  b2 = W * inv;
  return !mixed && det != 0.f && t > tmin && t <= tmax;
}

// The test on a triangle held in registers: the permuted components picked by
// selects.
DEV bool tri_test(const RayPre& r, const DTri& T, float tmin, float tmax, float& t_out, float& b1,
                  float& b2) {
  const f3 A = mk(T.p0x, T.p0y, T.p0z) - r.o, B = mk(T.p1x, T.p1y, T.p1z) - r.o;
  const f3 C = mk(T.p2x, T.p2y, T.p2z) - r.o;
  return tri_test_k(r, comp(A, r.kx), comp(A, r.ky), comp(A, r.kz), comp(B, r.kx), comp(B, r.ky),
                    comp(B, r.kz), comp(C, r.kx), comp(C, r.ky), comp(C, r.kz), tmin, tmax, t_out,
                    b1, b2);
}

// The test on a triangle record in LDS (vertex v's component c at tp[3 v + c]):
// the permuted components read directly, three address offsets per ray
// instead of selects per test.  In device memory the same reads would cost
// 64-bit addresses and registers in the kernels held to 128 VGPRs.
DEV bool tri_test_lds(const RayPre& r, const float* tp, float tmin, float tmax, float& t_out,
                      float& b1, float& b2) {
  return tri_test_k(r, tp[r.kx] - r.okx, tp[r.ky] - r.oky, tp[r.kz] - r.okz,
                    tp[3 + r.kx] - r.okx, tp[3 + r.ky] - r.oky, tp[3 + r.kz] - r.okz,
                    tp[6 + r.kx] - r.okx, tp[6 + r.ky] - r.oky, tp[6 + r.kz] - r.okz, tmin, tmax,
                    t_out, b1, b2);
}

DEV DTri load_tri(const DScene& s, int i) {
  const float4* p = reinterpret_cast<const float4*>(s.tris + i);
  float4 a = p[0], b = p[1], c = p[2];
  DTri t;
  t.p0x = a.x; t.p0y = a.y; t.p0z = a.z; t.p1x = a.w;
  t.p1y = b.x; t.p1z = b.y; t.p2x = b.z; t.p2y = b.w;
  t.p2z = c.x;
  t.prim = __float_as_int(c.y);
  t.flags = __float_as_int(c.z);
  t.pad = 0;
  return t;
}

// One traversal loop for both ray kinds, so the lanes of a wave traverse
// together whatever ray each carries.
// any = false: closest hit in (tmin, tmax), ties to the lowest original id.
// any = true: true iff a non-null triangle is hit in (tmin, tmax).
// compare-exchange by key, written as selects (no divergent branch)
DEV void cswap(float& ka, int& va, float& kb, int& vb) {
  const bool sw = kb < ka;
  const float k0 = sw ? kb : ka, k1 = sw ? ka : kb;
  const int v0 = sw ? vb : va, v1 = sw ? va : vb;
  ka = k0;
  kb = k1;
  va = v0;
  vb = v1;
}

// Closest (any = false) or any hit in (tmin, tmax] over the four-wide BVH.
// Per node: four slab tests; for a closest hit, hit interior children
// sorted near to far, the nearest visited next and the others pushed far
// first (an any-hit query takes them in slot order); the triangles of the
// node's hit leaf children form the lane's leaf batch, tested before its
// next node.
//
// Leaf batches are postponed across the wave: a lane that holds one stops
// visiting nodes until every lane of the wave holds one or has finished,
// and then all of them test their batches in one loop.  Testing a batch at
// once after its node (the wave looping over the largest batch while the
// lanes without one idle) kept only a fifth of the lanes busy in the
// triangle loop.  Each lane still does exactly what it did before, in the
// same order (node, its batch, the next node) -- only the interleaving of
// lanes changes -- so the nodes visited and the hit found are the same.
// LSC: the scene is the workgroup's LDS copy (triangle components read along
// the ray's permuted axes).  IDX: the near and far bounds of each axis read
// by the ray's signs; without it the six bound quadruples are read at fixed
// offsets and each slab pair ordered by min / max -- the same values, fewer
// live registers (the indexed form in device memory costs 64-bit addresses,
// which made the adjoint megakernels, held to 128 VGPRs, spill).
template <bool ST = false, bool LSC = false, bool IDX = true>
DEV bool traverse(const DScene& s, const RayPre& r, float tmin, float tmax, bool any, Hit& h,
                  int* stk, Counters& cnt) {
  float tbest = tmax;
  h.tri = -1;
  h.prim = 0x7fffffff;
  bool found = false;
  int node = 0, sp = 0;
  bool live = true;  // the lane has a node to visit
  // pending leaf batch: triangle j < e3 of the batch is j + the offset of
  // its range (range k covers [e_{k-1}, e_k); offsets f0..f3)
  int e0 = 0, e1 = 0, e2 = 0, e3 = 0, f0 = 0, f1 = 0, f2 = 0, f3 = 0;
  for (;;) {
    // node phase: visit nodes until this lane holds a leaf batch or has none left
    while (live && e3 == 0) {
      const float4* np = reinterpret_cast<const float4*>(s.nodes + node);
      const int4 ch = reinterpret_cast<const int4*>(np)[6], cn = reinterpret_cast<const int4*>(np)[7];
      cnt.nodes++;
      if constexpr (ST) cnt.wave_nodes += first_active_lane();
      float t0, t1, t2, t3;
      bool h0, h1, h2, h3;
      // The slab tests run whatever the counts say and are masked afterwards:
      // a short-circuit on the count would put the box loads behind the count
      // load and cost every node a second memory round trip.  Empty slots hold
      // a zero box, so the test on them is harmless.
      {  // entry (tn) and exit (tf) distances of the four boxes, axis by axis
        float4 tn, tf;
        if constexpr (IDX) {
          // the near and far bounds read by the ray's signs
          tn = slab4(np[r.nx], r.idir.x, r.ooi.x);
          tf = slab4(np[3 - r.nx], r.idir.x, r.ooi.x);
          tn = max4(tn, slab4(np[r.ny], r.idir.y, r.ooi.y));
          tf = min4(tf, slab4(np[5 - r.ny], r.idir.y, r.ooi.y));
          tn = max4(tn, slab4(np[r.nz], r.idir.z, r.ooi.z));
          tf = min4(tf, slab4(np[7 - r.nz], r.idir.z, r.ooi.z));
        } else {
          // fixed offsets, each slab pair ordered by min / max
          float4 a = slab4(np[0], r.idir.x, r.ooi.x), b = slab4(np[3], r.idir.x, r.ooi.x);
          tn = min4(a, b);
          tf = max4(a, b);
          a = slab4(np[1], r.idir.y, r.ooi.y);
          b = slab4(np[4], r.idir.y, r.ooi.y);
          tn = max4(tn, min4(a, b));
          tf = min4(tf, max4(a, b));
          a = slab4(np[2], r.idir.z, r.ooi.z);
          b = slab4(np[5], r.idir.z, r.ooi.z);
          tn = max4(tn, min4(a, b));
          tf = min4(tf, max4(a, b));
        }
        tn = max4(tn, make_float4(tmin, tmin, tmin, tmin));
        tf = min4(tf, make_float4(tbest, tbest, tbest, tbest));
        t0 = tn.x;
        t1 = tn.y;
        t2 = tn.z;
        t3 = tn.w;
        // conservative exit: the two roundings of the fma form plus slack
        h0 = (tn.x <= tf.x * 1.0000005f) & (cn.x >= 0);
        h1 = (tn.y <= tf.y * 1.0000005f) & (cn.y >= 0);
        h2 = (tn.z <= tf.z * 1.0000005f) & (cn.z >= 0);
        h3 = (tn.w <= tf.w * 1.0000005f) & (cn.w >= 0);
      }
      // the batch: the hit leaf children's ranges, offsets picked by selects
      e0 = (h0 && cn.x > 0) ? cn.x : 0;
      e1 = e0 + ((h1 && cn.y > 0) ? cn.y : 0);
      e2 = e1 + ((h2 && cn.z > 0) ? cn.z : 0);
      e3 = e2 + ((h3 && cn.w > 0) ? cn.w : 0);
      f0 = ch.x;
      f1 = ch.y - e0;
      f2 = ch.z - e1;
      f3 = ch.w - e2;
      // the next node (does not depend on the batch's outcome)
      if (any) {
        // whether anything is hit does not depend on the visiting order: the
        // hit interior children are taken in slot order, with no sort
        int next = -1;
        if (h0 && cn.x == 0) next = ch.x;
        if (h1 && cn.y == 0) {
          if (next < 0) next = ch.y; else stk[(sp++) * kBlock] = ch.y;
        }
        if (h2 && cn.z == 0) {
          if (next < 0) next = ch.z; else stk[(sp++) * kBlock] = ch.z;
        }
        if (h3 && cn.w == 0) {
          if (next < 0) next = ch.w; else stk[(sp++) * kBlock] = ch.w;
        }
        if (next >= 0) {
          node = next;
        } else if (sp == 0) {
          live = false;
        } else {
          --sp;
          node = stk[sp * kBlock];
        }
        continue;
      }
      // interior children hit: keys finite for them, +inf otherwise
      float k0 = (h0 && cn.x == 0) ? fminf(t0, 3.0e38f) : INFINITY;
      float k1 = (h1 && cn.y == 0) ? fminf(t1, 3.0e38f) : INFINITY;
      float k2 = (h2 && cn.z == 0) ? fminf(t2, 3.0e38f) : INFINITY;
      float k3 = (h3 && cn.w == 0) ? fminf(t3, 3.0e38f) : INFINITY;
      int v0 = ch.x, v1 = ch.y, v2 = ch.z, v3 = ch.w;
      cswap(k0, v0, k1, v1);
      cswap(k2, v2, k3, v3);
      cswap(k0, v0, k2, v2);
      cswap(k1, v1, k3, v3);
      cswap(k1, v1, k2, v2);
      if (k0 == INFINITY) {
        if (sp == 0) {
          live = false;
        } else {
          --sp;
          node = stk[sp * kBlock];
        }
        continue;
      }
      node = v0;
      if (k3 != INFINITY) stk[(sp++) * kBlock] = v3;
      if (k2 != INFINITY) stk[(sp++) * kBlock] = v2;
      if (k1 != INFINITY) stk[(sp++) * kBlock] = v1;
    }
    // leaf phase: every lane of the wave holds a batch or has finished
    if (e3 == 0) break;  // this lane has finished (no node, no batch)
    for (int j = 0; j < e3; ++j) {
      int off = j < e2 ? f2 : f3;
      off = j < e1 ? f1 : off;
      off = j < e0 ? f0 : off;
      const int i = j + off;
      int prim, flags;
      float t, b1, b2;
      bool ok;
      if constexpr (LSC) {
        const float* tp = reinterpret_cast<const float*>(s.tris + i);
        prim = __float_as_int(tp[9]);
        flags = __float_as_int(tp[10]);
        ok = tri_test_lds(r, tp, tmin, tbest, t, b1, b2);
      } else {
        const DTri T = load_tri(s, i);
        prim = T.prim;
        flags = T.flags;
        ok = tri_test(r, T, tmin, tbest, t, b1, b2);
      }
      cnt.tris++;
      if constexpr (ST) cnt.wave_tris += first_active_lane();
      if (any) {
        // shadow rays pass through null surfaces; the flag is tested after
        // the whole record has been loaded (no second memory round trip)
        if (ok && !(flags & 1) && t < tmax) {
          found = true;
          break;
        }
        continue;
      }
      // closest: strictly nearer, or an exact tie with a lower original id
      ok = ok && (t < tbest || (h.tri >= 0 && prim < h.prim));
      tbest = ok ? t : tbest;
      h.t = ok ? t : h.t;
      h.b1 = ok ? b1 : h.b1;
      h.b2 = ok ? b2 : h.b2;
      h.tri = ok ? i : h.tri;
      h.prim = ok ? prim : h.prim;
    }
    e3 = 0;
    if (found) break;
  }
  return any ? found : h.tri >= 0;
}

// ---------------------------------------------------------------------------
// frames, sampling helpers
// ---------------------------------------------------------------------------
struct Frame {
  f3 s, t, n;
};
// Orthonormal basis of a unit normal (Duff et al., JCGT 2017, branchless).
DEV Frame make_frame(f3 n) {
  float sign = copysignf(1.0f, n.z);
  float a = -1.0f / (sign + n.z);
  float b = n.x * n.y * a;
  Frame f;
  f.n = n;
  f.s = mk(1.0f + sign * n.x * n.x * a, sign * b, -sign * n.x);
  f.t = mk(b, sign + n.y * n.y * a, -n.y);
  return f;
}
DEV f3 to_local(const Frame& f, f3 v) { return mk(dot(v, f.s), dot(v, f.t), dot(v, f.n)); }
DEV f3 to_world(const Frame& f, f3 v) { return f.s * v.x + f.t * v.y + f.n * v.z; }

DEV f3 spawn(const DScene& s, f3 p, f3 n_g, f3 d) {
  float sg = dot(d, n_g) >= 0.f ? 1.0f : -1.0f;
  return p + n_g * (sg * s.eps);
}

// cosine-weighted hemisphere: phi = 2 pi u_a, sin^2(theta) = u_b
DEV f3 cosine_hemisphere(float ua, float ub) {
  float sp, cp;
  sincos_2pi(ua, &sp, &cp);
  float r = sqrtf(ub);
  return mk(cp * r, sp * r, sqrtf(1.0f - ub));
}

// ---------------------------------------------------------------------------
// microfacet terms (Walter et al. 2007), alpha = roughness
// ---------------------------------------------------------------------------
DEV float ggx_D(float a, float c) {
  if (c <= 0.f) return 0.f;
  float c2 = c * c, a2 = a * a;
  float den = c2 * (a2 - 1.0f) + 1.0f;
  return a2 / (kPi * den * den);
}
DEV float ggx_G1(float a, float vm, float vn) {
  if (vm * vn <= 0.f) return 0.f;
  float c2 = vn * vn;
  float tan2 = fmaxf(0.f, 1.0f - c2) / c2;
  return 2.0f / (1.0f + sqrtf(1.0f + a * a * tan2));
}
DEV float ggx_dlnD(float a, float c) {
  float c2 = c * c;
  float den = c2 * (a * a - 1.0f) + 1.0f;
  return 2.0f / a - 4.0f * a * c2 / den;
}
DEV float ggx_dlnG1(float a, float vn) {
  float c2 = vn * vn;
  float tan2 = fmaxf(0.f, 1.0f - c2) / c2;
  float r = sqrtf(1.0f + a * a * tan2);
  return -(a * tan2 / r) / (1.0f + r);
}
DEV f3 ggx_sample_m(float a, float u1, float u2) {
  float cos2 = (1.0f - u1) / (1.0f + (a * a - 1.0f) * u1);
  float ct = sqrtf(cos2);
  float st = sqrtf(fmaxf(0.f, 1.0f - cos2));
  float sp, cp;
  sincos_2pi(u2, &sp, &cp);
  return mk(st * cp, st * sp, ct);
}
// exact unpolarised dielectric Fresnel; cos_i >= 0 on the incident side,
// eta = n_transmitted / n_incident
DEV float fresnel_dielectric(float cos_i, float eta) {
  float sin2_t = (1.0f - cos_i * cos_i) / (eta * eta);
  if (sin2_t >= 1.0f) return 1.0f;
  float cos_t = sqrtf(1.0f - sin2_t);
  float rs = (cos_i - eta * cos_t) / (cos_i + eta * cos_t);
  float rp = (eta * cos_i - cos_t) / (eta * cos_i + cos_t);
  return 0.5f * (rs * rs + rp * rp);
}
DEV float schlick(float f0, float c) {
  float m = 1.0f - c;
  float m2 = m * m;
  return f0 + (1.0f - f0) * m2 * m2 * m;
}
DEV f3 reflect_about(f3 wi, f3 m) { return m * (2.0f * dot(wi, m)) - wi; }

// ---------------------------------------------------------------------------
// Material switch.  eval() returns f * |cos theta_o| per channel and the
// density of sample(); with DERIV also d/d albedo_c and d/d alpha per
// channel.  Work shared by all types (albedo/roughness fetch, frame) is done
// once outside the switch.
// ---------------------------------------------------------------------------
struct Shade {
  int type;
  f3 albedo;
  f3 f0;
  float alpha, eta, opacity;
};

struct BEval {
  f3 f;
  float pdf;
  f3 dalb, dalpha;
};

template <bool DERIV>
DEV void eval_lambert(f3 albedo, f3 wi, f3 wo, BEval& e) {
  if (wi.z <= 0.f || wo.z <= 0.f) return;
  float k = wo.z * kInvPi;
  e.f = albedo * k;
  if (DERIV) e.dalb = mk(k, k, k);
  e.pdf = k;
}

template <bool DERIV>
DEV BEval bsdf_eval(const Shade& m, f3 wi, f3 wo) {
  BEval e;
  e.f = mk(0, 0, 0);
  e.pdf = 0.f;
  e.dalb = mk(0, 0, 0);
  e.dalpha = mk(0, 0, 0);
  const float a = m.alpha;
  switch (m.type) {
    case DRT_BSDF_DIFFUSE:
    case DRT_BSDF_DIFFUSE_TEXTURED:
    case DRT_BSDF_MASK:
      eval_lambert<DERIV>(m.albedo, wi, wo, e);
      break;
    case DRT_BSDF_TWOSIDED:
      if (wi.z < 0.f) {
        wi.z = -wi.z;
        wo.z = -wo.z;
      }
      eval_lambert<DERIV>(m.albedo, wi, wo, e);
      break;
    case DRT_BSDF_CONDUCTOR: {
      if (wi.z <= 0.f || wo.z <= 0.f) break;
      f3 h = normalize(wi + wo);
      float D = ggx_D(a, h.z);
      float G = ggx_G1(a, dot(wi, h), wi.z) * ggx_G1(a, dot(wo, h), wo.z);
      float base = D * G / (4.0f * wi.z);
      float ih = dot(wi, h);
      e.f = mk(schlick(m.f0.x, ih), schlick(m.f0.y, ih), schlick(m.f0.z, ih)) * base;
      if (DERIV) e.dalpha = e.f * (ggx_dlnD(a, h.z) + ggx_dlnG1(a, wi.z) + ggx_dlnG1(a, wo.z));
      e.pdf = D * h.z / (4.0f * fabsf(dot(wo, h)));
      break;
    }
    case DRT_BSDF_PLASTIC: {
      if (wi.z <= 0.f || wo.z <= 0.f) break;
      f3 h = normalize(wi + wo);
      float D = ggx_D(a, h.z);
      float G = ggx_G1(a, dot(wi, h), wi.z) * ggx_G1(a, dot(wo, h), wo.z);
      float spec = fresnel_dielectric(dot(wi, h), m.eta) * D * G / (4.0f * wi.z);
      float Fi = fresnel_dielectric(wi.z, m.eta), Fo = fresnel_dielectric(wo.z, m.eta);
      float kd = (1.0f - Fi) * (1.0f - Fo) * wo.z * kInvPi;
      e.f = mk(spec, spec, spec) + m.albedo * kd;
      if (DERIV) {
        e.dalb = mk(kd, kd, kd);
        float sd = spec * (ggx_dlnD(a, h.z) + ggx_dlnG1(a, wi.z) + ggx_dlnG1(a, wo.z));
        e.dalpha = mk(sd, sd, sd);
      }
      float ps = fminf(fmaxf(Fi, 0.1f), 0.9f);
      e.pdf = ps * (D * h.z / (4.0f * fabsf(dot(wo, h)))) + (1.0f - ps) * wo.z * kInvPi;
      break;
    }
    case DRT_BSDF_DIELECTRIC: {
      float ci = wi.z, co = wo.z;
      if (ci == 0.f || co == 0.f) break;
      float eta = ci > 0.f ? m.eta : 1.0f / m.eta;
      bool refl = ci * co > 0.f;
      f3 h = refl ? normalize(wi + wo) : normalize(wi + wo * eta);
      if (h.z < 0.f) h = -h;
      float D = ggx_D(a, h.z);
      float G = ggx_G1(a, dot(wi, h), ci) * ggx_G1(a, dot(wo, h), co);
      if (D == 0.f || G == 0.f) break;
      float ih = dot(wi, h), oh = dot(wo, h);
      float F = fresnel_dielectric(fabsf(ih), eta);
      float val, pdf;
      if (refl) {
        val = F * D * G / (4.0f * fabsf(ci));
        pdf = F * D * h.z / (4.0f * fabsf(oh));
      } else {
        if (ih * oh >= 0.f) break;
        float den = ih + eta * oh;
        den *= den;
        val = fabsf(ih) * fabsf(oh) * (1.0f - F) * D * G / (fabsf(ci) * den);
        pdf = (1.0f - F) * D * h.z * eta * eta * fabsf(oh) / den;
      }
      e.f = mk(val, val, val);
      if (DERIV) {
        float dv = val * (ggx_dlnD(a, h.z) + ggx_dlnG1(a, ci) + ggx_dlnG1(a, co));
        e.dalpha = mk(dv, dv, dv);
      }
      e.pdf = pdf;
      break;
    }
    default:
      break;
  }
  return e;
}

// Draws a direction (local frame) with the density eval() reports.
// Returns false if the sample is rejected (below the surface, zero value).
template <bool DERIV>
DEV bool bsdf_sample(const Shade& m, f3 wi, float u1, float u2, float ulobe, f3& wo, BEval& e) {
  const float a = m.alpha;
  switch (m.type) {
    case DRT_BSDF_DIFFUSE:
    case DRT_BSDF_DIFFUSE_TEXTURED:
    case DRT_BSDF_MASK:
      if (wi.z <= 0.f) return false;
      wo = cosine_hemisphere(u1, u2);
      break;
    case DRT_BSDF_TWOSIDED:
      wo = cosine_hemisphere(u1, u2);
      if (wi.z < 0.f) wo.z = -wo.z;
      break;
    case DRT_BSDF_CONDUCTOR: {
      if (wi.z <= 0.f) return false;
      f3 mm = ggx_sample_m(a, u1, u2);
      if (dot(wi, mm) <= 0.f) return false;
      wo = reflect_about(wi, mm);
      if (wo.z <= 0.f) return false;
      break;
    }
    case DRT_BSDF_PLASTIC: {
      if (wi.z <= 0.f) return false;
      float ps = fminf(fmaxf(fresnel_dielectric(wi.z, m.eta), 0.1f), 0.9f);
      if (ulobe < ps) {
        f3 mm = ggx_sample_m(a, u1, u2);
        if (dot(wi, mm) <= 0.f) return false;
        wo = reflect_about(wi, mm);
        if (wo.z <= 0.f) return false;
      } else {
        wo = cosine_hemisphere(u1, u2);
      }
      break;
    }
    case DRT_BSDF_DIELECTRIC: {
      if (wi.z == 0.f) return false;
      float sg = wi.z > 0.f ? 1.0f : -1.0f;
      float eta = wi.z > 0.f ? m.eta : 1.0f / m.eta;
      f3 mm = ggx_sample_m(a, u1, u2) * sg;
      float c = dot(wi, mm);
      if (c <= 0.f) return false;
      float F = fresnel_dielectric(c, eta);
      if (ulobe < F) {
        wo = reflect_about(wi, mm);
        if (wo.z * sg <= 0.f) return false;
      } else {
        float sin2_t = (1.0f - c * c) / (eta * eta);
        if (sin2_t >= 1.0f) return false;
        float cos_t = sqrtf(1.0f - sin2_t);
        wo = wi * (-1.0f / eta) + mm * (c / eta - cos_t);
        if (wo.z * sg >= 0.f) return false;
      }
      break;
    }
    default:
      return false;
  }
  e = bsdf_eval<DERIV>(m, wi, wo);
  return e.pdf > 0.f && nonzero(e.f);
}

// ---------------------------------------------------------------------------
// environment map (latitude-longitude, row 0 = +y, theta from +y)
// ---------------------------------------------------------------------------
DEV void env_cell(const DScene& s, f3 d, int& row, int& col, float& sin_t) {
  float ct = fminf(1.0f, fmaxf(-1.0f, d.y));
  float th = acosf(ct);
  float ph = atan2f(d.z, d.x);
  if (ph < 0.f) ph += 2.0f * kPi;
  int c = (int)floorf(ph * (0.5f * kInvPi) * (float)s.env_w);
  int r = (int)floorf(th * kInvPi * (float)s.env_h);
  col = min(max(c, 0), s.env_w - 1);
  row = min(max(r, 0), s.env_h - 1);
  sin_t = sinf(th);
}
DEV f3 env_lookup(const DScene& s, int row, int col) {
  const float* p = s.env + 3 * ((size_t)row * s.env_w + col);
  return mk(p[0], p[1], p[2]);
}
// density (solid angle) of the environment sampler for a direction
DEV float env_pdf(const DScene& s, int row, int col, float sin_t) {
  if (sin_t <= 0.f) return 0.f;
  return s.env_puv[(size_t)row * s.env_w + col] / (2.0f * kPi * kPi * sin_t);
}
// largest i in [0, n) with cdf[i] <= u
DEV int cdf_find(const float* cdf, int n, float u) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (cdf[mid] <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}
DEV bool env_sample(const DScene& s, float u1, float u2, f3& d) {
  if (s.env_cdf_row[s.env_h] <= 0.f) return false;
  int r = cdf_find(s.env_cdf_row, s.env_h, u1);
  float r0 = s.env_cdf_row[r], r1 = s.env_cdf_row[r + 1];
  float v = ((float)r + (u1 - r0) / (r1 - r0)) / (float)s.env_h;
  const float* cc = s.env_cdf_col + (size_t)r * (s.env_w + 1);
  int c = cdf_find(cc, s.env_w, u2);
  float u = ((float)c + (u2 - cc[c]) / (cc[c + 1] - cc[c])) / (float)s.env_w;
  float st, ct, sp, cp;
  sincos_2pi(0.5f * v, &st, &ct);
  sincos_2pi(u, &sp, &cp);
  d = mk(st * cp, ct, st * sp);
  return true;
}

DEV float power_heuristic(float a, float b) {
  float a2 = a * a, b2 = b * b;
  return a2 / (a2 + b2);
}

// ---------------------------------------------------------------------------
// per-workgroup tables in LDS
// ---------------------------------------------------------------------------
struct LdsTables {
  const float* tex[DRT_MAX_TEXTURES];
  float* gtex[DRT_MAX_TEXTURES];
  int tw[DRT_MAX_TEXTURES], th[DRT_MAX_TEXTURES];
};

// Gradient sinks of the replay pass.
struct Sink {
  const LdsTables* tab;
  float* rough_lds;      // per-workgroup roughness accumulators (or null)
  float* rough_global;   // fallback when there are more slots than LDS holds
};

// Number of distinct values of `key` among the active lanes of the wave
// (the same on every active lane): leader by leader, each pass retires the
// lanes that share the leader's key.
DEV int wave_distinct(int key) {
  uint64_t todo = __ballot(1);
  int n = 0;
  while (todo) {
    const int key0 = __shfl(key, __ffsll((unsigned long long)todo) - 1, 64);
    todo &= ~(uint64_t)__ballot(key == key0);
    ++n;
  }
  return n;
}

DEV void scatter_tex(const Sink& k, int tex, int texel, f3 g, Counters& cnt, bool stats) {
  float* base = k.tab->gtex[tex];
  if (!base) return;
  if (stats) {
    // measurement only (stats launches): how often lanes of one wave-wide
    // scatter share a texel
    const int n = wave_distinct(tex * 0x01000000 ^ texel);
    cnt.tex_lanes++;
    if (__lane_id() == __ffsll((unsigned long long)__ballot(1)) - 1) cnt.tex_keys += n;
  }
  float* p = base + 3 * (size_t)texel;
  if (g.x != 0.f) { atomicAdd(p + 0, g.x); cnt.scatter++; }
  if (g.y != 0.f) { atomicAdd(p + 1, g.y); cnt.scatter++; }
  if (g.z != 0.f) { atomicAdd(p + 2, g.z); cnt.scatter++; }
}
DEV void scatter_rough(const Sink& k, int slot, float g, Counters& cnt) {
  if (g == 0.f) return;
  if (k.rough_lds) atomicAdd(k.rough_lds + slot, g);
  else if (k.rough_global) { atomicAdd(k.rough_global + slot, g); cnt.scatter++; }
}

// A lane's roughness gradient summed in a register while its slot stays the
// same (slot -1: nothing held).
struct RoughAcc {
  int slot;
  float v;
};

// Sum of x over the 64 lanes of the wave (butterfly of lane exchanges); all
// lanes must be active, and every lane receives the same sum.
DEV float wave_sum(float x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

// Flush of every lane's roughness accumulator, called by all 64 lanes of
// the wave together: the lanes holding the same slot are summed across the
// wave and one lane per distinct slot issues the atomic (one atomic per
// distinct key instead of one per lane).
DEV void wave_scatter_rough(const Sink& k, RoughAcc& a, Counters& cnt) {
  const bool want = a.slot >= 0 && a.v != 0.f;
  uint64_t todo = __ballot(want);
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const int key = __shfl(a.slot, leader, 64);
    const bool mine = want && a.slot == key;
    const float sum = wave_sum(mine ? a.v : 0.f);
    if (__lane_id() == leader) scatter_rough(k, key, sum, cnt);
    todo &= ~(uint64_t)__ballot(mine);
  }
  a.slot = -1;
  a.v = 0.f;
}

DEV void camera_ray(const DCam& c, int W, int H, int x, int y, uint32_t g_lo, uint32_t g_hi,
                    const DRender& R, f3& o, f3& d) {
  uint4 r = philox(g_lo, g_hi, 0xFFFFFFFFu, 0u, R.key0, R.key1);
  float px = ((float)x + u01(r.x)) / (float)W;
  float py = ((float)y + u01(r.y)) / (float)H;
  float sx = (2.0f * px - 1.0f) * c.tan_half * c.aspect;
  float sy = (1.0f - 2.0f * py) * c.tan_half;
  o = mk(c.ox, c.oy, c.oz);
  d = normalize(mk(c.fx, c.fy, c.fz) + mk(c.rx, c.ry, c.rz) * sx + mk(c.ux, c.uy, c.uz) * sy);
}

DEV void load_tables(LdsTables& tab, const DScene& s, const DParams& P, const DGrads* G) {
  int t = threadIdx.x;
  if (t < DRT_MAX_TEXTURES) {
    tab.tex[t] = P.tex[t];
    tab.gtex[t] = G ? G->tex[t] : nullptr;
    tab.tw[t] = s.tex_w[t];
    tab.th[t] = s.tex_h[t];
  }
}

}  // namespace drt
