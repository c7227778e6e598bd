// gfx950 kernels of the differentiable path tracer.
//
// One megakernel renders (Dr.Jit paper, Fig. "prb-structure", megakernel #1);
// a second fuses the paper's megakernels #2 and #3: per sample it traces the
// path once to obtain its radiance L, then replays it with identical Philox
// counters, recovering the radiance that arrives over each sampled direction
// by subtracting what the vertices before it contributed (Path Replay
// Backpropagation, Sec. "Physically Based Differentiable Rendering"), and
// scatter-adds the gradients of the attached BSDF values (Sec. "AD tape
// surgery": f'/f applied to the replayed radiance; Sec. "Differentiating
// polymorphism": implicit parameter reads become atomic scatter-reductions).
//
// Design for CDNA4: wave64, one-wave 8x8-pixel workgroups, BVH traversal stack in
// LDS (one column per lane, no bank conflicts), the paper's polymorphic BSDF
// call as a switch on the material id with the albedo/roughness fetch hoisted
// out of it, roughness gradients pre-reduced in LDS per workgroup, texel
// gradients as hardware float atomics (no return value).
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
};

// ---------------------------------------------------------------------------
// BVH traversal.  The per-lane stack lives in LDS at stk[i * kBlock], so the
// 64 lanes of a wave touch 64 consecutive words (conflict-free).
// ---------------------------------------------------------------------------
struct RayPre {
  f3 o, d;
  f3 idir, ooi;  // 1/d (finite) and o/d for the slab test
  int kx, ky, kz;
  float sx, sy, sz;
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
  return r;
}

// Slab test of one child box; returns entry distance in tn.
DEV bool slab(const RayPre& r, float lx, float ly, float lz, float hx, float hy, float hz,
              float tmin, float tmax, float& tn) {
  float t0x = fmaf(lx, r.idir.x, -r.ooi.x), t1x = fmaf(hx, r.idir.x, -r.ooi.x);
  float t0y = fmaf(ly, r.idir.y, -r.ooi.y), t1y = fmaf(hy, r.idir.y, -r.ooi.y);
  float t0z = fmaf(lz, r.idir.z, -r.ooi.z), t1z = fmaf(hz, r.idir.z, -r.ooi.z);
  float tnear = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), tmin));
  float tfar = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
  tn = tnear;
  // conservative far bound: the two roundings of the fma form plus slack
  return tnear <= tfar * 1.0000005f;
}

struct Hit {
  float t, b1, b2;
  int tri;   // BVH-order index, -1 on a miss
  int prim;  // original id
};

// Watertight ray/triangle test (no culling), t in (tmin, tmax] -- the caller
// decides about t == tmax.  Exactly-zero edge functions are re-evaluated in
// double precision, as the method asks.
DEV bool tri_test(const RayPre& r, const DTri& T, float tmin, float tmax, float& t_out, float& b1,
                  float& b2) {
  f3 A = mk(T.p0x, T.p0y, T.p0z) - r.o;
  f3 B = mk(T.p1x, T.p1y, T.p1z) - r.o;
  f3 C = mk(T.p2x, T.p2y, T.p2z) - r.o;
  float Akz = comp(A, r.kz), Bkz = comp(B, r.kz), Ckz = comp(C, r.kz);
  float Ax = comp(A, r.kx) - r.sx * Akz, Ay = comp(A, r.ky) - r.sy * Akz;
  float Bx = comp(B, r.kx) - r.sx * Bkz, By = comp(B, r.ky) - r.sy * Bkz;
  float Cx = comp(C, r.kx) - r.sx * Ckz, Cy = comp(C, r.ky) - r.sy * Ckz;
  float U = Cx * By - Cy * Bx;
  float V = Ax * Cy - Ay * Cx;
  float W = Bx * Ay - By * Ax;
  if (U == 0.f || V == 0.f || W == 0.f) {
    U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
    V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
    W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
  }
  if ((U < 0.f || V < 0.f || W < 0.f) && (U > 0.f || V > 0.f || W > 0.f)) return false;
  float det = U + V + W;
  if (det == 0.f) return false;
  float T_ = U * (r.sz * Akz) + V * (r.sz * Bkz) + W * (r.sz * Ckz);
  float inv = 1.0f / det;
  float t = T_ * inv;
  if (!(t > tmin && t <= tmax)) return false;
  t_out = t;
  b1 = V * inv;
  b2 = W * inv;
  return true;
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
DEV void cswap(float& ka, int& va, float& kb, int& vb) {
  if (kb < ka) {
    float k = ka; ka = kb; kb = k;
    int v = va; va = vb; vb = v;
  }
}

// Closest (any = false) or any hit in (tmin, tmax] over the four-wide BVH.
// Per node: four slab tests; the triangles of every hit leaf child in one
// loop; hit interior children sorted near to far, the nearest visited next
// and the others pushed far first.
DEV bool traverse(const DScene& s, const RayPre& r, float tmin, float tmax, bool any, Hit& h,
                  int* stk, Counters& cnt) {
  float tbest = tmax;
  h.tri = -1;
  h.prim = 0x7fffffff;
  bool found = false;
  int node = 0, sp = 0;
  for (;;) {
    const float4* np = reinterpret_cast<const float4*>(s.nodes + node);
    const int4 ch = reinterpret_cast<const int4*>(np)[6], cn = reinterpret_cast<const int4*>(np)[7];
    cnt.nodes++;
    float t0, t1, t2, t3;
    bool h0, h1, h2, h3;
    {  // children 0 and 1: three float4 (fewer live registers than all four boxes)
      const float4 a = np[0], b = np[1], c = np[2];
      h0 = cn.x >= 0 && slab(r, a.x, a.y, a.z, a.w, b.x, b.y, tmin, tbest, t0);
      h1 = cn.y >= 0 && slab(r, b.z, b.w, c.x, c.y, c.z, c.w, tmin, tbest, t1);
    }
    {  // children 2 and 3
      const float4 a = np[3], b = np[4], c = np[5];
      h2 = cn.z >= 0 && slab(r, a.x, a.y, a.z, a.w, b.x, b.y, tmin, tbest, t2);
      h3 = cn.w >= 0 && slab(r, b.z, b.w, c.x, c.y, c.z, c.w, tmin, tbest, t3);
    }
    // leaf children: test their triangles now (one loop over the ranges)
    const int e0 = (h0 && cn.x > 0) ? cn.x : 0;
    const int e1 = e0 + ((h1 && cn.y > 0) ? cn.y : 0);
    const int e2 = e1 + ((h2 && cn.z > 0) ? cn.z : 0);
    const int e3 = e2 + ((h3 && cn.w > 0) ? cn.w : 0);
    for (int j = 0; j < e3; ++j) {
      const int i = j < e0 ? ch.x + j : (j < e1 ? ch.y + (j - e0) : (j < e2 ? ch.z + (j - e1) : ch.w + (j - e2)));
      DTri T = load_tri(s, i);
      cnt.tris++;
      if (any && (T.flags & 1)) continue;
      float t, b1, b2;
      if (!tri_test(r, T, tmin, tbest, t, b1, b2)) continue;
      if (any) {
        if (t < tmax) {
          found = true;
          break;
        }
        continue;
      }
      // closest: strictly nearer, or an exact tie with a lower original id
      if (t < tbest || (h.tri >= 0 && T.prim < h.prim)) {
        tbest = t;
        h.t = t;
        h.b1 = b1;
        h.b2 = b2;
        h.tri = i;
        h.prim = T.prim;
      }
    }
    if (found) break;
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
      if (sp == 0) break;
      --sp;
      node = stk[sp * kBlock];
      continue;
    }
    node = v0;
    if (k3 != INFINITY) stk[(sp++) * kBlock] = v3;
    if (k2 != INFINITY) stk[(sp++) * kBlock] = v2;
    if (k1 != INFINITY) stk[(sp++) * kBlock] = v1;
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

DEV void scatter_tex(const Sink& k, int tex, int texel, f3 g, Counters& cnt) {
  float* base = k.tab->gtex[tex];
  if (!base) return;
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

// ---------------------------------------------------------------------------
// The megakernel body.  A lane owns one pixel and loops over its samples.
// Each iteration of the loop is one vertex for every lane of the wave, in
// two phases that all lanes take together: (A) trace the closest-hit ray and
// do the emission, next-event and BSDF-sampling work of the vertex it finds;
// (B) trace the vertex's shadow ray and resolve the next-event term.  A lane
// whose path has ended starts the pixel's next sample (in the adjoint: the
// replay of the same sample) at the end of the iteration, so lanes stay in
// phase and busy until their own pixel is done.
//
// Path conventions.  D = max_depth counts segments including the camera ray;
// emission found at vertex k counts if k <= D; next-event estimation and
// BSDF sampling happen at vertex k < D; Russian roulette after sampling at
// k >= rr_depth.  Null surfaces, and mask surfaces whose opacity test fails,
// are passed through and count as vertices.  Random numbers of vertex k come
// from Philox blocks (g, b = k-1, dim 0/1): dim 0 = (light choice, light u,
// light v, lobe choice), dim 1 = (bsdf u, bsdf v, roulette, mask).
//
// MODE_PRIMAL: `out` receives the sum of the sample radiances.
// MODE_ADJOINT: per sample, pass A traces the path for its radiance L; pass B
// replays it from Lrem = L, subtracts each collected term as it is met, and
// scatters dL . (d NEE_k + Lrem (d f_k)/f_k) at each scattering vertex.
// MODE_CACHED: a path stops at its record vertex -- the first scattering
// vertex with index >= K, after that vertex's emission -- and appends a query
// (features, throughput, pixel) for the radiance cache to answer.
// MODE_TRAIN: a path records the features of its record vertex, goes on as a
// plain path, and writes target = (radiance after the record point) / beta.
// MODE_CACHED_SAMPLES: as MODE_CACHED, but each sample's radiance goes to
// io.lsamp[g] and its query carries the sample index g instead of the pixel.
// MODE_ADJOINT_CACHED: pass B only, from Lrem = io.lsamp[g] (the cached
// estimate with the cache's answer already added); the replay stops at the
// record vertex, so the detached cache term reaches earlier vertices through
// Lrem and nothing is scattered for the network.
// MODE_JVP: forward-mode derivative along a parameter direction (tangent
// textures in tab.gtex, tangent roughness in sink.rough_global): the tangents
// of beta and L ride along the path; `out` receives the sum of the sample
// radiance tangents.  Attached and detached terms as in the replay.
// Samples g_base .. g_base + n_samples - 1 start at pixel (cam, x, y).
// ---------------------------------------------------------------------------
enum {
  MODE_PRIMAL = 0,
  MODE_ADJOINT = 1,
  MODE_CACHED = 2,
  MODE_TRAIN = 3,
  MODE_CACHED_SAMPLES = 4,
  MODE_ADJOINT_CACHED = 5,
  MODE_JVP = 6
};

template <int MODE>
DEV void render_pixel(const DScene& s, const DParams& P, const DCams& C, const DRender& R,
                      const LdsTables& tab, int cam, int x, int y, uint64_t g_base, int n_samples,
                      f3 dL, int* stk, Counters& cnt, const Sink& sink, const DNrcIO& io,
                      f3& out) {
  constexpr bool ADJ = MODE == MODE_ADJOINT || MODE == MODE_ADJOINT_CACHED;
  constexpr bool JVP = MODE == MODE_JVP;
  // modes with a record vertex (cache queries, training records, cached replay)
  constexpr bool HOOK = MODE == MODE_CACHED || MODE == MODE_TRAIN || MODE == MODE_CACHED_SAMPLES ||
                        MODE == MODE_ADJOINT_CACHED;
  constexpr bool QUERY = MODE == MODE_CACHED || MODE == MODE_CACHED_SAMPLES;
  const int W = C.width, H = C.height;
  const uint64_t pix = ((uint64_t)cam * H + y) * W + x;
  const int n_em = s.n_ems;
  const float p_sel = n_em > 0 ? 1.0f / (float)n_em : 0.f;
  const bool no_nee = (R.flags & DRT_FLAG_NO_NEE) != 0;

  f3 acc = mk(0, 0, 0);
  int sidx = 0;
  uint32_t glo = 0, ghi = 0;
  f3 beta, L, Lrem = mk(0, 0, 0), o, d, prev_p;
  f3 tbeta = mk(0, 0, 0), tL = mk(0, 0, 0);  // tangents (MODE_JVP)
  float prev_pdf;
  int k;
  // record vertex (MODE_TRAIN)
  bool recorded = false;
  f3 beta_at = mk(0, 0, 0), L_at = mk(0, 0, 0);

  auto start = [&]() {
    uint64_t g = g_base + (uint64_t)sidx;
    glo = (uint32_t)g;
    ghi = (uint32_t)(g >> 32);
    camera_ray(C.cam[cam], W, H, x, y, glo, ghi, R, o, d);
    beta = mk(1, 1, 1);
    L = mk(0, 0, 0);
    tbeta = mk(0, 0, 0);
    tL = mk(0, 0, 0);
    prev_pdf = 0.f;  // 0: the next emitter hit takes no MIS weight
    prev_p = o;
    k = 1;
    recorded = false;
    cnt.samples++;
  };

  // one vertex for this lane: returns true when the path has ended.  The
  // replay variant (pass B) carries the subtraction and the scatter; the
  // other passes compile without them.
  auto step = [&](auto replay) -> bool {
    constexpr bool RB = ADJ && decltype(replay)::value;
    constexpr bool DER = RB || JVP;  // BSDF parameter derivatives needed
    bool done = false, nee = false;
    f3 nee_c = mk(0, 0, 0), nee_gt = mk(0, 0, 0), nee_t = mk(0, 0, 0), so = o, sd = d;
    float nee_gr = 0.f, stmax = 0.f;
    bool bsdf_pend = false;
    f3 rat_alb = mk(0, 0, 0), rat_alpha = mk(0, 0, 0);
    int vtex = -1, vtexel = 0, vrslot = -1;
    // ---------------- phase A: closest hit and the vertex's work
    {
      RayPre rp = ray_pre(o, d);
      Hit h;
      cnt.rays++;
      const bool hit = traverse(s, rp, 0.f, INFINITY, false, h, stk, cnt);
      if (!hit) {
        if (s.env_emitter >= 0) {
          int row, col;
          float st;
          env_cell(s, d, row, col, st);
          float w = 1.0f;
          if (!(prev_pdf == 0.f || no_nee)) w = power_heuristic(prev_pdf, p_sel * env_pdf(s, row, col, st));
          f3 c = beta * env_lookup(s, row, col) * w;
          L = L + c;
          if (RB) Lrem = Lrem - c;
          if (JVP) tL = tL + tbeta * env_lookup(s, row, col) * w;
        }
        done = true;
      } else {
        DTri T = load_tri(s, h.tri);
        f3 p0 = mk(T.p0x, T.p0y, T.p0z), p1 = mk(T.p1x, T.p1y, T.p1z), p2 = mk(T.p2x, T.p2y, T.p2z);
        float b0 = 1.0f - h.b1 - h.b2;
        f3 p = p0 * b0 + p1 * h.b1 + p2 * h.b2;
        f3 n_g = normalize(cross(p1 - p0, p2 - p0));
        const float4* shp = reinterpret_cast<const float4*>(s.shade + T.prim);
        float4 sb = shp[1];
        int mat_id = __float_as_int(sb.z), em_id = __float_as_int(sb.w);
        float cos_y = -dot(d, n_g);
        if (em_id >= 0 && cos_y > 0.f) {
          const DEmitter& E = s.ems[em_id];
          float w = 1.0f;
          if (!(prev_pdf == 0.f || no_nee)) {
            f3 dv = p - prev_p;
            w = power_heuristic(prev_pdf, p_sel * dot(dv, dv) / (E.area * cos_y));
          }
          f3 c = beta * mk(E.radiance[0], E.radiance[1], E.radiance[2]) * w;
          L = L + c;
          if (RB) Lrem = Lrem - c;
          if (JVP) tL = tL + tbeta * mk(E.radiance[0], E.radiance[1], E.radiance[2]) * w;
        }
        if (k == R.max_depth) {
          done = true;
        } else {
          uint4 r0 = philox(glo, ghi, (uint32_t)(k - 1), 0u, R.key0, R.key1);
          uint4 r1 = philox(glo, ghi, (uint32_t)(k - 1), 1u, R.key0, R.key1);
          const DMaterial& M = s.mats[mat_id];
          const int type = M.type;
          if (type == DRT_BSDF_NULL || (type == DRT_BSDF_MASK && u01(r1.w) >= M.opacity)) {
            // pass-through: same direction, counts as a vertex
            if (type == DRT_BSDF_MASK) prev_pdf = 0.f;
            o = spawn(s, p, n_g, d);
            ++k;
          } else {
            cnt.verts++;
            // hoisted out of the switch: frame, albedo (texture or constant), roughness
            Frame fr = make_frame(n_g);
            f3 wi = to_local(fr, -d);
            Shade sh;
            sh.type = type;
            sh.albedo = mk(M.albedo[0], M.albedo[1], M.albedo[2]);
            sh.f0 = mk(M.f0[0], M.f0[1], M.f0[2]);
            sh.alpha = M.alpha;
            sh.eta = M.eta;
            sh.opacity = M.opacity;
            vtex = M.texture;
            if (vtex >= 0) {
              float4 sa = shp[0];
              float u = sa.x * b0 + sa.z * h.b1 + sb.x * h.b2;
              float v = sa.y * b0 + sa.w * h.b1 + sb.y * h.b2;
              int TW = tab.tw[vtex], TH = tab.th[vtex];
              int tx = (int)fminf(floorf(fmaxf(u, 0.f) * (float)TW), (float)(TW - 1));
              int ty = (int)fminf(floorf(fmaxf(v, 0.f) * (float)TH), (float)(TH - 1));
              vtexel = ty * TW + tx;
              const float* tp = tab.tex[vtex] + 3 * (size_t)vtexel;
              sh.albedo = mk(tp[0], tp[1], tp[2]);
            }
            vrslot = M.rough_slot;
            if (vrslot >= 0) sh.alpha = P.rough[vrslot];
            // the direction's components at this vertex (MODE_JVP)
            f3 vt = mk(0, 0, 0);
            float vr = 0.f;
            if (JVP) {
              if (vtex >= 0 && tab.gtex[vtex]) {
                const float* tp = tab.gtex[vtex] + 3 * (size_t)vtexel;
                vt = mk(tp[0], tp[1], tp[2]);
              }
              if (vrslot >= 0 && sink.rough_global) vr = sink.rough_global[vrslot];
            }
            bool stop_here = false;
            if (HOOK && !recorded && k >= io.K) {
              // features of the record vertex: position, direction back along
              // the ray, normal facing it, roughness (1 unless microfacet),
              // albedo (f0 for a conductor, 1 for a dielectric)
              f3 w = -d;
              f3 nn = dot(n_g, w) >= 0.f ? n_g : -n_g;
              bool ggx = type == DRT_BSDF_CONDUCTOR || type == DRT_BSDF_DIELECTRIC ||
                         type == DRT_BSDF_PLASTIC;
              f3 alb = type == DRT_BSDF_CONDUCTOR ? sh.f0
                       : (type == DRT_BSDF_DIELECTRIC ? mk(1, 1, 1) : sh.albedo);
              float* rec = nullptr;
              if (QUERY) {
                int slot = atomicAdd(io.count, 1);
                if (slot < io.capacity) {
                  rec = io.rec + (size_t)NRC_REC * slot;
                  io.qpix[slot] = MODE == MODE_CACHED_SAMPLES ? (int)glo : (int)pix;
                  if (io.qbin) io.qbin[slot] = query_bin(p.x, p.y, p.z, io.lo, io.inv_ext);
                  rec[13] = beta.x;
                  rec[14] = beta.y;
                  rec[15] = beta.z;
                }
              } else if (MODE == MODE_TRAIN) {
                rec = io.rec + (size_t)NRC_REC * g_base;
                recorded = true;
                beta_at = beta;
                L_at = L;
              }
              if (MODE != MODE_TRAIN) {
                stop_here = true;
                done = true;
              }
              if (rec) {
                rec[0] = p.x; rec[1] = p.y; rec[2] = p.z;
                rec[3] = w.x; rec[4] = w.y; rec[5] = w.z;
                rec[6] = nn.x; rec[7] = nn.y; rec[8] = nn.z;
                rec[9] = ggx ? sh.alpha : 1.0f;
                rec[10] = alb.x; rec[11] = alb.y; rec[12] = alb.z;
              }
            }
            // next-event candidate; its shadow ray is traced in phase B
            if (!stop_here && !no_nee && n_em > 0) {
              const DEmitter& E = s.ems[pick(r0.x, (uint32_t)n_em)];
              float lu = u01(r0.y), lv = u01(r0.z);
              bool valid = false, delta = false, finite = false;
              f3 wl = mk(0, 0, 1), y = mk(0, 0, 0), Le = mk(0, 0, 0);
              float pdf_l = 0.f;
              if (E.type == DRT_EMITTER_AREA) {
                y = mk(E.p0[0], E.p0[1], E.p0[2]) + mk(E.e1[0], E.e1[1], E.e1[2]) * lu +
                    mk(E.e2[0], E.e2[1], E.e2[2]) * lv;
                f3 dv = y - p;
                float dist2 = dot(dv, dv), dist = sqrtf(dist2);
                wl = dv * (1.0f / dist);
                float cy = -dot(wl, mk(E.n[0], E.n[1], E.n[2]));
                if (cy > 0.f) {
                  pdf_l = dist2 / (E.area * cy);
                  Le = mk(E.radiance[0], E.radiance[1], E.radiance[2]);
                  finite = true;
                  valid = true;
                }
              } else if (E.type == DRT_EMITTER_ENV) {
                if (env_sample(s, lu, lv, wl)) {
                  int row, col;
                  float st;
                  env_cell(s, wl, row, col, st);
                  pdf_l = env_pdf(s, row, col, st);
                  if (pdf_l > 0.f) {
                    Le = env_lookup(s, row, col);
                    valid = true;
                  }
                }
              } else {
                wl = mk(E.p0[0], E.p0[1], E.p0[2]);
                Le = mk(E.radiance[0], E.radiance[1], E.radiance[2]);
                pdf_l = 1.0f;
                delta = true;
                valid = true;
              }
              if (valid) {
                BEval fe = bsdf_eval<DER>(sh, wi, to_local(fr, wl));
                if (nonzero(fe.f)) {
                  float w = delta ? 1.0f : power_heuristic(p_sel * pdf_l, fe.pdf);
                  f3 coef = beta * Le * (w / (p_sel * pdf_l));
                  nee_c = coef * fe.f;
                  if (JVP)
                    nee_t = tbeta * Le * (w / (p_sel * pdf_l)) * fe.f +
                            coef * (fe.dalb * vt + fe.dalpha * vr);
                  if (RB) {
                    nee_gt = dL * coef * fe.dalb;
                    f3 g = dL * coef * fe.dalpha;
                    nee_gr = g.x + g.y + g.z;
                  }
                  // shadow ray from the offset origin; towards an area light it
                  // stops short of the sampled point by 1e-4 of its length
                  so = spawn(s, p, n_g, wl);
                  sd = wl;
                  stmax = INFINITY;
                  if (finite) {
                    f3 dv = y - so;
                    float dl = sqrtf(dot(dv, dv));
                    sd = dv * (1.0f / dl);
                    stmax = (1.0f - 1e-4f) * dl;
                  }
                  nee = true;
                }
              }
            }
            // BSDF sampling
            f3 wo;
            BEval be;
            const bool ok = !stop_here &&
                            bsdf_sample<DER>(sh, wi, u01(r1.x), u01(r1.y), u01(r0.w), wo, be);
            if (RB) {
              bsdf_pend = ok;
              if (bsdf_pend) {
                rat_alb = mk(be.f.x != 0.f ? be.dalb.x / be.f.x : 0.f,
                             be.f.y != 0.f ? be.dalb.y / be.f.y : 0.f,
                             be.f.z != 0.f ? be.dalb.z / be.f.z : 0.f);
                rat_alpha = mk(be.f.x != 0.f ? be.dalpha.x / be.f.x : 0.f,
                               be.f.y != 0.f ? be.dalpha.y / be.f.y : 0.f,
                               be.f.z != 0.f ? be.dalpha.z / be.f.z : 0.f);
              }
            }
            if (ok) {
              if (JVP) tbeta = (tbeta * be.f + beta * (be.dalb * vt + be.dalpha * vr)) * (1.0f / be.pdf);
              beta = beta * be.f * (1.0f / be.pdf);
              prev_pdf = be.pdf;
              prev_p = p;
              f3 wow = to_world(fr, wo);
              o = spawn(s, p, n_g, wow);
              d = wow;
              if (k >= R.rr_depth) {
                float q = fminf(maxc(beta), 0.95f);
                if (u01(r1.z) >= q) {
                  done = true;
                } else {
                  beta = beta * (1.0f / q);
                  if (JVP) tbeta = tbeta * (1.0f / q);
                }
              }
            } else {
              done = true;
            }
            ++k;
          }
        }
      }
    }
    // ---------------- phase B: the shadow ray of this vertex
    f3 gtex = mk(0, 0, 0);
    float grough = 0.f;
    if (nee) {
      RayPre rp = ray_pre(so, sd);
      Hit h;
      cnt.shadow++;
      if (!traverse(s, rp, 0.f, stmax, true, h, stk, cnt)) {
        L = L + nee_c;
        if (JVP) tL = tL + nee_t;
        if (RB) {
          Lrem = Lrem - nee_c;
          gtex = nee_gt;
          grough = nee_gr;
        }
      }
    }
    if (RB && bsdf_pend) {
      // radiance arriving over the sampled direction = what is left of L
      gtex = gtex + dL * Lrem * rat_alb;
      f3 g = dL * Lrem * rat_alpha;
      grough += g.x + g.y + g.z;
    }
    if (RB) {
      // one scatter per vertex for its next-event and continuation terms
      if (vtex >= 0) scatter_tex(sink, vtex, vtexel, gtex, cnt);
      if (vrslot >= 0) scatter_rough(sink, vrslot, grough, cnt);
    }
    return done;
  };
  // lanes start each path together (coherent primary rays); a lane whose
  // path ends early waits for the wave
  for (;;) {
    start();
    if constexpr (MODE == MODE_ADJOINT_CACHED) {
      const float* ls = io.lsamp + 3 * (g_base + (uint64_t)sidx);
      Lrem = mk(ls[0], ls[1], ls[2]);
      while (!step(std::true_type{})) {
      }
      if (++sidx == n_samples) break;
      continue;
    }
    while (!step(std::false_type{})) {
    }
    if (MODE == MODE_TRAIN) {
      float* rec = io.rec + (size_t)NRC_REC * g_base;
      if (recorded) {
        rec[13] = beta_at.x != 0.f ? (L.x - L_at.x) / beta_at.x : 0.f;
        rec[14] = beta_at.y != 0.f ? (L.y - L_at.y) / beta_at.y : 0.f;
        rec[15] = beta_at.z != 0.f ? (L.z - L_at.z) / beta_at.z : 0.f;
        atomicAdd(io.count, 1);
      } else {
        for (int c = 0; c < NRC_REC; ++c) rec[c] = 0.f;
      }
      io.valid[g_base] = recorded ? 1 : 0;
    }
    if (ADJ) {
      Lrem = L;  // pass B replays this sample from its full radiance
      start();
      while (!step(std::true_type{})) {
      }
      cnt.lrem_max = fmaxf(cnt.lrem_max, fmaxf(fabsf(Lrem.x), fmaxf(fabsf(Lrem.y), fabsf(Lrem.z))));
    } else if (JVP) {
      acc = acc + tL;
    } else if (MODE == MODE_CACHED_SAMPLES) {
      float* ls = io.lsamp + 3 * (g_base + (uint64_t)sidx);
      ls[0] = L.x;
      ls[1] = L.y;
      ls[2] = L.z;
    } else {
      acc = acc + L;
    }
    if (++sidx == n_samples) break;
  }
  out = acc;
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

DEV void flush_counters(const DRender& R, Counters& c) {
  if (!R.stats) return;
  atomicAdd((unsigned long long*)&R.stats[DRT_STAT_RAYS], (unsigned long long)c.rays);
  atomicAdd((unsigned long long*)&R.stats[DRT_STAT_SHADOW], (unsigned long long)c.shadow);
  atomicAdd((unsigned long long*)&R.stats[DRT_STAT_NODES], (unsigned long long)c.nodes);
  atomicAdd((unsigned long long*)&R.stats[DRT_STAT_TRIS], (unsigned long long)c.tris);
  atomicAdd((unsigned long long*)&R.stats[DRT_STAT_VERTICES], (unsigned long long)c.verts);
  atomicAdd((unsigned long long*)&R.stats[DRT_STAT_SCATTER], (unsigned long long)c.scatter);
  atomicAdd((unsigned long long*)&R.stats[DRT_STAT_SAMPLES], (unsigned long long)c.samples);
  atomicMax((unsigned long long*)&R.stats[DRT_STAT_LREM_MAX],
            (unsigned long long)__float_as_uint(c.lrem_max));
}

// ---------------------------------------------------------------------------
// megakernels: one 8x8 pixel tile per workgroup (one wave)
// ---------------------------------------------------------------------------
// STATS = false compiles the counters out (they are never read).
// MODE: MODE_PRIMAL, MODE_CACHED (paths stop at their record vertex and
// append cache queries) or MODE_CACHED_SAMPLES (per-sample radiance, no image).
template <bool STATS, int MODE>
__global__ __launch_bounds__(kBlock) void k_render_forward(DScene s, DParams P, DCams C, DRender R,
                                                           float* __restrict__ image, DNrcIO io) {
  __shared__ int stack[kStackDepth * kBlock];
  __shared__ LdsTables tab;
  load_tables(tab, s, P, nullptr);
  __syncthreads();
  const int W = C.width, H = C.height;
  const int x = blockIdx.x * kTile + (threadIdx.x % kTile);
  const int y = blockIdx.y * kTile + (threadIdx.x / kTile);
  const int cam = blockIdx.z;
  Counters cnt = {};
  if (x < W && y < H) {
    Sink none{&tab, nullptr, nullptr};
    f3 acc;
    const uint64_t pix = ((uint64_t)cam * H + y) * W + x;
    render_pixel<MODE>(s, P, C, R, tab, cam, x, y, pix * (uint64_t)R.spp, R.spp, mk(0, 0, 0),
                       stack + threadIdx.x, cnt, none, io, acc);
    if (MODE != MODE_CACHED_SAMPLES) {
      const float inv = 1.0f / (float)R.spp;
      float* out = image + 3 * (((size_t)cam * H + y) * W + x);
      out[0] = acc.x * inv;
      out[1] = acc.y * inv;
      out[2] = acc.z * inv;
    }
  }
  if constexpr (STATS) flush_counters(R, cnt);
}

// Held to 128 VGPRs (4 waves per SIMD): measured faster than 3 waves at 131.
// MODE: MODE_ADJOINT (both passes) or MODE_ADJOINT_CACHED (replay from the
// per-sample cached estimates in io.lsamp).
template <bool STATS, int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_render_adjoint(DScene s, DParams P, DCams C, DRender R,
                                                           const float* __restrict__ adj,
                                                           DGrads G, DNrcIO io) {
  __shared__ int stack[kStackDepth * kBlock];
  __shared__ LdsTables tab;
  __shared__ float rough_acc[kMaxRoughLds];
  const bool lds_rough = G.rough && s.n_rough <= kMaxRoughLds;
  load_tables(tab, s, P, &G);
  if (threadIdx.x < kMaxRoughLds) rough_acc[threadIdx.x] = 0.f;
  __syncthreads();
  const int W = C.width, H = C.height;
  const int x = blockIdx.x * kTile + (threadIdx.x % kTile);
  const int y = blockIdx.y * kTile + (threadIdx.x / kTile);
  const int cam = blockIdx.z;
  Counters cnt = {};
  if (x < W && y < H) {
    const size_t pix = ((size_t)cam * H + y) * W + x;
    const float inv = 1.0f / (float)R.spp;
    f3 dL = mk(adj[3 * pix] * inv, adj[3 * pix + 1] * inv, adj[3 * pix + 2] * inv);
    if (nonzero(dL)) {
      Sink sink{&tab, lds_rough ? rough_acc : nullptr, lds_rough ? nullptr : G.rough};
      f3 unused;
      render_pixel<MODE>(s, P, C, R, tab, cam, x, y, pix * (uint64_t)R.spp, R.spp, dL,
                         stack + threadIdx.x, cnt, sink, io, unused);
    }
  }
  __syncthreads();
  if (lds_rough && threadIdx.x < s.n_rough) {
    float v = rough_acc[threadIdx.x];
    if (v != 0.f) {
      atomicAdd(G.rough + threadIdx.x, v);
      cnt.scatter++;
    }
  }
  if constexpr (STATS) flush_counters(R, cnt);
}

// Forward-mode derivative of the image along the direction T (tangent
// textures and roughness): out = (1/spp) sum of the sample radiance tangents.
__global__ __launch_bounds__(kBlock) void k_render_jvp(DScene s, DParams P, DCams C, DRender R,
                                                       DGrads T, float* __restrict__ image) {
  __shared__ int stack[kStackDepth * kBlock];
  __shared__ LdsTables tab;
  load_tables(tab, s, P, &T);
  __syncthreads();
  const int W = C.width, H = C.height;
  const int x = blockIdx.x * kTile + (threadIdx.x % kTile);
  const int y = blockIdx.y * kTile + (threadIdx.x / kTile);
  const int cam = blockIdx.z;
  Counters cnt = {};
  if (x < W && y < H) {
    Sink dir{&tab, nullptr, T.rough};
    DNrcIO none = {};
    f3 acc;
    const uint64_t pix = ((uint64_t)cam * H + y) * W + x;
    render_pixel<MODE_JVP>(s, P, C, R, tab, cam, x, y, pix * (uint64_t)R.spp, R.spp, mk(0, 0, 0),
                           stack + threadIdx.x, cnt, dir, none, acc);
    const float inv = 1.0f / (float)R.spp;
    float* out = image + 3 * pix;
    out[0] = acc.x * inv;
    out[1] = acc.y * inv;
    out[2] = acc.z * inv;
  }
}

// Training paths of the radiance cache: path j (counter g = j) starts at the
// pixel chosen by the first word of its camera block dim 2, and writes record
// j (features, target) and valid[j].
__global__ __launch_bounds__(kBlock) void k_nrc_records(DScene s, DParams P, DCams C, DRender R,
                                                        int64_t n_paths, DNrcIO io) {
  __shared__ int stack[kStackDepth * kBlock];
  __shared__ LdsTables tab;
  load_tables(tab, s, P, nullptr);
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n_paths) return;
  const uint32_t n_pix = (uint32_t)((int64_t)C.n * C.width * C.height);
  uint4 r = philox((uint32_t)j, (uint32_t)((uint64_t)j >> 32), 0xFFFFFFFFu, 2u, R.key0, R.key1);
  const uint32_t pid = pick(r.x, n_pix);
  const int cam = (int)(pid / ((uint32_t)C.width * C.height));
  const int y = (int)((pid / C.width) % C.height), x = (int)(pid % C.width);
  Counters cnt = {};
  Sink none{&tab, nullptr, nullptr};
  f3 unused;
  render_pixel<MODE_TRAIN>(s, P, C, R, tab, cam, x, y, (uint64_t)j, 1, mk(0, 0, 0),
                           stack + threadIdx.x, cnt, none, io, unused);
}

// Ray queries (closest / any) for tests and traversal measurements.
__global__ __launch_bounds__(kBlock) void k_trace(DScene s, const float* __restrict__ rays,
                                                  int64_t n, int mode, drt_hit* __restrict__ out) {
  __shared__ int stack[kStackDepth * kBlock];
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float4* rp = reinterpret_cast<const float4*>(rays + 8 * i);
  float4 a = rp[0], b = rp[1];
  RayPre r = ray_pre(mk(a.x, a.y, a.z), mk(b.x, b.y, b.z));
  Counters cnt = {};
  Hit h;
  drt_hit o;
  if (mode == 0) {
    bool hit = traverse(s, r, a.w, b.w, false, h, stack + threadIdx.x, cnt);
    o.t = hit ? h.t : INFINITY;
    o.b1 = hit ? h.b1 : 0.f;
    o.b2 = hit ? h.b2 : 0.f;
    o.prim = hit ? h.prim : -1;
  } else {
    bool hit = traverse(s, r, a.w, b.w, true, h, stack + threadIdx.x, cnt);
    o.t = 0.f;
    o.b1 = 0.f;
    o.b2 = 0.f;
    o.prim = hit ? 1 : -1;
  }
  out[i] = o;
}

__global__ void k_philox(const uint32_t* __restrict__ ctr, const uint32_t* __restrict__ key,
                         int64_t n, uint32_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint4 r = philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], key[2 * i],
                   key[2 * i + 1]);
  out[4 * i] = r.x;
  out[4 * i + 1] = r.y;
  out[4 * i + 2] = r.z;
  out[4 * i + 3] = r.w;
}

// ---------------------------------------------------------------------------
// loss and optimiser (streaming, HBM-bound)
// ---------------------------------------------------------------------------
constexpr int kLossBlocks = 1024;

__global__ __launch_bounds__(256) void k_loss_partial(const float* __restrict__ img,
                                                      const float* __restrict__ tgt, int64_t n,
                                                      float* __restrict__ adj,
                                                      double* __restrict__ partial) {
  __shared__ double red[256];
  double acc = 0.0;
  const float scale = (float)(2.0 / (double)n);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    float r = img[i] - tgt[i];
    acc += (double)r * (double)r;
    if (adj) adj[i] = r * scale;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ partial, int nb,
                                                    int64_t n, float* __restrict__ loss) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)(red[0] / (double)n);
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2, float lo, float hi, int zero,
                                              uint16_t* __restrict__ half_out) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * 256;
  for (; i < n; i += stride) {
    float gi = g[i];
    if (zero) g[i] = 0.f;
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float x = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    x = fminf(fmaxf(x, lo), hi);
    p[i] = x;
    if (half_out) half_out[i] = __half_as_ushort(__float2half_rn(x));
  }
}

// ---------------------------------------------------------------------------
// launchers

// ---------------------------------------------------------------------------
hipError_t launch_render_forward(const DScene& s, const DParams& p, const DCams& c,
                                 const DRender& r, float* image, hipStream_t st) {
  dim3 grid((c.width + kTile - 1) / kTile, (c.height + kTile - 1) / kTile, c.n);
  DNrcIO none = {};
  if (r.stats)
    hipLaunchKernelGGL((k_render_forward<true, MODE_PRIMAL>), grid, dim3(kBlock), 0, st, s, p, c,
                       r, image, none);
  else
    hipLaunchKernelGGL((k_render_forward<false, MODE_PRIMAL>), grid, dim3(kBlock), 0, st, s, p,
                       c, r, image, none);
  return hipGetLastError();
}

hipError_t launch_render_cached(const DScene& s, const DParams& p, const DCams& c,
                                const DRender& r, float* image, const DNrcIO& io,
                                hipStream_t st) {
  dim3 grid((c.width + kTile - 1) / kTile, (c.height + kTile - 1) / kTile, c.n);
  if (io.lsamp)
    hipLaunchKernelGGL((k_render_forward<false, MODE_CACHED_SAMPLES>), grid, dim3(kBlock), 0, st,
                       s, p, c, r, image, io);
  else
    hipLaunchKernelGGL((k_render_forward<false, MODE_CACHED>), grid, dim3(kBlock), 0, st, s, p,
                       c, r, image, io);
  return hipGetLastError();
}

hipError_t launch_nrc_records(const DScene& s, const DParams& p, const DCams& c, const DRender& r,
                              int64_t n_paths, const DNrcIO& io, hipStream_t st) {
  int64_t blocks = (n_paths + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_nrc_records, dim3((unsigned)blocks), dim3(kBlock), 0, st, s, p, c, r,
                     n_paths, io);
  return hipGetLastError();
}

hipError_t launch_render_adjoint(const DScene& s, const DParams& p, const DCams& c,
                                 const DRender& r, const float* adj, const DGrads& g,
                                 hipStream_t st) {
  dim3 grid((c.width + kTile - 1) / kTile, (c.height + kTile - 1) / kTile, c.n);
  DNrcIO none = {};
  if (r.stats)
    hipLaunchKernelGGL((k_render_adjoint<true, MODE_ADJOINT>), grid, dim3(kBlock), 0, st, s, p,
                       c, r, adj, g, none);
  else
    hipLaunchKernelGGL((k_render_adjoint<false, MODE_ADJOINT>), grid, dim3(kBlock), 0, st, s, p,
                       c, r, adj, g, none);
  return hipGetLastError();
}

hipError_t launch_render_adjoint_cached(const DScene& s, const DParams& p, const DCams& c,
                                        const DRender& r, const float* adj, const DGrads& g,
                                        const DNrcIO& io, hipStream_t st) {
  dim3 grid((c.width + kTile - 1) / kTile, (c.height + kTile - 1) / kTile, c.n);
  if (r.stats)
    hipLaunchKernelGGL((k_render_adjoint<true, MODE_ADJOINT_CACHED>), grid, dim3(kBlock), 0, st,
                       s, p, c, r, adj, g, io);
  else
    hipLaunchKernelGGL((k_render_adjoint<false, MODE_ADJOINT_CACHED>), grid, dim3(kBlock), 0, st,
                       s, p, c, r, adj, g, io);
  return hipGetLastError();
}

hipError_t launch_render_jvp(const DScene& s, const DParams& p, const DCams& c, const DRender& r,
                             const DGrads& t, float* image, hipStream_t st) {
  dim3 grid((c.width + kTile - 1) / kTile, (c.height + kTile - 1) / kTile, c.n);
  hipLaunchKernelGGL(k_render_jvp, grid, dim3(kBlock), 0, st, s, p, c, r, t, image);
  return hipGetLastError();
}

hipError_t launch_trace(const DScene& s, const float* rays, int64_t n, int mode, drt_hit* hits,
                        hipStream_t st) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_trace, dim3((unsigned)blocks), dim3(kBlock), 0, st, s, rays, n, mode, hits);
  return hipGetLastError();
}

hipError_t launch_philox(const uint32_t* ctr, const uint32_t* key, int64_t n, uint32_t* out,
                         hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_philox, dim3((unsigned)blocks), dim3(256), 0, st, ctr, key, n, out);
  return hipGetLastError();
}

int64_t loss_workspace_floats(int64_t) { return 2 * kLossBlocks; }

hipError_t launch_loss_l2(const float* img, const float* tgt, int64_t n, float* adj, float* loss,
                          float* ws, hipStream_t st) {
  int64_t nb = (n + 255) / 256;
  if (nb > kLossBlocks) nb = kLossBlocks;
  double* partial = reinterpret_cast<double*>(ws);
  hipLaunchKernelGGL(k_loss_partial, dim3((unsigned)nb), dim3(256), 0, st, img, tgt, n, adj,
                     partial);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, partial, (int)nb, n, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, float* g, float* m, float* v, int64_t n,
                       const drt_adam_opts& o, hipStream_t st) {
  double c1 = 1.0 - pow((double)o.beta1, (double)o.step);
  double c2 = 1.0 - pow((double)o.beta2, (double)o.step);
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, st, p, g, m, v, n, o.lr,
                     o.beta1, o.beta2, o.eps, (float)c1, (float)c2, o.lo, o.hi, o.zero_grad,
                     o.half_out);
  return hipGetLastError();
}

__global__ void k_zero(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0u;
}

hipError_t launch_zero(void* p, int64_t n_words, hipStream_t st) {
  int64_t blocks = (n_words + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t*)p, n_words);
  return hipGetLastError();
}

}  // namespace drt
