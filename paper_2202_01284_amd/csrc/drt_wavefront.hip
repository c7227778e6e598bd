// Wavefront variants of the primal renderer and of the replayed adjoint:
// the same estimators as the megakernels (identical Philox counters,
// conventions, device functions and arithmetic order), but every bounce is
// split into separate kernels that pass the path state through HBM --
// closest hit, shading, shadow ray (in the replay: resolving the vertex and
// scattering its gradient) -- the execution model the paper compares its
// megakernels against (Sec. "Evaluation": wavefront versus megakernel).
// One lane per path g = ((cam H + y) W + x) spp + s; paths that have ended
// return at once (no compaction).  The adjoint runs pass A (the primal with
// the replay seed, for each path's radiance L) and then pass B, the replay
// from L_rem = L with the subtractions and the gradient scatter of Path
// Replay Backpropagation (Sec. "Physically Based Differentiable Rendering").
//
// Path state (structure of arrays, float4 each, in a caller workspace):
//   o4  = (origin, prev_pdf)        d4  = (direction, k as int bits)
//   b4  = (beta, alive as int bits) L4  = (radiance, or L_rem in the replay)
//   pp4 = (prev_p, unused)          h4  = (t, b1, b2, triangle as int bits)
//   so4 = (shadow origin, tmax)     sd4 = (shadow direction, pending flag)
//   sc4 = (next-event contribution, unused)
// and, for the replay, the vertex's pending derivative terms:
//   pa4 = ((d f/d albedo)/f, unused) pr4 = ((d f/d alpha)/f, unused)
//   pn4 = (next-event albedo gradient, next-event roughness gradient)
//   pv4 = (texture, texel, roughness slot, BSDF sample pending) as int bits
// and, for the checkpointed adjoint, pe4 = (emission found at the vertex,
// unused).  The shading kernel reads the ray state from o4, d4, b4, pp4 and
// writes the next bounce's to no4, nd4, nb4, npp4 (the same arrays, except
// in the checkpointed variant).
//
// Checkpointed adjoint (the naive alternative to Path Replay
// Backpropagation that Sec. "Evaluation" measures against it: a standard
// path tracer differentiated with one checkpoint per scattering event).
// The forward pass is the primal, with the ray state before every bounce
// kept in a tape slice of the workspace (o4, d4, b4, pp4: 64 B per path and
// bounce), so it costs memory in proportion to the path length.  The
// backward pass walks the bounces from the last to the first: it restores
// the ray of bounce i from its slice, recomputes the vertex (closest hit,
// shading with derivatives, shadow ray), forms the vertex's gradient with
// A = the radiance collected by the later vertices -- the quantity the
// replay obtains as L_rem by subtraction -- and then adds the vertex's own
// emission and next-event terms to A.
#include "drt_device.h"

namespace drt {

struct WState {
  float4 *o4, *d4, *b4, *L4, *pp4, *h4, *so4, *sd4, *sc4;
  float4 *pa4, *pr4, *pn4, *pv4, *pe4;
  float4 *no4, *nd4, *nb4, *npp4;  // where the shading kernel writes the next ray state
};

constexpr int kWfBlock = 64;    // one wave per workgroup (LDS traversal stack per lane)
constexpr int kWfArrays = 9;    // primal state
constexpr int kWfArraysAdj = 13;  // with the replay's pending terms
constexpr int kWfArraysCk = 10;   // checkpointed adjoint: L4 .. pe4 besides the tape
constexpr int kTapeArrays = 4;    // o4, d4, b4, pp4 per bounce

// what the shading kernel computes
enum { WF_PRIMAL = 0, WF_REPLAY = 1, WF_BACKWARD = 2 };

// the path's share of the image adjoint (zero: the path is not traced)
DEV f3 path_dL(const float* adj, int64_t g, int spp) {
  const int64_t pix = g / spp;
  const float inv = 1.0f / (float)spp;
  return mk(adj[3 * pix] * inv, adj[3 * pix + 1] * inv, adj[3 * pix + 2] * inv);
}

DEV f3 xyz(float4 v) { return mk(v.x, v.y, v.z); }
DEV float4 f4(f3 a, float w) { return make_float4(a.x, a.y, a.z, w); }

// camera rays of all paths.  ADJ: paths whose pixel has a zero adjoint are
// not traced; REPLAY: L4 keeps pass A's radiance as L_rem.
template <bool ADJ, bool REPLAY>
__global__ __launch_bounds__(kWfBlock) void k_wf_camera(DCams C, DRender R, int64_t n,
                                                        const float* __restrict__ adj, WState S) {
  const int64_t g = (int64_t)blockIdx.x * kWfBlock + threadIdx.x;
  if (g >= n) return;
  const bool live = !ADJ || nonzero(path_dL(adj, g, R.spp));
  const int64_t pix = g / R.spp;
  const int W = C.width, H = C.height;
  const int cam = (int)(pix / ((int64_t)W * H));
  const int y = (int)((pix / W) % H), x = (int)(pix % W);
  f3 o, d;
  camera_ray(C.cam[cam], W, H, x, y, (uint32_t)g, (uint32_t)((uint64_t)g >> 32), R, o, d);
  S.o4[g] = f4(o, 0.f);  // prev_pdf 0: the first emitter hit takes no MIS weight
  S.d4[g] = f4(d, __int_as_float(1));
  S.b4[g] = f4(mk(1, 1, 1), __int_as_float(live ? 1 : 0));
  if (!REPLAY) S.L4[g] = f4(mk(0, 0, 0), 0.f);
  S.pp4[g] = f4(o, 0.f);
  S.sd4[g] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (REPLAY) S.pv4[g] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// closest hit of every live path
__global__ __launch_bounds__(kWfBlock) void k_wf_trace(DScene s, int64_t n, WState S) {
  __shared__ int stack[kStackDepth * kWfBlock];
  const int64_t g = (int64_t)blockIdx.x * kWfBlock + threadIdx.x;
  if (g >= n) return;
  if (__float_as_int(S.b4[g].w) == 0) return;
  Counters cnt = {};
  Hit h;
  RayPre rp = ray_pre(xyz(S.o4[g]), xyz(S.d4[g]));
  const bool hit = traverse(s, rp, 0.f, INFINITY, false, h, stack + threadIdx.x, cnt);
  S.h4[g] = make_float4(h.t, h.b1, h.b2, __int_as_float(hit ? h.tri : -1));
}

// the vertex found by the closest hit: emission (MIS), then, below the
// maximum depth, a pass-through or the next-event candidate (its shadow ray
// left pending) and the BSDF sample with Russian roulette.  WF_REPLAY: the
// collected terms are subtracted from L_rem in L4 and the vertex's
// derivative terms are left pending for k_wf_resolve.  WF_BACKWARD: L4 (the
// radiance of the later vertices) is left alone; the emission goes to pe4
// and the derivative terms are left pending as in the replay.
template <int WM>
__global__ __launch_bounds__(kWfBlock) void k_wf_shade(DScene s, DParams P, DRender R, int64_t n,
                                                       const float* __restrict__ adj, WState S) {
  constexpr bool RB = WM == WF_REPLAY, CK = WM == WF_BACKWARD, DER = RB || CK;
  __shared__ LdsTables tab;
  load_tables(tab, s, P, nullptr);
  __syncthreads();
  const int64_t g = (int64_t)blockIdx.x * kWfBlock + threadIdx.x;
  if (g >= n) return;
  float4 b4 = S.b4[g];
  if (__float_as_int(b4.w) == 0) {
    if (S.nb4 != S.b4) S.nb4[g] = b4;  // an ended path stays ended in the next slice
    return;
  }
  const int n_em = s.n_ems;
  const float p_sel = n_em > 0 ? 1.0f / (float)n_em : 0.f;
  const bool no_nee = (R.flags & DRT_FLAG_NO_NEE) != 0;
  const uint32_t glo = (uint32_t)g, ghi = (uint32_t)((uint64_t)g >> 32);
  float4 o4 = S.o4[g], d4 = S.d4[g];
  f3 o = xyz(o4), d = xyz(d4), beta = xyz(b4), L = xyz(S.L4[g]), prev_p = xyz(S.pp4[g]);
  float prev_pdf = o4.w;
  int k = __float_as_int(d4.w);
  const float4 hv = S.h4[g];
  const int tri = __float_as_int(hv.w);
  bool done = false;
  bool nee = false;
  f3 nee_c = mk(0, 0, 0), so = o, sd = d;
  float stmax = 0.f;
  // replay: the vertex's derivative terms
  const f3 dL = DER ? path_dL(adj, g, R.spp) : mk(0, 0, 0);
  f3 e = mk(0, 0, 0);  // emission found here (WF_BACKWARD)
  f3 nee_gt = mk(0, 0, 0), rat_alb = mk(0, 0, 0), rat_alpha = mk(0, 0, 0);
  float nee_gr = 0.f;
  int vtex = -1, vtexel = 0, vrslot = -1;
  bool bsdf_pend = false, shaded = false;
  if (tri < 0) {
    if (s.env_emitter >= 0) {
      int row, col;
      float st;
      env_cell(s, d, row, col, st);
      float w = 1.0f;
      if (!(prev_pdf == 0.f || no_nee)) w = power_heuristic(prev_pdf, p_sel * env_pdf(s, row, col, st));
      f3 c = beta * env_lookup(s, row, col) * w;
      if (CK) e = c;
      else L = RB ? L - c : L + c;
    }
    done = true;
  } else {
    DTri T = load_tri(s, tri);
    f3 p0 = mk(T.p0x, T.p0y, T.p0z), p1 = mk(T.p1x, T.p1y, T.p1z), p2 = mk(T.p2x, T.p2y, T.p2z);
    float b0 = 1.0f - hv.y - hv.z;
    f3 p = p0 * b0 + p1 * hv.y + p2 * hv.z;
    const float4* shp = reinterpret_cast<const float4*>(s.shade + T.prim);
    float4 sb = shp[1];
    const float4 sn = shp[2];
    const f3 n_g = mk(sn.x, sn.y, sn.z);
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
      if (CK) e = c;
      else L = RB ? L - c : L + c;
    }
    if (k == R.max_depth) {
      done = true;
    } else {
      uint4 r0 = philox(glo, ghi, (uint32_t)(k - 1), 0u, R.key0, R.key1);
      uint4 r1 = philox(glo, ghi, (uint32_t)(k - 1), 1u, R.key0, R.key1);
      const DMaterial& M = s.mats[mat_id];
      const int type = M.type;
      if (type == DRT_BSDF_NULL || (type == DRT_BSDF_MASK && u01(r1.w) >= M.opacity)) {
        if (type == DRT_BSDF_MASK) prev_pdf = 0.f;
        o = spawn(s, p, n_g, d);
        ++k;
      } else {
        shaded = true;
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
          float u = sa.x * b0 + sa.z * hv.y + sb.x * hv.z;
          float v = sa.y * b0 + sa.w * hv.y + sb.y * hv.z;
          int TW = tab.tw[vtex], TH = tab.th[vtex];
          int tx = (int)fminf(floorf(fmaxf(u, 0.f) * (float)TW), (float)(TW - 1));
          int ty = (int)fminf(floorf(fmaxf(v, 0.f) * (float)TH), (float)(TH - 1));
          vtexel = ty * TW + tx;
          const float* tp = tab.tex[vtex] + 3 * (size_t)vtexel;
          sh.albedo = mk(tp[0], tp[1], tp[2]);
        }
        vrslot = M.rough_slot;
        if (vrslot >= 0) sh.alpha = P.rough[vrslot];
        if (!no_nee && n_em > 0) {
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
              if (DER) {
                nee_gt = dL * coef * fe.dalb;
                f3 gr = dL * coef * fe.dalpha;
                nee_gr = gr.x + gr.y + gr.z;
              }
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
        f3 wo;
        BEval be;
        const bool ok = bsdf_sample<DER>(sh, wi, u01(r1.x), u01(r1.y), u01(r0.w), wo, be);
        if (DER && ok) {
          bsdf_pend = true;
          rat_alb = mk(be.f.x != 0.f ? be.dalb.x / be.f.x : 0.f, be.f.y != 0.f ? be.dalb.y / be.f.y : 0.f,
                       be.f.z != 0.f ? be.dalb.z / be.f.z : 0.f);
          rat_alpha = mk(be.f.x != 0.f ? be.dalpha.x / be.f.x : 0.f,
                         be.f.y != 0.f ? be.dalpha.y / be.f.y : 0.f,
                         be.f.z != 0.f ? be.dalpha.z / be.f.z : 0.f);
        }
        if (ok) {
          beta = beta * be.f * (1.0f / be.pdf);
          prev_pdf = be.pdf;
          prev_p = p;
          f3 wow = to_world(fr, wo);
          o = spawn(s, p, n_g, wow);
          d = wow;
          if (k >= R.rr_depth) {
            float q = fminf(maxc(beta), 0.95f);
            if (u01(r1.z) >= q) done = true;
            else beta = beta * (1.0f / q);
          }
        } else {
          done = true;
        }
        ++k;
      }
    }
  }
  S.no4[g] = f4(o, prev_pdf);
  S.nd4[g] = f4(d, __int_as_float(k));
  S.nb4[g] = f4(beta, __int_as_float(done ? 0 : 1));
  if (CK) S.pe4[g] = f4(e, 0.f);
  else S.L4[g] = f4(L, 0.f);
  S.npp4[g] = f4(prev_p, 0.f);
  if (nee) {
    S.so4[g] = f4(so, stmax);
    S.sc4[g] = f4(nee_c, 0.f);
  }
  S.sd4[g] = f4(sd, __int_as_float(nee ? 1 : 0));
  if (DER) {
    if (shaded) {
      S.pa4[g] = f4(rat_alb, 0.f);
      S.pr4[g] = f4(rat_alpha, 0.f);
      S.pn4[g] = f4(nee_gt, nee_gr);
    }
    S.pv4[g] = make_float4(__int_as_float(shaded ? vtex : -1), __int_as_float(vtexel),
                           __int_as_float(shaded ? vrslot : -1), __int_as_float(bsdf_pend ? 1 : 0));
  }
}

// pending shadow rays: an unoccluded one adds its next-event contribution
__global__ __launch_bounds__(kWfBlock) void k_wf_shadow(DScene s, int64_t n, WState S) {
  __shared__ int stack[kStackDepth * kWfBlock];
  const int64_t g = (int64_t)blockIdx.x * kWfBlock + threadIdx.x;
  if (g >= n) return;
  const float4 sd4 = S.sd4[g];
  if (__float_as_int(sd4.w) == 0) return;
  const float4 so4 = S.so4[g];
  Counters cnt = {};
  Hit h;
  RayPre rp = ray_pre(xyz(so4), xyz(sd4));
  if (!traverse(s, rp, 0.f, so4.w, true, h, stack + threadIdx.x, cnt)) {
    const float4 l = S.L4[g];
    S.L4[g] = f4(xyz(l) + xyz(S.sc4[g]), 0.f);
  }
  S.sd4[g] = make_float4(sd4.x, sd4.y, sd4.z, 0.f);  // resolved (the path may have ended)
}

// replay: the vertex's shadow ray, then its gradient as the megakernel forms
// it -- the next-event term if visible (L_rem loses it first), plus dL L_rem
// (d f/f) for the sampled continuation -- scattered into its texel and
// roughness slot (roughness pre-reduced in LDS per workgroup).
// CK (checkpointed backward): L4 holds A, the radiance of the later
// vertices; the gradient is the next-event term if visible plus dL A (d f/f),
// and then A gains the vertex's emission and visible next-event term.  Every
// path live at this bounce takes part (its emission counts even where the
// vertex has no derivative).
template <bool CK>
__global__ __launch_bounds__(kWfBlock) void k_wf_resolve(DScene s, DParams P, DGrads G, DRender R,
                                                         int64_t n, const float* __restrict__ adj,
                                                         WState S) {
  __shared__ int stack[kStackDepth * kWfBlock];
  __shared__ LdsTables tab;
  __shared__ float rough_acc[kMaxRoughLds];
  const bool lds_rough = G.rough && s.n_rough <= kMaxRoughLds;
  load_tables(tab, s, P, &G);
  if (threadIdx.x < kMaxRoughLds) rough_acc[threadIdx.x] = 0.f;
  __syncthreads();
  const int64_t g = (int64_t)blockIdx.x * kWfBlock + threadIdx.x;
  Counters cnt = {};
  if (g < n) {
    const float4 sd4 = S.sd4[g], pv = S.pv4[g];
    const bool nee = __float_as_int(sd4.w) != 0;
    const int vtex = __float_as_int(pv.x), vtexel = __float_as_int(pv.y), vrslot = __float_as_int(pv.z);
    const bool bsdf_pend = __float_as_int(pv.w) != 0;
    const bool live = CK ? __float_as_int(S.b4[g].w) != 0 : (nee || bsdf_pend);
    if (live) {
      f3 Lrem = xyz(S.L4[g]);  // CK: A
      f3 gtex = mk(0, 0, 0), add = mk(0, 0, 0);
      float grough = 0.f;
      if (nee) {
        const float4 so4 = S.so4[g];
        Hit h;
        RayPre rp = ray_pre(xyz(so4), xyz(sd4));
        if (!traverse(s, rp, 0.f, so4.w, true, h, stack + threadIdx.x, cnt)) {
          if (CK) add = xyz(S.sc4[g]);
          else Lrem = Lrem - xyz(S.sc4[g]);
          const float4 pn = S.pn4[g];
          gtex = xyz(pn);
          grough = pn.w;
        }
      }
      if (bsdf_pend) {
        const f3 dL = path_dL(adj, g, R.spp);
        gtex = gtex + dL * Lrem * xyz(S.pa4[g]);
        f3 gr = dL * Lrem * xyz(S.pr4[g]);
        grough += gr.x + gr.y + gr.z;
      }
      Sink sink{&tab, lds_rough ? rough_acc : nullptr, lds_rough ? nullptr : G.rough};
      if (vtex >= 0) scatter_tex(sink, vtex, vtexel, gtex, cnt, false);
      if (vrslot >= 0) scatter_rough(sink, vrslot, grough, cnt);
      if (CK) Lrem = Lrem + xyz(S.pe4[g]) + add;
      S.L4[g] = f4(Lrem, 0.f);
      S.sd4[g] = make_float4(sd4.x, sd4.y, sd4.z, 0.f);
      S.pv4[g] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  __syncthreads();
  if (lds_rough && threadIdx.x < s.n_rough) {
    const float v = rough_acc[threadIdx.x];
    if (v != 0.f) atomicAdd(G.rough + threadIdx.x, v);
  }
}

// image = mean over each pixel's samples (in sample order, as the megakernel sums)
__global__ __launch_bounds__(256) void k_wf_accumulate(int64_t n_pix, int spp, WState S,
                                                       float* __restrict__ image) {
  const int64_t pix = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (pix >= n_pix) return;
  f3 acc = mk(0, 0, 0);
  for (int j = 0; j < spp; ++j) acc = acc + xyz(S.L4[pix * spp + j]);
  const float inv = 1.0f / (float)spp;
  image[3 * pix] = acc.x * inv;
  image[3 * pix + 1] = acc.y * inv;
  image[3 * pix + 2] = acc.z * inv;
}

int64_t wavefront_workspace_bytes(int64_t n_paths) { return n_paths * kWfArrays * 16; }
int64_t wavefront_adjoint_workspace_bytes(int64_t n_paths) { return n_paths * kWfArraysAdj * 16; }
int64_t checkpoint_workspace_bytes(int64_t n_paths, int max_depth) {
  return n_paths * (kWfArraysCk + kTapeArrays * (int64_t)(max_depth + 1)) * 16;
}

static WState state_in(void* ws, int64_t n, int n_arrays) {
  float4* base = static_cast<float4*>(ws);
  WState S = {};
  float4** arrays[kWfArraysAdj] = {&S.o4, &S.d4, &S.b4, &S.L4, &S.pp4, &S.h4, &S.so4,
                                   &S.sd4, &S.sc4, &S.pa4, &S.pr4, &S.pn4, &S.pv4};
  for (int a = 0; a < n_arrays; ++a) *arrays[a] = base + (size_t)a * n;
  S.no4 = S.o4;
  S.nd4 = S.d4;
  S.nb4 = S.b4;
  S.npp4 = S.pp4;
  return S;
}

// Checkpointed layout: L4 h4 so4 sd4 sc4 pa4 pr4 pn4 pv4 pe4, then the tape,
// slice i = (o4, d4, b4, pp4) of bounce i (i = 0 .. max_depth; the last is
// written by the last bounce and never read).  Bounce i reads slice i and
// writes slice `out`.
static WState state_ck(void* ws, int64_t n, int i, int out) {
  float4* base = static_cast<float4*>(ws);
  WState S = {};
  float4** arrays[kWfArraysCk] = {&S.L4, &S.h4, &S.so4, &S.sd4, &S.sc4,
                                  &S.pa4, &S.pr4, &S.pn4, &S.pv4, &S.pe4};
  for (int a = 0; a < kWfArraysCk; ++a) *arrays[a] = base + (size_t)a * n;
  float4* tape = base + (size_t)kWfArraysCk * n;
  float4* in = tape + (size_t)kTapeArrays * i * n;
  float4* nx = tape + (size_t)kTapeArrays * out * n;
  S.o4 = in;
  S.d4 = in + n;
  S.b4 = in + 2 * n;
  S.pp4 = in + 3 * n;
  S.no4 = nx;
  S.nd4 = nx + n;
  S.nb4 = nx + 2 * n;
  S.npp4 = nx + 3 * n;
  return S;
}

// one full primal pass over all paths (radiance per path in L4)
static void primal_passes(const DScene& s, const DParams& p, const DCams& c, const DRender& r,
                          int64_t n, const float* adj, const WState& S, hipStream_t st) {
  const unsigned blocks = (unsigned)((n + kWfBlock - 1) / kWfBlock);
  if (adj)
    hipLaunchKernelGGL((k_wf_camera<true, false>), dim3(blocks), dim3(kWfBlock), 0, st, c, r, n, adj, S);
  else
    hipLaunchKernelGGL((k_wf_camera<false, false>), dim3(blocks), dim3(kWfBlock), 0, st, c, r, n, adj, S);
  for (int depth = 1; depth <= r.max_depth; ++depth) {
    hipLaunchKernelGGL(k_wf_trace, dim3(blocks), dim3(kWfBlock), 0, st, s, n, S);
    hipLaunchKernelGGL(k_wf_shade<WF_PRIMAL>, dim3(blocks), dim3(kWfBlock), 0, st, s, p, r, n, adj, S);
    hipLaunchKernelGGL(k_wf_shadow, dim3(blocks), dim3(kWfBlock), 0, st, s, n, S);
  }
}

hipError_t launch_render_wavefront(const DScene& s, const DParams& p, const DCams& c,
                                   const DRender& r, void* ws, float* image, hipStream_t st) {
  const int64_t n_pix = (int64_t)c.n * c.width * c.height;
  const int64_t n = n_pix * r.spp;
  const WState S = state_in(ws, n, kWfArrays);
  primal_passes(s, p, c, r, n, nullptr, S, st);
  hipLaunchKernelGGL(k_wf_accumulate, dim3((unsigned)((n_pix + 255) / 256)), dim3(256), 0, st, n_pix,
                     r.spp, S, image);
  return hipGetLastError();
}

hipError_t launch_render_adjoint_wavefront(const DScene& s, const DParams& p, const DCams& c,
                                           const DRender& r, const float* adj, const DGrads& G,
                                           void* ws, hipStream_t st) {
  const int64_t n = (int64_t)c.n * c.width * c.height * r.spp;
  const WState S = state_in(ws, n, kWfArraysAdj);
  const unsigned blocks = (unsigned)((n + kWfBlock - 1) / kWfBlock);
  primal_passes(s, p, c, r, n, adj, S, st);  // pass A: L per path
  hipLaunchKernelGGL((k_wf_camera<true, true>), dim3(blocks), dim3(kWfBlock), 0, st, c, r, n, adj, S);
  for (int depth = 1; depth <= r.max_depth; ++depth) {
    hipLaunchKernelGGL(k_wf_trace, dim3(blocks), dim3(kWfBlock), 0, st, s, n, S);
    hipLaunchKernelGGL(k_wf_shade<WF_REPLAY>, dim3(blocks), dim3(kWfBlock), 0, st, s, p, r, n, adj, S);
    hipLaunchKernelGGL(k_wf_resolve<false>, dim3(blocks), dim3(kWfBlock), 0, st, s, p, G, r, n, adj, S);
  }
  return hipGetLastError();
}

hipError_t launch_render_checkpoint_forward(const DScene& s, const DParams& p, const DCams& c,
                                            const DRender& r, void* ws, float* image,
                                            hipStream_t st) {
  const int64_t n_pix = (int64_t)c.n * c.width * c.height;
  const int64_t n = n_pix * r.spp;
  const unsigned blocks = (unsigned)((n + kWfBlock - 1) / kWfBlock);
  const WState S0 = state_ck(ws, n, 0, 0);
  hipLaunchKernelGGL((k_wf_camera<false, false>), dim3(blocks), dim3(kWfBlock), 0, st, c, r, n,
                     nullptr, S0);
  for (int i = 0; i < r.max_depth; ++i) {
    const WState S = state_ck(ws, n, i, i + 1);
    hipLaunchKernelGGL(k_wf_trace, dim3(blocks), dim3(kWfBlock), 0, st, s, n, S);
    hipLaunchKernelGGL(k_wf_shade<WF_PRIMAL>, dim3(blocks), dim3(kWfBlock), 0, st, s, p, r, n,
                       nullptr, S);
    hipLaunchKernelGGL(k_wf_shadow, dim3(blocks), dim3(kWfBlock), 0, st, s, n, S);
  }
  hipLaunchKernelGGL(k_wf_accumulate, dim3((unsigned)((n_pix + 255) / 256)), dim3(256), 0, st, n_pix,
                     r.spp, S0, image);
  return hipGetLastError();
}

hipError_t launch_render_checkpoint_adjoint(const DScene& s, const DParams& p, const DCams& c,
                                            const DRender& r, const float* adj, const DGrads& G,
                                            void* ws, hipStream_t st) {
  const int64_t n = (int64_t)c.n * c.width * c.height * r.spp;
  const unsigned blocks = (unsigned)((n + kWfBlock - 1) / kWfBlock);
  hipError_t e = launch_zero(state_ck(ws, n, 0, 0).L4, 4 * n, st);  // A = 0 beyond the last vertex
  if (e != hipSuccess) return e;
  for (int i = r.max_depth - 1; i >= 0; --i) {
    // the next-ray outputs of the recomputed bounce go to the unused last slice
    const WState S = state_ck(ws, n, i, r.max_depth);
    hipLaunchKernelGGL(k_wf_trace, dim3(blocks), dim3(kWfBlock), 0, st, s, n, S);
    hipLaunchKernelGGL(k_wf_shade<WF_BACKWARD>, dim3(blocks), dim3(kWfBlock), 0, st, s, p, r, n,
                       adj, S);
    hipLaunchKernelGGL(k_wf_resolve<true>, dim3(blocks), dim3(kWfBlock), 0, st, s, p, G, r, n, adj, S);
  }
  return hipGetLastError();
}

}  // namespace drt
