// Wavefront variant of the primal renderer: the same estimator as the
// megakernel (identical Philox counters, conventions and device functions),
// but every bounce is split into separate kernels that pass the path state
// through HBM -- closest hit, shading, shadow ray -- the execution model the
// paper compares its megakernels against (Sec. "Evaluation": wavefront
// versus megakernel).  One lane per path g = ((cam H + y) W + x) spp + s;
// paths that have ended return at once (no compaction).
//
// Path state (structure of arrays, float4 each, in a caller workspace):
//   o4  = (origin, prev_pdf)        d4  = (direction, k as int bits)
//   b4  = (beta, alive as int bits) L4  = (radiance, unused)
//   pp4 = (prev_p, unused)          h4  = (t, b1, b2, triangle as int bits)
//   so4 = (shadow origin, tmax)     sd4 = (shadow direction, pending flag)
//   sc4 = (next-event contribution, unused)
#include "drt_device.h"

namespace drt {

struct WState {
  float4 *o4, *d4, *b4, *L4, *pp4, *h4, *so4, *sd4, *sc4;
};

constexpr int kWfBlock = 64;    // one wave per workgroup (LDS traversal stack per lane)
constexpr int kWfArrays = 9;

DEV f3 xyz(float4 v) { return mk(v.x, v.y, v.z); }
DEV float4 f4(f3 a, float w) { return make_float4(a.x, a.y, a.z, w); }

// camera rays of all paths
__global__ __launch_bounds__(kWfBlock) void k_wf_camera(DCams C, DRender R, int64_t n, WState S) {
  const int64_t g = (int64_t)blockIdx.x * kWfBlock + threadIdx.x;
  if (g >= n) return;
  const int64_t pix = g / R.spp;
  const int W = C.width, H = C.height;
  const int cam = (int)(pix / ((int64_t)W * H));
  const int y = (int)((pix / W) % H), x = (int)(pix % W);
  f3 o, d;
  camera_ray(C.cam[cam], W, H, x, y, (uint32_t)g, (uint32_t)((uint64_t)g >> 32), R, o, d);
  S.o4[g] = f4(o, 0.f);  // prev_pdf 0: the first emitter hit takes no MIS weight
  S.d4[g] = f4(d, __int_as_float(1));
  S.b4[g] = f4(mk(1, 1, 1), __int_as_float(1));
  S.L4[g] = f4(mk(0, 0, 0), 0.f);
  S.pp4[g] = f4(o, 0.f);
  S.sd4[g] = make_float4(0.f, 0.f, 0.f, 0.f);
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
// left pending) and the BSDF sample with Russian roulette
__global__ __launch_bounds__(kWfBlock) void k_wf_shade(DScene s, DParams P, DRender R, int64_t n,
                                                       WState S) {
  __shared__ LdsTables tab;
  load_tables(tab, s, P, nullptr);
  __syncthreads();
  const int64_t g = (int64_t)blockIdx.x * kWfBlock + threadIdx.x;
  if (g >= n) return;
  float4 b4 = S.b4[g];
  if (__float_as_int(b4.w) == 0) return;
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
  if (tri < 0) {
    if (s.env_emitter >= 0) {
      int row, col;
      float st;
      env_cell(s, d, row, col, st);
      float w = 1.0f;
      if (!(prev_pdf == 0.f || no_nee)) w = power_heuristic(prev_pdf, p_sel * env_pdf(s, row, col, st));
      L = L + beta * env_lookup(s, row, col) * w;
    }
    done = true;
  } else {
    DTri T = load_tri(s, tri);
    f3 p0 = mk(T.p0x, T.p0y, T.p0z), p1 = mk(T.p1x, T.p1y, T.p1z), p2 = mk(T.p2x, T.p2y, T.p2z);
    float b0 = 1.0f - hv.y - hv.z;
    f3 p = p0 * b0 + p1 * hv.y + p2 * hv.z;
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
      L = L + beta * mk(E.radiance[0], E.radiance[1], E.radiance[2]) * w;
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
        Frame fr = make_frame(n_g);
        f3 wi = to_local(fr, -d);
        Shade sh;
        sh.type = type;
        sh.albedo = mk(M.albedo[0], M.albedo[1], M.albedo[2]);
        sh.f0 = mk(M.f0[0], M.f0[1], M.f0[2]);
        sh.alpha = M.alpha;
        sh.eta = M.eta;
        sh.opacity = M.opacity;
        const int vtex = M.texture;
        if (vtex >= 0) {
          float4 sa = shp[0];
          float u = sa.x * b0 + sa.z * hv.y + sb.x * hv.z;
          float v = sa.y * b0 + sa.w * hv.y + sb.y * hv.z;
          int TW = tab.tw[vtex], TH = tab.th[vtex];
          int tx = (int)fminf(floorf(fmaxf(u, 0.f) * (float)TW), (float)(TW - 1));
          int ty = (int)fminf(floorf(fmaxf(v, 0.f) * (float)TH), (float)(TH - 1));
          const float* tp = tab.tex[vtex] + 3 * (size_t)(ty * TW + tx);
          sh.albedo = mk(tp[0], tp[1], tp[2]);
        }
        if (M.rough_slot >= 0) sh.alpha = P.rough[M.rough_slot];
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
            BEval fe = bsdf_eval<false>(sh, wi, to_local(fr, wl));
            if (nonzero(fe.f)) {
              float w = delta ? 1.0f : power_heuristic(p_sel * pdf_l, fe.pdf);
              nee_c = beta * Le * (w / (p_sel * pdf_l)) * fe.f;
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
        if (bsdf_sample<false>(sh, wi, u01(r1.x), u01(r1.y), u01(r0.w), wo, be)) {
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
  S.o4[g] = f4(o, prev_pdf);
  S.d4[g] = f4(d, __int_as_float(k));
  S.b4[g] = f4(beta, __int_as_float(done ? 0 : 1));
  S.L4[g] = f4(L, 0.f);
  S.pp4[g] = f4(prev_p, 0.f);
  if (nee) {
    S.so4[g] = f4(so, stmax);
    S.sc4[g] = f4(nee_c, 0.f);
  }
  S.sd4[g] = f4(sd, __int_as_float(nee ? 1 : 0));
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

hipError_t launch_render_wavefront(const DScene& s, const DParams& p, const DCams& c,
                                   const DRender& r, void* ws, float* image, hipStream_t st) {
  const int64_t n_pix = (int64_t)c.n * c.width * c.height;
  const int64_t n = n_pix * r.spp;
  float4* base = static_cast<float4*>(ws);
  WState S;
  float4** arrays[kWfArrays] = {&S.o4, &S.d4, &S.b4, &S.L4, &S.pp4, &S.h4, &S.so4, &S.sd4, &S.sc4};
  for (int a = 0; a < kWfArrays; ++a) *arrays[a] = base + (size_t)a * n;
  const unsigned blocks = (unsigned)((n + kWfBlock - 1) / kWfBlock);
  hipLaunchKernelGGL(k_wf_camera, dim3(blocks), dim3(kWfBlock), 0, st, c, r, n, S);
  for (int depth = 1; depth <= r.max_depth; ++depth) {
    hipLaunchKernelGGL(k_wf_trace, dim3(blocks), dim3(kWfBlock), 0, st, s, n, S);
    hipLaunchKernelGGL(k_wf_shade, dim3(blocks), dim3(kWfBlock), 0, st, s, p, r, n, S);
    hipLaunchKernelGGL(k_wf_shadow, dim3(blocks), dim3(kWfBlock), 0, st, s, n, S);
  }
  hipLaunchKernelGGL(k_wf_accumulate, dim3((unsigned)((n_pix + 255) / 256)), dim3(256), 0, st, n_pix,
                     r.spp, S, image);
  return hipGetLastError();
}

}  // namespace drt
