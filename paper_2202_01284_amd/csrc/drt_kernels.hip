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
#include <atomic>
#include <mutex>

#include "drt_device.h"

namespace drt {

// ---------------------------------------------------------------------------
// The megakernel body.  A lane owns one pixel and loops over its samples.
// Each iteration of the loop is one vertex for every lane of the wave, in
// two phases that all lanes take together: (A) trace the closest-hit ray and
// do the emission, next-event and BSDF-sampling work of the vertex it finds;
// (B) trace the vertex's shadow ray and resolve the next-event term.  The
// lanes of a wave start each sample together (coherent primary rays); a lane
// whose path ends early waits for the wave (per-lane restart was measured
// slower: it mixes primary and secondary rays in a wave).
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
// MODE_TRAIN_SELF: self-training path g: as MODE_CACHED_SAMPLES (radiance up
// to the record vertex to io.lsamp[g], query there with id g), and every
// scattering vertex k < K before it writes record g (K - 1) + k - 1 of
// io.trec (features, and for now the radiance collected so far in 13..15)
// and its throughput to io.tbeta; io.valid marks the records written.
// Samples g_base .. g_base + n_samples - 1 start at pixel (cam, x, y).
// HC (intersection records): the tracing pass stores each step's closest
// hit and shadow-ray outcome, and the replay reads them back instead of
// tracing the same rays again.  MODE_ADJOINT: pass A writes, the replay of
// the same sample reads, at hrec[(k - 1) kBlock] (reused sample after
// sample); MODE_CACHED_SAMPLES writes and MODE_ADJOINT_CACHED (a later
// launch) reads, at hrec[(sample max_depth + k - 1) kBlock].
// ---------------------------------------------------------------------------
enum {
  MODE_PRIMAL = 0,
  MODE_ADJOINT = 1,
  MODE_CACHED = 2,
  MODE_TRAIN = 3,
  MODE_CACHED_SAMPLES = 4,
  MODE_ADJOINT_CACHED = 5,
  MODE_JVP = 6,
  MODE_TRAIN_SELF = 7
};

template <int MODE, bool HC = false, bool ST = false, bool LS = false>
DEV void render_pixel(const DScene& s, const DParams& P, const DCams& C, const DRender& R,
                      const LdsTables& tab, int cam, int x, int y, uint64_t g_base, int n_samples,
                      f3 dL, int* stk, Counters& cnt, const Sink& sink, const DNrcIO& io,
                      f3& out, int4* hrec = nullptr, RoughAcc* racc_out = nullptr) {
  constexpr bool ADJ = MODE == MODE_ADJOINT || MODE == MODE_ADJOINT_CACHED;
  constexpr bool JVP = MODE == MODE_JVP;
  // the indexed node test except where the scene is read from device memory
  // by the kernels carrying derivatives (held to 128 VGPRs)
  constexpr bool IDX = LS || !(ADJ || JVP);
  // modes with a record vertex (cache queries, training records, cached replay)
  constexpr bool HOOK = MODE == MODE_CACHED || MODE == MODE_TRAIN || MODE == MODE_CACHED_SAMPLES ||
                        MODE == MODE_ADJOINT_CACHED || MODE == MODE_TRAIN_SELF;
  constexpr bool QUERY = MODE == MODE_CACHED || MODE == MODE_CACHED_SAMPLES || MODE == MODE_TRAIN_SELF;
  constexpr bool SELF = MODE == MODE_TRAIN_SELF;
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
  uint32_t self_mask = 0;  // records written by this path (MODE_TRAIN_SELF)
  // The lane's roughness gradient, summed in a register while its slot stays
  // the same and handed to the workgroup's accumulator when the slot changes;
  // after the last sample it is handed to the caller (racc_out), which
  // flushes it for the whole wave at once, or else added per lane: one
  // accumulator update per lane and work unit instead of one per vertex.
  int racc_slot = -1;
  float racc = 0.f;

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
    self_mask = 0;
    cnt.samples++;
  };

  // one vertex for this lane: returns true when the path has ended.  The
  // replay variant (pass B) carries the subtraction and the scatter; the
  // other passes compile without them.
  auto step = [&](auto replay) -> bool {
    constexpr bool RB = ADJ && decltype(replay)::value;
    if constexpr (ST) {
      cnt.lane_steps++;
      cnt.wave_steps += first_active_lane();
    }
    constexpr bool DER = RB || JVP;  // BSDF parameter derivatives needed
    constexpr bool HREAD = HC && ((MODE == MODE_ADJOINT && RB) || MODE == MODE_ADJOINT_CACHED);
    constexpr bool HWRITE = HC && ((MODE == MODE_ADJOINT && !RB) || MODE == MODE_CACHED_SAMPLES);
    const size_t rec_sample = MODE == MODE_ADJOINT ? 0 : (size_t)sidx * R.max_depth;
    int4* rec = (HREAD || HWRITE) ? hrec + (rec_sample + (size_t)(k - 1)) * kBlock : nullptr;
    int rec_tri = -1;
    float rec_b1 = 0.f, rec_b2 = 0.f;
    bool rec_vis = false;
    bool done = false, nee = false;
    f3 nee_c = mk(0, 0, 0), nee_gt = mk(0, 0, 0), nee_t = mk(0, 0, 0), so = o, sd = d;
    float nee_gr = 0.f, stmax = 0.f;
    bool bsdf_pend = false;
    f3 rat_alb = mk(0, 0, 0), rat_alpha = mk(0, 0, 0);
    int vtex = -1, vtexel = 0, vrslot = -1;
    // ---------------- phase A: closest hit and the vertex's work
    {
      Hit h;
      bool hit;
      if constexpr (HREAD) {
        const int4 r = *rec;
        h.tri = r.x;
        h.b1 = __int_as_float(r.y);
        h.b2 = __int_as_float(r.z);
        hit = r.x >= 0;
        rec_vis = r.w != 0;
      } else {
        RayPre rp = ray_pre(o, d);
        cnt.rays++;
        hit = traverse<ST, LS, IDX>(s, rp, 0.f, INFINITY, false, h, stk, cnt);
      }
      if constexpr (HWRITE) {
        rec_tri = hit ? h.tri : -1;
        rec_b1 = h.b1;
        rec_b2 = h.b2;
      }
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
            if constexpr (ST) cnt.wave_shade += first_active_lane();
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
            const bool at_hook = HOOK && !recorded && k >= io.K;
            if (at_hook || (SELF && k < io.K)) {
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
              if (SELF && !at_hook) {
                const size_t r = (size_t)g_base * (io.K - 1) + (k - 1);
                rec = io.trec + (size_t)NRC_REC * r;
                rec[13] = L.x;
                rec[14] = L.y;
                rec[15] = L.z;
                io.tbeta[3 * r] = beta.x;
                io.tbeta[3 * r + 1] = beta.y;
                io.tbeta[3 * r + 2] = beta.z;
                self_mask |= 1u << (k - 1);
              } else if (QUERY) {
                int slot = atomicAdd(io.count, 1);
                if (slot < io.capacity) {
                  rec = io.rec + (size_t)NRC_REC * slot;
                  io.qpix[slot] = MODE == MODE_CACHED ? (int)pix : (int)glo;
                  if (io.qbin) io.qbin[slot] = query_key(p.x, p.y, p.z, io.lo, io.inv_ext);
                  if (io.qref) {
                    const bool tex_in = vtex >= 0 && type != DRT_BSDF_CONDUCTOR &&
                                        type != DRT_BSDF_DIELECTRIC;
                    query_ref_put(io.qref + 2 * (size_t)slot, tex_in ? vtexel : -1, vtex,
                                  ggx ? vrslot : -1);
                  }
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
              if (MODE != MODE_TRAIN && at_hook) {
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
      bool vis;
      if constexpr (HREAD) {
        vis = rec_vis;
      } else {
        RayPre rp = ray_pre(so, sd);
        Hit h;
        cnt.shadow++;
        vis = !traverse<ST, LS, IDX>(s, rp, 0.f, stmax, true, h, stk, cnt);
      }
      if constexpr (HWRITE) rec_vis = vis;
      if (vis) {
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
      if (vtex >= 0) scatter_tex(sink, vtex, vtexel, gtex, cnt, R.stats != nullptr);
      if (vrslot >= 0 && grough != 0.f) {
        if (vrslot != racc_slot) {
          if (racc_slot >= 0) scatter_rough(sink, racc_slot, racc, cnt);
          racc_slot = vrslot;
          racc = 0.f;
        }
        racc += grough;
      }
    }
    if constexpr (HWRITE)
      *rec = make_int4(rec_tri, __float_as_int(rec_b1), __float_as_int(rec_b2), rec_vis ? 1 : 0);
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
      // replay residual relative to the sample's radiance (max norms; a
      // path that collected nothing must end at exactly zero)
      const float rmax = fmaxf(fabsf(Lrem.x), fmaxf(fabsf(Lrem.y), fabsf(Lrem.z)));
      const float lmax = fmaxf(fabsf(L.x), fmaxf(fabsf(L.y), fabsf(L.z)));
      cnt.lrem_max = fmaxf(cnt.lrem_max, lmax > 0.f ? rmax / lmax : rmax);
    } else if (JVP) {
      acc = acc + tL;
    } else if (MODE == MODE_CACHED_SAMPLES || SELF) {
      float* ls = io.lsamp + 3 * (g_base + (uint64_t)sidx);
      ls[0] = L.x;
      ls[1] = L.y;
      ls[2] = L.z;
      if (SELF) {
        int* v = io.valid + (size_t)g_base * (io.K - 1);
        for (int i = 0; i < io.K - 1; ++i) v[i] = (self_mask >> i) & 1u;
        if (self_mask) atomicAdd(io.rcount, __popc(self_mask));
      }
    } else {
      acc = acc + L;
    }
    if (++sidx == n_samples) break;
  }
  if (ADJ && racc_slot >= 0) {
    if (racc_out) {
      racc_out->slot = racc_slot;
      racc_out->v = racc;
    } else {
      scatter_rough(sink, racc_slot, racc, cnt);
    }
  }
  out = acc;
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
  atomicAdd((unsigned long long*)&R.stats[DRT_STAT_TEX_LANES], (unsigned long long)c.tex_lanes);
  atomicAdd((unsigned long long*)&R.stats[DRT_STAT_TEX_KEYS], (unsigned long long)c.tex_keys);
  atomicAdd((unsigned long long*)&R.stats[DRT_STAT_WAVE_NODES], (unsigned long long)c.wave_nodes);
  atomicAdd((unsigned long long*)&R.stats[DRT_STAT_WAVE_TRIS], (unsigned long long)c.wave_tris);
  atomicAdd((unsigned long long*)&R.stats[DRT_STAT_LANE_STEPS], (unsigned long long)c.lane_steps);
  atomicAdd((unsigned long long*)&R.stats[DRT_STAT_WAVE_STEPS], (unsigned long long)c.wave_steps);
  atomicAdd((unsigned long long*)&R.stats[DRT_STAT_WAVE_SHADE], (unsigned long long)c.wave_shade);
  atomicMax((unsigned long long*)&R.stats[DRT_STAT_LREM_MAX],
            (unsigned long long)__float_as_uint(c.lrem_max));
}

// The scene as a megakernel reads it.  LS: the tree, the triangles, their
// shading records, the materials and the emitters from the workgroup's LDS
// copy, filled here (the caller synchronizes before the first read); the
// host sets s.lds_scene only where they fit kLdsSceneBytes and the tree
// needs at most kStackDepthSmall stack entries.
DEV void lds_fill(float4* dst, const void* src, int n) {
  const float4* s4 = reinterpret_cast<const float4*>(src);
  for (int i = threadIdx.x; i < n; i += kBlock) dst[i] = s4[i];
}
template <bool LS>
DEV DScene scene_view(const DScene& s, float4* lds) {
  if constexpr (!LS) {
    return s;
  } else {
    // float4 per node / triangle / shading record / material / emitter: 8 / 3 / 3 / 4 / 6
    const int nn = 8 * s.n_nodes, nt = 3 * s.n_tris, ns = 3 * s.n_tris, nm = 4 * s.n_mats;
    const int ne = 6 * s.n_ems;
    float4* p = lds;
    lds_fill(p, s.nodes, nn);
    lds_fill(p + nn, s.tris, nt);
    lds_fill(p + nn + nt, s.shade, ns);
    lds_fill(p + nn + nt + ns, s.mats, nm);
    lds_fill(p + nn + nt + ns + nm, s.ems, ne);
    DScene v = s;
    v.nodes = reinterpret_cast<const DNode*>(p);
    v.tris = reinterpret_cast<const DTri*>(p + nn);
    v.shade = reinterpret_cast<const DShade*>(p + nn + nt);
    v.mats = reinterpret_cast<const DMaterial*>(p + nn + nt + ns);
    v.ems = reinterpret_cast<const DEmitter*>(p + nn + nt + ns + nm);
    return v;
  }
}

// ---------------------------------------------------------------------------
// megakernels: one 8x8 pixel tile per workgroup (one wave)
// ---------------------------------------------------------------------------
// STATS = false compiles the counters out (they are never read).
// MODE: MODE_PRIMAL, MODE_CACHED (paths stop at their record vertex and
// append cache queries) or MODE_CACHED_SAMPLES (per-sample radiance, no image;
// with HC also the intersection records of every sample).
template <bool STATS, int MODE, bool HC = false, bool LS = false>
__global__ __launch_bounds__(kBlock) void k_render_forward(DScene s, DParams P, DCams C, DRender R,
                                                           float* __restrict__ image, DNrcIO io) {
  __shared__ int stack[(LS ? kStackDepthSmall : kStackDepth) * kBlock];
  __shared__ LdsTables tab;
  __shared__ float4 lds_scene[LS ? kLdsSceneBytes / 16 : 1];
  load_tables(tab, s, P, nullptr);
  const DScene sv = scene_view<LS>(s, lds_scene);
  __syncthreads();
  const int W = C.width, H = C.height;
  const int x = blockIdx.x * kTile + (threadIdx.x % kTile);
  const int y = blockIdx.y * kTile + (threadIdx.x / kTile);
  // MODE_PRIMAL and MODE_CACHED may split a tile's samples over two
  // workgroups (blockIdx.z = camera x 2 + half), which then add their halves
  // onto a zeroed image:
  // two addends onto zero give the same sum in either order, so the image
  // stays deterministic
  const int split = (int)gridDim.z / C.n;
  const int cam = blockIdx.z / split, part = blockIdx.z % split;
  const int s0 = part * R.spp / split, s1 = (part + 1) * R.spp / split;
  Counters cnt = {};
  if (x < W && y < H && s1 > s0) {
    Sink none{&tab, nullptr, nullptr};
    f3 acc;
    const uint64_t pix = ((uint64_t)cam * H + y) * W + x;
    int4* hrec = nullptr;
    if (HC) {
      const size_t wg = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
      hrec = R.hits + wg * R.spp * R.max_depth * kBlock + threadIdx.x;
    }
    render_pixel<MODE, HC, STATS, LS>(sv, P, C, R, tab, cam, x, y, pix * (uint64_t)R.spp + s0, s1 - s0,
                                  mk(0, 0, 0), stack + threadIdx.x, cnt, none, io, acc, hrec);
    if (MODE != MODE_CACHED_SAMPLES) {
      const float inv = 1.0f / (float)R.spp;
      float* out = image + 3 * (((size_t)cam * H + y) * W + x);
      if (split == 1) {
        out[0] = acc.x * inv;
        out[1] = acc.y * inv;
        out[2] = acc.z * inv;
      } else {
        atomicAdd(out, acc.x * inv);
        atomicAdd(out + 1, acc.y * inv);
        atomicAdd(out + 2, acc.z * inv);
      }
    }
  }
  if constexpr (STATS) flush_counters(R, cnt);
}

// Held to 128 VGPRs (4 waves per SIMD): measured faster than 3 waves at 131.
// MODE: MODE_ADJOINT (both passes) or MODE_ADJOINT_CACHED (replay from the
// per-sample cached estimates in io.lsamp).  HC: the replay reads pass A's
// intersection records from R.hits (this workgroup's slice).
// Work units: (8x8 tile, sample range) -- a tile's samples split into
// adjoint_split(spp) ranges.  MODE_ADJOINT with records runs persistent
// workgroups (as many as are resident at once) that take the units from the
// counter R.items until none is left, each with one record slot; otherwise
// the grid has one workgroup per unit (blockIdx.z = camera x split + part).
template <bool STATS, int MODE, bool HC = false, bool LS = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_render_adjoint(DScene s, DParams P, DCams C, DRender R,
                                                           const float* __restrict__ adj,
                                                           DGrads G, DNrcIO io) {
  __shared__ int stack[(LS ? kStackDepthSmall : kStackDepth) * kBlock];
  __shared__ LdsTables tab;
  __shared__ float rough_acc[kMaxRoughLds];
  __shared__ float4 lds_scene[LS ? kLdsSceneBytes / 16 : 1];
  const bool lds_rough = G.rough && s.n_rough <= kMaxRoughLds;
  load_tables(tab, s, P, &G);
  if (threadIdx.x < kMaxRoughLds) rough_acc[threadIdx.x] = 0.f;
  const DScene sv = scene_view<LS>(s, lds_scene);
  __syncthreads();
  constexpr bool PERSIST = HC && MODE == MODE_ADJOINT;
  __shared__ uint32_t unit_s;
  const int W = C.width, H = C.height;
  const int tiles_x = tiles_of(W), tiles_y = tiles_of(H);
  const int split = PERSIST ? adjoint_split(R.spp) : (int)gridDim.z / C.n;
  const int64_t units = PERSIST ? (int64_t)tiles_x * tiles_y * C.n * split : 1;  // < 2^31 (host)
  Counters cnt = {};
  const Sink sink{&tab, lds_rough ? rough_acc : nullptr, lds_rough ? nullptr : G.rough};
  for (int round = 0;; ++round) {
    int bx, by, cam, part;
    if constexpr (PERSIST) {
      if (threadIdx.x == 0) unit_s = atomicAdd(R.items, 1u);
      __syncthreads();
      const int64_t unit = unit_s;
      __syncthreads();
      if (unit >= units) break;  // the counter only grows: every wave leaves
      const int tile = (int)(unit / split);
      part = (int)(unit % split);
      bx = tile % tiles_x;
      by = (tile / tiles_x) % tiles_y;
      cam = tile / (tiles_x * tiles_y);
    } else {
      if (round > 0) break;
      bx = blockIdx.x;
      by = blockIdx.y;
      cam = blockIdx.z / split;
      part = blockIdx.z % split;
    }
    const int x = bx * kTile + (threadIdx.x % kTile);
    const int y = by * kTile + (threadIdx.x / kTile);
    const int s0 = part * R.spp / split, s1 = (part + 1) * R.spp / split;
    RoughAcc racc{-1, 0.f};
    if (x < W && y < H && s1 > s0) {
      const size_t pix = ((size_t)cam * H + y) * W + x;
      const float inv = 1.0f / (float)R.spp;
      f3 dL = mk(adj[3 * pix] * inv, adj[3 * pix + 1] * inv, adj[3 * pix + 2] * inv);
      if (nonzero(dL)) {
        f3 unused;
        int4* hrec = nullptr;
        if (PERSIST) {
          // one sample's records at a time, in this workgroup's slot
          hrec = R.hits + (size_t)blockIdx.x * R.max_depth * kBlock + threadIdx.x;
        } else if (HC) {
          // MODE_ADJOINT_CACHED: every sample's records, per tile
          const size_t wg = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
          hrec = R.hits + wg * R.spp * R.max_depth * kBlock + threadIdx.x;
        }
        render_pixel<MODE, HC, STATS, LS>(sv, P, C, R, tab, cam, x, y, pix * (uint64_t)R.spp + s0,
                                      s1 - s0, dL, stack + threadIdx.x, cnt, sink, io, unused, hrec,
                                      &racc);
      }
    }
    // all 64 lanes again (the unit is the workgroup's): the lanes' roughness
    // sums, reduced across the wave per slot
    wave_scatter_rough(sink, racc, cnt);
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
// As the primal: LS reads the scene from the workgroup's LDS copy, and a
// tile's samples may be split over two workgroups adding onto a zeroed image
// (blockIdx.z = camera x split + part).  Held to 128 VGPRs (4 waves per
// SIMD): 4.20 -> 3.93 ms against 3 waves at 130 on 1024^2, 16 spp.
template <bool LS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_render_jvp(
    DScene s, DParams P, DCams C, DRender R, DGrads T, float* __restrict__ image) {
  __shared__ int stack[(LS ? kStackDepthSmall : kStackDepth) * kBlock];
  __shared__ LdsTables tab;
  __shared__ float4 lds_scene[LS ? kLdsSceneBytes / 16 : 1];
  load_tables(tab, s, P, &T);
  const DScene sv = scene_view<LS>(s, lds_scene);
  __syncthreads();
  const int W = C.width, H = C.height;
  const int x = blockIdx.x * kTile + (threadIdx.x % kTile);
  const int y = blockIdx.y * kTile + (threadIdx.x / kTile);
  const int split = (int)gridDim.z / C.n;
  const int cam = blockIdx.z / split, part = blockIdx.z % split;
  const int s0 = part * R.spp / split, s1 = (part + 1) * R.spp / split;
  Counters cnt = {};
  if (x < W && y < H && s1 > s0) {
    Sink dir{&tab, nullptr, T.rough};
    DNrcIO none = {};
    f3 acc;
    const uint64_t pix = ((uint64_t)cam * H + y) * W + x;
    render_pixel<MODE_JVP, false, false, LS>(sv, P, C, R, tab, cam, x, y, pix * (uint64_t)R.spp + s0,
                                             s1 - s0, mk(0, 0, 0), stack + threadIdx.x, cnt, dir,
                                             none, acc);
    const float inv = 1.0f / (float)R.spp;
    float* out = image + 3 * pix;
    if (split == 1) {
      out[0] = acc.x * inv;
      out[1] = acc.y * inv;
      out[2] = acc.z * inv;
    } else {
      atomicAdd(out, acc.x * inv);
      atomicAdd(out + 1, acc.y * inv);
      atomicAdd(out + 2, acc.z * inv);
    }
  }
}

// Training paths of the radiance cache: path j (counter g = j) starts at the
// pixel chosen by the first word of its camera block dim 2, and writes record
// j (features, target) and valid[j].  LS: the scene read from the
// workgroup's LDS copy, as in the megakernels.
template <bool LS>
__global__ __launch_bounds__(kBlock) void k_nrc_records(DScene s, DParams P, DCams C, DRender R,
                                                        int64_t n_paths, DNrcIO io) {
  __shared__ int stack[(LS ? kStackDepthSmall : kStackDepth) * kBlock];
  __shared__ LdsTables tab;
  __shared__ float4 lds_scene[LS ? kLdsSceneBytes / 16 : 1];
  load_tables(tab, s, P, nullptr);
  const DScene sv = scene_view<LS>(s, lds_scene);
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
  render_pixel<MODE_TRAIN, false, false, LS>(sv, P, C, R, tab, cam, x, y, (uint64_t)j, 1, mk(0, 0, 0),
                           stack + threadIdx.x, cnt, none, io, unused);
}

// Self-training paths: path j as in k_nrc_records, written by
// render_pixel<MODE_TRAIN_SELF>.
template <bool LS>
__global__ __launch_bounds__(kBlock) void k_nrc_records_self(DScene s, DParams P, DCams C, DRender R,
                                                             int64_t n_paths, DNrcIO io) {
  __shared__ int stack[(LS ? kStackDepthSmall : kStackDepth) * kBlock];
  __shared__ LdsTables tab;
  __shared__ float4 lds_scene[LS ? kLdsSceneBytes / 16 : 1];
  load_tables(tab, s, P, nullptr);
  const DScene sv = scene_view<LS>(s, lds_scene);
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
  render_pixel<MODE_TRAIN_SELF, false, false, LS>(sv, P, C, R, tab, cam, x, y, (uint64_t)j, 1, mk(0, 0, 0),
                                stack + threadIdx.x, cnt, none, io, unused);
}

// Targets of the self-training records: (path estimate - radiance before the
// record's scattering) / throughput, per channel (0 where beta is 0); the path
// estimate in io.lsamp already holds the cache's answer at the path's end.
__global__ __launch_bounds__(256) void k_nrc_self_targets(DNrcIO io, int64_t n_paths) {
  const int R = io.K - 1;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n_paths * R) return;
  float* rec = io.trec + (size_t)NRC_REC * i;
  if (!io.valid[i]) {
    for (int c = 0; c < NRC_REC; ++c) rec[c] = 0.f;
    return;
  }
  const float* L = io.lsamp + 3 * (size_t)(i / R);
  const float* b = io.tbeta + 3 * (size_t)i;
  for (int c = 0; c < 3; ++c) rec[13 + c] = b[c] != 0.f ? (L[c] - rec[13 + c]) / b[c] : 0.f;
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

// Float32 sums carried as unevaluated pairs (hi, lo) with |lo| <= ulp(hi)/2:
// error-free transformations (Knuth's two-sum, the fma product error) keep
// the rounding errors, so a sum of a few million squares keeps ~2^-44 of
// relative accuracy without double precision.
struct F2 {
  float hi, lo;
};
DEV F2 two_sum(float a, float b) {
  const float s = a + b;
  const float bb = s - a;
  const float e = (a - (s - bb)) + (b - bb);
  return F2{s, e};
}
DEV F2 f2_add(F2 a, F2 b) {
  const F2 s = two_sum(a.hi, b.hi);
  const float lo = s.lo + (a.lo + b.lo);
  const float hi = s.hi + lo;  // renormalise (fast two-sum: |s.hi| >= |lo|)
  return F2{hi, lo - (hi - s.hi)};
}
DEV F2 f2_add_square(F2 acc, float r) {
  const float p = __fmul_rn(r, r);
  const float pe = __builtin_fmaf(r, r, -p);  // r r - p, exactly
  return f2_add(acc, F2{p, pe});
}
DEV void f2_block_reduce(F2& v, F2* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = f2_add(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  v = red[0];
}

// partial[2 b], partial[2 b + 1] = (hi, lo) of block b's sum of squares.
__global__ __launch_bounds__(256) void k_loss_partial(const float* __restrict__ img,
                                                      const float* __restrict__ tgt, int64_t n,
                                                      float adj_scale, float* __restrict__ adj,
                                                      float* __restrict__ partial) {
  __shared__ F2 red[256];
  F2 acc{0.f, 0.f};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float r = img[i] - tgt[i];
    acc = f2_add_square(acc, r);
    if (adj) adj[i] = r * adj_scale;
  }
  f2_block_reduce(acc, red);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = acc.hi;
    partial[2 * blockIdx.x + 1] = acc.lo;
  }
}

// loss = (sum of the partial pairs) / n; inv_n = 1/n rounded to float.
__global__ __launch_bounds__(256) void k_loss_final(const float* __restrict__ partial, int nb,
                                                    float inv_n, float* __restrict__ loss) {
  __shared__ F2 red[256];
  F2 acc{0.f, 0.f};
  for (int i = threadIdx.x; i < nb; i += 256) acc = f2_add(acc, F2{partial[2 * i], partial[2 * i + 1]});
  f2_block_reduce(acc, red);
  if (threadIdx.x == 0) {
    // (hi + lo) / n with the pair's two roundings kept apart
    const float q = acc.hi * inv_n;
    loss[0] = __builtin_fmaf(acc.lo, inv_n, q);
  }
}

struct AdamArgs {
  float lr, b1, b2, eps, c1, c2, lo, hi;
};
// one parameter: moments updated in place, the new (clamped) value returned
DEV float adam1(const AdamArgs& a, float pi, float gi, float& mi, float& vi) {
  mi = a.b1 * mi + (1.0f - a.b1) * gi;
  vi = a.b2 * vi + (1.0f - a.b2) * gi * gi;
  const float x = pi - a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
  return fminf(fmaxf(x, a.lo), a.hi);
}

// Scalar form: parameters [i0, n) (the vector form's tail, or all of them
// when the arrays are not 16-byte aligned).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              int64_t i0, int64_t n, AdamArgs a, int zero,
                                              uint16_t* __restrict__ half_out) {
  int64_t i = i0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * 256;
  for (; i < n; i += stride) {
    float gi = g[i], mi = m[i], vi = v[i];
    if (zero) g[i] = 0.f;
    const float x = adam1(a, p[i], gi, mi, vi);
    m[i] = mi;
    v[i] = vi;
    p[i] = x;
    if (half_out) half_out[i] = __half_as_ushort(__float2half_rn(x));
  }
}

// Every stream of the vector form is touched once per step and is far larger
// than the caches: non-temporal loads and stores keep it from displacing
// other lines (measured 0.31 -> 0.25-0.28 ms on a 4096^2x3 texture).
typedef float nt_f4 __attribute__((ext_vector_type(4)));
DEV float4 load_nt(const float4* q) {
  const nt_f4 t = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(q));
  return make_float4(t.x, t.y, t.z, t.w);
}
DEV void store_nt(float4 x, float4* q) {
  const nt_f4 t = {x.x, x.y, x.z, x.w};
  __builtin_nontemporal_store(t, reinterpret_cast<nt_f4*>(q));
}

// Vector form: four parameters per thread and iteration (16-byte loads and
// stores), parameters [0, 4 n4).
__global__ __launch_bounds__(256) void k_adam4(float4* __restrict__ p, float4* __restrict__ g,
                                               float4* __restrict__ m, float4* __restrict__ v,
                                               int64_t n4, AdamArgs a, int zero,
                                               uint2* __restrict__ half_out) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * 256;
  for (; i < n4; i += stride) {
    const float4 gi = load_nt(g + i), pi = load_nt(p + i);
    float4 mi = load_nt(m + i), vi = load_nt(v + i);
    if (zero) store_nt(make_float4(0.f, 0.f, 0.f, 0.f), g + i);
    float4 x;
    x.x = adam1(a, pi.x, gi.x, mi.x, vi.x);
    x.y = adam1(a, pi.y, gi.y, mi.y, vi.y);
    x.z = adam1(a, pi.z, gi.z, mi.z, vi.z);
    x.w = adam1(a, pi.w, gi.w, mi.w, vi.w);
    store_nt(mi, m + i);
    store_nt(vi, v + i);
    store_nt(x, p + i);
    if (half_out) {
      const uint32_t lo = __half_as_ushort(__float2half_rn(x.x)) |
                          ((uint32_t)__half_as_ushort(__float2half_rn(x.y)) << 16);
      const uint32_t hi = __half_as_ushort(__float2half_rn(x.z)) |
                          ((uint32_t)__half_as_ushort(__float2half_rn(x.w)) << 16);
      half_out[i] = make_uint2(lo, hi);
    }
  }
}

// ---------------------------------------------------------------------------
// launchers

// ---------------------------------------------------------------------------
// The megakernels read the tree and triangles from a per-workgroup LDS copy
// where the scene fits (not for the counting runs, nor when the caller asks
// for device-memory reads).
static bool use_lds_scene(const DScene& s, const DRender& r) {
  return s.lds_scene && !r.stats && !(r.flags & DRT_FLAG_GLOBAL_SCENE);
}

hipError_t launch_render_forward(const DScene& s, const DParams& p, const DCams& c,
                                 const DRender& r, float* image, hipStream_t st) {
  // two workgroups per tile (sample halves) adding onto a zeroed image
  const int split = r.spp >= 2 ? 2 : 1;
  if (split > 1) {
    hipError_t e = launch_zero(image, 3 * (int64_t)c.n * c.width * c.height, st);
    if (e != hipSuccess) return e;
  }
  dim3 grid(tiles_of(c.width), tiles_of(c.height), c.n * split);
  DNrcIO none = {};
  if (r.stats)
    hipLaunchKernelGGL((k_render_forward<true, MODE_PRIMAL>), grid, dim3(kBlock), 0, st, s, p, c,
                       r, image, none);
  else if (use_lds_scene(s, r))
    hipLaunchKernelGGL((k_render_forward<false, MODE_PRIMAL, false, true>), grid, dim3(kBlock), 0, st,
                       s, p, c, r, image, none);
  else
    hipLaunchKernelGGL((k_render_forward<false, MODE_PRIMAL>), grid, dim3(kBlock), 0, st, s, p,
                       c, r, image, none);
  return hipGetLastError();
}

hipError_t launch_render_cached(const DScene& s, const DParams& p, const DCams& c,
                                const DRender& r, float* image, const DNrcIO& io,
                                hipStream_t st) {
  dim3 grid(tiles_of(c.width), tiles_of(c.height), c.n);
  const bool ls = use_lds_scene(s, r);
  if (io.lsamp && r.hits && ls)
    hipLaunchKernelGGL((k_render_forward<false, MODE_CACHED_SAMPLES, true, true>), grid, dim3(kBlock),
                       0, st, s, p, c, r, image, io);
  else if (io.lsamp && r.hits)
    hipLaunchKernelGGL((k_render_forward<false, MODE_CACHED_SAMPLES, true>), grid, dim3(kBlock), 0,
                       st, s, p, c, r, image, io);
  else if (io.lsamp && ls)
    hipLaunchKernelGGL((k_render_forward<false, MODE_CACHED_SAMPLES, false, true>), grid, dim3(kBlock),
                       0, st, s, p, c, r, image, io);
  else if (io.lsamp)
    hipLaunchKernelGGL((k_render_forward<false, MODE_CACHED_SAMPLES>), grid, dim3(kBlock), 0, st,
                       s, p, c, r, image, io);
  else {
    // the plain cached render splits a tile's samples over two workgroups as
    // the primal does (halves added onto a zeroed image; the queries take
    // their slots atomically either way): 22.4 -> 21.9 ms at 1024^2, 64 spp
    const int split = r.spp >= 2 ? 2 : 1;
    if (split > 1) {
      hipError_t e = launch_zero(image, 3 * (int64_t)c.n * c.width * c.height, st);
      if (e != hipSuccess) return e;
    }
    dim3 g2(tiles_of(c.width), tiles_of(c.height), c.n * split);
    if (ls)
      hipLaunchKernelGGL((k_render_forward<false, MODE_CACHED, false, true>), g2, dim3(kBlock), 0, st,
                         s, p, c, r, image, io);
    else
      hipLaunchKernelGGL((k_render_forward<false, MODE_CACHED>), g2, dim3(kBlock), 0, st, s, p,
                         c, r, image, io);
  }
  return hipGetLastError();
}

hipError_t launch_nrc_records(const DScene& s, const DParams& p, const DCams& c, const DRender& r,
                              int64_t n_paths, const DNrcIO& io, hipStream_t st) {
  int64_t blocks = (n_paths + kBlock - 1) / kBlock;
  if (use_lds_scene(s, r))
    hipLaunchKernelGGL((k_nrc_records<true>), dim3((unsigned)blocks), dim3(kBlock), 0, st, s, p, c,
                       r, n_paths, io);
  else
    hipLaunchKernelGGL((k_nrc_records<false>), dim3((unsigned)blocks), dim3(kBlock), 0, st, s, p, c,
                       r, n_paths, io);
  return hipGetLastError();
}

hipError_t launch_nrc_records_self(const DScene& s, const DParams& p, const DCams& c,
                                   const DRender& r, int64_t n_paths, const DNrcIO& io,
                                   hipStream_t st) {
  int64_t blocks = (n_paths + kBlock - 1) / kBlock;
  if (use_lds_scene(s, r))
    hipLaunchKernelGGL((k_nrc_records_self<true>), dim3((unsigned)blocks), dim3(kBlock), 0, st, s, p,
                       c, r, n_paths, io);
  else
    hipLaunchKernelGGL((k_nrc_records_self<false>), dim3((unsigned)blocks), dim3(kBlock), 0, st, s,
                       p, c, r, n_paths, io);
  return hipGetLastError();
}

hipError_t launch_nrc_self_targets(const DNrcIO& io, int64_t n_paths, hipStream_t st) {
  const int64_t n = n_paths * (io.K - 1);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_nrc_self_targets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, io,
                     n_paths);
  return hipGetLastError();
}

hipError_t launch_render_adjoint(const DScene& s, const DParams& p, const DCams& c,
                                 const DRender& r, const float* adj, const DGrads& g,
                                 hipStream_t st) {
  dim3 grid(tiles_of(c.width), tiles_of(c.height),
            c.n * adjoint_split(r.spp));
  DNrcIO none = {};
  if (r.hits) {
    // persistent workgroups, one record slot each; the host sized the slots
    // for this many
    const int64_t units = (int64_t)grid.x * grid.y * grid.z;
    const int resident = adjoint_resident_groups();
    const unsigned groups = (unsigned)(resident > 0 && resident < units ? resident : units);
    hipError_t e = launch_zero(r.items, 1, st);
    if (e != hipSuccess) return e;
    if (r.stats)
      hipLaunchKernelGGL((k_render_adjoint<true, MODE_ADJOINT, true>), dim3(groups), dim3(kBlock), 0,
                         st, s, p, c, r, adj, g, none);
    else if (use_lds_scene(s, r))
      hipLaunchKernelGGL((k_render_adjoint<false, MODE_ADJOINT, true, true>), dim3(groups),
                         dim3(kBlock), 0, st, s, p, c, r, adj, g, none);
    else
      hipLaunchKernelGGL((k_render_adjoint<false, MODE_ADJOINT, true>), dim3(groups), dim3(kBlock), 0,
                         st, s, p, c, r, adj, g, none);
  } else if (r.stats) {
    hipLaunchKernelGGL((k_render_adjoint<true, MODE_ADJOINT>), grid, dim3(kBlock), 0, st, s, p,
                       c, r, adj, g, none);
  } else if (use_lds_scene(s, r)) {
    hipLaunchKernelGGL((k_render_adjoint<false, MODE_ADJOINT, false, true>), grid, dim3(kBlock), 0, st,
                       s, p, c, r, adj, g, none);
  } else {
    hipLaunchKernelGGL((k_render_adjoint<false, MODE_ADJOINT>), grid, dim3(kBlock), 0, st, s, p,
                       c, r, adj, g, none);
  }
  return hipGetLastError();
}

int adjoint_resident_groups() {
  // per device, queried once (host threads may race to fill it; they store
  // the same value): compute units x workgroups of the kernel that fit on one
  // at a time
  static std::atomic<int> cached[kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 0;
  const int known = cached[dev].load(std::memory_order_relaxed);
  if (known > 0) return known;
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(&k_render_adjoint<false, MODE_ADJOINT, true>),
          kBlock, 0) != hipSuccess)
    return 0;
  if (cus <= 0 || per_cu <= 0) return 0;
  cached[dev].store(cus * per_cu, std::memory_order_relaxed);
  return cus * per_cu;
}

hipError_t launch_render_adjoint_cached(const DScene& s, const DParams& p, const DCams& c,
                                        const DRender& r, const float* adj, const DGrads& g,
                                        const DNrcIO& io, hipStream_t st) {
  dim3 grid(tiles_of(c.width), tiles_of(c.height), c.n);
  const bool ls = use_lds_scene(s, r);
  if (r.hits && r.stats)
    hipLaunchKernelGGL((k_render_adjoint<true, MODE_ADJOINT_CACHED, true>), grid, dim3(kBlock), 0,
                       st, s, p, c, r, adj, g, io);
  else if (r.hits && ls)
    hipLaunchKernelGGL((k_render_adjoint<false, MODE_ADJOINT_CACHED, true, true>), grid, dim3(kBlock),
                       0, st, s, p, c, r, adj, g, io);
  else if (r.hits)
    hipLaunchKernelGGL((k_render_adjoint<false, MODE_ADJOINT_CACHED, true>), grid, dim3(kBlock), 0,
                       st, s, p, c, r, adj, g, io);
  else if (ls)
    hipLaunchKernelGGL((k_render_adjoint<false, MODE_ADJOINT_CACHED, false, true>), grid, dim3(kBlock),
                       0, st, s, p, c, r, adj, g, io);
  else if (r.stats)
    hipLaunchKernelGGL((k_render_adjoint<true, MODE_ADJOINT_CACHED>), grid, dim3(kBlock), 0, st,
                       s, p, c, r, adj, g, io);
  else
    hipLaunchKernelGGL((k_render_adjoint<false, MODE_ADJOINT_CACHED>), grid, dim3(kBlock), 0, st,
                       s, p, c, r, adj, g, io);
  return hipGetLastError();
}

hipError_t launch_render_jvp(const DScene& s, const DParams& p, const DCams& c, const DRender& r,
                             const DGrads& t, float* image, hipStream_t st) {
  const int split = r.spp >= 2 ? 2 : 1;
  if (split > 1) {
    hipError_t e = launch_zero(image, 3 * (int64_t)c.n * c.width * c.height, st);
    if (e != hipSuccess) return e;
  }
  dim3 grid(tiles_of(c.width), tiles_of(c.height), c.n * split);
  if (use_lds_scene(s, r))
    hipLaunchKernelGGL((k_render_jvp<true>), grid, dim3(kBlock), 0, st, s, p, c, r, t, image);
  else
    hipLaunchKernelGGL((k_render_jvp<false>), grid, dim3(kBlock), 0, st, s, p, c, r, t, image);
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
  // the two scale factors are rounded to float once, here on the host
  const float adj_scale = (float)(2.0 / (double)n), inv_n = (float)(1.0 / (double)n);
  hipLaunchKernelGGL(k_loss_partial, dim3((unsigned)nb), dim3(256), 0, st, img, tgt, n, adj_scale,
                     adj, ws);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, ws, (int)nb, inv_n, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, float* g, float* m, float* v, int64_t n,
                       const drt_adam_opts& o, hipStream_t st) {
  const double c1 = 1.0 - pow((double)o.beta1, (double)o.step);
  const double c2 = 1.0 - pow((double)o.beta2, (double)o.step);
  const AdamArgs a = {o.lr, o.beta1, o.beta2, o.eps, (float)c1, (float)c2, o.lo, o.hi};
  auto aligned = [](const void* q, uintptr_t k) { return ((uintptr_t)q & (k - 1)) == 0; };
  const bool vec = aligned(p, 16) && aligned(g, 16) && aligned(m, 16) && aligned(v, 16) &&
                   (!o.half_out || aligned(o.half_out, 8));
  const int64_t n4 = vec ? n / 4 : 0;
  if (n4 > 0) {
    int64_t blocks = (n4 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_adam4, dim3((unsigned)blocks), dim3(256), 0, st,
                       reinterpret_cast<float4*>(p), reinterpret_cast<float4*>(g),
                       reinterpret_cast<float4*>(m), reinterpret_cast<float4*>(v), n4, a,
                       o.zero_grad, reinterpret_cast<uint2*>(o.half_out));
  }
  if (4 * n4 < n) {
    int64_t blocks = (n - 4 * n4 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, st, p, g, m, v, 4 * n4, n, a,
                       o.zero_grad, o.half_out);
  }
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

// ---------------------------------------------------------------------------
// Library-held scratch for the entry point that allocates nothing: the
// intersection records and work counter of the persistent replay.  Each GPU
// holds its own copy for the life of the process.  In host code the array's
// name is not a device address: kernels and fills only ever receive the
// address hipGetSymbolAddress returned for the current device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void** out) {
  static std::atomic<void*> ptrs[kMaxDevices];
  static std::mutex mu;
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  void* p = ptrs[dev].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> lock(mu);
    p = ptrs[dev].load(std::memory_order_relaxed);
    if (!p) {
      // once per device, with that device current (hipGetDevice above)
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return e;
      if (!p) return hipErrorInvalidSymbol;
      ptrs[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return hipSuccess;
}

}  // namespace drt
