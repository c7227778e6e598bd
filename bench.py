"""Throughput of one differentiable-rendering gradient step on one MI355X.

Workload (the reverse-mode configuration at 1024x1024): the Cornell-box-like
scene with a GGX conductor, a 4096x4096x3 float32 albedo texture on the back
wall and one roughness scalar; 1024x1024 pixels, 16 spp, max depth 3, no
Russian roulette.  One step = primal render (seed A) -> L2 loss and
image-space adjoint -> replayed adjoint (seed B) scattering texel and
roughness gradients -> Adam on texture and roughness (gradients re-zeroed by
the same kernel).  The replay reads pass A's intersections from a 12 MiB
record buffer instead of tracing the same rays again (identical gradients);
the re-tracing replay's time is reported beside it.  Inputs are resident in
HBM before timing starts.

Reported: Msamples/s = 1024*1024*16 / step time; the adjoint kernel's
roofline (ALU bound; algorithmic FLOPs from the traversal/shading counters of
a stats run, divided by its HIP-event launch duration); the FP64 CPU oracle's
throughput on a bounded sample of the same workload; and the radiance cache
against plain path tracing (depth 6, RR from 3): time to equal RMSE for the
primal at 1024^2 against a 4096-spp plain reference, and the gradient step
with the cache in the primal and in the replay (plus one training frame).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Algorithmic work per counted unit (derivation in the design notes):
FLOP_PER_NODE = 80.0      # four child slab tests (four-wide BVH node)
FLOP_PER_TRI = 40.0       # one watertight triangle test
FLOP_PER_VERTEX = 200.0   # shading a scattering vertex: frame, BSDF eval + sample, light sample, MIS
PEAK_FP32_VALU = 78.6     # TFLOP/s: 256 CU x 64 lanes x 2 (FMA) x 2.4 GHz, non-packed FP32


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--res", type=int, default=1024)
    ap.add_argument("--spp", type=int, default=16)
    ap.add_argument("--tex", type=int, default=4096)
    ap.add_argument("--target-spp", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-aux", action="store_true", help="skip the 1M-triangle primal figure")
    ap.add_argument("--no-cache", action="store_true",
                    help="skip the radiance-cache comparison (equal RMSE, cached gradient step)")
    ap.add_argument("--no-recovery", action="store_true",
                    help="skip the 200-step texture recovery, cache vs plain at matched time")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 256 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--strategies-only", action="store_true",
                    help="only the image + gradient strategies (PRB megakernel, PRB wavefront, "
                         "checkpointed) on the gradient-step workload, once each; prints their JSON")
    ap.add_argument("--scene-1m-only", action="store_true",
                    help="only the ~1M-triangle scene's primal (megakernel and wavefront, once "
                         "each after a warm-up) and its replayed adjoint; prints their JSON")
    ap.add_argument("--cache-render-only", action="store_true",
                    help="only the radiance cache's render at 1024^2, 64 spp (after 100 training "
                         "frames) and the plain render beside it, twice each; prints their times")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the design notes describe how the gradient step would shard).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2202_01284_amd as drt
    import scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda"
    if args.scene_1m_only:
        print(json.dumps(aux_primal_1m(drt, scenes, torch, reps=1)), flush=True)
        return
    if args.cache_render_only:
        print(json.dumps(cache_render_only(drt, scenes, torch, R=args.res)), flush=True)
        return
    if args.calib_copy:
        # a plain copy of known size: 256 MiB read + 256 MiB written
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    R, SPP, D = args.res, args.spp, 3
    sc = scenes.cornell(tex_size=args.tex, width=R, height=R, conductor=True)
    gs = drt.Scene(sc)
    cams = sc.cameras
    tex = torch.full((args.tex, args.tex, 3), 0.5, dtype=torch.float32, device=dev)
    if args.strategies_only:
        rough = torch.tensor([0.3], dtype=torch.float32, device=dev)
        a = torch.from_numpy(np.random.default_rng(4).normal(size=(1, R, R, 3)).astype(np.float32)
                             * 1e-3).to(dev)
        print(json.dumps(checkpoint_compare(drt, scenes, torch, sc, [tex], rough, a, R, SPP, D,
                                            depths=())), flush=True)
        return
    rough = torch.tensor([0.3], dtype=torch.float32, device=dev)
    # target: seeded random texture, roughness 0.2, rendered once at high spp
    tex_t = torch.from_numpy(scenes.random_texture(args.tex)).to(dev)
    rough_t = torch.tensor([0.2], dtype=torch.float32, device=dev)
    target = drt.render_forward(gs, [tex_t], rough_t, cams, args.target_spp, D, seed=1284)
    del tex_t
    gtex = torch.zeros_like(tex)
    grough = torch.zeros_like(rough)
    m_t, v_t = torch.zeros_like(tex), torch.zeros_like(tex)
    m_r, v_r = torch.zeros_like(rough), torch.zeros_like(rough)
    img = torch.empty((1, R, R, 3), dtype=torch.float32, device=dev)
    adj = torch.empty_like(img)
    ws = torch.empty(int(drt.lib.drt_loss_workspace_floats(img.numel())), dtype=torch.float32,
                     device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    hits = drt.adjoint_hit_records(cams, SPP, D)
    ev, step_ev = [], []

    def step(k, timed, records=True):
        # timed steps carry four HIP events (start, after the loss, after the
        # adjoint, end) on the launch stream: per-step parts and medians
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if timed else None
        if timed:
            e[0].record()
        drt.render_forward(gs, [tex], rough, cams, SPP, D, seed=2 * k + 1, out=img)
        drt.loss_l2(img, target, adj=adj)
        if timed:
            e[1].record()
        drt.render_adjoint(gs, [tex], rough, cams, adj, SPP, D, seed=2 * k + 2,
                           grad_textures=[gtex], grad_roughness=grough,
                           hit_records=hits if records else None)
        if timed:
            e[2].record()
            ev.append((e[1], e[2]))
        drt.adam_step(tex, gtex, m_t, v_t, k + 1, lr=1e-2, lo=0.0, hi=1.0, zero_grad=True)
        drt.adam_step(rough, grough, m_r, v_r, k + 1, lr=1e-2, lo=0.01, hi=1.0, zero_grad=True)
        if timed:
            e[3].record()
            step_ev.append(e)

    for k in range(args.warmup):
        step(k, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        step(k, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    samples = R * R * SPP
    value = samples / (ms * 1e-3) / 1e6
    adj_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    med = lambda i, j: round(float(np.median([e[i].elapsed_time(e[j]) for e in step_ev])), 3)  # noqa: E731
    step_parts = {"step_median": med(0, 3), "primal_and_loss_median": med(0, 1),
                  "adjoint_median": med(1, 2), "adam_median": med(2, 3)}
    # the same steps with the replay tracing its rays again (no records)
    k0 = args.warmup + args.steps
    step(k0, False, records=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(k0 + 1, k0 + 1 + args.steps):
        step(k, False, records=False)
    torch.cuda.synchronize()
    ms_retrace = (time.perf_counter() - t0) * 1e3 / args.steps

    # the primal of the same step by the wavefront variant (comparison only)
    ws = torch.empty(int(drt.lib.drt_render_wavefront_workspace_bytes(R * R * SPP)), dtype=torch.uint8,
                     device=dev)
    wf_img = torch.empty_like(img)
    drt.render_wavefront(gs, [tex], rough, cams, SPP, D, seed=1, out=wf_img, workspace=ws)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(3):
        drt.render_forward(gs, [tex], rough, cams, SPP, D, seed=3 + k, out=wf_img)
    e1.record()
    torch.cuda.synchronize()
    mk_ms = e0.elapsed_time(e1) / 3
    e0.record()
    for k in range(3):
        drt.render_wavefront(gs, [tex], rough, cams, SPP, D, seed=3 + k, out=wf_img, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    wf_ms = e0.elapsed_time(e1) / 3
    del ws, wf_img
    # and the replayed adjoint (gradients into scratch tensors)
    ws = torch.empty(int(drt.lib.drt_render_adjoint_wavefront_workspace_bytes(R * R * SPP)),
                     dtype=torch.uint8, device=dev)
    g_t, g_r = torch.zeros_like(tex), torch.zeros_like(rough)
    drt.render_adjoint_wavefront(gs, [tex], rough, cams, adj, SPP, D, seed=2, grad_textures=[g_t],
                                 grad_roughness=g_r, workspace=ws)
    e0.record()
    for k in range(2):
        drt.render_adjoint(gs, [tex], rough, cams, adj, SPP, D, seed=4 + k, grad_textures=[g_t],
                           grad_roughness=g_r)
    e1.record()
    torch.cuda.synchronize()
    mk_adj = e0.elapsed_time(e1) / 2  # the replay tracing its rays again
    e0.record()
    for k in range(2):
        drt.render_adjoint_wavefront(gs, [tex], rough, cams, adj, SPP, D, seed=4 + k, grad_textures=[g_t],
                                     grad_roughness=g_r, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    wf_adj = e0.elapsed_time(e1) / 2
    del ws, g_t, g_r
    wavefront = {"primal_ms_megakernel": round(mk_ms, 3), "primal_ms_wavefront": round(wf_ms, 3),
                 "adjoint_ms_megakernel": round(mk_adj, 3),
                 "adjoint_ms_megakernel_records": round(adj_ms, 3),
                 "adjoint_ms_wavefront": round(wf_adj, 3),
                 "wavefront_over_megakernel_time": {"primal": round(wf_ms / mk_ms, 3),
                                                    "adjoint": round(wf_adj / mk_adj, 3)}}

    # forward mode (one pass carrying tangents): the image derivative along a
    # random direction in the texture and the roughness, same workload
    gen = torch.Generator(device=dev).manual_seed(8)
    t_tex = torch.randn(tex.shape, generator=gen, device=dev)
    t_rough = torch.ones_like(rough)
    jvp_img = torch.empty((1, R, R, 3), dtype=torch.float32, device=dev)
    drt.render_jvp(gs, [tex], rough, cams, SPP, D, seed=2, tan_textures=[t_tex],
                   tan_roughness=t_rough, out=jvp_img)
    e0.record()
    for k in range(2):
        drt.render_jvp(gs, [tex], rough, cams, SPP, D, seed=3 + k, tan_textures=[t_tex],
                       tan_roughness=t_rough, out=jvp_img)
    e1.record()
    torch.cuda.synchronize()
    jvp_ms = e0.elapsed_time(e1) / 2
    jvp = {"ms": round(jvp_ms, 3), "msamples_s": round(R * R * SPP / (jvp_ms * 1e-3) / 1e6, 3),
           "primal_ms": round(mk_ms, 3),
           "what": "forward-mode image derivative along a random texture and roughness direction "
                   "(k_render_jvp, one pass carrying tangents), same scene, spp and depth"}
    del t_tex, jvp_img

    # algorithmic work of one adjoint launch (stats run, not timed)
    stats = drt.new_stats()
    drt.render_adjoint(gs, [tex], rough, cams, adj, SPP, D, seed=2 * args.warmup + 2,
                       grad_textures=[torch.zeros_like(tex)], grad_roughness=torch.zeros_like(rough),
                       stats=stats, hit_records=hits)
    st = drt.read_stats(stats)
    flops = st["nodes"] * FLOP_PER_NODE + st["tris"] * FLOP_PER_TRI + st["vertices"] * FLOP_PER_VERTEX
    achieved = flops / (adj_ms * 1e-3) / 1e12
    # the replay from intersection records; <.., true> when the scene fits the LDS copy
    kname = "k_render_adjoint<false, 1, true, %s>" % ("true" if gs.info["lds_copy"] else "false")
    roofline = {"kernel": kname, "bound": "alu", "achieved": round(achieved, 4),
                "peak": PEAK_FP32_VALU, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VALU, 5),
                "traffic": measured_traffic(), "launch_ms": round(adj_ms, 3),
                "units_per_launch": {k: st[k] for k in ("rays", "shadow_rays", "nodes", "tris",
                                                         "vertices", "scatter", "samples")},
                # lanes of a wave-wide texel scatter per distinct texel: the
                # most a wave-level merge of equal keys could cut the atomics by
                "texel_lanes_per_key": round(st["tex_lanes"] / max(st["tex_keys"], 1), 4),
                "simd_utilisation": simd_utilisation(st)}

    aux = None
    checkpointed = None
    if not args.no_aux:
        aux = aux_primal_1m(drt, scenes, torch)
        checkpointed = checkpoint_compare(drt, scenes, torch, sc, [tex], rough, adj, R, SPP, D)

    cache = None
    if not args.no_cache:
        cache = {"equal_rmse": cache_equal_rmse(drt, scenes, torch, R=args.res),
                 "gradient_step": cache_gradient_step(drt, scenes, torch, R=args.res, SPP=args.spp,
                                                      tex_size=args.tex),
                 "gradient_bias": cache_gradient_bias(drt, scenes, torch, tex_size=args.tex)}

    recovery = None
    if not args.no_recovery:
        recovery = texture_recovery(drt, scenes, torch, tex_size=args.tex)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(sc, R, SPP, D, args.cpu_seconds)

    line = {
        "metric": "Msamples/s primal+adjoint at 1024^2 (gradient step)",
        "value": round(value, 3),
        "unit": "Msamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "step_ms_hip_events": step_parts,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded procedural scene and textures)",
        "config": {"workload": "cornell-box + GGX conductor, 4096^2x3 texture + 1 roughness, "
                               "primal + L2 + replayed adjoint (replay from intersection records) "
                               "+ Adam",
                   "width": R, "height": R, "spp": SPP, "max_depth": D, "russian_roulette": False,
                   "texture": [args.tex, args.tex, 3], "triangles": sc.n_triangles,
                   "target_spp": args.target_spp},
        "retrace_step": {"ms_per_step": round(ms_retrace, 3),
                         "msamples_s": round(samples / (ms_retrace * 1e-3) / 1e6, 3),
                         "what": "the same gradient step with the replay tracing its rays again"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cache": cache,
        "wavefront": wavefront,
        "jvp": jvp,
        "checkpointed": checkpointed,
        "aux": aux,
        "texture_recovery": recovery,
    }
    print(json.dumps(line), flush=True)


def simd_utilisation(st):
    """Mean fraction of a wave's 64 lanes taking part in each phase, from a
    stats launch: node visits, triangle tests, vertex steps of live paths
    and shading blocks, each per-lane count over 64 x the wave's count."""
    def f(lanes, waves):
        return round(st[lanes] / (64.0 * st[waves]), 4) if st[waves] else None
    return {"node_loop": f("nodes", "wave_nodes"), "triangle_loop": f("tris", "wave_tris"),
            "vertex_steps": f("lane_steps", "wave_steps"), "shading": f("vertices", "wave_shade")}


def source_code_digest(paths):
    """SHA-256 of C/C++/HIP sources with their comments removed and runs of
    whitespace collapsed (string and character literals kept whole): it
    changes when the code does, not when a comment does."""
    import hashlib
    h = hashlib.sha256()
    for f in paths:
        text = open(os.path.join(ROOT, f), encoding="utf-8").read()
        out, i, n = [], 0, len(text)
        while i < n:
            c = text[i]
            if text.startswith("//", i):
                j = text.find("\n", i)
                i = n if j < 0 else j
                out.append(" ")
            elif text.startswith("/*", i):
                j = text.find("*/", i + 2)
                i = n if j < 0 else j + 2
                out.append(" ")
            elif c in "\"'":
                j = i + 1
                while j < n and text[j] != c:
                    j += 2 if text[j] == "\\" else 1
                out.append(text[i:j + 1])
                i = j + 1
            else:
                out.append(c)
                i += 1
        h.update(" ".join("".join(out).split()).encode())
        h.update(b"\0")
    return h.hexdigest()


def counter_record(name):
    """A committed counter summary (profiles/<name>), or None when the
    kernel code has changed since the counters were taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", name)))
        digest = source_code_digest(rec["sources"])  # every file the kernel is compiled from
    except (OSError, ValueError, KeyError, TypeError):
        return None
    if digest != rec.get("source_code_sha256"):
        return None
    return rec


def measured_traffic():
    """HBM bytes per adjoint launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, calibrated on a plain copy), or None when
    the kernel source has changed since the counters were taken."""
    rec = counter_record("adjoint_traffic.json")
    return int(rec["hbm_bytes"]) if rec else None


def checkpoint_compare(drt, scenes, torch, sc, tex, rough, adj, R, SPP, D,
                       depths=(3, 8, 16, 32), R_long=512, spp_long=4):
    """Image + gradient of <adj, image> by the three strategies the paper
    compares (Sec. "Evaluation", differentiating existing methods): PRB as
    megakernels (primal, then pass A + replay), PRB as wavefront kernels,
    and the checkpointed path tracer (forward with a checkpoint per bounce,
    then the backward walk; wavefront kernels).  HIP-event times; the
    checkpoints' memory beside them.  First on the gradient-step workload,
    then on the Cornell box at R_long^2, spp_long spp without Russian
    roulette for growing maximum depth."""
    gs = drt.Scene(sc)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def timed(fn, reps=2):
        fn()
        a, b = ev(), ev()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def measure(cams, spp, depth, a):
        img = torch.empty((len(cams), cams[0].height, cams[0].width, 3), device="cuda")
        gt, gr = [torch.zeros_like(t) for t in tex], torch.zeros_like(rough)
        n = len(cams) * cams[0].width * cams[0].height * spp
        ws_p = torch.empty(int(drt.lib.drt_render_wavefront_workspace_bytes(n)), dtype=torch.uint8,
                           device="cuda")
        ws_a = torch.empty(int(drt.lib.drt_render_adjoint_wavefront_workspace_bytes(n)),
                           dtype=torch.uint8, device="cuda")
        mk = timed(lambda: (drt.render_forward(gs, tex, rough, cams, spp, depth, seed=1, out=img),
                            drt.render_adjoint(gs, tex, rough, cams, a, spp, depth, seed=2,
                                               grad_textures=gt, grad_roughness=gr)))
        hits = drt.adjoint_hit_records(cams, spp, depth)
        mkr = timed(lambda: (drt.render_forward(gs, tex, rough, cams, spp, depth, seed=1, out=img),
                             drt.render_adjoint(gs, tex, rough, cams, a, spp, depth, seed=2,
                                                grad_textures=gt, grad_roughness=gr,
                                                hit_records=hits)))
        rec_mb = hits.numel() / 2 ** 20
        del hits
        wf = timed(lambda: (drt.render_wavefront(gs, tex, rough, cams, spp, depth, seed=1, out=img,
                                                 workspace=ws_p),
                            drt.render_adjoint_wavefront(gs, tex, rough, cams, a, spp, depth, seed=2,
                                                         grad_textures=gt, grad_roughness=gr,
                                                         workspace=ws_a)))
        del ws_p, ws_a
        ws_c = drt.checkpoint_workspace(cams, spp, depth)
        ck = timed(lambda: (drt.render_checkpointed_forward(gs, tex, rough, cams, spp, depth, seed=1,
                                                            workspace=ws_c, out=img),
                            drt.render_checkpointed_adjoint(gs, tex, rough, cams, a, spp, depth, ws_c,
                                                            seed=1, grad_textures=gt,
                                                            grad_roughness=gr)))
        mb = ws_c.numel() / 2 ** 20
        del ws_c
        return {"max_depth": depth, "prb_megakernel_ms": round(mk, 3),
                "prb_megakernel_records_ms": round(mkr, 3), "records_mib": round(rec_mb, 1),
                "prb_wavefront_ms": round(wf, 3),
                "checkpointed_wavefront_ms": round(ck, 3), "checkpointed_workspace_mib": round(mb, 1),
                "prb_wavefront_workspace_mib": round(n * 13 * 16 / 2 ** 20, 1)}

    head = measure(sc.cameras, SPP, D, adj)
    cams = scenes.cornell(width=R_long, height=R_long).cameras
    a = torch.from_numpy(np.random.default_rng(3).normal(size=(1, R_long, R_long, 3))
                         .astype(np.float32) * 1e-3).cuda()
    rows = [measure(cams, spp_long, d, a) for d in depths]
    return {"workload": f"image + gradient; {R}^2 {SPP} spp D{D} (gradient-step scene), then "
                        f"{R_long}^2 {spp_long} spp without RR at growing max depth",
            "gradient_step_workload": head, "by_depth": rows}


def aux_primal_1m(drt, scenes, torch, reps=2):
    """Primal Msamples/s on the ~1M-triangle procedural scene (1024^2, 64 spp,
    depth 6, Russian roulette from 3): reported beside the headline."""
    t = time.perf_counter()
    sc = scenes.procedural()
    gs = drt.Scene(sc)
    build_s = time.perf_counter() - t
    tex = [torch.from_numpy(x).cuda() for x in sc.textures]
    rough = torch.from_numpy(sc.roughness).cuda()
    img = torch.empty((1, 1024, 1024, 3), dtype=torch.float32, device="cuda")
    drt.render_forward(gs, tex, rough, sc.cameras, 64, 6, 3, seed=1, out=img)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(reps):
        drt.render_forward(gs, tex, rough, sc.cameras, 64, 6, 3, seed=2 + k, out=img)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    stats = drt.new_stats()
    drt.render_forward(gs, tex, rough, sc.cameras, 64, 6, 3, seed=2, out=img, stats=stats)
    st = drt.read_stats(stats)
    rays = st["rays"] + st["shadow_rays"]
    # traversal roofline: the nodes and triangles a ray must read (128 B per
    # four-wide node, 48 B per triangle) at the achieved ray rate, against
    # HBM; the HBM bytes and L2 requests per ray, VALU busy and lane
    # utilisation from the committed counter summary of this launch
    bpr = (st["nodes"] * 128.0 + st["tris"] * 48.0) / max(rays, 1)
    rec = counter_record("traversal_1m_counters.json")
    traversal = {"algorithmic_bytes_per_ray": round(bpr, 1),
                 "achieved_GBps": round(bpr * rays / (ms * 1e-3) / 1e9, 1),
                 "hbm_peak_GBps": 8000.0,
                 "frac_of_hbm_peak": round(bpr * rays / (ms * 1e-3) / 8e12, 4),
                 "hbm_bytes_per_ray": rec["hbm_bytes_per_ray"] if rec else None,
                 "l2_requests_per_ray": rec["l2_requests_per_ray"] if rec else None,
                 "l2_hit_rate": rec["l2_hit_rate"] if rec else None,
                 "valu_busy": rec["valu_busy"] if rec else None,
                 "valu_lane_utilisation": rec["valu_lane_utilisation"] if rec else None}
    # the same image by the wavefront variant (state through HBM between kernels)
    ws = torch.empty(int(drt.lib.drt_render_wavefront_workspace_bytes(1024 * 1024 * 64)),
                     dtype=torch.uint8, device="cuda")
    drt.render_wavefront(gs, tex, rough, sc.cameras, 64, 6, 3, seed=1, out=img, workspace=ws)
    e0.record()
    for k in range(reps):
        drt.render_wavefront(gs, tex, rough, sc.cameras, 64, 6, 3, seed=2 + k, out=img, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    wf_ms = e0.elapsed_time(e1) / reps
    del ws
    # replayed adjoint at 16 spp (random image adjoint), megakernel vs wavefront
    adj = torch.randn((1, 1024, 1024, 3), device="cuda") * 1e-3
    gt = [torch.zeros_like(x) for x in tex]
    gr = torch.zeros_like(rough)
    ws = torch.empty(int(drt.lib.drt_render_adjoint_wavefront_workspace_bytes(1024 * 1024 * 16)),
                     dtype=torch.uint8, device="cuda")
    drt.render_adjoint_wavefront(gs, tex, rough, sc.cameras, adj, 16, 6, 3, seed=5, grad_textures=gt,
                                 grad_roughness=gr, workspace=ws)
    e0.record()
    drt.render_adjoint(gs, tex, rough, sc.cameras, adj, 16, 6, 3, seed=6, grad_textures=gt, grad_roughness=gr)
    e1.record()
    torch.cuda.synchronize()
    adj_mk = e0.elapsed_time(e1)
    e0.record()
    drt.render_adjoint_wavefront(gs, tex, rough, sc.cameras, adj, 16, 6, 3, seed=6, grad_textures=gt,
                                 grad_roughness=gr, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    adj_wf = e0.elapsed_time(e1)
    del ws
    hits = drt.adjoint_hit_records(sc.cameras, 16, 6)
    drt.render_adjoint(gs, tex, rough, sc.cameras, adj, 16, 6, 3, seed=5, grad_textures=gt,
                       grad_roughness=gr, hit_records=hits)
    e0.record()
    drt.render_adjoint(gs, tex, rough, sc.cameras, adj, 16, 6, 3, seed=6, grad_textures=gt,
                       grad_roughness=gr, hit_records=hits)
    e1.record()
    torch.cuda.synchronize()
    adj_rec = e0.elapsed_time(e1)
    del gt, gr, adj, hits
    return {"workload": "procedural ~1M triangles, 8 BSDFs, env + 16 quad lights, 1024^2 64spp D6 RR3",
            "triangles": sc.n_triangles, "primal_msamples_s": round(1024 * 1024 * 64 / ms / 1e3, 2),
            "primal_ms": round(ms, 2), "wavefront_primal_ms": round(wf_ms, 2),
            "wavefront_over_megakernel_time": round(wf_ms / ms, 3),
            "adjoint_16spp_ms": {"megakernel": round(adj_mk, 2), "megakernel_records": round(adj_rec, 2),
                                 "wavefront": round(adj_wf, 2)},
            "mrays_s": round(rays / ms / 1e3, 1),
            "simd_utilisation": simd_utilisation(st),
            "traversal": traversal,
            "nodes_per_ray": round(st["nodes"] / max(rays, 1), 2),
            "tris_per_ray": round(st["tris"] / max(rays, 1), 2),
            "bvh": {k: gs.info[k] for k in ("n_nodes", "max_depth", "forced_leaves")},
            "host_build_s": round(build_s, 2)}


def cache_equal_rmse(drt, scenes, torch, R=1024, frames=300, spps=(1, 2, 4, 8, 16, 32, 64), ref_spp=4096):
    """Radiance cache vs plain path tracing at equal RMSE (Cornell box with
    the random back-wall texture, D = 6, RR from 3, truncation at v3).

    The reference is a plain render at ref_spp.  Both estimators are rendered
    at each spp in `spps`; RMSE^2 against the reference is corrected for the
    reference's own variance (V_plain / ref_spp).  The plain spp needed to
    reach the cache's RMSE is V_plain / RMSE_cache^2, and its time is that
    times the measured plain time per spp.  Training (65,536 paths a frame)
    is reported per frame beside it.  A second cache is trained for the same
    number of frames by self-training (16,384 paths a frame closed by the
    cache at v5, records at v1..v4) and measured the same way."""
    sc = scenes.cornell(texture=scenes.random_texture(64), width=R, height=R)
    cfg = scenes.nrc_config(sc)
    W0, grid0 = scenes.nrc_init(cfg, seed=16)
    gs = drt.Scene(sc)
    tex = [torch.from_numpy(sc.textures[0]).cuda()]
    cams = sc.cameras
    D, RR = 6, 3
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    ref = torch.zeros((1, R, R, 3), dtype=torch.float64, device="cuda")
    img = torch.empty((1, R, R, 3), dtype=torch.float32, device="cuda")
    chunk = 256
    for c in range(ref_spp // chunk):
        drt.render_forward(gs, tex, None, cams, chunk, D, RR, seed=100000 + c, out=img)
        ref += img.double()
    ref /= ref_spp // chunk

    def trained(**kw):
        c = drt.NrcCache(cfg, W0, grid0, lr=1e-2, **kw)
        c.train_frame(gs, tex, None, cams, seed=500)            # warm-up
        e0, e1 = ev(), ev()
        torch.cuda.synchronize()
        e0.record()
        for f in range(frames):
            c.train_frame(gs, tex, None, cams, seed=1000 + f)
        e1.record()
        torch.cuda.synchronize()
        return c, e0.elapsed_time(e1) / frames

    cache, train_ms = trained(n_paths=65536)
    cache_self, train_self_ms = trained(n_paths=16384, self_training=5)

    work = drt.cached_work(R * R * max(spps), "cuda")

    def timed(fn, reps=3):
        fn()
        a, b = ev(), ev()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def mse(x):
        return float(((x.double() - ref) ** 2).mean())

    rows = []
    for s in spps:
        plain_ms = timed(lambda: drt.render_forward(gs, tex, None, cams, s, D, RR, seed=7, out=img))
        m_plain = mse(img)
        cache_ms = timed(lambda: cache.render(gs, tex, None, cams, s, seed=7, out=img, work=work))
        m_cache = mse(img)
        self_ms = timed(lambda: cache_self.render(gs, tex, None, cams, s, seed=7, out=img, work=work))
        m_self = mse(img)
        v_plain = m_plain / (1.0 / s + 1.0 / ref_spp)            # per-sample variance of plain

        def equal(m, ms, tms):
            m_c = max(m - v_plain / ref_spp, 1e-30)                # cache MSE minus reference noise
            spp_eq = v_plain / m_c
            plain_eq_ms = spp_eq * plain_ms / s
            return spp_eq, plain_eq_ms / ms, plain_eq_ms / (ms + tms)

        spp_eq, sp, sp_t = equal(m_cache, cache_ms, train_ms)
        spp_eq_s, sp_s, sp_t_s = equal(m_self, self_ms, train_self_ms)
        rows.append({"spp": s, "plain_ms": round(plain_ms, 3), "cache_ms": round(cache_ms, 3),
                     "self_ms": round(self_ms, 3),
                     "rmse_plain": round(m_plain ** 0.5, 6), "rmse_cache": round(m_cache ** 0.5, 6),
                     "plain_spp_at_equal_rmse": round(spp_eq, 3),
                     "speedup_at_equal_rmse": round(sp, 3),
                     "speedup_incl_training": round(sp_t, 3),
                     "self_training": {"rmse_cache": round(m_self ** 0.5, 6),
                                       "plain_spp_at_equal_rmse": round(spp_eq_s, 3),
                                       "speedup_at_equal_rmse": round(sp_s, 3),
                                       "speedup_incl_training": round(sp_t_s, 3)}})
    at_target = {"cache": at_target_rmse(rows, "rmse_cache", "cache_ms", train_ms),
                 "self_training": at_target_rmse(rows, ("self_training", "rmse_cache"), "self_ms",
                                                 train_self_ms)}
    return {"workload": f"cornell-box, random 64^2 texture, {R}^2, D6 RR3, cache at v3, "
                        f"hash grid 16x2^19x2 fp16, 80-64x4-3 bf16 network",
            "at_target": at_target,
            "reference_spp": ref_spp, "train_frames": frames, "train_paths_per_frame": 65536,
            "train_ms_per_frame": round(train_ms, 3),
            "final_train_loss": round(float(cache.loss.item()), 4),
            "self_training": {"paths_per_frame": 16384, "tail_vertex": 5,
                              "train_ms_per_frame": round(train_self_ms, 3),
                              "final_train_loss": round(float(cache_self.loss.item()), 4)},
            "by_spp": rows}


def cache_render_only(drt, scenes, torch, R=1024, spp=64, frames=100, reps=2):
    """The cached render of the equal-RMSE comparison at its target spp
    (a cache trained for `frames` frames) and the plain render beside it,
    HIP-event times of `reps` launches each (for kernel traces and counters)."""
    sc = scenes.cornell(texture=scenes.random_texture(64), width=R, height=R)
    cfg = scenes.nrc_config(sc)
    W0, grid0 = scenes.nrc_init(cfg, seed=16)
    gs = drt.Scene(sc)
    tex = [torch.from_numpy(sc.textures[0]).cuda()]
    cache = drt.NrcCache(cfg, W0, grid0, lr=1e-2)
    for f in range(frames):
        cache.train_frame(gs, tex, None, sc.cameras, seed=1000 + f)
    work = drt.cached_work(R * R * spp, "cuda")
    img = torch.empty((1, R, R, 3), dtype=torch.float32, device="cuda")
    out = {}
    for name, fn in (("cache", lambda k: cache.render(gs, tex, None, sc.cameras, spp, seed=7 + k, out=img,
                                                      work=work)),
                     ("plain", lambda k: drt.render_forward(gs, tex, None, sc.cameras, spp, 6, 3,
                                                            seed=7 + k, out=img))):
        fn(0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for k in range(reps):
            fn(k + 1)
        b.record()
        torch.cuda.synchronize()
        out[name + "_ms"] = round(a.elapsed_time(b) / reps, 3)
    out["queries"] = int(work[2].item())
    out["workload"] = f"cornell-box, random 64^2 texture, {R}^2, {spp} spp, D6 RR3, cache at v3"
    return out


def at_target_rmse(rows, rmse_key, ms_key, train_ms):
    """Time for an estimator to reach the RMSE that plain path tracing
    reaches at the largest spp of `rows` (the target), against the plain
    render at that spp.  The estimator's spp at the target is interpolated
    between the two measured rows around the crossing (log RMSE linear in
    log spp), its time linearly in spp; one training frame per image is
    charged for 'incl_training'.  None where the estimator's RMSE at the
    largest spp is still above the target (bias dominates)."""
    import math

    def rm(r):
        return r[rmse_key[0]][rmse_key[1]] if isinstance(rmse_key, tuple) else r[rmse_key]
    last = rows[-1]
    target = last["rmse_plain"]
    out = {"target_rmse": target, "plain_spp": last["spp"], "plain_ms": last["plain_ms"]}
    if rm(last) > target:
        out.update({"spp": None, "ms": None, "speedup": None, "speedup_incl_training": None,
                    "note": "RMSE above the target at the largest spp"})
        return out
    lo = next((i for i in range(len(rows) - 1) if rm(rows[i]) > target >= rm(rows[i + 1])), None)
    if lo is None:  # already below the target at the smallest spp
        a = rows[0]
        spp = a["spp"] * (rm(a) / target) ** 2
        ms = a[ms_key] * spp / a["spp"]
    else:
        a, b = rows[lo], rows[lo + 1]
        f = (math.log(target) - math.log(rm(a))) / (math.log(rm(b)) - math.log(rm(a)))
        spp = math.exp(math.log(a["spp"]) + f * (math.log(b["spp"]) - math.log(a["spp"])))
        ms = a[ms_key] + (b[ms_key] - a[ms_key]) * (spp - a["spp"]) / (b["spp"] - a["spp"])
    out.update({"spp": round(spp, 2), "ms": round(ms, 3),
                "speedup": round(last["plain_ms"] / ms, 3),
                "speedup_incl_training": round(last["plain_ms"] / (ms + train_ms), 3)})
    return out


def cache_gradient_step(drt, scenes, torch, R=1024, SPP=16, tex_size=4096, steps=3):
    """Gradient step with paths of depth 6 (RR from 3) on the reverse-mode
    scene, plain vs radiance cache: primal (seed A) -> L2 -> replayed adjoint
    (seed B) -> Adam, and for the cache one training frame (65,536 paths,
    network + grid Adam) per step.  HIP-event times of each variant."""
    D, RR = 6, 3
    sc = scenes.cornell(tex_size=tex_size, width=R, height=R, conductor=True)
    cfg = scenes.nrc_config(sc)
    W0, grid0 = scenes.nrc_init(cfg, seed=16)
    gs = drt.Scene(sc)
    cams = sc.cameras
    dev = "cuda"
    tex = torch.full((tex_size, tex_size, 3), 0.5, dtype=torch.float32, device=dev)
    rough = torch.tensor([0.3], dtype=torch.float32, device=dev)
    tex_t = torch.from_numpy(scenes.random_texture(tex_size)).to(dev)
    target = drt.render_forward(gs, [tex_t], torch.tensor([0.2], device=dev), cams, 64, D, RR, seed=1284)
    del tex_t
    img = torch.empty((1, R, R, 3), dtype=torch.float32, device=dev)
    adj = torch.empty_like(img)
    gtex, grough = torch.zeros_like(tex), torch.zeros_like(rough)
    m_t, v_t, m_r, v_r = (torch.zeros_like(tex), torch.zeros_like(tex), torch.zeros_like(rough),
                          torch.zeros_like(rough))
    cache = drt.NrcCache(cfg, W0, grid0, n_paths=65536, lr=1e-2)
    for f in range(50):                                  # a briefly trained cache
        cache.train_frame(gs, [tex], rough, cams, seed=9000 + f)
    n = R * R * SPP
    work = drt.cached_work(n, dev, sample_radiance=True)
    hits = drt.adjoint_hit_records(cams, SPP, D)                # both replays read intersections
    hits_c = drt.cached_hit_records(cams, SPP, D)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def step(k, cached, input_grad=False):
        if cached:
            cache.render(gs, [tex], rough, cams, SPP, seed=2 * k + 1, out=img, work=work[:3])
        else:
            drt.render_forward(gs, [tex], rough, cams, SPP, D, RR, seed=2 * k + 1, out=img)
        drt.loss_l2(img, target, adj=adj)
        if cached:
            cache.adjoint(gs, [tex], rough, cams, adj, SPP, seed=2 * k + 2, grad_textures=[gtex],
                          grad_roughness=grough, work=work, input_grad=input_grad, hit_records=hits_c)
            cache.train_frame(gs, [tex], rough, cams, seed=20000 + k)
        else:
            drt.render_adjoint(gs, [tex], rough, cams, adj, SPP, D, RR, seed=2 * k + 2,
                               grad_textures=[gtex], grad_roughness=grough, hit_records=hits)
        drt.adam_step(tex, gtex, m_t, v_t, k + 1, lr=1e-2, lo=0.0, hi=1.0, zero_grad=True)
        drt.adam_step(rough, grough, m_r, v_r, k + 1, lr=1e-2, lo=0.01, hi=1.0, zero_grad=True)

    out = {}
    for name, cached, ig in (("plain", False, False), ("cache", True, False),
                             ("cache_input_grad", True, True)):
        step(0, cached, ig)
        a, b = ev(), ev()
        a.record()
        for k in range(1, 1 + steps):
            step(k, cached, ig)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        out[name] = {"ms_per_step": round(ms, 3), "msamples_s": round(n / ms / 1e3, 2)}
    return {"workload": f"cornell-box + GGX conductor, {tex_size}^2x3 texture, {R}^2 {SPP}spp D{D} "
                        f"RR{RR}, cache at v3 (one 65,536-path training frame per step)", **out}


def cache_gradient_bias(drt, scenes, torch, n_cams=16, R=512, spp=32, ref_spp=256, tex_size=4096,
                        train_frames=100):
    """Gradient error at matched wall time, cache vs plain (16 views at
    512^2 in one launch, depth 6, RR from 3, 4096^2x3 texture + roughness):
    the image adjoint is 2 (I - T) / N of a 32-spp primal against a 256-spp
    target; the reference gradient is the plain replayed adjoint at ref_spp;
    the cached gradient (32 spp, cache trained for train_frames frames; output
    detached, and through the network's albedo/roughness inputs) is timed,
    and the plain gradient is taken at the spp that costs the same time as
    the detached one.  Errors are ||g - g_ref|| / ||g_ref|| per texel and on the means of
    64x64-texel blocks (where sampling noise averages out and bias remains)."""
    D, RR = 6, 3
    sc = scenes.cornell(tex_size=tex_size, width=R, height=R, conductor=True)
    cams = scenes.ring_cameras(n_cams, R, R)
    cfg = scenes.nrc_config(sc)
    W0, grid0 = scenes.nrc_init(cfg, seed=16)
    gs = drt.Scene(sc)
    dev = "cuda"
    tex = torch.full((tex_size, tex_size, 3), 0.5, dtype=torch.float32, device=dev)
    rough = torch.tensor([0.3], dtype=torch.float32, device=dev)
    tex_t = torch.from_numpy(scenes.random_texture(tex_size)).to(dev)
    target = drt.render_forward(gs, [tex_t], torch.tensor([0.2], device=dev), cams, 256, D, RR, seed=1284)
    del tex_t
    img = drt.render_forward(gs, [tex], rough, cams, spp, D, RR, seed=11)
    adj = torch.empty_like(img)
    drt.loss_l2(img, target, adj=adj)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def grad(fn):
        gt, gr = torch.zeros_like(tex), torch.zeros_like(rough)
        fn(gt, gr)
        torch.cuda.synchronize()
        a, b = ev(), ev()
        gt.zero_()
        gr.zero_()
        a.record()
        fn(gt, gr)
        b.record()
        torch.cuda.synchronize()
        return gt, gr, a.elapsed_time(b)

    g_ref, _, _ = grad(lambda gt, gr: drt.render_adjoint(gs, [tex], rough, cams, adj, ref_spp, D, RR,
                                                           seed=101, grad_textures=[gt], grad_roughness=gr))
    cache = drt.NrcCache(cfg, W0, grid0, n_paths=65536, lr=1e-2)
    for f in range(train_frames):
        cache.train_frame(gs, [tex], rough, cams, seed=3000 + f)
    work = drt.cached_work(n_cams * R * R * spp, dev, sample_radiance=True)
    hits = drt.adjoint_hit_records(cams, spp, D)                # both replays read intersections
    hits_c = drt.cached_hit_records(cams, spp, D)
    g_c, _, t_c = grad(lambda gt, gr: cache.adjoint(gs, [tex], rough, cams, adj, spp, seed=103,
                                                    grad_textures=[gt], grad_roughness=gr, work=work,
                                                    hit_records=hits_c))
    g_ci, _, t_ci = grad(lambda gt, gr: cache.adjoint(gs, [tex], rough, cams, adj, spp, seed=103,
                                                      grad_textures=[gt], grad_roughness=gr, work=work,
                                                      input_grad=True, hit_records=hits_c))
    _, _, t_p32 = grad(lambda gt, gr: drt.render_adjoint(gs, [tex], rough, cams, adj, spp, D, RR, seed=105,
                                                         grad_textures=[gt], grad_roughness=gr,
                                                         hit_records=hits))
    spp_p = max(1, int(round(spp * t_c / t_p32)))
    g_p, _, t_p = grad(lambda gt, gr: drt.render_adjoint(gs, [tex], rough, cams, adj, spp_p, D, RR,
                                                         seed=107, grad_textures=[gt], grad_roughness=gr,
                                                         hit_records=hits))

    def err(g):
        d = (g - g_ref).double()
        full = float(d.norm() / g_ref.double().norm())
        b = tex_size // 64
        blk = lambda x: x.double().reshape(b, 64, b, 64, 3).mean((1, 3))  # noqa: E731
        block = float((blk(g) - blk(g_ref)).norm() / blk(g_ref).norm())
        return round(full, 4), round(block, 4)

    ec, ep, eci = err(g_c), err(g_p), err(g_ci)
    return {"workload": f"{n_cams} views x {R}^2, depth {D} RR{RR}, {tex_size}^2x3 texture, "
                        f"reference: plain adjoint at {ref_spp} spp",
            "cache": {"spp": spp, "ms": round(t_c, 2), "rel_err_texel": ec[0], "rel_err_64x64_blocks": ec[1]},
            "cache_input_grad": {"spp": spp, "ms": round(t_ci, 2), "rel_err_texel": eci[0],
                                 "rel_err_64x64_blocks": eci[1]},
            "plain_matched_time": {"spp": spp_p, "ms": round(t_p, 2), "rel_err_texel": ep[0],
                                   "rel_err_64x64_blocks": ep[1]},
            "train_frames": train_frames}


def texture_recovery(drt, scenes, torch, n_cams=16, R=512, spp=32, steps=200, tex_size=4096,
                     lr=1e-2, every=10, target_spp=256, warmup_frames=100):
    """Differentiable optimisation with the radiance cache (16 seeded views
    at 512^2 in one launch, depth 6, RR from 3): 200 Adam steps (lr 1e-2)
    recover the 4096^2x3 back-wall texture and the conductor roughness from
    target renders (roughness 0.2 and a random texture of 64x64 cells --
    scenes.cell_texture -- which the 512^2 views resolve; plain at
    target_spp).  Run twice from the same start (texture 0.5, roughness 0.3):
    with the cache in the primal and in the replay at `spp` (first trained
    for `warmup_frames` frames, then one 65,536-path frame per step on the
    current parameters; the warm-up's time is charged to the first step),
    and plain at the spp whose step costs the same wall time as the cached
    step.  Every `every` steps: the image loss, the texture error against the
    target (relative L2 per texel and of 64x64-texel cell means) and the
    roughness, with the accumulated HIP-event time."""
    D, RR = 6, 3
    dev = "cuda"
    sc = scenes.cornell(tex_size=tex_size, width=R, height=R, conductor=True)
    cams = scenes.ring_cameras(n_cams, R, R)
    cfg = scenes.nrc_config(sc)
    W0, grid0 = scenes.nrc_init(cfg, seed=16)
    gs = drt.Scene(sc)
    tex_t = torch.from_numpy(scenes.cell_texture(tex_size)).to(dev)
    target = drt.render_forward(gs, [tex_t], torch.tensor([0.2], device=dev), cams, target_spp, D, RR,
                                seed=1284)
    b = tex_size // 64
    blk = lambda x: x.double().reshape(b, 64, b, 64, 3).mean((1, 3))  # noqa: E731
    t_blk = blk(tex_t)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def run(cached, s, n_steps, record=True, warm=warmup_frames):
        tex = torch.full((tex_size, tex_size, 3), 0.5, dtype=torch.float32, device=dev)
        rough = torch.tensor([0.3], dtype=torch.float32, device=dev)
        gtex, grough = torch.zeros_like(tex), torch.zeros_like(rough)
        m_t, v_t, m_r, v_r = (torch.zeros_like(tex), torch.zeros_like(tex), torch.zeros_like(rough),
                              torch.zeros_like(rough))
        img = torch.empty((n_cams, R, R, 3), dtype=torch.float32, device=dev)
        adj = torch.empty_like(img)
        n = n_cams * R * R * s
        curve, total_ms = [], 0.0
        if cached:
            cache = drt.NrcCache(cfg, W0, grid0, n_paths=65536, lr=1e-2)
            work = drt.cached_work(n, dev, sample_radiance=True)
            hits = drt.cached_hit_records(cams, s, D)
            a, e = ev(), ev()
            a.record()
            for f in range(warm):
                cache.train_frame(gs, [tex], rough, cams, seed=40000 + f)
            e.record()
            torch.cuda.synchronize()
            total_ms += a.elapsed_time(e)
        else:
            hits = drt.adjoint_hit_records(cams, s, D)
        warm_ms = total_ms
        for k in range(n_steps):
            a, e = ev(), ev()
            a.record()
            if cached:
                cache.train_frame(gs, [tex], rough, cams, seed=50000 + k)
                cache.render(gs, [tex], rough, cams, s, seed=2 * k + 1, out=img, work=work[:3])
            else:
                drt.render_forward(gs, [tex], rough, cams, s, D, RR, seed=2 * k + 1, out=img)
            loss, _ = drt.loss_l2(img, target, adj=adj)
            if cached:
                cache.adjoint(gs, [tex], rough, cams, adj, s, seed=2 * k + 2, grad_textures=[gtex],
                              grad_roughness=grough, work=work, hit_records=hits)
            else:
                drt.render_adjoint(gs, [tex], rough, cams, adj, s, D, RR, seed=2 * k + 2,
                                   grad_textures=[gtex], grad_roughness=grough, hit_records=hits)
            drt.adam_step(tex, gtex, m_t, v_t, k + 1, lr=lr, lo=0.0, hi=1.0, zero_grad=True)
            drt.adam_step(rough, grough, m_r, v_r, k + 1, lr=lr, lo=0.01, hi=1.0, zero_grad=True)
            e.record()
            torch.cuda.synchronize()
            total_ms += a.elapsed_time(e)
            if record and ((k + 1) % every == 0 or k == 0):
                d = (tex - tex_t).double()
                curve.append({"step": k + 1, "ms": round(total_ms, 1),
                              "image_loss": float(loss.item()),
                              "tex_rel_err_texel": round(float(d.norm() / tex_t.double().norm()), 5),
                              "tex_rel_err_64x64_blocks": round(float((blk(tex) - t_blk).norm()
                                                                      / t_blk.norm()), 5),
                              "roughness": round(float(rough.item()), 5)})
        del hits
        return (total_ms - warm_ms) / n_steps, curve

    # per-step cost of each method (a few steps, not recorded), then the
    # plain spp whose step costs what the cached step costs
    run(True, spp, 2, record=False, warm=0)
    ms_cache, _ = run(True, spp, 4, record=False, warm=0)
    ms_plain_s, _ = run(False, spp, 4, record=False)
    spp_p = max(1, int(round(spp * ms_cache / ms_plain_s)))
    ms_c, curve_c = run(True, spp, steps)
    ms_p, curve_p = run(False, spp_p, steps)
    return {"workload": f"{n_cams} views x {R}^2 in one launch, depth {D} RR{RR}, {tex_size}^2x3 "
                        f"texture + roughness, {steps} Adam steps lr {lr}; target: random texture "
                        f"of 64x64 cells, roughness 0.2, {target_spp} spp",
            "cache": {"spp": spp, "ms_per_step": round(ms_c, 2), "warmup_frames": warmup_frames,
                      "train_paths_per_step": 65536, "curve": curve_c},
            "plain_matched_time": {"spp": spp_p, "ms_per_step": round(ms_p, 2), "curve": curve_p}}


def cpu_model():
    """The host CPU's model name (first processor entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(sc, R, SPP, D, budget_s):
    """FP64 oracle on a bounded, seeded sample of the workload's pixels:
    primal (seed A) + adjoint (seed B) per pixel, all host threads."""
    import oracle
    orc = oracle.OracleScene(sc)
    threads = oracle.n_threads_default()
    rng = np.random.default_rng(1284)
    n = 256
    total_t, total_pix = 0.0, 0
    while True:
        n = min(n, R * R)
        ids = rng.choice(R * R, n, replace=False).astype(np.int64)
        adj = rng.normal(size=(n, 3)) * 1e-6
        t = time.perf_counter()
        orc.render(spp=SPP, max_depth=D, seed=1, pixel_ids=ids, threads=threads)
        orc.adjoint(adj, spp=SPP, max_depth=D, seed=2, pixel_ids=ids, threads=threads)
        dt = time.perf_counter() - t
        total_t += dt
        total_pix += n
        # the whole image takes the oracle only a few seconds, so batches go on
        # (each of distinct pixels) until about two thirds of the budget
        if total_t >= 2.0 * budget_s / 3.0:
            break
        # next batch sized to land near the budget
        n = int(max(256, n * (budget_s - total_t) / max(dt, 1e-3)))
    return {"value": round(total_pix * SPP / total_t / 1e6, 5), "unit": "Msamples/s",
            "cores": threads, "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"{total_pix} random pixels (batches of distinct pixels) x {SPP} spp of "
                      f"the same scene/texture (primal + reverse-sweep adjoint), {total_t:.1f} s"}


if __name__ == "__main__":
    main()
