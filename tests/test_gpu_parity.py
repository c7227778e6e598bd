"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Tolerances (written here, applied element by element):
  images   -- a pixel passes if every channel has |g - o| <= 1e-3 |o| + 1e-6;
              at least 99.9% of pixels pass and the mean absolute error is
              <= 1e-4 (relative to max(1, mean |o|) for scenes brighter than 1).
  gradients -- ||g - o|| <= 1e-3 ||o|| and, per entry with |o| >= 1e-2 max|o|,
              |g - o| <= 1e-3 |o| on at least 99.9% of those entries.
  vs central differences -- |g - fd| <= 2e-2 max(|fd|, 1e-3 max|fd|).
Integer work (Philox words, hit triangle ids) is compared bit-exactly; hit
ids on rays whose answer lies within FP32 reach (the oracle's ambiguity flag)
are excluded and counted.
"""
import math

import numpy as np
import pytest

import oracle
import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2202_01284_amd  # noqa: F401  (fails loudly without libdrt.so)


def _drt():
    import paper_2202_01284_amd as drt
    return drt


def _params(sc):
    tex = [torch.from_numpy(np.ascontiguousarray(t)).cuda() for t in sc.textures]
    rough = torch.from_numpy(np.ascontiguousarray(sc.roughness)).cuda() if len(sc.roughness) else None
    return tex, rough


def check_image(g, o, what="", amb=None, max_amb_frac=0.25):
    """Image tolerance; pixels with a sample whose discrete decisions lie
    within FP32 reach (amb > 0, from the oracle) are set aside and counted."""
    g = np.asarray(g, np.float64).reshape(-1, 3)
    o = np.asarray(o, np.float64).reshape(-1, 3)
    keep = np.ones(g.shape[0], bool) if amb is None else (np.asarray(amb).reshape(-1) == 0)
    n_amb = int((~keep).sum())
    assert n_amb <= max_amb_frac * keep.size, (what, n_amb)
    g, o = g[keep], o[keep]
    err = np.abs(g - o)
    ok = (err <= 1e-3 * np.abs(o) + 1e-6).all(axis=1)
    frac = ok.mean()
    mae = err.mean()
    scale = max(1.0, float(np.abs(o).mean()))
    print(f"{what}: pass {frac:.5f} ({(~ok).sum()} px fail of {ok.size}, {n_amb} set aside), "
          f"mae {mae:.3g}, max err {err.max():.3g}", flush=True)
    assert frac >= 0.999, (what, frac)
    assert mae <= 1e-4 * scale, (what, mae)


def unambiguous_adjoint(orc, adj, amb):
    """Zero the image-space adjoint on pixels the oracle flags (a sample of
    theirs takes a decision within FP32 reach), for both implementations."""
    adj = adj.copy()
    adj.reshape(-1, 3)[np.asarray(amb).reshape(-1) > 0] = 0
    return adj


def check_grad(g, o, what=""):
    g = np.asarray(g, np.float64).reshape(-1)
    o = np.asarray(o, np.float64).reshape(-1)
    no = np.linalg.norm(o)
    assert no > 0, what
    rel = np.linalg.norm(g - o) / no
    big = np.abs(o) >= 1e-2 * np.abs(o).max()
    ok = np.abs(g - o)[big] <= 1e-3 * np.abs(o)[big]
    print(f"{what}: rel l2 {rel:.3g}, big entries {big.sum()}, pass {ok.mean():.5f}", flush=True)
    assert rel <= 1e-3, (what, rel)
    assert ok.mean() >= 0.999, (what, ok.mean())


# ---------------------------------------------------------------------------
# Philox
# ---------------------------------------------------------------------------

def test_philox_bit_exact():
    drt = _drt()
    rng = np.random.default_rng(1)
    n = 1 << 16
    ctr = rng.integers(0, 2 ** 32, (n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, (n, 2), dtype=np.uint64).astype(np.uint32)
    out = drt.philox(torch.from_numpy(ctr.view(np.int32)).cuda(),
                     torch.from_numpy(key.view(np.int32)).cuda())
    got = out.cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got, oracle.philox(ctr, key))


# ---------------------------------------------------------------------------
# traversal: hit ids bit-exact vs brute force
# ---------------------------------------------------------------------------

def _rays_for(sc, n, seed):
    if sc.cameras:
        cam = sc.cameras[0]
        rng = np.random.default_rng(seed)
        px, py = rng.uniform(0, cam.width, n), rng.uniform(0, cam.height, n)
        d = oracle.camera_dirs(cam, px, py).astype(np.float32)
        o = np.tile(np.array(cam.origin, np.float32), (n, 1))
        # secondary rays from points on the first hits, random directions
        return o, d
    return scenes.random_rays(n, seed=seed)


def _degenerate_soup():
    """Random triangles plus degenerate ones: 60 with a repeated vertex and
    20 with all three vertices equal (zero area: never hit), and 60 exact
    duplicates of existing triangles (equal t: the lower id wins)."""
    import dataclasses
    sc = scenes.triangle_soup(600, seed=4)
    P = sc.positions.reshape(-1, 3, 3)
    rep = P[:60].copy()
    rep[:, 1] = rep[:, 0]
    pts = np.repeat(P[60:80, :1], 3, axis=1)
    dup = P[100:160].copy()
    V = np.concatenate([P, rep, pts, dup]).astype(sc.positions.dtype)
    n = V.shape[0]
    return dataclasses.replace(
        sc, positions=V.reshape(-1, 3), uvs=np.zeros((3 * n, 2), sc.uvs.dtype),
        indices=np.arange(3 * n, dtype=sc.indices.dtype).reshape(-1, 3),
        tri_material=np.zeros(n, sc.tri_material.dtype),
        tri_emitter=np.full(n, -1, sc.tri_emitter.dtype), name="degenerate")


@pytest.mark.parametrize("name", ["soup", "cornell", "zoo", "grid", "degenerate"])
def test_trace_closest_and_any_vs_brute_force(name):
    drt = _drt()
    sc = {"soup": lambda: scenes.triangle_soup(2000, seed=3),
          "cornell": scenes.cornell,
          "zoo": scenes.bsdf_zoo,
          "grid": lambda: scenes.procedural(n_grid=64, n_spheres=20, sphere_res=(16, 8),
                                            env_size=(32, 16), n_lights=2, tex_size=16,
                                            width=32, height=32),
          "degenerate": _degenerate_soup}[name]()
    o, d = _rays_for(sc, 4096, seed=5)
    if name == "degenerate":
        # axis-aligned rays from inside the cube (zero direction components)
        rng = np.random.default_rng(17)
        oa = rng.uniform(-1.0, 1.0, (1536, 3)).astype(np.float32)
        da = np.zeros((1536, 3), np.float32)
        da[np.arange(1536), np.arange(1536) % 3] = np.where(np.arange(1536) % 6 < 3, 1.0, -1.0)
        o, d = np.concatenate([o, oa]), np.concatenate([d, da])
    rng = np.random.default_rng(9)
    # add random interior rays
    lo, hi = sc.positions.min(0), sc.positions.max(0)
    o2 = rng.uniform(lo, hi, (4096, 3)).astype(np.float32)
    d2 = rng.normal(size=(4096, 3))
    d2 = (d2 / np.linalg.norm(d2, axis=1, keepdims=True)).astype(np.float32)
    o = np.concatenate([o, o2])
    d = np.concatenate([d, d2])
    d = (d / np.linalg.norm(d.astype(np.float64), axis=1, keepdims=True)).astype(np.float32)
    n = o.shape[0]
    tmax = np.where(np.arange(n) % 3 == 0, 0.7, np.inf).astype(np.float32)
    rays = np.zeros((n, 8), np.float32)
    rays[:, 0:3], rays[:, 4:7], rays[:, 7] = o, d, tmax
    gs = drt.Scene(sc)
    print(name, gs.info, flush=True)
    hits = drt.trace(gs, torch.from_numpy(rays).cuda(), 0).cpu().numpy()
    prim_g = hits[:, 3].copy().view(np.int32)
    orc = oracle.OracleScene(sc)
    prim_o, t_o, _, amb = orc.trace(o.astype(np.float64), d.astype(np.float64), tmax=tmax.astype(np.float64))
    ok = ~amb
    print(f"{name}: ambiguous {amb.sum()} of {n}", flush=True)
    # (the oracle flags every hit on a duplicated triangle: its runner-up is at the same t)
    assert ok.mean() > (0.9 if name == "degenerate" else 0.97)
    np.testing.assert_array_equal(prim_g[ok], prim_o[ok])
    if name == "degenerate":
        # Against the same soup without the extra triangles (a different
        # tree): the closest hit is an order-free minimum, so ids and t agree
        # bit for bit -- no hit on a zero-area triangle, a duplicate never
        # wins over its original -- and so do the any-hit answers.
        clean = drt.Scene(scenes.triangle_soup(600, seed=4))
        rays_t = torch.from_numpy(rays).cuda()
        hc = drt.trace(clean, rays_t, 0).cpu().numpy()
        np.testing.assert_array_equal(hits[:, 3].copy().view(np.int32), hc[:, 3].copy().view(np.int32))
        np.testing.assert_array_equal(hits[:, 0].copy().view(np.int32), hc[:, 0].copy().view(np.int32))
        assert np.isin(prim_g, np.arange(100, 160)).sum() > 0
        ac = drt.trace(clean, rays_t, 1).cpu().numpy()[:, 3].copy().view(np.int32)
        ad = drt.trace(gs, rays_t, 1).cpu().numpy()[:, 3].copy().view(np.int32)
        np.testing.assert_array_equal(ad >= 0, ac >= 0)
    hit = ok & (prim_o >= 0)
    np.testing.assert_allclose(hits[hit, 0], t_o[hit], rtol=2e-5, atol=1e-6)
    anyh = drt.trace(gs, torch.from_numpy(rays).cuda(), 1).cpu().numpy()[:, 3].copy().view(np.int32)
    prim_a, _, _, amb_a = orc.trace(o.astype(np.float64), d.astype(np.float64),
                                    tmax=tmax.astype(np.float64), any_hit=True)
    ok = ~amb_a
    np.testing.assert_array_equal(anyh[ok], prim_a[ok])


# ---------------------------------------------------------------------------
# primal images
# ---------------------------------------------------------------------------

FWD_CASES = {
    "cornell_c1": (lambda: scenes.cornell(), dict(spp=4, max_depth=3)),
    "cornell_tex_conductor": (lambda: scenes.cornell(conductor=True, texture=scenes.random_texture(64)),
                              dict(spp=4, max_depth=4)),
    "furnace_sphere": (lambda: scenes.furnace_sphere(), dict(spp=4, max_depth=3)),
    "furnace_cube_nonee": (lambda: scenes.furnace_cube(), dict(spp=2, max_depth=5, flags=1)),
    "lit_plane": (lambda: scenes.lit_plane(), dict(spp=2, max_depth=3)),
    "zoo_rr": (lambda: scenes.bsdf_zoo(width=64, height=64), dict(spp=4, max_depth=6, rr_depth=3)),
    # odd spp: the primal's two sample halves are 2 + 3 samples
    "cornell_spp5": (lambda: scenes.cornell(conductor=True, texture=scenes.random_texture(64), width=40,
                                            height=24), dict(spp=5, max_depth=3)),
    # long paths: up to 48 vertices, no roulette (paths end by escaping the open front)
    "cornell_deep48": (lambda: scenes.cornell(conductor=True, texture=scenes.random_texture(64), width=16,
                                              height=16), dict(spp=2, max_depth=48)),
}


@pytest.mark.parametrize("case", list(FWD_CASES))
def test_forward_image_parity(case):
    drt = _drt()
    make, kw = FWD_CASES[case]
    sc = make()
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    rr = kw.get("rr_depth", drt.NO_RR)
    img = drt.render_forward(gs, tex, rough, sc.cameras, kw["spp"], kw["max_depth"], rr, seed=1,
                             flags=kw.get("flags", 0)).cpu().numpy()
    ref, amb = oracle.OracleScene(sc).render(spp=kw["spp"], max_depth=kw["max_depth"], rr_depth=rr,
                                             flags=kw.get("flags", 0), seed=1, ambiguity=True)
    check_image(img, ref, case, amb)


def test_forward_multi_camera_parity():
    drt = _drt()
    sc = scenes.cornell(conductor=True, texture=scenes.random_texture(64),
                        cameras=scenes.ring_cameras(3, 40, 24))
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    img = drt.render_forward(gs, tex, rough, sc.cameras, 3, 3, seed=7).cpu().numpy()
    ref, amb = oracle.OracleScene(sc).render(spp=3, max_depth=3, seed=7, ambiguity=True)
    check_image(img, ref, "ring3", amb)


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

ADJ_CASES = {
    "cornell_c1": (lambda: scenes.cornell(texture=scenes.random_texture(64)), dict(spp=4, max_depth=3)),
    "cornell_conductor": (lambda: scenes.cornell(conductor=True, texture=scenes.random_texture(64)),
                          dict(spp=4, max_depth=3)),
    "zoo": (lambda: scenes.bsdf_zoo(width=48, height=48), dict(spp=4, max_depth=6, rr_depth=3)),
    # odd spp and ragged tiles: the adjoint's four sample ranges are 1, 1, 1, 2
    "cornell_spp5": (lambda: scenes.cornell(conductor=True, texture=scenes.random_texture(64), width=40,
                                            height=24), dict(spp=5, max_depth=3)),
    # fewer samples than the four-way split: one range of one sample, direct
    # light only (the camera segment and one next-event segment)
    "cornell_spp1_direct": (lambda: scenes.cornell(conductor=True, texture=scenes.random_texture(64),
                                                   width=24, height=16), dict(spp=1, max_depth=2)),
    # three ranges of one sample each, two scattering bounces past the first
    "cornell_spp3_d4": (lambda: scenes.cornell(conductor=True, texture=scenes.random_texture(64),
                                               width=32, height=20), dict(spp=3, max_depth=4)),
    # long paths (up to 48 vertices, 48 records per lane and sample)
    "cornell_deep48": (lambda: scenes.cornell(conductor=True, texture=scenes.random_texture(64),
                                              width=16, height=16), dict(spp=2, max_depth=48)),
}


@pytest.mark.parametrize("case", list(ADJ_CASES))
def test_adjoint_parity(case):
    drt = _drt()
    make, kw = ADJ_CASES[case]
    sc = make()
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    c = sc.cameras[0]
    adj = np.random.default_rng(5).normal(size=(1, c.height, c.width, 3)).astype(np.float32)
    rr = kw.get("rr_depth", drt.NO_RR)
    orc = oracle.OracleScene(sc)
    _, amb = orc.render(spp=kw["spp"], max_depth=kw["max_depth"], rr_depth=rr, seed=2,
                        ambiguity=True)
    print(case, "pixels set aside:", int((amb > 0).sum()), flush=True)
    adj = unambiguous_adjoint(orc, adj, amb)
    stats = drt.new_stats()
    gt, gr = drt.render_adjoint(gs, tex, rough, sc.cameras, torch.from_numpy(adj).cuda(), kw["spp"],
                                kw["max_depth"], rr, seed=2, stats=stats)
    st = drt.read_stats(stats)
    print(case, st, flush=True)
    ot, orr = orc.adjoint(adj.astype(np.float64), spp=kw["spp"], max_depth=kw["max_depth"],
                          rr_depth=rr, seed=2)
    for i, (g, o) in enumerate(zip(gt, ot)):
        check_grad(g.cpu().numpy(), o, f"{case} texture {i}")
    if len(sc.roughness):
        check_grad(gr.cpu().numpy(), orr, f"{case} roughness")
    # replay residual: the subtraction recovers each sample's full radiance,
    # up to float32 rounding of its few terms (<= 1e-5 of the sample's
    # radiance, whatever the adjoint)
    assert st["lrem_max"] <= 1e-5, st


@pytest.mark.parametrize("case", list(ADJ_CASES))
def test_adjoint_with_intersection_records(case):
    """The replay reading pass A's intersection records: the same gradient
    as the re-tracing replay (up to atomic order), the oracle's within the
    gradient tolerance, no ray traced in the replay, and the replay residual
    as small (the records reproduce pass A's path exactly)."""
    drt = _drt()
    make, kw = ADJ_CASES[case]
    sc = make()
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    c = sc.cameras[0]
    rr = kw.get("rr_depth", drt.NO_RR)
    orc = oracle.OracleScene(sc)
    _, amb = orc.render(spp=kw["spp"], max_depth=kw["max_depth"], rr_depth=rr, seed=2, ambiguity=True)
    adj = unambiguous_adjoint(orc, np.random.default_rng(8).normal(size=(1, c.height, c.width, 3))
                              .astype(np.float32), amb)
    a = torch.from_numpy(adj).cuda()
    hits = drt.adjoint_hit_records(sc.cameras, kw["spp"], kw["max_depth"])
    st_h, st_p = drt.new_stats(), drt.new_stats()
    ht, hr = drt.render_adjoint(gs, tex, rough, sc.cameras, a, kw["spp"], kw["max_depth"], rr, seed=2,
                                stats=st_h, hit_records=hits)
    pt, pr = drt.render_adjoint(gs, tex, rough, sc.cameras, a, kw["spp"], kw["max_depth"], rr, seed=2,
                                stats=st_p)
    st_h, st_p = drt.read_stats(st_h), drt.read_stats(st_p)
    print(case, "rays with records", st_h["rays"], "re-traced", st_p["rays"], flush=True)
    assert 2 * st_h["rays"] == st_p["rays"] and 2 * st_h["shadow_rays"] == st_p["shadow_rays"]
    assert st_h["lrem_max"] <= 1e-5, st_h
    for i, (h, p) in enumerate(zip(ht, pt)):
        h, p = h.cpu().numpy().astype(np.float64), p.cpu().numpy().astype(np.float64)
        r = np.linalg.norm(h - p) / np.linalg.norm(p)
        print(case, f"texture {i}: records vs re-trace rel {r:.3g}", flush=True)
        assert r <= 1e-6
    if len(sc.roughness):
        # one float32 sum of ~1e4 signed terms, pre-summed per workgroup in
        # LDS: the persistent workgroups group the terms differently from the
        # per-tile launch (the texture gradients above show the terms
        # themselves agree), which moves the sum by 1e-6..2e-5 of its value --
        # the most where the terms cancel to a small total (depth 4)
        assert np.allclose(hr.cpu().numpy(), pr.cpu().numpy(), rtol=1e-4, atol=1e-9)
    ot, orr = orc.adjoint(adj.astype(np.float64), spp=kw["spp"], max_depth=kw["max_depth"], rr_depth=rr,
                          seed=2)
    for i, (g, o) in enumerate(zip(ht, ot)):
        check_grad(g.cpu().numpy(), o, f"{case} records texture {i}")
    if len(sc.roughness):
        check_grad(hr.cpu().numpy(), orr, f"{case} records roughness")


def test_intersection_records_multi_camera_ragged_and_size_check():
    """Ragged tiles (W, H not multiples of 8) over three cameras, and a
    record buffer one byte short is refused."""
    drt = _drt()
    sc = scenes.cornell(conductor=True, texture=scenes.random_texture(64),
                        cameras=scenes.ring_cameras(3, 44, 27))
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    a = torch.from_numpy(np.random.default_rng(9).normal(size=(3, 27, 44, 3)).astype(np.float32)).cuda()
    need = int(drt.lib.drt_render_adjoint_hit_bytes(3, 44, 27, 3, 4))
    assert need == 256 + 3 * 6 * 4 * 3 * 4 * 64 * 16   # 216 work units: fewer than resident workgroups
    with pytest.raises(RuntimeError, match="hit_records"):
        drt.render_adjoint(gs, tex, rough, sc.cameras, a, 3, 4, seed=5,
                           hit_records=torch.empty(need - 1, dtype=torch.uint8, device="cuda"))
    ht, hr = drt.render_adjoint(gs, tex, rough, sc.cameras, a, 3, 4, seed=5,
                                hit_records=drt.adjoint_hit_records(sc.cameras, 3, 4))
    pt, pr = drt.render_adjoint(gs, tex, rough, sc.cameras, a, 3, 4, seed=5)
    h, p = ht[0].cpu().numpy().astype(np.float64), pt[0].cpu().numpy().astype(np.float64)
    assert np.linalg.norm(h - p) <= 1e-6 * np.linalg.norm(p)
    assert abs(hr.item() - pr.item()) <= 1e-5 * abs(pr.item())   # summation grouping, as above


def test_adjoint_matches_central_differences_on_gpu():
    """Texel gradients of <adj, I> vs central differences of the GPU primal
    with common random numbers (the adjoint's seed), h = 1e-2."""
    drt = _drt()
    sc = scenes.cornell(texture=scenes.random_texture(64))
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    c = sc.cameras[0]
    adj = np.random.default_rng(6).normal(size=(1, c.height, c.width, 3))
    gt, _ = drt.render_adjoint(gs, tex, rough, sc.cameras,
                               torch.from_numpy(adj.astype(np.float32)).cuda(), 4, 3, seed=2)
    g = gt[0].cpu().numpy().reshape(-1).astype(np.float64)
    rng = np.random.default_rng(10)
    cand = np.flatnonzero(np.abs(g) > 1e-2 * np.abs(g).max())
    pick = rng.choice(cand, 32, replace=False)
    h = 1e-2
    fds = []
    for k in pick:
        tp = tex[0].clone().reshape(-1)
        tm = tex[0].clone().reshape(-1)
        tp[k] += h
        tm[k] -= h
        step = (tp[k].item() - tm[k].item()) / 2
        Ip = drt.render_forward(gs, [tp.reshape(tex[0].shape)], rough, sc.cameras, 4, 3, seed=2)
        Im = drt.render_forward(gs, [tm.reshape(tex[0].shape)], rough, sc.cameras, 4, 3, seed=2)
        dI = Ip.cpu().numpy().astype(np.float64) - Im.cpu().numpy().astype(np.float64)
        fds.append((adj * dI).sum() / (2 * step))
    fds = np.array(fds)
    scale = np.abs(fds).max()
    err = np.abs(g[pick] - fds)
    print("fd max rel err", (err / np.maximum(np.abs(fds), 1e-3 * scale)).max(), flush=True)
    assert np.all(err <= 2e-2 * np.maximum(np.abs(fds), 1e-3 * scale))


# ---------------------------------------------------------------------------
# loss and Adam
# ---------------------------------------------------------------------------

def test_loss_and_adam_vs_oracle():
    drt = _drt()
    rng = np.random.default_rng(2)
    n = 3 * 1000 * 37 + 5    # several blocks and a ragged tail
    img = rng.random(n).astype(np.float32)
    tgt = rng.random(n).astype(np.float32)
    loss, adj = drt.loss_l2(torch.from_numpy(img).cuda(), torch.from_numpy(tgt).cuda())
    lo, ao = oracle.loss_l2(img.astype(np.float64), tgt.astype(np.float64))
    assert abs(loss.item() - lo) <= 1e-6 * lo
    np.testing.assert_allclose(adj.cpu().numpy(), ao, rtol=1e-6, atol=1e-12)
    p = rng.random(n).astype(np.float32)
    g = rng.normal(size=n).astype(np.float32)
    pt, gt = torch.from_numpy(p).cuda(), torch.from_numpy(g).cuda()
    m, v = torch.zeros_like(pt), torch.zeros_like(pt)
    po, mo, vo = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in (1, 2, 3):
        drt.adam_step(pt, gt, m, v, t, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-8, lo=0.0, hi=1.0)
        oracle.adam(po, g.astype(np.float64), mo, vo, 1e-2, 0.9, 0.99, 1e-8, t, 0.0, 1.0)
    np.testing.assert_allclose(pt.cpu().numpy(), po, rtol=0, atol=2e-6)
    # arrays that start one element past a 16-byte boundary take the scalar
    # form; both forms write the FP16 copy
    base = torch.from_numpy(np.concatenate([[0.0], p]).astype(np.float32)).cuda()
    gb = torch.from_numpy(np.concatenate([[0.0], g]).astype(np.float32)).cuda()
    mb, vb = torch.zeros_like(base), torch.zeros_like(base)
    half = torch.empty(n, dtype=torch.float16, device="cuda")
    po, mo, vo = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in (1, 2):
        drt.adam_step(base[1:], gb[1:], mb[1:], vb[1:], t, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-8,
                      lo=0.0, hi=1.0, half_out=half)
        oracle.adam(po, g.astype(np.float64), mo, vo, 1e-2, 0.9, 0.99, 1e-8, t, 0.0, 1.0)
    np.testing.assert_allclose(base[1:].cpu().numpy(), po, rtol=0, atol=2e-6)
    np.testing.assert_array_equal(half.cpu().numpy(), base[1:].cpu().numpy().astype(np.float16))
    half2 = torch.empty(n, dtype=torch.float16, device="cuda")
    drt.adam_step(pt, gt, m, v, 4, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-8, lo=0.0, hi=1.0,
                  half_out=half2)
    np.testing.assert_array_equal(half2.cpu().numpy(), pt.cpu().numpy().astype(np.float16))


def test_empty_and_degenerate_inputs():
    drt = _drt()
    sc = scenes.triangle_soup(1, seed=1)
    gs = drt.Scene(sc)
    # zero rays is a no-op; a one-triangle scene is traversable
    drt.trace(gs, torch.zeros((0, 8), dtype=torch.float32, device="cuda"), 0)
    o, d = scenes.random_rays(64, seed=2)
    rays = np.zeros((64, 8), np.float32)
    rays[:, 0:3], rays[:, 4:7], rays[:, 7] = o, d, np.inf
    hits = drt.trace(gs, torch.from_numpy(rays).cuda(), 0).cpu().numpy()
    prim_o, _, _, amb = oracle.OracleScene(sc).trace(o.astype(np.float64), d.astype(np.float64))
    np.testing.assert_array_equal(hits[~amb, 3].copy().view(np.int32), prim_o[~amb])
    # a 1x1 image, 1 spp, depth 1 (camera ray only)
    sc2 = scenes.cornell(width=1, height=1)
    gs2 = drt.Scene(sc2)
    tex, _ = _params(sc2)
    img = drt.render_forward(gs2, tex, None, sc2.cameras, 1, 1, seed=3).cpu().numpy()
    ref = oracle.OracleScene(sc2).render(spp=1, max_depth=1, seed=3)
    check_image(img, ref, "1x1")
    # zero adjoint: no gradient, nothing traced
    z = torch.zeros((1, 1, 1, 3), dtype=torch.float32, device="cuda")
    gt, _ = drt.render_adjoint(gs2, tex, None, sc2.cameras, z, 1, 3)
    assert float(gt[0].abs().sum()) == 0.0
    # depth 1 (the camera segment alone sees only emission, which no
    # parameter changes): exactly zero gradients by both replays, as the
    # oracle's
    sc3 = scenes.cornell(conductor=True, texture=scenes.random_texture(64), width=16, height=8)
    gs3 = drt.Scene(sc3)
    tex3, rough3 = _params(sc3)
    a3 = torch.from_numpy(np.random.default_rng(5).normal(size=(1, 8, 16, 3)).astype(np.float32)).cuda()
    ot, orr = oracle.OracleScene(sc3).adjoint(a3.cpu().numpy().astype(np.float64), spp=2, max_depth=1,
                                              rr_depth=drt.NO_RR, seed=2)
    assert np.abs(ot[0]).sum() == 0.0 and np.abs(orr).sum() == 0.0
    for hits in (None, drt.adjoint_hit_records(sc3.cameras, 2, 1)):
        gt3, gr3 = drt.render_adjoint(gs3, tex3, rough3, sc3.cameras, a3, 2, 1, seed=2, hit_records=hits)
        assert float(gt3[0].abs().sum()) == 0.0 and float(gr3.abs().sum()) == 0.0
    # invalid arguments are rejected before any launch
    with pytest.raises(drt.DrtError):
        drt.render_forward(gs2, tex, None, sc2.cameras, 0, 3)


def test_binding_refuses_host_and_strided_tensors():
    """The kernels read raw addresses: the binding refuses a host tensor or a
    strided view before anything is launched."""
    drt = _drt()
    sc = scenes.cornell(width=16, height=16)
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    adj = torch.zeros((1, 16, 16, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError, match="hit_records"):
        drt.render_adjoint(gs, tex, rough, sc.cameras, adj, 1, 2,
                           hit_records=torch.empty(1 << 20, dtype=torch.uint8))
    with pytest.raises(ValueError, match="workspace"):
        drt.render_wavefront(gs, tex, rough, sc.cameras, 1, 2,
                             workspace=torch.empty(1 << 20, dtype=torch.uint8))
    ctr = torch.zeros((16, 8), dtype=torch.int32, device="cuda")[:, ::2]
    keys = torch.zeros((16, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError, match="counters"):
        drt.philox(ctr, keys)
    # the same calls with proper buffers go through
    out = drt.philox(ctr.contiguous(), keys)
    assert out.shape == (16, 4)


def test_stats_counters_are_consistent():
    """The stats launches' per-phase counters: each wave-level count is at
    least one active lane and at most 64 per event; the texel scatter counts
    at least one distinct texel per wave-wide scatter; counting changes no
    result (image and gradients bit-identical to the launch without it)."""
    drt = _drt()
    sc = scenes.bsdf_zoo(width=48, height=40)
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    kw = dict(spp=3, max_depth=6, rr_depth=3)
    st_f = drt.new_stats()
    img_s = drt.render_forward(gs, tex, rough, sc.cameras, kw["spp"], kw["max_depth"], kw["rr_depth"],
                               seed=4, stats=st_f)
    img = drt.render_forward(gs, tex, rough, sc.cameras, kw["spp"], kw["max_depth"], kw["rr_depth"],
                             seed=4)
    assert torch.equal(img_s, img)
    c = sc.cameras[0]
    adj = torch.from_numpy(np.random.default_rng(6).normal(size=(1, c.height, c.width, 3))
                           .astype(np.float32)).cuda()
    st_a = drt.new_stats()
    for hits in (None, drt.adjoint_hit_records(sc.cameras, kw["spp"], kw["max_depth"])):
        st_a.zero_()
        gt_s, gr_s = drt.render_adjoint(gs, tex, rough, sc.cameras, adj, kw["spp"], kw["max_depth"],
                                        kw["rr_depth"], seed=5, stats=st_a, hit_records=hits)
        gt, gr = drt.render_adjoint(gs, tex, rough, sc.cameras, adj, kw["spp"], kw["max_depth"],
                                    kw["rr_depth"], seed=5, hit_records=hits)
        for a, b in zip(gt_s, gt):
            # float atomics: the same terms, possibly added in another order
            np.testing.assert_allclose(a.cpu().numpy(), b.cpu().numpy(), rtol=1e-5, atol=1e-9)
        for st, what in ((drt.read_stats(st_f), "primal"), (drt.read_stats(st_a), "adjoint")):
            print(what, hits is not None, st, flush=True)
            for lanes, waves in (("nodes", "wave_nodes"), ("tris", "wave_tris"),
                                 ("lane_steps", "wave_steps"), ("vertices", "wave_shade")):
                assert st[waves] <= st[lanes] <= 64 * st[waves], (what, lanes, st)
            assert st["wave_nodes"] > 0 and st["wave_steps"] > 0 and st["wave_shade"] > 0
        st = drt.read_stats(st_a)
        assert 0 < st["tex_keys"] <= st["tex_lanes"], st
        assert drt.read_stats(st_f)["tex_lanes"] == 0


def test_primal_repeats_bit_for_bit():
    """The primal splits a tile's samples over two workgroups that add their
    halves onto a zeroed image: two addends onto zero give the same sum in
    either order, so repeated launches give the same bits (even and odd spp,
    scene in LDS and in device memory, several tiles and a ragged edge)."""
    drt = _drt()
    sc = scenes.cornell(conductor=True, texture=scenes.random_texture(64), width=100, height=60)
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    for flags in (0, drt.FLAG_GLOBAL_SCENE):
        for spp in (16, 15):
            a = drt.render_forward(gs, tex, rough, sc.cameras, spp, 4, 2, seed=11, flags=flags).cpu().numpy()
            assert np.isfinite(a).all() and a.max() > 0
            for _ in range(3):
                b = drt.render_forward(gs, tex, rough, sc.cameras, spp, 4, 2, seed=11, flags=flags).cpu().numpy()
                np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))


def test_lds_scene_copy_equals_device_memory_reads():
    """Scenes that fit the megakernels' per-workgroup LDS copy of the tree
    and triangles (the Cornell scenes) render from it; with
    DRT_FLAG_GLOBAL_SCENE the same kernels read device memory.  The same
    arithmetic on the same data: the primal image is bit-identical, the
    gradients equal up to the order of the float atomics, and the cached
    render equal up to that of its cache terms."""
    drt = _drt()
    sc = scenes.cornell(conductor=True, texture=scenes.random_texture(64), width=40, height=24)
    gs = drt.Scene(sc)
    assert gs.info["n_nodes"] * 128 + gs.info["n_triangles"] * 48 <= 5120
    tex, rough = _params(sc)
    G = drt.FLAG_GLOBAL_SCENE
    a = drt.render_forward(gs, tex, rough, sc.cameras, 5, 4, seed=3).cpu().numpy()
    b = drt.render_forward(gs, tex, rough, sc.cameras, 5, 4, seed=3, flags=G).cpu().numpy()
    np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))
    # forward mode likewise (the tangent image bit-identical)
    tt = [torch.from_numpy(np.random.default_rng(7).normal(size=t.shape).astype(np.float32)).cuda() for t in tex]
    tr = torch.ones_like(rough)
    ja = drt.render_jvp(gs, tex, rough, sc.cameras, 5, 4, seed=8, tan_textures=tt, tan_roughness=tr).cpu().numpy()
    jb = drt.render_jvp(gs, tex, rough, sc.cameras, 5, 4, seed=8, flags=G, tan_textures=tt,
                        tan_roughness=tr).cpu().numpy()
    assert np.abs(ja).max() > 0
    np.testing.assert_array_equal(ja.view(np.uint32), jb.view(np.uint32))
    adj = torch.from_numpy(np.random.default_rng(4).normal(size=(1, 24, 40, 3)).astype(np.float32)).cuda()
    for hits in (None, drt.adjoint_hit_records(sc.cameras, 5, 4)):
        ga, ra = drt.render_adjoint(gs, tex, rough, sc.cameras, adj, 5, 4, seed=6, hit_records=hits)
        gb, rb = drt.render_adjoint(gs, tex, rough, sc.cameras, adj, 5, 4, seed=6, flags=G, hit_records=hits)
        x, y = ga[0].cpu().numpy().astype(np.float64), gb[0].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(x - y) <= 1e-6 * np.linalg.norm(y)
        assert abs(ra.item() - rb.item()) <= 1e-5 * abs(rb.item())
    cfg = scenes.nrc_config(sc)
    W, grid = scenes.nrc_init(cfg, seed=10)
    Wg, gg = torch.from_numpy(W).cuda(), torch.from_numpy(grid.reshape(-1)).cuda()
    ca = drt.render_forward_cached(gs, tex, rough, sc.cameras, cfg, Wg, gg, spp=4, seed=5).cpu().numpy()
    cb = drt.render_forward_cached(gs, tex, rough, sc.cameras, cfg, Wg, gg, spp=4, seed=5,
                                   flags=G).cpu().numpy()
    np.testing.assert_allclose(ca, cb, rtol=1e-5, atol=1e-7)
