"""CPU-side checks of the HIP library: it loads, exports every entry point
the header declares, validates arguments before launching, and its host
scene build (binned-SAH BVH and tables) is correct -- checked by walking the
packed device layout in NumPy against the oracle's brute-force hits."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2202_01284_amd as drt
import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "drt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(drt_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert "drt_render_adjoint" in names and len(names) >= 14
    handle = ctypes.CDLL(drt.LIB_PATH)
    for n in names:
        assert hasattr(handle, n), n
    # the binding wraps each of them
    assert set(names) <= set(drt._SIGS)


def test_version_and_error_channel():
    assert b"gfx950" in drt.lib.drt_version()
    st = drt.lib.drt_scene_plan(None, None)
    assert st == -1
    assert b"NULL" in drt.lib.drt_last_error()


def test_invalid_arguments_rejected_before_launch():
    sc = scenes.cornell()
    d = drt.make_desc(sc)
    # bad index
    idx = sc.indices.copy()
    idx[3, 1] = 10 ** 6
    bad = drt.make_desc(scenes.Scene(**{**sc.__dict__, "indices": idx}))
    n = ctypes.c_uint64()
    assert drt.lib.drt_scene_plan(ctypes.byref(bad), ctypes.byref(n)) == -1
    assert b"vertex" in drt.lib.drt_last_error()
    # empty scene
    d2 = drt.make_desc(sc)
    d2.n_triangles = 0
    assert drt.lib.drt_scene_plan(ctypes.byref(d2), ctypes.byref(n)) == -1
    # render on a host-packed scene: wrong state, nothing launched
    buf = np.zeros(drt.scene_plan(sc), np.uint8)
    h = ctypes.c_void_p()
    assert drt.lib.drt_scene_pack(ctypes.byref(d), buf.ctypes.data, buf.size, ctypes.byref(h)) == 0
    p = drt.drt_params()
    cams = drt._cams(sc.cameras)
    o = drt._opts(0, 3, 1 << 30, 1, 0, None)
    assert drt.lib.drt_render_forward(h, ctypes.byref(p), cams, 1, ctypes.byref(o), 1, None) == -4
    assert drt.lib.drt_render_forward(None, ctypes.byref(p), cams, 1, ctypes.byref(o), 1, None) == -1
    assert drt.lib.drt_trace(None, None, 4, 0, None, None) == -1
    assert drt.lib.drt_philox(None, None, 0, None, None) == 0
    a = drt.drt_adam_opts()
    a.lr, a.beta1, a.beta2, a.eps, a.step = 1e-2, 0.9, 0.99, 1e-8, 0
    assert drt.lib.drt_adam_step(1, 1, 1, 1, 4, ctypes.byref(a), None) == -1
    drt.lib.drt_scene_destroy(h)


# ---------------------------------------------------------------------------
# packed BVH walked in NumPy
# ---------------------------------------------------------------------------

NODE = np.dtype([("box", "<f4", (6, 4)), ("child", "<i4", 4), ("count", "<i4", 4)])
TRI = np.dtype([("p", "<f4", 9), ("prim", "<i4"), ("flags", "<i4"), ("pad", "<i4")])


def _box(nd, s):
    return nd["box"][:3, s].copy(), nd["box"][3:, s].copy()


def _unpack(sc):
    buf, info = drt.scene_pack(sc)
    nodes = np.frombuffer(buf[:info["n_nodes"] * 128].tobytes(), NODE)
    off_tris = (max(1, sc.n_triangles) * 128 + 255) // 256 * 256
    tris = np.frombuffer(buf[off_tris:off_tris + 48 * sc.n_triangles].tobytes(), TRI)
    return nodes, tris, info


SHADE = np.dtype([("uv", "<f4", 6), ("material", "<i4"), ("emitter", "<i4"), ("n", "<f4", 3),
                  ("pad", "<i4")])


def _align256(x):
    return (x + 255) // 256 * 256


@pytest.mark.parametrize("name", ["cornell", "zoo", "soup"])
def test_packed_shading_records(name):
    """Shading records by original triangle id: the three uv pairs, material
    and emitter as given, and the unit geometric normal (p1 - p0) x (p2 - p0),
    computed in double and rounded once, so each component lies within one
    float ulp of 1 of the exact value; a zero-area triangle (never reported as
    hit) gets +z."""
    sc = {"cornell": lambda: scenes.cornell(conductor=True), "zoo": scenes.bsdf_zoo,
          "soup": lambda: scenes.triangle_soup(300, seed=4)}[name]()
    buf, info = drt.scene_pack(sc)
    nt = sc.n_triangles
    off_shade = _align256(_align256(max(1, nt) * 128) + 48 * nt)
    sh = np.frombuffer(buf[off_shade:off_shade + 48 * nt].tobytes(), SHADE)
    tri = np.asarray(sc.indices).reshape(-1, 3)
    P = np.asarray(sc.positions, np.float64).reshape(-1, 3)
    c = np.cross(P[tri[:, 1]] - P[tri[:, 0]], P[tri[:, 2]] - P[tri[:, 0]])
    length = np.linalg.norm(c, axis=1)
    ok = length > 0
    assert ok.any()
    np.testing.assert_allclose(sh["n"][ok], c[ok] / length[ok, None], rtol=0, atol=2.0 ** -24)
    assert (sh["n"][~ok] == np.array([0, 0, 1], np.float32)).all()
    np.testing.assert_array_equal(sh["material"], np.asarray(sc.tri_material).reshape(-1))
    np.testing.assert_array_equal(sh["emitter"], np.asarray(sc.tri_emitter).reshape(-1))
    uv = np.asarray(sc.uvs, np.float32).reshape(-1, 2)
    np.testing.assert_array_equal(sh["uv"], uv[tri].reshape(nt, 6))


def _depths(nodes):
    depth = {0: 0}
    for k, nd in enumerate(nodes):
        for s in range(4):
            if nd["count"][s] == 0:
                depth[int(nd["child"][s])] = depth[k] + 1
    return depth


@pytest.mark.parametrize("name", ["soup", "cornell", "zoo", "one", "big"])
def test_packed_bvh_structure(name):
    sc = {"soup": lambda: scenes.triangle_soup(500, seed=2), "cornell": scenes.cornell,
          "zoo": scenes.bsdf_zoo, "one": lambda: scenes.triangle_soup(1, seed=1),
          "big": lambda: scenes.triangle_soup(20000, seed=5)}[name]()
    nodes, tris, info = _unpack(sc)
    assert info["max_depth"] <= 24 and info["n_nodes"] == len(nodes)
    # the traversal stack bound: at most 12 levels of four-wide nodes
    assert max(_depths(nodes).values()) <= 11
    # every triangle referenced by exactly one leaf; boxes contain what they hold
    seen = np.zeros(sc.n_triangles, int)
    P = sc.positions
    for nd in nodes:
        for s in range(4):
            c, n = int(nd["child"][s]), int(nd["count"][s])
            if n < 0:
                continue
            lo, hi = _box(nd, s)
            if n > 0:
                for i in range(c, c + n):
                    seen[tris[i]["prim"]] += 1
                    v = tris[i]["p"].reshape(3, 3)
                    assert (v >= lo).all() and (v <= hi).all()
                    np.testing.assert_array_equal(v, P[sc.indices[tris[i]["prim"]]])
            else:
                ch = nodes[c]
                for s2 in range(4):
                    if ch["count"][s2] >= 0:
                        lo2, hi2 = _box(ch, s2)
                        assert (lo2 >= lo).all() and (hi2 <= hi).all()
    if name == "one":
        assert (seen == 2).all()   # a single triangle sits in both root children
    else:
        assert (seen == 1).all()


def _walk(nodes, tris, o, d):
    """Closest hit by walking the packed BVH (NumPy, FP64 ray-box and
    Moller-Trumbore, ties to the lowest id)."""
    best_t, best = np.inf, -1
    stack = [0]
    inv = 1.0 / np.where(np.abs(d) < 1e-30, 1e-30, d)
    while stack:
        nd = nodes[stack.pop()]
        for s in range(4):
            c, n = int(nd["child"][s]), int(nd["count"][s])
            if n < 0:
                continue
            lo, hi = (x.astype(float) for x in _box(nd, s))
            t0, t1 = (lo - o) * inv, (hi - o) * inv
            tn = max(np.minimum(t0, t1).max(), 0.0)
            tf = min(np.maximum(t0, t1).min(), best_t)
            if tn > tf * (1 + 1e-9):
                continue
            if n == 0:
                stack.append(c)
                continue
            for i in range(c, c + n):
                v = tris[i]["p"].reshape(3, 3).astype(float)
                e1, e2 = v[1] - v[0], v[2] - v[0]
                pv = np.cross(d, e2)
                det = e1 @ pv
                if det == 0:
                    continue
                tv = o - v[0]
                u = tv @ pv / det
                qv = np.cross(tv, e1)
                w = d @ qv / det
                t = e2 @ qv / det
                if u >= 0 and w >= 0 and u + w <= 1 and t > 0:
                    pr = tris[i]["prim"]
                    if t < best_t or (t == best_t and pr < best):
                        best_t, best = t, pr
    return best


@pytest.mark.parametrize("name", ["soup", "zoo"])
def test_packed_bvh_hits_equal_brute_force(name):
    sc = scenes.triangle_soup(300, seed=4) if name == "soup" else scenes.bsdf_zoo()
    nodes, tris, _ = _unpack(sc)
    if name == "soup":
        o, d = scenes.random_rays(300, seed=8)
    else:
        cam = sc.cameras[0]
        rng = np.random.default_rng(3)
        px, py = rng.uniform(0, cam.width, 300), rng.uniform(0, cam.height, 300)
        d = oracle.camera_dirs(cam, px, py)
        o = np.tile(cam.origin, (300, 1))
    orc = oracle.OracleScene(sc)
    prim, _, _, amb = orc.trace(o, d)
    got = np.array([_walk(nodes, tris, o[i].astype(float), d[i].astype(float)) for i in range(len(o))])
    ok = ~amb
    assert ok.mean() > 0.95
    np.testing.assert_array_equal(got[ok], prim[ok])


def test_scene_info_and_env_tables():
    sc = scenes.bsdf_zoo()
    buf, info = drt.scene_pack(sc)
    assert info["n_triangles"] == sc.n_triangles
    assert info["env_width"] == 64 and info["env_height"] == 32
    ext = (sc.positions.max(0) - sc.positions.min(0)).max()
    assert abs(info["eps"] - 1e-4 * ext) < 1e-9
    assert info["device_bytes"] <= drt.scene_plan(sc)


def test_cache_and_jvp_arguments_rejected_before_launch():
    """Argument checks of the radiance-cache and forward-mode entry points
    fail before anything is enqueued (the pointers below are never read)."""
    sc = scenes.cornell()
    cfg = scenes.nrc_config(sc)
    c = drt.nrc_config(cfg)
    fake = 1 << 20                       # non-null, never dereferenced
    n = 1000
    need = int(drt.lib.drt_nrc_train_workspace_bytes(n))
    assert need >= n * 1216
    assert drt.lib.drt_nrc_train_workspace_bytes(-1) == 0
    args = lambda ws, wsb: (ctypes.byref(c), fake, fake, fake, fake, fake, n, ws, wsb,  # noqa: E731
                            fake, fake, fake, None)
    assert drt.lib.drt_nrc_train(*args(fake, need - 1)) == -1          # workspace too small
    assert b"workspace" in drt.lib.drt_last_error()
    assert drt.lib.drt_nrc_train(*args(fake + 4, need)) == -1          # not 16-byte aligned
    assert drt.lib.drt_nrc_train(*args(None, need)) == -1
    bad = drt.nrc_config(dict(cfg, levels=8))
    assert drt.lib.drt_nrc_train(ctypes.byref(bad), fake, fake, fake, fake, fake, n, fake, need,
                                 fake, fake, fake, None) == -5         # unsupported
    bad = drt.nrc_config(dict(cfg, log2_table=30))
    assert drt.lib.drt_nrc_train(ctypes.byref(bad), fake, fake, fake, fake, fake, n, fake, need,
                                 fake, fake, fake, None) != 0
    assert drt.lib.drt_nrc_query_ints(10) == 7 * 10 + 32768
    assert drt.lib.drt_nrc_query_ints(11) == 7 * 11 + 1 + 32768  # pairs start 8-byte aligned
    assert drt.lib.drt_nrc_query_ints(-3) == 0
    # scenes packed on the host are rejected by every rendering entry point
    desc = drt.make_desc(sc)
    size = drt.scene_plan(sc)
    h = ctypes.c_void_p()
    raw = (ctypes.c_ubyte * size)()
    assert drt.lib.drt_scene_pack(ctypes.byref(desc), ctypes.addressof(raw), size, ctypes.byref(h)) == 0
    p = drt.drt_params()
    cams = drt._cams(sc.cameras)
    o = drt._opts(1, 3, 1 << 30, 1, 0, None)
    g = drt.drt_grads()
    assert drt.lib.drt_render_jvp(h, ctypes.byref(p), cams, 1, ctypes.byref(o), ctypes.byref(g),
                                  fake, None) == -4
    assert drt.lib.drt_render_jvp(None, ctypes.byref(p), cams, 1, ctypes.byref(o), ctypes.byref(g),
                                  fake, None) == -1
    assert drt.lib.drt_render_adjoint_cached(h, ctypes.byref(p), cams, 1, ctypes.byref(o),
                                             ctypes.byref(c), fake, fake, fake, fake, fake, 10, fake,
                                             fake, ctypes.byref(g), None, 0, None) == -4
    assert (drt.lib.drt_render_adjoint_cached_hit_bytes(1, 64, 64, 4, 6)
            == 4 * 8 * 8 * 6 * 64 * 16)
    assert drt.lib.drt_render_adjoint_cached_hit_bytes(1, 64, 64, 0, 6) == 0
    # intersection records of the replay: 8x8 workgroups x depth x 64 lanes x 16 B
    # without a device: a 256-byte counter header + one slot per work unit
    # (tile x one of min(spp, 4) sample ranges)
    assert drt.lib.drt_render_adjoint_hit_bytes(1, 1024, 1024, 16, 3) == 256 + 16384 * 4 * 3 * 64 * 16
    assert drt.lib.drt_render_adjoint_hit_bytes(2, 9, 17, 2, 2) == 256 + 2 * 2 * 3 * 2 * 2 * 64 * 16
    assert drt.lib.drt_render_adjoint_hit_bytes(1, 8, 8, 1, 3) == 256 + 3 * 64 * 16
    assert drt.lib.drt_render_adjoint_hit_bytes(1, 0, 8, 4, 3) == 0
    assert drt.lib.drt_render_adjoint_hit_bytes(1, 8, 8, 4, 0) == 0
    assert drt.lib.drt_render_adjoint_hit_bytes(1, 8, 8, 0, 3) == 0
    # sizes that would overflow int64 are 0, not wrapped values
    big = 2 ** 31 - 1
    assert drt.lib.drt_render_adjoint_hit_bytes(32, big, big, 16, 1 << 16) == 0
    assert drt.lib.drt_render_adjoint_hit_bytes(1, 8, 8, 4, (1 << 16) + 1) == 0
    assert drt.lib.drt_render_adjoint_cached_hit_bytes(32, big, big, 1 << 20, 6) == 0
    assert drt.lib.drt_render_adjoint_cached_hit_bytes(33, 8, 8, 4, 6) == 0
    assert drt.lib.drt_render_wavefront_workspace_bytes(2 ** 62) == 0
    assert drt.lib.drt_render_adjoint_wavefront_workspace_bytes(2 ** 62) == 0
    assert drt.lib.drt_render_wavefront_workspace_bytes(2 ** 46) > 0
    assert drt.lib.drt_nrc_train_workspace_bytes(2 ** 62) == 0
    assert drt.lib.drt_nrc_query_ints(2 ** 62) == 0
    assert drt.lib.drt_nrc_collect_self_workspace_bytes(2 ** 40, 2) == 0
    assert drt.lib.drt_render_adjoint_hits(h, ctypes.byref(p), cams, 1, ctypes.byref(o), fake,
                                           ctypes.byref(g), fake, 1 << 30, None) == -4
    # checkpointed calls: sizes grow by 64 B per path and bounce
    assert (drt.lib.drt_render_checkpointed_workspace_bytes(100, 4)
            - drt.lib.drt_render_checkpointed_workspace_bytes(100, 3)) == 100 * 64
    assert drt.lib.drt_render_checkpointed_workspace_bytes(100, 0) == 0
    assert drt.lib.drt_render_checkpointed_forward(h, ctypes.byref(p), cams, 1, ctypes.byref(o), fake,
                                                   1 << 30, fake, None) == -4
    # self-training: workspace sizes, and the scene check before anything else
    wsb = int(drt.lib.drt_nrc_collect_self_workspace_bytes(1000, 5))
    assert wsb >= 1000 * (16 * 4 + 5 * 4 + 3 * 4 + 4 * 3 * 4)
    assert drt.lib.drt_nrc_collect_self_workspace_bytes(1000, 1) == 0
    assert drt.lib.drt_nrc_collect_self_workspace_bytes(1000, 33) == 0
    assert drt.lib.drt_nrc_collect_self_workspace_bytes(-1, 5) == 0
    assert drt.lib.drt_nrc_collect_self(h, ctypes.byref(p), cams, 1, ctypes.byref(o), ctypes.byref(c),
                                        fake, fake, 5, 1000, fake, fake, fake, fake, wsb, None) == -4
    # the cache's training frame: scene state, then the frame and state structs
    fo = drt.drt_nrc_frame_opts(n_paths=1000, self_training=0, step=1, lr=1e-2, beta1=0.9, beta2=0.99,
                                eps=1e-8)
    stt = drt.drt_nrc_state()
    assert drt.lib.drt_nrc_train_frame(h, ctypes.byref(p), cams, 1, ctypes.byref(o), ctypes.byref(c),
                                       ctypes.byref(fo), ctypes.byref(stt), None) == -4
    assert drt.lib.drt_nrc_train_frame(None, ctypes.byref(p), cams, 1, ctypes.byref(o),
                                       ctypes.byref(c), ctypes.byref(fo), ctypes.byref(stt), None) == -1
    # the entry point that allocates nothing checks the scene before anything else
    assert drt.lib.drt_render_adjoint_noalloc(h, ctypes.byref(p), cams, 1, ctypes.byref(o), fake,
                                              ctypes.byref(g), None) == -4
    drt.lib.drt_scene_destroy(h)


@pytest.mark.parametrize("name", ["cornell", "cornell_conductor", "zoo", "soup40", "soup200", "one"])
def test_lds_copy_decision(name):
    """The megakernels keep a per-workgroup LDS copy of a scene's tree,
    triangles, shading records, materials and emitters when they take at
    most 5120 bytes and the tree needs at most 16 traversal-stack entries
    (3 per four-wide level)."""
    sc = {"cornell": scenes.cornell, "cornell_conductor": lambda: scenes.cornell(conductor=True),
          "zoo": scenes.bsdf_zoo, "soup40": lambda: scenes.triangle_soup(40, seed=3),
          "soup200": lambda: scenes.triangle_soup(200, seed=3),
          "one": lambda: scenes.triangle_soup(1, seed=1)}[name]()
    nodes, tris, info = _unpack(sc)
    levels = max(_depths(nodes).values()) + 1
    size = (info["n_nodes"] * 128 + info["n_triangles"] * (48 + 48) + info["n_materials"] * 64 +
            info["n_emitters"] * 96)
    want = int(size <= 5120 and 3 * levels <= 16)
    print(name, size, levels, info["lds_copy"], flush=True)
    assert info["lds_copy"] == want
    if name.startswith("cornell"):
        assert want == 1          # the gradient-step scenes take the LDS copy
    if name in ("zoo", "soup200"):
        assert want == 0
