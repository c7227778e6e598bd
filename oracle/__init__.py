"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

The oracle is the plain, slow, obviously-correct reference implementation the
HIP library is checked against.  Only the tests, the smoke check and the
bench's CPU-baseline leg use it; the product path never imports it.  It shares
no code with the HIP library: it reads the same seeded scene arrays produced
by ``scenes`` and nothing else.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

_c_int = ctypes.c_int
_c_i64 = ctypes.c_int64
_c_u32 = ctypes.c_uint32
_c_u64 = ctypes.c_uint64
_c_dbl = ctypes.c_double
_vp = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with the host compiler (IEEE double, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread",
                               "-fno-fast-math", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.oracle_scene_new.restype = _vp
        L.oracle_scene_free.argtypes = [_vp]
        L.oracle_scene_accel.argtypes = [_vp, _c_int]
        L.oracle_scene_eps.restype = _c_dbl
        L.oracle_scene_eps.argtypes = [_vp]
        L.oracle_env_pdf.restype = _c_dbl
        L.oracle_fresnel.restype = _c_dbl
        L.oracle_fresnel.argtypes = [_c_dbl, _c_dbl]
        L.oracle_loss_l2.restype = _c_dbl
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_vp) if a is not None else None


def n_threads_default() -> int:
    return max(1, min(os.cpu_count() or 1, 64))


def cam_array(cams) -> np.ndarray:
    out = np.zeros((len(cams), 12), np.float64)
    for i, c in enumerate(cams):
        out[i, 0:3] = c.origin
        out[i, 3:6] = c.target
        out[i, 6:9] = c.up
        out[i, 9] = c.fov_y_deg
        out[i, 10] = c.width
        out[i, 11] = c.height
    return out


# Scenes with at least this many triangles get the oracle's bounding-volume
# hierarchy by default (it returns what the loop over all triangles returns).
ACCEL_MIN_TRIANGLES = 4096


class OracleScene:
    """The oracle's own copy of a ``scenes.Scene`` (widened to FP64).

    accel: None = hierarchy from ACCEL_MIN_TRIANGLES triangles on; True /
    False = force it on / off (every query then loops over all triangles)."""

    def __init__(self, sc, accel: Optional[bool] = None):
        L = lib()
        self.sc = sc
        self._keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dt)
            self._keep.append(a)
            return _p(a)

        tw = np.array([s[1] for s in sc.tex_shapes] or [0], np.int32)
        th = np.array([s[0] for s in sc.tex_shapes] or [0], np.int32)
        env = sc.envmap
        self.h = L.oracle_scene_new(
            _c_int(sc.positions.shape[0]), arr(sc.positions, np.float32), arr(sc.uvs, np.float32),
            _c_int(sc.n_triangles), arr(sc.indices, np.int32), arr(sc.tri_material, np.int32),
            arr(sc.tri_emitter, np.int32), _c_int(sc.n_materials), arr(sc.mat_type, np.int32),
            arr(sc.mat_texture, np.int32), arr(sc.mat_rough_slot, np.int32),
            arr(sc.mat_albedo, np.float32), arr(sc.mat_alpha, np.float32),
            arr(sc.mat_f0, np.float32), arr(sc.mat_eta, np.float32),
            arr(sc.mat_opacity, np.float32), _c_int(sc.n_emitters), arr(sc.em_type, np.int32),
            arr(sc.em_p0, np.float32), arr(sc.em_e1, np.float32), arr(sc.em_e2, np.float32),
            arr(sc.em_radiance, np.float32), _c_int(len(sc.tex_shapes)), arr(tw, np.int32),
            arr(th, np.int32), _c_int(len(sc.roughness)),
            arr(env, np.float32) if env is not None else None,
            _c_int(0 if env is None else env.shape[1]), _c_int(0 if env is None else env.shape[0]))
        if not self.h:
            raise ValueError("oracle rejected the scene")
        self._keep = []  # the oracle copied everything
        self.accel = bool(sc.n_triangles >= ACCEL_MIN_TRIANGLES) if accel is None else bool(accel)
        L.oracle_scene_accel(_vp(self.h), _c_int(1 if self.accel else 0))

    def __del__(self):
        if getattr(self, "h", None):
            lib().oracle_scene_free(_vp(self.h))
            self.h = None

    @property
    def eps(self) -> float:
        return lib().oracle_scene_eps(_vp(self.h))

    # -- parameters --------------------------------------------------------
    def _params(self, textures, roughness):
        textures = self.sc.textures if textures is None else textures
        roughness = self.sc.roughness if roughness is None else roughness
        texs = [np.ascontiguousarray(t, np.float32) for t in textures]
        ptrs = (_vp * max(1, len(texs)))(*[_p(t) for t in texs])
        rough = np.ascontiguousarray(roughness, np.float32)
        if rough.size == 0:
            rough = np.zeros(1, np.float32)
        return texs, ptrs, rough

    # -- queries -------------------------------------------------------------
    def render(self, cams=None, spp=4, max_depth=3, rr_depth=1 << 30, flags=0, seed=1,
               pixel_ids: Optional[np.ndarray] = None, textures=None, roughness=None,
               threads: Optional[int] = None, ambiguity: bool = False):
        """Pixel estimates.  Full image [n_cams,H,W,3] if pixel_ids is None,
        else [len(pixel_ids),3].  With ambiguity=True also returns, per pixel,
        the number of samples with a discrete decision within FP32 reach."""
        cams = self.sc.cameras if cams is None else cams
        ca = cam_array(cams)
        W, H = cams[0].width, cams[0].height
        full = pixel_ids is None
        if full:
            pixel_ids = np.arange(len(cams) * W * H, dtype=np.int64)
        pixel_ids = np.ascontiguousarray(pixel_ids, np.int64)
        out = np.zeros((pixel_ids.size, 3), np.float64)
        amb = np.zeros(pixel_ids.size, np.int32) if ambiguity else None
        texs, tptr, rough = self._params(textures, roughness)
        lib().oracle_render(_vp(self.h), tptr, _p(rough), _p(ca), _c_int(len(cams)), _c_int(spp),
                            _c_int(max_depth), _c_int(rr_depth), _c_u32(flags), _c_u64(seed),
                            _c_i64(pixel_ids.size), _p(pixel_ids),
                            _c_int(threads or n_threads_default()), _p(out), _p(amb))
        if full:
            out = out.reshape(len(cams), H, W, 3)
            if ambiguity:
                amb = amb.reshape(len(cams), H, W)
        return (out, amb) if ambiguity else out

    def radiance(self, o, d, spp=16, max_depth=3, rr_depth=1 << 30, flags=0, seed=1,
                 textures=None, roughness=None, threads=None) -> np.ndarray:
        o = np.ascontiguousarray(o, np.float64).reshape(-1, 3)
        d = np.ascontiguousarray(d, np.float64).reshape(-1, 3)
        out = np.zeros((o.shape[0], 3), np.float64)
        texs, tptr, rough = self._params(textures, roughness)
        lib().oracle_radiance(_vp(self.h), tptr, _p(rough), _c_i64(o.shape[0]), _p(o), _p(d),
                              _c_int(spp), _c_int(max_depth), _c_int(rr_depth), _c_u32(flags),
                              _c_u64(seed), _c_int(threads or n_threads_default()), _p(out))
        return out

    def adjoint(self, adj, cams=None, spp=4, max_depth=3, rr_depth=1 << 30, flags=0, seed=2,
                pixel_ids=None, mode=0, textures=None, roughness=None, threads=None):
        """Gradient of sum_p <adj_p, I_p>: returns (list of texture grads, roughness grad)."""
        cams = self.sc.cameras if cams is None else cams
        ca = cam_array(cams)
        W, H = cams[0].width, cams[0].height
        adj = np.asarray(adj, np.float64)
        if pixel_ids is None:
            pixel_ids = np.arange(len(cams) * W * H, dtype=np.int64)
            adj = adj.reshape(-1, 3)
        pixel_ids = np.ascontiguousarray(pixel_ids, np.int64)
        adj = np.ascontiguousarray(adj.reshape(-1, 3), np.float64)
        assert adj.shape[0] == pixel_ids.size
        texs, tptr, rough = self._params(textures, roughness)
        gtex = [np.zeros(t.shape, np.float64) for t in texs]
        gptr = (_vp * max(1, len(gtex)))(*[_p(g) for g in gtex])
        grough = np.zeros(max(1, len(self.sc.roughness)), np.float64)
        lib().oracle_adjoint(_vp(self.h), tptr, _p(rough), _p(ca), _c_int(len(cams)), _c_int(spp),
                             _c_int(max_depth), _c_int(rr_depth), _c_u32(flags), _c_u64(seed),
                             _c_i64(pixel_ids.size), _p(pixel_ids), _p(adj), _c_int(mode),
                             _c_int(threads or n_threads_default()), gptr, _p(grough))
        return gtex, grough[:len(self.sc.roughness)]

    def jvp(self, tex_tangents, rough_tangent=None, cams=None, spp=4, max_depth=3, rr_depth=1 << 30,
            flags=0, seed=2, pixel_ids=None, textures=None, roughness=None, threads=None):
        """Forward-mode image derivative along (texture tangents, roughness
        tangent): [n_cams, H, W, 3], or [n, 3] for given pixel ids."""
        cams = self.sc.cameras if cams is None else cams
        ca = cam_array(cams)
        W, H = cams[0].width, cams[0].height
        full = pixel_ids is None
        if full:
            pixel_ids = np.arange(len(cams) * W * H, dtype=np.int64)
        pixel_ids = np.ascontiguousarray(pixel_ids, np.int64)
        texs, tptr, rough = self._params(textures, roughness)
        tt = [None if t is None else np.ascontiguousarray(t, np.float64) for t in tex_tangents]
        ttp = (_vp * max(1, len(tt)))(*[None if t is None else _p(t) for t in tt])
        rt = None if rough_tangent is None else np.ascontiguousarray(rough_tangent, np.float64)
        out = np.zeros((pixel_ids.size, 3))
        lib().oracle_jvp(_vp(self.h), tptr, _p(rough), _p(ca), _c_int(len(cams)), _c_int(spp),
                         _c_int(max_depth), _c_int(rr_depth), _c_u32(flags), _c_u64(seed), ttp,
                         None if rt is None else _p(rt), _c_i64(pixel_ids.size), _p(pixel_ids),
                         _c_int(threads or n_threads_default()), _p(out))
        return out.reshape(len(cams), H, W, 3) if full else out

    def trace(self, o, d, tmin=None, tmax=None, any_hit=False, threads=None):
        """Brute-force ray queries: (prim, t, bary[3], ambiguous)."""
        o = np.ascontiguousarray(o, np.float64).reshape(-1, 3)
        d = np.ascontiguousarray(d, np.float64).reshape(-1, 3)
        n = o.shape[0]
        tmin = np.zeros(n) if tmin is None else np.ascontiguousarray(np.broadcast_to(tmin, (n,)), np.float64)
        tmax = np.full(n, np.inf) if tmax is None else np.ascontiguousarray(np.broadcast_to(tmax, (n,)), np.float64)
        prim = np.zeros(n, np.int32)
        t = np.zeros(n, np.float64)
        b = np.zeros((n, 3), np.float64)
        amb = np.zeros(n, np.int32)
        lib().oracle_trace(_vp(self.h), _c_i64(n), _p(o), _p(d), _p(tmin), _p(tmax),
                           _c_int(1 if any_hit else 0), _c_int(threads or n_threads_default()),
                           _p(prim), _p(t), _p(b), _p(amb))
        return prim, t, b, amb.astype(bool)

    def ao(self, o, d, n_ao=128, seed=1, threads=None):
        o = np.ascontiguousarray(o, np.float64).reshape(-1, 3)
        d = np.ascontiguousarray(d, np.float64).reshape(-1, 3)
        out = np.zeros(o.shape[0], np.float64)
        lib().oracle_ao(_vp(self.h), _c_i64(o.shape[0]), _p(o), _p(d), _c_int(n_ao), _c_u64(seed),
                        _c_int(threads or n_threads_default()), _p(out))
        return out

    def env_pdf(self, d):
        d = np.ascontiguousarray(d, np.float64)
        return lib().oracle_env_pdf(_vp(self.h), _p(d))

    def env_sample(self, u1, u2):
        d = np.zeros(3)
        ok = lib().oracle_env_sample(_vp(self.h), _c_dbl(u1), _c_dbl(u2), _p(d))
        return bool(ok), d

    def env_lookup(self, d):
        d = np.ascontiguousarray(d, np.float64)
        out = np.zeros(3)
        lib().oracle_env_lookup(_vp(self.h), _p(d), _p(out))
        return out


# -- stand-alone pieces --------------------------------------------------------

def philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, np.uint32).reshape(-1, 2)
    out = np.zeros_like(ctr)
    lib().oracle_philox(_c_i64(ctr.shape[0]), _p(ctr), _p(key), _p(out))
    return out


def bsdf_eval(type_, wi, wo, albedo=(0.5, 0.5, 0.5), alpha=0.3, f0=(0.9, 0.9, 0.9), eta=1.5):
    a = np.ascontiguousarray(albedo, np.float64)
    f0 = np.ascontiguousarray(f0, np.float64)
    wi = np.ascontiguousarray(wi, np.float64)
    wo = np.ascontiguousarray(wo, np.float64)
    f = np.zeros(3)
    pdf = np.zeros(1)
    dalb = np.zeros(3)
    dal = np.zeros(3)
    lib().oracle_bsdf_eval(_c_int(type_), _p(a), _c_dbl(alpha), _p(f0), _c_dbl(eta), _p(wi),
                           _p(wo), _p(f), _p(pdf), _p(dalb), _p(dal))
    return f, float(pdf[0]), dalb, dal


def bsdf_sample(type_, wi, u1, u2, ulobe, albedo=(0.5, 0.5, 0.5), alpha=0.3,
                f0=(0.9, 0.9, 0.9), eta=1.5):
    a = np.ascontiguousarray(albedo, np.float64)
    f0 = np.ascontiguousarray(f0, np.float64)
    wi = np.ascontiguousarray(wi, np.float64)
    wo = np.zeros(3)
    f = np.zeros(3)
    pdf = np.zeros(1)
    ok = lib().oracle_bsdf_sample(_c_int(type_), _p(a), _c_dbl(alpha), _p(f0), _c_dbl(eta),
                                  _p(wi), _c_dbl(u1), _c_dbl(u2), _c_dbl(ulobe), _p(wo), _p(f),
                                  _p(pdf))
    return bool(ok), wo, f, float(pdf[0])


def ggx_terms(alpha, cos_m, cos_v):
    out = np.zeros(6)
    lib().oracle_ggx_terms(_c_dbl(alpha), _c_dbl(cos_m), _c_dbl(cos_v), _p(out))
    return dict(D=out[0], dlnD=out[1], dlnD_cs=out[2], G1=out[3], dlnG1=out[4], dlnG1_cs=out[5])


def ggx_sample(alpha, u1, u2):
    m = np.zeros(3)
    lib().oracle_ggx_sample(_c_dbl(alpha), _c_dbl(u1), _c_dbl(u2), _p(m))
    return m


def fresnel(cos_i, eta):
    return lib().oracle_fresnel(cos_i, eta)


def frame(n):
    n = np.ascontiguousarray(n, np.float64)
    s = np.zeros(3)
    t = np.zeros(3)
    lib().oracle_frame(_p(n), _p(s), _p(t))
    return s, t


def camera_dirs(cam, px, py):
    ca = cam_array([cam])
    px = np.ascontiguousarray(px, np.float64)
    py = np.ascontiguousarray(py, np.float64)
    out = np.zeros((px.size, 3))
    lib().oracle_camera_dirs(_p(ca), _c_i64(px.size), _p(px), _p(py), _p(out))
    return out


def loss_l2(img, target):
    img = np.ascontiguousarray(img, np.float64).reshape(-1)
    target = np.ascontiguousarray(target, np.float64).reshape(-1)
    adj = np.zeros_like(img)
    loss = lib().oracle_loss_l2(_c_i64(img.size), _p(img), _p(target), _p(adj))
    return loss, adj


def adam(p, g, m, v, lr, b1, b2, eps, t, lo=-np.inf, hi=np.inf):
    """In-place Adam step on float64 arrays."""
    lib().oracle_adam(_c_i64(p.size), _p(p), _p(np.ascontiguousarray(g, np.float64)), _p(m), _p(v),
                      _c_dbl(lr), _c_dbl(b1), _c_dbl(b2), _c_dbl(eps), _c_int(t), _c_dbl(lo),
                      _c_dbl(hi))


# -- radiance cache ------------------------------------------------------------

def nrc_cfg_array(cfg) -> np.ndarray:
    return np.array([cfg["levels"], cfg["features"], cfg["log2_table"], cfg["base_res"],
                     cfg["max_res"], *cfg["bbox_lo"], *cfg["bbox_hi"]], np.float64)


def sh16(d):
    out = np.zeros(16)
    lib().oracle_sh16(_p(np.ascontiguousarray(d, np.float64)), _p(out))
    return out


def level_res(cfg, l):
    return lib().oracle_level_res(_p(nrc_cfg_array(cfg)), _c_int(l))


def grid_corners(cfg, l, xn):
    idx = np.zeros(8, np.uint32)
    w = np.zeros(8)
    lib().oracle_grid_corners(_p(nrc_cfg_array(cfg)), _c_int(l), _p(np.ascontiguousarray(xn, np.float64)),
                              _p(idx), _p(w))
    return idx, w


def nrc_encode(feat, cfg, grid):
    """feat [n,13] raw records -> [n,80] network inputs (FP64)."""
    feat = np.ascontiguousarray(feat, np.float64).reshape(-1, 13)
    g = np.ascontiguousarray(grid, np.float32).reshape(-1)
    out = np.zeros((feat.shape[0], 80))
    lib().oracle_nrc_encode(_c_i64(feat.shape[0]), _p(feat), _p(nrc_cfg_array(cfg)), _p(g), _p(out))
    return out


def nrc_grid_backward(feat, cfg, dfeat, grad=None):
    feat = np.ascontiguousarray(feat, np.float64).reshape(-1, 13)
    dfeat = np.ascontiguousarray(dfeat, np.float64).reshape(-1, 80)
    if grad is None:
        grad = np.zeros(cfg["levels"] * (1 << cfg["log2_table"]) * cfg["features"])
    lib().oracle_nrc_grid_backward(_c_i64(feat.shape[0]), _p(feat), _p(nrc_cfg_array(cfg)), _p(dfeat),
                                   _p(grad))
    return grad


def mlp_num_weights() -> int:
    return lib().oracle_mlp_num_weights()


def mlp_forward(x, W, emu=False, threads=None):
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 80)
    W = np.ascontiguousarray(W, np.float64)
    y = np.zeros((x.shape[0], 3))
    lib().oracle_mlp_forward(_c_i64(x.shape[0]), _p(x), _p(W), _c_int(1 if emu else 0),
                             _c_int(threads or n_threads_default()), _p(y))
    return y


def mlp_backward(x, W, dy, emu=False):
    """(dW, dx) of sum_i <dy_i, y_i>."""
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 80)
    W = np.ascontiguousarray(W, np.float64)
    dy = np.ascontiguousarray(dy, np.float64).reshape(-1, 3)
    dW = np.zeros_like(W)
    dx = np.zeros_like(x)
    lib().oracle_mlp_backward(_c_i64(x.shape[0]), _p(x), _p(W), _p(dy), _c_int(1 if emu else 0),
                              _p(dW), _p(dx))
    return dW, dx


def mlp_term_magnitudes(x, W, dy, emu=False):
    """(aW, adx, ay): for every weight gradient, input gradient and output
    entry, the sum of the magnitudes of the terms it is summed from (the
    scale of a floating-point sum's rounding error), with the activations
    and backpropagated signals of mlp_backward.  For tolerances only."""
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 80)
    W = np.ascontiguousarray(W, np.float64)
    dy = np.ascontiguousarray(dy, np.float64).reshape(-1, 3)
    aW = np.zeros_like(W)
    adx = np.zeros_like(x)
    ay = np.zeros((x.shape[0], 3))
    lib().oracle_mlp_term_magnitudes(_c_i64(x.shape[0]), _p(x), _p(W), _p(dy),
                                     _c_int(1 if emu else 0), _p(aW), _p(adx), _p(ay))
    return aW, adx, ay


def rel_l2(y, t):
    y = np.ascontiguousarray(y, np.float64)
    t = np.ascontiguousarray(t, np.float64)
    dy = np.zeros_like(y)
    lib().oracle_rel_l2.restype = _c_dbl
    loss = lib().oracle_rel_l2(_c_i64(y.size // 3), _p(y), _p(t), _p(dy))
    return loss, dy


def _render_cached(self, cfg, grid, W, K=3, cams=None, spp=4, max_depth=6, rr_depth=3, flags=0,
                   seed=1, pixel_ids=None, emu=True, textures=None, roughness=None, threads=None,
                   ambiguity=False):
    cams = self.sc.cameras if cams is None else cams
    ca = cam_array(cams)
    Wd, H = cams[0].width, cams[0].height
    full = pixel_ids is None
    if full:
        pixel_ids = np.arange(len(cams) * Wd * H, dtype=np.int64)
    pixel_ids = np.ascontiguousarray(pixel_ids, np.int64)
    out = np.zeros((pixel_ids.size, 3))
    amb = np.zeros(pixel_ids.size, np.int32) if ambiguity else None
    texs, tptr, rough = self._params(textures, roughness)
    g = np.ascontiguousarray(grid, np.float32).reshape(-1)
    Wv = np.ascontiguousarray(W, np.float64)
    lib().oracle_render_cached(_vp(self.h), tptr, _p(rough), _p(ca), _c_int(len(cams)), _c_int(spp),
                               _c_int(max_depth), _c_int(rr_depth), _c_u32(flags), _c_u64(seed),
                               _c_int(K), _p(nrc_cfg_array(cfg)), _p(g), _p(Wv),
                               _c_int(1 if emu else 0), _c_i64(pixel_ids.size), _p(pixel_ids),
                               _c_int(threads or n_threads_default()), _p(out), _p(amb))
    if full:
        out = out.reshape(len(cams), H, Wd, 3)
        if ambiguity:
            amb = amb.reshape(len(cams), H, Wd)
    return (out, amb) if ambiguity else out


def _train_records(self, n_paths, K=3, cams=None, max_depth=6, rr_depth=3, flags=0, seed=7,
                   textures=None, roughness=None, threads=None, extra=False):
    """(features [n,13], targets [n,3], valid [n] bool, ambiguous [n] bool);
    with extra=True also (beta, L_before, L_total) [n,3]."""
    cams = self.sc.cameras if cams is None else cams
    ca = cam_array(cams)
    feat = np.zeros((n_paths, 13))
    tgt = np.zeros((n_paths, 3))
    valid = np.zeros(n_paths, np.int32)
    amb = np.zeros(n_paths, np.int32)
    beta, lat, ltot = np.zeros((n_paths, 3)), np.zeros((n_paths, 3)), np.zeros((n_paths, 3))
    texs, tptr, rough = self._params(textures, roughness)
    lib().oracle_train_records(_vp(self.h), tptr, _p(rough), _p(ca), _c_int(len(cams)),
                               _c_int(max_depth), _c_int(rr_depth), _c_u32(flags), _c_u64(seed),
                               _c_int(K), _c_i64(n_paths), _c_int(threads or n_threads_default()),
                               _p(feat), _p(tgt), _p(valid), _p(amb), _p(beta), _p(lat), _p(ltot))
    if extra:
        return feat, tgt, valid.astype(bool), amb.astype(bool), beta, lat, ltot
    return feat, tgt, valid.astype(bool), amb.astype(bool)


def _train_records_self(self, n_paths, cfg, grid, W, K=5, cams=None, max_depth=6, rr_depth=3, flags=0,
                        seed=7, emu=True, textures=None, roughness=None, threads=None):
    """Self-training records of n_paths paths, K - 1 slots per path (slot
    j (K-1) + k - 1 for vertex k): (features [n(K-1),13], targets [n(K-1),3],
    valid [n(K-1)] bool, ambiguous [n] bool)."""
    cams = self.sc.cameras if cams is None else cams
    ca = cam_array(cams)
    m = n_paths * (K - 1)
    feat, tgt = np.zeros((m, 13)), np.zeros((m, 3))
    valid = np.zeros(m, np.int32)
    amb = np.zeros(n_paths, np.int32)
    texs, tptr, rough = self._params(textures, roughness)
    g = np.ascontiguousarray(grid, np.float32).reshape(-1)
    Wv = np.ascontiguousarray(W, np.float64)
    lib().oracle_train_records_self(_vp(self.h), tptr, _p(rough), _p(ca), _c_int(len(cams)),
                                    _c_int(max_depth), _c_int(rr_depth), _c_u32(flags), _c_u64(seed),
                                    _c_int(K), _p(nrc_cfg_array(cfg)), _p(g), _p(Wv),
                                    _c_int(1 if emu else 0), _c_i64(n_paths),
                                    _c_int(threads or n_threads_default()), _p(feat), _p(tgt),
                                    _p(valid), _p(amb))
    return feat, tgt, valid.astype(bool), amb.astype(bool)


def _adjoint_cached(self, cfg, grid, W, adj, K=3, cams=None, spp=4, max_depth=6, rr_depth=3,
                    flags=0, seed=2, pixel_ids=None, emu=True, textures=None, roughness=None,
                    threads=None, input_grad=False):
    """Gradient of sum_p <adj_p, I_p> for the cached estimator: (list of
    texture grads, roughness grad).  input_grad=False: cache output detached;
    True: also through the network's albedo and roughness inputs."""
    cams = self.sc.cameras if cams is None else cams
    ca = cam_array(cams)
    Wd, H = cams[0].width, cams[0].height
    adj = np.asarray(adj, np.float64)
    if pixel_ids is None:
        pixel_ids = np.arange(len(cams) * Wd * H, dtype=np.int64)
    pixel_ids = np.ascontiguousarray(pixel_ids, np.int64)
    adj = np.ascontiguousarray(adj.reshape(-1, 3), np.float64)
    assert adj.shape[0] == pixel_ids.size
    texs, tptr, rough = self._params(textures, roughness)
    gtex = [np.zeros(t.shape, np.float64) for t in texs]
    gptr = (_vp * max(1, len(gtex)))(*[_p(g) for g in gtex])
    grough = np.zeros(max(1, len(self.sc.roughness)), np.float64)
    g = np.ascontiguousarray(grid, np.float32).reshape(-1)
    Wv = np.ascontiguousarray(W, np.float64)
    lib().oracle_adjoint_cached(_vp(self.h), tptr, _p(rough), _p(ca), _c_int(len(cams)), _c_int(spp),
                                _c_int(max_depth), _c_int(rr_depth), _c_u32(flags), _c_u64(seed),
                                _c_int(K), _p(nrc_cfg_array(cfg)), _p(g), _p(Wv),
                                _c_int(1 if emu else 0), _c_int(1 if input_grad else 0),
                                _c_i64(pixel_ids.size), _p(pixel_ids),
                                _p(adj), _c_int(threads or n_threads_default()), gptr, _p(grough))
    return gtex, grough[:len(self.sc.roughness)]


OracleScene.render_cached = _render_cached
OracleScene.adjoint_cached = _adjoint_cached
OracleScene.train_records = _train_records
OracleScene.train_records_self = _train_records_self
