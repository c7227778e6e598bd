"""MI355X differentiable path tracer: thin Python binding of the C ABI.

Every step of the rendering path runs in the HIP library ``libdrt.so``
(built for gfx950 by ``paper_2202_01284_amd.build``); this module only
marshals arguments.  PyTorch supplies device memory and the stream.  If the
library is missing the import fails -- there is no fallback.

Functions keep the C names without the ``drt_`` prefix where they wrap one
entry point (``render_forward``, ``render_adjoint``, ``trace``, ``philox``,
``loss_l2``, ``adam_step``, ``scene_upload``); ``RenderFn`` exposes the
primal/adjoint pair as a ``torch.autograd.Function`` (the paper's custom
adjoint, Sec. "Custom adjoints").
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DRT_LIBRARY may name another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("DRT_LIBRARY") or os.path.join(_HERE, "libdrt.so")

MAX_TEXTURES = 8
MAX_CAMERAS = 32
FLAG_NO_NEE = 1
FLAG_CACHE_INPUT_GRAD = 2   # cached adjoint: also through the cache's albedo/roughness inputs
FLAG_GLOBAL_SCENE = 4       # tree and triangles read from device memory even where they fit the LDS copy
STAT_NAMES = ["rays", "shadow_rays", "nodes", "tris", "vertices", "scatter", "lrem_max", "samples",
              "tex_lanes", "tex_keys", "wave_nodes", "wave_tris", "lane_steps", "wave_steps",
              "wave_shade"]

_c_i32 = ctypes.c_int32
_c_u32 = ctypes.c_uint32
_c_i64 = ctypes.c_int64
_c_u64 = ctypes.c_uint64
_c_f = ctypes.c_float
_vp = ctypes.c_void_p


class drt_material(ctypes.Structure):
    _fields_ = [("type", _c_i32), ("texture", _c_i32), ("rough_slot", _c_i32), ("reserved", _c_i32),
                ("albedo", _c_f * 3), ("alpha", _c_f), ("f0", _c_f * 3), ("eta", _c_f),
                ("opacity", _c_f), ("reserved2", _c_f * 3)]


class drt_emitter(ctypes.Structure):
    _fields_ = [("type", _c_i32), ("reserved", _c_i32 * 3), ("p0", _c_f * 3), ("e1", _c_f * 3),
                ("e2", _c_f * 3), ("radiance", _c_f * 3)]


class drt_texture_desc(ctypes.Structure):
    _fields_ = [("width", _c_i32), ("height", _c_i32)]


class drt_scene_desc(ctypes.Structure):
    _fields_ = [("n_vertices", _c_i32), ("n_triangles", _c_i32), ("positions", _vp), ("uvs", _vp),
                ("indices", _vp), ("tri_material", _vp), ("tri_emitter", _vp),
                ("n_materials", _c_i32), ("materials", _vp), ("n_emitters", _c_i32),
                ("emitters", _vp), ("n_textures", _c_i32), ("textures", _vp),
                ("n_roughness", _c_i32), ("envmap", _vp), ("env_width", _c_i32),
                ("env_height", _c_i32)]


class drt_scene_info(ctypes.Structure):
    _fields_ = [("n_nodes", _c_i32), ("n_leaves", _c_i32), ("max_depth", _c_i32),
                ("forced_leaves", _c_i32), ("n_triangles", _c_i32), ("n_materials", _c_i32),
                ("n_emitters", _c_i32), ("n_textures", _c_i32), ("n_roughness", _c_i32),
                ("env_width", _c_i32), ("env_height", _c_i32), ("eps", _c_f),
                ("bounds_lo", _c_f * 3), ("bounds_hi", _c_f * 3), ("device_bytes", _c_u64),
                ("lds_copy", _c_i32)]


class drt_camera(ctypes.Structure):
    _fields_ = [("origin", _c_f * 3), ("target", _c_f * 3), ("up", _c_f * 3), ("fov_y_deg", _c_f),
                ("width", _c_i32), ("height", _c_i32)]


class drt_params(ctypes.Structure):
    _fields_ = [("textures", _vp * MAX_TEXTURES), ("roughness", _vp)]


class drt_grads(ctypes.Structure):
    _fields_ = [("textures", _vp * MAX_TEXTURES), ("roughness", _vp)]


class drt_render_opts(ctypes.Structure):
    _fields_ = [("spp", _c_i32), ("max_depth", _c_i32), ("rr_depth", _c_i32), ("flags", _c_u32),
                ("seed", _c_u64), ("stats", _vp)]


class drt_hit(ctypes.Structure):
    _fields_ = [("t", _c_f), ("b1", _c_f), ("b2", _c_f), ("prim", _c_i32)]


class drt_adam_opts(ctypes.Structure):
    _fields_ = [("lr", _c_f), ("beta1", _c_f), ("beta2", _c_f), ("eps", _c_f), ("step", _c_i32),
                ("lo", _c_f), ("hi", _c_f), ("zero_grad", _c_i32), ("half_out", _vp)]


class drt_nrc_config(ctypes.Structure):
    _fields_ = [("levels", _c_i32), ("features", _c_i32), ("log2_table", _c_i32),
                ("base_res", _c_i32), ("max_res", _c_i32), ("trunc_vertex", _c_i32),
                ("bbox_lo", _c_f * 3), ("bbox_hi", _c_f * 3)]


class drt_nrc_state(ctypes.Structure):
    _fields_ = [("weights", _vp), ("weights_m", _vp), ("weights_v", _vp), ("weights_grad", _vp),
                ("grid", _vp), ("grid_m", _vp), ("grid_v", _vp), ("grid_grad", _vp),
                ("grid_half", _vp), ("records", _vp), ("valid", _vp), ("count", _vp),
                ("train_workspace", _vp), ("train_workspace_bytes", _c_i64),
                ("self_workspace", _vp), ("self_workspace_bytes", _c_i64), ("loss", _vp)]


class drt_nrc_frame_opts(ctypes.Structure):
    _fields_ = [("n_paths", _c_i64), ("self_training", _c_i32), ("step", _c_i32), ("lr", _c_f),
                ("beta1", _c_f), ("beta2", _c_f), ("eps", _c_f)]


# Every entry point of include/drt.h with its ctypes signature.
_SIGS = {
    "drt_last_error": (ctypes.c_char_p, []),
    "drt_version": (ctypes.c_char_p, []),
    "drt_scene_plan": (_c_i32, [ctypes.POINTER(drt_scene_desc), ctypes.POINTER(_c_u64)]),
    "drt_scene_upload": (_c_i32, [ctypes.POINTER(drt_scene_desc), _vp, _c_u64, _vp,
                                  ctypes.POINTER(_vp)]),
    "drt_scene_pack": (_c_i32, [ctypes.POINTER(drt_scene_desc), _vp, _c_u64, ctypes.POINTER(_vp)]),
    "drt_scene_info_get": (_c_i32, [_vp, ctypes.POINTER(drt_scene_info)]),
    "drt_scene_destroy": (_c_i32, [_vp]),
    "drt_render_forward": (_c_i32, [_vp, ctypes.POINTER(drt_params), ctypes.POINTER(drt_camera),
                                    _c_i32, ctypes.POINTER(drt_render_opts), _vp, _vp]),
    "drt_render_wavefront_workspace_bytes": (_c_i64, [_c_i64]),
    "drt_render_wavefront": (_c_i32, [_vp, ctypes.POINTER(drt_params), ctypes.POINTER(drt_camera),
                                      _c_i32, ctypes.POINTER(drt_render_opts), _vp, _c_i64, _vp, _vp]),
    "drt_render_adjoint_wavefront_workspace_bytes": (_c_i64, [_c_i64]),
    "drt_render_adjoint_wavefront": (_c_i32, [_vp, ctypes.POINTER(drt_params), ctypes.POINTER(drt_camera),
                                              _c_i32, ctypes.POINTER(drt_render_opts), _vp,
                                              ctypes.POINTER(drt_grads), _vp, _c_i64, _vp]),
    "drt_render_adjoint_hit_bytes": (_c_i64, [_c_i32, _c_i32, _c_i32, _c_i32, _c_i32]),
    "drt_render_adjoint_hits": (_c_i32, [_vp, ctypes.POINTER(drt_params), ctypes.POINTER(drt_camera),
                                         _c_i32, ctypes.POINTER(drt_render_opts), _vp,
                                         ctypes.POINTER(drt_grads), _vp, _c_i64, _vp]),
    "drt_render_adjoint_noalloc": (_c_i32, [_vp, ctypes.POINTER(drt_params), ctypes.POINTER(drt_camera),
                                            _c_i32, ctypes.POINTER(drt_render_opts), _vp,
                                            ctypes.POINTER(drt_grads), _vp]),
    "drt_render_checkpointed_workspace_bytes": (_c_i64, [_c_i64, _c_i32]),
    "drt_render_checkpointed_forward": (_c_i32, [_vp, ctypes.POINTER(drt_params),
                                                 ctypes.POINTER(drt_camera), _c_i32,
                                                 ctypes.POINTER(drt_render_opts), _vp, _c_i64, _vp,
                                                 _vp]),
    "drt_render_checkpointed_adjoint": (_c_i32, [_vp, ctypes.POINTER(drt_params),
                                                 ctypes.POINTER(drt_camera), _c_i32,
                                                 ctypes.POINTER(drt_render_opts), _vp,
                                                 ctypes.POINTER(drt_grads), _vp, _c_i64, _vp]),
    "drt_render_jvp": (_c_i32, [_vp, ctypes.POINTER(drt_params), ctypes.POINTER(drt_camera), _c_i32,
                                ctypes.POINTER(drt_render_opts), ctypes.POINTER(drt_grads), _vp, _vp]),
    "drt_render_adjoint": (_c_i32, [_vp, ctypes.POINTER(drt_params), ctypes.POINTER(drt_camera),
                                    _c_i32, ctypes.POINTER(drt_render_opts), _vp,
                                    ctypes.POINTER(drt_grads), _vp]),
    "drt_trace": (_c_i32, [_vp, _vp, _c_i64, _c_i32, _vp, _vp]),
    "drt_philox": (_c_i32, [_vp, _vp, _c_i64, _vp, _vp]),
    "drt_loss_workspace_floats": (_c_i64, [_c_i64]),
    "drt_loss_l2": (_c_i32, [_vp, _vp, _c_i64, _vp, _vp, _vp, _vp]),
    "drt_adam_step": (_c_i32, [_vp, _vp, _vp, _vp, _c_i64, ctypes.POINTER(drt_adam_opts), _vp]),
    "drt_nrc_encode": (_c_i32, [ctypes.POINTER(drt_nrc_config), _vp, _vp, _c_i64, _vp, _vp]),
    "drt_nrc_forward": (_c_i32, [_vp, _vp, _c_i64, _vp, _vp]),
    "drt_nrc_grid_backward": (_c_i32, [ctypes.POINTER(drt_nrc_config), _vp, _vp, _c_i64, _vp, _vp]),
    "drt_nrc_backward": (_c_i32, [_vp, _vp, _vp, _c_i64, _vp, _c_i64, _vp, _vp, _vp]),
    "drt_nrc_collect": (_c_i32, [_vp, ctypes.POINTER(drt_params), ctypes.POINTER(drt_camera), _c_i32,
                                 ctypes.POINTER(drt_render_opts), ctypes.POINTER(drt_nrc_config),
                                 _c_i64, _vp, _vp, _vp, _vp]),
    "drt_nrc_collect_self_workspace_bytes": (_c_i64, [_c_i64, _c_i32]),
    "drt_nrc_collect_self": (_c_i32, [_vp, ctypes.POINTER(drt_params), ctypes.POINTER(drt_camera),
                                      _c_i32, ctypes.POINTER(drt_render_opts),
                                      ctypes.POINTER(drt_nrc_config), _vp, _vp, _c_i32, _c_i64, _vp,
                                      _vp, _vp, _vp, _c_i64, _vp]),
    "drt_nrc_train_workspace_bytes": (_c_i64, [_c_i64]),
    "drt_nrc_train": (_c_i32, [ctypes.POINTER(drt_nrc_config), _vp, _vp, _vp, _vp, _vp, _c_i64, _vp,
                               _c_i64, _vp, _vp, _vp, _vp]),
    "drt_render_forward_cached": (_c_i32, [_vp, ctypes.POINTER(drt_params),
                                           ctypes.POINTER(drt_camera), _c_i32,
                                           ctypes.POINTER(drt_render_opts),
                                           ctypes.POINTER(drt_nrc_config), _vp, _vp, _vp, _vp,
                                           _vp, _c_i64, _vp, _vp]),
    "drt_nrc_query_ints": (_c_i64, [_c_i64]),
    "drt_nrc_train_frame": (_c_i32, [_vp, ctypes.POINTER(drt_params), ctypes.POINTER(drt_camera), _c_i32,
                                     ctypes.POINTER(drt_render_opts), ctypes.POINTER(drt_nrc_config),
                                     ctypes.POINTER(drt_nrc_frame_opts), ctypes.POINTER(drt_nrc_state),
                                     _vp]),
    "drt_render_adjoint_cached": (_c_i32, [_vp, ctypes.POINTER(drt_params), ctypes.POINTER(drt_camera),
                                           _c_i32, ctypes.POINTER(drt_render_opts),
                                           ctypes.POINTER(drt_nrc_config), _vp, _vp, _vp, _vp, _vp,
                                           _c_i64, _vp, _vp, ctypes.POINTER(drt_grads), _vp, _c_i64,
                                           _vp]),
    "drt_render_adjoint_cached_hit_bytes": (_c_i64, [_c_i32, _c_i32, _c_i32, _c_i32, _c_i32]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is not built: run paper_2202_01284_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()


class DrtError(RuntimeError):
    pass


def _check(status: int, what: str):
    if status != 0:
        msg = lib.drt_last_error().decode()
        raise DrtError(f"{what} failed ({status}): {msg}")


def _torch():
    import torch
    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t) -> Optional[int]:
    return None if t is None else _dp(t, "tensor")


def _dp(t, what: str) -> int:
    """Device address of a contiguous device tensor.  The kernels read raw
    addresses, so a host tensor or a strided view is rejected here."""
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous device tensor")
    return t.data_ptr()


def _nbytes(t) -> int:
    return t.numel() * t.element_size()


# ---------------------------------------------------------------------------
# scene
# ---------------------------------------------------------------------------

def make_desc(sc):
    """drt_scene_desc over the arrays of a ``scenes.Scene`` (kept alive on the
    returned object)."""
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dt)
        keep.append(a)
        return a.ctypes.data

    mats = (drt_material * sc.n_materials)()
    for i in range(sc.n_materials):
        m = mats[i]
        m.type = int(sc.mat_type[i])
        m.texture = int(sc.mat_texture[i])
        m.rough_slot = int(sc.mat_rough_slot[i])
        m.albedo[:] = [float(x) for x in sc.mat_albedo[i]]
        m.alpha = float(sc.mat_alpha[i])
        m.f0[:] = [float(x) for x in sc.mat_f0[i]]
        m.eta = float(sc.mat_eta[i])
        m.opacity = float(sc.mat_opacity[i])
    ems = (drt_emitter * max(1, sc.n_emitters))()
    for i in range(sc.n_emitters):
        e = ems[i]
        e.type = int(sc.em_type[i])
        e.p0[:] = [float(x) for x in sc.em_p0[i]]
        e.e1[:] = [float(x) for x in sc.em_e1[i]]
        e.e2[:] = [float(x) for x in sc.em_e2[i]]
        e.radiance[:] = [float(x) for x in sc.em_radiance[i]]
    texs = (drt_texture_desc * max(1, len(sc.tex_shapes)))()
    for i, (h, w) in enumerate(sc.tex_shapes):
        texs[i].width = int(w)
        texs[i].height = int(h)
    keep += [mats, ems, texs]
    d = drt_scene_desc()
    d.n_vertices = int(sc.positions.shape[0])
    d.n_triangles = int(sc.n_triangles)
    d.positions = arr(sc.positions, np.float32)
    d.uvs = arr(sc.uvs, np.float32)
    d.indices = arr(sc.indices, np.int32)
    d.tri_material = arr(sc.tri_material, np.int32)
    d.tri_emitter = arr(sc.tri_emitter, np.int32)
    d.n_materials = int(sc.n_materials)
    d.materials = ctypes.addressof(mats)
    d.n_emitters = int(sc.n_emitters)
    d.emitters = ctypes.addressof(ems)
    d.n_textures = len(sc.tex_shapes)
    d.textures = ctypes.addressof(texs)
    d.n_roughness = int(len(sc.roughness))
    if sc.envmap is not None:
        d.envmap = arr(sc.envmap, np.float32)
        d.env_width = int(sc.envmap.shape[1])
        d.env_height = int(sc.envmap.shape[0])
    d._keep = keep
    return d


def scene_plan(sc) -> int:
    d = make_desc(sc)
    n = _c_u64()
    _check(lib.drt_scene_plan(ctypes.byref(d), ctypes.byref(n)), "drt_scene_plan")
    return int(n.value)


def _info(h) -> dict:
    inf = drt_scene_info()
    _check(lib.drt_scene_info_get(h, ctypes.byref(inf)), "drt_scene_info_get")
    out = {}
    for name, _ in drt_scene_info._fields_:
        v = getattr(inf, name)
        out[name] = list(v) if not isinstance(v, (int, float)) else v
    return out


def scene_pack(sc):
    """Host-side build of the scene's device layout: (bytes, info)."""
    d = make_desc(sc)
    n = scene_plan(sc)
    buf = np.zeros(n, np.uint8)
    h = _vp()
    _check(lib.drt_scene_pack(ctypes.byref(d), buf.ctypes.data, n, ctypes.byref(h)), "drt_scene_pack")
    info = _info(h)
    lib.drt_scene_destroy(h)
    return buf[:info["device_bytes"]], info


class Scene:
    """A scene uploaded into a torch-owned device buffer."""

    def __init__(self, sc, device: str = "cuda"):
        torch = _torch()
        self.sc = sc
        d = make_desc(sc)
        n = _c_u64()
        _check(lib.drt_scene_plan(ctypes.byref(d), ctypes.byref(n)), "drt_scene_plan")
        self.buffer = torch.empty(int(n.value) + 256, dtype=torch.uint8, device=device)
        base = self.buffer.data_ptr()
        aligned = (base + 255) & ~255
        h = _vp()
        _check(lib.drt_scene_upload(ctypes.byref(d), aligned, int(n.value), _stream(),
                                    ctypes.byref(h)), "drt_scene_upload")
        self.handle = h
        self.info = _info(h)
        self.tex_shapes = [(int(t[0]), int(t[1]), 3) for t in sc.tex_shapes]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and lib is not None:          # module globals may be gone at interpreter exit
            lib.drt_scene_destroy(h)
            self.handle = None

    @property
    def n_textures(self) -> int:
        return self.info["n_textures"]

    @property
    def n_roughness(self) -> int:
        return self.info["n_roughness"]


def scene_upload(sc, device="cuda") -> Scene:
    return Scene(sc, device)


# ---------------------------------------------------------------------------
# rendering
# ---------------------------------------------------------------------------

def _cams(cams) -> "ctypes.Array":
    arr = (drt_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i].origin[:] = [float(x) for x in c.origin]
        arr[i].target[:] = [float(x) for x in c.target]
        arr[i].up[:] = [float(x) for x in c.up]
        arr[i].fov_y_deg = float(c.fov_y_deg)
        arr[i].width = int(c.width)
        arr[i].height = int(c.height)
    return arr


def _params(scene: Scene, textures, roughness):
    p = drt_params()
    textures = list(textures or [])
    if len(textures) != len(scene.tex_shapes):
        raise ValueError(f"scene has {len(scene.tex_shapes)} textures, got {len(textures)}")
    for i, t in enumerate(textures):
        _expect(t, f"texture {i}", scene.tex_shapes[i])
        p.textures[i] = _dp(t, f"texture {i}")
    if scene.n_roughness > 0:
        if roughness is None or roughness.numel() < scene.n_roughness:
            raise ValueError(f"scene has {scene.n_roughness} roughness slots")
    if roughness is not None and roughness.numel() > 0:
        _expect(roughness, "roughness")
        p.roughness = _dp(roughness, "roughness")
    return p


def _image_shape(cams):
    return (len(cams), cams[0].height, cams[0].width, 3)


def _expect(t, what, shape=None):
    torch = _torch()
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous float32 device tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _opts(spp, max_depth, rr_depth, seed, flags, stats):
    o = drt_render_opts()
    o.spp = int(spp)
    o.max_depth = int(max_depth)
    o.rr_depth = int(rr_depth)
    o.flags = int(flags)
    o.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    o.stats = None if stats is None else _dp(stats, "stats")
    return o


NO_RR = 1 << 30


def render_forward(scene: Scene, textures: Sequence, roughness, cams, spp: int, max_depth: int,
                   rr_depth: int = NO_RR, seed: int = 1, flags: int = 0, stats=None, out=None,
                   stream=None):
    """Image [n_cams, H, W, 3] (float32, device)."""
    torch = _torch()
    W, H = cams[0].width, cams[0].height
    if out is None:
        out = torch.empty((len(cams), H, W, 3), dtype=torch.float32, device=scene.buffer.device)
    _expect(out, "out", _image_shape(cams))
    ca = _cams(cams)
    p = _params(scene, textures, roughness)
    o = _opts(spp, max_depth, rr_depth, seed, flags, stats)
    _check(lib.drt_render_forward(scene.handle, ctypes.byref(p), ca, len(cams), ctypes.byref(o),
                                  _dp(out, "out"), _stream(stream)), "drt_render_forward")
    return out


def render_adjoint(scene: Scene, textures: Sequence, roughness, cams, adj_image, spp: int,
                   max_depth: int, rr_depth: int = NO_RR, seed: int = 2, flags: int = 0,
                   grad_textures=None, grad_roughness=None, stats=None, hit_records=None,
                   stream=None):
    """Adds d<adj, I>/d params into grad_textures / grad_roughness (allocated
    as zeros when not given) and returns them.  With hit_records (a device
    buffer of adjoint_hit_bytes(...) bytes) the replay reads pass A's
    intersections instead of tracing again."""
    torch = _torch()
    _expect(adj_image, "adj_image", _image_shape(cams))
    if grad_textures is None:
        grad_textures = [torch.zeros_like(t) for t in textures]
    if grad_roughness is None and roughness is not None and roughness.numel() > 0:
        grad_roughness = torch.zeros_like(roughness)
    g = drt_grads()
    if len(grad_textures) > len(scene.tex_shapes):
        raise ValueError("more gradient textures than scene textures")
    for i, t in enumerate(grad_textures):
        if t is not None:
            _expect(t, f"grad texture {i}", scene.tex_shapes[i])
            g.textures[i] = _dp(t, f"grad texture {i}")
    if grad_roughness is not None:
        _expect(grad_roughness, "grad roughness")
        if grad_roughness.numel() < scene.n_roughness:
            raise ValueError(f"grad roughness needs {scene.n_roughness} entries")
        g.roughness = _dp(grad_roughness, "grad_roughness")
    ca = _cams(cams)
    p = _params(scene, textures, roughness)
    o = _opts(spp, max_depth, rr_depth, seed, flags, stats)
    if hit_records is not None:
        _check(lib.drt_render_adjoint_hits(scene.handle, ctypes.byref(p), ca, len(cams),
                                           ctypes.byref(o), _dp(adj_image, "adj_image"), ctypes.byref(g),
                                           _dp(hit_records, "hit_records"), _nbytes(hit_records),
                                           _stream(stream)), "drt_render_adjoint_hits")
    else:
        _check(lib.drt_render_adjoint(scene.handle, ctypes.byref(p), ca, len(cams), ctypes.byref(o),
                                      _dp(adj_image, "adj_image"), ctypes.byref(g), _stream(stream)),
               "drt_render_adjoint")
    return grad_textures, grad_roughness


NOALLOC_SCRATCH_BYTES = 256 + (32 << 20)


def render_adjoint_noalloc(scene: Scene, textures: Sequence, roughness, cams, adj_image, spp: int,
                           max_depth: int, grad_textures, grad_roughness=None, rr_depth: int = NO_RR,
                           seed: int = 2, flags: int = 0, stats=None, stream=None):
    """drt_render_adjoint_noalloc: the replay from intersection records with
    the records in the library's own device scratch.  The caller passes the
    gradient buffers (added into); nothing is allocated here or in the
    library."""
    _expect(adj_image, "adj_image", _image_shape(cams))
    g = drt_grads()
    if len(grad_textures) > len(scene.tex_shapes):
        raise ValueError("more gradient textures than scene textures")
    for i, t in enumerate(grad_textures):
        if t is not None:
            _expect(t, f"grad texture {i}", scene.tex_shapes[i])
            g.textures[i] = _dp(t, f"grad texture {i}")
    if grad_roughness is not None:
        _expect(grad_roughness, "grad roughness")
        if grad_roughness.numel() < scene.n_roughness:
            raise ValueError(f"grad roughness needs {scene.n_roughness} entries")
        g.roughness = _dp(grad_roughness, "grad_roughness")
    ca = _cams(cams)
    p = _params(scene, textures, roughness)
    o = _opts(spp, max_depth, rr_depth, seed, flags, stats)
    _check(lib.drt_render_adjoint_noalloc(scene.handle, ctypes.byref(p), ca, len(cams), ctypes.byref(o),
                                          _dp(adj_image, "adj_image"), ctypes.byref(g), _stream(stream)),
           "drt_render_adjoint_noalloc")
    return grad_textures, grad_roughness


def adjoint_hit_records(cams, spp: int, max_depth: int, device="cuda"):
    """Intersection-record buffer for render_adjoint(hit_records=...)."""
    torch = _torch()
    nbytes = int(lib.drt_render_adjoint_hit_bytes(len(cams), cams[0].width, cams[0].height, spp,
                                                  max_depth))
    if nbytes <= 0:
        raise ValueError("no intersection records for these sizes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def render_wavefront(scene: Scene, textures: Sequence, roughness, cams, spp: int, max_depth: int,
                     rr_depth: int = NO_RR, seed: int = 1, flags: int = 0, out=None, workspace=None,
                     stream=None):
    """Primal image [n_cams, H, W, 3] by the wavefront variant (for the
    megakernel-versus-wavefront comparison)."""
    torch = _torch()
    W, H = cams[0].width, cams[0].height
    dev = scene.buffer.device
    if out is None:
        out = torch.empty((len(cams), H, W, 3), dtype=torch.float32, device=dev)
    _expect(out, "out", _image_shape(cams))
    need = int(lib.drt_render_wavefront_workspace_bytes(len(cams) * W * H * spp))
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    ca = _cams(cams)
    p = _params(scene, textures, roughness)
    o = _opts(spp, max_depth, rr_depth, seed, flags, None)
    _check(lib.drt_render_wavefront(scene.handle, ctypes.byref(p), ca, len(cams), ctypes.byref(o),
                                    _dp(workspace, "workspace"), _nbytes(workspace), _dp(out, "out"),
                                    _stream(stream)), "drt_render_wavefront")
    return out


def render_adjoint_wavefront(scene: Scene, textures: Sequence, roughness, cams, adj_image, spp: int,
                             max_depth: int, rr_depth: int = NO_RR, seed: int = 2, flags: int = 0,
                             grad_textures=None, grad_roughness=None, workspace=None, stream=None):
    """The replayed adjoint by the wavefront variant: adds the gradient of
    <adj, I> into grad_textures / grad_roughness and returns them."""
    torch = _torch()
    _expect(adj_image, "adj_image", _image_shape(cams))
    if grad_textures is None:
        grad_textures = [torch.zeros_like(t) for t in textures]
    if grad_roughness is None and roughness is not None and roughness.numel() > 0:
        grad_roughness = torch.zeros_like(roughness)
    g = drt_grads()
    for i, t in enumerate(grad_textures):
        if t is not None:
            _expect(t, f"grad texture {i}", scene.tex_shapes[i])
            g.textures[i] = _dp(t, f"grad texture {i}")
    if grad_roughness is not None:
        _expect(grad_roughness, "grad roughness")
        if grad_roughness.numel() < scene.n_roughness:
            raise ValueError(f"grad roughness needs {scene.n_roughness} entries")
        g.roughness = _dp(grad_roughness, "grad_roughness")
    n = len(cams) * cams[0].width * cams[0].height * spp
    if workspace is None:
        workspace = torch.empty(int(lib.drt_render_adjoint_wavefront_workspace_bytes(n)), dtype=torch.uint8,
                                device=scene.buffer.device)
    ca = _cams(cams)
    p = _params(scene, textures, roughness)
    o = _opts(spp, max_depth, rr_depth, seed, flags, None)
    _check(lib.drt_render_adjoint_wavefront(scene.handle, ctypes.byref(p), ca, len(cams), ctypes.byref(o),
                                            _dp(adj_image, "adj_image"), ctypes.byref(g),
                                            _dp(workspace, "workspace"), _nbytes(workspace),
                                            _stream(stream)),
           "drt_render_adjoint_wavefront")
    return grad_textures, grad_roughness


def checkpoint_workspace(cams, spp: int, max_depth: int, device="cuda"):
    """Workspace of the checkpointed calls: state plus one 64-byte checkpoint
    per path and bounce."""
    torch = _torch()
    n = len(cams) * cams[0].width * cams[0].height * spp
    nbytes = int(lib.drt_render_checkpointed_workspace_bytes(n, max_depth))
    if nbytes <= 0:
        raise ValueError("no checkpoint workspace for these sizes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def render_checkpointed_forward(scene: Scene, textures: Sequence, roughness, cams, spp: int,
                                max_depth: int, rr_depth: int = NO_RR, seed: int = 1, flags: int = 0,
                                workspace=None, out=None, stream=None):
    """Primal image whose per-bounce ray states stay in `workspace` for
    render_checkpointed_adjoint: (image, workspace)."""
    torch = _torch()
    dev = scene.buffer.device
    if out is None:
        out = torch.empty(_image_shape(cams), dtype=torch.float32, device=dev)
    _expect(out, "out", _image_shape(cams))
    if workspace is None:
        workspace = checkpoint_workspace(cams, spp, max_depth, dev)
    ca = _cams(cams)
    p = _params(scene, textures, roughness)
    o = _opts(spp, max_depth, rr_depth, seed, flags, None)
    _check(lib.drt_render_checkpointed_forward(scene.handle, ctypes.byref(p), ca, len(cams),
                                               ctypes.byref(o), _dp(workspace, "workspace"),
                                               _nbytes(workspace), _dp(out, "out"), _stream(stream)),
           "drt_render_checkpointed_forward")
    return out, workspace


def render_checkpointed_adjoint(scene: Scene, textures: Sequence, roughness, cams, adj_image,
                                spp: int, max_depth: int, workspace, rr_depth: int = NO_RR,
                                seed: int = 1, flags: int = 0, grad_textures=None,
                                grad_roughness=None, stream=None):
    """Gradient of <adj, I> from the checkpoints that
    render_checkpointed_forward left in `workspace` (same arguments), added
    into grad_textures / grad_roughness and returned."""
    torch = _torch()
    _expect(adj_image, "adj_image", _image_shape(cams))
    if grad_textures is None:
        grad_textures = [torch.zeros_like(t) for t in textures]
    if grad_roughness is None and roughness is not None and roughness.numel() > 0:
        grad_roughness = torch.zeros_like(roughness)
    g = drt_grads()
    for i, t in enumerate(grad_textures):
        if t is not None:
            _expect(t, f"grad texture {i}", scene.tex_shapes[i])
            g.textures[i] = _dp(t, f"grad texture {i}")
    if grad_roughness is not None:
        _expect(grad_roughness, "grad roughness")
        if grad_roughness.numel() < scene.n_roughness:
            raise ValueError(f"grad roughness needs {scene.n_roughness} entries")
        g.roughness = _dp(grad_roughness, "grad_roughness")
    ca = _cams(cams)
    p = _params(scene, textures, roughness)
    o = _opts(spp, max_depth, rr_depth, seed, flags, None)
    _check(lib.drt_render_checkpointed_adjoint(scene.handle, ctypes.byref(p), ca, len(cams),
                                               ctypes.byref(o), _dp(adj_image, "adj_image"),
                                               ctypes.byref(g), _dp(workspace, "workspace"),
                                               _nbytes(workspace), _stream(stream)),
           "drt_render_checkpointed_adjoint")
    return grad_textures, grad_roughness


def render_jvp(scene: Scene, textures: Sequence, roughness, cams, spp: int, max_depth: int,
               rr_depth: int = NO_RR, seed: int = 2, flags: int = 0, tan_textures=None,
               tan_roughness=None, out=None, stream=None):
    """Forward-mode image derivative along (tan_textures, tan_roughness):
    [n_cams, H, W, 3] float32 (device)."""
    torch = _torch()
    W, H = cams[0].width, cams[0].height
    if out is None:
        out = torch.empty((len(cams), H, W, 3), dtype=torch.float32, device=scene.buffer.device)
    _expect(out, "out", _image_shape(cams))
    t = drt_grads()
    tan_textures = list(tan_textures or [])
    if len(tan_textures) > len(scene.tex_shapes):
        raise ValueError("more tangent textures than scene textures")
    for i, x in enumerate(tan_textures):
        if x is not None:
            _expect(x, f"tangent texture {i}", scene.tex_shapes[i])
            t.textures[i] = _dp(x, f"tangent texture {i}")
    if tan_roughness is not None:
        _expect(tan_roughness, "tangent roughness")
        if tan_roughness.numel() < scene.n_roughness:
            raise ValueError(f"tangent roughness needs {scene.n_roughness} entries")
        t.roughness = _dp(tan_roughness, "tan_roughness")
    ca = _cams(cams)
    p = _params(scene, textures, roughness)
    o = _opts(spp, max_depth, rr_depth, seed, flags, None)
    _check(lib.drt_render_jvp(scene.handle, ctypes.byref(p), ca, len(cams), ctypes.byref(o),
                              ctypes.byref(t), _dp(out, "out"), _stream(stream)), "drt_render_jvp")
    return out


def trace(scene: Scene, rays, mode: int = 0, stream=None):
    """rays: float32 device [n, 8] = (o, tmin, d, tmax) -> hits int32/float32
    view as a float32 tensor [n, 4] (t, b1, b2, prim bits)."""
    torch = _torch()
    _expect(rays, "rays")
    n = rays.shape[0]
    out = torch.empty((n, 4), dtype=torch.float32, device=rays.device)
    _check(lib.drt_trace(scene.handle, _dp(rays, "rays"), n, mode, _dp(out, "out"), _stream(stream)),
           "drt_trace")
    return out


def philox(counters, keys, stream=None):
    """counters uint32-as-int32 [n,4], keys [n,2] (device) -> [n,4]."""
    torch = _torch()
    n = counters.shape[0]
    out = torch.empty((n, 4), dtype=torch.int32, device=counters.device)
    _check(lib.drt_philox(_dp(counters, "counters"), _dp(keys, "keys"), n, _dp(out, "out"),
                          _stream(stream)), "drt_philox")
    return out


def loss_l2(img, target, adj=None, stream=None):
    """(loss [1], adj) with adj = 2 (img - target) / n."""
    torch = _torch()
    _expect(img, "img")
    _expect(target, "target")
    n = img.numel()
    if adj is None:
        adj = torch.empty_like(img)
    loss = torch.empty(1, dtype=torch.float32, device=img.device)
    ws = torch.empty(int(lib.drt_loss_workspace_floats(n)), dtype=torch.float32, device=img.device)
    _check(lib.drt_loss_l2(_dp(img, "img"), _dp(target, "target"), n, _dp(adj, "adj"), _dp(loss, "loss"),
                           _dp(ws, "ws"), _stream(stream)), "drt_loss_l2")
    return loss, adj


def adam_step(param, grad, m, v, step: int, lr: float = 1e-2, beta1: float = 0.9,
              beta2: float = 0.99, eps: float = 1e-8, lo: float = -np.inf, hi: float = np.inf,
              zero_grad: bool = False, half_out=None, stream=None):
    torch = _torch()
    for t, w in ((param, "param"), (grad, "grad"), (m, "m"), (v, "v")):
        _expect(t, w)
        if t.numel() != param.numel():
            raise ValueError(f"{w} has {t.numel()} elements, param {param.numel()}")
    if half_out is not None and not (half_out.is_cuda and half_out.dtype == torch.float16 and
                                     half_out.is_contiguous() and half_out.numel() == param.numel()):
        raise ValueError("half_out must be a contiguous float16 device tensor of param's size")
    o = drt_adam_opts()
    o.lr, o.beta1, o.beta2, o.eps = lr, beta1, beta2, eps
    o.step = int(step)
    o.lo = float(max(lo, -3.0e38))
    o.hi = float(min(hi, 3.0e38))
    o.zero_grad = 1 if zero_grad else 0
    o.half_out = None if half_out is None else _dp(half_out, "half_out")
    _check(lib.drt_adam_step(_dp(param, "param"), _dp(grad, "grad"), _dp(m, "m"), _dp(v, "v"),
                             param.numel(), ctypes.byref(o), _stream(stream)), "drt_adam_step")


def new_stats():
    torch = _torch()
    return torch.zeros(len(STAT_NAMES), dtype=torch.int64, device="cuda")


def read_stats(stats) -> dict:
    v = stats.cpu().numpy().astype(np.int64)
    out = {k: int(v[i]) for i, k in enumerate(STAT_NAMES)}
    out["lrem_max"] = float(np.array([v[6]], np.int64).astype(np.uint32).view(np.float32)[0])
    return out


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------

def _make_render_fn():
    torch = _torch()

    class RenderFn(torch.autograd.Function):
        """image = render(params); backward runs the replayed adjoint with its
        own seed (a decorrelated second integration, Sec. "Physically Based
        Differentiable Rendering")."""

        @staticmethod
        def forward(ctx, scene, cams, spp, max_depth, rr_depth, seed_fwd, seed_adj, roughness,
                    *textures):
            rough = roughness.contiguous() if roughness is not None else None
            texs = [t.contiguous() for t in textures]
            img = render_forward(scene, texs, rough, cams, spp, max_depth, rr_depth, seed_fwd)
            ctx.scene, ctx.cams = scene, cams
            ctx.cfg = (spp, max_depth, rr_depth, seed_adj)
            ctx.save_for_backward(*( [rough] if rough is not None else [] ), *texs)
            ctx.has_rough = rough is not None
            return img

        @staticmethod
        def backward(ctx, grad_img):
            saved = ctx.saved_tensors
            rough = saved[0] if ctx.has_rough else None
            texs = list(saved[1:] if ctx.has_rough else saved)
            spp, max_depth, rr_depth, seed_adj = ctx.cfg
            gt, gr = render_adjoint(ctx.scene, texs, rough, ctx.cams, grad_img.contiguous(), spp,
                                    max_depth, rr_depth, seed_adj)
            return (None, None, None, None, None, None, None, gr, *gt)

    return RenderFn


_RenderFn = None


def render(scene: Scene, cams, textures, roughness=None, spp=4, max_depth=3, rr_depth=NO_RR,
           seed_fwd=1, seed_adj=2):
    """Differentiable render: gradients flow to ``textures`` and ``roughness``."""
    global _RenderFn
    if _RenderFn is None:
        _RenderFn = _make_render_fn()
    return _RenderFn.apply(scene, cams, spp, max_depth, rr_depth, seed_fwd, seed_adj, roughness,
                           *textures)


# ---------------------------------------------------------------------------
# neural radiance cache
# ---------------------------------------------------------------------------
NRC_INPUTS, NRC_WEIGHTS, NRC_RECORD = 80, 17600, 16


def nrc_config(cfg: dict) -> drt_nrc_config:
    c = drt_nrc_config()
    c.levels = int(cfg["levels"])
    c.features = int(cfg["features"])
    c.log2_table = int(cfg["log2_table"])
    c.base_res = int(cfg["base_res"])
    c.max_res = int(cfg["max_res"])
    c.trunc_vertex = int(cfg["trunc_vertex"])
    c.bbox_lo[:] = [float(x) for x in cfg["bbox_lo"]]
    c.bbox_hi[:] = [float(x) for x in cfg["bbox_hi"]]
    return c


def nrc_encode(cfg: dict, grid, records, stream=None):
    """records float [n,16] -> network inputs float [n,80] (before BF16)."""
    torch = _torch()
    n = records.shape[0]
    x = torch.empty((n, NRC_INPUTS), dtype=torch.float32, device=records.device)
    c = nrc_config(cfg)
    _check(lib.drt_nrc_encode(ctypes.byref(c), _dp(grid, "grid"), _dp(records, "records"), n,
                              _dp(x, "x"), _stream(stream)), "drt_nrc_encode")
    return x


def nrc_grid_backward(cfg: dict, records, dx, dgrid, stream=None):
    c = nrc_config(cfg)
    _check(lib.drt_nrc_grid_backward(ctypes.byref(c), _dp(records, "records"), _dp(dx, "dx"),
                                     records.shape[0], _dp(dgrid, "dgrid"), _stream(stream)),
           "drt_nrc_grid_backward")
    return dgrid


def nrc_forward(weights, x, stream=None):
    torch = _torch()
    n = x.shape[0]
    y = torch.empty((n, 3), dtype=torch.float32, device=x.device)
    _check(lib.drt_nrc_forward(_dp(weights, "weights"), _dp(x, "x"), n, _dp(y, "y"), _stream(stream)),
           "drt_nrc_forward")
    return y


def nrc_backward(weights, x, dy, dW=None, workspace=None, stream=None):
    torch = _torch()
    n = x.shape[0]
    if dW is None:
        dW = torch.zeros(NRC_WEIGHTS, dtype=torch.float32, device=x.device)
    if workspace is None:
        workspace = nrc_train_workspace(n, x.device)
    dx = torch.empty((n, NRC_INPUTS), dtype=torch.float32, device=x.device)
    _check(lib.drt_nrc_backward(_dp(weights, "weights"), _dp(x, "x"), _dp(dy, "dy"), n,
                                _dp(workspace, "workspace"), _nbytes(workspace), _dp(dW, "dW"),
                                _dp(dx, "dx"), _stream(stream)), "drt_nrc_backward")
    return dW, dx


def nrc_collect(scene: Scene, textures, roughness, cams, cfg: dict, n_paths: int, seed: int,
                max_depth: int = 6, rr_depth: int = 3, flags: int = 0, out=None, stream=None):
    """Training records of n_paths plain paths: (records [n,16], valid [n] int32, count [1])."""
    torch = _torch()
    dev = scene.buffer.device
    if out is None:
        out = (torch.empty((n_paths, NRC_RECORD), dtype=torch.float32, device=dev),
               torch.empty(n_paths, dtype=torch.int32, device=dev),
               torch.empty(1, dtype=torch.int32, device=dev))
    rec, valid, count = out
    ca = _cams(cams)
    p = _params(scene, textures, roughness)
    o = _opts(1, max_depth, rr_depth, seed, flags, None)
    c = nrc_config(cfg)
    _check(lib.drt_nrc_collect(scene.handle, ctypes.byref(p), ca, len(cams), ctypes.byref(o),
                               ctypes.byref(c), n_paths, _dp(rec, "rec"), _dp(valid, "valid"),
                               _dp(count, "count"), _stream(stream)), "drt_nrc_collect")
    return rec, valid, count


def nrc_collect_self(scene: Scene, textures, roughness, cams, cfg: dict, weights, grid, n_paths: int,
                     seed: int, tail_vertex: int = 5, max_depth: int = 6, rr_depth: int = 3,
                     flags: int = 0, out=None, workspace=None, stream=None):
    """Self-training records: n_paths paths closed by the cache's answer at
    vertex tail_vertex, one record slot per vertex before it.  Returns
    (records [n (tail_vertex-1), 16], valid [n (tail_vertex-1)] int32, count [1])."""
    torch = _torch()
    dev = scene.buffer.device
    m = n_paths * (tail_vertex - 1)
    if out is None:
        out = (torch.empty((m, NRC_RECORD), dtype=torch.float32, device=dev),
               torch.empty(m, dtype=torch.int32, device=dev),
               torch.empty(1, dtype=torch.int32, device=dev))
    rec, valid, count = out
    if rec.shape[0] < m or valid.numel() < m:
        raise ValueError(f"record buffers hold fewer than {m} records")
    need = int(lib.drt_nrc_collect_self_workspace_bytes(n_paths, tail_vertex))
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    ca = _cams(cams)
    p = _params(scene, textures, roughness)
    o = _opts(1, max_depth, rr_depth, seed, flags, None)
    c = nrc_config(cfg)
    _check(lib.drt_nrc_collect_self(scene.handle, ctypes.byref(p), ca, len(cams), ctypes.byref(o),
                                    ctypes.byref(c), _dp(weights, "weights"), _dp(grid, "grid"),
                                    tail_vertex, n_paths, _dp(rec, "rec"), _dp(valid, "valid"),
                                    _dp(count, "count"), _dp(workspace, "workspace"), _nbytes(workspace),
                                    _stream(stream)), "drt_nrc_collect_self")
    return rec, valid, count


def nrc_train_workspace(n: int, device="cuda"):
    torch = _torch()
    return torch.empty(int(lib.drt_nrc_train_workspace_bytes(n)), dtype=torch.uint8, device=device)


def nrc_train(cfg: dict, weights, grid, records, valid, count, dW, dgrid, loss=None, workspace=None,
              stream=None):
    torch = _torch()
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=weights.device)
    n = records.shape[0]
    if workspace is None:
        workspace = nrc_train_workspace(n, weights.device)
    c = nrc_config(cfg)
    _check(lib.drt_nrc_train(ctypes.byref(c), _dp(weights, "weights"), _dp(grid, "grid"),
                             _dp(records, "records"), _dp(valid, "valid"), _dp(count, "count"), n,
                             _dp(workspace, "workspace"), _nbytes(workspace), _dp(dW, "dW"),
                             _dp(dgrid, "dgrid"), _dp(loss, "loss"), _stream(stream)), "drt_nrc_train")
    return loss


def render_forward_cached(scene: Scene, textures, roughness, cams, cfg: dict, weights, grid,
                          spp: int, max_depth: int = 6, rr_depth: int = 3, seed: int = 1,
                          flags: int = 0, out=None, work=None, stream=None):
    """Primal image with path tails replaced by the cache at the record vertex."""
    torch = _torch()
    dev = scene.buffer.device
    W, H = cams[0].width, cams[0].height
    if out is None:
        out = torch.empty((len(cams), H, W, 3), dtype=torch.float32, device=dev)
    _expect(out, "out", _image_shape(cams))
    cap = len(cams) * W * H * spp
    if work is None:
        work = cached_work(cap, dev)
    q, qpix, qcount = work[:3]
    _check_work(q, qpix, cap)
    ca = _cams(cams)
    p = _params(scene, textures, roughness)
    o = _opts(spp, max_depth, rr_depth, seed, flags, None)
    c = nrc_config(cfg)
    _check(lib.drt_render_forward_cached(scene.handle, ctypes.byref(p), ca, len(cams),
                                         ctypes.byref(o), ctypes.byref(c), _dp(weights, "weights"),
                                         _dp(grid, "grid"), _dp(q, "q"), _dp(qpix, "qpix"),
                                         _dp(qcount, "qcount"), q.shape[0], _dp(out, "out"),
                                         _stream(stream)), "drt_render_forward_cached")
    return out


def cached_work(n_samples: int, device="cuda", sample_radiance: bool = False):
    """Scratch buffers of the cached render / adjoint for n_samples samples:
    (queries [n,16], query ints [drt_nrc_query_ints(n)], count [1]) and, for
    the adjoint, the per-sample radiance [n,3]."""
    torch = _torch()
    w = (torch.empty((n_samples, NRC_RECORD), dtype=torch.float32, device=device),
         torch.empty(int(lib.drt_nrc_query_ints(n_samples)), dtype=torch.int32, device=device),
         torch.empty(1, dtype=torch.int32, device=device))
    if sample_radiance:
        w = w + (torch.empty((n_samples, 3), dtype=torch.float32, device=device),)
    return w


def _check_work(q, ints, n):
    if q.shape[0] < n:
        raise ValueError(f"query buffer holds fewer than {n} queries")
    if ints.numel() < int(lib.drt_nrc_query_ints(q.shape[0])):
        raise ValueError("query int scratch is smaller than drt_nrc_query_ints(capacity)")


def render_adjoint_cached(scene: Scene, textures, roughness, cams, cfg: dict, weights, grid,
                          adj_image, spp: int, max_depth: int = 6, rr_depth: int = 3, seed: int = 2,
                          flags: int = 0, grad_textures=None, grad_roughness=None, work=None,
                          stats=None, hit_records=None, stream=None):
    """Adds the gradient of <adj, I_cached> into grad_textures /
    grad_roughness and returns them: with the cache output detached, or,
    with FLAG_CACHE_INPUT_GRAD in flags, also through the network's albedo
    and roughness inputs.  hit_records (cached_hit_records(...)): the replay
    reads the cached pass's intersections instead of tracing again."""
    torch = _torch()
    _expect(adj_image, "adj_image", _image_shape(cams))
    if grad_textures is None:
        grad_textures = [torch.zeros_like(t) for t in textures]
    if grad_roughness is None and roughness is not None and roughness.numel() > 0:
        grad_roughness = torch.zeros_like(roughness)
    g = drt_grads()
    if len(grad_textures) > len(scene.tex_shapes):
        raise ValueError("more gradient textures than scene textures")
    for i, t in enumerate(grad_textures):
        if t is not None:
            _expect(t, f"grad texture {i}", scene.tex_shapes[i])
            g.textures[i] = _dp(t, f"grad texture {i}")
    if grad_roughness is not None:
        _expect(grad_roughness, "grad roughness")
        if grad_roughness.numel() < scene.n_roughness:
            raise ValueError(f"grad roughness needs {scene.n_roughness} entries")
        g.roughness = _dp(grad_roughness, "grad_roughness")
    n = len(cams) * cams[0].width * cams[0].height * spp
    if work is None:
        work = cached_work(n, scene.buffer.device, sample_radiance=True)
    q, qid, qcount, lsamp = work
    _check_work(q, qid, n)
    if lsamp.shape[0] < n:
        raise ValueError(f"cached adjoint sample buffer holds fewer than {n} samples")
    ca = _cams(cams)
    p = _params(scene, textures, roughness)
    o = _opts(spp, max_depth, rr_depth, seed, flags, stats)
    c = nrc_config(cfg)
    _check(lib.drt_render_adjoint_cached(scene.handle, ctypes.byref(p), ca, len(cams),
                                         ctypes.byref(o), ctypes.byref(c), _dp(weights, "weights"),
                                         _dp(grid, "grid"), _dp(q, "q"), _dp(qid, "qid"),
                                         _dp(qcount, "qcount"), q.shape[0], _dp(lsamp, "lsamp"),
                                         _dp(adj_image, "adj_image"), ctypes.byref(g),
                                         None if hit_records is None else _dp(hit_records, "hit_records"),
                                         0 if hit_records is None else _nbytes(hit_records),
                                         _stream(stream)),
           "drt_render_adjoint_cached")
    return grad_textures, grad_roughness


def cached_hit_records(cams, spp: int, max_depth: int, device="cuda"):
    """Intersection-record buffer for render_adjoint_cached(hit_records=...)."""
    torch = _torch()
    nbytes = int(lib.drt_render_adjoint_cached_hit_bytes(len(cams), cams[0].width, cams[0].height,
                                                         spp, max_depth))
    if nbytes <= 0:
        raise ValueError("no intersection records for these sizes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


class NrcCache:
    """Radiance-cache state on the device: FP32 master weights and hash-grid
    features (with an FP16 copy of the grid for the kernels), Adam moments,
    gradient buffers, and the per-frame training loop
    (collect -> train -> Adam on the network -> Adam on the grid).
    self_training = 0: one record per path at the cache's truncation vertex
    from plain paths; self_training = K >= 2: self-training records at every
    vertex before K of paths closed by the cache's answer at K."""

    def __init__(self, cfg: dict, weights0, grid0, n_paths: int = 65536, lr: float = 1e-2,
                 device: str = "cuda", self_training: int = 0):
        torch = _torch()
        self.cfg = dict(cfg)
        self.W = torch.as_tensor(np.asarray(weights0, np.float32)).to(device).contiguous()
        g16 = torch.as_tensor(np.asarray(grid0, np.float16).reshape(-1)).to(device).contiguous()
        self.grid16 = g16
        self.grid = g16.float().contiguous()
        self.mW, self.vW = torch.zeros_like(self.W), torch.zeros_like(self.W)
        self.mG, self.vG = torch.zeros_like(self.grid), torch.zeros_like(self.grid)
        self.dW, self.dG = torch.zeros_like(self.W), torch.zeros_like(self.grid)
        self.n_paths = n_paths
        self.lr = lr
        self.step = 0
        self.buf = None
        self.ws = None
        self.self_training = int(self_training)
        if self.self_training == 1 or self.self_training < 0:
            raise ValueError("self_training is 0 or a tail vertex >= 2")
        self.ws_self = None
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)

    def train_frame(self, scene: Scene, textures, roughness, cams, seed: int, max_depth: int = 6,
                    rr_depth: int = 3, stream=None):
        """One training frame (drt_nrc_train_frame: records -> fused training
        pass -> Adam on the weights and the grid); returns the loss tensor."""
        torch = _torch()
        tail = self.self_training
        m = self.n_paths * (tail - 1 if tail else 1)
        dev = self.W.device
        if self.buf is None:
            self.buf = (torch.empty((m, NRC_RECORD), dtype=torch.float32, device=dev),
                        torch.empty(m, dtype=torch.int32, device=dev),
                        torch.empty(1, dtype=torch.int32, device=dev))
        if tail and self.ws_self is None:
            self.ws_self = torch.empty(int(lib.drt_nrc_collect_self_workspace_bytes(self.n_paths, tail)),
                                       dtype=torch.uint8, device=dev)
        if self.ws is None:
            self.ws = nrc_train_workspace(m, dev)
        st = drt_nrc_state()
        for name, t in (("weights", self.W), ("weights_m", self.mW), ("weights_v", self.vW),
                        ("weights_grad", self.dW), ("grid", self.grid), ("grid_m", self.mG),
                        ("grid_v", self.vG), ("grid_grad", self.dG), ("grid_half", self.grid16),
                        ("records", self.buf[0]), ("valid", self.buf[1]), ("count", self.buf[2]),
                        ("train_workspace", self.ws), ("loss", self.loss)):
            setattr(st, name, _dp(t, name))
        st.train_workspace_bytes = _nbytes(self.ws)
        if tail:
            st.self_workspace = _dp(self.ws_self, "self workspace")
            st.self_workspace_bytes = _nbytes(self.ws_self)
        fo = drt_nrc_frame_opts()
        fo.n_paths = self.n_paths
        fo.self_training = tail
        fo.step = self.step + 1
        fo.lr, fo.beta1, fo.beta2, fo.eps = self.lr, 0.9, 0.99, 1e-8
        ca = _cams(cams)
        p = _params(scene, textures, roughness)
        o = _opts(1, max_depth, rr_depth, seed, 0, None)
        c = nrc_config(self.cfg)
        _check(lib.drt_nrc_train_frame(scene.handle, ctypes.byref(p), ca, len(cams), ctypes.byref(o),
                                       ctypes.byref(c), ctypes.byref(fo), ctypes.byref(st),
                                       _stream(stream)), "drt_nrc_train_frame")
        self.step += 1
        return self.loss

    def adjoint(self, scene: Scene, textures, roughness, cams, adj_image, spp: int, seed: int,
                max_depth=6, rr_depth=3, grad_textures=None, grad_roughness=None, work=None,
                input_grad=False, hit_records=None):
        return render_adjoint_cached(scene, textures, roughness, cams, self.cfg, self.W,
                                     self.grid16, adj_image, spp, max_depth, rr_depth, seed,
                                     flags=FLAG_CACHE_INPUT_GRAD if input_grad else 0,
                                     grad_textures=grad_textures, grad_roughness=grad_roughness,
                                     work=work, hit_records=hit_records)

    def render(self, scene: Scene, textures, roughness, cams, spp: int, seed: int, max_depth=6,
               rr_depth=3, out=None, work=None):
        return render_forward_cached(scene, textures, roughness, cams, self.cfg, self.W,
                                     self.grid16, spp, max_depth, rr_depth, seed, out=out,
                                     work=work)
