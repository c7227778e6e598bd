"""Seeded synthetic scene generators (input data only).

This module is the one place that both the HIP library's tests/bench and the
CPU oracle take their inputs from.  It produces plain NumPy arrays -- triangle
meshes, material and emitter records, textures, environment maps, cameras --
and holds none of the rendering method's arithmetic: no sampling, no BSDFs,
no intersection, no random numbers that the renderer draws (those come from
counter-based Philox streams inside each implementation).

Asset randomness uses NumPy's PCG64 (``numpy.random.default_rng``).

Scene data format (shared by both consumers, documented here once):

* ``positions`` float32 [nv,3], ``uvs`` float32 [nv,2]
* ``indices`` int32 [nt,3]; triangle winding defines the geometric normal
  ``n_g = normalize((p1-p0) x (p2-p0))``
* ``tri_material`` int32 [nt]; ``tri_emitter`` int32 [nt] (-1: not emissive)
* materials: ``mat_type`` (BSDF code below), ``mat_texture`` (-1: constant
  albedo), ``mat_rough_slot`` (-1: constant ``mat_alpha``), ``mat_albedo``
  [nm,3], ``mat_alpha``, ``mat_f0`` [nm,3], ``mat_eta``, ``mat_opacity``
* emitters: ``em_type`` (emitter code below), ``em_p0``/``em_e1``/``em_e2``
  [ne,3] (area quads p0 + u e1 + v e2, front side along e1 x e2; for a
  directional light ``em_p0`` is the unit direction towards the light),
  ``em_radiance`` [ne,3] (radiance, or irradiance for directional lights)
* ``envmap`` float32 [h,w,3] or None (latitude-longitude, row 0 = +y)
* parameters (what the adjoint differentiates): ``textures`` (list of float32
  [H,W,3]) and ``roughness`` float32 [n_rough]
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# BSDF type codes of the scene format.
BSDF_NULL = 0
BSDF_DIFFUSE = 1
BSDF_DIFFUSE_TEXTURED = 2
BSDF_CONDUCTOR = 3
BSDF_DIELECTRIC = 4
BSDF_PLASTIC = 5
BSDF_TWOSIDED = 6
BSDF_MASK = 7

# Emitter type codes of the scene format.
EMITTER_AREA = 0
EMITTER_ENV = 1
EMITTER_DIRECTIONAL = 2

SEED_GEOMETRY = 2202
SEED_MATERIALS = 1284


@dataclasses.dataclass
class Camera:
    origin: tuple
    target: tuple
    up: tuple
    fov_y_deg: float
    width: int
    height: int


@dataclasses.dataclass
class Scene:
    positions: np.ndarray
    uvs: np.ndarray
    indices: np.ndarray
    tri_material: np.ndarray
    tri_emitter: np.ndarray
    mat_type: np.ndarray
    mat_texture: np.ndarray
    mat_rough_slot: np.ndarray
    mat_albedo: np.ndarray
    mat_alpha: np.ndarray
    mat_f0: np.ndarray
    mat_eta: np.ndarray
    mat_opacity: np.ndarray
    em_type: np.ndarray
    em_p0: np.ndarray
    em_e1: np.ndarray
    em_e2: np.ndarray
    em_radiance: np.ndarray
    tex_shapes: List[tuple]
    envmap: Optional[np.ndarray]
    textures: List[np.ndarray]
    roughness: np.ndarray
    cameras: List[Camera]
    name: str = ""

    @property
    def n_triangles(self) -> int:
        return int(self.indices.shape[0])

    @property
    def n_materials(self) -> int:
        return int(self.mat_type.shape[0])

    @property
    def n_emitters(self) -> int:
        return int(self.em_type.shape[0])


class _Builder:
    """Accumulates quads/meshes, materials and emitters into Scene arrays."""

    def __init__(self):
        self.pos: List[np.ndarray] = []
        self.uv: List[np.ndarray] = []
        self.idx: List[np.ndarray] = []
        self.tmat: List[np.ndarray] = []
        self.tem: List[np.ndarray] = []
        self.nv = 0
        self.mats: List[dict] = []
        self.ems: List[dict] = []

    def material(self, type_, albedo=(0.5, 0.5, 0.5), texture=-1, rough_slot=-1,
                 alpha=0.3, f0=(0.9, 0.9, 0.9), eta=1.5, opacity=1.0) -> int:
        self.mats.append(dict(type=type_, albedo=albedo, texture=texture,
                              rough_slot=rough_slot, alpha=alpha, f0=f0, eta=eta,
                              opacity=opacity))
        return len(self.mats) - 1

    def emitter(self, type_, p0=(0, 0, 0), e1=(0, 0, 0), e2=(0, 0, 0),
                radiance=(1, 1, 1)) -> int:
        self.ems.append(dict(type=type_, p0=p0, e1=e1, e2=e2, radiance=radiance))
        return len(self.ems) - 1

    def mesh(self, positions, uvs, indices, material: int, emitter: int = -1):
        positions = np.asarray(positions, np.float32).reshape(-1, 3)
        uvs = np.asarray(uvs, np.float32).reshape(-1, 2)
        indices = np.asarray(indices, np.int64).reshape(-1, 3)
        self.pos.append(positions)
        self.uv.append(uvs)
        self.idx.append((indices + self.nv).astype(np.int32))
        nt = indices.shape[0]
        self.tmat.append(np.full(nt, material, np.int32))
        self.tem.append(np.full(nt, emitter, np.int32))
        self.nv += positions.shape[0]

    def quad(self, p0, e1, e2, material: int, emitter: int = -1,
             uv=((0, 0), (1, 0), (1, 1), (0, 1))):
        """Quad p0 + u e1 + v e2 as two triangles whose normal is e1 x e2."""
        p0 = np.asarray(p0, np.float64)
        e1 = np.asarray(e1, np.float64)
        e2 = np.asarray(e2, np.float64)
        verts = np.stack([p0, p0 + e1, p0 + e1 + e2, p0 + e2])
        self.mesh(verts, uv, [[0, 1, 2], [0, 2, 3]], material, emitter)

    def area_light(self, p0, e1, e2, radiance, material: int):
        em = self.emitter(EMITTER_AREA, p0, e1, e2, radiance)
        self.quad(p0, e1, e2, material, em)
        return em

    def build(self, *, tex_shapes, textures, roughness, envmap, cameras, name) -> Scene:
        m = self.mats
        e = self.ems
        f32 = np.float32
        return Scene(
            positions=np.concatenate(self.pos).astype(f32),
            uvs=np.concatenate(self.uv).astype(f32),
            indices=np.concatenate(self.idx).astype(np.int32),
            tri_material=np.concatenate(self.tmat).astype(np.int32),
            tri_emitter=np.concatenate(self.tem).astype(np.int32),
            mat_type=np.array([x["type"] for x in m], np.int32),
            mat_texture=np.array([x["texture"] for x in m], np.int32),
            mat_rough_slot=np.array([x["rough_slot"] for x in m], np.int32),
            mat_albedo=np.array([x["albedo"] for x in m], f32).reshape(-1, 3),
            mat_alpha=np.array([x["alpha"] for x in m], f32),
            mat_f0=np.array([x["f0"] for x in m], f32).reshape(-1, 3),
            mat_eta=np.array([x["eta"] for x in m], f32),
            mat_opacity=np.array([x["opacity"] for x in m], f32),
            em_type=np.array([x["type"] for x in e], np.int32),
            em_p0=np.array([x["p0"] for x in e], f32).reshape(-1, 3),
            em_e1=np.array([x["e1"] for x in e], f32).reshape(-1, 3),
            em_e2=np.array([x["e2"] for x in e], f32).reshape(-1, 3),
            em_radiance=np.array([x["radiance"] for x in e], f32).reshape(-1, 3),
            tex_shapes=[tuple(s) for s in tex_shapes],
            envmap=None if envmap is None else np.ascontiguousarray(envmap, f32),
            textures=[np.ascontiguousarray(t, f32) for t in textures],
            roughness=np.asarray(roughness, f32).reshape(-1),
            cameras=list(cameras),
            name=name,
        )


# ----------------------------------------------------------------------------
# geometry helpers (pure mesh construction)
# ----------------------------------------------------------------------------

def _box_faces(b: _Builder, cx, cz, hx, hz, h, angle, material):
    """Open-bottom box (4 sides + top = 10 triangles), outward normals."""
    c, s = math.cos(angle), math.sin(angle)
    local = [(-hx, -hz), (hx, -hz), (hx, hz), (-hx, hz)]
    corners = [np.array([cx + c * x - s * z, 0.0, cz + s * x + c * z]) for x, z in local]
    center = np.array([cx, 0.0, cz])
    up = np.array([0.0, h, 0.0])
    for i in range(4):
        a, bb = corners[i], corners[(i + 1) % 4]
        e1 = bb - a
        n = np.cross(e1, up)
        mid = 0.5 * (a + bb)
        if np.dot(n, mid - center) > 0:
            b.quad(a, e1, up, material)
        else:
            b.quad(bb, -e1, up, material)
    # top, normal +y
    p0 = corners[0] + up
    e1 = corners[1] - corners[0]
    e2 = corners[3] - corners[0]
    if np.cross(e1, e2)[1] > 0:
        b.quad(p0, e1, e2, material)
    else:
        b.quad(p0, e2, e1, material)


def uv_sphere(center, radius, n_phi, n_theta, inward=False):
    """Closed UV sphere mesh (convex): returns positions, uvs, indices."""
    cx, cy, cz = center
    verts, uvs = [], []
    for j in range(n_theta + 1):
        th = math.pi * j / n_theta
        for i in range(n_phi + 1):
            ph = 2.0 * math.pi * i / n_phi
            verts.append((cx + radius * math.sin(th) * math.cos(ph),
                          cy + radius * math.cos(th),
                          cz + radius * math.sin(th) * math.sin(ph)))
            uvs.append((i / n_phi, j / n_theta))
    idx = []
    row = n_phi + 1
    for j in range(n_theta):
        for i in range(n_phi):
            a = j * row + i
            bq = a + 1
            cq = a + row
            d = cq + 1
            if j != 0:
                idx.append((a, bq, cq))
            if j != n_theta - 1:
                idx.append((bq, d, cq))
    idx = np.array(idx, np.int64)
    if inward:
        idx = idx[:, [0, 2, 1]]
    verts = np.array(verts)
    # orient every triangle consistently (outward unless inward=True)
    p0, p1, p2 = verts[idx[:, 0]], verts[idx[:, 1]], verts[idx[:, 2]]
    n = np.cross(p1 - p0, p2 - p0)
    outward = np.einsum("ij,ij->i", n, (p0 + p1 + p2) / 3.0 - np.array(center)) > 0
    flip = outward == inward
    idx[flip] = idx[flip][:, [0, 2, 1]]
    return verts, np.array(uvs), idx


def _sphere_arrays_vectorized(center, radius, n_phi, n_theta):
    """Vectorised outward UV sphere (used for large procedural scenes)."""
    th = np.pi * np.arange(n_theta + 1) / n_theta
    ph = 2.0 * np.pi * np.arange(n_phi + 1) / n_phi
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    verts = np.stack([center[0] + radius * np.sin(TH) * np.cos(PH),
                      center[1] + radius * np.cos(TH),
                      center[2] + radius * np.sin(TH) * np.sin(PH)], -1).reshape(-1, 3)
    uvs = np.stack([PH / (2 * np.pi), TH / np.pi], -1).reshape(-1, 2)
    row = n_phi + 1
    j, i = np.meshgrid(np.arange(n_theta), np.arange(n_phi), indexing="ij")
    a = (j * row + i).reshape(-1)
    jj = j.reshape(-1)
    b_ = a + 1
    c_ = a + row
    d_ = c_ + 1
    # with theta from +y downwards, (a, c, b) is outward-facing
    t1 = np.stack([a, c_, b_], -1)[jj != 0]
    t2 = np.stack([b_, c_, d_], -1)[jj != n_theta - 1]
    return verts, uvs, np.concatenate([t1, t2])


# ----------------------------------------------------------------------------
# Cornell-box-like scene (32 triangles)
# ----------------------------------------------------------------------------

def cornell_camera(width=64, height=64) -> Camera:
    return Camera((0.0, 1.0, 3.6), (0.0, 1.0, 0.0), (0.0, 1.0, 0.0), 40.0, width, height)


def random_texture(size: int, seed: int = SEED_MATERIALS) -> np.ndarray:
    """I.i.d. U(0.05, 0.95) RGB texels (the target texture of the optimisation)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.05, 0.95, size=(size, size, 3)).astype(np.float32)


def cell_texture(size: int, cells: int = 64, seed: int = SEED_MATERIALS) -> np.ndarray:
    """random_texture(cells) with each texel widened to a (size / cells)^2
    block: a target whose structure the views can resolve (an i.i.d. texel
    pattern at 4096^2 averages out over the texels one pixel covers)."""
    if size % cells:
        raise ValueError("size must be a multiple of cells")
    k = size // cells
    return np.repeat(np.repeat(random_texture(cells, seed), k, axis=0), k, axis=1)


def cornell(tex_size: int = 64, width: int = 64, height: int = 64, *,
            conductor: bool = False, texture: Optional[np.ndarray] = None,
            roughness: Optional[float] = None, seed: int = SEED_GEOMETRY,
            cameras: Optional[List[Camera]] = None) -> Scene:
    """Cornell-box-like room: 5 quads, 2 open-bottom boxes, 1 quad light.

    Materials: 0 = constant Lambertian 0.725, 1 = textured Lambertian (back
    wall), 2 = black Lambertian under the light; with ``conductor`` a GGX
    conductor (roughness slot 0) is added on the tall box.
    ``texture`` defaults to the constant 0.5 initial value; ``roughness``
    defaults to the initial value 0.3.
    """
    rng = np.random.default_rng(seed)
    b = _Builder()
    m_white = b.material(BSDF_DIFFUSE, albedo=(0.725, 0.725, 0.725))
    m_tex = b.material(BSDF_DIFFUSE_TEXTURED, texture=0)
    m_black = b.material(BSDF_DIFFUSE, albedo=(0.0, 0.0, 0.0))
    m_tall = m_white
    if conductor:
        f0 = tuple(np.random.default_rng(SEED_MATERIALS).uniform(0.5, 0.95, 3))
        m_tall = b.material(BSDF_CONDUCTOR, rough_slot=0, alpha=0.3, f0=f0)
    # room [-1,1] x [0,2] x [-1,1], open towards +z
    b.quad((-1, 0, 1), (2, 0, 0), (0, 0, -2), m_white)                  # floor (+y)
    b.quad((-1, 2, -1), (2, 0, 0), (0, 0, 2), m_white)                  # ceiling (-y)
    b.quad((-1, 0, -1), (2, 0, 0), (0, 2, 0), m_tex,                    # back wall (+z)
           uv=((0, 1), (1, 1), (1, 0), (0, 0)))
    b.quad((-1, 0, 1), (0, 0, -2), (0, 2, 0), m_white)                  # left wall (+x)
    b.quad((1, 0, -1), (0, 0, 2), (0, 2, 0), m_white)                   # right wall (-x)
    j = rng.uniform(-0.05, 0.05, 4)
    _box_faces(b, 0.35 + j[0], 0.35 + j[1], 0.3, 0.3, 0.6,
               rng.uniform(-0.4, -0.2), m_white)                        # short box
    _box_faces(b, -0.35 + j[2], -0.3 + j[3], 0.3, 0.3, 1.2,
               rng.uniform(0.2, 0.4), m_tall)                           # tall box
    b.area_light((-0.25, 1.98, -0.25), (0.5, 0, 0), (0, 0, 0.5), (10.0, 10.0, 10.0), m_black)
    tex = np.full((tex_size, tex_size, 3), 0.5, np.float32) if texture is None else texture
    rough = [0.3 if roughness is None else roughness] if conductor else []
    return b.build(tex_shapes=[tuple(tex.shape[:2])], textures=[tex], roughness=rough,
                   envmap=None, cameras=cameras or [cornell_camera(width, height)],
                   name="cornell")


def ring_cameras(n: int, width: int, height: int, seed: int = SEED_GEOMETRY) -> List[Camera]:
    """Seeded ring of cameras looking into the Cornell room."""
    rng = np.random.default_rng(seed + 16)
    cams = []
    for i in range(n):
        a = (i / n - 0.5) * 0.9 + rng.uniform(-0.03, 0.03)
        r = 3.6 + rng.uniform(-0.3, 0.3)
        y = 1.0 + rng.uniform(-0.25, 0.25)
        o = (r * math.sin(a), y, r * math.cos(a))
        cams.append(Camera(o, (0.0, 1.0, 0.0), (0.0, 1.0, 0.0), 40.0, width, height))
    return cams


# ----------------------------------------------------------------------------
# closed-form test scenes
# ----------------------------------------------------------------------------

def furnace_sphere(albedo=0.6, env_value=1.0, n_phi=24, n_theta=12, width=32, height=32,
                   env_size=(8, 16)) -> Scene:
    """Convex tessellated Lambertian sphere under a uniform environment."""
    b = _Builder()
    m = b.material(BSDF_DIFFUSE, albedo=(albedo, albedo, albedo))
    v, uv, idx = uv_sphere((0.0, 0.0, 0.0), 1.0, n_phi, n_theta)
    b.mesh(v, uv, idx, m)
    b.emitter(EMITTER_ENV)
    env = np.full(env_size + (3,), env_value, np.float32)
    cam = Camera((0.0, 0.3, 4.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 45.0, width, height)
    return b.build(tex_shapes=[], textures=[], roughness=[], envmap=env,
                   cameras=[cam], name="furnace_sphere")


def furnace_cube(albedo=0.5, radiance=1.0, width=16, height=16) -> Scene:
    """Camera inside a closed inward-facing cube whose 6 faces all emit."""
    b = _Builder()
    m = b.material(BSDF_DIFFUSE, albedo=(albedo, albedo, albedo))
    L = (radiance, radiance, radiance)
    s = 2.0
    # inward normals: e1 x e2 points into the cube [-1,1]^3
    faces = [((-1, -1, -1), (s, 0, 0), (0, 0, s)),    # y=-1, normal +y
             ((-1, 1, 1), (s, 0, 0), (0, 0, -s)),     # y=+1, normal -y
             ((-1, -1, -1), (0, s, 0), (s, 0, 0)),    # z=-1, normal +z
             ((-1, -1, 1), (s, 0, 0), (0, s, 0)),     # z=+1, normal -z
             ((-1, -1, 1), (0, 0, -s), (0, s, 0)),    # x=-1, normal +x ... fixed below
             ((1, -1, -1), (0, 0, s), (0, s, 0))]     # x=+1, normal -x
    for p0, e1, e2 in faces:
        p0 = np.array(p0, float)
        e1 = np.array(e1, float)
        e2 = np.array(e2, float)
        n = np.cross(e1, e2)
        c = p0 + 0.5 * (e1 + e2)
        if np.dot(n, -c) < 0:  # make the normal point at the cube centre
            p0, e1, e2 = p0 + e1, -e1, e2
        b.area_light(p0, e1, e2, L, m)
    cam = Camera((0.1, 0.2, 0.3), (0.5, -0.2, -1.0), (0.0, 1.0, 0.0), 60.0, width, height)
    return b.build(tex_shapes=[], textures=[], roughness=[], envmap=None,
                   cameras=[cam], name="furnace_cube")


def lit_plane(albedo=0.7, irradiance=2.0, theta_deg=30.0, width=16, height=16) -> Scene:
    """Large Lambertian plane y=0 under a directional light at ``theta_deg``."""
    b = _Builder()
    m = b.material(BSDF_DIFFUSE, albedo=(albedo, albedo * 0.5, albedo * 0.25))
    b.quad((-50, 0, 50), (100, 0, 0), (0, 0, -100), m)          # normal +y
    th = math.radians(theta_deg)
    d = (math.sin(th), math.cos(th), 0.0)
    b.emitter(EMITTER_DIRECTIONAL, p0=d, radiance=(irradiance, irradiance, irradiance))
    cam = Camera((0.0, 3.0, 2.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0, width, height)
    return b.build(tex_shapes=[], textures=[], roughness=[], envmap=None,
                   cameras=[cam], name="lit_plane")


def plane_under_rect_light(albedo=0.8, radiance=3.0, a=1.0, bsz=0.6, c=0.5) -> Scene:
    """Lambertian plane y=0 under a parallel, downward-facing a x b area light
    centred at height c above the origin (coaxial with the origin's normal)."""
    b = _Builder()
    m = b.material(BSDF_DIFFUSE, albedo=(albedo, albedo, albedo))
    m_black = b.material(BSDF_DIFFUSE, albedo=(0.0, 0.0, 0.0))
    b.quad((-2, 0, 2), (4, 0, 0), (0, 0, -4), m)
    # downward normal: e1 = +x, e2 = +z gives x cross z = -y
    b.area_light((-a / 2, c, -bsz / 2), (a, 0, 0), (0, 0, bsz), (radiance,) * 3, m_black)
    cam = Camera((0.0, 2.0, 3.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0, 8, 8)
    return b.build(tex_shapes=[], textures=[], roughness=[], envmap=None,
                   cameras=[cam], name="plane_rect_light")


def ao_occluder(h=0.5, half=0.3) -> Scene:
    """Ground plane y=0 with a square occluder of half-size ``half`` at height
    ``h`` centred above the origin (ambient-occlusion fixture)."""
    b = _Builder()
    m = b.material(BSDF_DIFFUSE, albedo=(0.5, 0.5, 0.5))
    b.quad((-1, 0, 1), (2, 0, 0), (0, 0, -2), m)
    b.quad((-half, h, -half), (2 * half, 0, 0), (0, 0, 2 * half), m)  # faces down
    return b.build(tex_shapes=[], textures=[], roughness=[], envmap=None,
                   cameras=[], name="ao_occluder")


def triangle_soup(n_tris=200, seed=7, extent=1.0, size=0.3) -> Scene:
    """Random triangles in a cube (intersection tests)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-extent, extent, (n_tris, 1, 3))
    v = c + rng.uniform(-size, size, (n_tris, 3, 3))
    b = _Builder()
    m = b.material(BSDF_DIFFUSE)
    b.mesh(v.reshape(-1, 3), np.zeros((3 * n_tris, 2)), np.arange(3 * n_tris).reshape(-1, 3), m)
    return b.build(tex_shapes=[], textures=[], roughness=[], envmap=None,
                   cameras=[], name="soup")


def random_rays(n, seed=11, extent=1.5):
    """Random ray origins on a sphere of radius 2*extent aimed into the cube."""
    rng = np.random.default_rng(seed)
    o = rng.normal(size=(n, 3))
    o = 2.0 * extent * o / np.linalg.norm(o, axis=1, keepdims=True)
    t = rng.uniform(-extent * 0.7, extent * 0.7, (n, 3))
    d = t - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)


# ----------------------------------------------------------------------------
# procedural environment map and textures
# ----------------------------------------------------------------------------

def sky_envmap(width=2048, height=1024, sun_dir=(0.4, 0.75, 0.3), sun_radius_deg=2.0,
               sun_intensity=2000.0) -> np.ndarray:
    """Latitude-longitude sky: gradient plus a small sun disk.  Pixel (row r,
    col c) covers theta in [r, r+1) * pi/height (theta from +y) and phi in
    [c, c+1) * 2pi/width, direction (sin t cos p, cos t, sin t sin p)."""
    th = (np.arange(height) + 0.5) / height * np.pi
    ph = (np.arange(width) + 0.5) / width * 2 * np.pi
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(TH) * np.cos(PH), np.cos(TH), np.sin(TH) * np.sin(PH)], -1)
    up = np.clip(d[..., 1], -1, 1)
    t = 0.5 * (up + 1.0)
    zen = np.array([0.25, 0.45, 0.9])
    hor = np.array([0.9, 0.85, 0.8])
    gnd = np.array([0.2, 0.18, 0.15])
    sky = np.where((up >= 0)[..., None], hor + (zen - hor) * np.sqrt(np.clip(up, 0, 1))[..., None],
                   gnd * (0.5 + 0.5 * t)[..., None])
    s = np.asarray(sun_dir, float)
    s /= np.linalg.norm(s)
    cosang = d @ s
    sun = cosang > math.cos(math.radians(sun_radius_deg))
    sky = sky.copy()
    sky[sun] = sun_intensity * np.array([1.0, 0.95, 0.85])
    return sky.astype(np.float32)


def checker_texture(size=1024, seed=SEED_MATERIALS) -> np.ndarray:
    """Procedural RGB texture: checkerboard modulated by seeded noise."""
    rng = np.random.default_rng(seed + 1)
    y, x = np.mgrid[0:size, 0:size]
    chk = ((x // (size // 16) + y // (size // 16)) % 2).astype(np.float32)
    base = rng.uniform(0.2, 0.9, (3,))
    alt = rng.uniform(0.05, 0.5, (3,))
    img = base * chk[..., None] + alt * (1 - chk[..., None])
    noise = rng.uniform(-0.05, 0.05, (size, size, 1))
    return np.clip(img + noise, 0.02, 0.98).astype(np.float32)


# ----------------------------------------------------------------------------
# procedural scene with all BSDF types
# ----------------------------------------------------------------------------

def _bsdf_for(b: _Builder, type_, rng, tex_slot: int, rough_slots: List[int]):
    alpha = float(rng.uniform(0.05, 0.6))
    albedo = tuple(rng.uniform(0.1, 0.9, 3))
    if type_ == BSDF_NULL:
        return b.material(BSDF_NULL)
    if type_ == BSDF_DIFFUSE:
        return b.material(BSDF_DIFFUSE, albedo=albedo)
    if type_ == BSDF_DIFFUSE_TEXTURED:
        return b.material(BSDF_DIFFUSE_TEXTURED, texture=tex_slot)
    if type_ == BSDF_CONDUCTOR:
        slot = len(rough_slots)
        rough_slots.append(alpha)
        return b.material(BSDF_CONDUCTOR, rough_slot=slot, alpha=alpha,
                          f0=tuple(rng.uniform(0.5, 0.95, 3)))
    if type_ == BSDF_DIELECTRIC:
        slot = len(rough_slots)
        rough_slots.append(alpha)
        return b.material(BSDF_DIELECTRIC, rough_slot=slot, alpha=alpha, eta=1.5)
    if type_ == BSDF_PLASTIC:
        slot = len(rough_slots)
        rough_slots.append(alpha)
        return b.material(BSDF_PLASTIC, rough_slot=slot, alpha=alpha, albedo=albedo, eta=1.5)
    if type_ == BSDF_TWOSIDED:
        return b.material(BSDF_TWOSIDED, texture=tex_slot)
    if type_ == BSDF_MASK:
        return b.material(BSDF_MASK, albedo=albedo, opacity=float(rng.uniform(0.3, 0.9)))
    raise ValueError(type_)


def _height_grid(n, x0, z0, size, amp, rng):
    """Height-displaced grid (n x n cells), normals +y. Returns v, uv, idx."""
    k = rng.uniform(0.5, 3.0, (4, 2))
    ph = rng.uniform(0, 2 * np.pi, 4)
    a = rng.uniform(0.2, 1.0, 4)
    a = amp * a / a.sum()
    xs = x0 + size * np.arange(n + 1) / n
    zs = z0 + size * np.arange(n + 1) / n
    X, Z = np.meshgrid(xs, zs, indexing="ij")
    Y = np.zeros_like(X)
    for i in range(4):
        Y += a[i] * np.sin(k[i, 0] * X + k[i, 1] * Z + ph[i])
    v = np.stack([X, Y, Z], -1).reshape(-1, 3)
    U, V = np.meshgrid(np.arange(n + 1) / n, np.arange(n + 1) / n, indexing="ij")
    uv = np.stack([U, V], -1).reshape(-1, 2)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    a0 = (i * (n + 1) + j).reshape(-1)
    a1 = a0 + 1
    a2 = a0 + (n + 1)
    a3 = a2 + 1
    # (a0, a1, a2): X increases along a2, Z along a1 -> (dz) x (dx) = +y
    idx = np.concatenate([np.stack([a0, a1, a2], -1), np.stack([a1, a3, a2], -1)])
    return v, uv, idx


def procedural(n_grid=512, n_spheres=215, sphere_res=(48, 24), env_size=(2048, 1024),
               n_lights=16, tex_size=1024, width=1024, height=1024, extent=12.0,
               seed_geometry=SEED_GEOMETRY, seed_materials=SEED_MATERIALS) -> Scene:
    """Large procedural scene: one height-displaced grid, UV spheres with
    radii U(0.1, 1) carrying all 8 BSDF types (assigned round-robin in a
    seeded order), 16 quad lights, a sky environment map and a procedural
    texture.  Default sizes give ~1.0M triangles."""
    rg = np.random.default_rng(seed_geometry)
    rm = np.random.default_rng(seed_materials)
    b = _Builder()
    rough: List[float] = []
    ground = b.material(BSDF_DIFFUSE_TEXTURED, texture=0)
    v, uv, idx = _height_grid(n_grid, -extent, -extent, 2 * extent, 0.2, rg)
    b.mesh(v, uv, idx, ground)
    types = [BSDF_DIFFUSE, BSDF_DIFFUSE_TEXTURED, BSDF_CONDUCTOR, BSDF_DIELECTRIC,
             BSDF_PLASTIC, BSDF_TWOSIDED, BSDF_MASK, BSDF_NULL]
    order = rm.permutation(n_spheres)
    mats = [_bsdf_for(b, types[k % 8], rm, 0, rough) for k in range(min(n_spheres, 64))]
    for s in range(n_spheres):
        r = rg.uniform(0.1, 1.0)
        cx, cz = rg.uniform(-extent * 0.8, extent * 0.8, 2)
        cy = r + rg.uniform(0.0, 0.6)
        mid = mats[order[s] % len(mats)]
        sv, suv, sidx = _sphere_arrays_vectorized((cx, cy, cz), r, *sphere_res)
        b.mesh(sv, suv, sidx, mid)
    black = b.material(BSDF_DIFFUSE, albedo=(0.0, 0.0, 0.0))
    for _ in range(n_lights):
        w, d = rg.uniform(0.2, 0.5, 2)
        cx, cz = rg.uniform(-extent * 0.7, extent * 0.7, 2)
        y = rg.uniform(2.5, 4.0) * max(extent / 12.0, 0.6)
        le = rm.uniform(5.0, 20.0)
        # downward facing: e1 = +x, e2 = +z
        b.area_light((cx - w / 2, y, cz - d / 2), (w, 0, 0), (0, 0, d), (le, le, le), black)
    b.emitter(EMITTER_ENV)
    env = sky_envmap(*env_size)
    tex = checker_texture(tex_size, seed_materials)
    k = extent / 12.0
    cam = Camera((0.0, 5.0 * k + 0.5, 14.0 * k), (0.0, 0.5, 0.0), (0.0, 1.0, 0.0), 50.0,
                 width, height)
    return b.build(tex_shapes=[tuple(tex.shape[:2])], textures=[tex], roughness=rough,
                   envmap=env, cameras=[cam], name="procedural")


def bsdf_zoo(width=64, height=64, seed=SEED_GEOMETRY, sun_intensity=200.0) -> Scene:
    """Small scene with every BSDF type, both emitter kinds and a texture:
    a textured displaced ground, eight spheres (one per BSDF type, in a
    seeded order) on a 4 x 2 grid in front of the camera, two quad lights and
    a 64 x 32 sky.  A procedural miniature for parity tests."""
    rg = np.random.default_rng(seed + 5)
    rm = np.random.default_rng(SEED_MATERIALS)
    b = _Builder()
    rough: List[float] = []
    ground = b.material(BSDF_DIFFUSE_TEXTURED, texture=0)
    v, uv, idx = _height_grid(8, -3.0, -3.0, 6.0, 0.1, rg)
    v[:, 1] -= 0.1
    b.mesh(v, uv, idx, ground)
    types = [BSDF_DIFFUSE, BSDF_DIFFUSE_TEXTURED, BSDF_CONDUCTOR, BSDF_DIELECTRIC,
             BSDF_PLASTIC, BSDF_TWOSIDED, BSDF_MASK, BSDF_NULL]
    mats = [_bsdf_for(b, t, rm, 0, rough) for t in types]
    order = rg.permutation(8)
    for s_ in range(8):
        cx = -1.5 + (s_ % 4) * 1.0 + rg.uniform(-0.1, 0.1)
        cz = -0.6 + (s_ // 4) * 1.2 + rg.uniform(-0.1, 0.1)
        r = rg.uniform(0.3, 0.45)
        sv, suv, sidx = _sphere_arrays_vectorized((cx, r, cz), r, 16, 8)
        b.mesh(sv, suv, sidx, mats[order[s_]])
    black = b.material(BSDF_DIFFUSE, albedo=(0.0, 0.0, 0.0))
    b.area_light((-1.5, 2.5, -0.5), (0.6, 0, 0), (0, 0, 0.5), (12.0, 11.0, 10.0), black)
    b.area_light((0.8, 2.0, 0.2), (0.5, 0, 0), (0, 0, 0.4), (6.0, 8.0, 12.0), black)
    b.emitter(EMITTER_ENV)
    env = sky_envmap(64, 32, sun_radius_deg=8.0, sun_intensity=sun_intensity)
    tex = checker_texture(64, SEED_MATERIALS)
    cam = Camera((0.0, 2.2, 4.0), (0.0, 0.3, 0.0), (0.0, 1.0, 0.0), 45.0, width, height)
    return b.build(tex_shapes=[(64, 64)], textures=[tex], roughness=rough,
                   envmap=env, cameras=[cam], name="bsdf_zoo")


# ----------------------------------------------------------------------------
# radiance-cache configuration and initial state (seeded inputs)
# ----------------------------------------------------------------------------

NRC_IN, NRC_HIDDEN, NRC_OUT = 80, 64, 3
NRC_LAYERS = [(NRC_HIDDEN, NRC_IN), (NRC_HIDDEN, NRC_HIDDEN), (NRC_HIDDEN, NRC_HIDDEN),
              (NRC_HIDDEN, NRC_HIDDEN), (NRC_OUT, NRC_HIDDEN)]
NRC_NUM_WEIGHTS = sum(r * c for r, c in NRC_LAYERS)


def nrc_config(sc: Scene, levels=16, features=2, log2_table=19, base_res=16, max_res=2048,
               trunc_vertex=3) -> dict:
    """Hash-grid configuration over the scene's vertex bounding box."""
    lo = sc.positions.min(0).astype(np.float64)
    hi = sc.positions.max(0).astype(np.float64)
    return dict(levels=levels, features=features, log2_table=log2_table, base_res=base_res,
                max_res=max_res, bbox_lo=[float(x) for x in np.float32(lo)],
                bbox_hi=[float(x) for x in np.float32(hi)], trunc_vertex=trunc_vertex)


def nrc_init(cfg: dict, seed: int = 16):
    """Initial network weights (He-uniform, float32 [NRC_NUM_WEIGHTS], layers
    row-major [out][in], input columns 68..79 zero) and hash-grid features
    (float16 [levels, 2^log2_table, features], U(-1e-4, 1e-4))."""
    rng = np.random.default_rng(seed)
    ws = []
    for li, (r, c) in enumerate(NRC_LAYERS):
        fan_in = 68 if li == 0 else c
        a = np.sqrt(6.0 / fan_in)
        w = rng.uniform(-a, a, (r, c))
        if li == 0:
            w[:, 68:] = 0.0
        ws.append(w.reshape(-1))
    W = np.concatenate(ws).astype(np.float32)
    T = 1 << cfg["log2_table"]
    grid = rng.uniform(-1e-4, 1e-4, (cfg["levels"], T, cfg["features"])).astype(np.float16)
    return W, grid
