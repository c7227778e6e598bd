"""Pins of the FP64 CPU oracle against values the paper prints, closed forms,
invariants and brute force -- never against the oracle itself.

Each test states what fixes the expected value.  CPU only.
"""
import math
import os

import numpy as np
import pytest

import oracle
import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Philox4x32-10
# ---------------------------------------------------------------------------

def _read_kat():
    rows = []
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers():
    """Random123's published known-answer vectors."""
    rows = _read_kat()
    ctr = np.array([r[0] for r in rows], np.uint32)
    key = np.array([r[1] for r in rows], np.uint32)
    want = np.array([r[2] for r in rows], np.uint32)
    np.testing.assert_array_equal(oracle.philox(ctr, key), want)


def test_philox_uniformity_chi2():
    """2^20 words folded to 24-bit uniforms: chi-square over 256 bins."""
    n = 1 << 18
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n, dtype=np.uint32)
    ctr[:, 2] = 5
    key = np.tile(np.array([1234, 99], np.uint32), (n, 1))
    out = oracle.philox(ctr, key).reshape(-1)
    u = (out >> 8).astype(np.float64) * 2.0 ** -24
    assert u.min() >= 0 and u.max() < 1
    counts = np.bincount((u * 256).astype(int), minlength=256)
    exp = u.size / 256
    chi2 = ((counts - exp) ** 2 / exp).sum()
    # 255 dof: mean 255, sd ~22.6; 6 sd band
    assert 255 - 6 * 22.6 < chi2 < 255 + 6 * 22.6


# ---------------------------------------------------------------------------
# intersection: brute force vs an independent Moller-Trumbore in NumPy
# ---------------------------------------------------------------------------

def _mt_closest(sc, o, d):
    """Independent brute-force closest hit (Moller-Trumbore, NumPy, FP64)."""
    P = sc.positions.astype(np.float64)
    I = sc.indices
    p0, p1, p2 = P[I[:, 0]], P[I[:, 1]], P[I[:, 2]]
    e1, e2 = p1 - p0, p2 - p0
    prims = np.full(o.shape[0], -1)
    ts = np.full(o.shape[0], np.inf)
    for r in range(o.shape[0]):
        pv = np.cross(d[r], e2)
        det = np.einsum("ij,ij->i", e1, pv)
        with np.errstate(divide="ignore", invalid="ignore"):
            tv = o[r] - p0
            u = np.einsum("ij,ij->i", tv, pv) / det
            qv = np.cross(tv, e1)
            v = (qv @ d[r]) / det
            t = np.einsum("ij,ij->i", e2, qv) / det
        ok = (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 0) & np.isfinite(t)
        if ok.any():
            tt = np.where(ok, t, np.inf)
            j = int(np.argmin(tt))
            prims[r] = j
            ts[r] = tt[j]
    return prims, ts


def test_closest_hit_matches_independent_brute_force():
    sc = scenes.triangle_soup(200, seed=3)
    o, d = scenes.random_rays(2000, seed=5)
    orc = oracle.OracleScene(sc)
    prim, t, b, amb = orc.trace(o, d)
    mp, mt = _mt_closest(sc, o.astype(np.float64), d.astype(np.float64))
    ok = ~amb
    assert ok.mean() > 0.97
    np.testing.assert_array_equal(prim[ok], mp[ok])
    hit = ok & (prim >= 0)
    assert hit.sum() > 300
    np.testing.assert_allclose(t[hit], mt[hit], rtol=1e-10)
    # barycentrics reproduce the hit point
    P = sc.positions.astype(np.float64)
    I = sc.indices[prim[hit]]
    ph = b[hit, 0:1] * P[I[:, 0]] + b[hit, 1:2] * P[I[:, 1]] + b[hit, 2:3] * P[I[:, 2]]
    pr = o[hit].astype(np.float64) + t[hit, None] * d[hit].astype(np.float64)
    np.testing.assert_allclose(ph, pr, atol=1e-9)


def test_watertight_closed_cube():
    """Rays from inside a closed mesh always hit, also through vertices and
    edges (the watertight test's defining property)."""
    sc = scenes.furnace_cube()
    orc = oracle.OracleScene(sc)
    targets = []
    for x in (-1, 0, 1):
        for y in (-1, 0, 1):
            for z in (-1, 0, 1):
                if (x, y, z) != (0, 0, 0):
                    targets.append((x, y, z))      # vertices, edge and face centres
    rng = np.random.default_rng(1)
    targets = np.array(targets, float)
    origins = np.concatenate([np.zeros((len(targets), 3)), rng.uniform(-0.5, 0.5, (len(targets), 3))])
    dirs = np.concatenate([targets, targets]) - origins
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    prim, t, _, _ = orc.trace(origins, dirs)
    assert (prim >= 0).all()


def test_closest_ties_take_lowest_id():
    """Two copies of one triangle: the lower id wins (exact tie)."""
    b = scenes._Builder()
    m = b.material(scenes.BSDF_DIFFUSE)
    tri = [(0, 0, 0), (1, 0, 0), (0, 1, 0)]
    b.mesh(tri, np.zeros((3, 2)), [[0, 1, 2]], m)
    b.mesh(tri, np.zeros((3, 2)), [[0, 2, 1]], m)
    sc = b.build(tex_shapes=[], textures=[], roughness=[], envmap=None, cameras=[], name="tie")
    orc = oracle.OracleScene(sc)
    prim, t, _, amb = orc.trace([[0.2, 0.2, 1.0]], [[0, 0, -1.0]])
    assert prim[0] == 0 and t[0] == 1.0


def test_any_hit_skips_null_and_respects_tmax():
    b = scenes._Builder()
    mn = b.material(scenes.BSDF_NULL)
    mm = b.material(scenes.BSDF_MASK, opacity=0.5)
    b.quad((-1, -1, 1), (2, 0, 0), (0, 2, 0), mn)   # null at z=1
    b.quad((-1, -1, 2), (2, 0, 0), (0, 2, 0), mm)   # mask at z=2
    sc = b.build(tex_shapes=[], textures=[], roughness=[], envmap=None, cameras=[], name="n")
    orc = oracle.OracleScene(sc)
    o = np.zeros((3, 3))
    d = np.tile([0, 0, 1.0], (3, 1))
    prim, _, _, _ = orc.trace(o, d, tmax=np.array([1.5, 2.5, np.inf]), any_hit=True)
    np.testing.assert_array_equal(prim, [-1, 1, 1])


def _small_procedural():
    return scenes.procedural(n_grid=64, n_spheres=24, sphere_res=(16, 8), env_size=(32, 16),
                             n_lights=3, tex_size=16, width=24, height=24)


@pytest.mark.parametrize("name", ["soup", "zoo", "procedural"])
def test_hierarchy_queries_equal_the_loop_over_all_triangles(name):
    """The oracle's bounding-volume hierarchy stands in for its loop over all
    triangles: closest hits (id, t, barycentrics), any hits and the
    ambiguity flags must be the loop's, bit for bit, on camera rays, rays
    between random interior points, finite and infinite t_max."""
    sc = {"soup": lambda: scenes.triangle_soup(3000, seed=4), "zoo": scenes.bsdf_zoo,
          "procedural": _small_procedural}[name]()
    fast, loop = oracle.OracleScene(sc, accel=True), oracle.OracleScene(sc, accel=False)
    assert fast.accel and not loop.accel
    rng = np.random.default_rng(8)
    n = 6000
    lo, hi = sc.positions.min(0), sc.positions.max(0)
    o = rng.uniform(lo, hi, (n, 3))
    d = rng.normal(size=(n, 3))
    if sc.cameras:
        cam = sc.cameras[0]
        k = n // 2
        o[:k] = cam.origin
        d[:k] = oracle.camera_dirs(cam, rng.uniform(0, cam.width, k), rng.uniform(0, cam.height, k))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    tmin = np.where(np.arange(n) % 5 == 0, 0.05, 0.0)
    tmax = np.where(np.arange(n) % 3 == 0, 0.7, np.inf)
    for any_hit in (False, True):
        a = fast.trace(o, d, tmin=tmin, tmax=tmax, any_hit=any_hit)
        b = loop.trace(o, d, tmin=tmin, tmax=tmax, any_hit=any_hit)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
        assert (b[0] >= 0).mean() > 0.1


def test_hierarchy_render_and_adjoint_equal_the_loop():
    """Images, per-pixel ambiguity counts and gradients of the procedural
    scene (all BSDF types, env map, quad lights, depth 6 with roulette) are
    identical with and without the hierarchy (one thread, so that the
    gradient sums run in the same order)."""
    sc = _small_procedural()
    fast, loop = oracle.OracleScene(sc, accel=True), oracle.OracleScene(sc, accel=False)
    kw = dict(spp=3, max_depth=6, rr_depth=3, seed=5)
    ia, ma = fast.render(ambiguity=True, **kw)
    ib, mb = loop.render(ambiguity=True, **kw)
    np.testing.assert_array_equal(ia, ib)
    np.testing.assert_array_equal(ma, mb)
    adj = np.random.default_rng(2).normal(size=ia.shape)
    ga, ra = fast.adjoint(adj, threads=1, **kw)
    gb, rb = loop.adjoint(adj, threads=1, **kw)
    for x, y in zip(ga, gb):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(ra, rb)
    assert np.abs(gb[0]).sum() > 0 and np.abs(rb).sum() > 0


# ---------------------------------------------------------------------------
# camera and frames
# ---------------------------------------------------------------------------

def test_camera_centre_and_edges():
    cam = scenes.Camera((0, 1, 3.6), (0, 1, 0), (0, 1, 0), 40.0, 64, 48)
    d = oracle.camera_dirs(cam, [32.0, 32.0, 0.0], [24.0, 0.0, 24.0])
    np.testing.assert_allclose(d[0], [0, 0, -1], atol=1e-15)
    # top edge: vertical angle = fov/2
    assert math.isclose(math.degrees(math.atan2(d[1][1], -d[1][2])), 20.0, rel_tol=1e-12)
    # left edge: horizontal tangent = tan(fov/2) * aspect, pointing to -x
    assert math.isclose(-d[2][0] / -d[2][2], math.tan(math.radians(20)) * 64 / 48, rel_tol=1e-12)


@pytest.mark.parametrize("n", [(0, 0, 1), (0, 0, -1), (1, 0, 0), (0.3, -0.4, 0.866), (0.6, 0.0, -0.8)])
def test_frame_orthonormal_right_handed(n):
    n = np.array(n, float)
    n /= np.linalg.norm(n)
    s, t = oracle.frame(n)
    M = np.stack([s, t, n])
    np.testing.assert_allclose(M @ M.T, np.eye(3), atol=1e-14)
    np.testing.assert_allclose(np.cross(s, t), n, atol=1e-14)


# ---------------------------------------------------------------------------
# ambient occlusion (the paper's running example) against a form factor
# ---------------------------------------------------------------------------

def _ff_corner(a, b, c):
    """Differential area to a parallel a x b rectangle at distance c whose
    corner lies on the area's normal (classic closed form)."""
    X, Y = a / c, b / c
    sx, sy = math.sqrt(1 + X * X), math.sqrt(1 + Y * Y)
    return (X / sx * math.atan(Y / sx) + Y / sy * math.atan(X / sy)) / (2 * math.pi)


def _ff_centred(a, b, c):
    return 4 * _ff_corner(a / 2, b / 2, c)


def test_form_factor_formula_by_quadrature():
    from scipy import integrate
    a, b, c = 0.6, 0.6, 0.5
    q, _ = integrate.dblquad(lambda y, x: c * c / (x * x + y * y + c * c) ** 2 / math.pi,
                             -a / 2, a / 2, -b / 2, b / 2, epsabs=1e-12)
    assert math.isclose(q, _ff_centred(a, b, c), rel_tol=1e-9)


def _linspace_pin():
    vals = {}
    for line in open(os.path.join(GOLDEN, "linspace_1024.txt")):
        if line.startswith("#"):
            continue
        k, v = line.split(":")
        vals[k] = [float(x) for x in v.split()]
    return vals


def test_ao_under_square_occluder():
    """AO with 128 cosine rays of length 1 (the running example) at points
    under a centred square occluder equals 1 - F (form factor)."""
    pin = _linspace_pin()
    x = np.linspace(-1, 1, 1024)
    np.testing.assert_allclose(np.round(x[:3], 3), pin["first"])
    np.testing.assert_allclose(np.round(x[-3:], 3), pin["last"])
    h, half = 0.5, 0.3
    sc = scenes.ao_occluder(h=h, half=half)
    orc = oracle.OracleScene(sc)
    g = x[::32] * 1e-3                      # orthographic offsets around the origin
    X, Z = np.meshgrid(g, g)
    o = np.stack([X.ravel(), np.full(X.size, 0.01), Z.ravel()], 1)
    d = np.tile([0.0, -1.0, 0.0], (o.shape[0], 1))
    ao = orc.ao(o, d, n_ao=128, seed=7)
    assert (ao >= 0).all()
    F = _ff_centred(2 * half, 2 * half, h - orc.eps)
    m = ao.mean()
    se = math.sqrt(m * (1 - m) / (ao.size * 128))
    assert abs(m - (1 - F)) < 4 * se + 1e-4, (m, 1 - F, se)


# ---------------------------------------------------------------------------
# closed-form scenes
# ---------------------------------------------------------------------------

def test_white_furnace_sphere_exact_without_nee():
    rho, Lenv = 0.6, 1.5
    sc = scenes.furnace_sphere(albedo=rho, env_value=Lenv, width=16, height=16)
    orc = oracle.OracleScene(sc)
    img = orc.render(spp=1, max_depth=4, flags=1, seed=3)
    vals = np.unique(img.round(12))
    rho32 = float(np.float32(rho))
    np.testing.assert_allclose(sorted(vals), sorted({round(rho32 * Lenv, 12), Lenv}), rtol=1e-12)


def test_white_furnace_sphere_with_nee_in_expectation():
    rho, Lenv = 0.6, 1.0
    sc = scenes.furnace_sphere(albedo=rho, env_value=Lenv)
    orc = oracle.OracleScene(sc)
    o = np.array([[0.0, 0.0, 4.0]] * 64)
    d = np.array([[0.0, 0.0, -1.0]] * 64)
    est = orc.radiance(o, d, spp=256, max_depth=2, seed=11)[:, 0]
    m, se = est.mean(), est.std() / math.sqrt(est.size)
    assert abs(m - float(np.float32(rho)) * Lenv) < 4 * se + 1e-12


def test_enclosed_furnace_depth_series():
    """Inside an emitting closed box: L = Le * sum_{j<D} rho^j per sample."""
    sc = scenes.furnace_cube(albedo=0.5, radiance=2.0)
    orc = oracle.OracleScene(sc)
    for D in (1, 2, 3, 6):
        img = orc.render(spp=1, max_depth=D, flags=1, seed=5)
        np.testing.assert_allclose(img, 2.0 * sum(0.5 ** j for j in range(D)), rtol=1e-12)


def test_directional_light_on_plane_exact():
    rho = np.array([0.7, 0.35, 0.175], np.float32).astype(float)
    E, th = 2.0, 30.0
    sc = scenes.lit_plane(albedo=0.7, irradiance=E, theta_deg=th)
    orc = oracle.OracleScene(sc)
    img = orc.render(spp=2, max_depth=3, seed=1)
    want = rho * E * math.cos(math.radians(th)) / math.pi
    np.testing.assert_allclose(img.reshape(-1, 3), np.tile(want, (img.size // 3, 1)), rtol=1e-6)


def test_area_light_form_factor_in_expectation():
    rho, Le, a, b, c = 0.8, 3.0, 1.0, 0.6, 0.5
    sc = scenes.plane_under_rect_light(albedo=rho, radiance=Le, a=a, bsz=b, c=c)
    orc = oracle.OracleScene(sc)
    o = np.array([[-1.5, 0.05, 0.0]] * 64)
    d = np.array([1.5, -0.05, 0.0]) / math.hypot(1.5, 0.05)
    d = np.tile(d, (64, 1))
    est = orc.radiance(o, d, spp=512, max_depth=2, seed=3)[:, 0]
    want = float(np.float32(rho)) * Le * _ff_centred(a, b, c)
    m, se = est.mean(), est.std() / math.sqrt(est.size)
    assert abs(m - want) < 4 * se + 2e-3 * want, (m, want, se)


# ---------------------------------------------------------------------------
# microfacet and Fresnel terms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("alpha", [0.05, 0.2, 0.6, 1.0])
def test_ggx_normalisation(alpha):
    """int D(m) cos(theta_m) dm = 1 over the hemisphere."""
    from scipy import integrate
    f = lambda th: oracle.ggx_terms(alpha, math.cos(th), 0.5)["D"] * math.cos(th) * math.sin(th) * 2 * math.pi
    val, _ = integrate.quad(f, 0, math.pi / 2, limit=400, points=[alpha * 0.5, alpha, 2 * alpha])
    assert abs(val - 1) < 1e-7


@pytest.mark.parametrize("alpha", [0.1, 0.45])
def test_ggx_sampling_matches_density(alpha):
    """Histogram of sampled cos(theta_m) vs the integral of D cos over bins."""
    from scipy import integrate
    rng = np.random.default_rng(3)
    n = 200000
    u = rng.random((n, 2))
    cs = np.array([oracle.ggx_sample(alpha, a, b)[2] for a, b in u[:20000]])
    edges = np.linspace(0, 1, 11)
    cnt, _ = np.histogram(cs, edges)
    for i in range(10):
        p, _ = integrate.quad(lambda c: oracle.ggx_terms(alpha, c, 0.5)["D"] * c * 2 * math.pi,
                              edges[i], edges[i + 1], limit=200)
        se = math.sqrt(max(p * (1 - p), 1e-12) / 20000)
        assert abs(cnt[i] / 20000 - p) < 5 * se + 1e-4


@pytest.mark.parametrize("alpha,cm,cv", [(0.05, 0.99, 0.3), (0.3, 0.8, 0.9), (0.6, 0.4, 0.2), (0.9, 0.95, 0.05)])
def test_ggx_roughness_derivatives_complex_step(alpha, cm, cv):
    t = oracle.ggx_terms(alpha, cm, cv)
    assert math.isclose(t["dlnD"], t["dlnD_cs"], rel_tol=1e-10, abs_tol=1e-12)
    assert math.isclose(t["dlnG1"], t["dlnG1_cs"], rel_tol=1e-10, abs_tol=1e-12)


def test_fresnel_closed_forms():
    assert math.isclose(oracle.fresnel(1.0, 1.5), 0.04, rel_tol=1e-12)
    crit = math.sqrt(1 - 1 / 1.5 ** 2)  # inside glass: cos of the critical angle
    assert oracle.fresnel(crit * 0.99, 1 / 1.5) == 1.0
    assert oracle.fresnel(crit * 1.01, 1 / 1.5) < 1.0
    assert oracle.fresnel(0.0, 1.5) == pytest.approx(1.0)
    # reciprocity: F(theta_i; eta) = F(theta_t; 1/eta)
    for ci in (0.2, 0.5, 0.9):
        ct = math.sqrt(1 - (1 - ci * ci) / 1.5 ** 2)
        assert math.isclose(oracle.fresnel(ci, 1.5), oracle.fresnel(ct, 1 / 1.5), rel_tol=1e-12)


# ---------------------------------------------------------------------------
# BSDF sampling consistency: integral of the density = success rate, and
# E[f/pdf] = integral of f over the sphere
# ---------------------------------------------------------------------------

BSDF_CASES = [
    (scenes.BSDF_DIFFUSE, 0.3, (0.3, 0.2, 0.9)),
    (scenes.BSDF_TWOSIDED, 0.3, (0.3, 0.2, -0.9)),
    (scenes.BSDF_CONDUCTOR, 0.25, (0.5, 0.1, 0.6)),
    (scenes.BSDF_PLASTIC, 0.3, (0.2, -0.4, 0.5)),
    (scenes.BSDF_DIELECTRIC, 0.35, (0.3, 0.1, 0.7)),
    (scenes.BSDF_DIELECTRIC, 0.35, (0.3, 0.1, -0.7)),
]


def _sphere_grid(n_th=240, n_ph=480):
    th = (np.arange(n_th) + 0.5) / n_th * math.pi
    ph = (np.arange(n_ph) + 0.5) / n_ph * 2 * math.pi
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    w = np.sin(TH) * (math.pi / n_th) * (2 * math.pi / n_ph)
    d = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1)
    return d.reshape(-1, 3), w.reshape(-1)


@pytest.mark.slow
@pytest.mark.parametrize("type_,alpha,wi", BSDF_CASES)
def test_bsdf_sampling_consistency(type_, alpha, wi):
    wi = np.array(wi, float)
    wi /= np.linalg.norm(wi)
    kw = dict(albedo=(0.7, 0.5, 0.3), alpha=alpha, f0=(0.9, 0.7, 0.5), eta=1.5)
    dirs, w = _sphere_grid()
    pdf_int = 0.0
    f_int = np.zeros(3)
    for dd, ww in zip(dirs, w):
        f, pdf, _, _ = oracle.bsdf_eval(type_, wi, dd, **kw)
        pdf_int += pdf * ww
        f_int += f * ww
    rng = np.random.default_rng(17)
    n = 40000
    u = rng.random((n, 3))
    acc = np.zeros((n, 3))
    ok = np.zeros(n, bool)
    for i in range(n):
        good, wo, f, pdf = oracle.bsdf_sample(type_, wi, u[i, 0], u[i, 1], u[i, 2], **kw)
        ok[i] = good
        if good:
            acc[i] = f / pdf
    rate = ok.mean()
    assert abs(pdf_int - rate) < 5 * math.sqrt(rate * (1 - rate) / n) + 4e-3
    m = acc.mean(0)
    se = acc.std(0) / math.sqrt(n)
    assert np.all(np.abs(m - f_int) < 5 * se + 5e-3 * np.abs(f_int) + 1e-4), (m, f_int, se)


@pytest.mark.parametrize("type_", [scenes.BSDF_DIFFUSE, scenes.BSDF_CONDUCTOR, scenes.BSDF_PLASTIC,
                                   scenes.BSDF_DIELECTRIC])
def test_bsdf_reflection_reciprocity(type_):
    rng = np.random.default_rng(2)
    for _ in range(20):
        a = rng.normal(size=3); a[2] = abs(a[2]); a /= np.linalg.norm(a)
        b = rng.normal(size=3); b[2] = abs(b[2]); b /= np.linalg.norm(b)
        fab, _, _, _ = oracle.bsdf_eval(type_, a, b, alpha=0.3)
        fba, _, _, _ = oracle.bsdf_eval(type_, b, a, alpha=0.3)
        np.testing.assert_allclose(fab / b[2], fba / a[2], rtol=1e-10, atol=1e-14)


def _half_angle_pair(th_i, th_o):
    """Directions at polar angles th_i, th_o on either side of the normal in
    one plane: their half vector is the normal tilted by (th_i - th_o) / 2, so
    the cosine between wi and it is cos((th_i + th_o) / 2)."""
    wi = np.array([math.sin(th_i), 0.0, math.cos(th_i)])
    wo = np.array([-math.sin(th_o), 0.0, math.cos(th_o)])
    return wi, wo, math.cos(0.5 * (th_i + th_o))


@pytest.mark.parametrize("alpha", [0.1, 0.4])
def test_conductor_fresnel_is_schlick(alpha):
    """Schlick's approximation F = f0 + (1 - f0)(1 - cos)^5, cos between the
    incident direction and the microfacet normal (Schlick 1994): the conductor
    value is F times terms that do not depend on f0, so its ratio at two f0
    isolates F.  At cos = 1 the ratio to f0 = 1 is f0, at cos = 1/2 it is
    f0 + (1 - f0)/32, at grazing it tends to 1, and with f0 = 0 it is
    (1 - cos)^5 at asymmetric angles (the cosine is taken at the half
    vector, not at either direction)."""
    C = scenes.BSDF_CONDUCTOR

    def ratio(f0, wi, wo):
        a = oracle.bsdf_eval(C, wi, wo, f0=(f0, f0, f0), alpha=alpha)[0]
        b = oracle.bsdf_eval(C, wi, wo, f0=(1.0, 1.0, 1.0), alpha=alpha)[0]
        assert np.all(b > 0)
        return a / b

    up = np.array([0.0, 0.0, 1.0])
    for f0 in (0.0, 0.3, 0.9):
        np.testing.assert_allclose(ratio(f0, up, up), f0, rtol=1e-12, atol=1e-15)
        wi, wo, c = _half_angle_pair(math.pi / 3, math.pi / 3)
        assert math.isclose(c, 0.5, rel_tol=1e-12)
        np.testing.assert_allclose(ratio(f0, wi, wo), f0 + (1 - f0) / 32, rtol=1e-10)
        wi, wo, c = _half_angle_pair(math.pi / 2 - 1e-6, math.pi / 2 - 1e-6)
        np.testing.assert_allclose(ratio(f0, wi, wo), 1.0, rtol=1e-5)
    for th_i, th_o in ((0.2, 1.1), (1.3, 0.4), (0.9, 0.0)):
        wi, wo, c = _half_angle_pair(th_i, th_o)
        np.testing.assert_allclose(ratio(0.0, wi, wo), (1 - c) ** 5, rtol=1e-10)


def test_dielectric_transmission_generalised_reciprocity():
    """Radiance BSDF of a refracting interface (Veach 1997, generalised
    reciprocity): f(a, b) / n_a^2 = f(b, a) / n_b^2 for a camera-side
    direction a in the medium of index n_a and a light-side direction b in
    index n_b (outside 1, inside eta = 1.5).  eval() returns f |cos theta_b|,
    so the values are divided by the cosine of their second argument."""
    D = scenes.BSDF_DIELECTRIC
    eta = 1.5
    rng = np.random.default_rng(12)
    n_checked = 0
    for _ in range(400):
        a = rng.normal(size=3); a /= np.linalg.norm(a)
        b = rng.normal(size=3); b /= np.linalg.norm(b)
        if a[2] * b[2] >= 0:
            b[2] = -b[2]   # opposite sides: transmission
        for alpha in (0.1, 0.35):
            fab = oracle.bsdf_eval(D, a, b, alpha=alpha, eta=eta)[0][0] / abs(b[2])
            fba = oracle.bsdf_eval(D, b, a, alpha=alpha, eta=eta)[0][0] / abs(a[2])
            na = 1.0 if a[2] > 0 else eta
            nb = 1.0 if b[2] > 0 else eta
            if fab == 0 and fba == 0:
                continue
            n_checked += 1
            assert math.isclose(fab / na ** 2, fba / nb ** 2, rel_tol=1e-10), (a, b, alpha)
    assert n_checked > 100


@pytest.mark.parametrize("inside", [False, True])
def test_dielectric_transmission_normal_incidence_smooth_limit(inside):
    """As the roughness goes to zero the transmitted part of a normally
    incident camera direction integrates to the smooth interface's radiance
    transmittance: (1 - F0) (n_camera / n_light)^2 with F0 = ((eta - 1) /
    (eta + 1))^2 = 0.04 -- 0.96 / 2.25 looking from outside into glass,
    0.96 x 2.25 looking out from inside (radiance scales with the square of
    the index, Veach 1997).  The integrand is symmetric about the normal;
    the polar integral runs in log(theta) to resolve the peak of width ~alpha."""
    D = scenes.BSDF_DIELECTRIC
    eta, alpha = 1.5, 2e-3
    s = -1.0 if inside else 1.0
    wi = np.array([0.0, 0.0, s])
    lt = np.linspace(math.log(1e-9), math.log(math.pi / 2), 20001)
    th = np.exp(lt)
    vals = np.empty(th.size)
    for i, t in enumerate(th):
        wo = np.array([math.sin(t), 0.0, -s * math.cos(t)])
        vals[i] = oracle.bsdf_eval(D, wi, wo, alpha=alpha, eta=eta)[0][0]
    g = vals * np.sin(th) * th   # d(omega) = sin(theta) dtheta dphi, dtheta = theta dlog(theta)
    integral = 2 * math.pi * float(np.sum(0.5 * (g[1:] + g[:-1]) * np.diff(lt)))
    f0 = ((eta - 1) / (eta + 1)) ** 2
    want = (1 - f0) * (eta ** 2 if inside else 1 / eta ** 2)
    assert math.isclose(integral, want, rel_tol=1e-4), (integral, want)


def test_plastic_diffuse_weight():
    """Plastic's diffuse lobe (1 - F(cos_i)) (1 - F(cos_o)) rho / pi, times
    cos_o: the value is affine in the albedo, so the difference of two evals
    isolates it from the specular coat.  Both directions normal: 0.96^2 / pi;
    incidence normal and outgoing at 60 degrees: 0.96 (1 - F(1/2)) 0.5 / pi,
    and swapped, 0.96 (1 - F(1/2)) / pi -- F the exact dielectric Fresnel
    pinned above."""
    P = scenes.BSDF_PLASTIC
    eta = 1.5

    def diffuse(wi, wo):
        one = oracle.bsdf_eval(P, wi, wo, albedo=(1.0, 1.0, 1.0), alpha=0.3, eta=eta)[0]
        zero = oracle.bsdf_eval(P, wi, wo, albedo=(0.0, 0.0, 0.0), alpha=0.3, eta=eta)[0]
        return one - zero

    up = np.array([0.0, 0.0, 1.0])
    tilt = np.array([math.sin(math.pi / 3), 0.0, 0.5])
    f_half = oracle.fresnel(0.5, eta)
    np.testing.assert_allclose(diffuse(up, up), 0.96 ** 2 / math.pi, rtol=1e-10)
    np.testing.assert_allclose(diffuse(up, tilt), 0.96 * (1 - f_half) * 0.5 / math.pi, rtol=1e-10)
    np.testing.assert_allclose(diffuse(tilt, up), (1 - f_half) * 0.96 / math.pi, rtol=1e-10)
    # the albedo enters linearly: rho = 0.25 gives a quarter of the lobe
    quarter = (oracle.bsdf_eval(P, up, up, albedo=(0.25, 0.25, 0.25), alpha=0.3, eta=eta)[0]
               - oracle.bsdf_eval(P, up, up, albedo=(0.0, 0.0, 0.0), alpha=0.3, eta=eta)[0])
    np.testing.assert_allclose(quarter, 0.25 * 0.96 ** 2 / math.pi, rtol=1e-10)


def test_bsdf_parameter_derivatives_by_finite_differences():
    """d f/d albedo and d f/d alpha of the eval() against FP64 central
    differences of eval() itself at perturbed parameters."""
    rng = np.random.default_rng(4)
    for type_ in (scenes.BSDF_DIFFUSE, scenes.BSDF_CONDUCTOR, scenes.BSDF_PLASTIC,
                  scenes.BSDF_DIELECTRIC, scenes.BSDF_TWOSIDED):
        for _ in range(10):
            wi = rng.normal(size=3); wi /= np.linalg.norm(wi)
            wo = rng.normal(size=3); wo /= np.linalg.norm(wo)
            if type_ not in (scenes.BSDF_DIELECTRIC, scenes.BSDF_TWOSIDED):
                wi[2], wo[2] = abs(wi[2]), abs(wo[2])
            alb = np.array([0.3, 0.5, 0.7])
            f, _, dalb, dal = oracle.bsdf_eval(type_, wi, wo, albedo=alb, alpha=0.3)
            h = 1e-6
            fp = oracle.bsdf_eval(type_, wi, wo, albedo=alb + h, alpha=0.3)[0]
            fm = oracle.bsdf_eval(type_, wi, wo, albedo=alb - h, alpha=0.3)[0]
            np.testing.assert_allclose(dalb, (fp - fm) / (2 * h), rtol=1e-6, atol=1e-9)
            fp = oracle.bsdf_eval(type_, wi, wo, albedo=alb, alpha=0.3 + h)[0]
            fm = oracle.bsdf_eval(type_, wi, wo, albedo=alb, alpha=0.3 - h)[0]
            np.testing.assert_allclose(dal, (fp - fm) / (2 * h), rtol=1e-5, atol=1e-8)


# ---------------------------------------------------------------------------
# environment map sampling
# ---------------------------------------------------------------------------

def _env_scene(w=64, h=32, sun=True):
    b = scenes._Builder()
    m = b.material(scenes.BSDF_DIFFUSE)
    b.quad((-0.1, -5, -0.1), (0.2, 0, 0), (0, 0, 0.2), m)
    b.emitter(scenes.EMITTER_ENV)
    env = scenes.sky_envmap(w, h, sun_radius_deg=10.0 if sun else 0.0, sun_intensity=50.0)
    return b.build(tex_shapes=[], textures=[], roughness=[], envmap=env, cameras=[], name="env")


def test_env_pdf_integrates_to_one_and_sampling_is_unbiased():
    sc = _env_scene()
    orc = oracle.OracleScene(sc)
    dirs, w = _sphere_grid(256, 512)
    # the (x, y, z) of _sphere_grid has z as the polar axis; the map's is y
    dirs = dirs[:, [0, 2, 1]]
    pdf = np.array([orc.env_pdf(d) for d in dirs])
    assert abs((pdf * w).sum() - 1) < 2e-3
    lum = lambda c: 0.2126 * c[0] + 0.7152 * c[1] + 0.0722 * c[2]
    ref = sum(lum(orc.env_lookup(d)) * ww for d, ww in zip(dirs, w))
    rng = np.random.default_rng(8)
    vals = []
    for u1, u2 in rng.random((20000, 2)):
        ok, d = orc.env_sample(u1, u2)
        assert ok
        vals.append(lum(orc.env_lookup(d)) / orc.env_pdf(d))
    vals = np.array(vals)
    assert abs(vals.mean() - ref) < 5 * vals.std() / math.sqrt(vals.size) + 3e-3 * ref


# ---------------------------------------------------------------------------
# estimator consistency: NEE + MIS, Russian roulette and pass-through rules
# leave the expectation unchanged
# ---------------------------------------------------------------------------

def _diff_se(a, b):
    d = (a - b).reshape(-1)
    return d.mean(), d.std() / math.sqrt(d.size)


def test_nee_mis_unbiased_cornell():
    sc = scenes.cornell()
    orc = oracle.OracleScene(sc)
    a = orc.render(spp=64, max_depth=4, seed=21)
    b = orc.render(spp=256, max_depth=4, flags=1, seed=22)
    m, se = _diff_se(a, b)
    assert abs(m) < 4 * se, (m, se)


@pytest.mark.slow
def test_nee_mis_rr_unbiased_all_bsdfs():
    sc = scenes.bsdf_zoo(width=24, height=24)
    sc.envmap = scenes.sky_envmap(64, 32, sun_intensity=0.0)   # no sun: keep NO_NEE variance finite
    orc = oracle.OracleScene(sc)
    a = orc.render(spp=512, max_depth=16, rr_depth=3, seed=31)
    b = orc.render(spp=1024, max_depth=16, flags=1, seed=32)
    m, se = _diff_se(a, b)
    assert abs(m) < 4 * se, (m, se)
    c = orc.render(spp=512, max_depth=16, seed=33)
    m, se = _diff_se(a, c)
    assert abs(m) < 4 * se, (m, se)


# ---------------------------------------------------------------------------
# the adjoint
# ---------------------------------------------------------------------------

def _adj_image(sc, seed=5):
    c = sc.cameras[0]
    return np.random.default_rng(seed).normal(size=(len(sc.cameras), c.height, c.width, 3))


@pytest.mark.parametrize("name", ["cornell", "zoo"])
def test_adjoint_reverse_sweep_equals_forward_mode(name):
    if name == "cornell":
        sc = scenes.cornell(conductor=True, texture=scenes.random_texture(64))
        kw = dict(spp=4, max_depth=3)
    else:
        sc = scenes.bsdf_zoo(width=32, height=32)
        kw = dict(spp=4, max_depth=6, rr_depth=3)
    orc = oracle.OracleScene(sc)
    adj = _adj_image(sc)
    gt0, gr0 = orc.adjoint(adj, mode=0, seed=2, **kw)
    gt1, gr1 = orc.adjoint(adj, mode=1, seed=2, **kw)
    for a, b in zip(gt0, gt1):
        assert np.abs(a).max() > 0
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(a).max())
    np.testing.assert_allclose(gr0, gr1, rtol=1e-12, atol=1e-15)
    if len(gr0):
        assert np.abs(gr0).max() > 0


def test_adjoint_albedo_matches_central_differences():
    """With sampling independent of albedo and RR off, the estimator is a
    polynomial of degree <= 2 in each texel at D = 3, so a central difference
    with common random numbers is exact up to round-off."""
    sc = scenes.cornell(texture=scenes.random_texture(64))
    orc = oracle.OracleScene(sc)
    kw = dict(spp=4, max_depth=3, seed=2)
    adj = _adj_image(sc)
    gtex, _ = orc.adjoint(adj, **kw)
    g = gtex[0].reshape(-1)
    rng = np.random.default_rng(9)
    cand = np.flatnonzero(np.abs(g) > 1e-3 * np.abs(g).max())
    pick = rng.choice(cand, 24, replace=False)
    h = 1e-2
    base = sc.textures[0].astype(np.float64)
    for k in pick:
        tp = base.copy().reshape(-1); tp[k] += h
        tm = base.copy().reshape(-1); tm[k] -= h
        Ip = orc.render(textures=[tp.reshape(base.shape).astype(np.float32)], **kw)
        Im = orc.render(textures=[tm.reshape(base.shape).astype(np.float32)], **kw)
        # perturbed texel values are FP32 in the scene data: use the exact step
        hh = (np.float32(base.reshape(-1)[k] + h) - np.float32(base.reshape(-1)[k] - h)) / 2
        fd = float((adj * (Ip - Im)).sum() / (2 * hh))
        assert math.isclose(fd, g[k], rel_tol=1e-6, abs_tol=1e-9 * np.abs(g).max()), (k, fd, g[k])


# ---------------------------------------------------------------------------
# loss and Adam
# ---------------------------------------------------------------------------

def test_roughness_gradient_matches_central_differences_in_expectation():
    """The oracle's roughness gradient (detached sampling) against central
    differences of its own estimator in the roughness (h = 1e-2, common
    random numbers, no roulette).  Sampling depends on the roughness, so a
    single seed's differences carry noise the detached gradient does not;
    both are unbiased for the derivative of the expected image.  16 seeds of
    128 spp: the mean difference within max(2e-2 |fd|, 3 SE) (3 SE is ~10%
    of the derivative here)."""
    sc = scenes.cornell(conductor=True, width=24, height=24)
    orc = oracle.OracleScene(sc)
    adj = np.ones((1, 24, 24, 3)) / (24 * 24 * 3)     # derivative of the mean brightness
    a0 = float(sc.roughness[0])
    h = 1e-2
    g, fd = [], []
    for s in range(16):
        seed = 300 + s
        _, gr = orc.adjoint(adj, spp=128, max_depth=3, seed=seed)
        ip = orc.render(spp=128, max_depth=3, seed=seed, roughness=np.array([a0 + h], np.float32))
        im = orc.render(spp=128, max_depth=3, seed=seed, roughness=np.array([a0 - h], np.float32))
        step = float(np.float32(a0 + h)) - float(np.float32(a0 - h))
        g.append(gr[0])
        fd.append(float((adj * (ip - im)).sum()) / step)
    g, fd = np.array(g), np.array(fd)
    diff = g - fd
    se = diff.std(ddof=1) / math.sqrt(len(diff))
    assert abs(fd.mean()) > 3 * fd.std(ddof=1) / math.sqrt(len(fd))
    assert abs(diff.mean()) <= max(2e-2 * abs(fd.mean()), 3 * se), (g.mean(), fd.mean(), se)
    assert 3 * se < 0.15 * abs(fd.mean())     # the comparison resolves a 15% error


def test_loss_l2_closed_form():
    img = np.array([1.0, 2.0, 3.0, 4.0])
    tgt = np.array([0.0, 2.0, 5.0, 3.0])
    loss, adj = oracle.loss_l2(img, tgt)
    assert loss == (1 + 0 + 4 + 1) / 4
    np.testing.assert_allclose(adj, [0.5, 0.0, -1.0, 0.5])


def test_adam_first_step_closed_form():
    g = np.array([1e-3, -2.0, 0.0, 5e-9])
    p = np.zeros(4); m = np.zeros(4); v = np.zeros(4)
    oracle.adam(p, g, m, v, lr=1e-2, b1=0.9, b2=0.99, eps=1e-8, t=1)
    np.testing.assert_allclose(p, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    oracle.adam(p, g, m, v, lr=1e-2, b1=0.9, b2=0.99, eps=1e-8, t=2, lo=-0.015, hi=1.0)
    assert p.min() >= -0.015
