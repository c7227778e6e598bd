"""Pins of the oracle's forward-mode image derivative (CPU only): central
differences along a texel direction (exact: at depth 3 the estimator is a
polynomial of degree <= 2 in the texels on any line) and the dot-product
identity <dI, J v> = <J^T dI, v> against the independent reverse sweep."""
import math

import numpy as np

import oracle
import scenes


def _scene():
    sc = scenes.cornell(texture=scenes.random_texture(8), width=16, height=16, conductor=True)
    # texels on a 2^-10 grid: perturbations by multiples of 2^-6 are exact in float32
    tex = (np.round(sc.textures[0].astype(np.float64) * 1024) / 1024).astype(np.float32)
    return sc, tex


def test_jvp_matches_central_differences_along_texels():
    sc, tex = _scene()
    orc = oracle.OracleScene(sc)
    rng = np.random.default_rng(1)
    v = rng.choice([-1.0, 1.0], tex.shape)
    kw = dict(spp=2, max_depth=3, seed=5)
    jv = orc.jvp([v], None, textures=[tex], **kw)
    h = 1.0 / 64
    ip = orc.render(textures=[(tex + h * v).astype(np.float32)], **kw)
    im = orc.render(textures=[(tex - h * v).astype(np.float32)], **kw)
    fd = (ip - im) / (2 * h)
    assert np.abs(jv).max() > 0
    np.testing.assert_allclose(jv, fd, rtol=1e-9, atol=1e-12)


def test_jvp_dot_product_identity_with_reverse_sweep():
    sc, tex = _scene()
    orc = oracle.OracleScene(sc)
    rng = np.random.default_rng(2)
    v = rng.normal(size=tex.shape)
    vr = np.array([0.7])
    adj = rng.normal(size=(1, 16, 16, 3))
    kw = dict(spp=2, max_depth=3, seed=6, textures=[tex])
    jv = orc.jvp([v], vr, **kw)
    (gt,), gr = orc.adjoint(adj, mode=0, **kw)
    lhs = float((adj * jv).sum())
    rhs = float((gt * v).sum() + (gr * vr).sum())
    assert math.isclose(lhs, rhs, rel_tol=1e-11), (lhs, rhs)
    # the roughness part alone
    jr = orc.jvp([np.zeros_like(v)], vr, **kw)
    assert math.isclose(float((adj * jr).sum()), float((gr * vr).sum()), rel_tol=1e-11)
