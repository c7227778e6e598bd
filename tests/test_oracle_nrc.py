"""Pins of the oracle's radiance-cache pieces (CPU only): spherical
harmonics identities, hash-grid interpolation and adjointness, the network's
gradients against finite differences, BF16 rounding against torch, the
relative-L2 loss, and the cached estimator's and training targets'
definitions."""
import math

import numpy as np
import pytest

import oracle
import scenes


def _sphere_grid(n_th=120, n_ph=240):
    th = (np.arange(n_th) + 0.5) / n_th * math.pi
    ph = (np.arange(n_ph) + 0.5) / n_ph * 2 * math.pi
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    w = np.sin(TH) * (math.pi / n_th) * (2 * math.pi / n_ph)
    d = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1)
    return d.reshape(-1, 3), w.reshape(-1)


def test_sh16_orthonormal_by_quadrature():
    d, w = _sphere_grid()
    Y = np.array([oracle.sh16(v) for v in d])
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=2e-4)


def test_sh16_band_sums():
    rng = np.random.default_rng(1)
    for _ in range(20):
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        Y = oracle.sh16(v)
        for l, (a, b) in enumerate([(0, 1), (1, 4), (4, 9), (9, 16)]):
            assert math.isclose((Y[a:b] ** 2).sum(), (2 * l + 1) / (4 * math.pi), rel_tol=1e-12)


def _cfg(log2_table=19):
    return dict(levels=16, features=2, log2_table=log2_table, base_res=16, max_res=2048,
                bbox_lo=[-1.0, 0.0, -1.0], bbox_hi=[1.0, 2.0, 1.0], trunc_vertex=3)


def test_level_resolutions_geometric():
    cfg = _cfg()
    res = [oracle.level_res(cfg, l) for l in range(16)]
    assert res[0] == 16 and res[-1] == 2048
    b = math.exp((math.log(2048) - math.log(16)) / 15)
    for l in range(16):
        assert res[l] == math.floor(16 * b ** l + 1e-6)


def test_grid_dense_level_reproduces_linear_function():
    """At a dense level, corner values a.c + k reproduce a linear function of
    the scaled position exactly (trilinear interpolation of a linear map)."""
    cfg = _cfg()
    T = 1 << cfg["log2_table"]
    grid = np.zeros((16, T, 2), np.float32)
    rng = np.random.default_rng(2)
    for l in range(3):                      # levels 0..2 are dense
        N = oracle.level_res(cfg, l)
        i, j, k = np.meshgrid(np.arange(N + 1), np.arange(N + 1), np.arange(N + 1), indexing="ij")
        lin = i + (N + 1) * j + (N + 1) ** 2 * k
        grid[l, lin.reshape(-1), 0] = (0.25 * i + 0.5 * j - 0.125 * k).reshape(-1)
        grid[l, lin.reshape(-1), 1] = (1.0 + 0.0625 * i).reshape(-1)
    lo, hi = np.array(cfg["bbox_lo"]), np.array(cfg["bbox_hi"])
    feat = np.zeros((200, 13))
    feat[:, 0:3] = lo + rng.random((200, 3)) * (hi - lo)
    feat[:, 3] = 1.0
    feat[:, 6] = 1.0
    enc = oracle.nrc_encode(feat, cfg, grid)
    xn = (feat[:, 0:3] - lo) / (hi - lo)
    for l in range(3):
        N = oracle.level_res(cfg, l)
        p = xn * N
        np.testing.assert_allclose(enc[:, 2 * l], 0.25 * p[:, 0] + 0.5 * p[:, 1] - 0.125 * p[:, 2],
                                   atol=1e-5)
        np.testing.assert_allclose(enc[:, 2 * l + 1], 1.0 + 0.0625 * p[:, 0], atol=1e-6)


def test_grid_weights_partition_unity_and_indices_in_range():
    cfg = _cfg()
    rng = np.random.default_rng(3)
    for l in (0, 4, 5, 10, 15):
        for xn in rng.random((20, 3)):
            idx, w = oracle.grid_corners(cfg, l, xn)
            assert abs(w.sum() - 1) < 1e-12 and (w >= 0).all()
            assert (idx < (1 << cfg["log2_table"])).all()


def test_grid_backward_is_adjoint_of_encode():
    """The encoding is linear in the table: <backward(dF), table> = <dF, encode(table)>."""
    cfg = _cfg(log2_table=12)              # small table: every level past 1 is hashed
    T = 1 << 12
    rng = np.random.default_rng(4)
    grid = rng.uniform(-1, 1, (16, T, 2)).astype(np.float32)
    lo, hi = np.array(cfg["bbox_lo"]), np.array(cfg["bbox_hi"])
    feat = np.zeros((64, 13))
    feat[:, 0:3] = lo + rng.random((64, 3)) * (hi - lo)
    feat[:, 3] = feat[:, 7] = 1.0
    enc = oracle.nrc_encode(feat, cfg, grid)
    dF = np.zeros((64, 80))
    dF[:, :32] = rng.normal(size=(64, 32))
    g = oracle.nrc_grid_backward(feat, cfg, dF)
    lhs = float(g @ grid.reshape(-1).astype(np.float64))
    rhs = float((dF[:, :32] * enc[:, :32]).sum())
    assert math.isclose(lhs, rhs, rel_tol=1e-10)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.normal(size=2000) * 10 ** rng.uniform(-8, 4, 2000),
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5 - 2 ** -7]])
    want = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    W = np.zeros(oracle.mlp_num_weights())
    # route through the network: identity-like first layer is not available,
    # so compare via the forward of a one-hot input selecting each value
    x = np.zeros((1, 80))
    x[0, 0] = 1.0
    got = []
    for val in v:
        W[:] = 0
        W[0] = val                      # W0[0][0]
        W[64 * 80 + 0] = 1.0            # W1[0][0]
        W[64 * 80 + 3 * 64 * 64 + 0] = 1.0  # W4[0][0]  (via W2, W3 below)
        W[64 * 80 + 64 * 64] = 1.0      # W2[0][0]
        W[64 * 80 + 2 * 64 * 64] = 1.0  # W3[0][0]
        y = oracle.mlp_forward(x, W, emu=True)[0, 0]
        got.append(y)
    got = np.array(got)
    pos = v > 0                          # ReLU passes positive values only
    np.testing.assert_array_equal(got[pos], want[pos])
    assert (got[~pos] == 0).all()


def test_mlp_gradients_against_finite_differences():
    rng = np.random.default_rng(6)
    W = rng.normal(size=oracle.mlp_num_weights()) * 0.2
    x = rng.normal(size=(4, 80))
    dy = rng.normal(size=(4, 3))
    dW, dx = oracle.mlp_backward(x, W, dy, emu=False)
    f = lambda Wv, xv: float((oracle.mlp_forward(xv, Wv) * dy).sum())
    h = 1e-6
    for k in rng.choice(W.size, 40, replace=False):
        Wp, Wm = W.copy(), W.copy()
        Wp[k] += h
        Wm[k] -= h
        assert math.isclose(dW[k], (f(Wp, x) - f(Wm, x)) / (2 * h), rel_tol=1e-5, abs_tol=1e-8)
    for (i, j) in [(0, 0), (1, 17), (2, 40), (3, 67)]:
        xp, xm = x.copy(), x.copy()
        xp[i, j] += h
        xm[i, j] -= h
        assert math.isclose(dx[i, j], (f(W, xp) - f(W, xm)) / (2 * h), rel_tol=1e-5, abs_tol=1e-8)


def test_mlp_term_magnitudes():
    """The tolerance scales of the network parity tests: for one sample a
    weight gradient is a single term, so its magnitude sum is |dW|; over
    samples the sums add; with non-negative weights, inputs and output
    gradients every term is non-negative, so the sums equal y, dW and dx;
    otherwise they bound them."""
    rng = np.random.default_rng(8)
    n_w = oracle.mlp_num_weights()
    W = rng.normal(size=n_w) * 0.2
    x = rng.normal(size=(2, 80))
    dy = rng.normal(size=(2, 3))
    for emu in (False, True):
        single = []
        for i in range(2):
            dWi, _ = oracle.mlp_backward(x[i:i + 1], W, dy[i:i + 1], emu=emu)
            aWi, _, _ = oracle.mlp_term_magnitudes(x[i:i + 1], W, dy[i:i + 1], emu=emu)
            np.testing.assert_array_equal(aWi, np.abs(dWi))
            single.append(aWi)
        dW, dx = oracle.mlp_backward(x, W, dy, emu=emu)
        aW, adx, ay = oracle.mlp_term_magnitudes(x, W, dy, emu=emu)
        np.testing.assert_allclose(aW, single[0] + single[1], rtol=1e-15, atol=0)
        assert np.all(aW >= np.abs(dW) * (1 - 1e-15))
        assert np.all(adx >= np.abs(dx) * (1 - 1e-12))
        y = oracle.mlp_forward(x, W, emu=emu)
        assert np.all(ay >= np.abs(y) * (1 - 1e-12))
        assert (adx > np.abs(dx) * 1.01).any() and (ay > np.abs(y) * 1.01).any()
    Wp, xp, dyp = np.abs(W), np.abs(x), np.abs(dy)
    dW, dx = oracle.mlp_backward(xp, Wp, dyp)
    aW, adx, ay = oracle.mlp_term_magnitudes(xp, Wp, dyp)
    np.testing.assert_allclose(aW, dW, rtol=1e-13)
    np.testing.assert_allclose(adx, dx, rtol=1e-13)
    np.testing.assert_allclose(ay, oracle.mlp_forward(xp, Wp), rtol=1e-13)


def test_mlp_bf16_mode_close_to_fp64():
    rng = np.random.default_rng(7)
    W = rng.normal(size=oracle.mlp_num_weights()) * 0.15
    x = rng.normal(size=(64, 80))
    y0 = oracle.mlp_forward(x, W, emu=False)
    y1 = oracle.mlp_forward(x, W, emu=True)
    rel = np.linalg.norm(y1 - y0) / np.linalg.norm(y0)
    assert 1e-5 < rel < 3e-2


def test_relative_l2_closed_form_and_gradient():
    y = np.array([[1.0, 0.0, -0.5]])
    t = np.array([[0.5, 0.1, 0.0]])
    loss, dy = oracle.rel_l2(y, t)
    want = ((0.5 ** 2) / 1.01 + 0.01 / 0.01 + 0.25 / 0.26) / 3
    assert math.isclose(loss, want, rel_tol=1e-12)
    np.testing.assert_allclose(dy, 2 * (y - t) / (y ** 2 + 0.01) / 3, rtol=1e-12)


def test_cached_estimator_with_zero_network_equals_truncated_plain():
    """C = 0: the cached estimator is the plain one with max depth K (no
    pass-through surfaces in this scene), sample for sample."""
    sc = scenes.cornell(texture=scenes.random_texture(64))
    cfg = scenes.nrc_config(sc)
    _, grid = scenes.nrc_init(cfg)
    W = np.zeros(oracle.mlp_num_weights())
    orc = oracle.OracleScene(sc)
    a = orc.render_cached(cfg, grid, W, K=3, spp=2, max_depth=6, rr_depth=3, seed=9)
    b = orc.render(spp=2, max_depth=3, seed=9)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)


def test_training_targets_reassemble_the_plain_estimator():
    """Per path, L_before + beta * target is the path's radiance; over paths
    started at uniformly chosen pixels its mean is the plain image's mean."""
    sc = scenes.cornell(texture=scenes.random_texture(64), width=32, height=32)
    orc = oracle.OracleScene(sc)
    n = 1 << 16
    feat, tgt, valid, _, beta, lat, ltot = orc.train_records(n, K=3, max_depth=6, rr_depth=3,
                                                             seed=21, extra=True)
    assert 0.2 < valid.mean() < 1.0
    assert np.isfinite(tgt).all() and (tgt[~valid] == 0).all()
    d, nn = feat[valid, 3:6], feat[valid, 6:9]
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1, atol=1e-12)
    assert ((d * nn).sum(1) >= 0).all()
    np.testing.assert_allclose((lat + beta * tgt)[valid], ltot[valid], rtol=1e-12, atol=1e-12)
    img = orc.render(spp=256, max_depth=6, rr_depth=3, seed=22)
    m, se = ltot.mean(), ltot.mean(1).std() / math.sqrt(n)
    assert abs(m - img.mean()) < 4 * se + 4 * img.mean(2).std() / math.sqrt(img.size // 3 * 256), (m, img.mean())


def _constant_network(c=(1.5, 1.0, 0.5)):
    """Weights whose output is the constant c * Y_00: only the band-0 SH input
    of the outgoing direction (input 32, constant over the sphere) feeds one
    ReLU chain."""
    W = np.zeros(oracle.mlp_num_weights())
    W[32] = 1.0                               # layer 0, row 0, column 32
    W[64 * 80] = W[64 * 80 + 4096] = W[64 * 80 + 2 * 4096] = 1.0
    for ch in range(3):
        W[64 * 80 + 3 * 4096 + ch * 64] = c[ch]
    return W


def test_constant_network_output():
    W = _constant_network()
    x = np.random.default_rng(3).normal(size=(5, 80))
    x[:, 32] = 0.5 / math.sqrt(math.pi)
    np.testing.assert_allclose(oracle.mlp_forward(x, W), np.tile([1.5, 1.0, 0.5], (5, 1)) * x[:, 32:33],
                               rtol=1e-14)


def test_cached_adjoint_with_zero_network_equals_truncated_plain():
    sc = scenes.cornell(texture=scenes.random_texture(16), width=16, height=16, conductor=True)
    cfg = scenes.nrc_config(sc)
    _, grid = scenes.nrc_init(cfg)
    orc = oracle.OracleScene(sc)
    adj = np.random.default_rng(5).normal(size=(1, 16, 16, 3))
    ga, ra = orc.adjoint_cached(cfg, grid, np.zeros(oracle.mlp_num_weights()), adj, K=3, spp=2,
                                max_depth=6, rr_depth=3, seed=4)
    gb, rb = orc.adjoint(adj, spp=2, max_depth=3, seed=4)
    np.testing.assert_allclose(ga[0], gb[0], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(ra, rb, rtol=1e-12, atol=1e-15)


def test_cached_adjoint_matches_central_differences():
    """With a cache whose output does not depend on its inputs the cached
    estimator is a polynomial of degree <= 2 in the texels (two scattering
    vertices before the record vertex, no RR before it), so central
    differences are exact up to rounding."""
    sc = scenes.cornell(texture=scenes.random_texture(8), width=16, height=16)
    cfg = scenes.nrc_config(sc)
    _, grid = scenes.nrc_init(cfg)
    W = _constant_network()
    orc = oracle.OracleScene(sc)
    rng = np.random.default_rng(6)
    adj = rng.normal(size=(1, 16, 16, 3))
    kw = dict(K=3, spp=2, max_depth=6, rr_depth=3, seed=8, emu=False)
    # texels on a 2^-10 grid, step 2^-6: the perturbed texels are exact in float32
    tex = (np.round(sc.textures[0].astype(np.float64) * 1024) / 1024).astype(np.float32)
    (g,), _ = orc.adjoint_cached(cfg, grid, W, adj, textures=[tex], **kw)
    assert np.abs(g).max() > 0
    h = 1.0 / 64
    for trial in range(6):
        v = np.zeros_like(tex)
        sel = rng.choice(tex.size, 12, replace=False)
        v.reshape(-1)[sel] = rng.choice([-1.0, 1.0], 12)
        if trial == 0:
            v = rng.choice([-1.0, 1.0], tex.shape).astype(np.float32)
        ip = orc.render_cached(cfg, grid, W, textures=[tex + h * v], **{k: kw[k] for k in kw})
        im = orc.render_cached(cfg, grid, W, textures=[tex - h * v], **{k: kw[k] for k in kw})
        fd = float(((ip - im) * adj).sum() / (2 * h))
        an = float((g * v).sum())
        assert math.isclose(an, fd, rel_tol=1e-9, abs_tol=1e-12), (trial, an, fd)


def _linear_network(c=(0.5, 0.4, 0.3), a=(0.8, 1.1, 0.6), b=(0.7, 0.2, 0.9)):
    """Weights whose output is c * Y_00 + a * albedo + b * roughness, per
    channel: hidden units 0..4 carry the band-0 SH input (32), the three
    albedo inputs (65..67) and the roughness input (64) unchanged through the
    ReLU layers (all of them are >= 0)."""
    W = np.zeros(oracle.mlp_num_weights())
    W[0 * 80 + 32] = 1.0
    for ch in range(3):
        W[(1 + ch) * 80 + 65 + ch] = 1.0
    W[4 * 80 + 64] = 1.0
    for layer in range(3):
        off = 64 * 80 + layer * 4096
        for r in range(5):
            W[off + r * 64 + r] = 1.0
    off = 64 * 80 + 3 * 4096
    for ch in range(3):
        W[off + ch * 64 + 0] = c[ch]
        W[off + ch * 64 + 1 + ch] = a[ch]
        W[off + ch * 64 + 4] = b[ch]
    return W


def test_linear_network_output():
    W = _linear_network()
    x = np.random.default_rng(4).uniform(0.0, 1.0, size=(6, 80))
    y = oracle.mlp_forward(x, W)
    want = (np.array([0.5, 0.4, 0.3]) * x[:, 32:33] + np.array([0.8, 1.1, 0.6]) * x[:, 65:68]
            + np.array([0.7, 0.2, 0.9]) * x[:, 64:65])
    np.testing.assert_allclose(y, want, rtol=1e-14)


def test_cached_adjoint_through_inputs_matches_differences_of_the_estimator():
    """With a network linear in the albedo input, the cached estimator at
    K = 3 is a polynomial of degree <= 3 in the texels (albedo at the two
    scattering vertices before the record vertex and at the record vertex),
    so the Richardson combination of central differences at h and 2h is
    exact up to rounding.  The gradient through the network's inputs must
    match it; the detached gradient must not."""
    sc = scenes.cornell(texture=scenes.random_texture(8), width=16, height=16)
    cfg = scenes.nrc_config(sc)
    _, grid = scenes.nrc_init(cfg)
    W = _linear_network()
    orc = oracle.OracleScene(sc)
    rng = np.random.default_rng(12)
    adj = rng.normal(size=(1, 16, 16, 3))
    kw = dict(K=3, spp=2, max_depth=6, rr_depth=3, seed=9, emu=False)
    # texels on a 2^-10 grid inside [0.1, 0.9], steps of 2^-6 and 2^-5: exact in float32
    t0 = np.clip(sc.textures[0].astype(np.float64), 0.1, 0.9)
    tex = (np.round(t0 * 1024) / 1024).astype(np.float32)
    (g,), _ = orc.adjoint_cached(cfg, grid, W, adj, textures=[tex], input_grad=True, **kw)
    (g0,), _ = orc.adjoint_cached(cfg, grid, W, adj, textures=[tex], **kw)

    def fd(v, h):
        ip = orc.render_cached(cfg, grid, W, textures=[tex + h * v], **kw)
        im = orc.render_cached(cfg, grid, W, textures=[tex - h * v], **kw)
        return float(((ip - im) * adj).sum() / (2 * h))

    for trial in range(4):
        v = np.zeros_like(tex)
        sel = rng.choice(tex.size, 16, replace=False)
        v.reshape(-1)[sel] = rng.choice([-1.0, 1.0], 16)
        if trial == 0:
            v = rng.choice([-1.0, 1.0], tex.shape).astype(np.float32)
        h = 1.0 / 64
        ref = (4.0 * fd(v, h) - fd(v, 2 * h)) / 3.0
        an, an0 = float((g * v).sum()), float((g0 * v).sum())
        assert math.isclose(an, ref, rel_tol=1e-8, abs_tol=1e-12), (trial, an, ref)
        if trial == 0:
            assert abs(an - an0) > 1e-3 * abs(an), (an, an0)


def test_cached_adjoint_through_roughness_input_at_the_first_vertex():
    """Record vertex K = 1: the cached estimator is the emission seen by the
    camera ray plus C(features of its hit), linear in the roughness of the
    GGX conductor and in the texels through this network, so central
    differences are exact.  This pins the roughness feature's slot and the
    texel lookup of the albedo feature."""
    sc = scenes.cornell(texture=scenes.random_texture(8), width=16, height=16, conductor=True,
                        roughness=0.25)
    cfg = scenes.nrc_config(sc)
    _, grid = scenes.nrc_init(cfg)
    W = _linear_network()
    orc = oracle.OracleScene(sc)
    rng = np.random.default_rng(13)
    adj = rng.normal(size=(1, 16, 16, 3))
    kw = dict(K=1, spp=2, max_depth=6, rr_depth=3, seed=10, emu=False)
    tex = (np.round(sc.textures[0].astype(np.float64) * 1024) / 1024).astype(np.float32)
    rough = np.array([0.25], np.float32)
    (g,), gr = orc.adjoint_cached(cfg, grid, W, adj, textures=[tex], roughness=rough,
                                  input_grad=True, **kw)
    (g0,), gr0 = orc.adjoint_cached(cfg, grid, W, adj, textures=[tex], roughness=rough, **kw)
    assert np.all(g0 == 0) and np.all(gr0 == 0)   # nothing before the record vertex
    h = 1.0 / 64
    ip = orc.render_cached(cfg, grid, W, textures=[tex], roughness=rough + h, **kw)
    im = orc.render_cached(cfg, grid, W, textures=[tex], roughness=rough - h, **kw)
    fd = float(((ip - im) * adj).sum() / (2 * h))
    assert abs(gr[0]) > 1e-6
    assert math.isclose(float(gr[0]), fd, rel_tol=1e-9, abs_tol=1e-13), (gr[0], fd)
    v = rng.choice([-1.0, 1.0], tex.shape).astype(np.float32)
    ip = orc.render_cached(cfg, grid, W, textures=[tex + h * v], roughness=rough, **kw)
    im = orc.render_cached(cfg, grid, W, textures=[tex - h * v], roughness=rough, **kw)
    fd = float(((ip - im) * adj).sum() / (2 * h))
    assert math.isclose(float((g * v).sum()), fd, rel_tol=1e-9, abs_tol=1e-13)


def test_cached_adjoint_input_term_vanishes_without_input_weights():
    """A network that ignores its albedo and roughness inputs adds nothing
    through them."""
    sc = scenes.cornell(texture=scenes.random_texture(8), width=16, height=16, conductor=True)
    cfg = scenes.nrc_config(sc)
    W, grid = scenes.nrc_init(cfg)
    W = np.array(W, np.float64)
    W[np.arange(64)[:, None] * 80 + np.arange(64, 68)[None, :]] = 0.0
    orc = oracle.OracleScene(sc)
    adj = np.random.default_rng(14).normal(size=(1, 16, 16, 3))
    kw = dict(K=3, spp=2, max_depth=6, rr_depth=3, seed=11, threads=1)  # one summation order
    (g,), gr = orc.adjoint_cached(cfg, grid, W, adj, input_grad=True, **kw)
    (g0,), gr0 = orc.adjoint_cached(cfg, grid, W, adj, **kw)
    np.testing.assert_array_equal(g, g0)
    np.testing.assert_array_equal(gr, gr0)


def test_self_training_records_without_tail_equal_single_vertex_records():
    """Zero network and max depth = K (so no vertex is ever handed to the
    cache): the self-training record of vertex k is the single-vertex
    training record with record vertex k, path for path (the Cornell scene
    has no pass-through surfaces, so vertex k is the k-th scattering one)."""
    sc = scenes.cornell(texture=scenes.random_texture(16), width=16, height=16, conductor=True)
    cfg = scenes.nrc_config(sc)
    _, grid = scenes.nrc_init(cfg)
    orc = oracle.OracleScene(sc)
    n, K = 2048, 6
    f, t, v, _ = orc.train_records_self(n, cfg, grid, np.zeros(oracle.mlp_num_weights()), K=K,
                                        max_depth=6, rr_depth=3, seed=21)
    f, t, v = f.reshape(n, K - 1, 13), t.reshape(n, K - 1, 3), v.reshape(n, K - 1)
    for k in range(1, K):
        f1, t1, v1, _ = orc.train_records(n, K=k, max_depth=6, rr_depth=3, seed=21)
        np.testing.assert_array_equal(v[:, k - 1], v1)
        np.testing.assert_array_equal(f[:, k - 1], f1)
        np.testing.assert_array_equal(t[:, k - 1], t1)
        assert v1.sum() > n // 16, (k, v1.sum())


def test_self_training_tail_is_the_cache_answer_at_vertex_K():
    """With a constant network c Y_00 the targets move by exactly
    beta_K / beta_k * c Y_00 when the path reaches a scattering vertex K (the
    throughputs from the single-vertex records), and not at all otherwise."""
    sc = scenes.cornell(texture=scenes.random_texture(16), width=16, height=16, conductor=True)
    cfg = scenes.nrc_config(sc)
    _, grid = scenes.nrc_init(cfg)
    orc = oracle.OracleScene(sc)
    n, K, D = 2048, 4, 5
    c = np.array([1.5, 1.0, 0.5]) * 0.5 / math.sqrt(math.pi)
    kw = dict(K=K, max_depth=D, rr_depth=3, seed=23, emu=False)
    _, t0, v0, _ = orc.train_records_self(n, cfg, grid, np.zeros(oracle.mlp_num_weights()), **kw)
    _, tc, vc, _ = orc.train_records_self(n, cfg, grid, _constant_network(), **kw)
    np.testing.assert_array_equal(v0, vc)
    t0, tc, v0 = t0.reshape(n, K - 1, 3), tc.reshape(n, K - 1, 3), v0.reshape(n, K - 1)
    _, _, vK, _, bK, _, _ = orc.train_records(n, K=K, max_depth=D, rr_depth=3, seed=23, extra=True)
    assert 0 < vK.sum() < n
    for k in range(1, K):
        _, _, vk, _, bk, _, _ = orc.train_records(n, K=k, max_depth=D, rr_depth=3, seed=23, extra=True)
        np.testing.assert_array_equal(vk, v0[:, k - 1])
        with np.errstate(divide="ignore", invalid="ignore"):
            want = np.where(vK[:, None] & vk[:, None] & (bk != 0), bK / bk * c, 0.0)
        np.testing.assert_allclose(tc[:, k - 1] - t0[:, k - 1], want, rtol=1e-12, atol=1e-12)
