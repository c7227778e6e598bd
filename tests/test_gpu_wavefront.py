"""Wavefront variant of the primal renderer against the megakernel on the
same sample streams (same device functions and arithmetic order: images
agree to float rounding -- |w - m| <= 1e-5 |m| + 1e-7 on >= 99.9% of pixel
channels, the rest are samples whose FP32 decision flips between two
contraction patterns), and against the oracle as the forward parity tests."""
import numpy as np
import pytest

import oracle
import scenes
from test_gpu_parity import FWD_CASES, _params, check_image

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _drt():
    import paper_2202_01284_amd as drt
    return drt


@pytest.mark.parametrize("case", list(FWD_CASES))
def test_wavefront_equals_megakernel_and_oracle(case):
    drt = _drt()
    make, kw = FWD_CASES[case]
    sc = make()
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    rr = kw.get("rr_depth", drt.NO_RR)
    args = (gs, tex, rough, sc.cameras, kw["spp"], kw["max_depth"], rr)
    wf = drt.render_wavefront(*args, seed=1, flags=kw.get("flags", 0)).cpu().numpy()
    mk = drt.render_forward(*args, seed=1, flags=kw.get("flags", 0)).cpu().numpy()
    close = np.abs(wf - mk) <= 1e-5 * np.abs(mk) + 1e-7
    print(case, "wavefront vs megakernel: identical", float((wf == mk).mean()), "close", float(close.mean()),
          flush=True)
    assert close.mean() >= 0.999
    ref, amb = oracle.OracleScene(sc).render(spp=kw["spp"], max_depth=kw["max_depth"], rr_depth=rr,
                                             flags=kw.get("flags", 0), seed=1, ambiguity=True)
    check_image(wf, ref, case + " wavefront", amb)


def test_wavefront_multi_camera_and_workspace_check():
    drt = _drt()
    sc = scenes.cornell(conductor=True, texture=scenes.random_texture(64),
                        cameras=scenes.ring_cameras(3, 40, 24))
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    wf = drt.render_wavefront(gs, tex, rough, sc.cameras, 3, 3, seed=7).cpu().numpy()
    mk = drt.render_forward(gs, tex, rough, sc.cameras, 3, 3, seed=7).cpu().numpy()
    assert (np.abs(wf - mk) <= 1e-5 * np.abs(mk) + 1e-7).mean() >= 0.999
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError, match="workspace"):
        drt.render_wavefront(gs, tex, rough, sc.cameras, 3, 3, seed=7, workspace=small)


@pytest.mark.parametrize("case", ["cornell_c1", "cornell_conductor", "zoo"])
def test_wavefront_adjoint_equals_megakernel_and_oracle(case):
    """The wavefront replay against the megakernel's (same seed: equal up to
    float rounding and atomic order, relative L2 <= 1e-5) and the oracle
    (gradient tolerance, pixels with FP32-reach decisions set aside)."""
    from test_gpu_parity import ADJ_CASES, check_grad, unambiguous_adjoint
    drt = _drt()
    make, kw = ADJ_CASES[case]
    sc = make()
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    c = sc.cameras[0]
    rr = kw.get("rr_depth", drt.NO_RR)
    orc = oracle.OracleScene(sc)
    _, amb = orc.render(spp=kw["spp"], max_depth=kw["max_depth"], rr_depth=rr, seed=2, ambiguity=True)
    adj = unambiguous_adjoint(orc, np.random.default_rng(5).normal(size=(1, c.height, c.width, 3))
                              .astype(np.float32), amb)
    a = torch.from_numpy(adj).cuda()
    wt, wr = drt.render_adjoint_wavefront(gs, tex, rough, sc.cameras, a, kw["spp"], kw["max_depth"], rr, seed=2)
    mt, mr = drt.render_adjoint(gs, tex, rough, sc.cameras, a, kw["spp"], kw["max_depth"], rr, seed=2)
    for i, (w, m) in enumerate(zip(wt, mt)):
        w, m = w.cpu().numpy().astype(np.float64), m.cpu().numpy().astype(np.float64)
        r = np.linalg.norm(w - m) / np.linalg.norm(m)
        print(case, f"texture {i}: wavefront vs megakernel rel {r:.3g}", flush=True)
        assert r <= 1e-5
    if len(sc.roughness):
        assert np.allclose(wr.cpu().numpy(), mr.cpu().numpy(), rtol=1e-5, atol=1e-9)
    ot, orr = orc.adjoint(adj.astype(np.float64), spp=kw["spp"], max_depth=kw["max_depth"], rr_depth=rr,
                          seed=2)
    for i, (g, o) in enumerate(zip(wt, ot)):
        check_grad(g.cpu().numpy(), o, f"{case} wavefront texture {i}")
    if len(sc.roughness):
        check_grad(wr.cpu().numpy(), orr, f"{case} wavefront roughness")


@pytest.mark.parametrize("case", ["cornell_c1", "cornell_conductor", "zoo"])
def test_checkpointed_adjoint_equals_replay_and_oracle(case):
    """Checkpointed adjoint (forward with one checkpoint per bounce, then the
    backward walk): its image is the wavefront primal's, bit for bit, and its
    gradient (same seed) the replayed adjoint's up to float rounding and
    atomic order, and the oracle's within the gradient tolerance."""
    from test_gpu_parity import ADJ_CASES, check_grad, unambiguous_adjoint
    drt = _drt()
    make, kw = ADJ_CASES[case]
    sc = make()
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    c = sc.cameras[0]
    rr = kw.get("rr_depth", drt.NO_RR)
    spp, D = kw["spp"], kw["max_depth"]
    orc = oracle.OracleScene(sc)
    _, amb = orc.render(spp=spp, max_depth=D, rr_depth=rr, seed=2, ambiguity=True)
    adj = unambiguous_adjoint(orc, np.random.default_rng(6).normal(size=(1, c.height, c.width, 3))
                              .astype(np.float32), amb)
    a = torch.from_numpy(adj).cuda()
    img, ws = drt.render_checkpointed_forward(gs, tex, rough, sc.cameras, spp, D, rr, seed=2)
    wf = drt.render_wavefront(gs, tex, rough, sc.cameras, spp, D, rr, seed=2)
    np.testing.assert_array_equal(img.cpu().numpy(), wf.cpu().numpy())
    ct, cr = drt.render_checkpointed_adjoint(gs, tex, rough, sc.cameras, a, spp, D, ws, rr, seed=2)
    mt, mr = drt.render_adjoint(gs, tex, rough, sc.cameras, a, spp, D, rr, seed=2)
    for i, (w, m) in enumerate(zip(ct, mt)):
        w, m = w.cpu().numpy().astype(np.float64), m.cpu().numpy().astype(np.float64)
        r = np.linalg.norm(w - m) / np.linalg.norm(m)
        print(case, f"texture {i}: checkpointed vs replay rel {r:.3g}", flush=True)
        assert r <= 1e-5
    if len(sc.roughness):
        assert np.allclose(cr.cpu().numpy(), mr.cpu().numpy(), rtol=1e-5, atol=1e-9)
    ot, orr = orc.adjoint(adj.astype(np.float64), spp=spp, max_depth=D, rr_depth=rr, seed=2)
    for i, (g, o) in enumerate(zip(ct, ot)):
        check_grad(g.cpu().numpy(), o, f"{case} checkpointed texture {i}")
    if len(sc.roughness):
        check_grad(cr.cpu().numpy(), orr, f"{case} checkpointed roughness")


def test_checkpointed_workspace_and_degenerate_depth():
    """The workspace grows by one 64-byte checkpoint per path and bounce and
    too small a one is refused; with max depth 1 (camera rays only) nothing
    is differentiable and the gradient stays zero."""
    drt = _drt()
    sc = scenes.cornell(conductor=True, texture=scenes.random_texture(64), width=24, height=16)
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    n = 24 * 16 * 2
    b3 = int(drt.lib.drt_render_checkpointed_workspace_bytes(n, 3))
    b4 = int(drt.lib.drt_render_checkpointed_workspace_bytes(n, 4))
    assert b4 - b3 == n * 64
    small = torch.empty(b3 - 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError, match="workspace"):
        drt.render_checkpointed_forward(gs, tex, rough, sc.cameras, 2, 3, workspace=small)
    img, ws = drt.render_checkpointed_forward(gs, tex, rough, sc.cameras, 2, 1, seed=3)
    ref = drt.render_forward(gs, tex, rough, sc.cameras, 2, 1, seed=3)
    assert (np.abs(img.cpu().numpy() - ref.cpu().numpy()) <= 1e-6).all()
    a = torch.ones((1, 16, 24, 3), device="cuda")
    gt, gr = drt.render_checkpointed_adjoint(gs, tex, rough, sc.cameras, a, 2, 1, ws, seed=3)
    assert float(gt[0].abs().max()) == 0.0 and float(gr.abs().max()) == 0.0
