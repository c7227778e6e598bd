"""Forward-mode image derivative on the GPU (drt_render_jvp) against the
oracle's, and the dot-product identity <dI, J v> = <J^T dI, v> between the
GPU forward mode and the GPU replayed adjoint on the same sample streams.

Tolerances: against the oracle as for gradients (relative L2 <= 1e-3, per
entry 1e-3 on entries >= 1e-2 of the largest), on pixels whose samples take
no FP32-reach decision; the identity within 1e-4 relative (both sides are
FP32 sums of the same per-vertex terms in different orders)."""
import numpy as np
import pytest

import oracle
import scenes
from test_gpu_parity import ADJ_CASES, _params, check_grad

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _drt():
    import paper_2202_01284_amd as drt
    return drt


def _direction(sc, seed):
    rng = np.random.default_rng(seed)
    vt = [rng.normal(size=t.shape).astype(np.float32) for t in sc.textures]
    vr = rng.normal(size=max(1, len(sc.roughness))).astype(np.float32)[:len(sc.roughness)]
    return vt, vr


@pytest.mark.parametrize("case", list(ADJ_CASES))
def test_jvp_vs_oracle(case):
    drt = _drt()
    make, kw = ADJ_CASES[case]
    sc = make()
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    rr = kw.get("rr_depth", drt.NO_RR)
    vt, vr = _direction(sc, 7)
    jv = drt.render_jvp(gs, tex, rough, sc.cameras, kw["spp"], kw["max_depth"], rr, seed=3,
                        tan_textures=[torch.from_numpy(v).cuda() for v in vt],
                        tan_roughness=torch.from_numpy(vr).cuda() if len(vr) else None).cpu().numpy()
    orc = oracle.OracleScene(sc)
    _, amb = orc.render(spp=kw["spp"], max_depth=kw["max_depth"], rr_depth=rr, seed=3, ambiguity=True)
    ref = orc.jvp([v.astype(np.float64) for v in vt], vr.astype(np.float64) if len(vr) else None,
                  spp=kw["spp"], max_depth=kw["max_depth"], rr_depth=rr, seed=3)
    ok = amb.reshape(-1) == 0
    print(case, "pixels set aside:", int((~ok).sum()), flush=True)
    check_grad(jv.reshape(-1, 3)[ok], ref.reshape(-1, 3)[ok], f"{case} jvp")


@pytest.mark.parametrize("case", list(ADJ_CASES))
def test_jvp_adjoint_dot_product_identity(case):
    drt = _drt()
    make, kw = ADJ_CASES[case]
    sc = make()
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    rr = kw.get("rr_depth", drt.NO_RR)
    c = sc.cameras[0]
    vt, vr = _direction(sc, 8)
    adj = np.random.default_rng(9).normal(size=(1, c.height, c.width, 3)).astype(np.float32)
    jv = drt.render_jvp(gs, tex, rough, sc.cameras, kw["spp"], kw["max_depth"], rr, seed=4,
                        tan_textures=[torch.from_numpy(v).cuda() for v in vt],
                        tan_roughness=torch.from_numpy(vr).cuda() if len(vr) else None).cpu().numpy()
    gt, gr = drt.render_adjoint(gs, tex, rough, sc.cameras, torch.from_numpy(adj).cuda(), kw["spp"],
                                kw["max_depth"], rr, seed=4)
    lhs = float((adj.astype(np.float64) * jv).sum())
    rhs = sum(float((g.cpu().numpy().astype(np.float64) * v).sum()) for g, v in zip(gt, vt))
    if len(vr):
        rhs += float((gr.cpu().numpy().astype(np.float64) * vr).sum())
    print(case, "<dI, Jv>", lhs, "<J^T dI, v>", rhs, flush=True)
    assert abs(lhs - rhs) <= 1e-4 * max(abs(lhs), abs(rhs))


def test_jvp_zero_direction_is_zero():
    drt = _drt()
    make, kw = ADJ_CASES["cornell_conductor"]
    sc = make()
    gs = drt.Scene(sc)
    tex, rough = _params(sc)
    jv = drt.render_jvp(gs, tex, rough, sc.cameras, 2, 3, seed=3).cpu().numpy()
    assert np.all(jv == 0)
