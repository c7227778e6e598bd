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
