"""drt_render_adjoint_noalloc (the replay from intersection records with the
records in the library's own device scratch) against drt_render_adjoint_hits
(the same replay with a caller buffer), through the C ABI, on two calls in a
row -- the second on a smaller input, so the scratch holds the first call's
records when it starts -- and both against the FP64 oracle.

Tolerances: gradients vs the oracle as in test_gpu_parity (check_grad); the
two GPU entry points run the same kernels and differ only in the order of
their float atomics and in which persistent workgroup sums which samples of
the roughness in LDS: texture gradients within 1e-6 (relative L2),
roughness within 1e-5 relative.
"""
import numpy as np
import pytest

import oracle
import scenes
from test_gpu_parity import check_grad, unambiguous_adjoint

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _drt():
    import paper_2202_01284_amd as drt
    return drt


CALLS = [
    # (width, height, spp, max_depth, seed): ragged tiles; the second is smaller
    (40, 24, 5, 3, 11),
    (24, 16, 3, 2, 12),
]


def test_noalloc_matches_caller_buffer_twice():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    drt = _drt()
    for W, H, spp, depth, seed in CALLS:
        print(f"noalloc call: {W}x{H} spp {spp} depth {depth} seed {seed}", flush=True)
        sc = scenes.cornell(conductor=True, texture=scenes.random_texture(64), width=W, height=H)
        gs = drt.Scene(sc)
        tex = [torch.from_numpy(np.ascontiguousarray(t)).cuda() for t in sc.textures]
        rough = torch.from_numpy(np.ascontiguousarray(sc.roughness)).cuda()
        orc = oracle.OracleScene(sc)
        _, amb = orc.render(spp=spp, max_depth=depth, seed=seed, ambiguity=True)
        adj = unambiguous_adjoint(orc, np.random.default_rng(seed).normal(size=(1, H, W, 3))
                                  .astype(np.float32), amb)
        a = torch.from_numpy(adj).cuda()
        gt_n = [torch.zeros_like(t) for t in tex]
        gr_n = torch.zeros_like(rough)
        drt.render_adjoint_noalloc(gs, tex, rough, sc.cameras, a, spp, depth, gt_n, gr_n, seed=seed)
        gt_h, gr_h = drt.render_adjoint(gs, tex, rough, sc.cameras, a, spp, depth, seed=seed,
                                        hit_records=drt.adjoint_hit_records(sc.cameras, spp, depth))
        torch.cuda.synchronize()
        n, h = gt_n[0].double(), gt_h[0].double()
        r = float((n - h).norm() / h.norm())
        print(f"  texture: noalloc vs caller buffer rel {r:.3g}", flush=True)
        assert r <= 1e-6
        assert np.allclose(gr_n.cpu().numpy(), gr_h.cpu().numpy(), rtol=1e-5, atol=1e-9)
        ot, orr = orc.adjoint(adj.astype(np.float64), spp=spp, max_depth=depth, seed=seed)
        check_grad(gt_n[0].cpu().numpy(), ot[0], f"noalloc {W}x{H} texture")
        check_grad(gr_n.cpu().numpy(), orr, f"noalloc {W}x{H} roughness")


def test_noalloc_refuses_sizes_beyond_its_scratch():
    drt = _drt()
    sc = scenes.cornell(conductor=True, texture=scenes.random_texture(64), width=1024, height=1024)
    gs = drt.Scene(sc)
    tex = [torch.from_numpy(np.ascontiguousarray(t)).cuda() for t in sc.textures]
    rough = torch.from_numpy(np.ascontiguousarray(sc.roughness)).cuda()
    need = int(drt.lib.drt_render_adjoint_hit_bytes(1, 1024, 1024, 16, 64))
    assert need > drt.NOALLOC_SCRATCH_BYTES
    a = torch.zeros((1, 1024, 1024, 3), dtype=torch.float32, device="cuda")
    g = [torch.zeros_like(t) for t in tex]
    with pytest.raises(drt.DrtError, match="scratch"):
        drt.render_adjoint_noalloc(gs, tex, rough, sc.cameras, a, 16, 64, g, torch.zeros_like(rough))
    # nothing was enqueued: the gradient buffers are untouched
    torch.cuda.synchronize()
    assert float(g[0].abs().sum()) == 0.0
