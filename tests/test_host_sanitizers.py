"""The library's host code (argument validation, the SAH build, the
four-wide collapse, the environment tables, packing) under AddressSanitizer
and UndefinedBehaviorSanitizer, on the CPU.

drt_host.cpp is compiled again with the sanitizers on its host pass only
(``-Xarch_host``: the GPU code is built as usual and never runs here), linked
with the library's other objects into a temporary copy of the library, and
driven through the ctypes binding in a child process that preloads the
sanitizer runtime: every scene builder of ``scenes`` plus degenerate and
invalid inputs.  Any report makes the child fail (no recovery).
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_01284_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]

CHILD = r'''
import ctypes, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import paper_2202_01284_amd as drt
import scenes

builders = [scenes.cornell(), scenes.cornell(conductor=True, texture=scenes.random_texture(64)),
            scenes.bsdf_zoo(), scenes.triangle_soup(1, seed=1), scenes.triangle_soup(700, seed=3),
            scenes.furnace_sphere(), scenes.furnace_cube(), scenes.lit_plane(),
            scenes.procedural(n_grid=24, n_spheres=10, sphere_res=(10, 5), env_size=(64, 32),
                              n_lights=3, tex_size=8, width=8, height=8)]
for sc in builders:
    buf, info = drt.scene_pack(sc)
    assert info["n_triangles"] == sc.n_triangles and len(buf) <= drt.scene_plan(sc)

# degenerate geometry: zero-area and repeated triangles, all on one point
b = scenes._Builder()
m = b.material(scenes.BSDF_DIFFUSE)
b.mesh([(0, 0, 0), (0, 0, 0), (0, 0, 0)], np.zeros((3, 2)), [[0, 1, 2]] * 40, m)
b.mesh([(0, 0, 0), (1, 0, 0), (2, 0, 0)], np.zeros((3, 2)), [[0, 1, 2]] * 9, m)
sc = b.build(tex_shapes=[], textures=[], roughness=[], envmap=None, cameras=[], name="degenerate")
drt.scene_pack(sc)

# invalid scenes are refused with a status, not a crash
def refused(mutate):
    sc = scenes.cornell()
    mutate(sc)
    try:
        drt.scene_pack(sc)
    except drt.DrtError:
        return True
    return False
assert refused(lambda sc: sc.indices.__setitem__((3, 1), 10 ** 6))
assert refused(lambda sc: sc.positions.__setitem__((2, 0), np.nan))
assert refused(lambda sc: sc.tri_material.__setitem__(0, 99))
assert refused(lambda sc: sc.mat_type.__setitem__(0, 42))

# size queries at their limits
L = drt.lib
for v in (L.drt_render_adjoint_hit_bytes(32, 2 ** 31 - 1, 2 ** 31 - 1, 16, 1 << 16),
          L.drt_render_wavefront_workspace_bytes(2 ** 62), L.drt_nrc_query_ints(-1),
          L.drt_nrc_collect_self_workspace_bytes(2 ** 40, 2), L.drt_nrc_train_workspace_bytes(-5)):
    assert v == 0
print("sanitized host code ok")
'''


@pytest.mark.slow
def test_host_code_under_asan_and_ubsan():
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    runtime = subprocess.check_output([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                                      text=True).strip()
    if not os.path.exists(runtime):
        pytest.skip("sanitizer runtime not found")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-fno-hip-fp32-correctly-rounded-divide-sqrt", "-fgpu-flush-denormals-to-zero"]
    with tempfile.TemporaryDirectory() as tmp:
        objs = []
        for src in ("drt_kernels.hip", "drt_nrc.hip", "drt_wavefront.hip"):
            prebuilt = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
            if os.path.exists(prebuilt):
                objs.append(prebuilt)
                continue
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            subprocess.check_call([HIPCC, *flags, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
            objs.append(obj)
        host = os.path.join(tmp, "drt_host_san.o")
        subprocess.check_call([HIPCC, *flags, *SAN, "-x", "hip", "-c", os.path.join(CSRC, "drt_host.cpp"),
                               "-o", host])
        lib = os.path.join(tmp, "libdrt_san.so")
        subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", host, *objs,
                               "-shared-libsan", "-Xarch_host", "-fsanitize=address", "-o", lib])
        env = dict(os.environ, DRT_LIBRARY=lib, LD_PRELOAD=runtime,
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True, text=True,
                           timeout=600)
        out = r.stdout + r.stderr
        assert r.returncode == 0, out[-4000:]
        assert "sanitized host code ok" in out
        assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
