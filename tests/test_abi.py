"""CPU checks of the C ABI: the library loads, exports every symbol include/pt.h declares, and
rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ptlib():
    from paper_2503_23412_amd import build, pt
    if not os.path.exists(pt.LIB_PATH):
        build.build()
    return pt


def test_header_symbols_exported(ptlib):
    hdr = open(os.path.join(ROOT, "include", "pt.h")).read()
    decl = set(re.findall(r"^(?:pt_status|const char \*)\s*(pt_\w+)\s*\(", hdr, re.M))
    assert {"pt_scene_upload", "pt_scene_release", "pt_build_subspaces", "pt_render_iteration",
            "pt_reciprocal_estimate", "pt_resolve_image", "pt_last_error"} <= decl
    L = ptlib.lib()
    for name in decl:
        assert hasattr(L, name), name
    assert set(ptlib.EXPORTED) == decl


def test_struct_sizes_match_header(ptlib):
    # the ctypes mirrors must have the C layouts (checked against hand-computed sizes)
    assert ctypes.sizeof(ptlib.SceneDesc) == 4 + 4 + 8 * 3 + 4 + 4 + 8 + 4 + 4 + 8 + 8 + 4 * 4
    assert ctypes.sizeof(ptlib.IterParams) == 18 * 4
    assert ctypes.sizeof(ptlib.IterStats) == (29 + 25) * 8
    assert ctypes.sizeof(ptlib.SubspaceParams) == 7 * 4
    assert ctypes.sizeof(ptlib.Totals) == 9 * 8
    assert ctypes.sizeof(ptlib.TuneResult) == 10 * 4


def test_invalid_arguments_rejected_without_device(ptlib):
    L = ptlib.lib()
    h = ctypes.c_void_p()
    assert L.pt_scene_upload(None, None, ctypes.byref(h)) == -1
    d = ptlib.SceneDesc()
    d.n_tri = 0
    assert L.pt_scene_upload(ctypes.byref(d), None, ctypes.byref(h)) == -1
    assert b"missing" in L.pt_last_error()
    # bad material index
    tri = np.zeros((1, 9), np.float32)
    tri[0, 3], tri[0, 7] = 1, 1
    mat = np.array([5], np.int32)
    uv = np.zeros((1, 6), np.float32)
    mats = np.zeros((1, 16), np.float32)
    tex = np.ones((1, 1), np.float32)
    cam = np.zeros(10, np.float32)
    d = ptlib.SceneDesc(1, tri.ctypes.data, mat.ctypes.data, uv.ctypes.data, 1, mats.ctypes.data, 1, 1,
                        tex.ctypes.data, cam.ctypes.data, 8, 8, 4, 16)
    assert L.pt_scene_upload(ctypes.byref(d), None, ctypes.byref(h)) == -1
    assert b"material" in L.pt_last_error()
    d.bvh_width = 6
    assert L.pt_scene_upload(ctypes.byref(d), None, ctypes.byref(h)) == -1
    assert b"bvh_width" in L.pt_last_error()
    assert L.pt_render_iteration(None, None, None, None, None, None) == -1
    assert L.pt_reciprocal_estimate(None, None, None, None, None) == -1
    assert L.pt_resolve_image(None, None, 1, None, None) == -1
    assert L.pt_scene_release(None) == 0


def test_bvh_stack_need_fits_the_kernels(ptlib):
    """The host BVH builds (what pt_scene_upload runs) for the config scenes and a 1.4 M-triangle
    variant of the glossy scene: worst-case traversal stacks within the kernels' 48 entries
    (4-wide) and 64 (8-wide), and the need at least the depth less one on these scenes (every
    level of a deep path of inner nodes has siblings there)."""
    from synth import scenes
    cases = [scenes.cornell_glass(8, 8), scenes.projector(8, 8), scenes.glossy_procedural(8, 8),
             scenes.glossy_procedural(8, 8, target_tris=2_000_000)]
    for sc in cases:
        nodes, need, depth = ptlib.bvh_stats(sc["tri"])
        n = sc["tri"].shape[0]
        assert n / 16 <= nodes <= n, (n, nodes)
        assert depth - 1 <= need <= 48, (n, need, depth)
        # the 8-wide tree over the same leaves: fewer nodes and levels, a walk within 64 entries
        nodes8, need8, depth8 = ptlib.bvh_stats(sc["tri"], width=8)
        assert n / 32 <= nodes8 < nodes and depth8 < depth, (n, nodes8, depth8)
        assert depth8 - 1 <= need8 <= 64, (n, need8, depth8)
    # one triangle: a single node with one leaf child needs no stack
    one = np.array([[0, 0, 0, 1, 0, 0, 0, 1, 0]], np.float32)
    assert ptlib.bvh_stats(one) == (1, 0, 1) and ptlib.bvh_stats(one, width=8) == (1, 0, 1)
