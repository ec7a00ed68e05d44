"""CPU checks of the C ABI: the library loads, exports every symbol include/pt.h declares, and
rejects invalid arguments before touching a device."""
import ctypes
import itertools
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
    assert ctypes.sizeof(ptlib.PlanesDesc) == (3 * 3 + 2 + 3 + 10 + 3) * 4 + 3 * 4
    assert ctypes.sizeof(ptlib.PlanesStats) == 4 * 8


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
    # photon planes: the description is validated before any device call
    from synth import scenes
    sc = scenes.planes_scene(8, 8)
    f = lambda v, n: (ctypes.c_float * n)(*[float(x) for x in v])  # noqa: E731
    def desc(**kw):
        v = dict(sc, max_planes=64)
        v.update(kw)
        return ptlib.PlanesDesc(f(v["light_c"], 3), f(v["light_u"], 3), f(v["light_v"], 3), v["light_eu"],
                                v["light_ev"], f(v["le"], 3), f(v["camera"], 10), v["sigma_s"], v["sigma_t"],
                                v["t_max"], v["width"], v["height"], v["max_planes"])
    hp = ctypes.c_void_p()
    for bad, msg in ((dict(light_v=[1.0, 0.0, 0.0]), b"orthonormal"), (dict(light_eu=0.0), b"half extents"),
                     (dict(sigma_t=-1.0), b"sigma"), (dict(width=0), b"image size"),
                     (dict(max_planes=0), b"max_planes"), (dict(max_planes=ptlib.PLANES_MAX + 1), b"max_planes"),
                     (dict(camera=[0, 0, 0, 0, 0, 0, 0, 1, 0, 30]), b"camera")):
        assert L.pt_planes_create(ctypes.byref(desc(**bad)), None, ctypes.byref(hp)) == -1, bad
        assert msg in L.pt_last_error(), (bad, L.pt_last_error())
    assert L.pt_planes_render(None, 1, 0, 0, None, None, None, None) == -1
    assert L.pt_planes_release(None) == 0


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


def test_proxy_class_matches_the_oracle_on_every_short_path(ptlib, oracle):
    """The proxy-class test the kernels apply (eye side, then the joined light tail from the light
    sub-path signature) against the oracle's on every path of 1..7 vertices over {specular,
    Lambertian, other diffuse}, every split into eye vertices and a joined light tail, u_max 1, 2,
    4, with and without class C."""
    n_paths = n_proxy = 0
    for n in range(1, 8):
        for mats in itertools.product("SLR", repeat=n):
            is_s = [m == "S" for m in mats]
            is_l = [m == "L" for m in mats]
            eye = np.array([(1 if s else 0) | (2 if l else 0) for s, l in zip(is_s, is_l)], np.uint8)
            for u_max in (1, 2, 4):
                for gcv in (0, 1):
                    want = oracle.proxy_class(is_s, is_l, u_max, gcv)
                    n_paths += 1
                    n_proxy += want
                    for ne in range(n + 1):
                        # z_1 .. z_ne on the eye side, the rest joined as y_j .. y_1 (y_k = z_{n+1-k})
                        j = n - ne
                        sig = 0
                        for k in range(1, j + 1):
                            z = n - k          # 0-based eye index of y_k
                            sig |= (1 << k) if is_s[z] else 0
                            sig |= (1 << (16 + k)) if is_l[z] else 0
                        got = ptlib.proxy_class(eye[:ne], sig, j, u_max, gcv)
                        assert got == want, ("".join(mats), ne, u_max, gcv, got, want)
    assert 0 < n_proxy < n_paths
    with pytest.raises(ptlib.PTError):
        ptlib.proxy_class([0], 0, 0, u_max=5)
