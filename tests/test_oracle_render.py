"""Pins of the oracle's in-scene estimators against closed forms and against each other.

P3  class A, u = 1: the incomplete sub-path density P at a point below a rectangular
    emitter is (1/A) x the form factor integral; checked against Gauss-Legendre
    quadrature, and the reciprocal estimate's mean against 1/P.
P4  class A, u = 2 through a perfect mirror: P equals the u = 1 density of the emitter
    mirrored about the mirror plane (image method); f/q is binary (Section 4.2's binary
    case), and the reciprocal estimate's mean is 1/P.
P5  diffuse furnace: a closed box of emitting Lambertian walls reads Le (1 - a^K) / (1 - a)
    with at most K segments (the white-furnace closed form), for O1 and O2.
P6  glass furnace: an emitting spherical enclosure (no corners, so the class B f/q stays
    bounded) around a lossless glass sphere; every pixel still reads the closed form (large
    K), for O1 and O2 (O2 routes the L S^u and L D S^u paths through the proxy).
P7  proxy-class paths only: O2's proxy strategy alone matches O1 restricted to the same
    signature class, per pixel within 4 combined standard errors (mirror room, u <= 2).
P8  the proxy class with a general control vertex (Section 5.2): the oracle's state machine
    agrees with the classes' definitions on every eye path of up to 8 vertices; O1's class
    filter with it still partitions the image exactly, and its proxy class is the one without
    it plus a non-empty set of L ... h_c D S^u paths.
P9  O2's proxy strategy with class C candidates alone on its class matches O1 restricted to the
    class with a general control vertex (spherical glass furnace, u <= 1), per pixel and in total.
"""
import itertools
import re
import math

import numpy as np
import pytest

from synth import scenes


def _gauss_rect(fun, x0, x1, z0, z1, n=64):
    xs, ws = np.polynomial.legendre.leggauss(n)
    X = 0.5 * (x1 - x0) * xs + 0.5 * (x1 + x0)
    Z = 0.5 * (z1 - z0) * xs + 0.5 * (z1 + z0)
    W = np.outer(ws, ws) * 0.25 * (x1 - x0) * (z1 - z0)
    XX, ZZ = np.meshgrid(X, Z, indexing="ij")
    return float((fun(XX, ZZ) * W).sum())


def _prim_containing(sc, p):
    tri = sc["tri"].reshape(-1, 3, 3).astype(np.float64)
    for i, t in enumerate(tri):
        e1, e2, w = t[1] - t[0], t[2] - t[0], p - t[0]
        n = np.cross(e1, e2)
        if abs(np.dot(n, w)) > 1e-9 * np.linalg.norm(n):
            continue
        # barycentrics
        d00, d01, d11 = np.dot(e1, e1), np.dot(e1, e2), np.dot(e2, e2)
        d20, d21 = np.dot(w, e1), np.dot(w, e2)
        den = d00 * d11 - d01 * d01
        b1 = (d11 * d20 - d01 * d21) / den
        b2 = (d00 * d21 - d01 * d20) / den
        if b1 >= 0 and b2 >= 0 and b1 + b2 <= 1:
            return i
    raise AssertionError("point not on any triangle")


def _density_parallel_rect(v, h, A):
    """(1/A) * integral over the emitter rectangle x in [-.5,.5], z in [-.25,.25] at height
    h above v of cos0 cosv / (pi d^2) = h^2 / (pi d^4)."""
    def fun(x, z):
        d2 = (x - v[0]) ** 2 + h * h + (z - v[2]) ** 2
        return h * h / (math.pi * d2 * d2)
    return _gauss_rect(fun, -0.5, 0.5, -0.25, 0.25) / A


@pytest.mark.parametrize("v", [(0.3, 0.0, 0.1), (1.4, 0.0, -0.7)])
def test_p3_form_factor_density_and_reciprocal(oracle, v):
    sc = scenes.formfactor_plane(mirror=False)
    S = oracle.Scene(sc)
    A = S.emitter_area
    assert abs(A - 0.5) < 1e-6
    v = np.array(v)
    prim = _prim_containing(sc, v)
    P = _density_parallel_rect(v, 1.0, A)
    # plain Monte Carlo mean of f/q estimates P; f/q <= 2/A on a one-sided conductor
    B = 2.0 / A
    pe, re, rn, tr = S.recip_candidate(0, 1, v, prim, B=B, n_est=100000, per=1, seed=7)
    assert tr == 0
    assert pe.max() <= B * (1 + 1e-9)
    assert abs(pe.mean() - P) < 4 * pe.std() / math.sqrt(len(pe)), (pe.mean(), P)
    assert abs(re.mean() - 1.0 / P) < 4 * re.std() / math.sqrt(len(re)), (re.mean(), 1 / P)
    # expected cost B / beta (geometric regime, Appendix E)
    assert abs(rn.mean() - B / P) < 4 * rn.std() / math.sqrt(len(rn))


def test_p4_mirror_image_method_binary(oracle):
    sc = scenes.formfactor_plane(mirror=True)
    S = oracle.Scene(sc)
    A = S.emitter_area
    v = np.array([2.0, 0.0, 0.1])
    prim = _prim_containing(sc, v)
    # emitter at y = 0.5 mirrored about y = 1.5 -> image at height 2.5 above the floor point
    P = _density_parallel_rect(v, 2.5, A)
    pe, re, rn, tr = S.recip_candidate(0, 2, v, prim, B=1.0 / A, n_est=60000, per=1, seed=8)
    assert tr == 0
    vals = np.unique(np.round(pe * A, 9))
    assert set(vals.tolist()) <= {0.0, 1.0}, vals          # f/q in {0, 1/A}
    assert abs(pe.mean() - P) < 4 * pe.std() / math.sqrt(len(pe)), (pe.mean(), P)
    assert abs(re.mean() - 1.0 / P) < 4 * re.std() / math.sqrt(len(re)), (re.mean(), 1 / P)
    assert np.allclose(re, rn * A)                          # I~ = N / B with B = 1/A


def _zscore_ok(mean, var_of_mean, expect, frac=0.999):
    z = (mean - expect) / np.sqrt(var_of_mean + 1e-300)
    return (np.abs(z) < 4).mean() >= frac, float(np.abs(z).max())


@pytest.mark.parametrize("method", [0, 1])
def test_p5_diffuse_furnace(oracle, method):
    a, le, K = 0.5, 1.0, 6
    sc = scenes.furnace(albedo=a, le=le, width=8, height=8)
    S = oracle.Scene(sc)
    N = 512
    s, s2, st = S.render(method=method, n_iter=N, max_depth=K, n_light=256, cand_cap=64, seed=3)
    m = s / N
    vm = (s2 / N - m * m) / N
    expect = le * (1 - a ** K) / (1 - a)
    ok, zmax = _zscore_ok(m, vm, expect, frac=1.0)
    assert ok, zmax
    assert abs(m.mean() - expect) < 4 * math.sqrt(vm.mean() / m.size)


@pytest.mark.parametrize("method", [0, 1])
def test_p6_glass_furnace(oracle, method):
    a, le, K = 0.5, 1.0, 120
    sc = scenes.furnace(albedo=a, le=le, glass_sphere=True, width=8, height=8, sphere_subdiv=2, enclosure="sphere")
    S = oracle.Scene(sc)
    N = 384
    s, s2, st = S.render(method=method, n_iter=N, max_depth=K, n_light=256, cand_cap=64, seed=4)
    m = s / N
    vm = (s2 / N - m * m) / N
    expect = le * (1 - a ** K) / (1 - a)
    ok, zmax = _zscore_ok(m, vm, expect, frac=1.0)
    assert ok, zmax
    if method == 1:
        assert st["n_kept"] > 0 and st["n_proxy_valid"] > 0 and st["n_recip_truncated"] == 0


def test_p7_proxy_class_matches_path_tracing(oracle):
    """Mirror room: light -> mirror/glass -> floor (class A) and light -> wall -> mirror ->
    floor (class B) paths, u <= 2; O2's proxy strategy alone vs O1 restricted to the class."""
    sc = scenes.mirror_room(16, 16)
    S = oracle.Scene(sc)
    N = 256
    s1, q1, _ = S.render(method=0, n_iter=N, max_depth=8, u_max=2, class_filter=1, seed=5)
    s2, q2, st = S.render(method=1, n_iter=N, max_depth=8, n_light=512, cand_cap=128, u_max=2,
                          class_filter=1, seed=6)
    m1, m2 = s1 / N, s2 / N
    v1, v2 = (q1 / N - m1 ** 2) / N, (q2 / N - m2 ** 2) / N
    z = (m1 - m2) / np.sqrt(v1 + v2 + 1e-300)
    assert (np.abs(z) < 4).mean() >= 0.99, np.abs(z).max()
    # whole-image total of the class agrees within 4 standard errors
    assert abs(m1.sum() - m2.sum()) < 4 * math.sqrt(v1.sum() + v2.sum())
    assert st["n_recip_truncated"] == 0 and st["n_proxy_valid"] > 0
    assert m1.sum() > 0.05 * (m1.sum() + 1e-9)


def _proxy_class_def(mats, u_max, gcv):
    """The classes written out on the light-order string (eye path z_1 .. z_n closed at the emitter
    y_0, so y_k = z_{n+1-k}): z_d is the first non-specular eye vertex and y_1 .. y_i the vertices
    between the emitter and z_d. Class A: y_1 .. y_i specular, 1 <= i <= u_max. Class B: y_1 not
    specular, then u = i - 1 specular vertices, 1 <= u <= u_max. Class C: some y_j (j >= 1)
    Lambertian, y_{j+1} not specular, then u = i - j - 1 specular vertices, 1 <= u <= u_max, and
    i <= 5 (the light vertices the strategy stores). Letters: S specular, L Lambertian, R other."""
    if all(m == "S" for m in mats):
        return 0
    zd = next(k for k, m in enumerate(mats) if m != "S")     # 0-based eye index of z_d
    light = "".join(reversed(mats[zd + 1:]))                  # y_1 .. y_i
    i = len(light)
    if re.fullmatch(r"S{1,%d}" % u_max, light):
        return 1
    if re.fullmatch(r"[LR]S{1,%d}" % u_max, light):
        return 1
    if gcv and i <= 5 and re.fullmatch(r"[SLR]*L[LR]S{1,%d}" % u_max, light):
        return 1
    return 0


def test_p8_general_cv_class_definition(oracle):
    """Every eye path of 1..8 vertices over {specular, Lambertian, other diffuse}: the oracle's
    proxy-class state machine equals the written-out definition, with and without class C."""
    n_c = 0
    for n in range(1, 9):
        for mats in itertools.product("SLR", repeat=n):
            is_s = [m == "S" for m in mats]
            is_l = [m == "L" for m in mats]
            for u_max in (1, 2, 4):
                for gcv in (0, 1):
                    want = _proxy_class_def(mats, u_max, gcv)
                    got = oracle.proxy_class(is_s, is_l, u_max, gcv)
                    assert got == want, ("".join(mats), u_max, gcv, got, want)
                    n_c += gcv and want and not _proxy_class_def(mats, u_max, 0)
    assert n_c > 0


def test_p8_general_cv_partition(oracle):
    """Mirror room, the same random streams: with class C, O1's proxy class and the other paths
    still add up to the unfiltered image; the proxy class grows by the class C paths only (never
    loses a path), and they carry a non-zero share."""
    sc = scenes.mirror_room(8, 8)
    S = oracle.Scene(sc)
    kw = dict(method=0, n_iter=24, max_depth=8, u_max=2, seed=3)
    a, _, _ = S.render(class_filter=0, **kw)
    p0, _, _ = S.render(class_filter=1, **kw)
    o0, _, _ = S.render(class_filter=2, **kw)
    p1, _, _ = S.render(class_filter=1, general_cv=1, **kw)
    o1, _, _ = S.render(class_filter=2, general_cv=1, **kw)
    scale = a.max()
    assert np.abs(p1 + o1 - a).max() <= 1e-12 * scale
    assert np.abs(p0 + o0 - a).max() <= 1e-12 * scale
    extra = p1 - p0
    assert extra.min() >= -1e-12 * scale
    assert np.abs(extra - (o0 - o1)).max() <= 1e-12 * scale
    assert extra.sum() > 1e-3 * p0.sum()
    with pytest.raises(ValueError):
        S.render(method=2, n_iter=1, general_cv=1)


def test_p9_o2_general_cv_matches_o1(oracle):
    """Spherical glass furnace (every diffuse vertex on the enclosure, so the connection h_c <-> y_{j+1}
    has a bounded geometry term), 8 segments, u <= 1: O2 with class C candidates, the proxy alone
    on its class, against O1 restricted to the same class; class C is about 20 % of it. The proxy
    alone carries the reciprocal estimates' right tail unweighted, so its per-pixel means are
    skewed low with standard errors that read low: the image total is the test of the
    expectation, and per pixel the upper side."""
    sc = scenes.furnace(albedo=0.5, le=1.0, glass_sphere=True, width=8, height=8, enclosure="sphere")
    S = oracle.Scene(sc)
    N1, N2 = 8192, 1024
    kw = dict(max_depth=8, u_max=1, class_filter=1)
    s1, q1, _ = S.render(method=0, n_iter=N1, general_cv=1, seed=11, **kw)
    s0, _, _ = S.render(method=0, n_iter=N1, seed=11, **kw)
    s2, q2, st = S.render(method=1, n_iter=N2, n_light=256, cand_cap=64, general_cv=1, seed=12, **kw)
    m1, m2 = s1 / N1, s2 / N2
    v1 = np.maximum(q1 / N1 - m1 ** 2, 0) / N1
    v2 = np.maximum(q2 / N2 - m2 ** 2, 0) / N2
    z = (m2 - m1) / np.sqrt(v1 + v2 + 1e-300)
    se = math.sqrt(v1.sum() + v2.sum())
    assert (z < 4).mean() >= 0.99, z.max()
    assert abs(m2.sum() - m1.sum()) < 4 * se
    assert m2.sum() - s0.sum() / N1 > 5 * se            # the class C paths are there
    assert st["n_recip_truncated"] == 0 and st["n_proxy_valid"] > 0
