"""Pins of the photon-plane oracle (oracle/planes.c; Section 6.7's photon planes with the CMIS
weight of the continuous chord-angle technique space).

PL1  chord length of the light rectangle through a point: brute force along the line.
PL2  J(y, m) = int_0^pi len(alpha; y) |u_alpha . m| dalpha: a fine midpoint sum.
PL3  the single-scattering reference: with no extinction its light integral is the solid angle the
     rectangle subtends (Van Oosterom and Strackee's closed form for two triangles), and the
     quadrature is converged (refined nodes agree).
PL4  the photon-plane estimator with the exact reciprocal (the density p(alpha, xbar) and the
     balance-heuristic weight) against the reference, per pixel within 4 standard errors.
"""
import math

import numpy as np
import pytest

from synth import scenes


def test_pl1_chord_length(oracle):
    rng = np.random.default_rng(11)
    eu, ev = 0.5, 0.3
    for _ in range(200):
        a, b = rng.uniform(-eu, eu), rng.uniform(-ev, ev)
        al = rng.uniform(0, math.pi)
        s = np.linspace(-2.0, 2.0, 400001)
        x, y = a + s * math.cos(al), b + s * math.sin(al)
        inside = (np.abs(x) <= eu) & (np.abs(y) <= ev)
        brute = inside.sum() * (s[1] - s[0])
        assert abs(oracle.planes_chord(eu, ev, a, b, al) - brute) < 2e-5
    # axis-parallel chords through any point: the side lengths
    assert oracle.planes_chord(eu, ev, 0.1, 0.2, 0.0) == pytest.approx(2 * eu)
    assert oracle.planes_chord(eu, ev, 0.1, 0.2, math.pi / 2) == pytest.approx(2 * ev)


def test_pl2_J_against_a_fine_sum(oracle):
    rng = np.random.default_rng(12)
    eu, ev = 0.5, 0.3
    n = 400000
    al = (np.arange(n) + 0.5) * math.pi / n
    ca, sa = np.cos(al), np.sin(al)
    for _ in range(12):
        a, b = rng.uniform(-eu, eu), rng.uniform(-ev, ev)
        mu, mv = rng.normal(size=2)
        with np.errstate(divide="ignore"):
            t = [(-eu - a) / ca, (eu - a) / ca, (-ev - b) / sa, (ev - b) / sa]
        lo = np.maximum(np.minimum(t[0], t[1]), np.minimum(t[2], t[3]))
        hi = np.minimum(np.maximum(t[0], t[1]), np.maximum(t[2], t[3]))
        brute = (np.maximum(hi - lo, 0) * np.abs(mu * ca + mv * sa)).sum() * math.pi / n
        assert oracle.planes_J(eu, ev, a, b, mu, mv) == pytest.approx(brute, rel=2e-5)
    # m along U only: J = int len |cos| dalpha, which for the centre of a square of side 2e is
    # 2 int_0^{pi/2} 2e cos / max(cos, sin) dalpha = 4 e (pi/4 + ln(2) / 2)
    e = 0.4
    assert oracle.planes_J(e, e, 0.0, 0.0, 1.0, 0.0) == pytest.approx(4 * e * (math.pi / 4 + math.log(2) / 2),
                                                                      rel=1e-10)


def _solid_angle_rect(x, corners):
    """Solid angle of a planar quadrilateral seen from x (two triangles, Van Oosterom-Strackee)."""
    tot = 0.0
    for tri in ((0, 1, 2), (0, 2, 3)):
        a, b, c = (corners[k] - x for k in tri)
        la, lb, lc = (np.linalg.norm(v) for v in (a, b, c))
        num = abs(np.dot(a, np.cross(b, c)))
        den = la * lb * lc + np.dot(a, b) * lc + np.dot(a, c) * lb + np.dot(b, c) * la
        tot += 2.0 * math.atan2(num, den)
    return tot


def test_pl3_reference_solid_angle_and_convergence(oracle):
    sc = scenes.planes_scene(4, 3, sigma_s=0.5, sigma_t=0.0)
    ref = oracle.planes_reference(sc, nt=16, ny=8)
    c, U, V = sc["light_c"], sc["light_u"], sc["light_v"]
    eu, ev = sc["light_eu"], sc["light_ev"]
    corners = [c - eu * U - ev * V, c + eu * U - ev * V, c + eu * U + ev * V, c - eu * U + ev * V]
    cam = sc["camera"]
    o = cam[:3]
    f = cam[3:6] - o
    f /= np.linalg.norm(f)
    r = np.cross(f, cam[6:9])
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(0.5 * math.radians(cam[9]))
    W, H = sc["width"], sc["height"]
    gx, gw = np.polynomial.legendre.leggauss(48)
    for py in range(H):
        for px in range(W):
            x = (2.0 * (px + 0.5) / W - 1.0) * th * W / H
            y = (1.0 - 2.0 * (py + 0.5) / H) * th
            d = f + x * r + y * u
            d /= np.linalg.norm(d)
            L = 0.0
            for k in range(8):
                t0, t1 = sc["t_max"] * k / 8, sc["t_max"] * (k + 1) / 8
                for xi, wi in zip(gx, gw):
                    t = 0.5 * (t0 + t1) + 0.5 * (t1 - t0) * xi
                    L += 0.5 * (t1 - t0) * wi * _solid_angle_rect(o + t * d, corners)
            L *= sc["sigma_s"] / (4 * math.pi) * sc["le"][0]
            assert ref[py, px, 0] == pytest.approx(L, rel=1e-6)
    sc = scenes.planes_scene(4, 3)
    a = oracle.planes_reference(sc, nt=16, ny=8)
    b = oracle.planes_reference(sc, nt=24, ny=12)
    assert np.abs(a - b).max() <= 1e-9 * a.max()


def test_pl4_plane_estimator_matches_reference(oracle):
    sc = scenes.planes_scene(6, 6)
    ref = oracle.planes_reference(sc)
    N = 32
    s, s2 = oracle.planes_render(sc, 1024, N, seed=7)
    m = s / N
    v = (s2 / N - m * m) / N
    z = (m - ref) / np.sqrt(v + 1e-300)
    assert np.abs(z[..., 0]).max() < 4, np.abs(z).max()
    assert np.all(m > 0)


def test_planes_scene_keeps_eye_rays_off_the_light_plane():
    """The workload's stated geometry: every eye ray leaves the light's plane at 15 to 40 degrees
    (none grazes it, where a plane's estimate would have unbounded variance) and stays at least
    0.25 from the light up to t_max."""
    sc = scenes.planes_scene(64, 64)
    c, U, V = sc["light_c"], sc["light_u"], sc["light_v"]
    N = np.cross(U, V)
    cam = sc["camera"]
    o = cam[:3]
    f = cam[3:6] - o
    f /= np.linalg.norm(f)
    r = np.cross(f, cam[6:9])
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(0.5 * math.radians(cam[9]))
    W, H = sc["width"], sc["height"]
    ang = []
    dmin = np.inf
    ts = np.linspace(0.0, sc["t_max"], 200)
    for py in (0, H // 2, H - 1):
        for px in (0, W // 2, W - 1):
            x = (2.0 * (px + 0.5) / W - 1.0) * th * W / H
            y = (1.0 - 2.0 * (py + 0.5) / H) * th
            d = f + x * r + y * u
            d /= np.linalg.norm(d)
            ang.append(math.degrees(math.asin(abs(np.dot(d, N)))))
            for t in ts:
                p = o + t * d - c
                a, b, h = np.dot(p, U), np.dot(p, V), np.dot(p, N)
                da, db = max(abs(a) - sc["light_eu"], 0.0), max(abs(b) - sc["light_ev"], 0.0)
                dmin = min(dmin, math.sqrt(da * da + db * db + h * h))
    assert 14.0 < min(ang) and max(ang) < 41.0, (min(ang), max(ang))
    assert dmin > 0.25, dmin
