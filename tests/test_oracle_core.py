"""Pins of the FP64 oracle's building blocks against facts that do not come from the oracle.

- Philox4x32-10 against the published known-answer vectors.
- The reciprocal estimator I~ (Section 4.2 and Appendix A) against its closed forms: the
  mean 1/int f (Appendix C), the exact variance and expected cost when B >= max f/q (the
  geometric regime of Appendix E), the sign estimator's variance q/(B-Bq)^2 (Appendix E),
  V[I~] <= V[I] (Appendix F), divergence for beta/B >= 2 (Appendix B).
- Booth's roulette (the RR ablation's baseline): identical to I~ on a binary f/q when its
  parameter is at most 1 (both then go on with probability 1 exactly when g = 1, from the same
  draws); on a constant f/q its estimate is a closed-form function of the chain length, whose
  law is known, and the weights are unbiased exactly.
- The binary BVH against brute force.
- BSDFs: sampling densities (chi-square), reciprocity, energy, Snell and Fresnel.
"""
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers(oracle):
    rows = [l.split() for l in open(os.path.join(GOLD, "philox4x32_10_kat.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = oracle.philox(v[0:4], v[4:6])
        assert list(out) == v[6:10]


def _tables():
    rng = np.random.Generator(np.random.Philox(key=11))
    out = [(np.array([0.3, 1.2, 0.5]), np.array([0.5, 0.25, 0.25]))]
    for n in (2, 3, 5, 8):
        f = rng.uniform(0.05, 1.0, n)
        q = rng.uniform(0.2, 1.0, n)
        out.append((f, q / q.sum()))
    return out


def _closed_forms(f, q, B):
    g = 1.0 - f / (q * B)
    Eg, Eg2 = float((q * g).sum()), float((q * g * g).sum())
    m1 = Eg / (1 - Eg)
    m2 = Eg2 * (1 + 2 * m1) / (1 - Eg)
    return dict(var=(m2 - m1 * m1) / B ** 2, var_sign=Eg / (B * (1 - Eg)) ** 2, cost=1.0 / (1 - Eg))


@pytest.mark.parametrize("mult", [0.7, 1.0, 3.0])
def test_recip_mean_all_regimes(oracle, mult):
    """E[I~] = 1 / int f for B in the splitting (0.7 max), optimal (max) and over-bound (3 max) regimes."""
    for i, (f, q) in enumerate(_tables()):
        B = mult * float((f / q).max())
        est, ns, tr = oracle.recip_table(f, q, B, 60000, 0, seed=100 + i)
        assert tr == 0
        se = est.std() / math.sqrt(len(est))
        assert abs(est.mean() - 1.0 / f.sum()) < 4 * se + 1e-12, (i, mult, est.mean(), 1 / f.sum(), se)


def test_recip_geometric_regime_closed_forms(oracle):
    """B >= max f/q: exact variance of I~, variance of the sign estimator, cost B/beta."""
    for i, (f, q) in enumerate(_tables()):
        for mult in (1.0, 1.6):
            B = mult * float((f / q).max())
            cf = _closed_forms(f, q, B)
            est, ns, _ = oracle.recip_table(f, q, B, 200000, 0, seed=200 + i)
            n = len(est)
            var = est.var()
            # standard error of a sample variance: sqrt((m4 - var^2) / n)
            m4 = np.mean((est - est.mean()) ** 4)
            assert abs(var - cf["var"]) < 5 * math.sqrt((m4 - var ** 2) / n), (i, var, cf["var"])
            assert abs(ns.mean() - cf["cost"]) < 5 * ns.std() / math.sqrt(n)
            assert abs(cf["cost"] - B / f.sum()) < 1e-9          # E[samples] = B / beta
            es, nss, _ = oracle.recip_table(f, q, B, 200000, 1, seed=300 + i)
            vs = es.var()
            m4s = np.mean((es - es.mean()) ** 4)
            assert abs(vs - cf["var_sign"]) < 5 * math.sqrt((m4s - vs ** 2) / n), (i, vs, cf["var_sign"])
            assert cf["var"] <= cf["var_sign"] + 1e-15               # Appendix F


def test_recip_closed_forms_worked_example(oracle):
    """f = (0.3, 1.2, 0.5), q = (1/2, 1/4, 1/4), B = 4.8, by hand: g = (7/8, 0, 7/12), E_g = 7/12,
    E_g2 = 0.46788, m1 = 1.4, m2 = 4.26708, so V[I~] = (m2 - m1^2) / B^2 = 0.10013 and
    V[I] = E_g / (B (1 - E_g))^2 = 7/48 = 0.14583 (Appendix E)."""
    f, q = np.array([0.3, 1.2, 0.5]), np.array([0.5, 0.25, 0.25])
    cf = _closed_forms(f, q, 4.8)
    assert abs(cf["var"] - 0.10013) < 1e-4
    assert abs(cf["var_sign"] - 0.14583) < 1e-4


def test_recip_binary_is_geometric(oracle):
    """Binary f/q in {0, c} with B = c: I~ = N/B with N ~ Geometric(success), as in the
    binary special case of Section 4.2."""
    f = np.array([0.0, 0.0, 0.4, 0.0])
    q = np.array([0.25, 0.25, 0.25, 0.25])
    B = 1.6                       # = f/q on the support
    est, ns, _ = oracle.recip_table(f, q, B, 100000, 0, seed=9)
    assert np.allclose(est * B, ns)                  # every estimate is (#samples) / B
    p = 0.25
    assert abs(ns.mean() - 1 / p) < 4 * ns.std() / math.sqrt(len(ns))
    k = np.bincount(ns.astype(int))
    for m in (1, 2, 3):
        assert abs(k[m] / len(ns) - p * (1 - p) ** (m - 1)) < 0.01


def test_recip_diverges_past_convergence_boundary(oracle):
    """beta / B >= 2 leaves the Taylor series' convergence domain (Appendix B): the
    splitting process explodes and hits the sample cap."""
    f, q = np.array([0.3, 1.2, 0.5]), np.array([0.5, 0.25, 0.25])
    _, _, tr_ok = oracle.recip_table(f, q, 0.7 * 4.8, 2000, 0, seed=5, cap=20000)
    _, _, tr_bad = oracle.recip_table(f, q, 0.4 * f.sum(), 200, 0, seed=5, cap=20000)
    assert tr_ok == 0
    assert tr_bad > 50


def test_booth_binary_identity_with_itilde(oracle):
    """f/q in {0, B}: g in {1, 0}. I~ splits into one child exactly when g = 1, and Booth's
    roulette (r <= 1) goes on with probability min(1, 1 / r) = 1 exactly then: the same chains."""
    f, q = np.array([0.0, 0.25, 0.0, 0.25]), np.full(4, 0.25)
    a, na, _ = oracle.recip_table(f, q, 1.0, 4000, 0, seed=7)
    for rhat in (1.0, 0.5):
        b, nb, _ = oracle.recip_table(f, q, 1.0, 4000, 2, seed=7, rhat=rhat)
        assert np.array_equal(na, nb)
        assert np.allclose(a, b, rtol=1e-12, atol=0)


@pytest.mark.parametrize("rhat", [0.25, 0.05])
def test_booth_constant_ratio_exact(oracle, rhat):
    """f/q constant = B (1 - gamma): every g is gamma, the prefix product after j samples is
    gamma^j, and the chain goes on after j samples with probability r_j = min(1, gamma^j / rhat).
    The chain length L then has a closed-form law, and the estimate is a function of L alone:
    est(L) = (1 + sum_{k<=L} gamma^k / prod_{j<k} r_j) / B. Checked: every estimate against
    est(its own sample count), and E[L] against the law. The term of length k is divided by
    prod_{j<k} r_j, the probability of reaching it, so its expectation is gamma^k and the sum is
    1/int f; the sample mean itself is useless here, since the terms grow like gamma^(-k^2/2)
    against their probability and the variance is infinite. A small sample cap makes a roulette
    that never stops (one on |g| instead of the product) fail fast."""
    gamma = 0.5
    f, q = np.array([0.25, 0.25]), np.array([0.5, 0.5])
    B = float((f / q).max()) / (1.0 - gamma)
    r = [min(1.0, gamma ** j / rhat) for j in range(1, 80)]
    est_of, p_of = [], []
    reach, w, acc = 1.0, 1.0, 1.0
    for L in range(1, 79):
        acc += gamma ** L / w                 # the term of length L
        est_of.append(acc / B)
        p_of.append(reach * (1.0 - r[L - 1]))   # reached L, stopped after it
        reach *= r[L - 1]
        w *= r[L - 1]
        if reach < 1e-30:                     # longer chains have no weight in the law
            p_of[-1] += reach
            break
    est_of, p_of = np.array(est_of), np.array(p_of)
    assert abs(p_of.sum() - 1.0) < 1e-12
    est, ns, tr = oracle.recip_table(f, q, B, 200000, 2, seed=13, cap=1000, rhat=rhat)
    assert tr == 0
    L = ns.astype(np.int64)
    assert np.allclose(est, est_of[L - 1], rtol=1e-12, atol=0)
    EL = (p_of * np.arange(1, len(p_of) + 1)).sum()
    assert abs(ns.mean() - EL) < 5 * ns.std() / math.sqrt(len(ns)), (ns.mean(), EL)


def test_booth_large_rhat_has_heavy_tail(oracle):
    """With rhat = 100 a chain goes on with probability at most 1 / 100 and carries the inverse
    weight: a few estimates exceed the mean by orders of magnitude (the ablation's point)."""
    f, q = np.array([0.2, 0.5, 0.3]), np.array([0.2, 0.25, 0.55])
    B = float((f / q).max())
    est, ns, _ = oracle.recip_table(f, q, B, 200000, 2, seed=12, rhat=100.0)
    assert ns.mean() < 1.02
    assert est.max() > 50.0 / f.sum()


# ---------------------------------------------------------------------------- BVH
def _random_rays(sc, n, seed):
    rng = np.random.Generator(np.random.Philox(key=seed))
    tri = sc["tri"].reshape(-1, 3, 3).astype(np.float64)
    lo, hi = tri.min((0, 1)), tri.max((0, 1))
    o = rng.uniform(lo, hi, (n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.concatenate([o, d, np.full((n, 1), 1e-9), np.full((n, 1), 1e30)], axis=1)


@pytest.mark.parametrize("which", ["cornell", "projector"])
def test_bvh_matches_brute_force(oracle, which):
    from synth import scenes
    sc = scenes.cornell_glass(8, 8) if which == "cornell" else scenes.projector(8, 8)
    S = oracle.Scene(sc)
    rays = _random_rays(sc, 3000, 4)
    t1, p1 = S.trace(rays, brute=False)
    t2, p2 = S.trace(rays, brute=True)
    assert (p1 == p2).all()
    assert np.allclose(t1, t2, rtol=1e-12, atol=0)
    assert (p1 >= 0).mean() > 0.5


# ---------------------------------------------------------------------------- BSDFs
def _lambert():
    from synth import scenes
    return scenes.material(scenes.MAT_LAMBERT, (0.8, 0.5, 0.2))


def _ggx(r):
    from synth import scenes
    return scenes.material(scenes.MAT_CONDUCTOR, (0.9, 0.6, 0.3), roughness=r)


def _glass():
    from synth import scenes
    return scenes.material(scenes.MAT_DIELECTRIC, ior=1.5)


N_UP = np.array([0.0, 0.0, 1.0])


def _dir(theta, phi):
    return np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)])


@pytest.mark.parametrize("mat", ["lambert", "ggx_0.3", "ggx_0.6"])
def test_bsdf_sampling_chi_square(oracle, mat):
    """Sampled directions follow the stated pdf: chi-square over (cos theta, phi) bins,
    expected counts from a fine numerical integral of the pdf."""
    rec = _lambert() if mat == "lambert" else _ggx(float(mat.split("_")[1]))
    wo = _dir(0.6, 0.3)
    rng = np.random.Generator(np.random.Philox(key=21))
    nb_t, nb_p, n = 10, 12, 40000
    counts = np.zeros((nb_t, nb_p))
    fails = 0
    for _ in range(n):
        s = oracle.bsdf_sample(rec, N_UP, wo, rng.uniform(size=3))
        if not s[7]:
            fails += 1
            continue
        wi = s[:3]
        ct = wi[2]
        it = min(int(ct * nb_t), nb_t - 1)
        ph = (math.atan2(wi[1], wi[0]) + 2 * math.pi) % (2 * math.pi)
        ip = min(int(ph / (2 * math.pi) * nb_p), nb_p - 1)
        counts[it, ip] += 1
    # expected: integrate pdf over each bin with a midpoint rule in (cos theta, phi)
    sub = 12
    exp = np.zeros((nb_t, nb_p))
    for it in range(nb_t):
        for ip in range(nb_p):
            acc = 0.0
            for a in range(sub):
                for b in range(sub):
                    ct = (it + (a + 0.5) / sub) / nb_t
                    ph = (ip + (b + 0.5) / sub) / nb_p * 2 * math.pi
                    wi = _dir(math.acos(ct), ph)
                    acc += oracle.bsdf_eval(rec, N_UP, wo, wi)[3]
            exp[it, ip] = acc / (sub * sub) * (1.0 / nb_t) * (2 * math.pi / nb_p) * n
    mask = exp > 5
    chi2 = ((counts[mask] - exp[mask]) ** 2 / exp[mask]).sum()
    dof = mask.sum() - 1
    # ~ 5 sigma above the mean of a chi-square with dof degrees of freedom
    assert chi2 < dof + 5 * math.sqrt(2 * dof), (chi2, dof)
    # the mass outside the front hemisphere shows up as failed samples only
    assert abs((n - fails) - exp.sum()) < 5 * math.sqrt(n) + 0.02 * n


@pytest.mark.parametrize("rough", [0.05, 0.3])
def test_ggx_reciprocity_and_energy(oracle, rough):
    rec = _ggx(rough)
    rng = np.random.Generator(np.random.Philox(key=22))
    for _ in range(50):
        a = _dir(rng.uniform(0, 1.4), rng.uniform(0, 6.28))
        b = _dir(rng.uniform(0, 1.4), rng.uniform(0, 6.28))
        fa = oracle.bsdf_eval(rec, N_UP, a, b)
        fb = oracle.bsdf_eval(rec, N_UP, b, a)
        assert np.allclose(fa[:3], fb[:3], rtol=1e-10)
        assert abs(fa[3] - fb[3]) <= 1e-10 * max(fa[3], 1)   # the reflection pdf is symmetric too
    # single-scattering albedo <= 1 (white furnace of one BSDF)
    wo = _dir(0.7, 0.0)
    w = np.zeros(3)
    n = 20000
    for _ in range(n):
        s = oracle.bsdf_sample(rec, N_UP, wo, rng.uniform(size=3))
        if s[7]:
            w += s[3:6]
    assert (w / n <= 1.0 + 0.02).all()


def test_lambert_albedo_and_sides(oracle):
    rec = _lambert()
    rng = np.random.Generator(np.random.Philox(key=23))
    for wo in (_dir(0.4, 1.0), -_dir(0.4, 1.0)):
        for _ in range(200):
            s = oracle.bsdf_sample(rec, N_UP, wo, rng.uniform(size=3))
            assert s[7] and np.sign(s[2]) == np.sign(wo[2])
            assert np.allclose(s[3:6], [0.8, 0.5, 0.2])
            assert abs(s[6] - abs(s[2]) / math.pi) < 1e-12


def test_dielectric_snell_fresnel_and_modes(oracle):
    rec = _glass()
    eta = 1.5
    for theta in (0.0, 0.3, 0.9, 1.3):
        wo = _dir(theta, 0.4)
        refl = oracle.bsdf_sample(rec, N_UP, wo, [0.0, 0.5, 0.5])       # u < F: reflection
        tran = oracle.bsdf_sample(rec, N_UP, wo, [0.999999, 0.5, 0.5])  # transmission
        F = refl[6]
        assert abs(F + tran[6] - 1.0) < 1e-12
        assert np.allclose(refl[:3], [-wo[0], -wo[1], wo[2]], atol=1e-12)
        sin_i = math.sin(theta)
        wt = tran[:3]
        assert abs(math.hypot(wt[0], wt[1]) - sin_i / eta) < 1e-12 and wt[2] < 0
        # radiance carried from inside to outside is divided by eta^2; importance is not
        assert abs(tran[3] - 1 / eta ** 2) < 1e-12
        light = oracle.bsdf_sample(rec, N_UP, wo, [0.999999, 0.5, 0.5], mode=1)
        assert abs(light[3] - 1.0) < 1e-12
        # normal incidence: F = ((eta-1)/(eta+1))^2
        if theta == 0.0:
            assert abs(F - ((eta - 1) / (eta + 1)) ** 2) < 1e-12
    # total internal reflection from inside beyond the critical angle
    wo_in = -_dir(0.9, 0.0)     # inside the glass, 0.9 rad > asin(1/1.5)
    s = oracle.bsdf_sample(rec, N_UP, wo_in, [0.999999, 0.5, 0.5])
    assert s[6] == 1.0 and s[2] < 0
