"""Host logic of the ablation script: the variant sets and the firefly-proof image mean."""
import os
import sys
import types

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), ".."))
import bench_ablation as ba  # noqa: E402


def _flags():
    names = ["NEE", "PROXY", "ONLY_PROXY_CLASS", "ONLY_OTHER", "GAMMA", "TILES", "TIMING", "COUNT", "MIS", "MLP",
             "SPC", "LT", "BOOTH", "MLP_DIR"]
    return types.SimpleNamespace(**{f"PT_FLAG_{n}": 1 << i for i, n in enumerate(names)})


def test_rr_variants_differ_only_in_the_roulette():
    pt = _flags()
    for study in ("rr", "rr_proxy"):
        v = ba.variants(study, pt)
        assert v[0][0] == "rrs" and not v[0][1] & pt.PT_FLAG_BOOTH
        rs = [r for _, _, r in v[1:]]
        assert rs == sorted(rs) and rs[0] < 1 < rs[-1]
        for name, flags, r in v[1:]:
            assert flags == v[0][1] | pt.PT_FLAG_BOOTH and name == f"booth_r={r:g}"
    assert ba.variants("rr", pt)[0][1] & pt.PT_FLAG_MIS
    proxy = ba.variants("rr_proxy", pt)[0][1]
    assert proxy & pt.PT_FLAG_ONLY_PROXY_CLASS and not proxy & pt.PT_FLAG_MIS


def test_gamma_variants_differ_only_in_gamma():
    pt = _flags()
    (n0, f0, _), (n1, f1, _) = ba.variants("gamma", pt)
    assert (n0, n1) == ("gamma", "uniform") and f0 == f1 | pt.PT_FLAG_GAMMA and not f1 & pt.PT_FLAG_GAMMA
    assert f0 & pt.PT_FLAG_ONLY_PROXY_CLASS


def test_trimmed_mean_ignores_a_single_firefly():
    rng = np.random.default_rng(5)
    m = rng.uniform(0.0, 1.0, (64, 64, 3))
    base = ba.trimmed_mean(m)
    m2 = m.copy()
    m2[3, 7, 1] = 1e6
    assert abs(ba.trimmed_mean(m2) - base) < 1e-3 * base
    assert m2.mean() > 50 * m.mean()
    assert abs(base - np.sort(m.ravel())[: int(0.999 * m.size)].mean()) < 1e-15
    assert abs(base - 0.5) < 0.02


def test_learned_variants_add_only_the_network():
    pt = _flags()
    v = ba.variants("learned", pt)
    assert [n for n, _, _ in v] == ["plain", "learned", "learned_selection"]
    plain = v[0][1]
    assert plain & pt.PT_FLAG_MIS and not plain & (pt.PT_FLAG_MLP | pt.PT_FLAG_MLP_DIR)
    assert v[1][1] == plain | pt.PT_FLAG_MLP | pt.PT_FLAG_MLP_DIR
    assert v[2][1] == plain | pt.PT_FLAG_MLP
