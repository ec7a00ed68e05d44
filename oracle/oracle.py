"""ctypes wrapper of the FP64 CPU oracle (oracle.c, and planes.c for the photon-plane workload).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the CPU
baseline leg of bench.py. The HIP library and its binding never import it.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")
SRC_PLANES = os.path.join(HERE, "planes.c")


def build(force=True):
    """Compile oracle.c and planes.c with gcc (O2, plain C11, pthreads)."""
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-pthread",
                           "-o", tmp, SRC, SRC_PLANES, "-lm"])
    os.replace(tmp, LIB)
    return LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int), ("n_iter", ctypes.c_int), ("first_iter", ctypes.c_int),
        ("max_depth", ctypes.c_int), ("n_light", ctypes.c_int), ("cand_cap", ctypes.c_int),
        ("repeats", ctypes.c_int), ("u_max", ctypes.c_int), ("class_filter", ctypes.c_int),
        ("threads", ctypes.c_int), ("seed", ctypes.c_uint32), ("pilot", ctypes.c_int),
        ("chain_cap", ctypes.c_long), ("cost_cap", ctypes.c_double), ("o3_weights", ctypes.c_int),
        ("general_cv", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_cand", ctypes.c_double), ("n_kept", ctypes.c_double), ("n_recip_samples", ctypes.c_double),
        ("n_recip_truncated", ctypes.c_double), ("n_proxy_attempts", ctypes.c_double),
        ("n_proxy_valid", ctypes.c_double), ("bucket_B", ctypes.c_double * 10),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L.or_scene_new.restype = P
        L.or_scene_new.argtypes = [P, ctypes.c_int, P, P, P, ctypes.c_int, P, ctypes.c_int, ctypes.c_int, P,
                                   ctypes.c_int, ctypes.c_int]
        L.or_scene_free.argtypes = [P]
        L.or_scene_emitter_area.restype = ctypes.c_double
        L.or_scene_emitter_area.argtypes = [P]
        L.or_trace.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P, P]
        L.or_render.argtypes = [P, ctypes.POINTER(Params), P, P, ctypes.POINTER(Stats)]
        L.or_recip_table.restype = ctypes.c_int
        L.or_recip_table.argtypes = [P, P, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_uint32, ctypes.c_long, P, P, ctypes.c_double]
        L.or_recip_candidate.restype = ctypes.c_int
        L.or_recip_candidate.argtypes = [P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_uint32, P, P, P]
        L.or_philox4x32_10.argtypes = [P, P, P]
        L.or_bsdf_sample.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, P]
        L.or_bsdf_eval.argtypes = [P, P, P, P, P]
        D = ctypes.c_double
        L.or_planes_chord.restype = D
        L.or_planes_chord.argtypes = [D, D, D, D, D]
        L.or_planes_J.restype = D
        L.or_planes_J.argtypes = [D, D, D, D, D, D]
        L.or_planes_reference.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
        L.or_planes_render.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, P,
                                       P]
        L.or_proxy_class.restype = ctypes.c_int
        L.or_proxy_class.argtypes = [P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox(ctr, key):
    c = np.asarray(ctr, np.uint32)
    k = np.asarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def recip_table(f, q, B, n_est, estimator=0, seed=1, cap=1 << 24, rhat=1.0):
    """estimator 0: I~, 1: the sign estimator I, 2: Booth's roulette with parameter rhat."""
    f = np.ascontiguousarray(f, np.float64)
    q = np.ascontiguousarray(q, np.float64)
    est = np.zeros(n_est)
    ns = np.zeros(n_est)
    tr = lib().or_recip_table(_p(f), _p(q), len(f), float(B), estimator, n_est, seed, cap, _p(est), _p(ns),
                              float(rhat))
    return est, ns, tr


def bsdf_sample(rec, n, wo, u, mode=0):
    rec = np.ascontiguousarray(rec, np.float32)
    n = np.ascontiguousarray(n, np.float64)
    wo = np.ascontiguousarray(wo, np.float64)
    out = np.zeros(9)
    lib().or_bsdf_sample(_p(rec), _p(n), _p(wo), float(u[0]), float(u[1]), float(u[2]), mode, _p(out))
    return out


def bsdf_eval(rec, n, wo, wi):
    rec = np.ascontiguousarray(rec, np.float32)
    n, wo, wi = (np.ascontiguousarray(x, np.float64) for x in (n, wo, wi))
    out = np.zeros(4)
    lib().or_bsdf_eval(_p(rec), _p(n), _p(wo), _p(wi), _p(out))
    return out


def planes_block(sc):
    """The 27-double scene block of planes.c from a synth.scenes.planes_scene dictionary."""
    b = np.concatenate([sc["light_c"], sc["light_u"], sc["light_v"], [sc["light_eu"], sc["light_ev"]], sc["le"],
                        sc["camera"], [sc["sigma_s"], sc["sigma_t"], sc["t_max"]]]).astype(np.float64)
    assert b.shape == (27,)
    return np.ascontiguousarray(b)


def planes_chord(eu, ev, a, b, alpha):
    """Length of the chord of [-eu, eu] x [-ev, ev] through (a, b) at angle alpha."""
    return lib().or_planes_chord(float(eu), float(ev), float(a), float(b), float(alpha))


def planes_J(eu, ev, a, b, mu, mv):
    """J = int_0^pi chord(alpha; a, b) |mu cos(alpha) + mv sin(alpha)| dalpha (piecewise Gauss-Legendre)."""
    return lib().or_planes_J(float(eu), float(ev), float(a), float(b), float(mu), float(mv))


def planes_reference(sc, nt=16, ny=8):
    """Per-pixel single-scattered radiance of the pixel-centre rays by quadrature, [H, W, 3]."""
    W, H = sc["width"], sc["height"]
    img = np.zeros((H, W, 3))
    blk = planes_block(sc)
    lib().or_planes_reference(_p(blk), W, H, nt, ny, _p(img))
    return img


def planes_render(sc, n_planes, n_iter, seed=1):
    """The photon-plane estimator with the exact reciprocal: per-pixel (sum, sumsq) over n_iter."""
    W, H = sc["width"], sc["height"]
    s = np.zeros((H, W, 3))
    s2 = np.zeros((H, W, 3))
    blk = planes_block(sc)
    lib().or_planes_render(_p(blk), W, H, int(n_planes), int(n_iter), int(seed), _p(s), _p(s2))
    return s, s2


def proxy_class(is_s, is_lambert, u_max=4, general_cv=0):
    """1 when the eye path z_1 .. z_n (flags per vertex) closed at the emitter after z_n belongs to
    the proxy class (classes A, B and, with general_cv, C)."""
    a = np.ascontiguousarray(is_s, np.int32)
    b = np.ascontiguousarray(is_lambert, np.int32)
    return int(lib().or_proxy_class(_p(a), _p(b), len(a), int(u_max), int(general_cv)))


class Scene:
    """Oracle-side copy of a scene dictionary from synth.scenes."""

    def __init__(self, sc):
        self._keep = [np.ascontiguousarray(sc[k]) for k in ("tri", "tri_mat", "tri_uv", "mats", "tex", "cam")]
        tri, tri_mat, tri_uv, mats, tex, cam = self._keep
        self.W, self.H = sc["width"], sc["height"]
        self.h = lib().or_scene_new(_p(tri), tri.shape[0], _p(tri_mat), _p(tri_uv), _p(mats), mats.shape[0],
                                    _p(tex), tex.shape[1], tex.shape[0], _p(cam), self.W, self.H)

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_scene_free(self.h)
            self.h = None

    @property
    def emitter_area(self):
        return lib().or_scene_emitter_area(self.h)

    def trace(self, rays, brute=False):
        rays = np.ascontiguousarray(rays, np.float64)
        n = rays.shape[0]
        t = np.zeros(n)
        prim = np.zeros(n, np.int32)
        lib().or_trace(self.h, _p(rays), n, int(brute), _p(t), _p(prim))
        return t, prim

    def render(self, method=0, n_iter=1, first_iter=0, max_depth=8, n_light=4096, cand_cap=400, repeats=5,
               u_max=4, class_filter=0, threads=None, seed=0, pilot=16, chain_cap=1 << 21, cost_cap=4096.0,
               o3_weights=0, general_cv=0):
        """Returns (sum, sumsq, stats): per-pixel sums of per-iteration values, shape (H, W, 3).

        method 0: O1 (PT + NEE), 1: O2 (proxy-sampling BDPT), 2: O3 (plain BDPT; o3_weights 0 balance
        heuristic, 1 uniform weights, 2 light tracing alone). general_cv (O1, O2): the proxy class of
        class_filter also holds the paths of a general control vertex (Section 5.2), which O2 builds
        from class C candidates."""
        if general_cv and method == 2:
            raise ValueError("general_cv applies to O1's class filter and to O2 only")
        threads = threads or os.cpu_count() or 1
        p = Params(method, n_iter, first_iter, max_depth, n_light, cand_cap, repeats, u_max, class_filter,
                   threads, seed, pilot, chain_cap, cost_cap, o3_weights, int(general_cv))
        s = np.zeros((self.H, self.W, 3))
        s2 = np.zeros((self.H, self.W, 3))
        st = Stats()
        lib().or_render(self.h, ctypes.byref(p), _p(s), _p(s2), ctypes.byref(st))
        stats = {k: getattr(st, k) for k, _ in Stats._fields_ if k != "bucket_B"}
        stats["bucket_B"] = np.array(list(st.bucket_B)).reshape(2, 5)
        return s, s2, stats

    def recip_candidate(self, cls, u, vpos, vprim, hcpos=None, hcprim=-1, B=1.0, n_est=1000, per=1, seed=3):
        vpos = np.ascontiguousarray(vpos, np.float64)
        hc = np.ascontiguousarray(hcpos if hcpos is not None else np.zeros(3), np.float64)
        pe = np.zeros(n_est)
        re = np.zeros(n_est)
        rn = np.zeros(n_est)
        tr = lib().or_recip_candidate(self.h, cls, u, _p(vpos), int(vprim), _p(hc), int(hcprim), float(B), n_est,
                                      per, seed, _p(pe), _p(re), _p(rn))
        return pe, re, rn, tr
