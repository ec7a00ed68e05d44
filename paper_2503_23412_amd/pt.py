"""ctypes binding of libpt.so (include/pt.h). Argument marshalling only: every step of the
rendering path runs in the library's HIP kernels. Device buffers are torch tensors on the
current HIP device; the stream is torch's current stream unless one is given.

The binding raises if libpt.so is missing or fails to load; there is no fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpt.so")

PT_FLAG_NEE = 1 << 0
PT_FLAG_PROXY = 1 << 1
PT_FLAG_ONLY_PROXY_CLASS = 1 << 2
PT_FLAG_ONLY_OTHER = 1 << 3
PT_FLAG_GAMMA = 1 << 4
PT_FLAG_TILES = 1 << 5
PT_FLAG_TIMING = 1 << 6
PT_FLAG_COUNT = 1 << 7
PT_FLAG_MIS = 1 << 8
PT_FLAG_MLP = 1 << 9
PT_FLAG_SPC = 1 << 10
PT_FLAG_LT = 1 << 11
PT_FLAG_BOOTH = 1 << 12
PT_FLAG_MLP_DIR = 1 << 13
PT_FLAG_GENERAL_CV = 1 << 14
MLP_VMF = 40   # outputs of the direction head after the n_spec logits

PT_EST_ITILDE = 0
PT_EST_SIGN = 1
PT_EST_BOOTH = 2

EXPORTED = ["pt_scene_upload", "pt_scene_release", "pt_build_subspaces", "pt_render_iteration", "pt_render_batch",
            "pt_render_scenes", "pt_autotune", "pt_set_schedule", "pt_get_schedule",
            "pt_mlp_param_count", "pt_mlp_set_params", "pt_mlp_get_params", "pt_mlp_forward", "pt_mlp_train_step",
            "pt_reciprocal_estimate", "pt_resolve_image", "pt_trace_closest", "pt_scene_totals",
            "pt_selection_tables", "pt_iteration_times", "pt_philox", "pt_bvh_stats", "pt_reciprocal_estimate_noalloc",
            "pt_proxy_class", "pt_vmf_sample", "pt_planes_create", "pt_planes_render", "pt_planes_release",
            "pt_last_error"]
NOALLOC_TABLE_MAX = 1 << 20
PLANES_MAX = 1 << 22


class SceneDesc(ctypes.Structure):
    _fields_ = [
        ("n_tri", ctypes.c_int32), ("tri", ctypes.c_void_p), ("tri_mat", ctypes.c_void_p),
        ("tri_uv", ctypes.c_void_p), ("n_mat", ctypes.c_int32), ("mats", ctypes.c_void_p),
        ("tex_w", ctypes.c_int32), ("tex_h", ctypes.c_int32), ("tex", ctypes.c_void_p),
        ("camera", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("bvh_width", ctypes.c_int32), ("max_light_paths", ctypes.c_int32),
    ]


class SubspaceParams(ctypes.Structure):
    _fields_ = [("n_pretrace", ctypes.c_int32), ("n_eye", ctypes.c_int32), ("n_spec", ctypes.c_int32),
                ("kmeans_iters", ctypes.c_int32), ("seed", ctypes.c_uint32), ("n_light", ctypes.c_int32),
                ("n_ctrl", ctypes.c_int32)]


class IterParams(ctypes.Structure):
    _fields_ = [
        ("iteration", ctypes.c_uint32), ("seed", ctypes.c_uint32), ("max_depth", ctypes.c_int32),
        ("n_light", ctypes.c_int32), ("cand_cap", ctypes.c_int32), ("recip_repeats", ctypes.c_int32),
        ("u_max", ctypes.c_int32), ("pilot", ctypes.c_int32), ("cost_cap", ctypes.c_float),
        ("train_iters", ctypes.c_int32), ("tile", ctypes.c_int32), ("tile_threshold", ctypes.c_float),
        ("tile_low_prob", ctypes.c_float), ("defensive", ctypes.c_float), ("flags", ctypes.c_uint32),
        ("mlp_lr", ctypes.c_float), ("mlp_mix", ctypes.c_float), ("booth_r", ctypes.c_float),
    ]


class IterStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "rays_extend_eye", "rays_extend_light", "rays_shadow", "rays_proxy", "rays_recip",
        "n_cand", "n_kept", "n_recip_samples", "n_recip_truncated",
        "n_proxy_attempts", "n_proxy_valid", "n_nan", "node_visits", "tri_tests",
        "ms_extend", "n_extend_launches", "n_pool", "n_connections", "n_lt_splats", "ms_recip", "ms_recip_stage_a",
        "node_visits_recip", "tri_tests_recip", "node_visits_stage_a", "tri_tests_stage_a", "n_samples_stage_a",
        "n_drawn_stage_a", "n_drawn_pilot", "wave_trips_stage_a")] + [
        ("chain_len_hist", ctypes.c_double * 24), ("chain_len_max", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["chain_len_hist"] = list(self.chain_len_hist)
        return d


class TuneResult(ctypes.Structure):
    _fields_ = [("stage_a_budget", ctypes.c_uint32), ("round_grid", ctypes.c_int32), ("ms_best", ctypes.c_float),
                ("ms_previous", ctypes.c_float), ("iterations_rendered", ctypes.c_uint32),
                ("ext_wg", ctypes.c_int32), ("queue_chunk", ctypes.c_int32), ("bvh_width", ctypes.c_int32),
                ("stage_a_ahead", ctypes.c_int32), ("stage_a_refill", ctypes.c_int32)]


class Totals(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("iterations", "n_nan", "n_recip_truncated", "n_proxy_valid",
                                               "n_recip_samples", "n_cand", "captures", "bvh_stack_need",
                                               "bvh_depth")]


class CandDesc(ctypes.Structure):
    _fields_ = [("cls", ctypes.c_int32), ("u", ctypes.c_int32), ("v", ctypes.c_float * 3), ("v_prim", ctypes.c_int32),
                ("hc", ctypes.c_float * 3), ("hc_prim", ctypes.c_int32), ("hc_b1", ctypes.c_float),
                ("hc_b2", ctypes.c_float)]


class RecipQuery(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("n", ctypes.c_int32), ("f_dev", ctypes.c_void_p),
                ("q_dev", ctypes.c_void_p), ("B", ctypes.c_float), ("n_est", ctypes.c_int32),
                ("estimator", ctypes.c_int32), ("seed", ctypes.c_uint32), ("cap", ctypes.c_uint32),
                ("cand", ctypes.POINTER(CandDesc)), ("per", ctypes.c_int32), ("out_p_dev", ctypes.c_void_p),
                ("booth_r", ctypes.c_float)]


_lib = None


def lib():
    """Load libpt.so (raises OSError when it is missing or does not load)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, I = ctypes.c_void_p, ctypes.c_int32
        L.pt_scene_upload.argtypes = [ctypes.POINTER(SceneDesc), P, ctypes.POINTER(P)]
        L.pt_scene_release.argtypes = [P]
        L.pt_build_subspaces.argtypes = [P, ctypes.POINTER(SubspaceParams), P]
        L.pt_render_iteration.argtypes = [P, ctypes.POINTER(IterParams), P, P, ctypes.POINTER(IterStats), P]
        L.pt_render_batch.argtypes = [P, ctypes.POINTER(IterParams), ctypes.c_uint32, P, P, P]
        L.pt_reciprocal_estimate.argtypes = [P, ctypes.POINTER(RecipQuery), P, P, P]
        L.pt_resolve_image.argtypes = [P, P, ctypes.c_uint32, P, P]
        L.pt_trace_closest.argtypes = [P, P, I, P, P, P]
        L.pt_render_scenes.argtypes = [P, P, I, ctypes.c_uint32, P, P, P]
        L.pt_autotune.argtypes = [P, ctypes.POINTER(IterParams), P, P, ctypes.POINTER(TuneResult), P]
        L.pt_set_schedule.argtypes = [P, ctypes.POINTER(TuneResult)]
        L.pt_get_schedule.argtypes = [P, ctypes.POINTER(TuneResult)]
        L.pt_mlp_param_count.argtypes = [P, ctypes.POINTER(I)]
        L.pt_mlp_set_params.argtypes = [P, P, I, P]
        L.pt_mlp_get_params.argtypes = [P, P, I, P]
        L.pt_mlp_forward.argtypes = [P, P, I, P, P]
        L.pt_mlp_train_step.argtypes = [P, P, P, P, I, P, P, P, I, ctypes.c_float, P, P]
        L.pt_vmf_sample.argtypes = [P, I, ctypes.c_uint32, P, P, P]
        L.pt_scene_totals.argtypes = [P, ctypes.POINTER(Totals), I, P]
        L.pt_selection_tables.argtypes = [P, I, I, I, P, P, P, P, P, P, P]
        L.pt_philox.argtypes = [P, I, P, P]
        L.pt_iteration_times.argtypes = [P, ctypes.c_uint32, I, P, P]
        L.pt_bvh_stats.argtypes = [P, I, I, P, P, P]
        L.pt_reciprocal_estimate_noalloc.argtypes = [ctypes.POINTER(RecipQuery), P, P, P]
        L.pt_proxy_class.argtypes = [P, I, ctypes.c_uint32, I, I, I, ctypes.POINTER(I)]
        L.pt_planes_create.argtypes = [ctypes.POINTER(PlanesDesc), P, ctypes.POINTER(P)]
        L.pt_planes_render.argtypes = [P, I, ctypes.c_uint32, ctypes.c_uint32, P, P, ctypes.POINTER(PlanesStats), P]
        L.pt_planes_release.argtypes = [P]
        L.pt_last_error.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name == "pt_last_error":
                continue
            getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


class PTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libpt error {code}: {msg}")
        self.code = code


def _check(code):
    if code != 0:
        raise PTError(code, lib().pt_last_error().decode())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def default_params(**kw):
    p = dict(iteration=0, seed=0, max_depth=8, n_light=4096, cand_cap=400, recip_repeats=5, u_max=4, pilot=16,
             cost_cap=4096.0, train_iters=40, tile=10, tile_threshold=0.05, tile_low_prob=0.2, defensive=0.1,
             flags=PT_FLAG_NEE | PT_FLAG_PROXY, mlp_lr=1e-3, mlp_mix=0.9, booth_r=1.0)
    p.update(kw)
    return p


class PlanesDesc(ctypes.Structure):
    _fields_ = [("light_c", ctypes.c_float * 3), ("light_u", ctypes.c_float * 3), ("light_v", ctypes.c_float * 3),
                ("light_eu", ctypes.c_float), ("light_ev", ctypes.c_float), ("le", ctypes.c_float * 3),
                ("camera", ctypes.c_float * 10), ("sigma_s", ctypes.c_float), ("sigma_t", ctypes.c_float),
                ("t_max", ctypes.c_float), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("max_planes", ctypes.c_int32)]


class PlanesStats(ctypes.Structure):
    _fields_ = [("n_hits", ctypes.c_double), ("n_samples", ctypes.c_double), ("n_truncated", ctypes.c_double),
                ("n_nan", ctypes.c_double)]


class Planes:
    """Photon-plane single scattering (pt_planes_*) for a synth.scenes.planes_scene dictionary."""

    def __init__(self, sc, max_planes, stream=None):
        f = lambda v, n: (ctypes.c_float * n)(*[float(x) for x in v])  # noqa: E731
        d = PlanesDesc(f(sc["light_c"], 3), f(sc["light_u"], 3), f(sc["light_v"], 3), float(sc["light_eu"]),
                       float(sc["light_ev"]), f(sc["le"], 3), f(sc["camera"], 10), float(sc["sigma_s"]),
                       float(sc["sigma_t"]), float(sc["t_max"]), int(sc["width"]), int(sc["height"]),
                       int(max_planes))
        self.h = ctypes.c_void_p()
        self.W, self.H = int(sc["width"]), int(sc["height"])
        _check(lib().pt_planes_create(ctypes.byref(d), _stream(stream), ctypes.byref(self.h)))

    def render(self, accum, accum_sq, n_planes, iteration=0, seed=1, stats=False, stream=None):
        st = PlanesStats() if stats else None
        _check(lib().pt_planes_render(self.h, int(n_planes), int(iteration), int(seed), _ptr(accum), _ptr(accum_sq),
                                      ctypes.byref(st) if st is not None else None, _stream(stream)))
        return {k: getattr(st, k) for k, _ in PlanesStats._fields_} if st is not None else None

    def release(self):
        if self.h:
            lib().pt_planes_release(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Scene:
    """A scene uploaded to the current HIP device."""

    def __init__(self, sc, max_light_paths=4096, stream=None, bvh_width=4):
        self._host = [np.ascontiguousarray(sc[k]) for k in ("tri", "tri_mat", "tri_uv", "mats", "tex", "cam")]
        tri, tri_mat, tri_uv, mats, tex, cam = self._host
        self.width, self.height = int(sc["width"]), int(sc["height"])
        d = SceneDesc(tri.shape[0], tri.ctypes.data, tri_mat.ctypes.data, tri_uv.ctypes.data, mats.shape[0],
                      mats.ctypes.data, tex.shape[1], tex.shape[0], tex.ctypes.data, cam.ctypes.data,
                      self.width, self.height, int(bvh_width), int(max_light_paths))
        h = ctypes.c_void_p()
        _check(lib().pt_scene_upload(ctypes.byref(d), _stream(stream), ctypes.byref(h)))
        self.h = h
        self.max_light_paths = int(max_light_paths)

    def release(self):
        if getattr(self, "h", None):
            lib().pt_scene_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def build_subspaces(self, n_pretrace=0, n_eye=64, n_spec=64, kmeans_iters=8, seed=0, n_light=0, n_ctrl=10,
                        stream=None):
        p = SubspaceParams(n_pretrace, n_eye, n_spec, kmeans_iters, seed, n_light, n_ctrl)
        _check(lib().pt_build_subspaces(self.h, ctypes.byref(p), _stream(stream)))

    def render_iteration(self, accum, accum_sq=None, stats=False, stream=None, **params):
        p = IterParams(**default_params(**params))
        st = IterStats() if stats else None
        _check(lib().pt_render_iteration(self.h, ctypes.byref(p), _ptr(accum), _ptr(accum_sq),
                                         ctypes.byref(st) if st is not None else None, _stream(stream)))
        return st.as_dict() if st is not None else None

    def render_batch(self, accum, accum_sq, n_iter, stream=None, **params):
        """n_iter iterations from params['iteration'] on, replaying one captured HIP graph."""
        p = IterParams(**default_params(**params))
        _check(lib().pt_render_batch(self.h, ctypes.byref(p), int(n_iter), _ptr(accum), _ptr(accum_sq),
                                     _stream(stream)))

    def resolve(self, accum, n_iter, out, stream=None):
        _check(lib().pt_resolve_image(self.h, _ptr(accum), int(n_iter), _ptr(out), _stream(stream)))

    def recip_candidate(self, cls, u, v, v_prim, B, n_est, out, nsamples, p_out=None, hc=(0.0, 0.0, 0.0), hc_prim=-1,
                        hc_b=(0.0, 0.0), per=1, seed=3, cap=0, stream=None):
        """Estimates of 1/P (out) and of P (p_out, `per` samples each) for one incomplete sub-path."""
        d = CandDesc(int(cls), int(u), (ctypes.c_float * 3)(*v), int(v_prim), (ctypes.c_float * 3)(*hc), int(hc_prim),
                     float(hc_b[0]), float(hc_b[1]))
        q = RecipQuery(1, 0, None, None, float(B), int(n_est), 0, int(seed), int(cap), ctypes.pointer(d), int(per),
                       p_out.data_ptr() if p_out is not None else None)
        _check(lib().pt_reciprocal_estimate(self.h, ctypes.byref(q), _ptr(out), _ptr(nsamples), _stream(stream)))

    def schedule(self):
        """The scene's current schedule knobs (as last tuned or set), named as in autotune's result."""
        r = TuneResult()
        _check(lib().pt_get_schedule(self.h, ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in r._fields_ if k not in ("ms_best", "ms_previous", "iterations_rendered")}

    def set_schedule(self, **knobs):
        """Set schedule knobs (names of the autotuner's result); the others keep their values."""
        cur = self.schedule()
        cur.update(knobs)
        r = TuneResult(**cur)
        _check(lib().pt_set_schedule(self.h, ctypes.byref(r)))

    def autotune(self, accum, accum_sq=None, stream=None, **params):
        """Time the reciprocal-chain schedule choices and keep the fastest (renders into accum)."""
        p = IterParams(**default_params(**params))
        r = TuneResult()
        _check(lib().pt_autotune(self.h, ctypes.byref(p), _ptr(accum), _ptr(accum_sq), ctypes.byref(r),
                                 _stream(stream)))
        return {k: getattr(r, k) for k, _ in r._fields_}

    # learned subspace selection (PT_FLAG_MLP): parameters and the network's two passes
    def mlp_param_count(self):
        n = ctypes.c_int32()
        _check(lib().pt_mlp_param_count(self.h, ctypes.byref(n)))
        return n.value

    def mlp_set_params(self, params, stream=None):
        a = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().pt_mlp_set_params(self.h, a.ctypes.data, int(a.size), _stream(stream)))

    def mlp_get_params(self, stream=None):
        a = np.empty(self.mlp_param_count(), dtype=np.float32)
        _check(lib().pt_mlp_get_params(self.h, a.ctypes.data, int(a.size), _stream(stream)))
        return a

    def mlp_forward(self, feat, out, stream=None):
        """feat: float32 device [n, 9]; out: float32 device [n, n_spec + MLP_VMF] (logits, then the
        direction head's mixture outputs; bias included)."""
        _check(lib().pt_mlp_forward(self.h, _ptr(feat), int(feat.shape[0]), _ptr(out), _stream(stream)))

    def mlp_train_step(self, feat, label, weight, lr, feat_dir=None, dirs=None, weight_dir=None, want_grad=False,
                       stream=None):
        """One Adam step on weighted subspace samples and (optionally) weighted direction samples
        (device tensors); returns the gradient when asked."""
        g = np.empty(self.mlp_param_count(), dtype=np.float32) if want_grad else None
        n = int(feat.shape[0]) if feat is not None else 0
        nd = int(feat_dir.shape[0]) if feat_dir is not None else 0
        _check(lib().pt_mlp_train_step(self.h, _ptr(feat), _ptr(label), _ptr(weight), n, _ptr(feat_dir), _ptr(dirs),
                                       _ptr(weight_dir), nd, float(lr), g.ctypes.data if g is not None else None,
                                       _stream(stream)))
        return g

    def totals(self, reset=False, stream=None):
        """Running totals over every iteration rendered so far (synchronises)."""
        t = Totals()
        _check(lib().pt_scene_totals(self.h, ctypes.byref(t), int(bool(reset)), _stream(stream)))
        return {k: getattr(t, k) for k, _ in t._fields_}

    def iteration_times(self, first, n, stream=None):
        """Device wall-clock duration (ms) of iterations first .. first + n - 1 (-1 where unrecorded)."""
        out = np.zeros(n, np.float64)
        _check(lib().pt_iteration_times(self.h, int(first), int(n), out.ctypes.data, _stream(stream)))
        return out

    def selection_tables(self, which, n_rows, n_cols, stream=None):
        """The latest iteration's alias rows (which 0: Gamma, 1: Q) as host arrays."""
        ne = ctypes.c_int32()
        nonempty = np.zeros(n_cols, np.int32)
        prob = np.zeros((n_rows, n_cols), np.float32)
        alias = np.zeros((n_rows, n_cols), np.int32)
        pmf = np.zeros((n_rows, n_cols), np.float32)
        w = np.zeros((n_rows, n_cols), np.float32)
        _check(lib().pt_selection_tables(self.h, int(which), int(n_rows), int(n_cols), ctypes.byref(ne),
                                         nonempty.ctypes.data, prob.ctypes.data, alias.ctypes.data, pmf.ctypes.data,
                                         w.ctypes.data, _stream(stream)))
        return dict(n_nonempty=ne.value, nonempty=nonempty, prob=prob, alias=alias, pmf=pmf, weights=w)

    def trace_closest(self, rays, t_out, prim_out, stream=None):
        _check(lib().pt_trace_closest(self.h, _ptr(rays), int(rays.shape[0]), _ptr(t_out), _ptr(prim_out),
                                      _stream(stream)))


def reciprocal_table(f, q, B, n_est, out, nsamples, estimator=PT_EST_ITILDE, seed=1, cap=0, booth_r=1.0,
                     stream=None):
    """f, q: float32 device tensors; out float32 [n_est], nsamples int32 [n_est] (device)."""
    qq = RecipQuery(0, int(f.shape[0]), f.data_ptr(), q.data_ptr(), float(B), int(n_est), int(estimator), int(seed),
                    int(cap), None, 0, None, float(booth_r))
    _check(lib().pt_reciprocal_estimate(None, ctypes.byref(qq), _ptr(out), _ptr(nsamples), _stream(stream)))


def philox(inp, out, stream=None):
    """inp: int32/uint32 device tensor [n, 6] (counter 0..3, key 0..1); out: [n, 4] (device)."""
    _check(lib().pt_philox(_ptr(inp), int(inp.shape[0]), _ptr(out), _stream(stream)))


def vmf_sample(raw, seed, dirs, pdf, stream=None):
    """raw: float32 device [n, 40] mixtures; writes dirs [n, 3] and pdf [n] (device)."""
    _check(lib().pt_vmf_sample(_ptr(raw), int(raw.shape[0]), int(seed), _ptr(dirs), _ptr(pdf), _stream(stream)))


def bvh_stats(tri, width=4):
    """Host-only: (nodes, worst-case traversal stack, depth) of the BVH of tri [n, 9] (width 4 or 8)."""
    t = np.ascontiguousarray(tri, np.float32).reshape(-1, 9)
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().pt_bvh_stats(t.ctypes.data, int(t.shape[0]), int(width), ctypes.byref(a), ctypes.byref(b),
                              ctypes.byref(c)))
    return a.value, b.value, c.value


def proxy_class(eye_flags, light_sig=0, j=0, u_max=4, general_cv=0):
    """Host-only: 1 when the path camera -> z_1 .. z_n (eye_flags: bit 0 specular, bit 1 Lambertian)
    -> y_j .. y_1 (from the light signature light_sig) -> emitter is in the proxy class."""
    e = np.ascontiguousarray(eye_flags, np.uint8)
    out = ctypes.c_int32()
    _check(lib().pt_proxy_class(e.ctypes.data if e.size else None, int(e.size), int(light_sig) & 0xFFFFFFFF, int(j),
                                int(u_max), int(general_cv), ctypes.byref(out)))
    return out.value


def reciprocal_table_noalloc(f, q, B, n_est, out, nsamples, estimator=PT_EST_ITILDE, seed=1, cap=0, booth_r=1.0,
                             stream=None):
    """reciprocal_table through the entry point that allocates nothing (tables <= NOALLOC_TABLE_MAX)."""
    qq = RecipQuery(0, int(f.shape[0]), f.data_ptr(), q.data_ptr(), float(B), int(n_est), int(estimator), int(seed),
                    int(cap), None, 0, None, float(booth_r))
    _check(lib().pt_reciprocal_estimate_noalloc(ctypes.byref(qq), _ptr(out), _ptr(nsamples), _stream(stream)))


def render_scenes(scenes, accums, accums_sq, n_iter, params, stream=None):
    """n_iter iterations of every scene from one captured multi-scene graph; params: one dict each."""
    n = len(scenes)
    hs = (ctypes.c_void_p * n)(*[sc.h.value for sc in scenes])
    ps = (IterParams * n)(*[IterParams(**default_params(**q)) for q in params])
    a = (ctypes.c_void_p * n)(*[t.data_ptr() for t in accums])
    b = (ctypes.c_void_p * n)(*[t.data_ptr() for t in accums_sq]) if accums_sq is not None else None
    _check(lib().pt_render_scenes(hs, ps, n, int(n_iter), a, b, _stream(stream)))
