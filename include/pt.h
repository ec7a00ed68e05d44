/*
 * pt.h -- C ABI of the MI355X (gfx950) proxy-sampling BDPT library, libpt.so.
 *
 * Method: Su et al., "Proxy Tracing: Unbiased Reciprocal Estimation for Optimized
 * Sampling in BDPT". Every rendering iteration estimates, for every pixel j, the path
 * integral I_j = int f_j(x) dmu(x) (Section 3.1, path integral equation) with one sample
 * per pixel (Section 6.1: one iteration = 1 spp), from a cache of M light sub-paths that
 * all pixels share (Section 3.2), reciprocal estimates of the densities of incomplete light
 * sub-paths (Sections 4.2 and 5.2) and proxy retraces at the eye's first diffuse vertex
 * (Section 5.1).
 *
 * Conventions shared by every call:
 *  - Pointers named *_dev are device pointers (HIP device memory, e.g. torch tensors on
 *    cuda:0); every other pointer is host memory. The library never frees caller memory.
 *  - hip_stream is a hipStream_t (may be NULL = the legacy default stream). All device work
 *    is enqueued on it in order; no call synchronises the host unless it says so.
 *  - The library owns everything reachable from a pt_scene (geometry, BVH, light cache,
 *    candidates, statistics, workspaces); pt_scene_release frees it.
 *  - Return value: PT_OK (0) or a negative pt_status. Invalid arguments return PT_EINVAL
 *    and change no state. pt_last_error() gives a message for the last failing call on the
 *    calling thread. No C++ exception crosses this interface.
 *  - Only gfx950 code objects are built; another device returns PT_EUNSUPPORTED.
 */
#ifndef PT_H
#define PT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pt_status;
enum {
    PT_OK = 0,
    PT_EINVAL = -1,       /* bad argument; nothing changed */
    PT_ENOMEM = -2,       /* device allocation failed; the scene stays valid */
    PT_EDEVICE = -3,      /* a HIP call failed */
    PT_ESTATE = -4,       /* call out of order (e.g. render before build_subspaces) */
    PT_EUNSUPPORTED = -5  /* not a gfx950 device, or a scene the kernels cannot hold (e.g. a BVH whose
                             traversal would need more stack entries than the kernels keep) */
};

typedef struct pt_scene pt_scene;

/* Material record: 16 floats per material, host memory.
 *  [0] type: 0 Lambert, 1 conductor (GGX, alpha = max(roughness^2, 1e-4); roughness exactly 0
 *      is a perfect mirror), 2 smooth dielectric (outside index 1)
 *  [1..3] albedo (Lambert) or F0 (conductor, Schlick Fresnel)
 *  [4] roughness   [5] index of refraction   [6..8] emitted radiance (Lambert only)
 *  [9] 1: emission is multiplied by the emission texture at the surface (u, v)
 * A vertex is specular (S) for a conductor or dielectric with roughness < 0.2 (Section 6.1);
 * every other vertex is diffuse (D). Emitters emit on the front side of their triangles. */
typedef struct {
    int32_t n_tri;
    const float *tri;        /* [n_tri * 9] v0, v1, v2; front = (v1-v0) x (v2-v0) */
    const int32_t *tri_mat;  /* [n_tri] material index */
    const float *tri_uv;     /* [n_tri * 6] per-vertex (u, v) */
    int32_t n_mat;
    const float *mats;       /* [n_mat * 16] */
    int32_t tex_w, tex_h;
    const float *tex;        /* [tex_h * tex_w] emission texture, row-major, nearest lookup */
    const float *camera;     /* [10] position, target, up, vertical fov (degrees) */
    int32_t width, height;   /* image size */
    int32_t bvh_width;       /* 4 or 8: the BVH width the walks use; 0: both trees are built and
                                the 4-wide one is used until pt_autotune picks */
    int32_t max_light_paths; /* capacity for M, light sub-paths per iteration */
} pt_scene_desc;

/* Upload a scene: the measurement's geometry, materials, emitters and sensor (Section 3.1: the
 * path integral's surfaces and the pixel filters f_j, here a pinhole camera whose pixel (x, y)
 * integrates over its square of the image plane), plus the capacity for the M light sub-paths
 * every iteration traces (Section 3.2). Validates the arrays, builds a binned-SAH BVH on the
 * host, collapses it to 4-wide 128-byte nodes and/or 8-wide 128-byte nodes with 8-bit quantised
 * child boxes (bvh_width; both share the leaves), copies everything to the current device and
 * allocates per-iteration workspaces sized for width x height pixels and max_light_paths light
 * sub-paths. Host arrays may be freed on return. On success *out receives the handle.
 * Synchronises hip_stream. Errors: PT_EINVAL for malformed arrays (nothing allocated),
 * PT_EUNSUPPORTED when the requested tree's worst-case traversal needs more stack entries than
 * the kernels hold (48 per thread for 4-wide walks, 64 for 8-wide ones; bvh_width 0: when
 * neither tree fits; a tree that does not fit is not kept),
 * PT_ENOMEM when a device allocation fails. */
pt_status pt_scene_upload(const pt_scene_desc *desc, void *hip_stream, pt_scene **out);

/* Free everything the scene owns. Synchronises the device first. NULL is a no-op. */
pt_status pt_scene_release(pt_scene *s);

/* Subspace construction (Section 3.2, SPCBPT's subspaces; Section 5.5's specular and control
 * subspaces): pre-traces n_pretrace paths and clusters eye first-diffuse vertices (T), specular
 * light vertices (S), connectable light vertices (S_L) and the control vertices of class-B
 * incomplete sub-paths (C) by (position, normal, incident direction) with k-means. Resets the selection matrices Gamma (Section 5.6) and Q (light-vertex
 * connections) to uniform and clears all running statistics.
 * Must be called once before pt_render_iteration. */
typedef struct {
    int32_t n_pretrace;      /* pre-traced samples (eye and light paths each) */
    int32_t n_eye;           /* eye subspaces T (<= 4096) */
    int32_t n_spec;          /* specular subspaces S (<= 4096) */
    int32_t kmeans_iters;    /* Lloyd iterations */
    uint32_t seed;
    int32_t n_light;         /* light subspaces S_L of the probabilistic connections (<= 4096; 0: n_eye) */
    int32_t n_ctrl;          /* control subspaces C (Section 5.5) of the class-B control vertices y_0 on the
                                emitters (<= 256; 0 or 1: none). The reciprocal statistics that feed the
                                MIS weights (Section 5.4) and the floor of B are kept per (class, u, S, C) */
} pt_subspace_params;
pt_status pt_build_subspaces(pt_scene *s, const pt_subspace_params *p, void *hip_stream);

/* flags of pt_iter_params */
enum {
    PT_FLAG_NEE = 1u << 0,          /* next-event estimation at non-Dirac eye vertices */
    PT_FLAG_PROXY = 1u << 1,        /* proxy connections (class A = L S^u, class B = L D S^u) */
    PT_FLAG_ONLY_PROXY_CLASS = 1u << 2,  /* score only paths the proxy strategy can build */
    PT_FLAG_ONLY_OTHER = 1u << 3,   /* score only the other paths */
    PT_FLAG_GAMMA = 1u << 4,        /* select incomplete sub-paths by Gamma[T, S] (else uniformly) */
    PT_FLAG_TILES = 1u << 5,        /* 10x10-pixel tile gating of proxy attempts (Section 6.1) */
    PT_FLAG_TIMING = 1u << 6,       /* time the extension kernels with HIP events into the stats */
    PT_FLAG_COUNT = 1u << 7,        /* count BVH node visits and triangle tests of extension rays */
    PT_FLAG_MIS = 1u << 8,          /* variance-aware MIS for proxy paths (Section 5.4) */
    PT_FLAG_SPC = 1u << 10,         /* probabilistic connections: each eye vertex to one light vertex
                                       drawn from the pool of all light sub-path vertices (max_depth <= 16) */
    PT_FLAG_LT = 1u << 11,          /* light tracing: every pool vertex splats onto the image (max_depth <= 16) */
    PT_FLAG_MLP = 1u << 9           /* learned subspace selection: mlp_mix x network softmax +
                                       (1 - mlp_mix) x the plain row (Gamma row with PT_FLAG_GAMMA,
                                       else uniform over the non-empty subspaces); trained online
                                       while iteration < train_iters */
    ,
    PT_FLAG_BOOTH = 1u << 12,       /* reciprocal chains with Booth's roulette (parameter booth_r)
                                       instead of the RRS function of equ:rr (RR ablation) */
    PT_FLAG_MLP_DIR = 1u << 13,     /* with PT_FLAG_MLP: the first retrace direction at a glossy
                                       (non-Dirac) y_{s-1} from mlp_mix x the network's vMF mixture +
                                       (1 - mlp_mix) x BSDF sampling; trained online like the logits */
    PT_FLAG_GENERAL_CV = 1u << 14   /* general control vertex (Sections 5.2, 5.3): proxy candidates
                                       of class C as well, h_c = y_j (j >= 1) on a Lambertian
                                       surface with the control direction from y_{j-1}, the retrace
                                       for u = 1 also sampling the BSDF at h_c (the cosine on the
                                       control direction's side); the proxy class then holds
                                       L ... D D S^u paths, which the other strategies then leave
                                       to it. Needs PT_FLAG_PROXY; not with PT_FLAG_MIS (the
                                       variance-aware weights over the larger class are not
                                       built), so the strategies partition the paths */
};

typedef struct {
    uint32_t iteration;      /* k: keys every random stream of this iteration */
    uint32_t seed;
    int32_t max_depth;       /* maximum number of segments of a full path (1 .. 127) */
    int32_t n_light;         /* M light sub-paths (<= max_light_paths) */
    int32_t cand_cap;        /* expected number of candidates kept per iteration (400) */
    int32_t recip_repeats;   /* reciprocal estimates averaged per candidate (5) */
    int32_t u_max;           /* longest specular run handled by the proxy strategy (<= 4) */
    int32_t pilot;           /* minimum pilot samples per candidate (B and cost estimate); 0: no pilot, B and
                                beta from the candidate's (class, u, S, C) bucket statistics of earlier
                                iterations (needs PT_FLAG_GAMMA, PT_FLAG_MIS or PT_FLAG_MLP) */
    float cost_cap;          /* expected chain samples per candidate above which it is roulette-kept */
    int32_t train_iters;     /* iterations during which Gamma and tile statistics learn (40) */
    int32_t tile;            /* tile edge in pixels (10) */
    float tile_threshold;    /* proxy share above which a tile always attempts (0.05) */
    float tile_low_prob;     /* attempt probability of the other tiles (0.2) */
    float defensive;         /* uniform fraction mixed into Gamma rows (0.1) */
    uint32_t flags;
    float mlp_lr;            /* Adam step size of the learned selection (1e-3) */
    float mlp_mix;           /* weight of the network in the selection mixture, in [0, 1) (0.9) */
    float booth_r;           /* PT_FLAG_BOOTH: parameter of Booth's roulette (> 0) */
} pt_iter_params;

/* Host-visible per-iteration statistics (valid once the stream is synchronised when
 * pt_render_iteration was given a non-NULL pointer; that call synchronises). */
typedef struct {
    double rays_extend_eye, rays_extend_light, rays_shadow, rays_proxy, rays_recip;
    double n_cand, n_kept, n_recip_samples, n_recip_truncated;
    double n_proxy_attempts, n_proxy_valid, n_nan;
    double node_visits, tri_tests;   /* eye extension rays, when PT_FLAG_COUNT is set */
    double ms_extend;                /* summed duration of the extension launches (PT_FLAG_TIMING) */
    double n_extend_launches;
    double n_pool, n_connections, n_lt_splats;   /* light vertices in the pool; connections and splats made */
    double ms_recip, ms_recip_stage_a;  /* reciprocal block (pilot to last round) and its first chain
                                           kernel, HIP events on the stream (PT_FLAG_TIMING) */
    double node_visits_recip, tri_tests_recip;   /* traversal work of the pilot and the chain rounds */
    double node_visits_stage_a, tri_tests_stage_a, n_samples_stage_a;   /* the first chain kernel's */
    double n_drawn_stage_a, n_drawn_pilot;   /* f/q samples drawn (64 per wavefront step) by the first
                                                chain kernel and by the pilot */
    double wave_trips_stage_a;               /* traversal loop trips of the first chain kernel's
                                                wavefronts: node visits / (64 trips) is its SIMD
                                                efficiency (PT_FLAG_COUNT) */
    double chain_len_hist[24];       /* reciprocal chains by samples used: bin b counts [2^b, 2^(b+1)) */
    double chain_len_max;            /* longest chain of the iteration (samples) */
} pt_iter_stats;

/* One iteration: 1 sample per pixel of every estimator strategy, added into the CALLER-OWNED
 * device buffers accum_rgb_dev[H*W*3] (+= the iteration's pixel value) and
 * accum_sq_dev[H*W*3] (+= its square; may be NULL). Row-major, pixel (x, y) at y*W + x.
 * stats may be NULL; when given, the call synchronises the stream and fills it. */
pt_status pt_render_iteration(pt_scene *s, const pt_iter_params *p, float *accum_rgb_dev, float *accum_sq_dev,
                              pt_iter_stats *stats, void *hip_stream);

/* n_iter consecutive iterations (p->iteration, p->iteration + 1, ...) by replaying one captured
 * HIP graph of an iteration; the same results as n_iter pt_render_iteration calls with the same
 * parameters. The graph is captured on first use and re-captured when the parameters (other
 * than the iteration index), the buffers or the scene's state generation (see pt_render_scenes)
 * change. No statistics; PT_FLAG_TIMING is rejected. */
pt_status pt_render_batch(pt_scene *s, const pt_iter_params *p, uint32_t n_iter, float *accum_rgb_dev,
                          float *accum_sq_dev, void *hip_stream);

/* Several scenes (1 .. 64, each appearing once) per launch: one HIP graph holds one iteration of
 * every scene, each on its own branch so that the device runs small scenes side by side, and is
 * replayed n_iter times on hip_stream (iterations params[i].iteration, +1, ...). With two or more
 * scenes the first stage of the reciprocal chains (the iteration's largest kernel) is one
 * persistent launch for all of them: the branches join after their roulette, one grid takes
 * (scene, chain) items from a single work queue over every scene's chains (scenes[0]'s queue
 * chunk, see pt_autotune), and the branches fork again for the chain rounds and the rest of the
 * iteration; each scene's estimates are those of pt_render_iteration with its parameters. Scene i
 * accumulates into accum_rgb[i] / accum_sq[i] (accum_sq may be NULL) as pt_render_iteration
 * does. The graph belongs to scenes[0] and is rebuilt when a scene, a parameter other than the
 * iteration index, a buffer or a scene's state changes: every scene carries a state generation,
 * unique in the process, that upload, pt_build_subspaces, the network's allocation and
 * pt_autotune advance, and the graph's key holds each scene's generation, so a graph is never
 * replayed on a scene it was not captured for (a scene released and another uploaded at the same
 * host address included). PT_FLAG_TIMING is rejected. */
pt_status pt_render_scenes(pt_scene *const *scenes, const pt_iter_params *params, int32_t n_scenes, uint32_t n_iter,
                           float *const *accum_rgb, float *const *accum_sq, void *hip_stream);

/* Schedule autotuning on this scene and parameters, by coordinate descent: each knob is timed over
 * three iterations (after one to settle) for each of its values, with the choices made before
 * it, and the fastest value is kept by the scene for later iterations. The knobs, in order: the
 * BVH width the walks use (4 or 8, when the scene was uploaded with bvh_width 0 and both trees
 * fit the stack); the sample budget of the reciprocal chains' one-wavefront stage (512 .. 8192)
 * with the grid of their round kernels (1,024 .. 8,192 blocks); the workgroup size of the ray
 * extension launches (64, 128, 256 threads: each thread's traversal stack lives in LDS, so the
 * size trades occupancy per CU against workgroups in flight); the number of chains a wavefront
 * of the one-wavefront stage takes from its work queue per visit (1, 2, 4; also used by the
 * multi-scene stage of pt_render_scenes); how many steps of 64 samples a lane of that stage may
 * compute beyond the oldest step its chain has not consumed (1: lockstep; 2: a lane whose sample
 * ended early starts the next while the others still trace); whether that stage walks the tree
 * one node at a time and restarts a lane whose walk ended (its next trip or next sample) while
 * the others still walk (4-wide trees). Every choice gives the same estimator (a ray's hit
 * does not depend on the tree's width or its workgroup, and the chains consume i.i.d. samples
 * whoever draws them), so it changes speed only. The timed iterations render into accum_rgb /
 * accum_sq (iterations p->iteration, +1, ...); their number is returned in iterations_rendered.
 * The knobs are timed one after another, so call it once the iteration's cost has settled: after
 * the first 40 iterations, in which the Gamma, Q and tile statistics learn (while they learn the
 * cost falls, and the value timed last would look best). The starting knobs are timed twice
 * before the descent, and at its end the chosen and the starting knobs are timed alternately
 * twice each; the starting ones stay if they were faster (a transient slowdown during the descent
 * leaves no slower schedule behind). Synchronises hip_stream. */
typedef struct {
    uint32_t stage_a_budget;     /* chosen sample budget of the one-wavefront stage */
    int32_t round_grid;          /* chosen blocks of the round kernels */
    float ms_best;               /* iteration time with the chosen schedule (final check) */
    float ms_previous;           /* iteration time with the knobs the scene had before */
    uint32_t iterations_rendered;
    int32_t ext_wg;              /* chosen workgroup size of the extension launches */
    int32_t queue_chunk;         /* chosen chains per take from stage A's work queue */
    int32_t bvh_width;           /* BVH width the walks use from now on (4 or 8) */
    int32_t stage_a_ahead;       /* chosen look-ahead of the one-wavefront stage (1 or 2 steps) */
    int32_t stage_a_refill;      /* 1: that stage refills its walks node by node (4-wide trees) */
} pt_tune_result;
pt_status pt_autotune(pt_scene *s, const pt_iter_params *p, float *accum_rgb_dev, float *accum_sq_dev,
                      pt_tune_result *out, void *hip_stream);

/* Set the schedule knobs pt_autotune chooses (the fields of pt_tune_result other than the
 * timings and iteration count), e.g. to reuse one tuning on scenes of the same kind or to fix a
 * schedule. Every schedule gives the same estimator. PT_EINVAL for a value out of range,
 * PT_EUNSUPPORTED for a BVH width the scene holds no tree of. Advances the scene's state
 * generation (a captured graph is re-captured). */
pt_status pt_set_schedule(pt_scene *s, const pt_tune_result *knobs);
/* The scene's current schedule knobs (timings and iteration count zero). */
pt_status pt_get_schedule(const pt_scene *s, pt_tune_result *knobs);

/* Learned proposal of the proxy strategy (PT_FLAG_MLP, PT_FLAG_MLP_DIR). Not part of the paper's
 * method: it replaces the Gamma row of Section 5.6 by a network's softmax mixed with that row
 * and, with PT_FLAG_MLP_DIR, proposes the first retrace direction at a glossy y_{s-1} (Section 5.1's
 * retrace samples the BSDF there) by an 8-lobe von Mises-Fisher mixture mixed with the BSDF. Every
 * selection probability and direction density is exact, so the proxy estimator stays unbiased.
 *
 * Network: input = 9 features of a vertex (position scaled to the scene's bounding box in [0, 1],
 * shading normal, unit direction toward the eye side's previous vertex), each encoded as
 * [raw, sin(2^b pi f), cos(2^b pi f) for b = 0..11] (225 values) and zero-padded to 256; three hidden
 * layers of 64 ReLU units; n_out = n_spec + 40 outputs: one logit per specular subspace, then per
 * lobe k = 0..7 the raw mean direction (3, normalised; +z when it vanishes), the log concentration
 * (clamped to [-3, 10]) and the lobe's mixture logit. Lobe density (solid angle):
 * kappa / (2 pi (1 - exp(-2 kappa))) exp(-kappa (1 - mu.w)). BF16 operands with FP32 accumulation.
 * Parameter vector (FP32, this order, row-major with the input index first): W1[256][64], b1[64],
 * W2[64][64], b2[64], W3[64][64], b3[64], W4[64][n_out], b4[n_out]; outputs = h3 W4 + b4. The logits
 * are queried at the eye's first diffuse vertex, the mixture at the chosen y_{s-1} (direction toward
 * z_d). The network is re-initialised by pt_build_subspaces (and on first use); the parameters live
 * with the scene. */
pt_status pt_mlp_param_count(const pt_scene *s, int32_t *count);   /* after pt_build_subspaces */
/* host_params[count] -> the scene's network; clears the Adam moments and step count. Synchronous. */
pt_status pt_mlp_set_params(pt_scene *s, const float *host_params, int32_t count, void *hip_stream);
/* the scene's network -> host_params[count]. Synchronous. */
pt_status pt_mlp_get_params(pt_scene *s, float *host_params, int32_t count, void *hip_stream);
/* out_dev[n][n_spec + 40] (bias included) of feat_dev[n][9] (device, FP32). 1 <= n <= 131072. */
pt_status pt_mlp_forward(pt_scene *s, const float *feat_dev, int32_t n, float *out_dev, void *hip_stream);
/* One training step on a batch of n subspace samples (device arrays feat[n][9], label[n] in
 * [0, n_spec), weight[n] >= 0) and n_dir direction samples (feat_dir[n_dir][9], unit dir[n_dir][3],
 * weight_dir[n_dir] >= 0): loss = sum_i w_i CE(softmax(logits_i), label_i) / sum_i w_i
 * - sum_j v_j log p_mix(dir_j | outputs_j) / sum_j v_j (either part absent when its count is 0);
 * the gradient is copied to grad_host[count] when it is not NULL, then one Adam step (b1 0.9,
 * b2 0.999, eps 1e-8, step size lr) is applied. Synchronous. 0 <= n, n_dir <= 65536, n + n_dir >= 1. */
pt_status pt_mlp_train_step(pt_scene *s, const float *feat_dev, const int32_t *label_dev, const float *weight_dev,
                            int32_t n, const float *feat_dir_dev, const float *dir_dev, const float *weight_dir_dev,
                            int32_t n_dir, float lr, float *grad_host, void *hip_stream);
/* Test hook: one direction from each of n vMF mixtures raw_dev[n][40] (the direction head's 40 outputs,
 * bias included) by the sampler of the proxy retrace, with the mixture density it is weighted by:
 * dir_dev[n][3], pdf_dev[n] (device). No scene needed. */
pt_status pt_vmf_sample(const float *raw_dev, int32_t n, uint32_t seed, float *dir_dev, float *pdf_dev,
                        void *hip_stream);

/* Reciprocal estimator (Section 4.2, RRS estimator with r = |g|, Appendix A). */
enum { PT_RECIP_TABLE = 0, PT_RECIP_CANDIDATE = 1 };
/* One incomplete light sub-path (Section 5.2): the kept specular vertex y_{s-1} and, for
 * class B, the control vertex y_0 on an emitter. Triangle indices are input indices. */
typedef struct {
    int32_t cls;             /* 0: class A (L S^u), 1: class B (L D S^u) */
    int32_t u;               /* 1 .. 4 */
    float v[3];              /* y_{s-1} */
    int32_t v_prim;
    float hc[3];             /* y_0 (class B) */
    int32_t hc_prim;         /* -1 for class A */
    float hc_b1, hc_b2;      /* barycentrics of y_0 on hc_prim (emission texture lookup) */
} pt_cand_desc;
/* PT_EST_BOOTH: Booth's Russian roulette (the comparison of Section 4.2 and the RR ablation of
 * Section 6): one chain without splitting that, after a prefix of j samples, goes on with
 * probability min(1, prod_{i<j} |1 - f/(Bq)| / booth_r). */
enum { PT_EST_ITILDE = 0, PT_EST_SIGN = 1, PT_EST_BOOTH = 2 };
typedef struct {
    int32_t mode;            /* PT_RECIP_TABLE */
    int32_t n;               /* table size */
    const float *f_dev;      /* [n] target f(x) >= 0 */
    const float *q_dev;      /* [n] supporting pmf q(x) > 0 where f > 0 (sums to 1) */
    float B;                 /* the constant B > 0 (B >= max f/q: no splitting) */
    int32_t n_est;           /* independent estimates of 1 / sum f */
    int32_t estimator;       /* PT_EST_ITILDE, PT_EST_SIGN or PT_EST_BOOTH */
    uint32_t seed;
    uint32_t cap;            /* sample cap per estimate (0: 65536); hitting it marks the count */
    /* PT_RECIP_CANDIDATE only (s required): the incomplete sub-path, in host memory; per =
     * samples of f/q averaged into each plain Monte Carlo estimate of P written to out_p_dev[n_est]
     * (device, may be NULL). f/q follows the supporting distribution of Section 5.3. */
    const pt_cand_desc *cand;
    int32_t per;
    float *out_p_dev;
    float booth_r;           /* PT_EST_BOOTH: the roulette's parameter (> 0) */
} pt_recip_query;
/* Writes out_est_dev[n_est] (float: estimates of 1 / sum f, or of 1 / P for a candidate) and
 * out_nsamples_dev[n_est] (samples used; bit 31 set when the cap truncated that estimate).
 * s may be NULL for PT_RECIP_TABLE. */
pt_status pt_reciprocal_estimate(pt_scene *s, const pt_recip_query *q, float *out_est_dev,
                                 uint32_t *out_nsamples_dev, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): pt_reciprocal_estimate in PT_RECIP_TABLE mode, with the same
 * arguments, kernels and results (bit for bit, for the same query), that allocates nothing. The
 * cumulative sums of q go to a fixed device array of PT_NOALLOC_TABLE_MAX + 1 doubles (8 MiB, one
 * per device, held until the process ends) instead of a per-call workspace. Tables longer than
 * PT_NOALLOC_TABLE_MAX entries and any other mode return PT_EINVAL. Every call on a device shares
 * that device's array: calls that overlap on one device (on different streams, or from different
 * threads without ordering) race and give wrong estimates; calls ordered on one stream do not.
 * No scene is needed. */
#define PT_NOALLOC_TABLE_MAX (1 << 20)
pt_status pt_reciprocal_estimate_noalloc(const pt_recip_query *q, float *out_est_dev, uint32_t *out_nsamples_dev,
                                         void *hip_stream);

/* Image = accum / n_iter: the per-pixel estimate of I_j (Section 3.1) as the mean of n_iter
 * iterations of one sample per pixel each (Section 6.1), written to the caller-owned
 * out_rgb_dev[H*W*3] (row-major, 3 floats per pixel, the layout of accum_rgb_dev). accum_rgb_dev
 * and out_rgb_dev may be the same buffer. PT_EINVAL for a NULL buffer or n_iter = 0. */
pt_status pt_resolve_image(pt_scene *s, const float *accum_rgb_dev, uint32_t n_iter, float *out_rgb_dev,
                           void *hip_stream);

/* Test hook: closest-hit queries against the scene's BVH. rays_dev[n*8] = origin, direction,
 * tmin, tmax (float); writes t_dev[n] (-1 on a miss) and prim_dev[n] (input triangle index or
 * -1). Ties in t go to the lower input triangle index. */
pt_status pt_trace_closest(pt_scene *s, const float *rays_dev, int32_t n, float *t_dev, int32_t *prim_dev,
                           void *hip_stream);

/* Running totals over every iteration the scene has rendered (pt_render_iteration, pt_render_batch,
 * pt_render_scenes, pt_autotune), kept on the device and read here (synchronises hip_stream);
 * reset != 0 clears them afterwards. The parity runs require n_nan = n_recip_truncated = 0 over
 * all their iterations. captures counts the HIP graphs pt_render_batch and pt_render_scenes have
 * captured for this scene; bvh_stack_need and bvh_depth describe the uploaded tree. */
typedef struct {
    double iterations, n_nan, n_recip_truncated, n_proxy_valid, n_recip_samples, n_cand;
    double captures, bvh_stack_need, bvh_depth;
} pt_totals;
pt_status pt_scene_totals(pt_scene *s, pt_totals *out, int32_t reset, void *hip_stream);

/* Per-iteration latency from the device's wall clock: the time from the first to the last kernel of
 * iterations first .. first + n - 1 (of any render call), in ms, to ms_host[n]; -1 for an iteration
 * whose record is not there (not rendered yet, still running, or more than PT_TS_CAP = 4096
 * iterations ago). n <= 4096. Synchronises hip_stream. */
pt_status pt_iteration_times(pt_scene *s, uint32_t first, int32_t n, double *ms_host, void *hip_stream);

/* Test hook: the selection tables of the latest iteration (Section 5.6's Gamma rows for which = 0,
 * the light-subspace rows Q of the probabilistic connections for which = 1), copied to host memory
 * (synchronises hip_stream). n_rows x n_cols must be the table's shape (eye subspaces x specular,
 * or light, subspaces). Writes *n_nonempty (columns non-empty this iteration), nonempty[n_cols]
 * (their subspace ids, the first *n_nonempty valid), and per row T: prob[T*n_cols + j] and
 * alias[T*n_cols + j] (the Walker alias row over column positions j < *n_nonempty),
 * pmf[T*n_cols + S] (the probability the row realises for subspace S, which the estimators divide
 * by; valid for non-empty S) and weights[T*n_cols + S] (the frozen learned weights the row was
 * built from). */
pt_status pt_selection_tables(pt_scene *s, int32_t which, int32_t n_rows, int32_t n_cols, int32_t *n_nonempty,
                              int32_t *nonempty, float *prob, int32_t *alias, float *pmf, float *weights,
                              void *hip_stream);

/* Test hook: Philox4x32-10 (Salmon et al. 2011), the counter-based generator every random decision
 * of the kernels draws from, on n rows of in_dev[6 n] = (counter 0..3, key 0..1) -> out_dev[4 n].
 * Device buffers. */
pt_status pt_philox(const uint32_t *in_dev, int32_t n, uint32_t *out_dev, void *hip_stream);

/* Host only (no device needed): builds the BVH of the given width (4 or 8) that pt_scene_upload
 * would build for tri[n_tri*9] and reports its node count, the worst-case traversal stack it
 * needs and its depth in levels. */
pt_status pt_bvh_stats(const float *tri, int32_t n_tri, int32_t width, int32_t *n_nodes, int32_t *stack_need,
                       int32_t *depth);

/* Host only (no device needed): the proxy-class test every strategy of the kernels applies to a
 * path under the partition (classes A and B of Section 5.1 within Section 6.1's limits, and class C
 * of Section 5.2 with general_cv), for tests of that partition. The path runs camera -> z_1 .. z_n
 * -> y_j .. y_1 -> the emitter y_0: eye[i] (i < n_eye) holds z_{i+1}'s flags (bit 0 specular, bit 1
 * Lambertian), light_sig a light sub-path signature (bit i: y_i specular, i < 16; bit 16 + i: y_i
 * Lambertian, i < 8) whose vertices y_j .. y_1 (0 <= j <= 15) are joined; 1 <= u_max <= 4. *out = 1
 * when the path belongs to the proxy class. */
pt_status pt_proxy_class(const uint8_t *eye, int32_t n_eye, uint32_t light_sig, int32_t j, int32_t u_max,
                         int32_t general_cv, int32_t *out);

/* ---------------------------------------------------------------------------------------------
 * Photon planes (Section 6.7): reciprocal estimation as the CMIS weight of a continuous technique
 * space. Single scattering in a homogeneous medium (isotropic phase function, filling space,
 * nothing occluding) lit by one rectangular Lambertian light, rendered with photon planes: a point
 * uniform on the light, a chord angle alpha uniform in [0, pi) (the light's chord through that
 * point) and a cosine-distributed direction w span a plane; each pixel's centre ray gathers every
 * plane it meets. alpha is the technique: the balance-heuristic weight over [0, pi) needs
 * 1 / int p(alpha, xbar) dalpha, which one chain of the RRS estimator (Section 4.2, r = |g|)
 * estimates without bias, with the supporting density q(alpha | xbar) read from a cached
 * piecewise approximation of q* ~ p(., xbar) indexed by the light point and the angle that the
 * eye and plane directions fix (4 MB, built at creation). */
#define PT_PLANES_MAX (1 << 22)
typedef struct pt_planes pt_planes;
typedef struct {
    float light_c[3];        /* light centre */
    float light_u[3], light_v[3];   /* orthonormal axes; the light emits toward u x v */
    float light_eu, light_ev;       /* half extents along u and v */
    float le[3];             /* emitted radiance */
    float camera[10];        /* position, target, up, vertical fov (degrees) */
    float sigma_s, sigma_t;  /* scattering and extinction coefficients */
    float t_max;             /* eye rays end at this distance */
    int32_t width, height;
    int32_t max_planes;      /* largest n_planes of a render call (<= PT_PLANES_MAX) */
} pt_planes_desc;
typedef struct {
    double n_hits;           /* ray-plane hits of the call */
    double n_samples;        /* f/q samples of their reciprocal chains */
    double n_truncated;      /* chains cut at 4,096 samples (their estimates are biased) */
    double n_nan;            /* pixels whose value was not finite (not accumulated) */
} pt_planes_stats;
/* Validates the description (PT_EINVAL), allocates the device buffers (PT_ENOMEM) and builds the
 * q* cache on hip_stream (synchronised). */
pt_status pt_planes_create(const pt_planes_desc *desc, void *hip_stream, pt_planes **out);
/* One iteration: n_planes planes (0 <= n_planes <= max_planes) keyed by (seed, iteration); adds
 * each pixel's value (the mean over the planes of the hits' estimates, RGB) to accum_rgb_dev
 * [width*height*3] and its square to accum_sq_dev (may be NULL). Device buffers, row-major pixels.
 * Kernel launches only, unless stats is non-NULL (then it synchronises and fills *stats). Calls on
 * one object share its plane buffer and counters: issue them on one stream (or order them). */
pt_status pt_planes_render(pt_planes *p, int32_t n_planes, uint32_t iteration, uint32_t seed, float *accum_rgb_dev,
                           float *accum_sq_dev, pt_planes_stats *stats, void *hip_stream);
/* Frees the object (synchronises the device). NULL is a no-op. */
pt_status pt_planes_release(pt_planes *p);

/* Message for the last non-OK return on this thread ("" if none). */
const char *pt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
