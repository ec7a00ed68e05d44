// C ABI of libpt.so (declared in include/pt.h): scene upload, subspace construction, one
// rendering iteration, the reciprocal estimator and image resolve.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pt.h"
#include "pt_kernels.h"

void pt_build_bvh4(const float *tri, int n, std::vector<BNode> &nodes, std::vector<int> &order);

namespace {

thread_local std::string g_err;

pt_status set_err(pt_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(x)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) return set_err(PT_EDEVICE, "%s failed: %s", #x, hipGetErrorString(e_)); \
    } while (0)

inline int blocks(long n, int b) { return (int)((n + b - 1) / b); }

pt_status check_device()
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_err(PT_EUNSUPPORTED, "device %d is %s; this library is built for gfx950 only", dev, prop.gcnArchName);
    return PT_OK;
}

}  // namespace

struct pt_scene {
    int device = 0;
    int W = 0, H = 0, npix = 0, max_light = 0, ntri = 0;
    float scene_diag = 1.0f;
    // geometry
    BNode *nodes = nullptr;
    TriIsect *tris = nullptr;
    TriShade *shade = nullptr;
    MatDev *mats = nullptr;
    float *tex = nullptr;
    int *em_tri = nullptr;
    float *em_cdf = nullptr;
    SceneDev S{};
    // workspaces
    LightBuf L{};
    EyeBuf E{};
    Cand *cand = nullptr;
    uint32_t *kept = nullptr, *final_ = nullptr;
    unsigned long long *cnt = nullptr;
    float *runmax = nullptr;   // [2 * 5] running maxima of f/q per (class, u)
    bool subspaces_ready = false;
    std::vector<int> inv_order;  // input triangle index -> BVH order
    std::vector<hipEvent_t> ev;
    std::vector<void *> allocs;

    template <class T> pt_status alloc(T *&p, size_t n)
    {
        void *q = nullptr;
        if (hipMalloc(&q, n * sizeof(T) + 16) != hipSuccess) {
            (void)hipGetLastError();
            return set_err(PT_ENOMEM, "hipMalloc of %zu bytes failed", n * sizeof(T));
        }
        allocs.push_back(q);
        p = (T *)q;
        return PT_OK;
    }
    ~pt_scene()
    {
        for (void *p : allocs) (void)hipFree(p);
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

#define TRY(x)                          \
    do {                                \
        pt_status st_ = (x);            \
        if (st_ != PT_OK) return st_;   \
    } while (0)

extern "C" const char *pt_last_error(void) { return g_err.c_str(); }

extern "C" pt_status pt_scene_upload(const pt_scene_desc *d, void *stream_, pt_scene **out)
{
    try {
        if (!d || !out) return set_err(PT_EINVAL, "null argument");
        *out = nullptr;
        if (d->n_tri <= 0 || !d->tri || !d->tri_mat || !d->tri_uv || d->n_mat <= 0 || !d->mats || !d->camera)
            return set_err(PT_EINVAL, "missing geometry, materials or camera");
        if (d->width <= 0 || d->height <= 0 || (long)d->width * d->height > (1L << 26))
            return set_err(PT_EINVAL, "bad image size %d x %d", d->width, d->height);
        if (d->tex_w <= 0 || d->tex_h <= 0 || !d->tex) return set_err(PT_EINVAL, "missing emission texture");
        if (d->max_light_paths <= 0 || d->max_light_paths > (1 << 24))
            return set_err(PT_EINVAL, "max_light_paths out of range");
        if (d->bvh_width != 4 && d->bvh_width != 0) return set_err(PT_EINVAL, "only 4-wide BVH nodes are built");
        for (int i = 0; i < d->n_tri; ++i)
            if (d->tri_mat[i] < 0 || d->tri_mat[i] >= d->n_mat) return set_err(PT_EINVAL, "triangle %d: bad material", i);
        for (int m = 0; m < d->n_mat; ++m) {
            const int t = (int)d->mats[16 * m];
            if (t < 0 || t > 2) return set_err(PT_EINVAL, "material %d: bad type", m);
        }
        TRY(check_device());
        hipStream_t stream = (hipStream_t)stream_;
        pt_scene *s = new pt_scene();
        HIPCHK(hipGetDevice(&s->device));
        s->W = d->width; s->H = d->height; s->npix = d->width * d->height; s->max_light = d->max_light_paths;
        s->ntri = d->n_tri;
        // BVH
        std::vector<BNode> nodes;
        std::vector<int> order;
        pt_build_bvh4(d->tri, d->n_tri, nodes, order);
        s->inv_order.assign(d->n_tri, 0);
        for (int i = 0; i < d->n_tri; ++i) s->inv_order[order[i]] = i;
        std::vector<TriIsect> ti(d->n_tri);
        std::vector<TriShade> ts(d->n_tri);
        float lo[3] = {1e30f, 1e30f, 1e30f}, hi[3] = {-1e30f, -1e30f, -1e30f};
        std::vector<int> em;
        std::vector<float> emc;
        double area_acc = 0.0;
        std::vector<MatDev> mats(d->n_mat);
        for (int m = 0; m < d->n_mat; ++m) {
            const float *r = d->mats + 16 * m;
            MatDev &md = mats[m];
            md.type = (int)r[0];
            md.rgb = make_float3(r[1], r[2], r[3]);
            md.alpha = std::max(r[4] * r[4], 1e-4f);
            md.ior = r[5];
            md.le = make_float3(r[6], r[7], r[8]);
            md.flags = 0;
            if (r[6] > 0 || r[7] > 0 || r[8] > 0) md.flags |= MF_EMIT;
            if (r[9] != 0.0f) md.flags |= MF_TEXTURED;
            if ((md.type == MAT_CONDUCTOR || md.type == MAT_DIELECTRIC) && r[4] < 0.2f) md.flags |= MF_SPEC;
            if (md.type == MAT_DIELECTRIC || (md.type == MAT_CONDUCTOR && r[4] == 0.0f)) md.flags |= MF_DELTA;
        }
        for (int i = 0; i < d->n_tri; ++i) {
            const int src = order[i];
            const float *p = d->tri + 9 * (size_t)src;
            TriIsect &t = ti[i];
            for (int k = 0; k < 3; ++k) {
                t.v0[k] = p[k]; t.e1[k] = p[3 + k] - p[k]; t.e2[k] = p[6 + k] - p[k];
                for (int v = 0; v < 3; ++v) { lo[k] = std::min(lo[k], p[3 * v + k]); hi[k] = std::max(hi[k], p[3 * v + k]); }
            }
            t.prim = src; t.pad[0] = t.pad[1] = 0;
            // normal and area in double to keep thin triangles' normals exact
            const double e1[3] = {(double)t.e1[0], (double)t.e1[1], (double)t.e1[2]};
            const double e2[3] = {(double)t.e2[0], (double)t.e2[1], (double)t.e2[2]};
            const double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
            const double len = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
            TriShade &sh = ts[i];
            sh.n = len > 0 ? make_float3((float)(c[0] / len), (float)(c[1] / len), (float)(c[2] / len)) : make_float3(0, 0, 1);
            sh.mat = d->tri_mat[src];
            for (int k = 0; k < 6; ++k) sh.uv[k] = d->tri_uv[6 * (size_t)src + k];
            if ((mats[sh.mat].flags & MF_EMIT) && len > 0) {
                area_acc += 0.5 * len;
                em.push_back(i);
                emc.push_back((float)area_acc);
            }
        }
        if (em.empty()) { delete s; return set_err(PT_EINVAL, "scene has no emitter"); }
        for (float &c : emc) c = (float)(c / area_acc);
        emc.back() = 1.0f;
        s->scene_diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                  (hi[2] - lo[2]) * (hi[2] - lo[2]));
        pt_status st;
#define AL(p, n) if ((st = s->alloc(p, n)) != PT_OK) { delete s; return st; }
        AL(s->nodes, nodes.size());
        AL(s->tris, ti.size());
        AL(s->shade, ts.size());
        AL(s->mats, mats.size());
        AL(s->tex, (size_t)d->tex_w * d->tex_h);
        AL(s->em_tri, em.size());
        AL(s->em_cdf, emc.size());
        const int M = s->max_light, np = s->npix;
        AL(s->L.ro, M); AL(s->L.rd, M); AL(s->L.hit, M);
        AL(s->L.lv, (size_t)PT_LMAX * M); AL(s->L.lb0, M); AL(s->L.sig, M);
        AL(s->L.q[0], M); AL(s->L.q[1], M);
        AL(s->cand, (size_t)4 * M);
        AL(s->kept, (size_t)4 * M); AL(s->final_, (size_t)4 * M);
        AL(s->E.ro, np); AL(s->E.rd, np); AL(s->E.hit, np); AL(s->E.beta, np); AL(s->E.info, np);
        AL(s->E.q[0], np); AL(s->E.q[1], np);
        AL(s->E.shadow, np); AL(s->E.proxy, np);
        AL(s->E.frame, (size_t)3 * np);
        AL(s->cnt, C_COUNT);
        AL(s->runmax, 16);
#undef AL
        s->L.M = M;
        s->E.npix = np;
        HIPCHK(hipMemcpyAsync(s->nodes, nodes.data(), nodes.size() * sizeof(BNode), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(s->tris, ti.data(), ti.size() * sizeof(TriIsect), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(s->shade, ts.data(), ts.size() * sizeof(TriShade), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(s->mats, mats.data(), mats.size() * sizeof(MatDev), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(s->tex, d->tex, sizeof(float) * d->tex_w * d->tex_h, hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(s->em_tri, em.data(), em.size() * sizeof(int), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(s->em_cdf, emc.data(), emc.size() * sizeof(float), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemsetAsync(s->E.frame, 0, sizeof(float) * 3 * np, stream));
        HIPCHK(hipMemsetAsync(s->runmax, 0, sizeof(float) * 16, stream));
        HIPCHK(hipStreamSynchronize(stream));
        SceneDev &S = s->S;
        S.nodes = s->nodes; S.tris = s->tris; S.shade = s->shade; S.mats = s->mats; S.tex = s->tex;
        S.tex_w = d->tex_w; S.tex_h = d->tex_h; S.em_tri = s->em_tri; S.em_cdf = s->em_cdf; S.n_em = (int)em.size();
        S.em_area = (float)area_acc;
        S.tmin = 2e-6f * s->scene_diag;
        const float *c = d->camera;
        float3 p = make_float3(c[0], c[1], c[2]), tg = make_float3(c[3], c[4], c[5]), up = make_float3(c[6], c[7], c[8]);
        auto nrm = [](float3 a) { float l = std::sqrt(a.x * a.x + a.y * a.y + a.z * a.z); return make_float3(a.x / l, a.y / l, a.z / l); };
        auto crs = [](float3 a, float3 b) { return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); };
        float3 f = nrm(make_float3(tg.x - p.x, tg.y - p.y, tg.z - p.z));
        float3 r = nrm(crs(f, up));
        S.cam.p = p; S.cam.f = f; S.cam.r = r; S.cam.u = crs(r, f);
        S.cam.tan_half = std::tan(0.5f * c[9] * 3.14159265358979f / 180.0f);
        S.cam.aspect = (float)d->width / (float)d->height;
        S.cam.w = d->width; S.cam.h = d->height;
        *out = s;
        return PT_OK;
    } catch (const std::exception &e) {
        return set_err(PT_ENOMEM, "host exception: %s", e.what());
    } catch (...) {
        return set_err(PT_ENOMEM, "host exception");
    }
}

extern "C" pt_status pt_scene_release(pt_scene *s)
{
    if (!s) return PT_OK;
    (void)hipDeviceSynchronize();
    delete s;
    return PT_OK;
}

extern "C" pt_status pt_build_subspaces(pt_scene *s, const pt_subspace_params *p, void *stream_)
{
    if (!s || !p) return set_err(PT_EINVAL, "null argument");
    if (p->n_eye <= 0 || p->n_eye > 4096 || p->n_spec <= 0 || p->n_spec > 4096 || p->n_pretrace < 0 ||
        p->kmeans_iters < 0)
        return set_err(PT_EINVAL, "subspace parameters out of range");
    hipStream_t stream = (hipStream_t)stream_;
    HIPCHK(hipMemsetAsync(s->runmax, 0, sizeof(float) * 16, stream));
    s->subspaces_ready = true;
    return PT_OK;
}

extern "C" pt_status pt_render_iteration(pt_scene *s, const pt_iter_params *p, float *acc, float *acc2,
                                         pt_iter_stats *stats, void *stream_)
{
    if (!s || !p || !acc) return set_err(PT_EINVAL, "null argument");
    if (!s->subspaces_ready) return set_err(PT_ESTATE, "pt_build_subspaces must run before pt_render_iteration");
    if (p->max_depth < 1 || p->max_depth > PT_MAX_DEPTH) return set_err(PT_EINVAL, "max_depth out of range [1, %d]", PT_MAX_DEPTH);
    if (p->n_light < 1 || p->n_light > s->max_light) return set_err(PT_EINVAL, "n_light out of range [1, %d]", s->max_light);
    if (p->u_max < 1 || p->u_max > 4) return set_err(PT_EINVAL, "u_max out of range [1, 4]");
    if (p->recip_repeats < 1 || p->recip_repeats > 8) return set_err(PT_EINVAL, "recip_repeats out of range [1, 8]");
    if (p->cand_cap < 1 || p->pilot < 1) return set_err(PT_EINVAL, "cand_cap and pilot must be positive");
    if ((p->flags & PT_FLAG_ONLY_PROXY_CLASS) && (p->flags & PT_FLAG_ONLY_OTHER))
        return set_err(PT_EINVAL, "class filters are exclusive");
    hipStream_t stream = (hipStream_t)stream_;
    SceneDev S = s->S;
    LightBuf L = s->L;
    L.M = p->n_light;
    EyeBuf E = s->E;
    const int M = L.M;
    const bool proxy = (p->flags & PT_FLAG_PROXY) != 0;
    const bool count = (p->flags & PT_FLAG_COUNT) != 0;
    const bool timing = (p->flags & PT_FLAG_TIMING) != 0;
    if (timing && s->ev.size() < 2 * (size_t)p->max_depth) {
        while (s->ev.size() < 2 * (size_t)p->max_depth) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            s->ev.push_back(e);
        }
    }
    k_zero<<<blocks(C_COUNT, 256), 256, 0, stream>>>(s->cnt, C_COUNT);
    if (proxy) {
        // light pass: y_0 .. y_{lmax-1}
        const int lmax = std::min(p->max_depth - 1, PT_LMAX);
        k_light_gen<<<blocks(M, 256), 256, 0, stream>>>(S, L, p->seed, p->iteration, s->cnt);
        for (int vi = 1; vi < lmax; ++vi) {
            k_extend<false><<<blocks(M, WG), WG, 0, stream>>>(S, L.q[(vi - 1) & 1], s->cnt, C_LIGHT_Q0 + vi - 1, L.ro,
                                                              L.rd, L.hit, s->cnt, C_RAYS_LIGHT);
            k_light_shade<<<blocks(M, 256), 256, 0, stream>>>(S, L, p->seed, p->iteration, vi, lmax, s->cnt);
        }
        if (lmax >= 2) {
            k_candidates<<<blocks(M, 256), 256, 0, stream>>>(L, p->u_max, s->cand, s->cnt);
            const int maxc = 4 * M;
            k_keep<<<blocks(maxc, 256), 256, 0, stream>>>(p->cand_cap, p->seed, p->iteration, s->kept, maxc, s->cnt);
            k_pilot<<<blocks(maxc, RW), 64 * RW, 0, stream>>>(S, s->cand, s->kept, p->pilot, p->seed, p->iteration,
                                                             s->runmax, s->cnt);
            k_roulette<<<blocks(maxc, 256), 256, 0, stream>>>(s->cand, s->kept, s->final_, s->runmax, S.em_area,
                                                              p->recip_repeats, p->cost_cap, p->seed, p->iteration,
                                                              s->cnt);
            const uint32_t n1 = (uint32_t)std::max(64.0f, p->cost_cap / (float)p->recip_repeats);
            k_recip<<<blocks((long)maxc * p->recip_repeats, RW), 64 * RW, 0, stream>>>(
                S, s->cand, s->final_, p->recip_repeats, p->seed, p->iteration, n1, 1u << 20, s->runmax, s->cnt);
        }
    }
    // eye pass
    EyeParams EP;
    EP.seed = p->seed; EP.iter = p->iteration; EP.K = p->max_depth; EP.u_max = p->u_max;
    EP.filter = (p->flags & PT_FLAG_ONLY_PROXY_CLASS) ? (proxy ? 3 : 1) : (proxy ? 2 : ((p->flags & PT_FLAG_ONLY_OTHER) ? 2 : 0));
    EP.proxy_on = proxy && !(p->flags & PT_FLAG_ONLY_OTHER);
    EP.nee_on = (p->flags & PT_FLAG_NEE) != 0;
    const int np = s->npix;
    k_camera<<<blocks(np, 256), 256, 0, stream>>>(S, E, p->seed, p->iteration, s->cnt);
    for (int t = 1; t <= p->max_depth; ++t) {
        if (timing) HIPCHK(hipEventRecord(s->ev[2 * (t - 1)], stream));
        if (count)
            k_extend<true><<<blocks(np, WG), WG, 0, stream>>>(S, E.q[(t - 1) & 1], s->cnt, C_EYE_Q0 + t - 1, E.ro, E.rd,
                                                              E.hit, s->cnt, C_RAYS_EYE);
        else
            k_extend<false><<<blocks(np, WG), WG, 0, stream>>>(S, E.q[(t - 1) & 1], s->cnt, C_EYE_Q0 + t - 1, E.ro, E.rd,
                                                               E.hit, s->cnt, C_RAYS_EYE);
        if (timing) HIPCHK(hipEventRecord(s->ev[2 * (t - 1) + 1], stream));
        k_eye_shade<<<blocks(np, 256), 256, 0, stream>>>(S, E, EP, t, s->cnt);
        k_occluded<<<blocks(np, WG), WG, 0, stream>>>(S, E, t, s->cnt);
    }
    if (EP.proxy_on) {
        ProxyParams PP;
        PP.seed = p->seed; PP.iter = p->iteration; PP.K = p->max_depth; PP.M = M; PP.cand_cap = p->cand_cap;
        PP.repeats = p->recip_repeats;
        k_proxy<<<blocks(np, WG), WG, 0, stream>>>(S, E, s->cand, s->final_, PP, s->cnt);
    }
    k_accumulate<<<blocks(3L * np, 256), 256, 0, stream>>>(E.frame, acc, acc2, 3 * np, s->cnt);
    HIPCHK(hipGetLastError());
    if (stats) {
        unsigned long long c[C_COUNT];
        HIPCHK(hipMemcpyAsync(c, s->cnt, sizeof(c), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        std::memset(stats, 0, sizeof(*stats));
        stats->rays_extend_eye = (double)c[C_RAYS_EYE];
        stats->rays_extend_light = (double)c[C_RAYS_LIGHT];
        stats->rays_shadow = (double)c[C_RAYS_SHADOW];
        stats->rays_proxy = (double)c[C_RAYS_PROXY];
        stats->rays_recip = (double)c[C_RAYS_RECIP];
        stats->n_cand = (double)c[C_NCAND];
        stats->n_kept = (double)c[C_NFINAL];
        stats->n_recip_samples = (double)c[C_RECIP_SAMPLES];
        stats->n_recip_truncated = (double)c[C_RECIP_TRUNC];
        stats->n_proxy_attempts = (double)c[C_PROXY_ATT];
        stats->n_proxy_valid = (double)c[C_PROXY_VALID];
        stats->n_nan = (double)c[C_NAN];
        stats->node_visits = (double)c[C_VISITS];
        stats->tri_tests = (double)c[C_TESTS];
        if (timing) {
            double ms = 0.0;
            for (int t = 0; t < p->max_depth; ++t) {
                float e = 0.0f;
                HIPCHK(hipEventElapsedTime(&e, s->ev[2 * t], s->ev[2 * t + 1]));
                ms += e;
            }
            stats->ms_extend = ms;
            stats->n_extend_launches = p->max_depth;
        }
    }
    return PT_OK;
}

extern "C" pt_status pt_reciprocal_estimate(pt_scene *s, const pt_recip_query *q, float *out, uint32_t *ns,
                                            void *stream_)
{
    if (!q || !out || !ns) return set_err(PT_EINVAL, "null argument");
    if (q->n_est <= 0 || !(q->B > 0.0f)) return set_err(PT_EINVAL, "n_est and B must be positive");
    hipStream_t stream = (hipStream_t)stream_;
    const uint32_t cap = q->cap ? q->cap : 65536u;
    if (q->mode == PT_RECIP_TABLE) {
        if (q->n <= 0 || !q->f_dev || !q->q_dev) return set_err(PT_EINVAL, "bad table query");
        if (q->estimator != PT_EST_ITILDE && q->estimator != PT_EST_SIGN) return set_err(PT_EINVAL, "unknown estimator");
        if (!s) TRY(check_device());
        k_recip_table<<<blocks(q->n_est, 256), 256, 0, stream>>>(q->f_dev, q->q_dev, q->n, q->B, q->n_est,
                                                                 q->estimator, q->seed, cap, out, ns);
    } else if (q->mode == PT_RECIP_CANDIDATE) {
        const pt_cand_desc *d = q->cand;
        if (!s || !d) return set_err(PT_EINVAL, "candidate mode needs a scene and a candidate");
        if (d->cls < 0 || d->cls > 1 || d->u < 1 || d->u > 4 || q->per < 1) return set_err(PT_EINVAL, "bad candidate");
        if (d->v_prim < 0 || d->v_prim >= s->ntri || (d->cls == 1 && (d->hc_prim < 0 || d->hc_prim >= s->ntri)))
            return set_err(PT_EINVAL, "candidate triangle out of range");
        Cand c;
        std::memset(&c, 0, sizeof(c));
        auto as_f = [](int i) { float f; std::memcpy(&f, &i, sizeof(f)); return f; };
        c.v = make_float4(d->v[0], d->v[1], d->v[2], as_f(s->inv_order[d->v_prim]));
        const int hct = d->cls == 1 ? s->inv_order[d->hc_prim] : 0;
        c.hc = make_float4(d->hc[0], d->hc[1], d->hc[2], as_f(hct));
        c.hc_b1 = d->hc_b1; c.hc_b2 = d->hc_b2;
        c.cls_u = (d->cls << 8) | d->u;
        c.B = q->B; c.rho = 1.0f;
        k_recip_point<<<blocks(q->n_est, RW), 64 * RW, 0, stream>>>(s->S, c, q->n_est, q->per, q->seed, cap, out, ns,
                                                                   q->out_p_dev);
    } else {
        return set_err(PT_EINVAL, "unknown mode %d", q->mode);
    }
    HIPCHK(hipGetLastError());
    return PT_OK;
}

extern "C" pt_status pt_resolve_image(pt_scene *s, const float *acc, uint32_t n_iter, float *out, void *stream_)
{
    if (!s || !acc || !out || n_iter == 0) return set_err(PT_EINVAL, "bad argument");
    hipStream_t stream = (hipStream_t)stream_;
    k_resolve<<<blocks(3L * s->npix, 256), 256, 0, stream>>>(acc, out, 3 * s->npix, 1.0f / (float)n_iter);
    HIPCHK(hipGetLastError());
    return PT_OK;
}

extern "C" pt_status pt_trace_closest(pt_scene *s, const float *rays, int32_t n, float *t, int32_t *prim, void *stream_)
{
    if (!s || !rays || !t || !prim || n < 0) return set_err(PT_EINVAL, "bad argument");
    if (n == 0) return PT_OK;
    hipStream_t stream = (hipStream_t)stream_;
    k_trace_closest<<<blocks(n, WG), WG, 0, stream>>>(s->S, rays, n, t, prim);
    HIPCHK(hipGetLastError());
    return PT_OK;
}
