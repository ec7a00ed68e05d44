// C ABI of libpt.so (declared in include/pt.h): scene upload, subspace construction, one
// rendering iteration, the reciprocal estimator and image resolve.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pt.h"
#include "pt_kernels.h"
#include "pt_planes.h"

void pt_build_bvh(const float *tri, int n, std::vector<BNode> &nodes, std::vector<BNode8> *nodes8,
                  std::vector<int> &order);
int pt_bvh4_stack_need(const std::vector<BNode> &nodes, int *depth);
int pt_bvh8_stack_need(const std::vector<BNode8> &nodes, int *depth);

namespace {

thread_local std::string g_err;
// state generations: every change of a scene's device buffers or schedule takes the next value,
// unique over the process, so that a captured graph is never replayed on a scene (or a scene
// uploaded at the same host address) it was not captured for
std::atomic<unsigned long long> g_generation{0};
unsigned long long next_generation() { return ++g_generation; }

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

#ifndef PT_PERSIST_PER_CU
#define PT_PERSIST_PER_CU 4   // workgroups per CU of the persistent pilot and stage-A grids
#endif

// launch a traversal kernel with the scene's stack entry type: 16-bit for trees below 65,536
// nodes, and a type of the same size that walks the 8-wide tree when the scene uses it
// (uint16_t / int: 4-wide; int16_t / uint32_t: 8-wide)
#define PT_STK(sc, kern, grid, block, strm, ...)                                                \
    do {                                                                                        \
        if ((sc)->bvh_cur == 8) {                                                               \
            if ((sc)->stk16) kern<int16_t><<<(grid), (block), 0, (strm)>>>(__VA_ARGS__);        \
            else kern<uint32_t><<<(grid), (block), 0, (strm)>>>(__VA_ARGS__);                   \
        } else {                                                                                \
            if ((sc)->stk16) kern<uint16_t><<<(grid), (block), 0, (strm)>>>(__VA_ARGS__);       \
            else kern<int><<<(grid), (block), 0, (strm)>>>(__VA_ARGS__);                        \
        }                                                                                       \
    } while (0)
// extension launches over n rays with the scene's tuned workgroup size (64, 128 or 256)
#define PT_EXT_WG(sc, counting, SEt, WGv, n, strm, ...)                                                        \
    do {                                                                                                     \
        if (counting) k_extend<true, SEt, WGv><<<blocks((n), WGv), WGv, 0, (strm)>>>(__VA_ARGS__);           \
        else k_extend<false, SEt, WGv><<<blocks((n), WGv), WGv, 0, (strm)>>>(__VA_ARGS__);                   \
    } while (0)
#define PT_EXT_SE(sc, counting, SEt, n, strm, ...)                                                           \
    do {                                                                                                     \
        if ((sc)->ext_wg == 64) PT_EXT_WG(sc, counting, SEt, 64, n, strm, __VA_ARGS__);                      \
        else if ((sc)->ext_wg == 256) PT_EXT_WG(sc, counting, SEt, 256, n, strm, __VA_ARGS__);               \
        else PT_EXT_WG(sc, counting, SEt, 128, n, strm, __VA_ARGS__);                                        \
    } while (0)
#define PT_STK_EXT(sc, counting, n, strm, ...)                                                              \
    do {                                                                                                     \
        if ((sc)->bvh_cur == 8) {                                                                            \
            if ((sc)->stk16) PT_EXT_SE(sc, counting, int16_t, n, strm, __VA_ARGS__);                         \
            else PT_EXT_SE(sc, counting, uint32_t, n, strm, __VA_ARGS__);                                    \
        } else {                                                                                             \
            if ((sc)->stk16) PT_EXT_SE(sc, counting, uint16_t, n, strm, __VA_ARGS__);                        \
            else PT_EXT_SE(sc, counting, int, n, strm, __VA_ARGS__);                                         \
        }                                                                                                    \
    } while (0)
// PT_STK for kernels with a second (bool) template argument
#define PT_STK_B(sc, kern, B, grid, block, strm, ...)                                           \
    do {                                                                                        \
        if ((sc)->bvh_cur == 8) {                                                               \
            if ((sc)->stk16) kern<int16_t, B><<<(grid), (block), 0, (strm)>>>(__VA_ARGS__);     \
            else kern<uint32_t, B><<<(grid), (block), 0, (strm)>>>(__VA_ARGS__);                \
        } else {                                                                                \
            if ((sc)->stk16) kern<uint16_t, B><<<(grid), (block), 0, (strm)>>>(__VA_ARGS__);    \
            else kern<int, B><<<(grid), (block), 0, (strm)>>>(__VA_ARGS__);                     \
        }                                                                                       \
    } while (0)
// the stack entry choice of a multi-scene launch (PT_STK_B reads these two fields)
struct MultiStk {
    bool stk16;
    int bvh_cur;
};
// stage A with Booth's roulette: its own instances (template argument BOOTH)
template <typename SE>
static void launch_recip_booth(int grid, hipStream_t st, SceneDev S, Cand *cand, const uint32_t *final_,
                               const uint32_t *order, int repeats, uint32_t seed, uint32_t n1, uint32_t budget,
                               float *runmax, ChainState *longq, float booth_r, unsigned long long *cnt, int chunk,
                               int ahead)
{
    k_recip<SE, true><<<grid, 64 * RW, 0, st>>>(S, cand, final_, order, repeats, seed, n1, budget, runmax, longq,
                                                booth_r, cnt, chunk, ahead);
}

// alias rows of a T x n table over its non-empty columns: one wavefront per row when the row
// fits LDS, else one thread per row
static void alias_rows(const float *tab, int ne, int n, const int *nonempty, const int *n_nonempty, float defensive,
                       float *al_prob, int *al_idx, float *row_sum, float *pmf, int *scratch, hipStream_t st)
{
    if (n <= ALIAS_LDS_COLS)
        k_alias_rows_wave<<<ne, 64, (size_t)16 * n, st>>>(tab, ne, n, nonempty, n_nonempty, defensive, al_prob, al_idx,
                                                          row_sum, pmf);
    else
        k_alias_rows<<<blocks(ne, 64), 64, 0, st>>>(tab, ne, n, nonempty, n_nonempty, defensive, al_prob, al_idx, row_sum,
                                                   pmf, scratch);
}

struct pt_scene {
    int device = 0;
    unsigned long long gen = 0;   // state generation (next_generation)
    int stack_need = 0, bvh_depth = 0;
    int W = 0, H = 0, npix = 0, max_light = 0, ntri = 0;
    float scene_diag = 1.0f;
    // geometry
    BNode *nodes = nullptr;
    BNode8 *nodes8 = nullptr;   // the 8-wide tree (uploaded when bvh_width is 0 or 8 and its walk fits)
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
    uint32_t *cost_bin = nullptr, *order = nullptr;   // chain scheduling (longest expected first)
    unsigned long long *cnt = nullptr;
    unsigned long long *tot = nullptr;   // [TOT_COUNT] running totals over iterations (k_totals)
    long long *ts = nullptr;             // [2 PT_TS_CAP] wall-clock start / end of the latest iterations
    int wall_khz = 0;                    // device wall-clock rate
    float *runmax = nullptr;   // [16]: running maxima of f/q per (class, u), PT_STAT_CU used
    // subspace-based connections: light subspaces, buckets of the pool, Q (learned, frozen), alias rows
    int n_lsub = 0;
    float *light_c = nullptr, *qacc = nullptr, *qfrz = nullptr, *q_alprob = nullptr, *q_alpmf = nullptr, *q_rowsum = nullptr,
          *q_rowtot = nullptr, *lne_prev = nullptr;
    int *lcount = nullptr, *loff = nullptr, *lfill = nullptr, *lnonempty = nullptr, *ln_ne = nullptr, *llist = nullptr,
        *plab = nullptr, *prank = nullptr, *q_alidx = nullptr, *q_scratch = nullptr, *lcount_prev = nullptr;
    ChainState *chq[2] = {nullptr, nullptr};   // running reciprocal chains between rounds
    float2 *chbuf = nullptr;                   // (f/q, u) samples of one round
    bool subspaces_ready = false;
    // subspaces, selection and statistics (allocated by pt_build_subspaces)
    int n_eye = 0, n_spec = 0, tile = 10, tiles_x = 0, n_tiles = 0, km_cap = 0;
    float *eye_c = nullptr, *spec_c = nullptr, *km_sum = nullptr, *km_cnt = nullptr, *feat = nullptr;
    int *s_count = nullptr, *s_off = nullptr, *s_fill = nullptr, *s_list = nullptr, *nonempty = nullptr, *n_ne = nullptr;
    float *al_prob = nullptr, *al_pmf = nullptr, *row_sum = nullptr, *gamma_acc = nullptr, *gamma_frz = nullptr;
    int *al_idx = nullptr, *al_scratch = nullptr;
    float *rstat_acc = nullptr, *rstat_frz = nullptr, *tile_proxy = nullptr, *tile_total = nullptr;
    // control subspaces (Section 5.5) and the bucket maxima of f/q by (class, u, S, C)
    int n_ctrl = 1, stat_cap = 0;
    float *ctrl_c = nullptr, *bstat_acc = nullptr, *bstat_frz = nullptr;
    float *prev = nullptr, *row_tot = nullptr;
    int *s_count_prev = nullptr;
    // learned selection: parameters (FP32 master, BF16 copy, gradient, Adam moments) and
    // activations for max(npix, 2 MLP_CAP) rows
    int mlp_nout = 0, mlp_rows = 0, mlp_np = 0;
    bool mlp_ready = false;
    float *mw = nullptr, *mg = nullptr, *mm = nullptr, *mv = nullptr;
    uint16_t *mwt = nullptr;   // transposed BF16 weight matrices (k_mlp_transpose) for the fused forward pass
    uint16_t *mwb = nullptr, *mx = nullptr, *mh[3] = {nullptr, nullptr, nullptr}, *mdz[2] = {nullptr, nullptr},
             *mg4 = nullptr;
    float *mz = nullptr, *ml = nullptr, *mdh = nullptr;
    float *mvmf = nullptr;   // [npix x MLP_VMF] mixture outputs (bias included) of every proxy item's y_{s-1}
    MlpTrain MT{};
    // group searches of the centroid sets (eye T, specular S, light S_L)
    struct GroupSet {
        float *g = nullptr;
        int *start = nullptr, *mem = nullptr;
        int G = 0, K = 0, cap_G = 0, cap_K = 0;
    } gs_eye, gs_spec, gs_light;
    std::vector<int> inv_order;  // input triangle index -> BVH order
    std::vector<hipEvent_t> ev;
    std::vector<void *> allocs;
    // captured iteration graph (pt_render_batch) and the key it was captured for
    hipStream_t cap_stream = nullptr;
    // reciprocal-chain schedule (pt_autotune): stage-A sample budget, blocks of the round kernels
    uint32_t tune_budget = 1024;
    int tune_gen_grid = 8192;
    // workgroups of the persistent pilot and stage-A launches: four per CU
    int persist_wg = 1024;
    // workgroup size of the extension (closest-hit) launches (pt_autotune: 64, 128 or 256)
    int ext_wg = 128;
    int ahead = 2;   // steps a stage-A lane may compute beyond the oldest unconsumed one (1 or 2)
    int refill = 0;  // stage A refills its walks node by node (4-wide trees)
    // the chain kernels keep 16-bit traversal stack entries when the tree has fewer than 65,536 nodes
    bool stk16 = false;
    // BVH widths available to the walks, and the one in use (S.nodes8 set when it is 8)
    bool has4 = false, has8 = false;
    int bvh_cur = 4;
    int stack_need4 = 0, bvh_depth4 = 0, stack_need8 = 0, bvh_depth8 = 0;
    // second stream of an iteration: the eye pass and light tracing run on it beside the
    // reciprocal estimates (default priority), forked and joined with these events
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // multi-scene graph (pt_render_scenes) owned by the first scene of a batch
    hipGraphExec_t mgexec = nullptr;
    std::vector<char> mgkey;
    RecipJob *mjobs = nullptr;           // multi-scene stage A: one job per scene (device)
    uint32_t *mbase = nullptr;           // the scenes' first items, then the total (device)
    unsigned long long *mwork = nullptr; // the shared work counter (device)
    int queue_chunk = 1;                 // chains per take from the multi-scene work queue
    std::vector<hipStream_t> mstreams;
    std::vector<hipEvent_t> mevents;
    hipGraphExec_t gexec = nullptr;
    std::vector<char> gkey;
    unsigned long long n_captures = 0;   // graphs captured by pt_render_batch / pt_render_scenes

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
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (mgexec) (void)hipGraphExecDestroy(mgexec);
        if (mjobs) (void)hipFree(mjobs);
        if (mbase) (void)hipFree(mbase);
        if (mwork) (void)hipFree(mwork);
        for (hipStream_t q : mstreams) (void)hipStreamDestroy(q);
        for (hipEvent_t e : mevents) (void)hipEventDestroy(e);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (side) { (void)hipStreamSynchronize(side); (void)hipStreamDestroy(side); }
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
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
        if (d->bvh_width != 4 && d->bvh_width != 8 && d->bvh_width != 0)
            return set_err(PT_EINVAL, "bvh_width must be 0, 4 or 8");
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
        {
            int ncu = 0;
            HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, s->device));
            s->persist_wg = PT_PERSIST_PER_CU * std::max(ncu, 1);
            HIPCHK(hipDeviceGetAttribute(&s->wall_khz, hipDeviceAttributeWallClockRate, s->device));
            // the second stream of an iteration (default priority) and its fork / join events
            HIPCHK(hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
        }
        s->W = d->width; s->H = d->height; s->npix = d->width * d->height; s->max_light = d->max_light_paths;
        s->ntri = d->n_tri;
        // BVH
        std::vector<BNode> nodes;
        std::vector<BNode8> nodes8;
        std::vector<int> order;
        const bool want8 = d->bvh_width != 4;
        pt_build_bvh(d->tri, d->n_tri, nodes, want8 ? &nodes8 : nullptr, order);
        s->stack_need4 = pt_bvh4_stack_need(nodes, &s->bvh_depth4);
        if (want8) s->stack_need8 = pt_bvh8_stack_need(nodes8, &s->bvh_depth8);
        // a width is available when its worst-case walk fits the kernels' stack
        s->has4 = d->bvh_width != 8 && s->stack_need4 <= PT_STACK;
        s->has8 = want8 && s->stack_need8 <= PT_STACK8;
        if ((d->bvh_width == 4 && !s->has4) || (d->bvh_width == 8 && !s->has8) || (!s->has4 && !s->has8)) {
            const bool w8 = d->bvh_width == 8;
            const int need = w8 ? s->stack_need8 : s->stack_need4;
            delete s;
            return set_err(PT_EUNSUPPORTED, "the %d-wide BVH needs a traversal stack of %d entries; the kernels hold %d",
                           w8 ? 8 : 4, need, w8 ? PT_STACK8 : PT_STACK);
        }
        s->bvh_cur = s->has4 ? 4 : 8;
        s->stack_need = s->bvh_cur == 4 ? s->stack_need4 : s->stack_need8;
        s->bvh_depth = s->bvh_cur == 4 ? s->bvh_depth4 : s->bvh_depth8;
        s->stk16 = nodes.size() < 65536 && nodes8.size() < 65536;
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
        if (s->has8) AL(s->nodes8, nodes8.size());
        AL(s->tris, ti.size());
        AL(s->shade, ts.size());
        AL(s->mats, mats.size());
        AL(s->tex, (size_t)d->tex_w * d->tex_h);
        AL(s->em_tri, em.size());
        AL(s->em_cdf, emc.size());
        const int M = s->max_light, np = s->npix;
        AL(s->L.ro, M); AL(s->L.rd, M); AL(s->L.hit, M);
        AL(s->L.lv, (size_t)PT_LSTORE * M); AL(s->L.lt, (size_t)PT_LSTORE * M); AL(s->L.lphi, (size_t)PT_LSTORE * M);
        AL(s->L.lfl, (size_t)PT_LSTORE * M); AL(s->L.pool, (size_t)PT_LSTORE * M); AL(s->L.lbeta, M);
        AL(s->L.lb0, M); AL(s->L.sig, M);
        AL(s->L.q[0], M); AL(s->L.q[1], M);
        AL(s->cand, (size_t)4 * M);
        AL(s->kept, (size_t)4 * M); AL(s->final_, (size_t)4 * M);
        AL(s->cost_bin, (size_t)4 * M); AL(s->order, (size_t)4 * M);
        AL(s->E.ro, np); AL(s->E.rd, np); AL(s->E.hit, np); AL(s->E.beta, np); AL(s->E.info, np); AL(s->E.mis, np);
        AL(s->E.q[0], np); AL(s->E.q[1], np);
        AL(s->E.shadow, 2 * (size_t)np); AL(s->E.proxy, np); AL(s->E.mis2, np);
        AL(s->llist, (size_t)PT_LSTORE * M); AL(s->plab, (size_t)PT_LSTORE * M); AL(s->prank, (size_t)PT_LSTORE * M);
        AL(s->E.frame, (size_t)3 * np);
        AL(s->cnt, C_COUNT);
        AL(s->tot, TOT_COUNT);
        AL(s->ts, 2 * PT_TS_CAP);
        AL(s->runmax, 16);
        AL(s->chq[0], CHAIN_LIST_CAP); AL(s->chq[1], CHAIN_LIST_CAP);
        AL(s->chbuf, CHAIN_BUF);
#undef AL
        s->L.M = M;
        s->E.npix = np;
        HIPCHK(hipMemcpyAsync(s->nodes, nodes.data(), nodes.size() * sizeof(BNode), hipMemcpyHostToDevice, stream));
        if (s->has8)
            HIPCHK(hipMemcpyAsync(s->nodes8, nodes8.data(), nodes8.size() * sizeof(BNode8), hipMemcpyHostToDevice,
                                  stream));
        HIPCHK(hipMemcpyAsync(s->tris, ti.data(), ti.size() * sizeof(TriIsect), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(s->shade, ts.data(), ts.size() * sizeof(TriShade), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(s->mats, mats.data(), mats.size() * sizeof(MatDev), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(s->tex, d->tex, sizeof(float) * d->tex_w * d->tex_h, hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(s->em_tri, em.data(), em.size() * sizeof(int), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(s->em_cdf, emc.data(), emc.size() * sizeof(float), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemsetAsync(s->E.frame, 0, sizeof(float) * 3 * np, stream));
        HIPCHK(hipMemsetAsync(s->runmax, 0, sizeof(float) * 16, stream));
        HIPCHK(hipMemsetAsync(s->tot, 0, sizeof(unsigned long long) * TOT_COUNT, stream));
        HIPCHK(hipMemsetAsync(s->ts, 0, sizeof(long long) * 2 * PT_TS_CAP, stream));
        HIPCHK(hipStreamSynchronize(stream));
        SceneDev &S = s->S;
        S.nodes = s->nodes; S.nodes8 = s->nodes8; S.tris = s->tris; S.shade = s->shade; S.mats = s->mats; S.tex = s->tex;
        S.tex_w = d->tex_w; S.tex_h = d->tex_h; S.em_tri = s->em_tri; S.em_cdf = s->em_cdf; S.n_em = (int)em.size();
        S.em_area = (float)area_acc;
        S.tmin = 2e-6f * s->scene_diag;
        S.lo = make_float3(lo[0], lo[1], lo[2]);
        S.inv_ext = make_float3(1.0f / std::max(hi[0] - lo[0], 1e-6f), 1.0f / std::max(hi[1] - lo[1], 1e-6f),
                                1.0f / std::max(hi[2] - lo[2], 1e-6f));
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
        s->gen = next_generation();
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

namespace {
pt_status run_kmeans(pt_scene *s, const float *feat, int n, float *cent, int K, int iters, hipStream_t st)
{
    k_km_init<<<blocks(K, 256), 256, 0, st>>>(feat, n, cent, K);
    for (int it = 0; it < iters && n > 0; ++it) {
        k_fill<<<blocks((long)K * FEAT, 256), 256, 0, st>>>(s->km_sum, 0.0f, (size_t)K * FEAT);
        k_fill<<<blocks(K, 256), 256, 0, st>>>(s->km_cnt, 0.0f, (size_t)K);
        k_km_assign<<<blocks(n, 256), 256, 0, st>>>(feat, n, cent, K, s->km_sum, s->km_cnt);
        k_km_update<<<blocks(K, 256), 256, 0, st>>>(cent, s->km_sum, s->km_cnt, K);
    }
    HIPCHK(hipGetLastError());
    return PT_OK;
}
// groups for the two-level centroid search: k-means of the K centroids into ceil(sqrt K) groups,
// each centroid a member of its nearest group (flat search for K <= 64)
pt_status build_groups(pt_scene *s, const float *cent, int K, pt_scene::GroupSet &gs, int iters, hipStream_t st)
{
    gs.K = K;
    gs.G = 0;
    if (K <= 64) return PT_OK;
    const int G = (int)std::ceil(std::sqrt((double)K));
    if (gs.cap_G < G || gs.cap_K < K) {
        pt_status e;
        if ((e = s->alloc(gs.g, (size_t)G * FEAT)) != PT_OK) return e;
        if ((e = s->alloc(gs.start, (size_t)G + 1)) != PT_OK) return e;
        if ((e = s->alloc(gs.mem, (size_t)K)) != PT_OK) return e;
        gs.cap_G = G; gs.cap_K = K;
    }
    TRY(run_kmeans(s, cent, K, gs.g, G, std::max(iters, 4), st));
    std::vector<float> hc((size_t)K * FEAT), hg((size_t)G * FEAT);
    HIPCHK(hipMemcpyAsync(hc.data(), cent, hc.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hg.data(), gs.g, hg.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<int> grp(K), start(G + 1, 0), mem(K);
    for (int k = 0; k < K; ++k) {
        float bd = 3.0e38f;
        for (int g = 0; g < G; ++g) {
            float d = 0.0f;
            for (int j = 0; j < 9; ++j) {
                const float t = hc[(size_t)FEAT * k + j] - hg[(size_t)FEAT * g + j];
                d += t * t;
            }
            if (d < bd) { bd = d; grp[k] = g; }
        }
        start[grp[k] + 1]++;
    }
    for (int g = 0; g < G; ++g) start[g + 1] += start[g];
    std::vector<int> fill(start.begin(), start.end() - 1);
    for (int k = 0; k < K; ++k) mem[fill[grp[k]]++] = k;
    HIPCHK(hipMemcpyAsync(gs.start, start.data(), start.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(gs.mem, mem.data(), mem.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    gs.G = G;
    return PT_OK;
}
CentSet cent_set(const float *c, const pt_scene::GroupSet &gs)
{
    return CentSet{c, gs.g, gs.start, gs.mem, gs.K, gs.G};
}

__global__ void k_feat_cands(SceneDev S, const Cand *cand, const unsigned long long *cnt, float *feat)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int)cnt[C_NCAND]) return;
    const Cand &c = cand[i];
    float f[9];
    feat9(S, xyz(c.v), S.shade[__float_as_int(c.v.w)].n, oct_dec(make_float2(c.pad[0], c.pad[1])), f);
    for (int j = 0; j < 9; ++j) feat[FEAT * (size_t)i + j] = f[j];
}
__global__ void k_set_counter(unsigned long long *cnt, int idx, unsigned long long v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) cnt[idx] = v;
}
// features of the class-B candidates' control vertices y_0 (position, emitter normal, no
// direction), compacted with the counter cnt[slot]
__global__ void k_feat_ctrl(SceneDev S, const Cand *cand, unsigned long long *cnt, float *feat, int slot)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int)cnt[C_NCAND]) return;
    const Cand &c = cand[i];
    if (!cand_cls(c.cls_u)) return;
    float f[9];
    feat9(S, xyz(c.hc), S.shade[__float_as_int(c.hc.w)].n, f3(0.f, 0.f, 0.f), f);
    const int k = (int)atomicAdd(cnt + slot, 1ull);
    for (int j = 0; j < 9; ++j) feat[FEAT * (size_t)k + j] = f[j];
}
__global__ void k_feat_proxy(SceneDev S, const ProxyItem *items, const unsigned long long *cnt, float *feat)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int)cnt[C_PROXYQ]) return;
    const ProxyItem &p = items[i];
    float f[9];
    feat9(S, xyz(p.x), S.shade[__float_as_int(p.x.w)].n, xyz(p.wo), f);
    for (int j = 0; j < 9; ++j) feat[FEAT * (size_t)i + j] = f[j];
}
}  // namespace

extern "C" pt_status pt_build_subspaces(pt_scene *s, const pt_subspace_params *p, void *stream_)
{
    if (!s || !p) return set_err(PT_EINVAL, "null argument");
    if (p->n_eye <= 0 || p->n_eye > 4096 || p->n_spec <= 0 || p->n_spec > 4096 || p->n_pretrace < 0 ||
        p->kmeans_iters < 0 || p->kmeans_iters > 64 || p->n_light < 0 || p->n_light > 4096 || p->n_ctrl < 0 ||
        p->n_ctrl > 256)
        return set_err(PT_EINVAL, "subspace parameters out of range");
    const int nl = p->n_light > 0 ? p->n_light : p->n_eye;
    const int nc = std::max(1, p->n_ctrl);
    hipStream_t st = (hipStream_t)stream_;
    const int M = s->max_light, np = s->npix;
    const int ne = p->n_eye, ns = p->n_spec;
    // k-means scratch for the largest clustering
    const int kmax = std::max(std::max(ne, ns), nl);
    if (kmax > s->km_cap) {
        pt_status e;
        if ((e = s->alloc(s->km_sum, (size_t)kmax * FEAT)) != PT_OK) return e;
        if ((e = s->alloc(s->km_cnt, (size_t)kmax)) != PT_OK) return e;
        s->km_cap = kmax;
    }
    if (nl != s->n_lsub || ne != s->n_eye || !s->light_c) {
        pt_status e;
#define AL(ptr, n) if ((e = s->alloc(ptr, n)) != PT_OK) return e;
        AL(s->light_c, (size_t)nl * FEAT); AL(s->lcount, nl); AL(s->loff, nl); AL(s->lfill, nl); AL(s->lnonempty, nl);
        if (!s->ln_ne) { AL(s->ln_ne, 1); AL(s->lne_prev, 1); }
        AL(s->lcount_prev, nl);
        AL(s->qacc, (size_t)ne * nl); AL(s->qfrz, (size_t)ne * nl); AL(s->q_alprob, (size_t)ne * nl);
        AL(s->q_alpmf, (size_t)ne * nl);
        AL(s->q_alidx, (size_t)ne * nl); AL(s->q_scratch, (size_t)2 * ne * nl); AL(s->q_rowsum, ne); AL(s->q_rowtot, ne);
#undef AL
        s->n_lsub = nl;
    }
    if (ne != s->n_eye || ns != s->n_spec || !s->eye_c) {
        pt_status e;
#define AL(ptr, n) if ((e = s->alloc(ptr, n)) != PT_OK) return e;
        AL(s->eye_c, (size_t)ne * FEAT); AL(s->spec_c, (size_t)ns * FEAT);

        if (!s->feat) AL(s->feat, (size_t)std::max(np, 4 * M) * FEAT);
        AL(s->s_count, ns); AL(s->s_off, ns); AL(s->s_fill, ns); AL(s->nonempty, ns); AL(s->n_ne, 1);
        if (!s->s_list) AL(s->s_list, (size_t)4 * M);
        AL(s->al_prob, (size_t)ne * ns); AL(s->al_idx, (size_t)ne * ns); AL(s->al_scratch, (size_t)2 * ne * ns);
        AL(s->al_pmf, (size_t)ne * ns);
        AL(s->row_sum, ne); AL(s->gamma_acc, (size_t)ne * ns); AL(s->gamma_frz, (size_t)ne * ns);
        AL(s->s_count_prev, ns); AL(s->row_tot, ne);
        if (!s->prev) AL(s->prev, 4);
        s->tiles_x = (s->W + s->tile - 1) / s->tile;
        s->n_tiles = s->tiles_x * ((s->H + s->tile - 1) / s->tile);
        if (!s->tile_proxy) { AL(s->tile_proxy, s->n_tiles); AL(s->tile_total, s->n_tiles); }
#undef AL
        s->n_eye = ne; s->n_spec = ns;
    }
    // statistics by (class, u, S, C): PT_STAT_CU (3 classes x 5 values of u) x n_ctrl x n_spec buckets
    if ((long)PT_STAT_CU * nc * ns > s->stat_cap) {
        pt_status e;
#define AL(ptr, n) if ((e = s->alloc(ptr, n)) != PT_OK) return e;
        AL(s->rstat_acc, (size_t)3 * PT_STAT_CU * nc * ns); AL(s->rstat_frz, (size_t)3 * PT_STAT_CU * nc * ns);
        AL(s->bstat_acc, (size_t)3 * PT_STAT_CU * nc * ns); AL(s->bstat_frz, (size_t)3 * PT_STAT_CU * nc * ns);
        AL(s->ctrl_c, (size_t)256 * FEAT);
#undef AL
        s->stat_cap = PT_STAT_CU * nc * ns;
    }
    s->n_ctrl = nc;
    // pre-trace: light sub-paths -> candidate specular vertices; eye paths -> first diffuse vertices
    SceneDev S = s->S;
    LightBuf L = s->L;
    L.M = std::max(1, std::min(M, p->n_pretrace > 0 ? p->n_pretrace : M));
    const uint32_t key = 0xFFFFFF00u;
    k_zero<<<blocks(C_COUNT, 256), 256, 0, st>>>(s->cnt, C_COUNT);
    k_iter<<<1, 1, 0, st>>>(s->cnt, key, 0, 0, nullptr, 0);
    k_light_gen<<<blocks(L.M, 256), 256, 0, st>>>(S, L, p->seed, s->cnt);
    for (int vi = 1; vi < PT_LMAX; ++vi) {
        PT_STK_EXT(s, false, L.M, st, S, L.q[(vi - 1) & 1], s->cnt, C_LIGHT_Q0 + vi - 1, L.ro, L.rd,
                   L.hit, s->cnt, C_RAYS_LIGHT);
        k_light_shade<<<blocks(L.M, 256), 256, 0, st>>>(S, L, p->seed, vi, PT_LMAX, s->cnt);
    }
    unsigned long long c[C_COUNT];
    // light subspaces: non-Dirac light vertices y_i, i >= 1 (the connection pool's vertices)
    {
        const int cap = std::max(np, 4 * M);
        k_feat_light<<<blocks((long)(PT_LMAX - 1) * L.M, 256), 256, 0, st>>>(S, L, PT_LMAX, s->feat, cap, s->cnt, C_POOL);
        HIPCHK(hipMemcpyAsync(c, s->cnt, sizeof(c), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        TRY(run_kmeans(s, s->feat, (int)std::min<unsigned long long>(c[C_POOL], (unsigned long long)cap), s->light_c,
                       nl, p->kmeans_iters, st));
        TRY(build_groups(s, s->light_c, nl, s->gs_light, p->kmeans_iters, st));
    }
    k_candidates<<<blocks(L.M, 256), 256, 0, st>>>(L, 4, 0, s->cand, s->cnt);
    k_feat_cands<<<blocks(4L * L.M, 256), 256, 0, st>>>(S, s->cand, s->cnt, s->feat);
    HIPCHK(hipMemcpyAsync(c, s->cnt, sizeof(c), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    TRY(run_kmeans(s, s->feat, (int)c[C_NCAND], s->spec_c, ns, p->kmeans_iters, st));
    TRY(build_groups(s, s->spec_c, ns, s->gs_spec, p->kmeans_iters, st));
    // control subspaces: the control vertices y_0 of the class-B candidates (position, normal)
    if (nc > 1) {
        k_set_counter<<<1, 1, 0, st>>>(s->cnt, C_MLP_ROWS, 0ull);
        k_feat_ctrl<<<blocks(4L * L.M, 256), 256, 0, st>>>(S, s->cand, s->cnt, s->feat, C_MLP_ROWS);
        HIPCHK(hipMemcpyAsync(c, s->cnt, sizeof(c), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        TRY(run_kmeans(s, s->feat, (int)c[C_MLP_ROWS], s->ctrl_c, nc, p->kmeans_iters, st));
        k_set_counter<<<1, 1, 0, st>>>(s->cnt, C_MLP_ROWS, 0ull);
    }
    // eye: first diffuse vertices of one pass (the proxy queue collects them)
    EyeBuf E = s->E;
    EyeParams EP{};
    EP.seed = p->seed; EP.K = 8; EP.u_max = 4; EP.filter = 3; EP.proxy_on = 1; EP.nee_on = 0;
    SubDev D{};
    k_zero<<<blocks(C_COUNT, 256), 256, 0, st>>>(s->cnt, C_COUNT);
    k_camera<<<blocks(np, 256), 256, 0, st>>>(S, E, p->seed, s->cnt);
    for (int t = 1; t <= EP.K; ++t) {
        PT_STK_EXT(s, false, np, st, S, E.q[(t - 1) & 1], s->cnt, C_EYE_Q0 + t - 1, E.ro, E.rd, E.hit,
                   s->cnt, C_RAYS_EYE);
        k_eye_shade<<<blocks(np, 256), 256, 0, st>>>(S, E, EP, D, L, ConnDev{}, t, s->cnt);
    }
    k_fill<<<blocks(3L * np, 256), 256, 0, st>>>(E.frame, 0.0f, (size_t)3 * np);
    k_feat_proxy<<<blocks(np, 256), 256, 0, st>>>(S, E.proxy, s->cnt, s->feat);
    HIPCHK(hipMemcpyAsync(c, s->cnt, sizeof(c), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    TRY(run_kmeans(s, s->feat, (int)c[C_PROXYQ], s->eye_c, ne, p->kmeans_iters, st));
    TRY(build_groups(s, s->eye_c, ne, s->gs_eye, p->kmeans_iters, st));
    // statistics start from nothing
    k_fill<<<blocks((long)ne * ns, 256), 256, 0, st>>>(s->gamma_acc, 0.0f, (size_t)ne * ns);
    k_fill<<<blocks(3L * PT_STAT_CU * nc * ns, 256), 256, 0, st>>>(s->rstat_acc, 0.0f, (size_t)3 * PT_STAT_CU * nc * ns);
    k_fill<<<blocks(3L * PT_STAT_CU * nc * ns, 256), 256, 0, st>>>(s->bstat_acc, 0.0f, (size_t)3 * PT_STAT_CU * nc * ns);
    k_fill<<<blocks(s->n_tiles, 256), 256, 0, st>>>(s->tile_proxy, 0.0f, (size_t)s->n_tiles);
    k_fill<<<blocks(s->n_tiles, 256), 256, 0, st>>>(s->tile_total, 0.0f, (size_t)s->n_tiles);
    k_fill<<<1, 16, 0, st>>>(s->runmax, 0.0f, 16);
    k_fill_i<<<blocks(ns, 256), 256, 0, st>>>(s->s_count, 0, (size_t)ns);
    k_fill_i<<<1, 64, 0, st>>>(s->n_ne, 0, 1);
    k_fill_i<<<blocks(ns, 256), 256, 0, st>>>(s->s_count_prev, 0, (size_t)ns);
    k_fill<<<1, 64, 0, st>>>(s->prev, 0.0f, 4);
    k_fill<<<blocks((long)ne * nl, 256), 256, 0, st>>>(s->qacc, 0.0f, (size_t)ne * nl);
    k_fill_i<<<blocks(nl, 256), 256, 0, st>>>(s->lcount_prev, 0, (size_t)nl);
    k_fill_i<<<blocks(nl, 256), 256, 0, st>>>(s->lcount, 0, (size_t)nl);
    k_fill_i<<<1, 64, 0, st>>>(s->ln_ne, 0, 1);
    k_fill<<<1, 64, 0, st>>>(s->lne_prev, 0.0f, 1);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    s->subspaces_ready = true;
    s->mlp_ready = false;   // the network starts again with the new subspaces
    s->gen = next_generation();
    return PT_OK;
}

namespace {
#define MLP_CAP 65536   // training samples per iteration (each head)
#define MLP_CHUNK (2 * MLP_CAP)   // proxy items per chunk of the per-iteration queries
#define MLP_KSPLIT 32   // K splits of the weight-gradient products (K = samples)

struct MlpOff {
    size_t W1, b1, W2, b2, W3, b3, W4, b4, n;
};
MlpOff mlp_off(int nout)
{
    MlpOff o;
    o.W1 = 0; o.b1 = o.W1 + MLP_IN * MLP_H;
    o.W2 = o.b1 + MLP_H; o.b2 = o.W2 + MLP_H * MLP_H;
    o.W3 = o.b2 + MLP_H; o.b3 = o.W3 + MLP_H * MLP_H;
    o.W4 = o.b3 + MLP_H; o.b4 = o.W4 + (size_t)MLP_H * nout;
    o.n = o.b4 + nout;
    return o;
}

__global__ void k_to_bf16(const float *w, uint16_t *wb, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = f2bf(w[i]);
}
__global__ void k_sum1(const float *x, int n, float *out)
{
    __shared__ float red[256];
    float a = 0.0f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) a += x[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// C = A B on MFMA (see k_gemm); ksplit > 1 adds into C with atomics
void gemm(hipStream_t st, int M, int N, int K, const uint16_t *A, int sam, int sak, const uint16_t *B, int sbk, int sbn,
          float *C, int scm, const unsigned long long *cnt, int m_cidx, int k_cidx, int ksplit)
{
    const long waves = (long)((M + 15) / 16) * ((N + 15) / 16);
    dim3 grid(blocks(waves, 4), 1, ksplit);
    k_gemm<<<grid, 256, 0, st>>>(M, N, K, A, sam, sak, B, sbk, sbn, C, scm, 0, cnt, m_cidx, k_cidx);
}

// the transposed BF16 weight matrices the fused forward pass reads, from the BF16 copy
void mlp_transpose(pt_scene *s, hipStream_t st)
{
    const MlpOff o = mlp_off(s->mlp_nout);
    const long n = (long)MLP_IN * MLP_H + 2L * MLP_H * MLP_H + (long)MLP_H * s->mlp_nout;
    k_mlp_transpose<<<blocks(n, 256), 256, 0, st>>>(s->mwb, s->mwt, s->mlp_nout, o.W1, o.W2, o.W3, o.W4);
}

// allocation (once per output width: n_spec logits + MLP_VMF mixture outputs) and, unless ready,
// initialisation of the network
pt_status ensure_mlp(pt_scene *s, hipStream_t st)
{
    if (!s->subspaces_ready) return set_err(PT_ESTATE, "pt_build_subspaces must run first");
    const int nout = s->n_spec + MLP_VMF;
    if (s->mlp_nout != nout) {
        const MlpOff o = mlp_off(nout);
        // rows: one chunk of the per-item queries, or a training batch of both heads' samples
        const int R = 2 * MLP_CAP;
        pt_status e;
#define AL(ptr, n) if ((e = s->alloc(ptr, n)) != PT_OK) return e;
        AL(s->mw, o.n); AL(s->mg, o.n); AL(s->mm, o.n); AL(s->mv, o.n); AL(s->mwb, o.n); AL(s->mwt, o.n);
        AL(s->mx, (size_t)R * MLP_IN);
        for (int k = 0; k < 3; ++k) AL(s->mh[k], (size_t)R * MLP_H);
        for (int k = 0; k < 2; ++k) AL(s->mdz[k], (size_t)R * MLP_H);
        AL(s->mg4, (size_t)2 * MLP_CAP * nout);
        AL(s->mz, (size_t)R * MLP_H); AL(s->mdh, (size_t)R * MLP_H);
        AL(s->ml, (size_t)R * nout);
        AL(s->mvmf, (size_t)s->npix * MLP_VMF);
        if (!s->MT.feat) {
            AL(s->MT.feat, (size_t)MLP_CAP * 9); AL(s->MT.label, MLP_CAP); AL(s->MT.weight, MLP_CAP);
            AL(s->MT.wsum, 1);
            AL(s->MT.vfeat, (size_t)MLP_CAP * 9); AL(s->MT.vdir, (size_t)MLP_CAP * 3); AL(s->MT.vweight, MLP_CAP);
            AL(s->MT.vwsum, 1);
            s->MT.cap = MLP_CAP;
        }
#undef AL
        s->mlp_nout = nout; s->mlp_rows = R; s->mlp_np = (int)o.n;
        s->mlp_ready = false;
        s->gen = next_generation();
    }
    if (!s->mlp_ready) {
        k_mlp_init<<<blocks(s->mlp_np, 256), 256, 0, st>>>(s->mw, s->mwb, s->mg, s->mm, s->mv, nout, 0x6d6c7001u);
        mlp_transpose(s, st);
        k_set_counter<<<1, 1, 0, st>>>(s->cnt, C_MLP_T, 0ull);
        HIPCHK(hipGetLastError());
        s->mlp_ready = true;
    }
    return PT_OK;
}

// outputs col0 .. col0 + ncols - 1 of the first rows of s->mx into out (row stride ncols), with
// bias_out[col] added when given: rows = min(M, cnt[m_cidx] - off) (or M), one fused launch;
// keep_h: the hidden activations go to mh[0..2] for the backward pass
void mlp_forward(pt_scene *s, int M, const unsigned long long *cnt, int m_cidx, float *out, int col0, int ncols,
                 hipStream_t st, const float *bias_out = nullptr, bool keep_h = false, int off = 0)
{
    const int nout = s->mlp_nout;
    const MlpOff o = mlp_off(nout);
    const int grid = std::max(1, std::min(blocks(M, MLP_FT_ROWS), 2048));
    if (keep_h)
        k_mlp_fwd<true><<<grid, 256, 0, st>>>(s->mx, M, cnt, m_cidx, s->mwt, s->mw, o.W1, o.b1, o.W2, o.b2, o.W3, o.b3,
                                              o.W4, nout, col0, ncols, out, bias_out, s->mh[0], s->mh[1], s->mh[2], off);
    else
        k_mlp_fwd<false><<<grid, 256, 0, st>>>(s->mx, M, cnt, m_cidx, s->mwt, s->mw, o.W1, o.b1, o.W2, o.b2, o.W3,
                                               o.b3, o.W4, nout, col0, ncols, out, bias_out, nullptr, nullptr, nullptr,
                                               off);
}

// gradient of the training batch's loss (rows: T's min(cap, C_MLP_N) subspace samples, then its
// min(cap, C_MLP_NV) direction samples, encoded in s->mx; cnt[C_MLP_ROWS] set): the weighted
// cross entropy of the logits plus the weighted negative log-likelihood of the directions under
// the vMF mixture, each over its own weight sum, added into s->mg (which is zero before)
void mlp_backward(pt_scene *s, const MlpTrain &T, hipStream_t st)
{
    const int R = 2 * MLP_CAP, N = s->mlp_nout, ns = s->n_spec;
    const MlpOff o = mlp_off(N);
    unsigned long long *cnt = s->cnt;
    mlp_forward(s, R, cnt, C_MLP_ROWS, s->ml, 0, N, st, nullptr, true);
    k_ce_grad<<<MLP_CAP, 256, 0, st>>>(s->ml, s->mw + o.b4, T.label, T.weight, T.wsum, MLP_CAP, ns, N, s->mg4, cnt,
                                       C_MLP_N);
    k_vmf_grad<<<blocks(MLP_CAP, 256), 256, 0, st>>>(s->ml, s->mw + o.b4, T.vdir, T.vweight, T.vwsum, N, ns, s->mg4,
                                                     cnt, MLP_CAP);
    k_colsum<<<dim3(blocks(N, 64), R / MLP_STRIP), 64, 0, st>>>(s->mg4, R, N, s->mg + o.b4, cnt, C_MLP_ROWS);
    // layer 4: dW4 = H3^T G4, dH3 = G4 W4^T
    gemm(st, MLP_H, N, R, s->mh[2], 1, MLP_H, s->mg4, N, 1, s->mg + o.W4, N, cnt, -1, C_MLP_ROWS, MLP_KSPLIT);
    gemm(st, R, MLP_H, N, s->mg4, N, 1, s->mwb + o.W4, 1, N, s->mdh, MLP_H, cnt, C_MLP_ROWS, -1, 1);
    const size_t Wo[3] = {o.W1, o.W2, o.W3}, bo[3] = {o.b1, o.b2, o.b3};
    for (int l = 2; l >= 0; --l) {
        uint16_t *dz = s->mdz[l & 1];
        k_relu_back<<<blocks((long)R * MLP_H, 256), 256, 0, st>>>(s->mdh, s->mh[l], dz, R, MLP_H, cnt, C_MLP_ROWS);
        k_colsum<<<dim3(1, R / MLP_STRIP), 64, 0, st>>>(dz, R, MLP_H, s->mg + bo[l], cnt, C_MLP_ROWS);
        const uint16_t *in = l == 0 ? s->mx : s->mh[l - 1];
        const int K = l == 0 ? MLP_IN : MLP_H;
        gemm(st, K, MLP_H, R, in, 1, K, dz, MLP_H, 1, s->mg + Wo[l], MLP_H, cnt, -1, C_MLP_ROWS, MLP_KSPLIT);
        if (l > 0)
            gemm(st, R, MLP_H, MLP_H, dz, MLP_H, 1, s->mwb + Wo[l], 1, MLP_H, s->mdh, MLP_H, cnt, C_MLP_ROWS, -1, 1);
    }
}

void mlp_adam(pt_scene *s, float lr, hipStream_t st)
{
    k_adam<<<blocks(s->mlp_np, 256), 256, 0, st>>>(s->mw, s->mwb, s->mg, s->mm, s->mv, s->mlp_np, lr, 0.9f, 0.999f,
                                                   1e-8f, s->cnt);
    mlp_transpose(s, st);
    k_mlp_tick<<<1, 1, 0, st>>>(s->cnt);
}

pt_status check_params(pt_scene *s, const pt_iter_params *p, float *acc)
{
    if (!s || !p || !acc) return set_err(PT_EINVAL, "null argument");
    if (!s->subspaces_ready) return set_err(PT_ESTATE, "pt_build_subspaces must run before pt_render_iteration");
    if (p->max_depth < 1 || p->max_depth > PT_MAX_DEPTH) return set_err(PT_EINVAL, "max_depth out of range [1, %d]", PT_MAX_DEPTH);
    if (p->n_light < 1 || p->n_light > s->max_light) return set_err(PT_EINVAL, "n_light out of range [1, %d]", s->max_light);
    if (p->u_max < 1 || p->u_max > 4) return set_err(PT_EINVAL, "u_max out of range [1, 4]");
    if (p->recip_repeats < 1 || p->recip_repeats > 8) return set_err(PT_EINVAL, "recip_repeats out of range [1, 8]");
    if (p->cand_cap < 1 || p->pilot < 0) return set_err(PT_EINVAL, "cand_cap must be positive, pilot not negative");
    if (p->pilot == 0 && (p->flags & PT_FLAG_PROXY) && !(p->flags & (PT_FLAG_GAMMA | PT_FLAG_MIS | PT_FLAG_MLP)))
        return set_err(PT_EINVAL, "pilot = 0 needs the subspace statistics (PT_FLAG_GAMMA, PT_FLAG_MIS or PT_FLAG_MLP)");
    if ((p->flags & PT_FLAG_ONLY_PROXY_CLASS) && (p->flags & PT_FLAG_ONLY_OTHER))
        return set_err(PT_EINVAL, "class filters are exclusive");
    if ((p->flags & (PT_FLAG_SPC | PT_FLAG_LT)) && p->max_depth > PT_LSTORE)
        return set_err(PT_EINVAL, "light-vertex connections and light tracing support max_depth <= %d", PT_LSTORE);
    if ((p->flags & PT_FLAG_MLP) && !(p->mlp_mix >= 0.0f && p->mlp_mix < 1.0f && p->mlp_lr > 0.0f))
        return set_err(PT_EINVAL, "PT_FLAG_MLP needs 0 <= mlp_mix < 1 and mlp_lr > 0");
    if ((p->flags & PT_FLAG_BOOTH) && !(p->booth_r > 0.0f)) return set_err(PT_EINVAL, "PT_FLAG_BOOTH needs booth_r > 0");
    if ((p->flags & PT_FLAG_GENERAL_CV) && (!(p->flags & PT_FLAG_PROXY) || (p->flags & PT_FLAG_MIS)))
        return set_err(PT_EINVAL, "PT_FLAG_GENERAL_CV needs PT_FLAG_PROXY, without PT_FLAG_MIS");
    return PT_OK;
}



// Enqueues one iteration on `stream`: kernel launches only (no host synchronisation, no
// memset), so the sequence can be captured into a HIP graph. graph = true: the iteration index
// in device memory is advanced by one instead of being set from p->iteration.
// stage A's first-round sample count of a chain
uint32_t stage_a_n1(const pt_iter_params *p) { return (uint32_t)std::max(64.0f, p->cost_cap / (float)p->recip_repeats); }

// part: 0 = the whole iteration; 1 = up to the reciprocal chains' stage A (exclusive); 2 = from
// the chain rounds on (a multi-scene graph runs stage A of all its scenes in one launch between)
pt_status enqueue_iteration(pt_scene *s, const pt_iter_params *p, float *acc, float *acc2, hipStream_t stream,
                            bool graph, int part = 0)
{
    const bool pre = part != 2, post = part != 1;
    SceneDev S = s->S;
    LightBuf L = s->L;
    L.M = p->n_light;
    EyeBuf E = s->E;
    const int M = L.M;
    const bool proxy = (p->flags & PT_FLAG_PROXY) != 0;
    const bool count = (p->flags & PT_FLAG_COUNT) != 0;
    const bool timing = (p->flags & PT_FLAG_TIMING) != 0;
    // events: two per eye extension launch, then four around the reciprocal block
    const size_t n_ev = 2 * (size_t)p->max_depth + 4;
    if (timing && s->ev.size() < n_ev) {
        while (s->ev.size() < n_ev) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            s->ev.push_back(e);
        }
    }
    const bool gamma = proxy && (p->flags & PT_FLAG_GAMMA);
    const bool mis = proxy && (p->flags & PT_FLAG_MIS);
    const bool tiles = proxy && (p->flags & PT_FLAG_TILES) && p->tile == s->tile;
    const bool mlp = proxy && (p->flags & PT_FLAG_MLP) && s->mlp_ready && s->mlp_nout == s->n_spec + MLP_VMF;
    const bool labels = gamma || mis || mlp;
    const int ne = s->n_eye, ns = s->n_spec;
    if (pre) k_zero<<<blocks(C_COUNT, 256), 256, 0, stream>>>(s->cnt, C_COUNT);
    if (pre) k_iter<<<1, 1, 0, stream>>>(s->cnt, p->iteration, graph ? 1 : 0, p->train_iters, s->ts, 1);
    if (labels && pre) {
        // statistics of earlier iterations only: frozen copies for this iteration
        k_copy<<<blocks((long)ne * ns, 256), 256, 0, stream>>>(s->gamma_acc, s->gamma_frz, (size_t)ne * ns);
        const size_t nst = (size_t)PT_STAT_CU * s->n_ctrl * ns;
        k_copy<<<blocks((long)(3 * nst), 256), 256, 0, stream>>>(s->rstat_acc, s->rstat_frz, 3 * nst);
        k_copy<<<blocks((long)(3 * nst), 256), 256, 0, stream>>>(s->bstat_acc, s->bstat_frz, 3 * nst);
        k_row_tot<<<blocks(ne, 256), 256, 0, stream>>>(s->gamma_frz, ne, ns, s->row_tot);
    }
    const bool conn = (p->flags & PT_FLAG_SPC) != 0, ltr = (p->flags & PT_FLAG_LT) != 0;
    // light sub-paths: y_0 .. y_{lmax-1}; connections and light tracing use every vertex a path
    // within max_depth segments can have, the proxy candidates the first PT_LMAX
    const int lmax = (conn || ltr) ? p->max_depth : std::min(p->max_depth - 1, PT_LMAX);
    if (pre && (proxy || conn || ltr)) {
        k_light_gen<<<blocks(M, 256), 256, 0, stream>>>(S, L, p->seed, s->cnt);
        for (int vi = 1; vi < lmax; ++vi) {
            PT_STK_EXT(s, false, M, stream, S, L.q[(vi - 1) & 1], s->cnt, C_LIGHT_Q0 + vi - 1, L.ro,
                       L.rd, L.hit, s->cnt, C_RAYS_LIGHT);
            k_light_shade<<<blocks(M, 256), 256, 0, stream>>>(S, L, p->seed, vi, lmax, s->cnt);
        }
    }
    // The connection pool, the eye pass, light tracing and the bucket sizes kept for the next
    // iteration read the light store and frozen statistics only, none of the reciprocal
    // estimates, and the reciprocal block reads none of theirs, so they run on a second stream
    // beside the reciprocal block, forked after the light pass and joined before the proxy
    // connections. Iterations with PT_FLAG_TIMING stay on one stream so that each timed kernel has
    // the device to itself, and so do captured iterations (pt_render_batch, pt_render_scenes: a
    // fork inside the multi-scene capture ended the process; their scenes already run side by
    // side as the graph's branches).
    const bool overlap = !timing && !graph && proxy && s->side && part == 0;
    hipStream_t es = stream;
    if (overlap) {
        HIPCHK(hipEventRecord(s->ev_fork, stream));
        HIPCHK(hipStreamWaitEvent(s->side, s->ev_fork, 0));
        es = s->side;
    }
    const MisK mk{(p->flags & PT_FLAG_NEE) ? 1.0f : 0.0f, conn ? 1.0f : 0.0f, ltr ? (float)M : 0.0f};
    const int nl = s->n_lsub;
    ConnDev CD{};
    if (conn) {
        CD.light = cent_set(s->light_c, s->gs_light); CD.eye = cent_set(s->eye_c, s->gs_eye);
        CD.n_lsub = nl; CD.n_eye = ne; CD.M = M;
        CD.lab = s->plab; CD.rank = s->prank; CD.count = s->lcount; CD.off = s->loff; CD.fill = s->lfill; CD.list = s->llist;
        CD.nonempty = s->lnonempty; CD.n_nonempty = s->ln_ne;
        CD.al_prob = s->q_alprob; CD.al_idx = s->q_alidx; CD.al_pmf = s->q_alpmf; CD.row_sum = s->q_rowsum; CD.q = s->qfrz;
        CD.row_tot = s->q_rowtot; CD.count_prev = s->lcount_prev; CD.ne_prev = s->lne_prev;
        CD.defensive = p->defensive; CD.qacc = s->qacc;
        // Q of earlier iterations only
        if (pre) k_copy<<<blocks((long)ne * nl, 256), 256, 0, es>>>(s->qacc, s->qfrz, (size_t)ne * nl);
        if (pre) k_row_tot<<<blocks(ne, 256), 256, 0, es>>>(s->qfrz, ne, nl, s->q_rowtot);
    }
    if (pre && (conn || ltr) && lmax >= 2) {
        const long maxp = (long)(lmax - 1) * M;
        if (!conn) k_pool<<<blocks(maxp, 256), 256, 0, es>>>(L, lmax, s->cnt);
        if (conn) {
            // the pool, bucketed by light subspace; alias rows of Q over the non-empty buckets
            k_fill_i<<<blocks(nl, 256), 256, 0, es>>>(s->lcount, 0, (size_t)nl);
            k_pool_label<<<blocks(maxp, 256), 256, 0, es>>>(S, L, lmax, CD, s->cnt);
            k_scan_sub<<<1, 1024, 0, es>>>(s->lcount, s->loff, s->lfill, s->lnonempty, s->ln_ne, nl);
            k_scatter_pool<<<blocks(maxp, 256), 256, 0, es>>>(L, CD, s->cnt);
            alias_rows(s->qfrz, ne, nl, s->lnonempty, s->ln_ne, p->defensive, s->q_alprob, s->q_alidx, s->q_rowsum,
                       s->q_alpmf, s->q_scratch, es);
        }
        k_light_phi<<<blocks(M, 256), 256, 0, es>>>(S, L, mk, CD, s->cnt);
    }
    // eye pass. Without MIS the proxy strategy alone scores the proxy-class paths (a partition);
    // with MIS, PT/NEE keep them with the weights of Section 5.4.
    EyeParams EP{};
    EP.seed = p->seed; EP.K = p->max_depth; EP.u_max = p->u_max;
    EP.proxy_on = proxy && !(p->flags & PT_FLAG_ONLY_OTHER);
    const bool only_cls = (p->flags & PT_FLAG_ONLY_PROXY_CLASS) != 0, only_oth = (p->flags & PT_FLAG_ONLY_OTHER) != 0;
    if (EP.proxy_on && !mis) EP.filter = only_cls ? 3 : 2;
    else EP.filter = only_cls ? 1 : (only_oth ? 2 : 0);
    EP.nee_on = (p->flags & PT_FLAG_NEE) != 0;
    EP.mis_on = mis && EP.proxy_on;
    EP.labels_on = labels && EP.proxy_on;
    EP.gamma_on = gamma;
    EP.mlp_on = mlp && EP.proxy_on;
    EP.tiles_on = tiles;
    EP.M = M; EP.cand_cap = p->cand_cap;
    EP.mk = mk; EP.conn_on = conn && lmax >= 2;
    EP.gcv = (p->flags & PT_FLAG_GENERAL_CV) != 0;
    SubDev D{};
    if (s->n_eye > 0) {
        D.eye_c = s->eye_c; D.spec_c = s->spec_c; D.n_eye = ne; D.n_spec = ns;
        D.eye = cent_set(s->eye_c, s->gs_eye); D.spec = cent_set(s->spec_c, s->gs_spec);
        D.s_count = s->s_count; D.s_off = s->s_off; D.s_list = s->s_list; D.nonempty = s->nonempty; D.n_nonempty = s->n_ne;
        D.al_prob = s->al_prob; D.al_idx = s->al_idx; D.al_pmf = s->al_pmf; D.row_sum = s->row_sum; D.gamma = s->gamma_frz;
        D.defensive = p->defensive; D.rstat = s->rstat_frz; D.bstat = s->bstat_frz;
        D.ctrl_c = s->ctrl_c; D.n_ctrl = s->n_ctrl;
        D.prev = s->prev; D.s_count_prev = s->s_count_prev; D.row_tot = s->row_tot;
        D.tile_proxy = s->tile_proxy; D.tile_total = s->tile_total; D.tile = s->tile; D.tiles_x = s->tiles_x;
        D.tile_thr = p->tile_threshold; D.tile_low = p->tile_low_prob;
    }
    const int np = s->npix;
    if (pre) k_camera<<<blocks(np, 256), 256, 0, es>>>(S, E, p->seed, s->cnt);
    for (int t = 1; pre && t <= p->max_depth; ++t) {
        if (timing) HIPCHK(hipEventRecord(s->ev[2 * (t - 1)], es));
        PT_STK_EXT(s, count, np, es, S, E.q[(t - 1) & 1], s->cnt, C_EYE_Q0 + t - 1, E.ro, E.rd, E.hit,
                   s->cnt, C_RAYS_EYE);
        if (timing) HIPCHK(hipEventRecord(s->ev[2 * (t - 1) + 1], es));
        k_eye_shade<<<blocks(np, 256), 256, 0, es>>>(S, E, EP, D, L, CD, t, s->cnt);
        PT_STK(s, k_occluded, blocks(2L * np, WG), WG, es, S, E, CD, t, s->cnt);
    }
    if (pre && ltr && lmax >= 2)
        PT_STK(s, k_lt, blocks((long)(lmax - 1) * M, WG), WG, es, S, L, EP, D, CD, E.frame, s->cnt);
    if (pre && conn && lmax >= 2) k_conn_prev<<<blocks(nl, 256), 256, 0, es>>>(CD, s->lcount_prev, s->lne_prev);
    if (proxy) {
        if (lmax >= 2) {
            const int maxc = 4 * M;
            const size_t e0 = 2 * (size_t)p->max_depth;
            if (pre) {
                k_candidates<<<blocks(M, 256), 256, 0, stream>>>(L, p->u_max, (p->flags & PT_FLAG_GENERAL_CV) ? 1 : 0,
                                                                 s->cand, s->cnt);
                k_keep<<<blocks(maxc, 256), 256, 0, stream>>>(p->cand_cap, p->seed, s->kept, maxc, s->cnt);
                // subspace labels (S, C) of the kept candidates: their buckets' statistics give B a floor
                if (labels) k_label_kept<<<blocks(maxc, 256), 256, 0, stream>>>(S, D, s->cand, s->kept, s->cnt);
                if (timing) HIPCHK(hipEventRecord(s->ev[e0], stream));
                // pilot = 0: B and beta of a candidate from its (class, u, S, C) bucket's statistics alone
                if (p->pilot > 0)
                    PT_STK(s, k_pilot, s->persist_wg, 64 * RW, stream, S, s->cand, s->kept, p->pilot, p->seed,
                           s->runmax, s->cnt);
                k_roulette<<<blocks(maxc, 256), 256, 0, stream>>>(s->cand, s->kept, s->final_, s->cost_bin, s->runmax,
                                                                  D, labels ? 1 : 0, S.em_area, p->recip_repeats,
                                                                  p->cost_cap, p->seed, s->cnt);
                k_order<<<blocks(maxc, 256), 256, 0, stream>>>(s->cost_bin, s->order, s->cnt);
            }
            const uint32_t n1 = stage_a_n1(p);
            const float booth_r = (p->flags & PT_FLAG_BOOTH) ? p->booth_r : 0.0f;
            if (timing) HIPCHK(hipEventRecord(s->ev[e0 + 1], stream));
            if (part != 0) {
                // stage A belongs to the multi-scene launch between the two parts
            } else if (booth_r > 0.0f) {
                if (s->bvh_cur == 8) {
                    if (s->stk16) launch_recip_booth<int16_t>(s->persist_wg, stream, S, s->cand, s->final_, s->order,
                                                              p->recip_repeats, p->seed, n1, s->tune_budget, s->runmax,
                                                              s->chq[0], booth_r, s->cnt, s->queue_chunk, s->ahead);
                    else launch_recip_booth<uint32_t>(s->persist_wg, stream, S, s->cand, s->final_, s->order,
                                                      p->recip_repeats, p->seed, n1, s->tune_budget, s->runmax,
                                                      s->chq[0], booth_r, s->cnt, s->queue_chunk, s->ahead);
                } else {
                    if (s->stk16) launch_recip_booth<uint16_t>(s->persist_wg, stream, S, s->cand, s->final_, s->order,
                                                               p->recip_repeats, p->seed, n1, s->tune_budget, s->runmax,
                                                               s->chq[0], booth_r, s->cnt, s->queue_chunk, s->ahead);
                    else launch_recip_booth<int>(s->persist_wg, stream, S, s->cand, s->final_, s->order,
                                                 p->recip_repeats, p->seed, n1, s->tune_budget, s->runmax, s->chq[0],
                                                 booth_r, s->cnt, s->queue_chunk, s->ahead);
                }
            } else if (s->refill && s->bvh_cur == 4) {
                // walks refilled node by node (4-wide trees)
                if (s->stk16)
                    k_recip<uint16_t, false, true><<<s->persist_wg, 64 * RW, 0, stream>>>(
                        S, s->cand, s->final_, s->order, p->recip_repeats, p->seed, n1, s->tune_budget, s->runmax,
                        s->chq[0], booth_r, s->cnt, s->queue_chunk, s->ahead);
                else
                    k_recip<int, false, true><<<s->persist_wg, 64 * RW, 0, stream>>>(
                        S, s->cand, s->final_, s->order, p->recip_repeats, p->seed, n1, s->tune_budget, s->runmax,
                        s->chq[0], booth_r, s->cnt, s->queue_chunk, s->ahead);
            } else {
                PT_STK(s, k_recip, s->persist_wg, 64 * RW, stream, S, s->cand, s->final_, s->order, p->recip_repeats,
                       p->seed, n1, s->tune_budget, s->runmax, s->chq[0], booth_r, s->cnt, s->queue_chunk, s->ahead);
            }
            if (timing) HIPCHK(hipEventRecord(s->ev[e0 + 2], stream));
            for (int r = 0; post && r < CHAIN_ROUNDS; ++r) {
                const int in = r & 1, out = in ^ 1;
                k_set_counter<<<1, 1, 0, stream>>>(s->cnt, C_LONGQ0 + out, 0ull);
                PT_STK(s, k_chain_gen, s->tune_gen_grid, WG, stream, S, s->cand, s->chq[in], C_LONGQ0 + in, r, p->seed,
                              s->chbuf, s->cnt);
                k_chain_consume<<<2048, 64 * RW, 0, stream>>>(s->cand, s->chq[in], C_LONGQ0 + in, s->chq[out],
                                                              C_LONGQ0 + out, r, r == CHAIN_ROUNDS - 1 ? 1 : 0,
                                                              p->seed, s->chbuf, s->runmax, booth_r, s->cnt);
            }
            if (timing) HIPCHK(hipEventRecord(s->ev[e0 + 3], stream));
            if (labels && post) {
                k_fill_i<<<blocks(ns, 256), 256, 0, stream>>>(s->s_count, 0, (size_t)ns);
                k_count_sub<<<blocks(maxc, 256), 256, 0, stream>>>(s->cand, s->final_, s->cnt, s->s_count);
                k_scan_sub<<<1, 1024, 0, stream>>>(s->s_count, s->s_off, s->s_fill, s->nonempty, s->n_ne, ns);
                k_scatter_sub<<<blocks(maxc, 256), 256, 0, stream>>>(s->cand, s->final_, s->cnt, s->s_fill, s->s_list);
                if (gamma)
                    alias_rows(s->gamma_frz, ne, ns, s->nonempty, s->n_ne, p->defensive, s->al_prob, s->al_idx,
                               s->row_sum, s->al_pmf, s->al_scratch, stream);
                k_rstat<<<blocks(maxc, 256), 256, 0, stream>>>(s->cand, s->final_, s->cnt, p->recip_repeats, D,
                                                                  s->rstat_acc, s->bstat_acc);
            }
        }
    }
    if (part == 1) {
        HIPCHK(hipGetLastError());
        return PT_OK;
    }
    if (overlap) {
        HIPCHK(hipEventRecord(s->ev_join, es));
        HIPCHK(hipStreamWaitEvent(stream, s->ev_join, 0));
    }
    StatBuf SB{s->gamma_acc, s->tile_proxy, s->tile_total};
    const bool vmf = EP.mlp_on && (p->flags & PT_FLAG_MLP_DIR);
    if (EP.mlp_on) {
        // the network's logits for every queued first diffuse vertex, then S and the incomplete
        // sub-path per item; for the direction head, the mixture at each chosen y_{s-1}
        const MlpOff o = mlp_off(s->mlp_nout);
        k_fill<<<1, 64, 0, stream>>>(s->MT.wsum, 0.0f, 1);
        k_fill<<<1, 64, 0, stream>>>(s->MT.vwsum, 0.0f, 1);
        // in chunks of MLP_CHUNK items, so that the logits of a chunk (MLP_CHUNK x n_spec) bound the
        // workspace whatever the image size
        for (int c0 = 0; c0 < np; c0 += MLP_CHUNK) {
            const int m = std::min(MLP_CHUNK, np - c0);
            k_mlp_enc_items<<<blocks(m, 256), 256, 0, stream>>>(S, E.proxy, s->cnt, s->mx, c0, m);
            mlp_forward(s, m, s->cnt, C_PROXYQ, s->ml, 0, ns, stream, nullptr, false, c0);
            // one thread per item over a few subspaces, one wavefront per item over many
            if (ns > 32)
                k_mlp_select_wave<<<blocks(m, 4), 256, 0, stream>>>(E, D, s->ml, s->mw + o.b4, ns, p->mlp_mix,
                                                                    gamma ? 1 : 0, p->seed, s->cnt, c0, m);
            else
                k_mlp_select<<<blocks(m, 256), 256, 0, stream>>>(E, D, s->ml, s->mw + o.b4, ns, p->mlp_mix,
                                                                 gamma ? 1 : 0, p->seed, s->cnt, c0, m);
            if (vmf) {
                k_mlp_enc_retrace<<<blocks(m, 256), 256, 0, stream>>>(S, E.proxy, s->cand, s->cnt, s->mx, c0, m);
                mlp_forward(s, m, s->cnt, C_PROXYQ, s->mvmf + (size_t)c0 * MLP_VMF, ns, MLP_VMF, stream,
                            s->mw + o.b4 + ns, false, c0);
            }
        }
    }
    EP.vmf_on = vmf ? 1 : 0;
    EP.mix = p->mlp_mix;
    if (EP.proxy_on)
        PT_STK(s, k_proxy, blocks(np, WG), WG, stream, S, E, s->cand, s->final_, EP, D, SB, s->MT, s->mvmf,
               p->recip_repeats, s->cnt);
    if (EP.mlp_on) {
        // online training on this iteration's samples (no work unless the iteration recorded some)
        k_mlp_rows<<<1, 1, 0, stream>>>(s->cnt, MLP_CAP);
        k_mlp_enc_train<<<blocks(2 * MLP_CAP, 256), 256, 0, stream>>>(s->MT, s->cnt, s->mx);
        mlp_backward(s, s->MT, stream);
        mlp_adam(s, p->mlp_lr, stream);
    }
    if (labels && s->prev)
        k_prev_store<<<blocks(ns, 256), 256, 0, stream>>>(s->cnt, s->s_count, s->n_ne, ns, s->prev, s->s_count_prev);
    k_accumulate<<<blocks(np, 256), 256, 0, stream>>>(E.frame, acc, acc2, np, s->W, s->tile, s->tiles_x,
                                                      tiles ? s->tile_total : nullptr, s->cnt);
    k_totals<<<1, 64, 0, stream>>>(s->cnt, s->tot, s->ts);
    HIPCHK(hipGetLastError());
    return PT_OK;
}
}  // namespace

extern "C" pt_status pt_render_iteration(pt_scene *s, const pt_iter_params *p, float *acc, float *acc2,
                                         pt_iter_stats *stats, void *stream_)
{
    TRY(check_params(s, p, acc));
    hipStream_t stream = (hipStream_t)stream_;
    const bool timing = (p->flags & PT_FLAG_TIMING) != 0;
    if (p->flags & PT_FLAG_MLP) TRY(ensure_mlp(s, stream));
    TRY(enqueue_iteration(s, p, acc, acc2, stream, false));
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
            if ((p->flags & PT_FLAG_PROXY) && std::min(p->max_depth - 1, PT_LMAX) >= 2) {
                const size_t e0 = 2 * (size_t)p->max_depth;
                float a = 0.0f, b = 0.0f;
                HIPCHK(hipEventElapsedTime(&a, s->ev[e0], s->ev[e0 + 3]));
                HIPCHK(hipEventElapsedTime(&b, s->ev[e0 + 1], s->ev[e0 + 2]));
                stats->ms_recip = a;
                stats->ms_recip_stage_a = b;
            }
        }
        stats->node_visits_recip = (double)c[C_VISITS_R];
        stats->tri_tests_recip = (double)c[C_TESTS_R];
        stats->node_visits_stage_a = (double)c[C_VISITS_A];
        stats->tri_tests_stage_a = (double)c[C_TESTS_A];
        stats->n_samples_stage_a = (double)c[C_SAMPLES_A];
        stats->n_drawn_stage_a = (double)c[C_DRAWN_A];
        stats->n_drawn_pilot = (double)c[C_DRAWN_P];
        stats->wave_trips_stage_a = (double)c[C_TRIPS_A];
        stats->n_pool = (double)c[C_POOL];
        stats->n_connections = (double)c[C_SPC];
        stats->n_lt_splats = (double)c[C_LT];
        for (int b = 0; b < 24; ++b) stats->chain_len_hist[b] = (double)c[C_CHAIN_HIST + b];
        stats->chain_len_max = (double)c[C_CHAIN_MAX];
    }
    return PT_OK;
}

extern "C" pt_status pt_render_batch(pt_scene *s, const pt_iter_params *p, uint32_t n_iter, float *acc, float *acc2,
                                     void *stream_)
{
    TRY(check_params(s, p, acc));
    if (n_iter == 0) return set_err(PT_EINVAL, "n_iter must be positive");
    if (p->flags & PT_FLAG_TIMING) return set_err(PT_EINVAL, "PT_FLAG_TIMING cannot be captured");
    hipStream_t stream = (hipStream_t)stream_;
    if (p->flags & PT_FLAG_MLP) {
        TRY(ensure_mlp(s, stream));
        // the capture stream does not wait on `stream`: finish the initialisation first
        HIPCHK(hipStreamSynchronize(stream));
    }
    // the graph depends on everything but the iteration index
    pt_iter_params key = *p;
    key.iteration = 0;
    std::vector<char> k((const char *)&key, (const char *)&key + sizeof(key));
    k.insert(k.end(), (const char *)&acc, (const char *)&acc + sizeof(acc));
    k.insert(k.end(), (const char *)&acc2, (const char *)&acc2 + sizeof(acc2));
    k.insert(k.end(), (const char *)&s->gen, (const char *)&s->gen + sizeof(s->gen));
    k.insert(k.end(), (const char *)&s->tune_budget, (const char *)&s->tune_budget + sizeof(s->tune_budget));
    k.insert(k.end(), (const char *)&s->tune_gen_grid, (const char *)&s->tune_gen_grid + sizeof(s->tune_gen_grid));
    k.insert(k.end(), (const char *)&s->ext_wg, (const char *)&s->ext_wg + sizeof(s->ext_wg));
    k.insert(k.end(), (const char *)&s->queue_chunk, (const char *)&s->queue_chunk + sizeof(s->queue_chunk));
    k.insert(k.end(), (const char *)&s->ahead, (const char *)&s->ahead + sizeof(s->ahead));
    k.insert(k.end(), (const char *)&s->refill, (const char *)&s->refill + sizeof(s->refill));
    if (!s->gexec || k != s->gkey) {
        ++s->n_captures;
        if (s->gexec) { HIPCHK(hipGraphExecDestroy(s->gexec)); s->gexec = nullptr; }
        if (!s->cap_stream) HIPCHK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
        pt_status st = enqueue_iteration(s, p, acc, acc2, s->cap_stream, true);
        hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
        if (st != PT_OK) { if (g) (void)hipGraphDestroy(g); return st; }
        if (e != hipSuccess) return set_err(PT_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) { s->gexec = nullptr; return set_err(PT_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e)); }
        s->gkey = k;
    }
    // the captured iteration advances the device-side index first: start one below
    k_iter<<<1, 1, 0, stream>>>(s->cnt, p->iteration - 1u, 0, p->train_iters, nullptr, 0);
    for (uint32_t i = 0; i < n_iter; ++i) HIPCHK(hipGraphLaunch(s->gexec, stream));
    HIPCHK(hipGetLastError());
    return PT_OK;
}

namespace {
// validation shared by both table-mode entry points
pt_status check_table_query(const pt_recip_query *q, const float *out, const uint32_t *ns)
{
    if (!q || !out || !ns) return set_err(PT_EINVAL, "null argument");
    if (q->n_est <= 0 || !(q->B > 0.0f)) return set_err(PT_EINVAL, "n_est and B must be positive");
    if (q->mode != PT_RECIP_TABLE) return set_err(PT_EINVAL, "not a table query");
    if (q->n <= 0 || !q->f_dev || !q->q_dev) return set_err(PT_EINVAL, "bad table query");
    if (q->estimator != PT_EST_ITILDE && q->estimator != PT_EST_SIGN && q->estimator != PT_EST_BOOTH)
        return set_err(PT_EINVAL, "unknown estimator");
    if (q->estimator == PT_EST_BOOTH && !(q->booth_r > 0.0f)) return set_err(PT_EINVAL, "booth_r must be positive");
    return PT_OK;
}
}  // namespace

extern "C" pt_status pt_reciprocal_estimate(pt_scene *s, const pt_recip_query *q, float *out, uint32_t *ns,
                                            void *stream_)
{
    if (!q || !out || !ns) return set_err(PT_EINVAL, "null argument");
    if (q->n_est <= 0 || !(q->B > 0.0f)) return set_err(PT_EINVAL, "n_est and B must be positive");
    hipStream_t stream = (hipStream_t)stream_;
    const uint32_t cap = q->cap ? q->cap : 65536u;
    if (q->mode == PT_RECIP_TABLE) {
        TRY(check_table_query(q, out, ns));
        if (!s) TRY(check_device());
        // the cumulative sums of q in a stream-ordered workspace, released after the estimates
        double *cdf = nullptr;
        if (hipMallocAsync((void **)&cdf, sizeof(double) * ((size_t)q->n + 1), stream) != hipSuccess) {
            (void)hipGetLastError();
            return set_err(PT_ENOMEM, "workspace of %d doubles", q->n + 1);
        }
        k_table_cdf<<<1, 1024, 0, stream>>>(q->q_dev, q->n, cdf);
        k_recip_table<<<blocks(q->n_est, 256), 256, 0, stream>>>(q->f_dev, cdf, q->n, q->B, q->n_est, q->estimator,
                                                                 q->booth_r, q->seed, cap, out, ns);
        HIPCHK(hipFreeAsync(cdf, stream));
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
    PT_STK(s, k_trace_closest, blocks(n, WG), WG, stream, s->S, rays, n, t, prim);
    HIPCHK(hipGetLastError());
    return PT_OK;
}

extern "C" pt_status pt_mlp_param_count(const pt_scene *s, int32_t *count)
{
    if (!s || !count) return set_err(PT_EINVAL, "null argument");
    if (!s->subspaces_ready) return set_err(PT_ESTATE, "pt_build_subspaces must run first");
    *count = (int32_t)mlp_off(s->n_spec + MLP_VMF).n;
    return PT_OK;
}

extern "C" pt_status pt_mlp_set_params(pt_scene *s, const float *host, int32_t count, void *stream_)
{
    if (!s || !host) return set_err(PT_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream_;
    TRY(ensure_mlp(s, st));
    if (count != s->mlp_np) return set_err(PT_EINVAL, "parameter count %d, expected %d", count, s->mlp_np);
    const size_t n = (size_t)count;
    HIPCHK(hipMemcpyAsync(s->mw, host, n * sizeof(float), hipMemcpyHostToDevice, st));
    k_to_bf16<<<blocks((long)n, 256), 256, 0, st>>>(s->mw, s->mwb, n);
    mlp_transpose(s, st);
    k_fill<<<blocks((long)n, 256), 256, 0, st>>>(s->mg, 0.0f, n);
    k_fill<<<blocks((long)n, 256), 256, 0, st>>>(s->mm, 0.0f, n);
    k_fill<<<blocks((long)n, 256), 256, 0, st>>>(s->mv, 0.0f, n);
    k_set_counter<<<1, 1, 0, st>>>(s->cnt, C_MLP_T, 0ull);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return PT_OK;
}

extern "C" pt_status pt_mlp_get_params(pt_scene *s, float *host, int32_t count, void *stream_)
{
    if (!s || !host) return set_err(PT_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream_;
    TRY(ensure_mlp(s, st));
    if (count != s->mlp_np) return set_err(PT_EINVAL, "parameter count %d, expected %d", count, s->mlp_np);
    HIPCHK(hipMemcpyAsync(host, s->mw, (size_t)count * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return PT_OK;
}

extern "C" pt_status pt_mlp_forward(pt_scene *s, const float *feat, int32_t n, float *out, void *stream_)
{
    if (!s || !feat || !out) return set_err(PT_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream_;
    TRY(ensure_mlp(s, st));
    if (n < 1 || n > s->mlp_rows) return set_err(PT_EINVAL, "n out of range [1, %d]", s->mlp_rows);
    const MlpOff o = mlp_off(s->mlp_nout);
    k_mlp_enc_feat<<<blocks(n, 256), 256, 0, st>>>(feat, n, s->cnt, -1, s->mx);
    mlp_forward(s, n, s->cnt, -1, out, 0, s->mlp_nout, st);
    k_add_bias<<<blocks((long)n * s->mlp_nout, 256), 256, 0, st>>>(out, s->mw + o.b4, n, s->mlp_nout);
    HIPCHK(hipGetLastError());
    return PT_OK;
}

extern "C" pt_status pt_mlp_train_step(pt_scene *s, const float *feat, const int32_t *label, const float *weight,
                                       int32_t n, const float *feat_dir, const float *dir, const float *weight_dir,
                                       int32_t n_dir, float lr, float *grad_host, void *stream_)
{
    if (!s || (n > 0 && (!feat || !label || !weight)) || (n_dir > 0 && (!feat_dir || !dir || !weight_dir)))
        return set_err(PT_EINVAL, "null argument");
    if (n < 0 || n > MLP_CAP || n_dir < 0 || n_dir > MLP_CAP || n + n_dir < 1)
        return set_err(PT_EINVAL, "n and n_dir out of range [0, %d], not both 0", MLP_CAP);
    if (!(lr > 0.0f)) return set_err(PT_EINVAL, "lr must be positive");
    hipStream_t st = (hipStream_t)stream_;
    TRY(ensure_mlp(s, st));
    // the caller's arrays as this step's training batch
    MlpTrain T = s->MT;
    T.feat = const_cast<float *>(feat); T.label = const_cast<int *>(label); T.weight = const_cast<float *>(weight);
    T.vfeat = const_cast<float *>(feat_dir); T.vdir = const_cast<float *>(dir);
    T.vweight = const_cast<float *>(weight_dir);
    k_set_counter<<<1, 1, 0, st>>>(s->cnt, C_MLP_N, (unsigned long long)n);
    k_set_counter<<<1, 1, 0, st>>>(s->cnt, C_MLP_NV, (unsigned long long)n_dir);
    k_mlp_rows<<<1, 1, 0, st>>>(s->cnt, MLP_CAP);
    k_fill<<<1, 64, 0, st>>>(T.wsum, 0.0f, 1);
    k_fill<<<1, 64, 0, st>>>(T.vwsum, 0.0f, 1);
    if (n > 0) k_sum1<<<1, 256, 0, st>>>(weight, n, T.wsum);
    if (n_dir > 0) k_sum1<<<1, 256, 0, st>>>(weight_dir, n_dir, T.vwsum);
    k_mlp_enc_train<<<blocks(n + n_dir, 256), 256, 0, st>>>(T, s->cnt, s->mx);
    mlp_backward(s, T, st);
    if (grad_host) {
        HIPCHK(hipMemcpyAsync(grad_host, s->mg, (size_t)s->mlp_np * sizeof(float), hipMemcpyDeviceToHost, st));
    }
    mlp_adam(s, lr, st);
    k_set_counter<<<1, 1, 0, st>>>(s->cnt, C_MLP_N, 0ull);
    k_set_counter<<<1, 1, 0, st>>>(s->cnt, C_MLP_NV, 0ull);
    k_set_counter<<<1, 1, 0, st>>>(s->cnt, C_MLP_ROWS, 0ull);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return PT_OK;
}

extern "C" pt_status pt_vmf_sample(const float *raw_dev, int32_t n, uint32_t seed, float *dir_dev, float *pdf_dev,
                                   void *stream_)
{
    if (!raw_dev || !dir_dev || !pdf_dev || n < 0) return set_err(PT_EINVAL, "bad argument");
    if (n == 0) return PT_OK;
    TRY(check_device());
    k_vmf_hook<<<blocks(n, 256), 256, 0, (hipStream_t)stream_>>>(raw_dev, n, seed, dir_dev, pdf_dev);
    HIPCHK(hipGetLastError());
    return PT_OK;
}

extern "C" pt_status pt_render_scenes(pt_scene *const *scenes, const pt_iter_params *params, int32_t n, uint32_t n_iter,
                                      float *const *acc, float *const *acc2, void *stream_)
{
    if (!scenes || !params || !acc || n <= 0 || n > 64) return set_err(PT_EINVAL, "bad scene batch (1 .. 64 scenes)");
    if (n_iter == 0) return set_err(PT_EINVAL, "n_iter must be positive");
    for (int i = 0; i < n; ++i) {
        TRY(check_params(scenes[i], &params[i], acc[i]));
        if (params[i].flags & PT_FLAG_TIMING) return set_err(PT_EINVAL, "PT_FLAG_TIMING cannot be captured");
        for (int j = 0; j < i; ++j)
            if (scenes[j] == scenes[i]) return set_err(PT_EINVAL, "a scene appears twice in the batch");
    }
    hipStream_t stream = (hipStream_t)stream_;
    pt_scene *own = scenes[0];
    for (int i = 0; i < n; ++i)
        if (params[i].flags & PT_FLAG_MLP) {
            TRY(ensure_mlp(scenes[i], stream));
            HIPCHK(hipStreamSynchronize(stream));
        }
    // the graph depends on every scene, its parameters but the iteration index, and the buffers
    std::vector<char> k;
    for (int i = 0; i < n; ++i) {
        pt_iter_params key = params[i];
        key.iteration = 0;
        const pt_scene *sp = scenes[i];
        float *a = acc[i], *b = acc2 ? acc2[i] : nullptr;
        k.insert(k.end(), (const char *)&sp, (const char *)&sp + sizeof(sp));
        k.insert(k.end(), (const char *)&key, (const char *)&key + sizeof(key));
        k.insert(k.end(), (const char *)&a, (const char *)&a + sizeof(a));
        k.insert(k.end(), (const char *)&b, (const char *)&b + sizeof(b));
        k.insert(k.end(), (const char *)&sp->tune_budget, (const char *)&sp->tune_budget + sizeof(uint32_t));
        k.insert(k.end(), (const char *)&sp->tune_gen_grid, (const char *)&sp->tune_gen_grid + sizeof(int));
        k.insert(k.end(), (const char *)&sp->gen, (const char *)&sp->gen + sizeof(sp->gen));
        k.insert(k.end(), (const char *)&sp->queue_chunk, (const char *)&sp->queue_chunk + sizeof(int));
        k.insert(k.end(), (const char *)&sp->ext_wg, (const char *)&sp->ext_wg + sizeof(int));
        k.insert(k.end(), (const char *)&sp->ahead, (const char *)&sp->ahead + sizeof(int));
        k.insert(k.end(), (const char *)&sp->refill, (const char *)&sp->refill + sizeof(int));
    }
    if (!own->mgexec || k != own->mgkey) {
        ++own->n_captures;
        if (own->mgexec) { HIPCHK(hipGraphExecDestroy(own->mgexec)); own->mgexec = nullptr; }
        if (!own->cap_stream) HIPCHK(hipStreamCreateWithFlags(&own->cap_stream, hipStreamNonBlocking));
        while ((int)own->mstreams.size() < n) {
            hipStream_t q;
            HIPCHK(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
            own->mstreams.push_back(q);
        }
        // stage A of every scene in one persistent launch: the jobs (device copies of what k_recip
        // takes per scene) are written before the capture
        // (one instance walks one tree width: the scenes must agree on it, else every branch keeps
        // its own stage A; 32-bit stack entries when any scene needs them)
        bool multi = false, same = true, booth = false, wide = false;
        for (int i = 0; i < n; ++i) {
            const pt_scene *sp = scenes[i];
            const pt_iter_params *q = &params[i];
            const bool conn = (q->flags & PT_FLAG_SPC) != 0, ltr = (q->flags & PT_FLAG_LT) != 0;
            const int lmax = (conn || ltr) ? q->max_depth : std::min(q->max_depth - 1, PT_LMAX);
            multi |= (q->flags & PT_FLAG_PROXY) && lmax >= 2;
            same &= sp->bvh_cur == own->bvh_cur;
            wide |= !sp->stk16;
            booth |= (q->flags & PT_FLAG_BOOTH) && q->booth_r > 0.0f;
        }
        multi = multi && same && n > 1;
        if (multi) {
            if (!own->mjobs) {
                HIPCHK(hipMalloc(&own->mjobs, 64 * sizeof(RecipJob)));
                HIPCHK(hipMalloc(&own->mbase, 65 * sizeof(uint32_t)));
                HIPCHK(hipMalloc(&own->mwork, sizeof(unsigned long long)));
            }
            std::vector<RecipJob> jobs((size_t)n);
            for (int i = 0; i < n; ++i) {
                pt_scene *sp = scenes[i];
                const pt_iter_params *q = &params[i];
                RecipJob &J = jobs[(size_t)i];
                J.S = sp->S;
                J.cand = sp->cand; J.final_ = sp->final_; J.order = sp->order; J.runmax = sp->runmax;
                J.longq = sp->chq[0]; J.cnt = sp->cnt; J.repeats = q->recip_repeats; J.seed = q->seed;
                J.n1 = stage_a_n1(q); J.budget = sp->tune_budget;
                J.booth_r = (q->flags & PT_FLAG_BOOTH) ? q->booth_r : 0.0f;
            }
            HIPCHK(hipMemcpy(own->mjobs, jobs.data(), jobs.size() * sizeof(RecipJob), hipMemcpyHostToDevice));
        }
        while ((int)own->mevents.size() < 2 * n + 2) {
            hipEvent_t e;
            HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            own->mevents.push_back(e);
        }
        // fork: every scene's iteration on its own stream, joined back into the capture stream (in
        // two parts around the shared stage A when there is one)
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(own->cap_stream, hipStreamCaptureModeThreadLocal));
        pt_status st = PT_OK;
        hipError_t e = hipSuccess;
        for (int part = multi ? 1 : 0; part <= (multi ? 2 : 0) && st == PT_OK && e == hipSuccess; ++part) {
            hipEvent_t *ev = own->mevents.data() + (part == 2 ? n + 1 : 0);
            e = hipEventRecord(ev[0], own->cap_stream);
            for (int i = 0; i < n && st == PT_OK && e == hipSuccess; ++i) {
                e = hipStreamWaitEvent(own->mstreams[i], ev[0], 0);
                if (e != hipSuccess) break;
                st = enqueue_iteration(scenes[i], &params[i], acc[i], acc2 ? acc2[i] : nullptr, own->mstreams[i], true,
                                       part);
                if (st != PT_OK) break;
                e = hipEventRecord(ev[i + 1], own->mstreams[i]);
                if (e == hipSuccess) e = hipStreamWaitEvent(own->cap_stream, ev[i + 1], 0);
            }
            if (part == 1 && st == PT_OK && e == hipSuccess) {
                k_multi_base<<<1, 64, 0, own->cap_stream>>>(own->mjobs, n, own->mbase, own->mwork);
                const int grid = own->persist_wg, chunk = std::max(1, own->queue_chunk);
                const MultiStk ms{!wide, own->bvh_cur};
                if (booth) PT_STK_B(&ms, k_recip_multi, true, grid, 64 * RW, own->cap_stream, own->mjobs, n, own->mbase,
                                    own->mwork, chunk, own->ahead);
                else PT_STK_B(&ms, k_recip_multi, false, grid, 64 * RW, own->cap_stream, own->mjobs, n, own->mbase,
                              own->mwork, chunk, own->ahead);
                e = hipGetLastError();
            }
        }
        const hipError_t e2 = hipStreamEndCapture(own->cap_stream, &g);
        if (st != PT_OK) { if (g) (void)hipGraphDestroy(g); return st; }
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return set_err(PT_EDEVICE, "multi-scene capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
        }
        e = hipGraphInstantiate(&own->mgexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) { own->mgexec = nullptr; return set_err(PT_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e)); }
        own->mgkey = k;
    }
    for (int i = 0; i < n; ++i)
        k_iter<<<1, 1, 0, stream>>>(scenes[i]->cnt, params[i].iteration - 1u, 0, params[i].train_iters, nullptr, 0);
    for (uint32_t it = 0; it < n_iter; ++it) HIPCHK(hipGraphLaunch(own->mgexec, stream));
    HIPCHK(hipGetLastError());
    return PT_OK;
}

extern "C" pt_status pt_get_schedule(const pt_scene *s, pt_tune_result *k)
{
    if (!s || !k) return set_err(PT_EINVAL, "null argument");
    *k = pt_tune_result{};
    k->stage_a_budget = s->tune_budget;
    k->round_grid = s->tune_gen_grid;
    k->ext_wg = s->ext_wg;
    k->queue_chunk = s->queue_chunk;
    k->bvh_width = s->bvh_cur;
    k->stage_a_ahead = s->ahead;
    k->stage_a_refill = s->refill;
    return PT_OK;
}

extern "C" pt_status pt_set_schedule(pt_scene *s, const pt_tune_result *k)
{
    if (!s || !k) return set_err(PT_EINVAL, "null argument");
    const uint32_t b = k->stage_a_budget;
    if (b < 64u || b > (1u << 20)) return set_err(PT_EINVAL, "stage_a_budget %u out of range", b);
    if (k->round_grid < 64 || k->round_grid > 65536) return set_err(PT_EINVAL, "round_grid %d out of range", k->round_grid);
    if (k->ext_wg != 64 && k->ext_wg != 128 && k->ext_wg != 256) return set_err(PT_EINVAL, "ext_wg must be 64, 128 or 256");
    if (k->queue_chunk < 1 || k->queue_chunk > 64) return set_err(PT_EINVAL, "queue_chunk %d out of range", k->queue_chunk);
    if (k->stage_a_ahead < 1 || k->stage_a_ahead > 2) return set_err(PT_EINVAL, "stage_a_ahead must be 1 or 2");
    if (k->stage_a_refill != 0 && k->stage_a_refill != 1) return set_err(PT_EINVAL, "stage_a_refill must be 0 or 1");
    if (k->bvh_width != 4 && k->bvh_width != 8) return set_err(PT_EINVAL, "bvh_width must be 4 or 8");
    if ((k->bvh_width == 4 && !s->has4) || (k->bvh_width == 8 && !s->has8))
        return set_err(PT_EUNSUPPORTED, "the scene holds no %d-wide tree", k->bvh_width);
    s->tune_budget = b;
    s->tune_gen_grid = k->round_grid;
    s->ext_wg = k->ext_wg;
    s->queue_chunk = k->queue_chunk;
    s->ahead = k->stage_a_ahead;
    s->refill = k->stage_a_refill;
    s->bvh_cur = k->bvh_width;
    s->stack_need = s->bvh_cur == 8 ? s->stack_need8 : s->stack_need4;
    s->bvh_depth = s->bvh_cur == 8 ? s->bvh_depth8 : s->bvh_depth4;
    s->gen = next_generation();
    return PT_OK;
}

extern "C" pt_status pt_autotune(pt_scene *s, const pt_iter_params *p, float *acc, float *acc2, pt_tune_result *out,
                                 void *stream_)
{
    TRY(check_params(s, p, acc));
    if (!out) return set_err(PT_EINVAL, "null result");
    hipStream_t stream = (hipStream_t)stream_;
    if (p->flags & PT_FLAG_MLP) TRY(ensure_mlp(s, stream));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    pt_iter_params q = *p;
    q.flags &= ~(uint32_t)(PT_FLAG_TIMING | PT_FLAG_COUNT);
    int used = 0;
    // iteration time with the scene's current knobs: one iteration to settle, three timed
    auto timed = [&](float &ms) -> pt_status {
        q.iteration = p->iteration + (uint32_t)used++;
        pt_status st = enqueue_iteration(s, &q, acc, acc2, stream, false);
        if (st != PT_OK) return st;
        if (hipEventRecord(e0, stream) != hipSuccess) return set_err(PT_EDEVICE, "event record failed");
        for (int r = 0; r < 3; ++r) {
            q.iteration = p->iteration + (uint32_t)used++;
            if ((st = enqueue_iteration(s, &q, acc, acc2, stream, false)) != PT_OK) return st;
        }
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return set_err(PT_EDEVICE, "event timing failed");
        ms *= 1.0f / 3.0f;
        return PT_OK;
    };
    auto set_width = [&](int w) {
        s->bvh_cur = w;
        s->stack_need = w == 8 ? s->stack_need8 : s->stack_need4;
        s->bvh_depth = w == 8 ? s->bvh_depth8 : s->bvh_depth4;
    };
    const uint32_t b0 = s->tune_budget;
    const int g0 = s->tune_gen_grid, w0 = s->ext_wg, c0 = s->queue_chunk, v0 = s->bvh_cur;
    pt_status st = PT_OK;
    float dflt = 0.0f, best = 3.0e38f, ms = 0.0f;
    // coordinate descent, each knob timed with the choices made before it: the BVH width (when
    // both trees are there), the chain schedule (stage-A budget x round grid), the extension
    // workgroup size, the queue chunk
    int bv = v0;
    // the incumbent twice (the faster counts), so that one slow measurement at the start (a
    // transient of the device) does not make every alternative look better
    st = timed(dflt);
    if (st == PT_OK && (st = timed(ms)) == PT_OK) dflt = std::min(dflt, ms);
    best = dflt;
    if (st == PT_OK && s->has4 && s->has8) {
        set_width(v0 == 4 ? 8 : 4);
        if ((st = timed(ms)) == PT_OK && ms < best) { best = ms; bv = s->bvh_cur; }
        set_width(bv);
    }
    static const uint32_t budgets[5] = {512u, 1024u, 2048u, 4096u, 8192u};
    static const int grids[3] = {1024, 2048, 8192};
    uint32_t bb = b0;
    int bg = g0;
    float best_s = 3.0e38f;
    for (int bi = 0; bi < 5 && st == PT_OK; ++bi)
        for (int gi = 0; gi < 3 && st == PT_OK; ++gi) {
            s->tune_budget = budgets[bi];
            s->tune_gen_grid = grids[gi];
            if ((st = timed(ms)) == PT_OK && ms < best_s) { best_s = ms; bb = budgets[bi]; bg = grids[gi]; }
        }
    s->tune_budget = bb;
    s->tune_gen_grid = bg;
    static const int wgs[3] = {64, 128, 256};
    int bw = w0;
    float best_w = 3.0e38f;
    for (int wi = 0; wi < 3 && st == PT_OK; ++wi) {
        s->ext_wg = wgs[wi];
        if ((st = timed(ms)) == PT_OK && ms < best_w) { best_w = ms; bw = wgs[wi]; }
    }
    s->ext_wg = bw;
    static const int chunks[3] = {1, 2, 4};
    int bc = c0;
    float best_c = 3.0e38f;
    for (int ci = 0; ci < 3 && st == PT_OK; ++ci) {
        s->queue_chunk = chunks[ci];
        if ((st = timed(ms)) == PT_OK && ms < best_c) { best_c = ms; bc = chunks[ci]; }
    }
    s->queue_chunk = bc;
    // how far a stage-A lane may run ahead of the chain's oldest unconsumed step
    const int a0 = s->ahead;
    int ba = a0;
    float best_a = 3.0e38f;
    for (int ai = 1; ai <= 2 && st == PT_OK; ++ai) {
        s->ahead = ai;
        if ((st = timed(ms)) == PT_OK && ms < best_a) { best_a = ms; ba = ai; }
    }
    s->ahead = ba;
    // and whether stage A refills its walks node by node (4-wide trees only)
    const int r0 = s->refill;
    int br = r0;
    float best_r = 3.0e38f;
    for (int ri = 0; ri <= (s->bvh_cur == 4 ? 1 : 0) && st == PT_OK; ++ri) {
        s->refill = ri;
        if ((st = timed(ms)) == PT_OK && ms < best_r) { best_r = ms; br = ri; }
    }
    s->refill = br;
    // the chosen knobs against the ones the descent started from, timed alternately twice each:
    // a transient slowdown during the descent must not leave a slower schedule in place
    float ms_chosen = 3.0e38f, ms_start = 3.0e38f;
    for (int r = 0; r < 2 && st == PT_OK; ++r) {
        s->tune_budget = b0; s->tune_gen_grid = g0; s->ext_wg = w0; s->queue_chunk = c0; s->ahead = a0;
        s->refill = r0;
        set_width(v0);
        if ((st = timed(ms)) != PT_OK) break;
        ms_start = std::min(ms_start, ms);
        s->tune_budget = bb; s->tune_gen_grid = bg; s->ext_wg = bw; s->queue_chunk = bc; s->ahead = ba;
        s->refill = br;
        set_width(bv);
        if ((st = timed(ms)) != PT_OK) break;
        ms_chosen = std::min(ms_chosen, ms);
    }
    if (st == PT_OK && ms_start < ms_chosen) {
        bb = b0; bg = g0; bw = w0; bc = c0; ba = a0; br = r0; bv = v0;
        s->tune_budget = bb; s->tune_gen_grid = bg; s->ext_wg = bw; s->queue_chunk = bc; s->ahead = ba;
        s->refill = br;
        set_width(bv);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PT_OK) {
        s->tune_budget = b0; s->tune_gen_grid = g0; s->ext_wg = w0; s->queue_chunk = c0; s->ahead = a0;
        s->refill = r0;
        set_width(v0);
        return st;
    }
    s->gen = next_generation();
    out->stage_a_budget = bb;
    out->round_grid = bg;
    out->ext_wg = bw;
    out->queue_chunk = bc;
    out->stage_a_ahead = ba;
    out->stage_a_refill = br;
    out->bvh_width = s->bvh_cur;
    out->ms_best = std::min(ms_start, ms_chosen);
    out->ms_previous = std::min(dflt, ms_start);
    out->iterations_rendered = (uint32_t)used;
    return PT_OK;
}

extern "C" pt_status pt_scene_totals(pt_scene *s, pt_totals *out, int32_t reset, void *stream_)
{
    if (!s || !out) return set_err(PT_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream_;
    unsigned long long t[TOT_COUNT];
    HIPCHK(hipMemcpyAsync(t, s->tot, sizeof(t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    out->iterations = (double)t[TOT_ITERS];
    out->n_nan = (double)t[TOT_NAN];
    out->n_recip_truncated = (double)t[TOT_TRUNC];
    out->n_proxy_valid = (double)t[TOT_PROXY_VALID];
    out->n_recip_samples = (double)t[TOT_RECIP_SAMPLES];
    out->n_cand = (double)t[TOT_CAND];
    out->captures = (double)s->n_captures;
    out->bvh_stack_need = (double)s->stack_need;
    out->bvh_depth = (double)s->bvh_depth;
    if (reset) {
        k_fill_u64<<<1, 64, 0, st>>>(s->tot, 0ull, TOT_COUNT);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
    }
    return PT_OK;
}

extern "C" pt_status pt_iteration_times(pt_scene *s, uint32_t first, int32_t n, double *ms, void *stream_)
{
    if (!s || !ms || n < 0 || n > PT_TS_CAP) return set_err(PT_EINVAL, "bad argument (n <= %d)", PT_TS_CAP);
    hipStream_t st = (hipStream_t)stream_;
    std::vector<long long> t(2 * PT_TS_CAP);
    HIPCHK(hipMemcpyAsync(t.data(), s->ts, t.size() * sizeof(long long), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) {
        const uint32_t slot = (first + (uint32_t)i) % PT_TS_CAP;
        const long long a = t[2 * slot], b = t[2 * slot + 1];
        ms[i] = (b > a && a > 0 && s->wall_khz > 0) ? (double)(b - a) / (double)s->wall_khz : -1.0;
    }
    return PT_OK;
}

extern "C" pt_status pt_selection_tables(pt_scene *s, int32_t which, int32_t n_rows, int32_t n_cols,
                                         int32_t *n_nonempty, int32_t *nonempty, float *prob, int32_t *alias,
                                         float *pmf, float *weights, void *stream_)
{
    if (!s || !n_nonempty || !nonempty || !prob || !alias || !pmf || !weights) return set_err(PT_EINVAL, "null argument");
    if (!s->subspaces_ready) return set_err(PT_ESTATE, "pt_build_subspaces must run first");
    if (which != 0 && which != 1) return set_err(PT_EINVAL, "which must be 0 (Gamma) or 1 (Q)");
    const int R = s->n_eye, C = which == 0 ? s->n_spec : s->n_lsub;
    if (n_rows != R || n_cols != C) return set_err(PT_EINVAL, "table is %d x %d, not %d x %d", R, C, n_rows, n_cols);
    hipStream_t st = (hipStream_t)stream_;
    const size_t n = (size_t)R * C;
    HIPCHK(hipMemcpyAsync(n_nonempty, which == 0 ? s->n_ne : s->ln_ne, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(nonempty, which == 0 ? s->nonempty : s->lnonempty, C * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(prob, which == 0 ? s->al_prob : s->q_alprob, n * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(alias, which == 0 ? s->al_idx : s->q_alidx, n * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(pmf, which == 0 ? s->al_pmf : s->q_alpmf, n * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(weights, which == 0 ? s->gamma_frz : s->qfrz, n * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return PT_OK;
}

extern "C" pt_status pt_philox(const uint32_t *in_dev, int32_t n, uint32_t *out_dev, void *stream_)
{
    if (!in_dev || !out_dev || n < 0) return set_err(PT_EINVAL, "bad argument");
    if (n == 0) return PT_OK;
    TRY(check_device());
    k_philox_hook<<<blocks(n, 256), 256, 0, (hipStream_t)stream_>>>(in_dev, n, out_dev);
    HIPCHK(hipGetLastError());
    return PT_OK;
}

extern "C" pt_status pt_bvh_stats(const float *tri, int32_t n_tri, int32_t width, int32_t *n_nodes,
                                  int32_t *stack_need, int32_t *depth)
{
    if (!tri || n_tri <= 0 || !n_nodes || !stack_need || !depth) return set_err(PT_EINVAL, "bad argument");
    if (width != 4 && width != 8) return set_err(PT_EINVAL, "width must be 4 or 8");
    try {
        std::vector<BNode> nodes;
        std::vector<BNode8> nodes8;
        std::vector<int> order;
        pt_build_bvh(tri, n_tri, nodes, width == 8 ? &nodes8 : nullptr, order);
        int dp = 0;
        *stack_need = width == 8 ? pt_bvh8_stack_need(nodes8, &dp) : pt_bvh4_stack_need(nodes, &dp);
        *depth = dp;
        *n_nodes = (int32_t)(width == 8 ? nodes8.size() : nodes.size());
        return PT_OK;
    } catch (const std::exception &e) {
        return set_err(PT_ENOMEM, "host exception: %s", e.what());
    }
}

// ---------------------------------------------------------------------------------------------
// Photon planes (single scattering, Section 6.7)
struct pt_planes {
    PlaneDev P{};
    uint32_t *alias = nullptr;
    float *pk = nullptr;
    float *z = nullptr;
    PlaneRec *planes = nullptr;
    unsigned long long *cnt = nullptr;
    int max_planes = 0;
    ~pt_planes()
    {
        (void)hipFree(alias); (void)hipFree(pk); (void)hipFree(z); (void)hipFree(planes); (void)hipFree(cnt);
    }
};

extern "C" pt_status pt_planes_create(const pt_planes_desc *d, void *stream_, pt_planes **out)
{
    if (!d || !out) return set_err(PT_EINVAL, "null argument");
    *out = nullptr;
    const float *U = d->light_u, *V = d->light_v;
    const float uu = U[0] * U[0] + U[1] * U[1] + U[2] * U[2], vv = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
    const float uv = U[0] * V[0] + U[1] * V[1] + U[2] * V[2];
    if (!(fabsf(uu - 1.0f) < 1e-4f && fabsf(vv - 1.0f) < 1e-4f && fabsf(uv) < 1e-4f))
        return set_err(PT_EINVAL, "light axes must be orthonormal");
    if (!(d->light_eu > 0.0f && d->light_ev > 0.0f)) return set_err(PT_EINVAL, "light half extents must be positive");
    if (!(d->sigma_s >= 0.0f && d->sigma_t >= 0.0f && d->t_max > 0.0f))
        return set_err(PT_EINVAL, "need sigma_s >= 0, sigma_t >= 0, t_max > 0");
    if (d->width <= 0 || d->height <= 0 || (long)d->width * d->height > (1L << 26))
        return set_err(PT_EINVAL, "bad image size %d x %d", d->width, d->height);
    if (d->max_planes <= 0 || d->max_planes > PT_PLANES_MAX)
        return set_err(PT_EINVAL, "max_planes must be in [1, %d]", PT_PLANES_MAX);
    const float *cam = d->camera;
    const float3 cp = make_float3(cam[0], cam[1], cam[2]), tg = make_float3(cam[3], cam[4], cam[5]), up = make_float3(cam[6], cam[7], cam[8]);
    float3 fw = make_float3(tg.x - cp.x, tg.y - cp.y, tg.z - cp.z);
    const float lf = sqrtf(fw.x * fw.x + fw.y * fw.y + fw.z * fw.z);
    float3 rt = make_float3(fw.y * up.z - fw.z * up.y, fw.z * up.x - fw.x * up.z, fw.x * up.y - fw.y * up.x);
    const float lr = sqrtf(rt.x * rt.x + rt.y * rt.y + rt.z * rt.z);
    if (!(lf > 0.0f && lr > 0.0f && cam[9] > 0.0f && cam[9] < 180.0f))
        return set_err(PT_EINVAL, "degenerate camera");
    TRY(check_device());
    hipStream_t st = (hipStream_t)stream_;
    pt_planes *p = new pt_planes();
    PlaneDev &P = p->P;
    P.c = make_float3(d->light_c[0], d->light_c[1], d->light_c[2]);
    P.U = make_float3(U[0], U[1], U[2]);
    P.V = make_float3(V[0], V[1], V[2]);
    P.N = make_float3(U[1] * V[2] - U[2] * V[1], U[2] * V[0] - U[0] * V[2], U[0] * V[1] - U[1] * V[0]);
    P.eu = d->light_eu; P.ev = d->light_ev; P.area = 4.0f * d->light_eu * d->light_ev;
    P.le = make_float3(d->le[0], d->le[1], d->le[2]);
    P.cam_p = cp;
    P.cam_f = make_float3(fw.x / lf, fw.y / lf, fw.z / lf);
    P.cam_r = make_float3(rt.x / lr, rt.y / lr, rt.z / lr);
    P.cam_u = make_float3(P.cam_r.y * P.cam_f.z - P.cam_r.z * P.cam_f.y, P.cam_r.z * P.cam_f.x - P.cam_r.x * P.cam_f.z,
                 P.cam_r.x * P.cam_f.y - P.cam_r.y * P.cam_f.x);
    P.tan_half = tanf(0.5f * cam[9] * 3.14159265358979f / 180.0f);
    P.aspect = (float)d->width / (float)d->height;
    P.ss = d->sigma_s; P.st = d->sigma_t; P.tmax = d->t_max;
    P.w = d->width; P.h = d->height;
    p->max_planes = d->max_planes;
    if (hipMalloc((void **)&p->alias, sizeof(uint32_t) * PL_ENTRIES * PL_BINS) != hipSuccess ||
        hipMalloc((void **)&p->pk, sizeof(float) * PL_ENTRIES * PL_BINS) != hipSuccess ||
        hipMalloc((void **)&p->z, sizeof(float) * PL_ENTRIES) != hipSuccess ||
        hipMalloc((void **)&p->planes, sizeof(PlaneRec) * (size_t)d->max_planes) != hipSuccess ||
        hipMalloc((void **)&p->cnt, sizeof(unsigned long long) * PC_COUNT) != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        return set_err(PT_ENOMEM, "photon-plane buffers");
    }
    P.alias = p->alias; P.pk = p->pk; P.z = p->z;
    k_planes_cache<<<blocks(PL_ENTRIES, 256), 256, 0, st>>>(P, p->alias, p->pk, p->z);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        delete p;
        return set_err(PT_EDEVICE, "photon-plane cache");
    }
    *out = p;
    return PT_OK;
}

extern "C" pt_status pt_planes_render(pt_planes *p, int32_t n_planes, uint32_t iteration, uint32_t seed,
                                      float *acc, float *acc2, pt_planes_stats *stats, void *stream_)
{
    if (!p || !acc) return set_err(PT_EINVAL, "null argument");
    if (n_planes < 0 || n_planes > p->max_planes)
        return set_err(PT_EINVAL, "n_planes %d outside [0, %d]", n_planes, p->max_planes);
    hipStream_t st = (hipStream_t)stream_;
    k_fill_u64<<<1, 64, 0, st>>>(p->cnt, 0ull, PC_COUNT);
    if (n_planes > 0) k_planes_gen<<<blocks(n_planes, 256), 256, 0, st>>>(p->P, n_planes, seed, iteration, p->planes);
    k_planes_gather<<<blocks((long)p->P.w * p->P.h, 256), 256, 0, st>>>(p->P, p->planes, n_planes, seed, iteration,
                                                                        acc, acc2, p->cnt);
    HIPCHK(hipGetLastError());
    if (stats) {
        unsigned long long c[PC_COUNT];
        HIPCHK(hipMemcpyAsync(c, p->cnt, sizeof(c), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        stats->n_hits = (double)c[PC_HITS];
        stats->n_samples = (double)c[PC_SAMPLES];
        stats->n_truncated = (double)c[PC_TRUNC];
        stats->n_nan = (double)c[PC_NAN];
    }
    return PT_OK;
}

extern "C" pt_status pt_planes_release(pt_planes *p)
{
    if (!p) return PT_OK;
    (void)hipDeviceSynchronize();
    delete p;
    return PT_OK;
}

extern "C" pt_status pt_proxy_class(const uint8_t *eye, int32_t n_eye, uint32_t light_sig, int32_t j, int32_t u_max,
                                    int32_t general_cv, int32_t *out)
{
    if (!out || n_eye < 0 || (n_eye > 0 && !eye) || j < 0 || j > 15 || u_max < 1 || u_max > 4)
        return set_err(PT_EINVAL, "bad argument");
    uint32_t ph = 0, uu = 0, kk = 0;
    for (int i = 0; i < n_eye; ++i)
        pstate_push(ph, uu, kk, (eye[i] & 1u) != 0, (eye[i] & 2u) != 0, u_max, general_cv != 0);
    *out = light_tail_class(ph, uu, kk, light_sig, j, u_max, general_cv != 0) ? 1 : 0;
    return PT_OK;
}

// ---------------------------------------------------------------------------------------------
// Table-mode reciprocal estimates without allocation. The cumulative sums of q live in this
// file-scope device array instead of a per-call workspace; each device holds its own copy for the
// life of the process. Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): its device address is taken once per device with
// hipGetSymbolAddress and kept in table_scratch_dev.
static __device__ __align__(256) double table_scratch[PT_NOALLOC_TABLE_MAX + 1];   // 8 MiB

namespace {
std::mutex g_table_scratch_mu;
std::vector<double *> g_table_scratch_dev;   // per device ordinal

// the current device's address of table_scratch (looked up on the first call on that device)
pt_status table_scratch_dev(double **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_table_scratch_mu);
    if ((int)g_table_scratch_dev.size() <= dev) g_table_scratch_dev.resize((size_t)dev + 1, nullptr);
    if (!g_table_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(table_scratch));
        if (e != hipSuccess || !p)
            return set_err(PT_EDEVICE, "hipGetSymbolAddress(table_scratch) failed: %s", hipGetErrorString(e));
        g_table_scratch_dev[dev] = (double *)p;
    }
    *out = g_table_scratch_dev[dev];
    return PT_OK;
}
}  // namespace

extern "C" pt_status pt_reciprocal_estimate_noalloc(const pt_recip_query *q, float *out, uint32_t *ns, void *stream_)
{
    TRY(check_table_query(q, out, ns));
    if (q->n > PT_NOALLOC_TABLE_MAX)
        return set_err(PT_EINVAL, "table of %d entries: pt_reciprocal_estimate_noalloc holds at most %d", q->n,
                       PT_NOALLOC_TABLE_MAX);
    TRY(check_device());
    double *cdf = nullptr;
    TRY(table_scratch_dev(&cdf));
    hipStream_t stream = (hipStream_t)stream_;
    const uint32_t cap = q->cap ? q->cap : 65536u;
    // k_table_cdf writes cdf[0 .. n] before k_recip_table reads it, so nothing of an earlier call
    // (a longer table's tail included) is read
    k_table_cdf<<<1, 1024, 0, stream>>>(q->q_dev, q->n, cdf);
    k_recip_table<<<blocks(q->n_est, 256), 256, 0, stream>>>(q->f_dev, cdf, q->n, q->B, q->n_est, q->estimator,
                                                             q->booth_r, q->seed, cap, out, ns);
    HIPCHK(hipGetLastError());
    return PT_OK;
}
