/*
 * FP64 CPU oracle for proxy-sampling BDPT (Su et al., "Proxy Tracing: Unbiased
 * Reciprocal Estimation for Optimized Sampling in BDPT").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The HIP library never
 * links, includes or calls anything here, and this file includes nothing from
 * the HIP tree.
 *
 * It is deliberately plain and slow: double precision throughout, a binary
 * median-split BVH (pinned against brute force), recursion where the paper's
 * algorithms recurse, pthreads only for independent per-pixel / per-path work.
 *
 * What it computes:
 *   - the path integral I = int f dmu of every pixel (Section 3.1, path integral
 *     equation), estimated two ways:
 *       O1  unidirectional path tracing with next-event estimation, balance
 *           heuristic between the two (the plain definition);
 *       O3  plain bidirectional path tracing: one light and one eye sub-path
 *           per pixel sample, every (s, t) strategy, balance-heuristic weights
 *           from explicit products of vertex densities (Section 3.1);
 *       O2  proxy-sampling BDPT: light sub-path cache, incomplete sub-path
 *           candidates, reciprocal estimates of 1/P (Section 5), proxy
 *           connections at the eye's first diffuse vertex; every path that the
 *           proxy strategy can build is scored by it alone, all others by O1's
 *           strategies (a partition of unity, hence valid MIS weights in {0,1});
 *   - the reciprocal estimator of 1/int f (Section 4.2, RRS estimator and
 *     Appendix A, Algorithm "Estimator I~", plus the sign estimator I).
 *
 * Readings of points the paper leaves open are restated next to the code that
 * takes them.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* vectors                                                                   */
/* ------------------------------------------------------------------------- */
typedef struct { double x, y, z; } v3;
static inline v3 vmk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static inline v3 vadd(v3 a, v3 b) { return vmk(a.x + b.x, a.y + b.y, a.z + b.z); }
static inline v3 vsub(v3 a, v3 b) { return vmk(a.x - b.x, a.y - b.y, a.z - b.z); }
static inline v3 vscl(v3 a, double s) { return vmk(a.x * s, a.y * s, a.z * s); }
static inline double vdot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline v3 vcross(v3 a, v3 b) { return vmk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static inline double vlen(v3 a) { return sqrt(vdot(a, a)); }
static inline v3 vnorm(v3 a) { return vscl(a, 1.0 / vlen(a)); }
static inline double vmaxc(v3 a) { return a.x > a.y ? (a.x > a.z ? a.x : a.z) : (a.y > a.z ? a.y : a.z); }
static inline double vcomp(v3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), from its published      */
/* definition: 10 rounds of two 32x32->64 multiplies with Weyl key bumps.    */
/* ------------------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A stream: key = (seed, purpose), counter = (a, b, c, running block). */
typedef struct { uint32_t key[2]; uint32_t ctr[4]; uint32_t buf[4]; int pos; } rng_t;
enum { ST_PT = 1, ST_LIGHT = 2, ST_CAND = 3, ST_RECIP = 4, ST_EYE = 5, ST_PILOT = 6, ST_TABLE = 7, ST_TEST = 8, ST_BDPT = 9 };

static void rng_init(rng_t *r, uint32_t seed, uint32_t purpose, uint32_t a, uint32_t b, uint32_t c)
{
    r->key[0] = seed; r->key[1] = purpose * 0x01000193u + 0x5bd1e995u;
    r->ctr[0] = a; r->ctr[1] = b; r->ctr[2] = c; r->ctr[3] = 0;
    r->pos = 4;
}
static uint32_t rng_u32(rng_t *r)
{
    if (r->pos == 4) { or_philox4x32_10(r->ctr, r->key, r->buf); r->ctr[3]++; r->pos = 0; }
    return r->buf[r->pos++];
}
/* uniform double in [0,1) with 53 random bits */
static double rng_u01(rng_t *r)
{
    uint32_t a = rng_u32(r) >> 5, b = rng_u32(r) >> 6;
    return ((double)a * 67108864.0 + (double)b) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------- */
/* scene                                                                     */
/* ------------------------------------------------------------------------- */
enum { MAT_LAMBERT = 0, MAT_CONDUCTOR = 1, MAT_DIELECTRIC = 2 };

typedef struct {
    int type;
    double rgb[3];
    double rough, alpha, ior;
    double le[3];
    int textured, emissive;
    int spec;   /* S vertex: conductor or dielectric with roughness < 0.2 (Section 6.1) */
    int delta;  /* Dirac BSDF: smooth dielectric, or conductor of roughness exactly 0 */
} mat_t;

typedef struct { v3 v0, e1, e2, n; double area; int mat; double uv[6]; } tri_t;
typedef struct { double lo[3], hi[3]; int left, right, first, count; } bnode_t;

typedef struct {
    int ntri; tri_t *tri;
    int nmat; mat_t *mat;
    int tw, th; double *tex;
    v3 cam_p, cam_f, cam_r, cam_u; double tan_half; int W, H;
    int nem; int *em_tri; double *em_cdf; double em_area;
    bnode_t *nodes; int nnodes; int *prim;
    double tmin;
} scene_t;

static void tri_bounds(const tri_t *t, double lo[3], double hi[3])
{
    v3 p[3] = {t->v0, vadd(t->v0, t->e1), vadd(t->v0, t->e2)};
    for (int k = 0; k < 3; ++k) { lo[k] = 1e300; hi[k] = -1e300; }
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) {
            double c = vcomp(p[i], k);
            if (c < lo[k]) lo[k] = c;
            if (c > hi[k]) hi[k] = c;
        }
}

/* binary BVH, median split of centroids along the widest centroid axis */
static double *g_cent; static int g_axis;
static int cmp_cent(const void *a, const void *b)
{
    double ca = g_cent[3 * *(const int *)a + g_axis], cb = g_cent[3 * *(const int *)b + g_axis];
    return ca < cb ? -1 : (ca > cb ? 1 : (*(const int *)a - *(const int *)b));
}
static int bvh_build(scene_t *s, double *cent, int first, int count)
{
    int id = s->nnodes++;
    bnode_t *nd = &s->nodes[id];
    for (int k = 0; k < 3; ++k) { nd->lo[k] = 1e300; nd->hi[k] = -1e300; }
    double clo[3] = {1e300, 1e300, 1e300}, chi[3] = {-1e300, -1e300, -1e300};
    for (int i = first; i < first + count; ++i) {
        double lo[3], hi[3];
        tri_bounds(&s->tri[s->prim[i]], lo, hi);
        for (int k = 0; k < 3; ++k) {
            if (lo[k] < nd->lo[k]) nd->lo[k] = lo[k];
            if (hi[k] > nd->hi[k]) nd->hi[k] = hi[k];
            double c = cent[3 * s->prim[i] + k];
            if (c < clo[k]) clo[k] = c;
            if (c > chi[k]) chi[k] = c;
        }
    }
    if (count <= 4) { nd->first = first; nd->count = count; nd->left = nd->right = -1; return id; }
    int axis = 0;
    for (int k = 1; k < 3; ++k) if (chi[k] - clo[k] > chi[axis] - clo[axis]) axis = k;
    g_cent = cent; g_axis = axis;
    qsort(s->prim + first, (size_t)count, sizeof(int), cmp_cent);
    int half = count / 2;
    int l = bvh_build(s, cent, first, half);
    int r = bvh_build(s, cent, first + half, count - half);
    nd = &s->nodes[id];
    nd->left = l; nd->right = r; nd->count = 0; nd->first = -1;
    return id;
}

void *or_scene_new(const float *tri, int ntri, const int *tri_mat, const float *tri_uv,
                   const float *mats, int nmat, const float *tex, int tw, int th,
                   const float *cam, int W, int H)
{
    scene_t *s = (scene_t *)calloc(1, sizeof(scene_t));
    s->ntri = ntri; s->nmat = nmat; s->tw = tw; s->th = th; s->W = W; s->H = H;
    s->mat = (mat_t *)calloc((size_t)nmat, sizeof(mat_t));
    for (int m = 0; m < nmat; ++m) {
        const float *r = mats + 16 * m;
        mat_t *mt = &s->mat[m];
        mt->type = (int)r[0];
        for (int k = 0; k < 3; ++k) { mt->rgb[k] = r[1 + k]; mt->le[k] = r[6 + k]; }
        mt->rough = r[4];
        mt->alpha = r[4] * (double)r[4];
        if (mt->alpha < 1e-4) mt->alpha = 1e-4;
        mt->ior = r[5];
        mt->textured = r[9] != 0.0f;
        mt->emissive = (r[6] > 0 || r[7] > 0 || r[8] > 0);
        mt->spec = (mt->type == MAT_CONDUCTOR || mt->type == MAT_DIELECTRIC) && mt->rough < 0.2;
        mt->delta = (mt->type == MAT_DIELECTRIC) || (mt->type == MAT_CONDUCTOR && mt->rough == 0.0);
    }
    s->tex = (double *)malloc(sizeof(double) * (size_t)tw * th);
    for (int i = 0; i < tw * th; ++i) s->tex[i] = tex[i];
    s->tri = (tri_t *)calloc((size_t)ntri, sizeof(tri_t));
    double scene_lo[3] = {1e300, 1e300, 1e300}, scene_hi[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < ntri; ++i) {
        const float *p = tri + 9 * i;
        v3 a = vmk(p[0], p[1], p[2]), b = vmk(p[3], p[4], p[5]), c = vmk(p[6], p[7], p[8]);
        tri_t *t = &s->tri[i];
        t->v0 = a; t->e1 = vsub(b, a); t->e2 = vsub(c, a);
        v3 cr = vcross(t->e1, t->e2);
        t->area = 0.5 * vlen(cr);
        t->n = t->area > 0 ? vnorm(cr) : vmk(0, 0, 1);
        t->mat = tri_mat[i];
        for (int k = 0; k < 6; ++k) t->uv[k] = tri_uv[6 * i + k];
        double lo[3], hi[3];
        tri_bounds(t, lo, hi);
        for (int k = 0; k < 3; ++k) {
            if (lo[k] < scene_lo[k]) scene_lo[k] = lo[k];
            if (hi[k] > scene_hi[k]) scene_hi[k] = hi[k];
        }
    }
    double diag = sqrt((scene_hi[0] - scene_lo[0]) * (scene_hi[0] - scene_lo[0]) +
                       (scene_hi[1] - scene_lo[1]) * (scene_hi[1] - scene_lo[1]) +
                       (scene_hi[2] - scene_lo[2]) * (scene_hi[2] - scene_lo[2]));
    s->tmin = 1e-9 * (diag > 0 ? diag : 1.0);
    /* emitters: uniform by area over all emissive triangles (light sampling reading R7) */
    s->em_tri = (int *)malloc(sizeof(int) * (size_t)(ntri + 1));
    s->em_cdf = (double *)malloc(sizeof(double) * (size_t)(ntri + 1));
    s->nem = 0; s->em_area = 0;
    for (int i = 0; i < ntri; ++i)
        if (s->mat[s->tri[i].mat].emissive && s->tri[i].area > 0) {
            s->em_area += s->tri[i].area;
            s->em_tri[s->nem] = i;
            s->em_cdf[s->nem] = s->em_area;
            s->nem++;
        }
    /* camera */
    s->cam_p = vmk(cam[0], cam[1], cam[2]);
    v3 tgt = vmk(cam[3], cam[4], cam[5]), up = vmk(cam[6], cam[7], cam[8]);
    s->cam_f = vnorm(vsub(tgt, s->cam_p));
    s->cam_r = vnorm(vcross(s->cam_f, up));
    s->cam_u = vcross(s->cam_r, s->cam_f);
    s->tan_half = tan(0.5 * cam[9] * PI / 180.0);
    /* BVH */
    double *cent = (double *)malloc(sizeof(double) * 3 * (size_t)ntri);
    s->prim = (int *)malloc(sizeof(int) * (size_t)ntri);
    for (int i = 0; i < ntri; ++i) {
        v3 c = vadd(s->tri[i].v0, vscl(vadd(s->tri[i].e1, s->tri[i].e2), 1.0 / 3.0));
        cent[3 * i] = c.x; cent[3 * i + 1] = c.y; cent[3 * i + 2] = c.z;
        s->prim[i] = i;
    }
    s->nodes = (bnode_t *)calloc((size_t)(2 * ntri + 2), sizeof(bnode_t));
    s->nnodes = 0;
    if (ntri > 0) bvh_build(s, cent, 0, ntri);
    free(cent);
    return s;
}

void or_scene_free(void *p)
{
    scene_t *s = (scene_t *)p;
    if (!s) return;
    free(s->tri); free(s->mat); free(s->tex); free(s->em_tri); free(s->em_cdf);
    free(s->nodes); free(s->prim); free(s);
}

double or_scene_emitter_area(void *p) { return ((scene_t *)p)->em_area; }

/* ------------------------------------------------------------------------- */
/* ray queries                                                               */
/* ------------------------------------------------------------------------- */
typedef struct { double t, b1, b2; int prim; } hit_t;

/* Moller-Trumbore; returns 1 and t, b1, b2 on a hit with t in (tmin, tmax) */
static int isect_tri(const tri_t *t, v3 o, v3 d, double tmin, double tmax, double *tt, double *ob1, double *ob2)
{
    v3 pv = vcross(d, t->e2);
    double det = vdot(t->e1, pv);
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    v3 tv = vsub(o, t->v0);
    double b1 = vdot(tv, pv) * inv;
    if (b1 < 0.0 || b1 > 1.0) return 0;
    v3 qv = vcross(tv, t->e1);
    double b2 = vdot(d, qv) * inv;
    if (b2 < 0.0 || b1 + b2 > 1.0) return 0;
    double th = vdot(t->e2, qv) * inv;
    if (!(th > tmin && th < tmax)) return 0;
    *tt = th; *ob1 = b1; *ob2 = b2;
    return 1;
}

static int box_hit(const bnode_t *n, v3 o, v3 inv, double tmax)
{
    double t0 = 0.0, t1 = tmax;
    for (int k = 0; k < 3; ++k) {
        double ok = vcomp(o, k), ik = vcomp(inv, k);
        double a = (n->lo[k] - ok) * ik, b = (n->hi[k] - ok) * ik;
        if (a > b) { double tmp = a; a = b; b = tmp; }
        if (a != a) a = -1e300; /* NaN from 0 * inf: slab is infinite */
        if (b != b) b = 1e300;
        if (a > t0) t0 = a;
        if (b < t1) t1 = b;
        if (t0 > t1 * (1.0 + 1e-12) + 1e-15) return 0;
    }
    return 1;
}

/* closest hit; ties in t go to the lower triangle index; ign0/ign1 are skipped */
static int trace_closest(const scene_t *s, v3 o, v3 d, double tmin, double tmax, int ign0, int ign1, hit_t *h)
{
    h->prim = -1; h->t = tmax;
    if (s->ntri == 0) return 0;
    v3 inv = vmk(1.0 / d.x, 1.0 / d.y, 1.0 / d.z);
    int stack[128]; int sp = 0; stack[sp++] = 0;
    while (sp) {
        const bnode_t *n = &s->nodes[stack[--sp]];
        if (!box_hit(n, o, inv, h->t)) continue;
        if (n->count > 0) {
            for (int i = n->first; i < n->first + n->count; ++i) {
                int p = s->prim[i];
                if (p == ign0 || p == ign1) continue;
                double t, b1, b2;
                if (isect_tri(&s->tri[p], o, d, tmin, tmax, &t, &b1, &b2)) {
                    if (t < h->t || (t == h->t && (h->prim < 0 || p < h->prim))) {
                        h->t = t; h->b1 = b1; h->b2 = b2; h->prim = p;
                    }
                }
            }
        } else {
            stack[sp++] = n->left;
            stack[sp++] = n->right;
        }
    }
    return h->prim >= 0;
}

static int trace_brute(const scene_t *s, v3 o, v3 d, double tmin, double tmax, int ign0, int ign1, hit_t *h)
{
    h->prim = -1; h->t = tmax;
    for (int p = 0; p < s->ntri; ++p) {
        if (p == ign0 || p == ign1) continue;
        double t, b1, b2;
        if (isect_tri(&s->tri[p], o, d, tmin, tmax, &t, &b1, &b2))
            if (t < h->t || (t == h->t && (h->prim < 0 || p < h->prim))) {
                h->t = t; h->b1 = b1; h->b2 = b2; h->prim = p;
            }
    }
    return h->prim >= 0;
}

/* visibility between surface points a (on triangle pa) and b (on triangle pb) */
static int visible(const scene_t *s, v3 a, int pa, v3 b, int pb)
{
    v3 d = vsub(b, a);
    double dist = vlen(d);
    if (dist <= 0) return 0;
    d = vscl(d, 1.0 / dist);
    hit_t h;
    return !trace_closest(s, a, d, s->tmin, dist * (1.0 - 1e-9), pa, pb, &h);
}

/* batch query: rays[n*8] = o(3), d(3), tmin, tmax; writes t (or -1) and prim (or -1) */
void or_trace(void *p, const double *rays, int n, int brute, double *t_out, int *prim_out)
{
    scene_t *s = (scene_t *)p;
    for (int i = 0; i < n; ++i) {
        const double *r = rays + 8 * i;
        hit_t h;
        int ok = brute ? trace_brute(s, vmk(r[0], r[1], r[2]), vmk(r[3], r[4], r[5]), r[6], r[7], -1, -1, &h)
                       : trace_closest(s, vmk(r[0], r[1], r[2]), vmk(r[3], r[4], r[5]), r[6], r[7], -1, -1, &h);
        t_out[i] = ok ? h.t : -1.0;
        prim_out[i] = ok ? h.prim : -1;
    }
}

/* ------------------------------------------------------------------------- */
/* materials and BSDFs                                                       */
/* ------------------------------------------------------------------------- */
static void onb(v3 n, v3 *t, v3 *b)
{
    if (fabs(n.x) > fabs(n.z)) *t = vnorm(vmk(-n.y, n.x, 0.0));
    else *t = vnorm(vmk(0.0, -n.z, n.y));
    *b = vcross(n, *t);
}
static v3 cosine_dir(v3 n, double u1, double u2)
{
    double r = sqrt(u1), phi = 2.0 * PI * u2;
    v3 t, b;
    onb(n, &t, &b);
    double z = sqrt(fmax(0.0, 1.0 - u1));
    return vnorm(vadd(vadd(vscl(t, r * cos(phi)), vscl(b, r * sin(phi))), vscl(n, z)));
}

static double schlick(double f0, double c) { double m = 1.0 - c; return f0 + (1.0 - f0) * m * m * m * m * m; }

/* exact unpolarised Fresnel reflectance from index eta_o (incident side) into eta_i */
static double fresnel_dielectric(double cos_o, double eta_o, double eta_i, double *cos_t_out)
{
    double r = eta_o / eta_i;
    double s2 = r * r * (1.0 - cos_o * cos_o);
    if (s2 >= 1.0) { *cos_t_out = 0.0; return 1.0; }
    double ct = sqrt(1.0 - s2);
    double rs = (eta_o * cos_o - eta_i * ct) / (eta_o * cos_o + eta_i * ct);
    double rp = (eta_i * cos_o - eta_o * ct) / (eta_i * cos_o + eta_o * ct);
    *cos_t_out = ct;
    return 0.5 * (rs * rs + rp * rp);
}

/* GGX microfacet distribution and separable Smith masking, alpha = max(rough^2, 1e-4) */
static double ggx_D(double alpha, v3 n, v3 h)
{
    double c = vdot(n, h);
    if (c <= 0) return 0.0;
    double s2 = vdot(vcross(n, h), vcross(n, h));
    double a2 = alpha * alpha;
    double den = c * c * a2 + s2;
    return a2 / (PI * den * den);
}
static double ggx_G1(double alpha, v3 n, v3 w)
{
    double c = vdot(n, w);
    if (c <= 0) return 0.0;
    double s2 = vdot(vcross(n, w), vcross(n, w));
    double t2 = s2 / (c * c);
    return 2.0 / (1.0 + sqrt(1.0 + alpha * alpha * t2));
}

/* f_s(wo, wi) for non-Dirac materials (both are symmetric, so the transport mode is irrelevant).
 * wo and wi point away from the surface. Lambert reflects on the side of wo; a conductor
 * reflects only on its front side. */
static void bsdf_eval(const mat_t *m, v3 n, v3 wo, v3 wi, double f[3])
{
    f[0] = f[1] = f[2] = 0.0;
    double co = vdot(n, wo), ci = vdot(n, wi);
    if (m->type == MAT_LAMBERT) {
        if (co * ci <= 0) return;
        for (int k = 0; k < 3; ++k) f[k] = m->rgb[k] / PI;
    } else if (m->type == MAT_CONDUCTOR && !m->delta) {
        if (co <= 0 || ci <= 0) return;
        v3 h = vnorm(vadd(wo, wi));
        double D = ggx_D(m->alpha, n, h), G = ggx_G1(m->alpha, n, wo) * ggx_G1(m->alpha, n, wi);
        double c = vdot(wi, h);
        for (int k = 0; k < 3; ++k) f[k] = schlick(m->rgb[k], c) * D * G / (4.0 * co * ci);
    }
}

/* solid-angle density of sampling wi given wo, for non-Dirac materials */
static double bsdf_pdf(const mat_t *m, v3 n, v3 wo, v3 wi)
{
    double co = vdot(n, wo), ci = vdot(n, wi);
    if (m->type == MAT_LAMBERT) return co * ci > 0 ? fabs(ci) / PI : 0.0;
    if (m->type == MAT_CONDUCTOR && !m->delta) {
        if (co <= 0 || ci <= 0) return 0.0;
        v3 h = vnorm(vadd(wo, wi));
        double oh = vdot(wo, h);
        if (oh <= 0) return 0.0;
        return ggx_D(m->alpha, n, h) * vdot(n, h) / (4.0 * oh);
    }
    return 0.0;
}

typedef struct {
    int ok, delta, transmit;
    v3 wi;
    double w[3];      /* f |cos wi| / pdf in the requested transport mode */
    double pdf;       /* solid-angle pdf (non-Dirac) or the discrete lobe probability (Dirac) */
} bsample_t;

enum { MODE_CAMERA = 0, MODE_LIGHT = 1 };

/* Sample wi given wo. MODE_CAMERA: wo points toward the camera side of the path and the
 * weight carries radiance (through a refraction it is (eta_o/eta_i)^2). MODE_LIGHT: wo points
 * toward the light side and the weight of a refraction is 1 (the adjoint of the same BSDF). */
static bsample_t bsdf_sample(const mat_t *m, v3 n, v3 wo, double u1, double u2, double u3, int mode)
{
    bsample_t s;
    memset(&s, 0, sizeof(s));
    double co = vdot(n, wo);
    if (m->type == MAT_LAMBERT) {
        v3 ns = co > 0 ? n : vscl(n, -1.0);
        if (co == 0) return s;
        s.wi = cosine_dir(ns, u1, u2);
        double ci = vdot(ns, s.wi);
        if (ci <= 0) return s;
        s.pdf = ci / PI;
        for (int k = 0; k < 3; ++k) s.w[k] = m->rgb[k];
        s.ok = 1;
        return s;
    }
    if (m->type == MAT_CONDUCTOR) {
        if (co <= 0) return s;
        if (m->delta) {
            s.wi = vsub(vscl(n, 2.0 * co), wo);
            for (int k = 0; k < 3; ++k) s.w[k] = schlick(m->rgb[k], co);
            s.pdf = 1.0; s.delta = 1; s.ok = 1;
            return s;
        }
        double a = m->alpha;
        double t2 = a * a * u1 / (1.0 - u1);
        double ch = 1.0 / sqrt(1.0 + t2), sh = sqrt(t2) * ch, phi = 2.0 * PI * u2;
        v3 t, b;
        onb(n, &t, &b);
        v3 h = vnorm(vadd(vadd(vscl(t, sh * cos(phi)), vscl(b, sh * sin(phi))), vscl(n, ch)));
        double oh = vdot(wo, h);
        if (oh <= 0) return s;
        s.wi = vsub(vscl(h, 2.0 * oh), wo);
        if (vdot(n, s.wi) <= 0) return s;
        double f[3];
        bsdf_eval(m, n, wo, s.wi, f);
        s.pdf = bsdf_pdf(m, n, wo, s.wi);
        if (s.pdf <= 0) return s;
        double ci = vdot(n, s.wi);
        for (int k = 0; k < 3; ++k) s.w[k] = f[k] * ci / s.pdf;
        s.ok = 1;
        return s;
    }
    /* smooth dielectric: the geometric normal points to the outside (index 1) */
    if (co == 0) return s;
    int outside = co > 0;
    v3 ns = outside ? n : vscl(n, -1.0);
    double eo = outside ? 1.0 : m->ior, ei = outside ? m->ior : 1.0;
    double c = fabs(co), ct;
    double F = fresnel_dielectric(c, eo, ei, &ct);
    s.delta = 1; s.ok = 1;
    if (u1 < F) {
        s.wi = vsub(vscl(ns, 2.0 * c), wo);
        s.pdf = F;
        s.w[0] = s.w[1] = s.w[2] = 1.0;
    } else {
        double r = eo / ei;
        s.wi = vnorm(vadd(vscl(wo, -r), vscl(ns, r * c - ct)));
        s.pdf = 1.0 - F;
        s.transmit = 1;
        double wt = mode == MODE_CAMERA ? r * r : 1.0;
        s.w[0] = s.w[1] = s.w[2] = wt;
    }
    return s;
}

/* discrete lobe probability that a Dirac vertex maps wo to wi (0 if wi is not one of its lobes) */
static double delta_lobe_prob(const mat_t *m, v3 n, v3 wo, v3 wi)
{
    double co = vdot(n, wo);
    if (m->type == MAT_CONDUCTOR) return co > 0 && vdot(n, wi) > 0 ? 1.0 : 0.0;
    if (co == 0) return 0.0;
    int outside = co > 0;
    double eo = outside ? 1.0 : m->ior, ei = outside ? m->ior : 1.0, ct;
    double F = fresnel_dielectric(fabs(co), eo, ei, &ct);
    return (co * vdot(n, wi) > 0) ? F : 1.0 - F;
}

static void emitted(const scene_t *s, int prim, double b1, double b2, v3 w_out, double le[3])
{
    const tri_t *t = &s->tri[prim];
    const mat_t *m = &s->mat[t->mat];
    le[0] = le[1] = le[2] = 0.0;
    if (!m->emissive || vdot(t->n, w_out) <= 0) return;
    double sc = 1.0;
    if (m->textured) {
        double b0 = 1.0 - b1 - b2;
        double u = b0 * t->uv[0] + b1 * t->uv[2] + b2 * t->uv[4];
        double v = b0 * t->uv[1] + b1 * t->uv[3] + b2 * t->uv[5];
        int ix = (int)floor(u * s->tw), iy = (int)floor(v * s->th);
        if (ix < 0) ix = 0;
        if (ix >= s->tw) ix = s->tw - 1;
        if (iy < 0) iy = 0;
        if (iy >= s->th) iy = s->th - 1;
        sc = s->tex[iy * s->tw + ix];
    }
    for (int k = 0; k < 3; ++k) le[k] = m->le[k] * sc;
}

/* uniform point on the emitters by area: p = 1 / A (reading R7) */
typedef struct { v3 p, n; int prim; double b1, b2; } lpoint_t;
static int sample_light(const scene_t *s, rng_t *r, lpoint_t *lp)
{
    if (s->nem == 0) return 0;
    double x = rng_u01(r) * s->em_area;
    int lo = 0, hi = s->nem - 1;
    while (lo < hi) { int mid = (lo + hi) / 2; if (s->em_cdf[mid] > x) hi = mid; else lo = mid + 1; }
    const tri_t *t = &s->tri[s->em_tri[lo]];
    double u1 = rng_u01(r), u2 = rng_u01(r), su = sqrt(u1);
    lp->b1 = su * (1.0 - u2); lp->b2 = su * u2;
    lp->p = vadd(t->v0, vadd(vscl(t->e1, lp->b1), vscl(t->e2, lp->b2)));
    lp->n = t->n; lp->prim = s->em_tri[lo];
    return 1;
}

static v3 hit_point(const scene_t *s, const hit_t *h)
{
    const tri_t *t = &s->tri[h->prim];
    return vadd(t->v0, vadd(vscl(t->e1, h->b1), vscl(t->e2, h->b2)));
}

/* ------------------------------------------------------------------------- */
/* exported BSDF hooks for the sampling tests                                 */
/* ------------------------------------------------------------------------- */
static mat_t mat_from_record(const float *r)
{
    mat_t m;
    memset(&m, 0, sizeof(m));
    m.type = (int)r[0];
    for (int k = 0; k < 3; ++k) { m.rgb[k] = r[1 + k]; m.le[k] = r[6 + k]; }
    m.rough = r[4]; m.alpha = r[4] * (double)r[4]; if (m.alpha < 1e-4) m.alpha = 1e-4;
    m.ior = r[5];
    m.spec = (m.type == MAT_CONDUCTOR || m.type == MAT_DIELECTRIC) && m.rough < 0.2;
    m.delta = (m.type == MAT_DIELECTRIC) || (m.type == MAT_CONDUCTOR && m.rough == 0.0);
    return m;
}
/* out[0..2] wi, out[3..5] weight, out[6] pdf, out[7] ok, out[8] delta */
void or_bsdf_sample(const float *rec, const double *n, const double *wo, double u1, double u2, double u3,
                    int mode, double *out)
{
    mat_t m = mat_from_record(rec);
    bsample_t s = bsdf_sample(&m, vmk(n[0], n[1], n[2]), vmk(wo[0], wo[1], wo[2]), u1, u2, u3, mode);
    out[0] = s.wi.x; out[1] = s.wi.y; out[2] = s.wi.z;
    out[3] = s.w[0]; out[4] = s.w[1]; out[5] = s.w[2];
    out[6] = s.pdf; out[7] = s.ok; out[8] = s.delta;
}
/* out[0..2] f, out[3] pdf */
void or_bsdf_eval(const float *rec, const double *n, const double *wo, const double *wi, double *out)
{
    mat_t m = mat_from_record(rec);
    double f[3];
    bsdf_eval(&m, vmk(n[0], n[1], n[2]), vmk(wo[0], wo[1], wo[2]), vmk(wi[0], wi[1], wi[2]), f);
    out[0] = f[0]; out[1] = f[1]; out[2] = f[2];
    out[3] = bsdf_pdf(&m, vmk(n[0], n[1], n[2]), vmk(wo[0], wo[1], wo[2]), vmk(wi[0], wi[1], wi[2]));
}

/* ------------------------------------------------------------------------- */
/* reciprocal estimators (Section 4.2 and Appendix A)                        */
/* ------------------------------------------------------------------------- */
/* A sampler returns one sample of f(x)/q(x) with x ~ q; the estimator only sees that ratio. */
typedef double (*fq_sampler)(void *ctx, rng_t *r);

typedef struct {
    fq_sampler sample;
    void *ctx;
    rng_t *rng;
    double B;
    long nsamp, cap;
    int truncated;
} recip_ctx;

/* Estimator I~' of Appendix A: estimates 1/int f - 1/B. Sample x0 ~ q, g0 = 1 - f/(B q),
 * r0 = |g0| (the RRS function of equ:rr), split into floor(r0) (+1 with probability
 * r0 - floor(r0)) children, each weighted g0 / r0. The loop runs the integer split count
 * (reading R1); a zero g0 spawns nothing. */
static double itilde_prime(recip_ctx *c)
{
    if (c->nsamp >= c->cap) { c->truncated = 1; return 0.0; }
    c->nsamp++;
    double fq = c->sample(c->ctx, c->rng);
    double g0 = 1.0 - fq / c->B;
    double r0 = fabs(g0);
    double ans = g0 / c->B;
    if (r0 == 0.0) return ans;
    long n = (long)floor(r0);
    if (rng_u01(c->rng) < r0 - floor(r0)) n++;
    for (long i = 0; i < n; ++i) ans += g0 * itilde_prime(c) / r0;
    return ans;
}
static double itilde(recip_ctx *c) { return itilde_prime(c) + 1.0 / c->B; }

/* Estimator I of Appendix A (the sign estimator I_sign of Section 4.2): adds 1/B per node. */
static double isign(recip_ctx *c)
{
    if (c->nsamp >= c->cap) { c->truncated = 1; return 0.0; }
    c->nsamp++;
    double fq = c->sample(c->ctx, c->rng);
    double g0 = 1.0 - fq / c->B;
    double r0 = fabs(g0);
    double ans = 1.0 / c->B;
    if (r0 == 0.0) return ans;
    long n = (long)floor(r0);
    if (rng_u01(c->rng) < r0 - floor(r0)) n++;
    for (long i = 0; i < n; ++i) ans += g0 * isign(c) / r0;
    return ans;
}

/* Booth's Russian roulette for 1/int f (Section 4.2, the comparison with Booth 2007; the RR
 * ablation of Section 6): one chain, no splitting. After the prefix of j samples the chain goes
 * on with probability r_j = min(1, prod_{i<j} |g_i| / rhat) and the terms beyond it are divided
 * by r_j, so the estimate is [1 + sum_k prod_{i<k} g_i / prod_{1<=j<k} r_j] / B (equ:RRS_estimator
 * with Booth's RR function; reading R26). One uniform number is drawn per sample after it, as
 * I~ draws one for its split, so that on a binary f/q with rhat <= 1 both take the same
 * decisions from the same stream. */
static double ibooth(recip_ctx *c, double rhat)
{
    double ans = 1.0, prod = 1.0, w = 1.0;
    for (;;) {
        if (c->nsamp >= c->cap) { c->truncated = 1; break; }
        c->nsamp++;
        double fq = c->sample(c->ctx, c->rng);
        double g = 1.0 - fq / c->B;
        prod *= g;
        ans += prod / w;
        double r = fmin(1.0, fabs(prod) / rhat);
        if (!(rng_u01(c->rng) < r)) break;
        w *= r;
    }
    return ans / c->B;
}

typedef struct { const double *f, *q; double *cdf; int n; } table_ctx;
static double table_sample(void *p, rng_t *r)
{
    table_ctx *t = (table_ctx *)p;
    double x = rng_u01(r) * t->cdf[t->n - 1];
    int i = 0;
    while (i < t->n - 1 && t->cdf[i] <= x) ++i;
    return t->f[i] / t->q[i];
}

/* Discrete problem: target 1 / sum_i f[i], supporting pmf q (q[i] > 0 wherever f[i] > 0).
 * estimator 0 = I~ (the paper's estimator), 1 = I (sign estimator), 2 = Booth's roulette with
 * parameter rhat. est[i] and nsamp[i] receive each independent estimate and its sample count.
 * Returns the number of truncated estimates (sample cap reached). */
int or_recip_table(const double *f, const double *q, int n, double B, int estimator, int n_est,
                   uint32_t seed, long cap, double *est, double *nsamp, double rhat)
{
    table_ctx t = {f, q, (double *)malloc(sizeof(double) * (size_t)n), n};
    double acc = 0;
    for (int i = 0; i < n; ++i) { acc += q[i]; t.cdf[i] = acc; }
    int trunc = 0;
    for (int e = 0; e < n_est; ++e) {
        rng_t r;
        rng_init(&r, seed, ST_TABLE, (uint32_t)e, 0, 0);
        recip_ctx c = {table_sample, &t, &r, B, 0, cap > 0 ? cap : (1L << 24), 0};
        est[e] = estimator == 0 ? itilde(&c) : estimator == 1 ? isign(&c) : ibooth(&c, rhat);
        nsamp[e] = (double)c.nsamp;
        trunc += c.truncated;
    }
    free(t.cdf);
    return trunc;
}

/* ------------------------------------------------------------------------- */
/* path classes for the partition of strategies                              */
/* ------------------------------------------------------------------------- */
/* The proxy strategy builds, at the eye's first diffuse vertex z_d, paths whose part beyond z_d is
 * L S^u (class A) or L D S^u (class B), 1 <= u <= 4 (Section 6.1's limits) and, with a general
 * control vertex (Section 5.2), L ... h_c D S^u (class C, h_c = y_j, j >= 1, a Lambertian vertex).
 * The state machine walks eye vertices z_1, z_2, ... (emitters count as diffuse):
 *   phase 0  no diffuse vertex yet
 *   phase 1  at / after z_d, only specular vertices since (u of them)
 *   phase 2  S^u (1 <= u <= 4) then exactly one diffuse vertex (y_1, or y_{j+1} for class C)
 *   phase 4  (general control vertex only) S^u D then a Lambertian h_c, k vertices pushed since h_c
 *            entered (h_c = y_k when the path closes at the vertex pushed last)
 *   phase 3  anything else (never a proxy path). */
typedef struct { int phase, u, k; } pstate_t;
static void pstate_push(pstate_t *st, int is_s, int is_lambert, int umax, int gcv)
{
    switch (st->phase) {
    case 0: if (!is_s) { st->phase = 1; st->u = 0; } break;
    case 1:
        if (is_s) { if (++st->u > umax) st->phase = 3; }
        else st->phase = st->u >= 1 ? 2 : 3;
        break;
    case 2:
        if (gcv && is_lambert) { st->phase = 4; st->k = 1; }
        else st->phase = 3;
        break;
    case 4: st->k++; break;
    default: break;
    }
}
#define LMAX_GCV 6   /* light vertices the proxy strategy keeps per sub-path (y_0 .. y_5) */
/* does a path closed at the emitter after the vertices pushed so far (an emission hit of the next
 * vertex, or a light sample connected to the vertex pushed last) belong to the proxy class? Class
 * A: S^u then the emitter; B: S^u D then the emitter (h_c = y_0); C: S^u D then h_c = y_k, k >= 1,
 * with y_{k+1+u} among the stored light vertices */
static int pstate_closes_proxy(const pstate_t *st)
{
    if (st->phase == 4) return st->k + 1 + st->u <= LMAX_GCV - 1;
    return (st->phase == 1 && st->u >= 1) || st->phase == 2;
}
/* the proxy-class test of one eye path z_1 .. z_n closed at the emitter after z_n (is_s[i],
 * is_lambert[i] of z_{i+1}): the state machine above, exported so that tests can check it against
 * the classes' definitions on every short path */
int or_proxy_class(const int *is_s, const int *is_lambert, int n, int umax, int gcv)
{
    pstate_t st = {0, 0, 0};
    for (int i = 0; i < n; ++i) pstate_push(&st, is_s[i], is_lambert[i], umax, gcv);
    return pstate_closes_proxy(&st);
}

/* ------------------------------------------------------------------------- */
/* thread pool helper                                                         */
/* ------------------------------------------------------------------------- */
typedef void (*work_fn)(void *ctx, int i);
typedef struct { work_fn fn; void *ctx; int n; int next; pthread_mutex_t mu; } pool_t;
static void *pool_worker(void *p)
{
    pool_t *pl = (pool_t *)p;
    for (;;) {
        pthread_mutex_lock(&pl->mu);
        int i = pl->next++;
        pthread_mutex_unlock(&pl->mu);
        if (i >= pl->n) break;
        pl->fn(pl->ctx, i);
    }
    return NULL;
}
static void parallel_for(int n, int threads, work_fn fn, void *ctx)
{
    /* always run on pool threads: their large stacks hold the recursion of I~' */
    if (n <= 0) return;
    if (threads > n) threads = n;
    if (threads < 1) threads = 1;
    pool_t pl = {fn, ctx, n, 0, PTHREAD_MUTEX_INITIALIZER};
    pthread_t th[256];
    if (threads > 256) threads = 256;
    pthread_attr_t at;
    pthread_attr_init(&at);
    pthread_attr_setstacksize(&at, (size_t)1 << 30);   /* deep recursion in I~' */
    for (int t = 0; t < threads; ++t) pthread_create(&th[t], &at, pool_worker, &pl);
    for (int t = 0; t < threads; ++t) pthread_join(th[t], NULL);
    pthread_attr_destroy(&at);
}

/* ------------------------------------------------------------------------- */
/* render parameters and statistics                                           */
/* ------------------------------------------------------------------------- */
typedef struct {
    int method;        /* 0 = O1 (PT + NEE), 1 = O2 (proxy-sampling BDPT), 2 = O3 (plain BDPT) */
    int n_iter;        /* iterations = samples per pixel (1 spp each, Section 6.1) */
    int first_iter;    /* index of the first iteration (streams are keyed by it) */
    int max_depth;     /* maximum number of path segments */
    int n_light;       /* M light sub-paths per iteration */
    int cand_cap;      /* expected number of kept candidates per iteration */
    int repeats;       /* reciprocal repeats averaged per candidate (5 in Section 6.1) */
    int u_max;         /* longest specular run handled by the proxy (4 in Section 6.1) */
    int class_filter;  /* 0 all paths, 1 proxy-class paths only, 2 all other paths only */
    int threads;
    uint32_t seed;
    int pilot;         /* minimum pilot samples per candidate (B and cost estimate) */
    long chain_cap;    /* sample cap per reciprocal estimate */
    double cost_cap;   /* expected chain samples per candidate above which it is roulette-kept */
    int o3_weights;    /* O3 only: 0 balance heuristic, 1 uniform over the strategies that can
                        * build the path, 2 light tracing alone (pins of the strategies) */
    int general_cv;    /* O1's class filter and O2: 1 when the proxy class also holds the paths of a
                        * general control vertex (Section 5.2): ... h_c D S^u z_d with h_c = y_j,
                        * j >= 1, a Lambertian vertex, and j + 1 + u < LMAX_GCV (the stored light
                        * vertices); O2 then builds them from class C candidates */
} or_params;

typedef struct {
    double n_cand, n_kept, n_recip_samples, n_recip_truncated, n_proxy_attempts, n_proxy_valid;
    double bucket_B[2][5];
} or_stats;

/* ------------------------------------------------------------------------- */
/* O1: path tracing with next-event estimation                                */
/* ------------------------------------------------------------------------- */
typedef struct {
    const scene_t *s; const or_params *p;
    double *sum, *sumsq;
    int iter;
    /* O2 data (NULL for O1) */
    struct o2_iter *o2;
} eye_ctx;

static void camera_ray(const scene_t *s, int px, int py, double jx, double jy, v3 *o, v3 *d)
{
    double aspect = (double)s->W / s->H;
    double x = (2.0 * (px + jx) / s->W - 1.0) * s->tan_half * aspect;
    double y = (1.0 - 2.0 * (py + jy) / s->H) * s->tan_half;
    *o = s->cam_p;
    *d = vnorm(vadd(s->cam_f, vadd(vscl(s->cam_r, x), vscl(s->cam_u, y))));
}

/* filter: 0 every path, 1 proxy-class paths only, 2 all other paths only, 3 none */
static int class_ok(int filter, int is_proxy_class)
{
    if (filter == 1) return is_proxy_class;
    if (filter == 2) return !is_proxy_class;
    return filter == 0;
}

struct o2_iter;
static double proxy_connect(const scene_t *s, const or_params *p, struct o2_iter *it, v3 xd, v3 nd, int primd,
                            const mat_t *md, v3 wo, int d, rng_t *r, double out[3]);

/* One eye path for one pixel and iteration: PT with NEE (balance heuristic). For O2 the
 * proxy-class paths are left to proxy_connect at the first diffuse vertex. */
static void eye_path(const eye_ctx *c, int px, int py, rng_t *r, double L[3])
{
    const scene_t *s = c->s;
    const or_params *p = c->p;
    /* O2: PT/NEE score the non-proxy paths (filter 2) unless only the proxy class is wanted
     * (then they score nothing); the proxy strategy runs unless only non-proxy paths are wanted. */
    int filter = p->class_filter;
    int do_proxy = 0;
    if (c->o2) { do_proxy = p->class_filter != 2; filter = p->class_filter == 1 ? 3 : 2; }
    L[0] = L[1] = L[2] = 0.0;
    v3 o, d;
    camera_ray(s, px, py, rng_u01(r), rng_u01(r), &o, &d);
    double beta[3] = {1, 1, 1};
    double prev_pdf = 0.0;
    int prev_delta = 1, ign = -1;
    pstate_t st = {0, 0, 0};
    for (int t = 1; t <= p->max_depth; ++t) {
        hit_t h;
        if (!trace_closest(s, o, d, s->tmin, 1e300, ign, -1, &h)) break;
        v3 x = hit_point(s, &h);
        const tri_t *tr = &s->tri[h.prim];
        const mat_t *m = &s->mat[tr->mat];
        v3 wo = vscl(d, -1.0);
        if (m->emissive) {
            double le[3];
            emitted(s, h.prim, h.b1, h.b2, wo, le);
            if ((le[0] > 0 || le[1] > 0 || le[2] > 0) && class_ok(filter, pstate_closes_proxy(&st))) {
                double w = 1.0;
                if (!(t == 1 || prev_delta)) {
                    double cl = fabs(vdot(tr->n, wo));
                    double pl = h.t * h.t / (cl * s->em_area);
                    w = prev_pdf / (prev_pdf + pl);
                }
                for (int k = 0; k < 3; ++k) L[k] += beta[k] * le[k] * w;
            }
        }
        if (t == p->max_depth) break;
        pstate_push(&st, m->spec, m->type == MAT_LAMBERT, p->u_max, p->general_cv);
        /* proxy connection at the first diffuse vertex (O2 only) */
        if (do_proxy && st.phase == 1 && st.u == 0 && !m->spec) {
            double pc[3];
            proxy_connect(s, p, c->o2, x, tr->n, h.prim, m, wo, t, r, pc);
            for (int k = 0; k < 3; ++k) L[k] += beta[k] * pc[k];
        }
        /* next-event estimation */
        if (!m->delta && s->nem > 0) {
            lpoint_t lp;
            sample_light(s, r, &lp);
            v3 dl = vsub(lp.p, x);
            double dist = vlen(dl);
            v3 wl = vscl(dl, 1.0 / dist);
            double cl = vdot(lp.n, vscl(wl, -1.0));
            int cls = pstate_closes_proxy(&st);
            if (cl > 0 && class_ok(filter, cls)) {
                double f[3];
                bsdf_eval(m, tr->n, wo, wl, f);
                if ((f[0] > 0 || f[1] > 0 || f[2] > 0) && visible(s, x, h.prim, lp.p, lp.prim)) {
                    double le[3];
                    emitted(s, lp.prim, lp.b1, lp.b2, vscl(wl, -1.0), le);
                    double pl = dist * dist / (cl * s->em_area);
                    double pb = bsdf_pdf(m, tr->n, wo, wl);
                    double w = pl / (pl + pb);
                    double ci = fabs(vdot(tr->n, wl));
                    for (int k = 0; k < 3; ++k) L[k] += beta[k] * f[k] * ci * le[k] / pl * w;
                }
            }
        }
        bsample_t bs = bsdf_sample(m, tr->n, wo, rng_u01(r), rng_u01(r), rng_u01(r), MODE_CAMERA);
        if (!bs.ok) break;
        for (int k = 0; k < 3; ++k) beta[k] *= bs.w[k];
        if (beta[0] == 0 && beta[1] == 0 && beta[2] == 0) break;
        prev_pdf = bs.pdf; prev_delta = bs.delta;
        o = x; d = bs.wi; ign = h.prim;
    }
}

static void eye_row(void *ctx, int py)
{
    const eye_ctx *c = (const eye_ctx *)ctx;
    const scene_t *s = c->s;
    for (int px = 0; px < s->W; ++px) {
        int pix = py * s->W + px;
        rng_t r;
        rng_init(&r, c->p->seed, c->o2 ? ST_EYE : ST_PT, (uint32_t)pix, (uint32_t)c->iter, 0);
        double L[3];
        eye_path(c, px, py, &r, L);
        for (int k = 0; k < 3; ++k) {
            c->sum[3 * pix + k] += L[k];
            c->sumsq[3 * pix + k] += L[k] * L[k];
        }
    }
}

/* ------------------------------------------------------------------------- */
/* O2: light sub-paths, incomplete sub-path candidates, reciprocal estimates  */
/* ------------------------------------------------------------------------- */
#define LMAX 6   /* light vertices stored per sub-path: y_0 .. y_5 (class B with u = 4) */
typedef struct {
    v3 p, n; int prim; double b1, b2; int is_s;
    int is_lam;       /* Lambertian (a possible general control vertex) */
    double beta[3];   /* the light tracer's throughput arriving at the vertex: L_e A pi at y_1, then
                       * times the adjoint BSDF weight f |cos| / pdf of every vertex passed */
} lvert_t;
typedef struct { lvert_t v[LMAX]; int nv; } lpath_t;

typedef struct {
    int cls;          /* 0: class A = L_DD S^u, h_c null; 1: class B = L_DD D S^u, h_c = y_0;
                       * 2: class C (general control vertex), h_c = y_j on a Lambertian surface */
    int u;            /* length of the trailing specular run */
    int j;            /* class C: the light-order index of h_c */
    lvert_t v;        /* y_{s-1}, the specular vertex that is kept */
    lvert_t hc;       /* y_0 for class B; y_j for class C with its normal turned toward y_{j-1}
                       * (the side its BSDF is sampled on from the control direction) */
    v3 wc;            /* class C: the direction from h_c toward y_{j-1} */
    double recip;     /* averaged reciprocal estimate of 1 / P(u, h_c, y_{s-1}, w_c) */
    double B;         /* the constant B used by this candidate's chains */
    double rho;       /* probability of keeping it after the pilot (cost roulette) */
} cand_t;

struct o2_iter {
    lpath_t *paths; int M;
    cand_t *cand; int ncand;
    int *kept; int nkept;
    double pi_inc;
    double B[3][5];
    /* per-iteration statistics of f/q samples, per (class, u) bucket */
    double fq_max[3][5], fq_sum[3][5], fq_n[3][5];
    double n_samples, n_trunc;
    long proxy_attempts, proxy_valid;
    pthread_mutex_t mu;
};

/* Section 3.1 tracing pdf chain: light sub-path sampling. y_0 uniform on the emitters by
 * area, cosine emission about its normal, then the BSDF (adjoint mode) at every vertex; no
 * Russian roulette (reading R8). */
typedef struct { const scene_t *s; const or_params *p; struct o2_iter *it; int iter; } light_ctx;
static void light_path(void *ctx, int l)
{
    light_ctx *c = (light_ctx *)ctx;
    const scene_t *s = c->s;
    lpath_t *lp = &c->it->paths[l];
    lp->nv = 0;
    rng_t r;
    rng_init(&r, c->p->seed, ST_LIGHT, (uint32_t)l, (uint32_t)c->iter, 0);
    lpoint_t y0;
    if (!sample_light(s, &r, &y0)) return;
    lvert_t *v0 = &lp->v[0];
    v0->p = y0.p; v0->n = y0.n; v0->prim = y0.prim; v0->b1 = y0.b1; v0->b2 = y0.b2; v0->is_s = 0;
    v0->is_lam = 0; v0->beta[0] = v0->beta[1] = v0->beta[2] = 0.0;
    lp->nv = 1;
    v3 d = cosine_dir(y0.n, rng_u01(&r), rng_u01(&r));
    /* throughput of the ray leaving y_0: L_e cos / (p_A p_w) with p_A = 1/A, p_w = cos/pi */
    double beta[3];
    emitted(s, y0.prim, y0.b1, y0.b2, d, beta);
    for (int k = 0; k < 3; ++k) beta[k] *= s->em_area * PI;
    v3 o = y0.p;
    int ign = y0.prim;
    int lmax = c->p->max_depth - 1 < LMAX ? c->p->max_depth - 1 : LMAX;
    while (lp->nv < lmax) {
        hit_t h;
        if (!trace_closest(s, o, d, s->tmin, 1e300, ign, -1, &h)) break;
        lvert_t *v = &lp->v[lp->nv++];
        v->p = hit_point(s, &h); v->n = s->tri[h.prim].n; v->prim = h.prim; v->b1 = h.b1; v->b2 = h.b2;
        const mat_t *m = &s->mat[s->tri[h.prim].mat];
        v->is_s = m->spec;
        v->is_lam = m->type == MAT_LAMBERT;
        for (int k = 0; k < 3; ++k) v->beta[k] = beta[k];
        bsample_t bs = bsdf_sample(m, v->n, vscl(d, -1.0), rng_u01(&r), rng_u01(&r), rng_u01(&r), MODE_LIGHT);
        if (!bs.ok) break;
        for (int k = 0; k < 3; ++k) beta[k] *= bs.w[k];
        o = v->p; d = bs.wi; ign = h.prim;
    }
}

/* Section 5.1 / 6.1: every prefix ending at a specular vertex whose trailing specular run
 * (length u in [1, u_max]) starts at y_1 (class A, h_c null) or at y_2 after a diffuse y_1
 * (class B, h_c = y_0) is an incomplete sub-path candidate (reading R11); with gcv also a run
 * that starts at y_{j+2} after a diffuse y_{j+1} and a Lambertian y_j, j >= 1 (class C, h_c =
 * y_j, Section 5.2). */
static int collect_candidates(const lpath_t *lp, int u_max, int gcv, cand_t *out)
{
    int n = 0;
    if (lp->nv < 2) return 0;
    if (lp->v[1].is_s) {
        for (int i = 1; i < lp->nv && lp->v[i].is_s && i <= u_max; ++i) {
            cand_t *c = &out[n++];
            c->cls = 0; c->u = i; c->v = lp->v[i]; c->hc = lp->v[0];
        }
    } else {
        for (int i = 2; i < lp->nv && lp->v[i].is_s && i - 1 <= u_max; ++i) {
            cand_t *c = &out[n++];
            c->cls = 1; c->u = i - 1; c->v = lp->v[i]; c->hc = lp->v[0];
        }
    }
    if (gcv)
        for (int j = 1; j + 2 < lp->nv; ++j) {
            if (!lp->v[j].is_lam || lp->v[j + 1].is_s) continue;
            for (int i = j + 2; i < lp->nv && lp->v[i].is_s && i - j - 1 <= u_max; ++i) {
                cand_t *c = &out[n++];
                c->cls = 2; c->u = i - j - 1; c->j = j; c->v = lp->v[i]; c->hc = lp->v[j];
                c->wc = vnorm(vsub(lp->v[j - 1].p, lp->v[j].p));
                if (vdot(c->hc.n, c->wc) < 0) c->hc.n = vscl(c->hc.n, -1.0);
            }
        }
    return n;
}

/* ---- supporting distribution q and target f for 1/P (Sections 5.2 and 5.3) ----
 * P(u, h_c, y_{s-1}, w_c) = int p(g | h_c, w_c) p(y_{s-1} | g, h_c) dmu(g)   (equ:reciprocalFinal)
 * f(g) is the light tracer's own density of the dropped vertices and of y_{s-1}, with
 * visibility and the S/D signature (S for the intermediate vertices, an emitter for class
 * A's y_0, D for class B's y_1). q is the uniform mixture of the available strategies
 * (reading R5): light-source sampling (u = 1, class A), tracing from the control vertex
 * (u = 1, class B; h_c is on the light so its cosine lobe is used), and tracing from the
 * specular vertex (cosine at y_{s-1}, then the BSDF at each intermediate vertex). On a
 * transmissive y_{s-1} each side's cosine hemisphere is taken with probability 1/2 (R6). */

/* probability of picking the hemisphere of direction w at the specular vertex */
static double side_prob(const mat_t *m, v3 n, v3 w)
{
    if (m->type == MAT_DIELECTRIC) return 0.5;
    return vdot(n, w) > 0 ? 1.0 : 0.0;
}

typedef struct { const scene_t *s; const cand_t *c; long rays; } cq_ctx;

/* cosine-hemisphere direction at y_{s-1} on a chosen side */
static v3 spec_start_dir(const mat_t *m, v3 n, rng_t *r)
{
    v3 ns = n;
    if (m->type == MAT_DIELECTRIC && rng_u01(r) < 0.5) ns = vscl(n, -1.0);
    double u1 = rng_u01(r), u2 = rng_u01(r);
    return cosine_dir(ns, u1, u2);
}

/* u = 1: every density in plain area measure (no Dirac vertex lies inside g). */
static double fq_u1(cq_ctx *cc, rng_t *r)
{
    const scene_t *s = cc->s;
    const cand_t *c = cc->c;
    const mat_t *mv = &s->mat[s->tri[c->v.prim].mat];
    int strat = rng_u01(r) < 0.5 ? 0 : 1;   /* 0: light / control vertex, 1: from y_{s-1} */
    v3 y; v3 ny; int prim;
    if (c->cls == 0) {
        /* g = y_0 on the emitters */
        lpoint_t lp;
        if (strat == 0) {
            if (!sample_light(s, r, &lp)) return 0.0;
            if (!visible(s, lp.p, lp.prim, c->v.p, c->v.prim)) { cc->rays++; return 0.0; }
            cc->rays++;
            y = lp.p; ny = lp.n; prim = lp.prim;
        } else {
            v3 w = spec_start_dir(mv, c->v.n, r);
            hit_t h;
            cc->rays++;
            if (!trace_closest(s, c->v.p, w, s->tmin, 1e300, c->v.prim, -1, &h)) return 0.0;
            if (!s->mat[s->tri[h.prim].mat].emissive) return 0.0;
            y = hit_point(s, &h); ny = s->tri[h.prim].n; prim = h.prim;
        }
        (void)prim;
        v3 dv = vsub(c->v.p, y);
        double d2 = vdot(dv, dv), dist = sqrt(d2);
        v3 w = vscl(dv, 1.0 / dist);
        double c0 = vdot(ny, w), cv = fabs(vdot(c->v.n, w));
        /* f = p(y_0) p(y_1 | y_0): uniform area, cosine emission to the front, area conversion */
        double f = c0 > 0 ? (1.0 / s->em_area) * (c0 / PI) * cv / d2 : 0.0;
        double q1 = 1.0 / s->em_area;
        double q3 = side_prob(mv, c->v.n, vscl(w, -1.0)) * (cv / PI) * fabs(c0) / d2;
        return f / (0.5 * (q1 + q3));
    }
    /* class B: g = y_1 (diffuse), h_c = y_0 on the light */
    v3 y0 = c->hc.p, n0 = c->hc.n;
    int p0 = c->hc.prim;
    hit_t h;
    if (strat == 0) {
        v3 w = cosine_dir(n0, rng_u01(r), rng_u01(r));
        cc->rays++;
        if (!trace_closest(s, y0, w, s->tmin, 1e300, p0, -1, &h)) return 0.0;
        if (s->mat[s->tri[h.prim].mat].spec) return 0.0;
        y = hit_point(s, &h); ny = s->tri[h.prim].n; prim = h.prim;
        cc->rays++;
        if (!visible(s, y, prim, c->v.p, c->v.prim)) return 0.0;
    } else {
        v3 w = spec_start_dir(mv, c->v.n, r);
        cc->rays++;
        if (!trace_closest(s, c->v.p, w, s->tmin, 1e300, c->v.prim, -1, &h)) return 0.0;
        if (s->mat[s->tri[h.prim].mat].spec) return 0.0;
        y = hit_point(s, &h); ny = s->tri[h.prim].n; prim = h.prim;
        cc->rays++;
        if (!visible(s, y0, p0, y, prim)) return 0.0;
    }
    const mat_t *m1 = &s->mat[s->tri[prim].mat];
    v3 a = vsub(y, y0);
    double d01s = vdot(a, a), d01 = sqrt(d01s);
    v3 w01 = vscl(a, 1.0 / d01);
    double c0 = vdot(n0, w01), c1a = fabs(vdot(ny, w01));
    v3 b = vsub(c->v.p, y);
    double d1vs = vdot(b, b), d1v = sqrt(d1vs);
    v3 w1v = vscl(b, 1.0 / d1v);
    double c1b = fabs(vdot(ny, w1v)), cv = fabs(vdot(c->v.n, w1v));
    /* p(y_1 | y_0): cosine emission, area conversion at y_1 */
    double p1 = c0 > 0 ? (c0 / PI) * c1a / d01s : 0.0;
    /* p(y_2 | y_1, y_0): the light tracer's BSDF sampling at y_1, area conversion at y_2 */
    double pb = bsdf_pdf(m1, ny, vscl(w01, -1.0), w1v);
    double f = p1 * pb * cv / d1vs;
    double q2 = p1;
    double q3 = side_prob(mv, c->v.n, vscl(w1v, -1.0)) * (cv / PI) * c1b / d1vs;
    return f / (0.5 * (q2 + q3));
}

/* u >= 2: only tracing from y_{s-1} is available (Section 5.3). Dirac vertices inside g are
 * not integration variables (reading R10): both f and q carry the discrete lobe
 * probabilities, and the solid angle sampled at each non-Dirac vertex a is converted to area
 * at the next non-Dirac vertex b through a Jacobian J(a->b). Light's etendue is conserved
 * along the run, so J(a->b) / J(b->a) = (eta_b^2 |cos b|) / (eta_a^2 |cos a|), with eta the
 * index of the medium the run leaves a into and arrives at b from. Only that ratio enters
 * f/q; the common generalised geometry factor cancels. */
static double medium_eta(const mat_t *m, v3 n, v3 w_away)
{
    /* index of the medium on the side of w_away at a dielectric interface */
    if (m->type == MAT_DIELECTRIC) return vdot(n, w_away) > 0 ? 1.0 : m->ior;
    return 1.0;
}

static double fq_chain(cq_ctx *cc, rng_t *r)
{
    const scene_t *s = cc->s;
    const cand_t *c = cc->c;
    int u = c->u;
    /* trace g in reverse order: x[0] = y_{s-1}, x[1] = y_{s-2}, ..., x[u] = last dropped vertex */
    v3 xp[6], xn[6]; int xprim[6];
    const mat_t *xm[6];
    xp[0] = c->v.p; xn[0] = c->v.n; xprim[0] = c->v.prim; xm[0] = &s->mat[s->tri[c->v.prim].mat];
    v3 w = spec_start_dir(xm[0], xn[0], r);
    double q = side_prob(xm[0], xn[0], w) * fabs(vdot(xn[0], w)) / PI;   /* solid angle at y_{s-1} */
    double f = 1.0;
    for (int k = 1; k <= u; ++k) {
        hit_t h;
        cc->rays++;
        if (!trace_closest(s, xp[k - 1], w, s->tmin, 1e300, xprim[k - 1], -1, &h)) return 0.0;
        xp[k] = hit_point(s, &h); xn[k] = s->tri[h.prim].n; xprim[k] = h.prim; xm[k] = &s->mat[s->tri[h.prim].mat];
        if (k < u) {
            if (!xm[k]->spec) return 0.0;
            /* continue with the BSDF at this intermediate vertex, given the direction toward x[k-1] */
            v3 wo = vscl(w, -1.0);
            bsample_t bs = bsdf_sample(xm[k], xn[k], wo, rng_u01(r), rng_u01(r), rng_u01(r), MODE_CAMERA);
            if (!bs.ok) return 0.0;
            q *= bs.pdf;
            w = bs.wi;
        }
    }
    /* signature at the last vertex */
    if (c->cls == 0) { if (!xm[u]->emissive) return 0.0; }
    else { if (xm[u]->spec) return 0.0; }
    /* f: the light tracer's densities in light order, evaluated on the traced vertices.
     * light order index: y_j = x[u - j] for class A (y_0 = x[u]); for class B y_1 = x[u]. */
    /* density of each intermediate vertex's forward sampling (light mode), and the ratio of
     * the run Jacobians; anchors are the non-Dirac vertices. */
    /* the first light-order vertex of g: */
    int last = u;
    v3 dir_first = vnorm(vsub(xp[last - 1], xp[last]));     /* from the first dropped vertex toward the next */
    if (c->cls == 0) {
        double c0 = vdot(xn[last], dir_first);
        if (c0 <= 0) return 0.0;
        f *= (1.0 / s->em_area) * c0 / PI;                    /* p(y_0) and the cosine lobe (solid angle) */
    } else {
        /* y_1 = x[u] (diffuse): p(y_1 | y_0) in area measure, then its BSDF lobe toward y_2 */
        v3 a = vsub(xp[last], c->hc.p);
        double d2 = vdot(a, a), dist = sqrt(d2);
        v3 w01 = vscl(a, 1.0 / dist);
        double c0 = vdot(c->hc.n, w01);
        if (c0 <= 0) return 0.0;
        cc->rays++;
        if (!visible(s, c->hc.p, c->hc.prim, xp[last], xprim[last])) return 0.0;
        f *= (c0 / PI) * fabs(vdot(xn[last], w01)) / d2;
        f *= bsdf_pdf(xm[last], xn[last], vscl(w01, -1.0), dir_first);
    }
    if (f == 0.0) return 0.0;
    /* intermediate vertices x[u-1] .. x[1] in light order, and run Jacobians */
    int anchor = last;               /* current non-Dirac anchor (light side) */
    for (int k = last - 1; k >= 1; --k) {
        v3 w_light = vnorm(vsub(xp[k + 1], xp[k]));  /* toward the light side */
        v3 w_cam = vnorm(vsub(xp[k - 1], xp[k]));    /* toward y_{s-1} */
        if (xm[k]->delta) {
            f *= delta_lobe_prob(xm[k], xn[k], w_light, w_cam);
            if (f == 0.0) return 0.0;
        } else {
            /* close the run anchor -> k, then sample at k */
            v3 w_a = vnorm(vsub(xp[anchor - 1], xp[anchor]));
            double eta_a = medium_eta(xm[anchor], xn[anchor], w_a);
            double eta_b = medium_eta(xm[k], xn[k], w_light);
            f *= (eta_b * eta_b * fabs(vdot(xn[k], w_light))) / (eta_a * eta_a * fabs(vdot(xn[anchor], w_a)));
            f *= bsdf_pdf(xm[k], xn[k], w_light, w_cam);
            if (f == 0.0) return 0.0;
            anchor = k;
        }
    }
    /* final run anchor -> y_{s-1} */
    {
        v3 w_a = vnorm(vsub(xp[anchor - 1], xp[anchor]));
        v3 w_in = vnorm(vsub(xp[1], xp[0]));         /* at y_{s-1}, toward the light side */
        double eta_a = medium_eta(xm[anchor], xn[anchor], w_a);
        double eta_b = medium_eta(xm[0], xn[0], w_in);
        f *= (eta_b * eta_b * fabs(vdot(xn[0], w_in))) / (eta_a * eta_a * fabs(vdot(xn[anchor], w_a)));
    }
    return f / q;
}

static double cand_fq(void *p, rng_t *r)
{
    cq_ctx *cc = (cq_ctx *)p;
    return cc->c->u == 1 ? fq_u1(cc, r) : fq_chain(cc, r);
}

/* ---- per-iteration candidate processing ---- */
typedef struct {
    const scene_t *s; const or_params *p; struct o2_iter *it; int iter;
    double *fqmax, *fqsum, *fqn;   /* per kept candidate, per-chain sample statistics */
    double *trunc, *nsamp;
} recip_job;

/* wrapper sampler that records the f/q statistics of the samples it draws */
typedef struct { cq_ctx cq; double mx, sum, n; } rec_ctx;
static double rec_sample(void *p, rng_t *r)
{
    rec_ctx *rc = (rec_ctx *)p;
    double v = cand_fq(&rc->cq, r);
    if (v > rc->mx) rc->mx = v;
    rc->sum += v; rc->n += 1;
    return v;
}

/* pilot: fresh samples of the candidate's f/q, at least `pilot` of them, continuing until 8
 * non-zero values were seen or 16 x `pilot` samples were drawn */
static void pilot_one(void *ctx, int k)
{
    recip_job *j = (recip_job *)ctx;
    cand_t *c = &j->it->cand[j->it->kept[k]];
    rng_t r;
    rng_init(&r, j->p->seed, ST_PILOT, (uint32_t)k, (uint32_t)j->iter, 0);
    rec_ctx rc = {{j->s, c, 0}, 0, 0, 0};
    int nz = 0;
    for (int i = 0; i < 16 * j->p->pilot; ++i) {
        if (rec_sample(&rc, &r) > 0) nz++;
        if (i + 1 >= j->p->pilot && nz >= 8) break;
    }
    j->fqmax[k] = rc.mx; j->fqsum[k] = rc.sum; j->fqn[k] = rc.n;
}

static void recip_one(void *ctx, int k)
{
    recip_job *j = (recip_job *)ctx;
    cand_t *c = &j->it->cand[j->it->kept[k]];
    double B = c->B;
    rec_ctx rc = {{j->s, c, 0}, 0, 0, 0};
    double acc = 0, ns = 0, tr = 0;
    for (int e = 0; e < j->p->repeats; ++e) {
        rng_t r;
        rng_init(&r, j->p->seed, ST_RECIP, (uint32_t)k, (uint32_t)j->iter, (uint32_t)e);
        recip_ctx rcx = {rec_sample, &rc, &r, B, 0, j->p->chain_cap > 0 ? j->p->chain_cap : (1L << 21), 0};
        acc += itilde(&rcx);
        ns += (double)rcx.nsamp;
        tr += rcx.truncated;
    }
    c->recip = acc / j->p->repeats;
    j->fqmax[k] = rc.mx; j->fqsum[k] = rc.sum; j->fqn[k] = rc.n;
    j->nsamp[k] = ns; j->trunc[k] = tr;
}

/* Proxy connection at z_d (Sections 5.1, 5.4 and the settings of Section 6.1):
 * pick a kept candidate uniformly (pi_j = 1 / n_kept), connect z_d to y_{s-1}, retrace the
 * u dropped vertices by sampling the BSDF at y_{s-1} given the direction to z_d and then at
 * each new vertex, abort on an S/D mismatch (Section 5.1), and weight with the candidate's
 * reciprocal estimate. Normalisation M * pi_inc * pi_j (reading R12); p(h*) = 1 (class A) or
 * 1 / A (class B). Returns the contribution relative to the eye throughput at z_d. */
static double proxy_connect(const scene_t *s, const or_params *p, struct o2_iter *it, v3 xd, v3 nd, int primd,
                            const mat_t *md, v3 wo, int d, rng_t *r, double out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    if (it->nkept == 0) return 0.0;
    int k = (int)floor(rng_u01(r) * it->nkept);
    if (k >= it->nkept) k = it->nkept - 1;
    const cand_t *c = &it->cand[it->kept[k]];
    double pi_j = 1.0 / it->nkept;
    pthread_mutex_lock(&it->mu); it->proxy_attempts++; pthread_mutex_unlock(&it->mu);
    int segs = d + 1 + c->u + (c->cls == 0 ? 0 : 1 + c->j);
    if (segs > p->max_depth) return 0.0;
    v3 dv = vsub(c->v.p, xd);
    double d2 = vdot(dv, dv), dist = sqrt(d2);
    v3 wzv = vscl(dv, 1.0 / dist);
    double fz[3];
    bsdf_eval(md, nd, wo, wzv, fz);
    if (fz[0] == 0 && fz[1] == 0 && fz[2] == 0) return 0.0;
    double G = fabs(vdot(nd, wzv)) * fabs(vdot(c->v.n, wzv)) / d2;
    if (!visible(s, xd, primd, c->v.p, c->v.prim)) return 0.0;
    double thr[3] = {1, 1, 1};
    v3 cur = c->v.p, w_o = vscl(wzv, -1.0);
    int curprim = c->v.prim;
    v3 curn = c->v.n;
    double term[3] = {0, 0, 0};
    for (int step = 1; step <= c->u; ++step) {
        const mat_t *m = &s->mat[s->tri[curprim].mat];
        bsample_t bs = bsdf_sample(m, curn, w_o, rng_u01(r), rng_u01(r), rng_u01(r), MODE_CAMERA);
        if (!bs.ok) return 0.0;
        for (int q = 0; q < 3; ++q) thr[q] *= bs.w[q];
        hit_t h;
        if (!trace_closest(s, cur, bs.wi, s->tmin, 1e300, curprim, -1, &h)) return 0.0;
        const mat_t *mh = &s->mat[s->tri[h.prim].mat];
        v3 x = hit_point(s, &h);
        if (step < c->u) {
            if (!mh->spec) return 0.0;
        } else if (c->cls == 0) {
            if (!mh->emissive) return 0.0;
            emitted(s, h.prim, h.b1, h.b2, vscl(bs.wi, -1.0), term);
        } else {
            if (mh->spec) return 0.0;
            v3 a = vsub(c->hc.p, x);
            double e2 = vdot(a, a), e = sqrt(e2);
            v3 wl = vscl(a, 1.0 / e);
            double c0 = vdot(c->hc.n, vscl(wl, -1.0));
            if (c0 <= 0) return 0.0;
            double f1[3];
            bsdf_eval(mh, s->tri[h.prim].n, vscl(bs.wi, -1.0), wl, f1);
            if (f1[0] == 0 && f1[1] == 0 && f1[2] == 0) return 0.0;
            if (!visible(s, x, h.prim, c->hc.p, c->hc.prim)) return 0.0;
            double G01 = c0 * fabs(vdot(s->tri[h.prim].n, wl)) / e2;
            if (c->cls == 1) {
                double le[3];
                emitted(s, c->hc.prim, c->hc.b1, c->hc.b2, vscl(wl, -1.0), le);
                for (int q = 0; q < 3; ++q) term[q] = f1[q] * G01 * le[q] * s->em_area;   /* / p(h*) */
            } else {
                /* class C: the light throughput arriving at h_c, its BSDF from the control
                 * direction toward x, the geometry term h_c <-> x */
                double f0[3];
                bsdf_eval(&s->mat[s->tri[c->hc.prim].mat], s->tri[c->hc.prim].n, c->wc, vscl(wl, -1.0), f0);
                for (int q = 0; q < 3; ++q) term[q] = f1[q] * G01 * f0[q] * c->hc.beta[q];
            }
        }
        cur = x; curprim = h.prim; curn = s->tri[h.prim].n; w_o = vscl(bs.wi, -1.0);
    }
    double scale = c->recip / ((double)it->M * it->pi_inc * c->rho * pi_j);
    for (int q = 0; q < 3; ++q) out[q] = fz[q] * G * thr[q] * term[q] * scale;
    if (out[0] > 0 || out[1] > 0 || out[2] > 0) {
        pthread_mutex_lock(&it->mu); it->proxy_valid++; pthread_mutex_unlock(&it->mu);
    }
    return 1.0;
}

/* ------------------------------------------------------------------------- */
/* render entry point                                                         */
/* ------------------------------------------------------------------------- */
/* ------------------------------------------------------------------------- */
/* O3: plain bidirectional path tracing (Section 3.1)                         */
/* ------------------------------------------------------------------------- */
/* Every pixel sample traces one eye sub-path z_0 (the pinhole) z_1 .. z_D and one light
 * sub-path y_0 .. y_{D-1} (D = max_depth) and forms every full path x = y_0..y_{s-1}
 * z_{t-1}..z_0 of at most D segments (n = s + t - 1): s = 0 is an eye sub-path that hits an
 * emitter, s = 1 joins z_{t-1} to y_0, s >= 2 joins z_{t-1} to y_{s-1}, and t = 1 joins
 * y_{s-1} to the pinhole and adds the result to the pixel that the join passes through (light
 * tracing; the W * H light sub-paths of an iteration all do this, so each splat is divided by
 * W * H). The contribution of a strategy is f(x) / p_s(x) with f = L_e T W_e (path integral
 * equation, Section 3.1) and p_s = p(y) p(z), the product of the tracing densities of its
 * vertices in area measure (tracing pdf equation).
 *
 * Weights: the balance heuristic over the strategies s' = 0 .. n that can build x, each
 * density q_s' written out as the product over the path's vertices of the density with which
 * the light side (vertices below s') or the eye side (the others) generates them; light
 * tracing counts W * H samples per pixel, every other strategy one. A Dirac vertex has no
 * area density: the factor for the vertex generated across it is taken as 1 from both sides,
 * and a strategy whose joining segment ends at a Dirac vertex cannot build x (weight 0).
 * Any weights that sum to one over the strategies able to build x keep the sum unbiased
 * (the weights only need to be a partition of unity), so the uniform and the light-tracing-
 * only variants (o3_weights 1, 2) estimate the same image and pin each strategy's raw
 * contribution. */
#define O3_MAXD 128
typedef struct {
    v3 p, n;
    int prim;
    double b1, b2;
    const mat_t *m;
    double beta[3];   /* eye: W_e / p product up to here; light: L_e / p up to here (no BSDF at this vertex) */
} o3_vert;

typedef struct {
    const scene_t *s; const or_params *p;
    int iter;
    double *frame;          /* per-iteration pixel values (H * W * 3) */
    int *spl_pix;           /* per-row splat lists: row py holds at most W * D entries */
    double *spl_val;
    int *spl_n;
} o3_ctx;

/* image-plane position of direction d from the pinhole; 0 if it misses the image */
static int o3_project(const scene_t *s, v3 d, int *pix, double *cos_cam)
{
    double cf = vdot(d, s->cam_f);
    if (cf <= 0) return 0;
    double aspect = (double)s->W / s->H;
    double X = vdot(d, s->cam_r) / cf, Y = vdot(d, s->cam_u) / cf;
    double fx = (X / (s->tan_half * aspect) + 1.0) * 0.5 * s->W;
    double fy = (1.0 - Y / s->tan_half) * 0.5 * s->H;
    if (!(fx >= 0 && fx < s->W && fy >= 0 && fy < s->H)) return 0;
    *pix = (int)floor(fy) * s->W + (int)floor(fx);
    *cos_cam = cf;
    return 1;
}

/* pixel sensitivity per solid angle, W_e = 1 / (a_pix cos^3): uniform over the pixel's area on
 * the image plane at unit distance, which is also the eye sub-path's density of its first direction */
static double o3_we(const scene_t *s, double cos_cam)
{
    double aspect = (double)s->W / s->H;
    double a_pix = (2.0 * s->tan_half * aspect / s->W) * (2.0 * s->tan_half / s->H);
    return 1.0 / (a_pix * cos_cam * cos_cam * cos_cam);
}

/* vertex i of the full path for strategy s: x_0..x_{s-1} = y, x_s..x_{n-1} = z_{n-s}..z_1 */
static const o3_vert *o3_x(const o3_vert *Y, const o3_vert *Z, int s, int n, int i)
{
    return i < s ? &Y[i] : &Z[n - i];
}

static double o3_geo(v3 a, v3 na, v3 b, v3 nb, double *ca, double *cb)
{
    v3 d = vsub(b, a);
    double r2 = vdot(d, d);
    v3 w = vscl(d, 1.0 / sqrt(r2));
    *ca = vdot(na, w); *cb = -vdot(nb, w);
    return r2;
}

/* the weight of strategy s for the path it built (n segments) */
static double o3_weight(const scene_t *s, const or_params *p, const o3_vert *Y, const o3_vert *Z, int st, int n)
{
    if (p->o3_weights == 2) return st == n ? 1.0 : 0.0;
    double pl[O3_MAXD + 1], pe[O3_MAXD + 1];
    int dirac[O3_MAXD + 1];
    const double NL = (double)s->W * s->H;
    for (int i = 0; i < n; ++i) {
        const o3_vert *v = o3_x(Y, Z, st, n, i);
        dirac[i] = i > 0 && v->m->delta;
    }
    /* light-side densities: y_0 by area, y_1 by cosine emission, then BSDF sampling */
    for (int i = 0; i < n; ++i) {
        const o3_vert *v = o3_x(Y, Z, st, n, i);
        if (i == 0) { pl[0] = 1.0 / s->em_area; continue; }
        const o3_vert *a = o3_x(Y, Z, st, n, i - 1);
        double ca, cb, r2 = o3_geo(a->p, a->n, v->p, v->n, &ca, &cb);
        if (i == 1) { pl[1] = fmax(ca, 0.0) / PI * fabs(cb) / r2; continue; }
        if (dirac[i - 1]) { pl[i] = 1.0; continue; }
        const o3_vert *b = o3_x(Y, Z, st, n, i - 2);
        v3 wo = vnorm(vsub(b->p, a->p)), wi = vnorm(vsub(v->p, a->p));
        pl[i] = bsdf_pdf(a->m, a->n, wo, wi) * fabs(cb) / r2;
    }
    /* eye-side densities: x_{n-1} through the pixel, then BSDF sampling toward the light */
    for (int i = n - 1; i >= 0; --i) {
        const o3_vert *v = o3_x(Y, Z, st, n, i);
        if (i == n - 1) {
            v3 d = vsub(v->p, s->cam_p);
            double r2 = vdot(d, d);
            v3 w = vscl(d, 1.0 / sqrt(r2));
            double cf = vdot(w, s->cam_f);
            pe[i] = cf > 0 ? o3_we(s, cf) * fabs(vdot(v->n, w)) / r2 : 0.0;
            continue;
        }
        const o3_vert *a = o3_x(Y, Z, st, n, i + 1);
        if (dirac[i + 1]) { pe[i] = 1.0; continue; }
        v3 bp = i + 2 == n ? s->cam_p : o3_x(Y, Z, st, n, i + 2)->p;
        double ca, cb, r2 = o3_geo(a->p, a->n, v->p, v->n, &ca, &cb);
        v3 wo = vnorm(vsub(bp, a->p)), wi = vnorm(vsub(v->p, a->p));
        pe[i] = bsdf_pdf(a->m, a->n, wo, wi) * fabs(cb) / r2;
    }
    double qs = 0.0, sum = 0.0;
    int nvalid = 0;
    for (int sp = 0; sp <= n; ++sp) {
        /* the joining segment x_{sp-1} x_sp may not end at a Dirac vertex */
        if (sp >= 1 && sp <= n - 1 && (dirac[sp - 1] || dirac[sp])) continue;
        if (sp == n && dirac[n - 1]) continue;
        double q = sp == n ? NL : 1.0;
        for (int i = 0; i < sp; ++i) q *= pl[i];
        for (int i = sp; i < n; ++i) q *= pe[i];
        if (!(q > 0)) continue;
        nvalid++;
        sum += q;
        if (sp == st) qs = q;
    }
    if (p->o3_weights == 1) return qs > 0 ? 1.0 / nvalid : 0.0;
    return sum > 0 ? qs / sum : 0.0;
}

static void o3_pixel(const o3_ctx *c, int px, int py)
{
    const scene_t *s = c->s;
    const or_params *p = c->p;
    const int D = p->max_depth, pix = py * s->W + px;
    o3_vert Z[O3_MAXD + 2], Y[O3_MAXD + 1];
    int nz = 0, ny = 0;   /* eye vertices z_1..z_nz, light vertices y_0..y_{ny-1} */
    rng_t r;
    /* eye sub-path */
    rng_init(&r, p->seed, ST_BDPT, (uint32_t)pix, (uint32_t)c->iter, 0);
    v3 o, d;
    camera_ray(s, px, py, rng_u01(&r), rng_u01(&r), &o, &d);
    Z[0].p = s->cam_p; Z[0].n = s->cam_f; Z[0].prim = -1; Z[0].m = NULL;
    double beta[3] = {1, 1, 1};
    int ign = -1;
    while (nz < D) {
        hit_t h;
        if (!trace_closest(s, o, d, s->tmin, 1e300, ign, -1, &h)) break;
        o3_vert *v = &Z[++nz];
        v->p = hit_point(s, &h); v->n = s->tri[h.prim].n; v->prim = h.prim; v->b1 = h.b1; v->b2 = h.b2;
        v->m = &s->mat[s->tri[h.prim].mat];
        for (int k = 0; k < 3; ++k) v->beta[k] = beta[k];
        if (nz == D) break;
        bsample_t bs = bsdf_sample(v->m, v->n, vscl(d, -1.0), rng_u01(&r), rng_u01(&r), rng_u01(&r), MODE_CAMERA);
        if (!bs.ok) break;
        for (int k = 0; k < 3; ++k) beta[k] *= bs.w[k];
        if (beta[0] == 0 && beta[1] == 0 && beta[2] == 0) break;
        o = v->p; d = bs.wi; ign = h.prim;
    }
    /* light sub-path: y_0 uniform by area, cosine emission, BSDF sampling (adjoint) */
    rng_init(&r, p->seed, ST_BDPT, (uint32_t)pix, (uint32_t)c->iter, 1);
    lpoint_t lp;
    if (D >= 1 && sample_light(s, &r, &lp)) {
        o3_vert *y0 = &Y[ny++];
        y0->p = lp.p; y0->n = lp.n; y0->prim = lp.prim; y0->b1 = lp.b1; y0->b2 = lp.b2;
        y0->m = &s->mat[s->tri[lp.prim].mat];
        y0->beta[0] = y0->beta[1] = y0->beta[2] = s->em_area;
        d = cosine_dir(lp.n, rng_u01(&r), rng_u01(&r));
        double le[3];
        emitted(s, lp.prim, lp.b1, lp.b2, d, le);
        for (int k = 0; k < 3; ++k) beta[k] = s->em_area * le[k] * PI;
        o = lp.p; ign = lp.prim;
        while (ny < D && (beta[0] > 0 || beta[1] > 0 || beta[2] > 0)) {
            hit_t h;
            if (!trace_closest(s, o, d, s->tmin, 1e300, ign, -1, &h)) break;
            o3_vert *v = &Y[ny++];
            v->p = hit_point(s, &h); v->n = s->tri[h.prim].n; v->prim = h.prim; v->b1 = h.b1; v->b2 = h.b2;
            v->m = &s->mat[s->tri[h.prim].mat];
            for (int k = 0; k < 3; ++k) v->beta[k] = beta[k];
            bsample_t bs = bsdf_sample(v->m, v->n, vscl(d, -1.0), rng_u01(&r), rng_u01(&r), rng_u01(&r), MODE_LIGHT);
            if (!bs.ok) break;
            for (int k = 0; k < 3; ++k) beta[k] *= bs.w[k];
            o = v->p; d = bs.wi; ign = h.prim;
        }
    }
    double L[3] = {0, 0, 0};
    /* t >= 2: strategies that end at the eye vertex z_{t-1} */
    for (int t = 2; t <= nz + 1; ++t) {
        const o3_vert *z = &Z[t - 1];
        v3 zprev = Z[t - 2].p;
        v3 wo = vnorm(vsub(zprev, z->p));
        if (z->m->emissive && t - 1 <= D) {   /* s = 0: the eye sub-path reached an emitter */
            double le[3];
            emitted(s, z->prim, z->b1, z->b2, wo, le);
            if (le[0] > 0 || le[1] > 0 || le[2] > 0) {
                double w = o3_weight(s, p, Y, Z, 0, t - 1);
                for (int k = 0; k < 3; ++k) L[k] += w * z->beta[k] * le[k];
            }
        }
        if (z->m->delta) continue;
        for (int sn = 1; sn <= ny && sn + t - 1 <= D; ++sn) {
            const o3_vert *y = &Y[sn - 1];
            if (sn >= 2 && y->m->delta) continue;
            double cy, cz, r2 = o3_geo(y->p, y->n, z->p, z->n, &cy, &cz);
            v3 wyz = vscl(vsub(z->p, y->p), 1.0 / sqrt(r2));
            double fy[3], fz[3];
            if (sn == 1) emitted(s, y->prim, y->b1, y->b2, wyz, fy);
            else bsdf_eval(y->m, y->n, vnorm(vsub(Y[sn - 2].p, y->p)), wyz, fy);
            bsdf_eval(z->m, z->n, wo, vscl(wyz, -1.0), fz);
            double g = (sn == 1 ? fmax(cy, 0.0) : fabs(cy)) * fabs(cz) / r2;
            double c[3];
            int any = 0;
            for (int k = 0; k < 3; ++k) { c[k] = y->beta[k] * fy[k] * g * fz[k] * z->beta[k]; any |= c[k] > 0; }
            if (!any || !visible(s, y->p, y->prim, z->p, z->prim)) continue;
            double w = o3_weight(s, p, Y, Z, sn, sn + t - 1);
            for (int k = 0; k < 3; ++k) L[k] += w * c[k];
        }
    }
    for (int k = 0; k < 3; ++k) c->frame[3 * pix + k] += L[k];
    /* t = 1: light tracing, the light vertex y_{s-1} joined to the pinhole */
    const double NL = (double)s->W * s->H;
    for (int sn = 1; sn <= ny && sn <= D; ++sn) {
        const o3_vert *y = &Y[sn - 1];
        if (sn >= 2 && y->m->delta) continue;
        v3 dc = vsub(y->p, s->cam_p);
        double r2 = vdot(dc, dc);
        v3 w = vscl(dc, 1.0 / sqrt(r2));
        int tp;
        double cf;
        if (!o3_project(s, w, &tp, &cf)) continue;
        double fy[3];
        v3 to_cam = vscl(w, -1.0);
        if (sn == 1) emitted(s, y->prim, y->b1, y->b2, to_cam, fy);
        else bsdf_eval(y->m, y->n, vnorm(vsub(Y[sn - 2].p, y->p)), to_cam, fy);
        double cy = vdot(y->n, to_cam);
        double g = (sn == 1 ? fmax(cy, 0.0) : fabs(cy)) / r2 * o3_we(s, cf) / NL;
        double cc[3];
        int any = 0;
        for (int k = 0; k < 3; ++k) { cc[k] = y->beta[k] * fy[k] * g; any |= cc[k] > 0; }
        if (!any || !visible(s, y->p, y->prim, s->cam_p, -1)) continue;
        /* the eye side of this path is the pinhole alone */
        double wgt = o3_weight(s, p, Y, Z, sn, sn);
        int *cnt = &c->spl_n[py];
        size_t at = (size_t)py * s->W * D + (size_t)*cnt;
        c->spl_pix[at] = tp;
        for (int k = 0; k < 3; ++k) c->spl_val[3 * at + k] = wgt * cc[k];
        (*cnt)++;
    }
}

static void o3_row(void *ctx, int py)
{
    const o3_ctx *c = (const o3_ctx *)ctx;
    c->spl_n[py] = 0;
    for (int px = 0; px < c->s->W; ++px) o3_pixel(c, px, py);
}

static int o3_render(const scene_t *s, const or_params *p, double *sum, double *sumsq)
{
    if (p->max_depth < 1 || p->max_depth > O3_MAXD) return -1;
    int threads = p->threads > 0 ? p->threads : 1;
    size_t npix = (size_t)s->W * s->H;
    o3_ctx c;
    c.s = s; c.p = p;
    c.frame = (double *)calloc(npix * 3, sizeof(double));
    c.spl_pix = (int *)malloc(sizeof(int) * npix * (size_t)p->max_depth);
    c.spl_val = (double *)malloc(sizeof(double) * 3 * npix * (size_t)p->max_depth);
    c.spl_n = (int *)calloc((size_t)s->H, sizeof(int));
    for (int it = 0; it < p->n_iter; ++it) {
        c.iter = p->first_iter + it;
        memset(c.frame, 0, sizeof(double) * npix * 3);
        parallel_for(s->H, threads, o3_row, &c);
        /* splats in row order, so the sums do not depend on the thread count */
        for (int py = 0; py < s->H; ++py)
            for (int e = 0; e < c.spl_n[py]; ++e) {
                size_t at = (size_t)py * s->W * p->max_depth + (size_t)e;
                for (int k = 0; k < 3; ++k) c.frame[3 * c.spl_pix[at] + k] += c.spl_val[3 * at + k];
            }
        for (size_t i = 0; i < npix * 3; ++i) { sum[i] += c.frame[i]; sumsq[i] += c.frame[i] * c.frame[i]; }
    }
    free(c.frame); free(c.spl_pix); free(c.spl_val); free(c.spl_n);
    return 0;
}

int or_render(void *sp, const or_params *p, double *sum, double *sumsq, or_stats *stats)
{
    scene_t *s = (scene_t *)sp;
    int npix = s->W * s->H;
    int threads = p->threads > 0 ? p->threads : 1;
    if (stats) memset(stats, 0, sizeof(*stats));
    if (p->method == 2) return o3_render(s, p, sum, sumsq);
    if (p->method == 0) {
        for (int it = 0; it < p->n_iter; ++it) {
            eye_ctx c = {s, p, sum, sumsq, p->first_iter + it, NULL};
            parallel_for(s->H, threads, eye_row, &c);
        }
        return 0;
    }
    /* O2 */
    struct o2_iter it;
    memset(&it, 0, sizeof(it));
    pthread_mutex_init(&it.mu, NULL);
    it.M = p->n_light;
    it.paths = (lpath_t *)calloc((size_t)it.M, sizeof(lpath_t));
    it.cand = (cand_t *)calloc((size_t)it.M * 4 + 1, sizeof(cand_t));
    it.kept = (int *)calloc((size_t)it.M * 4 + 1, sizeof(int));
    double *fqmax = (double *)calloc((size_t)it.M * 4 + 1, sizeof(double));
    double *fqsum = (double *)calloc((size_t)it.M * 4 + 1, sizeof(double));
    double *fqn = (double *)calloc((size_t)it.M * 4 + 1, sizeof(double));
    double *trunc = (double *)calloc((size_t)it.M * 4 + 1, sizeof(double));
    double *nsamp = (double *)calloc((size_t)it.M * 4 + 1, sizeof(double));
    /* running (class, u) statistics across iterations (reading R3) */
    double run_max[3][5], run_sum[3][5], run_n[3][5];
    memset(run_max, 0, sizeof(run_max)); memset(run_sum, 0, sizeof(run_sum)); memset(run_n, 0, sizeof(run_n));
    for (int iter = 0; iter < p->n_iter; ++iter) {
        int k = p->first_iter + iter;
        light_ctx lc = {s, p, &it, k};
        parallel_for(it.M, threads, light_path, &lc);
        it.ncand = 0;
        for (int l = 0; l < it.M; ++l)
            it.ncand += collect_candidates(&it.paths[l], p->u_max, p->general_cv, it.cand + it.ncand);
        /* keep each candidate independently with probability pi_inc = min(1, cap / n_cand) */
        it.pi_inc = it.ncand > 0 ? fmin(1.0, (double)p->cand_cap / it.ncand) : 1.0;
        rng_t rk;
        rng_init(&rk, p->seed, ST_CAND, (uint32_t)k, 0, 0);
        it.nkept = 0;
        for (int i = 0; i < it.ncand; ++i)
            if (rng_u01(&rk) < it.pi_inc) it.kept[it.nkept++] = i;
        /* B = max f/q (Section 4.2 / Appendix E), taken per candidate as the maximum of a pilot
         * of fresh samples of that candidate's own f/q (reading R3). A candidate whose pilot
         * saw only zeros falls back to its (class, u) bucket's running maximum over earlier
         * samples, then to the maximum over all buckets, then to 1 / A. */
        recip_job job = {s, p, &it, k, fqmax, fqsum, fqn, trunc, nsamp};
        if (p->pilot > 0) parallel_for(it.nkept, threads, pilot_one, &job);
        for (int i = 0; i < it.nkept; ++i) {
            const cand_t *c = &it.cand[it.kept[i]];
            if (p->pilot <= 0) { fqmax[i] = 0; continue; }
            if (fqmax[i] > run_max[c->cls][c->u]) run_max[c->cls][c->u] = fqmax[i];
            run_sum[c->cls][c->u] += fqsum[i]; run_n[c->cls][c->u] += fqn[i];
        }
        double gmax = 0;
        for (int a = 0; a < 3; ++a) for (int b = 0; b < 5; ++b) if (run_max[a][b] > gmax) gmax = run_max[a][b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 5; ++b) it.B[a][b] = run_max[a][b] > 0 ? run_max[a][b] : (gmax > 0 ? gmax : 1.0 / s->em_area);
        /* B_j = max(the candidate's pilot maximum, its (class, u) bucket's running maximum over
         * all earlier pilot and chain samples): the paper's per-bucket maximum of f/q (reading R3),
         * never below what this candidate's own pilot saw.
         * Cost roulette (reading R12b): the expected cost of candidate j's chains is
         * repeats * B_j / beta_j (Appendix E), beta_j estimated by the pilot mean (or by
         * B_j / (2 n_pilot) when the pilot saw only zeros). A candidate above cost_cap is kept with
         * probability rho_j = cost_cap / cost_j and its contribution is divided by rho_j. */
        rng_t rr;
        rng_init(&rr, p->seed, ST_CAND, (uint32_t)k, 1, 0);
        int nk = 0;
        for (int i = 0; i < it.nkept; ++i) {
            cand_t *c = &it.cand[it.kept[i]];
            double rho = 1.0;
            c->B = fqmax[i] > it.B[c->cls][c->u] ? fqmax[i] : it.B[c->cls][c->u];
            double beta = fqmax[i] > 0 ? fqsum[i] / fqn[i] : c->B / (2.0 * (fqn[i] > 0 ? fqn[i] : 1.0));
            double cost = p->repeats * c->B / beta;
            if (p->cost_cap > 0 && cost > p->cost_cap) rho = p->cost_cap / cost;
            c->rho = rho;
            if (rho >= 1.0 || rng_u01(&rr) < rho) {
                it.kept[nk] = it.kept[i];
                fqmax[nk] = fqmax[i]; fqsum[nk] = fqsum[i]; fqn[nk] = fqn[i];
                nk++;
            }
        }
        it.nkept = nk;
        parallel_for(it.nkept, threads, recip_one, &job);
        for (int i = 0; i < it.nkept; ++i) {
            const cand_t *c = &it.cand[it.kept[i]];
            if (fqmax[i] > run_max[c->cls][c->u]) run_max[c->cls][c->u] = fqmax[i];
            run_sum[c->cls][c->u] += fqsum[i]; run_n[c->cls][c->u] += fqn[i];
            if (stats) { stats->n_recip_samples += nsamp[i]; stats->n_recip_truncated += trunc[i]; }
            if (getenv("ORACLE_TRACE_CHAINS") && nsamp[i] > 20000)
                fprintf(stderr, "cand cls=%d u=%d B=%g pilot_mean=%g pilot_n=%g rho=%g samples=%g trunc=%g\n",
                        c->cls, c->u, c->B, fqsum[i] / (fqn[i] > 0 ? fqn[i] : 1), fqn[i], c->rho, nsamp[i], trunc[i]);
        }
        if (stats) { stats->n_cand += it.ncand; stats->n_kept += it.nkept; }
        eye_ctx c = {s, p, sum, sumsq, k, &it};
        parallel_for(s->H, threads, eye_row, &c);
    }
    if (stats) {
        stats->n_proxy_attempts = (double)it.proxy_attempts;
        stats->n_proxy_valid = (double)it.proxy_valid;
        for (int a = 0; a < 2; ++a) for (int b = 0; b < 5; ++b) stats->bucket_B[a][b] = it.B[a][b];
    }
    free(it.paths); free(it.cand); free(it.kept); free(fqmax); free(fqsum); free(fqn); free(trunc); free(nsamp);
    pthread_mutex_destroy(&it.mu);
    (void)npix;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* single-candidate reciprocal hook (pins of P for fixed incomplete sub-paths) */
/* ------------------------------------------------------------------------- */
/* vpos/vn: y_{s-1} and its triangle vprim; hc*: y_0 for class B. Writes n_est values of
 * the averaged f/q (a plain Monte Carlo estimate of P with `per` samples each) into
 * p_est, and n_est reciprocal estimates I~ with constant B into r_est. */
typedef struct {
    scene_t *s; cand_t *c; double B; int n_est, per; uint32_t seed;
    double *p_est, *r_est, *r_ns; int trunc;
} rc_job;
static void rc_run(void *ctx, int unused)
{
    (void)unused;
    rc_job *j = (rc_job *)ctx;
    for (int e = 0; e < j->n_est; ++e) {
        rng_t r;
        rng_init(&r, j->seed, ST_TEST, (uint32_t)e, 1, 0);
        cq_ctx cc = {j->s, j->c, 0};
        double acc = 0;
        for (int i = 0; i < j->per; ++i) acc += cand_fq(&cc, &r);
        j->p_est[e] = acc / j->per;
        rng_t r2;
        rng_init(&r2, j->seed, ST_TEST, (uint32_t)e, 2, 0);
        recip_ctx rc = {cand_fq, &cc, &r2, j->B, 0, 1L << 21, 0};
        j->r_est[e] = itilde(&rc);
        j->r_ns[e] = (double)rc.nsamp;
        j->trunc += rc.truncated;
    }
}
int or_recip_candidate(void *sp, int cls, int u, const double *vpos, int vprim, const double *hcpos, int hcprim,
                       double B, int n_est, int per, uint32_t seed, double *p_est, double *r_est, double *r_ns)
{
    scene_t *s = (scene_t *)sp;
    cand_t c;
    memset(&c, 0, sizeof(c));
    c.cls = cls; c.u = u;
    c.v.p = vmk(vpos[0], vpos[1], vpos[2]); c.v.prim = vprim; c.v.n = s->tri[vprim].n;
    c.v.is_s = 1;
    if (hcprim >= 0) { c.hc.p = vmk(hcpos[0], hcpos[1], hcpos[2]); c.hc.prim = hcprim; c.hc.n = s->tri[hcprim].n; }
    rc_job j = {s, &c, B, n_est, per, seed, p_est, r_est, r_ns, 0};
    parallel_for(1, 1, rc_run, &j);   /* on a pool thread: its large stack holds the recursion */
    return j.trunc;
}
