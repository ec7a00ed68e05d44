// Device-side building blocks of the gfx950 proxy-sampling BDPT path: float3 math, the
// Philox4x32-10 counter-based generator, the three BSDFs in FP32, emitter sampling, and
// the 4-wide BVH traversal (closest hit and any hit) with its stack in LDS.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pt_layout.h"

#define PT_PI 3.14159265358979323846f

// ----------------------------------------------------------------------------- float3
__device__ __forceinline__ float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ __forceinline__ float3 operator+(float3 a, float3 b) { return f3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 operator-(float3 a, float3 b) { return f3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 operator-(float3 a) { return f3(-a.x, -a.y, -a.z); }
__device__ __forceinline__ float3 operator*(float3 a, float s) { return f3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ float3 operator*(float3 a, float3 b) { return f3(a.x * b.x, a.y * b.y, a.z * b.z); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 cross3(float3 a, float3 b)
{
    return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float3 normalize3(float3 a) { return a * rsqrtf(dot3(a, a)); }
__device__ __forceinline__ bool nonzero3(float3 a) { return a.x > 0.f || a.y > 0.f || a.z > 0.f; }
__device__ __forceinline__ float3 xyz(float4 a) { return f3(a.x, a.y, a.z); }
__device__ __forceinline__ float lum(float3 a) { return 0.2126f * a.x + 0.7152f * a.y + 0.0722f * a.z; }

// ----------------------------------------------------------------------------- Philox4x32-10
// Salmon et al. 2011: ten rounds; each round multiplies words 0 and 2 by fixed odd constants
// (high/low halves of the 64-bit products), mixes with words 1 and 3 and the key, and the key
// advances by the golden-ratio Weyl constants between rounds.
struct Rng {
    uint32_t k0, k1, c0, c1, c2, c3;
    uint32_t b[4];
    int pos;
};
__device__ __forceinline__ void philox10(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                                         uint32_t c3, uint32_t out[4])
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}
// key = (seed, stream), counter = (a, b, c, block)
__device__ __forceinline__ Rng rng_make(uint32_t seed, uint32_t stream, uint32_t a, uint32_t b, uint32_t c)
{
    Rng r;
    r.k0 = seed; r.k1 = stream * 0x9E3779B1u + 0x7F4A7C15u;
    r.c0 = a; r.c1 = b; r.c2 = c; r.c3 = 0;
    r.pos = 4;
    return r;
}
__device__ __forceinline__ uint32_t rng_u32(Rng &r)
{
    if (r.pos == 4) { philox10(r.k0, r.k1, r.c0, r.c1, r.c2, r.c3, r.b); r.c3++; r.pos = 0; }
    // pos is uniform per thread but dynamic; select without indexing a private array
    const uint32_t v = r.pos == 0 ? r.b[0] : r.pos == 1 ? r.b[1] : r.pos == 2 ? r.b[2] : r.b[3];
    r.pos++;
    return v;
}
// uniform float in [0, 1) with 24 random bits
__device__ __forceinline__ float rng_f(Rng &r) { return (float)(rng_u32(r) >> 8) * (1.0f / 16777216.0f); }
// index in [0, n) from 32 random bits x: floor(x n / 2^32)
__device__ __forceinline__ int index_of(uint32_t x, int n) { return (int)__umulhi(x, (uint32_t)n); }
__device__ __forceinline__ int rng_index(Rng &r, int n) { return index_of(rng_u32(r), n); }
// the probability with which index_of returns i: the number of x with floor(x n / 2^32) = i,
// ceil((i + 1) 2^32 / n) - ceil(i 2^32 / n), over 2^32 (within n / 2^32 of 1 / n)
__device__ __forceinline__ double index_prob(int i, int n)
{
    const uint64_t a = (((uint64_t)i << 32) + (uint64_t)n - 1) / (uint64_t)n;
    const uint64_t b = (((uint64_t)(i + 1) << 32) + (uint64_t)n - 1) / (uint64_t)n;
    return (double)(b - a) * 2.3283064365386962890625e-10;
}
// the probability that a 24-bit rng_f draw lies below p: ceil(p 2^24) / 2^24, clamped to [0, 1]
__device__ __forceinline__ double below_prob(float p)
{
    if (!(p > 0.0f)) return 0.0;
    if (p >= 1.0f) return 1.0;
    return ceil((double)p * 16777216.0) * (1.0 / 16777216.0);
}

enum { S_LIGHT = 11, S_CAND = 12, S_PILOT = 13, S_RECIP = 14, S_EYE = 15, S_PROXY = 16, S_TABLE = 17,
       S_ROUL = 18, S_PRE = 19, S_KMEANS = 20, S_TILE = 21, S_MLP = 22 };

// ----------------------------------------------------------------------------- frames
// branchless orthonormal basis about a unit normal (Duff et al. 2017)
__device__ __forceinline__ void basis(float3 n, float3 &t, float3 &b)
{
    const float s = copysignf(1.0f, n.z);
    const float a = -1.0f / (s + n.z);
    const float c = n.x * n.y * a;
    t = f3(1.0f + s * n.x * n.x * a, s * c, -s * n.x);
    b = f3(c, s + n.y * n.y * a, -n.y);
}
__device__ __forceinline__ float3 cos_hemi(float3 n, float u1, float u2)
{
    float3 t, b;
    basis(n, t, b);
    const float r = sqrtf(u1);
    float sp, cp;
    __sincosf(2.0f * PT_PI * u2, &sp, &cp);
    const float z = sqrtf(fmaxf(0.0f, 1.0f - u1));
    return normalize3(t * (r * cp) + b * (r * sp) + n * z);
}

// ----------------------------------------------------------------------------- materials
__device__ __forceinline__ float schlick1(float f0, float c)
{
    const float m = 1.0f - c, m2 = m * m;
    return f0 + (1.0f - f0) * m2 * m2 * m;
}
// exact dielectric reflectance for light going from index ei (the side of the incident
// direction, cosine ci) to index et; writes the transmitted cosine
__device__ __forceinline__ float fresnel_exact(float ci, float ei, float et, float &ct)
{
    const float eta = ei / et;
    const float st2 = eta * eta * fmaxf(0.0f, 1.0f - ci * ci);
    if (st2 >= 1.0f) { ct = 0.0f; return 1.0f; }
    ct = sqrtf(1.0f - st2);
    const float a = ei * ci, b = et * ct, c = et * ci, d = ei * ct;
    const float rs = (a - b) / (a + b), rp = (c - d) / (c + d);
    return 0.5f * (rs * rs + rp * rp);
}
// GGX normal distribution with the sine computed from the cross product (no 1 - cos^2)
__device__ __forceinline__ float ggx_d(float alpha, float3 n, float3 h)
{
    const float c = dot3(n, h);
    if (c <= 0.0f) return 0.0f;
    const float3 x = cross3(n, h);
    const float a2 = alpha * alpha;
    const float den = c * c * a2 + dot3(x, x);
    return a2 / (PT_PI * den * den);
}
__device__ __forceinline__ float ggx_g1(float alpha, float3 n, float3 w)
{
    const float c = dot3(n, w);
    if (c <= 0.0f) return 0.0f;
    const float3 x = cross3(n, w);
    const float t2 = dot3(x, x) / (c * c);
    return 2.0f / (1.0f + sqrtf(1.0f + alpha * alpha * t2));
}

__device__ __forceinline__ float3 bsdf_f(const MatDev &m, float3 n, float3 wo, float3 wi)
{
    const float co = dot3(n, wo), ci = dot3(n, wi);
    if (m.type == MAT_LAMBERT) return co * ci > 0.0f ? m.rgb * (1.0f / PT_PI) : f3(0.f, 0.f, 0.f);
    if (m.type == MAT_CONDUCTOR && !(m.flags & MF_DELTA)) {
        if (co <= 0.0f || ci <= 0.0f) return f3(0.f, 0.f, 0.f);
        const float3 h = normalize3(wo + wi);
        const float k = ggx_d(m.alpha, n, h) * ggx_g1(m.alpha, n, wo) * ggx_g1(m.alpha, n, wi) / (4.0f * co * ci);
        const float c = dot3(wi, h);
        return f3(schlick1(m.rgb.x, c), schlick1(m.rgb.y, c), schlick1(m.rgb.z, c)) * k;
    }
    return f3(0.f, 0.f, 0.f);
}
__device__ __forceinline__ float bsdf_pdf(const MatDev &m, float3 n, float3 wo, float3 wi)
{
    const float co = dot3(n, wo), ci = dot3(n, wi);
    if (m.type == MAT_LAMBERT) return co * ci > 0.0f ? fabsf(ci) * (1.0f / PT_PI) : 0.0f;
    if (m.type == MAT_CONDUCTOR && !(m.flags & MF_DELTA)) {
        if (co <= 0.0f || ci <= 0.0f) return 0.0f;
        const float3 h = normalize3(wo + wi);
        const float oh = dot3(wo, h);
        return oh > 0.0f ? ggx_d(m.alpha, n, h) * dot3(n, h) / (4.0f * oh) : 0.0f;
    }
    return 0.0f;
}

struct BS {
    float3 wi;
    float3 w;       // f |cos| / pdf in the requested mode
    float pdf;      // solid angle (smooth lobes) or lobe probability (Dirac)
    bool ok, delta;
};
// radiance = true: wo faces the camera side and refraction scales by (eta_o / eta_i)^2;
// false: wo faces the light side and refraction carries weight 1
__device__ __forceinline__ BS bsdf_sample(const MatDev &m, float3 n, float3 wo, float u1, float u2, float u3,
                                          bool radiance)
{
    BS s;
    s.ok = false; s.delta = false; s.pdf = 0.0f; s.w = f3(0.f, 0.f, 0.f); s.wi = f3(0.f, 0.f, 1.f);
    const float co = dot3(n, wo);
    if (m.type == MAT_LAMBERT) {
        if (co == 0.0f) return s;
        const float3 ns = co > 0.0f ? n : -n;
        s.wi = cos_hemi(ns, u1, u2);
        const float ci = dot3(ns, s.wi);
        if (ci <= 0.0f) return s;
        s.pdf = ci * (1.0f / PT_PI);
        s.w = m.rgb;
        s.ok = true;
        return s;
    }
    if (m.type == MAT_CONDUCTOR) {
        if (co <= 0.0f) return s;
        if (m.flags & MF_DELTA) {
            s.wi = n * (2.0f * co) - wo;
            s.w = f3(schlick1(m.rgb.x, co), schlick1(m.rgb.y, co), schlick1(m.rgb.z, co));
            s.pdf = 1.0f; s.delta = true; s.ok = true;
            return s;
        }
        const float t2 = m.alpha * m.alpha * u1 / (1.0f - u1);
        const float ch = rsqrtf(1.0f + t2), sh = sqrtf(t2) * ch;
        float sp, cp;
        __sincosf(2.0f * PT_PI * u2, &sp, &cp);
        float3 t, b;
        basis(n, t, b);
        const float3 h = normalize3(t * (sh * cp) + b * (sh * sp) + n * ch);
        const float oh = dot3(wo, h);
        if (oh <= 0.0f) return s;
        s.wi = h * (2.0f * oh) - wo;
        const float ci = dot3(n, s.wi);
        if (ci <= 0.0f) return s;
        s.pdf = bsdf_pdf(m, n, wo, s.wi);
        if (!(s.pdf > 0.0f)) return s;
        s.w = bsdf_f(m, n, wo, s.wi) * (ci / s.pdf);
        s.ok = true;
        return s;
    }
    // smooth dielectric; the geometric normal points outside (index 1)
    if (co == 0.0f) return s;
    const bool out = co > 0.0f;
    const float3 ns = out ? n : -n;
    const float eo = out ? 1.0f : m.ior, ei = out ? m.ior : 1.0f;
    const float c = fabsf(co);
    float ct;
    const float F = fresnel_exact(c, eo, ei, ct);
    s.delta = true; s.ok = true;
    if (u1 < F) {
        s.wi = ns * (2.0f * c) - wo;
        s.pdf = F;
        s.w = f3(1.f, 1.f, 1.f);
    } else {
        const float r = eo / ei;
        s.wi = normalize3(wo * (-r) + ns * (r * c - ct));
        s.pdf = 1.0f - F;
        const float k = radiance ? r * r : 1.0f;
        s.w = f3(k, k, k);
    }
    return s;
}
// discrete lobe probability of a Dirac vertex mapping wa to wb
__device__ __forceinline__ float dirac_prob(const MatDev &m, float3 n, float3 wa, float3 wb)
{
    const float ca = dot3(n, wa);
    if (m.type == MAT_CONDUCTOR) return (ca > 0.0f && dot3(n, wb) > 0.0f) ? 1.0f : 0.0f;
    if (ca == 0.0f) return 0.0f;
    const bool out = ca > 0.0f;
    float ct;
    const float F = fresnel_exact(fabsf(ca), out ? 1.0f : m.ior, out ? m.ior : 1.0f, ct);
    return ca * dot3(n, wb) > 0.0f ? F : 1.0f - F;
}
// refractive index of the medium on the side of w at a surface of material m
__device__ __forceinline__ float side_eta(const MatDev &m, float3 n, float3 w)
{
    return (m.type == MAT_DIELECTRIC && dot3(n, w) < 0.0f) ? m.ior : 1.0f;
}

// ----------------------------------------------------------------------------- scene access
struct SceneDev {
    const BNode *__restrict__ nodes;
    const BNode8 *__restrict__ nodes8;     // the 8-wide tree (walked by kernels with 8-wide stacks), or null
    const TriIsect *__restrict__ tris;     // BVH order
    const TriShade *__restrict__ shade;    // BVH order
    const MatDev *__restrict__ mats;
    const float *__restrict__ tex;
    int tex_w, tex_h;
    const int *__restrict__ em_tri;        // emissive triangles (BVH order)
    const float *__restrict__ em_cdf;      // normalised cumulative areas
    int n_em;
    float em_area;
    float tmin;
    CamDev cam;
    float3 lo, inv_ext;   // scene box, for subspace features
};

__device__ __forceinline__ float3 emission(const SceneDev &S, int tri, float b1, float b2, float3 w_out)
{
    const TriShade &sh = S.shade[tri];
    const MatDev &m = S.mats[sh.mat];
    if (!(m.flags & MF_EMIT) || dot3(sh.n, w_out) <= 0.0f) return f3(0.f, 0.f, 0.f);
    float k = 1.0f;
    if (m.flags & MF_TEXTURED) {
        const float b0 = 1.0f - b1 - b2;
        const float u = b0 * sh.uv[0] + b1 * sh.uv[2] + b2 * sh.uv[4];
        const float v = b0 * sh.uv[1] + b1 * sh.uv[3] + b2 * sh.uv[5];
        const int ix = min(max((int)floorf(u * S.tex_w), 0), S.tex_w - 1);
        const int iy = min(max((int)floorf(v * S.tex_h), 0), S.tex_h - 1);
        k = S.tex[iy * S.tex_w + ix];
    }
    return m.le * k;
}

struct LPoint { float3 p, n; int tri; float b1, b2; };
__device__ __forceinline__ LPoint sample_emitter(const SceneDev &S, float u0, float u1, float u2)
{
    int lo = 0, hi = S.n_em - 1;
    while (lo < hi) { const int mid = (lo + hi) >> 1; if (S.em_cdf[mid] > u0) hi = mid; else lo = mid + 1; }
    LPoint L;
    L.tri = S.em_tri[lo];
    const TriIsect &t = S.tris[L.tri];
    const float su = sqrtf(u1);
    L.b1 = su * (1.0f - u2); L.b2 = su * u2;
    L.p = f3(t.v0[0], t.v0[1], t.v0[2]) + f3(t.e1[0], t.e1[1], t.e1[2]) * L.b1 + f3(t.e2[0], t.e2[1], t.e2[2]) * L.b2;
    L.n = S.shade[L.tri].n;
    return L;
}
__device__ __forceinline__ float3 tri_point(const SceneDev &S, int tri, float b1, float b2)
{
    const TriIsect &t = S.tris[tri];
    return f3(t.v0[0], t.v0[1], t.v0[2]) + f3(t.e1[0], t.e1[1], t.e1[2]) * b1 + f3(t.e2[0], t.e2[1], t.e2[2]) * b2;
}

// ----------------------------------------------------------------------------- traversal
struct Hit { float t, b1, b2; int tri; };

// Moller-Trumbore in FP32. The barycentric and distance bounds are tested on the numerators,
// scaled by the sign of the determinant against |det| (the same inequalities times |det| > 0), so
// a rejected triangle costs no division; an accepted one takes one hardware reciprocal.
__device__ __forceinline__ bool isect(const TriIsect &T, float3 o, float3 d, float tmin, float tmax, float &t,
                                      float &b1, float &b2)
{
    const float3 e1 = f3(T.e1[0], T.e1[1], T.e1[2]), e2 = f3(T.e2[0], T.e2[1], T.e2[2]);
    const float3 pv = cross3(d, e2);
    const float det = dot3(e1, pv);
    if (det == 0.0f) return false;
    const float sg = det > 0.0f ? 1.0f : -1.0f, adet = fabsf(det);
    const float3 tv = o - f3(T.v0[0], T.v0[1], T.v0[2]);
    const float u = dot3(tv, pv) * sg;
    if (u < 0.0f || u > adet) return false;
    const float3 qv = cross3(tv, e1);
    const float v = dot3(d, qv) * sg;
    if (v < 0.0f || u + v > adet) return false;
    const float tt = dot3(e2, qv) * sg;
    if (!(tt > tmin * adet && tt < tmax * adet)) return false;
    const float inv = __builtin_amdgcn_rcpf(adet);
    t = tt * inv; b1 = u * inv; b2 = v * inv;
    return t > tmin && t < tmax;
}

// The traversal stack lives in LDS, column-major so that a wavefront's pushes and pops hit
// different banks: 32-bit entries put entry k of thread i at k * nthreads + i; 16-bit entries
// (trees of fewer than 65,536 nodes, half the LDS) pack entries 2j and 2j + 1 of thread i into
// the two halves of dword j * nthreads + i. A thread's pointer is its column's first element
// (stk_col).
//
// The entry type also selects the tree a kernel walks, at compile time: uint16_t and int walk the
// 4-wide nodes, int16_t and uint32_t (the same sizes) the 8-wide ones, so that a kernel holds the
// registers of one walk only. 16-bit entries hold node indices below 65,536 (int16_t ones read
// back through uint16_t).
template <typename SE> struct stk_wide8 { static constexpr bool value = false; };
template <> struct stk_wide8<int16_t> { static constexpr bool value = true; };
template <> struct stk_wide8<uint32_t> { static constexpr bool value = true; };
// entries per thread: the 8-wide walk pushes up to seven children a node
template <typename SE>
__host__ __device__ constexpr int stk_depth() { return stk_wide8<SE>::value ? PT_STACK8 : PT_STACK; }
template <typename SE>
__device__ __forceinline__ SE &stk_at(SE *stk, int k, int stride)
{
    if constexpr (sizeof(SE) == 2) return stk[(k >> 1) * 2 * stride + (k & 1)];
    else return stk[k * stride];
}
template <typename SE>
__device__ __forceinline__ int stk_node(SE v)
{
    if constexpr (sizeof(SE) == 2) return (int)(uint16_t)v;
    else return (int)v;
}
template <typename SE>
__device__ __forceinline__ SE *stk_col(SE *base, int thread) { return base + (sizeof(SE) == 2 ? 2 : 1) * thread; }

// the 8-wide walk (BNode8): the contract of traverse_rt below. A node is one 128-byte line read
// as seven 16-byte loads; a child plane at grid cell q lies at t = q * (2^(e-127) / d) +
// (org - o) / d, one FMA per plane. Children are taken in entry order through a 19-comparator
// network (Batcher's odd-even merge sort of eight).
template <bool COUNT, typename SE>
__device__ __forceinline__ bool traverse8_rt(const SceneDev &S, float3 o, float3 d, float tmin, float tmax, int ign0,
                                             int ign1, bool any, SE *stk, int stride, Hit &h, uint32_t *visits,
                                             uint32_t *tests, uint32_t *wave_trips)
{
    const float3 inv = f3(1.0f / d.x, 1.0f / d.y, 1.0f / d.z);
    h.tri = -1; h.t = tmax;
    int sp = 0;
    int node = 0;
    for (;;) {
        const uint4 *P = (const uint4 *)(S.nodes8 + node);
        if (COUNT) {
            (*visits)++;
            if (wave_trips && __lane_id() == __ffsll((long long)__ballot(1)) - 1) (*wave_trips)++;
        }
        const uint4 w0 = P[0], qx = P[1], qy = P[2], qz = P[3], c0 = P[4], c1 = P[5];
        const uint2 cn = *(const uint2 *)(P + 6);
        const float ax = __uint_as_float((w0.w & 0xFFu) << 23) * inv.x;
        const float ay = __uint_as_float(((w0.w >> 8) & 0xFFu) << 23) * inv.y;
        const float az = __uint_as_float(((w0.w >> 16) & 0xFFu) << 23) * inv.z;
        const float bx = (__uint_as_float(w0.x) - o.x) * inv.x;
        const float by = (__uint_as_float(w0.y) - o.y) * inv.y;
        const float bz = (__uint_as_float(w0.z) - o.z) * inv.z;
        const int cha[8] = {(int)c0.x, (int)c0.y, (int)c0.z, (int)c0.w, (int)c1.x, (int)c1.y, (int)c1.z, (int)c1.w};
        float tn[8];
        bool hitc[8];
        int cna[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int sh = 8 * (k & 3);
            const uint32_t lox = k < 4 ? qx.x : qx.y, hix = k < 4 ? qx.z : qx.w;
            const uint32_t loy = k < 4 ? qy.x : qy.y, hiy = k < 4 ? qy.z : qy.w;
            const uint32_t loz = k < 4 ? qz.x : qz.y, hiz = k < 4 ? qz.z : qz.w;
            const float tlx = (float)((lox >> sh) & 0xFFu) * ax + bx, thx = (float)((hix >> sh) & 0xFFu) * ax + bx;
            const float tly = (float)((loy >> sh) & 0xFFu) * ay + by, thy = (float)((hiy >> sh) & 0xFFu) * ay + by;
            const float tlz = (float)((loz >> sh) & 0xFFu) * az + bz, thz = (float)((hiz >> sh) & 0xFFu) * az + bz;
            const float t0 = fmaxf(fmaxf(fminf(tlx, thx), fminf(tly, thy)), fmaxf(fminf(tlz, thz), 0.0f));
            const float t1 = fminf(fminf(fmaxf(tlx, thx), fmaxf(tly, thy)), fminf(fmaxf(tlz, thz), h.t));
            cna[k] = (int)(((k < 4 ? cn.x : cn.y) >> sh) & 0xFFu);
            hitc[k] = t0 <= t1 * 1.00000024f && cna[k] != PT_CHILD_EMPTY;
            tn[k] = t0;
        }
        // leaves: one run over the hit leaves' triangles (as in the 4-wide walk)
        int e[8];
        int ntot = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            ntot += (hitc[k] && cna[k] > 0) ? cna[k] : 0;
            e[k] = ntot;
        }
        for (int j = 0; j < ntot; ++j) {
            int i = cha[7] + (j - e[6]);
#pragma unroll
            for (int k = 6; k >= 0; --k)
                if (j < e[k]) i = cha[k] + (j - (k > 0 ? e[k - 1] : 0));
            const TriIsect &T = S.tris[i];
            if (COUNT) (*tests)++;
            const int pid = T.prim;
            if (i == ign0 || i == ign1) continue;
            float t, b1, b2;
            if (isect(T, o, d, tmin, tmax, t, b1, b2)) {
                if (t < h.t || (t == h.t && h.tri >= 0 && pid < S.tris[h.tri].prim)) {
                    h.t = t; h.b1 = b1; h.b2 = b2; h.tri = i;
                    if (any) return true;
                }
            }
        }
        float key[8];
        int cid[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const bool take = hitc[k] && cna[k] == 0 && tn[k] <= h.t;
            key[k] = take ? tn[k] : 3.0e38f;
            cid[k] = take ? cha[k] : -1;
        }
#define PT_CSWAP(a, b)                                                                     \
        {                                                                                  \
            const bool sw = key[b] < key[a];                                               \
            const float ka = key[a], kb = key[b];                                          \
            const int ca = cid[a], cb = cid[b];                                            \
            key[a] = sw ? kb : ka; key[b] = sw ? ka : kb;                                  \
            cid[a] = sw ? cb : ca; cid[b] = sw ? ca : cb;                                  \
        }
        PT_CSWAP(0, 1) PT_CSWAP(2, 3) PT_CSWAP(4, 5) PT_CSWAP(6, 7)
        PT_CSWAP(0, 2) PT_CSWAP(1, 3) PT_CSWAP(4, 6) PT_CSWAP(5, 7)
        PT_CSWAP(1, 2) PT_CSWAP(5, 6)
        PT_CSWAP(0, 4) PT_CSWAP(1, 5) PT_CSWAP(2, 6) PT_CSWAP(3, 7)
        PT_CSWAP(2, 4) PT_CSWAP(3, 5)
        PT_CSWAP(1, 2) PT_CSWAP(3, 4) PT_CSWAP(5, 6)
#undef PT_CSWAP
        // as in the 4-wide walk, pt_scene_upload keeps the 8-wide tree only when its worst-case
        // walk fits the stack (PT_STACK8 entries); the bound only guards a malformed tree
        if (cid[0] >= 0) {
#pragma unroll
            for (int k = 7; k >= 1; --k)
                if (cid[k] >= 0 && sp < stk_depth<SE>()) stk_at(stk, sp++, stride) = (SE)cid[k];
            node = cid[0];
        } else {
            if (sp == 0) break;
            node = stk_node(stk_at(stk, --sp, stride));
        }
    }
    return h.tri >= 0;
}

// One walk of the 4-wide tree in progress: the ray, its reciprocal direction, the nearest hit so
// far, the node to visit next and the depth of the lane's stack. walk_step visits one node, so a
// kernel can interleave the walks of its lanes with other work (a lane whose walk ended can start
// another while the others still walk); traverse_rt runs walk_step to the end.
struct Walk {
    float3 o, d, inv, oi;
    float tmin, tmax;
    int ign0, ign1;
    bool any;
    int node, sp;
    Hit h;
};
__device__ __forceinline__ void walk_begin(Walk &w, float3 o, float3 d, float tmin, float tmax, int ign0, int ign1,
                                           bool any)
{
    w.o = o; w.d = d;
    w.inv = f3(1.0f / d.x, 1.0f / d.y, 1.0f / d.z);
    w.oi = o * w.inv;
    w.tmin = tmin; w.tmax = tmax; w.ign0 = ign0; w.ign1 = ign1; w.any = any;
    w.node = 0; w.sp = 0;
    w.h.tri = -1; w.h.t = tmax; w.h.b1 = w.h.b2 = 0.0f;
}
// visit w.node: true when the walk has ended (w.h holds the nearest hit, tri -1 for none; with
// `any` the first hit found)
template <bool COUNT, typename SE>
__device__ __forceinline__ bool walk_step(const SceneDev &S, Walk &w, SE *stk, int stride, uint32_t *visits,
                                          uint32_t *tests, uint32_t *wave_trips)
{
    const BNode &N = S.nodes[w.node];
    if (COUNT) {
        (*visits)++;
        // loop trips of the wavefront (counted by its first active lane): node visits over
        // 64 x trips is the SIMD efficiency of the traversal
        if (wave_trips && __lane_id() == __ffsll((long long)__ballot(1)) - 1) (*wave_trips)++;
    }
    // slab tests of the four children
    const float4 lx = *(const float4 *)N.lo_x, hx = *(const float4 *)N.hi_x;
    const float4 ly = *(const float4 *)N.lo_y, hy = *(const float4 *)N.hi_y;
    const float4 lz = *(const float4 *)N.lo_z, hz = *(const float4 *)N.hi_z;
    const int4 ch = *(const int4 *)N.child;
    const int4 cn = *(const int4 *)N.count;
    float tn[4];
    bool hitc[4];
    const float lxa[4] = {lx.x, lx.y, lx.z, lx.w}, hxa[4] = {hx.x, hx.y, hx.z, hx.w};
    const float lya[4] = {ly.x, ly.y, ly.z, ly.w}, hya[4] = {hy.x, hy.y, hy.z, hy.w};
    const float lza[4] = {lz.x, lz.y, lz.z, lz.w}, hza[4] = {hz.x, hz.y, hz.z, hz.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float ax = lxa[k] * w.inv.x - w.oi.x, bx = hxa[k] * w.inv.x - w.oi.x;
        const float ay = lya[k] * w.inv.y - w.oi.y, by = hya[k] * w.inv.y - w.oi.y;
        const float az = lza[k] * w.inv.z - w.oi.z, bz = hza[k] * w.inv.z - w.oi.z;
        const float t0 = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), 0.0f));
        const float t1 = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), w.h.t));
        hitc[k] = t0 <= t1 * 1.00000024f;
        tn[k] = t0;
    }
    const int cha[4] = {ch.x, ch.y, ch.z, ch.w}, cna[4] = {cn.x, cn.y, cn.z, cn.w};
    // leaves: test their triangles now, as one run over the hit leaves' triangles, so that a
    // wavefront's lanes step through their leaves together whichever children they are
    int e[4];
    int ntot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ntot += (hitc[k] && cna[k] > 0) ? cna[k] : 0;
        e[k] = ntot;   // end of child k's triangles in the run
    }
    for (int j = 0; j < ntot; ++j) {
        const int i = j < e[0] ? cha[0] + j
                    : j < e[1] ? cha[1] + (j - e[0])
                    : j < e[2] ? cha[2] + (j - e[1])
                               : cha[3] + (j - e[2]);
        const TriIsect &T = S.tris[i];
        if (COUNT) (*tests)++;
        const int pid = T.prim;
        if (i == w.ign0 || i == w.ign1) continue;
        float t, b1, b2;
        if (isect(T, w.o, w.d, w.tmin, w.tmax, t, b1, b2)) {
            if (t < w.h.t || (t == w.h.t && w.h.tri >= 0 && pid < S.tris[w.h.tri].prim)) {
                w.h.t = t; w.h.b1 = b1; w.h.b2 = b2; w.h.tri = i;
                if (w.any) return true;
            }
        }
    }
    // inner children still in front of the nearest hit, sorted by entry distance with a
    // five-comparator network in registers (children that are not taken sort last)
    float key[4];
    int cid[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool take = hitc[k] && cna[k] == 0 && cha[k] >= 0 && tn[k] <= w.h.t;
        key[k] = take ? tn[k] : 3.0e38f;
        cid[k] = take ? cha[k] : -1;
    }
#define PT_CSWAP(a, b)                                                                     \
    {                                                                                      \
        const bool sw = key[b] < key[a];                                                   \
        const float ka = key[a], kb = key[b];                                              \
        const int ca = cid[a], cb = cid[b];                                                \
        key[a] = sw ? kb : ka; key[b] = sw ? ka : kb;                                      \
        cid[a] = sw ? cb : ca; cid[b] = sw ? ca : cb;                                      \
    }
    PT_CSWAP(0, 1) PT_CSWAP(2, 3) PT_CSWAP(0, 2) PT_CSWAP(1, 3) PT_CSWAP(1, 2)
#undef PT_CSWAP
    // the nearest child continues in a register, the others are pushed far to near. The
    // stack holds PT_STACK entries, and pt_scene_upload rejects a tree whose worst-case walk
    // (the largest sum over a root-to-leaf path of inner children less one) needs more, so
    // the bound below only keeps a malformed tree from writing past the stack
    if (cid[0] >= 0) {
#pragma unroll
        for (int k = 3; k >= 1; --k)
            if (cid[k] >= 0 && w.sp < stk_depth<SE>()) stk_at(stk, w.sp++, stride) = (SE)cid[k];
        w.node = cid[0];
        return false;
    }
    if (w.sp == 0) return true;
    w.node = stk_node(stk_at(stk, --w.sp, stride));
    return false;
}

// `any` ends the walk at the first hit (visibility); it is a run-time argument so that a kernel
// can trace visibility and closest-hit rays at one call site, and constant-folds where the
// caller passes a constant. Stacks of int16_t or uint32_t entries walk the 8-wide tree.
template <bool COUNT, typename SE>
__device__ __forceinline__ bool traverse_rt(const SceneDev &S, float3 o, float3 d, float tmin, float tmax, int ign0,
                                            int ign1, bool any, SE *stk, int stride, Hit &h,
                                            uint32_t *visits = nullptr, uint32_t *tests = nullptr,
                                            uint32_t *wave_trips = nullptr)
{
    if constexpr (stk_wide8<SE>::value) {
        return traverse8_rt<COUNT>(S, o, d, tmin, tmax, ign0, ign1, any, stk, stride, h, visits, tests, wave_trips);
    } else {
        Walk w;
        walk_begin(w, o, d, tmin, tmax, ign0, ign1, any);
        while (!walk_step<COUNT>(S, w, stk, stride, visits, tests, wave_trips)) {
        }
        h = w.h;
        return h.tri >= 0;
    }
}

template <bool ANY, bool COUNT, typename SE>
__device__ __forceinline__ bool traverse(const SceneDev &S, float3 o, float3 d, float tmin, float tmax, int ign0,
                                         int ign1, SE *stk, int stride, Hit &h, uint32_t *visits = nullptr,
                                         uint32_t *tests = nullptr)
{
    return traverse_rt<COUNT>(S, o, d, tmin, tmax, ign0, ign1, ANY, stk, stride, h, visits, tests);
}
