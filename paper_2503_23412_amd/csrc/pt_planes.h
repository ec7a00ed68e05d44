// Photon planes for single scattering with the CMIS weight from reciprocal estimation
// (Section 6.7).
//
// A photon plane is drawn from a rectangular Lambertian light: a point y0 uniform on the light, a
// chord angle alpha uniform in [0, pi) (the chord of the rectangle through y0 along
// u_alpha = cos(alpha) U + sin(alpha) V) and a direction w cosine-distributed about the light's
// normal N = U x V; the plane is {y0 + s u_alpha + lambda w : s on the chord, lambda > 0}. An eye
// ray o + t d that meets it at x (t <= t_max) yields the single-scattering path (camera, x, y),
// y = y0 + s u_alpha on the light. The chord angle is the technique (continuous technique space
// [0, pi)); the density of the path under angle alpha, in measure dt dA(y), is
//     p(alpha, xbar) = (1/pi) (len(alpha; y) / A) (cos theta / pi) |u_alpha . m| / R^2,
// m = w x d, R = lambda, len(alpha; y) the chord through y at angle alpha (y0 uniform on the light
// gives the chord offset density len / A; the Jacobian of (offset, w) -> (t, y) is
// |(d x u_alpha) . w| / R^2). The balance-heuristic CMIS estimate of a hit is then
//     f / int_0^pi p(alpha', xbar) dalpha' = ss Le e^{-st (t + R)} pi A / (4 J),
//     J(y, m) = int_0^pi len(alpha; y) |u_alpha . m| dalpha,
// with the reciprocal 1/J estimated without bias by the RRS estimator of Section 4.2 (r = |g|):
// samples alpha' ~ q(alpha' | xbar), f/q = len(alpha'; y) |u_alpha' . m| / q(alpha'), mean J.
//
// The supporting density q is the cached piecewise approximation of q* ~ p(., xbar): a table
// over 16 x 16 cells of the light position and 32 bins of the angle of m's in-plane part (the
// only way d and w enter p's shape), each entry a 64-bin histogram of len(alpha; cell centre)
// |cos(alpha - phi)| over alpha, mixed with 10 % uniform (1/64 of it per bin) so that q covers p
// everywhere. Its integral Z (per unit |m|) sets B = 1.25 |m_in-plane| Z, near J. Each entry is a
// Walker alias table over its 64 bins of the mixture (a 6-bit column and a 24-bit threshold from
// one 32-bit draw; alpha then uniform in the bin) with the probability of every bin that this draw
// realises stored beside it, which q divides by: 4 MB.
//
// One launch gathers every plane of the iteration for every pixel's centre ray: a workgroup
// stages a tile of planes in LDS; each lane tests the whole tile against its ray (broadcast
// reads), keeps its hits as bits, and then the wavefront processes the hits of all its lanes
// together, one per lane per round, so the reciprocal chains run with most lanes busy.
#pragma once
#include "pt_kernels.h"

#define PL_CELLS 16     // light cells per axis
#define PL_PHI 32       // bins of the angle of m's in-plane part, over [0, pi)
#define PL_BINS 64      // alpha bins of one cached q
#define PL_ENTRIES (PL_CELLS * PL_CELLS * PL_PHI)
#define PL_TILE 256     // planes per LDS tile
#define PL_DEF 0.1f     // defensive uniform share of q
#define PL_CAP 4096u    // samples per reciprocal chain before it counts as truncated
#define PL_BSCALE 1.25f

enum { S_PLANE_GEN = 40, S_PLANE_HIT = 41 };
enum { PC_HITS = 0, PC_SAMPLES = 1, PC_TRUNC = 2, PC_NAN = 3, PC_COUNT = 4 };

struct PlaneDev {
    float3 c, U, V, N;
    float eu, ev, area;
    float3 le;
    float3 cam_p, cam_f, cam_r, cam_u;
    float tan_half, aspect;
    float ss, st, tmax;
    int w, h;
    const uint32_t *alias; // [PL_ENTRIES * PL_BINS] threshold (0 .. 2^24, low 25 bits) | alias bin << 25
    const float *pk;       // [PL_ENTRIES * PL_BINS] probability the alias draw realises per bin
    const float *z;        // [PL_ENTRIES] integral of the entry's profile over alpha
};

// one plane: y0.xyz = y0 - o for a point y0 on its chord and the camera position o; y0.w =
// (y0 - o) . n with n = u x w (both shared by every eye ray); n.w / u.w = the chord's parameter
// range; w.w = u . w
struct PlaneRec {
    float4 y0, n, u, w;
};

// length of the chord of [-eu, eu] x [-ev, ev] through (a, b) along (ca, sa)
__device__ __forceinline__ float pl_chord(float eu, float ev, float a, float b, float ca, float sa)
{
    float lo = -3.0e38f, hi = 3.0e38f;
    if (fabsf(ca) > 1e-20f) {
        const float r = __builtin_amdgcn_rcpf(ca);
        const float t0 = (-eu - a) * r, t1 = (eu - a) * r;
        lo = fmaxf(lo, fminf(t0, t1));
        hi = fminf(hi, fmaxf(t0, t1));
    }
    if (fabsf(sa) > 1e-20f) {
        const float r = __builtin_amdgcn_rcpf(sa);
        const float t0 = (-ev - b) * r, t1 = (ev - b) * r;
        lo = fmaxf(lo, fminf(t0, t1));
        hi = fminf(hi, fmaxf(t0, t1));
    }
    return fmaxf(hi - lo, 0.0f);
}

// the cache: one thread per (cell, phi) entry; the profile len(alpha; cell centre) |cos(alpha -
// phi)| integrated over each alpha bin (8-point midpoint rule), then Walker's alias table of the
// normalised bin masses (Vose's construction) with 24-bit thresholds, and the exact probability
// of each bin under the draw column = x >> 26, bin = (x & 0xFFFFFF) < threshold ? column : alias
__global__ void k_planes_cache(PlaneDev P, uint32_t *alias, float *pk, float *z)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= PL_ENTRIES) return;
    const int ip = e % PL_PHI, ic = e / PL_PHI;
    const int ia = ic % PL_CELLS, ib = ic / PL_CELLS;
    const float a = -P.eu + (ia + 0.5f) * (2.0f * P.eu / PL_CELLS);
    const float b = -P.ev + (ib + 0.5f) * (2.0f * P.ev / PL_CELLS);
    const float phi = (ip + 0.5f) * (PT_PI / PL_PHI);
    float mass[PL_BINS];
    float tot = 0.0f;
    const float h = PT_PI / PL_BINS;
#pragma unroll 1
    for (int k = 0; k < PL_BINS; ++k) {
        float s = 0.0f;
        for (int j = 0; j < 8; ++j) {
            const float al = (k + (j + 0.5f) / 8.0f) * h;
            s += pl_chord(P.eu, P.ev, a, b, cosf(al), sinf(al)) * fabsf(cosf(al - phi));
        }
        mass[k] = s * (h / 8.0f);
        tot += mass[k];
    }
    z[e] = tot;
    // the bin masses of the mixture with the defensive uniform share
#pragma unroll 1
    for (int k = 0; k < PL_BINS; ++k)
        mass[k] = PL_DEF / PL_BINS + (1.0f - PL_DEF) * (tot > 0.0f ? mass[k] / tot : 1.0f / PL_BINS);
    tot = 1.0f;
    // scaled masses n p_k; columns below 1 are filled by the alias of one at or above 1
    float sc[PL_BINS];
    int small[PL_BINS], large[PL_BINS], ns = 0, nl = 0;
    uint32_t *al = alias + (size_t)e * PL_BINS;
#pragma unroll 1
    for (int k = 0; k < PL_BINS; ++k) {
        sc[k] = mass[k] * PL_BINS;
        if (sc[k] < 1.0f) small[ns++] = k; else large[nl++] = k;
    }
    while (ns > 0 && nl > 0) {
        const int s0 = small[--ns], l0 = large[--nl];
        const uint32_t thr = (uint32_t)fminf(16777216.0f, fmaxf(0.0f, rintf(sc[s0] * 16777216.0f)));
        al[s0] = thr | ((uint32_t)l0 << 25);
        sc[l0] -= 1.0f - sc[s0];
        if (sc[l0] < 1.0f) small[ns++] = l0; else large[nl++] = l0;
    }
    while (nl > 0) { const int l0 = large[--nl]; al[l0] = 16777216u | ((uint32_t)l0 << 25); }
    while (ns > 0) { const int s0 = small[--ns]; al[s0] = 16777216u | ((uint32_t)s0 << 25); }
    // what the draw realises: column j keeps bin j below its threshold, else gives its alias
    float *pe = pk + (size_t)e * PL_BINS;
#pragma unroll 1
    for (int k = 0; k < PL_BINS; ++k) pe[k] = 0.0f;
#pragma unroll 1
    for (int j = 0; j < PL_BINS; ++j) {
        const uint32_t thr = min(al[j] & 0x1FFFFFFu, 16777216u), to = al[j] >> 25;
        pe[j] += (float)((double)thr / (16777216.0 * PL_BINS));
        if (thr < 16777216u) pe[to & 63u] += (float)((double)(16777216u - thr) / (16777216.0 * PL_BINS));
    }
}

// the planes of one iteration
__global__ void k_planes_gen(PlaneDev P, int n, uint32_t seed, uint32_t iter, PlaneRec *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Rng r = rng_make(seed, S_PLANE_GEN, (uint32_t)i, iter, 0u);
    const float a = (2.0f * rng_f(r) - 1.0f) * P.eu, b = (2.0f * rng_f(r) - 1.0f) * P.ev;
    const float al = PT_PI * rng_f(r);
    const float r1 = rng_f(r), r2 = rng_f(r);
    const float ph = 2.0f * PT_PI * r1, sr = sqrtf(r2), wz = sqrtf(fmaxf(0.0f, 1.0f - r2));
    const float3 y0 = P.c + P.U * a + P.V * b;
    const float3 w = P.N * wz + P.U * (sr * cosf(ph)) + P.V * (sr * sinf(ph));
    const float ca = cosf(al), sa = sinf(al);
    const float3 u = P.U * ca + P.V * sa;
    const float3 nn = cross3(u, w);
    float lo = -3.0e38f, hi = 3.0e38f;
    if (fabsf(ca) > 1e-20f) {
        const float t0 = (-P.eu - a) / ca, t1 = (P.eu - a) / ca;
        lo = fmaxf(lo, fminf(t0, t1)); hi = fminf(hi, fmaxf(t0, t1));
    }
    if (fabsf(sa) > 1e-20f) {
        const float t0 = (-P.ev - b) / sa, t1 = (P.ev - b) / sa;
        lo = fmaxf(lo, fminf(t0, t1)); hi = fminf(hi, fmaxf(t0, t1));
    }
    PlaneRec rec;
    const float3 yo = y0 - P.cam_p;
    rec.y0 = make_float4(yo.x, yo.y, yo.z, dot3(yo, nn));
    rec.n = make_float4(nn.x, nn.y, nn.z, lo);
    rec.u = make_float4(u.x, u.y, u.z, hi);
    rec.w = make_float4(w.x, w.y, w.z, dot3(u, w));
    out[i] = rec;
}

// the angle of (x, y) reduced to [0, pi) by a polynomial arctangent (error about 1e-3 rad)
__device__ __forceinline__ float pl_angle_pi(float x, float y)
{
    if (y < 0.0f || (y == 0.0f && x < 0.0f)) { x = -x; y = -y; }
    const float ax = fabsf(x), ay = fabsf(y);
    const float mn = fminf(ax, ay), mx = fmaxf(ax, ay);
    const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    float a = t * (0.78539816f + 0.273f * (1.0f - t));   // atan(t), 0 <= t <= 1
    if (ay > ax) a = 0.5f * PT_PI - a;
    return x < 0.0f ? PT_PI - a : a;
}

// the hit of plane R by the ray (o, d), if any: t, chord parameter s, lambda
__device__ __forceinline__ bool pl_hit(const PlaneDev &P, const PlaneRec &R, float3 d, float &t, float &sp,
                                       float &lam)
{
    const float den = d.x * R.n.x + d.y * R.n.y + d.z * R.n.z;
    t = R.y0.w * __builtin_amdgcn_rcpf(den);
    if (!(t > 0.0f && t <= P.tmax)) return false;
    const float3 q = d * t - xyz(R.y0);
    const float3 u = xyz(R.u), w = xyz(R.w);
    const float uw = R.w.w, idet = __builtin_amdgcn_rcpf(1.0f - uw * uw);
    const float qu = dot3(q, u), qw = dot3(q, w);
    sp = (qu - uw * qw) * idet;
    lam = (qw - uw * qu) * idet;
    return lam > 0.0f && sp >= R.n.w && sp <= R.u.w;
}

// the CMIS estimate of one hit (per unit Le), with 1/J from one RRS chain; ns += its samples,
// trunc += 1 when it reached PL_CAP samples
__device__ __forceinline__ float pl_estimate(const PlaneDev &P, const PlaneRec &R, float3 d, float t, float sp,
                                             float lam, Rng &r, uint32_t &ns, uint32_t &trunc)
{
    const float3 u = xyz(R.u), w = xyz(R.w);
    const float3 y = P.cam_p + xyz(R.y0) + u * sp;
    const float3 yc = y - P.c;
    const float a = dot3(yc, P.U), b = dot3(yc, P.V);
    const float3 m = cross3(w, d);
    const float mu = dot3(m, P.U), mv = dot3(m, P.V);
    const float mn = sqrtf(mu * mu + mv * mv);
    if (!(mn > 0.0f)) return 0.0f;
    const int ia = min(PL_CELLS - 1, max(0, (int)((a + P.eu) * (PL_CELLS / (2.0f * P.eu)))));
    const int ib = min(PL_CELLS - 1, max(0, (int)((b + P.ev) * (PL_CELLS / (2.0f * P.ev)))));
    // the bin of m's in-plane angle in [0, pi): a rough arctangent is enough (the entry only
    // chooses q, and the same entry gives q's density)
    const int ip = min(PL_PHI - 1, max(0, (int)(pl_angle_pi(mu, mv) * (PL_PHI / PT_PI))));
    const int e = (ib * PL_CELLS + ia) * PL_PHI + ip;
    const uint32_t *at = P.alias + (size_t)e * PL_BINS;
    const float *pe = P.pk + (size_t)e * PL_BINS;
    const float B = PL_BSCALE * mn * P.z[e];
    if (!(B > 0.0f)) return 0.0f;
    const float invB = 1.0f / B;
    const float h = PT_PI / PL_BINS;
    // Algorithm I~ with r = |g|: pending nodes counted by the sign of their prefix products
    float ans = invB;
    uint32_t pos = 1, neg = 0, nc = 0;
    while (pos + neg > 0) {
        if (nc >= PL_CAP) { trunc++; break; }
        float s = 1.0f;
        if (pos > 0) pos--; else { neg--; s = -1.0f; }
        // alpha' from the cached mixture: a bin by the alias draw, then uniform in the bin
        const uint32_t x = rng_u32(r);
        const uint32_t col = x >> 26, cell = at[col];
        const int k = (x & 0xFFFFFFu) < (cell & 0x1FFFFFFu) ? (int)col : (int)(cell >> 25);
        const float al = (k + rng_f(r)) * h;
        const float q = pe[k] * (PL_BINS / PT_PI);
        const float ca = __cosf(al), sa = __sinf(al);
        const float f = pl_chord(P.eu, P.ev, a, b, ca, sa) * fabsf(mu * ca + mv * sa);
        const float g = 1.0f - f * __builtin_amdgcn_rcpf(q * B);
        nc++;
        ans += s * g * invB;
        const float ag = fabsf(g), fl = floorf(ag);
        const uint32_t kids = (uint32_t)fminf(fl, 1.0e6f) + (rng_f(r) < ag - fl ? 1u : 0u);
        if ((s > 0.0f) == (g >= 0.0f)) pos += kids; else neg += kids;
    }
    ns += nc;
    return P.ss * __expf(-P.st * (t + lam)) * (PT_PI * 0.25f) * P.area * ans;
}

// every plane against every pixel's centre ray; acc/acc2 += the iteration's value / its square
__global__ void __launch_bounds__(256) k_planes_gather(PlaneDev P, const PlaneRec *__restrict__ planes, int n,
                                                       uint32_t seed, uint32_t iter, float *acc, float *acc2,
                                                       unsigned long long *cnt)
{
    __shared__ PlaneRec tile[PL_TILE];
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = pix < P.w * P.h;
    float3 d = f3(0.0f, 0.0f, 1.0f);
    if (live) {
        const int px = pix % P.w, py = pix / P.w;
        const float x = (2.0f * (px + 0.5f) / P.w - 1.0f) * P.tan_half * P.aspect;
        const float y = (1.0f - 2.0f * (py + 0.5f) / P.h) * P.tan_half;
        d = normalize3(P.cam_f + P.cam_r * x + P.cam_u * y);
    }
    float sum = 0.0f;
    uint32_t hits = 0, ns = 0, trunc = 0;
    for (int base = 0; base < n; base += PL_TILE) {
        const int cnt_t = min(PL_TILE, n - base);
        __syncthreads();
        for (int k = threadIdx.x; k < cnt_t; k += blockDim.x) tile[k] = planes[base + k];
        __syncthreads();
        // pass 1: which planes of the tile this lane's ray meets, as bits
        uint32_t mk[PL_TILE / 32];
#pragma unroll
        for (int wi = 0; wi < PL_TILE / 32; ++wi) {
            uint32_t bits = 0;
            for (int j = 0; j < 32; ++j) {
                const int k = wi * 32 + j;
                float t, sp, lam;
                if (live && k < cnt_t && pl_hit(P, tile[k], d, t, sp, lam)) bits |= 1u << j;
            }
            mk[wi] = bits;
        }
        // pass 2: the wavefront takes one hit per lane per round
#pragma unroll
        for (int wi = 0; wi < PL_TILE / 32; ++wi) {
            uint32_t bits = mk[wi];
            while (__any(bits != 0u)) {
                if (bits) {
                    const int j = __ffs(bits) - 1;
                    bits &= bits - 1u;
                    const int k = wi * 32 + j;
                    float t, sp, lam;
                    if (pl_hit(P, tile[k], d, t, sp, lam)) {
                        Rng r = rng_make(seed, S_PLANE_HIT, (uint32_t)pix, iter, (uint32_t)(base + k));
                        sum += pl_estimate(P, tile[k], d, t, sp, lam, r, ns, trunc);
                        hits++;
                    }
                }
            }
        }
    }
    if (live) {
        const float v = sum / (float)max(n, 1);
        const float3 c = P.le * v;
        const bool bad = !(v == v) || isinf(v);
        if (!bad) {
            acc[3 * pix + 0] += c.x; acc[3 * pix + 1] += c.y; acc[3 * pix + 2] += c.z;
            if (acc2) { acc2[3 * pix + 0] += c.x * c.x; acc2[3 * pix + 1] += c.y * c.y; acc2[3 * pix + 2] += c.z * c.z; }
        }
        if (bad) atomicAdd(cnt + PC_NAN, 1ull);
    }
    wave_count(cnt + PC_HITS, hits);
    wave_count(cnt + PC_SAMPLES, ns);
    wave_count(cnt + PC_TRUNC, trunc);
}
