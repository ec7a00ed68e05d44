// Memory layouts shared by the host code and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// 4-wide BVH node: one 128-byte line. Child k is empty when count[k] < 0, a leaf of
// count[k] > 0 consecutive triangles starting at child[k], or an inner node (count[k] == 0).
struct alignas(128) BNode {
    float lo_x[4], hi_x[4], lo_y[4], hi_y[4], lo_z[4], hi_z[4];
    int32_t child[4];
    int32_t count[4];
};
static_assert(sizeof(BNode) == 128, "BNode must be one 128-byte line");

// 8-wide BVH node, also one 128-byte line: the child boxes are quantised to 8 bits per plane
// on a per-node grid (compressed wide nodes in the manner of Ylitie, Karras and Laine, HPG 2017):
// child k spans [org + qlo[k] * 2^(e - 127), org + qhi[k] * 2^(e - 127)] on each axis, with e the
// biased float exponent of the axis's scale. The quantised box contains the child's exact box
// (lower planes rounded down, upper planes up). count[k]: 0 inner node child[k], 1..4 a leaf of
// that many consecutive triangles from child[k], PT_CHILD_EMPTY no child (child[k] = -1).
#define PT_CHILD_EMPTY 0xFF
struct alignas(128) BNode8 {
    float org[3];
    uint8_t e[3];
    uint8_t pad0;
    uint8_t qlo_x[8], qhi_x[8], qlo_y[8], qhi_y[8], qlo_z[8], qhi_z[8];
    int32_t child[8];
    uint8_t count[8];
    uint32_t pad1[6];
};
static_assert(sizeof(BNode8) == 128, "BNode8 must be one 128-byte line");

// Triangle for intersection (BVH order): 48 bytes.
struct alignas(16) TriIsect {
    float v0[3];
    float e1[3];
    float e2[3];
    int32_t prim;   // input triangle index
    int32_t pad[2];
};
static_assert(sizeof(TriIsect) == 48, "TriIsect must be 48 bytes");

// Shading data (BVH order): normal, material, per-vertex (u, v).
struct TriShade {
    float3 n;
    int32_t mat;
    float uv[6];
};

enum { MAT_LAMBERT = 0, MAT_CONDUCTOR = 1, MAT_DIELECTRIC = 2 };
enum { MF_EMIT = 1, MF_TEXTURED = 2, MF_SPEC = 4, MF_DELTA = 8 };

struct MatDev {
    int32_t type;
    uint32_t flags;
    float alpha, ior;
    float3 rgb;
    float3 le;
};

struct CamDev {
    float3 p, f, r, u;
    float tan_half, aspect;
    int32_t w, h;
};

// at most this many light vertices are kept per light sub-path: y_0 .. y_5, enough for a
// class B candidate with a specular run of 4
#define PT_LMAX 6
#define PT_LSTORE 16   // light vertices stored per path when light vertices are connected (SPC, LT)
#define PT_MAX_DEPTH 127   // longest path, in segments
enum { LV_S = 1, LV_DIRAC = 2 };   // per light vertex flags
#define PT_STACK 48    // traversal stack entries per thread, 4-wide walks
#define PT_STACK8 64   // and 8-wide walks

// Incomplete light sub-path candidate (y_{s-1} plus the control vertex), 96 bytes. Class A: h_c
// null; class B: h_c = y_0 on an emitter; class C (general control vertex): h_c = y_j, j >= 1, on a
// Lambertian surface, with its control direction and the light throughput arriving there.
struct Cand {
    float4 v;        // y_{s-1} position, w = triangle (bits)
    float4 hc;       // classes B, C: h_c position, w = triangle (bits)
    float hc_b1, hc_b2;   // class B: barycentrics of y_0; class C: octahedral encoding of the
                          // direction from h_c toward y_{j-1} (the reverse of the control direction)
    int32_t cls_u;   // j << 16 | class << 8 | u  (j: class C's light vertex index of h_c)
    float B;
    float rho;       // probability it survived the cost roulette
    float recip_sum; // sum of the reciprocal estimates of this iteration
    float pmax, psum, pn;
    int32_t spec_sub;// specular subspace S
    float pad[2];    // octahedral encoding of y_{s-1}'s incident direction (toward y_{s-2})
    float4 beta_c;   // class C: throughput arriving at h_c (rgb) from the light sub-path
};
static_assert(sizeof(Cand) == 96, "Cand layout");
#define PT_STAT_CU 15   // (class, u) pairs of the statistics: 3 classes x u = 0 .. 4
__host__ __device__ inline int cand_cls(int cls_u) { return (cls_u >> 8) & 0xFF; }
__host__ __device__ inline int cand_u(int cls_u) { return cls_u & 0xFF; }
__host__ __device__ inline int cand_j(int cls_u) { return cls_u >> 16; }

// Device counters of one iteration (64-bit so that large runs do not wrap).
enum {
    C_LIGHT_Q0 = 0,          // light queue counts per vertex index: 0 .. PT_LSTORE - 1
    C_EYE_Q0 = C_LIGHT_Q0 + PT_LSTORE,   // eye queue counts per depth 0 .. PT_MAX_DEPTH
    C_SHD0 = C_EYE_Q0 + PT_MAX_DEPTH + 1,   // shadow-ray queue counts per depth 0 .. PT_MAX_DEPTH
    C_PROXYQ = C_SHD0 + PT_MAX_DEPTH + 1, C_NCAND, C_NKEPT, C_NFINAL,
    C_RAYS_EYE, C_RAYS_LIGHT, C_RAYS_SHADOW, C_RAYS_PROXY, C_RAYS_RECIP,
    C_RECIP_SAMPLES, C_RECIP_TRUNC, C_LONGQ0, C_LONGQ1, C_CHAIN_HIST, C_CHAIN_MAX = C_CHAIN_HIST + 24, C_POOL, C_SPC, C_LT, C_PROXY_ATT, C_PROXY_VALID, C_NAN, C_VISITS, C_TESTS, C_VISITS_R, C_TESTS_R, C_VISITS_A, C_TESTS_A, C_TRIPS_A, C_SAMPLES_A, C_DRAWN_A, C_DRAWN_P, C_WORK_A, C_WORK_P, C_COSTH0, C_COSTF0 = C_COSTH0 + 16, C_STACK_OVF = C_COSTF0 + 16,
    C_MLP_N,                 // training samples of the subspace head recorded this iteration
    C_MLP_NV,                // training samples of the retrace-direction head recorded this iteration
    C_MLP_ROWS,              // training rows of this iteration (both heads, each capped)
    C_ITER, C_LEARN,         // iteration index and "still learning" flag (kept across k_zero)
    C_MLP_T,                 // Adam steps taken (kept across k_zero)
    C_COUNT
};
// a light sub-path has at most PT_LSTORE vertices and an eye path at most PT_MAX_DEPTH segments:
// every queue count has its own slot
static_assert(C_EYE_Q0 - C_LIGHT_Q0 >= PT_LSTORE, "light queue counters overlap");
static_assert(C_SHD0 - C_EYE_Q0 >= PT_MAX_DEPTH + 1 && C_PROXYQ - C_SHD0 >= PT_MAX_DEPTH + 1, "queue counters overlap");

// device wall-clock stamps of the start and end of the latest PT_TS_CAP iterations (ring by index)
#define PT_TS_CAP 4096

// running totals over the iterations of a scene (not cleared per iteration)
enum { TOT_ITERS = 0, TOT_NAN, TOT_TRUNC, TOT_PROXY_VALID, TOT_RECIP_SAMPLES, TOT_CAND, TOT_COUNT };

// queued shadow ray: origin + first ignored triangle, direction + tmax, contribution + pixel,
// second ignored triangle
struct ShadowRay {
    float4 o, d, c;
    int32_t ign1;
    int32_t tag;     // connection rays: eye subspace T << 12 | light subspace S_L (learning); else -1
    int32_t pad[2];
};
// proxy work item at an eye path's first diffuse vertex
struct ProxyItem {
    float4 x;        // position, w = triangle (bits)
    float4 wo;       // direction toward the previous eye vertex, w = segments so far (bits)
    float4 beta;     // eye throughput, w = pixel (bits)
    float4 aux;      // x = eye subspace T (bits), y = tile attempt probability c, z/w = learned selection
    float4 mis;      // x = eye-side area density of z_d, y = eye-side MIS partial at z_d (no connections)
};
