// gfx950 kernels of one proxy-sampling BDPT iteration.
//
// Light pass (Section 3.1's tracing pdf chain): k_light_gen -> (k_extend -> k_light_shade) per
// vertex, wavefront queues compacted with ballot + mbcnt, light vertices stored SoA.
// Candidates (Sections 5.1 and 6.1): k_candidates -> k_keep.
// Reciprocal estimates of 1/P (Sections 4.2, 5.2, 5.3): k_pilot -> k_roulette -> k_recip.
// Eye pass: k_camera -> (k_extend -> k_eye_shade -> k_occluded) per depth, then k_proxy
// (Section 5.1's retrace) and k_accumulate.
#pragma once
#include "pt_device.h"
#include "pt_subspace.h"

#define WG 128   // workgroup size of the traversal kernels (LDS stack 128 x 48 x 4 B = 24 KB)

__device__ __forceinline__ int fbits(float f) { return __float_as_int(f); }
__device__ __forceinline__ float ibits(int i) { return __int_as_float(i); }

// Wave-aggregated queue push: one atomic per wavefront, slots from the ballot prefix (mbcnt).
// Every lane of the wavefront must call it.
__device__ __forceinline__ int wave_push(unsigned long long *counter, bool pred)
{
    const unsigned long long mask = __ballot(pred);
    const int lane = __lane_id();
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    int base = 0;
    if (mask) {
        const int leader = __ffsll((long long)mask) - 1;
        if (lane == leader) base = (int)atomicAdd(counter, (unsigned long long)__popcll(mask));
        base = __shfl(base, leader);
    }
    return pred ? base + (int)below : -1;
}
__device__ __forceinline__ void wave_count(unsigned long long *counter, uint32_t v)
{
    // sum over the wavefront, one atomic
    uint32_t s = v;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (__lane_id() == 0 && s) atomicAdd(counter, (unsigned long long)s);
}
__device__ __forceinline__ void atomic_add3(float *p, float3 v)
{
    if (v.x != 0.0f) unsafeAtomicAdd(p + 0, v.x);
    if (v.y != 0.0f) unsafeAtomicAdd(p + 1, v.y);
    if (v.z != 0.0f) unsafeAtomicAdd(p + 2, v.z);
}
// max of non-negative floats through their integer bit patterns
__device__ __forceinline__ void atomic_maxf(float *p, float v)
{
    if (v > 0.0f) atomicMax((int *)p, __float_as_int(v));
}

// ---------------------------------------------------------------------------------- queues
__global__ void k_zero(unsigned long long *cnt, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && i != C_ITER && i != C_LEARN && i != C_MLP_T) cnt[i] = 0ull;
}
// iteration index in device memory: set (direct calls) or advanced by one (graph replays)
// (stamp: the iteration starts here; its device wall-clock time goes to the ring ts)
__global__ void k_iter(unsigned long long *cnt, uint32_t value, int advance, int train_iters, long long *ts, int stamp)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint32_t it = advance ? (uint32_t)cnt[C_ITER] + 1u : value;
        cnt[C_ITER] = it;
        cnt[C_LEARN] = (int)it < train_iters ? 1ull : 0ull;
        if (stamp && ts) {
            ts[2 * (it % PT_TS_CAP)] = wall_clock64();
            ts[2 * (it % PT_TS_CAP) + 1] = 0;
        }
    }
}
__device__ __forceinline__ uint32_t iter_of(const unsigned long long *cnt) { return (uint32_t)cnt[C_ITER]; }

// closest hit for every queued ray; rays live in (ro, rd) by path id, ro.w = ignored triangle,
// rd.w = tmax; writes hit[pid] = (t, b1, b2, triangle or -1). WGS threads per workgroup (the
// autotuner's choice of 64, 128 or 256; the LDS stack is stk_depth<SE>() x WGS entries)
template <bool COUNT, typename SE, int WGS = WG>
__global__ void __launch_bounds__(WGS) k_extend(SceneDev S, const uint32_t *__restrict__ q,
                                                const unsigned long long *__restrict__ cnt, int cidx,
                                                const float4 *__restrict__ ro, const float4 *__restrict__ rd,
                                                float4 *__restrict__ hit, unsigned long long *stats, int ray_ctr)
{
    __shared__ SE stk[stk_depth<SE>() * WGS];
    const int i = blockIdx.x * WGS + threadIdx.x;
    const int n = (int)cnt[cidx];
    uint32_t visits = 0, tests = 0;
    const bool act = i < n;
    if (act) {
        const int pid = q[i];
        const float4 o = ro[pid], d = rd[pid];
        Hit h;
        traverse<false, COUNT>(S, xyz(o), xyz(d), S.tmin, d.w, fbits(o.w), -1, stk_col(stk, (int)threadIdx.x), WGS, h,
                               &visits, &tests);
        hit[pid] = make_float4(h.t, h.b1, h.b2, ibits(h.tri));
    }
    wave_count(stats + ray_ctr, act ? 1u : 0u);
    if (COUNT) { wave_count(stats + C_VISITS, visits); wave_count(stats + C_TESTS, tests); }
}

// ---------------------------------------------------------------------------------- light pass
struct LightBuf {
    float4 *ro, *rd, *hit;
    float4 *lv;          // [PT_LSTORE * M]: position, w = triangle
    float4 *lt;          // [PT_LSTORE * M]: throughput arriving at the vertex (rgb), w = its forward
                         // area density (the light tracer's density of this vertex given the previous)
    float4 *lphi;        // [PT_LSTORE * M]: MIS partial sums of the strategies with fewer light vertices:
                         // x with connections, y without (proxy-class paths), z the emission-hit term alone
    uint8_t *lfl;        // [PT_LSTORE * M]: LV_S, LV_DIRAC
    float4 *lbeta;       // [M]: throughput and solid-angle pdf of the ray in flight
    float2 *lb0;         // [M]: barycentrics of y_0
    uint32_t *sig;       // [M]: bits 0..15 = vertex i specular, 16..23 = vertex i (< 8) Lambertian,
                         // 24..28 = vertex count
    uint32_t *q[2];
    uint32_t *pool;      // [PT_LSTORE * M]: vertices eye vertices may connect to (index i * M + path)
    int M;
};
__device__ __forceinline__ int sig_count(uint32_t sg) { return (int)((sg >> 24) & 0x1Fu); }

__global__ void k_light_gen(SceneDev S, LightBuf L, uint32_t seed, unsigned long long *cnt)
{
    const uint32_t iter = iter_of(cnt);
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l == 0) cnt[C_LIGHT_Q0] = (unsigned long long)L.M;
    if (l >= L.M) return;
    Rng r = rng_make(seed, S_LIGHT, (uint32_t)l, iter, 0u);
    const float u0 = rng_f(r), u1 = rng_f(r), u2 = rng_f(r);
    const LPoint y0 = sample_emitter(S, u0, u1, u2);
    const float3 w = cos_hemi(y0.n, rng_f(r), rng_f(r));
    L.lv[l] = make_float4(y0.p.x, y0.p.y, y0.p.z, ibits(y0.tri));
    L.lt[l] = make_float4(0.f, 0.f, 0.f, 1.0f / S.em_area);
    L.lfl[l] = 0;
    L.lb0[l] = make_float2(y0.b1, y0.b2);
    L.sig[l] = 1u << 24;
    // cosine emission: L_e cos / (p_A p_w) = L_e A pi
    const float3 le = emission(S, y0.tri, y0.b1, y0.b2, w) * (S.em_area * PT_PI);
    L.lbeta[l] = make_float4(le.x, le.y, le.z, fmaxf(dot3(y0.n, w), 0.0f) / PT_PI);
    L.ro[l] = make_float4(y0.p.x, y0.p.y, y0.p.z, ibits(y0.tri));
    L.rd[l] = make_float4(w.x, w.y, w.z, 3.0e38f);
    L.q[0][l] = (uint32_t)l;
}

// vertex `vi` of every queued light path: store it (position, arriving throughput, forward
// area density, flags) and sample the adjoint BSDF for the next
__global__ void k_light_shade(SceneDev S, LightBuf L, uint32_t seed, int vi, int lmax, unsigned long long *cnt)
{
    const uint32_t iter = iter_of(cnt);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = (int)cnt[C_LIGHT_Q0 + vi - 1];
    const uint32_t *qin = L.q[(vi - 1) & 1];
    uint32_t *qout = L.q[vi & 1];
    bool cont = false;
    int pid = 0;
    if (i < n) {
        pid = qin[i];
        const float4 h = L.hit[pid];
        const int tri = fbits(h.w);
        if (tri >= 0) {
            const float4 o = L.ro[pid], d = L.rd[pid];
            const float3 x = xyz(o) + xyz(d) * h.x;
            const TriShade &sh = S.shade[tri];
            const MatDev &m = S.mats[sh.mat];
            const float4 bt = L.lbeta[pid];
            const size_t v = (size_t)vi * L.M + pid;
            L.lv[v] = make_float4(x.x, x.y, x.z, ibits(tri));
            L.lt[v] = make_float4(bt.x, bt.y, bt.z, bt.w * fabsf(dot3(sh.n, xyz(d))) / (h.x * h.x));
            L.lfl[v] = (uint8_t)(((m.flags & MF_SPEC) ? LV_S : 0) | ((m.flags & MF_DELTA) ? LV_DIRAC : 0));
            uint32_t sg = L.sig[pid];
            if (m.flags & MF_SPEC) sg |= 1u << vi;
            if (m.type == MAT_LAMBERT && vi < 8) sg |= 1u << (16 + vi);
            sg = (sg & 0xFFFFFFu) | ((uint32_t)(vi + 1) << 24);
            L.sig[pid] = sg;
            if (vi + 1 < lmax) {
                Rng r = rng_make(seed, S_LIGHT, (uint32_t)pid, iter, (uint32_t)vi);
                const float a = rng_f(r), b = rng_f(r), c = rng_f(r);
                const BS bs = bsdf_sample(m, sh.n, -xyz(d), a, b, c, false);
                if (bs.ok) {
                    const float3 nb = xyz(bt) * bs.w;
                    L.lbeta[pid] = make_float4(nb.x, nb.y, nb.z, bs.pdf);
                    L.ro[pid] = make_float4(x.x, x.y, x.z, ibits(tri));
                    L.rd[pid] = make_float4(bs.wi.x, bs.wi.y, bs.wi.z, 3.0e38f);
                    cont = true;
                }
            }
        }
    }
    const int slot = wave_push(cnt + C_LIGHT_Q0 + vi, cont);
    if (cont) qout[slot] = (uint32_t)pid;
}

// proxy-class state machine over eye vertices (emitters count as D): phase 0 before the first
// diffuse vertex z_d; 1 at/after z_d with only specular vertices since (u of them); 2 after
// S^u then one diffuse vertex (y_1, or y_{j+1} of class C); 4 (general control vertex, gcv)
// after a further Lambertian vertex h_c, k vertices pushed since h_c entered (h_c = y_k if the
// path closes now) while y_{k+1+u} is still among the stored light vertices; 3 never a proxy path
__host__ __device__ inline void pstate_push(uint32_t &ph, uint32_t &u, uint32_t &k, bool spec, bool lambert, int umax,
                                            bool gcv)
{
    if (ph == 0) { if (!spec) { ph = 1; u = 0; } }
    else if (ph == 1) {
        if (spec) { if (++u > (uint32_t)umax) ph = 3; }
        else ph = u >= 1 ? 2 : 3;
    } else if (ph == 2) {
        k = 1;
        ph = (gcv && lambert && k + 1 + u <= PT_LMAX - 1) ? 4 : 3;
    } else if (ph == 4) {
        if (++k + 1 + u > PT_LMAX - 1) ph = 3;
    }
}
// does a path closed at an emitter after the vertices pushed so far belong to the proxy class?
__host__ __device__ inline bool pstate_closes(uint32_t ph, uint32_t u)
{
    return (ph == 1 && u >= 1) || ph == 2 || ph == 4;
}
__device__ __forceinline__ bool class_ok(int filter, bool proxy_class)
{
    return filter == 0 || (filter == 1 && proxy_class) || (filter == 2 && !proxy_class);
}

// ---------------------------------------------------------------------------------- connections
// Light-vertex connections (Section 3.2's subspace-based probabilistic connections): every
// non-Dirac light vertex y_i, i >= 1, of this iteration's M light sub-paths enters one pool,
// bucketed by its light subspace S_L (nearest centroid of position, normal, direction toward
// y_{i-1}). An eye vertex z in eye subspace T picks S_L from row T of the selection matrix Q
// (alias table over the non-empty subspaces, a defensive fraction uniform), then one vertex of
// that bucket uniformly: sigma = pi(S_L | T) / |S_L|, and the contribution is divided by
// M sigma. Q is learned like Gamma, from the connections' contributions of earlier iterations.
// Light tracing splats every pool vertex onto the image.
//
// MIS: balance heuristic over every strategy that builds the path. With light vertices
// x_0..x_{s-1} and eye vertices x_s..x_k (x_k the camera), strategy s has density
//   P_s = prod_{i<s} fwd_i * prod_{i>=s} rev_i * K_s,
// fwd_i / rev_i the area densities of x_i from the light / eye side, and K_0 = 1 (emission hit),
// K_1 = 1 (next-event estimation), K_s = M sigma(x_{s-1} | x_s) for a connection
// (2 <= s <= k-1), K_k = M (light tracing); K_s = 0 when x_{s-1} or x_s is Dirac or the strategy
// is off. Then w_s = K_s / (K_s + A_s + C_s) with
//   A_s = sum_{s'<s} K_s' prod_{i=s'}^{s-1} rev_i / fwd_i   (recursion A_{s+1} = (A_s + K_s) rev_s / fwd_s)
//   C_s = sum_{s'>s} K_s' prod_{i=s}^{s'-1} fwd_i / rev_i   (recursion C_s = fwd_s / rev_s (K_{s+1} + C_{s+1})).
// Every factor that does not depend on the other sub-path is accumulated while tracing: the
// light side stores phi_j = (A_{j-1} + K_{j-1}) |cos_{j-1}| / (d_{j-1,j}^2 fwd_{j-1}), so that
// A_j = phi_j rev-pdf(y_j) once the direction leaving y_j is known; the eye side carries the
// analogous quantity along the path. sigma in the weights comes from the frozen Q and the
// previous iteration's bucket sizes (any function the strategies share keeps the weights
// summing to one; one that does not depend on this iteration's light paths keeps them
// independent of the sample they weigh). Paths of the proxy class are weighed by the proxy
// combination (emission hit, NEE, light tracing, proxy) and never by a connection.

__global__ void k_pool(LightBuf L, int lmax, unsigned long long *cnt)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + (int)(idx / L.M), pid = (int)(idx % L.M);
    bool in = false;
    if (j < lmax) {
        const uint32_t v = (uint32_t)j * (uint32_t)L.M + (uint32_t)pid;
        in = j < sig_count(L.sig[pid]) && !(L.lfl[v] & LV_DIRAC);
    }
    const int slot = wave_push(cnt + C_POOL, in);
    if (in) L.pool[slot] = (uint32_t)j * (uint32_t)L.M + (uint32_t)pid;
}

// reverse density (solid angle) at a vertex of direction `wi` given the direction `wo` toward
// the other neighbour; a Dirac vertex gives its lobe probability
__device__ __forceinline__ float rev_pdf(const MatDev &m, float3 n, float3 wo, float3 wi)
{
    return (m.flags & MF_DELTA) ? dirac_prob(m, n, wo, wi) : bsdf_pdf(m, n, wo, wi);
}

struct MisK {
    float kN, kS, kL;   // next-event estimation, connections (on/off), light tracing (M)
};

// subspace-based selection of the light vertex a connection joins
struct ConnDev {
    CentSet light, eye;        // light subspace (S_L) and eye subspace (T) centroids
    int n_lsub, n_eye, M;
    // this iteration: label of every pool vertex (index i * M + path), buckets, alias rows
    int *lab;
    int *rank;                 // place of every pool vertex within its bucket (index i * M + path)
    int *count, *off, *fill, *list, *nonempty, *n_nonempty;
    const float *al_prob, *row_sum;
    const int *al_idx;
    const float *al_pmf;       // [n_eye * n_lsub] probability the alias row draws S_L (non-empty S_L only)
    const float *q;            // [n_eye * n_lsub] Q frozen for this iteration
    // MIS inputs from earlier iterations only
    const float *row_tot;      // [n_eye] row totals of the frozen Q
    const int *count_prev;     // [n_lsub] bucket sizes of the previous iteration
    const float *ne_prev;      // [1] non-empty light subspaces of the previous iteration
    float defensive;
    float *qacc;               // [n_eye * n_lsub] learning accumulator
};
__device__ __forceinline__ int conn_label_light(const SceneDev &S, const ConnDev &C, float3 p, float3 n, float3 w)
{
    float f[9];
    feat9(S, p, n, w, f);
    return nearest_set(C.light, f);
}
__device__ __forceinline__ int conn_label_eye(const SceneDev &S, const ConnDev &C, float3 p, float3 n, float3 w)
{
    float f[9];
    feat9(S, p, n, w, f);
    return nearest_set(C.eye, f);
}
// the weights' factor M sigma of a connection joining light vertex label Sl to eye label T,
// from frozen inputs (the selection probability the previous iteration's buckets would give)
__device__ __forceinline__ float conn_k(const ConnDev &C, float on, int T, int Sl)
{
    if (!(on > 0.0f) || Sl < 0) return 0.0f;
    const float ne = *C.ne_prev;
    if (!(ne > 0.0f)) return 0.0f;
    const int cp = C.count_prev[Sl];
    if (cp <= 0) return 0.0f;
    const float rt = C.row_tot[T];
    const float pi = rt > 0.0f ? (1.0f - C.defensive) * C.q[(size_t)T * C.n_lsub + Sl] / rt + C.defensive / ne : 1.0f / ne;
    return (float)C.M * pi / (float)cp;
}
// this iteration's selection probability of bucket Sl from row T: what the alias row realises
__device__ __forceinline__ float conn_sel(const ConnDev &C, int T, int Sl)
{
    const int ne = *C.n_nonempty;
    if (ne <= 0 || C.count[Sl] <= 0) return 0.0f;
    return C.al_pmf[(size_t)T * C.n_lsub + Sl];
}

// label every pool vertex and count the buckets
// the pool as in k_pool, and at once every pool vertex's light subspace label and its place in
// that label's bucket (the bucket counter before the increment), so that the scatter after the
// scan of the counts needs no atomics
__global__ void k_pool_label(SceneDev S, LightBuf L, int lmax, ConnDev C, unsigned long long *cnt)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + (int)(idx / L.M), pid = (int)(idx % L.M);
    bool in = false;
    uint32_t v = 0;
    if (j < lmax) {
        v = (uint32_t)j * (uint32_t)L.M + (uint32_t)pid;
        in = j < sig_count(L.sig[pid]) && !(L.lfl[v] & LV_DIRAC);
    }
    const int slot = wave_push(cnt + C_POOL, in);
    if (!in) return;
    L.pool[slot] = v;
    const float4 y = L.lv[v];
    const float3 w = normalize3(xyz(L.lv[v - (uint32_t)L.M]) - xyz(y));
    const int lab = conn_label_light(S, C, xyz(y), S.shade[fbits(y.w)].n, w);
    C.lab[v] = lab;
    C.rank[v] = atomicAdd(C.count + lab, 1);
}
__global__ void k_scatter_pool(LightBuf L, ConnDev C, const unsigned long long *cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int)cnt[C_POOL]) return;
    const uint32_t v = L.pool[i];
    C.list[C.off[C.lab[v]] + C.rank[v]] = (int)v;
}
// end of an iteration: its bucket sizes become the next iteration's frozen inputs
__global__ void k_conn_prev(ConnDev C, int *count_prev, float *ne_prev)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < C.n_lsub) count_prev[i] = C.count[i];
    if (i == 0) *ne_prev = (float)*C.n_nonempty;
}

// one thread per light path: phi_j for j = 1 .. count - 1 (x: every strategy; y: without the
// connections, the combination of proxy-class paths; z: the emission-hit strategy alone)
__global__ void k_light_phi(SceneDev S, LightBuf L, MisK K, ConnDev C, unsigned long long *cnt)
{
    const int pid = blockIdx.x * blockDim.x + threadIdx.x;
    if (pid >= L.M) return;
    const int nv = sig_count(L.sig[pid]);
    if (nv < 2) return;
    float3 yp = xyz(L.lv[pid]);
    float3 y = xyz(L.lv[(size_t)L.M + pid]);
    float phi, phi0, pt;
    {
        const float3 d = y - yp;
        const float d2 = dot3(d, d);
        const float c0 = fabsf(dot3(S.shade[fbits(L.lv[pid].w)].n, d)) * rsqrtf(d2);
        phi = phi0 = pt = c0 / d2 * S.em_area;   // (A_0 + K_0) g_0 / fwd_0, fwd_0 = 1 / A
        L.lphi[(size_t)L.M + pid] = make_float4(phi, phi0, pt, 0.0f);
    }
    for (int j = 2; j < nv; ++j) {
        const size_t v1 = (size_t)(j - 1) * L.M + pid;
        const float4 a = L.lv[v1], b = L.lv[(size_t)j * L.M + pid];
        const int t1 = fbits(a.w);
        const float3 n1 = S.shade[t1].n;
        const MatDev m1 = S.mats[S.shade[t1].mat];
        const float3 toj = xyz(b) - y;
        const float d2 = dot3(toj, toj);
        const float3 wj = toj * rsqrtf(d2);
        const float3 wp = normalize3(yp - y);
        const float rho = rev_pdf(m1, n1, wj, wp);
        const bool dirac1 = (L.lfl[v1] & LV_DIRAC) != 0;
        const bool dirac0 = j - 2 >= 1 ? (L.lfl[(size_t)(j - 2) * L.M + pid] & LV_DIRAC) != 0 : false;
        // split between x_{j-2} (light end) and x_{j-1} (eye end, its eye subspace taken with the
        // direction toward x_j)
        float Kp = 0.0f;
        if (!dirac1) {
            if (j - 1 == 1) Kp = K.kN;
            else if (!dirac0 && K.kS > 0.0f)
                Kp = conn_k(C, K.kS, conn_label_eye(S, C, y, n1, wj), C.lab[(size_t)(j - 2) * L.M + pid]);
        }
        const float Kp0 = (dirac1 || j - 1 != 1) ? 0.0f : K.kN;
        const float fwd = L.lt[v1].w;
        const float gf = fwd > 0.0f ? fabsf(dot3(n1, wj)) / (d2 * fwd) : 0.0f;
        phi = (phi * rho + Kp) * gf;
        phi0 = (phi0 * rho + Kp0) * gf;
        pt = pt * rho * gf;
        L.lphi[(size_t)j * L.M + pid] = make_float4(phi, phi0, pt, 0.0f);
        yp = y;
        y = xyz(b);
    }
}

// features of pre-traced light vertices y_i, i >= 1, non-Dirac (direction toward y_{i-1}), for
// the light subspaces; at most `cap` rows
__global__ void k_feat_light(SceneDev S, LightBuf L, int lmax, float *feat, int cap, unsigned long long *cnt,
                             int cidx)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + (int)(idx / L.M), pid = (int)(idx % L.M);
    bool in = false;
    if (j < lmax) {
        const size_t v = (size_t)j * L.M + pid;
        in = j < sig_count(L.sig[pid]) && !(L.lfl[v] & LV_DIRAC);
    }
    const int slot = wave_push(cnt + cidx, in);
    if (in && slot < cap) {
        const size_t v = (size_t)j * L.M + pid;
        const float4 y = L.lv[v];
        float f[9];
        feat9(S, xyz(y), S.shade[fbits(y.w)].n, normalize3(xyz(L.lv[v - L.M]) - xyz(y)), f);
        for (int k = 0; k < 9; ++k) feat[FEAT * (size_t)slot + k] = f[k];
    }
}

// eye-side state machine over a connected light sub-path y_j .. y_1 (then the emitter, a D
// vertex): is the full path in the proxy class? (Lambertian flags exist for y_1 .. y_7; a class C
// control vertex is never further along.)
__host__ __device__ inline bool light_tail_class(uint32_t ph, uint32_t uu, uint32_t kk, uint32_t sg, int j, int umax,
                                                 bool gcv)
{
    for (int i = j; i >= 1; --i)
        pstate_push(ph, uu, kk, (sg >> i) & 1u, i < 8 && ((sg >> (16 + i)) & 1u), umax, gcv);
    return pstate_closes(ph, uu);
}

// ---------------------------------------------------------------------------------- candidates
// Every prefix ending at a specular vertex whose trailing specular run (length u <= u_max)
// starts at y_1 (class A, L S^u) or at y_2 after a diffuse y_1 (class B, L D S^u, control
// vertex y_0 on the light) is a candidate (Section 5.1; Section 6.1's restrictions).
// the candidates of light sub-path l (signature sg, nv stored vertices): class A (y_1 .. y_i
// specular, h_c null), class B (y_1 diffuse, y_2 .. y_i specular, h_c = y_0) and, with gcv, class
// C (y_j Lambertian, j >= 1, y_{j+1} non-specular, y_{j+2} .. y_i specular, h_c = y_j); u <=
// u_max. emit(k, i, cls, j, u) is called for each in order, k counting from 0; returns the count.
// The specular run that ends at y_i fixes its class and j, so each y_i (1 <= i < nv <= 6) ends at
// most one candidate, and the five cannot all be candidates (y_1 .. y_5 all specular is one class
// A run with u = 5 > u_max at i = 5): at most 4 per sub-path, the capacity of the buffers.
template <typename F>
__device__ __forceinline__ int cand_walk(uint32_t sg, int nv, int u_max, int gcv, F emit)
{
    int k = 0;
    if (nv < 2) return 0;
    const auto spec = [&](int i) { return ((sg >> i) & 1u) != 0u; };
    const int cls = spec(1) ? 0 : 1;
    const int first = cls == 0 ? 1 : 2;
    for (int i = first; i < nv && spec(i) && i - first + 1 <= u_max; ++i) emit(k++, i, cls, 0, i - first + 1);
    if (gcv)
        for (int j = 1; j + 2 < nv; ++j) {
            if (!((sg >> (16 + j)) & 1u) || spec(j + 1)) continue;
            for (int i = j + 2; i < nv && spec(i) && i - j - 1 <= u_max; ++i) emit(k++, i, 2, j, i - j - 1);
        }
    return k;
}

__global__ void k_candidates(LightBuf L, int u_max, int gcv, Cand *cand, unsigned long long *cnt)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    int nc = 0, nv = 0;
    uint32_t sg = 0;
    if (l < L.M) {
        sg = L.sig[l];
        nv = min(sig_count(sg), PT_LMAX);
        nc = cand_walk(sg, nv, u_max, gcv, [](int, int, int, int, int) {});
    }
    // wavefront exclusive scan of the counts
    int incl = nc;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (__lane_id() >= off) incl += v;
    }
    const int total = __shfl(incl, 63);
    int base = 0;
    if (__lane_id() == 63 && total) base = (int)atomicAdd(cnt + C_NCAND, (unsigned long long)total);
    base = __shfl(base, 63);
    const int o = base + incl - nc;
    if (nc == 0) return;
    cand_walk(sg, nv, u_max, gcv, [&](int k, int vi, int cls, int j, int u) {
        Cand c;
        c.v = L.lv[vi * L.M + l];
        c.hc = L.lv[j * L.M + l];
        if (cls == 2) {
            const float2 wc = oct_enc(normalize3(xyz(L.lv[(j - 1) * L.M + l]) - xyz(c.hc)));
            c.hc_b1 = wc.x; c.hc_b2 = wc.y;
            c.beta_c = L.lt[j * L.M + l];
        } else {
            const float2 b = L.lb0[l];
            c.hc_b1 = b.x; c.hc_b2 = b.y;
            c.beta_c = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        c.cls_u = (j << 16) | (cls << 8) | u;
        c.B = 0.f; c.rho = 1.f; c.recip_sum = 0.f; c.pmax = 0.f; c.psum = 0.f; c.pn = 0.f; c.spec_sub = 0;
        const float2 wi = oct_enc(normalize3(xyz(L.lv[(vi - 1) * L.M + l]) - xyz(c.v)));
        c.pad[0] = wi.x; c.pad[1] = wi.y;
        cand[o + k] = c;
    });
}

// keep each candidate with probability pi_inc = min(1, cap / n_cand) (Horvitz-Thompson form of
// Section 6.1's cap of 400 incomplete sub-paths)
__global__ void k_keep(int cap, uint32_t seed, uint32_t *kept, int max_cand, unsigned long long *cnt)
{
    const uint32_t iter = iter_of(cnt);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = (int)cnt[C_NCAND];
    bool keep = false;
    if (i < n && i < max_cand) {
        const float pi = fminf(1.0f, (float)cap / (float)n);
        Rng r = rng_make(seed, S_CAND, (uint32_t)i, iter, 0u);
        keep = pi >= 1.0f || rng_f(r) < pi;
    }
    const int slot = wave_push(cnt + C_NKEPT, keep);
    if (keep) kept[slot] = (uint32_t)i;
}

// ---------------------------------------------------------------------------------- f/q samples
// One sample of f(g)/q(g) for the candidate (Sections 5.2-5.3). f is the light tracer's own
// density of the dropped vertices g and of y_{s-1} (visibility and the S/D signature
// included); q is the uniform mixture of the available strategies: light-source sampling
// (u = 1, class A), tracing from the control vertex (u = 1, class B; cosine lobe at the light
// vertex), tracing from y_{s-1} (cosine hemisphere, each side with probability 1/2 on a
// dielectric, then the BSDF at every intermediate vertex).
template <typename SE>
struct CtxT {
    const SceneDev &S;
    SE *stk;         // this thread's column of the workgroup's LDS stack (stk_col)
    uint32_t rays;
    int stride;      // threads per workgroup
    uint32_t visits = 0, tests = 0;   // BVH nodes visited and triangles tested (traffic accounting)
    uint32_t trips = 0;               // traversal loop trips of the wavefront (first active lane)
};
using Ctx = CtxT<int>;

template <typename SE>
__device__ __forceinline__ bool occluded(CtxT<SE> &C, float3 a, int ta, float3 b, int tb)
{
    const float3 d = b - a;
    const float dist = sqrtf(dot3(d, d));
    Hit h;
    C.rays++;
    return traverse<true, true>(C.S, a, d * (1.0f / dist), C.S.tmin, dist * 0.9999f, ta, tb, C.stk, C.stride, h,
                                &C.visits, &C.tests);
}
template <typename SE>
__device__ __forceinline__ bool closest(CtxT<SE> &C, float3 o, float3 d, int ign, Hit &h)
{
    C.rays++;
    return traverse<false, true>(C.S, o, d, C.S.tmin, 3.0e38f, ign, -1, C.stk, C.stride, h, &C.visits, &C.tests);
}
// a kernel's traversal work, one atomic per wavefront
template <typename SE>
__device__ __forceinline__ void count_traversal(const CtxT<SE> &C, unsigned long long *cnt, int cv = C_VISITS_R,
                                                int ct = C_TESTS_R, int cw = -1)
{
    wave_count(cnt + cv, C.visits);
    wave_count(cnt + ct, C.tests);
    if (cw >= 0) wave_count(cnt + cw, C.trips);
}
// cosine direction at y_{s-1}: on a dielectric each side with probability 1/2, else the front
__device__ __forceinline__ float3 spec_start(const MatDev &m, float3 n, Rng &r, float &side_p)
{
    float3 ns = n;
    side_p = 1.0f;
    if (m.type == MAT_DIELECTRIC) { side_p = 0.5f; if (rng_f(r) < 0.5f) ns = -n; }
    const float a = rng_f(r), b = rng_f(r);
    return cos_hemi(ns, a, b);
}
__device__ __forceinline__ float side_prob(const MatDev &m, float3 n, float3 w)
{
    return m.type == MAT_DIELECTRIC ? 0.5f : (dot3(n, w) > 0.0f ? 1.0f : 0.0f);
}

// f/q of the u = 1 class A sample that reached the emitter at y (normal ny)
__device__ __forceinline__ float fq_u1_a(const SceneDev &S, float3 v, float3 vn, const MatDev &mv, float3 y, float3 ny)
{
    const float invA = 1.0f / S.em_area;
    const float3 dv = v - y;
    const float d2 = dot3(dv, dv);
    const float3 w = dv * rsqrtf(d2);
    const float c0 = dot3(ny, w), cv = fabsf(dot3(vn, w));
    const float f = c0 > 0.0f ? invA * (c0 / PT_PI) * cv / d2 : 0.0f;
    const float q3 = side_prob(mv, vn, -w) * (cv / PT_PI) * fabsf(c0) / d2;
    return f / (0.5f * (invA + q3));
}
// One f/q sample is a small state machine: fq_begin draws its first choices and sets the ray of
// its first trip; after each trip fq_advance takes the hit, and either completes the sample or
// sets the next ray. The caller traces every trip at one call site, so lanes that took different
// strategies (u = 1) or reached different vertices still traverse together, and the traversal is
// inlined once. Modes: 0 u = 1 class A from the light (visibility y -> y_{s-1}), 1 u = 1 class A
// from y_{s-1} (toward the light), 2 / 3 u = 1 class B from y_0 / from y_{s-1} (ray to y_1, then
// the visibility of the other side), 4 u >= 2 (the retrace through the specular run, then for
// class B the visibility y_0 -> y_1).
struct FqCand {              // what a sample reads of its candidate
    float3 v, vn, y0, n0;    // y_{s-1} and h_c with their normals (h_c: classes B and C; for
                             // class C n0 faces the side of the control direction)
    int vt, t0, cls, u;
    MatDev mv;
};
struct FqState {             // a sample between two trips
    float3 ro, rd;           // the ray of the next trip (mode 0: ro is the emitter point; mode 4
                             // before the closing visibility: rd is the direction that left the
                             // last vertex)
    float rmax;
    int ig0, ig1;
    bool any;
    int mode, k;
    float3 nyl;              // mode 0: the emitter normal
    Hit h1;                  // modes 2, 3: y_1
    float f, q;
};
__device__ __forceinline__ FqCand fq_cand(const SceneDev &S, const Cand &c)
{
    FqCand K;
    K.cls = cand_cls(c.cls_u); K.u = cand_u(c.cls_u);
    K.v = xyz(c.v);
    K.vt = fbits(c.v.w);
    K.vn = S.shade[K.vt].n;
    K.mv = S.mats[S.shade[K.vt].mat];
    K.y0 = xyz(c.hc);        // control vertex h_c (classes B, C)
    K.t0 = fbits(c.hc.w);
    K.n0 = K.cls ? S.shade[K.t0].n : f3(0.0f, 0.0f, 1.0f);
    // class C: h_c is Lambertian, and sampling its BSDF from the control direction is the cosine
    // hemisphere on that direction's side, the density class B's emitter has about its normal
    if (K.cls == 2 && dot3(K.n0, oct_dec(make_float2(c.hc_b1, c.hc_b2))) < 0.0f) K.n0 = -K.n0;
    return K;
}
// f/q of the u = 1 sample of class B or C whose diffuse vertex y_1 (y_{j+1} for class C) is the
// hit h1: f = the light tracer's density of y_1 from h_c (cosine about n0) and of y_{s-1} from
// y_1 (area measure), q = the mixture of that density and of tracing from y_{s-1}
__device__ __forceinline__ float fq_u1_b(const SceneDev &S, const FqCand &K, const Hit &h1)
{
    const float3 y1 = tri_point(S, h1.tri, h1.b1, h1.b2);
    const float3 n1 = S.shade[h1.tri].n;
    const MatDev m1 = S.mats[S.shade[h1.tri].mat];
    const float3 a = y1 - K.y0;
    const float d01 = dot3(a, a);
    const float3 w01 = a * rsqrtf(d01);
    const float3 b = K.v - y1;
    const float d1v = dot3(b, b);
    const float3 w1v = b * rsqrtf(d1v);
    const float c0 = dot3(K.n0, w01);
    const float p1 = c0 > 0.0f ? (c0 / PT_PI) * fabsf(dot3(n1, w01)) / d01 : 0.0f;
    const float cv = fabsf(dot3(K.vn, w1v));
    const float f = p1 * bsdf_pdf(m1, n1, -w01, w1v) * cv / d1v;
    const float q3 = side_prob(K.mv, K.vn, -w1v) * (cv / PT_PI) * fabsf(dot3(n1, w1v)) / d1v;
    return f / (0.5f * (p1 + q3));
}
__device__ __forceinline__ void fq_begin(const SceneDev &S, const FqCand &K, Rng &r, FqState &s)
{
    s.ro = K.v; s.rd = f3(0.0f, 0.0f, 1.0f);
    s.rmax = 3.0e38f;
    s.ig0 = K.vt; s.ig1 = -1;
    s.any = false;
    s.k = 1;
    s.nyl = K.vn;
    s.h1.tri = -1; s.h1.b1 = s.h1.b2 = 0.0f; s.h1.t = 0.0f;
    s.f = 1.0f; s.q = 1.0f;
    if (K.u == 1) {
        const bool from_spec = rng_f(r) >= 0.5f;
        if (K.cls == 0) {
            if (!from_spec) {
                const float a = rng_f(r), b = rng_f(r), d = rng_f(r);
                const LPoint L = sample_emitter(S, a, b, d);
                s.nyl = L.n;
                const float3 dd = K.v - L.p;
                const float dist = sqrtf(dot3(dd, dd));
                s.ro = L.p; s.rd = dd * (1.0f / dist); s.rmax = dist * 0.9999f; s.ig0 = L.tri; s.ig1 = K.vt;
                s.any = true;
                s.mode = 0;
            } else {
                float sp;
                s.rd = spec_start(K.mv, K.vn, r, sp);
                s.mode = 1;
            }
        } else {
            if (!from_spec) {
                const float a = rng_f(r), b = rng_f(r);
                s.ro = K.y0; s.rd = cos_hemi(K.n0, a, b); s.ig0 = K.t0;
                s.mode = 2;
            } else {
                float sp;
                s.rd = spec_start(K.mv, K.vn, r, sp);
                s.mode = 3;
            }
        }
    } else {
        // u >= 2: trace from y_{s-1} only. Dirac vertices enter through their lobe
        // probabilities; the solid angle at each smooth vertex is carried to area at the next
        // smooth vertex, and only the ratio of the two directions' Jacobians,
        // (eta_b^2 |cos b|) / (eta_a^2 |cos a|), survives in f/q (etendue is conserved along a
        // Dirac run).
        float sp;
        s.rd = spec_start(K.mv, K.vn, r, sp);
        s.q = sp * fabsf(dot3(K.vn, s.rd)) / PT_PI;
        const float e = side_eta(K.mv, K.vn, s.rd);
        s.f = e * e * fabsf(dot3(K.vn, s.rd));   // numerator of the run leaving y_{s-1}
        s.mode = 4;
    }
}
// after the trip of s traced to (hit, h): true with the sample's f/q in out when it is complete
__device__ __forceinline__ bool fq_advance(const SceneDev &S, const FqCand &K, Rng &r, FqState &s, bool hit,
                                           const Hit &h, float &out)
{
    const int u = K.u;
    if (s.mode == 0) { out = hit ? 0.0f : fq_u1_a(S, K.v, K.vn, K.mv, s.ro, s.nyl); return true; }
    if (s.mode == 1) {
        if (!hit || !(S.mats[S.shade[h.tri].mat].flags & MF_EMIT)) { out = 0.0f; return true; }
        out = fq_u1_a(S, K.v, K.vn, K.mv, tri_point(S, h.tri, h.b1, h.b2), S.shade[h.tri].n);
        return true;
    }
    if (s.mode <= 3) {
        if (s.k == 2) { out = hit ? 0.0f : fq_u1_b(S, K, s.h1); return true; }
        // the ray to y_1, which must be diffuse; then the visibility of its other side
        if (!hit || (S.mats[S.shade[h.tri].mat].flags & MF_SPEC)) { out = 0.0f; return true; }
        s.h1 = h;
        const float3 p1 = tri_point(S, h.tri, h.b1, h.b2);
        const float3 a = s.mode == 2 ? p1 : K.y0, b = s.mode == 2 ? K.v : p1;
        const float3 dd = b - a;
        const float dist = sqrtf(dot3(dd, dd));
        s.ro = a; s.rd = dd * (1.0f / dist); s.rmax = dist * 0.9999f; s.any = true;
        s.ig0 = s.mode == 2 ? h.tri : K.t0; s.ig1 = s.mode == 2 ? K.vt : h.tri;
        s.k = 2;
        return false;
    }
    // mode 4
    if (s.k > u) { out = hit ? 0.0f : (s.f > 0.0f ? s.f / s.q : 0.0f); return true; }   // class B: y_0 -> y_1
    if (!hit) { out = 0.0f; return true; }
    const float3 y = tri_point(S, h.tri, h.b1, h.b2);
    const float3 ny = S.shade[h.tri].n;
    const MatDev m = S.mats[S.shade[h.tri].mat];
    const float3 w_cam = -s.rd;       // toward y_{s-1}
    if (s.k < u) {
        if (!(m.flags & MF_SPEC)) { out = 0.0f; return true; }
        const float a = rng_f(r), b = rng_f(r), cc = rng_f(r);
        const BS bs = bsdf_sample(m, ny, w_cam, a, b, cc, true);
        if (!bs.ok) { out = 0.0f; return true; }
        s.q *= bs.pdf;
        const float3 w_light = bs.wi;
        if (m.flags & MF_DELTA) {
            s.f *= dirac_prob(m, ny, w_light, w_cam);
        } else {
            // close the run arriving here, account the forward density, open the next run
            const float ea = side_eta(m, ny, w_cam);
            s.f /= ea * ea * fabsf(dot3(ny, w_cam));
            s.f *= bsdf_pdf(m, ny, w_light, w_cam);
            const float eb = side_eta(m, ny, w_light);
            s.f *= eb * eb * fabsf(dot3(ny, w_light));
        }
        if (!(s.f > 0.0f)) { out = 0.0f; return true; }
        s.ro = y; s.rd = w_light; s.ig0 = h.tri;
        ++s.k;
        return false;
    }
    // k == u: the vertex that closes the run
    const float ea = side_eta(m, ny, w_cam);
    s.f /= ea * ea * fabsf(dot3(ny, w_cam));
    if (K.cls == 0) {
        if (!(m.flags & MF_EMIT)) { out = 0.0f; return true; }
        const float c0 = dot3(ny, w_cam);
        if (c0 <= 0.0f) { out = 0.0f; return true; }
        s.f *= (1.0f / S.em_area) * c0 / PT_PI;
        out = s.f > 0.0f ? s.f / s.q : 0.0f;
        return true;
    }
    if (m.flags & MF_SPEC) { out = 0.0f; return true; }
    const float3 a = y - K.y0;
    const float d2 = dot3(a, a);
    const float3 w01 = a * rsqrtf(d2);
    const float c0 = dot3(K.n0, w01);   // the cosine density of leaving h_c (classes B and C)
    if (c0 <= 0.0f) { out = 0.0f; return true; }
    s.f *= (c0 / PT_PI) * fabsf(dot3(ny, w01)) / d2;
    s.f *= bsdf_pdf(m, ny, -w01, w_cam);
    // visibility y_0 -> y (ignoring both triangles), traced on the next trip
    const float dist = sqrtf(d2);
    s.ro = K.y0; s.rd = w01; s.rmax = dist * 0.9999f; s.ig0 = K.t0; s.ig1 = h.tri; s.any = true;
    s.k = u + 1;
    return false;
}
// one whole sample of candidate c with the random stream r
template <typename SE>
__device__ float fq_sample(CtxT<SE> &C, const Cand &c, Rng &r)
{
    const FqCand K = fq_cand(C.S, c);
    FqState s;
    fq_begin(C.S, K, r, s);
    for (;;) {
        Hit h;
        C.rays++;
        const bool hit = traverse_rt<true>(C.S, s.ro, s.rd, C.S.tmin, s.rmax, s.ig0, s.ig1, s.any, C.stk, C.stride, h,
                                           &C.visits, &C.tests, &C.trips);
        float out;
        if (fq_advance(C.S, K, r, s, hit, h, out)) return out;
    }
}

// The pilot and the chains run one wavefront per candidate / chain: each step the 64 lanes
// draw 64 i.i.d. samples of f/q (sample index = step * 64 + lane, each with its own Philox
// counter), and the wavefront then consumes them in order with a uniform scalar loop. Samples
// are i.i.d. whatever the chain's state, so drawing them ahead of need changes nothing but the
// number of discarded draws (fewer than 64 per chain).
#define RW 4                       // wavefronts per workgroup
// minimum waves per SIMD the chain kernels are compiled for (register budget 512 / waves);
// with 16-bit stack entries LDS allows more than three
#ifndef PT_RECIP_WAVES
#define PT_RECIP_WAVES 4
#endif
#ifndef PT_PILOT_WAVES
#define PT_PILOT_WAVES 4
#endif
#ifndef PT_GEN_WAVES
#define PT_GEN_WAVES 1
#endif

// The pilot and the stage-A chains run on a persistent grid (a few workgroups per CU): each
// wavefront takes the next item from a device counter until the items, counted on the device,
// run out, so the launch does not depend on the number of candidates and no wavefront is
// dispatched only to exit. Item k keeps its own Philox stream whichever wavefront runs it.
__device__ __forceinline__ int next_item(unsigned long long *counter)
{
    int k = 0;
    if (__lane_id() == 0) k = (int)atomicAdd(counter, 1ull);
    // readfirstlane (lane 0: the whole wavefront is active here) marks the item wave-uniform, so
    // that the item's candidate record and chain state are scalar loads and scalar registers
    return __builtin_amdgcn_readfirstlane(k);
}
// value of lane l (l wave-uniform) as a wave-uniform scalar
__device__ __forceinline__ float lane_f(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
__device__ __forceinline__ uint32_t lane_u(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }
// a value every lane holds equally (after a butterfly reduction), as a wave-uniform scalar
__device__ __forceinline__ float uni_f(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ int uni_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// pilot: 64-sample steps until at least `pilot` samples with 8 non-zero values, or 256 samples
template <typename SE>
__global__ void __launch_bounds__(64 * RW, PT_PILOT_WAVES) k_pilot(SceneDev S, Cand *cand, const uint32_t *kept, int pilot,
                                                   uint32_t seed, float *runmax, unsigned long long *cnt)
{
    const uint32_t iter = iter_of(cnt);
    __shared__ SE stk[stk_depth<SE>() * 64 * RW];
    const int lane = threadIdx.x & 63;
    const int n = (int)cnt[C_NKEPT];
    CtxT<SE> C{S, stk_col(stk, (int)threadIdx.x), 0u, (int)blockDim.x};
    for (int wave = next_item(cnt + C_WORK_P); wave < n; wave = next_item(cnt + C_WORK_P)) {   // wave-uniform
        Cand &c = cand[kept[wave]];
        float mx = 0.f, sm = 0.f;
        int nz = 0, k = 0;
        const int maxn = max(256, pilot);
        for (int step = 0; k < maxn; ++step) {
            Rng r = rng_make(seed, S_PILOT, (uint32_t)wave, iter, (uint32_t)(step * 64 + lane));
            const float v = fq_sample(C, c, r);
            float wm = v, ws = v;
            int wz = v > 0.0f ? 1 : 0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                wm = fmaxf(wm, __shfl_xor(wm, off));
                ws += __shfl_xor(ws, off);
                wz += __shfl_xor(wz, off);
            }
            mx = fmaxf(mx, wm); sm += ws; nz += wz; k += 64;
            if (k >= pilot && nz >= 8) break;
        }
        if (lane == 0) atomicAdd(cnt + C_DRAWN_P, (unsigned long long)k);
        if (lane == 0) {
            c.pmax = mx; c.psum = sm; c.pn = (float)k;
            atomic_maxf(runmax + cand_cls(c.cls_u) * 5 + cand_u(c.cls_u), mx);
        }
    }
    wave_count(cnt + C_RAYS_RECIP, C.rays);
    count_traversal(C, cnt);
}

// B_j (Appendix E's B = max f/q): from the candidate's pilot and the (class, u) running max, or,
// without a pilot, from its (class, u, S, C) bucket's statistics (Section 5.5); cost roulette: keep
// with rho = min(1, cost_cap / (R B / beta))
__global__ void k_roulette(Cand *cand, const uint32_t *kept, uint32_t *final_, uint32_t *cost_bin,
                           const float *runmax, SubDev D, int labelled, float em_area, int repeats, float cost_cap,
                           uint32_t seed, unsigned long long *cnt)
{
    const uint32_t iter = iter_of(cnt);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = (int)cnt[C_NKEPT];
    bool keep = false;
    uint32_t ci = 0, bin = 0;
    if (i < n) {
        ci = kept[i];
        Cand &c = cand[ci];
        const int b = cand_cls(c.cls_u) * 5 + cand_u(c.cls_u);
        float gmax = 0.f;
        for (int k = 0; k < PT_STAT_CU; ++k) gmax = fmaxf(gmax, runmax[k]);
        const float Bb = runmax[b] > 0.f ? runmax[b] : (gmax > 0.f ? gmax : 1.0f / em_area);
        // The (class, u, S, C) bucket's f/q statistics of earlier iterations (Section 5.5) when the
        // subspace labels exist: the largest value and the mean. With a pilot (c.pn > 0): B =
        // max(pilot max, the bucket's max, or the (class, u) running max while the bucket has
        // none), beta the pilot mean. Without one: B the bucket's max and beta its mean (the (class,
        // u) running max and B / 2 while the bucket has none). Any B with beta / B in (0, 2) leaves
        // the estimate unbiased (Appendix B); the pilot keeps B at or above what the candidate's own
        // samples reached.
        const int sb = labelled ? 3 * stat_bucket(D, cand_cls(c.cls_u), cand_u(c.cls_u), c.spec_sub & 0xFFFF,
                                                  c.spec_sub >> 16) : 0;
        const bool piloted = c.pn > 0.f;
        const bool has_bucket = labelled && D.bstat[sb] > 0.f && D.bstat[sb + 2] > 0.f;
        const bool bucket = !piloted && has_bucket;
        const float B = piloted ? fmaxf(c.pmax, has_bucket ? D.bstat[sb] : Bb) : (bucket ? D.bstat[sb] : Bb);
        float beta;
        if (piloted) beta = c.pmax > 0.f ? c.psum / c.pn : B / (2.0f * c.pn);
        else beta = (bucket && D.bstat[sb + 1] > 0.f) ? D.bstat[sb + 1] / D.bstat[sb + 2] : 0.5f * B;
        const float cost = (float)repeats * B / beta;
        const float rho = (cost_cap > 0.f && cost > cost_cap) ? cost_cap / cost : 1.0f;
        Rng r = rng_make(seed, S_ROUL, (uint32_t)i, iter, 0u);
        keep = rho >= 1.0f || rng_f(r) < rho;
        c.B = B; c.rho = rho; c.recip_sum = 0.0f;
        // class of the expected samples per chain, B / beta: log2, 0 .. 15
        bin = (uint32_t)min(15, max(0, (int)log2f(fmaxf(B / beta, 1.0f))));
    }
    const int slot = wave_push(cnt + C_NFINAL, keep);
    if (keep) {
        final_[slot] = ci;
        cost_bin[slot] = bin;
        atomicAdd(cnt + C_COSTH0 + bin, 1ull);
    }
}

// order of the final candidates for the chains: the classes of expected chain length from the
// longest down, so that the persistent stage-A grid starts the long chains first and does not end
// on one (longest-first scheduling); within a class in any order
__global__ void k_order(const uint32_t *cost_bin, uint32_t *order, unsigned long long *cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = (int)cnt[C_NFINAL];
    if (i >= n) return;
    const uint32_t b = cost_bin[i];
    unsigned long long base = 0;
    for (int k = 15; k > (int)b; --k) base += cnt[C_COSTH0 + k];
    order[base + atomicAdd(cnt + C_COSTF0 + b, 1ull)] = (uint32_t)i;
}

// One estimate I~ per chain (Section 4.2 with r = |g|). Pending nodes of the splitting tree
// are kept as two counters by the sign of their prefix product: a node of sign s adds s g / B
// and spawns floor(|g|) (+1 with probability |g| - floor|g|) children of sign s sgn(g).
// Chain roulette (reading R12c): when the chain has used n1, 2 n1, 4 n1, ... samples it goes on
// with probability 1/2 and its estimate is doubled, otherwise its estimate is 0; the flip times
// depend on the sample count only and the flips are independent, so the expectation is kept and
// the expected cost stays O(n1 log) however small beta is.
//
// Samples are i.i.d. (sample k of a chain is Philox counter k of its stream), so they can be
// drawn ahead of need and by any lanes: stage A runs one wavefront per chain, 64 samples per
// step, up to a budget; the chains still running then continue in rounds in which the whole
// GPU draws a block of samples for every remaining chain (k_chain_gen) and one wavefront per
// chain consumes its block in order (k_chain_consume). While a chain holds exactly one positive
// pending node and g is in [0, 1] (f/q <= B, the usual case) each sample either continues the
// chain or ends it, so a ballot finds the next event among 64 samples at once.
struct ChainState {
    uint32_t ci, chain;        // candidate index; chain id = ci * 8 + repeat
    double ans;                // 1 + sum of s g so far (the estimate is ans weight / B)
    float weight, mx;          // roulette weight; largest f/q drawn (bucket statistics)
    uint32_t pos, neg, ns, next_flip, coin;
    float bprod, bw;           // Booth's roulette: product of g so far, product of continuation probabilities
};
struct ChainRun {
    double ans;
    float weight;
    uint32_t pos, neg, ns, next_flip, coin;
    bool alive;
    float bprod, bw;
};
#define CHAIN_COIN 0x80000000u   // Philox counters of the roulette coins
#define CHAIN_LONG 0x00100000u   // Philox counters of the samples drawn in rounds
#define CHAIN_UNI 0x40000000u    // Philox counters of stage A's child-count uniforms
#define CHAIN_ROUNDS 11
#define CHAIN_BUF (1u << 24)     // samples per round over all chains
#define CHAIN_LIST_CAP (CHAIN_BUF / 64)   // running chains carried between rounds

__device__ __forceinline__ float chain_coin(uint32_t seed, uint32_t chain, uint32_t iter, uint32_t k)
{
    Rng r = rng_make(seed, S_RECIP, chain, iter, CHAIN_COIN + k);
    return rng_f(r);
}

// consume lanes 0 .. nv-1 of (fq, u) in lane order; wave-uniform state
// Booth's roulette on sample values g (lane order, from lane l): no splitting; after a prefix the
// chain goes on with probability min(1, |prod g| / booth_r) and later terms are divided by the
// product of those probabilities; the chain roulette's flips apply as in the RRS chains
__device__ __forceinline__ void booth_step(float gl, float ul, float booth_r, ChainRun &st, uint32_t seed,
                                           uint32_t chain, uint32_t iter)
{
    if (st.ns == st.next_flip) {
        if (chain_coin(seed, chain, iter, st.coin++) < 0.5f) st.weight *= 2.0f;
        else { st.alive = false; return; }
        st.next_flip *= 2u;
    }
    st.ns++;
    st.bprod *= gl;
    st.ans += (double)(st.bprod / st.bw);
    const float r = fminf(1.0f, fabsf(st.bprod) / booth_r);
    if (!(ul < r)) { st.pos = 0; return; }
    st.bw *= r;
}

__device__ __forceinline__ void chain_consume(float fq, float u, int nv, float invB, ChainRun &st, uint32_t seed,
                                              uint32_t chain, uint32_t iter, float booth_r = 0.0f)
{
    const int lane = __lane_id();
    const float g = 1.0f - fq * invB;
    if (booth_r > 0.0f) {
        for (int l = 0; l < nv && st.alive && st.pos > 0; ++l)
            booth_step(lane_f(g, l), lane_f(u, l), booth_r, st, seed, chain, iter);
        return;
    }
    const float ag = fabsf(g), fl = floorf(ag);
    const uint32_t kids = (uint32_t)fminf(fl, 1.0e6f) + (u < ag - fl ? 1u : 0u);
    int l = 0;
    while (l < nv && st.alive && st.pos + st.neg > 0) {
        if (st.pos == 1 && st.neg == 0) {
            // lanes before the first event continue the chain by one positive node each
            const bool ev = lane >= l && lane < nv &&
                            (kids == 0u || g < 0.0f || st.ns + (uint32_t)(lane - l) == st.next_flip);
            const unsigned long long m = __ballot(ev);
            const int e = m ? (__ffsll((long long)m) - 1) : nv;
            float sum = (lane >= l && lane < e) ? g : 0.0f;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
            st.ans += (double)uni_f(sum);
            st.ns += (uint32_t)(e - l);
            l = e;
            if (l >= nv) break;
        }
        // one sample through the general rule
        if (st.ns == st.next_flip) {
            if (chain_coin(seed, chain, iter, st.coin++) < 0.5f) st.weight *= 2.0f;
            else { st.alive = false; break; }
            st.next_flip *= 2u;
        }
        const float gl = lane_f(g, l);
        const uint32_t kl = lane_u(kids, l);
        bool positive = st.pos > 0;
        if (positive) st.pos--; else st.neg--;
        st.ns++;
        st.ans += positive ? (double)gl : -(double)gl;
        if (positive == (gl >= 0.0f)) st.pos += kl; else st.neg += kl;
        ++l;
    }
}

// the same for 256 samples held four per lane (sample 4 * lane + i), in sample order: one
// memory round trip of the rounds' consumer covers four times as many samples
__device__ __forceinline__ void chain_consume4(const float (&fq)[4], const float (&uu)[4], float invB, ChainRun &st,
                                               uint32_t seed, uint32_t chain, uint32_t iter, float booth_r = 0.0f)
{
    const int lane = __lane_id();
    float g[4];
    uint32_t kids[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        g[i] = 1.0f - fq[i] * invB;
        const float ag = fabsf(g[i]), fl = floorf(ag);
        kids[i] = (uint32_t)fminf(fl, 1.0e6f) + (uu[i] < ag - fl ? 1u : 0u);
    }
    if (booth_r > 0.0f) {
        for (int l = 0; l < 256 && st.alive && st.pos > 0; ++l) {
            const int li = l & 3;
            const float gs = li == 0 ? g[0] : li == 1 ? g[1] : li == 2 ? g[2] : g[3];
            const float us = li == 0 ? uu[0] : li == 1 ? uu[1] : li == 2 ? uu[2] : uu[3];
            booth_step(lane_f(gs, l >> 2), lane_f(us, l >> 2), booth_r, st, seed, chain, iter);
        }
        return;
    }
    int l = 0;
    while (l < 256 && st.alive && st.pos + st.neg > 0) {
        if (st.pos == 1 && st.neg == 0) {
            // the first event at or after sample l; samples before it continue the chain
            int e = 256;
#pragma unroll
            for (int i = 3; i >= 0; --i) {
                const int j = 4 * lane + i;
                if (j >= l && (kids[i] == 0u || g[i] < 0.0f || st.ns + (uint32_t)(j - l) == st.next_flip)) e = j;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) e = min(e, __shfl_xor(e, off));
            e = uni_i(e);
            float sum = 0.0f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = 4 * lane + i;
                sum += (j >= l && j < e) ? g[i] : 0.0f;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
            st.ans += (double)uni_f(sum);
            st.ns += (uint32_t)(e - l);
            l = e;
            if (l >= 256) break;
        }
        // one sample through the general rule
        if (st.ns == st.next_flip) {
            if (chain_coin(seed, chain, iter, st.coin++) < 0.5f) st.weight *= 2.0f;
            else { st.alive = false; break; }
            st.next_flip *= 2u;
        }
        const int li = l & 3;
        const float gs = li == 0 ? g[0] : li == 1 ? g[1] : li == 2 ? g[2] : g[3];
        const uint32_t ks = li == 0 ? kids[0] : li == 1 ? kids[1] : li == 2 ? kids[2] : kids[3];
        const float gl = lane_f(gs, l >> 2);
        const uint32_t kl = lane_u(ks, l >> 2);
        bool positive = st.pos > 0;
        if (positive) st.pos--; else st.neg--;
        st.ns++;
        st.ans += positive ? (double)gl : -(double)gl;
        if (positive == (gl >= 0.0f)) st.pos += kl; else st.neg += kl;
        ++l;
    }
}

__device__ __forceinline__ void chain_finish(Cand &c, const ChainRun &st, bool trunc, float mx, float *runmax,
                                             unsigned long long *cnt)
{
    // lane 0 of the chain's wavefront
    atomicAdd(cnt + C_CHAIN_HIST + min(23, 31 - __clz((int)max(st.ns, 1u))), 1ull);
    atomicMax(cnt + C_CHAIN_MAX, (unsigned long long)st.ns);
    const float est = (st.alive || trunc) ? (float)(st.ans * (double)st.weight / (double)c.B) : 0.0f;
    unsafeAtomicAdd(&c.recip_sum, est);
    atomic_maxf(runmax + cand_cls(c.cls_u) * 5 + cand_u(c.cls_u), mx);
    atomic_maxf(&c.pmax, mx);   // the candidate's largest f/q, pilot and chains (bucket statistics)
}

// stage A of one chain (item `wave` of a scene's (candidate, repeat) list, wave-uniform): one
// wavefront draws at most `budget` samples, then hands a running chain over to the rounds.
// Lane l computes samples l, 64 + l, 128 + l, ... (sample step * 64 + l has its own Philox
// counter, so its value does not depend on when it is computed); the chain consumes whole steps
// of 64 in order. A lane whose sample ends early (a miss, a zero) starts its next one while the
// others still trace, up to `ahead` steps beyond the oldest step not yet consumed (1: the lanes
// move in lockstep, one sample each per step); the values of up to two steps wait in registers.
// The uniform that splits a sample's |g| into whole and fractional children has a Philox counter
// of its own (CHAIN_UNI + sample index), drawn when the sample is consumed.
template <typename SE, bool BOOTH>
__device__ __forceinline__ void stage_a_chain(CtxT<SE> &C, Cand *cand, const uint32_t *final_, const uint32_t *order,
                                              int wave, int repeats, uint32_t seed, uint32_t iter, uint32_t n1,
                                              uint32_t budget, float *runmax, ChainState *longq, float booth_r,
                                              unsigned long long *cnt, int lane, int ahead, uint32_t &ns,
                                              uint32_t &drawn)
{
    const uint32_t ci = final_[order[wave / repeats]];
    const uint32_t chain = ci * 8u + (uint32_t)(wave % repeats);
    Cand &c = cand[ci];
    const float invB = 1.0f / c.B;
    ChainRun st{1.0, 1.0f, 1u, 0u, 0u, n1, 0u, true, 1.0f, 1.0f};
    float mx = 0.0f, fs = 0.0f;
    uint32_t nd = 0;
    const FqCand K = fq_cand(C.S, c);
    const int smax = (int)((budget + 63u) / 64u);   // steps stage A may consume
    ahead = min(max(ahead, 1), 2);                   // the register ring holds two steps
    int t = 0, head = 0;                             // this lane's step; the oldest unconsumed step
    Rng r = rng_make(seed, S_RECIP, chain, iter, (uint32_t)lane);
    FqState s;
    fq_begin(C.S, K, r, s);
    float v0 = 0.0f, v1 = 0.0f;   // f/q of the steps by step & 1
    while (st.alive && st.pos + st.neg > 0 && st.ns < budget && head < smax) {
        if (t < smax && t < head + ahead) {
            Hit h;
            C.rays++;
            const bool hit = traverse_rt<true>(C.S, s.ro, s.rd, C.S.tmin, s.rmax, s.ig0, s.ig1, s.any, C.stk,
                                               C.stride, h, &C.visits, &C.tests, &C.trips);
            float fq;
            if (fq_advance(C.S, K, r, s, hit, h, fq)) {
                v0 = (t & 1) == 0 ? fq : v0;
                v1 = (t & 1) == 1 ? fq : v1;
                ++t;
                if (t < smax) {
                    r = rng_make(seed, S_RECIP, chain, iter, (uint32_t)(t * 64 + lane));
                    fq_begin(C.S, K, r, s);
                }
            }
        }
        // the oldest step is complete once every lane has computed its sample of it
        while (st.alive && st.pos + st.neg > 0 && st.ns < budget && head < smax && __ballot(t <= head) == 0ull) {
            const float fq = (head & 1) == 0 ? v0 : v1;
            Rng ru = rng_make(seed, S_RECIP, chain, iter, CHAIN_UNI + (uint32_t)(head * 64 + lane));
            const float uu = rng_f(ru);
            // the step's largest and summed f/q (wave-uniform)
            float smx = fq, ssum = fq;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                smx = fmaxf(smx, __shfl_xor(smx, off));
                ssum += __shfl_xor(ssum, off);
            }
            mx = fmaxf(mx, uni_f(smx));
            fs += uni_f(ssum);
            nd += 64u;
            chain_consume(fq, uu, 64, invB, st, seed, chain, iter, BOOTH ? booth_r : 0.0f);
            ++head;
        }
    }
    drawn += (uint32_t)t;   // samples this lane computed (some beyond the last consumed step)
    // every f/q of the consumed steps is an i.i.d. sample of the candidate's ratio: its (class, u,
    // S, C) bucket's mean estimates beta for later iterations
    if (lane == 0 && nd > 0) {
        unsafeAtomicAdd(&c.psum, fs);
        unsafeAtomicAdd(&c.pn, (float)nd);
    }
    ns += st.ns;
    if (lane == 0) {
        const bool running = st.alive && st.pos + st.neg > 0;
        int slot = -1;
        if (running) {
            slot = (int)atomicAdd(cnt + C_LONGQ0, 1ull);
            if (slot >= CHAIN_LIST_CAP) slot = -1;
        }
        if (slot >= 0) {
            ChainState q{ci, chain, st.ans, st.weight, mx, st.pos, st.neg, st.ns, st.next_flip, st.coin,
                         st.bprod, st.bw};
            longq[slot] = q;
        } else {
            if (running) atomicAdd(cnt + C_RECIP_TRUNC, 1ull);
            chain_finish(c, st, running, mx, runmax, cnt);
        }
    }
}

// Stage A of one chain with walks refilled node by node (4-wide trees): the lanes walk one node
// at a time while at least PT_REFILL_MIN of them still walk; then every lane whose walk ended
// advances its sample and, if the sample goes on, starts the walk of its next trip, or, if it is
// complete, starts its next sample within the look-ahead; then the chain consumes the complete
// steps. So a lane whose ray ended early starts more work instead of waiting for the longest walk
// of the wavefront. The samples, their counters and the order of consumption are those of
// stage_a_chain.
#ifndef PT_REFILL_MIN
#define PT_REFILL_MIN 40
#endif
template <typename SE, bool BOOTH>
__device__ __forceinline__ void stage_a_chain_refill(CtxT<SE> &C, Cand *cand, const uint32_t *final_,
                                                     const uint32_t *order, int wave, int repeats, uint32_t seed,
                                                     uint32_t iter, uint32_t n1, uint32_t budget, float *runmax,
                                                     ChainState *longq, float booth_r, unsigned long long *cnt,
                                                     int lane, int ahead, uint32_t &ns, uint32_t &drawn)
{
    const uint32_t ci = final_[order[wave / repeats]];
    const uint32_t chain = ci * 8u + (uint32_t)(wave % repeats);
    Cand &c = cand[ci];
    const float invB = 1.0f / c.B;
    ChainRun st{1.0, 1.0f, 1u, 0u, 0u, n1, 0u, true, 1.0f, 1.0f};
    float mx = 0.0f, fs = 0.0f;
    uint32_t nd = 0;
    const FqCand K = fq_cand(C.S, c);
    const int smax = (int)((budget + 63u) / 64u);
    ahead = min(max(ahead, 1), 2);
    int t = 0, head = 0;
    Rng r = rng_make(seed, S_RECIP, chain, iter, (uint32_t)lane);
    FqState s;
    fq_begin(C.S, K, r, s);
    Walk w;
    walk_begin(w, s.ro, s.rd, C.S.tmin, s.rmax, s.ig0, s.ig1, s.any);
    C.rays++;
    bool walking = true, busy = true;   // a ray in flight; a sample in flight
    float v0 = 0.0f, v1 = 0.0f;
    while (st.alive && st.pos + st.neg > 0 && st.ns < budget && head < smax) {
        do {
            if (walking && walk_step<true>(C.S, w, C.stk, C.stride, &C.visits, &C.tests, &C.trips)) walking = false;
        } while (__popcll(__ballot(walking)) >= PT_REFILL_MIN);
        if (busy && !walking) {
            float fq;
            if (fq_advance(C.S, K, r, s, w.h.tri >= 0, w.h, fq)) {
                v0 = (t & 1) == 0 ? fq : v0;
                v1 = (t & 1) == 1 ? fq : v1;
                ++t;
                busy = false;
            } else {
                walk_begin(w, s.ro, s.rd, C.S.tmin, s.rmax, s.ig0, s.ig1, s.any);
                C.rays++;
                walking = true;
            }
        }
        if (!busy && t < smax && t < head + ahead) {
            r = rng_make(seed, S_RECIP, chain, iter, (uint32_t)(t * 64 + lane));
            fq_begin(C.S, K, r, s);
            walk_begin(w, s.ro, s.rd, C.S.tmin, s.rmax, s.ig0, s.ig1, s.any);
            C.rays++;
            walking = true;
            busy = true;
        }
        while (st.alive && st.pos + st.neg > 0 && st.ns < budget && head < smax && __ballot(t <= head) == 0ull) {
            const float fq = (head & 1) == 0 ? v0 : v1;
            Rng ru = rng_make(seed, S_RECIP, chain, iter, CHAIN_UNI + (uint32_t)(head * 64 + lane));
            const float uu = rng_f(ru);
            float smx = fq, ssum = fq;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                smx = fmaxf(smx, __shfl_xor(smx, off));
                ssum += __shfl_xor(ssum, off);
            }
            mx = fmaxf(mx, uni_f(smx));
            fs += uni_f(ssum);
            nd += 64u;
            chain_consume(fq, uu, 64, invB, st, seed, chain, iter, BOOTH ? booth_r : 0.0f);
            ++head;
        }
    }
    drawn += (uint32_t)t;
    if (lane == 0 && nd > 0) {
        unsafeAtomicAdd(&c.psum, fs);
        unsafeAtomicAdd(&c.pn, (float)nd);
    }
    ns += st.ns;
    if (lane == 0) {
        const bool running = st.alive && st.pos + st.neg > 0;
        int slot = -1;
        if (running) {
            slot = (int)atomicAdd(cnt + C_LONGQ0, 1ull);
            if (slot >= CHAIN_LIST_CAP) slot = -1;
        }
        if (slot >= 0) {
            ChainState q{ci, chain, st.ans, st.weight, mx, st.pos, st.neg, st.ns, st.next_flip, st.coin,
                         st.bprod, st.bw};
            longq[slot] = q;
        } else {
            if (running) atomicAdd(cnt + C_RECIP_TRUNC, 1ull);
            chain_finish(c, st, running, mx, runmax, cnt);
        }
    }
}

// stage A over one scene's chains: a persistent grid whose wavefronts take the next chains from a
// device counter; BOOTH selects Booth's roulette (booth_r) at compile time, so that the default
// instance carries none of its state
template <typename SE, bool BOOTH = false, bool REFILL = false>
__global__ void __launch_bounds__(64 * RW, PT_RECIP_WAVES) k_recip(SceneDev S, Cand *cand, const uint32_t *final_,
                                                   const uint32_t *order, int repeats,
                                                   uint32_t seed, uint32_t n1, uint32_t budget, float *runmax,
                                                   ChainState *longq, float booth_r, unsigned long long *cnt,
                                                   int chunk, int ahead)
{
    const uint32_t iter = iter_of(cnt);
    __shared__ SE stk[stk_depth<SE>() * 64 * RW];
    const int lane = threadIdx.x & 63;
    const int n = (int)cnt[C_NFINAL] * repeats;
    CtxT<SE> C{S, stk_col(stk, (int)threadIdx.x), 0u, (int)blockDim.x};
    uint32_t ns = 0, drawn = 0;
    // chunk consecutive chains per take from the counter (wave-uniform)
    for (int w0 = next_item(cnt + C_WORK_A) * chunk; w0 < n; w0 = next_item(cnt + C_WORK_A) * chunk)
        for (int wave = w0; wave < min(w0 + chunk, n); ++wave) {
            if constexpr (REFILL && !stk_wide8<SE>::value)
                stage_a_chain_refill<SE, BOOTH>(C, cand, final_, order, wave, repeats, seed, iter, n1, budget, runmax,
                                                longq, booth_r, cnt, lane, ahead, ns, drawn);
            else
                stage_a_chain<SE, BOOTH>(C, cand, final_, order, wave, repeats, seed, iter, n1, budget, runmax, longq,
                                         booth_r, cnt, lane, ahead, ns, drawn);
        }
    wave_count(cnt + C_RECIP_SAMPLES, lane == 0 ? ns : 0u);
    wave_count(cnt + C_SAMPLES_A, lane == 0 ? ns : 0u);
    wave_count(cnt + C_DRAWN_A, drawn);
    wave_count(cnt + C_RAYS_RECIP, C.rays);
    count_traversal(C, cnt, C_VISITS_A, C_TESTS_A, C_TRIPS_A);
}

// one scene's share of a multi-scene stage A (what k_recip takes as arguments)
struct RecipJob {
    SceneDev S;
    Cand *cand;
    const uint32_t *final_, *order;
    float *runmax;
    ChainState *longq;
    unsigned long long *cnt;
    int repeats;
    uint32_t seed, n1, budget;
    float booth_r;
};
// the scenes' chain lists laid end to end: base[j] = first item of scene j, base[n] = all items;
// the shared work counter restarts at zero
__global__ void k_multi_base(const RecipJob *jobs, int n, uint32_t *base, unsigned long long *work)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t b = 0;
    for (int j = 0; j < n; ++j) {
        base[j] = b;
        b += (uint32_t)jobs[j].cnt[C_NFINAL] * (uint32_t)jobs[j].repeats;
    }
    base[n] = b;
    *work = 0ull;
}
// stage A of several scenes in one persistent launch: the wavefronts take items from one work
// queue over every scene's chains (chunk consecutive items per take), so that the scenes' uneven
// chain counts share the device without a tail per scene; counts go to each item's scene
template <typename SE, bool BOOTH>
__global__ void __launch_bounds__(64 * RW, PT_RECIP_WAVES) k_recip_multi(const RecipJob *__restrict__ jobs, int n_jobs,
                                                                         const uint32_t *__restrict__ base,
                                                                         unsigned long long *work, int chunk,
                                                                         int ahead)
{
    __shared__ SE stk[stk_depth<SE>() * 64 * RW];
    const int lane = threadIdx.x & 63;
    const int total = (int)base[n_jobs];
    for (int w0 = next_item(work) * chunk; w0 < total; w0 = next_item(work) * chunk) {   // wave-uniform
        const int w1 = min(w0 + chunk, total);
        for (int w = w0; w < w1; ++w) {
            int j = 0;
            while (j + 1 < n_jobs && (int)base[j + 1] <= w) ++j;
            j = __builtin_amdgcn_readfirstlane(j);
            const RecipJob &J = jobs[j];
            CtxT<SE> C{J.S, stk_col(stk, (int)threadIdx.x), 0u, (int)blockDim.x};
            uint32_t ns = 0, drawn = 0;
            stage_a_chain<SE, BOOTH>(C, J.cand, J.final_, J.order, w - (int)base[j], J.repeats, J.seed, iter_of(J.cnt),
                                     J.n1, J.budget, J.runmax, J.longq, J.booth_r, J.cnt, lane, ahead, ns, drawn);
            wave_count(J.cnt + C_RECIP_SAMPLES, lane == 0 ? ns : 0u);
            wave_count(J.cnt + C_SAMPLES_A, lane == 0 ? ns : 0u);
            wave_count(J.cnt + C_DRAWN_A, drawn);
            wave_count(J.cnt + C_RAYS_RECIP, C.rays);
            count_traversal(C, J.cnt, C_VISITS_A, C_TESTS_A, C_TRIPS_A);
        }
    }
}

// samples per chain in round r for n running chains: doubling from 1024, so that a chain draws at
// most about twice the samples it uses; when few chains remain, enough to fill the device in one
// launch (CHAIN_FILL samples over all chains), so that long chains end in fewer latency-bound
// rounds; within the buffer; a multiple of 256 (the consumer's block)
// (2^17 measured about 1 ms per iteration faster than 2^16 or 2^18 on the 512^2 projector)
#ifndef CHAIN_FILL
#define CHAIN_FILL (1u << 17)
#endif
__device__ __forceinline__ uint32_t chain_round_size(uint32_t n, int round)
{
    const uint32_t want = max(1024u << round, CHAIN_FILL / max(n, 1u)) & ~255u;
    const uint32_t fit = (CHAIN_BUF / max(n, 1u)) & ~255u;
    return max(256u, min(want, fit));
}

// round r, part 1: every lane of the grid draws samples for the running chains
template <typename SE>
__global__ void __launch_bounds__(WG, PT_GEN_WAVES) k_chain_gen(SceneDev S, const Cand *__restrict__ cand,
                                                  const ChainState *__restrict__ list, int cidx, int round,
                                                  uint32_t seed, float2 *buf, unsigned long long *cnt)
{
    __shared__ SE stk[stk_depth<SE>() * WG];
    const uint32_t iter = iter_of(cnt);
    const uint32_t n = (uint32_t)min(cnt[cidx], (unsigned long long)CHAIN_LIST_CAP);
    CtxT<SE> C{S, stk_col(stk, (int)threadIdx.x), 0u, WG};
    if (n > 0) {
        const uint32_t G = chain_round_size(n, round);
        const uint64_t total = (uint64_t)n * G;
        for (uint64_t idx = (uint64_t)blockIdx.x * WG + threadIdx.x; idx < total; idx += (uint64_t)gridDim.x * WG) {
            const uint32_t slot = (uint32_t)(idx / G), j = (uint32_t)(idx % G);
            const ChainState &q = list[slot];
            Rng r = rng_make(seed, S_RECIP, q.chain, iter, CHAIN_LONG + ((uint32_t)round << 21) + j);
            const float fq = fq_sample(C, cand[q.ci], r);
            buf[idx] = make_float2(fq, rng_f(r));
        }
    }
    wave_count(cnt + C_RAYS_RECIP, C.rays);
    count_traversal(C, cnt);
}

// round r, part 2: one wavefront per running chain consumes its block in order; chains that
// still run move to the other list (or, after the last round, end as truncated)
__global__ void __launch_bounds__(64 * RW) k_chain_consume(Cand *cand, const ChainState *__restrict__ list, int cidx,
                                                           ChainState *next, int cidx_next, int round, int last,
                                                           uint32_t seed, const float2 *__restrict__ buf,
                                                           float *runmax, float booth_r, unsigned long long *cnt)
{
    const uint32_t iter = iter_of(cnt);
    const int lane = threadIdx.x & 63;
    const uint32_t n = (uint32_t)min(cnt[cidx], (unsigned long long)CHAIN_LIST_CAP);
    uint32_t used = 0;
    for (uint32_t wave = blockIdx.x * RW + (threadIdx.x >> 6); wave < n; wave += gridDim.x * RW) {   // wave-uniform
        const ChainState q = list[wave];
        Cand &c = cand[q.ci];
        const float invB = 1.0f / c.B;
        ChainRun st{q.ans, q.weight, q.pos, q.neg, q.ns, q.next_flip, q.coin, true, q.bprod, q.bw};
        const uint32_t G = chain_round_size(n, round);
        const float2 *b = buf + (size_t)wave * G;
        float mx = q.mx;
        for (uint32_t base = 0; base < G && st.alive && st.pos + st.neg > 0; base += 256) {
            const float4 v0 = *(const float4 *)(b + base + 4 * lane), v1 = *(const float4 *)(b + base + 4 * lane + 2);
            const float fq[4] = {v0.x, v0.z, v1.x, v1.z}, uu[4] = {v0.y, v0.w, v1.y, v1.w};
            mx = fmaxf(mx, fmaxf(fmaxf(fq[0], fq[1]), fmaxf(fq[2], fq[3])));
            chain_consume4(fq, uu, invB, st, seed, q.chain, iter, booth_r);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
        used += st.ns - q.ns;
        if (lane == 0) {
            const bool running = st.alive && st.pos + st.neg > 0;
            int slot = -1;
            if (running && !last) {
                slot = (int)atomicAdd(cnt + cidx_next, 1ull);
                if (slot >= CHAIN_LIST_CAP) slot = -1;
            }
            if (slot >= 0) {
                ChainState o{q.ci, q.chain, st.ans, st.weight, mx, st.pos, st.neg, st.ns, st.next_flip, st.coin,
                             st.bprod, st.bw};
                next[slot] = o;
            } else {
                if (running) atomicAdd(cnt + C_RECIP_TRUNC, 1ull);
                chain_finish(c, st, running, mx, runmax, cnt);
            }
        }
    }
    wave_count(cnt + C_RECIP_SAMPLES, lane == 0 ? used : 0u);
}

// Candidate probe: one wavefront per estimate; `per` samples of f/q averaged into a plain
// Monte Carlo estimate of P, then one chain of I~ with the given B (no roulette).
__global__ void __launch_bounds__(64 * RW) k_recip_point(SceneDev S, Cand c, int n_est, int per, uint32_t seed,
                                                         uint32_t cap, float *est, uint32_t *ns_out, float *p_out)
{
    __shared__ int stk[PT_STACK * 64 * RW];
    const int wave = blockIdx.x * RW + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    Ctx C{S, stk + threadIdx.x, 0u, (int)blockDim.x};
    if (wave >= n_est) return;   // wave-uniform
    float acc = 0.0f;
    for (int base = 0; base < per; base += 64) {
        Rng r = rng_make(seed, S_TABLE, (uint32_t)wave, 1u, (uint32_t)(base + lane));
        float v = base + lane < per ? fq_sample(C, c, r) : 0.0f;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        acc += v;
    }
    const float invB = 1.0f / c.B;
    float ans = invB;
    uint32_t pos = 1, neg = 0, ns = 0, trunc = 0;
    for (int step = 0; pos + neg > 0; ++step) {
        if (ns >= cap) { trunc = 1; break; }
        Rng r = rng_make(seed, S_TABLE, (uint32_t)wave, 2u, (uint32_t)(step * 64 + lane));
        const float fq = fq_sample(C, c, r);
        const float u = rng_f(r);
        for (int l = 0; l < 64; ++l) {
            if (pos + neg == 0) break;
            const float g = 1.0f - lane_f(fq, l) * invB;
            const float ul = lane_f(u, l);
            float sgn = 1.0f;
            if (pos > 0) pos--; else { neg--; sgn = -1.0f; }
            ns++;
            ans += sgn * g * invB;
            const float ag = fabsf(g), fl = floorf(ag);
            const uint32_t kids = (uint32_t)fminf(fl, 1.0e6f) + (ul < ag - fl ? 1u : 0u);
            if ((sgn > 0.0f) == (g >= 0.0f)) pos += kids; else neg += kids;
        }
    }
    if (lane == 0) {
        est[wave] = ans;
        ns_out[wave] = ns | (trunc << 31);
        if (p_out) p_out[wave] = acc / (float)per;
    }
}

// ---------------------------------------------------------------------------------- eye pass
struct EyeBuf {
    float4 *ro, *rd, *hit, *beta;   // beta.w = solid-angle pdf of the last sampled direction
    uint32_t *info;                 // bits 0..7 depth, 8 previous vertex Dirac, 9..10 phase, 11..14 u
    float4 *mis;                    // x = p(z_d -> y_{s-1}) in area measure, y = T, z = S (bits)
    float4 *mis2;                   // eye-side MIS partials of the ray in flight (times its d^2):
                                    // x with connections, y without (proxy-class paths); z = eye
                                    // subspace of the vertex the ray left (bits)
    uint32_t *q[2];
    ShadowRay *shadow;
    ProxyItem *proxy;
    float *frame;                   // [npix * 3] this iteration's pixel values
    int npix;
};

// solid-angle density of the camera direction d for a uniform point on its pixel (image plane at
// distance 1): 1 / (pixel area cos^3)
__device__ __forceinline__ float camera_pdf(const CamDev &c, float3 d)
{
    const float ct = dot3(d, c.f);
    if (!(ct > 0.0f)) return 0.0f;
    const float a_pix = 4.0f * c.tan_half * c.tan_half * c.aspect / ((float)c.w * (float)c.h);
    return 1.0f / (a_pix * ct * ct * ct);
}

__global__ void k_camera(SceneDev S, EyeBuf E, uint32_t seed, unsigned long long *cnt)
{
    const uint32_t iter = iter_of(cnt);
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) cnt[C_EYE_Q0] = (unsigned long long)E.npix;
    if (p >= E.npix) return;
    const int px = p % S.cam.w, py = p / S.cam.w;
    Rng r = rng_make(seed, S_EYE, (uint32_t)p, iter, 0u);
    const float jx = rng_f(r), jy = rng_f(r);
    const float x = (2.0f * (px + jx) / S.cam.w - 1.0f) * S.cam.tan_half * S.cam.aspect;
    const float y = (1.0f - 2.0f * (py + jy) / S.cam.h) * S.cam.tan_half;
    const float3 d = normalize3(S.cam.f + S.cam.r * x + S.cam.u * y);
    E.ro[p] = make_float4(S.cam.p.x, S.cam.p.y, S.cam.p.z, ibits(-1));
    E.rd[p] = make_float4(d.x, d.y, d.z, 3.0e38f);
    E.beta[p] = make_float4(1.f, 1.f, 1.f, camera_pdf(S.cam, d));
    E.mis2[p] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    E.info[p] = 1u << 8;   // camera counts as a Dirac predecessor for the first hit
    E.mis[p] = make_float4(0.f, 0.f, 0.f, 0.f);
    E.q[0][p] = (uint32_t)p;
}

struct EyeParams {
    uint32_t seed;
    int K, u_max;
    int filter;      // 0 all, 1 proxy class only, 2 other only, 3 none (for PT/NEE)
    int proxy_on;
    int nee_on;
    int mis_on;      // variance-aware MIS between the proxy strategy and PT/NEE (else a partition)
    int labels_on;   // compute eye subspaces T (Gamma selection or MIS)
    int gamma_on;
    int mlp_on;      // subspace S chosen by k_mlp_select (learned mixture) before k_proxy
    int vmf_on;      // first retrace direction at a glossy y_{s-1} from the learned vMF mixture
    float mix;       // weight of the learned densities in their mixtures with plain sampling
    int tiles_on;
    int M, cand_cap;
    MisK mk;             // strategy factors of the connection MIS
    int conn_on;         // light-vertex connections
    int gcv;             // the proxy class holds class C (general control vertex) as well
};
// k_sel = M pi_inc c pi_sel: the proxy strategy's selection factor for a path whose first
// diffuse eye vertex lies in T and whose y_{s-1} lies in S (surrogate used by both strategies)
__device__ __forceinline__ float proxy_ksel(const SubDev &D, const EyeParams &P, const unsigned long long *cnt, int T,
                                            int S, float c)
{
    // frozen inputs only (the previous iteration's counts), so that the weight of a proxy
    // sample does not depend on the light paths that produced it
    const float ncand = D.prev[0], nk = D.prev[1];
    if (!(nk > 0.0f) || !(ncand > 0.0f)) return 0.0f;
    const float pi_inc = fminf(1.0f, (float)P.cand_cap / ncand);
    float ps;
    if (P.gamma_on) {
        const int cs = D.s_count_prev[S];
        ps = cs > 0 ? sel_prob_frozen(D, T, S) / (float)cs : 0.0f;
    } else {
        ps = 1.0f / nk;
    }
    return (float)P.M * pi_inc * c * ps;
}

// eye-side factor K of the split whose light end is z_t and whose eye end is z_{t-1} (z_t not
// the emitter x_0): light tracing when z_{t-1} is the camera, else a connection (z_t labelled as
// a light vertex with the direction toward its light-side neighbour w_light, z_{t-1} by T_prev);
// conn = false leaves the connections out (proxy-class paths)
__device__ __forceinline__ float eye_split(const EyeParams &P, const ConnDev &C, const SceneDev &S, bool conn, int t,
                                           bool z_dirac, bool prev_dirac, int T_prev, float3 x, float3 n,
                                           float3 w_light)
{
    if (z_dirac) return 0.0f;
    if (t == 1) return P.mk.kL;
    if (!conn || prev_dirac || !(P.mk.kS > 0.0f)) return 0.0f;
    return conn_k(C, P.mk.kS, T_prev, conn_label_light(S, C, x, n, w_light));
}
// may a light-vertex connection or splat score a path of this class?
__device__ __forceinline__ bool conn_ok(const EyeParams &P, bool cls)
{
    return P.proxy_on ? (!cls && (P.filter == 0 || P.filter == 2)) : class_ok(P.filter, cls);
}

__global__ void k_eye_shade(SceneDev S, EyeBuf E, EyeParams P, SubDev D, LightBuf L, ConnDev C, int t,
                            unsigned long long *cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = (int)cnt[C_EYE_Q0 + t - 1];
    const uint32_t *qin = E.q[(t - 1) & 1];
    uint32_t *qout = E.q[t & 1];
    bool cont = false, shadow = false, shadow2 = false, proxy = false;
    int pid = 0;
    ShadowRay sr, sr2;
    ProxyItem pi;
    float4 nro, nrd, nbeta, nmis;
    float4 nmis2 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    uint32_t ninfo = 0;
    if (i < n) {
        pid = qin[i];
        const float4 h = E.hit[pid];
        const int tri = fbits(h.w);
        if (tri >= 0) {
            const float4 o = E.ro[pid], d = E.rd[pid];
            const float3 x = xyz(o) + xyz(d) * h.x;
            const TriShade &sh = S.shade[tri];
            const MatDev m = S.mats[sh.mat];
            const float3 wo = -xyz(d);
            const float4 bt = E.beta[pid];
            const float3 beta = xyz(bt);
            uint32_t info = E.info[pid];
            uint32_t ph = (info >> 9) & 7u, uu = (info >> 12) & 15u, kk = (info >> 16) & 7u;
            const bool prev_delta = (info >> 8) & 1u;
            float4 mis = P.labels_on ? E.mis[pid] : make_float4(0.f, 0.f, 0.f, 0.f);
            const int Tl = fbits(mis.y), Sl = fbits(mis.z);
            const float c_pix = P.tiles_on ? tile_prob(D, pid, S.cam.w) : 1.0f;
            // eye-side MIS state at z_t: its density from the eye side, and e_t with
            // C(z_{t-1}) = e_t * (density at z_t of the direction toward z_{t-1})
            const float d2 = h.x * h.x;
            const float cos_o = fabsf(dot3(sh.n, wo));
            const float rev_z = bt.w * cos_o / d2;
            const float4 m2 = t >= 2 ? E.mis2[pid] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            const float e_t = m2.x / d2, e0_t = m2.y / d2;
            const int T_prev = fbits(m2.z);
            float3 add = f3(0.f, 0.f, 0.f);
            if (m.flags & MF_EMIT) {
                const bool cls = pstate_closes(ph, uu);
                if (class_ok(P.filter, cls)) {
                    const float3 le = emission(S, tri, h.y, h.z, wo);
                    if (nonzero3(le)) {
                        float w = 1.0f;
                        const float cl = fabsf(dot3(sh.n, wo));
                        if (cls && P.mis_on && P.proxy_on) {
                            // three strategies build this proxy-class path (area measure at y_0,
                            // common factors dropped): BSDF hit, NEE at the previous vertex, proxy
                            const float J0 = cl / d2;
                            // class B: this emitter point is the control vertex y_0
                            const int Cl = ph == 2 ? ctrl_label(S, D, x, tri) : 0;
                            const float Ap = proxy_mis_factor(D, ph == 2 ? 1 : 0, (int)uu, Sl, Cl,
                                                              proxy_ksel(D, P, cnt, Tl, Sl, c_pix));
                            // w = 1 / (1 + C_0 + P_proxy / P_0), C_0 without the connections
                            const float hit = mis.x * bt.w * J0;
                            const float prx = ph == 2 ? Ap / S.em_area : Ap * bt.w * J0;
                            const float K1 = prev_delta ? 0.0f : P.mk.kN;
                            const float C0 = (1.0f / S.em_area) / rev_z * (K1 + e0_t * (cl / PT_PI));
                            w = hit > 0.0f ? hit / (hit * (1.0f + C0) + prx) : 0.0f;
                        } else if (t >= 2) {
                            // emission hit (s = 0): w = 1 / (1 + C_0), C_0 = fwd(x_0) / rev(x_0) (K_1 + C_1)
                            const float K1 = prev_delta ? 0.0f : P.mk.kN;
                            const float c1 = e_t * (cl / PT_PI);
                            const float C0 = (1.0f / S.em_area) / rev_z * (K1 + c1);
                            w = 1.0f / (1.0f + C0);
                        }
                        add = beta * le * w;
                    }
                }
            }
            if (nonzero3(add)) atomic_add3(E.frame + 3 * pid, add);
            if (t < P.K) {
                const bool spec = (m.flags & MF_SPEC) != 0;
                const bool z_dirac = (m.flags & MF_DELTA) != 0;
                const uint32_t ph0 = ph, uu0 = uu;
                pstate_push(ph, uu, kk, spec, m.type == MAT_LAMBERT, P.u_max, P.gcv != 0);
                Rng r = rng_make(P.seed, S_EYE, (uint32_t)pid, iter_of(cnt), (uint32_t)t);
                const bool at_zd = ph == 1 && uu == 0 && !spec;
                int Tnew = Tl;
                if (at_zd && P.labels_on) {
                    float f[9];
                    feat9(S, x, sh.n, wo, f);
                    Tnew = nearest_set(D.eye, f);
                }
                const float u0 = rng_f(r), u1 = rng_f(r), u2 = rng_f(r);
                const float ut = rng_f(r);
                if (P.proxy_on && at_zd && ut < c_pix) {
                    proxy = true;
                    pi.x = make_float4(x.x, x.y, x.z, ibits(tri));
                    pi.wo = make_float4(wo.x, wo.y, wo.z, ibits(t));
                    pi.beta = make_float4(beta.x, beta.y, beta.z, ibits(pid));
                    pi.aux = make_float4(ibits(Tnew), c_pix, 0.f, 0.f);
                    pi.mis = make_float4(rev_z, e0_t, 0.f, 0.f);
                }
                if (P.nee_on && !z_dirac && S.n_em > 0) {
                    const bool cls = pstate_closes(ph, uu);
                    const bool mis3 = cls && P.mis_on && P.proxy_on;
                    if (class_ok(P.filter, cls)) {
                        const LPoint Lp = sample_emitter(S, u0, u1, u2);
                        const float3 dl = Lp.p - x;
                        const float dist2 = dot3(dl, dl), dist = sqrtf(dist2);
                        const float3 wl = dl * (1.0f / dist);
                        const float cl = -dot3(Lp.n, wl);
                        if (cl > 0.0f) {
                            const float3 fs = bsdf_f(m, sh.n, wo, wl);
                            if (nonzero3(fs)) {
                                const float3 le = emission(S, Lp.tri, Lp.b1, Lp.b2, -wl);
                                const float pl = dist2 / (cl * S.em_area);
                                const float pb = bsdf_pdf(m, sh.n, wo, wl);
                                float w;
                                if (mis3) {
                                    // this vertex is y_1. If it is y_{s-1} itself (class A, u = 1), its
                                    // density from z_d and its subspace (with the direction toward this
                                    // path's light-side neighbour, here the light sample) are taken now
                                    const bool at_v = ph == 1 && uu == 1;
                                    float pz = mis.x;
                                    int Sv = Sl;
                                    if (at_v) {
                                        pz = bt.w * cos_o / d2;
                                        float f[9];
                                        feat9(S, x, sh.n, wl, f);
                                        Sv = nearest_set(D.spec, f);
                                    }
                                    const float J0 = cl / dist2;
                                    // class B: the light sample is the control vertex y_0
                                    const int Cv = ph == 2 ? ctrl_label(S, D, Lp.p, Lp.tri) : 0;
                                    const float Ap = proxy_mis_factor(D, ph == 2 ? 1 : 0, (int)uu, Sv, Cv,
                                                                      proxy_ksel(D, P, cnt, Tl, Sv, c_pix));
                                    const float hitp = pz * pb * J0, nee = pz / S.em_area;
                                    const float prx = ph == 2 ? Ap / S.em_area : Ap * pb * J0;
                                    // w = K_1 / (K_1 + A_1 + C_1 + A_1 P_proxy / P_0), without connections
                                    const float fwd_z = (cl / PT_PI) * fabsf(dot3(sh.n, wl)) / dist2;
                                    const float C1 = fwd_z / rev_z *
                                                     (eye_split(P, C, S, false, t, false, prev_delta, T_prev, x, sh.n, wl) +
                                                      e0_t * bsdf_pdf(m, sh.n, wl, wo));
                                    w = nee > 0.0f ? P.mk.kN / (P.mk.kN + (hitp + prx) / nee + C1) : 0.0f;
                                } else {
                                    // s = 1: A_1 = rev(x_0) / fwd(x_0); C_1 = fwd(z) / rev(z) (K + e_t rev-pdf)
                                    const float A1 = pb / pl;
                                    const float fwd_z = (cl / PT_PI) * fabsf(dot3(sh.n, wl)) / dist2;
                                    const float c = e_t * bsdf_pdf(m, sh.n, wl, wo);
                                    const float C1 = fwd_z / rev_z *
                                                     (eye_split(P, C, S, true, t, false, prev_delta, T_prev, x, sh.n, wl) + c);
                                    w = P.mk.kN / (P.mk.kN + A1 + C1);
                                }
                                const float3 c = beta * fs * le * (fabsf(dot3(sh.n, wl)) / pl * w);
                                if (nonzero3(c)) {
                                    shadow = true;
                                    sr.o = make_float4(x.x, x.y, x.z, ibits(tri));
                                    sr.d = make_float4(wl.x, wl.y, wl.z, dist * 0.9999f);
                                    sr.c = make_float4(c.x, c.y, c.z, ibits(pid));
                                    sr.ign1 = Lp.tri;
                                    sr.tag = -1;
                                }
                            }
                        }
                    }
                }
                // connection: light subspace from row T of Q, then one vertex of that bucket
                const uint32_t xc = rng_u32(r);
                const float uc1 = rng_f(r);
                const uint32_t xc2 = rng_u32(r);
                const int T_z = (P.conn_on && !z_dirac) ? conn_label_eye(S, C, x, sh.n, wo) : 0;
                const int ne_l = P.conn_on ? *C.n_nonempty : 0;
                if (P.conn_on && !z_dirac && ne_l > 0 && P.mk.kS > 0.0f) {
                    const size_t row = (size_t)T_z * C.n_lsub;
                    const int Sl = C.nonempty[alias_draw(C.al_prob + row, C.al_idx + row, ne_l, xc, uc1)];
                    const int cs = C.count[Sl];
                    // the bucket's vertex uniformly: index_of realises index_prob(k, cs)
                    const int kv = cs > 0 ? index_of(xc2, cs) : 0;
                    const float sel = cs > 0 ? conn_sel(C, T_z, Sl) * (float)(index_prob(kv, cs) * (double)cs) : 0.0f;
                    const uint32_t v = (uint32_t)C.list[C.off[Sl] + kv];
                    const int j = (int)(v / (uint32_t)L.M), lp = (int)(v % (uint32_t)L.M);
                    const uint32_t sg = L.sig[lp];
                    if (sel > 0.0f && t + j + 1 <= P.K && conn_ok(P, light_tail_class(ph, uu, kk, sg, j, P.u_max, P.gcv != 0))) {
                        const float4 yv = L.lv[v];
                        const int ty = fbits(yv.w);
                        const float3 y = xyz(yv), ny = S.shade[ty].n;
                        const MatDev my = S.mats[S.shade[ty].mat];
                        const float3 wyp = normalize3(xyz(L.lv[v - (uint32_t)L.M]) - y);
                        const float3 dv = y - x;
                        const float dd2 = dot3(dv, dv), dist = sqrtf(dd2);
                        const float3 wzy = dv * (1.0f / dist), wyz = -wzy;
                        const float3 fz = bsdf_f(m, sh.n, wo, wzy);
                        const float3 fy = bsdf_f(my, ny, wyz, wyp);
                        if (nonzero3(fz) && nonzero3(fy)) {
                            const float cy = fabsf(dot3(ny, wyz)), cz = fabsf(dot3(sh.n, wzy));
                            const float4 lt = L.lt[v];
                            const float Kown = conn_k(C, P.mk.kS, T_z, Sl);
                            // light side: A_s = (phi_j rev-pdf(y_j) + K_j) rev(y_j) / fwd(y_j); K_j is the
                            // split before y_j, with y_j's eye subspace taken toward z
                            const bool prev_y_dirac = j >= 2 && (L.lfl[v - (uint32_t)L.M] & LV_DIRAC);
                            const float Kj = j == 1 ? P.mk.kN
                                                    : (prev_y_dirac ? 0.0f
                                                                    : conn_k(C, P.mk.kS, conn_label_eye(S, C, y, ny, wyz),
                                                                             C.lab[v - (uint32_t)L.M]));
                            const float rev_y = bsdf_pdf(m, sh.n, wo, wzy) * cy / dd2;
                            const float As = (L.lphi[v].x * bsdf_pdf(my, ny, wyz, wyp) + Kj) * rev_y / lt.w;
                            // eye side: C_s = fwd(z) / rev(z) (K + e_t rev-pdf(z))
                            const float fwd_z = bsdf_pdf(my, ny, wyp, wyz) * cz / dd2;
                            const float c = e_t * bsdf_pdf(m, sh.n, wzy, wo);
                            const float Cs = fwd_z / rev_z *
                                             (eye_split(P, C, S, true, t, false, prev_delta, T_prev, x, sh.n, wzy) + c);
                            const float w = Kown > 0.0f ? Kown / (Kown + As + Cs) : 0.0f;
                            const float3 cc = beta * fz * fy * xyz(lt) *
                                              (cy * cz / dd2 * ((float)cs / ((float)P.M * sel)) * w);
                            if (nonzero3(cc) && lt.w > 0.0f) {
                                shadow2 = true;
                                sr2.o = make_float4(x.x, x.y, x.z, ibits(tri));
                                sr2.d = make_float4(wzy.x, wzy.y, wzy.z, dist * 0.9999f);
                                sr2.c = make_float4(cc.x, cc.y, cc.z, ibits(pid));
                                sr2.ign1 = ty;
                                sr2.tag = (T_z << 12) | Sl;
                            }
                        }
                    }
                }
                const float a = rng_f(r), b = rng_f(r), cc = rng_f(r);
                const BS bs = bsdf_sample(m, sh.n, wo, a, b, cc, true);
                if (bs.ok) {
                    const float3 nb = beta * bs.w;
                    if (nonzero3(nb)) {
                        cont = true;
                        nro = make_float4(x.x, x.y, x.z, ibits(tri));
                        nrd = make_float4(bs.wi.x, bs.wi.y, bs.wi.z, 3.0e38f);
                        nbeta = make_float4(nb.x, nb.y, nb.z, bs.pdf);
                        ninfo = (uint32_t)t | (bs.delta ? 1u << 8 : 0u) | (ph << 9) | (uu << 12) | (kk << 16);
                        nmis = make_float4(mis.x, ibits(Tnew), mis.z, 0.f);
                        // e_{t+1} d^2 = (K + e_t rev-pdf(z)) |cos| / rev(z), the light side being z_{t+1}
                        const float rp = rev_pdf(m, sh.n, bs.wi, wo), cw = fabsf(dot3(sh.n, bs.wi)) / rev_z;
                        nmis2.x = (eye_split(P, C, S, true, t, z_dirac, prev_delta, T_prev, x, sh.n, bs.wi) + e_t * rp) * cw;
                        nmis2.y = (eye_split(P, C, S, false, t, z_dirac, prev_delta, T_prev, x, sh.n, bs.wi) + e0_t * rp) * cw;
                        nmis2.z = ibits(T_z);
                        if (P.labels_on && ph0 == 1 && uu0 == 0 && ph == 1 && uu == 1) {
                            // this vertex is y_{s-1}: record p(z_d -> y_{s-1}) (area) and its specular
                            // subspace from (position, normal, direction toward the light side)
                            float f[9];
                            feat9(S, x, sh.n, bs.wi, f);
                            nmis.x = bt.w * cos_o / d2;
                            nmis.z = ibits(nearest_set(D.spec, f));
                        }
                    }
                }
            }
        }
    }
    const int ss = wave_push(cnt + C_SHD0 + t, shadow);
    if (shadow) E.shadow[ss] = sr;
    const int ss2 = wave_push(cnt + C_SHD0 + t, shadow2);
    if (shadow2) E.shadow[ss2] = sr2;
    wave_count(cnt + C_SPC, shadow2 ? 1u : 0u);
    const int ps = wave_push(cnt + C_PROXYQ, proxy);
    if (proxy) E.proxy[ps] = pi;
    const int cs = wave_push(cnt + C_EYE_Q0 + t, cont);
    if (cont) {
        qout[cs] = (uint32_t)pid;
        E.ro[pid] = nro; E.rd[pid] = nrd; E.beta[pid] = nbeta; E.info[pid] = ninfo;
        E.mis2[pid] = nmis2;
        if (P.labels_on) E.mis[pid] = nmis;
    }
}

// Light tracing: every pool vertex y_j connects to the camera and splats onto its pixel,
// weighted against the other strategies (w = M / (M + A_k)); with the proxy strategy and its MIS,
// proxy-class paths are weighed against emission hits, NEE and the proxy (w = M / (M + A'_k +
// B_k P_proxy / P_0), A' without connections, B_k the emission-hit term of A_k).
template <typename SE>
__global__ void __launch_bounds__(WG) k_lt(SceneDev S, LightBuf L, EyeParams P, SubDev D, ConnDev C, float *frame,
                                           unsigned long long *cnt)
{
    __shared__ SE stk[stk_depth<SE>() * WG];
    const int i = blockIdx.x * WG + threadIdx.x;
    const uint32_t npool = (uint32_t)cnt[C_POOL];
    uint32_t done = 0, rays = 0;
    if ((uint32_t)i < npool) {
        const uint32_t v = L.pool[i];
        const int j = (int)(v / (uint32_t)L.M), lp = (int)(v % (uint32_t)L.M);
        const CamDev &cam = S.cam;
        const float4 yv = L.lv[v];
        const int ty = fbits(yv.w);
        const float3 y = xyz(yv), ny = S.shade[ty].n;
        const float3 dc = cam.p - y;
        const float dd2 = dot3(dc, dc), dist = sqrtf(dd2);
        const float3 wyc = dc * (1.0f / dist), dir = -wyc;
        const float ct = dot3(dir, cam.f);
        const uint32_t sg = L.sig[lp];
        const bool cls = light_tail_class(0u, 0u, 0u, sg, j, P.u_max, P.gcv != 0);
        const bool with_proxy = P.proxy_on && P.mis_on;
        const bool ok = P.proxy_on ? (with_proxy ? class_ok(P.filter, cls) : (!cls && (P.filter == 0 || P.filter == 2)))
                                   : class_ok(P.filter, cls);
        if (ct > 0.0f && ok) {
            const float sx = dot3(dir, cam.r) / ct / (cam.tan_half * cam.aspect);
            const float sy = dot3(dir, cam.u) / ct / cam.tan_half;
            const float fx = (sx + 1.0f) * 0.5f * (float)cam.w, fy = (1.0f - sy) * 0.5f * (float)cam.h;
            if (fx >= 0.0f && fy >= 0.0f && fx < (float)cam.w && fy < (float)cam.h) {
                const int px = min((int)fx, cam.w - 1), py = min((int)fy, cam.h - 1);
                const MatDev my = S.mats[S.shade[ty].mat];
                const float3 yprev = xyz(L.lv[v - (uint32_t)L.M]);
                const float3 wyp = normalize3(yprev - y);
                const float3 fy3 = bsdf_f(my, ny, wyc, wyp);
                const float4 lt = L.lt[v];
                if (nonzero3(fy3) && lt.w > 0.0f) {
                    const float cy = fabsf(dot3(ny, wyc));
                    const float pw = camera_pdf(cam, dir);
                    const float rev_y = pw * cy / dd2;
                    const float rho = bsdf_pdf(my, ny, wyc, wyp);
                    const float4 ph4 = L.lphi[v];
                    const bool prev_y_dirac = j >= 2 && (L.lfl[v - (uint32_t)L.M] & LV_DIRAC);
                    float w;
                    if (cls && with_proxy) {
                        // A'_k and B_k; P_proxy / P_0 from the proxy's surrogate at this path's z_d
                        const float K0j = j == 1 ? P.mk.kN : 0.0f;
                        const float Ak = (ph4.y * rho + K0j) * rev_y / lt.w;
                        const float Bk = ph4.z * rho * rev_y / lt.w;
                        int m = j;
                        while (m >= 1 && ((sg >> m) & 1u)) --m;   // z_d: first non-specular vertex from the camera
                        float BX = 0.0f;
                        if (m >= 2) {
                            const bool clsB = !((sg >> 1) & 1u);
                            const int u = clsB ? m - 2 : m - 1;
                            const size_t vm = (size_t)m * L.M + lp, vs = (size_t)(m - 1) * L.M + lp;
                            const float4 zd4 = L.lv[vm], ys4 = L.lv[vs];
                            const float3 zd = xyz(zd4), ys = xyz(ys4), ys2 = xyz(L.lv[vs - L.M]);
                            const int tz = fbits(zd4.w), ts = fbits(ys4.w);
                            const float3 nz = S.shade[tz].n, ns = S.shade[ts].n;
                            const MatDev mz = S.mats[S.shade[tz].mat];
                            const float3 eprev = m == j ? cam.p : xyz(L.lv[vm + L.M]);
                            const float3 wze = normalize3(eprev - zd);
                            const float3 dzs = ys - zd;
                            const float dzs2 = dot3(dzs, dzs);
                            const float3 wzs = dzs * rsqrtf(dzs2);
                            const float pz = bsdf_pdf(mz, nz, wze, wzs) * fabsf(dot3(ns, wzs)) / dzs2;
                            if (pz > 0.0f && P.labels_on) {
                                float f[9];
                                feat9(S, zd, nz, wze, f);
                                const int Tl = nearest_set(D.eye, f);
                                feat9(S, ys, ns, normalize3(ys2 - ys), f);
                                const int Sl = nearest_set(D.spec, f);
                                const float c_pix = P.tiles_on ? tile_prob(D, py * cam.w + px, cam.w) : 1.0f;
                                // class B: the path's emitter point y_0 is the control vertex
                                const int Cl = clsB ? ctrl_label(S, D, xyz(L.lv[lp]), fbits(L.lv[lp].w)) : 0;
                                const float Ap = proxy_mis_factor(D, clsB ? 1 : 0, u, Sl, Cl,
                                                                  proxy_ksel(D, P, cnt, Tl, Sl, c_pix));
                                float X;
                                if (clsB) {
                                    const float3 y0 = xyz(L.lv[lp]), y1 = xyz(L.lv[(size_t)L.M + lp]), y2 = xyz(L.lv[2 * (size_t)L.M + lp]);
                                    const int t1 = fbits(L.lv[(size_t)L.M + lp].w), t0 = fbits(L.lv[lp].w);
                                    const float3 d10 = y0 - y1;
                                    const float d102 = dot3(d10, d10);
                                    const float3 w10 = d10 * rsqrtf(d102);
                                    const float pb = bsdf_pdf(S.mats[S.shade[t1].mat], S.shade[t1].n, normalize3(y2 - y1), w10);
                                    const float J0 = fabsf(dot3(S.shade[t0].n, w10)) / d102;
                                    X = pb * J0 > 0.0f ? (Ap / S.em_area) / (pz * pb * J0) : 0.0f;
                                } else {
                                    X = Ap / pz;
                                }
                                BX = Bk * X;
                            }
                        }
                        w = P.mk.kL / (P.mk.kL + Ak + BX);
                    } else {
                        float Kj = j == 1 ? P.mk.kN : 0.0f;
                        if (j >= 2 && !prev_y_dirac && P.mk.kS > 0.0f)
                            Kj = conn_k(C, P.mk.kS, conn_label_eye(S, C, y, ny, wyc), C.lab[v - (uint32_t)L.M]);
                        const float Ak = (ph4.x * rho + Kj) * rev_y / lt.w;
                        w = P.mk.kL / (P.mk.kL + Ak);
                    }
                    const float3 c = xyz(lt) * fy3 * (pw * cy / dd2 / (float)P.M * w);
                    if (nonzero3(c)) {
                        Hit hh;
                        rays = 1;
                        if (!traverse<true, false>(S, y, wyc, S.tmin, dist * 0.9999f, ty, -1, stk_col(stk, (int)threadIdx.x), WG, hh)) {
                            atomic_add3(frame + 3 * (py * cam.w + px), c);
                            done = 1;
                        }
                    }
                }
            }
        }
    }
    wave_count(cnt + C_LT, done);
    wave_count(cnt + C_RAYS_SHADOW, rays);
}

// shadow rays of NEE and connections; a visible connection's luminance trains Q while learning
template <typename SE>
__global__ void __launch_bounds__(WG) k_occluded(SceneDev S, EyeBuf E, ConnDev C, int t, unsigned long long *cnt)
{
    __shared__ SE stk[stk_depth<SE>() * WG];
    const int i = blockIdx.x * WG + threadIdx.x;
    const int n = (int)cnt[C_SHD0 + t];
    const bool act = i < n;
    if (act) {
        const ShadowRay sr = E.shadow[i];
        Hit h;
        if (!traverse<true, false>(S, xyz(sr.o), xyz(sr.d), S.tmin, sr.d.w, fbits(sr.o.w), sr.ign1, stk_col(stk, (int)threadIdx.x),
                                   WG, h)) {
            atomic_add3(E.frame + 3 * fbits(sr.c.w), xyz(sr.c));
            if (sr.tag >= 0 && C.qacc && cnt[C_LEARN])
                unsafeAtomicAdd(C.qacc + (size_t)(sr.tag >> 12) * C.n_lsub + (sr.tag & 0xFFF), lum(xyz(sr.c)));
        }
    }
    wave_count(cnt + C_RAYS_SHADOW, act ? 1u : 0u);
}

struct StatBuf {
    float *gamma_acc;      // [n_eye * n_spec] accumulated proxy luminance per (T, S)
    float *tile_proxy, *tile_total;
};

// the learned selection's kernels (they read the proxy queue filled above)
#include "pt_mlp.h"

// Proxy connection (Section 5.1): pick a kept incomplete sub-path (Gamma[T, S] row by its alias
// table, then uniformly within S, Section 5.6; or uniformly among all), connect z_d to y_{s-1},
// retrace the u dropped vertices by sampling the BSDF at y_{s-1} given the direction to z_d and
// then at each new vertex, abort on an S/D mismatch, weight with 1/P's estimate and normalise by
// M pi_inc rho pi_j c; p(h*) = 1 (class A) or 1/A (class B). With MIS the contribution is
// weighted against PT and NEE (Section 5.4) with the same surrogate densities the eye pass uses.
template <typename SE>
__global__ void __launch_bounds__(WG) k_proxy(SceneDev S, EyeBuf E, const Cand *__restrict__ cand,
                                              const uint32_t *__restrict__ final_, EyeParams P, SubDev D,
                                              StatBuf SB, MlpTrain MT, const float *vmf, int repeats,
                                              unsigned long long *cnt)
{
    __shared__ SE stk[stk_depth<SE>() * WG];
    const int i = blockIdx.x * WG + threadIdx.x;
    const int n = (int)cnt[C_PROXYQ];
    const int nk = (int)cnt[C_NFINAL];
    CtxT<SE> C{S, stk_col(stk, (int)threadIdx.x), 0u, (int)blockDim.x};
    uint32_t valid = 0;
    if (i < n && nk > 0) {
        const ProxyItem it = E.proxy[i];
        const int pix = fbits(it.beta.w);
        const int T = fbits(it.aux.x);
        const float c_pix = it.aux.y;
        Rng r = rng_make(P.seed, S_PROXY, (uint32_t)pix, iter_of(cnt), 0u);
        int ci;
        float pi_j;
        int Ssel = 0;
        // every selection divides by the probability its draw realises (index_prob, the alias
        // row's realised pmf, the network mixture's), not by the nominal one
        const uint32_t x0 = rng_u32(r);
        const float u1 = rng_f(r);
        const uint32_t x2 = rng_u32(r);
        if (P.mlp_on) {
            // S from the learned mixture and the sub-path within it, with their probability,
            // drawn by k_mlp_select
            Ssel = fbits(it.aux.z);
            ci = fbits(it.mis.z);
            pi_j = ci >= 0 ? it.mis.w : 0.0f;
            if (ci < 0) ci = 0;
        } else if (P.gamma_on) {
            const int ne = *D.n_nonempty;
            const size_t row = (size_t)T * D.n_spec;
            Ssel = D.nonempty[alias_draw(D.al_prob + row, D.al_idx + row, ne, x0, u1)];
            const int cs = D.s_count[Ssel];
            const int k = index_of(x2, cs);
            ci = D.s_list[D.s_off[Ssel] + k];
            pi_j = (float)((double)sel_prob(D, T, Ssel) * index_prob(k, cs));
        } else {
            const int k = index_of(x0, nk);
            ci = (int)final_[k];
            pi_j = (float)index_prob(k, nk);
        }
        const Cand c = cand[ci];
        const int cls = cand_cls(c.cls_u), u = cand_u(c.cls_u);
        const int d = fbits(it.wo.w);
        float3 zn = f3(0.f, 0.f, 1.f);
        float3 add = f3(0.f, 0.f, 0.f);
        // the direction head's training sample of this contribution (glossy y_{s-1} only)
        bool glossy_rec = false;
        float3 rv = f3(0.f, 0.f, 0.f), rvn = rv, rwo = rv, rdir = rv;
        // segments of the path: d on the eye side, z_d -> y_{s-1}, u down to the dropped diffuse
        // vertex (classes B, C) or the emitter (A), then one to h_c = y_j and j along the light
        // prefix (j = 0 for class B)
        const int seg = d + 1 + u + (cls == 0 ? 0 : 1 + cand_j(c.cls_u));
        if (seg <= P.K && pi_j > 0.0f) {
            const float3 xd = xyz(it.x);
            const int td = fbits(it.x.w);
            const TriShade &shd = S.shade[td];
            const MatDev md = S.mats[shd.mat];
            zn = shd.n;
            const float3 v = xyz(c.v);
            const int vt = fbits(c.v.w);
            const float3 vn = S.shade[vt].n;
            const float3 dv = v - xd;
            const float d2 = dot3(dv, dv);
            const float3 wzv = dv * rsqrtf(d2);
            const float3 fz = bsdf_f(md, shd.n, xyz(it.wo), wzv);
            if (nonzero3(fz) && !occluded(C, xd, td, v, vt)) {
                const float G = fabsf(dot3(shd.n, wzv)) * fabsf(dot3(vn, wzv)) / d2;
                float3 thr = f3(1.f, 1.f, 1.f), term = f3(0.f, 0.f, 0.f);
                float3 cur = v, wo = -wzv, curn = vn, first_dir = f3(0.f, 0.f, 1.f);
                int curt = vt;
                // the path from z_d toward the light, for the light-tracing term of the weight
                float3 qp[PT_LMAX + 2];
                int qt[PT_LMAX + 2];
                int nq = 2;
                qp[0] = xd; qt[0] = td; qp[1] = v; qt[1] = vt;
                bool ok = true, last_delta = false;
                float last_pdf = 0.0f, J0 = 0.0f, pb_y1 = 0.0f;
                bool glossy_first = false;
                for (int k = 1; k <= u && ok; ++k) {
                    const MatDev m = S.mats[S.shade[curt].mat];
                    const float a = rng_f(r), b = rng_f(r), cc = rng_f(r);
                    BS bs;
                    if (k == 1 && P.vmf_on && !(m.flags & MF_DELTA)) {
                        // a glossy y_{s-1}: mix x learned vMF mixture + (1 - mix) x BSDF sampling,
                        // weighted by f |cos| over the mixture's density (the realised mixture
                        // weight of the 24-bit draw); the MIS weights keep the BSDF density
                        glossy_first = true;
                        const float *R = vmf + (size_t)i * MLP_VMF;
                        const float um = rng_f(r);
                        const double mw = below_prob(P.mix);
                        float3 wi;
                        if (um < P.mix) {
                            wi = vmf_mix_sample(R, a, b, cc);
                        } else {
                            const BS b0 = bsdf_sample(m, curn, wo, a, b, cc, true);
                            wi = b0.wi;
                            if (!b0.ok) wi = f3(0.f, 0.f, 0.f);
                        }
                        const float pb = bsdf_pdf(m, curn, wo, wi);
                        const float pm = (float)(mw * (double)vmf_mix_pdf(R, wi) + (1.0 - mw) * (double)pb);
                        const float3 fv = bsdf_f(m, curn, wo, wi);
                        bs.wi = wi;
                        bs.delta = false;
                        bs.pdf = pb;
                        bs.ok = pm > 0.0f && nonzero3(fv) && dot3(wi, wi) > 0.5f;
                        bs.w = bs.ok ? fv * (fabsf(dot3(curn, wi)) / pm) : f3(0.f, 0.f, 0.f);
                    } else {
                        bs = bsdf_sample(m, curn, wo, a, b, cc, true);
                    }
                    Hit h;
                    if (!bs.ok || !closest(C, cur, bs.wi, curt, h)) { ok = false; break; }
                    if (k == 1) first_dir = bs.wi;
                    thr = thr * bs.w;
                    last_pdf = bs.pdf; last_delta = bs.delta;
                    const MatDev mh = S.mats[S.shade[h.tri].mat];
                    const float3 y = tri_point(S, h.tri, h.b1, h.b2);
                    const float3 ny = S.shade[h.tri].n;
                    if (k < u) {
                        if (!(mh.flags & MF_SPEC)) { ok = false; break; }
                    } else if (cls == 0) {
                        if (!(mh.flags & MF_EMIT)) { ok = false; break; }
                        term = emission(S, h.tri, h.b1, h.b2, -bs.wi);
                        J0 = fabsf(dot3(ny, bs.wi)) / (h.t * h.t);
                    } else {
                        if (mh.flags & MF_SPEC) { ok = false; break; }
                        const float3 y0 = xyz(c.hc);
                        const int t0 = fbits(c.hc.w);
                        const float3 a0 = y0 - y;
                        const float e2 = dot3(a0, a0);
                        const float3 wl = a0 * rsqrtf(e2);
                        const float3 f1 = bsdf_f(mh, ny, -bs.wi, wl);
                        if (cls == 2) {
                            // class C: the light throughput arriving at h_c, the BSDF there from
                            // the control direction toward y, and the geometry term h_c <-> y
                            const float3 n0 = S.shade[t0].n;
                            const float3 f0 = bsdf_f(S.mats[S.shade[t0].mat], n0,
                                                     oct_dec(make_float2(c.hc_b1, c.hc_b2)), -wl);
                            if (!nonzero3(f0) || !nonzero3(f1) || occluded(C, y, h.tri, y0, t0)) { ok = false; break; }
                            term = f1 * xyz(c.beta_c) * f0 * (fabsf(dot3(n0, wl)) * fabsf(dot3(ny, wl)) / e2);
                        } else {
                            const float c0 = -dot3(S.shade[t0].n, wl);
                            if (c0 <= 0.0f || !nonzero3(f1) || occluded(C, y, h.tri, y0, t0)) { ok = false; break; }
                            const float3 le = emission(S, t0, c.hc_b1, c.hc_b2, -wl);
                            term = f1 * le * (c0 * fabsf(dot3(ny, wl)) / e2 * S.em_area);
                            J0 = c0 / e2;
                            pb_y1 = bsdf_pdf(mh, ny, -bs.wi, wl);
                        }
                    }
                    cur = y; curt = h.tri; curn = ny; wo = -bs.wi;
                    qp[nq] = y; qt[nq] = h.tri; ++nq;
                }
                if (ok && cls == 1) { qp[nq] = xyz(c.hc); qt[nq] = fbits(c.hc.w); ++nq; }
                if (ok) {
                    const float pi_inc = fminf(1.0f, (float)P.cand_cap / (float)cnt[C_NCAND]);
                    const float scale = (c.recip_sum / (float)repeats) /
                                        ((float)P.M * pi_inc * c.rho * pi_j * c_pix);
                    float w = 1.0f;
                    if (P.mis_on) {
                        // the same three densities the eye pass weighs with (area measure at y_0,
                        // common factors dropped): BSDF hit from y_1, NEE at y_1, proxy
                        float f[9];
                        feat9(S, v, vn, first_dir, f);
                        const int Sm = nearest_set(D.spec, f);
                        const float pz = bsdf_pdf(md, shd.n, xyz(it.wo), wzv) * fabsf(dot3(vn, wzv)) / d2;
                        const int Cm = cls ? ctrl_label(S, D, xyz(c.hc), fbits(c.hc.w)) : 0;
                        const float Ap = proxy_mis_factor(D, cls, u, Sm, Cm, proxy_ksel(D, P, cnt, T, Sm, c_pix));
                        float hit, nee, prx;
                        if (cls == 0) {
                            hit = pz * last_pdf * J0;
                            nee = last_delta ? 0.0f : pz / S.em_area;
                            prx = Ap * last_pdf * J0;
                        } else {
                            hit = pz * pb_y1 * J0;
                            nee = pz / S.em_area;
                            prx = Ap / S.em_area;
                        }
                        // light tracing and the eye-side strategies beyond z_d, relative to the
                        // emission hit: prod over q_0 = z_d .. q_n = y_0 of fwd / rev, times the
                        // eye-side factor at z_d (light tracing if z_d is the first vertex)
                        float lt = 0.0f;
                        const float e0 = it.mis.y;
                        const float kz = (d == 1 ? P.mk.kL : 0.0f) +
                                         e0 * rev_pdf(md, shd.n, wzv, xyz(it.wo));
                        if (kz > 0.0f && it.mis.x > 0.0f) {
                            float R = 1.0f;
                            for (int q = 0; q < nq; ++q) {
                                const float3 yq = qp[q];
                                // eye-side density of q_q
                                float rev;
                                if (q == 0) {
                                    rev = it.mis.x;
                                } else {
                                    const float3 a = qp[q - 1];
                                    const TriShade &sa = S.shade[qt[q - 1]];
                                    const float3 wi = normalize3(yq - a);
                                    const float3 wo2 = q == 1 ? xyz(it.wo) : normalize3(qp[q - 2] - a);
                                    const float3 dd = yq - a;
                                    rev = rev_pdf(S.mats[sa.mat], sa.n, wo2, wi) * fabsf(dot3(S.shade[qt[q]].n, wi)) /
                                          dot3(dd, dd);
                                }
                                // light-side density of q_q
                                float fwd;
                                if (q == nq - 1) {
                                    fwd = 1.0f / S.em_area;
                                } else {
                                    const float3 b = qp[q + 1];
                                    const TriShade &sb = S.shade[qt[q + 1]];
                                    const float3 dd = yq - b;
                                    const float dd2 = dot3(dd, dd);
                                    const float3 wq = dd * rsqrtf(dd2);
                                    float pdir;
                                    if (q + 1 == nq - 1) pdir = fmaxf(dot3(sb.n, wq), 0.0f) / PT_PI;   // cosine emission
                                    else pdir = rev_pdf(S.mats[sb.mat], sb.n, normalize3(qp[q + 2] - b), wq);
                                    fwd = pdir * fabsf(dot3(S.shade[qt[q]].n, wq)) / dd2;
                                }
                                R = rev > 0.0f ? R * fwd / rev : 0.0f;
                            }
                            lt = hit * R * kz;
                        }
                        w = prx > 0.0f ? prx / (hit + lt + nee + prx) : 0.0f;
                    }
                    add = xyz(it.beta) * fz * thr * term * (G * scale * w);
                    if (glossy_first) { glossy_rec = true; rv = v; rvn = vn; rwo = -wzv; rdir = first_dir; }
                }
            }
        }
        if (nonzero3(add)) {
            atomic_add3(E.frame + 3 * pix, add);
            valid = 1;
            if (cnt[C_LEARN]) {
                const float l = lum(add);
                if (P.gamma_on) unsafeAtomicAdd(SB.gamma_acc + (size_t)T * D.n_spec + Ssel, l);
                if (P.mlp_on && l > 0.0f) mlp_record(S, MT, cnt, xyz(it.x), zn, xyz(it.wo), Ssel, l);
                if (P.vmf_on && glossy_rec && l > 0.0f) mlp_record_dir(S, MT, cnt, rv, rvn, rwo, rdir, l);
                if (P.tiles_on) {
                    const int tl = (pix / S.cam.w) / D.tile * D.tiles_x + (pix % S.cam.w) / D.tile;
                    unsafeAtomicAdd(SB.tile_proxy + tl, l);
                }
            }
        }
    }
    wave_count(cnt + C_PROXY_ATT, (i < n && nk > 0) ? 1u : 0u);
    wave_count(cnt + C_PROXY_VALID, valid);
    wave_count(cnt + C_RAYS_PROXY, C.rays);
}

// frame -> caller accumulators; non-finite values are counted and dropped; frame cleared;
// while learning, each tile's total luminance is accumulated for the tile rule
__global__ void k_accumulate(float *frame, float *acc, float *acc2, int npix, int W, int tile, int tiles_x,
                             float *tile_total, unsigned long long *cnt)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t bad = 0;
    if (p < npix) {
        float v[3];
        for (int k = 0; k < 3; ++k) {
            v[k] = frame[3 * p + k];
            if (!isfinite(v[k])) { v[k] = 0.0f; bad = 1; }
            acc[3 * p + k] += v[k];
            if (acc2) acc2[3 * p + k] += v[k] * v[k];
            frame[3 * p + k] = 0.0f;
        }
        if (tile_total && cnt[C_LEARN]) {
            const float l = lum(f3(v[0], v[1], v[2]));
            if (l > 0.0f) unsafeAtomicAdd(tile_total + (p / W) / tile * tiles_x + (p % W) / tile, l);
        }
    }
    wave_count(cnt + C_NAN, bad);
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
// Philox4x32-10 of n (counter, key) rows: in[6 i .. 6 i + 5] = c0 c1 c2 c3 k0 k1 -> out[4 i .. 4 i + 3]
__global__ void k_philox_hook(const uint32_t *in, int n, uint32_t *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t *a = in + 6 * (size_t)i;
    uint32_t o[4];
    philox10(a[4], a[5], a[0], a[1], a[2], a[3], o);
    for (int k = 0; k < 4; ++k) out[4 * (size_t)i + k] = o[k];
}
// the iteration's counts added to the scene's running totals; the iteration's end stamp
__global__ void k_totals(const unsigned long long *cnt, unsigned long long *tot, long long *ts)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (ts) ts[2 * ((uint32_t)cnt[C_ITER] % PT_TS_CAP) + 1] = wall_clock64();
    tot[TOT_ITERS] += 1ull;
    tot[TOT_NAN] += cnt[C_NAN];
    tot[TOT_TRUNC] += cnt[C_RECIP_TRUNC];
    tot[TOT_PROXY_VALID] += cnt[C_PROXY_VALID];
    tot[TOT_RECIP_SAMPLES] += cnt[C_RECIP_SAMPLES];
    tot[TOT_CAND] += cnt[C_NCAND];
}

__global__ void k_copy(const float *src, float *dst, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}
__global__ void k_fill(float *p, float v, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_i(int *p, int v, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_resolve(const float *acc, float *out, int n, float inv)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = acc[i] * inv;
}

// ---------------------------------------------------------------------------------- test hooks
template <typename SE>
__global__ void __launch_bounds__(WG) k_trace_closest(SceneDev S, const float *rays, int n, float *t_out, int *prim_out)
{
    __shared__ SE stk[stk_depth<SE>() * WG];
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= n) return;
    const float *r = rays + 8 * (size_t)i;
    Hit h;
    const bool ok = traverse<false, false>(S, f3(r[0], r[1], r[2]), f3(r[3], r[4], r[5]), r[6], r[7], -1, -1,
                                           stk_col(stk, (int)threadIdx.x), WG, h);
    t_out[i] = ok ? h.t : -1.0f;
    prim_out[i] = ok ? S.tris[h.tri].prim : -1;
}

// Table mode of the reciprocal estimator: target 1 / sum f, supporting pmf q (inverse-CDF by a
// linear scan), estimator I~ (sign_est = 0) or the sign estimator I (sign_est = 1).
// Cumulative sums of the supporting pmf q of a table problem, in double, by one workgroup of
// 1024 threads (each a contiguous chunk): cdf[0] = 0, cdf[k + 1] = q[0] + ... + q[k].
__global__ void __launch_bounds__(1024) k_table_cdf(const float *q, int n, double *cdf)
{
    __shared__ double part[1024];
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int a = min(n, t * per), b = min(n, a + per);
    double acc = 0.0;
    for (int k = a; k < b; ++k) acc += (double)q[k];
    part[t] = acc;
    __syncthreads();
    // inclusive scan of the 1024 chunk sums (Hillis-Steele)
    for (int off = 1; off < 1024; off <<= 1) {
        const double v = t >= off ? part[t - off] : 0.0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    double run = t > 0 ? part[t - 1] : 0.0;
    if (t == 0) cdf[0] = 0.0;
    for (int k = a; k < b; ++k) {
        run += (double)q[k];
        cdf[k + 1] = run;
    }
}
// One draw from the table's supporting pmf by inverse CDF: a 53-bit uniform scaled by the total,
// binary search for the interval [cdf[k], cdf[k + 1]) that holds it. qk receives the probability
// that this draw realises, (cdf[k + 1] - cdf[k]) / cdf[n], which the estimator divides by.
__device__ __forceinline__ int table_draw(Rng &r, const double *cdf, int n, double &qk)
{
    const uint32_t xa = rng_u32(r), xb = rng_u32(r);
    const double u = (double)(((uint64_t)xa << 21) | (uint64_t)(xb >> 11)) * (1.0 / 9007199254740992.0);
    const double tot = cdf[n], t = u * tot;
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cdf[mid] <= t) lo = mid; else hi = mid;
    }
    qk = (cdf[lo + 1] - cdf[lo]) / tot;
    return lo;
}
__global__ void k_recip_table(const float *f, const double *cdf, int n, float B, int n_est, int est, float booth_r,
                              uint32_t seed, uint32_t cap, float *out, uint32_t *ns_out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_est) return;
    Rng r = rng_make(seed, S_TABLE, (uint32_t)e, 0u, 0u);
    const float invB = 1.0f / B;
    const int sign_est = est == 1;
    if (est == 2) {
        // Booth's roulette: one chain, go on with probability min(1, |prod g| / booth_r), the
        // terms beyond divided by the product of those probabilities; one uniform number per
        // sample after it, drawn where I~ draws its split
        float ans = 1.0f, prod = 1.0f, w = 1.0f;
        uint32_t ns = 0, trunc = 0;
        for (;;) {
            if (ns >= cap) { trunc = 1; break; }
            double qk;
            const int k = table_draw(r, cdf, n, qk);
            const float g = (float)(1.0 - (double)f[k] / (qk * (double)B));
            ns++;
            prod *= g;
            ans += prod / w;
            const float rr = fminf(1.0f, fabsf(prod) / booth_r);
            if (!(rng_f(r) < rr)) break;
            w *= rr;
        }
        out[e] = ans * invB;
        ns_out[e] = ns | (trunc << 31);
        return;
    }
    float ans = invB;
    uint32_t pos = 1, neg = 0, ns = 0, trunc = 0;
    while (pos + neg > 0) {
        if (ns >= cap) { trunc = 1; break; }
        float s = 1.0f;
        if (pos > 0) pos--; else { neg--; s = -1.0f; }
        double qk;
        const int k = table_draw(r, cdf, n, qk);
        const float g = (float)(1.0 - (double)f[k] / (qk * (double)B));
        ns++;
        ans += sign_est ? (ns > 1 ? s * invB : 0.0f) : s * g * invB;
        const float ag = fabsf(g), fl = floorf(ag);
        const uint32_t kids = (uint32_t)fl + (rng_f(r) < ag - fl ? 1u : 0u);
        if ((s > 0.0f) == (g >= 0.0f)) pos += kids; else neg += kids;
    }
    out[e] = ans;
    ns_out[e] = ns | (trunc << 31);
}
