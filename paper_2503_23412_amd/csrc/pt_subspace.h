// Subspaces and probabilistic selection (Section 3.2's subspaces, Sections 5.5 and 5.6):
// k-means over 9-D features (position normalised to the scene box, normal, incident
// direction), per-iteration bucketing of kept incomplete sub-paths by specular subspace S,
// Walker/Vose alias rows of the selection matrix Gamma[T, S], and the frozen statistics the
// MIS weights of Section 5.4 use.
#pragma once
#include "pt_device.h"

#define FEAT 12   // 9 features padded to 12 floats (three float4 loads)

// A set of K centroids with a two-level search: the nearest of G group centroids, then the
// nearest member of that group (the groups cluster the centroids themselves). The label is a
// deterministic function of the features, which is all the estimators and weights need; an
// empty nearest group falls back to the full search. G = 0: flat search.
struct CentSet {
    const float *c;          // [K * FEAT]
    const float *g;          // [G * FEAT]
    const int *start;        // [G + 1] member ranges
    const int *mem;          // [K] centroid ids by group
    int K, G;
};
__device__ __forceinline__ float feat_d2(const float *__restrict__ c, const float f[9])
{
    const float4 a = *(const float4 *)c, b = *(const float4 *)(c + 4), e = *(const float4 *)(c + 8);
    const float d0 = a.x - f[0], d1 = a.y - f[1], d2 = a.z - f[2], d3 = a.w - f[3], d4 = b.x - f[4],
                d5 = b.y - f[5], d6 = b.z - f[6], d7 = b.w - f[7], d8 = e.x - f[8];
    return d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3 + d4 * d4 + d5 * d5 + d6 * d6 + d7 * d7 + d8 * d8;
}

struct SubDev {
    const float *eye_c;      // [n_eye * FEAT] centroids of eye first-diffuse vertices (T)
    const float *spec_c;     // [n_spec * FEAT] centroids of specular vertices y_{s-1} (S)
    CentSet eye, spec;       // the same centroids with their group search
    int n_eye, n_spec;
    // this iteration's bucketing of the final candidates
    const int *s_count, *s_off, *s_list, *nonempty;
    const int *n_nonempty;
    // alias rows over the non-empty subspaces, and the row normalisers
    const float *al_prob;    // [n_eye * n_spec]
    const int *al_idx;       // [n_eye * n_spec]
    const float *row_sum;    // [n_eye] sum of Gamma over non-empty S (0 = uniform row)
    const float *al_pmf;     // [n_eye * n_spec] probability the alias row draws S (non-empty S only)
    const float *gamma;      // [n_eye * n_spec] frozen Gamma of this iteration
    float defensive;
    // control subspaces C of the incomplete sub-paths' control vertices (class B: y_0 on an
    // emitter; class A has none and takes C = 0), Section 5.5
    const float *ctrl_c;     // [n_ctrl * FEAT]
    int n_ctrl;
    // frozen reciprocal statistics per (class, u, S, C): sum R, sum R^2 / rho, count; and the
    // bucket's f/q samples: largest value (a floor of its B), sum, count (its mean estimates beta)
    const float *rstat;      // [PT_STAT_CU * n_ctrl * n_spec * 3]
    const float *bstat;      // [PT_STAT_CU * n_ctrl * n_spec * 3]
    // the previous iteration's candidate counts (n_cand, n_final, non-empty subspaces), its
    // per-subspace counts and the frozen Gamma row totals: the MIS surrogate's inputs, none of
    // which depends on this iteration's light paths
    const float *prev;       // [3]
    const int *s_count_prev; // [n_spec]
    const float *row_tot;    // [n_eye]
    // tiles
    const float *tile_proxy, *tile_total;
    int tile, tiles_x;
    float tile_thr, tile_low;
};

__device__ __forceinline__ void feat9(const SceneDev &S, float3 p, float3 n, float3 w, float f[9])
{
    f[0] = (p.x - S.lo.x) * S.inv_ext.x; f[1] = (p.y - S.lo.y) * S.inv_ext.y; f[2] = (p.z - S.lo.z) * S.inv_ext.z;
    f[3] = n.x; f[4] = n.y; f[5] = n.z;
    f[6] = w.x; f[7] = w.y; f[8] = w.z;
}
__device__ __forceinline__ int nearest(const float *__restrict__ cent, int K, const float f[9])
{
    int best = 0;
    float bd = 3.0e38f;
    for (int k = 0; k < K; ++k) {
        const float4 a = *(const float4 *)(cent + FEAT * k), b = *(const float4 *)(cent + FEAT * k + 4),
                     c = *(const float4 *)(cent + FEAT * k + 8);
        const float d0 = a.x - f[0], d1 = a.y - f[1], d2 = a.z - f[2], d3 = a.w - f[3], d4 = b.x - f[4],
                    d5 = b.y - f[5], d6 = b.z - f[6], d7 = b.w - f[7], d8 = c.x - f[8];
        const float d = d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3 + d4 * d4 + d5 * d5 + d6 * d6 + d7 * d7 + d8 * d8;
        if (d < bd) { bd = d; best = k; }
    }
    return best;
}

__device__ __forceinline__ int nearest_set(const CentSet &C, const float f[9])
{
    if (C.G <= 0) return nearest(C.c, C.K, f);
    const int g = nearest(C.g, C.G, f);
    const int a = C.start[g], b = C.start[g + 1];
    if (a >= b) return nearest(C.c, C.K, f);
    int best = C.mem[a];
    float bd = 3.0e38f;
    for (int i = a; i < b; ++i) {
        const int k = C.mem[i];
        const float d = feat_d2(C.c + FEAT * k, f);
        if (d < bd) { bd = d; best = k; }
    }
    return best;
}

// octahedral encoding of a unit vector into two floats
__device__ __forceinline__ float2 oct_enc(float3 v)
{
    const float s = fabsf(v.x) + fabsf(v.y) + fabsf(v.z);
    float x = v.x / s, y = v.y / s;
    if (v.z < 0.0f) {
        const float ox = (1.0f - fabsf(y)) * copysignf(1.0f, x), oy = (1.0f - fabsf(x)) * copysignf(1.0f, y);
        x = ox; y = oy;
    }
    return make_float2(x, y);
}
__device__ __forceinline__ float3 oct_dec(float2 e)
{
    float3 v = f3(e.x, e.y, 1.0f - fabsf(e.x) - fabsf(e.y));
    if (v.z < 0.0f) {
        const float ox = (1.0f - fabsf(v.y)) * copysignf(1.0f, v.x), oy = (1.0f - fabsf(v.x)) * copysignf(1.0f, v.y);
        v.x = ox; v.y = oy;
    }
    return normalize3(v);
}

// ------------------------------------------------------------------------------ k-means
__global__ void k_km_init(const float *feat, int n, float *cent, int K)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const int src = n > 0 ? (int)(((long)k * n) / K) : -1;
    for (int j = 0; j < FEAT; ++j) cent[FEAT * k + j] = src >= 0 ? feat[FEAT * (size_t)src + j] : 0.0f;
}
__global__ void k_km_assign(const float *feat, int n, const float *cent, int K, float *sums, float *counts)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float f[9];
    for (int j = 0; j < 9; ++j) f[j] = feat[FEAT * (size_t)i + j];
    const int k = nearest(cent, K, f);
    for (int j = 0; j < 9; ++j) unsafeAtomicAdd(sums + FEAT * k + j, f[j]);
    unsafeAtomicAdd(counts + k, 1.0f);
}
__global__ void k_km_update(float *cent, const float *sums, const float *counts, int K)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K || counts[k] <= 0.0f) return;
    for (int j = 0; j < 9; ++j) cent[FEAT * k + j] = sums[FEAT * k + j] / counts[k];
}

// ------------------------------------------------------------------------------ bucketing
// control subspace of a control vertex y_0 on emitter triangle t0 (features: position, normal and
// no direction, since the control vertex of class B carries no direction); 0 with one subspace
__device__ __forceinline__ int ctrl_label(const SceneDev &S, const SubDev &D, float3 y0, int t0)
{
    if (D.n_ctrl <= 1) return 0;
    float f[9];
    feat9(S, y0, S.shade[t0].n, f3(0.f, 0.f, 0.f), f);
    return nearest(D.ctrl_c, D.n_ctrl, f);
}
// bucket of the (class, u, S, C) statistics
__device__ __forceinline__ int stat_bucket(const SubDev &D, int cls, int u, int S, int C)
{
    return ((cls * 5 + u) * D.n_ctrl + C) * D.n_spec + S;
}
// labels of the kept candidates, before their reciprocal estimates: specular subspace S of
// y_{s-1} (with its incident direction) and control subspace C, as spec_sub = S | C << 16
__global__ void k_label_kept(SceneDev S, SubDev D, Cand *cand, const uint32_t *kept, const unsigned long long *cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int)cnt[C_NKEPT]) return;
    Cand &c = cand[kept[i]];
    float f[9];
    feat9(S, xyz(c.v), S.shade[__float_as_int(c.v.w)].n, oct_dec(make_float2(c.pad[0], c.pad[1])), f);
    const int s = nearest_set(D.spec, f);
    const int C = cand_cls(c.cls_u) ? ctrl_label(S, D, xyz(c.hc), __float_as_int(c.hc.w)) : 0;
    c.spec_sub = s | (C << 16);
}
// bucket sizes of the final candidates by S
__global__ void k_count_sub(const Cand *cand, const uint32_t *final_, const unsigned long long *cnt, int *s_count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int)cnt[C_NFINAL]) return;
    atomicAdd(s_count + (cand[final_[i]].spec_sub & 0xFFFF), 1);
}
// one workgroup: exclusive scan of the counts and the list of non-empty subspaces
__global__ void k_scan_sub(const int *s_count, int *s_off, int *s_fill, int *nonempty, int *n_nonempty, int K)
{
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int per = (K + blockDim.x - 1) / blockDim.x;
    int acc = 0;
    for (int j = t * per; j < min(K, (t + 1) * per); ++j) acc += s_count[j];
    part[t] = acc;
    __syncthreads();
    if (t == 0) {
        int run = 0, ne = 0;
        for (int b = 0; b < (int)blockDim.x; ++b) { const int v = part[b]; part[b] = run; run += v; }
        for (int j = 0; j < K; ++j) if (s_count[j] > 0) nonempty[ne++] = j;
        *n_nonempty = ne;
    }
    __syncthreads();
    int run = part[t];
    for (int j = t * per; j < min(K, (t + 1) * per); ++j) { s_off[j] = run; s_fill[j] = run; run += s_count[j]; }
}
__global__ void k_scatter_sub(const Cand *cand, const uint32_t *final_, const unsigned long long *cnt, int *s_fill,
                              int *s_list)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int)cnt[C_NFINAL]) return;
    const int s = cand[final_[i]].spec_sub & 0xFFFF;
    s_list[atomicAdd(s_fill + s, 1)] = (int)final_[i];
}

// Walker alias draw over the ne columns of a row: column index_of(x, ne), kept when the 24-bit
// uniform u lies below its probability, else its alias
__device__ __forceinline__ int alias_draw(const float *pr, const int *ai, int ne, uint32_t x, float u)
{
    const int c = index_of(x, ne);
    return u < pr[c] ? c : ai[c];
}
// The probabilities with which alias_draw returns each column, from the table as stored: column
// c is drawn with index_prob(c, ne) and kept with below_prob(pr[c]), else it gives ai[c]. These
// are the selection probabilities the estimators divide by, so that the FP32 rounding of the
// construction changes the sampling density and never the expectation. pm[ne] (double).
__device__ __forceinline__ void alias_pmf(const float *pr, const int *ai, int ne, double *pm)
{
    for (int j = 0; j < ne; ++j) pm[j] = 0.0;
    for (int c = 0; c < ne; ++c) {
        const double w = index_prob(c, ne), st = below_prob(pr[c]);
        pm[c] += w * st;
        pm[ai[c]] += w * (1.0 - st);
    }
}

// Gamma row T -> alias table over the non-empty subspaces (Vose's construction, one thread per
// row, worklists in global scratch). Row probabilities: (1 - defensive) Gamma[T, S] / sum over
// non-empty S + defensive / n_nonempty, or uniform when the row has no data. pmf[T, S] receives
// the probability the stored table realises for every non-empty S.
__global__ void k_alias_rows(const float *gamma, int n_eye, int n_spec, const int *nonempty, const int *n_nonempty,
                             float defensive, float *al_prob, int *al_idx, float *row_sum, float *pmf, int *scratch)
{
    const int T = blockIdx.x * blockDim.x + threadIdx.x;
    if (T >= n_eye) return;
    const int ne = *n_nonempty;
    const float *g = gamma + (size_t)T * n_spec;
    float rs = 0.0f;
    for (int j = 0; j < ne; ++j) rs += g[nonempty[j]];
    row_sum[T] = rs;
    if (ne == 0) return;
    float *pr = al_prob + (size_t)T * n_spec;
    int *ai = al_idx + (size_t)T * n_spec;
    int *small = scratch + (size_t)T * 2 * n_spec, *large = small + n_spec;
    int ns = 0, nl = 0;
    for (int j = 0; j < ne; ++j) {
        const float p = rs > 0.0f ? (1.0f - defensive) * g[nonempty[j]] / rs + defensive / ne : 1.0f / ne;
        pr[j] = p * ne;
        if (pr[j] < 1.0f) small[ns++] = j; else large[nl++] = j;
    }
    while (ns > 0 && nl > 0) {
        const int l = small[--ns], gg = large[--nl];
        ai[l] = gg;
        pr[gg] = (pr[gg] + pr[l]) - 1.0f;
        if (pr[gg] < 1.0f) small[ns++] = gg; else large[nl++] = gg;
    }
    while (nl > 0) { const int gg = large[--nl]; pr[gg] = 1.0f; ai[gg] = gg; }
    while (ns > 0) { const int l = small[--ns]; pr[l] = 1.0f; ai[l] = l; }
    // the worklists are free now: the realised probabilities in their place
    double *pm = (double *)small;
    alias_pmf(pr, ai, ne, pm);
    float *po = pmf + (size_t)T * n_spec;
    for (int j = 0; j < ne; ++j) po[nonempty[j]] = (float)pm[j];
}
// The same tables with one wavefront per row: the row's probabilities and Vose's worklists in LDS
// (16 bytes per column, dynamic), the sums and probabilities formed by the 64 lanes, the
// sequential construction by lane 0 on LDS. Same output as k_alias_rows.
#define ALIAS_LDS_COLS 2048
__global__ void __launch_bounds__(64) k_alias_rows_wave(const float *gamma, int n_eye, int n_spec, const int *nonempty,
                                                        const int *n_nonempty, float defensive, float *al_prob,
                                                        int *al_idx, float *row_sum, float *pmf)
{
    extern __shared__ float alias_sh[];
    const int T = blockIdx.x, lane = threadIdx.x;
    if (T >= n_eye) return;   // block-uniform
    const int ne = *n_nonempty;
    const float *g = gamma + (size_t)T * n_spec;
    float rs = 0.0f;
    for (int j = lane; j < ne; j += 64) rs += g[nonempty[j]];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) rs += __shfl_xor(rs, off);
    if (lane == 0) row_sum[T] = rs;
    if (ne == 0) return;
    float *pr = alias_sh;
    int *ai = (int *)(pr + n_spec), *small = ai + n_spec, *large = small + n_spec;
    for (int j = lane; j < ne; j += 64) {
        const float p = rs > 0.0f ? (1.0f - defensive) * g[nonempty[j]] / rs + defensive / ne : 1.0f / ne;
        pr[j] = p * ne;
    }
    __syncthreads();
    // the worklists (8 bytes per column from byte offset 8 n_spec) hold the realised
    // probabilities once the construction is done
    double *pm = (double *)small;
    if (lane == 0) {
        int ns = 0, nl = 0;
        for (int j = 0; j < ne; ++j) {
            if (pr[j] < 1.0f) small[ns++] = j; else large[nl++] = j;
        }
        while (ns > 0 && nl > 0) {
            const int l = small[--ns], gg = large[--nl];
            ai[l] = gg;
            pr[gg] = (pr[gg] + pr[l]) - 1.0f;
            if (pr[gg] < 1.0f) small[ns++] = gg; else large[nl++] = gg;
        }
        while (nl > 0) { const int gg = large[--nl]; pr[gg] = 1.0f; ai[gg] = gg; }
        while (ns > 0) { const int l = small[--ns]; pr[l] = 1.0f; ai[l] = l; }
        alias_pmf(pr, ai, ne, pm);
    }
    __syncthreads();
    float *po = al_prob + (size_t)T * n_spec;
    int *io = al_idx + (size_t)T * n_spec;
    float *qo = pmf + (size_t)T * n_spec;
    for (int j = lane; j < ne; j += 64) { po[j] = pr[j]; io[j] = ai[j]; qo[nonempty[j]] = (float)pm[j]; }
}

// selection probability of subspace S from eye subspace T: what the alias row realises
__device__ __forceinline__ float sel_prob(const SubDev &D, int T, int S)
{
    const int ne = *D.n_nonempty;
    if (ne == 0 || D.s_count[S] == 0) return 0.0f;
    return D.al_pmf[(size_t)T * D.n_spec + S];
}

// selection probability of S from T under the frozen Gamma row (defensive mixture over the
// previous iteration's non-empty subspaces): the surrogate the MIS weights use
__device__ __forceinline__ float sel_prob_frozen(const SubDev &D, int T, int S)
{
    const float ne = fmaxf(D.prev[2], 1.0f);
    const float rt = D.row_tot[T];
    return rt > 0.0f ? (1.0f - D.defensive) * D.gamma[(size_t)T * D.n_spec + S] / rt + D.defensive / ne : 1.0f / ne;
}
__global__ void k_row_tot(const float *gamma, int n_eye, int n_spec, float *row_tot)
{
    const int T = blockIdx.x * blockDim.x + threadIdx.x;
    if (T >= n_eye) return;
    float a = 0.0f;
    for (int j = 0; j < n_spec; ++j) a += gamma[(size_t)T * n_spec + j];
    row_tot[T] = a;
}
// end of an iteration: its counts become the next iteration's frozen inputs
__global__ void k_prev_store(const unsigned long long *cnt, const int *s_count, const int *n_ne, int n_spec,
                             float *prev, int *s_count_prev)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_spec) s_count_prev[i] = s_count[i];
    if (i == 0) {
        prev[0] = (float)cnt[C_NCAND];
        prev[1] = (float)cnt[C_NFINAL];
        prev[2] = cnt[C_NFINAL] > 0 ? (float)*n_ne : 0.0f;
    }
}

// reciprocal statistics of the final candidates by (class, u, S, C) (accumulated for later
// iterations), and the bucket's f/q samples: largest value (the candidates' pilot and chain
// maxima), sum and count of every f/q the pilot and the first chain stage drew
__global__ void k_rstat(const Cand *cand, const uint32_t *final_, const unsigned long long *cnt, int repeats, SubDev D,
                        float *rstat_acc, float *bstat_acc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int)cnt[C_NFINAL] || !cnt[C_LEARN]) return;
    const Cand &c = cand[final_[i]];
    const float R = c.recip_sum / (float)repeats;
    const int b = stat_bucket(D, cand_cls(c.cls_u), cand_u(c.cls_u), c.spec_sub & 0xFFFF, c.spec_sub >> 16);
    // the second moment of the unbiased factor R 1{kept} / rho is E[R^2] / rho
    unsafeAtomicAdd(rstat_acc + 3 * b + 0, R);
    unsafeAtomicAdd(rstat_acc + 3 * b + 1, R * R / fmaxf(c.rho, 1e-6f));
    unsafeAtomicAdd(rstat_acc + 3 * b + 2, 1.0f);
    if (c.pmax > 0.0f) atomicMax((int *)(bstat_acc + 3 * b), __float_as_int(c.pmax));
    unsafeAtomicAdd(bstat_acc + 3 * b + 1, c.psum);
    unsafeAtomicAdd(bstat_acc + 3 * b + 2, c.pn);
}

// Surrogate of the proxy strategy's density factor for MIS (Section 5.4, equ:MIS_1 with
// E[1/p~^2] p = (1 + V_rel) / p): K' P^ / (1 + V_rel), with P^ = 1 / mean R and V_rel the
// relative variance of R 1{kept} / rho (second moment E[R^2 / rho]) in the (class, u, S, C) bucket
// of Section 5.5 from earlier iterations, K' = M pi_inc c pi_sel.
__device__ __forceinline__ float proxy_mis_factor(const SubDev &D, int cls, int u, int S, int C, float k_sel)
{
    const int b = stat_bucket(D, cls, u, S, C);
    const float n = D.rstat[3 * b + 2];
    if (!(n > 0.0f) || !(k_sel > 0.0f)) return 0.0f;
    const float m = D.rstat[3 * b + 0] / n, m2 = D.rstat[3 * b + 1] / n;
    if (!(m > 0.0f)) return 0.0f;
    const float vrel = fmaxf(0.0f, m2 / (m * m) - 1.0f);
    return k_sel / (m * (1.0f + vrel));
}
// tile attempt probability c (Section 6.1): 1 when the proxy's share of the tile's contribution
// (previous iterations) exceeds the threshold or nothing is known yet, else the low probability
__device__ __forceinline__ float tile_prob(const SubDev &D, int pix, int W)
{
    if (D.tile <= 0) return 1.0f;
    const int t = (pix / W) / D.tile * D.tiles_x + (pix % W) / D.tile;
    const float tot = D.tile_total[t];
    if (!(tot > 0.0f)) return 1.0f;
    return D.tile_proxy[t] > D.tile_thr * tot ? 1.0f : D.tile_low;
}
