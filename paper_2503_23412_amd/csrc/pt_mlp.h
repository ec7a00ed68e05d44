// Learned proposal for the selection of incomplete sub-paths: an MLP maps the features of the
// eye's first diffuse vertex (9-D: position in the scene box, normal, direction toward the
// previous eye vertex; 12-band sin/cos encoding + raw = 225, padded to 256) through three
// hidden layers of 64 ReLU units to one logit per specular subspace. The proxy strategy picks
// S from 0.9 softmax(logits over the non-empty subspaces) + 0.1 plain row (defensive), so every
// selection probability stays positive and exactly known. It is trained online on the proxy
// contributions of earlier iterations (contribution-weighted cross entropy) with Adam.
//
// The dense layers run on MFMA: v_mfma_f32_16x16x32_bf16, BF16 operands, FP32 accumulation.
#pragma once
#include "pt_subspace.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

#define MLP_IN 256
#define MLP_H 64
#define MLP_BANDS 12

__device__ __forceinline__ uint16_t f2bf(float f)
{
    // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(u >> 16);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// encode features into row `row` of X (bf16, MLP_IN wide)
__device__ __forceinline__ void mlp_encode(const float f[9], uint16_t *X)
{
    int o = 0;
    for (int j = 0; j < 9; ++j) {
        X[o++] = f2bf(f[j]);
        float s = f[j] * PT_PI;
        for (int b = 0; b < MLP_BANDS; ++b) {
            float sn, cs;
            sincosf(s, &sn, &cs);   // accurate form: the top band's argument reaches 2^11 pi
            X[o++] = f2bf(sn);
            X[o++] = f2bf(cs);
            s *= 2.0f;
        }
    }
    while (o < MLP_IN) X[o++] = 0;
}

// C (+)= A B with A(m, k) = A[m*sam + k*sak], B(k, n) = B[k*sbk + n*sbn] (bf16), C(m, n) =
// C[m*scm + n] (fp32). One wavefront per 16 x 16 tile of C; K is split over gridDim.z with
// atomic accumulation when splits > 1. Rows m >= *m_count (device count) are skipped when
// m_count is given. Lane l of the 16x16x32 MFMA holds A[l%16][8(l/16) .. +7],
// B[8(l/16) .. +7][l%16] and returns C[4(l/16) .. +3][l%16].
__global__ void k_gemm(int M, int N, int K, const uint16_t *__restrict__ A, int sam, int sak,
                       const uint16_t *__restrict__ B, int sbk, int sbn, float *C, int scm, int accumulate,
                       const unsigned long long *cnt, int m_cidx, int k_cidx)
{
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int tiles_n = (N + 15) >> 4;
    const int tm = wave / tiles_n, tn = wave % tiles_n;
    const int Mv = m_cidx >= 0 ? min(M, (int)cnt[m_cidx]) : M;
    if (k_cidx >= 0) K = min(K, (int)cnt[k_cidx]);
    if (tm * 16 >= Mv) return;   // wave-uniform
    const int ksplit = gridDim.z, kz = blockIdx.z;
    const int kchunk = ((K + 31) / 32 + ksplit - 1) / ksplit * 32;
    const int k_begin = kz * kchunk, k_end = min(K, k_begin + kchunk);
    const int r = lane & 15, g = lane >> 4;
    const int am = tm * 16 + r, bn = tn * 16 + r;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = k_begin; k0 < k_end; k0 += 32) {
        bf16x8 a, b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = k0 + 8 * g + j;
            const uint16_t av = (am < Mv && k < K) ? A[(size_t)am * sam + (size_t)k * sak] : (uint16_t)0;
            const uint16_t bv = (bn < N && k < K) ? B[(size_t)k * sbk + (size_t)bn * sbn] : (uint16_t)0;
            a[j] = __builtin_bit_cast(__bf16, av);
            b[j] = __builtin_bit_cast(__bf16, bv);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int m = tm * 16 + 4 * g + j, n = tn * 16 + r;
        if (m < Mv && n < N) {
            float *p = C + (size_t)m * scm + n;
            if (ksplit > 1) { if (acc[j] != 0.0f) unsafeAtomicAdd(p, acc[j]); }
            else *p = accumulate ? *p + acc[j] : acc[j];
        }
    }
}

// H = relu(Z + b) as bf16, rows < count
__global__ void k_bias_relu(const float *Z, const float *bias, uint16_t *H, int M, int N,
                            const unsigned long long *cnt, int m_cidx)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int Mv = m_cidx >= 0 ? min(M, (int)cnt[m_cidx]) : M;
    if (i >= (size_t)Mv * N) return;
    H[i] = f2bf(fmaxf(Z[i] + bias[i % N], 0.0f));
}

// softmax cross entropy gradient of weighted samples: G = w_i (softmax(L_i + b) - onehot(S_i))
// / sum w (bf16), over all n_out logits (one 256-thread block per row)
__global__ void k_ce_grad(const float *L, const float *bias, const int *label, const float *weight,
                          const float *wsum, int M, int N, uint16_t *G, const unsigned long long *cnt, int m_cidx)
{
    const int row = blockIdx.x;
    const int Mv = m_cidx >= 0 ? min(M, (int)cnt[m_cidx]) : M;
    if (row >= Mv) return;
    const float wsum_inv = *wsum > 0.0f ? 1.0f / *wsum : 0.0f;
    __shared__ float red[256];
    const float *l = L + (size_t)row * N;
    float mx = -3.0e38f;
    for (int j = threadIdx.x; j < N; j += blockDim.x) mx = fmaxf(mx, l[j] + bias[j]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    mx = red[0];
    __syncthreads();
    float sm = 0.f;
    for (int j = threadIdx.x; j < N; j += blockDim.x) sm += __expf(l[j] + bias[j] - mx);
    red[threadIdx.x] = sm;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const float inv = 1.0f / red[0];
    const float w = weight[row] * wsum_inv;
    const int lab = label[row];
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
        const float gj = w * (__expf(l[j] + bias[j] - mx) * inv - (j == lab ? 1.0f : 0.0f));
        G[(size_t)row * N + j] = f2bf(gj);
    }
}

// dZ = dH * (H > 0) as bf16
__global__ void k_relu_back(const float *dH, const uint16_t *H, uint16_t *dZ, int M, int N,
                            const unsigned long long *cnt, int m_cidx)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int Mv = m_cidx >= 0 ? min(M, (int)cnt[m_cidx]) : M;
    if (i >= (size_t)Mv * N) return;
    dZ[i] = f2bf(bf2f(H[i]) > 0.0f ? dH[i] : 0.0f);
}

// db[n] += sum over rows of G[m][n] (bf16): each thread sums one column over a strip of
// MLP_STRIP rows, then one atomic per (strip, column)
#define MLP_STRIP 256
__global__ void k_colsum(const uint16_t *G, int M, int N, float *db, const unsigned long long *cnt, int m_cidx)
{
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int Mv = m_cidx >= 0 ? min(M, (int)cnt[m_cidx]) : M;
    const int r0 = blockIdx.y * MLP_STRIP;
    if (col >= N || r0 >= Mv) return;
    const int r1 = min(Mv, r0 + MLP_STRIP);
    float s = 0.0f;
    for (int r = r0; r < r1; ++r) s += bf2f(G[(size_t)r * N + col]);
    if (s != 0.0f) unsafeAtomicAdd(db + col, s);
}

// Adam (Kingma and Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, w -= lr mhat / (sqrt(vhat) + eps)
// with the bias corrections of step t = cnt[C_MLP_T] + 1; refreshes the bf16 copy and clears the
// gradient. Runs only when this iteration recorded training samples.
__global__ void k_adam(float *w, uint16_t *wb, float *g, float *m, float *v, int n, float lr, float b1, float b2,
                       float eps, const unsigned long long *cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || cnt[C_MLP_N] == 0) return;
    const float t = (float)(cnt[C_MLP_T] + 1ull);
    const float bc1 = 1.0f - powf(b1, t), bc2 = 1.0f - powf(b2, t);
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi, vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi; v[i] = vi;
    const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    w[i] = wi;
    if (wb) wb[i] = f2bf(wi);
    g[i] = 0.0f;
}

// Adam step counter, after k_adam
__global__ void k_mlp_tick(unsigned long long *cnt)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && cnt[C_MLP_N] != 0) cnt[C_MLP_T] += 1ull;
}

// He-uniform weights, zero biases (output layer scaled by 0.1 so the first softmax is near
// uniform); Adam moments and gradients cleared
__global__ void k_mlp_init(float *w, uint16_t *wb, float *g, float *m, float *v, int n_out, uint32_t seed)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int sz[8] = {MLP_IN * MLP_H, MLP_H, MLP_H * MLP_H, MLP_H, MLP_H * MLP_H, MLP_H, MLP_H * n_out, n_out};
    const int fan[4] = {225, MLP_H, MLP_H, MLP_H};
    int off = 0, seg = 0;
    while (seg < 8 && i >= off + sz[seg]) off += sz[seg++];
    if (seg >= 8) return;
    float x = 0.0f;
    if ((seg & 1) == 0) {
        Rng r = rng_make(seed, S_MLP, (uint32_t)i, 0u, 0u);
        const float a = sqrtf(6.0f / (float)fan[seg >> 1]) * (seg == 6 ? 0.1f : 1.0f);
        x = (2.0f * rng_f(r) - 1.0f) * a;
        // rows of W1 beyond the 225 encoded inputs only ever see zeros
        if (seg == 0 && (i - off) / MLP_H >= 225) x = 0.0f;
    }
    w[i] = x; wb[i] = f2bf(x); g[i] = 0.0f; m[i] = 0.0f; v[i] = 0.0f;
}

// features of the proxy items' first diffuse vertices -> encoded rows of X
__global__ void k_mlp_enc_items(SceneDev S, const ProxyItem *items, const unsigned long long *cnt, uint16_t *X)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int)cnt[C_PROXYQ]) return;
    const ProxyItem &p = items[i];
    float f[9];
    feat9(S, xyz(p.x), S.shade[__float_as_int(p.x.w)].n, xyz(p.wo), f);
    mlp_encode(f, X + (size_t)i * MLP_IN);
}
// training features (n x 9, fp32) -> encoded rows
__global__ void k_mlp_enc_feat(const float *feat, int n, const unsigned long long *cnt, int m_cidx, uint16_t *X)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nv = m_cidx >= 0 ? min(n, (int)cnt[m_cidx]) : n;
    if (i >= nv) return;
    float f[9];
    for (int j = 0; j < 9; ++j) f[j] = feat[9 * (size_t)i + j];
    mlp_encode(f, X + (size_t)i * MLP_IN);
}
// logits + bias as fp32 output (for the forward hook)
__global__ void k_add_bias(float *L, const float *bias, int M, int N)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (size_t)M * N) L[i] += bias[i % N];
}

// Selection of the specular subspace for every proxy item: with probability `mix` from the
// network's softmax restricted to the non-empty subspaces (inverse CDF), otherwise from the
// plain row (Gamma alias row, or uniform over the non-empty subspaces). The probability of
// the chosen S under the mixture is written with it: aux.z = S (bits), aux.w = pi_S.
__global__ void k_mlp_select(EyeBuf E, SubDev D, const float *L, const float *bias, int n_out, float mix, int gamma_on,
                             uint32_t seed, const unsigned long long *cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int)cnt[C_PROXYQ]) return;
    ProxyItem &it = E.proxy[i];
    // the subspace lists are rebuilt only in iterations that keep candidates
    const int ne = cnt[C_NFINAL] > 0 ? min(*D.n_nonempty, D.n_spec) : 0;
    if (ne <= 0) { it.aux.z = __int_as_float(-1); it.aux.w = 0.0f; return; }
    const int T = __float_as_int(it.aux.x);
    const float *l = L + (size_t)i * n_out;
    Rng r = rng_make(seed, S_MLP, (uint32_t)__float_as_int(it.beta.w), (uint32_t)cnt[C_ITER], 1u);
    float mx = -3.0e38f;
    for (int j = 0; j < ne; ++j) mx = fmaxf(mx, l[D.nonempty[j]] + bias[D.nonempty[j]]);
    // softmax terms summed in double: the inverse CDF below, with a 53-bit uniform, then draws
    // S = nonempty[j] with probability e_j / sum to within 2^-52, the probability written out
    double sum = 0.0;
    for (int j = 0; j < ne; ++j) sum += (double)__expf(l[D.nonempty[j]] + bias[D.nonempty[j]] - mx);
    const float u0 = rng_f(r);
    const uint32_t xa = rng_u32(r), xb = rng_u32(r);
    int S;
    if (u0 < mix) {
        const double u = (double)(((uint64_t)xa << 21) | (uint64_t)(xb >> 11)) * (1.0 / 9007199254740992.0);
        const double target = u * sum;
        double c = 0.0;
        S = -1;
        for (int j = 0; j < ne; ++j) {
            const double e = (double)__expf(l[D.nonempty[j]] + bias[D.nonempty[j]] - mx);
            c += e;
            if (e > 0.0) S = D.nonempty[j];
            if (target < c) break;
        }
    } else if (gamma_on) {
        const size_t row = (size_t)T * D.n_spec;
        S = D.nonempty[alias_draw(D.al_prob + row, D.al_idx + row, ne, xa, (float)(xb >> 8) * (1.0f / 16777216.0f))];
    } else {
        S = D.nonempty[index_of(xa, ne)];
    }
    const double learned = (double)__expf(l[S] + bias[S] - mx) / sum;
    double plain;
    if (gamma_on) {
        plain = (double)sel_prob(D, T, S);
    } else {
        int j = 0;
        while (j < ne && D.nonempty[j] != S) ++j;
        plain = index_prob(j, ne);
    }
    // the mixture weight the 24-bit draw u0 < mix realises
    const double m = below_prob(mix);
    it.aux.z = __int_as_float(S);
    it.aux.w = (float)(m * learned + (1.0 - m) * plain);
}

// One training sample per valid proxy contribution of a learning iteration: the features of the
// first diffuse eye vertex, the selected subspace and the contribution's luminance as weight.
struct MlpTrain {
    float *feat;     // [cap x 9]
    int *label;      // [cap]
    float *weight;   // [cap]
    float *wsum;     // [1]
    int cap;
};
__device__ __forceinline__ void mlp_record(const SceneDev &S, const MlpTrain &T, unsigned long long *cnt, float3 x,
                                           float3 n, float3 wo, int Ssel, float w)
{
    const int slot = (int)atomicAdd(cnt + C_MLP_N, 1ull);
    if (slot >= T.cap) return;
    float f[9];
    feat9(S, x, n, wo, f);
    for (int j = 0; j < 9; ++j) T.feat[9 * (size_t)slot + j] = f[j];
    T.label[slot] = Ssel;
    T.weight[slot] = w;
    unsafeAtomicAdd(T.wsum, w);
}
