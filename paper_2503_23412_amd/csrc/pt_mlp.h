// Learned proposal of the proxy strategy: an MLP maps 9 features of a vertex (position in the
// scene box, normal, direction toward the previous vertex of the eye side; 12-band sin/cos
// encoding + raw = 225, padded to 256) through three hidden layers of 64 ReLU units to n_spec
// subspace logits followed by an 8-lobe von Mises-Fisher mixture over directions (5 outputs per
// lobe: mean direction, log concentration, mixture logit).
//  * Queried at the eye's first diffuse vertex, the logits pick the specular subspace S from
//    mix softmax(logits over the non-empty subspaces) + (1 - mix) plain row (defensive).
//  * Queried at the chosen incomplete sub-path's y_{s-1} (direction toward z_d), the mixture
//    proposes the first retrace direction at a glossy (non-Dirac) y_{s-1}: mix vMF mixture +
//    (1 - mix) BSDF sampling, with the mixture density in the retrace pdf.
// Every probability stays positive wherever the plain sampling's does and is exactly known, so
// the estimator stays unbiased. Both heads train online on the proxy contributions of the
// iterations (contribution-weighted cross entropy and negative log-likelihood) with Adam.
//
// The dense layers run on MFMA: v_mfma_f32_16x16x32_bf16, BF16 operands, FP32 accumulation.
#pragma once
#include "pt_subspace.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

#define MLP_IN 256
#define MLP_H 64
#define MLP_BANDS 12
#define MLP_LOBES 8
#define MLP_VMF (5 * MLP_LOBES)
#define VMF_LOGK_MIN (-3.0f)
#define VMF_LOGK_MAX 10.0f

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

// Transposed BF16 copies of the four weight matrices for the fused forward pass: for layer l with
// W_l[K][N] (row-major at offset off_l of the parameter vector), Wt_l[n][k] = W_l[k][n] at the same
// offset of wt, so that one lane's 8 consecutive k of a column are one 16-byte load.
__global__ void k_mlp_transpose(const uint16_t *wb, uint16_t *wt, int nout, size_t oW1, size_t oW2, size_t oW3,
                                size_t oW4)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n1 = (size_t)MLP_IN * MLP_H, n2 = (size_t)MLP_H * MLP_H, n4 = (size_t)MLP_H * nout;
    size_t off, K, N, j;
    if (i < n1) { off = oW1; K = MLP_IN; N = MLP_H; j = i; }
    else if (i < n1 + n2) { off = oW2; K = MLP_H; N = MLP_H; j = i - n1; }
    else if (i < n1 + 2 * n2) { off = oW3; K = MLP_H; N = MLP_H; j = i - n1 - n2; }
    else if (i < n1 + 2 * n2 + n4) { off = oW4; K = MLP_H; N = (size_t)nout; j = i - n1 - 2 * n2; }
    else return;
    const size_t k = j / N, n = j % N;
    wt[off + n * K + k] = wb[off + j];
}

// Fused forward pass of the whole network on MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulation)
// over one chunk of rows (rows off .. off + M - 1 of the queue, at X row 0):
// one workgroup of four wavefronts per 64-row tile (a persistent loop over tiles), each wavefront a
// strip of 16 rows through all four layers. Lane (r, g) = (lane % 16, lane / 16) feeds row r's
// inputs 8 g .. 8 g + 7 of each 32-wide k step (one 16-byte load) and column r's weights
// (16-byte loads from the transposed copies, which every tile rereads from the caches); hidden
// activations (bias, ReLU, BF16) go through a per-wavefront LDS strip that turns the MFMA's output
// layout (rows 4 g .. 4 g + 3 of column r) into the next layer's input layout. Writes the outputs
// col0 .. col0 + ncols - 1 of rows < min(M, cnt[m_cidx]) (or M) to out (row stride ncols), with
// bias_out[col] added when given; keep_h: the hidden activations also go to H1..H3 (row stride 64)
// for the backward pass.
#define MLP_FT_ROWS 64
#define MLP_STRIP_LD (MLP_H + 8)   // padded LDS row (144 bytes): 16-byte lane reads fall in distinct banks
__device__ __forceinline__ bf16x8 ld8(const uint16_t *p)
{
    return __builtin_bit_cast(bf16x8, *(const uint4 *)p);
}
// one hidden layer for the wavefront's 16 rows: inputs from X (layer 1) or from the LDS strip,
// 64 outputs in four 16 x 16 MFMA tiles, then bias, ReLU and BF16 back into the strip (and to H)
template <int K, bool FROM_X, bool KEEP_H>
__device__ __forceinline__ void mlp_fwd_layer(const uint16_t *__restrict__ X, int row0, int Mv,
                                              const uint16_t *__restrict__ Wt, const float *__restrict__ bias,
                                              uint16_t *hs, uint16_t *H, int r, int g)
{
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // two k steps in flight: enough loads to cover the latency without holding every step's
    // fragments in registers
#pragma unroll 2
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 a;
        if (FROM_X) {
            const int row = row0 + r;
            a = row < Mv ? ld8(X + (size_t)row * MLP_IN + k0 + 8 * g) : bf16x8{};
        } else {
            a = ld8(hs + r * MLP_STRIP_LD + k0 + 8 * g);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const bf16x8 b = ld8(Wt + (size_t)(t * 16 + r) * K + k0 + 8 * g);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
        }
    }
    __syncthreads();   // every lane's reads of the strip precede its overwrite
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float b = bias[t * 16 + r];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint16_t h = f2bf(fmaxf(acc[t][j] + b, 0.0f));
            hs[(4 * g + j) * MLP_STRIP_LD + t * 16 + r] = h;
            const int m = row0 + 4 * g + j;
            if (KEEP_H && m < Mv) H[(size_t)m * MLP_H + t * 16 + r] = h;
        }
    }
    __syncthreads();
}
template <bool KEEP_H>
__global__ void __launch_bounds__(256, 4) k_mlp_fwd(const uint16_t *__restrict__ X, int M, const unsigned long long *cnt,
                                                   int m_cidx, const uint16_t *__restrict__ wt,
                                                   const float *__restrict__ w, size_t oW1, size_t ob1, size_t oW2,
                                                   size_t ob2, size_t oW3, size_t ob3, size_t oW4, int nout, int col0,
                                                   int ncols, float *__restrict__ out,
                                                   const float *__restrict__ bias_out, uint16_t *H1, uint16_t *H2,
                                                   uint16_t *H3, int off)
{
    __shared__ __align__(16) uint16_t strip[4][16 * MLP_STRIP_LD];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    // rows of this chunk: the device count less the chunk's offset, at most M
    const int Mv = m_cidx >= 0 ? max(0, min(M, (int)cnt[m_cidx] - off)) : M;
    uint16_t *hs = strip[wave];
    for (int tile = blockIdx.x; tile * MLP_FT_ROWS < Mv; tile += gridDim.x) {
        const int row0 = tile * MLP_FT_ROWS + wave * 16;
        mlp_fwd_layer<MLP_IN, true, KEEP_H>(X, row0, Mv, wt + oW1, w + ob1, hs, H1, r, g);
        mlp_fwd_layer<MLP_H, false, KEEP_H>(X, row0, Mv, wt + oW2, w + ob2, hs, H2, r, g);
        mlp_fwd_layer<MLP_H, false, KEEP_H>(X, row0, Mv, wt + oW3, w + ob3, hs, H3, r, g);
        // output layer: 16 columns per MFMA tile, K = 64 in two steps
        const bf16x8 a0 = ld8(hs + r * MLP_STRIP_LD + 8 * g), a1 = ld8(hs + r * MLP_STRIP_LD + 32 + 8 * g);
#pragma unroll 1
        for (int c0 = 0; c0 < ncols; c0 += 16) {
            const int n = col0 + c0 + r;
            const bool nin = c0 + r < ncols;
            const uint16_t *wc = wt + oW4 + (size_t)n * MLP_H;
            const bf16x8 b0 = nin ? ld8(wc + 8 * g) : bf16x8{}, b1 = nin ? ld8(wc + 32 + 8 * g) : bf16x8{};
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc, 0, 0, 0);
            if (nin) {
                const float bo = bias_out ? bias_out[c0 + r] : 0.0f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int m = row0 + 4 * g + j;
                    if (m < Mv) out[(size_t)m * ncols + c0 + r] = acc[j] + bo;
                }
            }
        }
        __syncthreads();   // the strip is rewritten by the next tile
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
// / sum w (bf16) over the first N columns of rows of stride ld (the other ld - N columns of G are
// cleared), rows < min(M, cnt[m_cidx]) (one 256-thread block per row)
__global__ void k_ce_grad(const float *L, const float *bias, const int *label, const float *weight,
                          const float *wsum, int M, int N, int ld, uint16_t *G, const unsigned long long *cnt, int m_cidx)
{
    const int row = blockIdx.x;
    const int Mv = m_cidx >= 0 ? min(M, (int)cnt[m_cidx]) : M;
    if (row >= Mv) return;
    const float wsum_inv = *wsum > 0.0f ? 1.0f / *wsum : 0.0f;
    __shared__ float red[256];
    const float *l = L + (size_t)row * ld;
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
    for (int j = threadIdx.x; j < ld; j += blockDim.x) {
        const float gj = j < N ? w * (__expf(l[j] + bias[j] - mx) * inv - (j == lab ? 1.0f : 0.0f)) : 0.0f;
        G[(size_t)row * ld + j] = f2bf(gj);
    }
}

// ------------------------------------------------------------------ vMF retrace-direction head
// Lobe k of the raw outputs R (40 floats, bias included): unit mean (the raw direction
// normalised; +z if it vanishes), concentration exp(clamp(log kappa)), mixture logit.
__device__ __forceinline__ void vmf_lobe(const float *R, int k, float3 &mu, float &kappa, float &nrm)
{
    const float3 m = f3(R[5 * k], R[5 * k + 1], R[5 * k + 2]);
    nrm = sqrtf(dot3(m, m));
    mu = nrm > 1e-20f ? m * (1.0f / nrm) : f3(0.f, 0.f, 1.f);
    kappa = expf(fminf(fmaxf(R[5 * k + 3], VMF_LOGK_MIN), VMF_LOGK_MAX));
}
// von Mises-Fisher density (solid angle): kappa / (2 pi (1 - exp(-2 kappa))) exp(-kappa h), with
// h = 1 - mu.w written as |mu - w|^2 / 2 (no cancellation near the mean)
__device__ __forceinline__ float vmf_lobe_pdf(float3 mu, float kappa, float3 w)
{
    const float3 d = mu - w;
    const float h = 0.5f * dot3(d, d);
    return kappa / (2.0f * PT_PI * -expm1f(-2.0f * kappa)) * expf(-kappa * h);
}
// lobe probabilities that the inverse-CDF draw below realises with a 24-bit uniform u0: lobe k
// for c_{k-1} <= u0 < c_k (c = cumulative softmax of the lobe logits, the last one forced to 1),
// so P(k) = below_prob(c_k) - below_prob(c_{k-1})
__device__ __forceinline__ void vmf_weights(const float *R, float cdf[MLP_LOBES], float pr[MLP_LOBES])
{
    float mx = -3.0e38f;
    for (int k = 0; k < MLP_LOBES; ++k) mx = fmaxf(mx, R[5 * k + 4]);
    float e[MLP_LOBES], sum = 0.0f;
    for (int k = 0; k < MLP_LOBES; ++k) { e[k] = expf(R[5 * k + 4] - mx); sum += e[k]; }
    float c = 0.0f;
    double prev = 0.0;
    for (int k = 0; k < MLP_LOBES; ++k) {
        c += e[k] / sum;
        cdf[k] = k == MLP_LOBES - 1 ? 2.0f : c;
        const double b = k == MLP_LOBES - 1 ? 1.0 : below_prob(c);
        pr[k] = (float)(b - prev);
        prev = b;
    }
}
__device__ __forceinline__ float vmf_mix_pdf(const float *R, float3 w)
{
    float cdf[MLP_LOBES], pr[MLP_LOBES];
    vmf_weights(R, cdf, pr);
    float p = 0.0f;
    for (int k = 0; k < MLP_LOBES; ++k) {
        float3 mu;
        float kappa, nrm;
        vmf_lobe(R, k, mu, kappa, nrm);
        p += pr[k] * vmf_lobe_pdf(mu, kappa, w);
    }
    return p;
}
// a direction from the mixture: the lobe by inverse CDF (u0), then h = 1 - mu.w =
// -log(v + (1 - v) exp(-2 kappa)) / kappa with v = 1 - u1 in (0, 1] (the inverse CDF of the vMF's
// cosine), the azimuth 2 pi u2 about the mean
__device__ __forceinline__ float3 vmf_mix_sample(const float *R, float u0, float u1, float u2)
{
    float cdf[MLP_LOBES], pr[MLP_LOBES];
    vmf_weights(R, cdf, pr);
    int k = 0;
    while (k < MLP_LOBES - 1 && !(u0 < cdf[k])) ++k;
    float3 mu;
    float kappa, nrm;
    vmf_lobe(R, k, mu, kappa, nrm);
    const float v = 1.0f - u1;
    const float h = fminf(-logf(v + (1.0f - v) * expf(-2.0f * kappa)) / kappa, 2.0f);
    const float st = sqrtf(fmaxf(h * (2.0f - h), 0.0f));
    float3 t, b;
    basis(mu, t, b);
    float sp, cp;
    sincosf(2.0f * PT_PI * u2, &sp, &cp);
    return normalize3(mu * (1.0f - h) + (t * cp + b * sp) * st);
}
// gradient of the weighted negative log-likelihood of directions (rows [r0, r0 + nv) of L, stride
// ld, the 40 mixture outputs from column c0; weights over their sum) into G (bf16, the other
// columns of those rows cleared): lobe logit pi_k - r_k; log concentration
// -r_k (1 - 2 kappa / (exp(2 kappa) - 1) - kappa h) inside the clamp; raw direction
// -r_k kappa (w - (mu.w) mu) / |m|; r_k = pi_k p_k / p the lobe's responsibility
__global__ void k_vmf_grad(const float *L, const float *bias, const float *dir, const float *weight,
                           const float *wsum, int ld, int c0, uint16_t *G, const unsigned long long *cnt, int cap)
{
    const int nce = min((int)cnt[C_MLP_N], cap), nv = min((int)cnt[C_MLP_NV], cap);
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv) return;
    const int row = nce + j;
    float R[MLP_VMF];
    for (int q = 0; q < MLP_VMF; ++q) R[q] = L[(size_t)row * ld + c0 + q] + bias[c0 + q];
    const float3 w = f3(dir[3 * (size_t)j], dir[3 * (size_t)j + 1], dir[3 * (size_t)j + 2]);
    const float ws = *wsum > 0.0f ? weight[j] / *wsum : 0.0f;
    float mx = -3.0e38f;
    for (int k = 0; k < MLP_LOBES; ++k) mx = fmaxf(mx, R[5 * k + 4]);
    float pi[MLP_LOBES], pk[MLP_LOBES], sum = 0.0f, p = 0.0f;
    for (int k = 0; k < MLP_LOBES; ++k) { pi[k] = expf(R[5 * k + 4] - mx); sum += pi[k]; }
    for (int k = 0; k < MLP_LOBES; ++k) {
        pi[k] /= sum;
        float3 mu;
        float kappa, nrm;
        vmf_lobe(R, k, mu, kappa, nrm);
        pk[k] = vmf_lobe_pdf(mu, kappa, w);
        p += pi[k] * pk[k];
    }
    uint16_t *g = G + (size_t)row * ld;
    for (int q = 0; q < c0; ++q) g[q] = 0;
    for (int q = c0 + MLP_VMF; q < ld; ++q) g[q] = 0;
    for (int k = 0; k < MLP_LOBES; ++k) {
        float3 mu;
        float kappa, nrm;
        vmf_lobe(R, k, mu, kappa, nrm);
        const float r = p > 0.0f ? pi[k] * pk[k] / p : 0.0f;
        const float3 d = mu - w;
        const float h = 0.5f * dot3(d, d);
        const float two_k = 2.0f * kappa;
        const float ratio = two_k < 80.0f ? two_k / expm1f(two_k) : 0.0f;
        const float s = R[5 * k + 3];
        const float gs = (s > VMF_LOGK_MIN && s < VMF_LOGK_MAX) ? -r * (1.0f - ratio - kappa * h) : 0.0f;
        const float cw = dot3(mu, w);
        const float3 gm = nrm > 1e-20f ? (w - mu * cw) * (-r * kappa / nrm) : f3(0.f, 0.f, 0.f);
        g[c0 + 5 * k + 0] = f2bf(ws * gm.x);
        g[c0 + 5 * k + 1] = f2bf(ws * gm.y);
        g[c0 + 5 * k + 2] = f2bf(ws * gm.z);
        g[c0 + 5 * k + 3] = f2bf(ws * gs);
        g[c0 + 5 * k + 4] = f2bf(ws * (pi[k] - r));
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
// gradient. Runs only when this iteration has training rows.
__global__ void k_adam(float *w, uint16_t *wb, float *g, float *m, float *v, int n, float lr, float b1, float b2,
                       float eps, const unsigned long long *cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || cnt[C_MLP_ROWS] == 0) return;
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
    if (threadIdx.x == 0 && blockIdx.x == 0 && cnt[C_MLP_ROWS] != 0) cnt[C_MLP_T] += 1ull;
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

// features of the proxy items' first diffuse vertices (items off .. off + M - 1) -> encoded rows of X
__global__ void k_mlp_enc_items(SceneDev S, const ProxyItem *items, const unsigned long long *cnt, uint16_t *X, int off,
                                int M)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M || off + i >= (int)cnt[C_PROXYQ]) return;
    const ProxyItem &p = items[off + i];
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
// the chosen S under the mixture is written with it: aux.z = S (bits), aux.w = pi_S; then an
// incomplete sub-path of S uniformly: mis.z = its index (bits), mis.w = its overall selection
// probability. Items off .. off + M - 1; L holds n_out logits per item of the chunk (bias not
// included).
__global__ void k_mlp_select(EyeBuf E, SubDev D, const float *L, const float *bias, int n_out, float mix, int gamma_on,
                             uint32_t seed, const unsigned long long *cnt, int off, int M)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M || off + i >= (int)cnt[C_PROXYQ]) return;
    ProxyItem &it = E.proxy[off + i];
    // the subspace lists are rebuilt only in iterations that keep candidates
    const int ne = cnt[C_NFINAL] > 0 ? min(*D.n_nonempty, D.n_spec) : 0;
    if (ne <= 0) {
        it.aux.z = __int_as_float(-1); it.aux.w = 0.0f;
        it.mis.z = __int_as_float(-1); it.mis.w = 0.0f;
        return;
    }
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
    const double piS = m * learned + (1.0 - m) * plain;
    it.aux.z = __int_as_float(S);
    it.aux.w = (float)piS;
    // then the incomplete sub-path uniformly within S: its index and overall selection probability
    const int cs = D.s_count[S];
    if (cs > 0) {
        const int k = index_of(rng_u32(r), cs);
        it.mis.z = __int_as_float(D.s_list[D.s_off[S] + k]);
        it.mis.w = (float)(piS * index_prob(k, cs));
    } else {
        it.mis.z = __int_as_float(-1);
        it.mis.w = 0.0f;
    }
}

// The same selection with one wavefront per item, for many subspaces: the lanes read the item's
// logits row together (coalesced) for the maximum and the sum of the softmax terms, and the
// inverse CDF walks the row in blocks of 64 with a wavefront prefix sum in double. The draws
// (the same Philox counters), the probability written out and the choice of the block-ordered
// cumulative sum crossing the target are those of k_mlp_select up to the order of the double
// additions; the probability divides by the sum the draw used.
__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__global__ void __launch_bounds__(256) k_mlp_select_wave(EyeBuf E, SubDev D, const float *L, const float *bias,
                                                         int n_out, float mix, int gamma_on, uint32_t seed,
                                                         const unsigned long long *cnt, int off, int M)
{
    const int lane = threadIdx.x & 63;
    const int i = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));   // one item per wave
    if (i >= M || off + i >= (int)cnt[C_PROXYQ]) return;
    ProxyItem &it = E.proxy[off + i];
    const int ne = cnt[C_NFINAL] > 0 ? min(*D.n_nonempty, D.n_spec) : 0;
    if (ne <= 0) {
        if (lane == 0) {
            it.aux.z = __int_as_float(-1); it.aux.w = 0.0f;
            it.mis.z = __int_as_float(-1); it.mis.w = 0.0f;
        }
        return;
    }
    const int T = __float_as_int(it.aux.x);
    const float *l = L + (size_t)i * n_out;
    Rng r = rng_make(seed, S_MLP, (uint32_t)__float_as_int(it.beta.w), (uint32_t)cnt[C_ITER], 1u);
    float mx = -3.0e38f;
    for (int j = lane; j < ne; j += 64) mx = fmaxf(mx, l[D.nonempty[j]] + bias[D.nonempty[j]]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    double part = 0.0;
    for (int j = lane; j < ne; j += 64) part += (double)__expf(l[D.nonempty[j]] + bias[D.nonempty[j]] - mx);
    const double sum = wave_sum_d(part);
    const float u0 = rng_f(r);
    const uint32_t xa = rng_u32(r), xb = rng_u32(r);
    int S, jS;
    if (u0 < mix) {
        const double u = (double)(((uint64_t)xa << 21) | (uint64_t)(xb >> 11)) * (1.0 / 9007199254740992.0);
        const double target = u * sum;
        double base = 0.0;
        int last = -1;   // the last index with a non-zero term so far (the draw when rounding leaves no crossing)
        jS = -1;
        for (int b = 0; b < ne && jS < 0; b += 64) {
            const int j = b + lane;
            const double e = j < ne ? (double)__expf(l[D.nonempty[j]] + bias[D.nonempty[j]] - mx) : 0.0;
            double c = e;   // inclusive prefix sum over the block
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const double t = __shfl_up(c, o);
                if (lane >= o) c += t;
            }
            const unsigned long long cross = __ballot(e > 0.0 && target < base + c);
            if (cross) {
                jS = b + __ffsll((long long)cross) - 1;
            } else {
                const unsigned long long nz = __ballot(e > 0.0);
                if (nz) last = b + 63 - __clzll((long long)nz);
                base += __shfl(c, 63);
            }
        }
        if (jS < 0) jS = last >= 0 ? last : 0;
        S = D.nonempty[jS];
    } else if (gamma_on) {
        const size_t row = (size_t)T * D.n_spec;
        jS = alias_draw(D.al_prob + row, D.al_idx + row, ne, xa, (float)(xb >> 8) * (1.0f / 16777216.0f));
        S = D.nonempty[jS];
    } else {
        jS = index_of(xa, ne);
        S = D.nonempty[jS];
    }
    if (lane != 0) return;
    const double learned = (double)__expf(l[S] + bias[S] - mx) / sum;
    const double plain = gamma_on ? (double)sel_prob(D, T, S) : index_prob(jS, ne);
    const double m = below_prob(mix);
    const double piS = m * learned + (1.0 - m) * plain;
    it.aux.z = __int_as_float(S);
    it.aux.w = (float)piS;
    const int cs = D.s_count[S];
    if (cs > 0) {
        const int k = index_of(rng_u32(r), cs);
        it.mis.z = __int_as_float(D.s_list[D.s_off[S] + k]);
        it.mis.w = (float)(piS * index_prob(k, cs));
    } else {
        it.mis.z = __int_as_float(-1);
        it.mis.w = 0.0f;
    }
}

// Training samples of a learning iteration, one per valid proxy contribution: for the subspace
// head the features of the first diffuse eye vertex, the selected subspace and the
// contribution's luminance as weight; for the direction head the features of y_{s-1} (direction
// toward z_d), the first retrace direction and the same weight (retraces from glossy y_{s-1}).
struct MlpTrain {
    float *feat;     // [cap x 9]
    int *label;      // [cap]
    float *weight;   // [cap]
    float *wsum;     // [1]
    float *vfeat;    // [cap x 9]
    float *vdir;     // [cap x 3]
    float *vweight;  // [cap]
    float *vwsum;    // [1]
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
__device__ __forceinline__ void mlp_record_dir(const SceneDev &S, const MlpTrain &T, unsigned long long *cnt, float3 x,
                                               float3 n, float3 wo, float3 dir, float w)
{
    const int slot = (int)atomicAdd(cnt + C_MLP_NV, 1ull);
    if (slot >= T.cap) return;
    float f[9];
    feat9(S, x, n, wo, f);
    for (int j = 0; j < 9; ++j) T.vfeat[9 * (size_t)slot + j] = f[j];
    T.vdir[3 * (size_t)slot] = dir.x; T.vdir[3 * (size_t)slot + 1] = dir.y; T.vdir[3 * (size_t)slot + 2] = dir.z;
    T.vweight[slot] = w;
    unsafeAtomicAdd(T.vwsum, w);
}
// rows of this iteration's training batch: the subspace samples, then the direction samples
__global__ void k_mlp_rows(unsigned long long *cnt, int cap)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        cnt[C_MLP_ROWS] = (unsigned long long)(min((int)cnt[C_MLP_N], cap) + min((int)cnt[C_MLP_NV], cap));
}
// encoded rows of the training batch (subspace rows first)
__global__ void k_mlp_enc_train(MlpTrain T, const unsigned long long *cnt, uint16_t *X)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nce = min((int)cnt[C_MLP_N], T.cap), nv = min((int)cnt[C_MLP_NV], T.cap);
    if (i >= nce + nv) return;
    const float *src = i < nce ? T.feat + 9 * (size_t)i : T.vfeat + 9 * (size_t)(i - nce);
    float f[9];
    for (int j = 0; j < 9; ++j) f[j] = src[j];
    mlp_encode(f, X + (size_t)i * MLP_IN);
}
// features of every proxy item's chosen y_{s-1} (position, normal, direction toward z_d) ->
// encoded rows of X (zeros for an item without a choice); items off .. off + M - 1
__global__ void k_mlp_enc_retrace(SceneDev S, const ProxyItem *items, const Cand *cand, const unsigned long long *cnt,
                                  uint16_t *X, int off, int M)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M || off + i >= (int)cnt[C_PROXYQ]) return;
    const ProxyItem &p = items[off + i];
    const int ci = __float_as_int(p.mis.z);
    float f[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (ci >= 0 && p.mis.w > 0.0f) {
        const Cand &c = cand[ci];
        const float3 v = xyz(c.v);
        feat9(S, v, S.shade[__float_as_int(c.v.w)].n, normalize3(xyz(p.x) - v), f);
    }
    mlp_encode(f, X + (size_t)i * MLP_IN);
}
// test hook: n draws from the mixtures raw[n][40] (bias included) with their mixture density
__global__ void k_vmf_hook(const float *raw, int n, uint32_t seed, float *dir, float *pdf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float R[MLP_VMF];
    for (int q = 0; q < MLP_VMF; ++q) R[q] = raw[(size_t)i * MLP_VMF + q];
    Rng r = rng_make(seed, S_MLP, (uint32_t)i, 7u, 0u);
    const float u0 = rng_f(r), u1 = rng_f(r), u2 = rng_f(r);
    const float3 w = vmf_mix_sample(R, u0, u1, u2);
    dir[3 * (size_t)i] = w.x; dir[3 * (size_t)i + 1] = w.y; dir[3 * (size_t)i + 2] = w.z;
    pdf[i] = vmf_mix_pdf(R, w);
}
