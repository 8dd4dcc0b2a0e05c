// swim_mlp.hip -- gfx950 kernels of the MLP surrogate: a BF16 MFMA GEMM
// (v_mfma_f32_16x16x16bf16_1k, FP32 accumulation) with fused epilogues for
// the forward layers (bias, GELU) and the backward pass (GELU'), column sums
// for the bias gradients, the MSE loss gradient, Adam, and the prescreen
// distance of ABC proposals.
//
// GEMM operands are read as FP32 and rounded to bfloat16 (nearest, ties to
// even) while they are staged into LDS, so the network computes with BF16
// weights and activations and FP32 accumulation; FP32 master weights are
// kept for Adam.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <math.h>
#include <stdint.h>

#include "swim_internal.h"
#include "swim_philox.h"

namespace swim {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (one v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// erf by Abramowitz & Stegun, Handbook of Mathematical Functions, 7.1.26:
// erf(x) = 1 - (a1 t + a2 t^2 + ... + a5 t^5) exp(-x^2), t = 1 / (1 + p x),
// x >= 0, odd extension; absolute error at most 1.5e-7 (plus the hardware
// reciprocal and exp2 at 1 ulp each), far below the BF16 resolution at which
// every activation feeds the next layer.  About 12 instructions against ~44
// for the library erff, which bound the fused MLP on the vector ALUs.
__device__ __forceinline__ float erf_as(float x)
{
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
    float p = fmaf(1.061405429f, t, -1.453152027f);
    p = fmaf(p, t, 1.421413741f);
    p = fmaf(p, t, -0.284496736f);
    p = fmaf(p, t, 0.254829592f);
    p *= t;
    const float e = __builtin_amdgcn_exp2f(-ax * ax * 1.4426950408889634f);  // exp(-x^2)
    return copysignf(fmaf(-p, e, 1.0f), x);
}

// GELU(x) = (x/2)(1 + erf(x/sqrt 2)) with erf from 7.1.26 rearranged: with
// a = |x|, z = a/sqrt 2 and erf(z) = 1 - P(t) exp(-z^2), t = 1/(1 + p z),
// GELU(x) = max(x, 0) - (a/2) P(t) exp(-a^2/2) for either sign of x (no
// copysign, no 1 + erf); the same function as (x/2)(1 + erf_as(x/sqrt 2)).
__device__ __forceinline__ float gelu_f(float x)
{
    const float a = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, a, 1.0f));
    float p = fmaf(1.061405429f, t, -1.453152027f);
    p = fmaf(p, t, 1.421413741f);
    p = fmaf(p, t, -0.284496736f);
    p = fmaf(p, t, 0.254829592f);
    // exp(-a^2/2) / 2, the halving folded into the exponent
    const float e = __builtin_amdgcn_exp2f(fmaf(a * a, -0.5f * 1.4426950408889634f, -1.0f));
    return fmaf(-(a * t), p * e, fmaxf(x, 0.0f));
}

__device__ __forceinline__ float gelu_grad_f(float x)
{
    const float cdf = 0.5f * (1.0f + erf_as(x * 0.70710678118654752f));
    const float pdf = 0.39894228040143268f * __builtin_amdgcn_exp2f(-0.5f * x * x * 1.4426950408889634f);
    return fmaf(x, pdf, cdf);
}

// C(m, n) = sum_k A(m, k) B(k, n), A(m, k) = A[m*sam + k*sak],
// B(k, n) = B[k*sbk + n*sbn], C(m, n) at C[m*ldc + n].  Epilogues:
//   MLP_EPI_PLAIN  C = acc
//   MLP_EPI_GELU   pre = acc + bias[n] -> C;  H = gelu(pre) -> aux
//   MLP_EPI_BIAS   C = acc + bias[n]
//   MLP_EPI_DGELU  C = acc * gelu'(aux(m, n))   (aux = pre-activations)
//   MLP_EPI_MSE    Y = acc + bias[n] -> C; with d = Y - T(m, n):
//                  dY = sc d -> aux (sc = 2 / (M N)), d^2 -> sq  (ldc = N)
// Workgroup tile 64 x 64 (4 waves of 32 x 32 = 2 x 2 MFMA tiles), k chunks of 32.
constexpr int GT = 64, GK = 32, GPAD = 8;

// epilogue of one output element (the split-K fixup applies it too)
template <int EPI>
__device__ __forceinline__ void gemm_epilogue(float v, int n, int64_t o, float* __restrict__ C, const GemmEpi& E)
{
    if (EPI == 1) {
        v += E.bias[n];
        C[o] = v;
        E.aux[o] = gelu_f(v);
    } else if (EPI == 2) {
        C[o] = v + E.bias[n];
    } else if (EPI == 3) {
        C[o] = v * gelu_grad_f(E.aux[o]);
    } else if (EPI == 4) {
        v += E.bias[n];
        C[o] = v;
        const float d = v - E.T[o];
        E.aux[o] = E.sc * d;
        E.sq[o] = d * d;
    } else {
        C[o] = v;
    }
}

// Split K: with part != nullptr, workgroup z of the grid's third dimension
// takes the k chunks [z kper, (z + 1) kper) and writes its raw sums to
// part[z][M][N]; k_gemm_reduce adds the slices in order of z and applies the
// epilogue (deterministic).  This fills the chip when the M x N tiles are
// few (the weight gradients: 256 x 256 outputs summed over a batch of 1024).
// (A last-arriving-workgroup reduction inside the GEMM was tried: its
// device-scope fences, which write back the L2 of the XCD, made the GEMMs
// 3-5x slower than the second launch.)
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const float* __restrict__ A, int64_t sam,
                                                   int64_t sak, const float* __restrict__ B, int64_t sbk, int64_t sbn,
                                                   float* __restrict__ C, int64_t ldc, GemmEpi E,
                                                   float* __restrict__ part, int kper)
{
    __shared__ uint16_t As[GT][GK + GPAD];   // [m][k]
    __shared__ uint16_t Bs[GT][GK + GPAD];   // [n][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    // consecutive threads take consecutive addresses of each operand: along k
    // when its k stride is 1, along m (n) otherwise (the transposed operands
    // of the backward pass)
    const bool a_k_fast = sak == 1, b_n_fast = sbn == 1 || sbk != 1;
    const int kbeg = part ? (int)blockIdx.z * kper * GK : 0;
    const int kend = part ? min(K, kbeg + kper * GK) : K;
    // the next chunk's operands are fetched into registers while the
    // current chunk's MFMAs run
    constexpr int PER = (GT * GK) / 256;
    float ra[PER], rb[PER];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            const int r = a_k_fast ? e / GK : e % GT, kk = a_k_fast ? e % GK : e / GT;
            const int m = m0 + r, k = k0 + kk;
            ra[i] = (m < M && k < K) ? A[(int64_t)m * sam + (int64_t)k * sak] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            const int kk = b_n_fast ? e / GT : e % GK, c = b_n_fast ? e % GT : e / GK;
            const int n = n0 + c, k = k0 + kk;
            rb[i] = (n < N && k < K) ? B[(int64_t)k * sbk + (int64_t)n * sbn] : 0.0f;
        }
    };
    if (kbeg < kend) fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            const int r = a_k_fast ? e / GK : e % GT, kk = a_k_fast ? e % GK : e / GT;
            As[r][kk] = f2bf(ra[i]);
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            const int kk = b_n_fast ? e / GT : e % GK, c = b_n_fast ? e % GT : e / GK;
            Bs[c][kk] = f2bf(rb[i]);
        }
        __syncthreads();
        if (k0 + GK < kend) fetch(k0 + GK);
#pragma unroll
        for (int ks = 0; ks < GK; ks += 16) {
            // operand layout of the 16x16x16 MFMA: lane l holds row (l % 16)
            // and k = 4 (l / 16) .. 4 (l / 16) + 3 of its 16-wide k slice
            const int kq = ks + 4 * (lane >> 4);
            bf16x4_t av[2], bv[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                // 8-byte aligned: rows of GK + GPAD = 40 elements, kq % 4 == 0
                av[t] = __builtin_bit_cast(bf16x4_t, *reinterpret_cast<const uint2*>(&As[wm + 16 * t + (lane & 15)][kq]));
                bv[t] = __builtin_bit_cast(bf16x4_t, *reinterpret_cast<const uint2*>(&Bs[wn + 16 * t + (lane & 15)][kq]));
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    // result layout: lane l holds column (l % 16), rows 4 (l / 16) + r
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * a + 4 * (lane >> 4) + r;
                const int n = n0 + wn + 16 * b + (lane & 15);
                if (m >= M || n >= N) continue;
                if (part)
                    part[((int64_t)blockIdx.z * M + m) * N + n] = acc[a][b][r];
                else
                    gemm_epilogue<EPI>(acc[a][b][r], n, (int64_t)m * ldc + n, C, E);
            }
}

// C(m, n) = sum over z of part[z][m][n], z ascending, then the epilogue.  The
// S <= GEMM_MAX_SPLIT loads are issued before the sum (independent, not a
// chain of dependent load latencies).
constexpr int GEMM_MAX_SPLIT = 16;
template <int EPI>
__global__ void k_gemm_reduce(int M, int N, int S, const float* __restrict__ part, float* __restrict__ C, int64_t ldc,
                              GemmEpi E)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)M * N) return;
    const int m = (int)(e / N), n = (int)(e % N);
    float p[GEMM_MAX_SPLIT];
#pragma unroll
    for (int z = 0; z < GEMM_MAX_SPLIT; ++z) p[z] = z < S ? part[(int64_t)z * M * N + e] : 0.0f;
    float v = 0.0f;
#pragma unroll
    for (int z = 0; z < GEMM_MAX_SPLIT; ++z)
        if (z < S) v += p[z];
    gemm_epilogue<EPI>(v, n, (int64_t)m * ldc + n, C, E);
}

// out[n] = sum_m A[m*lda + n]  (bias gradients): a workgroup of 1024
// threads sums 8 columns, 128 row groups each summing every 128th row (8
// rows for a batch of 1024, loads issued ahead of the adds), then the 128
// partial sums of a column in a fixed tree (deterministic)
__global__ __launch_bounds__(1024) void k_colsum(int M, int N, const float* __restrict__ A, int64_t lda,
                                                 float* __restrict__ out)
{
    __shared__ float part[128][9];
    const int c = threadIdx.x & 7, g = threadIdx.x >> 3;
    const int n = blockIdx.x * 8 + c;
    float s = 0.f;
    if (n < N) {
        int m = g;
        for (; m + 128 * 7 < M; m += 128 * 8) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = A[(int64_t)(m + 128 * j) * lda + n];
#pragma unroll
            for (int j = 0; j < 8; ++j) s += v[j];
        }
        for (; m < M; m += 128) s += A[(int64_t)m * lda + n];
    }
    part[g][c] = s;
    __syncthreads();
    for (int w = 64; w >= 1; w >>= 1) {
        if (g < w) part[g][c] += part[g + w][c];
        __syncthreads();
    }
    if (g == 0 && n < N) out[n] = part[0][c];
}

// out[0] = sum of v[0..n): one workgroup of 1024 threads, each summing a
// strided share, then a fixed tree (the training loss)
__global__ __launch_bounds__(1024) void k_sum(int64_t n, const float* __restrict__ v, float* __restrict__ out)
{
    __shared__ float part[1024];
    float s = 0.f;
    for (int64_t i = threadIdx.x; i < n; i += 1024) s += v[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0];
}

// rows of X and T picked by perm[0..M) into the batch buffers; an index
// outside [0, nrows) yields a NaN row (the loss turns NaN) instead of a read
// out of bounds
__global__ void k_gather_rows(int M, const int32_t* perm, int64_t nrows, const float* X, int nx, const float* T, int nt,
                              float* Xb, float* Tb)
{
    const int m = blockIdx.x;
    if (m >= M) return;
    const int64_t src = perm[m];
    const bool ok = src >= 0 && src < nrows;
    for (int c = threadIdx.x; c < nx + nt; c += blockDim.x) {
        if (c < nx) Xb[(int64_t)m * nx + c] = ok ? X[src * nx + c] : NAN;
        else Tb[(int64_t)m * nt + c - nx] = ok ? T[src * nt + c - nx] : NAN;
    }
}

// Adam with bias-corrected moments: p -= lr mhat / (sqrt(vhat) + eps)
__global__ void k_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float c1,
                       float c2, float eps)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// Prescreen distance: de-standardize the predicted summaries, compare with the
// observed summaries: d = sqrt(mean_j (mu_j + sd_j y_j - obs_j)^2) over the
// first n_sum outputs; keep[m] = d <= tol.
__global__ void k_prescreen(int M, int N, int n_sum, const float* Y, const float* mu, const float* sd,
                            const float* obs, float tol, float* dist, uint8_t* keep)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    float s = 0.f;
    for (int j = 0; j < n_sum; ++j) {
        const float d = fmaf(sd[j], Y[(int64_t)m * N + j], mu[j]) - obs[j];
        s = fmaf(d, d, s);
    }
    const float d = sqrtf(s / (float)n_sum);
    if (dist) dist[m] = d;
    keep[m] = (d <= tol) ? 1 : 0;
}

// stream compaction of keep[0..n) into idx (ascending): per-block counts,
// a single-block exclusive scan, then the scatter
__global__ void k_count_blocks(int64_t n, const uint8_t* keep, int32_t* counts)
{
    __shared__ int32_t s[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    s[threadIdx.x] = (i < n && keep[i]) ? 1 : 0;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = s[0];
}

__global__ void k_scan_counts(int64_t nb, int32_t* counts, int64_t* total)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t acc = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int32_t c = counts[b];
        counts[b] = (int32_t)acc;
        acc += c;
    }
    *total = acc;
}

__global__ void k_scatter(int64_t n, const uint8_t* keep, const int32_t* offs, int64_t* idx)
{
    __shared__ int32_t s[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int f = (i < n && keep[i]) ? 1 : 0;
    s[threadIdx.x] = f;
    __syncthreads();
    // inclusive scan inside the block (Hillis-Steele)
    for (int o = 1; o < 256; o <<= 1) {
        const int v = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += v;
        __syncthreads();
    }
    if (f) idx[offs[blockIdx.x] + s[threadIdx.x] - 1] = i;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_gemm_bf16(int epi, int M, int N, int K, const float* A, int64_t sam, int64_t sak, const float* B,
                            int64_t sbk, int64_t sbn, float* C, int64_t ldc, const GemmEpi& E, const MlpWs& ws,
                            hipStream_t st)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    if (epi == 4 && ldc != N) return hipErrorInvalidValue;
    const int gx = (N + GT - 1) / GT, gy = (M + GT - 1) / GT, chunks = (K + GK - 1) / GK;
    // split K into S slices when the output tiles alone leave CUs idle
    int S = 1, kper = chunks;
    if (ws.part && chunks >= 2 && gx * gy < 256) {
        S = std::min({chunks, (256 + gx * gy - 1) / (gx * gy), GEMM_MAX_SPLIT});
        while (S > 1 && (int64_t)S * M * N > ws.part_floats) --S;
        kper = (chunks + S - 1) / S;
        S = (chunks + kper - 1) / kper;
    }
    float* part = S > 1 ? ws.part : nullptr;
    const dim3 grid(gx, gy, S);
#define SWIM_GEMM_CASE(EP)                                                                                         \
    case EP:                                                                                                       \
        hipLaunchKernelGGL(k_gemm_bf16<EP>, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, E,  \
                           part, kper);                                                                            \
        if (part)                                                                                                  \
            hipLaunchKernelGGL(k_gemm_reduce<EP>, dim3((unsigned)(((int64_t)M * N + 255) / 256)), dim3(256), 0,    \
                               st, M, N, S, part, C, ldc, E);                                                      \
        break;
    switch (epi) {
        SWIM_GEMM_CASE(0)
        SWIM_GEMM_CASE(1)
        SWIM_GEMM_CASE(2)
        SWIM_GEMM_CASE(3)
        SWIM_GEMM_CASE(4)
    default: return hipErrorInvalidValue;
    }
#undef SWIM_GEMM_CASE
    return hipGetLastError();
}

hipError_t launch_colsum(int M, int N, const float* A, int64_t lda, float* out, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_colsum, dim3((N + 7) / 8), dim3(1024), 0, st, M, N, A, lda, out);
    return hipGetLastError();
}

hipError_t launch_sum(int64_t n, const float* v, float* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, st, n, v, out);
    return hipGetLastError();
}

hipError_t launch_gather_rows(int M, const int32_t* perm, int64_t nrows, const float* X, int nx, const float* T, int nt,
                              float* Xb, float* Tb, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_rows, dim3(M), dim3(64), 0, st, M, perm, nrows, X, nx, T, nt, Xb, Tb);
    return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float c1,
                       float c2, float eps, hipStream_t st)
{
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, p, g, m, v, lr, b1, b2, c1, c2,
                       eps);
    return hipGetLastError();
}

hipError_t launch_prescreen(int M, int N, int n_sum, const float* Y, const float* mu, const float* sd, const float* obs,
                            float tol, float* dist, uint8_t* keep, hipStream_t st)
{
    if (M <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prescreen, dim3((M + 255) / 256), dim3(256), 0, st, M, N, n_sum, Y, mu, sd, obs, tol, dist,
                       keep);
    return hipGetLastError();
}

hipError_t launch_compact(int64_t n, const uint8_t* keep, int32_t* counts, int64_t* idx, int64_t* total, hipStream_t st)
{
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_count_blocks, dim3((unsigned)nb), dim3(256), 0, st, n, keep, counts);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(64), 0, st, nb, counts, total);
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)nb), dim3(256), 0, st, n, keep, counts, idx);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// surrogate data preparation
// ---------------------------------------------------------------------------
// X[i] = (alpha, ln S_b, ln S_s, b, omega), standardized when mu/sd are given
__global__ void k_features(int64_t n, const double* theta, double b, double om, const float* mu, const float* sd,
                           float* X)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double f[5] = {theta[3 * i], log(theta[3 * i + 1]), log(theta[3 * i + 2]), b, om};
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        float v = (float)f[c];
        if (mu) v = (v - mu[c]) / sd[c];
        X[i * 5 + c] = v;
    }
}

// T[i] = (head displacement at the chosen samples, x then y, ..., speed)
template <typename T>
__global__ void k_targets(int64_t n, int n_obs, const T* obs, const T* speed, double x0, double y0, const int32_t* idx,
                          int n_sum, float* Tout)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int nt = 2 * n_sum + 1;
    for (int j = 0; j < n_sum; ++j) {
        const T* o = obs + (i * n_obs + idx[j]) * 2;
        Tout[i * nt + 2 * j] = (float)((double)o[0] - x0);
        Tout[i * nt + 2 * j + 1] = (float)((double)o[1] - y0);
    }
    Tout[i * nt + 2 * n_sum] = (float)speed[i];
}

// column mean and standard deviation (population), one workgroup per column,
// fixed summation order
__global__ __launch_bounds__(256) void k_colstats(int64_t n, int cols, const float* A, float* mu, float* sd)
{
    __shared__ double red[256];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)A[i * cols + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double m = red[0] / (double)n;
    __syncthreads();
    double q = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double d = (double)A[i * cols + c] - m;
        q += d * d;
    }
    red[threadIdx.x] = q;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        mu[c] = (float)m;
        const double v = red[0] / (double)n;
        sd[c] = v > 0.0 ? (float)sqrt(v) : 1.0f;
    }
}

__global__ void k_standardize(int64_t n, int cols, float* A, const float* mu, const float* sd)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * cols) return;
    const int c = (int)(e % cols);
    A[e] = (A[e] - mu[c]) / sd[c];
}

// prior draws on the device, identical to the host abc_prior_draw:
// theta[i][d] = lo[d] + (hi[d] - lo[d]) u_d, u from Philox stream 0, draws 0, 1
__global__ void k_prior_draw(uint64_t seed, int64_t n, double lo0, double lo1, double lo2, double hi0, double hi1,
                             double hi2, double* theta)
{
    // separately rounded multiply and add, as the host draw computes them
    // (the default contraction would fuse them into one FMA)
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double u[4];
    philox_uniforms2(seed, 0, (uint64_t)i, 0, u);
    philox_uniforms2(seed, 0, (uint64_t)i, 1, u + 2);
    const double lo[3] = {lo0, lo1, lo2}, hi[3] = {hi0, hi1, hi2};
#pragma unroll
    for (int d = 0; d < 3; ++d) theta[3 * i + d] = lo[d] + (hi[d] - lo[d]) * u[d];
}

// param rows (alpha, S_b, S_s, b, omega, k, 0, 0, 0) of the theta rows idx[j]
// (idx NULL: j itself), j < *n_dev; an index outside [0, n_theta) gives a
// NaN row (that system is then flagged SWIM_ST_BADPARAM)
__global__ void k_param_rows(int64_t cap, const int64_t* n_dev, const int64_t* idx, int64_t n_theta,
                             const double* theta, double b, double om, double kw, double* rows)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cap || (n_dev && j >= *n_dev)) return;
    const int64_t i = idx ? idx[j] : j;
    const bool ok = i >= 0 && i < n_theta;
    double* P = rows + 9 * j;
    P[0] = ok ? theta[3 * i] : NAN;
    P[1] = ok ? theta[3 * i + 1] : NAN;
    P[2] = ok ? theta[3 * i + 2] : NAN;
    P[3] = b;
    P[4] = om;
    P[5] = kw;
    P[6] = 0.0;
    P[7] = 0.0;
    P[8] = 0.0;
}

// dst[j] = src[idx[j]] (rows of `cols` floats), j < *n_dev; an index outside
// [0, n_src) gives a NaN row
__global__ void k_gather_f32(int64_t cap, const int64_t* n_dev, const int64_t* idx, int64_t n_src, const float* src,
                             int cols, float* dst)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j = e / cols;
    if (j >= cap || j >= *n_dev) return;
    const int c = (int)(e % cols);
    const int64_t i = idx[j];
    dst[j * cols + c] = (i >= 0 && i < n_src) ? src[i * cols + c] : NAN;
}

__global__ void k_flag_eq(int64_t n, const int32_t* v, int32_t want, uint8_t* keep)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) keep[i] = v[i] == want ? 1 : 0;
}

// keep[i] &= every one of the first n_disp entries of row i of T is finite
// with magnitude <= max_disp
__global__ void k_flag_bounded(int64_t n, const float* T, int nt, int n_disp, float max_disp, uint8_t* keep)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool ok = keep[i] != 0;
    for (int j = 0; j < n_disp; ++j) ok = ok && fabsf(T[i * nt + j]) <= max_disp;
    keep[i] = ok ? 1 : 0;
}

hipError_t launch_features(int64_t n, const double* theta, double b, double om, const float* mu, const float* sd,
                           float* X, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, theta, b, om, mu, sd, X);
    return hipGetLastError();
}

hipError_t launch_targets(int dtype, int64_t n, int n_obs, const void* obs, const void* speed, double x0, double y0,
                          const int32_t* idx, int n_sum, float* T, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const dim3 g((unsigned)((n + 255) / 256));
    if (dtype == 0)
        hipLaunchKernelGGL(k_targets<float>, g, dim3(256), 0, st, n, n_obs, (const float*)obs, (const float*)speed, x0,
                           y0, idx, n_sum, T);
    else
        hipLaunchKernelGGL(k_targets<double>, g, dim3(256), 0, st, n, n_obs, (const double*)obs, (const double*)speed,
                           x0, y0, idx, n_sum, T);
    return hipGetLastError();
}

hipError_t launch_colstats(int64_t n, int cols, const float* A, float* mu, float* sd, hipStream_t st)
{
    hipLaunchKernelGGL(k_colstats, dim3(cols), dim3(256), 0, st, n, cols, A, mu, sd);
    return hipGetLastError();
}

hipError_t launch_standardize(int64_t n, int cols, float* A, const float* mu, const float* sd, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_standardize, dim3((unsigned)((n * cols + 255) / 256)), dim3(256), 0, st, n, cols, A, mu, sd);
    return hipGetLastError();
}

hipError_t launch_prior_draw(uint64_t seed, int64_t n, const double* lo, const double* hi, double* theta,
                             hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prior_draw, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, seed, n, lo[0], lo[1], lo[2],
                       hi[0], hi[1], hi[2], theta);
    return hipGetLastError();
}

hipError_t launch_param_rows(int64_t cap, const int64_t* n_dev, const int64_t* idx, int64_t n_theta,
                             const double* theta, double b, double om, double kw, double* rows, hipStream_t st)
{
    if (cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_param_rows, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, st, cap, n_dev, idx, n_theta,
                       theta, b, om, kw, rows);
    return hipGetLastError();
}

hipError_t launch_gather_f32(int64_t cap, const int64_t* n_dev, const int64_t* idx, int64_t n_src, const float* src,
                             int cols, float* dst, hipStream_t st)
{
    if (cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_f32, dim3((unsigned)((cap * cols + 255) / 256)), dim3(256), 0, st, cap, n_dev, idx,
                       n_src, src, cols, dst);
    return hipGetLastError();
}

hipError_t launch_flag_eq(int64_t n, const int32_t* v, int32_t want, uint8_t* keep, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flag_eq, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, v, want, keep);
    return hipGetLastError();
}

hipError_t launch_flag_bounded(int64_t n, const float* T, int nt, int n_disp, float max_disp, uint8_t* keep,
                               hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flag_bounded, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, T, nt, n_disp,
                       max_disp, keep);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused inference: every workgroup carries MLP_RT = 64 rows through all
// five layers, one 16-row tile per wave, with the activations in
// registers.  The product is formed transposed, C^T = W^T H^T, with
// v_mfma_f32_16x16x32_bf16: the weights are the A operand (rows n), the
// activations the B operand (columns = rows m of the batch).  A lane's four
// results of output tile c are the outputs n = 16c + 4q + r (q = lane / 16,
// r = 0..3) of row m = lane % 16; bias, GELU and the rounding to bfloat16
// turn tiles 2p and 2p + 1 into the lane's eight operand values of the next
// layer's k slice p, i.e. the k order within each 32-wide slice is
//   slot 8q + j  <->  k = 4q + j (j < 4),  16 + 4q + (j - 4) (j >= 4),
// and the packed weights (k_pack_w16) use the same order.  So activations
// never touch LDS; the weights, a bfloat16 copy packed per layer as W^T
// [n][k] (k in that slot order, padded to a multiple of 32, n of the last
// layer to 48), pass through LDS in chunks of MLP_KC = 32 k,
// double-buffered: the next chunk (of this layer or the next) is read into
// registers while the current one feeds the MFMAs.  40 KB of LDS, 158
// VGPRs (three waves per SIMD); FP32 accumulation over the slices in order.  MODE 0 writes the outputs;
// MODE 1 computes the prescreen distance of every row.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
constexpr int TT = 1;  // 16-row tiles per wave (two: 256 registers and spills, no faster)
constexpr int MLP_RT = 64 * TT, MLP_KC = 32, MLP_WP = MLP_KC + 8;
constexpr int MLP_NL = 5;
constexpr int mlp_kp(int l) { return l == 0 ? 32 : 256; }   // padded K
constexpr int mlp_np(int l) { return l == MLP_NL - 1 ? 48 : 256; }  // padded N
constexpr int mlp_k(int l) { return l == 0 ? 5 : 256; }
constexpr int mlp_n(int l) { return l == MLP_NL - 1 ? 33 : 256; }
constexpr int64_t mlp_w16_off(int l)
{
    int64_t o = 0;
    for (int k = 0; k < l; ++k) o += (int64_t)mlp_np(k) * mlp_kp(k);
    return o;
}
constexpr int64_t MLP_W16_TOTAL = mlp_w16_off(MLP_NL);
constexpr int64_t mlp_offW_d(int l)
{
    int64_t o = 0;
    for (int k = 0; k < l; ++k) o += (int64_t)mlp_k(k) * mlp_n(k) + mlp_n(k);
    return o;
}
// the k of operand slot s (0..31) of a 32-wide slice (see above)
__host__ __device__ constexpr int mlp_slot_k(int s)
{
    return (s & 7) < 4 ? 4 * (s >> 3) + (s & 7) : 16 + 4 * (s >> 3) + (s & 7) - 4;
}

// bfloat16 copy of the weights, transposed, k in slot order, padded (zeros)
__global__ void k_pack_w16(const float* P, uint16_t* W16)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= MLP_W16_TOTAL) return;
    int l = 0;
    while (l + 1 < MLP_NL && e >= mlp_w16_off(l + 1)) ++l;
    const int64_t i = e - mlp_w16_off(l);
    const int n = (int)(i / mlp_kp(l)), kk = (int)(i % mlp_kp(l));
    const int k = (kk & ~31) + mlp_slot_k(kk & 31);
    const float v = (n < mlp_n(l) && k < mlp_k(l)) ? P[mlp_offW_d(l) + (int64_t)k * mlp_n(l) + n] : 0.0f;
    W16[e] = f2bf(v);
}

// weight chunk c of layer l (rows n < Np(l), slots [32c, 32c + 32)) as
// per-thread 16-byte pieces: global -> registers, registers -> LDS.  A row
// is 4 pieces; 256 rows are 1024 pieces, 4 per thread (the last layer's 48
// rows: the first 192 pieces).
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
struct WChunk {
    u32x4_t v[4];
};
__device__ __forceinline__ const uint16_t* mlp_wl(const uint16_t* W16, int l)
{
    return W16 + (l == 0 ? 0 : mlp_w16_off(1) + (int64_t)(l - 1) * 65536);
}
__device__ __forceinline__ int mlp_chunks(int l) { return l == 0 ? 1 : 256 / MLP_KC; }
// this thread's pieces of layer l's chunks: element offsets in the packed
// layer (chunk 0; chunk c adds 32 c) and in the LDS buffer (-1: none)
struct WAddr {
    int src[4], dst[4];
};
__device__ __forceinline__ void wchunk_addr(int l, int tid, WAddr& a)
{
    const int Kp = l == 0 ? 32 : 256, np4 = 4 * (l == MLP_NL - 1 ? 48 : 256);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = tid + 256 * q, ec = min(e, np4 - 1);  // clamped: always a valid piece
        a.src[q] = (ec >> 2) * Kp + 8 * (ec & 3);
        a.dst[q] = e < np4 ? (e >> 2) * MLP_WP + 8 * (e & 3) : -1;
    }
}
__device__ __forceinline__ void wchunk_load(const uint16_t* Wl, const WAddr& a, int c, WChunk& w)
{
#pragma unroll
    for (int q = 0; q < 4; ++q) w.v[q] = *reinterpret_cast<const u32x4_t*>(Wl + a.src[q] + MLP_KC * c);
}
__device__ __forceinline__ void wchunk_store(const WAddr& a, const WChunk& w, uint16_t* Ws)
{
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (a.dst[q] >= 0) *reinterpret_cast<u32x4_t*>(Ws + a.dst[q]) = w.v[q];
}
__device__ __forceinline__ uint32_t pack_bf2(float a, float b)
{
    return __builtin_bit_cast(uint32_t, bf16x2_t{(__bf16)a, (__bf16)b});
}

template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_mlp_fused(int64_t M, const float* __restrict__ X,
                                                   const uint16_t* __restrict__ W16, const float* __restrict__ P,
                                                   float* __restrict__ Y, const float* __restrict__ out_mu,
                                                   const float* __restrict__ out_sd, const float* __restrict__ obs,
                                                   int n_sum, float tol, float* __restrict__ dist,
                                                   uint8_t* __restrict__ keep)
{
    extern __shared__ __align__(16) uint16_t mlp_smem[];
    uint16_t* Wb = mlp_smem;  // [2][256][MLP_WP], double-buffered
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = lane >> 4;
    // this lane's rows of the batch (one per row tile) and output slots
    int64_t row[TT];
#pragma unroll
    for (int t = 0; t < TT; ++t) row[t] = (int64_t)blockIdx.x * MLP_RT + 16 * TT * wave + 16 * t + (lane & 15);
    // B operands of the current layer: 8 slices x 2 row tiles (layer 0: the
    // five inputs in slice 0, slot order, zeros elsewhere)
    u32x4_t hb[TT][8];
#pragma unroll
    for (int t = 0; t < TT; ++t) {
        float xin[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = mlp_slot_k(8 * q + j);
            xin[j] = (k < 5 && row[t] < M) ? X[row[t] * 5 + k] : 0.0f;
        }
        hb[t][0] = u32x4_t{pack_bf2(xin[0], xin[1]), pack_bf2(xin[2], xin[3]), pack_bf2(xin[4], xin[5]),
                           pack_bf2(xin[6], xin[7])};
#pragma unroll
        for (int p = 1; p < 8; ++p) hb[t][p] = u32x4_t{0u, 0u, 0u, 0u};
    }
    WChunk nxt;
    WAddr wa_cur, wa_next;
    wchunk_addr(0, tid, wa_cur);
    wchunk_load(mlp_wl(W16, 0), wa_cur, 0, nxt);
    wchunk_store(wa_cur, nxt, Wb);
    int g = 0;
#pragma unroll 1
    for (int l = 0; l < MLP_NL; ++l) {
        const int NT = l == MLP_NL - 1 ? 3 : 16;  // 16-row tiles of n
        const int nchunk = mlp_chunks(l);
        const uint16_t* Wl = mlp_wl(W16, l);
        const uint16_t* Wn = mlp_wl(W16, l + 1 < MLP_NL ? l + 1 : l);
        if (l + 1 < MLP_NL) wchunk_addr(l + 1, tid, wa_next);
        const float* bias = P + mlp_offW_d(l) + (int64_t)mlp_k(l) * mlp_n(l);
        // hidden layers start from the bias (C^T[n][m] = b[n]), the last
        // layer adds it to its 33 outputs
        f32x4_t acc[TT][16];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const f32x4_t b0 = l < MLP_NL - 1 ? *reinterpret_cast<const f32x4_t*>(bias + 16 * c + 4 * q)
                                              : f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < TT; ++t) acc[t][c] = b0;
        }
#pragma unroll
        for (int ch = 0; ch < 8; ++ch) {
            if (ch < nchunk) {
                // chunk g stored by every thread; the previous reader of
                // Wbuf[(g + 1) & 1] done
                __syncthreads();
                const bool same = ch + 1 < nchunk, more = same || l + 1 < MLP_NL;
                if (more) wchunk_load(same ? Wl : Wn, same ? wa_cur : wa_next, same ? ch + 1 : 0, nxt);
                const uint16_t* Ws = Wb + (g & 1) * 256 * MLP_WP;
#pragma unroll
                for (int c = 0; c < 16; ++c) {
                    if (c < NT) {
                        const bf16x8_t wv = __builtin_bit_cast(
                            bf16x8_t, *reinterpret_cast<const u32x4_t*>(Ws + (16 * c + (lane & 15)) * MLP_WP + 8 * q));
#pragma unroll
                        for (int t = 0; t < TT; ++t)
                            acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                wv, __builtin_bit_cast(bf16x8_t, hb[t][ch]), acc[t][c], 0, 0, 0);
                    }
                }
                if (more) wchunk_store(same ? wa_cur : wa_next, nxt, Wb + ((g + 1) & 1) * 256 * MLP_WP);
                ++g;
            }
        }
        if (l + 1 < MLP_NL) wa_cur = wa_next;
        if (l < MLP_NL - 1) {
            // GELU, bfloat16: tiles 2p, 2p + 1 -> slice p of the next
            // layer's operand
#pragma unroll
            for (int p = 0; p < 8; ++p) {
#pragma unroll
                for (int t = 0; t < TT; ++t) {
                    const f32x4_t a0 = acc[t][2 * p], a1 = acc[t][2 * p + 1];
                    hb[t][p] = u32x4_t{pack_bf2(gelu_f(a0[0]), gelu_f(a0[1])), pack_bf2(gelu_f(a0[2]), gelu_f(a0[3])),
                                       pack_bf2(gelu_f(a1[0]), gelu_f(a1[1])), pack_bf2(gelu_f(a1[2]), gelu_f(a1[3]))};
                }
            }
        } else if (MODE == 0) {
#pragma unroll
            for (int t = 0; t < TT; ++t)
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int n = 16 * c + 4 * q + r;
                        if (n < 33 && row[t] < M) Y[row[t] * 33 + n] = acc[t][c][r] + bias[n];
                    }
        } else {
            // prescreen: d = sqrt(mean_{n < n_sum} (mu_n + sd_n y_n - obs_n)^2)
#pragma unroll
            for (int t = 0; t < TT; ++t) {
                float sq = 0.f;
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int n = 16 * c + 4 * q + r;
                        if (n < n_sum) {
                            const float dv = fmaf(out_sd[n], acc[t][c][r] + bias[n], out_mu[n]) - obs[n];
                            sq = fmaf(dv, dv, sq);
                        }
                    }
                // the four lanes of row m (lane % 16 equal), fixed order
                sq += __shfl_xor(sq, 16, 64);
                sq += __shfl_xor(sq, 32, 64);
                if (q == 0 && row[t] < M) {
                    const float d = sqrtf(sq / (float)n_sum);
                    if (dist) dist[row[t]] = d;
                    keep[row[t]] = (d <= tol) ? 1 : 0;
                }
            }
        }
    }
}

size_t mlp_fused_lds_bytes() { return (size_t)(2 * 256 * MLP_WP) * sizeof(uint16_t); }
int64_t mlp_w16_count() { return MLP_W16_TOTAL; }

hipError_t launch_pack_w16(const float* P, uint16_t* W16, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_w16, dim3((unsigned)((MLP_W16_TOTAL + 255) / 256)), dim3(256), 0, st, P, W16);
    return hipGetLastError();
}

hipError_t launch_mlp_fused(int mode, int64_t M, const float* X, const uint16_t* W16, const float* P, float* Y,
                            const float* out_mu, const float* out_sd, const float* obs, int n_sum, float tol,
                            float* dist, uint8_t* keep, hipStream_t st)
{
    if (M <= 0) return hipSuccess;
    const size_t lds = mlp_fused_lds_bytes();
    const dim3 grid((unsigned)((M + MLP_RT - 1) / MLP_RT));
    if (mode == 0)
        hipLaunchKernelGGL(k_mlp_fused<0>, grid, dim3(256), lds, st, M, X, W16, P, Y, out_mu, out_sd, obs, n_sum, tol,
                           dist, keep);
    else
        hipLaunchKernelGGL(k_mlp_fused<1>, grid, dim3(256), lds, st, M, X, W16, P, Y, out_mu, out_sd, obs, n_sum, tol,
                           dist, keep);
    return hipGetLastError();
}

}  // namespace swim
