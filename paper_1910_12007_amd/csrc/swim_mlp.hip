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
#include <math.h>
#include <stdint.h>

#include "swim_internal.h"

namespace swim {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float gelu_f(float x)
{
    return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad_f(float x)
{
    const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
    const float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
    return fmaf(x, pdf, cdf);
}

// C(m, n) = sum_k A(m, k) B(k, n), A(m, k) = A[m*sam + k*sak],
// B(k, n) = B[k*sbk + n*sbn], C(m, n) at C[m*ldc + n].  Epilogues:
//   MLP_EPI_PLAIN  C = acc
//   MLP_EPI_GELU   pre = acc + bias[n] -> C;  H = gelu(pre) -> aux
//   MLP_EPI_BIAS   C = acc + bias[n]
//   MLP_EPI_DGELU  C = acc * gelu'(aux(m, n))   (aux = pre-activations)
// Workgroup tile 64 x 64 (4 waves of 32 x 32 = 2 x 2 MFMA tiles), k chunks of 32.
constexpr int GT = 64, GK = 32, GPAD = 8;

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const float* __restrict__ A, int64_t sam,
                                                   int64_t sak, const float* __restrict__ B, int64_t sbk, int64_t sbn,
                                                   float* __restrict__ C, int64_t ldc, const float* __restrict__ bias,
                                                   float* __restrict__ aux)
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
    for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
        for (int i = 0; i < (GT * GK) / 256; ++i) {
            const int e = tid + 256 * i;
            const int r = e / GK, kk = e % GK;
            const int m = m0 + r, k = k0 + kk;
            As[r][kk] = (m < M && k < K) ? f2bf(A[(int64_t)m * sam + (int64_t)k * sak]) : (uint16_t)0;
        }
#pragma unroll
        for (int i = 0; i < (GT * GK) / 256; ++i) {
            const int e = tid + 256 * i;
            const int kk = e / GT, c = e % GT;
            const int n = n0 + c, k = k0 + kk;
            Bs[c][kk] = (n < N && k < K) ? f2bf(B[(int64_t)k * sbk + (int64_t)n * sbn]) : (uint16_t)0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < GK; ks += 16) {
            // operand layout of the 16x16x16 MFMA: lane l holds row (l % 16)
            // and k = 4 (l / 16) .. 4 (l / 16) + 3 of its 16-wide k slice
            const int kq = ks + 4 * (lane >> 4);
            bf16x4_t av[2], bv[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const uint16_t* pa = &As[wm + 16 * t + (lane & 15)][kq];
                const uint16_t* pb = &Bs[wn + 16 * t + (lane & 15)][kq];
                av[t] = bf16x4_t{(short)pa[0], (short)pa[1], (short)pa[2], (short)pa[3]};
                bv[t] = bf16x4_t{(short)pb[0], (short)pb[1], (short)pb[2], (short)pb[3]};
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
                float v = acc[a][b][r];
                const int64_t o = (int64_t)m * ldc + n;
                if (EPI == 1) {
                    v += bias[n];
                    C[o] = v;
                    aux[o] = gelu_f(v);
                } else if (EPI == 2) {
                    C[o] = v + bias[n];
                } else if (EPI == 3) {
                    C[o] = v * gelu_grad_f(aux[o]);
                } else {
                    C[o] = v;
                }
            }
}

// out[n] = sum_m A[m*lda + n]  (bias gradients), fixed summation order
__global__ void k_colsum(int M, int N, const float* A, int64_t lda, float* out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += A[(int64_t)m * lda + n];
    out[n] = s;
}

// dY = 2 (Y - T) / (M * N); per-row squared error (for the loss)
__global__ void k_mse_grad(int M, int N, const float* Y, const float* T, float* dY, float* rowsq)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const float sc = 2.0f / ((float)M * (float)N);
    float sq = 0.f;
    for (int n = 0; n < N; ++n) {
        const float d = Y[(int64_t)m * N + n] - T[(int64_t)m * N + n];
        dY[(int64_t)m * N + n] = sc * d;
        sq = fmaf(d, d, sq);
    }
    if (rowsq) rowsq[m] = sq;
}

// rows of X and T picked by perm[0..M) into the batch buffers
__global__ void k_gather_rows(int M, const int32_t* perm, const float* X, int nx, const float* T, int nt, float* Xb,
                              float* Tb)
{
    const int m = blockIdx.x;
    if (m >= M) return;
    const int64_t src = perm[m];
    for (int c = threadIdx.x; c < nx + nt; c += blockDim.x) {
        if (c < nx) Xb[(int64_t)m * nx + c] = X[src * nx + c];
        else Tb[(int64_t)m * nt + c - nx] = T[src * nt + c - nx];
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
                            int64_t sbk, int64_t sbn, float* C, int64_t ldc, const float* bias, float* aux,
                            hipStream_t st)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    const dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
    switch (epi) {
    case 0: hipLaunchKernelGGL(k_gemm_bf16<0>, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, aux); break;
    case 1: hipLaunchKernelGGL(k_gemm_bf16<1>, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, aux); break;
    case 2: hipLaunchKernelGGL(k_gemm_bf16<2>, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, aux); break;
    case 3: hipLaunchKernelGGL(k_gemm_bf16<3>, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, aux); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_colsum(int M, int N, const float* A, int64_t lda, float* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, st, M, N, A, lda, out);
    return hipGetLastError();
}

hipError_t launch_mse_grad(int M, int N, const float* Y, const float* T, float* dY, float* rowsq, hipStream_t st)
{
    hipLaunchKernelGGL(k_mse_grad, dim3((M + 255) / 256), dim3(256), 0, st, M, N, Y, T, dY, rowsq);
    return hipGetLastError();
}

hipError_t launch_gather_rows(int M, const int32_t* perm, const float* X, int nx, const float* T, int nt, float* Xb,
                              float* Tb, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_rows, dim3(M), dim3(64), 0, st, M, perm, X, nx, T, nt, Xb, Tb);
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

}  // namespace swim
