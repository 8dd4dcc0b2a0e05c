// swim_field.hip -- velocity (eq. BrV) and pressure (eq. BrP) of the
// regularized point forces of one system at arbitrary target points (Sec.
// 2.1), for flow and pressure pictures of a swimmer.
//
// Pressure: p = sum_i F_i . grad G_eps(x - X_i) with Delta G_eps = phi, the
// blob of the velocity kernel.  For a radial blob grad G_eps(x) =
// x m(r) / (2 pi r^2), m(r) the blob mass inside r; from (Delta - alpha^2) g
// = phi, m/(2 pi) = r g' - alpha^2 M, so for this blob
//   Stokes:   m = r^2 / R^2,
//   Brinkman: m = 1 - eps K1(alpha R) / (R K1(alpha eps)),  R^2 = r^2 + eps^2,
// and near contact (delta = r^2/eps^2 < 1/4) w = m / (2 pi r^2) is a power
// series in delta whose coefficients the host computes per call.
//
// One thread per target; the sources pass through LDS in tiles; every sum is
// accumulated in FP64.  The pair kernel: FP32 from the system's table (as in
// the forward runs), FP64 by direct evaluation.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swim_internal.h"
#include "swim_math.h"
#include "swim_pairsum.h"

namespace swim {

namespace {

constexpr int FIELD_TILE = 1024;

// pressure weight m(r) / (2 pi r^2) at t = r^2, in FP64
__device__ double field_weight(const FieldConst& fc, double t)
{
    const double delta = t * fc.inv_e2;
    if (fc.paper) {
        // m = 1 - eps^3/R^3:  w = (R^2 + R eps + eps^2) / (2 pi R^3 (R + eps))
        const double R2 = t + fc.e2, R = sqrt(R2);
        return fc.inv_2pi * (R2 + R * fc.eps + fc.e2) / (R2 * R * (R + fc.eps));
    }
    if (fc.stokes) return fc.inv_2pi / (t + fc.e2);
    if (delta < 0.25) {
        double w = fc.ser[FIELD_NSER - 1];
        for (int q = FIELD_NSER - 2; q >= 0; --q) w = fma(w, delta, fc.ser[q]);
        return w;
    }
    const double R = sqrt(t + fc.e2);
    double K0, K1, Q;
    bessel_k01_q_f64(fc.alpha * R, &K0, &K1, &Q);
    return fc.inv_2pi * (1.0 - fc.eps * K1 / (R * fc.K1e)) / t;
}

// FP32 table of the pressure weight on the kernel table's intervals of
// v = 1 + sigma t: the cubic through its FP64 values at the nodes 0, 1/4,
// 3/4, 1 of each interval (one thread per interval)
__global__ __launch_bounds__(256) void k_weight_table(FieldConst fc, float4* wt)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= TAB_N) return;
    const int e = i >> TAB_M, j = i & ((1 << TAB_M) - 1);
    const double a = ldexp(1.0, e);
    const double v0 = a * (1.0 + (double)j / (double)(1 << TAB_M)), hv = a / (double)(1 << TAB_M);
    const double un[4] = {0.0, 0.25, 0.75, 1.0};
    double f[4];
    for (int k = 0; k < 4; ++k) f[k] = field_weight(fc, fmax((v0 - 1.0 + hv * un[k]) * fc.c64.its, 1e-300));
    float c[4];
    cubic_lobatto(f, ldexp(1.0, -TAB_SHIFT), 1.0, c);
    wt[i] = make_float4(c[0], c[1], c[2], c[3]);
}

// tab (FP32 only): the system's kernel table, used for every pair inside it;
// beyond it the direct evaluation (FP64: the direct evaluation throughout)
template <typename T>
__global__ __launch_bounds__(256) void k_flow_field(int64_t n, const T* x, const T* y, const T* fx, const T* fy,
                                                    FieldConst fc, int64_t nt, const T* tx, const T* ty, T* u, T* v,
                                                    T* p, const TabSys* tab, const float4* wtab)
{
    __shared__ Src4<T> tile[FIELD_TILE];
    const SysConst<T> C = *reinterpret_cast<const SysConst<T>*>(sizeof(T) == 4 ? (const void*)&fc.c32
                                                                                   : (const void*)&fc.c64);
    const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool live = a < nt;
    const double X = live ? (double)tx[a] : 0.0, Y = live ? (double)ty[a] : 0.0;
    double su = 0.0, sv = 0.0, sp = 0.0, sfx = 0.0, sfy = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += FIELD_TILE) {
        const int m = (int)min<int64_t>(FIELD_TILE, n - j0);
        __syncthreads();
        for (int k = threadIdx.x; k < m; k += 256) {
            Src4<T> s;
            s.x = x[j0 + k];
            s.y = y[j0 + k];
            s.fx = fx[j0 + k];
            s.fy = fy[j0 + k];
            tile[k] = s;
        }
        __syncthreads();
        for (int k = 0; k < m; ++k) {
            const Src4<T> s = tile[k];
            sfx += (double)s.fx;
            sfy += (double)s.fy;
            const double dxd = X - (double)s.x, dyd = Y - (double)s.y;
            const T dx = (T)dxd, dy = (T)dyd;
            T Ht = (T)0, H2 = (T)0;
            const T t2 = fma_t(dx, dx, dy * dy);
            bool direct = true;
            if constexpr (sizeof(T) == 4) {
                if (tab) {
                    const uint32_t bits = tab_bits(t2, C.ts);
                    const uint32_t id = bits >> TAB_SHIFT;
                    if (id < TAB_END) {
                        tab_eval(tab->e[id - TAB_BIAS], tab_u(bits), Ht, H2);
                        H2 *= C.ts;  // the table holds H2 / sigma
                        direct = false;
                    }
                }
            }
            if (direct) kernel_eval<T>(C, t2, Ht, H2);
            const T fd = fma_t(s.fx, dx, s.fy * dy);
            su += (double)fma_t(Ht, s.fx, H2 * fd * dx);
            sv += (double)fma_t(Ht, s.fy, H2 * fd * dy);
            // pressure weight m(r) / (2 pi r^2): FP32 from the weight table
            // inside it, else in FP64
            const double t = fma(dxd, dxd, dyd * dyd);
            double w = 0.0;
            bool wdirect = true;
            if constexpr (sizeof(T) == 4) {
                if (wtab) {
                    const uint32_t bits = tab_bits(t2, C.ts);
                    const uint32_t id = bits >> TAB_SHIFT;
                    if (id < TAB_END) {
                        const float4 c = wtab[id - TAB_BIAS];
                        const float uu = tab_u(bits);
                        w = (double)fmaf(fmaf(fmaf(c.w, uu, c.z), uu, c.y), uu, c.x);
                        wdirect = false;
                    }
                }
            }
            if (wdirect) w = field_weight(fc, t);
            sp = fma((double)s.fx * dxd + (double)s.fy * dyd, w, sp);
        }
    }
    if (live) {
        u[a] = (T)fma(fc.h1c, sfx, su);
        v[a] = (T)fma(fc.h1c, sfy, sv);
        p[a] = (T)sp;
    }
}

}  // namespace

hipError_t launch_flow_field(int dtype, int64_t n, const void* x, const void* y, const void* fx, const void* fy,
                             const FieldConst& fc, int64_t nt, const void* tx, const void* ty, void* u, void* v,
                             void* p, const void* tab, void* wtab, hipStream_t st)
{
    if (nt == 0) return hipSuccess;
    if (wtab) hipLaunchKernelGGL(k_weight_table, dim3((TAB_N + 255) / 256), dim3(256), 0, st, fc, (float4*)wtab);
    const unsigned nb = (unsigned)((nt + 255) / 256);
    if (dtype == 0)
        hipLaunchKernelGGL(k_flow_field<float>, dim3(nb), dim3(256), 0, st, n, (const float*)x, (const float*)y,
                           (const float*)fx, (const float*)fy, fc, nt, (const float*)tx, (const float*)ty, (float*)u,
                           (float*)v, (float*)p, (const TabSys*)tab, (const float4*)wtab);
    else
        hipLaunchKernelGGL(k_flow_field<double>, dim3(nb), dim3(256), 0, st, n, (const double*)x, (const double*)y,
                           (const double*)fx, (const double*)fy, fc, nt, (const double*)tx, (const double*)ty,
                           (double*)u, (double*)v, (double*)p, (const TabSys*)nullptr,
                           (const float4*)nullptr);
    return hipGetLastError();
}

}  // namespace swim
