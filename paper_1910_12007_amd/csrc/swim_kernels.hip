// swim_kernels.hip -- gfx950 kernels of the batched filament-swimmer forward
// model (Sec. 2.1 and the Appendix): preferred curvature and elastic forces
// (eqs. EFB, curva, EFT, Fenergy), the dense regularized-Brinkmanlet velocity
// sum (eq. BrV), the forward-Euler no-slip update, head observations, and the
// ABC distance / tolerance kernels around it.
//
// Precision: every kernel is one template instantiated for float and double.
// In float the filament positions are carried as (hi, lo) pairs updated by an
// error-free TwoSum, so the segment vectors that drive the stiff stretching
// springs keep full relative precision.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swim_internal.h"
#include "swim_math.h"

namespace swim {

constexpr int32_t SWIM_ST_BADPARAM_ = 3;

template <typename T> struct alignas(4 * sizeof(T)) Src4 {
    T x, y, fx, fy;
};

// LDS ordering between lanes of one wavefront: a wavefront's LDS operations
// execute in issue order, so a compiler-level fence around a wave barrier is
// enough to order a store by one lane before a later load by another.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ float sin_t(float x) { return sinf(x); }
__device__ __forceinline__ double sin_t(double x) { return sin(x); }
__device__ __forceinline__ bool bad_t(float x) { return !(fabsf(x) <= 1e3f); }
__device__ __forceinline__ bool bad_t(double x) { return !(fabs(x) <= 1e3); }

// parameters of one filament, in the working precision
template <typename T> struct FilP {
    T Sb, Ss, b, om, kw, ph, ds, inv2ds, invds2;
    int N;
};

template <typename T>
__device__ __forceinline__ FilP<T> load_filp(const double* params, int64_t f, int N)
{
    const double* P = params + 9 * f;
    FilP<T> q;
    q.Sb = (T)P[1];
    q.Ss = (T)P[2];
    q.b = (T)P[3];
    q.om = (T)P[4];
    q.kw = (T)P[5];
    q.ph = (T)P[6];
    const double ds = 1.0 / (double)(N - 1);
    q.ds = (T)ds;
    q.inv2ds = (T)(0.5 / ds);
    q.invds2 = (T)(1.0 / (ds * ds));
    q.N = N;
    return q;
}

// Force F_p = -dE/dX_p on point p of one filament from the discrete tensile
// energy S_s sum_k (l_k/ds - 1)^2 ds and bending energy
// S_b sum_{k=1}^{N-2} (kappa_k - kappa0_k)^2 ds (Appendix EFT, EFB, curva;
// centred differences, interior nodes only).  seg(k, dx, dy) returns the
// segment vector X_{k+1} - X_k.
template <typename T, typename Seg>
__device__ __forceinline__ void point_force(const Seg& seg, int p, const FilP<T>& q, T t, T& Fx, T& Fy)
{
    const int N = q.N;
    T dx[4], dy[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int k = p - 2 + c;
        if (k >= 0 && k <= N - 2) {
            seg(k, dx[c], dy[c]);
        } else {
            dx[c] = (T)0;
            dy[c] = (T)0;
        }
    }
    Fx = (T)0;
    Fy = (T)0;
    // stretching: +tau_p (segment p) - tau_{p-1} (segment p-1)
#pragma unroll
    for (int c = 1; c <= 2; ++c) {
        const int k = p - 2 + c;
        if (k >= 0 && k <= N - 2) {
            const T l = sqrt_t(fma_t(dx[c], dx[c], dy[c] * dy[c]));
            const T co = (T)2 * q.Ss * (l / q.ds - (T)1) / l;
            const T sg = (c == 2) ? (T)1 : (T)-1;
            Fx = fma_t(sg * co, dx[c], Fx);
            Fy = fma_t(sg * co, dy[c], Fy);
        }
    }
    // bending: curvature nodes k = p-1, p, p+1
#pragma unroll
    for (int kk = -1; kk <= 1; ++kk) {
        const int k = p + kk;
        if (k < 1 || k > N - 2) continue;
        const int ca = kk + 1, cb = kk + 2;  // d_{k-1}, d_k
        const T a = (dx[cb] + dx[ca]) * q.inv2ds;
        const T bb = (dy[cb] + dy[ca]) * q.inv2ds;
        const T pp = (dx[cb] - dx[ca]) * q.invds2;
        const T qq = (dy[cb] - dy[ca]) * q.invds2;
        const T S = fma_t(a, a, bb * bb);
        const T rS = (T)1 / S;
        const T rS32 = rS / sqrt_t(S);
        const T num = fma_t(qq, a, -pp * bb);
        const T kap = num * rS32;
        const T k0 = -q.kw * q.kw * q.b * sin_t(fma_t(q.kw * q.ds, (T)k, q.ph - q.om * t));
        const T co = (T)2 * q.Sb * (kap - k0) * q.ds;
        const T n3 = (T)3 * num * rS32 * rS;
        const T dka = qq * rS32 - a * n3;
        const T dkb = -pp * rS32 - bb * n3;
        const T dkp = -bb * rS32;
        const T dkq = a * rS32;
        T gx, gy;
        if (kk == 1) {          // p = k - 1
            gx = fma_t(-dka, q.inv2ds, dkp * q.invds2);
            gy = fma_t(-dkb, q.inv2ds, dkq * q.invds2);
        } else if (kk == 0) {   // p = k
            gx = (T)-2 * dkp * q.invds2;
            gy = (T)-2 * dkq * q.invds2;
        } else {                // p = k + 1
            gx = fma_t(dka, q.inv2ds, dkp * q.invds2);
            gy = fma_t(dkb, q.inv2ds, dkq * q.invds2);
        }
        Fx = fma_t(-co, gx, Fx);
        Fy = fma_t(-co, gy, Fy);
    }
}

// Accumulate the velocity sum of eq. (BrV) over sources src[0..n) for the
// TPL targets (xi, yi) of this lane; the constant H1(0) part is added by the
// caller once as h1c * sum_j F_j.  FP64 evaluates the kernel functions
// directly; FP32 reads them from the system's table in LDS (tab), with the
// direct evaluation for pairs beyond its last octave.
template <typename T, int TPL>
__device__ __forceinline__ void pair_accumulate(const SysConst<T>& C, const TabSys* tab, const Src4<T>* src, int n,
                                                const T (&xi)[TPL], const T (&yi)[TPL],
                                                T (&ax)[TPL], T (&ay)[TPL])
{
    if constexpr (sizeof(T) == 4) {
        // table pass; a pair beyond the table contributes nothing here and
        // flags its lane
        bool far = false;
        const float ie2 = C.inv_e2;
        for (int j = 0; j < n; ++j) {
            const Src4<T> s = src[j];
#pragma unroll
            for (int k = 0; k < TPL; ++k) {
                const T dx = xi[k] - s.x, dy = yi[k] - s.y;
                const T t = fma_t(dx, dx, dy * dy);
                float u, Ht, H2;
                const uint32_t id = tab_locate(t, ie2, u);
                const bool in = id < (uint32_t)TAB_N;
                far = far || !in;
                tab_eval(tab->e[in ? id : 0u], u, Ht, H2);
                Ht = in ? Ht : 0.0f;
                H2 = in ? H2 : 0.0f;
                const T h2fd = H2 * fma_t(s.fx, dx, s.fy * dy);
                ax[k] = fma_t(Ht, s.fx, fma_t(h2fd, dx, ax[k]));
                ay[k] = fma_t(Ht, s.fy, fma_t(h2fd, dy, ay[k]));
            }
        }
        // direct evaluation of the flagged pairs, only where a lane has one
        if (__any(far)) {
            for (int j = 0; j < n; ++j) {
                const Src4<T> s = src[j];
#pragma unroll
                for (int k = 0; k < TPL; ++k) {
                    const T dx = xi[k] - s.x, dy = yi[k] - s.y;
                    const T t = fma_t(dx, dx, dy * dy);
                    float u;
                    if (tab_locate(t, ie2, u) >= (uint32_t)TAB_N) {
                        T Ht, H2;
                        kernel_eval<T>(C, t, Ht, H2);
                        const T h2fd = H2 * fma_t(s.fx, dx, s.fy * dy);
                        ax[k] = fma_t(Ht, s.fx, fma_t(h2fd, dx, ax[k]));
                        ay[k] = fma_t(Ht, s.fy, fma_t(h2fd, dy, ay[k]));
                    }
                }
            }
        }
    } else {
        for (int j = 0; j < n; ++j) {
            const Src4<T> s = src[j];
#pragma unroll
            for (int k = 0; k < TPL; ++k) {
                const T dx = xi[k] - s.x, dy = yi[k] - s.y;
                const T t = fma_t(dx, dx, dy * dy);
                T Ht, H2;
                kernel_eval<T>(C, t, Ht, H2);
                const T h2fd = H2 * fma_t(s.fx, dx, s.fy * dy);
                ax[k] = fma_t(Ht, s.fx, fma_t(h2fd, dx, ax[k]));
                ay[k] = fma_t(Ht, s.fy, fma_t(h2fd, dy, ay[k]));
            }
        }
    }
}

// FP32 pair sum with FP64 accumulation, for lanes that sum whole large
// systems.  Filament forces alternate in sign with magnitudes far above the
// velocity they produce (bending forces ~4e2 against velocities ~10 for
// N = 512), so the FP32 rounding of Ht * F_j (Ht ~ 0.3) and of an FP32
// running sum each leave ~1e-5 of relative error over thousands of sources.
// Here Ht = h0 + (h0lo + increment) keeps the constant term in two floats,
// the small in-interval increment is evaluated in FP32, and the products
// (exact in FP64) accumulate in FP64, which this chip issues at the FP32
// rate.  The H2 term stays in FP32 up to its product.
template <int TPL>
__device__ __forceinline__ void pair_accumulate_x(const SysConst<float>& C, const TabSys* tab,
                                                  const Src4<float>* src, int n, const float (&xi)[TPL],
                                                  const float (&yi)[TPL], double (&ax)[TPL], double (&ay)[TPL])
{
    bool far = false;
    const float ie2 = C.inv_e2;
    for (int j = 0; j < n; ++j) {
        const Src4<float> s = src[j];
        const double fx = s.fx, fy = s.fy;
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
            const float dx = xi[k] - s.x, dy = yi[k] - s.y;
            const float t = fmaf(dx, dx, dy * dy);
            float u;
            const uint32_t id = tab_locate(t, ie2, u);
            const bool in = id < (uint32_t)TAB_N;
            far = far || !in;
            const uint32_t ic = in ? id : 0u;
            const TabE& e = tab->e[ic];
            const float inc = u * fmaf(fmaf(e.h[3], u, e.h[2]), u, e.h[1]);
            const float hi = in ? e.h[0] : 0.0f;
            const float lo = in ? tab->h0lo[ic] + inc : 0.0f;
            const float H2 = in ? fmaf(fmaf(fmaf(e.g[3], u, e.g[2]), u, e.g[1]), u, e.g[0]) : 0.0f;
            const float h2fd = H2 * fmaf(s.fx, dx, s.fy * dy);
            ax[k] = fma((double)hi, fx, fma((double)lo, fx, fma((double)h2fd, (double)dx, ax[k])));
            ay[k] = fma((double)hi, fy, fma((double)lo, fy, fma((double)h2fd, (double)dy, ay[k])));
        }
    }
    if (__any(far)) {
        for (int j = 0; j < n; ++j) {
            const Src4<float> s = src[j];
#pragma unroll
            for (int k = 0; k < TPL; ++k) {
                const float dx = xi[k] - s.x, dy = yi[k] - s.y;
                const float t = fmaf(dx, dx, dy * dy);
                float u;
                if (tab_locate(t, ie2, u) >= (uint32_t)TAB_N) {
                    float Ht, H2;
                    kernel_eval<float>(C, t, Ht, H2);
                    const float h2fd = H2 * fmaf(s.fx, dx, s.fy * dy);
                    ax[k] = fma((double)Ht, (double)s.fx, fma((double)h2fd, (double)dx, ax[k]));
                    ay[k] = fma((double)Ht, (double)s.fy, fma((double)h2fd, (double)dy, ay[k]));
                }
            }
        }
    }
}

// copy one system's FP32 kernel table from HBM into LDS (nthreads threads)
__device__ __forceinline__ void tab_load(const TabSys* g, TabSys* tab, int tid, int nthreads)
{
    const float4* src = reinterpret_cast<const float4*>(g);
    float4* dst = reinterpret_cast<float4*>(tab);
    constexpr int NV = (int)(sizeof(TabSys) / sizeof(float4));
    for (int i = tid; i < NV; i += nthreads) dst[i] = src[i];
}

// error-free (hi, lo) += d  (TwoSum, then renormalize)
template <typename T> __device__ __forceinline__ void acc2(T& hi, T& lo, T d)
{
    const T s = hi + d;
    const T bv = s - hi;
    const T e = (hi - (s - bv)) + (d - bv);
    const T l = lo + e;
    const T h = s + l;
    lo = l - (h - s);
    hi = h;
}

// ---------------------------------------------------------------------------
// set-up
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_sysconst(int64_t n, const double* alpha, const double* eps, SysConst<T>* out,
                           SysConst<double>* out64)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    sysconst_compute<T>(alpha[i], eps[i], out + i);
    if (out64) sysconst_compute<double>(alpha[i], eps[i], out64 + i);
}

// per-system constants of a forward batch; systems whose parameters leave
// the kernel's domain (alpha < 0, alpha*eps > 1, non-finite rows) are
// flagged SWIM_ST_BADPARAM_ and skipped by the run kernels.
template <typename T>
__global__ void k_sysconst_batch(int64_t n, const int64_t* sw_off, const int32_t* npt, const double* params,
                                 double eps_over_ds, SysConst<T>* out, SysConst<double>* out64, int32_t* status)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double alpha = params[9 * sw_off[s]];
    const double eps = eps_over_ds / (double)(npt[s] - 1);
    bool ok = isfinite(alpha) && alpha >= 0.0 && alpha * eps <= 1.0;
    for (int64_t f = sw_off[s]; f < sw_off[s + 1]; ++f)
        for (int c = 0; c < 9; ++c) ok = ok && isfinite(params[9 * f + c]);
    status[s] = ok ? 0 : SWIM_ST_BADPARAM_;
    sysconst_compute<T>(ok ? alpha : 0.0, eps, out + s);
    if (out64) sysconst_compute<double>(ok ? alpha : 0.0, eps, out64 + s);
}

// FP32 kernel tables of systems [s0, s0 + n), one thread per interval; the
// FP64 evaluation's registers stay out of the kernels that use the tables
__global__ __launch_bounds__(64) void k_table_build(int64_t s0, int64_t n, const SysConst<double>* sysc64, TabSys* tab)
{
    const int64_t e = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int64_t s = s0 + e / TAB_N;
    const int i = (int)(e % TAB_N);
    if (e >= n * TAB_N) return;
    const SysConst<double>& C = sysc64[s];
    tab_interval(C, C.e2, i, tab[s].e[i], &tab[s].h0lo[i]);
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// standalone dense velocity sum (one evaluation of eq. BrV)
// block b handles targets [blk_first[b], +256*TPL) of system blk_sys[b];
// sources stream through LDS in tiles of 256 points.
// ---------------------------------------------------------------------------
template <typename T, int TPL>
__global__ __launch_bounds__(256) void k_pair_velocity(const int64_t* blk_sys, const int64_t* blk_first,
                                                        const int64_t* pt_off, const SysConst<T>* sysc,
                                                        const TabSys* tabs, const T* x, const T* y, const T* fx,
                                                        const T* fy, T* ux, T* uy)
{
    __shared__ Src4<T> tile[256];
    __shared__ double red[2][4];
    __shared__ TabSys tab_s[1];
    TabSys* tab = tab_s;
    const int tid = threadIdx.x;
    const int64_t s = blk_sys[blockIdx.x];
    const int64_t first = blk_first[blockIdx.x];
    const int64_t p0 = pt_off[s];
    const int64_t n = pt_off[s + 1] - p0;
    const SysConst<T> C = sysc[s];
    if constexpr (sizeof(T) == 4) tab_load(tabs + s, tab, tid, 256);
    // FP32 accumulates in FP64 (pair_accumulate_x); FP64 in FP64
    T xi[TPL], yi[TPL], ax[TPL], ay[TPL];
    double axd[TPL], ayd[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int64_t i = first + tid + 256 * k;
        xi[k] = i < n ? x[p0 + i] : (T)0;
        yi[k] = i < n ? y[p0 + i] : (T)0;
        ax[k] = (T)0;
        ay[k] = (T)0;
        axd[k] = ayd[k] = 0.0;
    }
    // sum of the forces in FP64: it multiplies H1(0) in every target's
    // velocity, and the forces of a filament cancel to a small total
    double sfx = 0.0, sfy = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += 256) {
        const int64_t j = j0 + tid;
        Src4<T> v;
        if (j < n) {
            v.x = x[p0 + j];
            v.y = y[p0 + j];
            v.fx = fx[p0 + j];
            v.fy = fy[p0 + j];
            sfx += v.fx;
            sfy += v.fy;
        } else {
            v.x = v.y = v.fx = v.fy = (T)0;
        }
        __syncthreads();
        tile[tid] = v;
        __syncthreads();
        const int m = (int)((n - j0) < 256 ? (n - j0) : 256);
        if constexpr (sizeof(T) == 4)
            pair_accumulate_x<TPL>(C, tab, tile, m, xi, yi, axd, ayd);
        else
            pair_accumulate<T, TPL>(C, tab, tile, m, xi, yi, ax, ay);
    }
    sfx = wave_sum(sfx);
    sfy = wave_sum(sfy);
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = sfx;
        red[1][tid >> 6] = sfy;
    }
    __syncthreads();
    const double SFxd = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const double SFyd = red[1][0] + red[1][1] + red[1][2] + red[1][3];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int64_t i = first + tid + 256 * k;
        if (i < n) {
            if constexpr (sizeof(T) == 4) {
                ux[p0 + i] = (T)fma((double)C.h1c, SFxd, axd[k]);
                uy[p0 + i] = (T)fma((double)C.h1c, SFyd, ayd[k]);
            } else {
                ux[p0 + i] = fma_t(C.h1c, (T)SFxd, ax[k]);
                uy[p0 + i] = fma_t(C.h1c, (T)SFyd, ay[k]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// standalone elastic forces at time t (one thread per point)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_forces(int64_t n_fil, const int64_t* fil_off, const int32_t* npt, const double* params,
                         double t, const T* x, const T* y, T* fx, T* fy)
{
    const int64_t f = blockIdx.y;
    if (f >= n_fil) return;
    const int N = npt[f];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t b = fil_off[f];
    const FilP<T> q = load_filp<T>(params, f, N);
    auto seg = [&](int k, T& dx, T& dy) {
        dx = x[b + k + 1] - x[b + k];
        dy = y[b + k + 1] - y[b + k];
    };
    T Fx, Fy;
    point_force<T>(seg, p, q, (T)t, Fx, Fy);
    fx[b + p] = Fx;
    fy[b + p] = Fy;
}

// ---------------------------------------------------------------------------
// persistent forward run: one workgroup of WPS wavefronts per system, systems
// taken from a longest-first work queue; every time step (forces -> velocity
// sum -> Euler) stays inside the workgroup, positions and forces live in LDS.
// Each wavefront sums over 1/WPS of the sources for all targets; partial
// velocities are reduced through LDS in a fixed order (deterministic).
// ---------------------------------------------------------------------------
template <typename T> struct FwdLds {
    TabSys* tab;   // FP32 kernel table (FP32 runs)
    Src4<T>* src;  // [NMAX] positions (hi) and forces
    T* lox;        // [NMAX] lo parts
    T* loy;
    T* part;       // [WPS][2][NMAX] partial velocities (WPS > 1)
    T* red;        // [2][WPS] wave partial sums of the forces
};

template <typename T, int TPL, int WPS>
__device__ void run_system(const Batch& b, const Run& r, int s, const FwdLds<T>& L, T* obs, T* speed,
                           int32_t* status, int32_t* steps_done)
{
    constexpr bool COMP = sizeof(T) == 4;
    constexpr int NMAX = 64 * TPL, NT = 64 * WPS, OWN = (NMAX + NT - 1) / NT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int N = b.npt[s];
    const int nsw = b.nswim[s];
    const int n = N * nsw;
    const int64_t f0 = b.sw_off[s];
    if (status[s] == SWIM_ST_BADPARAM_) {
        // parameters outside the kernel's domain: no run, NaN outputs
        for (int m = tid; m < nsw; m += NT) {
            T* q = obs + (f0 + m) * (int64_t)r.n_obs * 2;
            for (int o = 0; o < 2 * r.n_obs; ++o) q[o] = (T)NAN;
            speed[f0 + m] = (T)NAN;
        }
        if (tid == 0 && steps_done) steps_done[s] = 0;
        __syncthreads();
        return;
    }
    const SysConst<T> C = ((const SysConst<T>*)b.sysc)[s];
    const double dsd = 1.0 / (double)(N - 1);
    if constexpr (COMP) tab_load((const TabSys*)b.tab + s, L.tab, tid, NT);

    // owned points i = tid + NT*q: positions as (hi, lo)
    T xh[OWN], yh[OWN], xl[OWN], yl[OWN];
#pragma unroll
    for (int q = 0; q < OWN; ++q) {
        const int i = tid + NT * q;
        const bool own = i < n;
        const int m = own ? i / N : 0;
        const int p = own ? i - m * N : 0;
        const double X = b.params[9 * (f0 + m) + 7] + (double)p * dsd;
        const double Y = b.params[9 * (f0 + m) + 8];
        xh[q] = (T)X;
        yh[q] = (T)Y;
        xl[q] = COMP ? (T)(X - (double)xh[q]) : (T)0;
        yl[q] = COMP ? (T)(Y - (double)yh[q]) : (T)0;
        if (own) {
            L.src[i].x = xh[q];
            L.src[i].y = yh[q];
            L.lox[i] = xl[q];
            L.loy[i] = yl[q];
            if (p == N - 1) {
                // samples a stopped run never reaches stay NaN
                T* o = obs + (f0 + m) * (int64_t)r.n_obs * 2;
                for (int k = 0; k < 2 * r.n_obs; ++k) o[k] = (T)NAN;
            }
        }
    }
    __syncthreads();
    int st = 0, done = r.steps;
    const T dt = (T)r.dt;
    const int chunk = (n + WPS - 1) / WPS;
    const int j0 = min(n, wave * chunk), j1 = min(n, j0 + chunk);
    for (int step = 0; step < r.steps; ++step) {
        const T t = (T)((double)step * r.dt);
        // forces of the owned points (reads positions only)
        // force sums: one point per thread, then a 64-lane tree and the
        // WPS wave sums (short sums, FP32 is enough here)
        T sfx = (T)0, sfy = (T)0;
#pragma unroll
        for (int q = 0; q < OWN; ++q) {
            const int i = tid + NT * q;
            if (i < n) {
                const int m = i / N, p = i - m * N;
                const int base = m * N;
                const FilP<T> fp = load_filp<T>(b.params, f0 + m, N);
                auto seg = [&](int kk, T& dx, T& dy) {
                    const int a = base + kk, c = base + kk + 1;
                    dx = (L.src[c].x - L.src[a].x) + (COMP ? L.lox[c] - L.lox[a] : (T)0);
                    dy = (L.src[c].y - L.src[a].y) + (COMP ? L.loy[c] - L.loy[a] : (T)0);
                };
                T Fx, Fy;
                point_force<T>(seg, p, fp, t, Fx, Fy);
                L.src[i].fx = Fx;
                L.src[i].fy = Fy;
                sfx += Fx;
                sfy += Fy;
            }
        }
        sfx = wave_sum(sfx);
        sfy = wave_sum(sfy);
        if (lane == 0) {
            L.red[wave] = sfx;
            L.red[WPS + wave] = sfy;
        }
        __syncthreads();
        T SFx = (T)0, SFy = (T)0;
#pragma unroll
        for (int w = 0; w < WPS; ++w) {
            SFx += L.red[w];
            SFy += L.red[WPS + w];
        }
        // pair sum: this wave's share of the sources, all targets
        T xi[TPL], yi[TPL], ax[TPL], ay[TPL];
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
            const int i = lane + 64 * k;
            xi[k] = i < n ? L.src[i].x : (T)0;
            yi[k] = i < n ? L.src[i].y : (T)0;
            ax[k] = ay[k] = (T)0;
        }
        pair_accumulate<T, TPL>(C, L.tab, L.src + j0, j1 - j0, xi, yi, ax, ay);
        if constexpr (WPS > 1) {
#pragma unroll
            for (int k = 0; k < TPL; ++k) {
                const int i = lane + 64 * k;
                if (i < n) {
                    L.part[(wave * 2 + 0) * NMAX + i] = ax[k];
                    L.part[(wave * 2 + 1) * NMAX + i] = ay[k];
                }
            }
            __syncthreads();
        }
        // Euler update of the owned points
        int bad = 0;
#pragma unroll
        for (int q = 0; q < OWN; ++q) {
            const int i = tid + NT * q;
            if (i >= n) continue;
            T ux, uy;
            if constexpr (WPS > 1) {
                ux = (T)0;
                uy = (T)0;
#pragma unroll
                for (int w = 0; w < WPS; ++w) {
                    ux += L.part[(w * 2 + 0) * NMAX + i];
                    uy += L.part[(w * 2 + 1) * NMAX + i];
                }
            } else {
                ux = ax[q];
                uy = ay[q];
            }
            ux = fma_t(C.h1c, SFx, ux);
            uy = fma_t(C.h1c, SFy, uy);
            if (COMP) {
                acc2(xh[q], xl[q], dt * ux);
                acc2(yh[q], yl[q], dt * uy);
            } else {
                xh[q] = fma_t(dt, ux, xh[q]);
                yh[q] = fma_t(dt, uy, yh[q]);
            }
            if (bad_t(xh[q]) || bad_t(yh[q])) bad = (isfinite(xh[q]) && isfinite(yh[q])) ? 2 : 1;
        }
        // every read of the old positions is done after this barrier
        const int any_bad = __syncthreads_or(bad);
#pragma unroll
        for (int q = 0; q < OWN; ++q) {
            const int i = tid + NT * q;
            if (i < n) {
                L.src[i].x = xh[q];
                L.src[i].y = yh[q];
                L.lox[i] = xl[q];
                L.loy[i] = yl[q];
            }
        }
        if (any_bad) {
            st = __syncthreads_or(bad == 1) ? 1 : 2;
            done = step + 1;
            break;
        }
        __syncthreads();
        if (r.obs_every > 0 && (step + 1) % r.obs_every == 0) {
            const int o = (step + 1) / r.obs_every - 1;
#pragma unroll
            for (int q = 0; q < OWN; ++q) {
                const int i = tid + NT * q;
                if (i < n && (i % N) == N - 1) {
                    T* d = obs + ((f0 + i / N) * (int64_t)r.n_obs + o) * 2;
                    d[0] = xh[q] + xl[q];
                    d[1] = yh[q] + yl[q];
                }
            }
        }
    }
    const T Tend = (T)((double)r.steps * r.dt);
#pragma unroll
    for (int q = 0; q < OWN; ++q) {
        const int i = tid + NT * q;
        if (i < n && (i % N) == N - 1) {
            const int64_t f = f0 + i / N;
            if (st) {
                speed[f] = (T)NAN;
            } else {
                const T hx0 = (T)(b.params[9 * f + 7] + (double)(N - 1) * dsd);
                const T hy0 = (T)b.params[9 * f + 8];
                const T dx = (xh[q] + xl[q]) - hx0, dy = (yh[q] + yl[q]) - hy0;
                speed[f] = sqrt_t(fma_t(dx, dx, dy * dy)) / Tend;
            }
        }
    }
    if (tid == 0) {
        status[s] = st;
        if (steps_done) steps_done[s] = done;
    }
    __syncthreads();
}

template <typename T, int TPL, int WPS>
__global__ __launch_bounds__(64 * WPS) void k_forward(Batch b, Run r, const int32_t* order, int32_t* queue, T* obs,
                                                      T* speed, int32_t* status, int32_t* steps_done)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NMAX = 64 * TPL;
    __shared__ int s_item;
    constexpr size_t TABB = sizeof(T) == 4 ? sizeof(TabSys) : 0;
    FwdLds<T> L;
    L.tab = reinterpret_cast<TabSys*>(smem);
    L.src = reinterpret_cast<Src4<T>*>(smem + TABB);
    L.lox = reinterpret_cast<T*>(smem + TABB + NMAX * sizeof(Src4<T>));
    L.loy = L.lox + NMAX;
    L.red = L.loy + NMAX;
    L.part = L.red + 2 * WPS;
    // Work queue: thread 0 takes the next system; the item reaches every
    // thread through LDS and readfirstlane makes it an SGPR, so the loop exit
    // is a uniform scalar branch.  A workgroup takes at most n_sys items.
    for (int64_t it = 0; it <= b.n_sys; ++it) {
        if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= b.n_sys) break;
        const int s = __builtin_amdgcn_readfirstlane(order[item]);
        run_system<T, TPL, WPS>(b, r, s, L, obs, speed, status, steps_done);
    }
}

// ---------------------------------------------------------------------------
// large systems: one launch per step, targets split over workgroups; every
// workgroup rebuilds the forces of the whole system into LDS (O(N) work next
// to its O(N * 256 * TPL) pair work), positions are double-buffered in HBM.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_big_init(const int64_t* list, Batch b, BigState S, int32_t* status, T* obs, int32_t n_obs)
{
    constexpr bool COMP = sizeof(T) == 4;
    const int64_t s = list[blockIdx.y];
    const int64_t p0 = b.pt_off[s];
    const int N = b.npt[s];
    const int n = N * b.nswim[s];
    if (status[s] == SWIM_ST_BADPARAM_) {
        for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < b.nswim[s]; m += gridDim.x * blockDim.x) {
            const int64_t f = b.sw_off[s] + m;
            for (int o = 0; o < 2 * n_obs; ++o) obs[f * (int64_t)n_obs * 2 + o] = (T)NAN;
        }
        return;
    }
    const double dsd = 1.0 / (double)(N - 1);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int m = i / N, p = i - m * N;
        const int64_t f = b.sw_off[s] + m;
        const double X = b.params[9 * f + 7] + (double)p * dsd;
        const double Y = b.params[9 * f + 8];
        const T xh = (T)X, yh = (T)Y;
        ((T*)S.xh[0])[p0 + i] = xh;
        ((T*)S.yh[0])[p0 + i] = yh;
        ((T*)S.xl[0])[p0 + i] = COMP ? (T)(X - (double)xh) : (T)0;
        ((T*)S.yl[0])[p0 + i] = COMP ? (T)(Y - (double)yh) : (T)0;
        if (p == N - 1) {
            ((T*)S.head0)[2 * f] = (T)X;
            ((T*)S.head0)[2 * f + 1] = (T)Y;
            for (int o = 0; o < 2 * n_obs; ++o) obs[f * (int64_t)n_obs * 2 + o] = (T)NAN;
        }
    }
}

template <typename T, int TPL>
__global__ __launch_bounds__(256) void k_big_step(const int64_t* blk_sys, const int64_t* blk_first, Batch b,
                                                  BigState S, int step, Run r, T* obs, int32_t* status,
                                                  int32_t* steps_done)
{
    constexpr bool COMP = sizeof(T) == 4;
    constexpr size_t TABB = COMP ? sizeof(TabSys) : 0;
    extern __shared__ __align__(16) unsigned char smem[];
    TabSys* tab = reinterpret_cast<TabSys*>(smem);
    Src4<T>* src = reinterpret_cast<Src4<T>*>(smem + TABB);
    __shared__ double red[2][4];
    const int tid = threadIdx.x;
    const int64_t s = blk_sys[blockIdx.x];
    if (status[s] != 0) return;
    if constexpr (COMP) tab_load((const TabSys*)b.tab + s, tab, tid, 256);
    const int64_t first = blk_first[blockIdx.x];
    const int64_t p0 = b.pt_off[s];
    const int N = b.npt[s];
    const int n = N * b.nswim[s];
    const int64_t f0 = b.sw_off[s];
    const int cur = step & 1, nxt = cur ^ 1;
    const T* xh = (const T*)S.xh[cur] + p0;
    const T* yh = (const T*)S.yh[cur] + p0;
    const T* xl = (const T*)S.xl[cur] + p0;
    const T* yl = (const T*)S.yl[cur] + p0;
    const T t = (T)((double)step * r.dt);
    double sfx = 0.0, sfy = 0.0;   // FP64: multiplies H1(0) in every velocity
    for (int i = tid; i < n; i += 256) {
        const int m = i / N, p = i - m * N;
        const FilP<T> q = load_filp<T>(b.params, f0 + m, N);
        const int base = m * N;
        auto seg = [&](int kk, T& dx, T& dy) {
            const int a = base + kk, c = base + kk + 1;
            dx = (xh[c] - xh[a]) + (COMP ? xl[c] - xl[a] : (T)0);
            dy = (yh[c] - yh[a]) + (COMP ? yl[c] - yl[a] : (T)0);
        };
        T Fx, Fy;
        point_force<T>(seg, p, q, t, Fx, Fy);
        Src4<T> v;
        v.x = xh[i];
        v.y = yh[i];
        v.fx = Fx;
        v.fy = Fy;
        src[i] = v;
        sfx += Fx;
        sfy += Fy;
    }
    sfx = wave_sum(sfx);
    sfy = wave_sum(sfy);
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = sfx;
        red[1][tid >> 6] = sfy;
    }
    __syncthreads();
    const double SFxd = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const double SFyd = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    const SysConst<T> C = ((const SysConst<T>*)b.sysc)[s];
    // FP32 sums whole large systems per lane: FP64 accumulation
    // (pair_accumulate_x); FP64 runs accumulate in FP64 anyway
    T xi[TPL], yi[TPL], ax[TPL], ay[TPL];
    double axd[TPL], ayd[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int64_t i = first + tid + 256 * k;
        xi[k] = i < n ? src[i].x : (T)0;
        yi[k] = i < n ? src[i].y : (T)0;
        ax[k] = ay[k] = (T)0;
        axd[k] = ayd[k] = 0.0;
    }
    if constexpr (COMP)
        pair_accumulate_x<TPL>(C, tab, src, n, xi, yi, axd, ayd);
    else
        pair_accumulate<T, TPL>(C, tab, src, n, xi, yi, ax, ay);
    const T dt = (T)r.dt;
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int64_t i = first + tid + 256 * k;
        if (i >= n) continue;
        T hx = xi[k], hy = yi[k], lx = xl[i], ly = yl[i];
        T ux, uy;
        if constexpr (COMP) {
            ux = (T)fma((double)C.h1c, SFxd, axd[k]);
            uy = (T)fma((double)C.h1c, SFyd, ayd[k]);
        } else {
            ux = fma_t(C.h1c, (T)SFxd, ax[k]);
            uy = fma_t(C.h1c, (T)SFyd, ay[k]);
        }
        if (COMP) {
            acc2(hx, lx, dt * ux);
            acc2(hy, ly, dt * uy);
        } else {
            hx = fma_t(dt, ux, hx);
            hy = fma_t(dt, uy, hy);
        }
        ((T*)S.xh[nxt])[p0 + i] = hx;
        ((T*)S.yh[nxt])[p0 + i] = hy;
        ((T*)S.xl[nxt])[p0 + i] = lx;
        ((T*)S.yl[nxt])[p0 + i] = ly;
        if (bad_t(hx) || bad_t(hy)) {
            atomicMax(&status[s], (isfinite(hx) && isfinite(hy)) ? 2 : 1);
            if (steps_done) steps_done[s] = step + 1;
        }
        if (r.obs_every > 0 && (step + 1) % r.obs_every == 0) {
            const int m = (int)(i / N), p = (int)(i - (int64_t)m * N);
            if (p == N - 1) {
                const int o = (step + 1) / r.obs_every - 1;
                T* q = obs + ((f0 + m) * (int64_t)r.n_obs + o) * 2;
                q[0] = hx + lx;
                q[1] = hy + ly;
            }
        }
    }
}

template <typename T>
__global__ void k_big_finish(const int64_t* list, Batch b, BigState S, int buf, Run r, T* speed,
                             const int32_t* status, int32_t* steps_done)
{
    const int64_t s = list[blockIdx.x];
    if (threadIdx.x == 0 && steps_done) {
        if (status[s] == 0) steps_done[s] = r.steps;
        else if (status[s] == SWIM_ST_BADPARAM_) steps_done[s] = 0;
    }
    const int64_t p0 = b.pt_off[s];
    const int N = b.npt[s];
    const int nsw = b.nswim[s];
    const T Tend = (T)((double)r.steps * r.dt);
    for (int m = threadIdx.x; m < nsw; m += blockDim.x) {
        const int64_t f = b.sw_off[s] + m;
        const int64_t i = p0 + (int64_t)m * N + N - 1;
        if (status[s]) {
            speed[f] = (T)NAN;
        } else {
            const T hx = ((const T*)S.xh[buf])[i] + ((const T*)S.xl[buf])[i];
            const T hy = ((const T*)S.yh[buf])[i] + ((const T*)S.yl[buf])[i];
            const T dx = hx - ((const T*)S.head0)[2 * f], dy = hy - ((const T*)S.head0)[2 * f + 1];
            speed[f] = sqrt_t(fma_t(dx, dx, dy * dy)) / Tend;
        }
    }
}

// ---------------------------------------------------------------------------
// ABC: RMS head-position distance, k-th smallest (radix select), accept mask
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_abc_distance(int64_t n, int32_t n_obs, const T* obs, const double* data, const int32_t* status,
                               double* dist)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T* o = obs + i * (int64_t)n_obs * 2;
    double acc = 0.0;
    for (int m = 0; m < 2 * n_obs; ++m) {
        const double d = (double)o[m] - data[m];
        acc = fma(d, d, acc);
    }
    double d = sqrt(acc / (2.0 * n_obs));
    if ((status && status[i] != 0) || !isfinite(d)) d = INFINITY;
    dist[i] = d;
}

__device__ __forceinline__ uint64_t dkey(double v)
{
    const uint64_t u = __double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double dunkey(uint64_t k)
{
    const uint64_t u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double(u);
}

// tolerance = k-th smallest finite value of v, k = ceil(q * n_finite)
// clamped to [1, n_finite] (+inf when no value is finite): count the finite
// values, then an 8-pass MSB-first radix select over the order-preserving
// 64-bit keys of the doubles.  One workgroup.
__global__ __launch_bounds__(1024) void k_select_kth(int64_t n, const double* v, double q, double* out)
{
    __shared__ unsigned int hist[256];
    __shared__ uint64_t s_prefix, s_mask;
    __shared__ int64_t s_rank;
    __shared__ unsigned long long s_nf;
    const int tid = threadIdx.x;
    if (tid == 0) s_nf = 0;
    __syncthreads();
    unsigned long long nf = 0;
    for (int64_t i = tid; i < n; i += blockDim.x) nf += isfinite(v[i]) ? 1 : 0;
    atomicAdd(&s_nf, nf);
    __syncthreads();
    const int64_t n_fin = (int64_t)s_nf;
    if (n_fin == 0) {
        if (tid == 0) *out = INFINITY;
        return;
    }
    if (tid == 0) {
        int64_t k = (int64_t)ceil(q * (double)n_fin);
        k = k < 1 ? 1 : (k > n_fin ? n_fin : k);
        s_prefix = 0;
        s_mask = 0;
        s_rank = k - 1;
    }
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 56 - 8 * pass;
        for (int h = tid; h < 256; h += blockDim.x) hist[h] = 0;
        __syncthreads();
        const uint64_t prefix = s_prefix, mask = s_mask;
        for (int64_t i = tid; i < n; i += blockDim.x) {
            const uint64_t key = dkey(v[i]);
            if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            int64_t r = s_rank, cum = 0;
            int d = 0;
            for (; d < 256; ++d) {
                if (r < cum + (int64_t)hist[d]) break;
                cum += hist[d];
            }
            s_rank = r - cum;
            s_prefix = prefix | ((uint64_t)d << shift);
            s_mask = mask | ((uint64_t)255 << shift);
        }
        __syncthreads();
    }
    if (tid == 0) *out = dunkey(s_prefix);
}

__global__ void k_accept(int64_t n, const double* dist, const double* tol, uint8_t* acc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) acc[i] = (isfinite(dist[i]) && dist[i] <= *tol) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_sysconst_batch(int dtype, int64_t n_sys, const int64_t* sw_off, const int32_t* npt,
                                 const double* params, double eps_over_ds, void* sysc, void* sysc64,
                                 int32_t* status, hipStream_t st)
{
    if (n_sys <= 0) return hipSuccess;
    if (dtype == 0)
        hipLaunchKernelGGL(k_sysconst_batch<float>, dim3(nblk(n_sys, 64)), dim3(64), 0, st, n_sys, sw_off, npt,
                           params, eps_over_ds, (SysConst<float>*)sysc, (SysConst<double>*)sysc64, status);
    else
        hipLaunchKernelGGL(k_sysconst_batch<double>, dim3(nblk(n_sys, 64)), dim3(64), 0, st, n_sys, sw_off, npt,
                           params, eps_over_ds, (SysConst<double>*)sysc, (SysConst<double>*)nullptr, status);
    return hipGetLastError();
}

hipError_t launch_sysconst(int dtype, int64_t n_sys, const double* alpha, const double* eps, void* sysc,
                           void* sysc64, hipStream_t st)
{
    if (n_sys <= 0) return hipSuccess;
    if (dtype == 0)
        hipLaunchKernelGGL(k_sysconst<float>, dim3(nblk(n_sys, 64)), dim3(64), 0, st, n_sys, alpha, eps,
                           (SysConst<float>*)sysc, (SysConst<double>*)sysc64);
    else
        hipLaunchKernelGGL(k_sysconst<double>, dim3(nblk(n_sys, 64)), dim3(64), 0, st, n_sys, alpha, eps,
                           (SysConst<double>*)sysc, (SysConst<double>*)nullptr);
    return hipGetLastError();
}

size_t table_bytes() { return sizeof(TabSys); }

hipError_t launch_table_build(int64_t s0, int64_t n, const void* sysc64, void* tab, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_table_build, dim3((unsigned)nblk(n * TAB_N, 64)), dim3(64), 0, st, s0, n,
                       (const SysConst<double>*)sysc64, (TabSys*)tab);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n, 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

template <typename T, int TPL>
static void pair_launch(int64_t nb, const int64_t* bs, const int64_t* bf, const int64_t* off, const void* sysc,
                        const void* tab, const void* x, const void* y, const void* fx, const void* fy, void* ux,
                        void* uy, hipStream_t st)
{
    hipLaunchKernelGGL((k_pair_velocity<T, TPL>), dim3((unsigned)nb), dim3(256), 0, st, bs, bf, off,
                       (const SysConst<T>*)sysc, (const TabSys*)tab, (const T*)x, (const T*)y, (const T*)fx,
                       (const T*)fy, (T*)ux, (T*)uy);
}

hipError_t launch_pair_velocity(int dtype, int tpl, int64_t nb, const int64_t* bs, const int64_t* bf,
                                const int64_t* off, const void* sysc, const void* tab, const void* x, const void* y,
                                const void* fx, const void* fy, void* ux, void* uy, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
#define PAIR_CASE(T, P) \
    case P: pair_launch<T, P>(nb, bs, bf, off, sysc, tab, x, y, fx, fy, ux, uy, st); break;
    if (dtype == 0) {
        switch (tpl) { PAIR_CASE(float, 1) PAIR_CASE(float, 2) PAIR_CASE(float, 4) default: return hipErrorInvalidValue; }
    } else {
        switch (tpl) { PAIR_CASE(double, 1) PAIR_CASE(double, 2) PAIR_CASE(double, 4) default: return hipErrorInvalidValue; }
    }
#undef PAIR_CASE
    return hipGetLastError();
}

hipError_t launch_forces(int dtype, int64_t n_fil, const int64_t* fil_off, const int32_t* npt, const double* params,
                         double t, const void* x, const void* y, void* fx, void* fy, hipStream_t st)
{
    if (n_fil <= 0) return hipSuccess;
    // grid.y covers filaments; grid.x covers up to 4096 points per filament
    const dim3 grid(16, (unsigned)n_fil);
    if (dtype == 0)
        hipLaunchKernelGGL(k_forces<float>, grid, dim3(256), 0, st, n_fil, fil_off, npt, params, t, (const float*)x,
                           (const float*)y, (float*)fx, (float*)fy);
    else
        hipLaunchKernelGGL(k_forces<double>, grid, dim3(256), 0, st, n_fil, fil_off, npt, params, t,
                           (const double*)x, (const double*)y, (double*)fx, (double*)fy);
    return hipGetLastError();
}

size_t forward_lds_bytes(int dtype, int tpl, int wps)
{
    const size_t e = dtype == 0 ? sizeof(float) : sizeof(double);
    const size_t nmax = 64 * (size_t)tpl;
    return (dtype == 0 ? table_bytes() : 0) + nmax * 4 * e + 2 * nmax * e + 2 * (size_t)wps * e +
           (wps > 1 ? (size_t)wps * 2 * nmax * e : 0);
}

// raise the kernel's dynamic-LDS limit to what its launches need (outside
// any stream capture: a launch inside a capture finds it already set)
template <typename T, int TPL, int WPS>
static hipError_t fwd_prepare()
{
    const size_t lds = forward_lds_bytes(sizeof(T) == 4 ? 0 : 1, TPL, WPS);
    static size_t attr_lds = 0;
    if (lds > attr_lds) {
        hipError_t e = hipFuncSetAttribute((const void*)k_forward<T, TPL, WPS>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_lds = lds;
    }
    return hipSuccess;
}

template <typename T, int TPL, int WPS>
static hipError_t fwd_launch(int nblocks, const Batch& b, const Run& r, const int32_t* order, int32_t* q, void* obs,
                             void* speed, int32_t* status, int32_t* done, hipStream_t st)
{
    const size_t lds = forward_lds_bytes(sizeof(T) == 4 ? 0 : 1, TPL, WPS);
    hipError_t e = fwd_prepare<T, TPL, WPS>();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_forward<T, TPL, WPS>), dim3(nblocks), dim3(64 * WPS), lds, st, b, r, order, q, (T*)obs,
                       (T*)speed, status, done);
    return hipGetLastError();
}

template <typename T, int TPL, int WPS>
static int fwd_occupancy()
{
    int nb = 0;
    const size_t lds = forward_lds_bytes(sizeof(T) == 4 ? 0 : 1, TPL, WPS);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_forward<T, TPL, WPS>, 64 * WPS, lds) != hipSuccess || nb < 1)
        nb = 1;
    return nb;
}

#define SWIM_FWD_TABLE(X, T)                                                                               \
    X(T, 1, 1) X(T, 1, 2) X(T, 1, 4) X(T, 1, 8) X(T, 1, 16) X(T, 2, 1) X(T, 2, 2) X(T, 2, 4) X(T, 2, 8)      \
    X(T, 2, 16) X(T, 3, 1) X(T, 3, 2) X(T, 3, 4) X(T, 3, 8) X(T, 3, 16) X(T, 4, 1) X(T, 4, 2) X(T, 4, 4)     \
    X(T, 4, 8) X(T, 4, 16) X(T, 6, 1) X(T, 6, 2) X(T, 6, 4) X(T, 6, 8) X(T, 6, 16) X(T, 8, 1) X(T, 8, 2)      \
    X(T, 8, 4) X(T, 8, 8) X(T, 8, 16)

hipError_t launch_forward(int dtype, int tpl, int wps, int nblocks, const Batch& b, const Run& r,
                          const int32_t* order, int32_t* queue, void* obs, void* speed, int32_t* status,
                          int32_t* steps_done, hipStream_t st)
{
#define FWD_CASE(T, P, W) \
    if (tpl == P && wps == W) return fwd_launch<T, P, W>(nblocks, b, r, order, queue, obs, speed, status, steps_done, st);
    if (dtype == 0) {
        SWIM_FWD_TABLE(FWD_CASE, float)
    } else {
        SWIM_FWD_TABLE(FWD_CASE, double)
    }
#undef FWD_CASE
    return hipErrorInvalidValue;
}

hipError_t prepare_forward(int dtype, int tpl, int wps)
{
#define PREP_CASE(T, P, W) \
    if (tpl == P && wps == W) return fwd_prepare<T, P, W>();
    if (dtype == 0) {
        SWIM_FWD_TABLE(PREP_CASE, float)
    } else {
        SWIM_FWD_TABLE(PREP_CASE, double)
    }
#undef PREP_CASE
    return hipErrorInvalidValue;
}

int forward_blocks_per_cu(int dtype, int tpl, int wps)
{
#define OCC_CASE(T, P, W) \
    if (tpl == P && wps == W) return fwd_occupancy<T, P, W>();
    if (dtype == 0) {
        SWIM_FWD_TABLE(OCC_CASE, float)
    } else {
        SWIM_FWD_TABLE(OCC_CASE, double)
    }
#undef OCC_CASE
    return 1;
}

hipError_t launch_big_init(int dtype, const int64_t* list, int64_t n_list, const Batch& b, const BigState& s,
                           int32_t* status, void* obs, int32_t n_obs, hipStream_t st)
{
    if (n_list <= 0) return hipSuccess;
    const dim3 grid(16, (unsigned)n_list);
    if (dtype == 0)
        hipLaunchKernelGGL(k_big_init<float>, grid, dim3(256), 0, st, list, b, s, status, (float*)obs, n_obs);
    else
        hipLaunchKernelGGL(k_big_init<double>, grid, dim3(256), 0, st, list, b, s, status, (double*)obs, n_obs);
    return hipGetLastError();
}

size_t big_step_lds_bytes(int dtype, int32_t max_pts)
{
    return (dtype == 0 ? table_bytes() : 0) + (size_t)max_pts * 4 * (dtype == 0 ? sizeof(float) : sizeof(double));
}

template <typename T, int TPL>
static hipError_t big_prepare(int32_t max_pts)
{
    const size_t lds = big_step_lds_bytes(sizeof(T) == 4 ? 0 : 1, max_pts);
    static size_t attr_lds = 0;
    if (lds > attr_lds) {
        hipError_t e = hipFuncSetAttribute((const void*)k_big_step<T, TPL>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_lds = lds;
    }
    return hipSuccess;
}

hipError_t prepare_big_step(int dtype, int tpl, int32_t max_pts)
{
    if (dtype == 0) {
        switch (tpl) {
            case 1: return big_prepare<float, 1>(max_pts);
            case 2: return big_prepare<float, 2>(max_pts);
            case 4: return big_prepare<float, 4>(max_pts);
            default: return hipErrorInvalidValue;
        }
    }
    switch (tpl) {
        case 1: return big_prepare<double, 1>(max_pts);
        case 2: return big_prepare<double, 2>(max_pts);
        case 4: return big_prepare<double, 4>(max_pts);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int TPL>
static hipError_t big_launch(int64_t nb, const int64_t* bs, const int64_t* bf, int32_t max_pts, const Batch& b,
                             const BigState& s, int step, const Run& r, void* obs, int32_t* status, int32_t* done,
                             hipStream_t st)
{
    const size_t lds = big_step_lds_bytes(sizeof(T) == 4 ? 0 : 1, max_pts);
    hipError_t e = big_prepare<T, TPL>(max_pts);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_big_step<T, TPL>), dim3((unsigned)nb), dim3(256), lds, st, bs, bf, b, s, step, r, (T*)obs,
                       status, done);
    return hipGetLastError();
}

hipError_t launch_big_step(int dtype, int tpl, int64_t nb, const int64_t* bs, const int64_t* bf, int32_t max_pts,
                           const Batch& b, const BigState& s, int step, const Run& r, void* obs, int32_t* status,
                           int32_t* steps_done, hipStream_t st)
{
#define BIG_CASE(T, P) \
    case P: return big_launch<T, P>(nb, bs, bf, max_pts, b, s, step, r, obs, status, steps_done, st);
    if (dtype == 0) {
        switch (tpl) { BIG_CASE(float, 1) BIG_CASE(float, 2) BIG_CASE(float, 4) default: return hipErrorInvalidValue; }
    } else {
        switch (tpl) { BIG_CASE(double, 1) BIG_CASE(double, 2) BIG_CASE(double, 4) default: return hipErrorInvalidValue; }
    }
#undef BIG_CASE
}

hipError_t launch_big_finish(int dtype, const int64_t* list, int64_t n_list, const Batch& b, const BigState& s,
                             int buf, const Run& r, void* speed, const int32_t* status, int32_t* steps_done,
                             hipStream_t st)
{
    if (n_list <= 0) return hipSuccess;
    if (dtype == 0)
        hipLaunchKernelGGL(k_big_finish<float>, dim3((unsigned)n_list), dim3(64), 0, st, list, b, s, buf, r,
                           (float*)speed, status, steps_done);
    else
        hipLaunchKernelGGL(k_big_finish<double>, dim3((unsigned)n_list), dim3(64), 0, st, list, b, s, buf, r,
                           (double*)speed, status, steps_done);
    return hipGetLastError();
}

hipError_t launch_abc_distance(int dtype, int64_t n, int32_t n_obs, const void* obs, const double* data,
                               const int32_t* status, double* dist, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (dtype == 0)
        hipLaunchKernelGGL(k_abc_distance<float>, dim3(nblk(n, 256)), dim3(256), 0, st, n, n_obs, (const float*)obs,
                           data, status, dist);
    else
        hipLaunchKernelGGL(k_abc_distance<double>, dim3(nblk(n, 256)), dim3(256), 0, st, n, n_obs,
                           (const double*)obs, data, status, dist);
    return hipGetLastError();
}

hipError_t launch_select_kth(int64_t n, const double* v, double q, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_select_kth, dim3(1), dim3(1024), 0, st, n, v, q, out);
    return hipGetLastError();
}

hipError_t launch_accept(int64_t n, const double* dist, const double* tol, uint8_t* acc, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_accept, dim3(nblk(n, 256)), dim3(256), 0, st, n, dist, tol, acc);
    return hipGetLastError();
}

}  // namespace swim

