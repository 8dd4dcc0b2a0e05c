// swim_sperm.hip -- gfx950 forward run of the full sperm model of the
// Appendix: a flagellum with the tapered beat, a circular head (ring and
// diameter springs, head bending), the neck springs and the neck-angle
// energy, several swimmers per fluid, the dense regularized-Brinkmanlet sum
// of eq. (BrV) and the forward-Euler no-slip update (Sec. 2.1).
//
// One workgroup runs one system for all its steps (a persistent kernel fed
// by a work queue).  The pair sum uses the symmetric lane schedule of
// swim_pairsum.h, with the partly filled last block of 64 points taken
// point by point (74 points per swimmer leave 10 in it).  The elastic forces are computed per point from the
// positions in LDS: every point evaluates the springs and curvature nodes it
// belongs to, so forces need no atomics and no per-term buffers.
//
// Discrete energy (trapezoid rule, centred differences; every spring has the
// form K (l/L0 - 1)^2 L0):
//   flagellum tension  K_T   segments k, k+1, rest ds
//   flagellum bending  K_C   (zeta_k - zhat_k)^2 ds at nodes 1..nf-2,
//                      zhat = d^2/ds^2 of a (1-s) sin(eta s - omega t + phase)
//   head ring          K_HT  neighbouring head points, rest the initial chord c
//   head diameters     K_HT  points pi apart, rest 2 H_r
//   head bending       K_HC  (kappa_m - 1/H_r)^2 c at every head node
//   neck springs       K_NT  last flagellum point to the head points at
//                      pi - dth, pi, pi + dth; the one before to pi -+ dth;
//                      rest the initial lengths
//   neck angle         K_NA  (z1 . z2)^2, z1 = H(pi) - F(nf-1),
//                      z2 = H(pi + dth) - H(pi - dth)
// F = -dE/dX (eq. Fenergy).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "swim.h"
#include "swim_internal.h"
#include "swim_math.h"
#include "swim_pairsum.h"

namespace swim {

namespace {

constexpr int32_t ST_BADPARAM = 3;

// positions of one point in LDS: FP32 (hi, lo) pairs, FP64 plain
template <typename T> struct PosE;
template <> struct alignas(16) PosE<float> {
    float xh, yh, xl, yl;
};
template <> struct alignas(16) PosE<double> {
    double xh, yh;
};

template <typename T> __device__ __forceinline__ PosE<T> pos_make(T xh, T yh, T xl, T yl)
{
    PosE<T> p;
    p.xh = xh;
    p.yh = yh;
    if constexpr (sizeof(T) == 4) {
        p.xl = xl;
        p.yl = yl;
    }
    return p;
}

// X_q - X_p (FP32: differences of the hi and of the lo parts)
template <typename T> __device__ __forceinline__ V2<T> pos_diff(const PosE<T>& q, const PosE<T>& p)
{
    V2<T> d;
    d.x = q.xh - p.xh;
    d.y = q.yh - p.yh;
    if constexpr (sizeof(T) == 4) {
        d.x += q.xl - p.xl;
        d.y += q.yl - p.yl;
    }
    return d;
}

// spring K (l/L0 - 1)^2 L0 between p and q: returns c with F_p += c (X_q - X_p),
// c = 2 K (l/L0 - 1)/l.  FP32 forms the strain as (l^2 - L0^2)/((l + L0) L0),
// free of the cancellation in l/L0 - 1.
template <typename T> __device__ __forceinline__ T spring_coef(V2<T> d, T L0, T L02, T K2)
{
    if constexpr (sizeof(T) == 4) {
        const float t2 = fmaf(d.x, d.x, d.y * d.y);
        const float rl = __builtin_amdgcn_rsqf(t2);
        const float l = t2 * rl;
        const float num = fmaf(d.x, d.x, fmaf(d.y, d.y, -L02));
        return K2 * num * __builtin_amdgcn_rcpf((l + L0) * L0) * rl;
    } else {
        const double l = sqrt(fma(d.x, d.x, d.y * d.y));
        return K2 * (l / L0 - 1.0) / l;
    }
}

// curvature node (A, B, C) with segments d1 = X_B - X_A, d2 = X_C - X_B and
// parameter step h: energy W (kappa - k0)^2 h; returns -dE/dX of the point
// in role r (0: A, 1: B, 2: C) of this node.
template <typename T>
__device__ __forceinline__ V2<T> node_force(V2<T> d1, V2<T> d2, T inv2h, T invh2, T h, T W2, T k0, int r)
{
    const T a = (d2.x + d1.x) * inv2h;
    const T b = (d2.y + d1.y) * inv2h;
    const T p = (d2.x - d1.x) * invh2;
    const T q = (d2.y - d1.y) * invh2;
    const T S = fma_t(a, a, b * b);
    T rS, rS32;  // 1/S, S^(-3/2)
    if constexpr (sizeof(T) == 4) {
        const float rs = __builtin_amdgcn_rsqf(S);
        rS = rs * rs;
        rS32 = rS * rs;
    } else {
        rS = 1.0 / S;
        rS32 = rS / sqrt(S);
    }
    const T num = fma_t(q, a, -p * b);
    const T co = W2 * (num * rS32 - k0) * h;  // dE/dkappa
    const T n3 = (T)3 * num * rS32 * rS;
    const T dka = q * rS32 - a * n3;
    const T dkb = -p * rS32 - b * n3;
    const T dkp = -b * rS32;
    const T dkq = a * rS32;
    V2<T> g;  // dkappa/dX of the point in role r
    if (r == 0) {
        g.x = fma_t(-dka, inv2h, dkp * invh2);
        g.y = fma_t(-dkb, inv2h, dkq * invh2);
    } else if (r == 1) {
        g.x = (T)-2 * dkp * invh2;
        g.y = (T)-2 * dkq * invh2;
    } else {
        g.x = fma_t(dka, inv2h, dkp * invh2);
        g.y = fma_t(dkb, inv2h, dkq * invh2);
    }
    g.x = -co * g.x;
    g.y = -co * g.y;
    return g;
}

// per-system stiffnesses (twice the energy coefficients) and lengths in T
template <typename T> struct SpermK {
    T kt2, kc2, kht2, khc2, knt2, kna2;
    T ds, inv2ds, invds2, ds2;
    T ch, inv2ch, invch2, ch2;
    T dh, dh2, kh0;  // diameter 2 H_r, its square, preferred head curvature 1/H_r
    T L0[5], L02[5];
};

// elastic force on point p (index within its swimmer; its swimmer's points
// start at P in LDS).  zh[0..2]: preferred curvature of flagellum nodes
// p-1, p, p+1 now.
template <typename T>
__device__ __forceinline__ V2<T> sperm_force(const SpermShape& g, const SpermK<T>& K, const PosE<T>* P, int p,
                                             const T (&zh)[3])
{
    const int nf = g.nf, nh = g.nh, c = nf + nh / 2;
    const PosE<T> X = P[p];
    V2<T> F;
    F.x = (T)0;
    F.y = (T)0;
    auto spring = [&](int q, T L0, T L02, T K2) {
        const V2<T> d = pos_diff(P[q], X);
        const T cf = spring_coef(d, L0, L02, K2);
        F.x = fma_t(cf, d.x, F.x);
        F.y = fma_t(cf, d.y, F.y);
    };
    auto node = [&](int a, int b, int cc, T inv2h, T invh2, T h, T W2, T k0, int r) {
        const PosE<T> A = P[a], B = P[b], C = P[cc];
        const V2<T> f = node_force(pos_diff(B, A), pos_diff(C, B), inv2h, invh2, h, W2, k0, r);
        F.x += f.x;
        F.y += f.y;
    };
    if (p < nf) {
        if (p >= 1) spring(p - 1, K.ds, K.ds2, K.kt2);
        if (p <= nf - 2) spring(p + 1, K.ds, K.ds2, K.kt2);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int j = p + 1 - r;  // node j, in which p has role r
            if (j >= 1 && j <= nf - 2) node(j - 1, j, j + 1, K.inv2ds, K.invds2, K.ds, K.kc2, zh[2 - r], r);
        }
        if (p == nf - 1) {
            spring(c - 1, K.L0[0], K.L02[0], K.knt2);
            spring(c, K.L0[1], K.L02[1], K.knt2);
            spring(c + 1, K.L0[2], K.L02[2], K.knt2);
        } else if (p == nf - 2) {
            spring(c - 1, K.L0[3], K.L02[3], K.knt2);
            spring(c + 1, K.L0[4], K.L02[4], K.knt2);
        }
    } else {
        const int m = p - nf;
        auto hp = [&](int k) { return nf + (k + nh) % nh; };
        spring(hp(m - 1), K.ch, K.ch2, K.kht2);
        spring(hp(m + 1), K.ch, K.ch2, K.kht2);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int j = m + 1 - r;
            node(hp(j - 1), hp(j), hp(j + 1), K.inv2ch, K.invch2, K.ch, K.khc2, K.kh0, r);
        }
        spring(hp(m + nh / 2), K.dh, K.dh2, K.kht2);
        if (p == c - 1) {
            spring(nf - 1, K.L0[0], K.L02[0], K.knt2);
            spring(nf - 2, K.L0[3], K.L02[3], K.knt2);
        } else if (p == c) {
            spring(nf - 1, K.L0[1], K.L02[1], K.knt2);
        } else if (p == c + 1) {
            spring(nf - 1, K.L0[2], K.L02[2], K.knt2);
            spring(nf - 2, K.L0[4], K.L02[4], K.knt2);
        }
    }
    // neck angle: E = K (z1.z2)^2, dE/dz1 = 2K (z1.z2) z2, dE/dz2 = 2K (z1.z2) z1
    if (p == nf - 1 || p == c - 1 || p == c || p == c + 1) {
        const V2<T> z1 = pos_diff(P[c], P[nf - 1]), z2 = pos_diff(P[c + 1], P[c - 1]);
        const T w = K.kna2 * fma_t(z1.x, z2.x, z1.y * z2.y);
        if (p == nf - 1) {
            F.x = fma_t(w, z2.x, F.x);
            F.y = fma_t(w, z2.y, F.y);
        } else if (p == c) {
            F.x = fma_t(-w, z2.x, F.x);
            F.y = fma_t(-w, z2.y, F.y);
        } else if (p == c + 1) {
            F.x = fma_t(-w, z1.x, F.x);
            F.y = fma_t(-w, z1.y, F.y);
        } else {
            F.x = fma_t(w, z1.x, F.x);
            F.y = fma_t(w, z1.y, F.y);
        }
    }
    return F;
}

// initial position of point p of a swimmer whose first flagellum point is (x0, y0)
__device__ __forceinline__ void sperm_initial(const SpermShape& g, double x0, double y0, int p, double& x, double& y)
{
    if (p < g.nf) {
        x = x0 + (double)p * g.ds;
        y = y0;
    } else {
        const int m = p - g.nf;
        const double xc = (x0 + (double)(g.nf - 1) * g.ds) + g.hr + g.dn;
        x = xc + g.hr * cos((double)m * g.dth);
        y = y0 + g.hr * sin((double)m * g.dth);
    }
}

struct SpermLdsLayout {
    size_t tab, src, part, pos, bad, total;
};
__host__ __device__ constexpr size_t al16(size_t x) { return (x + 15) & ~(size_t)15; }
__host__ __device__ constexpr SpermLdsLayout sperm_lds_layout(int dtype, int tpl, int wps)
{
    const size_t e = dtype == 0 ? 4 : 8, nmax = 64 * (size_t)tpl;
    SpermLdsLayout L{};
    L.tab = 0;
    L.src = dtype == 0 ? al16(sizeof(TabSys)) : 0;
    L.part = al16(L.src + 2 * nmax * 4 * e);
    L.pos = al16(L.part + (size_t)wps * nmax * 2 * e);
    L.bad = al16(L.pos + nmax * 16);
    L.total = al16(L.bad + 4 * (size_t)wps);
    return L;
}

template <typename T, int TPL, int WPS>
__device__ void sperm_system(const SpermShape& g, const SpermRun& r, int64_t s, const SysConst<T>& C,
                             const TabSys* tab_g, TabSys* tab, Src4<T>* src, V2<T>* part, PosE<T>* pos, int* badw,
                             T* head, T* tail, int32_t* status)
{
    constexpr bool COMP = sizeof(T) == 4;
    constexpr int NMAX = 64 * TPL, NT = 64 * WPS, PPT = (NMAX + NT - 1) / NT;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int np = g.nf + g.nh, nsw = g.nsw, n = np * nsw;
    const int nobs1 = r.n_obs + 1;
    const double* sp = r.sysp + (int64_t)SWIM_SP_NPARAM * s;
    const double* sw = r.swp + (int64_t)3 * nsw * s;
    T* hd = head + (int64_t)s * nsw * nobs1 * 2;
    T* tl = tail + (int64_t)s * nsw * nobs1 * 2;
    // samples a stopped (or not run) system does not reach stay NaN
    for (int k = tid; k < nsw * nobs1 * 2; k += NT) {
        hd[k] = (T)NAN;
        tl[k] = (T)NAN;
    }
    if (status[s] == ST_BADPARAM) {
        __syncthreads();
        return;
    }
    if constexpr (COMP) tab_load(tab_g + s, tab, tid, NT);
    SpermK<T> K;
    K.kc2 = (T)(2.0 * sp[SWIM_SP_KC]);
    K.kt2 = (T)(2.0 * sp[SWIM_SP_KT]);
    K.kht2 = (T)(2.0 * sp[SWIM_SP_KHT]);
    K.khc2 = (T)(2.0 * sp[SWIM_SP_KHC]);
    K.knt2 = (T)(2.0 * sp[SWIM_SP_KNT]);
    K.kna2 = (T)(2.0 * sp[SWIM_SP_KNA]);
    K.ds = (T)g.ds;
    K.inv2ds = (T)(0.5 / g.ds);
    K.invds2 = (T)(1.0 / (g.ds * g.ds));
    K.ds2 = (T)(g.ds * g.ds);
    K.ch = (T)g.ch;
    K.inv2ch = (T)(0.5 / g.ch);
    K.invch2 = (T)(1.0 / (g.ch * g.ch));
    K.ch2 = (T)(g.ch * g.ch);
    K.dh = (T)(2.0 * g.hr);
    K.dh2 = (T)(4.0 * g.hr * g.hr);
    K.kh0 = (T)(1.0 / g.hr);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        K.L0[i] = (T)g.L0[i];
        K.L02[i] = (T)(g.L0[i] * g.L0[i]);
    }
    const double a = sp[SWIM_SP_A], eta = sp[SWIM_SP_ETA], om = sp[SWIM_SP_OMEGA];
    const T dt = (T)r.dt;
    const T rho = COMP ? C.tr : (T)1;

    // owned points i = tid + NT k: positions in registers, and for flagellum
    // points the preferred-curvature coefficients of nodes p-1, p, p+1:
    // zhat_j(t) = A_j cos(omega t) + B_j sin(omega t)
    T xh[PPT], yh[PPT], xl[PPT], yl[PPT], zA[PPT][3], zB[PPT][3];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int i = tid + NT * k;
        const bool held = i < n;
        const int m = held ? i / np : 0, p = held ? i - m * np : 0;
        double X = 0.0, Y = 0.0;
        if (held) sperm_initial(g, sw[3 * m], sw[3 * m + 1], p, X, Y);
        xh[k] = (T)X;
        yh[k] = (T)Y;
        xl[k] = COMP ? (T)(X - (double)xh[k]) : (T)0;
        yl[k] = COMP ? (T)(Y - (double)yh[k]) : (T)0;
        if (held) pos[i] = pos_make<T>(xh[k], yh[k], xl[k], yl[k]);
        const double ph = held ? sw[3 * m + 2] : 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int j = p - 1 + q;
            const double sj = (double)j * g.ds, psi = eta * sj + ph;
            const double u = -2.0 * a * eta, v = a * (1.0 - sj) * eta * eta;
            const bool nd = held && p < g.nf && j >= 1 && j <= g.nf - 2;
            zA[k][q] = nd ? (T)(u * cos(psi) - v * sin(psi)) : (T)0;
            zB[k][q] = nd ? (T)(u * sin(psi) + v * cos(psi)) : (T)0;
        }
    }
    // padding points n .. 64 B - 1 of the last block: no force, at the start
    // position of point n - 1 (they add nothing to the sums)
    for (int i = n + tid; i < 64 * ((n + 63) >> 6); i += NT) {
        double X, Y;
        sperm_initial(g, sw[3 * (nsw - 1)], sw[3 * (nsw - 1) + 1], np - 1, X, Y);
        Src4<T> v;
        v.x = (T)X * rho;
        v.y = (T)Y * rho;
        v.fx = (T)0;
        v.fy = (T)0;
        const int slot = src2_slot(i);
        src[slot] = v;
        src[slot + 64] = v;
    }
    // cos, sin of omega t: FP32 runs rotate by omega dt in FP64, FP64 runs
    // evaluate them directly
    double rc = 1.0, rs = 0.0;
    const double cd = cos(om * r.dt), sd = sin(om * r.dt);
    __syncthreads();

    // forces at the current positions (pos in LDS) into src; observation
    // sample o of the head centres and tail ends
    auto forces = [&]() {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int i = tid + NT * k;
            if (i < n) {
                const int m = i / np, p = i - m * np;
                T zh[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) zh[q] = fma_t(zA[k][q], (T)rc, zB[k][q] * (T)rs);
                const V2<T> F = sperm_force<T>(g, K, pos + m * np, p, zh);
                Src4<T> v;
                v.x = xh[k] * rho;
                v.y = yh[k] * rho;
                v.fx = F.x;
                v.fy = F.y;
                const int slot = src2_slot(i);
                src[slot] = v;
                src[slot + 64] = v;
            }
        }
    };
    auto observe = [&](int o) {
        for (int m = tid; m < nsw; m += NT) {
            double cx = 0.0, cy = 0.0;
            const PosE<T>* P = pos + m * np;
            for (int j = g.nf; j < np; ++j) {
                cx += (double)P[j].xh;
                cy += (double)P[j].yh;
                if constexpr (COMP) {
                    cx += (double)P[j].xl;
                    cy += (double)P[j].yl;
                }
            }
            T* h = hd + ((int64_t)m * nobs1 + o) * 2;
            T* t = tl + ((int64_t)m * nobs1 + o) * 2;
            h[0] = (T)(cx / (double)g.nh);
            h[1] = (T)(cy / (double)g.nh);
            double tx = (double)P[0].xh, ty = (double)P[0].yh;
            if constexpr (COMP) {
                tx += (double)P[0].xl;
                ty += (double)P[0].yl;
            }
            t[0] = (T)tx;
            t[1] = (T)ty;
        }
    };
    observe(0);
    forces();
    __syncthreads();
    int st = 0;
    int obs_left = r.obs_every, obs_k = 1;
    // this wave's share of the symmetric schedule (of the full blocks when
    // the tail schedule takes the rest), found once when it is one segment
    const bool tail_sched = tail_pays(n);
    int seg[5] = {0, 0, 0, 0, 0};
    {
        int a = 0, b = 0, lo = 0, hi = 0;
        const bool one = sym_one_segment<WPS>(tail_sched ? 64 * (n >> 6) : n, wave, a, b, lo, hi);
        seg[0] = __builtin_amdgcn_readfirstlane(one ? 1 : 0);
        seg[1] = __builtin_amdgcn_readfirstlane(a);
        seg[2] = __builtin_amdgcn_readfirstlane(b);
        seg[3] = __builtin_amdgcn_readfirstlane(lo);
        seg[4] = __builtin_amdgcn_readfirstlane(hi);
    }
    for (int step = 0; step < r.steps; ++step) {
        {
            T ax[TPL], ay[TPL];
            if (tail_sched)
                pair_phase_tail<T, TPL, WPS>(C, tab, src, n, wave, lane, ax, ay, seg);
            else if (seg[0])
                pair_phase_seg<T, TPL>(C, tab, src, seg[1], seg[2], seg[3], seg[4], lane, ax, ay);
            else
                pair_phase_sym<T, TPL, WPS>(C, tab, src, n, wave, lane, ax, ay);
#pragma unroll
            for (int c = 0; c < TPL; ++c) {
                if (64 * c < n) {
                    V2<T> v;
                    v.x = ax[c];
                    v.y = ay[c];
                    part[wave * NMAX + 64 * c + lane] = v;
                }
            }
        }
        __syncthreads();
        // Euler step of the owned points; partial sums reduced in wave order
        int bad = 0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int i = tid + NT * k;
            if (i < n) {
                V2<T> pv[WPS];
#pragma unroll
                for (int w = 0; w < WPS; ++w) pv[w] = part[w * NMAX + i];
                T ux = (T)0, uy = (T)0;
#pragma unroll
                for (int w = 0; w < WPS; ++w) {
                    ux += pv[w].x;
                    uy += pv[w].y;
                }
                if constexpr (COMP) {
                    acc2(xh[k], xl[k], dt * ux);
                    acc2(yh[k], yl[k], dt * uy);
                } else {
                    xh[k] = fma_t(dt, ux, xh[k]);
                    yh[k] = fma_t(dt, uy, yh[k]);
                }
                if (bad_t(xh[k]) || bad_t(yh[k])) bad = max(bad, (isfinite(xh[k]) && isfinite(yh[k])) ? 2 : 1);
                pos[i] = pos_make<T>(xh[k], yh[k], xl[k], yl[k]);
            }
        }
        if constexpr (COMP) {
            const double c0 = rc;
            rc = fma(c0, cd, -rs * sd);
            rs = fma(rs, cd, c0 * sd);
        } else {
            const double wt = om * ((double)(step + 1) * r.dt);
            rc = cos(wt);
            rs = sin(wt);
        }
        {
            const bool b1 = __ballot(bad == 1) != 0, b2 = __ballot(bad == 2) != 0;
            if (lane == 0) badw[wave] = (b1 ? 1 : 0) | (b2 ? 2 : 0);
        }
        __syncthreads();
        const int bw = lane < WPS ? badw[lane] : 0;
        const int bflags = (__ballot(bw & 1) ? 1 : 0) | (__ballot(bw & 2) ? 2 : 0);
        if (bflags) {
            st = (bflags & 1) ? 1 : 2;
            break;
        }
        if (r.obs_every > 0 && --obs_left == 0) {
            obs_left = r.obs_every;
            observe(obs_k++);
        }
        forces();
        __syncthreads();
    }
    if (tid == 0) status[s] = st;
    __syncthreads();
}

template <typename T, int TPL, int WPS>
__global__ __launch_bounds__(64 * WPS) void k_sperm_forward(SpermShape g, SpermRun r, const SysConst<T>* sysc,
                                                            const TabSys* tabs, int32_t* queue, T* head, T* tail,
                                                            int32_t* status)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item;
    const SpermLdsLayout lay = sperm_lds_layout(sizeof(T) == 4 ? 0 : 1, TPL, WPS);
    TabSys* tab = reinterpret_cast<TabSys*>(smem + lay.tab);
    Src4<T>* src = reinterpret_cast<Src4<T>*>(smem + lay.src);
    V2<T>* part = reinterpret_cast<V2<T>*>(smem + lay.part);
    PosE<T>* pos = reinterpret_cast<PosE<T>*>(smem + lay.pos);
    int* badw = reinterpret_cast<int*>(smem + lay.bad);
    // work queue: a workgroup takes at most n_sys items, so the loop ends
    for (int64_t it = 0; it <= r.n_sys; ++it) {
        if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= r.n_sys) break;
        sperm_system<T, TPL, WPS>(g, r, item, sysc[item], tabs, tab, src, part, pos, badw, head, tail, status);
    }
}

// per-system constants; rows outside the model's domain are flagged
template <typename T>
__global__ void k_sperm_setup(int64_t n_sys, int32_t nsw, double eps, const double* sysp, const double* swp,
                              SysConst<T>* sysc, SysConst<double>* sysc64, int32_t* status, int blob)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sys) return;
    const double* p = sysp + (int64_t)SWIM_SP_NPARAM * s;
    const double alpha = p[SWIM_SP_ALPHA];
    bool ok = isfinite(alpha) && alpha >= 0.0 && alpha * eps <= 1.0;
    for (int c = 0; c < SWIM_SP_NPARAM; ++c) ok = ok && isfinite(p[c]);
    for (int c = 0; c < 3 * nsw; ++c) ok = ok && isfinite(swp[(int64_t)3 * nsw * s + c]);
    status[s] = ok ? 0 : ST_BADPARAM;
    sysconst_compute2<T>(ok ? alpha : 0.0, eps, sysc + s, sysc64 ? sysc64 + s : nullptr, blob);
}

// observables of a sperm run per system s and interval/sample k = 1..n_obs
// (Sec. 4): kind 0, the head-centre velocity of swimmer 0,
// (h_k - h_{k-1}) / dt_obs; kind 1, the distance between the tail ends and
// between the head centres of swimmers 0 and 1 at sample k.  Stopped runs
// give NaN.
template <typename T>
__global__ void k_sperm_observables(int kind, int64_t n_sys, int32_t nsw, int32_t n_obs, double dt_obs, const T* head,
                                    const T* tail, const int32_t* status, double* g)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_sys * n_obs) return;
    const int64_t s = e / n_obs;
    const int k = (int)(e - s * n_obs) + 1;
    double* o = g + 2 * e;
    if (status[s] != 0) {
        o[0] = NAN;
        o[1] = NAN;
        return;
    }
    const int64_t stride = (int64_t)(n_obs + 1) * 2;  // one swimmer's samples
    const T* h0 = head + s * nsw * stride;
    if (kind == 0) {
        o[0] = ((double)h0[2 * k] - (double)h0[2 * k - 2]) / dt_obs;
        o[1] = ((double)h0[2 * k + 1] - (double)h0[2 * k - 1]) / dt_obs;
    } else {
        const T* t0 = tail + s * nsw * stride;
        const T *h1 = h0 + stride, *t1 = t0 + stride;
        const double tx = (double)t0[2 * k] - (double)t1[2 * k], ty = (double)t0[2 * k + 1] - (double)t1[2 * k + 1];
        const double hx = (double)h0[2 * k] - (double)h1[2 * k], hy = (double)h0[2 * k + 1] - (double)h1[2 * k + 1];
        o[0] = sqrt(fma(tx, tx, ty * ty));
        o[1] = sqrt(fma(hx, hx, hy * hy));
    }
}

// Gaussian log-likelihood (eqs. likelihood, fitness) with a diagonal
// covariance of two levels: entries 0, 2, 4, ... (the odd entries in 1-based
// numbering) have standard deviation sig2[2i], the others sig2[2i+1].
// A stopped run or a non-finite output gives -inf.
__global__ void k_gauss_loglik2(int64_t n, int32_t n_obs, const double* g, const double* data, const double* sig2,
                                const int32_t* status, double* logl)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* gi = g + i * (int64_t)n_obs * 2;
    double Ja = 0.0, Jb = 0.0;
    bool ok = status == nullptr || status[i] == 0;
    for (int k = 0; k < n_obs && ok; ++k) {
        ok = isfinite(gi[2 * k]) && isfinite(gi[2 * k + 1]);
        const double ra = data[2 * k] - gi[2 * k], rb = data[2 * k + 1] - gi[2 * k + 1];
        Ja = fma(ra, ra, Ja);
        Jb = fma(rb, rb, Jb);
    }
    if (!ok) {
        logl[i] = -INFINITY;
        return;
    }
    const double sa = sig2[2 * i], sb = sig2[2 * i + 1], m = (double)n_obs;
    if (!(sa > 0.0 && sb > 0.0)) {
        logl[i] = -INFINITY;
        return;
    }
    logl[i] = -m * log(2.0 * M_PI) - m * (log(sa) + log(sb)) - 0.5 * (Ja / (sa * sa) + Jb / (sb * sb));
}

template <typename T, int TPL, int WPS>
hipError_t launch_sperm_t(int nblocks, const SpermShape& g, const SpermRun& r, const void* sysc, const void* tabs,
                          int32_t* queue, void* head, void* tail, int32_t* status, hipStream_t st)
{
    const size_t lds = sperm_lds_layout(sizeof(T) == 4 ? 0 : 1, TPL, WPS).total;
    hipLaunchKernelGGL((k_sperm_forward<T, TPL, WPS>), dim3(nblocks), dim3(64 * WPS), lds, st, g, r,
                       (const SysConst<T>*)sysc, (const TabSys*)tabs, queue, (T*)head, (T*)tail, status);
    return hipGetLastError();
}

template <typename T, int TPL, int WPS> const void* sperm_kernel_ptr()
{
    return reinterpret_cast<const void*>(&k_sperm_forward<T, TPL, WPS>);
}

// dispatch over (dtype, tpl, wps); f receives the instantiation's tag types
template <typename F> hipError_t sperm_dispatch(int dtype, int tpl, int wps, F f)
{
#define SWIM_SPERM_CASE(TT, TP, WP)                                      \
    if (tpl == TP && wps == WP) return f((TT*)nullptr, std::integral_constant<int, TP>(), \
                                         std::integral_constant<int, WP>());
#define SWIM_SPERM_WPS(TT, TP) SWIM_SPERM_CASE(TT, TP, 2) SWIM_SPERM_CASE(TT, TP, 4) SWIM_SPERM_CASE(TT, TP, 8)
#define SWIM_SPERM_ALL(TT) \
    SWIM_SPERM_WPS(TT, 1) SWIM_SPERM_WPS(TT, 2) SWIM_SPERM_WPS(TT, 3) SWIM_SPERM_WPS(TT, 4) SWIM_SPERM_WPS(TT, 6) \
    SWIM_SPERM_WPS(TT, 8)
    if (dtype == 0) {
        SWIM_SPERM_ALL(float)
    } else {
        SWIM_SPERM_ALL(double)
    }
#undef SWIM_SPERM_ALL
#undef SWIM_SPERM_WPS
#undef SWIM_SPERM_CASE
    return hipErrorInvalidValue;
}

}  // namespace

size_t sperm_lds_bytes(int dtype, int tpl, int wps) { return sperm_lds_layout(dtype, tpl, wps).total; }

hipError_t launch_sperm_setup(int dtype, int64_t n_sys, int32_t nsw, double eps, const double* sysp,
                              const double* swp, void* sysc, void* sysc64, int32_t* status, int blob,
                              hipStream_t st)
{
    if (n_sys == 0) return hipSuccess;
    const int nb = (int)((n_sys + 255) / 256);
    if (dtype == 0)
        hipLaunchKernelGGL(k_sperm_setup<float>, dim3(nb), dim3(256), 0, st, n_sys, nsw, eps, sysp, swp,
                           (SysConst<float>*)sysc, (SysConst<double>*)sysc64, status, blob);
    else
        hipLaunchKernelGGL(k_sperm_setup<double>, dim3(nb), dim3(256), 0, st, n_sys, nsw, eps, sysp, swp,
                           (SysConst<double>*)sysc, (SysConst<double>*)nullptr, status, blob);
    return hipGetLastError();
}

hipError_t prepare_sperm(int dtype, int tpl, int wps)
{
    return sperm_dispatch(dtype, tpl, wps, [&](auto* tt, auto tp, auto wp) {
        using T = std::remove_pointer_t<decltype(tt)>;
        const void* k = sperm_kernel_ptr<T, decltype(tp)::value, decltype(wp)::value>();
        return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)sperm_lds_bytes(dtype, tpl, wps));
    });
}

int sperm_blocks_per_cu(int dtype, int tpl, int wps)
{
    int nb = 0;
    const hipError_t e = sperm_dispatch(dtype, tpl, wps, [&](auto* tt, auto tp, auto wp) {
        using T = std::remove_pointer_t<decltype(tt)>;
        const void* k = sperm_kernel_ptr<T, decltype(tp)::value, decltype(wp)::value>();
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 64 * wps, sperm_lds_bytes(dtype, tpl, wps));
    });
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_sperm_forward(int dtype, int tpl, int wps, int nblocks, const SpermShape& g, const SpermRun& r,
                                const void* sysc, const void* tabs, int32_t* queue, void* head, void* tail,
                                int32_t* status, hipStream_t st)
{
    return sperm_dispatch(dtype, tpl, wps, [&](auto* tt, auto tp, auto wp) {
        using T = std::remove_pointer_t<decltype(tt)>;
        return launch_sperm_t<T, decltype(tp)::value, decltype(wp)::value>(nblocks, g, r, sysc, tabs, queue, head,
                                                                           tail, status, st);
    });
}

hipError_t launch_sperm_observables(int dtype, int kind, int64_t n_sys, int32_t nsw, int32_t n_obs, double dt_obs,
                                    const void* head, const void* tail, const int32_t* status, double* g,
                                    hipStream_t st)
{
    const int64_t m = n_sys * n_obs;
    if (m == 0) return hipSuccess;
    const unsigned nb = (unsigned)((m + 255) / 256);
    if (dtype == 0)
        hipLaunchKernelGGL(k_sperm_observables<float>, dim3(nb), dim3(256), 0, st, kind, n_sys, nsw, n_obs, dt_obs,
                           (const float*)head, (const float*)tail, status, g);
    else
        hipLaunchKernelGGL(k_sperm_observables<double>, dim3(nb), dim3(256), 0, st, kind, n_sys, nsw, n_obs, dt_obs,
                           (const double*)head, (const double*)tail, status, g);
    return hipGetLastError();
}

hipError_t launch_gauss_loglik2(int64_t n, int32_t n_obs, const double* g, const double* data, const double* sig2,
                                const int32_t* status, double* logl, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gauss_loglik2, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, n_obs, g, data, sig2,
                       status, logl);
    return hipGetLastError();
}

}  // namespace swim
