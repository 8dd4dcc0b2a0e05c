// swim_math.h -- kernel functions of the regularized Brinkmanlet (Sec. 2.1,
// eq. BrV) for the device, templated on the working precision.
//
// Velocity of point forces F_j at X_j:
//   u(x) = sum_j [ H1(r) F_j + H2(r) (F_j . d) d ],  d = x - X_j, r = |d|,
//   H1 = -B'',  H2 = (r B'' - B')/r^3,  (Delta - alpha^2) B = G,  Delta G = phi.
// Blob reading (the paper defers G, B to its references): with
// R = sqrt(r^2 + eps^2) and c = 1/(alpha eps K1(alpha eps)),
//   g = Delta B = -c K0(alpha R)/(2 pi),   M(r) = int_0^r s g ds,
//   H1 = M/r^2 - g,   H2 = (g - 2 M/r^2)/r^2;  alpha = 0 is the Stokes limit.
//
// Evaluation without cancellation.  Write t = r^2, w = alpha^2 R^2 =
// alpha^2 t + w0 (w0 = alpha^2 eps^2), delta = t/eps^2 and
// Q(w) = z K1(z) - 1 at z = sqrt(w).  Then
//   g(t) - g(0) = -(c/2pi) [K0(w) - K0(w0)],
//   H2 = (c/pi) alpha^2 Q[w0, w, w]   (second divided difference),
//   H1 = H1(0) + Ht,   Ht = -(g(t) - g(0) + t H2)/2.
// The constant H1(0) multiplies sum_j F_j and is added once per target.
// For z <= 2 the ascending series K0 = -1/2 ln(w/4) I0(w) + P0(w),
// Q = 1/2 ln(w/4) A(w) - B(w) (A&S 9.6.13, 9.6.11) turn these divided
// differences into
//   K0(w) - K0(w0) = -1/2 log1p(delta) I0(w) + U(t),
//   H2 = (c/pi) [ V(t) + (D(w) lambda + Abar(w) S2) / (2 eps^2) ],
// with lambda = log1p(delta)/delta, S2 = (1 - lambda)/delta (the Stokes
// part), Abar = A/w, D = A' - Abar, and U, V polynomials in t whose
// coefficients (Taylor coefficients of I0, P0, A, B at w0, times the log
// ln(w0/4) where it appears) are computed once per system.  Every term is
// then a sum of same-signed pieces.  For z > 2 the functions come from
// K_nu(z) = exp(-z) z^-1/2 f_nu(2/z) with Chebyshev fits f_nu
// (swim_kfit.h) and the closed form, which no longer cancels there.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "swim_kfit.h"

#define SWIM_HD __host__ __device__ __forceinline__

namespace swim {

constexpr double PI = 3.14159265358979323846;
constexpr double EULER_GAMMA = 0.57721566490153286061;
constexpr int NT_MAX = 16;      // per-system polynomial length (max)
constexpr int NSER_SETUP = 40;  // series length used by the FP64 set-up

// ---------------------------------------------------------------------------
// compile-time series coefficients
// ---------------------------------------------------------------------------
constexpr double fact(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; }
constexpr double pow4(int n) { double p = 1.0; for (int i = 0; i < n; ++i) p *= 4.0; return p; }
// I0(w) = sum_k w^k / (4^k (k!)^2)
constexpr double c_I0(int k) { return 1.0 / (pow4(k) * fact(k) * fact(k)); }
// A(w) = z I1(z) = sum_{m>=1} A_m w^m,  A_m = 2 / (4^m (m-1)! m!)
constexpr double c_A(int m) { return m < 1 ? 0.0 : 2.0 / (pow4(m) * fact(m - 1) * fact(m)); }
// Abar(w) = A(w)/w = sum_k A_{k+1} w^k ;  D(w) = A' - Abar = sum_k k A_{k+1} w^k
constexpr double c_Abar(int k) { return c_A(k + 1); }
constexpr double c_D(int k) { return k * c_A(k + 1); }

// precision traits: series lengths and thresholds per working type
template <typename T> struct Prec;
template <> struct Prec<float> {
    static constexpr int NW = 9;       // terms of the w-polynomial Abar (w <= 4)
    static constexpr int NT = 9;       // terms of the per-system U, V polynomials
    static constexpr int NA = 4;       // terms of the near-contact atanh series
    static constexpr float DSMALL = 0.25f;
    static constexpr int NKF = SWIM_KFIT_K0_F32_N;
};
template <> struct Prec<double> {
    static constexpr int NW = 15;
    static constexpr int NT = 16;
    static constexpr int NA = 9;
    static constexpr double DSMALL = 0.25;
    static constexpr int NKF = SWIM_KFIT_K0_F64_N;
};

template <typename T> SWIM_HD T kfit(int nu, T x);
template <> SWIM_HD float kfit<float>(int nu, float x)
{
    // Clenshaw recurrence for sum_j c_j T_j(u), u = 2x - 1
    const float u = 2.0f * x - 1.0f, u2 = 2.0f * u;
    float b1 = 0.0f, b2 = 0.0f;
#pragma unroll
    for (int j = SWIM_KFIT_K0_F32_N - 1; j >= 1; --j) {
        const float cj = nu ? (float)swim_kfit_k1_f32[j] : (float)swim_kfit_k0_f32[j];
        const float b0 = fmaf(u2, b1, cj - b2);
        b2 = b1;
        b1 = b0;
    }
    const float c0 = nu ? (float)swim_kfit_k1_f32[0] : (float)swim_kfit_k0_f32[0];
    return fmaf(u, b1, c0 - b2);
}
template <> SWIM_HD double kfit<double>(int nu, double x)
{
    const double u = 2.0 * x - 1.0, u2 = 2.0 * u;
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int j = SWIM_KFIT_K0_F64_N - 1; j >= 1; --j) {
        const double cj = nu ? swim_kfit_k1_f64[j] : swim_kfit_k0_f64[j];
        const double b0 = fma(u2, b1, cj - b2);
        b2 = b1;
        b1 = b0;
    }
    const double c0 = nu ? swim_kfit_k1_f64[0] : swim_kfit_k0_f64[0];
    return fma(u, b1, c0 - b2);
}
// sqrt(z) exp(-z) I_nu(z) at x = SWIM_IFIT_IS / z in (0, 1] (z >= 8)
SWIM_HD double ifit(int nu, double x)
{
    const double u = 2.0 * x - 1.0, u2 = 2.0 * u;
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int j = SWIM_IFIT_I0_F64_N - 1; j >= 1; --j) {
        const double cj = nu ? swim_ifit_i1_f64[j] : swim_ifit_i0_f64[j];
        const double b0 = fma(u2, b1, cj - b2);
        b2 = b1;
        b1 = b0;
    }
    const double c0 = nu ? swim_ifit_i1_f64[0] : swim_ifit_i0_f64[0];
    return fma(u, b1, c0 - b2);
}

// Ascending series of fixed length in y = z^2/4 (A&S 9.6.10, 9.6.13),
// summed by Horner's rule with compile-time coefficients (no divisions, no
// data-dependent exits): all terms are positive, and the first omitted term
// is below 1e-19 of the sum on the range each serves (z <= 8 for I0 and I1,
// 24 terms; z <= 2 for the K0 pieces and the (I0 - 1) series, 16 terms).
constexpr int NSER_I = 24, NSER_K = 16;
struct BesselSeries {
    double i0[NSER_I];  // 1/(k!)^2:                 I0 = sum i0_k y^k
    double i1[NSER_I];  // 1/(k!(k+1)!):             I1 = (z/2) sum i1_k y^k
    double hk[NSER_K];  // H_k/(k!)^2, H_k = sum_{j<=k} 1/j
    double iq[NSER_K];  // 1/((k+1)!)^2:             (I0 - 1)/y = sum iq_k y^k
    constexpr BesselSeries() : i0(), i1(), hk(), iq()
    {
        double a = 1.0, b = 1.0, h = 0.0;
        for (int k = 0; k < NSER_I; ++k) {
            i0[k] = a;
            i1[k] = b;
            if (k < NSER_K) {
                hk[k] = h * a;
                iq[k] = a / ((double)(k + 1) * (double)(k + 1));
            }
            a /= (double)(k + 1) * (double)(k + 1);
            b /= (double)(k + 1) * (double)(k + 2);
            h += 1.0 / (double)(k + 1);
        }
    }
};
static constexpr BesselSeries BSER{};
template <int N> SWIM_HD double horner(const double (&c)[N], double y)
{
    double s = c[N - 1];
#pragma unroll
    for (int k = N - 2; k >= 0; --k) s = fma(s, y, c[k]);
    return s;
}

// ---------------------------------------------------------------------------
// per-system constants
// ---------------------------------------------------------------------------

// exponent m of the FP32 table scale: rho = 2^m is the smallest power of two
// above 1/eps (eps = f 2^e with f in [1/2, 1): m = 1 - e), so sigma = rho^2
// has sigma eps^2 = 4 f^2 in [1, 4).  Exact, so host and device agree.
SWIM_HD int tab_scale_exp(double eps)
{
    int e = 0;
    frexp(eps, &e);
    return 1 - e;
}

template <typename T> struct alignas(16) SysConst {
    T a2, e2, inv_e2, half_inv_e2;   // alpha^2, eps^2, 1/eps^2, 1/(2 eps^2)
    T w0, inv_a2;                    // alpha^2 eps^2, 1/alpha^2 (0 if alpha = 0)
    T cpi, c2pi;                     // c/pi, c/(2 pi)
    T K0z0, q0, h1c, paper;          // K0(alpha eps), Q(w0), H1(0); 1: the paper's blob
    T ts, its, tr, eps;              // FP32 table scale sigma = rho^2, 1/sigma, rho = 2^m; eps
    T U[NT_MAX];                     // U(t) = t * sum_n U[n] t^n
    T V[NT_MAX];                     // V(t) = sum_n V[n] t^n
    // FP32 constants of the paper's blob at alpha > 0 (paper = 0 there): the
    // direct evaluation, used only beyond the table's last octave (r > 2^21
    // eps), takes the blob of the reading above, whose kernel differs from
    // the paper blob's there by O(eps^2/r^2) apart from the constant
    // H1(0); hoff = H1(0) of that blob - H1(0) of the paper's is added to Ht.
    // 0 for every other system.
    T hoff;
};

// power-series coefficients in w of I0, P0 = sum_k psi(k+1) w^k/(4^k (k!)^2),
// A = z I1 and B = sum_{m>=1} [psi(m) + psi(m+1)] w^m/(4^m (m-1)! m!), the
// ascending series of the K0/K1 closed forms, fixed at compile time
struct SetupSeries {
    double I0[NSER_SETUP], P0[NSER_SETUP], A[NSER_SETUP], B[NSER_SETUP];
    constexpr SetupSeries() : I0(), P0(), A(), B()
    {
        double psi = -EULER_GAMMA;  // psi(k+1)
        for (int k = 0; k < NSER_SETUP; ++k) {
            const double ik = 1.0 / (pow4(k) * fact(k) * fact(k));
            I0[k] = ik;
            P0[k] = psi * ik;
            if (k > 0) {
                const double am = 1.0 / (pow4(k) * fact(k - 1) * fact(k));  // 1/(4^m (m-1)! m!), m = k
                A[k] = 2.0 * am;
                B[k] = ((psi - 1.0 / k) + psi) * am;                         // psi(m) + psi(m+1)
            }
            psi += 1.0 / (k + 1);
        }
    }
};
static constexpr SetupSeries SETUP_SERIES{};

// FP64 values of K0, K1 and Q at small or large argument (set-up only)
SWIM_HD void bessel_k01_q_f64(double z, double* K0, double* K1, double* Q)
{
    if (z <= 2.0) {
        // the ascending series in w = z^2 (A&S 9.6.13, 9.6.11), NSER_K
        // terms: their first omitted term is below 1e-24
        const double w = z * z, L = log(0.25 * w);
        double I0 = 0, P0 = 0, A = 0, B = 0;
#pragma unroll
        for (int k = NSER_K - 1; k >= 0; --k) {
            I0 = fma(I0, w, SETUP_SERIES.I0[k]);
            P0 = fma(P0, w, SETUP_SERIES.P0[k]);
            A = fma(A, w, SETUP_SERIES.A[k]);
            B = fma(B, w, SETUP_SERIES.B[k]);
        }
        *K0 = -0.5 * L * I0 + P0;
        *Q = 0.5 * L * A - B;
        *K1 = (1.0 + *Q) / z;
    } else {
        const double e = exp(-z) / sqrt(z), x = SWIM_KFIT_ZS / z;
        *K0 = e * kfit<double>(0, x);
        *K1 = e * kfit<double>(1, x);
        *Q = z * *K1 - 1.0;
    }
}

// reciprocals 1/(k+1) for the series recurrences of the set-up (a
// multiplication per term instead of an FP64 division)
struct PbRecip {
    double lin[80];
    constexpr PbRecip() : lin()
    {
        for (int k = 0; k < 80; ++k) lin[k] = 1.0 / (double)(k + 1);
    }
};
static constexpr PbRecip PB_RECIP{};


// Taylor coefficients at w0 of a power series p(w) = sum_m p_m w^m:
// phat_n = sum_{m>=n} C(m, n) p_m w0^(m-n)
SWIM_HD double taylor_at(const double* p, int M, int n, double w0)
{
    double s = 0.0, binom = 1.0, wp = 1.0;  // C(m, n), w0^(m-n) for m = n
    for (int m = n; m < M; ++m) {
        s += binom * p[m] * wp;
        binom = binom * (m + 1) * PB_RECIP.lin[m - n];  // C(m+1, n) = C(m, n) (m+1)/(m+1-n)
        wp *= w0;
    }
    return s;
}

// ---------------------------------------------------------------------------
// The paper's blob phi = 3 eps^3 / (2 pi R^5) (eq. eqnblob) for alpha > 0,
// whose regularized Brinkmanlet has no closed form.  g, the solution of
// (Delta - alpha^2) g = phi that vanishes at infinity, is phi convolved with
// -K0(alpha r)/(2 pi); the angular average of K0(alpha |x - y|) is
// I0(alpha s<) K0(alpha s>) (Graf's addition theorem), so with z = alpha r
//   g(r) = -[K0(z) A(r) + I0(z) B(r)],
//   A = int_0^r phi I0(alpha s) s ds,   B = int_r^inf phi K0(alpha s) s ds,
//   r g'(r) = z [K1(z) A - I1(z) B].
// The equation integrated over the disc of radius r gives
// r g' - alpha^2 M = m/(2 pi), M = int_0^r s g ds, m = 1 - eps^3/R^3 the blob
// mass inside r; for z <= 2 M is formed as
//   M = Cq + r^2 [q(z)/z^2] A - r^2 [I1(z)/z] B,
//   Cq = int_0^r phi s (I0(alpha s) - 1)/alpha^2 ds,
// which adds no two nearly equal terms.  The integrals are taken in
// u = asinh(s/eps), in which phi s ds = (3/2pi) sinh u / cosh^4 u du (poles
// pi/2 off the real axis), by 10-point Gauss-Legendre panels at most 1/2
// wide in u, and at most 1 + x/4 wide in x = alpha |s - r|, over which
// exp(-x) (the ratio of the Bessel factors) varies.  A and B are carried as
// As = exp(-z) A and Bs = exp(z) B, so nothing overflows; each integral stops
// where its integrand has fallen below e^-42 of its value at s = r.  Near
// contact (delta = r^2/eps^2 < 1/4) g is its power series in delta, whose
// coefficients the equation gives from gam_0 = g(0):
//   gam_{n+1} = eps^2 (phi_n + alpha^2 gam_n) / (4 (n+1)^2),
//   phi_n = 3/(2 pi eps^2) C(-5/2, n).
// All of this runs in FP64 and costs ~1e3 Bessel evaluations per kernel
// value: it builds the FP32 tables once per system and is the direct FP64
// evaluation.
// ---------------------------------------------------------------------------
constexpr double GL10_X[5] = {0.14887433898163122, 0.4333953941292472, 0.6794095682990244,
                              0.8650633666889845, 0.9739065285171717};
constexpr double GL10_W[5] = {0.295524224714753, 0.2692667193099965, 0.219086362515982,
                              0.14945134915058036, 0.06667134430868807};
constexpr int PB_NSER = 32;  // near-contact series length (delta < 1/4)

// exp(-z) I0(z), exp(-z) I1(z): the ascending series (A&S 9.6.10,
// positive terms) for z <= 8, the Chebyshev fits of sqrt(z) exp(-z) I_nu(z)
// in 8/z above (swim_kfit.h)
SWIM_HD void bessel_i01e_f64(double z, double* i0e, double* i1e)
{
    if (z <= SWIM_IFIT_IS) {
        const double y = 0.25 * z * z, e = exp(-z);
        *i0e = horner(BSER.i0, y) * e;
        *i1e = 0.5 * z * horner(BSER.i1, y) * e;
    } else {
        const double c = 1.0 / sqrt(z), x = SWIM_IFIT_IS / z;
        *i0e = c * ifit(0, x);
        *i1e = c * ifit(1, x);
    }
}

// exp(z) K0(z), exp(z) K1(z)
SWIM_HD void bessel_k01e_f64(double z, double* k0e, double* k1e)
{
    if (z <= SWIM_KFIT_ZS) {
        double K0, K1, Q;
        bessel_k01_q_f64(z, &K0, &K1, &Q);
        const double e = exp(z);
        *k0e = K0 * e;
        *k1e = K1 * e;
    } else {
        const double c = 1.0 / sqrt(z), x = SWIM_KFIT_ZS / z;
        *k0e = c * kfit<double>(0, x);
        *k1e = c * kfit<double>(1, x);
    }
}

// sinh(u) and the density (3/2pi) sinh u / cosh^4 u from one expm1
// (e^u - e^-u = em + em/e with em = e^u - 1: no cancellation at small u)
SWIM_HD void pb_point(double u, double* sh, double* dens)
{
    const double em = expm1(u), e = em + 1.0;
    const double sn = 0.5 * (em + em / e), c = 0.5 * (e + 1.0 / e), c2 = c * c;
    *sh = sn;
    *dens = (1.5 / PI) * sn / (c2 * c2);
}


// K0(x) e^z for x >= z >= 0: the ascending series (A&S 9.6.13) times ez = e^z
// for x <= 2, the K0 fit times e^(z - x) above
SWIM_HD double pb_k0x(double x, double z, double ez)
{
    if (x <= SWIM_KFIT_ZS) {
        const double y = 0.25 * x * x, L = log(0.5 * x) + EULER_GAMMA;
        double i0 = 0.0, sp = 0.0;  // sum y^k/(k!)^2, sum H_k y^k/(k!)^2
#pragma unroll
        for (int k = NSER_K - 1; k >= 0; --k) {
            i0 = fma(i0, y, BSER.i0[k]);
            sp = fma(sp, y, BSER.hk[k]);
        }
        return (sp - L * i0) * ez;
    }
    return kfit<double>(0, SWIM_KFIT_ZS / x) * exp(z - x) / sqrt(x);
}

// I0(x) e^-z for 0 <= x <= z: the ascending series times enz = e^-z for
// x <= 8, the fit of sqrt(x) e^-x I0(x) times e^(x - z) / sqrt(x) above
SWIM_HD double pb_i0x(double x, double z, double enz)
{
    if (x <= SWIM_IFIT_IS) return horner(BSER.i0, 0.25 * x * x) * enz;
    return ifit(0, SWIM_IFIT_IS / x) * exp(x - z) / sqrt(x);
}

// Panel rule: widest panel in u and the cut-off exponent.  The direct FP64
// evaluation takes (1/2, 42): ~1e-15 relative.  The FP32 tables, whose
// cubic pieces are good to ~1e-7, are built with (3/2, 26): 10-point rules
// on panels 3/4 wide in half-width against poles pi/2 off the axis leave
// ~1e-13, the cut-off e^-26 ~5e-12, at about a third of the panels.
struct PbRule {
    double du, cut;
};
constexpr PbRule PB_EXACT = {0.5, 42.0};
constexpr PbRule PB_TABLE = {1.5, 26.0};

// exp(alpha r) int_{u0}^inf (3/2pi) sinh u/cosh^4 u K0(alpha eps sinh u) du
SWIM_HD double pb_outer(double alpha, double eps, double r, double u0, PbRule q = PB_EXACT)
{
    const double z = alpha * r, ez = exp(fmin(z, SWIM_KFIT_ZS));
    double b = 0.0, ul = u0;
    for (int p = 0; p < 400; ++p) {
        const double sl = eps * sinh(ul), x = alpha * (sl - r);
        if (x + 3.0 * (ul - u0) > q.cut) break;
        const double uh = fmin(ul + q.du, asinh((sl + (1.0 + 0.25 * x) / alpha) / eps));
        const double hm = 0.5 * (uh - ul), ct = 0.5 * (uh + ul);
        for (int i = 0; i < 10; ++i) {
            const double u = i < 5 ? ct - hm * GL10_X[4 - i] : ct + hm * GL10_X[i - 5];
            const double w = i < 5 ? GL10_W[4 - i] : GL10_W[i - 5];
            double sh, dens;
            pb_point(u, &sh, &dens);
            b += hm * w * dens * pb_k0x(alpha * eps * sh, z, ez);
        }
        ul = uh;
    }
    return b;
}

// g(0) = -int_0^inf phi K0(alpha s) s ds; panels [2^-(j+2), 2^-(j+1)] in u
// towards the logarithm of K0 at s = 0, then pb_outer from u = 1/2
SWIM_HD double pb_g0(double alpha, double eps)
{
    double b = 0.0;
    for (int j = 52; j >= 0; --j) {
        const double ul = ldexp(1.0, -(j + 2)), uh = 2.0 * ul;
        const double hm = 0.5 * (uh - ul), ct = 0.5 * (uh + ul);
        for (int i = 0; i < 10; ++i) {
            const double u = i < 5 ? ct - hm * GL10_X[4 - i] : ct + hm * GL10_X[i - 5];
            const double w = i < 5 ? GL10_W[4 - i] : GL10_W[i - 5];
            double sh, dens;
            pb_point(u, &sh, &dens);
            b += hm * w * dens * pb_k0x(alpha * eps * sh, 0.0, 1.0);
        }
    }
    return -(b + pb_outer(alpha, eps, 0.0, 0.5));
}

// g(0) of the paper's blob in closed form.  The blob's Hankel transform is
// (1 + k eps) exp(-k eps) and (Delta - alpha^2) g = phi, so with a = alpha eps
//   g(0) = -(1/2pi) int_0^inf (1 + x) exp(-x) x / (x^2 + a^2) dx
//        = -(1/2pi) [ gaux(a) + 1 - a faux(a) ],
// faux = Ci(a) sin a - si(a) cos a and gaux = -Ci(a) cos a - si(a) sin a the
// auxiliary functions of the sine and cosine integrals (A&S 5.2.6-5.2.7 and
// their Laplace integrals 5.2.12-5.2.13), si = Si - pi/2, Ci and Si by their
// power series (A&S 5.2.14, 5.2.16; a <= 1 in this library's domain).
SWIM_HD double pb_g0_closed(double a)
{
    const double a2 = a * a;
    double p = a, q = 1.0;  // (-1)^k a^(2k+1)/(2k+1)!, (-1)^k a^(2k)/(2k)!
    double S = 0.0, Cs = 0.0;
    for (int k = 0; k < 16; ++k) {
        S += p * PB_RECIP.lin[2 * k];               // / (2k + 1)
        if (k >= 1) Cs += q * (0.5 * PB_RECIP.lin[k - 1]);  // / (2k)
        p *= -a2 * PB_RECIP.lin[2 * k + 1] * PB_RECIP.lin[2 * k + 2];  // / ((2k+2)(2k+3))
        q *= -a2 * PB_RECIP.lin[2 * k] * PB_RECIP.lin[2 * k + 1];      // / ((2k+1)(2k+2))
    }
    const double Ci = EULER_GAMMA + log(a) + Cs;
    const double si = S - 0.5 * PI;
    const double sn = sin(a), cs = cos(a);
    const double fa = Ci * sn - si * cs;
    const double ga = -Ci * cs - si * sn;
    return -(ga + 1.0 - a * fa) / (2.0 * PI);
}

// g(r) and M(r) for delta >= 1/4
SWIM_HD void pb_gM(double alpha, double eps, double t, double* g, double* M, PbRule q = PB_EXACT)
{
    const double r = sqrt(t), z = alpha * r, ur = asinh(r / eps);
    const bool small = z <= 2.0;
    const double enz = exp(-z);
    double as = 0.0, cq = 0.0, uh = ur;
    for (int p = 0; p < 400 && uh > 0.0; ++p) {
        const double sh = eps * sinh(uh), x = alpha * (r - sh);
        if (x - 3.0 * (ur - uh) > q.cut) break;
        const double sl = sh - (1.0 + 0.25 * x) / alpha;
        const double ul = fmax(fmax(uh - q.du, 0.0), sl > 0.0 ? asinh(sl / eps) : 0.0);
        const double hm = 0.5 * (uh - ul), ct = 0.5 * (uh + ul);
        for (int i = 0; i < 10; ++i) {
            const double u = i < 5 ? ct - hm * GL10_X[4 - i] : ct + hm * GL10_X[i - 5];
            double sh, dens;
            pb_point(u, &sh, &dens);
            const double w = hm * (i < 5 ? GL10_W[4 - i] : GL10_W[i - 5]) * dens;
            const double s = eps * sh, xs = alpha * s;
            as += w * pb_i0x(xs, z, enz);
            if (small) {
                // (I0(xs) - 1)/alpha^2 = (s^2/4) sum_k (xs^2/4)^k / ((k+1)!)^2
                cq += w * 0.25 * s * s * horner(BSER.iq, 0.25 * xs * xs);
            }
        }
        uh = ul;
    }
    const double bs = pb_outer(alpha, eps, r, ur, q);
    double k0e, k1e, i0e, i1e;
    bessel_k01e_f64(z, &k0e, &k1e);
    bessel_i01e_f64(z, &i0e, &i1e);
    *g = -(k0e * as + i0e * bs);
    if (small) {
        double K0, K1, Q;
        bessel_k01_q_f64(z, &K0, &K1, &Q);
        const double ez = exp(z);
        *M = cq + t * (Q / (z * z)) * as * ez - t * (i1e * ez / z) * bs / ez;
    } else {
        const double R = sqrt(t + eps * eps);
        const double m = 1.0 - eps * eps * eps / (R * R * R);
        *M = (z * (k1e * as - i1e * bs) - m / (2.0 * PI)) / (alpha * alpha);
    }
}

// Constants of the closed forms: the reading's blob (blob 0) for every
// alpha, the paper's blob (blob 1) at alpha = 0.
template <typename T> SWIM_HD void sysconst_base(double alpha, double eps, SysConst<T>* out, int blob)
{
    const double a2 = alpha * alpha, e2 = eps * eps, w0 = a2 * e2;
    SysConst<T> C;
    C.hoff = (T)0;
    C.a2 = (T)a2;
    C.e2 = (T)e2;
    C.inv_e2 = (T)(1.0 / e2);
    C.half_inv_e2 = (T)(0.5 / e2);
    C.w0 = (T)w0;
    C.paper = (T)(blob == 1 ? 1 : 0);
    const int m = tab_scale_exp(eps);
    C.ts = (T)ldexp(1.0, 2 * m);
    C.its = (T)ldexp(1.0, -2 * m);
    C.tr = (T)ldexp(1.0, m);
    C.eps = (T)eps;
    for (int n = 0; n < NT_MAX; ++n) { C.U[n] = (T)0; C.V[n] = (T)0; }
    if (alpha == 0.0) {
        C.inv_a2 = (T)0;
        C.cpi = (T)(1.0 / PI);
        C.c2pi = (T)(0.5 / PI);
        C.K0z0 = (T)0;
        C.q0 = (T)0;
        // H1(0): -ln(eps)/(4 pi) for the blob of the reading above;
        // (1 - ln(2 eps))/(4 pi) for the paper's blob
        C.h1c = blob == 1 ? (T)((1.0 - log(2.0 * eps)) / (4.0 * PI)) : (T)(-log(eps) / (4.0 * PI));
        *out = C;
        return;
    }
    const double z0 = alpha * eps;
    double K0, K1, Q0;
    bessel_k01_q_f64(z0, &K0, &K1, &Q0);
    const double c = 1.0 / (z0 * K1);
    C.inv_a2 = (T)(1.0 / a2);
    C.cpi = (T)(c / PI);
    C.c2pi = (T)(0.5 * c / PI);
    C.K0z0 = (T)K0;
    C.q0 = (T)Q0;
    C.h1c = (T)(c * K0 / (4.0 * PI));
    const double* pI0 = SETUP_SERIES.I0;
    const double* pP0 = SETUP_SERIES.P0;
    const double* pA = SETUP_SERIES.A;
    const double* pB = SETUP_SERIES.B;
    const double L0 = log(0.25 * w0);
    // U(t) = sum_{n>=1} [-L0/2 I0hat_n + P0hat_n] a2^n t^n,  stored as U[n-1]
    // V(t) = sum_{n>=2} (n-1) [L0/2 Ahat_n - Bhat_n] a2^(n-1) t^(n-2), stored as V[n-2]
    double a2n = a2;  // a2^n for n = 1
    for (int n = 1; n <= NT_MAX; ++n) {
        const double u = -0.5 * L0 * taylor_at(pI0, NSER_SETUP, n, w0) + taylor_at(pP0, NSER_SETUP, n, w0);
        C.U[n - 1] = (T)(u * a2n);
        a2n *= a2;
    }
    double a2m = a2;  // a2^(n-1) for n = 2
    for (int n = 2; n < NT_MAX + 2; ++n) {
        const double v = (n - 1) * (0.5 * L0 * taylor_at(pA, NSER_SETUP, n, w0) - taylor_at(pB, NSER_SETUP, n, w0));
        C.V[n - 2] = (T)(v * a2m);
        a2m *= a2;
    }
    *out = C;
}

// the paper's blob at alpha > 0, given g(0)
template <typename T> SWIM_HD void sysconst_paper(double alpha, double eps, double g0, SysConst<T>* out)
{
    if constexpr (sizeof(T) == 8) {
        const double a2 = alpha * alpha, e2 = eps * eps;
        SysConst<T> C{};
        C.a2 = a2;
        C.e2 = e2;
        C.inv_e2 = 1.0 / e2;
        C.half_inv_e2 = 0.5 / e2;
        C.w0 = a2 * e2;
        C.inv_a2 = 1.0 / a2;
        C.K0z0 = g0;
        C.h1c = -0.5 * g0;
        C.paper = 2.0;
        const int m = tab_scale_exp(eps);
        C.ts = ldexp(1.0, 2 * m);
        C.its = ldexp(1.0, -2 * m);
        C.tr = ldexp(1.0, m);
        C.eps = eps;
        *out = C;
    } else {
        SysConst<double> R;
        sysconst_base<double>(alpha, eps, &R, 0);
        sysconst_base<T>(alpha, eps, out, 0);
        out->h1c = (T)(-0.5 * g0);
        out->hoff = (T)(R.h1c + 0.5 * g0);
    }
}

// Computes the constants of one system in FP64 and rounds them to T.
// Requires alpha >= 0, eps > 0, alpha * eps <= 1 (checked by the caller).
// blob 1 selects the paper's blob 3 eps^3 / (2 pi R^5) (eq. eqnblob): closed
// forms at alpha = 0; for alpha > 0 the FP64 constants select the quadrature
// (paper = 2, K0z0 = g(0)) and the FP32 ones those of the reading's blob with
// H1(0) and hoff of the paper's (its FP32 values come from the tables).
template <typename T> SWIM_HD void sysconst_compute(double alpha, double eps, SysConst<T>* out, int blob = 0)
{
    if (blob == 1 && alpha > 0.0)
        sysconst_paper<T>(alpha, eps, pb_g0_closed(alpha * eps), out);
    else
        sysconst_base<T>(alpha, eps, out, blob);
}

// FP64 constants rounded to T field by field (what sysconst_base<T> forms)
template <typename T> SWIM_HD void sysconst_cast(const SysConst<double>& D, SysConst<T>* out)
{
    SysConst<T> C;
    C.a2 = (T)D.a2;
    C.e2 = (T)D.e2;
    C.inv_e2 = (T)D.inv_e2;
    C.half_inv_e2 = (T)D.half_inv_e2;
    C.w0 = (T)D.w0;
    C.inv_a2 = (T)D.inv_a2;
    C.cpi = (T)D.cpi;
    C.c2pi = (T)D.c2pi;
    C.K0z0 = (T)D.K0z0;
    C.q0 = (T)D.q0;
    C.h1c = (T)D.h1c;
    C.paper = (T)D.paper;
    C.ts = (T)D.ts;
    C.its = (T)D.its;
    C.tr = (T)D.tr;
    C.eps = (T)D.eps;
    for (int n = 0; n < NT_MAX; ++n) {
        C.U[n] = (T)D.U[n];
        C.V[n] = (T)D.V[n];
    }
    C.hoff = (T)D.hoff;
    *out = C;
}

// the constants in T and, if out64 is not null, in FP64 (one FP64 pass for
// both; g(0) of the paper's blob integrated once)
template <typename T>
SWIM_HD void sysconst_compute2(double alpha, double eps, SysConst<T>* out, SysConst<double>* out64, int blob)
{
    if (blob == 1 && alpha > 0.0) {
        const double g0 = pb_g0_closed(alpha * eps);
        sysconst_paper<T>(alpha, eps, g0, out);
        if (out64) sysconst_paper<double>(alpha, eps, g0, out64);
        return;
    }
    if (out64) {
        sysconst_base<double>(alpha, eps, out64, blob);
        sysconst_cast<T>(*out64, out);
    } else {
        sysconst_base<T>(alpha, eps, out, blob);
    }
}

// ---------------------------------------------------------------------------
// per-pair kernel values:  Ht = H1(t) - H1(0),  H2(t)
// t = 0 returns Ht = 0 and a finite H2 (the pair contributes nothing then).
// ---------------------------------------------------------------------------
SWIM_HD float log1p_t(float x) { return log1pf(x); }
SWIM_HD double log1p_t(double x) { return log1p(x); }
SWIM_HD float exp_t(float x) { return expf(x); }
SWIM_HD double exp_t(double x) { return exp(x); }
SWIM_HD float sqrt_t(float x) { return sqrtf(x); }
SWIM_HD double sqrt_t(double x) { return sqrt(x); }

// Fast FP32 forms for the pair loop.  On the device they are single VALU
// transcendentals (v_rcp_f32, v_log_f32, v_sqrt_f32, v_rsq_f32; about 1 ulp);
// the host pass of this header (used only by the host test hook) takes the
// libm equivalents.  FP64 keeps the correctly rounded library calls.
SWIM_HD float rcp_fast(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
SWIM_HD double rcp_fast(double x) { return 1.0 / x; }
SWIM_HD float sqrt_fast(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return sqrtf(x);
#endif
}
SWIM_HD double sqrt_fast(double x) { return sqrt(x); }
SWIM_HD float rsqrt_fast(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsqf(x);
#else
    return 1.0f / sqrtf(x);
#endif
}
SWIM_HD double rsqrt_fast(double x) { return 1.0 / sqrt(x); }
// log1p(x) for x >= 1/4: u = 1 + x is rounded, u - 1 is exact, and the
// factor x / (u - 1) restores the part of x the rounding dropped.
SWIM_HD float log1p_fast(float x)
{
    const float u = 1.0f + x;
#if defined(__HIP_DEVICE_COMPILE__)
    const float l = __builtin_amdgcn_logf(u) * 0.693147180559945309f;
#else
    const float l = logf(u);
#endif
    return l * (x * rcp_fast(u - 1.0f));
}
SWIM_HD double log1p_fast(double x) { return log1p(x); }
SWIM_HD float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
SWIM_HD double fma_t(double a, double b, double c) { return fma(a, b, c); }

template <typename T, int N>
SWIM_HD T horner_const(T x, double (*cf)(int))
{
    T s = (T)cf(N - 1);
#pragma unroll
    for (int k = N - 2; k >= 0; --k) s = fma_t(s, x, (T)cf(k));
    return s;
}

template <typename T, int N>
SWIM_HD T horner_arr(T x, const T* c)
{
    T s = c[N - 1];
#pragma unroll
    for (int k = N - 2; k >= 0; --k) s = fma_t(s, x, c[k]);
    return s;
}

template <typename T>
SWIM_HD void kernel_small_z(const SysConst<T>& C, T t, T w, T& Ht, T& H2)
{
    using P = Prec<T>;
    const T delta = t * C.inv_e2;
    T ell, lam, S2;
    if (delta >= (T)P::DSMALL || delta == (T)0) {
        // delta = 0 is the self pair: its value is multiplied by zero, so
        // lambda and S2 are taken at the clamped delta
        const T dc = delta >= (T)P::DSMALL ? delta : (T)P::DSMALL;
        const T lc = log1p_fast(dc);
        ell = delta == (T)0 ? (T)0 : lc;
        const T rd = rcp_fast(dc);
        lam = lc * rd;
        S2 = ((T)1 - lam) * rd;
    } else {
        // near contact (rare): log1p(d) = 2 atanh(y), y = d/(2+d), so with
        // Y = y^2 and Pa(Y) = sum_{m>=1} Y^(m-1)/(2m+1):
        //   lambda = 2 (1 + Y Pa)/(2+d),  S2 = 1/(2+d) - 2 d Pa/(2+d)^3,
        // both free of cancellation
        const T r2 = (T)1 / ((T)2 + delta);
        const T y = delta * r2, Y = y * y;
        T pa = (T)(1.0 / (2 * P::NA + 1));
#pragma unroll
        for (int m = P::NA - 1; m >= 1; --m) pa = fma_t(pa, Y, (T)(1.0 / (2 * m + 1)));
        const T Q = fma_t(Y, pa, (T)1);
        ell = (T)2 * y * Q;
        lam = (T)2 * Q * r2;
        S2 = r2 - (T)2 * delta * r2 * r2 * r2 * pa;
    }
    // Abar(w) and its derivative in one Horner pass; D = w Abar' and
    // I0 = 2 (Abar + w Abar') follow from the series coefficients
    T Ab = (T)c_Abar(P::NW - 1), dA = (T)0;
#pragma unroll
    for (int k = P::NW - 2; k >= 0; --k) {
        dA = fma_t(dA, w, Ab);
        Ab = fma_t(Ab, w, (T)c_Abar(k));
    }
    const T Dw = w * dA;
    const T I0w = (T)2 * (Ab + Dw);
    const T Ut = t * horner_arr<T, P::NT>(t, C.U);
    const T Vt = horner_arr<T, P::NT>(t, C.V);
    H2 = C.cpi * fma_t(C.half_inv_e2, fma_t(Dw, lam, Ab * S2), Vt);
    const T gt = -C.c2pi * fma_t((T)-0.5 * ell, I0w, Ut);
    Ht = (T)-0.5 * fma_t(t, H2, gt);
}

template <typename T>
SWIM_HD void kernel_large_z(const SysConst<T>& C, T t, T w, T& Ht, T& H2)
{
    const T z = sqrt_fast(w);
    const T rz = rcp_fast(z);
    const T e = exp_t(-z) * rsqrt_fast(z);
    const T x = (T)SWIM_KFIT_ZS * rz;
    const T K0 = e * kfit<T>(0, x);
    const T K1 = e * kfit<T>(1, x);
    const T g = -C.c2pi * K0;
    const T gt = -C.c2pi * (K0 - C.K0z0);
    const T q = fma_t(z, K1, (T)-1);
    const T rt = rcp_fast(t);
    const T Mt = C.c2pi * (q - C.q0) * C.inv_a2 * rt;  // M(r)/r^2
    H2 = (g - (T)2 * Mt) * rt;
    Ht = (T)-0.5 * fma_t(t, H2, gt);
}

// The paper's blob in the Stokes limit (G = (ln(R + eps) - eps/R)/(2 pi),
// H1 = M/r^2 - G, H2 = (G - 2M/r^2)/r^2), in cancellation-free form:
//   H2 = (R + 2 eps) / (4 pi R (R + eps)^2),
//   Ht = (1/2pi) [ -1/2 log1p(t / (2 eps (R + eps))) - (3R + 4 eps) t / (4 R (R + eps)^2) ]
template <typename T>
SWIM_HD void kernel_paper_stokes(const SysConst<T>& C, T t, T& Ht, T& H2)
{
    const T e = C.eps;
    const T R = sqrt_t(t + C.e2);
    const T Re = R + e;
    const T q = (T)1 / (R * Re * Re);
    H2 = (T)(0.25 / PI) * (R + (T)2 * e) * q;
    Ht = (T)(0.5 / PI) * ((T)-0.5 * log1p_t(t / ((T)2 * e * Re)) - (T)0.25 * ((T)3 * R + (T)4 * e) * t * q);
}

// The paper's blob at alpha > 0 (FP64 constants with paper = 2): near
// contact the series of g, Ht = -sum_{n>=1} gam_n delta^n (2n+1)/(2(n+1)),
// H2 = (1/eps^2) sum_{n>=1} gam_n delta^(n-1) n/(n+1); beyond it
// H1 = M/r^2 - g, H2 = (g - 2M/r^2)/r^2 from the quadrature.  Not inlined:
// it is large and only systems of this blob call it.
__host__ __device__ __attribute__((noinline)) inline void kernel_paper_brinkman(const SysConst<double>& C, double t,
                                                                              double& Ht, double& H2,
                                                                              PbRule q = PB_EXACT)
{
    const double delta = t * C.inv_e2;
    if (delta < 0.25) {
        double gam = C.K0z0, phin = 1.5 / PI * C.inv_e2, p = 1.0, ht = 0.0, h2 = 0.0;
        for (int n = 0; n + 1 < PB_NSER; ++n) {
            gam = C.e2 * (phin + C.a2 * gam) / (4.0 * (n + 1) * (n + 1));  // gam_{n+1}
            phin *= (-2.5 - n) / (n + 1);
            h2 += gam * p * (n + 1) / (n + 2);
            p *= delta;
            ht -= gam * p * (2 * n + 3) / (2.0 * (n + 2));
        }
        Ht = ht;
        H2 = h2 * C.inv_e2;
        return;
    }
    double g, M;
    pb_gM(sqrt(C.a2), C.eps, t, &g, &M, q);
    const double Mt = M / t;
    H2 = (g - 2.0 * Mt) / t;
    Ht = Mt - g - C.h1c;
}

template <typename T>
SWIM_HD void kernel_eval(const SysConst<T>& C, T t, T& Ht, T& H2)
{
    if (C.paper != (T)0) {
        if constexpr (sizeof(T) == 8) {
            if (C.paper != 1.0) {
                kernel_paper_brinkman(C, t, Ht, H2);
                return;
            }
        }
        kernel_paper_stokes<T>(C, t, Ht, H2);
        return;
    }
    const T w = fma_t(C.a2, t, C.w0);
    if (w <= (T)(SWIM_KFIT_ZS * SWIM_KFIT_ZS))
        kernel_small_z<T>(C, t, w, Ht, H2);
    else
        kernel_large_z<T>(C, t, w, Ht, H2);
    if constexpr (sizeof(T) == 4) Ht += C.hoff;
}

// ---------------------------------------------------------------------------
// FP32 evaluation by table.  In the variable v = 1 + sigma t (t = r^2, sigma
// the system's power of four with sigma eps^2 in [1, 4)) the functions
// Ht(t) and H2(t) are smooth on every interval
// [2^e (1 + j/16), 2^e (1 + (j+1)/16)), e = 0..TAB_OCT-1, j = 0..15, whose
// index is read straight from the bits of the float v (exponent and the top
// four mantissa bits) and whose local coordinate is the rest of the mantissa,
// taken as the integer u in [0, 2^19) (the interval coordinate times 2^19).
// On each interval both functions are the cubic through their values at the
// Chebyshev-Lobatto nodes 0, 1/4, 3/4, 1 of the interval, evaluated once per
// system in FP64 by kernel_eval<double> (for the paper's blob at alpha > 0
// by its quadrature with the table's panel rule).  The relative width 1/16 of an
// interval bounds the interpolation error by about 4e-3 (1/16)^4 max|f''''|
// in units of the function's own scale (about 1e-7 for the log and 1/t
// behaviour of these kernels); rounding the coefficients to FP32 adds one
// unit roundoff.  The stored coefficients absorb exact powers of two: the
// 2^-19 of u in every power of u, and 1/sigma in those of H2, so that with
// positions scaled by rho = sqrt(sigma) (d' = rho d, v = |d'|^2 + 1) a pair
// contributes Ht F + H2' (F . d') d' with H2' = H2 / sigma.  Entry TAB_N is
// all zero: pairs beyond the last octave index it (and contribute nothing)
// and fall back to the direct evaluation.  Far octaves cost nothing per
// pair, and runs that drift far apart before they stop stay on the table.
// ---------------------------------------------------------------------------
#ifndef SWIM_TAB_M
#define SWIM_TAB_M 4
#endif
constexpr int TAB_M = SWIM_TAB_M;            // intervals per octave: 2^TAB_M
// octaves of v, which covers [1, 2^44): positions stay within 1e3 of the
// origin (runs stop beyond), so pair distances are below 2830 and every pair
// of a system with eps >= 1.4e-3 (N <= 1100 at eps = 1.5 ds) is in the table
constexpr int TAB_OCT = 44;
constexpr int TAB_N = TAB_OCT << TAB_M;      // intervals per system
constexpr int TAB_SHIFT = 23 - TAB_M;        // mantissa bits of u
constexpr uint32_t TAB_BIAS = 0x3F800000u >> TAB_SHIFT;  // bits(1.0f) >> TAB_SHIFT
constexpr uint32_t TAB_END = TAB_BIAS + TAB_N;           // first index beyond the table
struct alignas(16) TabE {
    float h[4];  // Ht(u) = h0 + u (h1 + u (h2 + u h3))
    float g[4];  // H2(u) / sigma
};
static_assert(sizeof(TabE) == 32, "table entries are addressed as index << 5");
// one system's table (entry TAB_N: zeros); h0lo[i] = Ht at the start of
// interval i minus its FP32 value e[i].h[0], for the kernels that accumulate
// in FP64
struct alignas(16) TabSys {
    TabE e[TAB_N + 1];
    float h0lo[TAB_N + 1];
};

// cubic through (0, f0), (1/4, f1), (3/4, f2), (1, f3): monomial
// coefficients of the local coordinate scaled by sc (c_k sc^k), times mul
SWIM_HD void cubic_lobatto(const double (&f)[4], double sc, double mul, float (&c)[4])
{
    // Newton divided differences on the nodes 0, 1/4, 3/4, 1
    const double x1 = 0.25, x2 = 0.75;
    const double d01 = (f[1] - f[0]) / x1;
    const double d12 = (f[2] - f[1]) / (x2 - x1);
    const double d23 = (f[3] - f[2]) / (1.0 - x2);
    const double d012 = (d12 - d01) / x2;
    const double d123 = (d23 - d12) / (1.0 - x1);
    const double d0123 = d123 - d012;
    // p = f0 + d01 u + d012 u (u - x1) + d0123 u (u - x1) (u - x2)
    c[0] = (float)(mul * f[0]);
    c[1] = (float)(mul * sc * (d01 - d012 * x1 + d0123 * x1 * x2));
    c[2] = (float)(mul * sc * sc * (d012 - d0123 * (x1 + x2)));
    c[3] = (float)(mul * sc * sc * sc * d0123);
}

// FP64 kernel values at node k (coordinate 0, 1/4, 3/4, 1) of interval i
// (i <= TAB_N; node 0 of i = TAB_N is the end of the last interval).  t = 0
// is taken as a vanishing positive t, whose evaluation follows the
// near-contact series and gives the limits H2(0) and Ht(0) = 0.  The end
// of interval i and the start of interval i + 1 are the same t exactly
// (dyadic values of v), so either evaluation serves both.
SWIM_HD void tab_node(const SysConst<double>& C, int i, int k, double& fh, double& fg)
{
    const int e = i >> TAB_M, j = i & ((1 << TAB_M) - 1);
    const double a = ldexp(1.0, e);
    const double v0 = a * (1.0 + (double)j / (double)(1 << TAB_M)), hv = a / (double)(1 << TAB_M);
    const double un = k == 0 ? 0.0 : k == 1 ? 0.25 : k == 2 ? 0.75 : 1.0;
    const double t = fmax((v0 - 1.0 + hv * un) * C.its, 1e-300);
    if (C.paper == 2.0)
        kernel_paper_brinkman(C, t, fh, fg, PB_TABLE);
    else
        kernel_eval<double>(C, t, fh, fg);
}

// the table entry from its four node values; h0lo, if not null: the FP32
// remainder of the constant coefficient of Ht
SWIM_HD void tab_assemble(const SysConst<double>& C, const double (&fh)[4], const double (&fg)[4], TabE& out,
                          float* h0lo)
{
    const double sc = ldexp(1.0, -TAB_SHIFT);
    cubic_lobatto(fh, sc, 1.0, out.h);
    cubic_lobatto(fg, sc, C.its, out.g);
    if (h0lo) *h0lo = (float)(fh[0] - (double)out.h[0]);
}

// interval i of the table of the system with FP64 constants C (i = TAB_N:
// the zero entry)
SWIM_HD void tab_interval(const SysConst<double>& C, int i, TabE& out, float* h0lo = nullptr)
{
    if (i >= TAB_N) {
        for (int k = 0; k < 4; ++k) out.h[k] = out.g[k] = 0.0f;
        if (h0lo) *h0lo = 0.0f;
        return;
    }
    double fh[4], fg[4];
#pragma unroll 1
    for (int k = 0; k < 4; ++k) tab_node(C, i, k, fh[k], fg[k]);
    tab_assemble(C, fh, fg, out, h0lo);
}

// bits of v = 1 + sigma t: their index bits >> TAB_SHIFT (>= TAB_END beyond
// the table, non-finite t included) and u, the low mantissa bits as a float
SWIM_HD uint32_t tab_bits(float t, float sigma) { return __builtin_bit_cast(uint32_t, fmaf(t, sigma, 1.0f)); }
SWIM_HD float tab_u(uint32_t bits) { return (float)(bits & ((1u << TAB_SHIFT) - 1u)); }

SWIM_HD void tab_eval(const TabE& e, float u, float& Ht, float& H2s)
{
    Ht = fmaf(fmaf(fmaf(e.h[3], u, e.h[2]), u, e.h[1]), u, e.h[0]);
    H2s = fmaf(fmaf(fmaf(e.g[3], u, e.g[2]), u, e.g[1]), u, e.g[0]);
}

// ---------------------------------------------------------------------------
// The paper's blob at alpha > 0: all table nodes of one system in one sweep.
//
// The nodes of the FP32 table (node k: interval k/3 at coordinate 0, 1/4,
// 3/4; node 3 TAB_N the end of the last interval) have increasing r.  With
// A, B and Cq the integrals of pb_gM, each node needs
//   A(r_k) = sum of the integrals of phi I0(alpha s) s over the gaps
//            [r_{m-1}, r_m], m <= k (a prefix sum from s = 0),
//   Cq(r_k) likewise (only where alpha r_k <= 2),
//   B(r_k) = B(r_L) + the gaps m > k up to the last node L of the sweep
//            (a suffix sum; B(r_L) is one tail integral, pb_outer),
// and then g and M follow exactly as in pb_gM.  The gaps are narrow (at
// most 1/64 in u beyond the first octave), so a 6-point Gauss-Legendre rule
// per gap is exact to rounding for the blob's density (poles pi/2 off the
// axis) and for the Bessel factors up to alpha r = PB_ZF (they change by at
// most exp(PB_ZF/64) over a gap).  The sweep covers the nodes with
// delta = t/eps^2 >= 1/4 and alpha r <= PB_ZF; below, g is the near-contact
// series of kernel_paper_brinkman; beyond, the far-field expansion of
// pb_node_far.  Every node value is one gap quadrature and one set of Bessel
// functions instead of a panel quadrature of its own.
// ---------------------------------------------------------------------------
constexpr int PB_NODES = 3 * TAB_N + 1;  // table nodes of one system
constexpr double PB_ZF = 40.0;           // alpha r beyond which the far-field expansion serves
constexpr int PB_NA = 14;                // terms of the far-field expansion
constexpr double GL6_X[3] = {0.23861918608319693, 0.66120938646626448, 0.93246951420315205};
constexpr double GL6_W[3] = {0.46791393457269137, 0.36076157304813894, 0.17132449237916975};

// t = r^2 of table node k (the t of tab_node: node k % 3 of interval k / 3)
SWIM_HD double pb_node_t(double its, int k)
{
    const int i = k / 3, kk = k - 3 * i;
    const int e = i >> TAB_M, j = i & ((1 << TAB_M) - 1);
    const double a = ldexp(1.0, e);
    const double v0 = a * (1.0 + (double)j / (double)(1 << TAB_M)), hv = a / (double)(1 << TAB_M);
    const double un = kk == 0 ? 0.0 : kk == 1 ? 0.25 : 0.75;
    return fmax((v0 - 1.0 + hv * un) * its, 1e-300);
}

// integrals over the gap [ulo, uhi] in u = asinh(s/eps) of the blob measure
// phi s ds = (3/2pi) sinh u/cosh^4 u du times I0(alpha s) (ga), K0(alpha s)
// (gb, if wantB) and (I0(alpha s) - 1)/alpha^2 (gc, if wantC)
SWIM_HD void pb_gap(double alpha, double eps, double ulo, double uhi, bool wantB, bool wantC, double* ga, double* gb,
                    double* gc)
{
    const double hm = 0.5 * (uhi - ulo), ct = 0.5 * (uhi + ulo);
    double A = 0.0, B = 0.0, Cq = 0.0;
#pragma unroll 1
    for (int i = 0; i < 6; ++i) {
        const double u = i < 3 ? ct - hm * GL6_X[2 - i] : ct + hm * GL6_X[i - 3];
        double sh, dens;
        pb_point(u, &sh, &dens);
        const double wd = hm * (i < 3 ? GL6_W[2 - i] : GL6_W[i - 3]) * dens;
        const double s = eps * sh, xs = alpha * s;
        A += wd * pb_i0x(xs, 0.0, 1.0);
        if (wantB) B += wd * pb_k0x(xs, 0.0, 1.0);
        if (wantC) {
            // (I0(xs) - 1)/alpha^2 = (s^2/4) sum_k (xs^2/4)^k / ((k+1)!)^2
            Cq += wd * 0.25 * s * s * horner(BSER.iq, 0.25 * xs * xs);
        }
    }
    *ga = A;
    *gb = B;
    *gc = Cq;
}

// The tail B(r) = int_r^inf phi K0(alpha s) s ds beyond the sweep's last
// node, as np panels in d = u - u(r): panel p of [0, dmax] by 10-point
// Gauss-Legendre.  Its integrand falls like exp(-x - 3 d) with
// x = alpha (s - r), so dmax is where x + 3 d reaches 44 (at most 15): the
// neglected remainder is below e^-44 of the integrand at s = r, and a panel
// of dmax/np (np = 64) changes the exponent by at most (alpha r + 3) dmax/np.
SWIM_HD double pb_tail_dmax(double alpha, double eps, double r)
{
    const double u0 = asinh(r / eps);
    double lo = 0.0, hi = 15.0;
    for (int it = 0; it < 24; ++it) {
        const double d = 0.5 * (lo + hi);
        const double x = alpha * (eps * sinh(u0 + d) - r);
        if (x + 3.0 * d > 44.0) hi = d;
        else lo = d;
    }
    return hi;
}
SWIM_HD double pb_tail_panel(double alpha, double eps, double r, int p, int np)
{
    const double u0 = asinh(r / eps), dmax = pb_tail_dmax(alpha, eps, r);
    const double ul = u0 + dmax * p / np, uh = u0 + dmax * (p + 1) / np;
    const double hm = 0.5 * (uh - ul), ct = 0.5 * (uh + ul);
    double b = 0.0;
#pragma unroll 1
    for (int i = 0; i < 10; ++i) {
        const double u = i < 5 ? ct - hm * GL10_X[4 - i] : ct + hm * GL10_X[i - 5];
        double sh, dens;
        pb_point(u, &sh, &dens);
        b += hm * (i < 5 ? GL10_W[4 - i] : GL10_W[i - 5]) * dens * pb_k0x(alpha * eps * sh, 0.0, 1.0);
    }
    return b;
}

// node values Ht, H2 from A(r), B(r), Cq(r) (the formulas of pb_gM)
SWIM_HD void pb_node_sweep(double alpha, double eps, double t, double A, double B, double Cq, double h1c, double& fh,
                           double& fg)
{
    const double r = sqrt(t), z = alpha * r;
    double K0, K1, Q, i0e, i1e;
    bessel_k01_q_f64(z, &K0, &K1, &Q);
    bessel_i01e_f64(z, &i0e, &i1e);
    const double ez = exp(z), I0 = i0e * ez, I1 = i1e * ez;
    const double g = -(K0 * A + I0 * B);
    double M;
    if (z <= 2.0) {
        M = Cq + t * (Q / (z * z)) * A - t * (I1 / z) * B;
    } else {
        const double R = sqrt(t + eps * eps);
        const double m = 1.0 - eps * eps * eps / (R * R * R);
        M = (z * (K1 * A - I1 * B) - m / (2.0 * PI)) / (alpha * alpha);
    }
    const double Mt = M / t;
    fg = (g - 2.0 * Mt) / t;
    fh = Mt - g - h1c;
}

// Far field (alpha r > PB_ZF).  There g is the decaying particular solution
//   g = -sum_n Delta^n phi / alpha^(2n+2)
// up to a multiple of K0(alpha r) (below exp(-PB_ZF)), and Delta maps
// (R^2)^-q to 4 q^2 (R^2)^(-q-1) - 4 q (q+1) eps^2 (R^2)^(-q-2), so with
// w = 1/(alpha R)^2, y = eps^2/R^2:
//   g    = -(3 eps^3/(2 pi alpha^2 R^5)) sum_n w^n sum_j d_nj y^j,
//   r g' = -(3 eps^3/(2 pi alpha^2 R^5)) (r^2/R^2) sum_n w^n sum_j -2 p_nj d_nj y^j,
// p_nj = 5/2 + n + j; then M = (r g' - m/(2 pi))/alpha^2 (the equation
// integrated over the disc of radius r).
struct PbAsym {
    double d[PB_NA][PB_NA], e[PB_NA][PB_NA];  // d_nj and -2 p_nj d_nj
    constexpr PbAsym() : d(), e()
    {
        d[0][0] = 1.0;
        for (int n = 0; n + 1 < PB_NA; ++n) {
            for (int j = 0; j <= n + 1; ++j) {
                double v = 0.0;
                if (j <= n) {
                    const double q = 2.5 + n + j;
                    v += 4.0 * q * q * d[n][j];
                }
                if (j >= 1) {
                    const double q = 2.5 + n + (j - 1);
                    v -= 4.0 * q * (q + 1.0) * d[n][j - 1];
                }
                d[n + 1][j] = v;
            }
        }
        for (int n = 0; n < PB_NA; ++n)
            for (int j = 0; j <= n; ++j) e[n][j] = -2.0 * (2.5 + n + j) * d[n][j];
    }
};
static constexpr PbAsym PB_ASYM{};

SWIM_HD void pb_node_far(double alpha, double eps, double t, double h1c, double& fh, double& fg)
{
    const double e2 = eps * eps, R2 = t + e2, R = sqrt(R2), a2 = alpha * alpha;
    const double w = 1.0 / (a2 * R2), y = e2 / R2;
    double sg = 0.0, sr = 0.0, wn = 1.0;
#pragma unroll 1
    for (int n = 0; n < PB_NA; ++n) {
        double pg = PB_ASYM.d[n][n], pr = PB_ASYM.e[n][n];
#pragma unroll 1
        for (int j = n - 1; j >= 0; --j) {
            pg = pg * y + PB_ASYM.d[n][j];
            pr = pr * y + PB_ASYM.e[n][j];
        }
        sg += wn * pg;
        sr += wn * pr;
        wn *= w;
    }
    const double pre = 3.0 * e2 * eps / (2.0 * PI * a2 * R2 * R2 * R);
    const double g = -pre * sg;
    const double rg = -pre * (t / R2) * sr;
    const double m = 1.0 - y * (eps / R);
    const double M = (rg - m / (2.0 * PI)) / a2;
    const double Mt = M / t;
    fg = (g - 2.0 * Mt) / t;
    fh = Mt - g - h1c;
}

// the sweep's node range of a system: nodes [kS, kL] take pb_node_sweep
// (delta >= 1/4 and alpha r <= PB_ZF); below kS the near-contact series,
// beyond kL the far field
SWIM_HD void pb_sweep_range(const SysConst<double>& C, int& kS, int& kL)
{
    const double alpha = sqrt(C.a2);
    int lo = 0, hi = PB_NODES;  // first node with delta >= 1/4
    while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (pb_node_t(C.its, mid) * C.inv_e2 >= 0.25) hi = mid;
        else lo = mid + 1;
    }
    kS = lo;
    lo = 0;
    hi = PB_NODES;  // first node with alpha r > PB_ZF
    while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (alpha * sqrt(pb_node_t(C.its, mid)) > PB_ZF) hi = mid;
        else lo = mid + 1;
    }
    kL = lo - 1;
}

// the node values of a system outside the sweep (k < kS or k > kL)
SWIM_HD void pb_node_outside(const SysConst<double>& C, int k, int kS, double& fh, double& fg)
{
    const double t = pb_node_t(C.its, k);
    if (k < kS)
        kernel_paper_brinkman(C, t, fh, fg);  // delta < 1/4: the series
    else
        pb_node_far(sqrt(C.a2), C.eps, t, C.h1c, fh, fg);
}

// Host form of the sweep (the device kernel splits the same sums over a
// workgroup): FP64 values Ht, H2 of every table node of a system with the
// paper's blob at alpha > 0 (C.paper == 2).
inline void pb_table_nodes_host(const SysConst<double>& C, double* fh, double* fg)
{
    const double alpha = sqrt(C.a2), eps = C.eps;
    int kS, kL;
    pb_sweep_range(C, kS, kL);
    for (int k = 0; k < PB_NODES; ++k)
        if (k < kS || k > kL) pb_node_outside(C, k, kS, fh[k], fg[k]);
    if (kL < kS) return;
    const int ng = kL + 1;
    double* ga = new double[ng];
    double* gb = new double[ng];
    double* gc = new double[ng];
    double ulo = 0.0;
    for (int k = 1; k <= kL; ++k) {
        const double t = pb_node_t(C.its, k);
        const double uhi = asinh(sqrt(t) / eps);
        pb_gap(alpha, eps, ulo, uhi, k > kS, alpha * sqrt(t) <= 2.0, &ga[k], &gb[k], &gc[k]);
        ulo = uhi;
    }
    const double rL = sqrt(pb_node_t(C.its, kL));
    double B = 0.0;
    for (int p = 0; p < 64; ++p) B += pb_tail_panel(alpha, eps, rL, p, 64);
    double* Bk = new double[ng];
    for (int k = kL; k >= kS; --k) {
        Bk[k] = B;
        if (k > kS) B += gb[k];
    }
    double A = 0.0, Cq = 0.0;
    for (int k = 1; k <= kL; ++k) {
        A += ga[k];
        Cq += gc[k];
        if (k >= kS) pb_node_sweep(alpha, eps, pb_node_t(C.its, k), A, Bk[k], Cq, C.h1c, fh[k], fg[k]);
    }
    delete[] ga;
    delete[] gb;
    delete[] gc;
    delete[] Bk;
}

}  // namespace swim
