/*
 * swim_oracle.c -- plain, slow FP64 CPU oracle for the regularized-Brinkmanlet
 * filament swimmer (Larson, Olson & Matzavinos, "Bayesian uncertainty
 * quantification for micro-swimmers with fully resolved hydrodynamics").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The product library
 * (libswim) never links, loads or calls it, and shares no code with it.
 *
 * What it computes, step by step, in the paper's order:
 *   - regularized Brinkmanlet velocity of point forces, eq. (BrV) of Sec. 2.1,
 *     v(x) = sum_i [ -F_i B''(r) + (F_i . x_i)(x_i) (r B'' - B')/r^3 ],
 *     with (Delta - alpha^2) B = G and Delta G = phi (Sec. 2.1).
 *     The paper defers the closed forms of G and B to its references; the
 *     reading used here (blob phi_K, see kernel_init) is written out below.
 *   - forces F = -dE/dX of the discrete flagellum energy, eq. (Fenergy), with
 *     the bending energy (EFB), the signed curvature (curva) and the
 *     tensile energy (EFT) of the Appendix, second-order centred differences
 *     and the trapezoid rule (Appendix, numerical algorithm paragraph).
 *   - no-slip update dX/dt = v(X) by forward Euler (Sec. 2.1, Appendix).
 *
 * Floating point: positions, forces and sums are FP64.  The kernel functions
 * are evaluated in x87 extended precision (long double, 64-bit mantissa) and
 * rounded to double, so the cancellations inside the closed forms cost no
 * FP64 digits.  Velocity sums use Neumaier compensated summation in index
 * order j = 0, 1, ...
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long double ld;

static const ld PI_L = 3.14159265358979323846264338327950288L;
static const ld EULER_GAMMA_L = 0.57721566490153286060651209008240243L;

/* ------------------------------------------------------------------------ */
/* Modified Bessel functions of the second kind, orders 0 and 1.            */
/*                                                                          */
/* Integral representation K_nu(z) = int_0^inf exp(-z cosh u) cosh(nu u) du */
/* (Abramowitz & Stegun 9.6.24).  The integrand is even and analytic in the */
/* strip |Im u| < pi/2, so the trapezoid rule with step h converges like    */
/* exp(-pi^2/h); h = 0.2 gives ~e^-49 relative error, below long double     */
/* rounding.  For large z the integrand is a Gaussian of width 1/sqrt(z)    */
/* near u = 0, whose trapezoid error is ~exp(-2 pi^2/(z h^2)); h is capped  */
/* at 0.6/sqrt(z) to keep that below e^-54.  The factor exp(-z) is pulled   */
/* out.                                                                     */
/* ------------------------------------------------------------------------ */
static void bessel_k01_scaled(ld z, ld *k0e, ld *k1e)
{
    /* returns exp(z) K0(z), exp(z) K1(z) */
    ld h = 0.2L;
    if (z > 9.0L) h = 0.6L / sqrtl(z);
    ld umax = acoshl(1.0L + 70.0L / z); /* exp(-z (cosh u - 1)) < e^-70 beyond */
    int n = (int)(umax / h) + 2;
    ld s0 = 0.5L, s1 = 0.5L;            /* u = 0 node carries weight 1/2      */
    for (int k = 1; k <= n; ++k) {
        ld u = h * (ld)k;
        ld c = coshl(u);
        ld e = expl(-z * (c - 1.0L));
        s0 += e;
        s1 += e * c;
    }
    *k0e = h * s0;
    *k1e = h * s1;
}

static void bessel_k01(ld z, ld *k0, ld *k1)
{
    ld a, b;
    bessel_k01_scaled(z, &a, &b);
    ld ez = expl(-z);
    *k0 = a * ez;
    *k1 = b * ez;
}

/* q(z) = z K1(z) - 1.  For z <= 2 the ascending series of A&S 9.6.11 (n = 1):
 *   z K1(z) = 1 + z ln(z/2) I1(z)
 *               - (z^2/4) sum_k [psi(k+1) + psi(k+2)] (z^2/4)^k / (k! (k+1)!),
 *   z I1(z) = (z^2/2) sum_k (z^2/4)^k / (k! (k+1)!),
 * which never forms "1 - 1" for small z.  Above that, z K1(z) - 1 directly. */
static ld q_of(ld z)
{
    if (z > 2.0L) {
        ld k0, k1;
        bessel_k01(z, &k0, &k1);
        return z * k1 - 1.0L;
    }
    ld y = 0.25L * z * z;
    ld lg = logl(0.5L * z);
    ld term = 1.0L;                /* y^k / (k! (k+1)!) */
    ld psi1 = -EULER_GAMMA_L;      /* psi(k+1) */
    ld psi2 = 1.0L - EULER_GAMMA_L;/* psi(k+2) */
    ld sI = 0.0L, sP = 0.0L;
    for (int k = 0; k < 60; ++k) {
        sI += term;
        sP += (psi1 + psi2) * term;
        term *= y / ((ld)(k + 1) * (ld)(k + 2));
        psi1 += 1.0L / (ld)(k + 1);
        psi2 += 1.0L / (ld)(k + 2);
        if (term < 1e-30L * sI) break;
    }
    return 2.0L * y * lg * sI - y * sP;
}

/* ------------------------------------------------------------------------ */
/* Modified Bessel functions of the first kind, orders 0 and 1, scaled:     */
/*   exp(-z) I_n(z) = (1/pi) int_0^pi exp(z (cos th - 1)) cos(n th) dth     */
/* (A&S 9.6.19).  The integrand is even, 2 pi-periodic and entire, so the   */
/* trapezoid rule on [0, pi] with half weights at both ends converges       */
/* geometrically (64 nodes: aliasing error ~ I_128(z) e^-z); for large z it */
/* is a Gaussian of width 1/sqrt(z) at th = 0, and the step is capped at    */
/* 0.6/sqrt(z) as for K above.  For z <= 9 the ascending series            */
/*   I0 = sum_k y^k/(k!)^2,  I1 = (z/2) sum_k y^k/(k! (k+1)!),  y = z^2/4    */
/* (A&S 9.6.10) is used instead: in the integral for I1 the cos(th) factor  */
/* cancels to O(z), which would cost relative digits at small z.           */
/* ------------------------------------------------------------------------ */
static void bessel_i01_scaled(ld z, ld *i0e, ld *i1e)
{
    if (z <= 9.0L) {
        ld y = 0.25L * z * z, a = 1.0L, b = 1.0L, s0 = 0.0L, s1 = 0.0L;
        for (int k = 0; k < 100; ++k) {
            s0 += a;
            s1 += b;
            a *= y / ((ld)(k + 1) * (ld)(k + 1));
            b *= y / ((ld)(k + 1) * (ld)(k + 2));
            if (a < 1e-24L * s0) break;
        }
        ld e = expl(-z);
        *i0e = s0 * e;
        *i1e = 0.5L * z * s1 * e;
        return;
    }
    int n = 64;
    if (z > 9.0L) {
        int m = (int)(PI_L * sqrtl(z) / 0.6L) + 1;
        if (m > n) n = m;
    }
    ld h = PI_L / (ld)n;
    ld em = expl(-2.0L * z);
    ld s0 = 0.5L * (1.0L + em), s1 = 0.5L * (1.0L - em);
    for (int k = 1; k < n; ++k) {
        ld c = cosl(h * (ld)k);
        ld e = expl(z * (c - 1.0L));
        s0 += e;
        s1 += e * c;
    }
    *i0e = s0 / (ld)n;
    *i1e = s1 / (ld)n;
}

/* 20-point Gauss-Legendre rule on [-1, 1]: nodes by Newton's method on    */
/* P_20 from the standard initial guesses, weights 2/((1 - x^2) P_20'^2).   */
#define NGL 20
static ld gl_x[NGL], gl_w[NGL];
static volatile int gl_ready = 0;
static void gl_init(void)
{
    if (gl_ready) return;
    ld xs[NGL], ws[NGL];
    for (int i = 0; i < NGL; ++i) {
        ld x = cosl(PI_L * ((ld)i + 0.75L) / ((ld)NGL + 0.5L)), dp = 1.0L;
        for (int it = 0; it < 100; ++it) {
            ld p0 = 1.0L, p1 = x;
            for (int k = 2; k <= NGL; ++k) {
                ld p2 = ((ld)(2 * k - 1) * x * p1 - (ld)(k - 1) * p0) / (ld)k;
                p0 = p1;
                p1 = p2;
            }
            dp = (ld)NGL * (x * p1 - p0) / (x * x - 1.0L);
            ld dx = p1 / dp;
            x -= dx;
            if (fabsl(dx) < 1e-24L) break;
        }
        ld p0 = 1.0L, p1 = x;
        for (int k = 2; k <= NGL; ++k) {
            ld p2 = ((ld)(2 * k - 1) * x * p1 - (ld)(k - 1) * p0) / (ld)k;
            p0 = p1;
            p1 = p2;
        }
        dp = (ld)NGL * (x * p1 - p0) / (x * x - 1.0L);
        xs[i] = x;
        ws[i] = 2.0L / ((1.0L - x * x) * dp * dp);
    }
    for (int i = 0; i < NGL; ++i) {
        gl_x[i] = xs[i];
        gl_w[i] = ws[i];
    }
    gl_ready = 1;
}

/* ------------------------------------------------------------------------ */
/* The paper's blob (eq. eqnblob) for alpha > 0, where its Brinkmanlet has */
/* no closed form.  g solves (Delta - alpha^2) g = phi, i.e. g is the       */
/* convolution of phi with the free-space Green function -K0(alpha r)/2pi;  */
/* averaging K0(alpha |x - y|) over the angle of y (Graf's addition theorem)*/
/* leaves I0(alpha s<) K0(alpha s>), so with z = alpha r                    */
/*   g(r) = -[K0(z) A(r) + I0(z) B(r)],                                     */
/*   A = int_0^r phi(s) I0(alpha s) s ds,  B = int_r^inf phi(s) K0(alpha s) s ds. */
/* Differentiating, r g' = z [K1(z) A - I1(z) B]; integrating the equation  */
/* over the disc of radius r, r g' - alpha^2 M = m/(2 pi) with M = int_0^r  */
/* s g ds and the blob mass m = 1 - eps^3/R^3, so                           */
/*   M = (z K1 A - z I1 B - m/(2 pi)) / alpha^2.                            */
/* For z <= 2 the same M is taken in the form                               */
/*   M = Cq + r^2 [q(z)/z^2] A - r^2 [I1(z)/z] B,                           */
/*   Cq = int_0^r phi(s) s (I0(alpha s) - 1)/alpha^2 ds,                    */
/* (m/(2 pi) = A - alpha^2 Cq), in which no two large terms cancel.         */
/* Quadrature: s = eps sinh(u) turns phi(s) s ds into (3/2pi) sinh u/cosh^4 u du, */
/* analytic within pi/2 of the real axis; 20-point Gauss-Legendre panels of */
/* width <= 1/2 in u, and, near s = r where exp(-alpha |s - r|) varies, of  */
/* width <= 1 + x/4 in x = alpha |s - r|.  A and B are carried scaled,      */
/* As = e^-z A and Bs = e^z B, so that no exponential overflows; panels     */
/* stop once the integrand is below e^-50 of its size at s = r.             */
/* Near contact (delta = r^2/eps^2 < 1/4) the kernel uses the series of g   */
/* in delta: inserting g = sum gam_n delta^n and phi = sum phi_n delta^n,   */
/* phi_n = 3/(2 pi eps^2) C(-5/2, n), into the equation gives               */
/*   gam_{n+1} = eps^2 (phi_n + alpha^2 gam_n) / (4 (n+1)^2),               */
/* so only gam_0 = g(0) = -int_0^inf phi(s) K0(alpha s) s ds is integrated  */
/* (on panels refined geometrically towards the log singularity at s = 0). */
/* ------------------------------------------------------------------------ */
static ld pb_w(ld u)
{
    ld c = coshl(u);
    return 3.0L * sinhl(u) / (2.0L * PI_L * c * c * c * c);
}

/* (I0(x) - 1) / alpha^2 at x = alpha s, from the ascending series (x <= 2) */
static ld pb_i0m1(ld alpha, ld s)
{
    ld y = 0.25L * alpha * alpha * s * s, term = 1.0L, acc = 0.0L;
    for (int k = 0; k < 60; ++k) {
        acc += term;
        term *= y / ((ld)(k + 2) * (ld)(k + 2));
        if (term < 1e-30L * acc) break;
    }
    return 0.25L * s * s * acc;
}

static ld pb_b_tail(ld alpha, ld eps, ld r, ld u0);

/* As, Bs and (z <= 2) Cq at radius r */
static void pb_parts(ld alpha, ld eps, ld r, ld *As, ld *Bs, ld *Cq)
{
    ld z = alpha * r, ur = asinhl(r / eps);
    int want_c = z <= 2.0L;
    ld a = 0.0L, c = 0.0L, b = 0.0L;
    ld uh = ur;
    while (uh > 0.0L) {
        ld x = alpha * (r - eps * sinhl(uh));
        if (x - 3.0L * (ur - uh) > 50.0L) break;
        ld sl = eps * sinhl(uh) - (1.0L + 0.25L * x) / alpha;
        ld ul = sl > 0.0L ? asinhl(sl / eps) : 0.0L;
        if (ul < uh - 0.5L) ul = uh - 0.5L;
        if (ul < 0.0L) ul = 0.0L;
        ld hm = 0.5L * (uh - ul), ct = 0.5L * (uh + ul);
        for (int i = 0; i < NGL; ++i) {
            ld u = ct + hm * gl_x[i], s = eps * sinhl(u), wq = hm * gl_w[i] * pb_w(u);
            ld i0e, i1e;
            bessel_i01_scaled(alpha * s, &i0e, &i1e);
            a += wq * i0e * expl(alpha * s - z);
            if (want_c) c += wq * pb_i0m1(alpha, s);
        }
        uh = ul;
    }
    b = pb_b_tail(alpha, eps, r, ur);
    *As = a;
    *Bs = b;
    *Cq = c;
}

/* int over [ul, uh] of (3/2pi) sinh u/cosh^4 u K0(alpha s) exp(z) du */
static ld pb_b_panel(ld alpha, ld eps, ld z, ld ul, ld uh)
{
    ld hm = 0.5L * (uh - ul), ct = 0.5L * (uh + ul), b = 0.0L;
    for (int i = 0; i < NGL; ++i) {
        ld u = ct + hm * gl_x[i], s = eps * sinhl(u), k0e, k1e;
        bessel_k01_scaled(alpha * s, &k0e, &k1e);
        b += hm * gl_w[i] * pb_w(u) * k0e * expl(z - alpha * s);
    }
    return b;
}

/* Bs = e^z int_{u0}^inf ..., panels from u0 upwards */
static ld pb_b_tail(ld alpha, ld eps, ld r, ld u0)
{
    ld z = alpha * r, ul = u0, b = 0.0L;
    for (;;) {
        ld x = alpha * (eps * sinhl(ul) - r);
        if (x + 3.0L * (ul - u0) > 50.0L) break;
        ld uh = asinhl((eps * sinhl(ul) + (1.0L + 0.25L * x) / alpha) / eps);
        if (uh > ul + 0.5L) uh = ul + 0.5L;
        b += pb_b_panel(alpha, eps, z, ul, uh);
        ul = uh;
    }
    return b;
}

/* g(0) = -int_0^inf phi K0(alpha s) s ds: panels [2^-(j+2), 2^-(j+1)],
 * j = 0..63, towards the logarithm of K0 at s = 0, then from u = 1/2 on */
static ld pb_g0(ld alpha, ld eps)
{
    ld b = 0.0L;
    for (int j = 63; j >= 0; --j) b += pb_b_panel(alpha, eps, 0.0L, ldexpl(1.0L, -(j + 2)), ldexpl(1.0L, -(j + 1)));
    return -(b + pb_b_tail(alpha, eps, 0.0L, 0.5L));
}

/* g(r) and M(r) of the paper's blob at alpha > 0 */
static void pb_gM(ld alpha, ld eps, ld t, ld *g, ld *M)
{
    ld r = sqrtl(t), z = alpha * r;
    ld As, Bs, Cq;
    pb_parts(alpha, eps, r, &As, &Bs, &Cq);
    ld k0e, k1e, i0e, i1e;
    bessel_k01_scaled(z, &k0e, &k1e);
    bessel_i01_scaled(z, &i0e, &i1e);
    *g = -(k0e * As + i0e * Bs);
    if (z <= 2.0L) {
        ld ez = expl(z);
        ld qz2 = q_of(z) / (z * z);
        ld i1z = i1e * ez / z;
        *M = Cq + t * qz2 * As * ez - t * i1z * Bs / ez;
    } else {
        ld R = sqrtl(t + eps * eps);
        ld m = 1.0L - eps * eps * eps / (R * R * R);
        *M = (z * (k1e * As - i1e * Bs) - m / (2.0L * PI_L)) / (alpha * alpha);
    }
}

/* ------------------------------------------------------------------------ */
/* Kernel of eq. (BrV): v = sum_j [ H1(r) F_j + H2(r) (F_j . x) x ],       */
/* H1 = -B'',  H2 = (r B'' - B')/r^3,  x = x_i - X_j, r = |x|.              */
/*                                                                          */
/* Reading of the blob (the paper defers G and B to its references):        */
/*   g(r) = -c K0(alpha R) / (2 pi),  R = sqrt(r^2 + eps^2),               */
/*   c = 1 / (alpha eps K1(alpha eps)),                                     */
/* solves (Delta - alpha^2) g = phi with the positive, unit-mass blob       */
/*   phi = c eps^2/(2 pi) [alpha^2 K0(alpha R)/R^2 + 2 alpha K1(alpha R)/R^3]*/
/* which tends to eps^2/(pi R^4) as alpha -> 0.  With B = (g - G)/alpha^2   */
/* one has Delta B = g, so B' = M/r with M(r) = int_0^r s g(s) ds and       */
/* B'' = g - M/r^2:                                                         */
/*   M  = c [q(alpha R) - q(alpha eps)] / (2 pi alpha^2)                   */
/*   H1 = M/r^2 - g,   H2 = (g - 2 M/r^2)/r^2.                              */
/* At alpha = 0 (Stokes limit, same blob), with delta = r^2/eps^2:         */
/*   H1 = (1/4pi)[-ln R + log1p(delta)/(2 delta) - 1/2],                    */
/*   H2 = (1/2pi)[1/(2 r^2) - log1p(delta)/(2 r^2 delta)].                  */
/* Near contact (delta < 0.25) both use the Taylor series of g in delta,    */
/* g = sum_n gam_n delta^n, for which                                       */
/*   H1 = -sum_{n>=0} gam_n delta^n (2n+1)/(2(n+1)),                        */
/*   H2 = (1/eps^2) sum_{n>=1} gam_n delta^(n-1) n/(n+1).                   */
/* Brinkman: gam_n = -(c/2pi)(-1)^n kap_n, kap_n = (z0/2)^n K_n(z0)/n!,     */
/* z0 = alpha eps, from the recurrence K_{n+1} = K_{n-1} + (2n/z) K_n.      */
/* Stokes:   gam_0 = ln(eps^2)/(4pi), gam_n = (-1)^(n+1)/(4 pi n).          */
/* ------------------------------------------------------------------------ */
#define NGAM 32
#define DELTA_TAYLOR 0.25L

typedef struct {
    ld alpha, eps, e2;
    int stokes;
    int paper; /* the paper's blob (eq. eqnblob): 1 Stokes limit, 2 alpha > 0 */
    ld c, q0;
    ld gam[NGAM];
} okern;

/* Blob selection for the kernel functions below (test infrastructure:
 * set by the Python wrapper).  1 (the default): the paper's blob
 * phi = 3 eps^3 / (2 pi R^5) of eq. (eqnblob); 0: the blob of the reading
 * above.  The paper's blob, whose
 * Stokes Green function G (Delta G = phi) is
 *   G = (ln(R + eps) - eps/R) / (2 pi)
 * (r G' = m/(2 pi) with the blob mass m = 1 - eps^3/R^3).  Its kernel uses
 * the same route as the other blob: M = int_0^r s G ds =
 * [(r^2/2) ln(R + eps) - (R + 3 eps)(R - eps)/4] / (2 pi), H1 = M/r^2 - G,
 * H2 = (G - 2M/r^2)/r^2; near contact the series of G in delta with the
 * same formulas.  For alpha > 0 (no closed form) g and M come from the
 * quadrature of pb_gM and the series from gam_0 = g(0) (see above). */
static int g_blob = 1;
void oracle_set_blob(int b) { g_blob = b; }
int oracle_get_blob(void) { return g_blob; }

/* threads the OpenMP loops of the velocity sums use, and setting them */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static void kernel_init(okern *k, double alpha, double eps)
{
    memset(k, 0, sizeof(*k));
    k->alpha = alpha;
    k->eps = eps;
    k->e2 = (ld)eps * (ld)eps;
    k->stokes = (alpha == 0.0);
    if (g_blob == 1 && alpha > 0.0) {
        gl_init();
        k->paper = 2;
        k->c = 1.0L;
        ld phin = 3.0L / (2.0L * PI_L * k->e2); /* phi_0; phi_n = phi_0 C(-5/2, n) */
        k->gam[0] = pb_g0((ld)alpha, (ld)eps);
        for (int n = 0; n + 1 < NGAM; ++n) {
            k->gam[n + 1] = k->e2 * (phin + (ld)alpha * (ld)alpha * k->gam[n]) / (4.0L * (ld)(n + 1) * (ld)(n + 1));
            phin *= (-2.5L - (ld)n) / (ld)(n + 1);
        }
        return;
    }
    if (g_blob == 1) {
        /* Taylor coefficients of G in delta: with a = sqrt(1 + delta) and
         * u = (a - 1)/2, ln(1 + a) = ln 2 + ln(1 + u), whose coefficients L_n
         * satisfy n L_n = n u_n - sum_{j=1}^{n-1} j L_j u_{n-j};
         * eps/R = (1 + delta)^(-1/2). */
        k->paper = 1;
        k->c = 1.0L;
        ld an[NGAM], bn[NGAM], un[NGAM], Ln[NGAM];
        an[0] = 1.0L;
        bn[0] = 1.0L;
        for (int n = 1; n < NGAM; ++n) {
            an[n] = an[n - 1] * (0.5L - (ld)(n - 1)) / (ld)n;
            bn[n] = bn[n - 1] * (-0.5L - (ld)(n - 1)) / (ld)n;
        }
        un[0] = 0.0L;
        for (int n = 1; n < NGAM; ++n) un[n] = 0.5L * an[n];
        Ln[0] = 0.0L;
        for (int n = 1; n < NGAM; ++n) {
            ld acc = (ld)n * un[n];
            for (int j = 1; j < n; ++j) acc -= (ld)j * Ln[j] * un[n - j];
            Ln[n] = acc / (ld)n;
        }
        k->gam[0] = (logl((ld)eps) + logl(2.0L) - 1.0L) / (2.0L * PI_L);
        for (int n = 1; n < NGAM; ++n) k->gam[n] = (Ln[n] - bn[n]) / (2.0L * PI_L);
        return;
    }
    if (k->stokes) {
        k->c = 1.0L;
        k->gam[0] = logl(k->e2) / (4.0L * PI_L);
        for (int n = 1; n < NGAM; ++n)
            k->gam[n] = ((n % 2) ? 1.0L : -1.0L) / (4.0L * PI_L * (ld)n);
        return;
    }
    ld z0 = (ld)alpha * (ld)eps;
    ld K0, K1;
    bessel_k01(z0, &K0, &K1);
    k->c = 1.0L / (z0 * K1);
    k->q0 = q_of(z0);
    ld kap[NGAM];
    kap[0] = K0;
    kap[1] = 0.5L * z0 * K1;
    for (int n = 1; n + 1 < NGAM; ++n)
        kap[n + 1] = 0.25L * z0 * z0 * kap[n - 1] / ((ld)n * (ld)(n + 1))
                   + (ld)n * kap[n] / (ld)(n + 1);
    for (int n = 0; n < NGAM; ++n)
        k->gam[n] = -(k->c / (2.0L * PI_L)) * ((n % 2) ? -1.0L : 1.0L) * kap[n];
}

static void kernel_eval(const okern *k, double t_d, ld *H1, ld *H2)
{
    ld t = t_d;
    ld delta = t / k->e2;
    if (delta < DELTA_TAYLOR) {
        ld p = 1.0L, h1 = 0.0L, h2 = 0.0L;
        for (int n = 0; n < NGAM; ++n) {
            h1 -= k->gam[n] * p * (ld)(2 * n + 1) / (ld)(2 * (n + 1));
            if (n + 1 < NGAM)
                h2 += k->gam[n + 1] * p * (ld)(n + 1) / (ld)(n + 2);
            p *= delta;
        }
        *H1 = h1;
        *H2 = h2 / k->e2;
        return;
    }
    if (k->paper == 2) {
        ld g, M;
        pb_gM((ld)k->alpha, (ld)k->eps, t, &g, &M);
        *H1 = M / t - g;
        *H2 = (g - 2.0L * M / t) / t;
        return;
    }
    if (k->paper) {
        ld R = sqrtl(t + k->e2), e = (ld)k->eps;
        ld G = (logl(R + e) - e / R) / (2.0L * PI_L);
        ld M = (0.5L * t * logl(R + e) - 0.25L * (R + 3.0L * e) * (R - e)) / (2.0L * PI_L);
        *H1 = M / t - G;
        *H2 = (G - 2.0L * M / t) / t;
        return;
    }
    if (k->stokes) {
        ld R2 = t + k->e2;
        ld L1 = log1pl(delta);
        *H1 = (1.0L / (4.0L * PI_L)) * (-0.5L * logl(R2) + L1 / (2.0L * delta) - 0.5L);
        *H2 = (1.0L / (2.0L * PI_L)) * (1.0L / (2.0L * t) - L1 / (2.0L * t * delta));
        return;
    }
    ld R = sqrtl(t + k->e2);
    ld z = k->alpha * R;
    ld K0, K1;
    bessel_k01(z, &K0, &K1);
    ld qz = (z > 2.0L) ? z * K1 - 1.0L : q_of(z);
    ld g = -k->c * K0 / (2.0L * PI_L);
    ld M = k->c * (qz - k->q0) / (2.0L * PI_L * k->alpha * k->alpha);
    *H1 = M / t - g;
    *H2 = (g - 2.0L * M / t) / t;
}

/* ------------------------------------------------------------------------ */
/* Exported: kernel and special-function values (for the pins).             */
/* ------------------------------------------------------------------------ */
void oracle_bessel(int64_t n, const double *z, double *k0, double *k1, double *q)
{
    for (int64_t i = 0; i < n; ++i) {
        ld a, b;
        bessel_k01((ld)z[i], &a, &b);
        k0[i] = (double)a;
        k1[i] = (double)b;
        q[i] = (double)q_of((ld)z[i]);
    }
}

void oracle_kernel(double alpha, double eps, int64_t n, const double *t, double *H1, double *H2)
{
    okern k;
    kernel_init(&k, alpha, eps);
    for (int64_t i = 0; i < n; ++i) {
        ld a, b;
        kernel_eval(&k, t[i], &a, &b);
        H1[i] = (double)a;
        H2[i] = (double)b;
    }
}

/* ------------------------------------------------------------------------ */
/* Dense velocity sum, eq. (BrV), over all n points of one system.          */
/* ------------------------------------------------------------------------ */
static void velocity_sum(const okern *k, int64_t n, const double *x, const double *y,
                         const double *fx, const double *fy, double *ux, double *uy)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        double sx = 0.0, cx = 0.0, sy = 0.0, cy = 0.0; /* Neumaier sums */
        for (int64_t j = 0; j < n; ++j) {
            double dx = x[i] - x[j], dy = y[i] - y[j];
            double t = dx * dx + dy * dy;
            ld H1, H2;
            kernel_eval(k, t, &H1, &H2);
            double h1 = (double)H1, h2 = (double)H2;
            double fd = fx[j] * dx + fy[j] * dy;
            double vx = h1 * fx[j] + h2 * fd * dx;
            double vy = h1 * fy[j] + h2 * fd * dy;
            double s;
            s = sx + vx;
            cx += (fabs(sx) >= fabs(vx)) ? (sx - s) + vx : (vx - s) + sx;
            sx = s;
            s = sy + vy;
            cy += (fabs(sy) >= fabs(vy)) ? (sy - s) + vy : (vy - s) + sy;
            sy = s;
        }
        ux[i] = sx + cx;
        uy[i] = sy + cy;
    }
}

void oracle_velocity(int64_t n, const double *x, const double *y, const double *fx,
                     const double *fy, double alpha, double eps, double *ux, double *uy)
{
    okern k;
    kernel_init(&k, alpha, eps);
    velocity_sum(&k, n, x, y, fx, fy, ux, uy);
}

/* Velocity at a subset of targets only (targets idx[0..m-1]), for sampled
 * checks of systems too large to sum in full. */
void oracle_velocity_at(int64_t n, const double *x, const double *y, const double *fx,
                        const double *fy, double alpha, double eps, int64_t m,
                        const int64_t *idx, double *ux, double *uy)
{
    okern k;
    kernel_init(&k, alpha, eps);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t a = 0; a < m; ++a) {
        int64_t i = idx[a];
        double sx = 0.0, cx = 0.0, sy = 0.0, cy = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double dx = x[i] - x[j], dy = y[i] - y[j];
            double t = dx * dx + dy * dy;
            ld H1, H2;
            kernel_eval(&k, t, &H1, &H2);
            double h1 = (double)H1, h2 = (double)H2;
            double fd = fx[j] * dx + fy[j] * dy;
            double vx = h1 * fx[j] + h2 * fd * dx;
            double vy = h1 * fy[j] + h2 * fd * dy;
            double s;
            s = sx + vx;
            cx += (fabs(sx) >= fabs(vx)) ? (sx - s) + vx : (vx - s) + sx;
            sx = s;
            s = sy + vy;
            cy += (fabs(sy) >= fabs(vy)) ? (sy - s) + vy : (vy - s) + sy;
            sy = s;
        }
        ux[a] = sx + cx;
        uy[a] = sy + cy;
    }
}

/* ------------------------------------------------------------------------ */
/* Flagellum energy and forces, Appendix eqs. (EFB), (curva), (EFT).        */
/*   E_tens = S_s sum_{k=0}^{N-2} (l_k/ds - 1)^2 ds,  l_k = |X_{k+1}-X_k|   */
/*   (Hookean springs between neighbouring points; the derivative inside    */
/*    the norm is the first one, the printed second derivative is read as   */
/*    a typo since the text calls the discrete form springs).               */
/*   E_bend = S_b sum_{k=1}^{N-2} (kappa_k - kappa0_k)^2 ds                 */
/*   kappa = (y'' x' - x'' y') / (x'^2 + y'^2)^(3/2), centred differences.  */
/*   Only interior nodes carry curvature (end nodes contribute nothing).    */
/*   F = -dE/dX (eq. Fenergy), the exact gradient of the discrete energy.   */
/* ------------------------------------------------------------------------ */
double oracle_energy(int N, double ds, const double *x, const double *y, double Sb,
                     double Ss, const double *kappa0)
{
    double E = 0.0;
    for (int k = 0; k + 1 < N; ++k) {
        double dx = x[k + 1] - x[k], dy = y[k + 1] - y[k];
        double l = sqrt(dx * dx + dy * dy);
        double e = l / ds - 1.0;
        E += Ss * e * e * ds;
    }
    for (int k = 1; k + 1 < N; ++k) {
        double xp = (x[k + 1] - x[k - 1]) / (2.0 * ds);
        double yp = (y[k + 1] - y[k - 1]) / (2.0 * ds);
        double xpp = (x[k + 1] - 2.0 * x[k] + x[k - 1]) / (ds * ds);
        double ypp = (y[k + 1] - 2.0 * y[k] + y[k - 1]) / (ds * ds);
        double S = xp * xp + yp * yp;
        double kap = (ypp * xp - xpp * yp) / pow(S, 1.5);
        double d = kap - kappa0[k];
        E += Sb * d * d * ds;
    }
    return E;
}

void oracle_forces(int N, double ds, const double *x, const double *y, double Sb, double Ss,
                   const double *kappa0, double *fx, double *fy)
{
    for (int k = 0; k < N; ++k) {
        fx[k] = 0.0;
        fy[k] = 0.0;
    }
    /* stretching: dE/dX_{k+1} = 2 S_s (l/ds - 1) d/l from segment k */
    for (int k = 0; k + 1 < N; ++k) {
        double dx = x[k + 1] - x[k], dy = y[k + 1] - y[k];
        double l = sqrt(dx * dx + dy * dy);
        double e = l / ds - 1.0;
        double gx = 2.0 * Ss * e * dx / l;
        double gy = 2.0 * Ss * e * dy / l;
        fx[k + 1] -= gx;
        fy[k + 1] -= gy;
        fx[k] += gx;
        fy[k] += gy;
    }
    /* bending: chain rule through kappa_k(X_{k-1}, X_k, X_{k+1}) */
    for (int k = 1; k + 1 < N; ++k) {
        double a = (x[k + 1] - x[k - 1]) / (2.0 * ds);        /* x'  */
        double b = (y[k + 1] - y[k - 1]) / (2.0 * ds);        /* y'  */
        double p = (x[k + 1] - 2.0 * x[k] + x[k - 1]) / (ds * ds); /* x'' */
        double q = (y[k + 1] - 2.0 * y[k] + y[k - 1]) / (ds * ds); /* y'' */
        double S = a * a + b * b;
        double S32 = pow(S, 1.5);
        double num = q * a - p * b;
        double kap = num / S32;
        double co = 2.0 * Sb * (kap - kappa0[k]) * ds;       /* dE/dkappa_k */
        double dk_da = q / S32 - 3.0 * a * num / (S32 * S);
        double dk_db = -p / S32 - 3.0 * b * num / (S32 * S);
        double dk_dp = -b / S32;
        double dk_dq = a / S32;
        /* da/dx_{k-1} = -1/(2ds), da/dx_{k+1} = 1/(2ds);
           dp/dx_{k-1} = dp/dx_{k+1} = 1/ds^2, dp/dx_k = -2/ds^2 (same for y) */
        double i2 = 1.0 / (2.0 * ds), i1 = 1.0 / (ds * ds);
        fx[k - 1] -= co * (-dk_da * i2 + dk_dp * i1);
        fy[k - 1] -= co * (-dk_db * i2 + dk_dq * i1);
        fx[k] -= co * (-2.0 * dk_dp * i1);
        fy[k] -= co * (-2.0 * dk_dq * i1);
        fx[k + 1] -= co * (dk_da * i2 + dk_dp * i1);
        fy[k + 1] -= co * (dk_db * i2 + dk_dq * i1);
    }
}

/* preferred curvature kappa0(s, t) = -k^2 b sin(k s - omega t + phase), the
 * untapered case of the Appendix beat with zeta_hat = d^2 y_hat / ds^2. */
static void preferred_curvature(int N, double ds, double b, double kw, double omega,
                                double phase, double t, double *kappa0)
{
    for (int k = 0; k < N; ++k)
        kappa0[k] = -kw * kw * b * sin(kw * (double)k * ds - omega * t + phase);
}

void oracle_kappa0(int N, double ds, double b, double kw, double omega, double phase,
                   double t, double *kappa0)
{
    preferred_curvature(N, ds, b, kw, omega, phase, t, kappa0);
}

/* ------------------------------------------------------------------------ */
/* Forward model: one system of n_swim filaments of N points each.          */
/* params: n_swim rows of 9 doubles (alpha, Sb, Ss, b, omega, k, phase,     */
/* x0, y0); alpha is taken from row 0 (one fluid per system).               */
/* Filament m starts straight along x: X_k = (x0 + k ds, y0), ds = 1/(N-1), */
/* eps = eps_over_ds * ds.  Each step n (t = n dt): kappa0, forces of each  */
/* filament, velocity sum over all n_swim*N points, Euler update; after the */
/* update, if (n+1) % obs_every == 0, store the head X_{N-1} of every       */
/* filament.  Status 1 = non-finite, 2 = |X| > 1e3 (run stops there).       */
/* speed[m] = |X_h(T) - X_h(0)| / T.                                        */
/* ------------------------------------------------------------------------ */
int oracle_forward(int n_swim, int N, const double *params, double eps_over_ds, int steps,
                   double dt, int obs_every, double *obs, double *speed, double *xout,
                   double *yout, int *status)
{
    int64_t n = (int64_t)n_swim * N;
    double ds = 1.0 / (double)(N - 1);
    double eps = eps_over_ds * ds;
    double *x = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * n);
    double *fx = malloc(sizeof(double) * n), *fy = malloc(sizeof(double) * n);
    double *ux = malloc(sizeof(double) * n), *uy = malloc(sizeof(double) * n);
    double *k0 = malloc(sizeof(double) * N);
    double *h0 = malloc(sizeof(double) * 2 * n_swim);
    okern k;
    kernel_init(&k, params[0], eps);
    for (int m = 0; m < n_swim; ++m) {
        const double *P = params + 9 * m;
        for (int i = 0; i < N; ++i) {
            x[m * N + i] = P[7] + (double)i * ds;
            y[m * N + i] = P[8];
        }
        h0[2 * m] = x[m * N + N - 1];
        h0[2 * m + 1] = y[m * N + N - 1];
    }
    int st = 0;
    int n_obs = obs_every > 0 ? steps / obs_every : 0;
    for (int s = 0; s < steps && st == 0; ++s) {
        double t = (double)s * dt;
        for (int m = 0; m < n_swim; ++m) {
            const double *P = params + 9 * m;
            preferred_curvature(N, ds, P[3], P[5], P[4], P[6], t, k0);
            oracle_forces(N, ds, x + m * N, y + m * N, P[1], P[2], k0, fx + m * N, fy + m * N);
        }
        velocity_sum(&k, n, x, y, fx, fy, ux, uy);
        for (int64_t i = 0; i < n; ++i) {
            x[i] += dt * ux[i];
            y[i] += dt * uy[i];
        }
        for (int64_t i = 0; i < n; ++i) {
            if (!isfinite(x[i]) || !isfinite(y[i])) { st = 1; break; }
            if (fabs(x[i]) > 1e3 || fabs(y[i]) > 1e3) { st = 2; break; }
        }
        if (st == 0 && obs_every > 0 && (s + 1) % obs_every == 0) {
            int o = (s + 1) / obs_every - 1;
            for (int m = 0; m < n_swim; ++m) {
                obs[((int64_t)m * n_obs + o) * 2] = x[m * N + N - 1];
                obs[((int64_t)m * n_obs + o) * 2 + 1] = y[m * N + N - 1];
            }
        }
    }
    double T = (double)steps * dt;
    for (int m = 0; m < n_swim; ++m) {
        double dx = x[m * N + N - 1] - h0[2 * m], dy = y[m * N + N - 1] - h0[2 * m + 1];
        speed[m] = st ? NAN : sqrt(dx * dx + dy * dy) / T;
    }
    if (xout) memcpy(xout, x, sizeof(double) * n);
    if (yout) memcpy(yout, y, sizeof(double) * n);
    *status = st;
    free(x); free(y); free(fx); free(fy); free(ux); free(uy); free(k0); free(h0);
    return 0;
}

/* ======================================================================== */
/* Full sperm model (Appendix): flagellum of nf points with the tapered     */
/* beat, a circular head of nh points, the neck, n_swim swimmers per fluid. */
/*                                                                          */
/* Geometry of one swimmer (left to right, Appendix): flagellum point k at  */
/* (x0 + k ds, y0), ds = 1/(nf-1); head centre at the last flagellum point  */
/* shifted right by H_r + dN; head point m at angle m dth, dth = 2 pi/nh,   */
/* so m = nh/2 is the point at angle pi, nearest the flagellum.             */
/*                                                                          */
/* Discrete energy (trapezoid rule, centred differences, Appendix):          */
/*   flagellum tension  K_T  sum_k (l_k/ds - 1)^2 ds          (EFT)         */
/*   flagellum bending  K_C  sum_{k=1}^{nf-2} (zeta_k - zhat_k)^2 ds (EFB)  */
/*       zhat = d^2/ds^2 of a (1-s) sin(eta s - omega t + phase)            */
/*   head tension       K_HT sum_m (l_m/c - 1)^2 c, ring springs, rest c =  */
/*                      the initial chord 2 H_r sin(dth/2)                  */
/*   head diameters     K_HT sum_{m<nh/2} (d_m/(2 H_r) - 1)^2 (2 H_r),      */
/*                      springs between points pi apart                     */
/*   head bending       K_HC sum_m (kappa_m - 1/H_r)^2 c, closed curve      */
/*   neck tension       K_NT sum over 5 springs (l/L0 - 1)^2 L0, L0 = the   */
/*                      initial lengths: last flagellum point to the head   */
/*                      points at pi - dth, pi, pi + dth; the one before it */
/*                      to pi - dth and pi + dth                            */
/*   neck angle         K_NA (z1 . z2)^2, z1 = H(pi) - F(nf-1),             */
/*                      z2 = H(pi + dth) - H(pi - dth)                      */
/* Every spring has the form K (l/L0 - 1)^2 L0 of the flagellum's discrete */
/* tension.  F = -dE/dX (eq. Fenergy), the exact gradient of this energy.   */
/* ------------------------------------------------------------------------ */

/* system row: alpha, K_C, K_T, K_HT, K_HC, K_NT, K_NA, a, eta, omega */
enum { SP_ALPHA, SP_KC, SP_KT, SP_KHT, SP_KHC, SP_KNT, SP_KNA, SP_A, SP_ETA, SP_OMEGA, SP_N };

typedef struct {
    int nf, nh;
    double ds, hr, dn, dth, ch;
    double L0[5];
    int na[5], nb[5]; /* neck springs: point indices within the swimmer */
} osperm;

static void sperm_geom(osperm *g, int nf, int nh, double hr, double dn)
{
    g->nf = nf;
    g->nh = nh;
    g->ds = 1.0 / (double)(nf - 1);
    g->hr = hr;
    g->dn = dn;
    g->dth = 2.0 * (double)PI_L / (double)nh;
    g->ch = 2.0 * hr * sin(0.5 * g->dth);
    const int c = nf + nh / 2;
    const int a[5] = {nf - 1, nf - 1, nf - 1, nf - 2, nf - 2};
    const int b[5] = {c - 1, c, c + 1, c - 1, c + 1};
    for (int i = 0; i < 5; ++i) {
        g->na[i] = a[i];
        g->nb[i] = b[i];
    }
}

/* initial positions of one swimmer whose first flagellum point is (x0, y0) */
static void sperm_initial(const osperm *g, double x0, double y0, double *x, double *y)
{
    for (int k = 0; k < g->nf; ++k) {
        x[k] = x0 + (double)k * g->ds;
        y[k] = y0;
    }
    const double xc = x[g->nf - 1] + g->hr + g->dn, yc = y0;
    for (int m = 0; m < g->nh; ++m) {
        x[g->nf + m] = xc + g->hr * cos((double)m * g->dth);
        y[g->nf + m] = yc + g->hr * sin((double)m * g->dth);
    }
}

static void sperm_rest_lengths(osperm *g)
{
    double *x = malloc(sizeof(double) * (g->nf + g->nh)), *y = malloc(sizeof(double) * (g->nf + g->nh));
    sperm_initial(g, 0.0, 0.0, x, y);
    for (int i = 0; i < 5; ++i)
        g->L0[i] = hypot(x[g->nb[i]] - x[g->na[i]], y[g->nb[i]] - y[g->na[i]]);
    free(x);
    free(y);
}

/* preferred flagellum curvature zhat(s, t) = d^2/ds^2 [a (1-s) sin(eta s - omega t + phase)]
 *   = -2 a eta cos(psi) - a (1-s) eta^2 sin(psi),  psi = eta s - omega t + phase */
static double sperm_zhat(double a, double eta, double omega, double phase, double s, double t)
{
    const double psi = eta * s - omega * t + phase;
    return -2.0 * a * eta * cos(psi) - a * (1.0 - s) * eta * eta * sin(psi);
}

void oracle_sperm_zhat(int n, const double *s, double a, double eta, double omega, double phase, double t,
                       double *out)
{
    for (int i = 0; i < n; ++i) out[i] = sperm_zhat(a, eta, omega, phase, s[i], t);
}

/* curvature (curva) at B from A, B, C with parameter step h */
static double node_curvature(double xa, double ya, double xb, double yb, double xc, double yc, double h)
{
    const double xp = (xc - xa) / (2.0 * h), yp = (yc - ya) / (2.0 * h);
    const double xpp = (xc - 2.0 * xb + xa) / (h * h), ypp = (yc - 2.0 * yb + ya) / (h * h);
    return (ypp * xp - xpp * yp) / pow(xp * xp + yp * yp, 1.5);
}

static double spring_energy(double xa, double ya, double xb, double yb, double L0, double K)
{
    const double e = hypot(xb - xa, yb - ya) / L0 - 1.0;
    return K * e * e * L0;
}

/* energy of one swimmer; sp = system row, phase = the swimmer's beat phase */
static double sperm_energy(const osperm *g, const double *sp, double phase, double t, const double *x,
                           const double *y)
{
    const int nf = g->nf, nh = g->nh;
    const double *hx = x + nf, *hy = y + nf;
    double E = 0.0;
    for (int k = 0; k + 1 < nf; ++k) E += spring_energy(x[k], y[k], x[k + 1], y[k + 1], g->ds, sp[SP_KT]);
    for (int k = 1; k + 1 < nf; ++k) {
        const double z = node_curvature(x[k - 1], y[k - 1], x[k], y[k], x[k + 1], y[k + 1], g->ds);
        const double d = z - sperm_zhat(sp[SP_A], sp[SP_ETA], sp[SP_OMEGA], phase, (double)k * g->ds, t);
        E += sp[SP_KC] * d * d * g->ds;
    }
    for (int m = 0; m < nh; ++m) {
        const int n = (m + 1) % nh, p = (m + nh - 1) % nh;
        E += spring_energy(hx[m], hy[m], hx[n], hy[n], g->ch, sp[SP_KHT]);
        const double d = node_curvature(hx[p], hy[p], hx[m], hy[m], hx[n], hy[n], g->ch) - 1.0 / g->hr;
        E += sp[SP_KHC] * d * d * g->ch;
    }
    for (int m = 0; m < nh / 2; ++m)
        E += spring_energy(hx[m], hy[m], hx[m + nh / 2], hy[m + nh / 2], 2.0 * g->hr, sp[SP_KHT]);
    for (int i = 0; i < 5; ++i)
        E += spring_energy(x[g->na[i]], y[g->na[i]], x[g->nb[i]], y[g->nb[i]], g->L0[i], sp[SP_KNT]);
    const int c = nf + nh / 2, F = nf - 1;
    const double z1x = x[c] - x[F], z1y = y[c] - y[F];
    const double z2x = x[c + 1] - x[c - 1], z2y = y[c + 1] - y[c - 1];
    const double dot = z1x * z2x + z1y * z2y;
    E += sp[SP_KNA] * dot * dot;
    return E;
}

/* dE/dX of K (l/L0 - 1)^2 L0 between points a and b, subtracted from the forces */
static void spring_force(const double *x, const double *y, int a, int b, double L0, double K, double *fx,
                         double *fy)
{
    const double dx = x[b] - x[a], dy = y[b] - y[a];
    const double l = hypot(dx, dy);
    const double g = 2.0 * K * (l / L0 - 1.0) / l; /* dE/dX_b = g (X_b - X_a) */
    fx[b] -= g * dx;
    fy[b] -= g * dy;
    fx[a] += g * dx;
    fy[a] += g * dy;
}

/* dE/dX of W (kappa_B - k0)^2 h at the node B of (A, B, C), step h */
static void bend_force(const double *x, const double *y, int A, int B, int C, double h, double W, double k0,
                       double *fx, double *fy)
{
    const double a = (x[C] - x[A]) / (2.0 * h), b = (y[C] - y[A]) / (2.0 * h);
    const double p = (x[C] - 2.0 * x[B] + x[A]) / (h * h), q = (y[C] - 2.0 * y[B] + y[A]) / (h * h);
    const double S = a * a + b * b, S32 = pow(S, 1.5);
    const double num = q * a - p * b;
    const double co = 2.0 * W * (num / S32 - k0) * h; /* dE/dkappa */
    const double dka = q / S32 - 3.0 * a * num / (S32 * S);
    const double dkb = -p / S32 - 3.0 * b * num / (S32 * S);
    const double dkp = -b / S32, dkq = a / S32;
    const double i2 = 1.0 / (2.0 * h), i1 = 1.0 / (h * h);
    fx[A] -= co * (-dka * i2 + dkp * i1);
    fy[A] -= co * (-dkb * i2 + dkq * i1);
    fx[B] -= co * (-2.0 * dkp * i1);
    fy[B] -= co * (-2.0 * dkq * i1);
    fx[C] -= co * (dka * i2 + dkp * i1);
    fy[C] -= co * (dkb * i2 + dkq * i1);
}

static void sperm_forces(const osperm *g, const double *sp, double phase, double t, const double *x,
                         const double *y, double *fx, double *fy)
{
    const int nf = g->nf, nh = g->nh, n = nf + nh;
    for (int i = 0; i < n; ++i) fx[i] = fy[i] = 0.0;
    for (int k = 0; k + 1 < nf; ++k) spring_force(x, y, k, k + 1, g->ds, sp[SP_KT], fx, fy);
    for (int k = 1; k + 1 < nf; ++k)
        bend_force(x, y, k - 1, k, k + 1, g->ds, sp[SP_KC],
                   sperm_zhat(sp[SP_A], sp[SP_ETA], sp[SP_OMEGA], phase, (double)k * g->ds, t), fx, fy);
    for (int m = 0; m < nh; ++m) {
        const int nx = nf + (m + 1) % nh, pv = nf + (m + nh - 1) % nh;
        spring_force(x, y, nf + m, nx, g->ch, sp[SP_KHT], fx, fy);
        bend_force(x, y, pv, nf + m, nx, g->ch, sp[SP_KHC], 1.0 / g->hr, fx, fy);
    }
    for (int m = 0; m < nh / 2; ++m) spring_force(x, y, nf + m, nf + m + nh / 2, 2.0 * g->hr, sp[SP_KHT], fx, fy);
    for (int i = 0; i < 5; ++i) spring_force(x, y, g->na[i], g->nb[i], g->L0[i], sp[SP_KNT], fx, fy);
    /* angle: E = K (z1.z2)^2; dE/dz1 = 2 K (z1.z2) z2, dE/dz2 = 2 K (z1.z2) z1 */
    const int c = nf + nh / 2, F = nf - 1;
    const double z1x = x[c] - x[F], z1y = y[c] - y[F];
    const double z2x = x[c + 1] - x[c - 1], z2y = y[c + 1] - y[c - 1];
    const double w = 2.0 * sp[SP_KNA] * (z1x * z2x + z1y * z2y);
    fx[c] -= w * z2x;
    fy[c] -= w * z2y;
    fx[F] += w * z2x;
    fy[F] += w * z2y;
    fx[c + 1] -= w * z1x;
    fy[c + 1] -= w * z1y;
    fx[c - 1] += w * z1x;
    fy[c - 1] += w * z1y;
}

void oracle_sperm_initial(int nf, int nh, double hr, double dn, double x0, double y0, double *x, double *y)
{
    osperm g;
    sperm_geom(&g, nf, nh, hr, dn);
    sperm_initial(&g, x0, y0, x, y);
}

double oracle_sperm_energy(int nf, int nh, double hr, double dn, const double *sp, double phase, double t,
                           const double *x, const double *y)
{
    osperm g;
    sperm_geom(&g, nf, nh, hr, dn);
    sperm_rest_lengths(&g);
    return sperm_energy(&g, sp, phase, t, x, y);
}

void oracle_sperm_forces(int nf, int nh, double hr, double dn, const double *sp, double phase, double t,
                         const double *x, const double *y, double *fx, double *fy)
{
    osperm g;
    sperm_geom(&g, nf, nh, hr, dn);
    sperm_rest_lengths(&g);
    sperm_forces(&g, sp, phase, t, x, y, fx, fy);
}

/* ------------------------------------------------------------------------ */
/* Forward run of one system of n_swim sperm swimmers in one fluid (alpha   */
/* from the system row), blob width eps.  swp: n_swim rows (x0, y0, phase). */
/* Each step n (t = n dt): forces of every swimmer, velocity sum over all   */
/* points, Euler update, bound check.  Samples: index 0 is the initial      */
/* state, index j >= 1 follows step j*obs_every; each sample stores the     */
/* head centre (mean of the head points) and the tail end (flagellum point  */
/* 0) of every swimmer: head[(m*(n_obs+1) + j)*2 + {0,1}], same for tail.   */
/* Samples a stopped run does not reach are left untouched.                 */
/* ------------------------------------------------------------------------ */
int oracle_sperm_forward(int n_swim, int nf, int nh, double eps, double hr, double dn, const double *sp,
                         const double *swp, int steps, double dt, int obs_every, double *head, double *tail,
                         double *xout, double *yout, int *status)
{
    osperm g;
    sperm_geom(&g, nf, nh, hr, dn);
    sperm_rest_lengths(&g);
    const int np = nf + nh;
    const int64_t n = (int64_t)n_swim * np;
    const int n_obs = obs_every > 0 ? steps / obs_every : 0;
    double *x = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * n);
    double *fx = malloc(sizeof(double) * n), *fy = malloc(sizeof(double) * n);
    double *ux = malloc(sizeof(double) * n), *uy = malloc(sizeof(double) * n);
    okern k;
    kernel_init(&k, sp[SP_ALPHA], eps);
    for (int m = 0; m < n_swim; ++m) sperm_initial(&g, swp[3 * m], swp[3 * m + 1], x + m * np, y + m * np);
    int st = 0;
    for (int s = 0; s <= steps && st == 0; ++s) {
        if (s % (obs_every > 0 ? obs_every : steps + 1) == 0 && s / (obs_every > 0 ? obs_every : 1) <= n_obs) {
            const int j = obs_every > 0 ? s / obs_every : 0;
            for (int m = 0; m < n_swim; ++m) {
                double cx = 0.0, cy = 0.0;
                for (int i = 0; i < nh; ++i) {
                    cx += x[m * np + nf + i];
                    cy += y[m * np + nf + i];
                }
                double *hd = head + ((int64_t)m * (n_obs + 1) + j) * 2;
                double *tl = tail + ((int64_t)m * (n_obs + 1) + j) * 2;
                hd[0] = cx / (double)nh;
                hd[1] = cy / (double)nh;
                tl[0] = x[m * np];
                tl[1] = y[m * np];
            }
        }
        if (s == steps) break;
        const double t = (double)s * dt;
        for (int m = 0; m < n_swim; ++m)
            sperm_forces(&g, sp, swp[3 * m + 2], t, x + m * np, y + m * np, fx + m * np, fy + m * np);
        velocity_sum(&k, n, x, y, fx, fy, ux, uy);
        for (int64_t i = 0; i < n; ++i) {
            x[i] += dt * ux[i];
            y[i] += dt * uy[i];
        }
        for (int64_t i = 0; i < n; ++i) {
            if (!isfinite(x[i]) || !isfinite(y[i])) { st = 1; break; }
            if (fabs(x[i]) > 1e3 || fabs(y[i]) > 1e3) { st = 2; break; }
        }
    }
    if (xout) memcpy(xout, x, sizeof(double) * n);
    if (yout) memcpy(yout, y, sizeof(double) * n);
    *status = st;
    free(x); free(y); free(fx); free(fy); free(ux); free(uy);
    return 0;
}

/* ======================================================================== */
/* Flow and pressure at arbitrary points, eqs. (BrV) and (BrP) of Sec. 2.1. */
/*                                                                          */
/* The pressure of a regularized point force is p = F . grad G_eps with     */
/* Delta G_eps = phi (the same blob as the velocity), so for a radial blob  */
/* grad G_eps(x) = x m(r) / (2 pi r^2), m(r) = 2 pi int_0^r s phi(s) ds the */
/* blob mass inside r.  From (Delta - alpha^2) g = phi (see kernel_init),   */
/* m/(2 pi) = r g'(r) - alpha^2 M(r):                                       */
/*   Stokes:   m = r^2 / R^2                                                */
/*   Brinkman: m = 1 - eps K1(alpha R) / (R K1(alpha eps))                  */
/* Near contact (delta = r^2/eps^2 < 1/4), with g = sum gam_n delta^n,      */
/*   m / r^2 = (2 pi / eps^2) [ 2 sum_{n>=1} n gam_n delta^(n-1)            */
/*                              - (alpha^2 eps^2 / 2) sum_n gam_n delta^n / (n+1) ]. */
/* ------------------------------------------------------------------------ */
static ld mass_over_r2(const okern *k, double t_d)
{
    ld t = t_d;
    ld delta = t / k->e2;
    if (delta < DELTA_TAYLOR) {
        ld p = 1.0L, a = 0.0L, b = 0.0L;
        for (int n = 0; n < NGAM; ++n) {
            if (n + 1 < NGAM) a += (ld)(n + 1) * k->gam[n + 1] * p;
            b += k->gam[n] * p / (ld)(n + 1);
            p *= delta;
        }
        ld a2e2 = k->stokes ? 0.0L : (ld)k->alpha * (ld)k->alpha * k->e2;
        return (2.0L * PI_L / k->e2) * (2.0L * a - 0.5L * a2e2 * b);
    }
    ld R2 = t + k->e2;
    if (k->paper) {
        ld R = sqrtl(R2), e = (ld)k->eps;
        return (1.0L - e * e * e / (R2 * R)) / t;
    }
    if (k->stokes) return 1.0L / R2;
    ld R = sqrtl(R2);
    ld K0R, K1R, K0e, K1e;
    bessel_k01((ld)k->alpha * R, &K0R, &K1R);
    bessel_k01((ld)k->alpha * (ld)k->eps, &K0e, &K1e);
    return (1.0L - (ld)k->eps * K1R / (R * K1e)) / t;
}

/* blob of the kernel reading (kernel_init): phi(r) */
static ld blob_phi(const okern *k, double t_d)
{
    ld R2 = (ld)t_d + k->e2, R = sqrtl(R2);
    if (k->paper) return 3.0L * k->e2 * (ld)k->eps / (2.0L * PI_L * R2 * R2 * R);
    if (k->stokes) return k->e2 / (PI_L * R2 * R2);
    ld K0, K1, a = k->alpha;
    bessel_k01(a * R, &K0, &K1);
    return k->c * k->e2 / (2.0L * PI_L) * (a * a * K0 / R2 + 2.0L * a * K1 / (R2 * R));
}

void oracle_blob(double alpha, double eps, int64_t n, const double *t, double *phi, double *m_over_r2)
{
    okern k;
    kernel_init(&k, alpha, eps);
    for (int64_t i = 0; i < n; ++i) {
        phi[i] = (double)blob_phi(&k, t[i]);
        m_over_r2[i] = (double)mass_over_r2(&k, t[i]);
    }
}

/* velocity (eq. BrV) and pressure (eq. BrP) at nt target points from the n
 * regularized point forces of one system; index-order Neumaier sums */
void oracle_field(int64_t n, const double *x, const double *y, const double *fx, const double *fy,
                  double alpha, double eps, int64_t nt, const double *tx, const double *ty, double *u,
                  double *v, double *p)
{
    okern k;
    kernel_init(&k, alpha, eps);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t a = 0; a < nt; ++a) {
        double s[3] = {0, 0, 0}, c[3] = {0, 0, 0};
        for (int64_t j = 0; j < n; ++j) {
            double dx = tx[a] - x[j], dy = ty[a] - y[j];
            double t = dx * dx + dy * dy;
            ld H1, H2;
            kernel_eval(&k, t, &H1, &H2);
            double h1 = (double)H1, h2 = (double)H2;
            double fd = fx[j] * dx + fy[j] * dy;
            double w = (double)(mass_over_r2(&k, t) / (2.0L * PI_L));
            double val[3] = {h1 * fx[j] + h2 * fd * dx, h1 * fy[j] + h2 * fd * dy, fd * w};
            for (int q = 0; q < 3; ++q) {
                double z = s[q] + val[q];
                c[q] += (fabs(s[q]) >= fabs(val[q])) ? (s[q] - z) + val[q] : (val[q] - z) + s[q];
                s[q] = z;
            }
        }
        u[a] = s[0] + c[0];
        v[a] = s[1] + c[1];
        p[a] = s[2] + c[2];
    }
}
