/*
 * FP64 CPU oracle for the coarse-grained Green's-function Brownian-dynamics
 * step of Pruestel & Meier-Schellersheim (arXiv:1107.0270).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It is plain,
 * single-threaded C99 in binary64, written for checking by eye against the
 * paper: the simulation step follows Sec. 3 (steps 1-5 and the Details list),
 * the Green's functions follow Secs. 2.2 and 4.  Where a quantity is a plain
 * ratio of Green's functions (encounter probability, reaction probability)
 * the code evaluates that ratio after cancelling the common factors by exact
 * algebra; the derivation is written next to each function, and the tests pin
 * each one against the literal ratio evaluated in 50-digit arithmetic.
 *
 * Readings of points the paper leaves open (all listed in the design doc):
 *   - cut-off: r_cut solves 1 - S(dt | r_cut) = eps (Sec. 3, Details);
 *   - overlapping pairs get p_enc = 1; a pre-step separation below a is
 *     clamped to a;
 *   - candidate lists are ordered by slot index; the A side picks first, then
 *     each B arbitrates among the A's that picked it (Sec. 3, Details);
 *   - the propagated pair keeps the direction of its free end point, only the
 *     radius is redrawn (radial propagator of Sec. 3, Details);
 *   - the product C is placed at the diffusion-weighted centre (eq. Rcoo);
 *   - C diffuses with D_C; a C made in this step does not decay in it.
 */
#define _DEFAULT_SOURCE /* the Bessel functions j0, j1, y0, y1 of the C library */
#include "gfbd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846
#define SQRTPI 1.77245385090551602730

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: ten rounds of the Philox S-P network with the published    */
/* multipliers and Weyl key schedule (Salmon, Moraes, Dror, Shaw, SC'11).    */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t m0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t m1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(m0 >> 32), lo0 = (uint32_t)m0;
        uint32_t hi1 = (uint32_t)(m1 >> 32), lo1 = (uint32_t)m1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double orc_u01(uint32_t x) { return ((double)x + 0.5) * 2.3283064365386962890625e-10; }

static void draw(const uint32_t ctr[4], const uint32_t key[2], double u[4], uint32_t w[4])
{
    orc_philox4x32_10(ctr, key, w);
    for (int k = 0; k < 4; ++k) u[k] = orc_u01(w[k]);
}

/* ------------------------------------------------------------------------ */
/* Special functions                                                         */
/* ------------------------------------------------------------------------ */

/* e^{x^2} erfc(x).  Below 3 the library erfc times exp(x^2); above, the     */
/* Laplace continued fraction  sqrt(pi) e^{x^2} erfc(x) =                    */
/*   1/(x + (1/2)/(x + 1/(x + (3/2)/(x + ...))))  evaluated bottom-up.       */
double orc_erfcx(double x)
{
    if (x < 3.0) return exp(x * x) * erfc(x);
    double f = x;
    for (int k = 80; k >= 1; --k) f = x + (0.5 * k) / f;
    return 1.0 / (SQRTPI * f);
}

/* Repeated integrals of erfc scaled by e^{x^2}: out[k+1] = e^{x^2} i^k erfc(x)
 * for k = -1..kmax, with i^{-1}erfc = (2/sqrt(pi)) e^{-x^2}, i^0 erfc = erfc
 * and the recursion 2k i^k = i^{k-2} - 2x i^{k-1} of Sec. 4.2 (eq. iErf). */
void orc_ierfcx(double x, int kmax, double *out)
{
    out[0] = 2.0 / SQRTPI;
    out[1] = orc_erfcx(x);
    for (int k = 1; k <= kmax; ++k) out[k + 1] = (out[k - 1] - 2.0 * x * out[k]) / (2.0 * k);
}

/* Large-argument coefficients a_k(nu) of the modified Bessel functions
 * (Sec. 4.2, eq. coeffDef): a_k = prod_{m=1..k} (4 nu^2 - (2m-1)^2) / (k! 8^k). */
void orc_asym_coeffs(double nu, int n, double *a)
{
    a[0] = 1.0;
    for (int k = 1; k <= n; ++k) a[k] = a[k - 1] * (4.0 * nu * nu - (2.0 * k - 1.0) * (2.0 * k - 1.0)) / (8.0 * k);
}

/* e^{-x} I_0(x): ascending series sum (x^2/4)^k/(k!)^2 up to x = 20, above it
 * the large-argument series e^x/sqrt(2 pi x) sum_k (-1)^k a_k(0) x^-k (the
 * expansion quoted in Sec. 4.2), truncated at its smallest term. */
double orc_i0e(double x)
{
    x = fabs(x);
    if (x <= 20.0) {
        double q = 0.25 * x * x, term = 1.0, sum = 1.0;
        for (int k = 1; k < 400; ++k) {
            term *= q / ((double)k * (double)k);
            sum += term;
            if (term < 1e-18 * sum) break;
        }
        return sum * exp(-x);
    }
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 200; ++k) {
        double t = term * ((2.0 * k - 1.0) * (2.0 * k - 1.0)) / (8.0 * k * x);
        if (t >= term) break;
        term = t;
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum / sqrt(2.0 * PI * x);
}

/* ln erfc(y) for y >= 0 */
static double lnerfc(double y) { return -y * y + log(orc_erfcx(y)); }

/* The y >= yc (yc >= 0) with erfc(y) = u erfc(yc), 0 < u <= 1: safeguarded
 * Newton iteration on ln erfc, whose derivative is -2/(sqrt(pi) erfcx(y)). */
double orc_erfc_tail_inv(double yc, double u)
{
    if (u >= 1.0) return yc;
    double target = log(u) + lnerfc(yc);
    double lo = yc, hi = yc + 1.0;
    while (lnerfc(hi) > target) hi = 2.0 * hi + 1.0;
    double y = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        double f = lnerfc(y) - target; /* decreasing in y */
        if (f > 0) lo = y; else hi = y;
        double step = f * SQRTPI * orc_erfcx(y) / 2.0; /* -f / f' */
        double yn = y + step;
        if (!(yn > lo && yn < hi)) yn = 0.5 * (lo + hi);
        if (fabs(yn - y) <= 1e-16 * (1.0 + fabs(y))) { y = yn; break; }
        y = yn;
    }
    return y;
}

/* ------------------------------------------------------------------------ */
/* 3D radial Green's functions (Sec. 4.1), multiplied by a^3.                */
/* ------------------------------------------------------------------------ */

/* Free radial Green's function: the angular average (eq. radialGF) of the
 * Gaussian (eq. gaussian) with D = D_eff:
 *   a^3 g_free = [e^{-(R-R0)^2/4tau} - e^{-(R+R0)^2/4tau}] / (8 pi R R0 sqrt(pi tau)). */
double orc_g3_free(double R, double R0, double tau)
{
    double pre = 1.0 / (8.0 * PI * R * R0 * sqrt(PI * tau));
    return pre * (exp(-(R - R0) * (R - R0) / (4.0 * tau)) - exp(-(R + R0) * (R + R0) / (4.0 * tau)));
}

/* Absorbing closed form of Sec. 4.1. */
double orc_g3_abs(double R, double R0, double tau)
{
    double w = R + R0 - 2.0;
    double pre = 1.0 / (8.0 * PI * R * R0 * sqrt(PI * tau));
    return pre * (exp(-(R - R0) * (R - R0) / (4.0 * tau)) - exp(-w * w / (4.0 * tau)));
}

/* Radiation closed form of Sec. 4.1 with kappa = 1 + h (h = kappa_a/(4 pi a D));
 * h = 0 gives the reflecting function.  The product exp(kappa^2 tau + w kappa)
 * erfc(z), z = kappa sqrt(tau) + w/(2 sqrt(tau)), equals e^{-w^2/4tau} erfcx(z)
 * exactly (z^2 = kappa^2 tau + w kappa + w^2/4tau); that form is used so the
 * product neither overflows nor underflows.  The term carries a minus sign
 * (the paper's line break shows "+ -"). */
double orc_g3_rad(double R, double R0, double tau, double hh)
{
    double w = R + R0 - 2.0, kap = 1.0 + hh, st = sqrt(tau);
    double pre = 1.0 / (8.0 * PI * R * R0 * sqrt(PI * tau));
    double ew = exp(-w * w / (4.0 * tau));
    double z = kap * st + w / (2.0 * st);
    return pre * (exp(-(R - R0) * (R - R0) / (4.0 * tau)) + ew - kap * sqrt(4.0 * PI * tau) * ew * orc_erfcx(z));
}

/* Encounter probability p_enc = 1 - g_abs/g_free (Sec. 2.2.1, eq. bayes1D,
 * radial form of Sec. 2.2.4).  Both functions share the prefactor; after
 * multiplying numerator and denominator by e^{(R-R0)^2/4tau} and using
 * (R+R0-2)^2 - (R-R0)^2 = 4(R-1)(R0-1), (R+R0)^2 - (R-R0)^2 = 4 R R0:
 *   p_enc = [e^{-(R-1)(R0-1)/tau} - e^{-R R0/tau}] / [1 - e^{-R R0/tau}]
 *         = e^{-(R-1)(R0-1)/tau} (1 - e^{-(R+R0-1)/tau}) / (1 - e^{-R R0/tau}). */
double orc_penc3(double R, double R0, double tau)
{
    if (R <= 1.0) return 1.0;
    return exp(-(R - 1.0) * (R0 - 1.0) / tau) * (-expm1(-(R + R0 - 1.0) / tau)) / (-expm1(-R * R0 / tau));
}

/* Reaction probability (g_ref - g_rad)/(g_ref - g_abs) of Sec. 2.2.3
 * (eq. psurv_radII) with the Sec. 4.1 closed forms.  The free-space term
 * e^{-(R-R0)^2/4tau} cancels in both differences, and so does the common
 * factor e^{-w^2/4tau} pre:
 *   g_ref - g_rad = 2 sqrt(pi tau) [kappa erfcx(z_kappa) - erfcx(z_1)]
 *   g_ref - g_abs = 2 - 2 sqrt(pi tau) erfcx(z_1). */
double orc_preac3(double R, double R0, double tau, double hh)
{
    double w = R + R0 - 2.0, st = sqrt(tau), kap = 1.0 + hh;
    double z1 = st + w / (2.0 * st), zk = kap * st + w / (2.0 * st);
    double spt = sqrt(PI * tau);
    return spt * (kap * orc_erfcx(zk) - orc_erfcx(z1)) / (1.0 - spt * orc_erfcx(z1));
}

/* 1 - S_abs(tau | R0): the integral of eq. SurvRad over the absorbing closed
 * form, erfc((R0-1)/(2 sqrt tau)) / R0. */
double orc_loss3_abs(double R0, double tau)
{
    return erfc((R0 - 1.0) / (2.0 * sqrt(tau))) / R0;
}

/* 1 - S_rad(tau | R0) for the radiation closed form:
 *   (1/R0) (h/kappa) [erfc(u0) - e^{-u0^2} erfcx(u0 + kappa sqrt(tau))],
 * u0 = (R0-1)/(2 sqrt tau), kappa = 1 + h. */
double orc_loss3_rad(double R0, double tau, double hh)
{
    double st = sqrt(tau), u0 = (R0 - 1.0) / (2.0 * st), kap = 1.0 + hh;
    return (hh / kap) * (erfc(u0) - exp(-u0 * u0) * orc_erfcx(u0 + kap * st)) / R0;
}

/* Radial propagator density w_3 r^2 (g_ref - g_abs), per unit R' (Sec. 3,
 * Details), from the literal Green's functions. */
double orc_prop3_density(double Rp, double R0, double tau)
{
    return 4.0 * PI * Rp * Rp * (orc_g3_rad(Rp, R0, tau, 0.0) - orc_g3_abs(Rp, R0, tau));
}

/* ------------------------------------------------------------------------ */
/* 2D small-time expansions (Sec. 4.2).                                      */
/* ------------------------------------------------------------------------ */

#define MAXN 64

static void ser_mul(const double *x, const double *y, int n, double *z)
{
    for (int k = 0; k <= n; ++k) {
        double s = 0.0;
        for (int m = 0; m <= k; ++m) s += x[m] * y[k - m];
        z[k] = s;
    }
}

static void ser_div(const double *x, const double *y, int n, double *z)
{
    for (int k = 0; k <= n; ++k) {
        double s = x[k];
        for (int m = 1; m <= k; ++m) s -= y[m] * z[k - m];
        z[k] = s / y[0];
    }
}

/* Expansion coefficients gamma_k(R, R0), k = 0..n, of eq. expansionLaplace.
 * With s = 1/q~, K_nu(x) ~ sqrt(pi/2x) e^{-x} A_nu(1/x) and
 * I_nu(x) ~ e^x/sqrt(2 pi x) Abar_nu(1/x), A_nu(s) = sum a_k(nu) s^k,
 * Abar_nu(s) = sum (-1)^k a_k(nu) s^k, and I_0' = I_1, K_0' = -K_1, the three
 * boundary components (eqs. absPert, refPert, radPert) become
 *   abs: [Abar_0(s)/A_0(s)]                                  A_0(s/R0) A_0(s/R)
 *   rad: [(Abar_1(s) - h s Abar_0(s))/(A_1(s) + h s A_0(s))] A_0(s/R0) A_0(s/R)
 *   ref: the rad series at h = 0,
 * times the common factor e^{-q~(R+R0-2)}/(4 pi D sqrt(R R0) q~) (sign - for
 * abs).  The truncated power series are multiplied and divided term by term. */
void orc_gamma2(double R, double R0, double hh, int n, double *g_abs, double *g_ref, double *g_rad)
{
    double a0[MAXN + 1], a1[MAXN + 1], b0[MAXN + 1], b1[MAXN + 1];
    double x[MAXN + 1], y[MAXN + 1], P[MAXN + 1], Q[MAXN + 1], num[MAXN + 1], den[MAXN + 1];
    orc_asym_coeffs(0.0, n, a0);
    orc_asym_coeffs(1.0, n, a1);
    for (int k = 0; k <= n; ++k) {
        double sg = (k & 1) ? -1.0 : 1.0;
        b0[k] = sg * a0[k];
        b1[k] = sg * a1[k];
        x[k] = a0[k] * pow(R0, -k);
        y[k] = a0[k] * pow(R, -k);
    }
    ser_mul(x, y, n, P);
    if (g_abs) {
        ser_div(b0, a0, n, Q);
        ser_mul(Q, P, n, g_abs);
    }
    if (g_ref) {
        ser_div(b1, a1, n, Q);
        ser_mul(Q, P, n, g_ref);
    }
    if (g_rad) {
        for (int k = 0; k <= n; ++k) {
            num[k] = b1[k] - (k >= 1 ? hh * b0[k - 1] : 0.0);
            den[k] = a1[k] + (k >= 1 ? hh * a0[k - 1] : 0.0);
        }
        ser_div(num, den, n, Q);
        ser_mul(Q, P, n, g_rad);
    }
}

/* Boundary components of the 2D radial Green's functions in the time domain
 * (eqs. smallTEabs, smallTEabsII), times a^2:
 *   +-[pi^{-1/2} e^{-x^2} + (1/2) sum_{k=1..n} gamma_k i^{k-1}erfc(x) (2 sqrt tau)^k]
 *   / (4 pi sqrt(tau R R0)),   x = (R+R0-2)/(2 sqrt tau),
 * with the minus sign for kind 0 (absorbing); kind 1 = reflecting, 2 = radiation. */
double orc_g2_bc(int kind, double R, double R0, double tau, double hh, int n)
{
    double ga[MAXN + 1], gf[MAXN + 1], gr[MAXN + 1], it[MAXN + 2];
    orc_gamma2(R, R0, hh, n, ga, gf, gr);
    const double *g = kind == 0 ? ga : (kind == 1 ? gf : gr);
    double st = sqrt(tau), x = (R + R0 - 2.0) / (2.0 * st);
    orc_ierfcx(x, n, it);
    double S = 1.0 / SQRTPI, pw = 1.0;
    for (int k = 1; k <= n; ++k) {
        pw *= 2.0 * st;
        S += 0.5 * g[k] * it[k] * pw; /* it[k] = e^{x^2} i^{k-1} erfc(x) */
    }
    double val = exp(-x * x) * S / (4.0 * PI * sqrt(tau * R * R0));
    return kind == 0 ? -val : val;
}

/* Free 2D radial Green's function: the angular average of the planar
 * Gaussian, e^{-(R^2+R0^2)/4tau} I_0(R R0/2tau) / (4 pi tau), times a^2. */
double orc_g2_free(double R, double R0, double tau)
{
    return exp(-(R - R0) * (R - R0) / (4.0 * tau)) * orc_i0e(R * R0 / (2.0 * tau)) / (4.0 * PI * tau);
}

/* p_enc = 1 - g_abs/g_free = -g_abs,bc/g_free (eq. laplaceAnsatz).  Dividing
 * the expansion by the free function and combining the exponentials,
 * -x^2 + (R-R0)^2/4tau = -(R-1)(R0-1)/tau:
 *   p_enc = sqrt(tau/(R R0)) e^{-(R-1)(R0-1)/tau} S_abs / i0e(R R0/2tau),
 *   S_abs = pi^{-1/2} + (1/2) sum gamma^abs_k e^{x^2} i^{k-1}erfc(x) (2 sqrt tau)^k. */
double orc_penc2(double R, double R0, double tau, int n)
{
    if (R <= 1.0) return 1.0;
    double ga[MAXN + 1], it[MAXN + 2];
    orc_gamma2(R, R0, 0.0, n, ga, NULL, NULL);
    double st = sqrt(tau), x = (R + R0 - 2.0) / (2.0 * st);
    orc_ierfcx(x, n, it);
    double S = 1.0 / SQRTPI, pw = 1.0;
    for (int k = 1; k <= n; ++k) {
        pw *= 2.0 * st;
        S += 0.5 * ga[k] * it[k] * pw;
    }
    return sqrt(tau / (R * R0)) * exp(-(R - 1.0) * (R0 - 1.0) / tau) * S / orc_i0e(R * R0 / (2.0 * tau));
}

/* p_reac = (g_ref - g_rad)/(g_ref - g_abs) (eq. psurv_radII).  The free parts
 * cancel; so does the common factor e^{-x^2}/(4 pi sqrt(tau R R0)):
 *   p_reac = sum (g^ref_k - g^rad_k) T_k / [4 pi^{-1/2} + sum (g^ref_k + g^abs_k) T_k],
 *   T_k = e^{x^2} i^{k-1}erfc(x) (2 sqrt tau)^k. */
double orc_preac2(double R, double R0, double tau, double hh, int n)
{
    double ga[MAXN + 1], gf[MAXN + 1], gr[MAXN + 1], it[MAXN + 2];
    orc_gamma2(R, R0, hh, n, ga, gf, gr);
    double st = sqrt(tau), x = (R + R0 - 2.0) / (2.0 * st);
    orc_ierfcx(x, n, it);
    double num = 0.0, den = 4.0 / SQRTPI, pw = 1.0;
    for (int k = 1; k <= n; ++k) {
        pw *= 2.0 * st;
        double T = it[k] * pw;
        num += (gf[k] - gr[k]) * T;
        den += (gf[k] + ga[k]) * T;
    }
    return num / den;
}

/* Radial propagator density w_2 r (g_ref - g_abs) per unit R' (Sec. 3,
 * Details), from the expansions of the boundary components. */
double orc_prop2_density(double Rp, double R0, double tau, int n)
{
    return 2.0 * PI * Rp * (orc_g2_bc(1, Rp, R0, tau, 0.0, n) - orc_g2_bc(0, Rp, R0, tau, 0.0, n));
}

/* 1 + (sqrt(pi)/4) sum (g^ref_k + g^abs_k) T_k at (R', R0): the 2D propagator
 * density divided by its leading term (1/2) sqrt(R'/(tau R0)) e^{-x'^2} (2/sqrt(pi)). */
static double prop2_corr(double Rp, double R0, double tau, int n)
{
    double ga[MAXN + 1], gf[MAXN + 1], it[MAXN + 2];
    orc_gamma2(Rp, R0, 0.0, n, ga, gf, NULL);
    double st = sqrt(tau), x = (Rp + R0 - 2.0) / (2.0 * st);
    orc_ierfcx(x, n, it);
    double s = 0.0, pw = 1.0;
    for (int k = 1; k <= n; ++k) {
        pw *= 2.0 * st;
        s += (gf[k] + ga[k]) * it[k] * pw;
    }
    return 1.0 + 0.25 * SQRTPI * s;
}

/* ------------------------------------------------------------------------ */
/* Exact 2D radial Green's functions, beyond the small-time regime: the       */
/* n = 0 term of the 2D Green's function (eq. genericGF) with the radial      */
/* function of eq. fRad, by quadrature of its integral over x (times a^2):    */
/*   g(R, tau | R0) = (1/2 pi) int_0^inf e^{-tau x^2} C0(R,x) C0(R0,x) x dx,  */
/*   C0(R, x) = [J0(Rx) A(x) - Y0(Rx) B(x)] / sqrt(A^2 + B^2),               */
/* radiation A = x Y0'(x) - h Y0(x), B = x J0'(x) - h J0(x) (reflecting:     */
/* h = 0); absorbing A = Y0(x), B = J0(x) (the limit h -> inf, up to a sign   */
/* common to both factors).  The mass within R of the boundary, used by the   */
/* propagator, integrates the R' factor in closed form:                       */
/*   int_1^R 2 pi R' g(R'|R0) dR' = int_0^inf e^{-tau x^2} C0(R0,x) K(R,x) x dx,*/
/*   K(R, x) = [A (R J1(Rx) - J1(x)) - B (R Y1(Rx) - Y1(x))] / (x sqrt(A^2+B^2)).*/
/* Quadrature: 16-point Gauss-Legendre panels, geometric (ratio 2) from       */
/* 2^-30/4 up to 1/4 where the absorbing and radiation kernels vary like      */
/* 1/ln x, then of width <= min(1/4, pi/f) with f = R + R0 + 1 (the fastest   */
/* oscillation of the integrand), up to x = sqrt(50/tau) (e^{-50}).           */
/* ------------------------------------------------------------------------ */
#define GLN 16
static double gl_x[GLN], gl_w[GLN];
static int gl_ready;

static void gl_init(void)
{
    if (gl_ready) return;
    for (int i = 0; i < GLN; ++i) {
        double z = cos(PI * (i + 0.75) / (GLN + 0.5)), p0 = 1.0, p1 = z, dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            p0 = 1.0;
            p1 = z;
            for (int k = 2; k <= GLN; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = GLN * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        gl_x[i] = z;
        gl_w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    gl_ready = 1;
}

/* A, B of C0 for kind 0 (absorbing), 1 (reflecting), 2 (radiation) */
static void c0_ab(int kind, double x, double hh, double j0x, double y0x, double j1x, double y1x, double *A, double *B)
{
    if (kind == 0) {
        *A = y0x;
        *B = j0x;
        return;
    }
    double h = kind == 1 ? 0.0 : hh;
    *A = -x * y1x - h * y0x;
    *B = -x * j1x - h * j0x;
}

/* The integrals at one node x: g-integrands of the three kinds at (R, R0)
 * (mode 0), or the mass integrands of the absorbing and reflecting kinds
 * together with their g-integrands at (R, R0) (mode 1). */
static void x_terms(int mode, double x, double R, double R0, double hh, double out[4])
{
    double j0x = j0(x), y0x = y0(x), j1x = j1(x), y1x = y1(x);
    double jr = j0(R * x), yr = y0(R * x), jq = j0(R0 * x), yq = y0(R0 * x);
    if (mode == 0) {
        for (int kind = 0; kind < 3; ++kind) {
            double A, B;
            c0_ab(kind, x, hh, j0x, y0x, j1x, y1x, &A, &B);
            double N2 = A * A + B * B;
            out[kind] = (jr * A - yr * B) * (jq * A - yq * B) / N2 * x;
        }
        return;
    }
    double j1r = j1(R * x), y1r = y1(R * x);
    for (int kind = 0; kind < 2; ++kind) {
        double A, B;
        c0_ab(kind, x, hh, j0x, y0x, j1x, y1x, &A, &B);
        double N2 = A * A + B * B, cq = jq * A - yq * B;
        out[kind] = cq * (A * (R * j1r - j1x) - B * (R * y1r - y1x)) / N2;        /* x C0(R0) K(R) */
        out[2 + kind] = (jr * A - yr * B) * cq / N2 * x;                           /* x C0(R0) C0(R) */
    }
}

static void x_integrate(int mode, double R, double R0, double tau, double hh, double freq, double acc[4])
{
    gl_init();
    for (int k = 0; k < 4; ++k) acc[k] = 0.0;
    double xmax = sqrt(50.0 / tau), x1 = xmax < 0.25 ? xmax : 0.25;
    double wmax = PI / freq;
    if (wmax > 0.25) wmax = 0.25;
    int ngeo = 30, nuni = (int)ceil((xmax - x1) / wmax);
    double wuni = nuni > 0 ? (xmax - x1) / nuni : 0.0;
    for (int p = 0; p < ngeo + nuni; ++p) {
        double lo, hi;
        if (p < ngeo) {
            lo = ldexp(x1, p - ngeo);
            hi = 2.0 * lo;
        } else {
            lo = x1 + (p - ngeo) * wuni;
            hi = lo + wuni;
        }
        double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
        for (int i = 0; i < GLN; ++i) {
            double x = c + h * gl_x[i], t[4];
            x_terms(mode, x, R, R0, hh, t);
            double wgt = h * gl_w[i] * exp(-tau * x * x);
            for (int k = 0; k < 4; ++k) acc[k] += wgt * t[k];
        }
    }
}

void orc_g2x(double R, double R0, double tau, double hh, double out[3])
{
    double acc[4];
    x_integrate(0, R, R0, tau, hh, R + R0 + 1.0, acc);
    for (int k = 0; k < 3; ++k) out[k] = acc[k] / (2.0 * PI);
}

void orc_m2x(double R, double R0, double tau, double out[2])
{
    double acc[4];
    x_integrate(1, R, R0, tau, 0.0, R + R0 + 1.0, acc);
    out[0] = acc[0];
    out[1] = acc[1];
}

/* p_enc = 1 - g_abs/g_free (eq. laplaceAnsatz) with the exact g_abs */
double orc_penc2x(double R, double R0, double tau)
{
    if (R <= 1.0) return 1.0;
    double g[3];
    orc_g2x(R, R0, tau, 0.0, g);
    return 1.0 - g[0] / orc_g2_free(R, R0, tau);
}

/* p_reac = (g_ref - g_rad)/(g_ref - g_abs) (eq. psurv_radII) with the exact functions */
double orc_preac2x(double R, double R0, double tau, double hh)
{
    double g[3];
    orc_g2x(R, R0, tau, hh, g);
    return (g[1] - g[2]) / (g[1] - g[0]);
}

/* R'' >= 1 from w_2 r (g_ref - g_abs)(.|R0) by inversion with one uniform u:
 * the root of M(R) = u M(R_top), M(R) = int_1^R 2 pi R'(g_ref - g_abs) dR',
 * R_top = R0 + 12 sqrt(tau) + 1 (the mass beyond it is below e^{-36}).
 * Newton steps on M with its derivative 2 pi R (g_ref - g_abs), kept inside
 * a bracket that bisection takes over whenever a step leaves it. */
double orc_sample_prop2x(double R0, double tau, double u)
{
    double top = R0 + 12.0 * sqrt(tau) + 1.0, acc[4];
    double freq = top + R0 + 1.0;
    x_integrate(1, top, R0, tau, 0.0, freq, acc);
    double target = u * (acc[1] - acc[0]);
    double lo = 1.0, hi = top, x = R0 > 1.0 ? R0 : 1.0 + sqrt(tau);
    for (int it = 0; it < 200; ++it) {
        x_integrate(1, x, R0, tau, 0.0, freq, acc);
        double f = (acc[1] - acc[0]) - target, df = (acc[3] - acc[2]) * x;
        if (f < 0.0) lo = x;
        else hi = x;
        double nx = df > 0.0 ? x - f / df : 0.5 * (lo + hi);
        if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
        if (fabs(nx - x) <= 1e-13 * x || hi - lo <= 1e-13 * x) return nx;
        x = nx;
    }
    return x;
}

/* ------------------------------------------------------------------------ */
/* Radial propagator sampler.  With c = R0 - 1 and v = R' + R0 - 2 >= c:     */
/*   3D: density ~ (1 + v - c) e^{-v^2/4tau} [1 - sqrt(pi tau) erfcx(z1)],   */
/*       z1 = sqrt(tau) + v/(2 sqrt(tau))  (ref minus abs closed forms);     */
/*   2D: density ~ sqrt(1 + v - c) e^{-v^2/4tau} corr(v)  (expansions).      */
/* Proposal ~ (1 + beta (v - c)) e^{-v^2/4tau} with beta = 1 (3D), 1/2 (2D), */
/* a two-part mixture of a Gaussian tail and a Rayleigh tail when            */
/* beta c <= 1, else the Rayleigh tail beta v e^{-v^2/4tau} alone.  Attempt  */
/* k uses the counter with k in the upper 24 bits of word 3; of its four     */
/* words, 0 picks the mixture part, 1 inverts the part's tail, 2 accepts.    */
/* ------------------------------------------------------------------------ */
#define MAX_ATTEMPTS 4096u

double orc_sample_prop(int dim, double R0, double tau, int n_terms, const uint32_t ctr[4],
                       const uint32_t key[2], uint32_t *attempts, uint32_t *bound_hits)
{
    double c = R0 - 1.0;
    if (c < 0.0) c = 0.0;
    double st = sqrt(tau), yc = c / (2.0 * st);
    double beta = dim == 3 ? 1.0 : 0.5;
    int mixture = beta * c <= 1.0;
    double w1 = 0.0, w2 = 0.0;
    if (mixture) {
        w1 = (1.0 - beta * c) * sqrt(PI * tau) * orc_erfcx(yc);
        w2 = 2.0 * tau * beta;
    }
    double v = c;
    for (uint32_t k = 0; k < MAX_ATTEMPTS; ++k) {
        uint32_t ct[4] = {ctr[0], ctr[1], ctr[2], (ctr[3] & 0xFFu) | (k << 8)};
        double u[4];
        uint32_t w[4];
        draw(ct, key, u, w);
        double acc;
        if (mixture) {
            if (u[0] * (w1 + w2) < w1) v = 2.0 * st * orc_erfc_tail_inv(yc, u[1]);
            else v = sqrt(c * c - 4.0 * tau * log(u[1]));
            acc = 1.0;
        } else {
            v = sqrt(c * c - 4.0 * tau * log(u[1]));
            acc = (1.0 + beta * (v - c)) / (beta * v);
        }
        double Rp = 1.0 + v - c;
        if (dim == 3) {
            acc *= 1.0 - sqrt(PI * tau) * orc_erfcx(st + v / (2.0 * st));
        } else {
            double corr = prop2_corr(Rp, R0, tau, n_terms);
            if (corr > 1.0) {
                if (bound_hits) ++*bound_hits;
                corr = 1.0;
            }
            if (corr < 0.0) corr = 0.0;
            acc *= sqrt(Rp) / (1.0 + 0.5 * (Rp - 1.0)) * corr;
        }
        if (u[2] < acc) {
            *attempts = k + 1;
            return Rp;
        }
    }
    *attempts = MAX_ATTEMPTS;
    return 1.0 + v - c;
}

/* ------------------------------------------------------------------------ */
/* Cut-off radius: 1 - S(dt | r_cut) = eps (Sec. 3, Details), S_abs for      */
/* absorbing and reflecting pairs, S_rad for radiation pairs (3D closed      */
/* forms).  2D has no closed form; the planar loss erfc((R0-1)/(2 sqrt tau)) */
/* bounds the 2D loss from above, so its root is a conservative cut-off.     */
/* ------------------------------------------------------------------------ */
static double loss_at(int dim, int bc, double R0, double tau, double hh)
{
    if (dim == 2) return erfc((R0 - 1.0) / (2.0 * sqrt(tau)));
    if (bc == ORC_BC_RAD) return orc_loss3_rad(R0, tau, hh);
    return orc_loss3_abs(R0, tau);
}

double orc_rcut(int dim, int bc, double a, double Deff, double dt, double kappa_a, double eps)
{
    double tau = Deff * dt / (a * a);
    double hh = dim == 3 ? kappa_a / (4.0 * PI * a * Deff) : kappa_a / (2.0 * PI * Deff);
    if (loss_at(dim, bc, 1.0, tau, hh) <= eps) return a;
    double lo = 1.0, hi = 2.0;
    while (loss_at(dim, bc, hi, tau, hh) > eps) hi = 1.0 + 2.0 * (hi - 1.0);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (loss_at(dim, bc, mid, tau, hh) > eps) lo = mid; else hi = mid;
    }
    return a * hi;
}

/* ------------------------------------------------------------------------ */
/* The simulation step (Sec. 3).                                             */
/* Random draws: key = {seed_lo, seed_hi ^ replica}; counter =               */
/* {slot i, partner j or 0xFFFFFFFF, step, tag | attempt << 8}.             */
/* ------------------------------------------------------------------------ */
enum { TAG_MOVE = 1, TAG_ENC = 2, TAG_SELA = 3, TAG_SELB = 4, TAG_PROP = 5, TAG_REAC = 6,
       TAG_UNI = 7, TAG_DPROP = 8, TAG_DIR = 9, TAG_GEM = 10, TAG_FPT = 11, TAG_FPTU = 12, TAG_ANG = 13 };
#define NOSLOT 0xFFFFFFFFu

struct orc_sim {
    orc_params p;
    uint64_t cap, step;
    int32_t *sp;
    double *x, *xm, *dx;
    /* stage parity: the next step takes its post-move positions and displacements from the
     * caller (orc_sim_set_moved); its own move goes to xo for comparison */
    int given;
    double *xg, *dg, *xo;
    uint32_t *partner;
    uint8_t *born;
    double Deff, tau, hh, rcut, a, p_uni;
    uint32_t key[2];
    orc_pair *pairs;
    uint64_t n_pairs, c_pairs;
    orc_pick *picks;
    uint64_t n_picks, c_picks;
    orc_match *matches;
    uint64_t n_matches, c_matches;
    orc_diss *diss;
    uint64_t n_diss, c_diss;
    uint64_t st[ORC_ST_N];
};

static void *grow(void *ptr, uint64_t *capn, uint64_t need, size_t elt)
{
    if (need <= *capn) return ptr;
    uint64_t nc = *capn ? *capn : 1024;
    while (nc < need) nc *= 2;
    *capn = nc;
    return realloc(ptr, nc * elt);
}

/* Wrap into [0, L) and round to the state precision; a value that the
 * rounding carries up to L wraps to 0. */
static double wrap_store(const orc_sim *s, double y, double L)
{
    while (y < 0.0) y += L;
    while (y >= L) y -= L;
    if (s->p.store_f32) y = (double)(float)y;
    if (y >= L) y -= L;
    return y;
}

static double min_image(double d, double L)
{
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

orc_sim *orc_sim_create(const orc_params *p, uint64_t n, const int32_t *species, const double *pos,
                        const uint32_t *partner)
{
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->p = *p;
    s->cap = n;
    s->sp = (int32_t *)malloc(n * sizeof(int32_t));
    s->x = (double *)calloc(n * 3, sizeof(double));
    s->xm = (double *)calloc(n * 3, sizeof(double));
    s->dx = (double *)calloc(n * 3, sizeof(double));
    s->partner = (uint32_t *)malloc(n * sizeof(uint32_t));
    s->born = (uint8_t *)calloc(n, 1);
    int d = p->dim;
    for (uint64_t i = 0; i < n; ++i) {
        s->sp[i] = species[i];
        s->partner[i] = partner ? partner[i] : NOSLOT;
        for (int k = 0; k < d; ++k) s->x[i * 3 + k] = wrap_store(s, pos[i * d + k], p->box[k]);
    }
    s->a = p->sigma;
    s->Deff = p->D[0] + p->D[1];
    s->tau = s->Deff * p->dt / (s->a * s->a);
    if (p->bc == ORC_BC_REF) s->hh = 0.0;
    else if (d == 3) s->hh = p->kappa_a / (4.0 * PI * s->a * s->Deff);
    else s->hh = p->kappa_a / (2.0 * PI * s->Deff);
    s->rcut = p->rcut > 0.0 ? p->rcut : orc_rcut(d, p->bc, s->a, s->Deff, p->dt, p->kappa_a, p->eps_cut);
    s->p_uni = -expm1(-p->k_off * p->dt);
    s->key[0] = (uint32_t)p->seed;
    s->key[1] = (uint32_t)(p->seed >> 32) ^ p->replica;
    return s;
}

void orc_sim_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->sp); free(s->x); free(s->xm); free(s->dx); free(s->partner); free(s->born);
    free(s->xg); free(s->dg); free(s->xo);
    free(s->pairs); free(s->picks); free(s->matches); free(s->diss);
    free(s);
}

static int cmp_pair(const void *a, const void *b)
{
    const orc_pair *x = (const orc_pair *)a, *y = (const orc_pair *)b;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    if (x->j != y->j) return x->j < y->j ? -1 : 1;
    return 0;
}

static int cmp_pick_bj(const void *a, const void *b)
{
    const orc_pick *x = (const orc_pick *)a, *y = (const orc_pick *)b;
    if (x->j != y->j) return x->j < y->j ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    return 0;
}

/* The exact 2D functions serve pairs with R0 <= 1 + c sqrt(tau): there the
 * propagator's mass 1 - S_abs(R0) exceeds about erfc(c/2) and is resolved by
 * the quadrature.  Farther out every argument x = (R + R0 - 2)/(2 sqrt tau) of
 * the pair is >= c/2, where the order-12 small-time expansion (Sec. 4.2, eq.
 * smallTEabs) holds, and it is used.  c = 8.4 up to tau = 0.5; above, the
 * expansion's error at contact reaches 1e-6 only a little farther out, c = 9
 * (both measured against a numerical inversion of the Laplace-domain forms,
 * eqs. absPert, refPert, radPert). */
double orc_x2_switch(double tau) { return 1.0 + (tau <= 0.5 ? 8.4 : 9.0) * sqrt(tau); }

/* The propagator's distribution function is a ratio of masses of size
 * 1 - S_abs(R0), which the quadrature resolves down to about erfc(4.2) ~ 3e-9:
 * its switch stays at 1 + 8.4 sqrt(tau) for every tau. */
double orc_x2_prop_switch(double tau) { return 1.0 + 8.4 * sqrt(tau); }

static int use_x2(const orc_sim *s, double R0) { return s->p.dim == 2 && s->p.exact2d && R0 <= orc_x2_switch(s->tau); }
static int use_x2_prop(const orc_sim *s, double R0)
{
    return s->p.dim == 2 && s->p.exact2d && R0 <= orc_x2_prop_switch(s->tau);
}

static double pair_prob(const orc_sim *s, double R, double R0)
{
    if (R <= 1.0) return 1.0;
    if (s->p.dim == 3) return orc_penc3(R, R0, s->tau);
    return use_x2(s, R0) ? orc_penc2x(R, R0, s->tau) : orc_penc2(R, R0, s->tau, s->p.n_terms);
}

static double reac_prob(const orc_sim *s, double R, double R0)
{
    if (s->p.bc == ORC_BC_ABS) return 1.0;
    if (s->p.bc == ORC_BC_REF) return 0.0;
    if (s->p.dim == 3) return orc_preac3(R, R0, s->tau, s->hh);
    return use_x2(s, R0) ? orc_preac2x(R, R0, s->tau, s->hh) : orc_preac2(R, R0, s->tau, s->hh, s->p.n_terms);
}

/* R'' of a propagation: keyed rejection, or with the exact 2D functions
 * inversion with word 0 of the counter's attempt 0 */
static double propagate(const orc_sim *s, double R0, const uint32_t ctr[4], uint32_t *att, uint32_t *hits)
{
    if (use_x2_prop(s, R0)) {
        uint32_t w[4];
        uint32_t ct[4] = {ctr[0], ctr[1], ctr[2], ctr[3] & 0xFFu};
        orc_philox4x32_10(ct, s->key, w);
        *att = 1;
        return orc_sample_prop2x(R0, s->tau, orc_u01(w[0]));
    }
    return orc_sample_prop(s->p.dim, R0, s->tau, s->p.n_terms, ctr, s->key, att, hits);
}

/* post-move separation vector of (i, j) and the pre-step one, and their
 * scaled lengths (Sec. 2.1: r = r_B - r_A, eq. relCoo) */
static void separation(const orc_sim *s, uint32_t i, uint32_t j, double rv[3], double *R, double *R0)
{
    int d = s->p.dim;
    double r2 = 0.0, r02 = 0.0;
    for (int k = 0; k < 3; ++k) rv[k] = 0.0;
    for (int k = 0; k < d; ++k) {
        rv[k] = min_image(s->x[j * 3 + k] - s->x[i * 3 + k], s->p.box[k]);
        double r0 = rv[k] - (s->dx[j * 3 + k] - s->dx[i * 3 + k]);
        r2 += rv[k] * rv[k];
        r02 += r0 * r0;
    }
    *R = sqrt(r2) / s->a;
    *R0 = sqrt(r02) / s->a;
}

/* Direction of a propagated pair's new separation (Sec. 3, Details, second item
 * of the propagation): the angle Theta between the new separation and the
 * pre-step one r0v is drawn from J (G_ref - G_abs) given the new radius R''
 * (eqs. genericGF3D and genericGF), with u = U(word 0) of the counter
 * {i, j, step, ANG}.  In 3D the azimuth about r0v is uniform, 2 pi U(word 1),
 * measured in the frame b1, b2 orthogonal to r0v of Duff et al., "Building an
 * Orthonormal Basis, Revisited" (JCGT 2017); in 2D the side of the rotation is
 * the top bit of word 1 (set: clockwise).  e receives the unit direction and
 * *cth cos Theta.  A pre-step separation of length zero, or radii beyond any
 * encounter (the sampler's NaN), keep the direction ef of the free end point
 * (*cth = NaN). */
static void new_direction(const orc_sim *s, const double r0v[3], const double ef[3], double Rpp, double R0,
                          uint32_t i, uint32_t j, uint32_t stp, double e[3], double *cth)
{
    const int d = s->p.dim;
    double n0 = 0.0;
    for (int k = 0; k < d; ++k) n0 += r0v[k] * r0v[k];
    n0 = sqrt(n0);
    uint32_t ctr[4] = {i, j, stp, TAG_ANG}, w[4];
    orc_philox4x32_10(ctr, s->key, w);
    const double u = orc_u01(w[0]);
    double c = NAN;
    if (n0 > 0.0) c = d == 3 ? orc_sample_angle3(Rpp, R0, s->tau, u) : cos(orc_sample_angle2(Rpp, R0, s->tau, u));
    *cth = c;
    if (!(c == c)) {
        for (int k = 0; k < 3; ++k) e[k] = ef[k];
        return;
    }
    double n[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < d; ++k) n[k] = r0v[k] / n0;
    if (d == 3) {
        const double sg = n[2] >= 0.0 ? 1.0 : -1.0, a = -1.0 / (sg + n[2]), b = n[0] * n[1] * a;
        const double b1[3] = {1.0 + sg * n[0] * n[0] * a, sg * b, -sg * n[0]};
        const double b2[3] = {b, sg + n[1] * n[1] * a, -n[1]};
        const double sn = sqrt(fmax(0.0, 1.0 - c * c)), ph = 2.0 * PI * orc_u01(w[1]);
        const double cp = cos(ph), spp = sin(ph);
        for (int k = 0; k < 3; ++k) e[k] = c * n[k] + sn * (cp * b1[k] + spp * b2[k]);
    } else {
        const double sn = (w[1] >> 31 ? -1.0 : 1.0) * sqrt(fmax(0.0, 1.0 - c * c));
        e[0] = c * n[0] - sn * n[1];
        e[1] = sn * n[0] + c * n[1];
        e[2] = 0.0;
    }
}

void orc_sim_step(orc_sim *s)
{
    const int d = s->p.dim;
    const uint64_t n = s->cap;
    const uint32_t stp = (uint32_t)s->step;
    memset(s->st, 0, sizeof(s->st));
    s->n_pairs = s->n_picks = s->n_matches = s->n_diss = 0;
    memset(s->born, 0, n);

    /* Step 1: free Brownian displacement sqrt(2 D dt) N(0,1) for every
     * particle (Sec. 3, step 1), Box-Muller normals from one draw. */
    for (uint64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 3; ++k) s->dx[i * 3 + k] = 0.0;
        int sp = s->sp[i];
        if (sp > ORC_SP_C) continue;
        uint32_t ctr[4] = {(uint32_t)i, NOSLOT, stp, TAG_MOVE}, w[4];
        double u[4], z[4];
        draw(ctr, s->key, u, w);
        double r0 = sqrt(-2.0 * log(u[0])), t0 = 2.0 * PI * u[1];
        double r1 = sqrt(-2.0 * log(u[2])), t1 = 2.0 * PI * u[3];
        z[0] = r0 * cos(t0); z[1] = r0 * sin(t0); z[2] = r1 * cos(t1); z[3] = r1 * sin(t1);
        double sc = sqrt(2.0 * s->p.D[sp] * s->p.dt);
        for (int k = 0; k < d; ++k) {
            double dk = sc * z[k];
            double y = wrap_store(s, s->x[i * 3 + k] + dk, s->p.box[k]);
            if (s->given) {  /* its own move, kept for comparison; the step goes on from the caller's */
                s->xo[i * 3 + k] = y;
                s->dx[i * 3 + k] = s->dg[i * 3 + k];
                s->x[i * 3 + k] = s->xg[i * 3 + k];
            } else {
                s->dx[i * 3 + k] = dk;
                s->x[i * 3 + k] = y;
            }
        }
    }
    s->given = 0;
    memcpy(s->xm, s->x, n * 3 * sizeof(double));

    /* Steps 2 and 3: all A-B pairs within r_cut (Sec. 3, Details, cut-off),
     * found with a cell list of B particles. */
    int nc[3] = {1, 1, 1};
    for (int k = 0; k < d; ++k) {
        double m = floor(s->p.box[k] / s->rcut);
        nc[k] = m > 128.0 ? 128 : (int)m;
        if (nc[k] < 3) nc[k] = 1;
    }
    uint64_t ncell = (uint64_t)nc[0] * nc[1] * nc[2];
    int64_t *head = (int64_t *)malloc(ncell * sizeof(int64_t));
    int64_t *next = (int64_t *)malloc(n * sizeof(int64_t));
    for (uint64_t c = 0; c < ncell; ++c) head[c] = -1;
    int cidx[3];
#define CELL_OF(i, out)                                                                  \
    for (int k = 0; k < 3; ++k) {                                                        \
        int ci = 0;                                                                      \
        if (k < d && nc[k] > 1) {                                                        \
            ci = (int)floor(s->x[(i) * 3 + k] * nc[k] / s->p.box[k]);                    \
            if (ci < 0) ci = 0;                                                          \
            if (ci >= nc[k]) ci = nc[k] - 1;                                             \
        }                                                                                \
        out[k] = ci;                                                                     \
    }
    for (uint64_t j = 0; j < n; ++j) {
        if (s->sp[j] != ORC_SP_B) continue;
        CELL_OF(j, cidx);
        uint64_t c = ((uint64_t)cidx[2] * nc[1] + cidx[1]) * nc[0] + cidx[0];
        next[j] = head[c];
        head[c] = (int64_t)j;
    }
    const double rc2 = s->rcut * s->rcut;
    for (uint64_t i = 0; i < n; ++i) {
        if (s->sp[i] != ORC_SP_A) continue;
        CELL_OF(i, cidx);
        int lo[3], hi[3];
        for (int k = 0; k < 3; ++k) {
            lo[k] = nc[k] >= 3 ? -1 : 0;
            hi[k] = nc[k] >= 3 ? 1 : 0;
        }
        for (int oz = lo[2]; oz <= hi[2]; ++oz)
            for (int oy = lo[1]; oy <= hi[1]; ++oy)
                for (int ox = lo[0]; ox <= hi[0]; ++ox) {
                    int cx = (cidx[0] + ox + nc[0]) % nc[0];
                    int cy = (cidx[1] + oy + nc[1]) % nc[1];
                    int cz = (cidx[2] + oz + nc[2]) % nc[2];
                    uint64_t c = ((uint64_t)cz * nc[1] + cy) * nc[0] + cx;
                    for (int64_t j = head[c]; j >= 0; j = next[j]) {
                        double r2 = 0.0;
                        for (int k = 0; k < d; ++k) {
                            double dk = min_image(s->x[j * 3 + k] - s->x[i * 3 + k], s->p.box[k]);
                            r2 += dk * dk;
                        }
                        if (!(r2 < rc2)) continue;
                        s->pairs = (orc_pair *)grow(s->pairs, &s->c_pairs, s->n_pairs + 1, sizeof(orc_pair));
                        orc_pair *pr = &s->pairs[s->n_pairs++];
                        pr->i = (uint32_t)i;
                        pr->j = (uint32_t)j;
                    }
                }
    }
    free(head);
    free(next);
#undef CELL_OF
    qsort(s->pairs, s->n_pairs, sizeof(orc_pair), cmp_pair);
    s->st[ORC_ST_PAIRS] = s->n_pairs;

    /* Encounter probability for every pair (overlap: p = 1, step 2), and the
     * Bernoulli draw xi < p_enc (step 3). */
    for (uint64_t q = 0; q < s->n_pairs; ++q) {
        orc_pair *pr = &s->pairs[q];
        double rv[3], R, R0;
        separation(s, pr->i, pr->j, rv, &R, &R0);
        if (R0 < 1.0) {
            R0 = 1.0;
            s->st[ORC_ST_R0CLAMP]++;
        }
        pr->R = R;
        pr->R0 = R0;
        pr->p = pair_prob(s, R, R0);
        uint32_t ctr[4] = {pr->i, pr->j, stp, TAG_ENC}, w[4];
        orc_philox4x32_10(ctr, s->key, w);
        pr->draw = w[0];
        pr->cand = (R <= 1.0) || (orc_u01(w[0]) < pr->p);
        if (R <= 1.0) s->st[ORC_ST_OVERLAP]++;
        if (pr->cand) s->st[ORC_ST_CAND]++;
    }

    /* Several candidates (Sec. 3, Details): the A particle picks one with
     * probability p_enc / sum p_enc by the cumulative rule, candidates in
     * ascending slot order; then each B picked by several A's chooses among
     * them by the same rule. */
    for (uint64_t q = 0; q < s->n_pairs;) {
        uint64_t e = q;
        while (e < s->n_pairs && s->pairs[e].i == s->pairs[q].i) ++e;
        double T = 0.0;
        uint64_t m = 0;
        for (uint64_t t = q; t < e; ++t)
            if (s->pairs[t].cand) {
                T += s->pairs[t].p;
                ++m;
            }
        if (m > 0) {
            uint32_t ctr[4] = {s->pairs[q].i, NOSLOT, stp, TAG_SELA}, w[4];
            orc_philox4x32_10(ctr, s->key, w);
            double target = orc_u01(w[0]) * T, C = 0.0;
            uint64_t chosen = e;
            for (uint64_t t = q; t < e; ++t) {
                if (!s->pairs[t].cand) continue;
                C += s->pairs[t].p;
                chosen = t;
                if (target <= C) break;
            }
            s->picks = (orc_pick *)grow(s->picks, &s->c_picks, s->n_picks + 1, sizeof(orc_pick));
            orc_pick *pk = &s->picks[s->n_picks++];
            pk->i = s->pairs[chosen].i;
            pk->j = s->pairs[chosen].j;
            pk->p = s->pairs[chosen].p;
        }
        q = e;
    }
    s->st[ORC_ST_PICKS] = s->n_picks;
    qsort(s->picks, s->n_picks, sizeof(orc_pick), cmp_pick_bj);
    for (uint64_t q = 0; q < s->n_picks;) {
        uint64_t e = q;
        while (e < s->n_picks && s->picks[e].j == s->picks[q].j) ++e;
        double T = 0.0;
        for (uint64_t t = q; t < e; ++t) T += s->picks[t].p;
        uint32_t ctr[4] = {s->picks[q].j, NOSLOT, stp, TAG_SELB}, w[4];
        orc_philox4x32_10(ctr, s->key, w);
        double target = orc_u01(w[0]) * T, C = 0.0;
        uint64_t chosen = e - 1;
        for (uint64_t t = q; t < e; ++t) {
            C += s->picks[t].p;
            if (target <= C) {
                chosen = t;
                break;
            }
        }
        s->matches = (orc_match *)grow(s->matches, &s->c_matches, s->n_matches + 1, sizeof(orc_match));
        orc_match *mt = &s->matches[s->n_matches++];
        memset(mt, 0, sizeof(*mt));
        mt->i = s->picks[chosen].i;
        mt->j = s->picks[chosen].j;
        mt->cos_theta = NAN;
        q = e;
    }
    s->st[ORC_ST_MATCHES] = s->n_matches;

    /* Encountered pairs (steps 2a-2c): absorbing pairs react; reflecting and
     * radiation pairs get a new separation from the radial propagator
     * w_d r^{d-1}(g_ref - g_abs) (eq. passage_prob), and radiation pairs then
     * react with probability p_reac (eq. psurv_radII).  The centre
     * R = (D_B r_A + D_A r_B)/D_eff (eq. Rcoo) keeps its free end point. */
    const double fA = s->p.D[0] / s->Deff, fB = s->p.D[1] / s->Deff;
    for (uint64_t q = 0; q < s->n_matches; ++q) {
        orc_match *mt = &s->matches[q];
        uint32_t i = mt->i, j = mt->j;
        double rv[3], R, R0;
        separation(s, i, j, rv, &R, &R0);
        if (R0 < 1.0) R0 = 1.0;
        int react;
        if (s->p.bc == ORC_BC_ABS) {
            react = 1;
            mt->Rpp = R;
            mt->preac = 1.0;
        } else {
            uint32_t ctr[4] = {i, j, stp, TAG_PROP}, att = 0, hits = 0;
            double Rpp = propagate(s, R0, ctr, &att, &hits);
            s->st[ORC_ST_ATTEMPTS] += att;
            s->st[ORC_ST_BOUND] += hits;
            mt->attempts = att;
            mt->Rpp = Rpp;
            mt->preac = reac_prob(s, Rpp, R0);
            uint32_t c2[4] = {i, j, stp, TAG_REAC}, w[4];
            orc_philox4x32_10(c2, s->key, w);
            mt->draw = w[0];
            react = orc_u01(w[0]) < mt->preac;
            if (!react) {
                /* the free end point's direction, and unless the step keeps it, the
                 * drawn one (Sec. 3, Details) */
                double rn = 0.0, ef[3] = {0.0, 0.0, 0.0}, e[3], r0v[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k < d; ++k) rn += rv[k] * rv[k];
                rn = sqrt(rn);
                for (int k = 0; k < d; ++k) ef[k] = rn > 0.0 ? rv[k] / rn : (k == d - 1 ? 1.0 : 0.0);
                if (s->p.keep_dir) {
                    for (int k = 0; k < 3; ++k) e[k] = ef[k];
                } else {
                    for (int k = 0; k < d; ++k) r0v[k] = rv[k] - (s->dx[j * 3 + k] - s->dx[i * 3 + k]);
                    new_direction(s, r0v, ef, Rpp, R0, i, j, stp, e, &mt->cos_theta);
                }
                for (int k = 0; k < d; ++k) {
                    double cen = s->x[i * 3 + k] + fA * rv[k];
                    double xi = cen - fA * s->a * Rpp * e[k];
                    double xj = cen + fB * s->a * Rpp * e[k];
                    s->x[i * 3 + k] = wrap_store(s, xi, s->p.box[k]);
                    s->x[j * 3 + k] = wrap_store(s, xj, s->p.box[k]);
                }
            }
        }
        mt->reacted = react;
        if (react) {
            s->st[ORC_ST_REACT]++;
            for (int k = 0; k < d; ++k) s->x[i * 3 + k] = wrap_store(s, s->x[i * 3 + k] + fA * rv[k], s->p.box[k]);
            s->sp[i] = ORC_SP_C;
            s->born[i] = 1;
            for (int k = 0; k < 3; ++k) s->x[j * 3 + k] = 0.0;
            if (s->p.k_off > 0.0) {
                s->sp[j] = ORC_SP_RESERVED;
                s->partner[i] = j;
            } else {
                s->sp[j] = ORC_SP_FREE;
                s->partner[i] = NOSLOT;
            }
        }
    }

    /* Step 4: C -> A + B as a Poisson decay, p = 1 - e^{-k_off dt}
     * (eq. rad_prob); the products start at contact, get a separation from
     * the propagator with r0 = a, and recombine with probability p_reac
     * (Sec. 2.2.5). */
    if (s->p.k_off > 0.0) {
        for (uint64_t c = 0; c < n; ++c) {
            if (s->sp[c] != ORC_SP_C || s->born[c]) continue;
            uint32_t ctr[4] = {(uint32_t)c, NOSLOT, stp, TAG_UNI}, w[4];
            orc_philox4x32_10(ctr, s->key, w);
            if (!(orc_u01(w[0]) < s->p_uni)) continue;
            s->diss = (orc_diss *)grow(s->diss, &s->c_diss, s->n_diss + 1, sizeof(orc_diss));
            orc_diss *ds = &s->diss[s->n_diss++];
            memset(ds, 0, sizeof(*ds));
            ds->c = (uint32_t)c;
            ds->j = s->partner[c];
            ds->decayed = 1;
            s->st[ORC_ST_DECAY]++;
            uint32_t cp[4] = {(uint32_t)c, NOSLOT, stp, TAG_DPROP}, att = 0, hits = 0;
            double Rpp = propagate(s, 1.0, cp, &att, &hits);
            s->st[ORC_ST_ATTEMPTS] += att;
            s->st[ORC_ST_BOUND] += hits;
            ds->attempts = att;
            ds->Rpp = Rpp;
            ds->preac = reac_prob(s, Rpp, 1.0);
            uint32_t cg[4] = {(uint32_t)c, NOSLOT, stp, TAG_GEM};
            orc_philox4x32_10(cg, s->key, w);
            ds->draw = w[0];
            if (orc_u01(w[0]) < ds->preac) {
                ds->recombined = 1;
                s->st[ORC_ST_GEMINATE]++;
                continue;
            }
            uint32_t cd[4] = {(uint32_t)c, NOSLOT, stp, TAG_DIR};
            double u[4];
            draw(cd, s->key, u, w);
            double e[3] = {0.0, 0.0, 0.0};
            if (d == 3) {
                double z = 2.0 * u[0] - 1.0, ph = 2.0 * PI * u[1], rho = sqrt(1.0 - z * z);
                e[0] = rho * cos(ph); e[1] = rho * sin(ph); e[2] = z;
            } else {
                double ph = 2.0 * PI * u[0];
                e[0] = cos(ph); e[1] = sin(ph);
            }
            uint32_t j = s->partner[c];
            for (int k = 0; k < d; ++k) {
                double X = s->x[c * 3 + k];
                s->x[c * 3 + k] = wrap_store(s, X - fA * s->a * Rpp * e[k], s->p.box[k]);
                s->x[j * 3 + k] = wrap_store(s, X + fB * s->a * Rpp * e[k], s->p.box[k]);
            }
            s->sp[c] = ORC_SP_A;
            s->sp[j] = ORC_SP_B;
            s->partner[c] = NOSLOT;
        }
    }

    /* Step 5 */
    s->step++;
}

uint64_t orc_sim_cap(const orc_sim *s) { return s->cap; }
uint64_t orc_sim_stepno(const orc_sim *s) { return s->step; }

void orc_sim_derived(const orc_sim *s, double out[6])
{
    out[0] = s->Deff; out[1] = s->tau; out[2] = s->hh; out[3] = s->rcut; out[4] = s->a; out[5] = s->p_uni;
}

void orc_sim_state(const orc_sim *s, int32_t *species, double *pos, uint32_t *partner)
{
    int d = s->p.dim;
    for (uint64_t i = 0; i < s->cap; ++i) {
        if (species) species[i] = s->sp[i];
        if (partner) partner[i] = s->partner[i];
        if (pos)
            for (int k = 0; k < d; ++k) pos[i * d + k] = s->x[i * 3 + k];
    }
}

/* Stage parity: the next step uses these post-move positions and displacements (n * dim
 * each, by slot; entries of FREE and RESERVED slots are ignored) in place of its own move,
 * and runs every later stage on them; its own move is kept for orc_sim_moved_own. */
void orc_sim_set_moved(orc_sim *s, const double *pos, const double *disp)
{
    const int d = s->p.dim;
    const uint64_t n = s->cap;
    if (!s->xg) {
        s->xg = (double *)calloc(n * 3, sizeof(double));
        s->dg = (double *)calloc(n * 3, sizeof(double));
        s->xo = (double *)calloc(n * 3, sizeof(double));
    }
    for (uint64_t i = 0; i < n; ++i)
        for (int k = 0; k < d; ++k) {
            s->xg[i * 3 + k] = pos[i * d + k];
            s->dg[i * 3 + k] = disp[i * d + k];
        }
    s->given = 1;
}

/* The oracle's own post-move positions of the last step taken after orc_sim_set_moved. */
void orc_sim_moved_own(const orc_sim *s, double *pos)
{
    int d = s->p.dim;
    for (uint64_t i = 0; i < s->cap; ++i)
        for (int k = 0; k < d; ++k) pos[i * d + k] = s->xo ? s->xo[i * 3 + k] : NAN;
}

void orc_sim_moved(const orc_sim *s, double *pos)
{
    int d = s->p.dim;
    for (uint64_t i = 0; i < s->cap; ++i)
        for (int k = 0; k < d; ++k) pos[i * d + k] = s->xm[i * 3 + k];
}

void orc_sim_stats(const orc_sim *s, uint64_t out[ORC_ST_N]) { memcpy(out, s->st, sizeof(s->st)); }
uint64_t orc_sim_n_pairs(const orc_sim *s) { return s->n_pairs; }
uint64_t orc_sim_n_picks(const orc_sim *s) { return s->n_picks; }
uint64_t orc_sim_n_matches(const orc_sim *s) { return s->n_matches; }
uint64_t orc_sim_n_diss(const orc_sim *s) { return s->n_diss; }
void orc_sim_pairs(const orc_sim *s, orc_pair *out) { memcpy(out, s->pairs, s->n_pairs * sizeof(orc_pair)); }
void orc_sim_picks(const orc_sim *s, orc_pick *out) { memcpy(out, s->picks, s->n_picks * sizeof(orc_pick)); }
void orc_sim_matches(const orc_sim *s, orc_match *out) { memcpy(out, s->matches, s->n_matches * sizeof(orc_match)); }
void orc_sim_diss(const orc_sim *s, orc_diss *out) { memcpy(out, s->diss, s->n_diss * sizeof(orc_diss)); }

/* ------------------------------------------------------------------------ */
/* First-passage time by bisection (Appendix).  A pair whose separation went */
/* from x_i to x_f over one step of tau = D_eff dt / a^2, with at least one  */
/* encounter, has its first contact time located by halving the interval:   */
/* the separation at the midpoint is drawn from the Brownian bridge (eq.     */
/* midPGauss, per coordinate mean (x_a + x_b)/2 and variance tau_h, the      */
/* dimensionless half-interval), and p_enc of each half decides where the    */
/* first encounter lies.  Reading: both the midpoint and the choice are      */
/* conditioned on the encounter known to lie in the interval.  Given x_m the */
/* halves are independent, so that encounter has probability                 */
/* q = 1 - (1 - p1)(1 - p2): the midpoint is drawn from the bridge times q   */
/* (a bridge proposal accepted with probability q), and the first half is    */
/* chosen with probability p1 / q.  The located interval is then distributed */
/* as the first-passage time given the end points and the encounter.        */
/* Lengths are in units of a (contact at |x| = 1).  dim = 1 is the half line */
/* x > 1 with eq. bayes1D, p_enc = e^{-(x-1)(x0-1)/tau}; dim = 2 and 3 use    */
/* the radial encounter probabilities of Sec. 2.2.4 (3D: the closed form,   */
/* 2D: the expansion of order n_terms).                                      */
/* Draws per attempt k at level l: {c0, l, step, FPT | k << 8} gives the     */
/* normals (Box-Muller on words 0, 1 and 2, 3: z0 = r0 cos, z1 = r0 sin,     */
/* z2 = r1 cos), {c0, l, step, FPTU | k << 8} the uniforms (word 0 accepts,  */
/* word 1 chooses the half).  A level whose MAX_ATTEMPTS proposals are all   */
/* rejected (an interval whose encounter probability is far below their     */
/* inverse) ends the refinement: the interval reached is returned at the     */
/* requested resolution (its lower end) and bit 31 of *attempts is set.      */
/* ------------------------------------------------------------------------ */
static double fp_penc(int dim, double R, double R0, double tau, int n_terms)
{
    if (R <= 1.0 || R0 <= 1.0) return 1.0;
    if (dim == 1) return exp(-(R - 1.0) * (R0 - 1.0) / tau);
    if (dim == 2) return orc_penc2(R, R0, tau, n_terms);
    return orc_penc3(R, R0, tau);
}

static double fp_norm(int dim, const double *x)
{
    if (dim == 1) return x[0];
    double s = 0.0;
    for (int k = 0; k < dim; ++k) s += x[k] * x[k];
    return sqrt(s);
}

uint64_t orc_first_passage(int dim, const double *xi, const double *xf, double tau, int levels, int n_terms,
                           uint32_t c0, uint32_t step, const uint32_t key[2], uint32_t *attempts)
{
    double xa[3] = {0, 0, 0}, xb[3] = {0, 0, 0}, xm[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) {
        xa[k] = xi[k];
        xb[k] = xf[k];
    }
    uint64_t lo = 0;  /* the interval is [lo, lo + 1) in units of dt / 2^level */
    uint32_t att = 0;
    for (int l = 0; l < levels; ++l) {
        double th = tau / (double)(2ull << l);  /* the half-interval */
        double sd = sqrt(th), ra = fp_norm(dim, xa), rb = fp_norm(dim, xb);
        double p1 = 1.0, q = 1.0;
        double V = 0.0;
        int accepted = 0;
        for (uint32_t k = 0; k < MAX_ATTEMPTS; ++k) {
            uint32_t cz[4] = {c0, (uint32_t)l, step, TAG_FPT | (k << 8)}, cu[4] = {c0, (uint32_t)l, step, TAG_FPTU | (k << 8)};
            double u[4], v[4], z[3];
            uint32_t w[4];
            draw(cz, key, u, w);
            double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
            z[0] = r0 * cos(2.0 * PI * u[1]);
            z[1] = r0 * sin(2.0 * PI * u[1]);
            z[2] = r1 * cos(2.0 * PI * u[3]);
            for (int d = 0; d < dim; ++d) xm[d] = 0.5 * (xa[d] + xb[d]) + sd * z[d];
            double rm = fp_norm(dim, xm);
            p1 = fp_penc(dim, rm, ra, th, n_terms);
            double p2 = fp_penc(dim, rb, rm, th, n_terms);
            q = 1.0 - (1.0 - p1) * (1.0 - p2);
            draw(cu, key, v, w);
            ++att;
            V = v[1];
            if (v[0] < q) {
                accepted = 1;
                break;
            }
        }
        if (!accepted) {  /* exhausted: keep the interval reached */
            lo <<= (levels - l);
            att |= 0x80000000u;
            break;
        }
        lo *= 2;
        if (V * q < p1) {  /* first half: the end point becomes the midpoint */
            for (int d = 0; d < dim; ++d) xb[d] = xm[d];
        } else {           /* second half: the start point becomes the midpoint */
            for (int d = 0; d < dim; ++d) xa[d] = xm[d];
            lo += 1;
        }
    }
    if (attempts) *attempts = att;
    return lo;
}

/* ------------------------------------------------------------------------ */
/* Angular propagator in 3D (Sec. 3, Details: the angle between the pair's   */
/* separations before and after the step is drawn from J(G_ref - G_abs),    */
/* J = 2 pi sin(Theta) r^2, given the radius already drawn).                */
/*                                                                          */
/* With eq. genericGF3D for h -> 0 (reflecting) and h -> infinity           */
/* (absorbing), units a = 1 and D_eff = 1:                                   */
/*   G_ref - G_abs = sum_n (2n+1) P_n(cos Theta) w_n / (4 pi sqrt(R R0)),    */
/*   w_n = int_0^inf e^{-tau x^2} [F^r(R,x) F^r(R0,x) - F^a(R,x) F^a(R0,x)] x dx,*/
/* F^{r,a} the functions F_{n+1/2} of that equation.  Writing F as          */
/* [J(Rx) A - Y(Rx) B] / sqrt(A^2 + B^2) with A = (2h+1) Y(x) - 2x Y'(x),    */
/* B = (2h+1) J(x) - 2x J'(x) and C'_nu = C_{nu-1} - (nu/x) C_nu:           */
/*   reflecting: A = (2n+2) Y_nu(x) - 2x Y_{nu-1}(x), B likewise with J;    */
/*   absorbing (divide by 2h+1, h -> inf): A = Y_nu(x), B = J_nu(x).        */
/* Integrating over the sphere, the Legendre orthogonality leaves w_0:      */
/*   w_0 = 4 pi sqrt(R R0) (g_ref - g_abs)(R | R0), and the density of       */
/* c = cos Theta given R is sum_n (2n+1) P_n(c) w_n / (2 w_0), whose         */
/* integral from -1 (int P_n = (P_{n+1} - P_{n-1}) / (2n+1), n >= 1) is      */
/*   F(c) = [1 + c + sum_{n>=1} (w_n / w_0)(P_{n+1}(c) - P_{n-1}(c))] / 2.   */
/* The draw is the root of F(c) = u, located by bisection.                  */
/*                                                                          */
/* Bessel functions of half-integer order (Sec. 4.1, eq. 3termBessel):      */
/* J by the downward recurrence from a start above both the highest order   */
/* and the turning point (Miller's method), normalised to the elementary    */
/* J_{1/2} and J_{-1/2}; Y by the upward recurrence from Y_{-1/2} and        */
/* Y_{1/2}.  The integral over x: 16-point Gauss-Legendre panels of equal   */
/* width, at most min(1, 2 pi / f) with f = R + R0 - 1 (the fastest          */
/* oscillation of the integrand is at R + R0 - 2), over [0, sqrt(50/tau)].  */
/* Terms n = 0 .. N, N = min(160, 8 + ceil(sqrt(45 R R0 / tau))): the       */
/* coefficients fall like e^{-n(n+1) tau / (R R0)} (angular diffusion at    */
/* radius about sqrt(R R0)).  A node stops adding orders once |Y_nu(x)|      */
/* exceeds 2^500: there the products are below 1e-220 (and A^2 + B^2 stays  */
/* finite).                                                                 */
/* kind 1 replaces the bracket by J_nu(Rx) J_nu(R0x) (the free-space terms,   */
/* a check of the Bessel functions and the rule against Weber's integral)   */
/* and takes f = R + R0 + 1.                                                */
/* ------------------------------------------------------------------------ */
#define ANG_NCAP 160

int orc_angle3_terms(double R, double R0, double tau)
{
    int n = 8 + (int)ceil(sqrt(45.0 * R * R0 / tau));
    return n < ANG_NCAP ? n : ANG_NCAP;
}

/* J[k] = J_{k-1/2}(z), Y[k] = Y_{k-1/2}(z), k = 0 .. kmax (z > 0). */
void orc_bessel_half(int kmax, double z, double *J, double *Y)
{
    double zc = ceil(z);
    int m = (kmax > (int)zc + (int)ceil(12.0 * cbrt(z)) ? kmax : (int)zc + (int)ceil(12.0 * cbrt(z))) + 20;
    double *t = (double *)calloc((size_t)m + 2, sizeof(double));
    t[m + 1] = 0.0;
    t[m] = 1.0;
    for (int k = m; k >= 1; --k) {  /* C_{nu-1} = (2 nu / z) C_nu - C_{nu+1}, nu = k - 1/2 */
        t[k - 1] = (2.0 * k - 1.0) / z * t[k] - t[k + 1];
        if (fabs(t[k - 1]) > 1e250)
            for (int j = k - 1; j <= m + 1; ++j) t[j] *= 1e-250;
    }
    double s = sqrt(2.0 / (PI * z)), sz = sin(z), cz = cos(z);
    double M = fmax(fabs(t[0]), fabs(t[1])), a0 = t[0] / M, a1 = t[1] / M;
    double lam = s * (sz * a1 + cz * a0) / (a1 * a1 + a0 * a0) / M;
    for (int k = 0; k <= kmax; ++k) J[k] = lam * t[k];
    free(t);
    Y[0] = s * sz;
    if (kmax >= 1) Y[1] = -s * cz;
    for (int k = 1; k < kmax; ++k) Y[k + 1] = (2.0 * k - 1.0) / z * Y[k] - Y[k - 1];
}

void orc_angle3_coef(int kind, double R, double R0, double tau, int N, double *w)
{
    gl_init();
    double X = sqrt(50.0 / tau), f = R + R0 + (kind == 1 ? 1.0 : -1.0);
    double hmax = fmin(1.0, 2.0 * PI / f);
    int P = (int)ceil(X / hmax);
    double h = X / P;
    double *Jx = (double *)malloc(sizeof(double) * (size_t)(N + 2) * 6);
    double *Yx = Jx + (N + 2), *Jr = Yx + (N + 2), *Yr = Jr + (N + 2), *Jq = Yr + (N + 2), *Yq = Jq + (N + 2);
    for (int n = 0; n <= N; ++n) w[n] = 0.0;
    for (int p = 0; p < P; ++p) {
        for (int i = 0; i < GLN; ++i) {
            double x = h * (p + 0.5 + 0.5 * gl_x[i]);
            double g = 0.5 * h * gl_w[i] * exp(-tau * x * x) * x;
            orc_bessel_half(N + 1, x, Jx, Yx);
            orc_bessel_half(N + 1, R * x, Jr, Yr);
            orc_bessel_half(N + 1, R0 * x, Jq, Yq);
            for (int n = 0; n <= N; ++n) {
                int k = n + 1;  /* nu = n + 1/2 */
                if (kind == 1) {
                    w[n] += g * Jr[k] * Jq[k];
                    continue;
                }
                if (fabs(Yx[k]) > 0x1p500) break;
                double Ar = (2.0 * n + 2.0) * Yx[k] - 2.0 * x * Yx[k - 1];
                double Br = (2.0 * n + 2.0) * Jx[k] - 2.0 * x * Jx[k - 1];
                double Aa = Yx[k], Ba = Jx[k];
                double nr = sqrt(Ar * Ar + Br * Br), na = sqrt(Aa * Aa + Ba * Ba);
                double frR = (Jr[k] * Ar - Yr[k] * Br) / nr, frQ = (Jq[k] * Ar - Yq[k] * Br) / nr;
                double faR = (Jr[k] * Aa - Yr[k] * Ba) / na, faQ = (Jq[k] * Aa - Yq[k] * Ba) / na;
                w[n] += g * (frR * frQ - faR * faQ);
            }
        }
    }
    free(Jx);
}

double orc_angle3_cdf(const double *w, int N, double c)
{
    double s = 1.0 + c, pm = 1.0, p = c;  /* P_{n-1}, P_n at n = 1 */
    for (int n = 1; n <= N; ++n) {
        double pn1 = ((2.0 * n + 1.0) * c * p - n * pm) / (n + 1.0);
        s += w[n] / w[0] * (pn1 - pm);
        pm = p;
        p = pn1;
    }
    return 0.5 * s;
}

double orc_sample_angle3(double R, double R0, double tau, double u)
{
    if (!(R + R0 - 2.0 <= 40.0 * sqrt(tau))) return NAN;  /* beyond any encounter (e^{-400}), or not a number */
    R = fmax(R, 1.0);  /* a separation below contact is taken at contact */
    R0 = fmax(R0, 1.0);
    int N = orc_angle3_terms(R, R0, tau);
    double *w = (double *)malloc(sizeof(double) * (size_t)(N + 1));
    orc_angle3_coef(0, R, R0, tau, N, w);
    double lo = -1.0, hi = 1.0;
    for (int it = 0; it < 200 && hi - lo > 4e-16; ++it) {
        double mid = 0.5 * (lo + hi);
        if (orc_angle3_cdf(w, N, mid) < u) lo = mid;
        else hi = mid;
    }
    free(w);
    return 0.5 * (lo + hi);
}

/* ------------------------------------------------------------------------ */
/* Angular propagator in 2D (Sec. 3, Details, with J = r; eq. genericGF).    */
/*                                                                          */
/* With h -> 0 (reflecting) and h -> infinity (absorbing), units a = 1 and  */
/* D_eff = 1:                                                               */
/*   G_ref - G_abs = [w_0 + 2 sum_{n>=1} w_n cos(n theta)] / (2 pi),          */
/*   w_n = int_0^inf e^{-tau x^2} [C^r_n(R,x) C^r_n(R0,x) - C^a_n C^a_n] x dx,*/
/* (C_{-n} C_{-n} = C_n C_n), C_n = [J_n(Rx) A - Y_n(Rx) B] / sqrt(A^2+B^2)  */
/* from eq. fRad with x C'_n = x C_{n-1} - n C_n:                           */
/*   reflecting: A = x Y_{n-1}(x) - n Y_n(x), B likewise with J;            */
/*   absorbing (divide by -h, h -> inf): A = Y_n(x), B = J_n(x).            */
/* The angular integral leaves w_0 = 2 pi (g_ref - g_abs)(R | R0) (radial    */
/* functions of the exact 2D section above).  |theta| in [0, pi] given R    */
/* has the distribution function                                            */
/*   F(t) = [w_0 t + 2 sum_{n>=1} w_n sin(n t) / n] / (pi w_0),               */
/* and the draw is its root at u; the side (sign of theta) is the caller's. */
/*                                                                          */
/* Bessel functions of integer order (eq. 3termBessel): J by Miller's       */
/* downward recurrence normalised to the C library's j0, j1; Y upward from  */
/* its y0, y1.  The x integral: 32 Gauss-Legendre panels of ratio 2 on      */
/* [2^-32, 1] (Y_0 has a logarithm at x = 0), then panels of equal width at */
/* most min(1, 2 pi / (R + R0 - 1)) up to sqrt(50/tau).  Terms and order    */
/* cut-off as in 3D.  kind 1 gives the free-space terms J_n(Rx) J_n(R0x).    */
/* ------------------------------------------------------------------------ */

/* J[k] = J_{k-1}(z), Y[k] = Y_{k-1}(z), k = 0 .. kmax (z > 0): index 0 is order -1. */
void orc_bessel_int(int kmax, double z, double *J, double *Y)
{
    int nmax = kmax - 1;  /* highest order */
    double zc = ceil(z);
    int m = (nmax > (int)zc + (int)ceil(12.0 * cbrt(z)) ? nmax : (int)zc + (int)ceil(12.0 * cbrt(z))) + 20;
    double *t = (double *)calloc((size_t)m + 2, sizeof(double));  /* t[n] ~ J_n, n = 0 .. m + 1 */
    t[m + 1] = 0.0;
    t[m] = 1.0;
    for (int n = m; n >= 1; --n) {  /* J_{n-1} = (2n / z) J_n - J_{n+1} */
        t[n - 1] = 2.0 * n / z * t[n] - t[n + 1];
        if (fabs(t[n - 1]) > 1e250)
            for (int j = n - 1; j <= m + 1; ++j) t[j] *= 1e-250;
    }
    double a0 = j0(z), a1 = j1(z);
    double M = fmax(fabs(t[0]), fabs(t[1])), b0 = t[0] / M, b1 = t[1] / M;
    double lam = (a0 * b0 + a1 * b1) / (b0 * b0 + b1 * b1) / M;
    for (int n = 0; n <= nmax; ++n) J[n + 1] = lam * t[n];
    J[0] = -J[2];
    free(t);
    Y[1] = y0(z);
    if (kmax >= 2) Y[2] = y1(z);
    Y[0] = -y1(z);
    for (int n = 1; n < nmax; ++n) Y[n + 2] = 2.0 * n / z * Y[n + 1] - Y[n];
}

void orc_angle2_coef(int kind, double R, double R0, double tau, int N, double *w)
{
    gl_init();
    double X = sqrt(50.0 / tau), x1 = X < 1.0 ? X : 1.0, f = R + R0 + (kind == 1 ? 1.0 : -1.0);
    double hmax = fmin(1.0, 2.0 * PI / f);
    int ngeo = 32, nuni = X > x1 ? (int)ceil((X - x1) / hmax) : 0;
    double huni = nuni > 0 ? (X - x1) / nuni : 0.0;
    double *Jx = (double *)malloc(sizeof(double) * (size_t)(N + 2) * 6);
    double *Yx = Jx + (N + 2), *Jr = Yx + (N + 2), *Yr = Jr + (N + 2), *Jq = Yr + (N + 2), *Yq = Jq + (N + 2);
    for (int n = 0; n <= N; ++n) w[n] = 0.0;
    for (int p = 0; p < ngeo + nuni; ++p) {
        double lo, hi;
        if (p < ngeo) {
            lo = ldexp(x1, p - ngeo);
            hi = 2.0 * lo;
        } else {
            lo = x1 + (p - ngeo) * huni;
            hi = lo + huni;
        }
        double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
        for (int i = 0; i < GLN; ++i) {
            double x = c + h * gl_x[i];
            double g = h * gl_w[i] * exp(-tau * x * x) * x;
            orc_bessel_int(N + 1, x, Jx, Yx);
            orc_bessel_int(N + 1, R * x, Jr, Yr);
            orc_bessel_int(N + 1, R0 * x, Jq, Yq);
            for (int n = 0; n <= N; ++n) {
                int k = n + 1;  /* order n */
                if (kind == 1) {
                    w[n] += g * Jr[k] * Jq[k];
                    continue;
                }
                if (fabs(Yx[k]) > 0x1p500) break;
                double Ar = x * Yx[k - 1] - n * Yx[k], Br = x * Jx[k - 1] - n * Jx[k];
                double Aa = Yx[k], Ba = Jx[k];
                double nr = sqrt(Ar * Ar + Br * Br), na = sqrt(Aa * Aa + Ba * Ba);
                double crR = (Jr[k] * Ar - Yr[k] * Br) / nr, crQ = (Jq[k] * Ar - Yq[k] * Br) / nr;
                double caR = (Jr[k] * Aa - Yr[k] * Ba) / na, caQ = (Jq[k] * Aa - Yq[k] * Ba) / na;
                w[n] += g * (crR * crQ - caR * caQ);
            }
        }
    }
    free(Jx);
}

double orc_angle2_cdf(const double *w, int N, double t)
{
    double s = w[0] * t;
    for (int n = 1; n <= N; ++n) s += 2.0 * w[n] * sin(n * t) / n;
    return s / (PI * w[0]);
}

double orc_sample_angle2(double R, double R0, double tau, double u)
{
    if (!(R + R0 - 2.0 <= 40.0 * sqrt(tau))) return NAN;  /* beyond any encounter (e^{-400}), or not a number */
    R = fmax(R, 1.0);
    R0 = fmax(R0, 1.0);
    int N = orc_angle3_terms(R, R0, tau);
    double *w = (double *)malloc(sizeof(double) * (size_t)(N + 1));
    orc_angle2_coef(0, R, R0, tau, N, w);
    double lo = 0.0, hi = PI;
    for (int it = 0; it < 200 && hi - lo > 8e-16; ++it) {
        double mid = 0.5 * (lo + hi);
        if (orc_angle2_cdf(w, N, mid) < u) lo = mid;
        else hi = mid;
    }
    free(w);
    return 0.5 * (lo + hi);
}
