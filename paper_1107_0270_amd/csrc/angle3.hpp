// Angular propagator in 3D: the angle Theta between a pair's separations before
// and after a non-reactive encounter, drawn from J (G_ref - G_abs) given the new
// radius (Sec. 3, Details, second item of the propagation; J = 2 pi sin(Theta) r^2).
//
// In units a = 1, D_eff = 1 (eq. genericGF3D with h -> 0 and h -> infinity),
//   G_ref - G_abs = sum_n (2n+1) P_n(cos Theta) w_n / (4 pi sqrt(R R0)),
//   w_n = int_0^inf e^{-tau x^2} [F^r(R,x) F^r(R0,x) - F^a(R,x) F^a(R0,x)] x dx,
// F = [J_nu(Rx) A - Y_nu(Rx) B] / sqrt(A^2 + B^2), nu = n + 1/2, with
//   reflecting: A = (2n+2) Y_nu(x) - 2x Y_{nu-1}(x), B = (2n+2) J_nu(x) - 2x J_{nu-1}(x),
//   absorbing:  A = Y_nu(x), B = J_nu(x)
// (the boundary terms of that equation with C'_nu = C_{nu-1} - (nu/x) C_nu).  The
// distribution function of c = cos Theta given R is
//   F(c) = [1 + c + sum_{n>=1} (w_n / w_0)(P_{n+1}(c) - P_{n-1}(c))] / 2,
// and the draw is its root at the caller's uniform u.
//
// Evaluation:
//   - terms n = 0 .. N, N = min(ANG_NCAP, 8 + ceil(sqrt(45 R R0 / tau))) (the
//     coefficients fall like e^{-n(n+1) tau / (R R0)});
//   - x integral: 16-point Gauss-Legendre panels of equal width, at most
//     min(1, 2 pi / (R + R0 - 1)), over [0, sqrt(50 / tau)];
//   - Bessel functions of half-integer order (eq. 3termBessel): J by the downward
//     recurrence from above both N and the turning point (start below), normalised to the
//     elementary J_{1/2}, J_{-1/2}; Y by the upward recurrence from Y_{-1/2}, Y_{1/2};
//     a node stops adding orders once |Y_nu(x)| exceeds 2^500 (its products are
//     then below 1e-220, and A^2 + B^2 stays finite);
//   - pairs with R + R0 - 2 > 40 sqrt(tau) (beyond any encounter) or not a number give NaN;
//   - inversion: the root of F(c) = u by a search over [-1, 1].
// This file holds the series' pieces (terms, Bessel recurrences, F); the kernels that
// lay a pair's nodes over a workgroup and draw the angle are in angle_wg.hpp.
#pragma once

#include "kernels.hpp"

namespace gfbd {

constexpr int ANG_NCAP = 160;

struct GL16 {
    double x[16], w[16];
};

__device__ __forceinline__ int ang_terms(double R, double R0, double tau)
{
    const int n = 8 + (int)ceil(sqrt(45.0 * R * R0 / tau));
    return n < ANG_NCAP ? n : ANG_NCAP;
}

__device__ __forceinline__ double wave_allsum(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// J_{k-1/2}(z) for k = 0 .. kmax, for three arguments at once (the downward recurrence
// C_{nu-1} = (2 nu / z) C_nu - C_{nu+1}, nu = k - 1/2, from k = m down): t[j][k] times lam[j].
__device__ __forceinline__ void ang_miller3(int kmax, const double z[3], double (*t)[ANG_NCAP + 2], double lam[3])
{
    // start: J_m / |Y_m| at m = z + t falls like e^{-0.94 t^{3/2} / sqrt(z)} (beyond the turning
    // point), below 1e-18 for t >= 8 z^{1/3}; and at least 8 orders above kmax
    const double zm = fmax(z[0], fmax(z[1], z[2]));
    const int zc = (int)ceil(zm + 8.0 * cbrt(zm));
    const int m = (kmax > zc ? kmax : zc) + 8;
    double a[3], b[3], inv[3];  // a = C_{k}, b = C_{k+1}
    for (int j = 0; j < 3; ++j) {
        a[j] = 1.0;
        b[j] = 0.0;
        inv[j] = 1.0 / z[j];
    }
    if (m <= kmax)
        for (int j = 0; j < 3; ++j) t[j][m] = a[j];
    for (int k = m; k >= 1; --k) {
        for (int j = 0; j < 3; ++j) {
            const double c = (2.0 * k - 1.0) * inv[j] * a[j] - b[j];
            b[j] = a[j];
            a[j] = c;
            if (fabs(c) > 1e250) {  // rescale, including what is already stored
                a[j] *= 1e-250;
                b[j] *= 1e-250;
                for (int q = k; q <= kmax; ++q) t[j][q] *= 1e-250;
            }
            if (k - 1 <= kmax) t[j][k - 1] = a[j];
        }
    }
    for (int j = 0; j < 3; ++j) {
        double s0, c0;
        sincos(z[j], &s0, &c0);
        const double s = sqrt(2.0 / (PI_D * z[j]));
        const double M = fmax(fabs(t[j][0]), fabs(t[j][1])), a0 = t[j][0] / M, a1 = t[j][1] / M;
        lam[j] = s * (s0 * a1 + c0 * a0) / (a1 * a1 + a0 * a0) / M;
    }
}

struct InvTable {
    double v[ANG_NCAP + 2];
    constexpr InvTable() : v()
    {
        for (int n = 0; n < ANG_NCAP + 2; ++n) v[n] = 1.0 / (n + 1.0);
    }
};
__constant__ constexpr InvTable ANG_INV{};  // 1 / (n + 1)

__device__ __forceinline__ double ang_cdf(const double *W, int N, double c)
{
    double s = 1.0 + c, pm = 1.0, p = c;
    const double inv0 = 1.0 / W[0];
    for (int n = 1; n <= N; ++n) {
        const double pn1 = ((2.0 * n + 1.0) * c * p - n * pm) * ANG_INV.v[n];
        s += W[n] * inv0 * (pn1 - pm);
        pm = p;
        p = pn1;
    }
    return 0.5 * s;
}

} // namespace gfbd
