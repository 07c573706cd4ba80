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

} // namespace gfbd
