// Angular propagator in 2D: the angle theta between a membrane pair's separations before
// and after a non-reactive encounter, drawn from r (G_ref - G_abs) given the new radius
// (Sec. 3, Details, with J = r).
//
// In units a = 1, D_eff = 1 (eq. genericGF with h -> 0 and h -> infinity, eq. fRad),
//   G_ref - G_abs = [w_0 + 2 sum_{n>=1} w_n cos(n theta)] / (2 pi),
//   w_n = int_0^inf e^{-tau x^2} [C^r_n(R,x) C^r_n(R0,x) - C^a_n(R,x) C^a_n(R0,x)] x dx,
// C_n = [J_n(Rx) A - Y_n(Rx) B] / sqrt(A^2 + B^2) with
//   reflecting: A = x Y_{n-1}(x) - n Y_n(x), B = x J_{n-1}(x) - n J_n(x),
//   absorbing:  A = Y_n(x), B = J_n(x)
// (x C'_n = x C_{n-1} - n C_n; C_{-1} = -C_1).  |theta| in [0, pi] given R has the
// distribution function F(t) = [w_0 t + 2 sum_{n>=1} w_n sin(n t) / n] / (pi w_0), and the
// draw is its root at the caller's u.
//
// Evaluation as in 3D (angle3.hpp) except:
//   - Bessel functions of integer order: J by the downward recurrence, normalised by the
//     Neumann sum J_0 + 2 sum J_{2k} = 1; Y upward from Y_0, Y_1, which the Neumann series
//     give from the same J sequence (angle_wg.hpp);
//   - x integral: geometric Gauss-Legendre panels on (0, 1] (Y_0 has a logarithm at
//     x = 0; the kernel's layout is in angle_wg.hpp), then panels of equal width at most
//     min(1, 2 pi / (R + R0 - 1)) up to sqrt(50 / tau);
//   - sin(n t) by the three-term recurrence s_{n+1} = 2 cos(t) s_n - s_{n-1}.
#pragma once

#include "angle3.hpp"
