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
//   - Bessel functions of integer order: J by the downward recurrence normalised to j0, j1;
//     Y upward from y0, y1;
//   - x integral: geometric Gauss-Legendre panels on (0, 1] (Y_0 has a logarithm at
//     x = 0; the kernel's layout is in angle_wg.hpp), then panels of equal width at most
//     min(1, 2 pi / (R + R0 - 1)) up to sqrt(50 / tau);
//   - sin(n t) by the three-term recurrence s_{n+1} = 2 cos(t) s_n - s_{n-1}.
#pragma once

#include "angle3.hpp"

namespace gfbd {

// J_0, J_1, Y_0, Y_1 at z (kept out of line: the four library functions are long)
__device__ __noinline__ void ang_bessel01(double z, double *j0z, double *j1z, double *y0z, double *y1z)
{
    *j0z = j0(z);
    *j1z = j1(z);
    *y0z = y0(z);
    *y1z = y1(z);
}

// J_n(z) for n = 0 .. kmax, three arguments at once: t[j][n] times lam[j].
__device__ __forceinline__ void ang_miller3_int(int kmax, const double z[3], double (*t)[ANG_NCAP + 2], double lam[3],
                                                const double j0z[3], const double j1z[3])
{
    const double zm = fmax(z[0], fmax(z[1], z[2]));
    const int zc = (int)ceil(zm + 8.0 * cbrt(zm));
    const int m = (kmax > zc ? kmax : zc) + 8;
    double a[3], b[3], inv[3];  // a = J_n, b = J_{n+1}
    for (int j = 0; j < 3; ++j) {
        a[j] = 1.0;
        b[j] = 0.0;
        inv[j] = 1.0 / z[j];
    }
    for (int n = m; n >= 1; --n) {
        for (int j = 0; j < 3; ++j) {
            const double c = (2.0 * n) * inv[j] * a[j] - b[j];  // J_{n-1} = (2n / z) J_n - J_{n+1}
            b[j] = a[j];
            a[j] = c;
            if (fabs(c) > 1e250) {  // rescale, including what is already stored
                a[j] *= 1e-250;
                b[j] *= 1e-250;
                for (int q = n; q <= kmax; ++q) t[j][q] *= 1e-250;
            }
            if (n - 1 <= kmax) t[j][n - 1] = a[j];
        }
    }
    for (int j = 0; j < 3; ++j) {
        const double a0 = j0z[j], a1 = j1z[j];
        const double M = fmax(fabs(t[j][0]), fabs(t[j][1])), b0 = t[j][0] / M, b1 = t[j][1] / M;
        lam[j] = (a0 * b0 + a1 * b1) / (b0 * b0 + b1 * b1) / M;
    }
}

__device__ __forceinline__ double ang2_cdf(const double *W, int N, double t)
{
    const double c2 = 2.0 * cos(t);
    double sm = 0.0, s = sin(t), acc = W[0] * t;  // s_{n-1}, s_n at n = 1
    for (int n = 1; n <= N; ++n) {
        acc += 2.0 * W[n] * s * ANG_INV.v[n - 1];
        const double sn = c2 * s - sm;
        sm = s;
        s = sn;
    }
    return acc / (PI_D * W[0]);
}

} // namespace gfbd
