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
//   - x integral: 32 Gauss-Legendre panels of ratio 2 on [2^-32, 1] (Y_0 has a logarithm at
//     x = 0), then panels of equal width at most min(1, 2 pi / (R + R0 - 1)) up to
//     sqrt(50 / tau);
//   - sin(n t) by the three-term recurrence s_{n+1} = 2 cos(t) s_n - s_{n-1}.
#pragma once

#include "angle3.hpp"

namespace gfbd {

constexpr int ANG2_GEO = 32;  // geometric panels on [2^-32, 1]

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

__global__ __launch_bounds__(BLOCK) void k_angle2(double tau, uint64_t n, const double *__restrict__ Rv,
                                                  const double *__restrict__ R0v, const double *__restrict__ uv,
                                                  double *__restrict__ th_out, GL16 gl)
{
    constexpr int NW = BLOCK / 64;
    __shared__ double wsh[NW][ANG_NCAP + 1];
    const int lane = lane_id();
    double *W = wsh[threadIdx.x / 64];
    const uint64_t nwaves = (uint64_t)gridDim.x * NW;
    for (uint64_t i = (uint64_t)blockIdx.x * NW + threadIdx.x / 64; i < n; i += nwaves) {  // uniform over the wave
        const double Rin = Rv[i], R0in = R0v[i], u = uv[i];
        if (!(Rin + R0in - 2.0 <= 40.0 * sqrt(tau))) {  // no encounter reaches that far (e^{-400}), or not a number
            if (lane == 0) th_out[i] = __builtin_nan("");
            continue;
        }
        const double R = fmax(Rin, 1.0), R0 = fmax(R0in, 1.0);  // separations below contact count as contact
        const int N = ang_terms(R, R0, tau);
        const double X = sqrt(50.0 / tau), x1 = X < 1.0 ? X : 1.0;
        const double hmax = fmin(1.0, 2.0 * PI_D / (R + R0 - 1.0));
        const int nuni = X > x1 ? (int)ceil((X - x1) / hmax) : 0;
        const double huni = nuni > 0 ? (X - x1) / nuni : 0.0;
        const int Q = 16 * (ANG2_GEO + nuni);
        for (int k = 0; k <= N; ++k) W[k] = 0.0;
        for (int q0 = 0; q0 < Q; q0 += 64) {  // uniform over the wave
            const int q = q0 + lane;
            const bool live = q < Q;
            const int p = live ? q >> 4 : 0;
            double lo, hi;
            if (p < ANG2_GEO) {
                lo = ldexp(x1, p - ANG2_GEO);
                hi = 2.0 * lo;
            } else {
                lo = x1 + (p - ANG2_GEO) * huni;
                hi = lo + huni;
            }
            const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
            const double x = c + h * gl.x[q & 15];
            const double g = live ? h * gl.w[q & 15] * exp(-tau * x * x) * x : 0.0;
            double t[3][ANG_NCAP + 2], lam[3], y0v[3], ym[3], iz[3], j0z[3], j1z[3];  // Y_n, Y_{n-1}, 1/z
            const double z[3] = {x, R * x, R0 * x};
            for (int j = 0; j < 3; ++j) {
                ang_bessel01(z[j], &j0z[j], &j1z[j], &y0v[j], &ym[j]);
                ym[j] = -ym[j];  // Y_{-1} = -Y_1
                iz[j] = 1.0 / z[j];
            }
            // the first order whose |Y_n(x)| exceeds 2^500 ends the node's terms (the same
            // recurrence as below): J is needed only up to there
            int nd = N + 1;
            {
                double a = ym[0], b = y0v[0];
                for (int nn = 0; nn <= N; ++nn) {
                    if (fabs(b) > 0x1p500) {
                        nd = nn;
                        break;
                    }
                    const double c = (2.0 * nn) * iz[0] * b - a;
                    a = b;
                    b = c;
                }
            }
            const int kmax = nd + 1 < N + 1 ? nd + 1 : N + 1;  // >= 1
            ang_miller3_int(kmax, z, t, lam, j0z, j1z);
            bool dead = !live;
            double jm = -lam[0] * t[0][1];  // J_{-1}(x) = -J_1(x)
            for (int nn = 0; nn <= N; ++nn) {  // uniform over the wave
                if (fabs(y0v[0]) > 0x1p500) dead = true;
                if (__ballot(!dead) == 0) break;  // every node of the wave is past its last order
                double term = 0.0;
                const double jx = nn <= kmax ? lam[0] * t[0][nn] : 0.0;
                if (!dead) {
                    // C(R) C(R0) = (J(Rx) A - Y(Rx) B)(J(R0x) A - Y(R0x) B) / (A^2 + B^2)
                    const double jr = lam[1] * t[1][nn], jq = lam[2] * t[2][nn];
                    const double Ar = x * ym[0] - nn * y0v[0], Br = x * jm - nn * jx;
                    const double Aa = y0v[0], Ba = jx;
                    const double pr = (jr * Ar - y0v[1] * Br) / (Ar * Ar + Br * Br) * (jq * Ar - y0v[2] * Br);
                    const double pa = (jr * Aa - y0v[1] * Ba) / (Aa * Aa + Ba * Ba) * (jq * Aa - y0v[2] * Ba);
                    term = g * (pr - pa);
                }
                jm = jx;
                W[nn] += wave_allsum(term);  // every lane writes the same value and reads its own
                for (int j = 0; j < 3; ++j) {  // Y_{n+1} = (2n / z) Y_n - Y_{n-1}
                    const double yn = (2.0 * nn) * iz[j] * y0v[j] - ym[j];
                    ym[j] = y0v[j];
                    y0v[j] = yn;
                }
            }
        }
        double lo = 0.0, hi = PI_D;
        for (int it = 0; it < 9; ++it) {
            const double d = (hi - lo) / 65.0;
            const double tt = lo + d * (lane + 1);
            const u64 ge = __ballot(ang2_cdf(W, N, tt) >= u);
            const int j = ge ? __ffsll((unsigned long long)ge) - 1 : 64;  // first point at or above u
            const double nlo = j == 0 ? lo : lo + d * j;
            const double nhi = j == 64 ? hi : lo + d * (j + 1);
            lo = nlo;
            hi = nhi;
        }
        if (lane == 0) th_out[i] = 0.5 * (lo + hi);
    }
}

} // namespace gfbd
