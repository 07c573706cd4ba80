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
//   - inversion: nine rounds of a 65-way search over [-1, 1] (one point per lane),
//     a final interval of 2 / 65^9 < 1.1e-16.
// One wavefront per pair, lanes over the quadrature nodes; the per-order sums are
// reduced over the wave, so every lane holds every w_n.
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

__global__ __launch_bounds__(BLOCK) void k_angle3(double tau, uint64_t n, const double *__restrict__ Rv,
                                                  const double *__restrict__ R0v, const double *__restrict__ uv,
                                                  double *__restrict__ c_out, GL16 gl)
{
    constexpr int NW = BLOCK / 64;
    __shared__ double wsh[NW][ANG_NCAP + 1];
    const int lane = lane_id();
    double *W = wsh[threadIdx.x / 64];
    const uint64_t nwaves = (uint64_t)gridDim.x * NW;
    for (uint64_t i = (uint64_t)blockIdx.x * NW + threadIdx.x / 64; i < n; i += nwaves) {  // uniform over the wave
        const double Rin = Rv[i], R0in = R0v[i], u = uv[i];
        if (!(Rin + R0in - 2.0 <= 40.0 * sqrt(tau))) {  // no encounter reaches that far (e^{-400}), or not a number
            if (lane == 0) c_out[i] = __builtin_nan("");
            continue;
        }
        const double R = fmax(Rin, 1.0), R0 = fmax(R0in, 1.0);  // separations below contact count as contact
        const int N = ang_terms(R, R0, tau);
        const double X = sqrt(50.0 / tau);
        const double hmax = fmin(1.0, 2.0 * PI_D / (R + R0 - 1.0));
        const int P = (int)ceil(X / hmax);
        const double h = X / P;
        for (int k = 0; k <= N; ++k) W[k] = 0.0;
        for (int q0 = 0; q0 < 16 * P; q0 += 64) {  // uniform over the wave
            const int q = q0 + lane;
            const bool live = q < 16 * P;
            const int qq = live ? q : 0;
            const double x = h * ((qq >> 4) + 0.5 + 0.5 * gl.x[qq & 15]);
            const double g = live ? 0.5 * h * gl.w[qq & 15] * exp(-tau * x * x) * x : 0.0;
            double t[3][ANG_NCAP + 2], lam[3];
            const double z[3] = {x, R * x, R0 * x};
            ang_miller3(N + 1, z, t, lam);
            double ym[3], y0[3], iz[3];  // Y_{nu-1}, Y_nu, 1/z
            for (int j = 0; j < 3; ++j) {
                double s0, c0;
                sincos(z[j], &s0, &c0);
                const double s = sqrt(2.0 / (PI_D * z[j]));
                ym[j] = s * s0;   // Y_{-1/2}
                y0[j] = -s * c0;  // Y_{1/2}
                iz[j] = 1.0 / z[j];
            }
            bool dead = !live;
            double jm = lam[0] * t[0][0];  // J_{nu-1}(x)
            for (int nn = 0; nn <= N; ++nn) {  // uniform over the wave
                const int k = nn + 1;
                if (fabs(y0[0]) > 0x1p500) dead = true;
                double term = 0.0;
                const double jx = lam[0] * t[0][k];
                if (!dead) {
                    // F(R) F(R0) = (J(Rx) A - Y(Rx) B)(J(R0x) A - Y(R0x) B) / (A^2 + B^2)
                    const double jr = lam[1] * t[1][k], jq = lam[2] * t[2][k];
                    const double Ar = (2.0 * nn + 2.0) * y0[0] - 2.0 * x * ym[0];
                    const double Br = (2.0 * nn + 2.0) * jx - 2.0 * x * jm;
                    const double Aa = y0[0], Ba = jx;
                    const double pr = (jr * Ar - y0[1] * Br) / (Ar * Ar + Br * Br) * (jq * Ar - y0[2] * Br);
                    const double pa = (jr * Aa - y0[1] * Ba) / (Aa * Aa + Ba * Ba) * (jq * Aa - y0[2] * Ba);
                    term = g * (pr - pa);
                }
                jm = jx;
                W[nn] += wave_allsum(term);  // every lane writes the same value and reads its own
                for (int j = 0; j < 3; ++j) {  // Y_{nu+1} = (2 nu / z) Y_nu - Y_{nu-1}
                    const double yn = (2.0 * k - 1.0) * iz[j] * y0[j] - ym[j];
                    ym[j] = y0[j];
                    y0[j] = yn;
                }
            }
        }
        double lo = -1.0, hi = 1.0;
        for (int it = 0; it < 9; ++it) {
            const double d = (hi - lo) / 65.0;
            const double c = lo + d * (lane + 1);
            const u64 ge = __ballot(ang_cdf(W, N, c) >= u);
            const int j = ge ? __ffsll((unsigned long long)ge) - 1 : 64;  // first point at or above u
            const double nlo = j == 0 ? lo : lo + d * j;
            const double nhi = j == 64 ? hi : lo + d * (j + 1);
            lo = nlo;
            hi = nhi;
        }
        if (lane == 0) c_out[i] = 0.5 * (lo + hi);
    }
}

} // namespace gfbd
