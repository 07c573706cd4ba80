// Exact 2D radial functions beyond the small-time regime: tables of p_enc,
// p_reac and the propagator's distribution function, built on the device by
// quadrature of the n = 0 term of the 2D Green's function (eqs. genericGF and
// fRad) and read by bicubic interpolation.
//
// With R, R0 in units of a and tau = D_eff dt / a^2:
//   a^2 g(R | R0) = (1/2 pi) int_0^inf e^{-tau x^2} C(R, x) C(R0, x) x dx,
//   C(R, x) = [J0(Rx) A(x) - Y0(Rx) B(x)] / sqrt(A^2 + B^2),
// radiation A = -x Y1(x) - h Y0(x), B = -x J1(x) - h J0(x) (reflecting: h = 0),
// absorbing A = Y0(x), B = J0(x); and the mass within R,
//   int_1^R 2 pi R' g(R' | R0) dR' = int_0^inf e^{-tau x^2} C(R0, x) K(R, x) dx,
//   K(R, x) = [A (R J1(Rx) - J1(x)) - B (R Y1(Rx) - Y1(x))] / sqrt(A^2 + B^2)
// (the R' integral of R' J0(R'x) is R' J1(R'x)/x).  On the grid R_i = 1 + i h,
// h = sqrt(tau)/160 (fine enough for the layer of width tau/(R0 - 1) that
// p_enc and the propagator have at contact), with R0 on every second row
// (p_enc varies in R0 on the scale tau/(R - 1)), the quadrature sums are
// matrix products over the nodes:
//   G[i][j] = sum_k C(R_i, x_k) C(R0_j, x_k) x_k w_k / 2 pi,
//   M[i][j] = sum_k K(R_i, x_k) C(R0_j, x_k) w_k,
// with w_k the Gauss-Legendre weight times e^{-tau x_k^2}.  The tables are
//   p_enc  = 1 - G_abs / g_free,   p_reac = (G_ref - G_rad) / (G_ref - G_abs),
//   F      = (M_ref - M_abs)(R_i) / (M_ref - M_abs)(R0_j + L),  L = 12 sqrt(tau) + 1,
// stored column by column (a column is one R0).  They cover R0 <= 1 + c
// sqrt(tau), c = 8.4 for tau <= 0.5 and 9 up to tau = 0.8: there the
// propagator's mass 1 - S_abs(R0) stays above about erfc(c/2), which the
// quadrature resolves; beyond it every pair has x = (R + R0 - 2)/(2 sqrt tau)
// >= c/2, where the order-12 small-time expansion holds.  Against a numerical
// inversion of the Laplace-domain forms of Sec. 4.2 both sides of the switch
// hold 1e-6 for tau <= 0.5; from 0.5 to 0.8 the expansion's floor at contact
// rises to about 1.3e-6 (higher orders do worse: the series is asymptotic) and
// the quadrature loses resolution a little farther out, so c = 9 keeps both
// within 1.5e-6.  The propagator's distribution function, a ratio of masses of
// size 1 - S_abs(R0), keeps c = 8.4 at every tau (x2_r0sw_prop): beyond it the
// expansion's rejection sampler draws R''.  tau > 0.8 is refused.
// Included by green.hpp inside namespace gfbd, after i0e_d.
#pragma once

constexpr int NC_EXACT = -1;  // the order argument of the kernels that read the tables
constexpr u32 X2S = 2;        // R0 grid step in R grid steps
constexpr double X2_TAU_MAX = 0.8;  // largest tau of the exact 2D mode

// c of the switch R0 = 1 + c sqrt(tau) between the tables and the expansion
__host__ __device__ inline double x2_switch_c(double tau) { return tau <= 0.5 ? 8.4 : 9.0; }

// Lagrange weights of the cubic through nodes 0, 1, 2, 3 at s.
__device__ __forceinline__ void lag4(double s, double w[4])
{
    w[0] = -(s - 1.0) * (s - 2.0) * (s - 3.0) * (1.0 / 6.0);
    w[1] = s * (s - 2.0) * (s - 3.0) * 0.5;
    w[2] = -s * (s - 1.0) * (s - 3.0) * 0.5;
    w[3] = s * (s - 1.0) * (s - 2.0) * (1.0 / 6.0);
}

// The first of four nodes around grid position f (n >= 4 nodes) and the
// weights at f.
__device__ __forceinline__ u32 lag_base(double f, u32 n, double w[4])
{
    double b = floor(f) - 1.0;
    b = fmin(fmax(b, 0.0), (double)(n - 4));
    lag4(f - b, w);
    return (u32)b;
}

// The p_enc and p_reac tables are read at pairs in cell order, that is at random
// (R, R0): each lookup gathers a 4 x 4 stencil.  They are kept in binary32 (p_enc and
// p_reac are probabilities: the rounding is below 6e-8, the interpolation sums it to
// below 1e-7) in tiles of 8 rows (R) by 4 columns (R0), one 128-byte line each, a
// tile's columns of 8 rows one after the other, tiles ordered row tile fastest.  A
// stencil then touches 2.4 lines on average (4 to 5 in column-major binary64), and
// the rows that pairs within the cut-off read take half the bytes.
constexpr u32 X2TR = 8, X2TC = 4;

// Index of element (row i, column j) of a blocked table with ntr row tiles.
__device__ __forceinline__ size_t x2_bidx(u32 i, u32 j, u32 ntr)
{
    return ((size_t)(j / X2TC) * ntr + i / X2TR) * (X2TR * X2TC) + (j % X2TC) * X2TR + i % X2TR;
}

// Bicubic value of blocked table T at (R, R0).
__device__ inline double x2_table(const Params &P, const float *__restrict__ T, double R, double R0)
{
    double wi[4], wj[4];
    const u32 bi = lag_base((R - 1.0) * P.x2_inv_h, P.x2_nr, wi);
    const u32 bj = lag_base((R0 - 1.0) * P.x2_inv_h0, P.x2_n0, wj);
    double v = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const float *c = T + x2_bidx(0, bj + m, P.x2_ntr);  // the column in its first row tile
        double f[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const u32 i = bi + k;
            f[k] = (double)c[(size_t)(i / X2TR) * (X2TR * X2TC) + i % X2TR];
        }
        v += wj[m] * (wi[0] * f[0] + wi[1] * f[1] + wi[2] * f[2] + wi[3] * f[3]);
    }
    return v;
}

__device__ inline double penc2x(const Params &P, double R, double R0)
{
    if (R <= 1.0) return 1.0;
    return fmin(fmax(x2_table(P, P.x2_enc, R, R0), 0.0), 1.0);
}

__device__ inline double preac2x(const Params &P, double R, double R0)
{
    return fmin(fmax(x2_table(P, P.x2_reac, R, R0), 0.0), 1.0);
}

// R'' with F(R'' | R0) = u: the distribution function interpolated across R0
// (cubic), bisection over the grid rows for the bracketing interval, then
// bisection on the cubic through the rows around it.
__device__ inline double sample2x(const Params &P, double R0, double u)
{
    double wj[4];
    const u32 nr = P.x2_nr;
    // the columns beyond the propagator's switch are not resolved for it: the stencil stays below
    const u32 bj = lag_base((R0 - 1.0) * P.x2_inv_h0, P.x2_n0_prop, wj);
    const double *c = P.x2_cdf + (size_t)bj * nr;
    auto F = [&](u32 i) { return wj[0] * c[i] + wj[1] * c[nr + i] + wj[2] * c[2 * nr + i] + wj[3] * c[3 * nr + i]; };
    if (!(u > F(0))) return 1.0;
    u32 lo = 0, hi = nr - 1;
    if (!(u < F(hi))) return 1.0 + hi * P.x2_h;
    while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (F(mid) <= u) lo = mid;
        else hi = mid;
    }
    const u32 b = lo == 0 ? 0u : (lo + 3 > nr ? nr - 4 : lo - 1);
    const double f0 = F(b), f1 = F(b + 1), f2 = F(b + 2), f3 = F(b + 3);
    double sl = (double)(lo - b), sh = sl + 1.0;
#pragma nounroll
    for (int it = 0; it < 44; ++it) {
        const double sm = 0.5 * (sl + sh);
        double w[4];
        lag4(sm, w);
        if (w[0] * f0 + w[1] * f1 + w[2] * f2 + w[3] * f3 <= u) sl = sm;
        else sh = sm;
    }
    return 1.0 + ((double)b + 0.5 * (sl + sh)) * P.x2_h;
}

// ---- table construction ----------------------------------------------------

// Per node: normalised A, B of the three kinds and J1(x), Y1(x).
// nd[k * 8 + ...] = {Aabs, Babs, Aref, Bref, Arad, Brad, J1(x), Y1(x)}
__global__ void k_x2_nodes(const double *__restrict__ xs, u32 K, double hh, double *__restrict__ nd)
{
    const u32 k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const double x = xs[k];
    const double j0x = j0(x), y0x = y0(x), j1x = j1(x), y1x = y1(x);
    double A[3], B[3];
    A[0] = y0x;
    B[0] = j0x;
    A[1] = -x * y1x;
    B[1] = -x * j1x;
    A[2] = -x * y1x - hh * y0x;
    B[2] = -x * j1x - hh * j0x;
    double *o = nd + (size_t)k * 8;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double inv = 1.0 / sqrt(A[q] * A[q] + B[q] * B[q]);
        o[2 * q] = A[q] * inv;
        o[2 * q + 1] = B[q] * inv;
    }
    o[6] = j1x;
    o[7] = y1x;
}

// Rows of the quadrature matrices at R_i = 1 + i h: C of the three kinds
// and K of the absorbing and reflecting kinds, each nr x K (k fastest).
__global__ void k_x2_rows(const double *__restrict__ xs, const double *__restrict__ nd, u32 K, u32 nr, double h,
                          double *__restrict__ Cabs, double *__restrict__ Cref, double *__restrict__ Crad,
                          double *__restrict__ Kabs, double *__restrict__ Kref)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)nr * K) return;
    const u32 i = (u32)(t / K), k = (u32)(t % K);
    const double R = 1.0 + i * h, x = xs[k], Rx = R * x;
    const double jr = j0(Rx), yr = y0(Rx), j1r = j1(Rx), y1r = y1(Rx);
    const double *o = nd + (size_t)k * 8;
    const double dj = R * j1r - o[6], dy = R * y1r - o[7];
    Cabs[t] = jr * o[0] - yr * o[1];
    Cref[t] = jr * o[2] - yr * o[3];
    Crad[t] = jr * o[4] - yr * o[5];
    Kabs[t] = o[0] * dj - o[1] * dy;
    Kref[t] = o[2] * dj - o[3] * dy;
}

// out[i][j] = sum_k L[i][k] s[k] Rm[X2S j][k] (i < nr, j < n0; both operands nr x K
// with k fastest, the right one read on every X2S-th row, the R0 grid).
// 64 x 64 tiles, 4 x 4 per thread, chunks of 16 nodes through LDS.
constexpr int X2T = 64, X2C = 16;
__global__ __launch_bounds__(256) void k_x2_gemm(const double *__restrict__ L, const double *__restrict__ Rm,
                                                  const double *__restrict__ s, u32 nr, u32 n0, u32 K,
                                                  double *__restrict__ out)
{
    __shared__ double la[X2C][X2T + 1], rb[X2C][X2T + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const u32 i0 = blockIdx.y * X2T, j0_ = blockIdx.x * X2T;
    double acc[4][4] = {};
    for (u32 k0 = 0; k0 < K; k0 += X2C) {
        for (int e = threadIdx.x; e < X2T * X2C; e += 256) {
            const int r = e / X2C, kk = e % X2C;
            const u32 i = i0 + r, j = j0_ + r, k = k0 + kk;
            la[kk][r] = (i < nr && k < K) ? L[(size_t)i * K + k] * s[k] : 0.0;
            rb[kk][r] = (j < n0 && k < K) ? Rm[(size_t)(X2S * j) * K + k] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < X2C; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = la[kk][ty * 4 + q];
                b[q] = rb[kk][tx * 4 + q];
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[p][q] = fma(a[p], b[q], acc[p][q]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const u32 i = i0 + ty * 4 + p, j = j0_ + tx * 4 + q;
            if (i < nr && j < n0) out[(size_t)i * n0 + j] = acc[p][q];
        }
}

// The tables from the products (row-major nr x n0): p_enc and p_reac blocked in
// binary32 (ntr row tiles), the distribution function column-major in binary64.
// top: rows from R_j to the top of its distribution function.
__global__ void k_x2_tables(const double *__restrict__ Gabs, const double *__restrict__ Gref, const double *__restrict__ Grad,
                            const double *__restrict__ Mabs, const double *__restrict__ Mref, u32 nr, u32 n0, double h,
                            double tau, u32 top, u32 ntr, float *__restrict__ enc, float *__restrict__ reac,
                            double *__restrict__ cdf)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)nr * n0) return;
    const u32 j = (u32)(t / nr), i = (u32)(t % nr);  // output in column-major order
    const size_t a = (size_t)i * n0 + j;
    const double R = 1.0 + i * h, R0 = 1.0 + (double)(X2S * j) * h;
    // free function e^{-(R-R0)^2/4tau} i0e(R R0/2tau) / (4 pi tau)
    const double gf = exp(-(R - R0) * (R - R0) / (4.0 * tau)) * i0e_d(R * R0 / (2.0 * tau)) / (4.0 * PI_D * tau);
    const size_t b = x2_bidx(i, j, ntr);
    enc[b] = (float)(i == 0 ? 1.0 : 1.0 - Gabs[a] / gf);
    const double den = Gref[a] - Gabs[a];
    reac[b] = (float)(den > 0.0 ? (Gref[a] - Grad[a]) / den : 0.0);
    const u32 it = min(X2S * j + top, nr - 1);
    const size_t at = (size_t)it * n0 + j;
    const double mt = Mref[at] - Mabs[at];
    cdf[t] = i >= it ? 1.0 : (mt > 0.0 ? (Mref[a] - Mabs[a]) / mt : 0.0);
}
