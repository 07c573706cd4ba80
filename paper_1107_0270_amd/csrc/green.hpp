// Device-side Green's-function quantities of the coarse-grained BD step:
// encounter and reaction probabilities (Secs. 2.2.1-2.2.4 with the 3D closed
// forms of Sec. 4.1 and the 2D small-time expansions of Sec. 4.2) and the
// radial propagator sampler (Sec. 2.2.2, Sec. 3 Details).
#pragma once

#include "common.hpp"

namespace gfbd {

constexpr double PI_D = 3.14159265358979323846;
constexpr double SQRTPI_D = 1.77245385090551602730;

// ---------------------------------------------------------------------------
// 3D encounter probability 1 - g_abs/g_free.  With the two closed forms over
// the same prefactor, and (R+R0-2)^2 - (R-R0)^2 = 4(R-1)(R0-1),
// (R+R0)^2 - (R-R0)^2 = 4 R R0:
//   p_enc = e^{-(R-1)(R0-1)/tau} (1 - e^{-(R+R0-1)/tau}) / (1 - e^{-R R0/tau}).
// The three exponent arguments are formed in T2, the exponentials in T1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double penc3_args(double e1, double e2, double e3)
{
    return exp(-e1) * expm1(-e2) / expm1(-e3);
}
__device__ __forceinline__ float penc3_args(float e1, float e2, float e3)
{
    return expf(-e1) * expm1f(-e2) / expm1f(-e3);
}

// 3D reaction probability (g_ref - g_rad)/(g_ref - g_abs): the free term and
// the common factor e^{-w^2/4tau} cancel, leaving
//   sqrt(pi tau) [kappa erfcx(z_kappa) - erfcx(z_1)] / (1 - sqrt(pi tau) erfcx(z_1)),
// z_k = k sqrt(tau) + w/(2 sqrt(tau)), w = R + R0 - 2, kappa = 1 + h.
__device__ inline double preac3(const Params &P, double R, double R0)
{
    const double w = R + R0 - 2.0, st = P.sqrt_tau, kap = 1.0 + P.hh;
    const double z1 = st + w / (2.0 * st), zk = kap * st + w / (2.0 * st);
    const double spt = SQRTPI_D * st;
    return spt * (kap * erfcx(zk) - erfcx(z1)) / (1.0 - spt * erfcx(z1));
}

// ---------------------------------------------------------------------------
// 2D: e^{-x} I_0(x); scaled repeated erfc integrals; expansion coefficients.
// ---------------------------------------------------------------------------

// e^{-x} I_0(x): the device library's I_0 below 500, above it the
// large-argument series e^x/sqrt(2 pi x) sum |a_k(0)| x^-k (cut at its
// smallest term, far below rounding there).
__device__ inline double i0e_d(double x)
{
    if (x <= 500.0) return cyl_bessel_i0(x) * exp(-x);
    double t = 1.0, s = 1.0;
    const double ix = 1.0 / x;
    for (int k = 1; k < 80; ++k) {
        const double r = (2.0 * k - 1.0) * (2.0 * k - 1.0) * 0.125 * ix / (double)k;
        if (r >= 1.0) break;
        t *= r;
        s += t;
        if (t < 1e-18 * s) break;
    }
    return s * rsqrt(2.0 * PI_D * x);
}

// The expansion to order n.  NC > 0 fixes n = NC at compile time: the loops
// unroll and the coefficient arrays stay in registers.  NC = 0 takes
// n = P.n_terms at run time (any order up to MAXTERMS).
template <int NC> struct Order {
    static constexpr int M = NC > 0 ? NC : MAXTERMS;
};

// T_k = e^{x^2} i^{k-1}erfc(x) (2 sqrt tau)^k, k = 1..n, by the upward
// recursion 2k i^k = i^{k-2} - 2x i^{k-1} (eq. iErf) started from
// i^{-1} = 2/sqrt(pi) and i^0 = erfcx(x).
template <int NC> __device__ __forceinline__ void t_terms(double x, double two_st, int n, double *T)
{
    double im2 = 2.0 / SQRTPI_D, im1 = erfcx(x), pw = two_st;
    T[1] = im1 * pw;
#pragma unroll
    for (int k = 2; k <= Order<NC>::M; ++k) {
        if (k > n) break;
        const double ik = (im2 - 2.0 * x * im1) / (2.0 * (k - 1));
        im2 = im1;
        im1 = ik;
        pw *= two_st;
        T[k] = ik * pw;
    }
}

// P_k: coefficients of A_0(s/R0) A_0(s/R), k = 0..n (a_k(0) from the table).
template <int NC> __device__ __forceinline__ void p_series(const double *a0, double R, double R0, int n, double *Pc)
{
    double x[Order<NC>::M + 1], y[Order<NC>::M + 1];
    const double iR = 1.0 / R, iR0 = 1.0 / R0;
    double px = 1.0, py = 1.0;
#pragma unroll
    for (int k = 0; k <= Order<NC>::M; ++k) {
        if (k > n) break;
        x[k] = a0[k] * px;
        y[k] = a0[k] * py;
        px *= iR0;
        py *= iR;
    }
#pragma unroll
    for (int k = 0; k <= Order<NC>::M; ++k) {
        if (k > n) break;
        double s = 0.0;
#pragma unroll
        for (int m = 0; m <= k; ++m) s += x[m] * y[k - m];
        Pc[k] = s;
    }
}

// gamma_k = sum_m Q_m P_{k-m} for one boundary condition's quotient series Q.
__device__ __forceinline__ double gamma_k(const double *Q, const double *Pc, int k)
{
    double s = 0.0;
#pragma unroll
    for (int m = 0; m <= k; ++m) s += Q[m] * Pc[k - m];
    return s;
}

// 2D encounter probability -g_abs,bc / g_free with eq. smallTEabs:
//   sqrt(tau/(R R0)) e^{-(R-1)(R0-1)/tau} [pi^{-1/2} + (1/2) sum gamma^abs_k T_k] / i0e(R R0/2tau).
// At a given tau (sqrt_tau and inv_tau its root and inverse): the step uses the
// handle's, the first-passage bisection those of its half intervals.
template <int NC>
__device__ inline double penc2_at(const Params &P, double R, double R0, double tau, double sqrt_tau, double inv_tau)
{
    const int n = NC > 0 ? NC : P.n_terms;
    const double *a0 = P.g2c, *Qa = P.g2c + (MAXTERMS + 1);
    double Pc[Order<NC>::M + 1], T[Order<NC>::M + 1];
    p_series<NC>(a0, R, R0, n, Pc);
    const double x = (R + R0 - 2.0) / (2.0 * sqrt_tau);
    t_terms<NC>(x, 2.0 * sqrt_tau, n, T);
    double S = 1.0 / SQRTPI_D;
#pragma unroll
    for (int k = 1; k <= Order<NC>::M; ++k) {
        if (k > n) break;
        S += 0.5 * gamma_k(Qa, Pc, k) * T[k];
    }
    return sqrt(tau / (R * R0)) * exp(-(R - 1.0) * (R0 - 1.0) * inv_tau) * S / i0e_d(R * R0 * 0.5 * inv_tau);
}
template <int NC> __device__ inline double penc2_n(const Params &P, double R, double R0)
{
    return penc2_at<NC>(P, R, R0, P.tau, P.sqrt_tau, P.inv_tau);
}

// 2D reaction probability: free parts and the common factor cancel,
//   sum (g^ref_k - g^rad_k) T_k / [4 pi^{-1/2} + sum (g^ref_k + g^abs_k) T_k].
template <int NC> __device__ inline double preac2_n(const Params &P, double R, double R0)
{
    const int n = NC > 0 ? NC : P.n_terms;
    const double *a0 = P.g2c, *Qa = a0 + (MAXTERMS + 1), *Qf = a0 + 2 * (MAXTERMS + 1), *Qr = a0 + 3 * (MAXTERMS + 1);
    double Pc[Order<NC>::M + 1], T[Order<NC>::M + 1];
    p_series<NC>(a0, R, R0, n, Pc);
    const double x = (R + R0 - 2.0) / (2.0 * P.sqrt_tau);
    t_terms<NC>(x, 2.0 * P.sqrt_tau, n, T);
    double num = 0.0, den = 4.0 / SQRTPI_D;
#pragma unroll
    for (int k = 1; k <= Order<NC>::M; ++k) {
        if (k > n) break;
        const double gf = gamma_k(Qf, Pc, k);
        num += (gf - gamma_k(Qr, Pc, k)) * T[k];
        den += (gf + gamma_k(Qa, Pc, k)) * T[k];
    }
    return num / den;
}

// The 2D propagator density over its leading term: 1 + (sqrt(pi)/4) sum (g^ref_k + g^abs_k) T_k.
template <int NC> __device__ inline double corr2_n(const Params &P, double Rp, double R0)
{
    const int n = NC > 0 ? NC : P.n_terms;
    const double *a0 = P.g2c, *Qa = a0 + (MAXTERMS + 1), *Qf = a0 + 2 * (MAXTERMS + 1);
    double Pc[Order<NC>::M + 1], T[Order<NC>::M + 1];
    p_series<NC>(a0, Rp, R0, n, Pc);
    const double x = (Rp + R0 - 2.0) / (2.0 * P.sqrt_tau);
    t_terms<NC>(x, 2.0 * P.sqrt_tau, n, T);
    double s = 0.0;
#pragma unroll
    for (int k = 1; k <= Order<NC>::M; ++k) {
        if (k > n) break;
        s += (gamma_k(Qf, Pc, k) + gamma_k(Qa, Pc, k)) * T[k];
    }
    return 1.0 + 0.25 * SQRTPI_D * s;
}

#include "green2x.hpp"

// The order NC (12, or 0 for any order; NC_EXACT: the tables of green2x.hpp) is a template parameter of the
// kernels that evaluate the expansion, chosen on the host; NC = 0 takes the
// run-time order (its arrays sized for MAXTERMS).
__device__ inline double penc2_any(const Params &P, double R, double R0) { return penc2_n<0>(P, R, R0); }
__device__ inline double preac2_any(const Params &P, double R, double R0) { return preac2_n<0>(P, R, R0); }
__device__ inline double corr2_any(const Params &P, double Rp, double R0) { return corr2_n<0>(P, Rp, R0); }
// Beyond the tables' switch (NC_EXACT) the expansion runs at the handle's order, in its
// compiled form when that is the default order 12 (uniform branch): a wave whose pairs
// straddle the switch runs both forms, and the run-time-order one costs several times more.
template <int NC> __device__ inline double penc2(const Params &P, double R, double R0)
{
    if constexpr (NC == NC_EXACT) {
        if (R0 <= P.x2_r0sw) return penc2x(P, R, R0);
        return P.n_terms == 12 ? penc2_n<12>(P, R, R0) : penc2_any(P, R, R0);
    }
    else if constexpr (NC == 0) return penc2_any(P, R, R0);
    else return penc2_n<NC>(P, R, R0);
}
template <int NC> __device__ inline double preac2(const Params &P, double R, double R0)
{
    if constexpr (NC == NC_EXACT) {
        if (R0 <= P.x2_r0sw) return preac2x(P, R, R0);
        return P.n_terms == 12 ? preac2_n<12>(P, R, R0) : preac2_any(P, R, R0);
    }
    else if constexpr (NC == 0) return preac2_any(P, R, R0);
    else return preac2_n<NC>(P, R, R0);
}
template <int NC> __device__ inline double corr2(const Params &P, double Rp, double R0)
{
    if constexpr (NC == NC_EXACT) return 1.0;  // not reached: the exact form samples by inversion
    else if constexpr (NC == 0) return corr2_any(P, Rp, R0);
    else return corr2_n<NC>(P, Rp, R0);
}

template <int NC> __device__ inline double reac_prob(const Params &P, int dim, double R, double R0)
{
    if (P.bc == 0) return 1.0;
    if (P.bc == 1) return 0.0;
    return dim == 3 ? preac3(P, R, R0) : preac2<NC>(P, R, R0);
}

// ---------------------------------------------------------------------------
// Radial propagator sampler.
// ---------------------------------------------------------------------------

// The y >= yc with erfc(y) = u erfc(yc).  Start from the binary32 erfcinv
// of the target (about 1e-7 relative; where the target is below the binary32
// range, from the leading large-y form erfc(y) ~ e^{-y^2}/(y sqrt(pi)), within
// 1% there), then binary64 Newton steps on
// f(y) = ln erfcx(y) - y^2 - ln(u erfc(yc)), f'(y) = -2/(sqrt(pi) erfcx(y)),
// which converge quadratically: two or three reach the root to rounding.
// Called, not inlined: its registers would otherwise add to its callers'.
__device__ __forceinline__ double erfc_tail_inv(double yc, double u)
{
    const double lt = log(u) + log(erfcx(yc)) - yc * yc;  // ln of the target
    double y;
    if (lt > -80.0) {
        y = (double)erfcinvf(expf((float)lt));
    } else {
        const double s = sqrt(-lt);
        y = sqrt(fmax(-lt - log(s * SQRTPI_D), 0.0));
    }
    if (!(y >= yc)) y = yc;
#pragma nounroll
    for (int it = 0; it < 8; ++it) {
        const double ex = erfcx(y);
        const double dy = (log(ex) - y * y - lt) * ex * (0.5 * SQRTPI_D);
        double yn = y + dy;
        if (!(yn >= yc)) yn = yc;
        const bool done = fabs(yn - y) <= 2e-16 * y;
        y = yn;
        if (done) break;
    }
    return y;
}

constexpr u32 MAX_ATTEMPTS = 4096u;

// R'' >= 1 from w_d r^{d-1}(g_ref - g_abs)(.|R0) (Sec. 3, Details).  With
// c = R0 - 1, v = R' + R0 - 2 >= c, the target is
//   3D: (1 + v - c) e^{-v^2/4tau} [1 - sqrt(pi tau) erfcx(sqrt(tau) + v/(2 sqrt(tau)))],
//   2D: sqrt(1 + v - c) e^{-v^2/4tau} corr2(v),
// proposed from (1 + beta (v - c)) e^{-v^2/4tau}, beta = 1 (3D) or 1/2 (2D):
// a Gaussian-tail / Rayleigh-tail mixture when beta c <= 1, else the Rayleigh
// tail alone.  Attempt k draws Philox {c0, c1, step, tag | k << 8}: word 0
// chooses the mixture part, word 1 inverts its tail, word 2 accepts.  The
// result is the proposal of the first accepted attempt.
struct PropSetup {
    double c, yc, beta, w1, w2;
    bool mixture;
};

template <int DIM> __device__ inline PropSetup prop_setup(const Params &P, double R0)
{
    PropSetup S;
    S.c = R0 - 1.0;
    if (S.c < 0.0) S.c = 0.0;
    S.yc = S.c / (2.0 * P.sqrt_tau);
    S.beta = DIM == 3 ? 1.0 : 0.5;
    S.mixture = S.beta * S.c <= 1.0;
    S.w1 = S.w2 = 0.0;
    if (S.mixture) {
        S.w1 = (1.0 - S.beta * S.c) * (SQRTPI_D * P.sqrt_tau) * erfcx(S.yc);
        S.w2 = 2.0 * P.tau * S.beta;
    }
    return S;
}

// One attempt: the proposed R' and whether it is accepted.
template <int DIM, int NC>
__device__ inline double prop_attempt(const Params &P, const PropSetup &S, double R0, u32 c0, u32 c1, u32 step, u32 tag, u32 k,
                                      bool *accepted, bool *hit)
{
    const double tau = P.tau, st = P.sqrt_tau, c = S.c;
    const uint4 r = philox(c0, c1, step, (tag & 0xFFu) | (k << 8), P.key);
    const double u0 = u01(r.x), u1 = u01(r.y), u2 = u01(r.z);
    double v, acc;
    if (S.mixture) {
        if (u0 * (S.w1 + S.w2) < S.w1) v = 2.0 * st * erfc_tail_inv(S.yc, u1);
        else v = sqrt(c * c - 4.0 * tau * log(u1));
        acc = 1.0;
    } else {
        v = sqrt(c * c - 4.0 * tau * log(u1));
        acc = (1.0 + S.beta * (v - c)) / (S.beta * v);
    }
    const double Rp = 1.0 + v - c;
    *hit = false;
    if (DIM == 3) {
        acc *= 1.0 - (SQRTPI_D * st) * erfcx(st + v / (2.0 * st));
    } else {
        double corr = corr2<NC>(P, Rp, R0);
        if (corr > 1.0) {
            *hit = true;
            corr = 1.0;
        }
        if (corr < 0.0) corr = 0.0;
        acc *= sqrt(Rp) / (1.0 + 0.5 * (Rp - 1.0)) * corr;
    }
    *accepted = u2 < acc;
    return Rp;
}

// The sampler for a whole wave working on one pair: lane l evaluates attempts
// l, l + 64, ...; the first accepted attempt in order wins, exactly as if the
// attempts were tried one after another.  Every lane of the wave must call it
// with the same arguments; every lane gets the result.
// The exact 2D form (tables, R0 up to the switch) draws by inversion with
// word 0 of attempt 0; beyond the switch it samples by rejection from the
// small-time expansions.
__device__ inline double sample_radius_x2(const Params &P, double R0, u32 c0, u32 c1, u32 step, u32 tag, u32 *attempts, u32 *hits)
{
    const uint4 r = philox(c0, c1, step, tag & 0xFFu, P.key);
    *attempts = 1;
    *hits = 0;
    return sample2x(P, R0, u01(r.x));
}

template <int DIM, int NC>
__device__ double sample_radius_wave(const Params &P, double R0, u32 c0, u32 c1, u32 step, u32 tag, u32 *attempts, u32 *hits)
{
    if constexpr (DIM == 2 && NC == NC_EXACT) {
        if (R0 > P.x2_r0sw_prop) return sample_radius_wave<DIM, 0>(P, R0, c0, c1, step, tag, attempts, hits);
        return sample_radius_x2(P, R0, c0, c1, step, tag, attempts, hits);
    }
    const PropSetup S = prop_setup<DIM>(P, R0);
    const int lane = threadIdx.x & 63;
    u32 nh = 0;
    double Rp = 1.0;
    for (u32 k0 = 0; k0 < MAX_ATTEMPTS; k0 += 64) {
        bool ok, hit;
        Rp = prop_attempt<DIM, NC>(P, S, R0, c0, c1, step, tag, k0 + lane, &ok, &hit);
        const u64 okm = __ballot(ok), hm = __ballot(hit);
        if (okm) {
            const int first = __ffsll((unsigned long long)okm) - 1;
            const u64 upto = first == 63 ? ~0ull : ((2ull << first) - 1ull);
            *attempts = k0 + first + 1;
            *hits = nh + (u32)__popcll(hm & upto);
            return __shfl(Rp, first, 64);
        }
        nh += (u32)__popcll(hm);
    }
    *attempts = MAX_ATTEMPTS;
    *hits = nh;
    return __shfl(Rp, 63, 64);
}

// The same sampler for one lane working alone: attempts 0, 1, 2, ... in
// order until one is accepted (the definition the wave form reproduces).
template <int DIM, int NC>
__device__ double sample_radius_lane(const Params &P, double R0, u32 c0, u32 c1, u32 step, u32 tag, u32 *attempts, u32 *hits)
{
    if constexpr (DIM == 2 && NC == NC_EXACT) {
        if (R0 > P.x2_r0sw_prop) return sample_radius_lane<DIM, 0>(P, R0, c0, c1, step, tag, attempts, hits);
        return sample_radius_x2(P, R0, c0, c1, step, tag, attempts, hits);
    }
    const PropSetup S = prop_setup<DIM>(P, R0);
    u32 nh = 0;
    double Rp = 1.0;
    for (u32 k = 0; k < MAX_ATTEMPTS; ++k) {
        bool ok, hit;
        Rp = prop_attempt<DIM, NC>(P, S, R0, c0, c1, step, tag, k, &ok, &hit);
        nh += hit;
        if (ok) {
            *attempts = k + 1;
            *hits = nh;
            return Rp;
        }
    }
    *attempts = MAX_ATTEMPTS;
    *hits = nh;
    return Rp;
}

} // namespace gfbd
