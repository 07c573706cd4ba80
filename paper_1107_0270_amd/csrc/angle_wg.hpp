// The angular propagator at step size: one workgroup of 128 threads per pair.
//
// After a non-reactive encounter the pair's new separation makes an angle Theta with
// its pre-step separation drawn from J (G_ref - G_abs) given the new radius (Sec. 3,
// Details, second item of the propagation; the series of eqs. genericGF3D and
// genericGF, the Bessel recurrences of eq. 3termBessel).  The series and the
// distribution functions are those of angle3.hpp (3D) and angle2.hpp (2D); what
// differs is how the work is laid out and how much of it is done:
//
//   - the pair's quadrature nodes are spread over the workgroup, one node per thread
//     (more than 128 nodes: batches of 128), so a pair's latency is about that of one
//     node.  A pair of the 3D workload at tau = 0.8 has exactly 128 nodes;
//   - a node computes the orders up to ceil(z + 8 z^{1/3}) + 8 only, z the largest of
//     its three Bessel arguments (and at most the series' N): beyond the turning point
//     by that much, J_n(z) and with it every product term is below 1e-28 of w_0 (the
//     terms fall like ((z/2)^n / n!)^2).  Nodes at small x, which would otherwise carry
//     all N orders, need a fraction of them;
//   - the Bessel sequence J of a node comes from the downward recurrence, which yields
//     it highest order first while the products need it lowest order first.  Instead
//     of storing the sequence per thread (per-lane scratch memory), the first sweep
//     keeps the pair (J_k, J_{k+1}) at every 16th order k (every 32nd when six such
//     checkpoints would not cover the wave's orders) in the thread's column of LDS, and
//     the second pass regenerates each 16-order chunk downward from its checkpoint into
//     registers (a lower chunk runs through the upper one first), then consumes it
//     upward beside the upward recurrence of Y.
//     Rescaling during the first sweep scales the checkpoints already kept, so every
//     value is the same solution of the recurrence up to one common factor, removed by
//     the normalisation to the elementary J_{-1/2}, J_{1/2} (3D) or to J_0, J_1 (2D).
//     Six checkpoints cover the series' cap of 160 terms in 37 KB of LDS, so four
//     workgroups (two waves per SIMD) share a compute unit;
//   - each chunk's sixteen per-order terms are summed over the wave by a transposing
//     reduction (halving the orders a lane holds at each exchange: 17 exchanges per
//     chunk instead of 6 per order, done by permlane swaps and DPP moves in the VALU)
//     and added into the wave's own row of LDS; the rows are summed in wave order at
//     the end.  Every sum runs in a fixed order, so the coefficients, and the draw, do
//     not depend on timing;
//   - the search evaluates the 3D distribution function as a Legendre series summed
//     downward (Clenshaw), its coefficients and recurrence constants in rows of LDS;
//   - 2D: the geometric panels near x = 0 have ratio 4 (twelve on [4^-12, 1]) instead
//     of the ratio 2 of angle2.hpp; below 4^-12 the integrand (x times a power of
//     1 / log x) adds less than 1e-17 of w_0;
//   - the x integral stops at sqrt(40 / tau), where e^{-tau x^2} = e^{-40}, instead of
//     sqrt(50 / tau): the rest is below 5e-18 of the integral of the terms' magnitudes,
//     far below the rounding the cancellation in G_ref - G_abs brings, and in 3D at
//     tau = 0.8 pairs with R + R0 up to 8.1 (up to 7.36 before) fit one batch of nodes;
//   - the root of F(.) = u is bracketed by four rounds of a 128-point search (one point
//     per thread, the ends of the range included), a cell h of 2 / 127^4 < 1e-8 (3D) or
//     pi / 127^4 (2D), and then taken from the quadratic through the cell's two ends and
//     the next point of the last round (one Newton step on it from the secant's root): F
//     is smooth there, so the error is about h^3 |F^(3) / F'| / 16, far below the rounding
//     of c even for the narrowest distributions allowed, where linear interpolation (error
//     about h^2 |F''/F'| / 8) left some 1e-15.
#pragma once

#include "angle2.hpp"

namespace gfbd {

constexpr int AWG = 128;               // threads per pair
constexpr int AW_NW = AWG / 64;        // waves per pair
constexpr int ACS = 16;                // orders per regenerated chunk
constexpr int ACK = 2 * ACS;           // most orders between checkpoints
constexpr int ANCK = 6;                // checkpoints: orders 0 .. 191 (the cap needs 0 .. 161)
constexpr int ANG_ROUNDS = 4;          // rounds of the 129-way root search
constexpr int ANG2_GEO4 = 12;          // 2D geometric panels of ratio 4 on [4^-12, 1]
static_assert(ACK * ANCK >= ANG_NCAP + 2, "checkpoints must cover the series' cap");
// below this tau the series would need more than ANG_NCAP terms (R R0 / tau > 500 near
// contact) and the quadrature grows like 1 / sqrt(tau) nodes per pair
constexpr double ANG_TAU_MIN = 2e-3;

struct AngShared {
    union {
        double ck[ANCK][3][2][AWG];  // checkpoints of the J sequences, a column per thread
        struct {                     // after the nodes:
            double W[ANG_NCAP + 1];  // the coefficients w_n
            alignas(16) double S[ANG_NCAP + 2][4];  // 3D: the search's series, a row per order
        } co;
    };
    double w[AW_NW][ANG_NCAP + 1];  // per-wave partial coefficient sums; 2D: then the search's series
    double Fv[AWG];                 // F at the search points of the last round
    int hit[AW_NW];
    int hitr[2][AW_NW];             // the search's per-wave first points, alternate rounds
};
static_assert(sizeof(AngShared) <= 40960, "four workgroups must share a compute unit's LDS");

// The largest v of the wave (every lane active), the same in every lane: within each row of
// 16 lanes by DPP moves (lanes l ^ 1 and l ^ 2 by quad_perm, l ^ 4 by a row shift either way,
// l ^ 8 by row_ror:8), then over the four rows by v_readlane.
__device__ __forceinline__ int wave_max_i(int v)
{
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xf, 0xf, true));
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xf, 0xf, true));
    const int up = __builtin_amdgcn_mov_dpp(v, 0x104, 0xf, 0xf, true), down = __builtin_amdgcn_mov_dpp(v, 0x114, 0xf, 0xf, true);
    v = max(v, (threadIdx.x & 4) ? down : up);
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0x128, 0xf, 0xf, true));
    return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// 1/d from the hardware estimate refined by two Newton steps (the estimate's relative
// error e becomes e^4): within an ulp or two of the correctly rounded quotient, at a
// third of the cost of the IEEE division sequence.  d > 0 and finite here.
__device__ __forceinline__ double ang_rcp(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// Coefficient of the downward step C_{k-1} = coef * C_k / z - C_{k+1}:
// half-integer orders nu = k - 1/2 (3D): 2 nu = 2k - 1; integer orders (2D): 2k.
template <int DIM> __device__ __forceinline__ double ang_coef(int k) { return DIM == 3 ? 2.0 * k - 1.0 : 2.0 * k; }

// The distribution functions (angle3.hpp, angle2.hpp), with V_n = w_n / w_0:
// 3D F(c) = (1 + c)/2 + sum_{n=1..N} (V_n / 2) (P_{n+1}(c) - P_{n-1}(c)), rewritten as
// sum_{m=0..N+1} a_m P_m(c) with a_m = (V_{m-1} - V_{m+1}) / 2 (V_0 and V_{>N} taken as 0)
// plus 1/2 in a_0 and a_1, and summed downward (Clenshaw) with Bonnet's recurrence
// P_{m+1} = (2m+1)/(m+1) c P_m - m/(m+1) P_{m-1}: one dependent FMA per order.  Row m of S
// holds a_m, (2m+1)/(m+1) and -(m+1)/(m+2);
// 2D F(t) = t / pi + sum_{n=1..N} a_n sin(n t), a_n = 2 V_n / (n pi), summed upward with
// the sines from their three-term recurrence.  The coefficients sit in LDS, the same
// address in every lane; eight rows are loaded before they are used, so that the loads
// overlap.
__device__ __forceinline__ double ang_cdf_n(const double (*S)[4], int M, double c)
{
    double b1 = 0.0, b2 = 0.0;
    int k = M;
    for (; k >= 8; k -= 8) {  // eight orders: their rows' loads first, then the recurrence
        double a[8], p[8], q[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            a[j] = S[k - j][0];
            p[j] = S[k - j][1];
            q[j] = S[k - j][2];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const double b = fma(p[j] * c, b1, fma(q[j], b2, a[j]));
            b2 = b1;
            b1 = b;
        }
    }
    for (; k >= 1; --k) {
        const double b = fma(S[k][1] * c, b1, fma(S[k][2], b2, S[k][0]));
        b2 = b1;
        b1 = b;
    }
    return fma(c, b1, fma(-0.5, b2, S[0][0]));
}

__device__ __forceinline__ double ang2_cdf_n(const double *a, int N, double t)
{
    double s, cs;
    sincos(t, &s, &cs);
    const double c2 = 2.0 * cs;
    double sm = 0.0, acc = t * (1.0 / PI_D);  // sin((n-1) t), sin(n t) at n = 1
    int n = 1;
    for (; n + 7 <= N; n += 8) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = a[n + j];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            acc = fma(v[j], s, acc);
            const double sn = fma(c2, s, -sm);
            sm = s;
            s = sn;
        }
    }
    for (; n <= N; ++n) {
        acc = fma(a[n], s, acc);
        const double sn = fma(c2, s, -sm);
        sm = s;
        s = sn;
    }
    return acc;
}

// Weights of the Neumann series of J_0, Y_0 and Y_1 in J_k(z), k = 0 .. ANG_KMAX - 1
// (Abramowitz & Stegun 9.1.88 and 9.1.89, and the derivative of 9.1.89 with Y_0' = -Y_1,
// J_k' = (J_{k-1} - J_{k+1}) / 2):
//   1   = J_0 + 2 sum_{k>=1} J_{2k},
//   Y_0 = (2/pi) [(log(z/2) + gamma) J_0 - 2 sum_{k>=1} (-1)^k J_{2k} / k],
//   Y_1 = (2/pi) [(log(z/2) + gamma) J_1 - J_0 / z + sum_{j>=0} d_{2j+1} J_{2j+1}],
//         d_1 = -1, d_{2j+1} = (-1)^{j+1} (1/j + 1/(j+1)).
// The Miller sweep of a 2D node accumulates the three sums beside the recurrence, so the
// normalisation and the Y recurrences' starting values need no Bessel function call.
// w[k]: (-1)^{k/2} / (k/2) at even k >= 2 (0 at k = 0), d_k at odd k.  A node's sweep
// starts below ANG_KMAX: its arguments are at most (1 + 40 sqrt(tau)) sqrt(40 / tau) <= 395
// for tau >= ANG_TAU_MIN, so the start z + 8 z^{1/3} + 16 stays below 470.
constexpr int ANG_KMAX = 1024;
struct NeumannTable {
    double w[ANG_KMAX];
    constexpr NeumannTable() : w()
    {
        for (int k = 0; k < ANG_KMAX; ++k) {
            if (k % 2 == 0) {
                const int h = k / 2;
                w[k] = h == 0 ? 0.0 : (h % 2 == 0 ? 1.0 : -1.0) / h;
            } else {
                const int j = (k - 1) / 2;
                w[k] = j == 0 ? -1.0 : (j % 2 == 1 ? 1.0 : -1.0) * (1.0 / j + 1.0 / (j + 1));
            }
        }
    }
};
__constant__ constexpr NeumannTable ANG_NEU{};
constexpr double EULER_GAMMA = 0.57721566490153286061;

// One step of the transposing reduction: lanes that differ in bit `m` exchange the half
// of their n values the other keeps, and add.  Afterwards lanes with bit m clear hold
// the lower half, lanes with it set the upper half.
// Lane exchanges of the reduction, in the VALU rather than through the LDS crossbar:
// v_permlane32_swap exchanges lanes 32-63 of a with lanes 0-31 of b, v_permlane16_swap the odd
// rows of a with the even rows of b (rows of 16 lanes); DPP moves read lane l ^ 8 (row_ror:8),
// l + 4 and l - 4 within a row (row_shl:4, row_shr:4) and l ^ 2, l ^ 1 (quad_perm).
__device__ __forceinline__ void ang_swap(double &a, double &b, bool rows16)
{
    const unsigned long long x = (unsigned long long)__double_as_longlong(a), y = (unsigned long long)__double_as_longlong(b);
    const unsigned xl = (unsigned)x, xh = (unsigned)(x >> 32), yl = (unsigned)y, yh = (unsigned)(y >> 32);
    unsigned al, ah, bl, bh;
    if (rows16) {
        const auto lo = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
        al = lo[0]; bl = lo[1]; ah = hi[0]; bh = hi[1];
    } else {
        const auto lo = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
        al = lo[0]; bl = lo[1]; ah = hi[0]; bh = hi[1];
    }
    a = __longlong_as_double((long long)(((unsigned long long)ah << 32) | al));
    b = __longlong_as_double((long long)(((unsigned long long)bh << 32) | bl));
}

template <int CTRL> __device__ __forceinline__ double ang_dpp(double v)
{
    const unsigned long long x = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)x, CTRL, 0xf, 0xf, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(x >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// v of lane l ^ m, m = 8, 4, 2 or 1 (every lane of the wave active)
template <int m> __device__ __forceinline__ double ang_xor(double v, int lane)
{
    static_assert(m == 8 || m == 4 || m == 2 || m == 1, "row-local exchanges only");
    if constexpr (m == 8) return ang_dpp<0x128>(v);
    else if constexpr (m == 4) {
        const double up = ang_dpp<0x104>(v), down = ang_dpp<0x114>(v);
        return (lane & 4) ? down : up;
    } else if constexpr (m == 2) return ang_dpp<0x4E>(v);
    else return ang_dpp<0xB1>(v);
}

// One fold of n values on lane bit m: the lane keeps the half of its values selected by
// that bit and adds its partner's (lane ^ m) copy of the same half.
template <int n, int m>
__device__ __forceinline__ void ang_fold(double *v, int lane)
{
    if constexpr (m == 32 || m == 16) {
        // after the swap a lane holds its kept value in one operand and its partner's in the
        // other: the sum of the two, in either order the same
#pragma unroll
        for (int k = 0; k < n / 2; ++k) {
            double a = v[k], b = v[k + n / 2];
            ang_swap(a, b, m == 16);
            v[k] = a + b;
        }
    } else {
        const bool up = lane & m;
#pragma unroll
        for (int k = 0; k < n / 2; ++k) {
            const double lo = v[k], hi = v[k + n / 2];
            const double give = up ? lo : hi, keep = up ? hi : lo;
            v[k] = keep + ang_xor<m>(give, lane);
        }
    }
}

// All folds of a chunk of `top` values: on lane bits 32, 16, .. (one per halving); returns
// the order the lane then holds, its folded bits read high to low.
template <int n, int top>
__device__ __forceinline__ int ang_fold_all(double *v, int lane)
{
    if constexpr (n == 1) {
        return 0;
    } else {
        constexpr int m = 32 * n / top;  // lane bit of this fold
        ang_fold<n, m>(v, lane);
        return ((lane & m) ? n / 2 : 0) + ang_fold_all<n / 2, top>(v, lane);
    }
}

// The terms of one node (x, weight g) for orders 0 .. N: each order's sum over the wave
// is added to wrow[order].  Uniform over the workgroup: N; over the wave: every call.
template <int DIM>
__device__ __forceinline__ void ang_node(double x, double g, bool live, double R, double R0, int N, double *wrow,
                                         AngShared &sh)
{
    const int tid = threadIdx.x, lane = lane_id();
    // stored indices k: 3D C_k = J_{k-1/2}, k = 0 .. N + 1; 2D J_k, k = 0 .. N
    const int KT = DIM == 3 ? N + 2 : N + 1;
    const double z[3] = {x, R * x, R0 * x};
    double inv[3], a[3], b[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        inv[j] = 1.0 / z[j];
        a[j] = 1.0;  // C_m
        b[j] = 0.0;  // C_{m+1}
    }
    // this node's indices: up to 8 z^{1/3} + 8 orders beyond the largest argument's turning
    // point, where every term has fallen below 1e-28 of w_0
    const double zm = fmax(z[0], fmax(z[1], z[2]));
    const int zc = (int)ceil(zm + 8.0 * (double)cbrtf((float)zm));  // a bound: binary32 serves
    const int kt = live ? min(KT, zc + 9) : 0;
    const int klast = kt - 1;                                 // last index this node uses
    // 16-order chunks, and checkpoints at every chunk when six of them cover the wave's
    // orders, else at every other chunk (uniform)
    const int nch = __builtin_amdgcn_readfirstlane(wave_max_i((max(kt, 1) + ACS - 1) / ACS));
    const int spc = nch <= ANCK ? 1 : 2;  // chunks per checkpoint
    const int nck = (nch + spc - 1) / spc;
    const int top = ACS * spc * nck;      // index of the highest checkpoint
    // first sweep, from above both the node's last index and the turning point (2D: from the
    // wave's highest start, so the index is uniform and the series weights are scalar loads)
    int m = max(klast, zc) + 8;
    if (m < top) m = top;
    if constexpr (DIM == 2) m = __builtin_amdgcn_readfirstlane(wave_max_i(m));
    // 2D: the Neumann sums (even indices: 2 C_k and w_k C_k; odd: w_k C_k), from C_m = 1
    double sn[3] = {0.0, 0.0, 0.0}, se[3] = {0.0, 0.0, 0.0}, so[3] = {0.0, 0.0, 0.0};
    if constexpr (DIM == 2) {
        const double wm = ANG_NEU.w[m];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (m & 1) {
                so[j] = wm;
            } else {
                sn[j] = 2.0;
                se[j] = wm;
            }
        }
    }
    for (int k = m; k > top; --k) {  // nothing kept yet: rescale by selects, no branch
        const double cf = ang_coef<DIM>(k);
        const double wk = DIM == 2 ? ANG_NEU.w[k - 1] : 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double c = cf * inv[j] * a[j] - b[j];
            const bool big = fabs(c) > 1e250;
            b[j] = big ? a[j] * 1e-250 : a[j];
            a[j] = big ? c * 1e-250 : c;
            if constexpr (DIM == 2) {
                const double f = big ? 1e-250 : 1.0;
                if ((k - 1) & 1) {
                    sn[j] *= f;
                    se[j] *= f;
                    so[j] = so[j] * f + wk * a[j];
                } else {
                    sn[j] = sn[j] * f + 2.0 * a[j];
                    se[j] = se[j] * f + wk * a[j];
                    so[j] *= f;
                }
            }
        }
    }
    for (int ch = spc * nck - 1; ch >= 0; --ch) {
        const int s = ch / spc;
        if (ch % spc == spc - 1) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                sh.ck[s][j][0][tid] = a[j];  // C at index ACS spc (s + 1)
                sh.ck[s][j][1][tid] = b[j];  // and the one above
            }
        }
        const double base = 2.0 * ACS * ch;
#pragma unroll
        for (int i = ACS - 1; i >= 0; --i) {
            const double cf = base + (DIM == 3 ? 2.0 * i + 1.0 : 2.0 * i + 2.0);  // of index ACS ch + i + 1
            double c[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                c[j] = cf * inv[j] * a[j] - b[j];
                b[j] = a[j];
                a[j] = c[j];
                if constexpr (DIM == 2) {
                    const double wk = ANG_NEU.w[ACS * ch + i];
                    if (i & 1) {
                        so[j] += wk * c[j];
                    } else {
                        sn[j] += 2.0 * c[j];
                        se[j] += wk * c[j];
                    }
                }
            }
            if (fmax(fabs(c[0]), fmax(fabs(c[1]), fabs(c[2]))) > 1e250) {  // rare: one test for the three
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    if (!(fabs(c[j]) > 1e250)) continue;
                    a[j] *= 1e-250;  // rescale, including the checkpoints and sums kept so far
                    b[j] *= 1e-250;
                    sn[j] *= 1e-250;
                    se[j] *= 1e-250;
                    so[j] *= 1e-250;
                    for (int t = s; t < nck; ++t) {
                        sh.ck[t][j][0][tid] *= 1e-250;
                        sh.ck[t][j][1][tid] *= 1e-250;
                    }
                }
            }
        }
    }
    // a = C_0, b = C_1: normalisation and the Y recurrences' starting values
    double lam[3], y0[3], ym[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if constexpr (DIM == 3) {
            const double M = fmax(fabs(a[j]), fabs(b[j])), a0 = a[j] / M, a1 = b[j] / M;
            double s0, c0;
            sincos(z[j], &s0, &c0);
            const double sc = sqrt(2.0 / (PI_D * z[j]));
            lam[j] = sc * (s0 * a1 + c0 * a0) / (a1 * a1 + a0 * a0) / M;
            ym[j] = sc * s0;   // Y_{-1/2}
            y0[j] = -sc * c0;  // Y_{1/2}
        } else {
            const double l = 1.0 / (sn[j] - a[j]);  // the sum counted C_0 twice
            const double J0 = l * a[j], J1 = l * b[j], L = log(0.5 * z[j]) + EULER_GAMMA;
            lam[j] = l;
            y0[j] = (2.0 / PI_D) * (L * J0 - 2.0 * l * se[j]);             // Y_0
            ym[j] = -(2.0 / PI_D) * (L * J1 - J0 * inv[j] + l * so[j]);  // Y_{-1} = -Y_1
        }
    }
    // J_{nu-1}(x) of the first order: 3D J_{-1/2} = lam C_0; 2D J_{-1} = -J_1
    double jm = DIM == 3 ? lam[0] * a[0] : -lam[0] * b[0];
    bool dead = !live;
    for (int ch = 0; ch < spc * nck; ++ch) {
        if (__ballot(!dead) == 0) break;  // every node of the wave is past its last order
        // the chunk, normalised (the recurrence is linear, so scaling its two starting values
        // scales every value it gives); a lower chunk of a checkpoint runs through the upper
        const int s = ch / spc, K = ACS * spc * (s + 1);
        double v[3][ACS];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double aa = lam[j] * sh.ck[s][j][0][tid], bb = lam[j] * sh.ck[s][j][1][tid];
#pragma unroll 1
            for (int k = K; k > ACS * (ch + 1); --k) {
                const double c = ang_coef<DIM>(k) * inv[j] * aa - bb;
                bb = aa;
                aa = c;
            }
            const double base = 2.0 * ACS * ch;
#pragma unroll
            for (int i = ACS - 1; i >= 0; --i) {
                const double cf = base + (DIM == 3 ? 2.0 * i + 1.0 : 2.0 * i + 2.0);  // of index ACS ch + i + 1
                const double c = cf * inv[j] * aa - bb;
                bb = aa;
                aa = c;
                v[j][i] = c;  // J at index ACS ch + i
            }
        }
        const int k0 = ACS * ch;                  // index of v[.][0]
        const int nn0 = k0 - (DIM == 3 ? 1 : 0);  // its series order
        const double dn0 = (double)nn0;
        double t[ACS];
#pragma unroll
        for (int i = 0; i < ACS; ++i) {
            const int nn = nn0 + i;
            const double dn = dn0 + i;
            t[i] = 0.0;
            if (nn < 0 || nn > N) continue;  // uniform
            if (k0 + i > klast || fabs(y0[0]) > 0x1p500) dead = true;
            const double jx = v[0][i];
            if (!dead) {
                // F(R) F(R0) = (J(Rx) A - Y(Rx) B)(J(R0x) A - Y(R0x) B) / (A^2 + B^2)
                const double jr = v[1][i], jq = v[2][i];
                double Ar, Br;
                if constexpr (DIM == 3) {
                    Ar = (2.0 * dn + 2.0) * y0[0] - 2.0 * x * ym[0];
                    Br = (2.0 * dn + 2.0) * jx - 2.0 * x * jm;
                } else {
                    Ar = x * ym[0] - dn * y0[0];
                    Br = x * jm - dn * jx;
                }
                const double Aa = y0[0], Ba = jx;
                const double pr = (jr * Ar - y0[1] * Br) * ang_rcp(Ar * Ar + Br * Br) * (jq * Ar - y0[2] * Br);
                const double pa = (jr * Aa - y0[1] * Ba) * ang_rcp(Aa * Aa + Ba * Ba) * (jq * Aa - y0[2] * Ba);
                t[i] = g * (pr - pa);
            }
            jm = jx;
            const double cy = DIM == 3 ? 2.0 * dn + 1.0 : 2.0 * dn;
#pragma unroll
            for (int j = 0; j < 3; ++j) {  // Y_{nu+1} = (2 nu / z) Y_nu - Y_{nu-1}
                const double yn = cy * inv[j] * y0[j] - ym[j];
                ym[j] = y0[j];
                y0[j] = yn;
            }
        }
        // sum the chunk's orders over the wave: the folds on lane bits 5, 4, .. leave a lane
        // holding one order (its folded bits, high to low), summed over the lanes that
        // differ in the remaining low bits
        const int o = ang_fold_all<ACS, ACS>(t, lane);
        static_assert(ACS == 16, "the last two exchanges below are those of 16-order chunks");
        double v0 = t[0];
        v0 += ang_xor<2>(v0, lane);
        v0 += ang_xor<1>(v0, lane);
        const int nn = nn0 + o;
        if ((lane & (64 / ACS - 1)) == 0 && nn >= 0 && nn <= N) wrow[nn] += v0;
    }
}

// The angle of one pair, cooperatively by the whole workgroup: cos Theta (3D) or
// |theta| (2D) at the uniform u, NaN for radii beyond any encounter or not a number.
// Every thread returns the value.  Uniform: all arguments.
template <int DIM>
__device__ __forceinline__ double ang_draw_wg(double tau, double Rin, double R0in, double u, const GL16 &gl, AngShared &sh)
{
    const int tid = threadIdx.x, wv = tid >> 6;
    if (!(Rin + R0in - 2.0 <= 40.0 * sqrt(tau))) return __builtin_nan("");  // no encounter reaches that far (e^{-400})
    const double R = fmax(Rin, 1.0), R0 = fmax(R0in, 1.0);                   // below contact counts as contact
    const int N = ang_terms(R, R0, tau);
    for (int t = tid; t < AW_NW * (ANG_NCAP + 1); t += AWG) (&sh.w[0][0])[t] = 0.0;
    __syncthreads();
    // nodes: 3D equal panels on [0, X]; 2D geometric panels on [4^-12, 1], then equal ones
    const double X = sqrt(40.0 / tau), hmax = fmin(1.0, 2.0 * PI_D / (R + R0 - 1.0));
    int Q, nuni;
    double h, x1 = 0.0;
    if constexpr (DIM == 3) {
        nuni = (int)ceil(X / hmax);
        h = X / nuni;
        Q = 16 * nuni;
    } else {
        x1 = X < 1.0 ? X : 1.0;
        nuni = X > x1 ? (int)ceil((X - x1) / hmax) : 0;
        h = nuni > 0 ? (X - x1) / nuni : 0.0;
        Q = 16 * (ANG2_GEO4 + nuni);
    }
    double *wrow = sh.w[wv];
    for (int q0 = 0; q0 < Q; q0 += AWG) {  // uniform
        const int q = q0 + tid;
        const bool live = q < Q;
        const int qq = live ? q : 0, p = qq >> 4;
        double x, g;
        if constexpr (DIM == 3) {
            x = h * (p + 0.5 + 0.5 * gl.x[qq & 15]);
            g = live ? 0.5 * h * gl.w[qq & 15] * exp(-tau * x * x) * x : 0.0;
        } else {
            double lo, hi;
            if (p < ANG2_GEO4) {
                lo = ldexp(x1, 2 * (p - ANG2_GEO4));
                hi = 4.0 * lo;
            } else {
                lo = x1 + (p - ANG2_GEO4) * h;
                hi = lo + h;
            }
            const double c = 0.5 * (lo + hi), hw = 0.5 * (hi - lo);
            x = c + hw * gl.x[qq & 15];
            g = live ? hw * gl.w[qq & 15] * exp(-tau * x * x) * x : 0.0;
        }
        ang_node<DIM>(x, g, live, R, R0, N, wrow, sh);
    }
    __syncthreads();
    for (int t = tid; t <= N; t += AWG) {
        double s = 0.0;
        for (int w = 0; w < AW_NW; ++w) s += sh.w[w][t];  // in wave order
        sh.co.W[t] = s;
    }
    __syncthreads();
    // the last order whose coefficient is above 1e-17 of w_0 (the rest change F by less
    // than 1e-16), then the series the search evaluates (ang_cdf_n, ang2_cdf_n)
    const double inv0 = 1.0 / sh.co.W[0];
    int last = 0;
    for (int t = tid; t <= N; t += AWG)
        if (t > 0 && fabs(sh.co.W[t] * inv0) > 1e-17) last = t;
    last = wave_max_i(last);
    if ((tid & 63) == 0) sh.hit[wv] = last;
    __syncthreads();
    int Ne = 0;
    for (int w = 0; w < AW_NW; ++w) Ne = max(Ne, sh.hit[w]);
    const int M = DIM == 3 ? Ne + 1 : Ne;
    for (int m = tid; m <= M; m += AWG) {
        if constexpr (DIM == 3) {
            const double lo = m >= 2 ? sh.co.W[m - 1] : 0.0, hi = m + 1 <= Ne ? sh.co.W[m + 1] : 0.0;
            sh.co.S[m][0] = 0.5 * (lo - hi) * inv0 + (m <= 1 ? 0.5 : 0.0);
            sh.co.S[m][1] = (2.0 * m + 1.0) / (m + 1.0);
            sh.co.S[m][2] = -(m + 1.0) / (m + 2.0);
        } else {
            sh.w[0][m] = m > 0 ? 2.0 * sh.co.W[m] * inv0 / (m * PI_D) : 0.0;
        }
    }
    __syncthreads();
    // root of F(.) = u: F is nondecreasing; each round evaluates AWG equally spaced points
    // from lo to hi (both ends included) and keeps the cell between the last point below u
    // and the first at or above it; the last round also keeps F at the cell's ends and at
    // the next point beyond it.  The rounds' first-point flags alternate between two LDS
    // slots, so a round needs one barrier.
    double lo = DIM == 3 ? -1.0 : 0.0, hi = DIM == 3 ? 1.0 : PI_D, Flo = 0.0, Fhi = 1.0, F3 = 0.0;
    bool above = true;  // the third point lies above the cell (else below it)
    for (int it = 0; it < ANG_ROUNDS; ++it) {
        const bool last_round = it == ANG_ROUNDS - 1;
        const double d = (hi - lo) * (1.0 / (AWG - 1));
        const double c = lo + d * tid;
        const double Fc = DIM == 3 ? ang_cdf_n(sh.co.S, M, c) : ang2_cdf_n(sh.w[0], M, c);
        if (last_round) sh.Fv[tid] = Fc;
        const u64 bal = __ballot(Fc >= u);
        int *hit = sh.hitr[it & 1];
        if ((tid & 63) == 0) hit[wv] = bal ? __ffsll((unsigned long long)bal) - 1 : 64;
        __syncthreads();
        int j = AWG;  // first point at or above u
        for (int w = AW_NW - 1; w >= 0; --w)
            if (hit[w] < 64) j = 64 * w + hit[w];
        j = min(max(j, 1), AWG - 1);  // the ends bracket the root up to rounding
        const double nlo = lo + d * (j - 1), nhi = lo + d * j;
        if (last_round) {
            Flo = sh.Fv[j - 1];
            Fhi = sh.Fv[j];
            above = j + 1 < AWG;
            F3 = sh.Fv[above ? j + 1 : j - 2];
        }
        lo = nlo;
        hi = nhi;
    }
    // on the cell, t in [0, 1]: F ~ Flo + s t + q t (t - 1), q half the second difference
    // (the third point at t = 2 or t = -1); one Newton step from the secant's root
    const double s = Fhi - Flo;
    if (!(s > 0.0)) return 0.5 * (lo + hi);
    const double q = 0.5 * (above ? F3 - 2.0 * Fhi + Flo : Fhi - 2.0 * Flo + F3);
    double t = fmin(fmax((u - Flo) / s, 0.0), 1.0);
    const double g = s + q * (2.0 * t - 1.0);
    if (g > 0.0) t = fmin(fmax(t - q * t * (t - 1.0) / g, 0.0), 1.0);
    return lo + t * (hi - lo);
}

// sim_eval_angle: one workgroup per pair.
template <int DIM>
__global__ __launch_bounds__(AWG, 2) void k_angle_wg(double tau, uint64_t n, const double *__restrict__ Rv,
                                                  const double *__restrict__ R0v, const double *__restrict__ uv,
                                                  double *__restrict__ out, GL16 gl)
{
    __shared__ AngShared sh;
    for (uint64_t i = blockIdx.x; i < n; i += gridDim.x) {  // uniform
        const double v = ang_draw_wg<DIM>(tau, Rv[i], R0v[i], uv[i], gl, sh);
        if (threadIdx.x == 0) out[i] = v;
        __syncthreads();
    }
}

// AngEnt (kernels.hpp): a propagated pair of this step waiting for its angle, its
// records (post-move positions, left in place by the event kernel), the radius R''
// drawn for it and the clamped pre-step radius R0 it was drawn from; on = 0 marks an
// event that needs none (a reaction or a decay); dbg: its entry in the match log.

// Step stage after the events: the angle of every propagated pair (Sec. 3, Details)
// and its new positions.  The pre-step separation r0 = r - (d_B - d_A) comes from the
// post-move separation r and the regenerated displacements; u = U(word 0) of
// {slot A, slot B, step, ANG}; in 3D the azimuth about r0 is 2 pi U(word 1) in the
// frame b1, b2 orthogonal to r0 of Duff et al., "Building an Orthonormal Basis,
// Revisited" (JCGT 2017); in 2D word 1's top bit turns the rotation clockwise.  The
// centre of diffusion keeps its free end point (eq. Rcoo), and the pair is placed
// R'' a apart along the drawn direction.  A pre-step separation of length zero, or
// radii beyond any encounter, keep the free end point's direction.
// One propagated pair (event e of the step): its angle and new positions, drawn by the whole
// workgroup.  Uniform: every argument.
template <int DIM, class T, int PM, bool BATCH>
__device__ __forceinline__ void ang_place(const Params &P, Rec<T> *__restrict__ rec, const AngEnt &e, u32 step, DbgMatch *dbg,
                                          const GL16 &gl, AngShared &sh)
{
#pragma clang fp contract(off)
    double v;
    {
        const u32 sa = meta_slot(rec_meta(rec[e.ia])), sb = meta_slot(rec_meta(rec[e.ib]));
        const Params &Q = rep_params<BATCH>(P, sa);
        const uint4 r = philox(sa - Q.slot_base, sb - Q.slot_base, step - Q.step_base, TAG_ANG, Q.key);
        v = ang_draw_wg<DIM>(Q.tau, e.Rpp, e.R0, u01(r.x), gl, sh);
    }
    if (threadIdx.x == 0) {  // the records again: nothing held across the draw
        Rec<T> ra = rec[e.ia], rb = rec[e.ib];
        const u32 sa = meta_slot(rec_meta(ra)), sb = meta_slot(rec_meta(rb));
        const Params &Q = rep_params<BATCH>(P, sa);
        const u32 la = sa - Q.slot_base, lb = sb - Q.slot_base, ls = step - Q.step_base;
        const uint4 r = philox(la, lb, ls, TAG_ANG, Q.key);
        const double xa[3] = {(double)ra.x, (double)ra.y, (double)ra.z};
        const double xb[3] = {(double)rb.x, (double)rb.y, (double)rb.z};
        double dA[3], dB[3];
        displacement<DIM, T, PM>(Q, la, SP_A, ls, dA);
        displacement<DIM, T, PM>(Q, lb, SP_B, ls, dB);
        double rv[3] = {0.0, 0.0, 0.0}, r0v[3] = {0.0, 0.0, 0.0}, rn = 0.0, n0 = 0.0;
        for (int d = 0; d < DIM; ++d) {
            rv[d] = min_image_d(xb[d] - xa[d], Q.L[d], Q.Lh[d]);
            r0v[d] = rv[d] - (dB[d] - dA[d]);
            rn += rv[d] * rv[d];
            n0 += r0v[d] * r0v[d];
        }
        rn = sqrt(rn);
        n0 = sqrt(n0);
        const double c = n0 > 0.0 ? (DIM == 3 ? v : cos(v)) : __builtin_nan("");
        double ev[3] = {0.0, 0.0, 0.0};
        if (!(c == c)) {  // the free end point's direction
            for (int d = 0; d < DIM; ++d) ev[d] = rn > 0.0 ? rv[d] / rn : (d == DIM - 1 ? 1.0 : 0.0);
        } else {
            double nv[3] = {0.0, 0.0, 0.0};
            for (int d = 0; d < DIM; ++d) nv[d] = r0v[d] / n0;
            if constexpr (DIM == 3) {
                const double sg = nv[2] >= 0.0 ? 1.0 : -1.0, aa = -1.0 / (sg + nv[2]), bb = nv[0] * nv[1] * aa;
                const double b1[3] = {1.0 + sg * nv[0] * nv[0] * aa, sg * bb, -sg * nv[0]};
                const double b2[3] = {bb, sg + nv[1] * nv[1] * aa, -nv[1]};
                const double sn = sqrt(fmax(0.0, 1.0 - c * c));
                double sp, cp;
                sincos_turn<T>(u01(r.y), &sp, &cp);
                for (int d = 0; d < 3; ++d) ev[d] = c * nv[d] + sn * (cp * b1[d] + sp * b2[d]);
            } else {
                const double sn = (r.y >> 31 ? -1.0 : 1.0) * sqrt(fmax(0.0, 1.0 - c * c));
                ev[0] = c * nv[0] - sn * nv[1];
                ev[1] = sn * nv[0] + c * nv[1];
            }
        }
        T na[3] = {0, 0, 0}, nb[3] = {0, 0, 0};
        for (int d = 0; d < DIM; ++d) {
            const double cen = xa[d] + Q.fA * rv[d];
            na[d] = wrap_store<T>(cen - Q.fA * Q.a * e.Rpp * ev[d], Q.L[d]);
            nb[d] = wrap_store<T>(cen + Q.fB * Q.a * e.Rpp * ev[d], Q.L[d]);
        }
        ra.x = na[0]; ra.y = na[1]; ra.z = na[2];
        rb.x = nb[0]; rb.y = nb[1]; rb.z = nb[2];
        rec[e.ia] = ra;
        rec[e.ib] = rb;
        if (P.debug && e.dbg < P.dbg_cap) dbg[e.dbg].cos_theta = c;
    }
}

template <int DIM, class T, int PM, bool BATCH>
__global__ __launch_bounds__(AWG, 2) void k_angles(const Params *__restrict__ Pd, Rec<T> *__restrict__ rec,
                                                const AngEnt *__restrict__ ang, const Counters *__restrict__ C,
                                                DbgMatch *dbg, GL16 gl)
{
    __shared__ AngShared sh;
    const Params &P = *Pd;
    const u32 n = min(C->n_ev, P.cap);
    const u32 step = C->step;
    for (u32 w = blockIdx.x; w < n; w += gridDim.x) {  // uniform
        const AngEnt e = ang[w];
        if (!e.on) continue;
        ang_place<DIM, T, PM, BATCH>(P, rec, e, step, dbg, gl, sh);
        __syncthreads();  // sh is reused by the next pair
    }
}

// Event w in the wave form (LANE false: every lane of the wave active; the counts and the
// hand-off in lane 0) or the lane form (one event per lane).
template <int DIM, class T, int NC, bool BATCH, bool LANE = false>
__device__ __forceinline__ EvCount ev_wave(const Params &P, Rec<T> *__restrict__ rec, const PairEnt *__restrict__ list,
                                           const CandEnt *__restrict__ cand, const u32 *__restrict__ ev, u32 *__restrict__ partner,
                                           u32 step, Counters *C, DbgMatch *dbg_m, DbgDiss *dbg_d, u32 w, AngEnt *g)
{
    const u32 e = ev[w];
    if (e & EV_DECAY) {
        const u32 i = e & ~EV_DECAY;
        return ev_decay<DIM, T, NC, LANE>(ev_params<BATCH>(P, rec, i), rec, i, partner, step, C, dbg_d);
    }
    return ev_match<DIM, T, NC, LANE>(rep_params<BATCH>(P, cand[e].a_slot), rec, list[e].a_idx, list[e].b_idx, cand[e].R0,
                                      partner, step, C, dbg_m, g);
}

// A hand-off that this workgroup wrote to device memory before its last barrier, read
// with vector loads (a scalar load could see a line cached before the write).
__device__ __forceinline__ AngEnt ang_load(const AngEnt *a)
{
    AngEnt e;
    e.ia = __hip_atomic_load(&a->ia, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    e.ib = __hip_atomic_load(&a->ib, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    e.on = __hip_atomic_load(&a->on, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    e.dbg = __hip_atomic_load(&a->dbg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    e.Rpp = __hip_atomic_load(&a->Rpp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    e.R0 = __hip_atomic_load(&a->R0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return e;
}

// The events of the step and the angles of their propagated pairs in one launch (a 3D step
// whose pairs draw angles): one workgroup per event.  Its first wave runs the event in the
// wave form of k_events (the same draws), hands the pair to the workgroup through LDS,
// and a propagated pair then takes its angle as in k_angles.  With fewer workgroups than
// events, a workgroup runs its events first and then their angles.  Records of different
// events are disjoint, so the workgroups share nothing; a pair's records are written and
// read again within its workgroup only.  This saves the second launch and the angle
// stage's reloading of the event list.
template <int DIM, class T, int NC, int PM, bool BATCH>
__global__ __launch_bounds__(AWG, 2) void k_events_angles(const Params *__restrict__ Pd, Rec<T> *__restrict__ rec,
                                                       const PairEnt *__restrict__ list, const CandEnt *__restrict__ cand,
                                                       const u32 *__restrict__ ev, u32 *__restrict__ partner, Counters *C,
                                                       DbgMatch *dbg_m, DbgDiss *dbg_d, AngEnt *ang, GL16 gl)
{
    __shared__ AngShared sh;
    __shared__ AngEnt hand;
    __shared__ u32 st[EV_ST];  // the wave form's counts (lane 0 of the first wave), kept out of registers
    const Params &P = *Pd;
    const u32 step = C->step;
    const u32 n = min(C->n_ev, P.cap);
    if (blockIdx.x >= n) return;  // no event for this workgroup (uniform): nothing to count either
    if (threadIdx.x == 0)
        for (int k = 0; k < EV_ST; ++k) st[k] = 0;
    if (n <= gridDim.x) {  // one event per workgroup, handed over in LDS (uniform)
        const u32 w = blockIdx.x;
        if (threadIdx.x < 64) {
            AngEnt g;
            g.on = 0;
            const EvCount c = ev_wave<DIM, T, NC, BATCH>(P, rec, list, cand, ev, partner, step, C, dbg_m, dbg_d, w, &g);
            if (threadIdx.x == 0) {
#pragma unroll
                for (int k = 0; k < EV_ST; ++k) st[k] += c.v[k];
                hand = g;
            }
        }
        __syncthreads();  // the records and the hand-off are written
        const AngEnt e = hand;
        if (e.on) ang_place<DIM, T, PM, BATCH>(P, rec, e, step, dbg_m, gl, sh);
    } else {
        // more events than workgroups: this workgroup's events first, one per thread (the
        // lane form: the same draws), their hand-offs in device memory, then their angles (two
        // loops rather than one, so that neither loop holds the other's invariants across
        // its body)
        __syncthreads();  // st is cleared
        for (u32 w = blockIdx.x + threadIdx.x * gridDim.x; w < n; w += AWG * gridDim.x) {
            AngEnt g;
            g.on = 0;
            const EvCount c = ev_wave<DIM, T, NC, BATCH, true>(P, rec, list, cand, ev, partner, step, C, dbg_m, dbg_d, w, &g);
#pragma unroll
            for (int k = 0; k < EV_ST; ++k)
                if (c.v[k]) atomicAdd(&st[k], c.v[k]);
            ang[w] = g;  // a decay's stays off
        }
        __syncthreads();  // the records, the hand-offs and the counts are written
        for (u32 w = blockIdx.x; w < n; w += gridDim.x) {  // uniform
            const AngEnt e = ang_load(ang + w);
            if (!e.on) continue;
            ang_place<DIM, T, PM, BATCH>(P, rec, e, step, dbg_m, gl, sh);
            __syncthreads();  // sh is reused by the next pair
        }
    }
    if (threadIdx.x == 0) {
        const int map[EV_ST] = {ST_REACT, ST_ATTEMPTS, ST_BOUND, ST_NEAR, ST_DECAY, ST_GEMINATE};
#pragma unroll
        for (int k = 0; k < EV_ST; ++k)
            if (st[k]) atomicAdd((unsigned long long *)&C->stats[map[k]], (unsigned long long)st[k]);
    }
}

} // namespace gfbd
