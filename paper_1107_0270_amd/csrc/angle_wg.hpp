// The angular propagator at step size: one workgroup of 256 threads per pair.
//
// After a non-reactive encounter the pair's new separation makes an angle Theta with
// its pre-step separation drawn from J (G_ref - G_abs) given the new radius (Sec. 3,
// Details, second item of the propagation; the series of eqs. genericGF3D and
// genericGF, the Bessel recurrences of eq. 3termBessel).  The series, its quadrature
// and the distribution functions are those of angle3.hpp (3D) and angle2.hpp (2D);
// what differs is how the work is laid out:
//
//   - the pair's quadrature nodes are spread over the workgroup, one node per thread
//     (more than 256 nodes: batches of 256), so a pair's latency is about that of one
//     node rather than of a wave's share of nodes;
//   - the Bessel sequence J of a node comes from the downward recurrence, which yields
//     it highest order first while the products need it lowest order first.  Instead
//     of storing it per thread (per-lane scratch memory), the first sweep keeps the
//     pair (J_k, J_{k+1}) at every eighth order k in registers (checkpoints), and the
//     second pass regenerates each chunk of eight orders downward from its checkpoint,
//     then consumes it upward beside the upward recurrence of Y.  Rescaling during the
//     first sweep scales the checkpoints already kept, so every value is the same
//     solution of the recurrence up to one common factor, removed by the normalisation
//     to the elementary J_{-1/2}, J_{1/2} (3D) or to J_0, J_1 (2D).  This covers
//     N <= ANG_FAST_N terms; pairs with more (small tau, far pairs) keep the stored
//     sequence;
//   - the per-order sums are reduced over each wave in a fixed order and added into
//     the wave's own row of LDS; the rows are summed in wave order at the end, so the
//     coefficients, and the draw, do not depend on timing;
//   - the root of F(.) = u is found by seven rounds of a 257-way search (one point per
//     thread), an interval of 2 / 257^7 < 3e-17 (3D) or pi / 257^7 (2D).
#pragma once

#include "angle2.hpp"

namespace gfbd {

constexpr int AWG = 256;               // threads per pair
constexpr int AW_NW = AWG / 64;        // waves per pair
constexpr int ACS = 8;                 // orders per regenerated chunk
constexpr int ANCK = 9;                // checkpoints kept in registers
constexpr int ANG_FAST_N = ACS * ANCK - 2;  // most terms of the register form (orders 0 .. 71 stored)
// below this tau the series would need more than ANG_NCAP terms (R R0 / tau > 500 near
// contact) and the quadrature grows like 1 / sqrt(tau) nodes per pair
constexpr double ANG_TAU_MIN = 2e-3;

struct AngShared {
    double w[AW_NW][ANG_NCAP + 1];  // per-wave partial coefficient sums
    double W[ANG_NCAP + 1];         // the coefficients w_n
    int hit[AW_NW];
};

// Coefficient of the downward step C_{k-1} = coef * C_k / z - C_{k+1}:
// half-integer orders nu = k - 1/2 (3D): 2 nu = 2k - 1; integer orders (2D): 2k.
template <int DIM> __device__ __forceinline__ double ang_coef(int k) { return DIM == 3 ? 2.0 * k - 1.0 : 2.0 * k; }

// The terms of one node (x, weight g) for orders 0 .. N, register form: each order's
// sum over the wave is added to wrow[order] by lane 0.  Uniform over the workgroup:
// N; over the wave: every call.
template <int DIM>
__device__ __forceinline__ void ang_node_fast(double x, double g, bool live, double R, double R0, int N, double *wrow)
{
    const int lane = lane_id();
    // stored indices k: 3D C_k = J_{k-1/2}, k = 0 .. N + 1; 2D J_k, k = 0 .. N
    const int KT = DIM == 3 ? N + 2 : N + 1;
    const int nck = (KT + ACS - 1) / ACS;  // <= ANCK
    const double z[3] = {x, R * x, R0 * x};
    double inv[3], a[3], b[3];
    double cka[3][ANCK], ckb[3][ANCK];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        inv[j] = 1.0 / z[j];
        a[j] = 1.0;  // C_m
        b[j] = 0.0;  // C_{m+1}
#pragma unroll
        for (int s = 0; s < ANCK; ++s) cka[j][s] = ckb[j][s] = 0.0;
    }
    // first sweep, from above both the last order and the turning point (as in angle3.hpp)
    const double zm = fmax(z[0], fmax(z[1], z[2]));
    const int zc = (int)ceil(zm + 8.0 * cbrt(zm));
    int m = (KT - 1 > zc ? KT - 1 : zc) + 8;
    if (m < ACS * nck) m = ACS * nck;
    for (int k = m; k > ACS * nck; --k) {
        const double cf = ang_coef<DIM>(k);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double c = cf * inv[j] * a[j] - b[j];
            b[j] = a[j];
            a[j] = c;
            if (fabs(c) > 1e250) {
                a[j] *= 1e-250;
                b[j] *= 1e-250;
            }
        }
    }
#pragma unroll
    for (int s = ANCK - 1; s >= 0; --s) {
        if (s < nck) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                cka[j][s] = a[j];  // C at order ACS (s + 1)
                ckb[j][s] = b[j];  // and ACS (s + 1) + 1
            }
#pragma unroll
            for (int i = ACS - 1; i >= 0; --i) {
                const double cf = ang_coef<DIM>(ACS * s + i + 1);
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const double c = cf * inv[j] * a[j] - b[j];
                    b[j] = a[j];
                    a[j] = c;
                    if (fabs(c) > 1e250) {  // rescale, including the checkpoints kept so far
                        a[j] *= 1e-250;
                        b[j] *= 1e-250;
#pragma unroll
                        for (int t = s; t < ANCK; ++t) {
                            cka[j][t] *= 1e-250;
                            ckb[j][t] *= 1e-250;
                        }
                    }
                }
            }
        }
    }
    // a = C_0, b = C_1: normalisation and the Y recurrences' starting values
    double lam[3], y0[3], ym[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double M = fmax(fabs(a[j]), fabs(b[j])), a0 = a[j] / M, a1 = b[j] / M;
        if constexpr (DIM == 3) {
            double s0, c0;
            sincos(z[j], &s0, &c0);
            const double sc = sqrt(2.0 / (PI_D * z[j]));
            lam[j] = sc * (s0 * a1 + c0 * a0) / (a1 * a1 + a0 * a0) / M;
            ym[j] = sc * s0;   // Y_{-1/2}
            y0[j] = -sc * c0;  // Y_{1/2}
        } else {
            double j0z, j1z, y0z, y1z;
            ang_bessel01(z[j], &j0z, &j1z, &y0z, &y1z);
            lam[j] = (j0z * a0 + j1z * a1) / (a0 * a0 + a1 * a1) / M;
            y0[j] = y0z;   // Y_0
            ym[j] = -y1z;  // Y_{-1} = -Y_1
        }
    }
    // J_{nu-1}(x) of the first order: 3D J_{-1/2} = lam C_0; 2D J_{-1} = -J_1
    double jm = DIM == 3 ? lam[0] * a[0] : -lam[0] * b[0];
    bool dead = !live;
#pragma unroll
    for (int s = 0; s < ANCK; ++s) {
        if (s < nck && __ballot(!dead) != 0) {  // uniform over the wave
            double v[3][ACS];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double aa = cka[j][s], bb = ckb[j][s];
#pragma unroll
                for (int i = ACS - 1; i >= 0; --i) {
                    const double c = ang_coef<DIM>(ACS * s + i + 1) * inv[j] * aa - bb;
                    bb = aa;
                    aa = c;
                    v[j][i] = c;  // C at order ACS s + i
                }
            }
#pragma unroll
            for (int i = 0; i < ACS; ++i) {
                const int k = ACS * s + i;
                const int nn = DIM == 3 ? k - 1 : k;  // the series order this index serves
                if (nn < 0 || nn > N) continue;      // uniform
                if (fabs(y0[0]) > 0x1p500) dead = true;
                const double jx = lam[0] * v[0][i];
                double term = 0.0;
                if (!dead) {
                    // F(R) F(R0) = (J(Rx) A - Y(Rx) B)(J(R0x) A - Y(R0x) B) / (A^2 + B^2)
                    const double jr = lam[1] * v[1][i], jq = lam[2] * v[2][i];
                    double Ar, Br;
                    if constexpr (DIM == 3) {
                        Ar = (2.0 * nn + 2.0) * y0[0] - 2.0 * x * ym[0];
                        Br = (2.0 * nn + 2.0) * jx - 2.0 * x * jm;
                    } else {
                        Ar = x * ym[0] - nn * y0[0];
                        Br = x * jm - nn * jx;
                    }
                    const double Aa = y0[0], Ba = jx;
                    const double pr = (jr * Ar - y0[1] * Br) / (Ar * Ar + Br * Br) * (jq * Ar - y0[2] * Br);
                    const double pa = (jr * Aa - y0[1] * Ba) / (Aa * Aa + Ba * Ba) * (jq * Aa - y0[2] * Ba);
                    term = g * (pr - pa);
                }
                jm = jx;
                const double sum = wave_allsum(term);
                if (lane == 0) wrow[nn] += sum;
#pragma unroll
                for (int j = 0; j < 3; ++j) {  // Y_{nu+1} = (2 nu / z) Y_nu - Y_{nu-1}
                    const double yn = (DIM == 3 ? 2.0 * nn + 1.0 : 2.0 * nn) * inv[j] * y0[j] - ym[j];
                    ym[j] = y0[j];
                    y0[j] = yn;
                }
            }
        }
    }
}

// The same terms from a stored sequence (per-lane memory), for pairs with more terms
// than the register form holds.
template <int DIM>
__device__ __noinline__ void ang_node_stored(double x, double g, bool live, double R, double R0, int N, double *wrow)
{
    const int lane = lane_id();
    double t[3][ANG_NCAP + 2], lam[3], y0[3], ym[3], iz[3];
    const double z[3] = {x, R * x, R0 * x};
    double jm;
    if constexpr (DIM == 3) {
        ang_miller3(N + 1, z, t, lam);
        for (int j = 0; j < 3; ++j) {
            double s0, c0;
            sincos(z[j], &s0, &c0);
            const double s = sqrt(2.0 / (PI_D * z[j]));
            ym[j] = s * s0;
            y0[j] = -s * c0;
            iz[j] = 1.0 / z[j];
        }
        jm = lam[0] * t[0][0];
    } else {
        double j0z[3], j1z[3];
        for (int j = 0; j < 3; ++j) {
            ang_bessel01(z[j], &j0z[j], &j1z[j], &y0[j], &ym[j]);
            ym[j] = -ym[j];
            iz[j] = 1.0 / z[j];
        }
        ang_miller3_int(N, z, t, lam, j0z, j1z);
        jm = -lam[0] * t[0][1];
    }
    bool dead = !live;
    for (int nn = 0; nn <= N; ++nn) {  // uniform over the wave
        if (fabs(y0[0]) > 0x1p500) dead = true;
        if (__ballot(!dead) == 0) break;
        const int k = DIM == 3 ? nn + 1 : nn;
        const double jx = lam[0] * t[0][k];
        double term = 0.0;
        if (!dead) {
            const double jr = lam[1] * t[1][k], jq = lam[2] * t[2][k];
            double Ar, Br;
            if constexpr (DIM == 3) {
                Ar = (2.0 * nn + 2.0) * y0[0] - 2.0 * x * ym[0];
                Br = (2.0 * nn + 2.0) * jx - 2.0 * x * jm;
            } else {
                Ar = x * ym[0] - nn * y0[0];
                Br = x * jm - nn * jx;
            }
            const double Aa = y0[0], Ba = jx;
            const double pr = (jr * Ar - y0[1] * Br) / (Ar * Ar + Br * Br) * (jq * Ar - y0[2] * Br);
            const double pa = (jr * Aa - y0[1] * Ba) / (Aa * Aa + Ba * Ba) * (jq * Aa - y0[2] * Ba);
            term = g * (pr - pa);
        }
        jm = jx;
        const double sum = wave_allsum(term);
        if (lane == 0) wrow[nn] += sum;
        for (int j = 0; j < 3; ++j) {
            const double yn = (DIM == 3 ? 2.0 * nn + 1.0 : 2.0 * nn) * iz[j] * y0[j] - ym[j];
            ym[j] = y0[j];
            y0[j] = yn;
        }
    }
}

// The angle of one pair, cooperatively by the whole workgroup: cos Theta (3D) or
// |theta| (2D) at the uniform u, NaN for radii beyond any encounter or not a number.
// Every thread returns the value.  Uniform: all arguments.
template <int DIM>
__device__ double ang_draw_wg(double tau, double Rin, double R0in, double u, const GL16 &gl, AngShared &sh)
{
    const int tid = threadIdx.x, wv = tid >> 6;
    if (!(Rin + R0in - 2.0 <= 40.0 * sqrt(tau))) return __builtin_nan("");  // no encounter reaches that far (e^{-400})
    const double R = fmax(Rin, 1.0), R0 = fmax(R0in, 1.0);                   // below contact counts as contact
    const int N = ang_terms(R, R0, tau);
    for (int t = tid; t < AW_NW * (ANG_NCAP + 1); t += AWG) (&sh.w[0][0])[t] = 0.0;
    __syncthreads();
    // nodes: 3D equal panels on [0, X]; 2D geometric panels on [2^-32, 1], then equal ones
    const double X = sqrt(50.0 / tau), hmax = fmin(1.0, 2.0 * PI_D / (R + R0 - 1.0));
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
        Q = 16 * (ANG2_GEO + nuni);
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
            if (p < ANG2_GEO) {
                lo = ldexp(x1, p - ANG2_GEO);
                hi = 2.0 * lo;
            } else {
                lo = x1 + (p - ANG2_GEO) * h;
                hi = lo + h;
            }
            const double c = 0.5 * (lo + hi), hw = 0.5 * (hi - lo);
            x = c + hw * gl.x[qq & 15];
            g = live ? hw * gl.w[qq & 15] * exp(-tau * x * x) * x : 0.0;
        }
        if (N <= ANG_FAST_N) ang_node_fast<DIM>(x, g, live, R, R0, N, wrow);
        else ang_node_stored<DIM>(x, g, live, R, R0, N, wrow);
    }
    __syncthreads();
    for (int t = tid; t <= N; t += AWG) {
        double s = 0.0;
        for (int w = 0; w < AW_NW; ++w) s += sh.w[w][t];  // in wave order
        sh.W[t] = s;
    }
    __syncthreads();
    // root of F(.) = u: F is nondecreasing; each round keeps the cell between the last point
    // below u and the first at or above it
    double lo = DIM == 3 ? -1.0 : 0.0, hi = DIM == 3 ? 1.0 : PI_D;
    for (int it = 0; it < 7; ++it) {
        const double d = (hi - lo) / (AWG + 1);
        const double c = lo + d * (tid + 1);
        const bool ge = (DIM == 3 ? ang_cdf(sh.W, N, c) : ang2_cdf(sh.W, N, c)) >= u;
        const u64 bal = __ballot(ge);
        if ((tid & 63) == 0) sh.hit[wv] = bal ? __ffsll((unsigned long long)bal) - 1 : 64;
        __syncthreads();
        int j = AWG;  // first point at or above u
        for (int w = AW_NW - 1; w >= 0; --w)
            if (sh.hit[w] < 64) j = 64 * w + sh.hit[w];
        const double nlo = j == 0 ? lo : lo + d * j;
        const double nhi = j == AWG ? hi : lo + d * (j + 1);
        lo = nlo;
        hi = nhi;
        __syncthreads();
    }
    return 0.5 * (lo + hi);
}

// sim_eval_angle: one workgroup per pair.
template <int DIM>
__global__ __launch_bounds__(AWG) void k_angle_wg(double tau, uint64_t n, const double *__restrict__ Rv,
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
template <int DIM, class T, int PM, bool BATCH>
__global__ __launch_bounds__(AWG) void k_angles(const Params *__restrict__ Pd, Rec<T> *__restrict__ rec,
                                                const AngEnt *__restrict__ ang, const Counters *__restrict__ C,
                                                DbgMatch *dbg, GL16 gl)
{
#pragma clang fp contract(off)
    __shared__ AngShared sh;
    const Params &P = *Pd;
    const u32 n = min(C->n_ev, P.cap);
    const u32 step = C->step;
    for (u32 w = blockIdx.x; w < n; w += gridDim.x) {  // uniform
        const AngEnt e = ang[w];
        if (!e.on) continue;
        Rec<T> ra = rec[e.ia], rb = rec[e.ib];
        const u32 sa = meta_slot(rec_meta(ra)), sb = meta_slot(rec_meta(rb));
        const Params &Q = rep_params<BATCH>(P, sa);
        const u32 la = sa - Q.slot_base, lb = sb - Q.slot_base, ls = step - Q.step_base;
        const uint4 r = philox(la, lb, ls, TAG_ANG, Q.key);
        const double v = ang_draw_wg<DIM>(Q.tau, e.Rpp, e.R0, u01(r.x), gl, sh);
        if (threadIdx.x == 0) {
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
        __syncthreads();  // sh is reused by the next pair
    }
}

} // namespace gfbd
