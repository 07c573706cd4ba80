// Kernels of one step of the coarse-grained Green's-function BD algorithm
// (Sec. 3) on gfx950.  State: records {x, y, z, meta} kept sorted by
// (species, cell) after every step; slot-indexed side array for the reserved
// partner of each C.  All data-dependent work sizes are read from device
// counters, so a step needs no host round trip.
#pragma once

#include "common.hpp"
#include "green.hpp"

namespace gfbd {

constexpr int BLOCK = 256;
constexpr int CMAX = 8;          // candidates per A kept in registers
constexpr int SCAN_ITEMS = 16;   // keys per thread in the bin scan
constexpr int SCAN_TILE = BLOCK * SCAN_ITEMS;

__device__ __forceinline__ u32 gtid() { return blockIdx.x * BLOCK + threadIdx.x; }
__device__ __forceinline__ u32 gstride() { return gridDim.x * BLOCK; }
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// ---------------------------------------------------------------------------
// State updates: binary64 arithmetic, one rounding into the state precision,
// no FMA contraction (so each rounding is the one written).
// ---------------------------------------------------------------------------
template <class T> __device__ inline T wrap_store(double y, double L)
{
#pragma clang fp contract(off)
    if (y < 0.0) y += L;
    else if (y >= L) y -= L;
    if (!(y >= 0.0 && y < L)) {  // only for steps longer than L, which sim_create rejects
        y -= L * floor(y / L);
        if (!(y >= 0.0 && y < L)) y = 0.0;
    }
    T v = (T)y;
    if ((double)v >= L) v = (T)0;  // rounding carried it to L (L is exact in T)
    return v;
}

// Free displacement sqrt(2 D dt) N(0,1) of a slot (Sec. 3, step 1):
// Box-Muller on one Philox draw {slot, -, step, MOVE}.
template <int DIM> __device__ inline void displacement(const Params &P, u32 slot, u32 sp, u32 step, double d[3])
{
#pragma clang fp contract(off)
    const uint4 r = philox(slot, NOSLOT, step, TAG_MOVE, P.key);
    const double s = P.sd[sp];
    const double r0 = sqrt(-2.0 * log(u01(r.x))), t0 = (2.0 * PI_D) * u01(r.y);
    d[0] = s * (r0 * cos(t0));
    d[1] = s * (r0 * sin(t0));
    if (DIM == 3) {
        const double r1 = sqrt(-2.0 * log(u01(r.z))), t1 = (2.0 * PI_D) * u01(r.w);
        d[2] = s * (r1 * cos(t1));
    } else {
        d[2] = 0.0;
    }
}

template <int DIM, class T> __device__ inline Rec<T> moved(const Params &P, const Rec<T> &r, u32 meta, u32 step)
{
#pragma clang fp contract(off)
    double d[3];
    displacement<DIM>(P, meta_slot(meta), meta_sp(meta), step, d);
    Rec<T> q;
    q.x = wrap_store<T>((double)r.x + d[0], P.L[0]);
    q.y = wrap_store<T>((double)r.y + d[1], P.L[1]);
    q.z = DIM == 3 ? wrap_store<T>((double)r.z + d[2], P.L[2]) : (T)0;
    q.w = r.w;
    return q;
}

__device__ __forceinline__ int cell1(double x, double s, int n)
{
    int c = (int)floor(x * s);
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

template <int DIM, class T> __device__ inline u32 cell_of(const Params &P, const Rec<T> &q)
{
    const int cx = cell1((double)q.x, P.cs[0], P.nc[0]);
    const int cy = cell1((double)q.y, P.cs[1], P.nc[1]);
    const int cz = DIM == 3 ? cell1((double)q.z, P.cs[2], P.nc[2]) : 0;
    return ((u32)cz * P.nc[1] + cy) * P.nc[0] + cx;
}

// ---------------------------------------------------------------------------
// K1: move every live record and count it into its (species, cell) bucket.
// ---------------------------------------------------------------------------
template <int DIM, class T>
__global__ __launch_bounds__(BLOCK) void k_move_count(Params P, const Rec<T> *__restrict__ rec, u32 *__restrict__ rank,
                                                       u32 *__restrict__ cnt, Counters *C, u32 step)
{
    if (gtid() == 0) {
        C->n_dbg[0] = C->n_dbg[1] = C->n_dbg[2] = C->n_dbg[3] = 0;
    }
    const u32 n = C->n_rec;
    for (u32 i = gtid(); i < n; i += gstride()) {
        const Rec<T> r = rec[i];
        const u32 m = rec_meta(r), sp = meta_sp(m);
        if (sp > SP_C) continue;
        const Rec<T> q = moved<DIM, T>(P, r, m, step);
        const u32 key = sp * P.n_cells + cell_of<DIM, T>(P, q);
        rank[i] = atomicAdd(&cnt[key], 1u);
    }
}

// ---------------------------------------------------------------------------
// K2: exclusive scan of the bucket counts into bucket starts (and clear the
// counts for the next step): reduce tiles, scan tile sums, scan tiles.
// ---------------------------------------------------------------------------
__device__ inline u32 wave_incl_scan(u32 v)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const u32 t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ inline u32 block_excl_scan(u32 v, u32 *lds, u32 &total)
{
    const u32 inc = wave_incl_scan(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) lds[w] = inc;
    __syncthreads();
    u32 off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < BLOCK / 64; ++i) {
        const u32 x = lds[i];
        off += i < w ? x : 0u;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

__device__ inline u32 block_sum(u32 v, u32 *lds)
{
    u32 t;
    block_excl_scan(v, lds, t);
    return t;
}

__global__ __launch_bounds__(BLOCK) void k_scan_reduce(const u32 *__restrict__ cnt, u32 n, u32 *__restrict__ bsum)
{
    __shared__ u32 lds[BLOCK / 64];
    const u32 base = blockIdx.x * SCAN_TILE;
    u32 s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const u32 i = base + j * BLOCK + threadIdx.x;
        s += i < n ? cnt[i] : 0u;
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

__global__ __launch_bounds__(BLOCK) void k_scan_top(u32 *__restrict__ bsum, u32 nb)
{
    __shared__ u32 lds[BLOCK / 64];
    u32 carry = 0;
    for (u32 b = 0; b < nb; b += BLOCK) {
        const u32 i = b + threadIdx.x;
        const u32 v = i < nb ? bsum[i] : 0u;
        u32 tot;
        const u32 ex = block_excl_scan(v, lds, tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(BLOCK) void k_scan_down(u32 *__restrict__ cnt, u32 n, const u32 *__restrict__ bsum,
                                                      u32 *__restrict__ start, Counters *C)
{
    __shared__ u32 lds[BLOCK / 64];
    const u32 base = blockIdx.x * SCAN_TILE;
    u32 carry = bsum[blockIdx.x];
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const u32 i = base + j * BLOCK + threadIdx.x;
        const u32 v = i < n ? cnt[i] : 0u;
        u32 tot;
        const u32 ex = block_excl_scan(v, lds, tot);
        if (i < n) {
            start[i] = carry + ex;
            cnt[i] = 0u;
        }
        carry += tot;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        start[n] = carry;
        C->n_live = carry;
    }
}

// ---------------------------------------------------------------------------
// K3: write each moved record to its sorted place.
// ---------------------------------------------------------------------------
template <int DIM, class T>
__global__ __launch_bounds__(BLOCK) void k_scatter(Params P, const Rec<T> *__restrict__ rec, const u32 *__restrict__ rank,
                                                    const u32 *__restrict__ start, Rec<T> *__restrict__ out, const Counters *C,
                                                    u32 step)
{
    const u32 n = C->n_rec;
    for (u32 i = gtid(); i < n; i += gstride()) {
        const Rec<T> r = rec[i];
        const u32 m = rec_meta(r), sp = meta_sp(m);
        if (sp > SP_C) continue;
        const Rec<T> q = moved<DIM, T>(P, r, m, step);
        const u32 key = sp * P.n_cells + cell_of<DIM, T>(P, q);
        const u32 dst = start[key] + rank[i];
        if (dst < P.cap) out[dst] = q;
    }
}

// ---------------------------------------------------------------------------
// Pair geometry and encounter probability.
// ---------------------------------------------------------------------------
struct PairQ {
    double R, R0, p;
    u32 draw;
    bool cand, overlap, clamped, near;
};

__device__ __forceinline__ double min_image_d(double d, double L, double Lh)
{
    if (d > Lh) d -= L;
    else if (d < -Lh) d += L;
    return d;
}

// binary32 minimum image: the coordinate in the upper half is shifted by -L
// first, which is exact (Sterbenz), then the difference is taken.
__device__ __forceinline__ float min_image_f(float xb, float xa, float L, float Lh)
{
    const float d = xb - xa;
    if (d > Lh) return (xb - L) - xa;
    if (d < -Lh) return xb - (xa - L);
    return d;
}

// Everything about one A-B pair within r_cut (Sec. 3, steps 2-3): separation r
// after the move, separation r0 = r - (dB - dA) before it (R0 < 1 clamped to
// 1), p_enc (overlap: 1) and the Bernoulli draw {a, b, step, ENC}.
template <int DIM, class T, int PM>
__device__ inline PairQ pair_quantities(const Params &P, const Rec<T> &ra, const Rec<T> &rb, u32 sa, u32 sb,
                                        const double dA[3], u32 step)
{
#pragma clang fp contract(off)
    PairQ q;
    double dB[3];
    displacement<DIM>(P, sb, SP_B, step, dB);
    if (PM == PM_F32) {
        const float rx = min_image_f((float)rb.x, (float)ra.x, P.Lf[0], P.Lhf[0]);
        const float ry = min_image_f((float)rb.y, (float)ra.y, P.Lf[1], P.Lhf[1]);
        const float rz = DIM == 3 ? min_image_f((float)rb.z, (float)ra.z, P.Lf[2], P.Lhf[2]) : 0.0f;
        const float ox = rx - (float)(dB[0] - dA[0]), oy = ry - (float)(dB[1] - dA[1]);
        const float oz = DIM == 3 ? rz - (float)(dB[2] - dA[2]) : 0.0f;
        const float Rf = sqrtf(rx * rx + ry * ry + rz * rz) * P.inv_af;
        float R0f = sqrtf(ox * ox + oy * oy + oz * oz) * P.inv_af;
        q.clamped = R0f < 1.0f;
        if (q.clamped) R0f = 1.0f;
        q.R = Rf;
        q.R0 = R0f;
        q.overlap = Rf <= 1.0f;
        if (q.overlap) q.p = 1.0;
        else if (DIM == 3) q.p = penc3_args((Rf - 1.0f) * (R0f - 1.0f) * P.inv_tauf, (Rf + R0f - 1.0f) * P.inv_tauf, Rf * R0f * P.inv_tauf);
        else q.p = penc2(P, (double)Rf, (double)R0f);
    } else {
        double rv[3] = {0.0, 0.0, 0.0}, r2 = 0.0, r02 = 0.0;
        const double xa[3] = {(double)ra.x, (double)ra.y, (double)ra.z};
        const double xb[3] = {(double)rb.x, (double)rb.y, (double)rb.z};
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            rv[k] = min_image_d(xb[k] - xa[k], P.L[k], P.Lh[k]);
            const double o = rv[k] - (dB[k] - dA[k]);
            r2 += rv[k] * rv[k];
            r02 += o * o;
        }
        const double R = sqrt(r2) / P.a;
        double R0 = sqrt(r02) / P.a;
        q.clamped = R0 < 1.0;
        if (q.clamped) R0 = 1.0;
        q.R = R;
        q.R0 = R0;
        q.overlap = R <= 1.0;
        if (q.overlap) {
            q.p = 1.0;
        } else if (DIM == 3) {
            const double e1 = (R - 1.0) * (R0 - 1.0) / P.tau, e2 = (R + R0 - 1.0) / P.tau, e3 = R * R0 / P.tau;
            q.p = PM == PM_F64 ? penc3_args(e1, e2, e3) : (double)penc3_args((float)e1, (float)e2, (float)e3);
        } else {
            q.p = penc2(P, R, R0);
        }
    }
    q.draw = philox(sa, sb, step, TAG_ENC, P.key).x;
    q.cand = q.overlap || below(q.draw, q.p);
    q.near = !q.overlap && fabs(u01(q.draw) - q.p) < 1e-6;
    return q;
}

// Is rb within r_cut of ra?  binary32 modes test in binary32 (FP32NC with a
// widened radius, then the exact binary64 test); FP64 tests in binary64.
template <int DIM, class T, int PM> __device__ __forceinline__ bool in_range(const Params &P, const Rec<T> &ra, const Rec<T> &rb)
{
#pragma clang fp contract(off)
    if (PM == PM_F64) {
        double r2 = 0.0;
        const double xa[3] = {(double)ra.x, (double)ra.y, (double)ra.z};
        const double xb[3] = {(double)rb.x, (double)rb.y, (double)rb.z};
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const double d = min_image_d(xb[k] - xa[k], P.L[k], P.Lh[k]);
            r2 += d * d;
        }
        return r2 < P.rcut2;
    } else {
        const float dx = min_image_f((float)rb.x, (float)ra.x, P.Lf[0], P.Lhf[0]);
        const float dy = min_image_f((float)rb.y, (float)ra.y, P.Lf[1], P.Lhf[1]);
        const float dz = DIM == 3 ? min_image_f((float)rb.z, (float)ra.z, P.Lf[2], P.Lhf[2]) : 0.0f;
        const float r2f = dx * dx + dy * dy + dz * dz;
        if (PM == PM_F32) return r2f < P.rcut2f;
        if (!(r2f < P.rcut2f_wide)) return false;
        double r2 = 0.0;
        const double xa[3] = {(double)ra.x, (double)ra.y, (double)ra.z};
        const double xb[3] = {(double)rb.x, (double)rb.y, (double)rb.z};
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const double d = min_image_d(xb[k] - xa[k], P.L[k], P.Lh[k]);
            r2 += d * d;
        }
        return r2 < P.rcut2;
    }
}

// Visit every B record within r_cut of the A record ra: the B buckets of the
// 3^d cells around ra's cell (rows along x are contiguous bucket ranges).
template <int DIM, class T, int PM, class F>
__device__ inline void for_pairs(const Params &P, const Rec<T> *__restrict__ rec, const u32 *__restrict__ start, const Rec<T> &ra,
                                 F &&emit)
{
    const int cx = cell1((double)ra.x, P.cs[0], P.nc[0]);
    const int cy = cell1((double)ra.y, P.cs[1], P.nc[1]);
    const int cz = DIM == 3 ? cell1((double)ra.z, P.cs[2], P.nc[2]) : 0;
    const int nx = P.nc[0], ny = P.nc[1], nz = P.nc[2];
    const int zlo = (DIM == 3 && nz >= 3) ? -1 : 0, zhi = -zlo;
    const int ylo = ny >= 3 ? -1 : 0, yhi = -ylo;
    const u32 bbase = P.n_cells;  // B buckets follow the A buckets
    for (int oz = zlo; oz <= zhi; ++oz) {
        int z = cz + oz;
        z = z < 0 ? z + nz : (z >= nz ? z - nz : z);
        for (int oy = ylo; oy <= yhi; ++oy) {
            int y = cy + oy;
            y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
            const u32 row = bbase + ((u32)z * ny + y) * nx;
            // up to three contiguous ranges along x
            u32 r0b, r0e, r1b = 0, r1e = 0;
            if (nx < 3) {
                r0b = start[row];
                r0e = start[row + nx];
            } else if (cx >= 1 && cx <= nx - 2) {
                r0b = start[row + cx - 1];
                r0e = start[row + cx + 2];
            } else if (cx == 0) {
                r0b = start[row];
                r0e = start[row + 2];
                r1b = start[row + nx - 1];
                r1e = start[row + nx];
            } else {
                r0b = start[row + nx - 2];
                r0e = start[row + nx];
                r1b = start[row];
                r1e = start[row + 1];
            }
            for (u32 j = r0b; j < r0e; ++j) {
                const Rec<T> rb = rec[j];
                if (in_range<DIM, T, PM>(P, ra, rb)) emit(j, rb);
            }
            for (u32 j = r1b; j < r1e; ++j) {
                const Rec<T> rb = rec[j];
                if (in_range<DIM, T, PM>(P, ra, rb)) emit(j, rb);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// K5: pairs, encounter probabilities, Bernoulli draws and the A-side choice
// among several candidates (Sec. 3, Details): candidates in ascending B slot,
// pick the first k with U sum(p) <= p_1 + ... + p_k, U = {a, -, step, SELA}.
// ---------------------------------------------------------------------------
__device__ inline void block_add_stats(u32 *vals, int nv, u64 *dst, u32 *lds)
{
    for (int s = 0; s < nv; ++s) {
        const u32 t = block_sum(vals[s], lds);
        if (threadIdx.x == 0 && t) atomicAdd((unsigned long long *)&dst[s], (unsigned long long)t);
    }
}

template <int DIM, class T, int PM>
__global__ __launch_bounds__(BLOCK) void k_pairs(Params P, const Rec<T> *__restrict__ rec, const u32 *__restrict__ start,
                                                  Pick *__restrict__ picks, u32 *__restrict__ ovf, Counters *C, DbgPair *dbg,
                                                  u32 step)
{
    __shared__ u32 lds[BLOCK / 64];
    const u32 a_beg = start[0], a_end = start[P.n_cells];
    u32 st[5] = {0, 0, 0, 0, 0};  // pairs, cand, overlap, r0clamp, near
    u32 n_ovf_local = 0;
    const u32 iters = (a_end - a_beg + gstride() - 1) / gstride();
    for (u32 it = 0; it < iters; ++it) {
        const u32 ia = a_beg + it * gstride() + gtid();
        const bool active = ia < a_end;
        u32 cs[CMAX], ci[CMAX];
        double cp[CMAX];
        int m = 0;
        u32 sa = 0;
        if (active) {
            const Rec<T> ra = rec[ia];
            sa = meta_slot(rec_meta(ra));
            double dA[3];
            bool have_dA = false;
            for_pairs<DIM, T, PM>(P, rec, start, ra, [&](u32 jb, const Rec<T> &rb) {
                if (!have_dA) {
                    displacement<DIM>(P, sa, SP_A, step, dA);
                    have_dA = true;
                }
                const u32 sb = meta_slot(rec_meta(rb));
                const PairQ q = pair_quantities<DIM, T, PM>(P, ra, rb, sa, sb, dA, step);
                st[0] += 1;
                st[1] += q.cand;
                st[2] += q.overlap;
                st[3] += q.clamped;
                st[4] += q.near;
                if (P.debug) {
                    const u32 k = atomicAdd(&C->n_dbg[0], 1u);
                    if (k < P.dbg_cap) {
                        DbgPair d;
                        d.i = sa; d.j = sb; d.R = q.R; d.R0 = q.R0; d.p = q.p; d.draw = q.draw; d.cand = q.cand;
                        dbg[k] = d;
                    }
                }
                if (!q.cand) return;
                // sorted insertion by B slot, static register indexing
                if (m < CMAX) {
                    int pos = 0;
#pragma unroll
                    for (int k = 0; k < CMAX; ++k) pos += (k < m && cs[k] < sb) ? 1 : 0;
#pragma unroll
                    for (int k = CMAX - 1; k > 0; --k)
                        if (k > pos && k <= m) {
                            cs[k] = cs[k - 1];
                            ci[k] = ci[k - 1];
                            cp[k] = cp[k - 1];
                        }
#pragma unroll
                    for (int k = 0; k < CMAX; ++k)
                        if (k == pos) {
                            cs[k] = sb;
                            ci[k] = jb;
                            cp[k] = q.p;
                        }
                }
                ++m;
            });
        }
        const bool has = active && m > 0 && m <= CMAX;
        u32 pb = 0, pslot = 0;
        double pp = 0.0;
        if (has) {
            double T_ = 0.0;
#pragma unroll
            for (int k = 0; k < CMAX; ++k)
                if (k < m) T_ += cp[k];
            const double tgt = u01(philox(sa, NOSLOT, step, TAG_SELA, P.key).x) * T_;
            double acc = 0.0;
            bool found = false;
#pragma unroll
            for (int k = 0; k < CMAX; ++k)
                if (k < m && !found) {
                    acc += cp[k];
                    pb = ci[k];
                    pslot = cs[k];
                    pp = cp[k];
                    if (tgt <= acc) found = true;
                }
        }
        const u64 mask = __ballot(has);
        if (mask) {
            const int leader = __ffsll((unsigned long long)mask) - 1;
            u32 base = 0;
            if (lane_id() == leader) base = atomicAdd(&C->n_picks, (u32)__popcll(mask));
            base = __shfl(base, leader, 64);
            if (has) {
                const u32 k = base + (u32)__popcll(mask & ((1ull << lane_id()) - 1ull));
                if (k < P.cap_picks) {
                    Pick pk;
                    pk.a_idx = ia; pk.b_idx = pb; pk.a_slot = sa; pk.b_slot = pslot; pk.p = pp;
                    picks[k] = pk;
                } else {
                    atomicOr(&C->err, (u32)ERR_PICKS);
                }
            }
        }
        if (active && m > CMAX) {
            const u32 k = atomicAdd(&C->n_ovf, 1u);
            ovf[k] = ia;
            ++n_ovf_local;
        }
    }
    u32 vals[6] = {st[0], st[1], st[2], st[3], st[4], n_ovf_local};
    block_add_stats(vals, 4, &C->stats[ST_PAIRS], lds);
    u32 v2[1] = {vals[4]};
    block_add_stats(v2, 1, &C->stats[ST_NEAR], lds);
    u32 v3[1] = {vals[5]};
    block_add_stats(v3, 1, &C->stats[ST_CAND_OVERFLOW], lds);
}

// K5b: A particles with more than CMAX candidates: visit the neighbours again,
// write all candidates to a scratch list, sort it by B slot, pick.
struct OvfCand {
    u32 slot, idx;
    double p;
};

template <int DIM, class T, int PM>
__global__ __launch_bounds__(BLOCK) void k_pairs_overflow(Params P, const Rec<T> *__restrict__ rec, const u32 *__restrict__ start,
                                                           const u32 *__restrict__ ovf, OvfCand *__restrict__ cand,
                                                           Pick *__restrict__ picks, Counters *C, u32 step)
{
    const u32 n = C->n_ovf;
    for (u32 k = gtid(); k < n; k += gstride()) {
        const u32 ia = ovf[k];
        const Rec<T> ra = rec[ia];
        const u32 sa = meta_slot(rec_meta(ra));
        double dA[3];
        displacement<DIM>(P, sa, SP_A, step, dA);
        u32 m = 0;
        for_pairs<DIM, T, PM>(P, rec, start, ra, [&](u32, const Rec<T> &rb) {
            const PairQ q = pair_quantities<DIM, T, PM>(P, ra, rb, sa, meta_slot(rec_meta(rb)), dA, step);
            m += q.cand;
        });
        const u32 base = atomicAdd(&C->n_ovf_cand, m);
        if (base + m > P.cap_ovf_cand) {
            atomicOr(&C->err, (u32)ERR_OVF_CAND);
            continue;
        }
        u32 w = 0;
        for_pairs<DIM, T, PM>(P, rec, start, ra, [&](u32 jb, const Rec<T> &rb) {
            const u32 sb = meta_slot(rec_meta(rb));
            const PairQ q = pair_quantities<DIM, T, PM>(P, ra, rb, sa, sb, dA, step);
            if (q.cand && w < m) {
                OvfCand c;
                c.slot = sb; c.idx = jb; c.p = q.p;
                cand[base + w++] = c;
            }
        });
        OvfCand *L = cand + base;
        for (u32 i = 1; i < m; ++i) {
            const OvfCand x = L[i];
            u32 j = i;
            while (j > 0 && L[j - 1].slot > x.slot) {
                L[j] = L[j - 1];
                --j;
            }
            L[j] = x;
        }
        double T_ = 0.0;
        for (u32 i = 0; i < m; ++i) T_ += L[i].p;
        const double tgt = u01(philox(sa, NOSLOT, step, TAG_SELA, P.key).x) * T_;
        double acc = 0.0;
        u32 ch = m - 1;
        for (u32 i = 0; i < m; ++i) {
            acc += L[i].p;
            if (tgt <= acc) {
                ch = i;
                break;
            }
        }
        const u32 q = atomicAdd(&C->n_picks, 1u);
        if (q < P.cap_picks) {
            Pick pk;
            pk.a_idx = ia; pk.b_idx = L[ch].idx; pk.a_slot = sa; pk.b_slot = L[ch].slot; pk.p = L[ch].p;
            picks[q] = pk;
        } else {
            atomicOr(&C->err, (u32)ERR_PICKS);
        }
    }
}

// ---------------------------------------------------------------------------
// K6: B-side choice.  Picks of the same B are chained through a per-record
// head word tagged with the step; the suitor with the smallest A slot walks
// the chain in ascending A slot and applies the cumulative rule with
// U = {b, -, step, SELB}.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_link(const Pick *__restrict__ picks, u64 *__restrict__ head, u32 *__restrict__ next,
                                                 Counters *C, Params P, u32 step)
{
    const u32 n = min(C->n_picks, P.cap_picks);
    const u64 tag = (u64)(step + 1u) << 32;
    for (u32 k = gtid(); k < n; k += gstride()) {
        const u64 prev = atomicExch((unsigned long long *)&head[picks[k].b_idx], (unsigned long long)(tag | k));
        next[k] = (prev >> 32) == (u64)(step + 1u) ? (u32)prev : NOSLOT;
    }
}

__global__ __launch_bounds__(BLOCK) void k_select_b(Params P, const Pick *__restrict__ picks, const u64 *__restrict__ head,
                                                     const u32 *__restrict__ next, Match *__restrict__ matches, Counters *C,
                                                     DbgPick *dbg, u32 step)
{
    const u32 n = min(C->n_picks, P.cap_picks);
    for (u32 k = gtid(); k < n; k += gstride()) {
        const Pick me = picks[k];
        if (P.debug) {
            const u32 q = atomicAdd(&C->n_dbg[1], 1u);
            if (q < P.dbg_cap) {
                DbgPick d;
                d.i = me.a_slot; d.j = me.b_slot; d.p = me.p;
                dbg[q] = d;
            }
        }
        const u32 h = (u32)head[me.b_idx];
        // leader: the suitor with the smallest A slot
        u32 mins = NOSLOT, count = 0;
        for (u32 e = h; e != NOSLOT; e = next[e]) {
            mins = min(mins, picks[e].a_slot);
            ++count;
        }
        if (me.a_slot != mins) continue;
        u32 win = k;
        if (count > 1) {
            double T_ = 0.0;
            u32 prev = 0;
            bool first = true;
            for (u32 r = 0; r < count; ++r) {  // ascending A slot
                u32 best = NOSLOT, be = NOSLOT;
                for (u32 e = h; e != NOSLOT; e = next[e]) {
                    const u32 s = picks[e].a_slot;
                    if ((first || s > prev) && s < best) {
                        best = s;
                        be = e;
                    }
                }
                if (be == NOSLOT) break;
                T_ += picks[be].p;
                prev = best;
                first = false;
            }
            const double tgt = u01(philox(me.b_slot, NOSLOT, step, TAG_SELB, P.key).x) * T_;
            double acc = 0.0;
            first = true;
            for (u32 r = 0; r < count; ++r) {
                u32 best = NOSLOT, be = NOSLOT;
                for (u32 e = h; e != NOSLOT; e = next[e]) {
                    const u32 s = picks[e].a_slot;
                    if ((first || s > prev) && s < best) {
                        best = s;
                        be = e;
                    }
                }
                if (be == NOSLOT) break;
                acc += picks[be].p;
                prev = best;
                first = false;
                win = be;
                if (tgt <= acc) break;
            }
        }
        const u32 q = atomicAdd(&C->n_matches, 1u);
        Match mt;
        mt.a_idx = picks[win].a_idx;
        mt.b_idx = picks[win].b_idx;
        matches[q] = mt;
    }
}

// ---------------------------------------------------------------------------
// K7: matched pairs (Sec. 3, steps 2a-2c).
// ---------------------------------------------------------------------------
template <int DIM, class T>
__global__ __launch_bounds__(BLOCK) void k_react(Params P, Rec<T> *__restrict__ rec, const Match *__restrict__ matches,
                                                  u32 *__restrict__ partner, Counters *C, DbgMatch *dbg, u32 step)
{
#pragma clang fp contract(off)
    const u32 n = C->n_matches;
    u32 n_react = 0, n_att = 0, n_hits = 0, n_near = 0;
    for (u32 k = gtid(); k < n; k += gstride()) {
        const Match mt = matches[k];
        Rec<T> ra = rec[mt.a_idx], rb = rec[mt.b_idx];
        const u32 sa = meta_slot(rec_meta(ra)), sb = meta_slot(rec_meta(rb));
        double dA[3], dB[3];
        displacement<DIM>(P, sa, SP_A, step, dA);
        displacement<DIM>(P, sb, SP_B, step, dB);
        const double xa[3] = {(double)ra.x, (double)ra.y, (double)ra.z};
        const double xb[3] = {(double)rb.x, (double)rb.y, (double)rb.z};
        double rv[3] = {0.0, 0.0, 0.0}, r2 = 0.0, r02 = 0.0;
        for (int d = 0; d < DIM; ++d) {
            rv[d] = min_image_d(xb[d] - xa[d], P.L[d], P.Lh[d]);
            const double o = rv[d] - (dB[d] - dA[d]);
            r2 += rv[d] * rv[d];
            r02 += o * o;
        }
        const double R = sqrt(r2) / P.a;
        double R0 = sqrt(r02) / P.a;
        if (R0 < 1.0) R0 = 1.0;
        bool react;
        double Rpp = R, preac = 1.0;
        u32 att = 0, hits = 0;
        if (P.bc == 0) {
            react = true;
        } else {
            Rpp = sample_radius<DIM>(P, R0, sa, sb, step, TAG_PROP, &att, &hits);
            preac = reac_prob(P, DIM, Rpp, R0);
            const u32 w = philox(sa, sb, step, TAG_REAC, P.key).x;
            react = below(w, preac);
            n_near += fabs(u01(w) - preac) < 1e-6;
            if (!react) {
                double rn = 0.0;
                for (int d = 0; d < DIM; ++d) rn += rv[d] * rv[d];
                rn = sqrt(rn);
                T na[3] = {0, 0, 0}, nb[3] = {0, 0, 0};
                for (int d = 0; d < DIM; ++d) {
                    const double e = rn > 0.0 ? rv[d] / rn : (d == DIM - 1 ? 1.0 : 0.0);
                    const double cen = xa[d] + P.fA * rv[d];
                    na[d] = wrap_store<T>(cen - P.fA * P.a * Rpp * e, P.L[d]);
                    nb[d] = wrap_store<T>(cen + P.fB * P.a * Rpp * e, P.L[d]);
                }
                ra.x = na[0]; ra.y = na[1]; ra.z = na[2];
                rb.x = nb[0]; rb.y = nb[1]; rb.z = nb[2];
            }
        }
        n_att += att;
        n_hits += hits;
        if (react) {
            ++n_react;
            T nc[3] = {0, 0, 0};
            for (int d = 0; d < DIM; ++d) nc[d] = wrap_store<T>(xa[d] + P.fA * rv[d], P.L[d]);
            ra.x = nc[0]; ra.y = nc[1]; ra.z = nc[2];
            rec_set_meta(ra, meta_make(SP_C, sa));
            rec_set_meta(rb, meta_make(SP_DEAD, sb));
            partner[sa] = P.reversible ? sb : NOSLOT;
        }
        rec[mt.a_idx] = ra;
        rec[mt.b_idx] = rb;
        if (P.debug) {
            const u32 q = atomicAdd(&C->n_dbg[2], 1u);
            if (q < P.dbg_cap) {
                DbgMatch d;
                d.i = sa; d.j = sb; d.reacted = react; d.attempts = att; d.Rpp = Rpp; d.preac = preac;
                dbg[q] = d;
            }
        }
    }
    if (n_react) atomicAdd((unsigned long long *)&C->stats[ST_REACT], (unsigned long long)n_react);
    if (n_att) atomicAdd((unsigned long long *)&C->stats[ST_ATTEMPTS], (unsigned long long)n_att);
    if (n_hits) atomicAdd((unsigned long long *)&C->stats[ST_BOUND], (unsigned long long)n_hits);
    if (n_near) atomicAdd((unsigned long long *)&C->stats[ST_NEAR], (unsigned long long)n_near);
}

// ---------------------------------------------------------------------------
// K8: C -> A + B (Sec. 2.2.5 and step 4) for the C records that existed at
// the start of the step (the C bucket range of this step's binning).
// ---------------------------------------------------------------------------
template <int DIM, class T>
__global__ __launch_bounds__(BLOCK) void k_dissociate(Params P, Rec<T> *__restrict__ rec, const u32 *__restrict__ start,
                                                       u32 *__restrict__ partner, Counters *C, DbgDiss *dbg, u32 step)
{
#pragma clang fp contract(off)
    const u32 beg = start[2 * P.n_cells], end = start[3 * P.n_cells];
    u32 n_dec = 0, n_gem = 0, n_att = 0, n_hits = 0;
    for (u32 i = beg + gtid(); i < end; i += gstride()) {
        Rec<T> rc = rec[i];
        const u32 sc = meta_slot(rec_meta(rc));
        if (!below(philox(sc, NOSLOT, step, TAG_UNI, P.key).x, P.p_uni)) continue;
        ++n_dec;
        u32 att = 0, hits = 0;
        const double Rpp = sample_radius<DIM>(P, 1.0, sc, NOSLOT, step, TAG_DPROP, &att, &hits);
        n_att += att;
        n_hits += hits;
        const double preac = reac_prob(P, DIM, Rpp, 1.0);
        const bool gem = below(philox(sc, NOSLOT, step, TAG_GEM, P.key).x, preac);
        const u32 sb = partner[sc];
        if (P.debug) {
            const u32 q = atomicAdd(&C->n_dbg[3], 1u);
            if (q < P.dbg_cap) {
                DbgDiss d;
                d.c = sc; d.j = sb; d.decayed = 1; d.recombined = gem; d.attempts = att; d.pad = 0; d.Rpp = Rpp; d.preac = preac;
                dbg[q] = d;
            }
        }
        if (gem) {
            ++n_gem;
            continue;
        }
        const uint4 r = philox(sc, NOSLOT, step, TAG_DIR, P.key);
        double e[3] = {0.0, 0.0, 0.0};
        if (DIM == 3) {
            const double z = 2.0 * u01(r.x) - 1.0, ph = (2.0 * PI_D) * u01(r.y), rho = sqrt(1.0 - z * z);
            e[0] = rho * cos(ph);
            e[1] = rho * sin(ph);
            e[2] = z;
        } else {
            const double ph = (2.0 * PI_D) * u01(r.x);
            e[0] = cos(ph);
            e[1] = sin(ph);
        }
        const double X[3] = {(double)rc.x, (double)rc.y, (double)rc.z};
        Rec<T> ra = rc, rb = rc;
        T pa[3] = {0, 0, 0}, pb[3] = {0, 0, 0};
        for (int d = 0; d < DIM; ++d) {
            pa[d] = wrap_store<T>(X[d] - P.fA * P.a * Rpp * e[d], P.L[d]);
            pb[d] = wrap_store<T>(X[d] + P.fB * P.a * Rpp * e[d], P.L[d]);
        }
        ra.x = pa[0]; ra.y = pa[1]; ra.z = pa[2];
        rb.x = pb[0]; rb.y = pb[1]; rb.z = pb[2];
        rec_set_meta(ra, meta_make(SP_A, sc));
        rec_set_meta(rb, meta_make(SP_B, sb));
        partner[sc] = NOSLOT;
        rec[i] = ra;
        const u32 q = C->n_live + atomicAdd(&C->n_append, 1u);
        if (q < P.cap) rec[q] = rb;
        else atomicOr(&C->err, (u32)ERR_APPEND);
    }
    if (n_dec) atomicAdd((unsigned long long *)&C->stats[ST_DECAY], (unsigned long long)n_dec);
    if (n_gem) atomicAdd((unsigned long long *)&C->stats[ST_GEMINATE], (unsigned long long)n_gem);
    if (n_att) atomicAdd((unsigned long long *)&C->stats[ST_ATTEMPTS], (unsigned long long)n_att);
    if (n_hits) atomicAdd((unsigned long long *)&C->stats[ST_BOUND], (unsigned long long)n_hits);
}

// K9: close the step.
__global__ void k_finish(Counters *C)
{
    C->stats[ST_PICKS] = C->n_picks;
    C->stats[ST_MATCHES] = C->n_matches;
    for (int s = 0; s < ST_N; ++s) {
        C->stats_last[s] = C->stats[s];
        C->stats_sum[s] += C->stats[s];
        C->stats[s] = 0;
    }
    C->n_rec = C->n_live + C->n_append;
    C->n_picks = C->n_matches = C->n_append = C->n_ovf = C->n_ovf_cand = 0;
}

// ---------------------------------------------------------------------------
// Reads and debug captures.
// ---------------------------------------------------------------------------
template <int DIM, class T>
__global__ void k_gather(const Rec<T> *__restrict__ rec, const u32 *__restrict__ partner, const Counters *C, int use_live,
                         double *__restrict__ pos, int *__restrict__ species, u32 cap)
{
    const u32 n = use_live ? C->n_live : C->n_rec;
    for (u32 i = gtid(); i < n; i += gstride()) {
        const Rec<T> r = rec[i];
        const u32 m = rec_meta(r), sp = meta_sp(m), s = meta_slot(m);
        if (sp > SP_C || s >= cap) continue;
        if (pos) {
            pos[(u64)s * DIM + 0] = (double)r.x;
            pos[(u64)s * DIM + 1] = (double)r.y;
            if (DIM == 3) pos[(u64)s * DIM + 2] = (double)r.z;
        }
        if (species) {
            species[s] = (int)sp;
            if (sp == SP_C && partner[s] < cap) species[partner[s]] = 4;
        }
    }
}

__global__ void k_fill(double *pos, u64 npos, int *species, u32 nsp)
{
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    for (u64 i = gtid(); i < npos; i += gstride()) pos[i] = nan;
    for (u32 i = gtid(); i < nsp; i += gstride()) species[i] = 3;
}

// bucket of every live record after binning, found from the bucket starts
__global__ void k_dbg_cells(Params P, const Rec<float> *recf, const Rec<double> *recd, const u32 *__restrict__ start,
                            const Counters *C, u32 *__restrict__ cells)
{
    const u32 n = C->n_live;
    for (u32 i = gtid(); i < n; i += gstride()) {
        const u32 m = recf ? rec_meta(recf[i]) : rec_meta(recd[i]);
        u32 lo = 0, hi = P.n_keys;  // largest key with start[key] <= i
        while (hi - lo > 1) {
            const u32 mid = (lo + hi) >> 1;
            if (start[mid] <= i) lo = mid;
            else hi = mid;
        }
        cells[meta_slot(m)] = lo;
    }
}

} // namespace gfbd
