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

// Bucket counters: key k is kept in region k % 16 at offset k / 16 (regions
// of region_len words).  A wave counts particles of consecutive cells, so its
// atomics then fall on 16 cache lines with a few words each instead of on two
// lines: same-line atomics serialise.
constexpr u32 CNT_REGIONS = 16;
__device__ __forceinline__ u32 cnt_index(u32 key, u32 region_len) { return (key % CNT_REGIONS) * region_len + key / CNT_REGIONS; }
__device__ __forceinline__ u32 gstride() { return gridDim.x * BLOCK; }
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// The dispatcher deals workgroups to the eight XCDs round-robin (workgroup b
// runs on XCD b % 8), and each XCD has its own L2.  Work items that share
// bucket data (neighbouring cells) are given to one XCD as a contiguous
// range: item = (b % 8) * per + b / 8 for a grid of 8 * per workgroups.
constexpr u32 N_XCD = 8;
__device__ __forceinline__ u32 xcd_item(u32 b, u32 per) { return (b % N_XCD) * per + b / N_XCD; }

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

// ln u for a uniform 0 < u < 1.  u = m 2^e with m in [sqrt(1/2), sqrt(2)), and
// ln m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...), s = (m - 1)/(m + 1),
// |s| <= 0.1716: the series to s^19 leaves out less than 2^-56 of the sum.
// m - 1 is exact (m lies within a factor 2 of 1).  Within a few binary64 ulps
// of the correctly rounded logarithm, at a third of the device library's
// operations (which carries extra precision it does not need here).
__device__ __forceinline__ double ln_unit(double u)
{
    int e;
    double m = frexp(u, &e);  // [1/2, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0), z = s * s;
    double p = 1.0 / 19.0;
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    p = fma(p, z, 1.0);
    constexpr double LN2 = 0.69314718055994530942;
    return fma((double)e, LN2, 2.0 * s * p);
}

// Free displacement sqrt(2 D dt) N(0,1) of a slot (Sec. 3, step 1):
// Box-Muller on one Philox draw {slot, -, step, MOVE}.
// Angles 2 pi u: a binary64 state rounds the update at the level of the
// angle's own rounding, so the angle is formed as the product 2 pi * u; for a
// binary32 state those bits lie far below the state's resolution and
// sincospi(2u), which needs no argument reduction, is used.
template <class T> __device__ __forceinline__ void sincos_turn(double u, double *s, double *c)
{
    if (sizeof(T) == 8) sincos((2.0 * PI_D) * u, s, c);
    else sincospi(2.0 * u, s, c);
}
template <class T> __device__ __forceinline__ double cos_turn(double u)
{
    return sizeof(T) == 8 ? cos((2.0 * PI_D) * u) : cospi(2.0 * u);
}

// The plain binary32 mode (PM_F32), and PM_F32D, take the same draws through a
// binary32 Box-Muller: their displacements differ from the binary64 ones by a
// few binary32 rounding errors of the displacement.
__device__ __forceinline__ float u01f(u32 w) { return ((float)w + 0.5f) * 0x1p-32f; }

template <int DIM, class T, int PM> __device__ inline void displacement(const Params &P, u32 slot, u32 sp, u32 step, double d[3])
{
#pragma clang fp contract(off)
    const uint4 r = philox(slot, NOSLOT, step, TAG_MOVE, P.key);
    if constexpr (PM == PM_F32 || PM == PM_F32D) {
        const float s = (float)P.sd[sp];
        const float r0 = sqrtf(-2.0f * logf(u01f(r.x)));
        float s0, c0;
        sincospif(2.0f * u01f(r.y), &s0, &c0);
        d[0] = (double)(s * (r0 * c0));
        d[1] = (double)(s * (r0 * s0));
        d[2] = DIM == 3 ? (double)(s * (sqrtf(-2.0f * logf(u01f(r.z))) * cospif(2.0f * u01f(r.w)))) : 0.0;
        return;
    }
    const double s = P.sd[sp];
    const double r0 = sqrt(-2.0 * ln_unit(u01(r.x)));
    double s0, c0;
    sincos_turn<T>(u01(r.y), &s0, &c0);
    d[0] = s * (r0 * c0);
    d[1] = s * (r0 * s0);
    if (DIM == 3) {
        const double r1 = sqrt(-2.0 * ln_unit(u01(r.z)));
        d[2] = s * (r1 * cos_turn<T>(u01(r.w)));
    } else {
        d[2] = 0.0;
    }
}

// The parameters of the replica a slot belongs to (a single system: its own)
// and the slot's index within its replica (what the draws are keyed on).
template <bool BATCH> __device__ __forceinline__ const Params &rep_params(const Params &P, u32 slot)
{
    if constexpr (BATCH) return P.reps[P.rep_of_slot[slot]];
    else return P;
}
template <bool BATCH> __device__ __forceinline__ u32 local_slot(const Params &Q, u32 slot)
{
    if constexpr (BATCH) return slot - Q.slot_base;
    else return slot;
}
// The replica owning a bucket key (batches): a bucket lies in one replica's
// cells, and sorted records know their keys, so this table lookup follows the
// record order where a lookup by slot would gather at random.
__device__ __forceinline__ u32 rep_of_key(const Params &P, u32 key)
{
    u32 c = key;
    if (c >= P.n_cells) c -= P.n_cells;
    if (c >= P.n_cells) c -= P.n_cells;
    return P.cell_rep[c];
}
// The replica's own step (replicas may join a batch at different steps).
template <bool BATCH> __device__ __forceinline__ u32 local_step(const Params &Q, u32 step)
{
    if constexpr (BATCH) return step - Q.step_base;
    else return step;
}

// x' = wrap(x + displacement) for the record of (replica-local) slot `slot`.
template <int DIM, class T, int PM> __device__ inline Rec<T> moved(const Params &P, const Rec<T> &r, u32 slot, u32 sp, u32 step)
{
#pragma clang fp contract(off)
    double d[3];
    displacement<DIM, T, PM>(P, slot, sp, step, d);
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

// Bucket key of a record of species sp at q: species block (each of
// P.n_cells keys, over all replicas), then the replica's cells, then its cell.
template <int DIM, class T, bool BATCH> __device__ inline u32 bucket_key(const Params &P, const Params &Q, u32 sp, const Rec<T> &q)
{
    return sp * P.n_cells + (BATCH ? Q.cell_base : 0u) + cell_of<DIM, T>(Q, q);
}

// ---------------------------------------------------------------------------
// Wave and workgroup scans.
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

// Append `val` to buf for every thread with `has`, one atomic on *counter per
// workgroup: a same-address atomic per entry would serialise.  Every thread
// of the workgroup calls it; the order of entries within the list is free.
__device__ inline void block_append(u32 *__restrict__ buf, u32 *counter, bool has, u32 val, u32 *lds, u32 *base)
{
    u32 total;
    const u32 r = block_excl_scan(has ? 1u : 0u, lds, total);
    if (total == 0) return;  // uniform: total is the workgroup's
    if (threadIdx.x == 0) *base = atomicAdd(counter, total);
    __syncthreads();
    if (has) buf[*base + r] = val;
    __syncthreads();  // *base is read before the next call writes it
}

// ---------------------------------------------------------------------------
// K1: move every live record and count it into its (species, cell) bucket.
// The records sit in the order of last step's buckets, whose keys okey[]
// holds for the first n_sorted of them, and a step takes only a few per cent
// of them to another bucket.  Each wave takes a chunk of 64 sorted records.
// A record that keeps its bucket (a stayer) is ranked among the stayers of
// that bucket in the chunk by a segmented scan across the wave (shuffles, no
// LDS and no barrier), and the chunk stores the bucket's stayer count: no
// atomics.  Every other live record (bucket changed, appended since the last
// binning, or in a bucket that began in an earlier chunk) takes its rank from
// an atomic counter.  Stayers fill a bucket from its start, the others from
// its end.  rank[i] = STAYER | rank for a stayer, else the atomic rank.
// ---------------------------------------------------------------------------
constexpr u32 STAYER = 0x80000000u;
constexpr u32 NOKEY = 0xFFFFFFFFu;

template <int DIM, class T, int PM, bool BATCH>
__global__ __launch_bounds__(BLOCK) void k_move_count(Params P, const Rec<T> *__restrict__ rec, const u32 *__restrict__ okey,
                                                       Rec<T> *__restrict__ tmp, u32 *__restrict__ rank, u32 *__restrict__ cnt,
                                                       u32 *__restrict__ scnt, u32 *__restrict__ nkey, Counters *C)
{
    const u32 step = C->step;
    if (gtid() == 0) {
        C->n_dbg[0] = C->n_dbg[1] = C->n_dbg[2] = C->n_dbg[3] = 0;
    }
    const u32 n = C->n_rec, ns = min(C->n_sorted, n);
    const int lane = lane_id();
    const u32 nw = gstride() >> 6;
    for (u32 b0 = (gtid() >> 6) * 64; b0 < n; b0 += nw * 64) {  // uniform over the wave
        const u32 i = b0 + lane;
        const bool valid = i < n, sorted = i < ns;
        Rec<T> r;
        u32 m = 0, sp = SP_DEAD;
        if (valid) {
            r = rec[i];
            m = rec_meta(r);
            sp = meta_sp(m);
        }
        const u32 ok = sorted ? okey[i] : NOKEY;
        const u32 before = (b0 > 0 && b0 - 1 < ns) ? okey[b0 - 1] : NOKEY;  // the record before the chunk
        const bool alive = valid && sp <= SP_C;
        u32 key = NOKEY;
        if (alive) {
            const u32 slot = meta_slot(m);
            // a batch record's replica: from its old bucket if it has one, else by slot
            const Params &Q = BATCH ? P.reps[sorted ? rep_of_key(P, ok) : P.rep_of_slot[slot]] : P;
            const Rec<T> q = moved<DIM, T, PM>(Q, r, local_slot<BATCH>(Q, slot), sp, local_step<BATCH>(Q, step));
            tmp[i] = q;
            key = bucket_key<DIM, T, BATCH>(P, Q, sp, q);
            if constexpr (BATCH) nkey[i] = key;  // the scatter needs no replica lookup
        } else if (valid) {
            tmp[i] = r;  // dead record: the scatter skips it
        }
        // segments: runs of equal old keys; the first one is not this chunk's
        // if it continues from the record before the chunk.  Every lane takes
        // part in every shuffle (a lane left out of one gives no value).
        const u32 left = __shfl_up(ok, 1, 64), right = __shfl_down(ok, 1, 64), first = __shfl(ok, 0, 64);
        const bool head = lane == 0 || left != ok;
        u32 seg0 = head ? (u32)lane : 0u;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const u32 x = __shfl_up(seg0, o, 64);
            if (lane >= o) seg0 = max(seg0, x);
        }
        const bool cont0 = before != NOKEY && before == first;
        const bool local = sorted && !(seg0 == 0 && cont0);
        const bool stay = alive && local && key == ok;
        const u32 ex = wave_incl_scan(stay ? 1u : 0u) - (stay ? 1u : 0u);
        const u32 rs = ex - (u32)__shfl((int)ex, (int)seg0, 64);
        const bool last = lane == 63 || right != ok;
        if (local && last) scnt[cnt_index(ok, P.cnt_region)] = rs + (stay ? 1u : 0u);
        if (alive) rank[i] = stay ? (STAYER | rs) : atomicAdd(&cnt[cnt_index(key, P.cnt_region)], 1u);
    }
}


// ---------------------------------------------------------------------------
// K2: exclusive scan of the bucket counts (atomic counts plus stayer counts)
// into bucket starts, clearing both for the next step.
// ---------------------------------------------------------------------------
// Two passes, no waiting.  Each thread owns SCAN_ITEMS consecutive keys; the
// count and start arrays are padded to whole tiles and the padding of the
// counts stays zero.  Pass 1 writes tile sums; pass 2 adds up the sums of the
// tiles before its own (a few hundred values) and scans its tile.
// The counts of the 16 keys of thread g sit in 16 regions at offset g
// (cnt_index), so each of a thread's 16 loads is coalesced across the wave.
static_assert(SCAN_ITEMS == CNT_REGIONS, "one key per region per thread");

__device__ __forceinline__ void load_counts(const u32 *cnt, u32 g, u32 region_len, u32 v[16])
{
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = cnt[(size_t)r * region_len + g];
}

// A tile of keys lying wholly in the unused tail of one species block (cells beyond the
// high-water mark hw, the first of them excluded: its start closes the last used bucket)
// holds no record: its counts stay zero and no kernel reads its starts.  A pool sized for
// its capacity has most of its tiles there, and the scan skips them.
__device__ __forceinline__ bool scan_tile_idle(u32 b, u32 n_cells, u32 hw)
{
    const uint64_t k0 = (uint64_t)b * SCAN_TILE, s0 = k0 / n_cells, c0 = k0 - s0 * n_cells;
    return c0 > hw && k0 + SCAN_TILE <= (s0 + 1) * n_cells;
}

// hw: the pool's high-water mark in its counters (null for a single system or a batch, whose
// keys are all in use: no dependent load in front of the scan).
__global__ __launch_bounds__(BLOCK) void k_scan_tiles(const u32 *__restrict__ cnt, const u32 *__restrict__ scnt, u32 *__restrict__ tsum,
                                                       const u32 *hw, u32 n_cells)
{
    __shared__ u32 lds[BLOCK / 64];
    if (hw && scan_tile_idle(blockIdx.x, n_cells, *hw)) {  // uniform
        if (threadIdx.x == 0) tsum[blockIdx.x] = 0u;
        return;
    }
    u32 v[16], w[16];
    load_counts(cnt, gtid(), gridDim.x * BLOCK, v);
    load_counts(scnt, gtid(), gridDim.x * BLOCK, w);
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] += w[k];
    u32 s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += v[k];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) tsum[blockIdx.x] = s;
}

__global__ __launch_bounds__(BLOCK) void k_scan(u32 *__restrict__ cnt, u32 *__restrict__ scnt, const u32 *__restrict__ tsum,
                                                 u32 *__restrict__ start, Counters *C, const u32 *hw, u32 n_cells)
{
    __shared__ u32 lds[BLOCK / 64];
    // an idle tile has nothing to write (the last one still writes the total)
    if (hw && blockIdx.x + 1 < gridDim.x && scan_tile_idle(blockIdx.x, n_cells, *hw)) return;  // uniform
    const size_t base = (size_t)blockIdx.x * SCAN_TILE + SCAN_ITEMS * threadIdx.x;
    const u32 rl = gridDim.x * BLOCK;
    u32 v[16], w[16];
    load_counts(cnt, gtid(), rl, v);
    load_counts(scnt, gtid(), rl, w);
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] += w[k];
    u32 before = 0;
    for (u32 t = threadIdx.x; t < blockIdx.x; t += BLOCK) before += tsum[t];
    const u32 carry = block_sum(before, lds);
    u32 mine = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) mine += v[k];
    u32 total;
    u32 run = carry + block_excl_scan(mine, lds, total);
    uint4 *o = reinterpret_cast<uint4 *>(start + base);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint4 t;
        t.x = run;
        run += v[4 * k];
        t.y = run;
        run += v[4 * k + 1];
        t.z = run;
        run += v[4 * k + 2];
        t.w = run;
        run += v[4 * k + 3];
        o[k] = t;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) cnt[(size_t)r * rl + gtid()] = 0u;
#pragma unroll
    for (int r = 0; r < 16; ++r) scnt[(size_t)r * rl + gtid()] = 0u;
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == BLOCK - 1) {
        start[(size_t)gridDim.x * SCAN_TILE] = run;
        C->n_live = run;
    }
}

// ---------------------------------------------------------------------------
// K3: write each moved record to its sorted place (stayers from the start of
// the bucket, the others from its end) and note its bucket key for the next
// step's stayer test.
// ---------------------------------------------------------------------------
template <int DIM, class T, bool BATCH>
__global__ __launch_bounds__(BLOCK) void k_scatter(Params P, const Rec<T> *__restrict__ tmp, const u32 *__restrict__ rank,
                                                    const u32 *__restrict__ start, Rec<T> *__restrict__ out, u32 *__restrict__ okey,
                                                    const u32 *__restrict__ nkey, const Counters *C)
{
    const u32 n = C->n_rec;
    for (u32 i = gtid(); i < n; i += gstride()) {
        const Rec<T> q = tmp[i];
        const u32 m = rec_meta(q), sp = meta_sp(m);
        if (sp > SP_C) continue;
        u32 key;
        if constexpr (BATCH) key = nkey[i];
        else key = bucket_key<DIM, T, false>(P, P, sp, q);
        const u32 rk = rank[i];
        const u32 dst = (rk & STAYER) ? start[key] + (rk & ~STAYER) : start[key + 1] - 1u - rk;
        if (dst < P.cap) {
            out[dst] = q;
            okey[dst] = key;
        }
    }
}

// ---------------------------------------------------------------------------
// Pair geometry and encounter probability.
// ---------------------------------------------------------------------------
struct PairQ {
    double R, R0, p;
    double R0d;  // R0 in binary64 (equal to R0 unless the pair arithmetic is binary32)
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
// p_enc of a pair that does not overlap (R > 1, R0 >= 1) in the pair
// arithmetic PM: binary64; binary32 from binary32 R and R0; or binary32
// exponentials of binary64 exponent arguments.  The 2D expansion is binary64.
template <int DIM, int PM, int NC> __device__ __forceinline__ double penc_R(const Params &P, double R, double R0)
{
#pragma clang fp contract(off)
    if (DIM == 2) return penc2<NC>(P, R, R0);
    if (PM == PM_F32) {
        const float Rf = (float)R, R0f = (float)R0;
        return penc3_args((Rf - 1.0f) * (R0f - 1.0f) * P.inv_tauf, (Rf + R0f - 1.0f) * P.inv_tauf, Rf * R0f * P.inv_tauf);
    }
    const double e1 = (R - 1.0) * (R0 - 1.0) / P.tau, e2 = (R + R0 - 1.0) / P.tau, e3 = R * R0 / P.tau;
    return PM == PM_F64 ? penc3_args(e1, e2, e3) : (double)penc3_args((float)e1, (float)e2, (float)e3);
}

template <int DIM, class T, int PM, int NC>
__device__ inline PairQ pair_quantities(const Params &P, const Rec<T> &ra, const Rec<T> &rb, u32 sa, u32 sb,
                                        const double dA[3], u32 step)
{
#pragma clang fp contract(off)
    PairQ q;
    double dB[3];
    displacement<DIM, T, PM>(P, sb, SP_B, step, dB);
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
        {
            // the binary64 R0 that the propagation of a matched pair uses
            const double xa[3] = {(double)ra.x, (double)ra.y, (double)ra.z};
            const double xb[3] = {(double)rb.x, (double)rb.y, (double)rb.z};
            double r02 = 0.0;
            for (int k = 0; k < DIM; ++k) {
                const double o = min_image_d(xb[k] - xa[k], P.L[k], P.Lh[k]) - (dB[k] - dA[k]);
                r02 += o * o;
            }
            double R0 = sqrt(r02) / P.a;
            if (R0 < 1.0) R0 = 1.0;
            q.R0d = R0;
        }
        q.overlap = Rf <= 1.0f;
        q.p = q.overlap ? 1.0 : penc_R<DIM, PM, NC>(P, (double)Rf, (double)R0f);
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
        q.R0d = R0;
        q.overlap = R <= 1.0;
        q.p = q.overlap ? 1.0 : penc_R<DIM, PM, NC>(P, R, R0);
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

// Which neighbour cells of ra's cell can hold a B within r_cut.  Cells are
// at least r_cut wide, so along each axis only the cell itself and a
// neighbour whose shared face lies within r_cut of ra qualify.  P.reach is
// r_cut widened by far more than the rounding of the face positions, of the
// binning and of the pair test, so a skipped cell holds no pair; the pair
// test itself still decides every candidate.  An axis with fewer than three
// cells has one cell.
template <int DIM, class T>
__device__ __forceinline__ void reach_of(const Params &P, const Rec<T> &ra, int c[3], int lo[3], int hi[3])
{
    const double x[3] = {(double)ra.x, (double)ra.y, (double)ra.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        c[k] = 0;
        lo[k] = hi[k] = 0;
        if (k < DIM) {
            c[k] = cell1(x[k], P.cs[k], P.nc[k]);
            if (P.nc[k] >= 3) {
                const double f = x[k] - c[k] * P.ce[k];
                lo[k] = f < P.reach ? -1 : 0;
                hi[k] = P.ce[k] - f < P.reach ? 1 : 0;
            }
        }
    }
}

// The B bucket ranges that can hold a partner of the A record ra: rows of
// cells along x are contiguous ranges, a row split in two where it wraps
// around the box.  With cells at least twice the reach (NARROW) an A needs
// at most one neighbour per axis, so 2 x 2 rows (2 in 2D); otherwise up to
// 3 x 3.  All bounds are loaded before any is used.
template <int DIM, bool NARROW> constexpr int n_slots() { return NARROW ? (DIM == 3 ? 4 : 2) : (DIM == 3 ? 9 : 3); }

// P: the grid of ra's replica; bbase: key of that replica's first B bucket.
template <int DIM, bool NARROW, class T>
__device__ __forceinline__ void collect_ranges(const Params &P, u32 bbase, const u32 *__restrict__ start, const Rec<T> &ra, u32 *b0,
                                               u32 *e0, u32 *b1, u32 *e1)
{
    int c[3], lo[3], hi[3];
    reach_of<DIM, T>(P, ra, c, lo, hi);
    const int nx = P.nc[0], ny = P.nc[1], nz = P.nc[2];
    const int xa = c[0] + lo[0], xb = c[0] + hi[0];
    const int sy = lo[1] + hi[1], sz = lo[2] + hi[2];  // NARROW: the one neighbour side, or 0
#pragma unroll
    for (int s = 0; s < n_slots<DIM, NARROW>(); ++s) {
        int oy, oz;
        bool use;
        if (NARROW) {
            oy = (s & 1) ? sy : 0;
            oz = (s & 2) ? sz : 0;
            use = (!(s & 1) || sy != 0) && (!(s & 2) || sz != 0);
        } else {
            oy = s % 3 - 1;
            oz = DIM == 3 ? s / 3 - 1 : 0;
            use = oy >= lo[1] && oy <= hi[1] && oz >= lo[2] && oz <= hi[2];
        }
        b0[s] = e0[s] = b1[s] = e1[s] = 0;
        if (!use) continue;
        int y = c[1] + oy, z = c[2] + oz;
        y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
        z = z < 0 ? z + nz : (z >= nz ? z - nz : z);
        const u32 row = bbase + ((u32)z * ny + y) * nx;
        // bucket indices first, then the loads (branch-free, so the bounds
        // stay in registers)
        const bool wl = xa < 0, wh = xb >= nx;
        const u32 ka = row + (wl ? 0 : xa), kb = row + (wh ? nx : xb + 1);
        const u32 kc = row + (wl ? nx - 1 : 0), kd = row + (wl ? nx : 1);
        b0[s] = start[ka];
        e0[s] = start[kb];
        if (wl || wh) {
            b1[s] = start[kc];
            e1[s] = start[kd];
        }
    }
}

// Visit every B record within r_cut of the A record ra, one range after the
// other (the per-lane form; the direct kernel balances the ranges over a wave).
template <int DIM, class T, int PM, class F>
__device__ inline void for_pairs(const Params &P, const Rec<T> *__restrict__ rec, const u32 *__restrict__ start, const Rec<T> &ra,
                                 F &&emit)
{
    constexpr int NS = n_slots<DIM, false>();
    u32 b0[NS], e0[NS], b1[NS], e1[NS];
    collect_ranges<DIM, false, T>(P, P.n_cells, start, ra, b0, e0, b1, e1);  // B buckets follow the A buckets
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        for (u32 j = b0[s]; j < e0[s]; ++j) {
            const Rec<T> rb = rec[j];
            if (in_range<DIM, T, PM>(P, ra, rb)) emit(j, rb);
        }
        for (u32 j = b1[s]; j < e1[s]; ++j) {
            const Rec<T> rb = rec[j];
            if (in_range<DIM, T, PM>(P, ra, rb)) emit(j, rb);
        }
    }
}

// ---------------------------------------------------------------------------
// K5a: A-B pairs within r_cut.  One workgroup per brick of bx*by*bz cells:
// the B records of the brick and its one-cell halo are staged in LDS (bucket
// ranges of consecutive cells are contiguous), then every A of the brick
// tests the B's of its 3^d neighbour cells from LDS.  Pairs go to an LDS
// queue that is appended to the global pair list once per workgroup.  A
// brick whose halo holds more B's than fit in LDS tests from global memory.
// ---------------------------------------------------------------------------
__device__ inline void block_add_stats(const u32 *vals, int nv, u64 *dst, u32 *lds)
{
    for (int s = 0; s < nv; ++s) {
        const u32 t = block_sum(vals[s], lds);
        if (threadIdx.x == 0 && t) atomicAdd((unsigned long long *)&dst[s], (unsigned long long)t);
    }
}

constexpr int PBLOCK = 256;      // threads per pair-search workgroup
constexpr int QCAP = 512;        // pairs queued in LDS per workgroup
constexpr int MAX_HALO = 1024;   // halo cells per brick
constexpr int CELLS_PER_T = MAX_HALO / PBLOCK;
constexpr int MAX_ROWS = 64;     // rows of A cells per brick

// exclusive scan over a workgroup of NT threads (NT / 64 waves)
template <int NT> __device__ inline u32 group_excl_scan(u32 v, u32 *lds, u32 &total)
{
    const u32 inc = wave_incl_scan(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) lds[w] = inc;
    __syncthreads();
    u32 off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        const u32 x = lds[i];
        off += i < w ? x : 0u;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

// This workgroup's segment of the pair list and its counter.
__device__ __forceinline__ u32 pl_segment() { return blockIdx.x % PL_SEGS; }

__device__ __forceinline__ void append_pair(PairEnt *q, u32 *nq, PairEnt *list, Counters *C, const Params &P, u32 a, u32 b)
{
    const u32 k = atomicAdd(nq, 1u);
    PairEnt e;
    e.a_idx = a;
    e.b_idx = b;
    if (k < (u32)QCAP) {
        q[k] = e;
    } else {
        const u32 x = pl_segment();
        const u32 g = atomicAdd(&C->pl_seg[x * PL_STRIDE], 1u);
        if (g < P.seg_cap) list[x * P.seg_cap + g] = e;
        else atomicOr(&C->err, (u32)ERR_PAIRS);
    }
}

// Append a workgroup's queued pairs to its segment with one atomic.
template <int NT>
__device__ __forceinline__ void flush_pairs(const PairEnt *q, const u32 &nq, u32 &qbase, PairEnt *list, Counters *C, const Params &P)
{
    __syncthreads();
    const u32 n = min(nq, (u32)QCAP), x = pl_segment();
    if (threadIdx.x == 0) qbase = n ? atomicAdd(&C->pl_seg[x * PL_STRIDE], n) : 0u;
    __syncthreads();
    for (u32 i = threadIdx.x; i < n; i += NT) {
        const u32 g = qbase + i;
        if (g < P.seg_cap) list[x * P.seg_cap + g] = q[i];
        else atomicOr(&C->err, (u32)ERR_PAIRS);
    }
}

// The pairs of the step across the segments: pre[x] = pairs in segments
// before x (wave-uniform values); returns the total.
struct PairIndex {
    u32 pre[PL_SEGS];
    u32 total, seg_cap;
    __device__ __forceinline__ PairIndex(const Counters *C, const Params &P) : seg_cap(P.seg_cap)
    {
        u32 s = 0;
#pragma unroll
        for (u32 x = 0; x < PL_SEGS; ++x) {
            pre[x] = s;
            s += min(C->pl_seg[x * PL_STRIDE], seg_cap);
        }
        total = s;
    }
    // the list entry of pair k < total
    __device__ __forceinline__ u32 entry(u32 k) const
    {
        u32 seg = 0, off = 0;
#pragma unroll
        for (u32 x = 1; x < PL_SEGS; ++x)
            if (k >= pre[x]) {
                seg = x;
                off = pre[x];
            }
        return seg * seg_cap + (k - off);
    }
};

__device__ __forceinline__ int wrapc(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

template <int DIM, class T, int PM>
__global__ __launch_bounds__(PBLOCK) void k_pair_scan(Params P, const Rec<T> *__restrict__ rec, const u32 *__restrict__ start,
                                                       PairEnt *__restrict__ list, Counters *C)
{
    constexpr int LCAP = 1024;
    // B positions relative to the brick origin (periodic image applied) and
    // the B record index in the fourth lane, in halo-cell order
    __shared__ float4 sbr[LCAP];
    __shared__ u32 off[MAX_HALO + 1];
    // source of each staged slot: B record index and periodic-shift code
    // (two bits per axis: 1 = -L, 2 = +L)
    __shared__ u32 srcj[LCAP];
    __shared__ unsigned char srcc[LCAP];
    __shared__ u32 rowpre[MAX_ROWS + 1], rowst[MAX_ROWS];
    __shared__ PairEnt q[QCAP];
    __shared__ u32 nq, qbase;
    __shared__ u32 lds[PBLOCK / 64];

    const int nx = P.nc[0], ny = P.nc[1], nz = P.nc[2];
    const u32 per = gridDim.x / N_XCD;
    u32 b = xcd_item(blockIdx.x, per);
    if (b >= P.nbx * P.nby * P.nbz) return;  // padding of the grid to a multiple of 8 (uniform)
    const int x0 = (int)(b % P.nbx) * P.bx;
    b /= P.nbx;
    const int y0 = (int)(b % P.nby) * P.by;
    b /= P.nby;
    const int z0 = DIM == 3 ? (int)b * P.bz : 0;
    const int ex = min(P.bx, nx - x0), ey = min(P.by, ny - y0), ez = DIM == 3 ? min(P.bz, nz - z0) : 1;
    const int hx = ex + 2, hy = ey + 2, hz = DIM == 3 ? ez + 2 : 1;
    const int nh = hx * hy * hz;
    const u32 bbase = P.n_cells;
    const double ox = x0 / P.cs[0], oy = y0 / P.cs[1], oz = DIM == 3 ? z0 / P.cs[2] : 0.0;

    // 1. this thread's halo cells h = CELLS_PER_T * t + c: bucket ranges (all
    //    loads issued together) and the periodic shift of each cell
    u32 hs[CELLS_PER_T], he[CELLS_PER_T], code[CELLS_PER_T];
    u32 local = 0;
#pragma unroll
    for (int c = 0; c < CELLS_PER_T; ++c) {
        const int h = CELLS_PER_T * threadIdx.x + c;
        hs[c] = he[c] = code[c] = 0;
        if (h < nh) {
            const int r = h / hx;
            const int ux = x0 - 1 + (h - r * hx), uy = y0 - 1 + r % hy, uz = z0 - 1 + r / hy;
            const int gx = wrapc(ux, nx), gy = wrapc(uy, ny), gz = DIM == 3 ? wrapc(uz, nz) : 0;
            const u32 k = bbase + ((u32)gz * ny + gy) * nx + gx;
            hs[c] = start[k];
            he[c] = start[k + 1];
            code[c] = (ux < 0 ? 1u : (ux >= nx ? 2u : 0u)) | (uy < 0 ? 4u : (uy >= ny ? 8u : 0u)) |
                      (DIM == 3 ? (uz < 0 ? 16u : (uz >= nz ? 32u : 0u)) : 0u);
        }
    }
    const int nr = ey * ez;
    u32 rs = 0, rc = 0;
    if ((int)threadIdx.x < nr) {
        const int r = threadIdx.x;
        const u32 akey = ((u32)(z0 + r / ey) * ny + (y0 + r % ey)) * nx + x0;
        rs = start[akey];
        rc = start[akey + ex] - rs;
    }
#pragma unroll
    for (int c = 0; c < CELLS_PER_T; ++c) local += he[c] - hs[c];
    u32 total;
    u32 pos = group_excl_scan<PBLOCK>(local, lds, total);
#pragma unroll
    for (int c = 0; c < CELLS_PER_T; ++c) {
        const int h = CELLS_PER_T * threadIdx.x + c;
        if (h < nh) off[h] = pos;
        pos += he[c] - hs[c];
    }
    if (threadIdx.x < 64) {
        const u32 inc = wave_incl_scan(rc);
        if ((int)threadIdx.x < nr) {
            rowpre[threadIdx.x + 1] = inc;
            rowst[threadIdx.x] = rs;
        }
        if (threadIdx.x == 0) rowpre[0] = 0;
    }
    if (threadIdx.x == 0) {
        off[nh] = total;
        nq = 0;
    }

    // 2. stage the B records: the owner of each cell writes the sources of
    //    its slots, then every thread converts up to LCAP / PBLOCK records
    //    (fixed trip count, so all loads are in flight together)
    const bool use_lds = total <= (u32)LCAP;
    if (use_lds) {
        pos -= local;  // start of this thread's first cell
#pragma unroll
        for (int c = 0; c < CELLS_PER_T; ++c)
            for (u32 j = hs[c]; j < he[c]; ++j, ++pos) {
                srcj[pos] = j;
                srcc[pos] = (unsigned char)code[c];
            }
    } else if (threadIdx.x == 0) {
        atomicAdd((unsigned long long *)&C->stats[ST_LDS_FALLBACK], 1ull);
    }
    __syncthreads();
    if (use_lds) {
        const float Lx = (float)P.L[0], Ly = (float)P.L[1], Lz = (float)P.L[2];
#pragma unroll
        for (int u = 0; u < LCAP / PBLOCK; ++u) {
            const u32 k = threadIdx.x + u * PBLOCK;
            if (k < total) {
                const u32 j = srcj[k], cd = srcc[k];
                const Rec<T> rb = rec[j];
                const float sx = (cd & 1u) ? -Lx : ((cd & 2u) ? Lx : 0.0f);
                const float sy = (cd & 4u) ? -Ly : ((cd & 8u) ? Ly : 0.0f);
                const float sz = (cd & 16u) ? -Lz : ((cd & 32u) ? Lz : 0.0f);
                const float px = (float)((double)rb.x - ox) + sx;
                const float py = (float)((double)rb.y - oy) + sy;
                const float pz = DIM == 3 ? (float)((double)rb.z - oz) + sz : 0.0f;
                sbr[k] = make_float4(px, py, pz, __uint_as_float(j));
            }
        }
    }
    __syncthreads();

    // 3. every A of the brick against the B's of its 3^d neighbour cells: a
    //    binary32 test against a radius widened by the rounding of the
    //    relative coordinates, then the exact test on the few that pass
    const u32 nA = rowpre[nr];
    const float rpre = P.rcut2f_pre;
    for (u32 i = threadIdx.x; i < nA; i += PBLOCK) {
        int lo = 0, hi = nr;  // rowpre[lo] <= i < rowpre[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (rowpre[mid] <= i) lo = mid;
            else hi = mid;
        }
        const u32 ia = rowst[lo] + (i - rowpre[lo]);
        const Rec<T> ra = rec[ia];
        if (use_lds) {
            int c[3], lo[3], hi[3];
            reach_of<DIM, T>(P, ra, c, lo, hi);
            const int lx = c[0] - x0 + 1, ly = c[1] - y0 + 1, lz = DIM == 3 ? c[2] - z0 + 1 : 0;
            const float ax = (float)((double)ra.x - ox), ay = (float)((double)ra.y - oy);
            const float az = DIM == 3 ? (float)((double)ra.z - oz) : 0.0f;
            for (int dz = lo[2]; dz <= hi[2]; ++dz)
                for (int dy = lo[1]; dy <= hi[1]; ++dy) {
                    const int h0 = ((lz + dz) * hy + (ly + dy)) * hx + lx;
                    const u32 je = off[h0 + hi[0] + 1];
                    for (u32 j = off[h0 + lo[0]]; j < je; ++j) {
                        const float4 v = sbr[j];
                        const float ddx = v.x - ax, ddy = v.y - ay, ddz = v.z - az;
                        if (ddx * ddx + ddy * ddy + ddz * ddz < rpre) {
                            const u32 jb = __float_as_uint(v.w);
                            if (in_range<DIM, T, PM>(P, ra, rec[jb])) append_pair(q, &nq, list, C, P, ia, jb);
                        }
                    }
                }
        } else {
            for_pairs<DIM, T, PM>(P, rec, start, ra, [&](u32 jb, const Rec<T> &) { append_pair(q, &nq, list, C, P, ia, jb); });
        }
    }
    flush_pairs<PBLOCK>(q, nq, qbase, list, C, P);
}

// K5b: the same pairs with one A record per thread and the neighbour
// buckets read through L2: no staging, so it wins where an A tests few B's;
// also the path for grids with fewer than three cells along some axis.
// The lanes of a wave write their (B record, owner lane) tests into one LDS
// list and the wave then works through it 2 x 64 tests at a time (loads in
// flight together), so a lane with many tests does not hold up the other 63.
// A wave with more than TCAP tests tests per lane instead.
constexpr int TCAP = 512;  // tests listed per wave

template <int DIM, class T, int PM, bool NARROW, bool BATCH>
__device__ __forceinline__ void pair_scan_direct(const Params &P, const Rec<T> *__restrict__ rec, const u32 *__restrict__ start,
                                                 const u32 *__restrict__ okey, PairEnt *__restrict__ list, Counters *C)
{
    constexpr int NS = n_slots<DIM, NARROW>();
    constexpr int NW = BLOCK / 64;
    constexpr int U = 2;
    __shared__ PairEnt q[QCAP];
    __shared__ u32 nq, qbase;
    __shared__ u32 tj[NW][TCAP];
    __shared__ unsigned char town[NW][TCAP];
    __shared__ Rec<T> sa[BLOCK];
    __shared__ u32 srep[BATCH ? BLOCK : 1];  // replica of each staged A
    if (threadIdx.x == 0) nq = 0;
    const int w = threadIdx.x >> 6, lane = lane_id();
    const u32 a_end = start[P.n_cells];  // A buckets are the keys below n_cells
    // batches of BLOCK A records; XCD x takes the contiguous range
    // [x * per, (x + 1) * per), its workgroups striding through it
    const u32 nbatch = (a_end + BLOCK - 1) / BLOCK, per = (nbatch + N_XCD - 1) / N_XCD;
    const u32 x = blockIdx.x % N_XCD, g8 = gridDim.x / N_XCD;
    for (u32 k = blockIdx.x / N_XCD; k < per && x * per + k < nbatch; k += g8) {
        const u32 b = (x * per + k) * BLOCK;
        const u32 ia = b + threadIdx.x;
        const bool act = ia < a_end;
        Rec<T> ra = rec[act ? ia : b];
        u32 b0[NS], e0[NS], b1[NS], e1[NS];
        u32 tot = 0;
        // an A's replica from its bucket (A keys are its cells)
        const u32 rep = BATCH && act ? P.cell_rep[okey[ia]] : 0u;
        if (act) {
            // B buckets follow the A buckets; a replica's cells start at its cell base
            const Params &Q = BATCH ? P.reps[rep] : P;
            collect_ranges<DIM, NARROW, T>(Q, P.n_cells + (BATCH ? Q.cell_base : 0u), start, ra, b0, e0, b1, e1);
#pragma unroll
            for (int s = 0; s < NS; ++s) tot += (e0[s] - b0[s]) + (e1[s] - b1[s]);
        } else {
#pragma unroll
            for (int s = 0; s < NS; ++s) b0[s] = e0[s] = b1[s] = e1[s] = 0;
        }
        const u32 tinc = wave_incl_scan(tot);
        const u32 T_ = __shfl(tinc, 63, 64);
        const bool fits = T_ <= (u32)TCAP;  // uniform over the wave
        if (fits) {
            u32 k = tinc - tot;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                for (u32 j = b0[s]; j < e0[s]; ++j, ++k) {
                    tj[w][k] = j;
                    town[w][k] = (unsigned char)lane;
                }
                for (u32 j = b1[s]; j < e1[s]; ++j, ++k) {
                    tj[w][k] = j;
                    town[w][k] = (unsigned char)lane;
                }
            }
            sa[threadIdx.x] = ra;
            if constexpr (BATCH) srep[threadIdx.x] = rep;
        }
        __syncthreads();
        if (fits) {
            for (u32 t0 = 0; t0 < T_; t0 += U * 64) {
                u32 jb[U];
                int own[U];
                Rec<T> rb[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const u32 t = t0 + u * 64 + lane;
                    jb[u] = t < T_ ? tj[w][t] : NOSLOT;
                    own[u] = t < T_ ? town[w][t] : 0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (jb[u] != NOSLOT) rb[u] = rec[jb[u]];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (jb[u] == NOSLOT) continue;
                    const Rec<T> ro = sa[w * 64 + own[u]];
                    if (in_range<DIM, T, PM>(BATCH ? P.reps[srep[w * 64 + own[u]]] : P, ro, rb[u]))
                        append_pair(q, &nq, list, C, P, b + w * 64 + own[u], jb[u]);
                }
            }
        } else {
            const Params &Q = BATCH ? P.reps[rep] : P;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                for (u32 j = b0[s]; j < e0[s]; ++j)
                    if (in_range<DIM, T, PM>(Q, ra, rec[j])) append_pair(q, &nq, list, C, P, ia, j);
                for (u32 j = b1[s]; j < e1[s]; ++j)
                    if (in_range<DIM, T, PM>(Q, ra, rec[j])) append_pair(q, &nq, list, C, P, ia, j);
            }
        }
        __syncthreads();  // the next batch reuses the LDS tables
    }
    flush_pairs<BLOCK>(q, nq, qbase, list, C, P);
}

// The narrow form fits 64 VGPRs: eight waves per SIMD hold all A's of a
// typical step at once.
template <int DIM, class T, int PM, bool BATCH>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8))) void k_pair_scan_direct_narrow(
    Params P, const Rec<T> *__restrict__ rec, const u32 *__restrict__ start, const u32 *__restrict__ okey, PairEnt *__restrict__ list,
    Counters *C)
{
    pair_scan_direct<DIM, T, PM, true, BATCH>(P, rec, start, okey, list, C);
}

template <int DIM, class T, int PM, bool BATCH>
__global__ __launch_bounds__(BLOCK) void k_pair_scan_direct(Params P, const Rec<T> *__restrict__ rec, const u32 *__restrict__ start,
                                                             const u32 *__restrict__ okey, PairEnt *__restrict__ list, Counters *C)
{
    pair_scan_direct<DIM, T, PM, false, BATCH>(P, rec, start, okey, list, C);
}

// ---------------------------------------------------------------------------
// K5b: encounter probability and Bernoulli draw of every pair (one thread per
// pair).  Candidates are chained per A record through a head word tagged
// with the step, so no list needs clearing between steps.
// ---------------------------------------------------------------------------
__device__ __forceinline__ u32 chain_push(u64 *head, u32 rec_idx, u32 entry, u32 step)
{
    const u64 tag = (u64)(step + 1u) << 32;
    const u64 prev = atomicExch((unsigned long long *)&head[rec_idx], (unsigned long long)(tag | entry));
    return (prev >> 32) == (u64)(step + 1u) ? (u32)prev : NOSLOT;
}

template <int DIM, class T, int PM, int NC, bool BATCH>
__global__ __launch_bounds__(BLOCK) void k_pair_eval(Params P, const Rec<T> *__restrict__ rec, const u32 *__restrict__ okey,
                                                      const PairEnt *__restrict__ list, CandEnt *__restrict__ cand,
                                                      u32 *__restrict__ flag, u64 *__restrict__ headA, u32 *__restrict__ nextA,
                                                      Counters *C, DbgPair *dbg)
{
    __shared__ u32 lds[BLOCK / 64];
    const u32 step = C->step;
    const PairIndex pi(C, P);
    if (blockIdx.x * BLOCK >= pi.total) return;  // no pair for this workgroup (uniform): nothing to count
    u32 st[5] = {0, 0, 0, 0, 0};  // pairs, cand, overlap, r0clamp, near
    for (u32 kk = gtid(); kk < pi.total; kk += gstride()) {
        const u32 k = pi.entry(kk);
        const PairEnt e = list[k];
        const Rec<T> ra = rec[e.a_idx], rb = rec[e.b_idx];
        const u32 sa = meta_slot(rec_meta(ra)), sb = meta_slot(rec_meta(rb));
        const Params &Q = BATCH ? P.reps[P.cell_rep[okey[e.a_idx]]] : P;  // the A's bucket; A and B share their replica
        double dA[3];
        const u32 ls = local_step<BATCH>(Q, step);
        displacement<DIM, T, PM>(Q, local_slot<BATCH>(Q, sa), SP_A, ls, dA);
        const PairQ q = pair_quantities<DIM, T, PM, NC>(Q, ra, rb, local_slot<BATCH>(Q, sa), local_slot<BATCH>(Q, sb), dA, ls);
        st[0] += 1;
        st[1] += q.cand;
        st[2] += q.overlap;
        st[3] += q.clamped;
        st[4] += q.near;
        if (P.debug) {
            const u32 d = atomicAdd(&C->n_dbg[0], 1u);
            if (d < P.dbg_cap) {
                DbgPair g;
                g.i = sa; g.j = sb; g.R = q.R; g.R0 = q.R0; g.p = q.p; g.draw = q.draw; g.cand = q.cand;
                dbg[d] = g;
            }
        }
        flag[k] = q.cand ? PE_CAND : PE_PAIR;
        if (q.cand) {
            CandEnt c;
            c.a_slot = sa;
            c.b_slot = sb;
            c.p = q.p;
            c.R0 = q.R0d;
            cand[k] = c;
            nextA[k] = chain_push(headA, e.a_idx, k, step);
        }
    }
    block_add_stats(st, 4, &C->stats[ST_PAIRS], lds);
    block_add_stats(st + 4, 1, &C->stats[ST_NEAR], lds);
}

// The cumulative rule of Sec. 3 (Details) over one chain, members in
// ascending order of `key` (a slot): the first member k with
// U * sum(p) <= p_1 + ... + p_k.  `key_of(e)` and `p_of(e)` read member e.
// A chain of up to CHAIN_REGS members is read once into registers and put in
// key order by a sorting network (Batcher's odd-even merge, 19 comparators;
// static indices only, so nothing goes to per-lane scratch): one pass of
// dependent loads instead of one per member and rank.  The sums run in the
// same order either way.
constexpr u32 CHAIN_REGS = 8;

template <class V> __device__ __forceinline__ void chain_cas(u32 *key, V *p, u32 *ent, int i, int j)
{
    if (key[j] < key[i]) {
        const u32 k = key[i], e = ent[i];
        const V v = p[i];
        key[i] = key[j];
        p[i] = p[j];
        ent[i] = ent[j];
        key[j] = k;
        p[j] = v;
        ent[j] = e;
    }
}

template <class K, class Pf>
__device__ inline u32 choose_in_chain(u32 head, const u32 *__restrict__ next, u32 count, double U, K &&key_of, Pf &&p_of)
{
    if (count <= CHAIN_REGS) {
        u32 key[CHAIN_REGS], ent[CHAIN_REGS];
        double p[CHAIN_REGS];
        u32 e = head;
#pragma unroll
        for (int j = 0; j < (int)CHAIN_REGS; ++j) {
            if ((u32)j < count && e != NOSLOT) {
                key[j] = key_of(e);
                p[j] = p_of(e);
                ent[j] = e;
                e = next[e];
            } else {
                key[j] = NOSLOT;
                p[j] = 0.0;
                ent[j] = NOSLOT;
            }
        }
        chain_cas(key, p, ent, 0, 1); chain_cas(key, p, ent, 2, 3); chain_cas(key, p, ent, 4, 5); chain_cas(key, p, ent, 6, 7);
        chain_cas(key, p, ent, 0, 2); chain_cas(key, p, ent, 1, 3); chain_cas(key, p, ent, 4, 6); chain_cas(key, p, ent, 5, 7);
        chain_cas(key, p, ent, 1, 2); chain_cas(key, p, ent, 5, 6);
        chain_cas(key, p, ent, 0, 4); chain_cas(key, p, ent, 1, 5); chain_cas(key, p, ent, 2, 6); chain_cas(key, p, ent, 3, 7);
        chain_cas(key, p, ent, 2, 4); chain_cas(key, p, ent, 3, 5);
        chain_cas(key, p, ent, 1, 2); chain_cas(key, p, ent, 3, 4); chain_cas(key, p, ent, 5, 6);
        double T_ = 0.0;
#pragma unroll
        for (int j = 0; j < (int)CHAIN_REGS; ++j)
            if (key[j] != NOSLOT) T_ += p[j];
        const double tgt = U * T_;
        double acc = 0.0;
        u32 win = NOSLOT;
        bool done = false;
#pragma unroll
        for (int j = 0; j < (int)CHAIN_REGS; ++j)
            if (!done && key[j] != NOSLOT) {
                acc += p[j];
                win = ent[j];
                done = tgt <= acc;
            }
        return win;
    }
    double T_ = 0.0;
    u32 prev = 0;
    bool first = true;
    for (u32 r = 0; r < count; ++r) {
        u32 best = NOSLOT, be = NOSLOT;
        for (u32 e = head; e != NOSLOT; e = next[e]) {
            const u32 s = key_of(e);
            if ((first || s > prev) && s < best) {
                best = s;
                be = e;
            }
        }
        if (be == NOSLOT) break;
        T_ += p_of(be);
        prev = best;
        first = false;
    }
    const double tgt = U * T_;
    double acc = 0.0;
    u32 win = NOSLOT;
    first = true;
    for (u32 r = 0; r < count; ++r) {
        u32 best = NOSLOT, be = NOSLOT;
        for (u32 e = head; e != NOSLOT; e = next[e]) {
            const u32 s = key_of(e);
            if ((first || s > prev) && s < best) {
                best = s;
                be = e;
            }
        }
        if (be == NOSLOT) break;
        acc += p_of(be);
        prev = best;
        first = false;
        win = be;
        if (tgt <= acc) break;
    }
    return win;
}

// ---------------------------------------------------------------------------
// K5c: A-side choice.  The candidate with the smallest B slot of each A
// chain leads; it applies the rule with U = {a, -, step, SELA} and chains
// the chosen entry under its B record.
// ---------------------------------------------------------------------------
template <bool BATCH>
__global__ __launch_bounds__(BLOCK) void k_select_a(Params P, const PairEnt *__restrict__ list, const CandEnt *__restrict__ cand,
                                                     u32 *__restrict__ flag, const u64 *__restrict__ headA,
                                                     const u32 *__restrict__ nextA, u64 *__restrict__ headB, u32 *__restrict__ nextB,
                                                     Counters *C, DbgPick *dbg)
{
    __shared__ u32 lds[BLOCK / 64];
    const u32 step = C->step;
    const PairIndex pi(C, P);
    if (blockIdx.x * BLOCK >= pi.total) return;  // no pair for this workgroup (uniform)
    u32 picks = 0;
    for (u32 kk = gtid(); kk < pi.total; kk += gstride()) {
        const u32 k = pi.entry(kk);
        if (flag[k] == PE_PAIR) continue;
        const CandEnt me = cand[k];
        const u32 h = (u32)headA[list[k].a_idx];
        u32 mins = NOSLOT, count = 0;
        for (u32 e = h; e != NOSLOT; e = nextA[e]) {
            mins = min(mins, cand[e].b_slot);
            ++count;
        }
        if (me.b_slot != mins) continue;
        u32 win = k;
        if (count > 1) {
            const Params &Q = rep_params<BATCH>(P, me.a_slot);
            const double U = u01(philox(local_slot<BATCH>(Q, me.a_slot), NOSLOT, local_step<BATCH>(Q, step), TAG_SELA, Q.key).x);
            win = choose_in_chain(h, nextA, count, U, [&](u32 e) { return cand[e].b_slot; }, [&](u32 e) { return cand[e].p; });
            if (win == NOSLOT) win = k;
        }
        flag[win] = PE_PICKED;
        ++picks;
        nextB[win] = chain_push(headB, list[win].b_idx, win, step);
        if (P.debug) {
            const u32 d = atomicAdd(&C->n_dbg[1], 1u);
            if (d < P.dbg_cap) {
                DbgPick g;
                g.i = cand[win].a_slot; g.j = cand[win].b_slot; g.p = cand[win].p;
                dbg[d] = g;
            }
        }
    }
    block_add_stats(&picks, 1, &C->stats[ST_PICKS], lds);
}

constexpr u32 EV_DECAY = 0x80000000u;

// ---------------------------------------------------------------------------
// K6: B-side choice.  The picked entry with the smallest A slot of each B
// chain leads; it applies the rule with U = {b, -, step, SELB} and queues the
// winning pair as an event.
// ---------------------------------------------------------------------------
// Blocks [0, nb_sel) run the B-side choice over the pair list; the others
// mark the C records (binned at the start of the step) that decay:
// xi < 1 - e^{-k_off dt}, xi = {c, -, step, UNI} (eq. rad_prob, step 4).
template <class T, bool BATCH>
__global__ __launch_bounds__(BLOCK) void k_select_b(Params P, const PairEnt *__restrict__ list, const CandEnt *__restrict__ cand,
                                                     const u32 *__restrict__ flag, const u64 *__restrict__ headB,
                                                     const u32 *__restrict__ nextB, const Rec<T> *__restrict__ rec,
                                                     const u32 *__restrict__ start, const u32 *__restrict__ okey, u32 *__restrict__ ev,
                                                     Counters *C, u32 nb_sel)
{
    __shared__ u32 lds[BLOCK / 64];
    __shared__ u32 base;
    const u32 step = C->step;
    if (blockIdx.x >= nb_sel) {
        if (!P.reversible) return;
        const u32 beg = start[2 * P.n_cells], end = start[3 * P.n_cells];
        const u32 ts = (gridDim.x - nb_sel) * BLOCK;
        for (u32 b0 = beg + (blockIdx.x - nb_sel) * BLOCK; b0 < end; b0 += ts) {  // uniform over the workgroup
            const u32 i = b0 + threadIdx.x;
            bool dec = false;
            if (i < end) {
                const u32 sc = meta_slot(rec_meta(rec[i]));
                const Params &Q = BATCH ? P.reps[rep_of_key(P, okey[i])] : P;  // C records binned this step
                dec = below(philox(local_slot<BATCH>(Q, sc), NOSLOT, local_step<BATCH>(Q, step), TAG_UNI, Q.key).x, P.p_uni);
            }
            block_append(ev, &C->n_ev, dec, EV_DECAY | i, lds, &base);
        }
        return;
    }
    const PairIndex pi(C, P);
    if (blockIdx.x * BLOCK >= pi.total) return;  // no pair for this workgroup (uniform)
    u32 n_match = 0;
    for (u32 b0 = blockIdx.x * BLOCK; b0 < pi.total; b0 += nb_sel * BLOCK) {  // uniform over the workgroup
        const u32 kk = b0 + threadIdx.x;
        u32 win = NOSLOT;
        if (kk < pi.total) {
            const u32 k = pi.entry(kk);
            if (flag[k] == PE_PICKED) {
                const u32 h = (u32)headB[list[k].b_idx];
                u32 mins = NOSLOT, count = 0;
                for (u32 e = h; e != NOSLOT; e = nextB[e]) {
                    mins = min(mins, cand[e].a_slot);
                    ++count;
                }
                if (cand[k].a_slot == mins) {
                    win = k;
                    if (count > 1) {
                        const Params &Q = rep_params<BATCH>(P, cand[k].b_slot);
                        const double U =
                            u01(philox(local_slot<BATCH>(Q, cand[k].b_slot), NOSLOT, local_step<BATCH>(Q, step), TAG_SELB, Q.key).x);
                        win = choose_in_chain(h, nextB, count, U, [&](u32 e) { return cand[e].a_slot; },
                                              [&](u32 e) { return cand[e].p; });
                        if (win == NOSLOT) win = k;
                    }
                }
            }
        }
        n_match += win != NOSLOT;
        block_append(ev, &C->n_ev, win != NOSLOT, win, lds, &base);
    }
    block_add_stats(&n_match, 1, &C->stats[ST_MATCHES], lds);
}

// K9: close the step (one workgroup, after the events): thread s < ST_N
// moves counter s into the per-step and running sums; thread 0 then sets up
// the next step.  A kernel of its own rather than a last-block test in the
// event kernel: that test costs one same-address atomic per workgroup.
__global__ void k_close(Counters *C)
{
    const int s = threadIdx.x;
    __shared__ u32 n_pl;
    if (s == 0) {
        u32 t = 0;
        for (u32 x = 0; x < PL_SEGS; ++x) t += C->pl_seg[x * PL_STRIDE];
        n_pl = t;
    }
    __syncthreads();
    if (s < ST_N) {
        const u64 v = s == ST_PAIRS ? (u64)n_pl : C->stats[s];
        C->stats_last[s] = v;
        C->stats_sum[s] += v;
        C->stats[s] = 0;
    }
    if (s < (int)PL_SEGS) C->pl_seg[s * PL_STRIDE] = 0;
    __syncthreads();
    if (s == 0) {
        C->n_rec = C->n_live + C->n_append;
        C->n_sorted = C->n_live;  // records [0, n_live) carry their bucket keys
        C->n_pl = n_pl;
        C->n_append = C->n_ev = 0;
        C->step += 1u;
    }
}

// ---------------------------------------------------------------------------
// K7: the events of the step, one wave per event.
//  match (Sec. 3, steps 2a-2c): absorbing pairs react; reflecting and
//    radiation pairs get R'' from the radial propagator and radiation pairs
//    react with p_reac; the centre R (eq. Rcoo) keeps its free end point and
//    the pair keeps the direction of its free separation.
//  decay (Sec. 2.2.5): R'' from the propagator with r0 = a, geminate
//    recombination with p_reac(R''|a), otherwise A and B placed R'' apart
//    along a uniform direction around the old C, B into the reserved slot.
// Wave form (LANE = false): one wave per event, every lane computes the same
// values, the rejection attempts are spread over the lanes, lane 0 writes.
// Lane form (LANE = true): one event per lane, attempts one after another.
// Both return their counts (react, attempts, bound hits, near, decay,
// geminate; zero on lanes other than 0 in the wave form), which the kernel
// sums per workgroup.
// ---------------------------------------------------------------------------
constexpr int EV_ST = 6;
struct EvCount {
    u32 v[EV_ST];
};

// A propagated pair's hand-off to the angle stage (angle_wg.hpp); on = 0: no angle.
struct AngEnt {
    u32 ia, ib, on, dbg;
    double Rpp, R0;
};

template <int DIM, class T, int NC, bool LANE>
__device__ __forceinline__ EvCount ev_match(const Params &P, Rec<T> *__restrict__ rec, u32 ia, u32 ib, double R0,
                                         u32 *__restrict__ partner, u32 step, Counters *C, DbgMatch *dbg, AngEnt *ang)
{
#pragma clang fp contract(off)
    Rec<T> ra = rec[ia], rb = rec[ib];
    const u32 sa = meta_slot(rec_meta(ra)), sb = meta_slot(rec_meta(rb));
    const u32 la = sa - P.slot_base, lb = sb - P.slot_base;  // the draws are keyed on replica-local slots
    step -= P.step_base;                                       // and on the replica's own step
    const double xa[3] = {(double)ra.x, (double)ra.y, (double)ra.z};
    const double xb[3] = {(double)rb.x, (double)rb.y, (double)rb.z};
    double rv[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
    for (int d = 0; d < DIM; ++d) {
        rv[d] = min_image_d(xb[d] - xa[d], P.L[d], P.Lh[d]);
        r2 += rv[d] * rv[d];
    }
    const double R = sqrt(r2) / P.a;
    bool react;
    double Rpp = R, preac = 1.0;
    u32 att = 0, hits = 0, near = 0, wreac = 0;
    if (P.bc == 0) {
        react = true;
    } else {
        Rpp = LANE ? sample_radius_lane<DIM, NC>(P, R0, la, lb, step, TAG_PROP, &att, &hits)
                   : sample_radius_wave<DIM, NC>(P, R0, la, lb, step, TAG_PROP, &att, &hits);
        preac = reac_prob<NC>(P, DIM, Rpp, R0);
        wreac = philox(la, lb, step, TAG_REAC, P.key).x;
        react = below(wreac, preac);
        near = fabs(u01(wreac) - preac) < 1e-6;
        if (!react && !P.angles) {  // keep the free end point's direction
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
    if (react) {
        T nc[3] = {0, 0, 0};
        for (int d = 0; d < DIM; ++d) nc[d] = wrap_store<T>(xa[d] + P.fA * rv[d], P.L[d]);
        ra.x = nc[0]; ra.y = nc[1]; ra.z = nc[2];
        rec_set_meta(ra, meta_make(SP_C, sa));
        rec_set_meta(rb, meta_make(SP_DEAD, sb));
    }
    EvCount cnt = {{0, 0, 0, 0, 0, 0}};
    if (LANE || lane_id() == 0) {
        if (react) partner[sa] = P.reversible ? sb : NOSLOT;
        rec[ia] = ra;
        rec[ib] = rb;
        cnt.v[0] = react;
        cnt.v[1] = att;
        cnt.v[2] = hits;
        cnt.v[3] = near;
        u32 q = NOSLOT;
        if (P.debug) {
            q = atomicAdd(&C->n_dbg[2], 1u);
            if (q < P.dbg_cap) {
                DbgMatch d;
                d.i = sa; d.j = sb; d.reacted = react; d.attempts = att; d.draw = wreac; d.pad = 0;
                d.Rpp = Rpp; d.preac = preac; d.cos_theta = __builtin_nan("");
                dbg[q] = d;
            }
        }
        // the angle stage places a propagated pair (its post-move positions are left as they are)
        if (ang) {
            AngEnt g;
            g.ia = ia; g.ib = ib; g.on = !react && P.angles; g.dbg = q; g.Rpp = Rpp; g.R0 = R0;
            *ang = g;
        }
    }
    return cnt;
}

template <int DIM, class T, int NC, bool LANE>
__device__ __forceinline__ EvCount ev_decay(const Params &P, Rec<T> *__restrict__ rec, u32 i, u32 *__restrict__ partner, u32 step,
                                         Counters *C, DbgDiss *dbg)
{
#pragma clang fp contract(off)
    const Rec<T> rc = rec[i];
    const u32 sc = meta_slot(rec_meta(rc)), lc = sc - P.slot_base;
    step -= P.step_base;
    u32 att = 0, hits = 0;
    const double Rpp = LANE ? sample_radius_lane<DIM, NC>(P, 1.0, lc, NOSLOT, step, TAG_DPROP, &att, &hits)
                            : sample_radius_wave<DIM, NC>(P, 1.0, lc, NOSLOT, step, TAG_DPROP, &att, &hits);
    const double preac = reac_prob<NC>(P, DIM, Rpp, 1.0);
    const u32 wgem = philox(lc, NOSLOT, step, TAG_GEM, P.key).x;
    const bool gem = below(wgem, preac);
    const u32 sb = partner[sc];
    EvCount cnt = {{0, 0, 0, 0, 0, 0}};
    if (LANE || lane_id() == 0) {
        cnt.v[4] = 1;
        cnt.v[5] = gem;
        cnt.v[1] = att;
        cnt.v[2] = hits;
        if (P.debug) {
            const u32 q = atomicAdd(&C->n_dbg[3], 1u);
            if (q < P.dbg_cap) {
                DbgDiss d;
                d.c = sc; d.j = sb; d.decayed = 1; d.recombined = gem; d.attempts = att; d.draw = wgem; d.Rpp = Rpp; d.preac = preac;
                dbg[q] = d;
            }
        }
    }
    if (gem) return cnt;
    const uint4 r = philox(lc, NOSLOT, step, TAG_DIR, P.key);
    double e[3] = {0.0, 0.0, 0.0};
    if (DIM == 3) {
        const double z = 2.0 * u01(r.x) - 1.0, rho = sqrt(1.0 - z * z);
        double sp, cp;
        sincos_turn<T>(u01(r.y), &sp, &cp);
        e[0] = rho * cp;
        e[1] = rho * sp;
        e[2] = z;
    } else {
        sincos_turn<T>(u01(r.x), &e[1], &e[0]);
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
    if (LANE || lane_id() == 0) {
        partner[sc] = NOSLOT;
        rec[i] = ra;
        const u32 q = C->n_live + atomicAdd(&C->n_append, 1u);
        if (q < P.cap) rec[q] = rb;
        else atomicOr(&C->err, (u32)ERR_APPEND);
    }
    return cnt;
}

// The handlers are inlined: called, they keep their frames and the registers
// saved around the calls in per-lane scratch memory, whose loads then sit on
// each event's chain of dependent operations.  They read the parameters from
// a device-resident copy (a by-value kernel argument would be copied to
// per-lane scratch to be passed by reference).  Up to EV_LANE_MIN - 1 events
// run one per wave, more run one per lane.
constexpr u32 EV_LANE_MIN = 4096;

// the parameters of the replica of record i (a single system: its own)
template <bool BATCH, class T> __device__ __forceinline__ const Params &ev_params(const Params &P, const Rec<T> *rec, u32 i)
{
    if constexpr (BATCH) return rep_params<true>(P, meta_slot(rec_meta(rec[i])));
    else return P;
}

// ang (null when no pair draws an angle): event w's hand-off to the angle stage.
template <int DIM, class T, int NC, bool BATCH>
__global__ __launch_bounds__(BLOCK) void k_events(const Params *__restrict__ Pd, Rec<T> *__restrict__ rec,
                                                   const PairEnt *__restrict__ list, const CandEnt *__restrict__ cand,
                                                   const u32 *__restrict__ ev, u32 *__restrict__ partner, Counters *C,
                                                   DbgMatch *dbg_m, DbgDiss *dbg_d, AngEnt *ang)
{
    __shared__ u32 lds[BLOCK / 64];
    const Params &P = *Pd;
    const u32 step = C->step;
    const u32 n = min(C->n_ev, P.cap);
    // a workgroup with no event (uniform) has nothing to count either
    if (blockIdx.x * (n >= EV_LANE_MIN ? BLOCK : BLOCK / 64) >= n) return;
    u32 st[EV_ST] = {0, 0, 0, 0, 0, 0};
    auto add = [&](const EvCount &c) {
#pragma unroll
        for (int k = 0; k < EV_ST; ++k) st[k] += c.v[k];
    };
    if (n >= EV_LANE_MIN) {
        for (u32 w = gtid(); w < n; w += gstride()) {
            const u32 e = ev[w];
            if (e & EV_DECAY) {
                const u32 i = e & ~EV_DECAY;
                add(ev_decay<DIM, T, NC, true>(ev_params<BATCH>(P, rec, i), rec, i, partner, step, C, dbg_d));
                if (ang) ang[w].on = 0;
            } else {
                add(ev_match<DIM, T, NC, true>(rep_params<BATCH>(P, cand[e].a_slot), rec, list[e].a_idx, list[e].b_idx,
                                               cand[e].R0, partner, step, C, dbg_m, ang ? ang + w : nullptr));
            }
        }
    } else {
        const u32 wave = (blockIdx.x * BLOCK + threadIdx.x) >> 6, nwaves = (gridDim.x * BLOCK) >> 6;
        for (u32 w = wave; w < n; w += nwaves) {
            const u32 e = ev[w];
            if (e & EV_DECAY) {
                const u32 i = e & ~EV_DECAY;
                add(ev_decay<DIM, T, NC, false>(ev_params<BATCH>(P, rec, i), rec, i, partner, step, C, dbg_d));
                if (ang && lane_id() == 0) ang[w].on = 0;
            } else {
                add(ev_match<DIM, T, NC, false>(rep_params<BATCH>(P, cand[e].a_slot), rec, list[e].a_idx, list[e].b_idx,
                                                cand[e].R0, partner, step, C, dbg_m, ang ? ang + w : nullptr));
            }
        }
    }
    // counts: one atomic per counter and workgroup
    const int map[EV_ST] = {ST_REACT, ST_ATTEMPTS, ST_BOUND, ST_NEAR, ST_DECAY, ST_GEMINATE};
#pragma unroll
    for (int k = 0; k < EV_ST; ++k) {
        const u32 t = block_sum(st[k], lds);
        if (threadIdx.x == 0 && t) atomicAdd((unsigned long long *)&C->stats[map[k]], (unsigned long long)t);
    }
}

// ---------------------------------------------------------------------------
// p_enc and p_reac of caller-given (R, R0) pairs with the step's own device
// functions (overlap rule included), one thread per pair.
// ---------------------------------------------------------------------------
template <int DIM, int PM, int NC>
__global__ __launch_bounds__(BLOCK) void k_eval_probs(Params P, uint64_t n, const double *__restrict__ R, const double *__restrict__ R0,
                                                       double *__restrict__ penc, double *__restrict__ preac)
{
    for (uint64_t i = gtid(); i < n; i += gstride()) {
        const double r = R[i], r0 = R0[i];
        if (penc) penc[i] = r <= 1.0 ? 1.0 : penc_R<DIM, PM, NC>(P, r, r0);
        if (preac) preac[i] = reac_prob<NC>(P, DIM, r, r0);
    }
}

// R'' draws of the radial propagator for caller-given R0 with the step's own
// sampler: draw i uses the counter {i, 0xFFFFFFFF, step, PROP | attempt << 8}
// and the handle's key; one wave per draw (WAVE) or one lane per draw.
template <int DIM, int NC, bool WAVE>
__global__ __launch_bounds__(BLOCK) void k_eval_prop(Params P, uint64_t n, const double *__restrict__ R0, u32 step,
                                                      double *__restrict__ Rpp, u32 *__restrict__ attempts)
{
    if (WAVE) {
        const u32 wave = gtid() >> 6, nwaves = gstride() >> 6;
        for (uint64_t i = wave; i < n; i += nwaves) {
            u32 att = 0, hits = 0;
            const double r = sample_radius_wave<DIM, NC>(P, R0[i], (u32)i, NOSLOT, step, TAG_PROP, &att, &hits);
            if (lane_id() == 0) {
                Rpp[i] = r;
                if (attempts) attempts[i] = att;
            }
        }
    } else {
        for (uint64_t i = gtid(); i < n; i += gstride()) {
            u32 att = 0, hits = 0;
            Rpp[i] = sample_radius_lane<DIM, NC>(P, R0[i], (u32)i, NOSLOT, step, TAG_PROP, &att, &hits);
            if (attempts) attempts[i] = att;
        }
    }
}

// ---------------------------------------------------------------------------
// First contact of a pair by bisection of the step (Appendix).  The pair's
// separation (units of a) went from xi to xf over tau = D_eff dt / a^2 with
// at least one encounter.  Each level halves the interval that holds the
// first contact: the midpoint separation is drawn from the Brownian bridge
// (eq. midPGauss: per coordinate mean (x_a + x_b)/2, variance tau_h for the
// half interval tau_h) conditioned on the encounter in the interval, i.e. a
// bridge proposal accepted with q = 1 - (1 - p1)(1 - p2), p1 and p2 the
// encounter probabilities of the halves (given the midpoint they are
// independent); the first half is kept with probability p1 / q.  Attempt k of
// level l draws {i, l, step, FPT | k << 8} (normals, by Box-Muller on words
// 0-1 and 2-3) and {i, l, step, FPTU | k << 8} (word 0 accepts, word 1
// chooses).  A level whose MAX_ATTEMPTS proposals are all rejected ends the
// refinement: the interval reached is kept (its lower end at the requested
// resolution) and bit 31 of the attempt count is set.  3D: the closed-form
// encounter probability; 2D: the expansion of compile-time order NC.
// The acceptance of the first level is the pair's whole encounter
// probability, which for some candidates is small, so one lane per pair would
// leave most lanes of a wave waiting for its slowest pair.  FP_GROUP lanes
// share a pair instead: lane s of the group evaluates attempts s, s + G, ...
// and the first accepted attempt in order wins, exactly as if the attempts
// were tried one after another.
// ---------------------------------------------------------------------------
constexpr u32 FP_GROUP = 16;

__device__ __forceinline__ double penc3_fp(double R, double R0, double tau)
{
    if (R <= 1.0 || R0 <= 1.0) return 1.0;
    return penc3_args((R - 1.0) * (R0 - 1.0) / tau, (R + R0 - 1.0) / tau, R * R0 / tau);
}

template <int DIM, int NC> __device__ __forceinline__ double penc_fp(const Params &P, double R, double R0, double tau)
{
    if constexpr (DIM == 3) return penc3_fp(R, R0, tau);
    if (R <= 1.0 || R0 <= 1.0) return 1.0;
    return penc2_at<NC>(P, R, R0, tau, sqrt(tau), 1.0 / tau);
}

template <int DIM, int NC>
__global__ __launch_bounds__(BLOCK) void k_first_passage(Params P, uint64_t n, const double *__restrict__ xi,
                                                          const double *__restrict__ xf, int levels, u32 step,
                                                          uint64_t *__restrict__ lo_out, u32 *__restrict__ att_out)
{
#pragma clang fp contract(off)
    const u32 lane = lane_id(), sub = lane % FP_GROUP, gbase = lane - sub;
    const uint64_t stride = gstride() / FP_GROUP;
    for (uint64_t i = gtid() / FP_GROUP; i < n; i += stride) {  // uniform over the group
        double xa[3], xb[3];
        for (int d = 0; d < 3; ++d) {
            xa[d] = d < DIM ? xi[3 * i + d] : 0.0;
            xb[d] = d < DIM ? xf[3 * i + d] : 0.0;
        }
        uint64_t lo = 0;
        u32 att = 0;
        for (int l = 0; l < levels; ++l) {
            const double th = P.tau / (double)(2ull << l);
            const double sd = sqrt(th);
            const double ra = sqrt(DIM == 3 ? xa[0] * xa[0] + xa[1] * xa[1] + xa[2] * xa[2] : xa[0] * xa[0] + xa[1] * xa[1]);
            const double rb = sqrt(DIM == 3 ? xb[0] * xb[0] + xb[1] * xb[1] + xb[2] * xb[2] : xb[0] * xb[0] + xb[1] * xb[1]);
            double xm[3], p1 = 1.0, q = 1.0, V = 0.0;
            int win = -1;
            for (u32 k0 = 0; k0 < MAX_ATTEMPTS; k0 += FP_GROUP) {  // uniform over the group
                const u32 k = k0 + sub;
                const uint4 rz = philox((u32)i, (u32)l, step, TAG_FPT | (k << 8), P.key);
                const uint4 ru = philox((u32)i, (u32)l, step, TAG_FPTU | (k << 8), P.key);
                const double r0 = sqrt(-2.0 * log(u01(rz.x))), r1 = sqrt(-2.0 * log(u01(rz.z)));
                double s0, c0;
                sincos((2.0 * PI_D) * u01(rz.y), &s0, &c0);
                const double z[3] = {r0 * c0, r0 * s0, r1 * cos((2.0 * PI_D) * u01(rz.w))};
                for (int d = 0; d < 3; ++d) xm[d] = d < DIM ? 0.5 * (xa[d] + xb[d]) + sd * z[d] : 0.0;
                const double rm = sqrt(DIM == 3 ? xm[0] * xm[0] + xm[1] * xm[1] + xm[2] * xm[2] : xm[0] * xm[0] + xm[1] * xm[1]);
                p1 = penc_fp<DIM, NC>(P, rm, ra, th);
                const double p2 = penc_fp<DIM, NC>(P, rb, rm, th);
                q = 1.0 - (1.0 - p1) * (1.0 - p2);
                V = u01(ru.y);
                const u64 m = __ballot(u01(ru.x) < q);
                const u64 gm = (m >> gbase) & (FP_GROUP == 64 ? ~0ull : ((1ull << (FP_GROUP % 64)) - 1ull));
                if (gm) {  // uniform over the group
                    win = __ffsll((unsigned long long)gm) - 1;
                    att += k0 + (u32)win + 1u;
                    break;
                }
            }
            if (win < 0) {  // exhausted: keep the interval reached
                lo <<= (levels - l);
                att = (att + MAX_ATTEMPTS) | 0x80000000u;
                break;
            }
            const int src = (int)gbase + win;
            for (int d = 0; d < 3; ++d) xm[d] = __shfl(xm[d], src, 64);
            p1 = __shfl(p1, src, 64);
            q = __shfl(q, src, 64);
            V = __shfl(V, src, 64);
            lo *= 2;
            if (V * q < p1) {
                for (int d = 0; d < 3; ++d) xb[d] = xm[d];
            } else {
                for (int d = 0; d < 3; ++d) xa[d] = xm[d];
                lo += 1;
            }
        }
        if (sub == 0) {
            lo_out[i] = lo;
            if (att_out) att_out[i] = att;
        }
    }
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

// The displacement every live record took in this step's move, by slot, as the
// later stages regenerate it (debug).
template <int DIM, class T, int PM, bool BATCH>
__global__ void k_dbg_disp(const Params P, const Rec<T> *__restrict__ rec, const Counters *C, double *__restrict__ disp,
                           u32 cap)
{
    const u32 n = C->n_live, step = C->step;
    for (u32 i = gtid(); i < n; i += gstride()) {
        const Rec<T> r = rec[i];
        const u32 m = rec_meta(r), sp = meta_sp(m), s = meta_slot(m);
        if (sp > SP_C || s >= cap) continue;
        const Params &Q = rep_params<BATCH>(P, s);
        double d[3];
        displacement<DIM, T, PM>(Q, local_slot<BATCH>(Q, s), sp, local_step<BATCH>(Q, step), d);
        for (int k = 0; k < DIM; ++k) disp[(u64)s * DIM + k] = d[k];
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

// ---------------------------------------------------------------------------
// Pool membership (between steps).  A member that leaves has its records
// marked dead in place, which keeps the buffer's order of bucket keys, and
// the next binning drops them.  A compaction moves the live records to the
// front of the other buffer in any order (no result depends on the order of
// records: every choice among candidates goes by slot) and makes the next
// binning treat every record as moved.
// ---------------------------------------------------------------------------
template <class T> __global__ __launch_bounds__(BLOCK) void k_retire(Rec<T> *__restrict__ rec, const Counters *C, u32 lo, u32 hi)
{
    const u32 n = C->n_rec;
    for (u32 i = gtid(); i < n; i += gstride()) {
        Rec<T> r = rec[i];
        const u32 m = rec_meta(r), s = meta_slot(m);
        if (meta_sp(m) <= SP_C && s >= lo && s < hi) {
            rec_set_meta(r, meta_make(SP_DEAD, s));
            rec[i] = r;
        }
    }
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_compact(const Rec<T> *__restrict__ in, Rec<T> *__restrict__ out, Counters *C)
{
    __shared__ u32 lds[BLOCK / 64];
    __shared__ u32 base;
    const u32 n = C->n_rec;
    for (u32 b0 = blockIdx.x * BLOCK; b0 < n; b0 += gridDim.x * BLOCK) {  // uniform over the workgroup
        const u32 i = b0 + threadIdx.x;
        Rec<T> r;
        bool keep = false;
        if (i < n) {
            r = in[i];
            keep = meta_sp(rec_meta(r)) <= SP_C;
        }
        u32 total;
        const u32 ex = block_excl_scan(keep ? 1u : 0u, lds, total);
        if (threadIdx.x == 0) base = total ? atomicAdd(&C->n_kept, total) : 0u;
        __syncthreads();
        if (keep) out[base + ex] = r;
        __syncthreads();  // base is rewritten by the next chunk
    }
}

__global__ void k_compact_done(Counters *C)
{
    if (gtid() == 0) {
        C->n_rec = C->n_live = C->n_kept;
        C->n_sorted = 0;  // the old bucket keys no longer line up with the records
        C->n_kept = 0;
    }
}

} // namespace gfbd
