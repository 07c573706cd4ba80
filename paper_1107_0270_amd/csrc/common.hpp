// Shared types of the gfx950 Green's-function Brownian-dynamics library:
// particle records, kernel parameters, device counters and the Philox4x32-10
// counter-based generator (Salmon et al., SC'11).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gfbd {

typedef uint32_t u32;
typedef uint64_t u64;

// Species code held in the top three bits of a record's meta word; the low
// 29 bits hold the slot.
constexpr u32 SP_A = 0, SP_B = 1, SP_C = 2, SP_DEAD = 7;
constexpr u32 SLOT_MASK = (1u << 29) - 1;
constexpr u32 NOSLOT = 0xFFFFFFFFu;
__host__ __device__ inline u32 meta_make(u32 sp, u32 slot) { return (sp << 29) | slot; }
__host__ __device__ inline u32 meta_sp(u32 m) { return m >> 29; }
__host__ __device__ inline u32 meta_slot(u32 m) { return m & SLOT_MASK; }

// Counter word 3: tag in the low byte, rejection-attempt index above it.
enum : u32 {
    TAG_MOVE = 1, TAG_ENC = 2, TAG_SELA = 3, TAG_SELB = 4, TAG_PROP = 5, TAG_REAC = 6,
    TAG_UNI = 7, TAG_DPROP = 8, TAG_DIR = 9, TAG_GEM = 10, TAG_FPT = 11, TAG_FPTU = 12, TAG_ANG = 13
};

// Arithmetic of the pair probability: binary64 throughout, binary32, or
// binary32 with binary64 separations and exponent arguments (displacements in
// binary64, or in binary32 as the plain mode takes them: PM_F32D).
enum { PM_F64 = 0, PM_F32 = 1, PM_F32NC = 2, PM_F32D = 3 };

struct Key {
    u32 k0, k1;
};

// Philox4x32-10: ten S-P rounds with multipliers 0xD2511F53, 0xCD9E8D57 and
// the Weyl key increments 0x9E3779B9, 0xBB67AE85.
__device__ __forceinline__ uint4 philox(u32 c0, u32 c1, u32 c2, u32 c3, Key k)
{
    u32 k0 = k.k0, k1 = k.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product gives both halves
        const u64 p0 = (u64)0xD2511F53u * c0, p1 = (u64)0xCD9E8D57u * c2;
        const u32 n0 = (u32)(p1 >> 32) ^ c1 ^ k0, n2 = (u32)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (u32)p1;
        c2 = n2;
        c3 = (u32)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Uniform (w + 1/2) 2^-32 in (0, 1), exact in binary64.
__device__ __forceinline__ double u01(u32 w) { return ((double)w + 0.5) * 0x1p-32; }

// The Bernoulli rule "xi < p" with xi = u01(w), evaluated exactly.
__device__ __forceinline__ bool below(u32 w, double p) { return ((double)w + 0.5) < p * 0x1p32; }

// Particle record: three coordinates and a meta word in the fourth lane
// (z is 0 in 2D).  16 bytes in binary32, 32 bytes in binary64.
template <class T> struct alignas(4 * sizeof(T)) Rec {
    T x, y, z, w;
};

__host__ __device__ inline u32 rec_meta(const Rec<float> &r)
{
    union { float f; u32 u; } c;
    c.f = r.w;
    return c.u;
}
__host__ __device__ inline u32 rec_meta(const Rec<double> &r)
{
    union { double f; u64 u; } c;
    c.f = r.w;
    return (u32)c.u;
}
__host__ __device__ inline void rec_set_meta(Rec<float> &r, u32 m)
{
    union { float f; u32 u; } c;
    c.u = m;
    r.w = c.f;
}
__host__ __device__ inline void rec_set_meta(Rec<double> &r, u32 m)
{
    union { double f; u64 u; } c;
    c.u = m;
    r.w = c.f;
}

constexpr int MAXTERMS = 32;

// Everything a kernel needs to know about the model and the grid.  Passed by
// value; derived once on the host in binary64.
struct Params {
    int dim;
    int bc;          // 0 absorbing, 1 reflecting, 2 radiation
    int reversible;  // k_off > 0
    int n_terms;     // 2D expansion order
    int angles;      // propagated pairs draw their angle to the old separation (else keep the free direction)
    double L[3], Lh[3];
    double cs[3];    // cells per um along each axis (n / L)
    double ce[3];    // cell edge along each axis (L / n)
    double reach;    // r_cut plus a rounding margin: neighbour cells farther away are skipped
    int nc[3];
    u32 n_cells, n_keys;
    double sd[3];    // sqrt(2 D dt) of A, B, C
    double a, inv_a, tau, inv_tau, sqrt_tau, hh;
    double rcut, rcut2;
    float rcut2f, rcut2f_wide, rcut2f_pre, inv_af, inv_tauf, Lf[3], Lhf[3];
    double fA, fB;   // D_A / D_eff, D_B / D_eff
    double p_uni;    // 1 - exp(-k_off dt)
    Key key;
    u32 cap;
    u32 cap_pl;          // capacity of the per-step pair list (PL_SEGS segments of seg_cap)
    u32 seg_cap;
    u32 cnt_region;      // words per region of the bucket counters (keys padded to whole scan tiles / 16)
    int tiled;           // pair search through LDS bricks (all edges >= 3 cells)
    int bx, by, bz;      // brick edges in cells
    u32 nbx, nby, nbz;   // bricks per axis
    u32 debug;
    u32 dbg_cap;
    const double *g2c;  // 2D constants: a_k(0), Q_abs, Q_ref, Q_rad (4 x (MAXTERMS+1))
    // exact 2D radial functions (green2x.hpp): tables over R = 1 + i h (i < x2_nr) and
    // R0 = 1 + 2 j h (j < x2_n0): p_enc and p_reac in binary32 tiles of 8 x 4 (x2_ntr row
    // tiles), the propagator's distribution function in binary64 with column j contiguous;
    // pairs with R0 > x2_r0sw take p_enc and p_reac from the small-time expansions, pairs with
    // R0 > x2_r0sw_prop their propagation
    const float *x2_enc, *x2_reac;
    const double *x2_cdf;
    double x2_h, x2_inv_h, x2_inv_h0, x2_r0sw, x2_r0sw_prop;
    u32 x2_nr, x2_n0, x2_n0_prop;  // rows, columns; columns the propagator's interpolation may read
    u32 x2_ntr;                    // row tiles of the p_enc and p_reac tables
    // Batches of independent replicas: replica r owns slots [slot_base,
    // slot_base + n) and cells [cell_base, cell_base + own cell count) of
    // every species block.  A single system is replica 0 with both bases 0.
    u32 slot_base, cell_base;
    u32 step_base;            // the replica's own step is the step counter minus this (mod 2^32)
    u32 n_rep;
    const u32 *rep_of_slot;   // replica of every slot (batches only)
    const u32 *cell_rep;      // replica of every cell (batches only)
    const Params *reps;       // per-replica parameters (batches only)
};

enum {
    ST_PAIRS = 0, ST_CAND, ST_OVERLAP, ST_R0CLAMP, ST_PICKS, ST_MATCHES, ST_REACT, ST_DECAY,
    ST_GEMINATE, ST_ATTEMPTS, ST_BOUND, ST_NEAR, ST_LDS_FALLBACK, ST_N
};

enum { ERR_PAIRS = 1, ERR_APPEND = 8 };

// The per-step pair list is cut into PL_SEGS segments of cap_pl / PL_SEGS
// entries, each with its own counter on its own 256-byte line: workgroup b
// appends to segment b mod PL_SEGS, so the appends of a step spread over
// PL_SEGS addresses (atomics on one address are serialised).  Pair k of the
// step (0 <= k < the sum of the counts) is entry k - (pairs in earlier
// segments) of its segment.
constexpr u32 PL_SEGS = 16;
constexpr u32 PL_STRIDE = 64;  // words between segment counters

// Device-resident counters; the work sizes of the data-dependent stages live
// here so that no stage needs the host to learn a count.
struct Counters {
    u32 n_rec;      // records in the current buffer (sorted + appended)
    u32 n_live;     // records placed by the last binning
    u32 n_pl;       // A-B pairs within r_cut found by the last step (its segments summed)
    u32 n_append;
    u32 step;       // step number used by every draw of this step
    u32 err;
    u32 n_dbg[4];   // pairs, picks, matches, dissociations logged this step
    u32 cell_hw;    // cells in use from the start of every species block (a pool's high-water mark)
    u32 n_sorted;   // leading records whose bucket keys the last binning noted
    u32 n_kept;     // records kept by a pool compaction (zero between compactions)
    u32 pad[3];
    u64 stats[ST_N];
    u64 stats_last[ST_N];
    u64 stats_sum[ST_N];
    u32 pl_seg[PL_SEGS * PL_STRIDE];  // pairs appended to each segment (count at [x * PL_STRIDE])
    // events (matched pairs and decays) queued this step, on a cache line of its
    // own (the preceding words are segment padding, the following ones padding)
    u32 n_ev;
    u32 pad_ev[PL_STRIDE - 1];
};

// An A-B pair within r_cut (record indices in the sorted buffer).
struct PairEnt {
    u32 a_idx, b_idx;
};

// A candidate (p_enc accepted): its slots, p_enc and the binary64 initial
// separation R0 (clamped to >= 1) that its propagation starts from.
struct CandEnt {
    u32 a_slot, b_slot;
    double p;
    double R0;
};

// pair-list entry state
enum : u32 { PE_PAIR = 0, PE_CAND = 1, PE_PICKED = 2 };

// Debug log entries (same layout as the public sim_dbg_* structs).
struct DbgPair { u32 i, j; double R, R0, p; u32 draw; int cand; };
struct DbgPick { u32 i, j; double p; };
struct DbgMatch { u32 i, j; int reacted; u32 attempts, draw, pad; double Rpp, preac, cos_theta; };
struct DbgDiss { u32 c, j; int decayed, recombined; u32 attempts, draw; double Rpp, preac; };

} // namespace gfbd
