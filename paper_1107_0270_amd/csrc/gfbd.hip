// Host side of the gfx950 Green's-function BD library: the C-ABI of
// include/gfbd.h, parameter derivation, device state and the launch sequence
// of one step (Sec. 3 of Pruestel & Meier-Schellersheim, arXiv:1107.0270).
#include "../../include/gfbd.h"
#include "kernels.hpp"
#include "angle_wg.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace gfbd;

// Device memory of sim_eval_pairs_noalloc (see there): the 2D expansion constants.
static __device__ __align__(256) double scratch[4 * (MAXTERMS + 1)];

namespace {

thread_local std::string g_err;

// ---------------------------------------------------------------------------
// Host numerics for the derived parameters (binary64).
// ---------------------------------------------------------------------------
double h_erfcx(double x)
{
    if (x < 26.0) return std::exp(x * x) * std::erfc(x);
    // large-argument series 1/(x sqrt(pi)) (1 - 1/(2x^2) + 3/(4x^4) - 15/(8x^6) + 105/(16x^8))
    const double t = 1.0 / (2.0 * x * x);
    return (1.0 - t * (1.0 - 3.0 * t * (1.0 - 5.0 * t * (1.0 - 7.0 * t)))) / (x * 1.77245385090551602730);
}

// 1 - S(tau | R0): 3D absorbing erfc(u0)/R0; 3D radiation
// (h/(1+h)) [erfc(u0) - e^{-u0^2} erfcx(u0 + (1+h) sqrt tau)]/R0; 2D the
// planar bound erfc(u0).  u0 = (R0 - 1)/(2 sqrt tau).
double h_loss(int dim, int bc, double R0, double tau, double hh)
{
    const double st = std::sqrt(tau), u0 = (R0 - 1.0) / (2.0 * st);
    if (dim == 2) return std::erfc(u0);
    if (bc == SIM_BC_RADIATION) {
        const double kap = 1.0 + hh;
        return (hh / kap) * (std::erfc(u0) - std::exp(-u0 * u0) * h_erfcx(u0 + kap * st)) / R0;
    }
    return std::erfc(u0) / R0;
}

// Cut-off: 1 - S(dt | r_cut) = eps (Sec. 3, Details), by bisection on R >= 1.
double h_rcut(int dim, int bc, double a, double tau, double hh, double eps)
{
    if (h_loss(dim, bc, 1.0, tau, hh) <= eps) return a;
    double lo = 1.0, hi = 2.0;
    while (h_loss(dim, bc, hi, tau, hh) > eps) hi = 1.0 + 2.0 * (hi - 1.0);
    for (int it = 0; it < 300; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        (h_loss(dim, bc, mid, tau, hh) > eps ? lo : hi) = mid;
    }
    return a * hi;
}

// Power-series quotient z = x / y, truncated after n.  Host and device run the same
// correctly rounded operations (no contraction), so both give the same bits.
__host__ __device__ void h_series_div(const double *x, const double *y, int n, double *z)
{
#pragma clang fp contract(off)
    for (int k = 0; k <= n; ++k) {
        double s = x[k];
        for (int m = 1; m <= k; ++m) s -= y[m] * z[k - m];
        z[k] = s / y[0];
    }
}

// 2D constants: a_k(0) and the R-independent quotient series of the three
// boundary components (Sec. 4.2): Abar_0/A_0, Abar_1/A_1 and
// (Abar_1 - h s Abar_0)/(A_1 + h s A_0).
__host__ __device__ void h_g2_constants(double hh, double *out)
{
#pragma clang fp contract(off)
    const int n = MAXTERMS;
    double a0[MAXTERMS + 1], a1[MAXTERMS + 1], b0[MAXTERMS + 1], b1[MAXTERMS + 1], nu[MAXTERMS + 1], de[MAXTERMS + 1];
    a0[0] = a1[0] = 1.0;
    for (int k = 1; k <= n; ++k) {
        const double odd = 2.0 * k - 1.0;
        a0[k] = a0[k - 1] * (0.0 - odd * odd) / (8.0 * k);
        a1[k] = a1[k - 1] * (4.0 - odd * odd) / (8.0 * k);
    }
    for (int k = 0; k <= n; ++k) {
        b0[k] = (k % 2 ? -a0[k] : a0[k]);
        b1[k] = (k % 2 ? -a1[k] : a1[k]);
        nu[k] = b1[k] - (k ? hh * b0[k - 1] : 0.0);
        de[k] = a1[k] + (k ? hh * a0[k - 1] : 0.0);
    }
    for (int k = 0; k <= n; ++k) out[k] = a0[k];
    h_series_div(b0, a0, n, out + (n + 1));
    h_series_div(b1, a1, n, out + 2 * (n + 1));
    h_series_div(nu, de, n, out + 3 * (n + 1));
}

template <class T> T h_wrap_store(double y, double L)
{
    if (y < 0.0) y += L;
    else if (y >= L) y -= L;
    if (!(y >= 0.0 && y < L)) {
        y -= L * std::floor(y / L);
        if (!(y >= 0.0 && y < L)) y = 0.0;
    }
    T v = (T)y;
    if ((double)v >= L) v = (T)0;
    return v;
}

} // namespace

// ---------------------------------------------------------------------------
// The handle.
// ---------------------------------------------------------------------------
struct sim {
    std::string err;
    virtual ~sim() {}
    virtual int step(uint32_t n) = 0;
    virtual int step_async(uint32_t n) = 0;
    virtual int sync() = 0;
    virtual int read(int what, void *dst, uint64_t cap, uint64_t *written) = 0;
    virtual int load(uint64_t step, const int32_t *sp, const double *pos, const uint32_t *partner) = 0;
    virtual int eval_pairs(uint64_t n, const double *R, const double *R0, double *penc, double *preac) = 0;
    virtual int eval_prop(uint64_t n, const double *R0, uint32_t step, int wave, double *Rpp, uint32_t *attempts) = 0;
    virtual int eval_first_passage(uint64_t n, const double *xi, const double *xf, int levels, uint32_t step, uint64_t *lo,
                                   uint32_t *attempts) = 0;
    virtual int eval_angle(uint64_t n, const double *R, const double *R0, const double *u, double *out) = 0;
    virtual int admit(const sim_replica &, uint32_t *) { return fail(SIM_ESTATE, "not a pool"); }
    virtual int retire(uint32_t) { return fail(SIM_ESTATE, "not a pool"); }
    virtual int read_member(uint32_t, int, void *, uint64_t, uint64_t *) { return fail(SIM_ESTATE, "not a pool"); }
    int fail(int code, const std::string &msg)
    {
        err = msg;
        g_err = msg;
        return code;
    }
};

namespace {

#define HIPCHECK(expr)                                                                          \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(SIM_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

// default workgroups of the event kernel (sim_config.event_blocks)
constexpr unsigned EV_BLOCKS = 1024;
// expected B's tested per A above which the LDS brick search is chosen
constexpr double PAIR_TESTS_TILED = 8.0;

struct Model {
    int dim, prec, bc;
    double box[3], dt, D[3], sigma, kappa, k_off, eps, rcut_req, cell_req;
    int pair_search;
    int green2d;
    uint32_t flags;  // SIM_F_*
    u32 pair_blocks, event_blocks;  // launch shapes of the pair stage and the event kernel
    uint64_t seed;
    uint32_t replica;
    int n_terms;
    uint32_t debug, timing;
    uint64_t dbg_cap;
    hipStream_t stream;
};

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }
int validate_box(int dim, int prec, const double *box);
int validate_state(int dim, bool reversible, uint64_t n, const int32_t *sp, const double *pos, const uint32_t *pt);

// The physics of one system (or one replica of a batch) from its configuration: what the
// step's device functions and the kernel-level evaluations read, cut-off included.
void phys_params(const Model &M, Params &P)
{
    std::memset(&P, 0, sizeof(P));
    P.dim = M.dim;
    P.bc = M.bc;
    P.reversible = M.k_off > 0.0;
    P.n_terms = M.n_terms;
    P.angles = M.bc != SIM_BC_ABSORBING && !(M.flags & SIM_F_KEEP_DIRECTION);
    const double Deff = M.D[0] + M.D[1];
    P.a = M.sigma;
    P.inv_a = 1.0 / M.sigma;
    P.tau = Deff * M.dt / (M.sigma * M.sigma);
    P.inv_tau = 1.0 / P.tau;
    P.sqrt_tau = std::sqrt(P.tau);
    if (M.bc == SIM_BC_RADIATION)
        P.hh = M.dim == 3 ? M.kappa / (4.0 * M_PI * M.sigma * Deff) : M.kappa / (2.0 * M_PI * Deff);
    P.rcut = M.rcut_req > 0.0 ? M.rcut_req : h_rcut(M.dim, M.bc, M.sigma, P.tau, P.hh, M.eps);
    P.rcut2 = P.rcut * P.rcut;
    P.rcut2f = (float)P.rcut2;
    P.rcut2f_wide = (float)(P.rcut2 * (1.0 + 1e-4));
    {
        // prefilter radius for brick-relative binary32 coordinates: each
        // coordinate is off by at most two binary32 roundings of a value
        // below the box edge
        double lmax = 0.0;
        for (int k = 0; k < M.dim; ++k) lmax = std::max(lmax, M.box[k]);
        const double slack = 4.0 * std::ldexp(1.0, std::ilogb(lmax) - 23) * std::sqrt((double)M.dim);
        P.rcut2f_pre = (float)((P.rcut + slack) * (P.rcut + slack) * (1.0 + 1e-5));
        // neighbour cells farther than this from an A are skipped: the
        // margin exceeds every rounding of a binary32 coordinate below
        // the box edge by a factor of 16 or more
        P.reach = P.rcut * (1.0 + 1e-6) + 64.0 * std::ldexp(1.0, std::ilogb(lmax) - 23);
    }
    P.inv_af = (float)P.inv_a;
    P.inv_tauf = (float)P.inv_tau;
    P.fA = M.D[0] / Deff;
    P.fB = M.D[1] / Deff;
    P.p_uni = -std::expm1(-M.k_off * M.dt);
    P.key.k0 = (u32)M.seed;
    P.key.k1 = (u32)(M.seed >> 32) ^ M.replica;
    for (int s = 0; s < 3; ++s) P.sd[s] = std::sqrt(2.0 * M.D[s] * M.dt);
}


// First-fit allocator of index ranges in [0, cap) (the slots and cells of a
// pool), merging neighbours on release.
struct RangeAlloc {
    std::map<uint64_t, uint64_t> free_;  // start -> length
    void reset(uint64_t cap)
    {
        free_.clear();
        if (cap) free_[0] = cap;
    }
    bool take(uint64_t len, uint64_t &at)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < len) continue;
            at = it->first;
            const uint64_t rest = it->second - len;
            free_.erase(it);
            if (rest) free_[at + len] = rest;
            return true;
        }
        return false;
    }
    void give(uint64_t at, uint64_t len)
    {
        auto it = free_.emplace(at, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && at + len == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

template <int DIM, class T, int PM> struct Engine final : sim {
    Model M;
    Params P;
    uint64_t n = 0, stepno = 0;
    int cur = 0;
    uint32_t maxA = 0, maxC = 0, nb_scan = 0;
    u32 cell_hw = 0;  // a pool: cells taken by its members so far, from the start of each species block
    double cell_edge = 0.0, pair_tests = 0.0;
    bool narrow = false;
    // device memory
    Rec<T> *rec[2] = {nullptr, nullptr}, *tmp = nullptr;
    u32 *rank = nullptr, *cnt = nullptr, *scnt = nullptr, *okey = nullptr, *start = nullptr, *bsum = nullptr, *partner = nullptr;
    u32 *nkey = nullptr;  // batches: each moved record's new bucket key
    PairEnt *plist = nullptr;
    CandEnt *cand = nullptr;
    u32 *flag = nullptr, *nextA = nullptr, *nextB = nullptr, *ev = nullptr;
    bool angles = false;    // propagated pairs draw their angle (otherwise they keep their direction)
    AngEnt *ang = nullptr;  // hand-offs of the events to their angles when the events outnumber the workgroups
    GL16 gl16;              // 16-point Gauss-Legendre rule of the angular series
    u64 *headA = nullptr, *headB = nullptr;
    Counters *ctr = nullptr;
    Params *dparams = nullptr;  // device copy of P for kernels that call out-of-line functions
    // batches
    bool batch = false;
    std::vector<Params> reps_h;
    std::vector<double> rep_box;
    std::vector<u32> rep_of_slot_h;
    Params *d_reps = nullptr;
    u32 *d_rep_of_slot = nullptr, *d_cell_rep = nullptr;
    double *d_g2c_reps = nullptr;
    // pools: members join and leave between steps
    bool pool = false;
    std::vector<uint64_t> member_n;  // slots of each member entry, 0 if the entry is free
    RangeAlloc slot_free, cell_free;
    std::vector<double> x2_build;  // exact 2D tables: quadrature nodes, rows, columns (the last built)
    // exact 2D tables, one set per (h~, r_cut): the members of a batch or pool with equal kappa
    // share theirs; every set lives as long as the handle
    bool exact2d = false;
    struct X2Set {
        double hh, rcut;
        Params tab;  // its x2_* fields
    };
    std::vector<X2Set> x2_sets;
    hipStream_t own_stream = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    uint32_t n_bricks = 0;
    double *g2c = nullptr;
    double *g_pos = nullptr, *dbg_moved = nullptr, *dbg_disp = nullptr;
    int *g_sp = nullptr;
    u32 *dbg_cells = nullptr;
    DbgPair *dbg_pairs = nullptr;
    DbgPick *dbg_picks = nullptr;
    DbgMatch *dbg_matches = nullptr;
    DbgDiss *dbg_diss = nullptr;
    std::vector<void *> allocs;
    // timing
    struct EvPair { hipEvent_t a, b; int k; };
    std::vector<EvPair> ev_pool, ev_used;
    double k_ms[SIM_K_N] = {0};
    uint64_t k_launches[SIM_K_N] = {0};

    ~Engine() override
    {
        (void)hipStreamSynchronize(M.stream);
        for (auto &g : gexec)
            if (g) (void)hipGraphExecDestroy(g);
        for (void *p : allocs) (void)hipFree(p);
        if (own_stream) (void)hipStreamDestroy(own_stream);
        for (auto &e : ev_pool) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
        for (auto &e : ev_used) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    }

    template <class U> int alloc(U *&p, uint64_t count)
    {
        void *q = nullptr;
        if (count == 0) count = 1;
        if (hipMalloc(&q, count * sizeof(U)) != hipSuccess) return fail(SIM_ENOMEM, "device allocation failed");
        allocs.push_back(q);
        p = (U *)q;
        return SIM_OK;
    }

    // Physics, cut-off and cell grid of one system (or one replica of a
    // batch) with n_r slots and species sp.
    int setup_replica(const Model &M, uint64_t n, const int32_t *sp, Params &P, double &cell_edge, double &pair_tests, bool &narrow)
    {
        phys_params(M, P);
        double Lmin = 1e300;
        for (int k = 0; k < DIM; ++k) Lmin = std::min(Lmin, M.box[k]);
        if (!(P.rcut < 0.5 * Lmin)) return fail(SIM_EINVAL, "r_cut must be below half the smallest box edge");
        const double smax = std::max(P.sd[0], std::max(P.sd[1], P.sd[2]));
        if (!(8.0 * smax < 0.5 * Lmin)) return fail(SIM_EINVAL, "displacement per step too large for the box");
        // counts
        uint64_t nA = 0, nB = 0, nC = 0;
        for (uint64_t i = 0; i < n; ++i) {
            nA += sp[i] == SIM_SP_A;
            nB += sp[i] == SIM_SP_B;
            nC += sp[i] == SIM_SP_C;
        }
        // grid: cells of edge >= r_cut, about one B per cell unless requested
        double vol = 1.0;
        for (int k = 0; k < DIM; ++k) vol *= M.box[k];
        double c = M.cell_req > 0.0 ? M.cell_req : std::pow(vol / (double)std::max<uint64_t>(nB + nC, 1), 1.0 / DIM);
        c = std::max(c, P.rcut);
        uint64_t ncell = 1;
        cell_edge = 1e300;
        for (int k = 0; k < 3; ++k) {
            int m_ = 1;
            if (k < DIM) {
                const double f = std::floor(M.box[k] / c);
                m_ = f > 2048.0 ? 2048 : (int)f;
                if (m_ < 3) m_ = 1;
                cell_edge = std::min(cell_edge, M.box[k] / m_);
            }
            P.nc[k] = m_;
            P.L[k] = k < DIM ? M.box[k] : 1.0;
            P.Lh[k] = 0.5 * P.L[k];
            P.Lf[k] = (float)P.L[k];
            P.Lhf[k] = (float)P.Lh[k];
            P.cs[k] = m_ / P.L[k];
            P.ce[k] = P.L[k] / m_;
            ncell *= (uint64_t)m_;
        }
        if (ncell > (1ull << 28)) return fail(SIM_EUNSUPPORTED, "too many cells");
        P.n_cells = (u32)ncell;
        P.n_keys = 3u * P.n_cells;
        // Pair search: LDS bricks pay off where every A tests many B's (each
        // staged B serves many A's); with few B's per A the direct kernel
        // (neighbour buckets through L2) has no staging to amortise.
        {
            const double bpc0 = (double)std::max<uint64_t>(nB + nC, 1) / (double)ncell;
            double tests = bpc0;
            for (int k = 0; k < DIM; ++k) tests *= P.nc[k] >= 3 ? std::min(3.0, 1.0 + 2.0 * P.reach / P.ce[k]) : 1.0;
            pair_tests = tests;
        }
        // an A needs at most one neighbour cell per axis when every axis with
        // three or more cells is at least twice the reach wide
        narrow = true;
        for (int k = 0; k < DIM; ++k)
            if (P.nc[k] >= 3 && !(P.ce[k] >= 2.0 * P.reach)) narrow = false;
        P.debug = M.debug;
        P.dbg_cap = (u32)M.dbg_cap;
        return SIM_OK;
    }

    // pair list: four entries per slot, at least 2^20, at most 2^30, in whole segments
    void set_pair_cap(Params &Q) const
    {
        Q.cap_pl = (u32)std::min<uint64_t>(std::max<uint64_t>(1u << 20, 4 * n), 1u << 30) & ~(PL_SEGS - 1);
        Q.seg_cap = Q.cap_pl / PL_SEGS;
    }

    int open_stream()
    {
        if (!M.stream) {  // a stream of our own: the null stream cannot be captured into a graph
            HIPCHECK(hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking));
            M.stream = own_stream;
        }
        return SIM_OK;
    }

    int init(const Model &m, uint64_t nslots, const int32_t *sp, const double *pos, const uint32_t *pt)
    {
        M = m;
        n = nslots;
        int rc;
        if ((rc = open_stream()) || (rc = setup_replica(M, n, sp, P, cell_edge, pair_tests, narrow))) return rc;
        P.cap = (u32)n;
        set_pair_cap(P);
        uint64_t nB = 0, nC = 0;
        for (uint64_t i = 0; i < n; ++i) {
            nB += sp[i] == SIM_SP_B;
            nC += sp[i] == SIM_SP_C;
        }
        const uint64_t ncell = P.n_cells;
        const bool can_tile = P.nc[0] >= 3 && P.nc[1] >= 3 && (DIM == 2 || P.nc[2] >= 3);
        P.tiled = can_tile && (M.pair_search == SIM_PAIRS_BRICKS ||
                               (M.pair_search == SIM_PAIRS_AUTO && pair_tests > PAIR_TESTS_TILED));
        // LDS bricks: about 256 cells (halo <= MAX_HALO), fewer when buckets are crowded
        if (P.tiled) {
            const double bpc = (double)std::max<uint64_t>(nB + nC, 1) / (double)ncell;
            const double lcap = 1024.0;
            int bb[3] = {std::min(DIM == 3 ? 8 : 16, P.nc[0] - 2), std::min(DIM == 3 ? 8 : 16, P.nc[1] - 2),
                         DIM == 3 ? std::min(4, P.nc[2] - 2) : 1};
            auto halo = [&] { return (bb[0] + 2.0) * (bb[1] + 2.0) * (DIM == 3 ? bb[2] + 2.0 : 1.0); };
            while (halo() * bpc > 0.6 * lcap && (bb[0] > 1 || bb[1] > 1 || bb[2] > 1)) {
                int k = 0;
                for (int d = 1; d < DIM; ++d)
                    if (bb[d] > bb[k]) k = d;
                bb[k] = (bb[k] + 1) / 2;
            }
            if (halo() > MAX_HALO || bb[1] * bb[2] > MAX_ROWS) return fail(SIM_EUNSUPPORTED, "pair-search brick too large");
            P.bx = bb[0];
            P.by = bb[1];
            P.bz = bb[2];
            P.nbx = (P.nc[0] + P.bx - 1) / P.bx;
            P.nby = (P.nc[1] + P.by - 1) / P.by;
            P.nbz = DIM == 3 ? (P.nc[2] + P.bz - 1) / P.bz : 1;
            n_bricks = P.nbx * P.nby * P.nbz;
        }
        if (DIM == 2 && M.green2d == SIM_G2_EXACT && (rc = x2_tables(P))) return rc;
        return finish_init(sp, pos, pt);
    }

    // 16-point Gauss-Legendre rule on [-1, 1]: the roots of P_16 by Newton's
    // method from Tricomi's estimate, weights 2 / ((1 - x^2) P_16'(x)^2).
    static void gauss_legendre16(double *x, double *w)
    {
        const int n = 16;
        for (int i = 0; i < n; ++i) {
            const double th = M_PI * (4.0 * i + 3.0) / (4.0 * n + 2.0);
            double t = (1.0 - (n - 1.0) / (8.0 * n * n * n)) * std::cos(th), d = 1.0;
            for (int it = 0; it < 60; ++it) {
                double pm = 1.0, p = t;  // P_0, P_1
                for (int k = 2; k <= n; ++k) {
                    const double pn = ((2 * k - 1) * t * p - (k - 1) * pm) / k;
                    pm = p;
                    p = pn;
                }
                d = n * (pm - t * p) / (1.0 - t * t);
                const double step = p / d;
                t -= step;
                if (std::fabs(step) < 1e-17) break;
            }
            x[i] = t;
            w[i] = 2.0 / ((1.0 - t * t) * d * d);
        }
    }

    // Tables of the exact 2D radial functions (green2x.hpp): R steps of
    // h = sqrt(tau)/160 and R0 steps of 2h, R0 up to the switch 1 + c
    // sqrt(tau) (x2_switch_c; plus the interpolation stencil), R up to the larger of
    // r_cut/a and the switch plus L = 12 sqrt(tau) + 1, the top of the
    // propagator's distribution function.  Quadrature nodes: 16-point
    // Gauss-Legendre panels, geometric (ratio 2) from 2^-30/4 to 1/4 where the
    // absorbing and radiation kernels vary like 1/ln x, then of width at most
    // min(1/4, pi / (R_top + R0_top + 1)) up to x = sqrt(50/tau).
    // The tables of a system (or of a replica or member, into its own parameters Q): from the
    // handle's sets when one was built for the same h~ and cut-off, else built.
    int x2_tables(Params &Q)
    {
        exact2d = true;
        for (const X2Set &x : x2_sets)
            if (x.hh == Q.hh && x.rcut == Q.rcut) {
                copy_x2(x.tab, Q);
                return SIM_OK;
            }
        int rc;
        if ((rc = build_x2(Q))) return rc;
        x2_sets.push_back({Q.hh, Q.rcut, Q});
        return SIM_OK;
    }

    static void copy_x2(const Params &src, Params &Q)
    {
        Q.x2_enc = src.x2_enc;
        Q.x2_reac = src.x2_reac;
        Q.x2_cdf = src.x2_cdf;
        Q.x2_h = src.x2_h;
        Q.x2_inv_h = src.x2_inv_h;
        Q.x2_inv_h0 = src.x2_inv_h0;
        Q.x2_r0sw = src.x2_r0sw;
        Q.x2_r0sw_prop = src.x2_r0sw_prop;
        Q.x2_n0_prop = src.x2_n0_prop;
        Q.x2_nr = src.x2_nr;
        Q.x2_n0 = src.x2_n0;
        Q.x2_ntr = src.x2_ntr;
    }

    int build_x2(Params &Q)
    {
        const double tau = Q.tau, st = Q.sqrt_tau, h = st / 160.0, h0 = X2S * h;
        if (!(tau * (1.0 - 1e-9) <= X2_TAU_MAX)) return fail(SIM_EUNSUPPORTED, "exact 2D functions need tau = D_eff dt / a^2 <= 0.8");
        const double r0sw = 1.0 + x2_switch_c(tau) * st, L = 12.0 * st + 1.0;
        const u32 n0 = (u32)std::ceil((r0sw - 1.0) / h0) + 4;
        const double r0top = 1.0 + (n0 - 1) * h0;
        const double rtop = std::max(Q.rcut / Q.a, r0top + L) + 4.0 * h;
        const u32 nr = (u32)std::ceil((rtop - 1.0) / h) + 1;
        const u32 top = (u32)std::ceil(L / h);
        if ((uint64_t)nr * n0 > (1ull << 26) || nr > 65535u * X2T)
            return fail(SIM_EUNSUPPORTED, "exact 2D tables would exceed 2^26 entries");
        double gx[16], gw[16];
        gauss_legendre16(gx, gw);
        std::vector<double> xs, s1, s2;
        const double xmax = std::sqrt(50.0 / tau), x1 = std::min(0.25, xmax);
        const double wmax = std::min(0.25, M_PI / (rtop + r0top + 1.0));
        const int ngeo = 30, nuni = (int)std::ceil((xmax - x1) / wmax);
        for (int p = 0; p < ngeo + nuni; ++p) {
            const double lo = p < ngeo ? std::ldexp(x1, p - ngeo) : x1 + (p - ngeo) * ((xmax - x1) / nuni);
            const double hi = p < ngeo ? 2.0 * lo : lo + (xmax - x1) / nuni;
            for (int q = 0; q < 16; ++q) {
                const double x = 0.5 * (lo + hi) + 0.5 * (hi - lo) * gx[q];
                const double wk = 0.5 * (hi - lo) * gw[q] * std::exp(-tau * x * x);
                xs.push_back(x);
                s1.push_back(wk * x / (2.0 * M_PI));  // G: x w / 2 pi
                s2.push_back(wk);                     // M: w
            }
        }
        const u32 K = (u32)xs.size();
        const size_t NK = (size_t)nr * K, NT = (size_t)nr * n0;
        if (NK > (1ull << 31)) return fail(SIM_EUNSUPPORTED, "exact 2D quadrature matrices too large");
        // scratch (freed below) and the tables (kept)
        double *tmp_buf = nullptr;
        const size_t n_tmp = 3 * (size_t)K + 8 * (size_t)K + 5 * NK + 5 * NT;
        if (hipMalloc(&tmp_buf, sizeof(double) * n_tmp) != hipSuccess) return fail(SIM_ENOMEM, "device allocation failed (exact 2D scratch)");
        double *d_x = tmp_buf, *d_s1 = d_x + K, *d_s2 = d_s1 + K, *d_nd = d_s2 + K;
        double *Cabs = d_nd + 8 * (size_t)K, *Cref = Cabs + NK, *Crad = Cref + NK, *Kabs = Crad + NK, *Kref = Kabs + NK;
        double *Gabs = Kref + NK, *Gref = Gabs + NT, *Grad = Gref + NT, *Mabs = Grad + NT, *Mref = Mabs + NT;
        // p_enc and p_reac in binary32 tiles of X2TR rows by X2TC columns (the padding is never read)
        const u32 ntr = (nr + X2TR - 1) / X2TR, ntc = (n0 + X2TC - 1) / X2TC;
        const size_t NB = (size_t)ntr * ntc * X2TR * X2TC;
        float *enc = nullptr, *reac = nullptr;
        double *cdf = nullptr;
        int rc;
        if ((rc = alloc(enc, NB)) || (rc = alloc(reac, NB)) || (rc = alloc(cdf, NT))) {
            (void)hipFree(tmp_buf);
            return rc;
        }
        hipStream_t sm = M.stream;
        auto run = [&]() -> hipError_t {
            hipError_t e;
            if ((e = hipMemsetAsync(enc, 0, sizeof(float) * NB, sm)) != hipSuccess) return e;
            if ((e = hipMemsetAsync(reac, 0, sizeof(float) * NB, sm)) != hipSuccess) return e;
            if ((e = hipMemcpyAsync(d_x, xs.data(), sizeof(double) * K, hipMemcpyHostToDevice, sm)) != hipSuccess) return e;
            if ((e = hipMemcpyAsync(d_s1, s1.data(), sizeof(double) * K, hipMemcpyHostToDevice, sm)) != hipSuccess) return e;
            if ((e = hipMemcpyAsync(d_s2, s2.data(), sizeof(double) * K, hipMemcpyHostToDevice, sm)) != hipSuccess) return e;
            k_x2_nodes<<<(K + 255) / 256, 256, 0, sm>>>(d_x, K, Q.hh, d_nd);
            k_x2_rows<<<(u32)((NK + 255) / 256), 256, 0, sm>>>(d_x, d_nd, K, nr, h, Cabs, Cref, Crad, Kabs, Kref);
            const dim3 g((n0 + X2T - 1) / X2T, (nr + X2T - 1) / X2T);
            k_x2_gemm<<<g, 256, 0, sm>>>(Cabs, Cabs, d_s1, nr, n0, K, Gabs);
            k_x2_gemm<<<g, 256, 0, sm>>>(Cref, Cref, d_s1, nr, n0, K, Gref);
            k_x2_gemm<<<g, 256, 0, sm>>>(Crad, Crad, d_s1, nr, n0, K, Grad);
            k_x2_gemm<<<g, 256, 0, sm>>>(Kabs, Cabs, d_s2, nr, n0, K, Mabs);
            k_x2_gemm<<<g, 256, 0, sm>>>(Kref, Cref, d_s2, nr, n0, K, Mref);
            k_x2_tables<<<(u32)((NT + 255) / 256), 256, 0, sm>>>(Gabs, Gref, Grad, Mabs, Mref, nr, n0, h, tau, top, ntr, enc, reac, cdf);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            return hipStreamSynchronize(sm);  // the host vectors are read by the copies
        };
        const hipError_t e = run();
        (void)hipFree(tmp_buf);
        if (e != hipSuccess) return fail(SIM_EDEVICE, std::string("exact 2D tables: ") + hipGetErrorString(e));
        Q.x2_enc = enc;
        Q.x2_reac = reac;
        Q.x2_cdf = cdf;
        Q.x2_h = h;
        Q.x2_inv_h = 1.0 / h;
        Q.x2_inv_h0 = 1.0 / h0;
        Q.x2_r0sw = r0sw;
        Q.x2_r0sw_prop = 1.0 + 8.4 * st;  // the propagator's mass is resolved to about erfc(4.2)
        Q.x2_n0_prop = std::min<u32>(n0, (u32)std::ceil(8.4 * st / h0) + 4);
        Q.x2_nr = nr;
        Q.x2_n0 = n0;
        Q.x2_ntr = ntr;
        x2_build = {(double)K, (double)nr, (double)n0};
        return SIM_OK;
    }

    // A batch of independent replicas (3D): each keeps its own box, kappa,
    // replica key, cut-off and grid; their slots and cells are laid out one
    // after the other.  The pair search is the direct one.
    int init_batch(const std::vector<Model> &ms, const std::vector<uint64_t> &nr, const std::vector<u32> &step0, const int32_t *sp,
                   const double *pos, const uint32_t *pt)
    {
        M = ms[0];
        n = 0;
        for (uint64_t x : nr) n += x;
        int rc;
        if ((rc = open_stream())) return rc;
        batch = true;
        const size_t R = ms.size();
        reps_h.resize(R);
        rep_box.resize(3 * R);
        rep_of_slot_h.resize(n);
        uint64_t sbase = 0, cbase = 0;
        narrow = true;
        for (size_t r = 0; r < R; ++r) {
            double ce = 0.0, tests = 0.0;
            bool nar = true;
            if ((rc = setup_replica(ms[r], nr[r], sp + sbase, reps_h[r], ce, tests, nar))) return rc;
            if (DIM == 2 && M.green2d == SIM_G2_EXACT && (rc = x2_tables(reps_h[r]))) return rc;
            reps_h[r].slot_base = (u32)sbase;
            reps_h[r].cell_base = (u32)cbase;
            reps_h[r].step_base = 0u - step0[r];  // own step = counter (0 at creation) - base
            for (int k = 0; k < 3; ++k) rep_box[3 * r + k] = ms[r].box[k];
            for (uint64_t i = 0; i < nr[r]; ++i) rep_of_slot_h[sbase + i] = (u32)r;
            narrow = narrow && nar;
            if (r == 0) {
                cell_edge = ce;
                pair_tests = tests;
            }
            sbase += nr[r];
            cbase += reps_h[r].n_cells;
            if (cbase > (1ull << 28)) return fail(SIM_EUNSUPPORTED, "too many cells in the batch");
        }
        P = reps_h[0];  // replica 0's physics; totals below
        P.n_cells = (u32)cbase;
        P.n_keys = 3u * P.n_cells;
        P.slot_base = P.cell_base = P.step_base = 0;
        P.n_rep = (u32)R;
        P.cap = (u32)n;
        set_pair_cap(P);
        P.tiled = 0;
        if ((rc = alloc(d_reps, R)) || (rc = alloc(d_rep_of_slot, n)) || (rc = alloc(d_cell_rep, cbase))) return rc;
        P.reps = d_reps;
        P.rep_of_slot = d_rep_of_slot;
        P.cell_rep = d_cell_rep;
        std::vector<u32> cell_rep_h(cbase);
        for (size_t r = 0; r < R; ++r)
            for (u32 c = 0; c < reps_h[r].n_cells; ++c) cell_rep_h[reps_h[r].cell_base + c] = (u32)r;
        for (auto &q : reps_h) {  // fields shared by the whole batch
            q.cap = P.cap;
            q.cap_pl = P.cap_pl;
            q.seg_cap = P.seg_cap;
            q.n_rep = P.n_rep;
            q.reps = d_reps;
            q.rep_of_slot = d_rep_of_slot;
            q.cell_rep = d_cell_rep;
        }
        HIPCHECK(hipMemcpyAsync(d_rep_of_slot, rep_of_slot_h.data(), sizeof(u32) * n, hipMemcpyHostToDevice, M.stream));
        HIPCHECK(hipMemcpyAsync(d_cell_rep, cell_rep_h.data(), sizeof(u32) * cbase, hipMemcpyHostToDevice, M.stream));
        HIPCHECK(hipStreamSynchronize(M.stream));  // cell_rep_h is host memory the copy reads
        return finish_init(sp, pos, pt);
    }

    // A pool: an empty batch with room for slot_cap slots, cell_cap cells and
    // rep_cap members.  The configuration's box stands in for the members'
    // boxes in the shared fields; members bring their own.
    int init_pool(const Model &m, uint64_t slot_cap, uint64_t cell_cap, uint32_t rep_cap)
    {
        M = m;
        n = slot_cap;
        int rc;
        if ((rc = open_stream())) return rc;
        batch = pool = true;
        exact2d = DIM == 2 && M.green2d == SIM_G2_EXACT;  // tables come with each member
        if ((rc = setup_replica(M, 0, nullptr, P, cell_edge, pair_tests, narrow))) return rc;
        narrow = true;  // until a member needs the general pair search
        reps_h.assign(rep_cap, P);
        member_n.assign(rep_cap, 0);
        rep_box.assign(3 * (size_t)rep_cap, 1.0);
        slot_free.reset(slot_cap);
        cell_free.reset(cell_cap);
        P.n_cells = (u32)cell_cap;
        P.n_keys = 3u * P.n_cells;
        P.slot_base = P.cell_base = P.step_base = 0;
        P.n_rep = rep_cap;
        P.cap = (u32)n;
        set_pair_cap(P);
        P.tiled = 0;
        if ((rc = alloc(d_reps, rep_cap)) || (rc = alloc(d_rep_of_slot, n)) || (rc = alloc(d_cell_rep, cell_cap))) return rc;
        P.reps = d_reps;
        P.rep_of_slot = d_rep_of_slot;
        P.cell_rep = d_cell_rep;
        for (auto &q : reps_h) {
            q.cap = P.cap;
            q.cap_pl = P.cap_pl;
            q.seg_cap = P.seg_cap;
            q.n_rep = P.n_rep;
            q.reps = d_reps;
            q.rep_of_slot = d_rep_of_slot;
            q.cell_rep = d_cell_rep;
        }
        return finish_init(nullptr, nullptr, nullptr);
    }

    // Buffers, constants and the initial state (P final apart from g2c).
    int finish_init(const int32_t *sp, const double *pos, const uint32_t *pt)
    {
        // A and C counts change with reactions and state loads; size by the slot count
        maxA = (u32)n;
        maxC = (u32)n;
        nb_scan = (P.n_keys + SCAN_TILE - 1) / SCAN_TILE;
        P.cnt_region = nb_scan * (SCAN_TILE / CNT_REGIONS);
        // device buffers
        int rc;
        if ((rc = alloc(rec[0], n)) || (rc = alloc(rec[1], n)) || (rc = alloc(tmp, n)) ||
            (rc = alloc(rank, n)) || (rc = alloc(cnt, (uint64_t)nb_scan * SCAN_TILE)) ||
            (rc = alloc(scnt, (uint64_t)nb_scan * SCAN_TILE)) || (rc = alloc(okey, n)) ||
            (rc = alloc(start, (uint64_t)nb_scan * SCAN_TILE + 1)) || (rc = alloc(bsum, nb_scan)) || (rc = alloc(partner, n)) ||
            (rc = alloc(plist, P.cap_pl)) || (rc = alloc(cand, P.cap_pl)) || (rc = alloc(flag, P.cap_pl)) ||
            (rc = alloc(nextA, P.cap_pl)) || (rc = alloc(nextB, P.cap_pl)) || (rc = alloc(headA, n)) ||
            (rc = alloc(headB, n)) || (rc = alloc(ev, n)) || (rc = alloc(ctr, 1)) || (rc = alloc(g2c, 4 * (MAXTERMS + 1))) ||
            (rc = alloc(g_pos, n * DIM)) || (rc = alloc(g_sp, n)) || (batch && (rc = alloc(nkey, n))) ||
            (P.angles && (rc = alloc(ang, n))))
            return rc;
        angles = P.angles != 0;
        gauss_legendre16(gl16.x, gl16.w);
        if (M.debug) {
            if ((rc = alloc(dbg_moved, n * DIM)) || (rc = alloc(dbg_disp, n * DIM)) || (rc = alloc(dbg_cells, n)) || (rc = alloc(dbg_pairs, M.dbg_cap)) ||
                (rc = alloc(dbg_picks, M.dbg_cap)) || (rc = alloc(dbg_matches, M.dbg_cap)) || (rc = alloc(dbg_diss, M.dbg_cap)))
                return rc;
        }
        HIPCHECK(hipMemsetAsync(cnt, 0, sizeof(u32) * nb_scan * SCAN_TILE, M.stream));  // padding stays zero
        HIPCHECK(hipMemsetAsync(scnt, 0, sizeof(u32) * nb_scan * SCAN_TILE, M.stream));
        double g2h[4 * (MAXTERMS + 1)];
        h_g2_constants(P.hh, g2h);
        HIPCHECK(hipMemcpyAsync(g2c, g2h, sizeof(g2h), hipMemcpyHostToDevice, M.stream));
        P.g2c = g2c;
        if ((rc = alloc(dparams, 1))) return rc;
        HIPCHECK(hipMemcpyAsync(dparams, &P, sizeof(P), hipMemcpyHostToDevice, M.stream));  // P is final here
        if (batch) {
            // each replica's 2D expansion constants (Q_rad depends on its h)
            const size_t G = 4 * (MAXTERMS + 1), R = reps_h.size();
            std::vector<double> g2all(G * R);
            if ((rc = alloc(d_g2c_reps, G * R))) return rc;
            for (size_t r = 0; r < R; ++r) {
                h_g2_constants(reps_h[r].hh, &g2all[G * r]);
                reps_h[r].g2c = d_g2c_reps + G * r;
            }
            HIPCHECK(hipMemcpyAsync(d_g2c_reps, g2all.data(), sizeof(double) * G * R, hipMemcpyHostToDevice, M.stream));
            HIPCHECK(hipMemcpyAsync(d_reps, reps_h.data(), sizeof(Params) * R, hipMemcpyHostToDevice, M.stream));
            HIPCHECK(hipStreamSynchronize(M.stream));  // g2all and reps_h are host memory the copies read
        }
        if (pool) return start_counters(0, 0);
        return load(0, sp, pos, pt);
    }

    // Counters of a freshly loaded state with `live` records at step step0.
    int start_counters(uint64_t live, uint64_t step0)
    {
        Counters c;
        std::memset(&c, 0, sizeof(c));
        c.n_rec = (u32)live;
        c.n_live = (u32)live;
        c.step = (u32)step0;
        c.cell_hw = pool ? cell_hw : P.n_cells;  // a pool: the cells its members have taken so far
        HIPCHECK(hipMemcpyAsync(ctr, &c, sizeof(c), hipMemcpyHostToDevice, M.stream));
        HIPCHECK(hipMemsetAsync(headA, 0, sizeof(u64) * n, M.stream));  // no chain survives a reload
        HIPCHECK(hipMemsetAsync(headB, 0, sizeof(u64) * n, M.stream));
        HIPCHECK(hipStreamSynchronize(M.stream));
        cur = 0;
        stepno = step0;
        return SIM_OK;
    }

    int load(uint64_t step0, const int32_t *sp, const double *pos, const uint32_t *pt) override
    {
        if (pool) return fail(SIM_ESTATE, "a pool's members are loaded by sim_pool_admit");
        std::vector<Rec<T>> h(n);
        std::vector<u32> hp(n, NOSLOT);
        uint64_t live = 0;
        for (uint64_t i = 0; i < n; ++i) {
            if (sp[i] > SIM_SP_C) continue;
            Rec<T> r;
            const double *bx = batch ? &rep_box[3 * rep_of_slot_h[i]] : M.box;
            r.x = h_wrap_store<T>(pos[i * DIM + 0], bx[0]);
            r.y = h_wrap_store<T>(pos[i * DIM + 1], bx[1]);
            r.z = DIM == 3 ? h_wrap_store<T>(pos[i * DIM + 2], bx[2]) : (T)0;
            rec_set_meta(r, meta_make((u32)sp[i], (u32)i));
            h[live++] = r;
            if (sp[i] == SIM_SP_C && pt) hp[i] = pt[i];
        }
        HIPCHECK(hipMemcpyAsync(rec[0], h.data(), sizeof(Rec<T>) * live, hipMemcpyHostToDevice, M.stream));
        HIPCHECK(hipMemcpyAsync(partner, hp.data(), sizeof(u32) * n, hipMemcpyHostToDevice, M.stream));
        return start_counters(live, step0);
    }

    // ---- pools ------------------------------------------------------------
    int admit(const sim_replica &rp, uint32_t *member) override
    {
        if (!pool) return fail(SIM_ESTATE, "not a pool");
        int rc;
        if ((rc = validate_box(DIM, M.prec, rp.box)) || (rc = validate_state(DIM, M.k_off > 0.0, rp.n, rp.species, rp.pos, rp.partner)))
            return fail(rc, g_err);
        if (!finite_nonneg(rp.kappa)) return fail(SIM_EINVAL, "kappa must be >= 0");
        uint32_t idx = 0;
        while (idx < member_n.size() && member_n[idx]) ++idx;
        if (idx == member_n.size()) return fail(SIM_ECAPACITY, "every member entry is taken");
        Model mr = M;
        for (int k = 0; k < 3; ++k) mr.box[k] = k < DIM ? rp.box[k] : 1.0;
        mr.kappa = rp.kappa;
        mr.replica = rp.replica;
        Params Q;
        double ce = 0.0, tests = 0.0;
        bool nar = true;
        if ((rc = setup_replica(mr, rp.n, rp.species, Q, ce, tests, nar))) return rc;
        if (DIM == 2 && M.green2d == SIM_G2_EXACT && (rc = x2_tables(Q))) return rc;  // before any slot is taken
        uint64_t s0 = 0, c0 = 0;
        if (!slot_free.take(rp.n, s0)) return fail(SIM_ECAPACITY, "no free range of slots");
        if (!cell_free.take(Q.n_cells, c0)) {
            slot_free.give(s0, rp.n);
            return fail(SIM_ECAPACITY, "no free range of cells");
        }
        rc = place(idx, rp, mr, Q, s0, c0);
        if (rc) {
            slot_free.give(s0, rp.n);
            cell_free.give(c0, Q.n_cells);
            return rc;
        }
        if (narrow && !nar) {  // the graphs were built for the narrow pair search
            narrow = false;
            for (auto &g : gexec)
                if (g) {
                    (void)hipGraphExecDestroy(g);
                    g = nullptr;
                }
        }
        *member = idx;
        return SIM_OK;
    }

    // Writes member idx's parameters, slot ownership, partners and records.
    int place(uint32_t idx, const sim_replica &rp, const Model &mr, Params &Q, uint64_t s0, uint64_t c0)
    {
        const uint64_t m = rp.n;
        Q.slot_base = (u32)s0;
        Q.cell_base = (u32)c0;
        Q.step_base = (u32)stepno - rp.step;  // the member's own step = pool step - base
        Q.cap = P.cap;
        Q.cap_pl = P.cap_pl;
        Q.seg_cap = P.seg_cap;
        Q.n_rep = P.n_rep;
        Q.reps = d_reps;
        Q.rep_of_slot = d_rep_of_slot;
        Q.cell_rep = d_cell_rep;
        const size_t G = 4 * (MAXTERMS + 1);
        Q.g2c = d_g2c_reps + G * idx;
        std::vector<double> g2h(G);
        h_g2_constants(Q.hh, g2h.data());
        std::vector<Rec<T>> h;
        h.reserve(m);
        std::vector<u32> hp(m, NOSLOT), ho(m, idx);
        for (uint64_t i = 0; i < m; ++i) {
            const int sp = rp.species[i];
            if (sp > SIM_SP_C) continue;
            Rec<T> r;
            r.x = h_wrap_store<T>(rp.pos[i * DIM + 0], mr.box[0]);
            r.y = h_wrap_store<T>(rp.pos[i * DIM + 1], mr.box[1]);
            r.z = DIM == 3 ? h_wrap_store<T>(rp.pos[i * DIM + 2], mr.box[2]) : (T)0;
            rec_set_meta(r, meta_make((u32)sp, (u32)(s0 + i)));
            h.push_back(r);
            if (sp == SIM_SP_C && rp.partner && rp.partner[i] < m) hp[i] = (u32)(s0 + rp.partner[i]);
        }
        // the records go after the current ones; records of members that left
        // stay (dead) until the next binning, so make room if they crowd the buffer
        u32 n_rec = 0;
        HIPCHECK(hipMemcpyAsync(&n_rec, &ctr->n_rec, sizeof(u32), hipMemcpyDeviceToHost, M.stream));
        HIPCHECK(hipStreamSynchronize(M.stream));
        if ((uint64_t)n_rec + h.size() > n) {
            int rc;
            if ((rc = compact())) return rc;
            HIPCHECK(hipMemcpyAsync(&n_rec, &ctr->n_rec, sizeof(u32), hipMemcpyDeviceToHost, M.stream));
            HIPCHECK(hipStreamSynchronize(M.stream));
            if ((uint64_t)n_rec + h.size() > n) return fail(SIM_ECAPACITY, "record buffer full");
        }
        const u32 n_new = n_rec + (u32)h.size();
        HIPCHECK(hipMemcpyAsync(d_g2c_reps + G * idx, g2h.data(), sizeof(double) * G, hipMemcpyHostToDevice, M.stream));
        HIPCHECK(hipMemcpyAsync(d_reps + idx, &Q, sizeof(Params), hipMemcpyHostToDevice, M.stream));
        HIPCHECK(hipMemcpyAsync(d_rep_of_slot + s0, ho.data(), sizeof(u32) * m, hipMemcpyHostToDevice, M.stream));
        std::vector<u32> hc(Q.n_cells, idx);
        HIPCHECK(hipMemcpyAsync(d_cell_rep + c0, hc.data(), sizeof(u32) * Q.n_cells, hipMemcpyHostToDevice, M.stream));
        HIPCHECK(hipMemcpyAsync(partner + s0, hp.data(), sizeof(u32) * m, hipMemcpyHostToDevice, M.stream));
        if (!h.empty()) HIPCHECK(hipMemcpyAsync(rec[cur] + n_rec, h.data(), sizeof(Rec<T>) * h.size(), hipMemcpyHostToDevice, M.stream));
        HIPCHECK(hipMemcpyAsync(&ctr->n_rec, &n_new, sizeof(u32), hipMemcpyHostToDevice, M.stream));
        cell_hw = std::max<u32>(cell_hw, (u32)(c0 + Q.n_cells));  // never lowered: cells of members that left may still hold dead records
        HIPCHECK(hipMemcpyAsync(&ctr->cell_hw, &cell_hw, sizeof(u32), hipMemcpyHostToDevice, M.stream));
        HIPCHECK(hipStreamSynchronize(M.stream));  // the host buffers above are read by the copies
        reps_h[idx] = Q;
        member_n[idx] = m;
        for (int k = 0; k < 3; ++k) rep_box[3 * idx + k] = mr.box[k];
        return SIM_OK;
    }

    // Drops the dead records: the live ones move to the other buffer.
    int compact()
    {
        k_compact<T><<<grid_for(n, 8192), BLOCK, 0, M.stream>>>(rec[cur], rec[cur ^ 1], ctr);
        k_compact_done<<<1, 64, 0, M.stream>>>(ctr);
        HIPCHECK(hipGetLastError());
        cur ^= 1;
        return SIM_OK;
    }

    int retire(uint32_t idx) override
    {
        if (!pool) return fail(SIM_ESTATE, "not a pool");
        if (idx >= member_n.size() || !member_n[idx]) return fail(SIM_EINVAL, "no such member");
        const Params &Q = reps_h[idx];
        const uint64_t m = member_n[idx];
        k_retire<T><<<grid_for(n, 8192), BLOCK, 0, M.stream>>>(rec[cur], ctr, Q.slot_base, (u32)(Q.slot_base + m));
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(M.stream));
        slot_free.give(Q.slot_base, m);
        cell_free.give(Q.cell_base, Q.n_cells);
        member_n[idx] = 0;
        return SIM_OK;
    }

    // A member's positions, species, partners (member-local) or counts.
    int read_member(uint32_t idx, int what, void *dst, uint64_t cap, uint64_t *written) override
    {
        if (!pool) return fail(SIM_ESTATE, "not a pool");
        if (idx >= member_n.size() || !member_n[idx]) return fail(SIM_EINVAL, "no such member");
        if (what != SIM_READ_POS && what != SIM_READ_SPECIES && what != SIM_READ_PARTNER && what != SIM_READ_COUNTS)
            return fail(SIM_EINVAL, "a member reads positions, species, partners or counts");
        hipStream_t st = M.stream;
        const uint64_t s0 = reps_h[idx].slot_base, m = member_n[idx];
        k_fill<<<grid_for(m * DIM, 2048), BLOCK, 0, st>>>(g_pos + s0 * DIM, m * DIM, g_sp + s0, (u32)m);
        k_gather<DIM, T><<<grid_for(n, 8192), BLOCK, 0, st>>>(rec[cur], partner, ctr, 0, g_pos, g_sp, (u32)n);
        HIPCHECK(hipGetLastError());
        if (what == SIM_READ_POS) return copy_out(g_pos + s0 * DIM, sizeof(double) * m * DIM, dst, cap, written);
        if (what == SIM_READ_SPECIES) return copy_out(g_sp + s0, sizeof(int) * m, dst, cap, written);
        std::vector<int> hs(m);
        std::vector<u32> hp(m);
        HIPCHECK(hipMemcpyAsync(hs.data(), g_sp + s0, sizeof(int) * m, hipMemcpyDeviceToHost, st));
        HIPCHECK(hipMemcpyAsync(hp.data(), partner + s0, sizeof(u32) * m, hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        if (what == SIM_READ_COUNTS) {
            int64_t cnts[5] = {0, 0, 0, 0, 0};
            for (int v : hs) cnts[v] += 1;
            if (cap < sizeof(cnts)) return fail(SIM_EINVAL, "destination buffer too small");
            std::memcpy(dst, cnts, sizeof(cnts));
            if (written) *written = sizeof(cnts);
            return SIM_OK;
        }
        for (uint64_t i = 0; i < m; ++i) hp[i] = hs[i] == SIM_SP_C ? (u32)(hp[i] - s0) : NOSLOT;
        if (cap < sizeof(u32) * m) return fail(SIM_EINVAL, "destination buffer too small");
        std::memcpy(dst, hp.data(), sizeof(u32) * m);
        if (written) *written = sizeof(u32) * m;
        return SIM_OK;
    }

    template <class F> void launch(int k, F &&f)
    {
        if (!M.timing) {
            f();
            return;
        }
        EvPair e;
        if (ev_pool.empty()) {
            (void)hipEventCreate(&e.a);
            (void)hipEventCreate(&e.b);
        } else {
            e = ev_pool.back();
            ev_pool.pop_back();
        }
        e.k = k;
        (void)hipEventRecord(e.a, M.stream);
        f();
        (void)hipEventRecord(e.b, M.stream);
        ev_used.push_back(e);
    }

    static u32 round8(u32 g) { return (g + 7u) & ~7u; }
    static u32 grid_for(uint64_t work, u32 maxg) { return (u32)std::max<uint64_t>(1, std::min<uint64_t>((work + BLOCK - 1) / BLOCK, maxg)); }

    // Launches one step reading record buffer c and writing buffer c ^ 1.
    // The kernels that evaluate the 2D expansion are compiled for its order
    // (12, the default, or any order at run time).
    void enqueue_step(int c)
    {
        if constexpr (DIM == 2) {
            if (exact2d) return enqueue_step_n<NC_EXACT>(c);
            if (P.n_terms == 12) return enqueue_step_n<12>(c);
        }
        enqueue_step_n<0>(c);
    }

    template <int NC2> void enqueue_step_n(int c)
    {
        if (batch) return enqueue_step_t<NC2, true>(c);
        enqueue_step_t<NC2, false>(c);
    }

    template <int NC2, bool BATCH> void enqueue_step_t(int c)
    {
        hipStream_t st = M.stream;
        Rec<T> *in = rec[c], *out = rec[c ^ 1];
        const u32 g_all = grid_for(n, 8192);
        const u32 g_pl = M.pair_blocks;
        launch(SIM_K_MOVE, [&] { k_move_count<DIM, T, PM, BATCH><<<g_all, BLOCK, 0, st>>>(P, in, okey, tmp, rank, cnt, scnt, nkey, ctr); });
        launch(SIM_K_SCAN, [&] {
            const u32 *hw = pool ? &ctr->cell_hw : nullptr;
            k_scan_tiles<<<nb_scan, BLOCK, 0, st>>>(cnt, scnt, bsum, hw, P.n_cells);
            k_scan<<<nb_scan, BLOCK, 0, st>>>(cnt, scnt, bsum, start, ctr, hw, P.n_cells);
        });
        launch(SIM_K_SCATTER, [&] { k_scatter<DIM, T, BATCH><<<g_all, BLOCK, 0, st>>>(P, tmp, rank, start, out, okey, nkey, ctr); });
        if (M.debug) {
            k_fill<<<grid_for(n * DIM, 2048), BLOCK, 0, st>>>(dbg_moved, n * DIM, (int *)dbg_cells, (u32)n);
            k_gather<DIM, T><<<g_all, BLOCK, 0, st>>>(out, partner, ctr, 1, dbg_moved, nullptr, (u32)n);
            k_fill<<<grid_for(n * DIM, 2048), BLOCK, 0, st>>>(dbg_disp, n * DIM, nullptr, 0);
            k_dbg_disp<DIM, T, PM, BATCH><<<g_all, BLOCK, 0, st>>>(P, out, ctr, dbg_disp, (u32)n);
            k_dbg_cells<<<g_all, BLOCK, 0, st>>>(P, std::is_same<T, float>::value ? (const Rec<float> *)out : nullptr,
                                                 std::is_same<T, double>::value ? (const Rec<double> *)out : nullptr, start, ctr,
                                                 dbg_cells);
        }
        launch(SIM_K_PAIRS, [&] {
            // grids in multiples of the eight XCDs; the direct search takes no
            // more workgroups than are resident at once (2048)
            const u32 g_pairs = round8(grid_for(maxA, 2048));
            if (!BATCH && P.tiled) k_pair_scan<DIM, T, PM><<<round8(n_bricks), PBLOCK, 0, st>>>(P, out, start, plist, ctr);
            else if (narrow) k_pair_scan_direct_narrow<DIM, T, PM, BATCH><<<g_pairs, BLOCK, 0, st>>>(P, out, start, okey, plist, ctr);
            else k_pair_scan_direct<DIM, T, PM, BATCH><<<g_pairs, BLOCK, 0, st>>>(P, out, start, okey, plist, ctr);
        });
        launch(SIM_K_EVAL, [&] { k_pair_eval<DIM, T, PM, NC2, BATCH><<<g_pl, BLOCK, 0, st>>>(P, out, okey, plist, cand, flag, headA, nextA, ctr, dbg_pairs); });
        launch(SIM_K_SELECT_A, [&] { k_select_a<BATCH><<<g_pl, BLOCK, 0, st>>>(P, plist, cand, flag, headA, nextA, headB, nextB, ctr, dbg_picks); });
        const u32 nb_sel = g_pl, nb_dec = P.reversible ? grid_for(maxC, 2048) : 0;
        launch(SIM_K_SELECT_B, [&] {
            k_select_b<T, BATCH><<<nb_sel + nb_dec, BLOCK, 0, st>>>(P, plist, cand, flag, headB, nextB, out, start, okey, ev, ctr, nb_sel);
        });
        if (DIM == 3 && angles) {  // 3D: events and angles in one launch (timed as the angle stage)
            if constexpr (DIM == 3)
                launch(SIM_K_ANGLES, [&] {
                    k_events_angles<DIM, T, NC2, PM, BATCH><<<M.event_blocks, AWG, 0, st>>>(dparams, out, plist, cand, ev, partner,
                                                                                            ctr, dbg_matches, dbg_diss, ang, gl16);
                });
        } else {
            // 2D: the two held together spill (the expansion's arrays beside the angle's), so apart
            launch(SIM_K_EVENTS, [&] {
                k_events<DIM, T, NC2, BATCH><<<M.event_blocks, BLOCK, 0, st>>>(dparams, out, plist, cand, ev, partner, ctr,
                                                                               dbg_matches, dbg_diss, angles ? ang : nullptr);
            });
            if (angles)
                launch(SIM_K_ANGLES, [&] {
                    k_angles<DIM, T, PM, BATCH><<<M.event_blocks, AWG, 0, st>>>(dparams, out, ang, ctr, dbg_matches, gl16);
                });
        }
        k_close<<<1, 64, 0, st>>>(ctr);
    }

    int one_step()
    {
        const bool graph = !M.debug && !M.timing;
        if (graph) {
            if (!gexec[cur]) {
                hipGraph_t g = nullptr;
                HIPCHECK(hipStreamBeginCapture(M.stream, hipStreamCaptureModeThreadLocal));
                enqueue_step(cur);
                HIPCHECK(hipStreamEndCapture(M.stream, &g));
                const hipError_t e = hipGraphInstantiate(&gexec[cur], g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) return fail(SIM_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
            }
            HIPCHECK(hipGraphLaunch(gexec[cur], M.stream));
        } else {
            enqueue_step(cur);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return fail(SIM_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
        }
        cur ^= 1;
        ++stepno;
        return SIM_OK;
    }

    int eval_pairs(uint64_t n, const double *R, const double *R0, double *penc, double *preac) override
    {
        if (exact2d && !P.x2_enc) return fail(SIM_EUNSUPPORTED, "the exact 2D tables of a pool are its members': evaluate on a handle of the system");
        const u32 g = grid_for(n, 16384);
        bool done = false;
        if constexpr (DIM == 2) {
            if (P.x2_enc) {
                k_eval_probs<DIM, PM, NC_EXACT><<<g, BLOCK, 0, M.stream>>>(P, n, R, R0, penc, preac);
                done = true;
            } else if (P.n_terms == 12) {
                k_eval_probs<DIM, PM, 12><<<g, BLOCK, 0, M.stream>>>(P, n, R, R0, penc, preac);
                done = true;
            }
        }
        if (!done) k_eval_probs<DIM, PM, 0><<<g, BLOCK, 0, M.stream>>>(P, n, R, R0, penc, preac);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(M.stream));
        return SIM_OK;
    }

    int eval_prop(uint64_t n, const double *R0, uint32_t step, int wave, double *Rpp, uint32_t *attempts) override
    {
        if (n > 0xFFFFFFFFull) return fail(SIM_EINVAL, "at most 2^32 draws");
        if (exact2d && !P.x2_enc) return fail(SIM_EUNSUPPORTED, "the exact 2D tables of a pool are its members': evaluate on a handle of the system");
        if (DIM == 2 && P.x2_enc) launch_prop<NC_EXACT>(n, R0, step, wave, Rpp, attempts);
        else if (DIM == 2 && P.n_terms == 12) launch_prop<12>(n, R0, step, wave, Rpp, attempts);
        else launch_prop<0>(n, R0, step, wave, Rpp, attempts);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(M.stream));
        return SIM_OK;
    }

    int eval_first_passage(uint64_t n, const double *xi, const double *xf, int levels, uint32_t step, uint64_t *lo,
                           uint32_t *attempts) override
    {
        if (DIM == 2 && (exact2d || P.n_terms != 12))
            return fail(SIM_EUNSUPPORTED, "the 2D first-passage bisection takes the expansion of order 12");
        if (n > 0xFFFFFFFFull) return fail(SIM_EINVAL, "at most 2^32 pairs");
        if (levels < 1 || levels > 52) return fail(SIM_EINVAL, "levels must be in [1, 52]");
        const u32 g = grid_for(n * FP_GROUP, 16384);
        if constexpr (DIM == 3) k_first_passage<3, 0><<<g, BLOCK, 0, M.stream>>>(P, n, xi, xf, levels, step, lo, attempts);
        else k_first_passage<2, 12><<<g, BLOCK, 0, M.stream>>>(P, n, xi, xf, levels, step, lo, attempts);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(M.stream));
        return SIM_OK;
    }

    int eval_angle(uint64_t n, const double *R, const double *R0, const double *u, double *out) override
    {
        if (n > 0xFFFFFFFFull) return fail(SIM_EINVAL, "at most 2^32 pairs");
        // below this the series needs more than its 160 terms (R R0 / tau > 500) and the
        // quadrature grows like 1 / sqrt(tau) nodes per pair
        if (!(P.tau >= ANG_TAU_MIN)) return fail(SIM_EUNSUPPORTED, "the angular series is built for tau >= 2e-3");
        k_angle_wg<DIM><<<(u32)std::min<uint64_t>(n, 16384), AWG, 0, M.stream>>>(P.tau, n, R, R0, u, out, gl16);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(M.stream));
        return SIM_OK;
    }

    template <int NC> void launch_prop(uint64_t n, const double *R0, uint32_t step, int wave, double *Rpp, uint32_t *attempts)
    {
        if (wave) k_eval_prop<DIM, NC, true><<<grid_for(64 * n, 8192), BLOCK, 0, M.stream>>>(P, n, R0, step, Rpp, attempts);
        else k_eval_prop<DIM, NC, false><<<grid_for(n, 8192), BLOCK, 0, M.stream>>>(P, n, R0, step, Rpp, attempts);
    }

    int step(uint32_t nsteps) override
    {
        for (uint32_t i = 0; i < nsteps; ++i) {
            const int rc = one_step();
            if (rc) return rc;
        }
        return sync();
    }

    int step_async(uint32_t nsteps) override
    {
        if (M.debug || M.timing) return fail(SIM_EINVAL, "sim_step_async needs a handle without debug logs or kernel timing");
        for (uint32_t i = 0; i < nsteps; ++i) {
            const int rc = one_step();
            if (rc) return rc;
        }
        return SIM_OK;
    }

    // Waits for the stream; the capacity flags of every step since the last check.
    int sync() override
    {
        u32 errflags = 0;
        HIPCHECK(hipMemcpyAsync(&errflags, &ctr->err, sizeof(u32), hipMemcpyDeviceToHost, M.stream));
        HIPCHECK(hipStreamSynchronize(M.stream));
        if (M.timing) {
            for (auto &e : ev_used) {
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e.a, e.b);
                k_ms[e.k] += ms;
                k_launches[e.k] += 1;
                ev_pool.push_back(e);
            }
            ev_used.clear();
        }
        if (errflags) {
            HIPCHECK(hipMemsetAsync(&ctr->err, 0, sizeof(u32), M.stream));
            return fail(SIM_ECAPACITY, "per-step buffer overflow (flags " + std::to_string(errflags) + ")");
        }
        return SIM_OK;
    }

    int copy_out(const void *src, uint64_t bytes, void *dst, uint64_t cap, uint64_t *written)
    {
        if (bytes > cap) return fail(SIM_EINVAL, "destination buffer too small");
        HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, M.stream));
        HIPCHECK(hipStreamSynchronize(M.stream));
        if (written) *written = bytes;
        return SIM_OK;
    }

    int read(int what, void *dst, uint64_t cap, uint64_t *written) override
    {
        hipStream_t st = M.stream;
        const u32 g_all = grid_for(n, 8192);
        Counters c;
        HIPCHECK(hipMemcpyAsync(&c, ctr, sizeof(c), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        switch (what) {
        case SIM_READ_POS:
        case SIM_READ_SPECIES:
        case SIM_READ_COUNTS: {
            k_fill<<<grid_for(n * DIM, 2048), BLOCK, 0, st>>>(g_pos, n * DIM, g_sp, (u32)n);
            k_gather<DIM, T><<<g_all, BLOCK, 0, st>>>(rec[cur], partner, ctr, 0, g_pos, g_sp, (u32)n);
            if (what == SIM_READ_POS) return copy_out(g_pos, sizeof(double) * n * DIM, dst, cap, written);
            if (what == SIM_READ_SPECIES) return copy_out(g_sp, sizeof(int) * n, dst, cap, written);
            std::vector<int> h(n);
            HIPCHECK(hipMemcpyAsync(h.data(), g_sp, sizeof(int) * n, hipMemcpyDeviceToHost, st));
            HIPCHECK(hipStreamSynchronize(st));
            int64_t cnts[5] = {0, 0, 0, 0, 0};
            for (int v : h) cnts[v] += 1;
            if (cap < sizeof(cnts)) return fail(SIM_EINVAL, "destination buffer too small");
            std::memcpy(dst, cnts, sizeof(cnts));
            if (written) *written = sizeof(cnts);
            return SIM_OK;
        }
        case SIM_READ_PARTNER: {
            std::vector<u32> h(n);
            std::vector<int> s_(n);
            HIPCHECK(hipMemcpyAsync(h.data(), partner, sizeof(u32) * n, hipMemcpyDeviceToHost, st));
            k_fill<<<grid_for(n * DIM, 2048), BLOCK, 0, st>>>(g_pos, n * DIM, g_sp, (u32)n);
            k_gather<DIM, T><<<g_all, BLOCK, 0, st>>>(rec[cur], partner, ctr, 0, nullptr, g_sp, (u32)n);
            HIPCHECK(hipMemcpyAsync(s_.data(), g_sp, sizeof(int) * n, hipMemcpyDeviceToHost, st));
            HIPCHECK(hipStreamSynchronize(st));
            for (uint64_t i = 0; i < n; ++i)
                if (s_[i] != SIM_SP_C) h[i] = NOSLOT;
            if (cap < sizeof(u32) * n) return fail(SIM_EINVAL, "destination buffer too small");
            std::memcpy(dst, h.data(), sizeof(u32) * n);
            if (written) *written = sizeof(u32) * n;
            return SIM_OK;
        }
        case SIM_READ_STATS:
        case SIM_READ_STATS_SUM: {
            const u64 *src = what == SIM_READ_STATS ? c.stats_last : c.stats_sum;
            if (cap < sizeof(u64) * SIM_STAT_N) return fail(SIM_EINVAL, "destination buffer too small");
            std::memcpy(dst, src, sizeof(u64) * SIM_STAT_N);
            if (written) *written = sizeof(u64) * SIM_STAT_N;
            return SIM_OK;
        }
        case SIM_READ_DERIVED: {
            const double d[8] = {M.D[0] + M.D[1], P.tau, P.hh, P.rcut, P.a, P.p_uni, cell_edge, (double)stepno};
            if (cap < sizeof(d)) return fail(SIM_EINVAL, "destination buffer too small");
            std::memcpy(dst, d, sizeof(d));
            if (written) *written = sizeof(d);
            return SIM_OK;
        }
        case SIM_READ_GRID: {
            const int64_t g[5] = {P.nc[0], P.nc[1], P.nc[2], (int64_t)P.n_cells, P.tiled ? SIM_PAIRS_BRICKS : SIM_PAIRS_DIRECT};
            if (cap < sizeof(g)) return fail(SIM_EINVAL, "destination buffer too small");
            std::memcpy(dst, g, sizeof(g));
            if (written) *written = sizeof(g);
            return SIM_OK;
        }
        case SIM_READ_TIMING: {
            sim_kernel_time t[SIM_K_N];
            for (int k = 0; k < SIM_K_N; ++k) {
                t[k].ms = k_ms[k];
                t[k].launches = k_launches[k];
                k_ms[k] = 0.0;
                k_launches[k] = 0;
            }
            if (cap < sizeof(t)) return fail(SIM_EINVAL, "destination buffer too small");
            std::memcpy(dst, t, sizeof(t));
            if (written) *written = sizeof(t);
            return SIM_OK;
        }
        default:
            break;
        }
        if (!M.debug) return fail(SIM_ESTATE, "debug logs need sim_config.debug = 1");
        switch (what) {
        case SIM_READ_DBG_MOVED: return copy_out(dbg_moved, sizeof(double) * n * DIM, dst, cap, written);
        case SIM_READ_DBG_DISP: return copy_out(dbg_disp, sizeof(double) * n * DIM, dst, cap, written);
        case SIM_READ_DBG_CELLS: return copy_out(dbg_cells, sizeof(u32) * n, dst, cap, written);
        case SIM_READ_DBG_PAIRS: return copy_out(dbg_pairs, sizeof(DbgPair) * std::min<uint64_t>(c.n_dbg[0], M.dbg_cap), dst, cap, written);
        case SIM_READ_DBG_PICKS: return copy_out(dbg_picks, sizeof(DbgPick) * std::min<uint64_t>(c.n_dbg[1], M.dbg_cap), dst, cap, written);
        case SIM_READ_DBG_MATCHES: return copy_out(dbg_matches, sizeof(DbgMatch) * std::min<uint64_t>(c.n_dbg[2], M.dbg_cap), dst, cap, written);
        case SIM_READ_DBG_DISS: return copy_out(dbg_diss, sizeof(DbgDiss) * std::min<uint64_t>(c.n_dbg[3], M.dbg_cap), dst, cap, written);
        default: return fail(SIM_EINVAL, "unknown read selector");
        }
    }
};

int validate_box(int dim, int prec, const double *box)
{
    for (int k = 0; k < dim; ++k) {
        if (!(std::isfinite(box[k]) && box[k] > 0.0)) { g_err = "box edges must be > 0"; return SIM_EINVAL; }
        if (prec != SIM_PREC_FP64 && (double)(float)box[k] != box[k]) {
            g_err = "binary32 states need box edges exactly representable in binary32";
            return SIM_EINVAL;
        }
    }
    return SIM_OK;
}

// Species codes, finite positions of the particles, and (reversible
// reaction) one RESERVED partner slot per C.
int validate_state(int dim, bool reversible, uint64_t n, const int32_t *sp, const double *pos, const uint32_t *pt)
{
    if (!sp || !pos) { g_err = "null argument"; return SIM_EINVAL; }
    if (n == 0 || n > SLOT_MASK) { g_err = "slot count must be in [1, 2^29)"; return SIM_EINVAL; }
    std::vector<int> owners(n, 0);
    for (uint64_t i = 0; i < n; ++i) {
        const int s = sp[i];
        if (s < 0 || s > SIM_SP_RESERVED) { g_err = "unknown species code"; return SIM_EINVAL; }
        if (s <= SIM_SP_C)
            for (int k = 0; k < dim; ++k)
                if (!std::isfinite(pos[i * dim + k])) { g_err = "non-finite position"; return SIM_EINVAL; }
        if (s == SIM_SP_C && reversible) {
            if (!pt || pt[i] >= n || sp[pt[i]] != SIM_SP_RESERVED) { g_err = "each C needs a RESERVED partner slot"; return SIM_EINVAL; }
            owners[pt[i]] += 1;
        }
    }
    for (uint64_t i = 0; i < n; ++i)
        if (sp[i] == SIM_SP_RESERVED && owners[i] != 1) { g_err = "each RESERVED slot must belong to exactly one C"; return SIM_EINVAL; }
    return SIM_OK;
}

// The largest tau = D_eff dt / a^2 at which the 2D small-time expansion of order n holds p_enc and
// p_reac to 1e-6: measured at contact (the worst place) against a numerical inversion of the
// Laplace-domain forms of Sec. 4.2 (eqs. absPert, refPert, radPert), on the grid 0.005, 0.01, 0.02,
// ..., 0.07, for intrinsic rates h up to 0.8.  Orders below 5 reach 1e-6 nowhere on it.
double g2_tau_max(int n)
{
    static const double lim[33] = {0.0,  0.0,  0.0,  0.0,  0.0,  0.005, 0.01, 0.02, 0.03, 0.04, 0.04,
                                   0.05, 0.05, 0.05, 0.06, 0.06, 0.06,  0.06, 0.06, 0.06, 0.07, 0.07,
                                   0.07, 0.07, 0.07, 0.07, 0.07, 0.07,  0.07, 0.07, 0.07, 0.07, 0.07};
    return n >= 0 && n <= 32 ? lim[n] : 0.0;
}

// Everything but the state.
int validate_cfg(const sim_config *cfg, Model &M)
{
    if (!cfg) { g_err = "null argument"; return SIM_EINVAL; }
    if (cfg->dim != 2 && cfg->dim != 3) { g_err = "dim must be 2 or 3"; return SIM_EINVAL; }
    if (cfg->precision < 0 || cfg->precision > 3) { g_err = "unknown precision"; return SIM_EINVAL; }
    if (cfg->n_species != 3 || !cfg->species) { g_err = "exactly three species (A, B, C) are supported"; return SIM_EUNSUPPORTED; }
    if (cfg->n_reactions != 1 || !cfg->reactions) { g_err = "exactly one reaction A + B <-> C is supported"; return SIM_EUNSUPPORTED; }
    const sim_reaction &r = cfg->reactions[0];
    if (r.a != 0 || r.b != 1 || r.c != 2) { g_err = "the reaction must be species 0 + 1 <-> 2"; return SIM_EUNSUPPORTED; }
    if (r.bc < 0 || r.bc > 2) { g_err = "unknown boundary condition"; return SIM_EINVAL; }
    if (!(std::isfinite(r.sigma) && r.sigma > 0.0) || !finite_nonneg(r.kappa) || !finite_nonneg(r.k_off)) {
        g_err = "sigma must be > 0, kappa and k_off >= 0";
        return SIM_EINVAL;
    }
    for (int s = 0; s < 3; ++s)
        if (!finite_nonneg(cfg->species[s].D)) { g_err = "diffusion constants must be finite and >= 0"; return SIM_EINVAL; }
    if (!(cfg->species[0].D + cfg->species[1].D > 0.0)) { g_err = "D_A + D_B must be > 0"; return SIM_EINVAL; }
    if (!(std::isfinite(cfg->dt) && cfg->dt > 0.0)) { g_err = "dt must be > 0"; return SIM_EINVAL; }
    int rc;
    if ((rc = validate_box(cfg->dim, cfg->precision, cfg->box))) return rc;
    if (cfg->n_terms < 0 || cfg->n_terms > MAXTERMS) { g_err = "n_terms must be in [0, 32]"; return SIM_EINVAL; }
    const double eps = cfg->eps_cut == 0.0 ? 1e-3 : cfg->eps_cut;
    if (!(eps > 0.0 && eps < 1.0)) { g_err = "eps_cut must be in (0, 1)"; return SIM_EINVAL; }
    if (!finite_nonneg(cfg->rcut) || !finite_nonneg(cfg->cell)) { g_err = "rcut and cell must be >= 0"; return SIM_EINVAL; }
    if (cfg->pair_search < SIM_PAIRS_AUTO || cfg->pair_search > SIM_PAIRS_DIRECT) { g_err = "unknown pair_search"; return SIM_EINVAL; }
    if (cfg->green2d != SIM_G2_EXPANSION && cfg->green2d != SIM_G2_EXACT) { g_err = "unknown green2d"; return SIM_EINVAL; }
    if (cfg->green2d == SIM_G2_EXACT && cfg->dim != 2) { g_err = "green2d = SIM_G2_EXACT is for 2D"; return SIM_EINVAL; }
    if (cfg->flags & ~(uint32_t)(SIM_F_UNVALIDATED_TAU | SIM_F_KEEP_DIRECTION)) { g_err = "unknown flags"; return SIM_EINVAL; }
    if (r.bc != SIM_BC_ABSORBING && !(cfg->flags & SIM_F_KEEP_DIRECTION) &&
        !((cfg->species[0].D + cfg->species[1].D) * cfg->dt / (r.sigma * r.sigma) >= ANG_TAU_MIN)) {
        g_err = "the angular propagator is built for tau = D_eff dt / a^2 >= 2e-3 (its series needs more than 160 terms "
                "below): set SIM_F_KEEP_DIRECTION to keep the free end point's direction instead";
        return SIM_EUNSUPPORTED;
    }
    if (cfg->dim == 2) {
        // tau computed from the inputs may round just above a limit it equals (0.04, 0.8)
        const double tau = (cfg->species[0].D + cfg->species[1].D) * cfg->dt / (r.sigma * r.sigma) * (1.0 - 1e-9);
        const int nt = cfg->n_terms == 0 ? 12 : cfg->n_terms;
        if (cfg->green2d == SIM_G2_EXACT && !(tau <= X2_TAU_MAX)) {
            g_err = "exact 2D functions are validated for tau = D_eff dt / a^2 <= 0.8";
            return SIM_EUNSUPPORTED;
        }
        if (cfg->green2d == SIM_G2_EXPANSION && !(cfg->flags & SIM_F_UNVALIDATED_TAU) && !(tau <= g2_tau_max(nt))) {
            g_err = "the 2D small-time expansion of order " + std::to_string(nt) + " holds p_enc and p_reac to 1e-6 only for tau <= " +
                    std::to_string(g2_tau_max(nt)) + " (tau = " + std::to_string(tau) +
                    "): use green2d = SIM_G2_EXACT, a smaller dt or a higher order, or set SIM_F_UNVALIDATED_TAU";
            return SIM_EUNSUPPORTED;
        }
    }
    if (cfg->pair_blocks != 0 && (cfg->pair_blocks < 8 || cfg->pair_blocks > 65536)) { g_err = "pair_blocks must be 0 or in [8, 65536]"; return SIM_EINVAL; }
    if (cfg->event_blocks < 0 || cfg->event_blocks > 65536) { g_err = "event_blocks must be in [0, 65536]"; return SIM_EINVAL; }
    M.dim = cfg->dim;
    M.prec = cfg->precision;
    M.bc = r.bc;
    for (int k = 0; k < 3; ++k) M.box[k] = k < cfg->dim ? cfg->box[k] : 1.0;
    M.dt = cfg->dt;
    for (int s = 0; s < 3; ++s) M.D[s] = cfg->species[s].D;
    M.sigma = r.sigma;
    M.kappa = r.kappa;
    M.k_off = r.k_off;
    M.eps = eps;
    M.rcut_req = cfg->rcut;
    M.cell_req = cfg->cell;
    M.pair_search = cfg->pair_search;
    M.green2d = cfg->green2d;
    M.flags = cfg->flags;
    M.pair_blocks = cfg->pair_blocks ? (u32)cfg->pair_blocks : 1024u;
    M.event_blocks = cfg->event_blocks ? (u32)cfg->event_blocks : EV_BLOCKS;
    M.seed = cfg->seed;
    M.replica = cfg->replica;
    M.n_terms = cfg->n_terms == 0 ? 12 : cfg->n_terms;
    M.debug = cfg->debug;
    M.timing = cfg->timing;
    M.dbg_cap = cfg->debug_cap == 0 ? (1u << 20) : cfg->debug_cap;
    M.stream = (hipStream_t)cfg->hip_stream;
    return SIM_OK;
}

int validate(const sim_config *cfg, uint64_t n, const int32_t *sp, const double *pos, const uint32_t *pt, Model &M)
{
    if (!cfg || !sp || !pos) { g_err = "null argument"; return SIM_EINVAL; }
    if (n == 0 || n > SLOT_MASK) { g_err = "slot count must be in [1, 2^29)"; return SIM_EINVAL; }
    int rc;
    if ((rc = validate_cfg(cfg, M))) return rc;
    return validate_state(cfg->dim, cfg->reactions[0].k_off > 0.0, n, sp, pos, pt);
}

template <int DIM, class T, int PM>
int make(const Model &M, uint64_t n, const int32_t *sp, const double *pos, const uint32_t *pt, sim_t **out)
{
    Engine<DIM, T, PM> *e = new (std::nothrow) Engine<DIM, T, PM>();
    if (!e) { g_err = "host allocation failed"; return SIM_ENOMEM; }
    const int rc = e->init(M, n, sp, pos, pt);
    if (rc) {
        g_err = e->err;
        delete e;
        return rc;
    }
    *out = e;
    return SIM_OK;
}

template <int DIM, class T, int PM>
int make_batch(const std::vector<Model> &ms, const std::vector<uint64_t> &nr, const std::vector<u32> &step0, const int32_t *sp,
               const double *pos, const uint32_t *pt, sim_t **out)
{
    Engine<DIM, T, PM> *e = new (std::nothrow) Engine<DIM, T, PM>();
    if (!e) { g_err = "host allocation failed"; return SIM_ENOMEM; }
    const int rc = e->init_batch(ms, nr, step0, sp, pos, pt);
    if (rc) {
        g_err = e->err;
        delete e;
        return rc;
    }
    *out = e;
    return SIM_OK;
}

template <int DIM, class T, int PM>
int make_pool(const Model &M, uint64_t slot_cap, uint64_t cell_cap, uint32_t rep_cap, sim_t **out)
{
    Engine<DIM, T, PM> *e = new (std::nothrow) Engine<DIM, T, PM>();
    if (!e) { g_err = "host allocation failed"; return SIM_ENOMEM; }
    const int rc = e->init_pool(M, slot_cap, cell_cap, rep_cap);
    if (rc) {
        g_err = e->err;
        delete e;
        return rc;
    }
    *out = e;
    return SIM_OK;
}

// ---------------------------------------------------------------------------
// sim_eval_pairs_noalloc: the pair probabilities of sim_eval_pairs without a handle
// and without allocating.  The kernel reads the 2D expansion constants from device
// memory; a handle keeps them in a buffer of its own, this entry point in `scratch`
// below, a file-scope array of which every device holds its own copy.  Host code
// never uses the array's name as an address: the address is looked up once per
// device (hipGetSymbolAddress, with that device current) and kept.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_DOUBLES = 4 * (MAXTERMS + 1);  // a_k(0) and three quotient series, orders 0 .. 32
constexpr int NOALLOC_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[NOALLOC_DEVICES] = {};

int scratch_address(double **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { g_err = "hipGetDevice failed"; return SIM_EDEVICE; }
    if (dev < 0 || dev >= NOALLOC_DEVICES) { g_err = "device index beyond the table of scratch addresses"; return SIM_EUNSUPPORTED; }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return SIM_EDEVICE;
        }
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return SIM_OK;
}

template <int DIM, int PM> void launch_probs(const Params &P, uint64_t n, const double *R, const double *R0, double *penc,
                                             double *preac, hipStream_t st)
{
    const u32 g = (u32)std::max<uint64_t>(1, std::min<uint64_t>((n + BLOCK - 1) / BLOCK, 16384));
    if (DIM == 2 && P.n_terms == 12) k_eval_probs<DIM, PM, 12><<<g, BLOCK, 0, st>>>(P, n, R, R0, penc, preac);
    else k_eval_probs<DIM, PM, 0><<<g, BLOCK, 0, st>>>(P, n, R, R0, penc, preac);
}

} // namespace

// the constants of the 2D expansion for intrinsic rate hh into out (one thread)
__global__ void k_g2_constants(double hh, double *out)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) h_g2_constants(hh, out);
}

extern "C" {

int sim_create(const sim_config *cfg, uint64_t n, const int32_t *species, const double *pos, const uint32_t *partner, sim_t **out)
{
    if (!out) { g_err = "null output handle"; return SIM_EINVAL; }
    *out = nullptr;
    Model M;
    const int rc = validate(cfg, n, species, pos, partner, M);
    if (rc) return rc;
    if (M.dim == 3) {
        if (M.prec == SIM_PREC_FP64) return make<3, double, PM_F64>(M, n, species, pos, partner, out);
        if (M.prec == SIM_PREC_FP32) return make<3, float, PM_F32>(M, n, species, pos, partner, out);
        if (M.prec == SIM_PREC_FP32D_FP64NC) return make<3, float, PM_F32D>(M, n, species, pos, partner, out);
        return make<3, float, PM_F32NC>(M, n, species, pos, partner, out);
    }
    if (M.prec == SIM_PREC_FP64) return make<2, double, PM_F64>(M, n, species, pos, partner, out);
    if (M.prec == SIM_PREC_FP32) return make<2, float, PM_F32>(M, n, species, pos, partner, out);
    if (M.prec == SIM_PREC_FP32D_FP64NC) return make<2, float, PM_F32D>(M, n, species, pos, partner, out);
    return make<2, float, PM_F32NC>(M, n, species, pos, partner, out);
}

int sim_step(sim_t *h, uint32_t nsteps)
{
    if (!h) { g_err = "null handle"; return SIM_EINVAL; }
    return h->step(nsteps);
}

int sim_step_async(sim_t *h, uint32_t nsteps)
{
    if (!h) { g_err = "null handle"; return SIM_EINVAL; }
    return h->step_async(nsteps);
}

int sim_sync(sim_t *h)
{
    if (!h) { g_err = "null handle"; return SIM_EINVAL; }
    return h->sync();
}

int sim_read(sim_t *h, int what, void *dst, uint64_t cap_bytes, uint64_t *written)
{
    if (!h || !dst) { g_err = "null argument"; return SIM_EINVAL; }
    return h->read(what, dst, cap_bytes, written);
}

int sim_load_state(sim_t *h, uint64_t step, const int32_t *species, const double *pos, const uint32_t *partner)
{
    if (!h || !species || !pos) { g_err = "null argument"; return SIM_EINVAL; }
    return h->load(step, species, pos, partner);
}

int sim_batch_create(const sim_config *cfg, uint32_t n_rep, const sim_replica *reps, sim_t **out)
{
    if (!out) { g_err = "null output handle"; return SIM_EINVAL; }
    *out = nullptr;
    if (!cfg || !reps || n_rep == 0) { g_err = "null argument or no replicas"; return SIM_EINVAL; }
    std::vector<Model> ms(n_rep);
    std::vector<uint64_t> nr(n_rep);
    std::vector<u32> step0(n_rep);
    uint64_t total = 0;
    for (uint32_t r = 0; r < n_rep; ++r) {
        // each replica is checked as a system of its own: its box, kappa and replica key
        sim_config c = *cfg;
        for (int k = 0; k < 3; ++k) c.box[k] = reps[r].box[k];
        if (cfg->dim != 2 && cfg->dim != 3) { g_err = "dim must be 2 or 3"; return SIM_EINVAL; }
        c.replica = reps[r].replica;
        sim_reaction rx = cfg->reactions ? cfg->reactions[0] : sim_reaction{};
        rx.kappa = reps[r].kappa;
        c.reactions = cfg->reactions ? &rx : nullptr;
        const int rc = validate(&c, reps[r].n, reps[r].species, reps[r].pos, reps[r].partner, ms[r]);
        if (rc) return rc;
        nr[r] = reps[r].n;
        step0[r] = reps[r].step;
        total += reps[r].n;
    }
    if (total > SLOT_MASK) { g_err = "more than 2^29 slots in the batch"; return SIM_EINVAL; }
    // global arrays: replica r's slots follow those of replicas 0..r-1; partners become global
    const int d = cfg->dim;
    std::vector<int32_t> sp(total);
    std::vector<double> pos(total * d);
    std::vector<uint32_t> pt(total, 0xFFFFFFFFu);
    uint64_t base = 0;
    for (uint32_t r = 0; r < n_rep; ++r) {
        for (uint64_t i = 0; i < nr[r]; ++i) {
            sp[base + i] = reps[r].species[i];
            for (int k = 0; k < d; ++k) pos[d * (base + i) + k] = reps[r].pos[d * i + k];
            if (reps[r].partner && reps[r].species[i] == SIM_SP_C && reps[r].partner[i] != 0xFFFFFFFFu)
                pt[base + i] = (uint32_t)(base + reps[r].partner[i]);
        }
        base += nr[r];
    }
    const Model &M = ms[0];
    if (d == 3) {
        if (M.prec == SIM_PREC_FP64) return make_batch<3, double, PM_F64>(ms, nr, step0, sp.data(), pos.data(), pt.data(), out);
        if (M.prec == SIM_PREC_FP32) return make_batch<3, float, PM_F32>(ms, nr, step0, sp.data(), pos.data(), pt.data(), out);
        if (M.prec == SIM_PREC_FP32D_FP64NC) return make_batch<3, float, PM_F32D>(ms, nr, step0, sp.data(), pos.data(), pt.data(), out);
        return make_batch<3, float, PM_F32NC>(ms, nr, step0, sp.data(), pos.data(), pt.data(), out);
    }
    if (M.prec == SIM_PREC_FP64) return make_batch<2, double, PM_F64>(ms, nr, step0, sp.data(), pos.data(), pt.data(), out);
    if (M.prec == SIM_PREC_FP32) return make_batch<2, float, PM_F32>(ms, nr, step0, sp.data(), pos.data(), pt.data(), out);
    if (M.prec == SIM_PREC_FP32D_FP64NC) return make_batch<2, float, PM_F32D>(ms, nr, step0, sp.data(), pos.data(), pt.data(), out);
    return make_batch<2, float, PM_F32NC>(ms, nr, step0, sp.data(), pos.data(), pt.data(), out);
}

int sim_pool_create(const sim_config *cfg, uint64_t slot_cap, uint64_t cell_cap, uint32_t rep_cap, sim_t **out)
{
    if (!out) { g_err = "null output handle"; return SIM_EINVAL; }
    *out = nullptr;
    Model M;
    int rc;
    if ((rc = validate_cfg(cfg, M))) return rc;
    if (slot_cap == 0 || slot_cap > SLOT_MASK) { g_err = "slot capacity must be in [1, 2^29)"; return SIM_EINVAL; }
    if (cell_cap == 0 || cell_cap > (1ull << 28)) { g_err = "cell capacity must be in [1, 2^28]"; return SIM_EINVAL; }
    if (rep_cap == 0 || rep_cap > (1u << 20)) { g_err = "member capacity must be in [1, 2^20]"; return SIM_EINVAL; }
    if (M.dim == 3) {
        if (M.prec == SIM_PREC_FP64) return make_pool<3, double, PM_F64>(M, slot_cap, cell_cap, rep_cap, out);
        if (M.prec == SIM_PREC_FP32) return make_pool<3, float, PM_F32>(M, slot_cap, cell_cap, rep_cap, out);
        if (M.prec == SIM_PREC_FP32D_FP64NC) return make_pool<3, float, PM_F32D>(M, slot_cap, cell_cap, rep_cap, out);
        return make_pool<3, float, PM_F32NC>(M, slot_cap, cell_cap, rep_cap, out);
    }
    if (M.prec == SIM_PREC_FP64) return make_pool<2, double, PM_F64>(M, slot_cap, cell_cap, rep_cap, out);
    if (M.prec == SIM_PREC_FP32) return make_pool<2, float, PM_F32>(M, slot_cap, cell_cap, rep_cap, out);
    if (M.prec == SIM_PREC_FP32D_FP64NC) return make_pool<2, float, PM_F32D>(M, slot_cap, cell_cap, rep_cap, out);
    return make_pool<2, float, PM_F32NC>(M, slot_cap, cell_cap, rep_cap, out);
}

int sim_pool_admit(sim_t *h, const sim_replica *rep, uint32_t *member)
{
    if (!h || !rep || !member) { g_err = "null argument"; return SIM_EINVAL; }
    return h->admit(*rep, member);
}

int sim_pool_retire(sim_t *h, uint32_t member)
{
    if (!h) { g_err = "null handle"; return SIM_EINVAL; }
    return h->retire(member);
}

int sim_pool_read(sim_t *h, uint32_t member, int what, void *dst, uint64_t cap_bytes, uint64_t *written)
{
    if (!h || !dst) { g_err = "null argument"; return SIM_EINVAL; }
    return h->read_member(member, what, dst, cap_bytes, written);
}

int sim_eval_pairs(sim_t *h, uint64_t n, const double *R, const double *R0, double *penc, double *preac)
{
    if (!h || !R || !R0 || n == 0) { g_err = "null argument or n = 0"; return SIM_EINVAL; }
    return h->eval_pairs(n, R, R0, penc, preac);
}

int sim_eval_pairs_noalloc(const sim_config *cfg, uint64_t n, const double *R, const double *R0, double *penc, double *preac)
{
    if (!cfg || !R || !R0 || n == 0) { g_err = "null argument or n = 0"; return SIM_EINVAL; }
    Model M;
    int rc;
    if ((rc = validate_cfg(cfg, M))) return rc;
    if (M.green2d == SIM_G2_EXACT) {
        g_err = "the exact 2D functions are tables a handle builds (device memory): use sim_eval_pairs";
        return SIM_EUNSUPPORTED;
    }
    static_assert(NOALLOC_DOUBLES == sizeof(scratch) / sizeof(double), "scratch holds the 2D constants");
    double *ptr = nullptr;
    if ((rc = scratch_address(&ptr))) return rc;
    Params P;
    phys_params(M, P);
    P.g2c = ptr;  // read by the 2D expansion only
    hipStream_t st = (hipStream_t)cfg->hip_stream;
    if (M.dim == 2) k_g2_constants<<<1, 64, 0, st>>>(P.hh, ptr);
    if (M.dim == 3) {
        if (M.prec == SIM_PREC_FP64) launch_probs<3, PM_F64>(P, n, R, R0, penc, preac, st);
        else if (M.prec == SIM_PREC_FP32) launch_probs<3, PM_F32>(P, n, R, R0, penc, preac, st);
        else if (M.prec == SIM_PREC_FP32D_FP64NC) launch_probs<3, PM_F32D>(P, n, R, R0, penc, preac, st);
        else launch_probs<3, PM_F32NC>(P, n, R, R0, penc, preac, st);
    } else {
        if (M.prec == SIM_PREC_FP64) launch_probs<2, PM_F64>(P, n, R, R0, penc, preac, st);
        else if (M.prec == SIM_PREC_FP32) launch_probs<2, PM_F32>(P, n, R, R0, penc, preac, st);
        else if (M.prec == SIM_PREC_FP32D_FP64NC) launch_probs<2, PM_F32D>(P, n, R, R0, penc, preac, st);
        else launch_probs<2, PM_F32NC>(P, n, R, R0, penc, preac, st);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) { g_err = std::string("sim_eval_pairs_noalloc: ") + hipGetErrorString(e); return SIM_EDEVICE; }
    return SIM_OK;
}

int sim_eval_propagator(sim_t *h, uint64_t n, const double *R0, uint32_t step, int wave, double *Rpp, uint32_t *attempts)
{
    if (!h || !R0 || !Rpp || n == 0) { g_err = "null argument or n = 0"; return SIM_EINVAL; }
    return h->eval_prop(n, R0, step, wave, Rpp, attempts);
}

int sim_eval_angle(sim_t *h, uint64_t n, const double *R, const double *R0, const double *u, double *out)
{
    if (!h || !R || !R0 || !u || !out || n == 0) { g_err = "null argument or n = 0"; return SIM_EINVAL; }
    return h->eval_angle(n, R, R0, u, out);
}

int sim_eval_first_passage(sim_t *h, uint64_t n, const double *xi, const double *xf, int32_t levels, uint32_t step,
                           uint64_t *lo, uint32_t *attempts)
{
    if (!h || !xi || !xf || !lo || n == 0) { g_err = "null argument or n = 0"; return SIM_EINVAL; }
    return h->eval_first_passage(n, xi, xf, levels, step, lo, attempts);
}

int sim_destroy(sim_t *h)
{
    delete h;
    return SIM_OK;
}

const char *sim_last_error(const sim_t *h)
{
    if (h) return h->err.c_str();
    return g_err.c_str();
}

} // extern "C"
