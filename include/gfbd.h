/*
 * gfbd.h - C-ABI of the MI355X (gfx950) implementation of the coarse-grained
 * Green's-function Brownian-dynamics step of T. Pruestel and M.
 * Meier-Schellersheim, "Coarse-Grained Stochastic Particle-based
 * Reaction-Diffusion Simulation Algorithm" (arXiv:1107.0270).
 *
 * One call of sim_step advances the state by one time step dt of the
 * algorithm of Sec. 3:
 *   1. every particle takes a free Gaussian step sqrt(2 D dt) N(0,1)  (step 1);
 *   2. all A-B pairs closer than the cut-off r_cut (Sec. 3, Details) are found;
 *   3. each pair gets the encounter probability p_enc = 1 - G_abs/G_free
 *      (Sec. 2.2.1, radial form Sec. 2.2.4; 3D closed forms of Sec. 4.1, 2D
 *      small-time expansions of Sec. 4.2), overlapping pairs p_enc = 1, and a
 *      Bernoulli draw (steps 2 and 3);
 *   4. each A picks one of its candidates with probability p_enc / sum p_enc,
 *      then each B picked several times picks one of those A's (Sec. 3, Details);
 *   5. matched pairs react (absorbing), or get a new separation from the radial
 *      propagator w_d r^{d-1}(g_ref - g_abs) (Sec. 2.2.2) and react with
 *      p_reac = (G_ref - G_rad)/(G_ref - G_abs) (Sec. 2.2.3);
 *   6. C decays to A + B with p = 1 - exp(-k_off dt), the products start at
 *      contact, are propagated from r0 = a and may recombine (Sec. 2.2.5, step 4).
 *
 * Units: lengths in um, times in s, D in um^2/s, kappa_a in um^3/s (3D) or
 * um^2/s (2D), k_off in 1/s.  Species: exactly one channel A + B <-> C.
 *
 * State model: a fixed set of slots 0..n-1.  A slot holds an A, B or C, is
 * FREE, or is RESERVED by the C that consumed its B (reversible channel only);
 * when that C dissociates, its B returns to the reserved slot.  Positions are
 * kept in the precision of the state (binary64 for SIM_PREC_FP64, binary32
 * otherwise); every update is computed in binary64 and rounded once.
 *
 * Random numbers: Philox4x32-10 with key {seed_lo, seed_hi ^ replica} and
 * counter {slot, partner slot or 0xFFFFFFFF, step, tag | attempt << 8}; every
 * draw is a pure function of the particles and the step it belongs to.
 *
 * Errors: every call returns SIM_OK or a negative code and never throws.
 * sim_last_error(h) describes the last failure on that handle.  Handles are
 * not thread-safe; use one handle per host thread and stream.
 */
#ifndef GFBD_H
#define GFBD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sim sim_t; /* opaque, owned by the library */

enum {
    SIM_OK = 0,
    SIM_EINVAL = -1,      /* an argument is out of range; nothing changed */
    SIM_ENOMEM = -2,      /* device or host allocation failed */
    SIM_EDEVICE = -3,     /* a HIP call failed; the handle should be destroyed */
    SIM_ESTATE = -4,      /* call not valid in the handle's current state */
    SIM_EUNSUPPORTED = -5,/* valid input outside what this library supports */
    SIM_ECAPACITY = -6    /* a per-step buffer overflowed; the step's results are invalid */
};

enum { SIM_SP_A = 0, SIM_SP_B = 1, SIM_SP_C = 2, SIM_SP_FREE = 3, SIM_SP_RESERVED = 4 };
enum { SIM_BC_ABSORBING = 0, SIM_BC_REFLECTING = 1, SIM_BC_RADIATION = 2 };

/* Precision of the state and of the pair probabilities:
 *  FP64          state and all arithmetic in binary64;
 *  FP32          binary32 state; displacements (Box-Muller), pair search and p_enc in binary32;
 *  FP32_FP64NC   binary32 state, binary64 displacements, binary32 p_enc whose arguments (r, r - a,
 *                r0 - a and the exponent arguments) are formed in binary64;
 *  FP32D_FP64NC  as FP32_FP64NC, with the displacements of FP32 (binary32 Box-Muller).  Its moves
 *                differ from the binary64 ones by binary32 roundings of the displacement, so its
 *                trajectories are compared stage by stage from the step's own post-move state
 *                (SIM_READ_DBG_MOVED, SIM_READ_DBG_DISP).
 * Placements, the propagator and p_reac are binary64 in all modes. */
enum { SIM_PREC_FP64 = 0, SIM_PREC_FP32 = 1, SIM_PREC_FP32_FP64NC = 2, SIM_PREC_FP32D_FP64NC = 3 };

/* Kernel of the pair search (step 2); both find exactly the same pairs.
 *  BRICKS  one workgroup per brick of cells stages the B records of the brick
 *          and its one-cell halo in LDS (pays off with many B's per A);
 *  DIRECT  one thread per A reads the neighbour buckets through L2;
 *  AUTO    BRICKS when an A is expected to test more than 8 B's, else DIRECT.
 * Grids with fewer than three cells along some axis always use DIRECT. */
enum { SIM_PAIRS_AUTO = 0, SIM_PAIRS_BRICKS = 1, SIM_PAIRS_DIRECT = 2 };

typedef struct {
    double D; /* diffusion constant, um^2/s, >= 0 */
} sim_species;

typedef struct {
    int32_t a, b, c;  /* species indices: must be 0, 1, 2 */
    int32_t bc;       /* SIM_BC_* of the A-B encounter surface */
    double sigma;     /* encounter radius a_eff, um, > 0 (eq. smol_bc) */
    double kappa;     /* intrinsic association rate kappa_a (eq. robin_bc), >= 0 */
    double k_off;     /* C -> A + B rate (eq. single_rate), 1/s; 0 = irreversible */
} sim_reaction;

typedef struct {
    int32_t dim;                   /* 2 or 3 */
    int32_t precision;             /* SIM_PREC_* */
    double box[3];                 /* periodic box edges, um (box[2] ignored in 2D) */
    double dt;                     /* time step, s, > 0 */
    uint64_t seed;                 /* Philox key material */
    uint32_t replica;              /* folded into the Philox key */
    int32_t n_terms;               /* order of the 2D small-time expansion, 1..32 (0 = 12) */
    double eps_cut;                /* cut-off: 1 - S(dt | r_cut) = eps_cut (0 = 1e-3) */
    double rcut;                   /* > 0: use this cut-off (um) instead of deriving it */
    double cell;                   /* > 0: requested cell edge (um, raised to >= r_cut); 0 = automatic */
    int32_t pair_search;           /* SIM_PAIRS_* */
    int32_t n_species;             /* must be 3: A, B, C */
    const sim_species *species;    /* n_species entries; D_C is the C diffusion constant */
    int32_t n_reactions;           /* must be 1 */
    const sim_reaction *reactions;
    uint32_t debug;                /* 1: record the last step's stage logs for sim_read */
    uint32_t timing;               /* 1: time every kernel with HIP events (sim_read SIM_READ_TIMING) */
    uint64_t debug_cap;            /* entries per stage log (0 = 1 << 20) */
    void *hip_stream;              /* hipStream_t to run on; NULL = the null stream */
    int32_t green2d;               /* 2D radial functions: SIM_G2_EXPANSION or SIM_G2_EXACT (2D only) */
    int32_t pair_blocks;           /* workgroups of the pair-evaluation and selection kernels, 8..65536 (0 = 1024) */
    int32_t event_blocks;          /* workgroups of the event kernel, 1..65536 (0 = 1024) */
    uint32_t flags;                /* SIM_F_* bits (0: the paper's method, validated ranges only) */
} sim_config;

/* sim_config.green2d.
 * EXPANSION: the small-time expansions of Sec. 4.2 (eq. smallTEabs and its reflecting and radiation
 *   forms) to order n_terms.  Each order holds p_enc and p_reac to 1e-6 (measured against a numerical
 *   inversion of the Laplace-domain forms eqs. absPert, refPert and radPert, worst case at contact,
 *   h up to 0.8) only up to a tau = D_eff dt / a^2 that grows with the order: n_terms 5: 0.005,
 *   6: 0.01, 7: 0.02, 8: 0.03, 9-10: 0.04, 11-13: 0.05, 14-19: 0.06, 20-32: 0.07; orders 1-4 reach
 *   1e-6 nowhere.  Beyond that limit a 2D handle is refused (SIM_EUNSUPPORTED) unless flags has
 *   SIM_F_UNVALIDATED_TAU.
 * EXACT: the n = 0 term of the 2D Green's function (Sec. 4.2, its Bessel-function form, eqs.
 *   genericGF and fRad) by quadrature, tabulated on the device when the handle is created (a grid of
 *   step sqrt(tau)/160 in R, twice that in R0, read by bicubic interpolation): p_enc, p_reac and
 *   the propagator's distribution function, R'' then drawn by inversion of one uniform, word 0 of
 *   the counter of attempt 0.  Pairs with R0 beyond 1 + c sqrt(tau) (c = 8.4 for tau <= 0.5, 9 above)
 *   use the order-n_terms expansion, which holds there.  Accuracy against the Laplace inversion:
 *   1e-6 for tau <= 0.5, 1.5e-6 up to tau = 0.8; tau > 0.8 is refused (SIM_EUNSUPPORTED), as are
 *   EXACT in 3D (SIM_EINVAL) and tables over 2^26 entries (SIM_EUNSUPPORTED).  Batches and pools
 *   build one set of tables per distinct kappa (per cut-off) of their replicas or members, kept
 *   until the handle is destroyed: about 60 MB at tau = 0.8 (three tables of 3,500 x 720 doubles). */
enum { SIM_G2_EXPANSION = 0, SIM_G2_EXACT = 1 };

/* sim_config.flags.
 * UNVALIDATED_TAU  accept the 2D expansion beyond the tau its order holds to 1e-6 (see green2d);
 *                  the probabilities are then those of the truncated series, not the paper's.
 * KEEP_DIRECTION   after a non-reactive encounter keep the direction of the pair's free end point
 *                  and redraw only its length, instead of drawing the angle to the old separation
 *                  from the full propagator (Sec. 3, Details); exact for every single-pair radial
 *                  statistic, not for many-body geometry.  For comparison with that reading. */
enum { SIM_F_UNVALIDATED_TAU = 1u, SIM_F_KEEP_DIRECTION = 2u };

/* Creates a simulation with n slots.  species[i] in {A, B, C, FREE, RESERVED};
 * pos is n*dim doubles (slot-major, ignored for FREE/RESERVED); partner[i] is
 * the reserved slot of C slot i (may be NULL if there is no C).  Host buffers
 * are copied; the caller keeps ownership.  The library allocates all device
 * memory.  Returns SIM_EINVAL for NaN or negative parameters, dim not 2 or 3,
 * r_cut >= min(box)/2, or an inconsistent C/RESERVED map. */
int sim_create(const sim_config *cfg, uint64_t n, const int32_t *species, const double *pos,
               const uint32_t *partner, sim_t **out);

/* One replica of a batch: its own slots (n, species, positions, partners as in sim_create,
 * partner indices local to the replica), periodic box, intrinsic rate kappa_a, replica number
 * (folded into its Philox key) and own step counter (replicas may join at different points of
 * their trajectories; a replica continued from a state read at its step s is created with s). */
typedef struct {
    uint64_t n;
    const int32_t *species;
    const double *pos;
    const uint32_t *partner;
    double box[3];
    double kappa;
    uint32_t replica;
    uint32_t step;          /* the replica's own step counter at creation (its draws are keyed on it) */
} sim_replica;

/* Creates one handle that steps n_rep independent replicas together: every step of the
 * algorithm of Sec. 3 runs once for all of them (one graph replay per step).  cfg supplies
 * what the replicas share (precision, dt, species D, sigma, boundary condition, k_off, seed,
 * eps_cut, cell, ...); cfg->box, cfg->replica and the reaction's kappa are taken per replica
 * from reps[].  Each replica gets its own r_cut, cell grid and draws (keyed on its replica
 * number, local slots and own step), so its trajectory is the one sim_create would give for it
 * alone.  Afterwards the handle behaves like one system of
 * sum(n) slots: replica r owns slots [n_0 + ... + n_{r-1}, + n_r) in every read, and partner
 * indices in sim_read / sim_load_state are global.  SIM_READ_DERIVED and SIM_READ_GRID
 * describe replica 0; sim_eval_pairs, sim_eval_propagator, sim_eval_first_passage and sim_eval_angle use replica 0's
 * parameters (its exact 2D tables too).
 * pos of replica r holds n * dim values.  Errors as sim_create (reported for the first replica
 * that fails). */
int sim_batch_create(const sim_config *cfg, uint32_t n_rep, const sim_replica *reps, sim_t **out);

/* Continuous batching.  A pool is a batch created empty, with device memory for slot_cap
 * slots, cell_cap cells (over all members; a member takes its own cell grid, about one cell
 * per B, at most n) and rep_cap members.  Systems join it (sim_pool_admit) and leave it
 * (sim_pool_retire) between steps; each member owns a contiguous range of slots and of cells
 * while it is in, and every sim_step advances all members together (one graph replay per
 * step).  cfg supplies what the members share, as for sim_batch_create; cfg->box must be a
 * valid box for the configuration (it is checked like a system's and otherwise unused).
 * Returns SIM_EINVAL for capacities outside [1, 2^29) slots, [1, 2^28] cells or [1, 2^20]
 * members, SIM_ENOMEM if the device memory cannot be had, other errors as sim_create. */
int sim_pool_create(const sim_config *cfg, uint64_t slot_cap, uint64_t cell_cap, uint32_t rep_cap, sim_t **out);

/* Adds one system to the pool: rep as for sim_batch_create (species, positions, partners local
 * to it, box, kappa, replica number and its own step counter, all copied).  Its trajectory is
 * the one sim_create would give it alone from that state and step, whatever else is in the
 * pool and whenever it joins.  *member receives its entry, valid until it is retired.
 * SIM_ECAPACITY if no member entry, no contiguous range of rep->n slots or of its cells is free
 * (nothing changes then: retire members or wait); SIM_EINVAL for an invalid state or box;
 * SIM_ESTATE if h is not a pool; SIM_ENOMEM if the exact 2D tables of a new kappa (green2d =
 * SIM_G2_EXACT, built here before any slot is taken) cannot be allocated.  Synchronises the
 * pool's stream.  A pool's own sim_eval_pairs and sim_eval_propagator refuse the exact mode
 * (SIM_EUNSUPPORTED): its tables are its members'. */
int sim_pool_admit(sim_t *h, const sim_replica *rep, uint32_t *member);

/* Removes a member; its slots and cells are free for later admissions.  SIM_EINVAL if member
 * is not a current entry; SIM_ESTATE if h is not a pool.  Synchronises the pool's stream. */
int sim_pool_retire(sim_t *h, uint32_t member);

/* sim_read for one member: SIM_READ_POS, SIM_READ_SPECIES, SIM_READ_PARTNER (indices local to
 * the member) or SIM_READ_COUNTS, over its own slots in the layout it was admitted with.
 * SIM_EINVAL for another selector or an unknown member. */
int sim_pool_read(sim_t *h, uint32_t member, int what, void *dst, uint64_t cap_bytes, uint64_t *written);

/* Enqueues nsteps steps on the handle's stream and waits for them.  Without
 * debug or timing, each step is one replay of a captured HIP graph.  The
 * capacity flags are read back once at the end of the call, so SIM_ECAPACITY
 * reports an overflow of the per-step pair list in any of the steps. */
int sim_step(sim_t *h, uint32_t nsteps);

/* The same steps, enqueued on the handle's stream without waiting (Sec. 3: each step depends
 * only on the device state the previous one left, so no host round trip is needed between
 * steps).  The call returns once the graph replays are enqueued; host work, or work the
 * caller orders after them on the same stream (sim_config.stream), overlaps them.  Calls on
 * one handle are ordered by its stream.  SIM_EINVAL on a handle with debug logs or kernel
 * timing (they read back after every step).  A per-step buffer overflow is reported by the
 * next sim_sync or sim_step.  sim_read, sim_load_state and the pool calls wait for the stream
 * as they always do; sim_destroy waits for it before freeing. */
int sim_step_async(sim_t *h, uint32_t nsteps);

/* Waits for every step enqueued on the handle and reports SIM_ECAPACITY if any of them
 * overflowed a per-step buffer since the last sim_sync or sim_step. */
int sim_sync(sim_t *h);

/* What sim_read copies to the host buffer dst (cap_bytes long); *written gets
 * the number of bytes.  Reads synchronise the handle's stream. */
enum {
    SIM_READ_POS = 0,       /* double[n*dim], by slot; NaN for FREE/RESERVED */
    SIM_READ_SPECIES = 1,   /* int32[n], by slot */
    SIM_READ_PARTNER = 2,   /* uint32[n]: reserved slot of each C, else 0xFFFFFFFF */
    SIM_READ_COUNTS = 3,    /* int64[5]: number of A, B, C, FREE, RESERVED slots */
    SIM_READ_STATS = 4,     /* uint64[SIM_STAT_N]: counters of the last step */
    SIM_READ_STATS_SUM = 5, /* uint64[SIM_STAT_N]: counters summed since creation */
    SIM_READ_DERIVED = 6,   /* double[8]: D_eff, tau, h, r_cut, a, p_uni, cell edge, step */
    SIM_READ_DBG_MOVED = 7, /* double[n*dim]: positions after the move of the last step (debug) */
    SIM_READ_DBG_PAIRS = 8, /* sim_dbg_pair[]: every pair within r_cut of the last step (debug) */
    SIM_READ_DBG_PICKS = 9, /* sim_dbg_pick[]: the A-side choices (debug) */
    SIM_READ_DBG_MATCHES = 10, /* sim_dbg_match[] (debug) */
    SIM_READ_DBG_DISS = 11, /* sim_dbg_diss[] (debug) */
    SIM_READ_DBG_CELLS = 12,/* uint32[n]: sort key (species * n_cells + cell) of each live slot after binning, else 0xFFFFFFFF (debug) */
    SIM_READ_TIMING = 13,   /* sim_kernel_time[SIM_K_N]: accumulated kernel times (timing) */
    SIM_READ_GRID = 14,     /* int64[5]: cells per edge x, y, z, total cells, pair-search kernel (SIM_PAIRS_BRICKS or _DIRECT) */
    SIM_READ_DBG_DISP = 15  /* double[n*dim]: the displacement each live slot took in the move of the last step, as
                             * the step's later stages regenerate it (debug); NaN for FREE/RESERVED */
};

enum {
    SIM_STAT_PAIRS = 0, SIM_STAT_CAND, SIM_STAT_OVERLAP, SIM_STAT_R0CLAMP, SIM_STAT_PICKS,
    SIM_STAT_MATCHES, SIM_STAT_REACT, SIM_STAT_DECAY, SIM_STAT_GEMINATE, SIM_STAT_ATTEMPTS,
    SIM_STAT_BOUND, SIM_STAT_NEAR, SIM_STAT_LDS_FALLBACK, SIM_STAT_N
};

typedef struct { uint32_t i, j; double R, R0, p; uint32_t draw; int32_t cand; } sim_dbg_pair;
typedef struct { uint32_t i, j; double p; } sim_dbg_pick;
/* draw: the Philox word of the reaction test (TAG_REAC, word 0) of a matched pair, or of the
 * geminate test (TAG_GEM) of a decay; cos_theta: the cosine of the angle between the pair's
 * separations before and after a non-reactive propagation, NaN where none was drawn */
typedef struct { uint32_t i, j; int32_t reacted; uint32_t attempts, draw, pad; double Rpp, preac, cos_theta; } sim_dbg_match;
typedef struct { uint32_t c, j; int32_t decayed, recombined; uint32_t attempts, draw; double Rpp, preac; } sim_dbg_diss;

/* Kernels timed with sim_config.timing: move + bucket count, bucket scan,
 * scatter into sorted order, pair search, p_enc + draw per pair, A-side
 * choice, B-side choice + decay draws, matched pairs and decays (propagated
 * radius, reaction, dissociation), the angles of the propagated pairs (one
 * workgroup each; not run with SIM_F_KEEP_DIRECTION) and the one-workgroup step close. */
enum {
    SIM_K_MOVE = 0, SIM_K_SCAN, SIM_K_SCATTER, SIM_K_PAIRS, SIM_K_EVAL, SIM_K_SELECT_A, SIM_K_SELECT_B,
    SIM_K_EVENTS, SIM_K_ANGLES, SIM_K_N
};
typedef struct { double ms; uint64_t launches; } sim_kernel_time;

int sim_read(sim_t *h, int what, void *dst, uint64_t cap_bytes, uint64_t *written);

/* Replaces the state (same layout as sim_create) and sets the step counter;
 * n must equal the handle's slot count. */
int sim_load_state(sim_t *h, uint64_t step, const int32_t *species, const double *pos, const uint32_t *partner);

/* Evaluates p_enc = 1 - g_abs/g_free (Secs. 2.2.1 and 2.2.4, with the closed forms of Sec. 4.1
 * in 3D and the small-time expansion of Sec. 4.2 in 2D) and p_reac = (g_ref - g_rad)/(g_ref - g_abs)
 * (Sec. 2.2.3) for n caller-given pairs, with the step's own device functions and the handle's
 * dim, precision, boundary condition, tau, h and n_terms.  R[i] = r/a is the separation after
 * the move and R0[i] = r0/a >= 1 the one before it (a = sigma); for p_reac R[i] is the
 * propagated R'' >= 1.  R, R0, penc and preac are DEVICE pointers to n doubles owned by the
 * caller; penc or preac may be NULL to skip it.  p_enc is 1 for R <= 1 (overlap); p_reac is 1
 * for an absorbing and 0 for a reflecting surface.  Runs on the handle's stream and returns
 * when done.  SIM_EINVAL for NULL R, R0 or n = 0; SIM_EDEVICE if a HIP call fails. */
int sim_eval_pairs(sim_t *h, uint64_t n, const double *R, const double *R0, double *penc, double *preac);

/* For callers that cannot allocate device memory: code under HIP graph capture, serving loops
 * that may not call hipMalloc, harnesses that forbid it.  The same p_enc and p_reac as
 * sim_eval_pairs, bit for bit, for a system described by cfg instead of a handle (which
 * allocates when it is created): it validates cfg as sim_create does, enqueues the evaluation
 * on cfg->hip_stream (NULL: the null stream) and returns without waiting; the caller
 * synchronises that stream before reading penc and preac.  R, R0, penc, preac: DEVICE pointers,
 * as for sim_eval_pairs.  It allocates nothing: the one piece of device memory its kernel
 * needs beyond them, the constants of the 2D expansion (4 x 33 doubles, expansion orders up
 * to 32, the largest n_terms accepted), lives in a fixed array of the library that each GPU
 * holds for the life of the process; the entry point rewrites it on every 2D call.  Calls
 * that overlap on one GPU (on different streams, or from different threads) race on that
 * array; calls on one stream are ordered.  SIM_EINVAL for NULL R or R0, n = 0 or an invalid
 * cfg (n_terms above 32 among them); SIM_EUNSUPPORTED for green2d = SIM_G2_EXACT (its tables
 * are device memory a handle builds); SIM_EDEVICE if a HIP call fails. */
int sim_eval_pairs_noalloc(const sim_config *cfg, uint64_t n, const double *R, const double *R0, double *penc,
                           double *preac);

/* Draws n radii R'' >= 1 (in units of a) from the radial propagator w_d r^{d-1}(g_ref - g_abs)(.|R0)
 * (Sec. 2.2.2; 3D closed forms of Sec. 4.1, 2D expansion of Sec. 4.2) with the step's own rejection
 * sampler and the handle's parameters.  Draw i starts from R0[i] >= 1 and uses the Philox counter
 * {i, 0xFFFFFFFF, step, 5 | attempt << 8} with the handle's key.  wave != 0 spreads each draw's
 * attempts over a wave (the step's form for few events), wave = 0 takes one draw per lane (its
 * form for many); both give the same draws.  R0, Rpp (n doubles) and attempts (n uint32, may be
 * NULL) are DEVICE pointers owned by the caller.  Returns when done; SIM_EINVAL for NULL R0 or
 * Rpp, n = 0 or n > 2^32; SIM_EDEVICE if a HIP call fails. */
int sim_eval_propagator(sim_t *h, uint64_t n, const double *R0, uint32_t step, int wave, double *Rpp, uint32_t *attempts);

/* Locates the first contact of n pairs within one step by bisection (the paper's Appendix).
 * Pair i's separation vector went from xi[3i..3i+2] to xf[3i..3i+2] (units of a = sigma; a 2D
 * handle reads the first two components) over the
 * handle's dt (tau = D_eff dt / a^2), with at least one encounter in that step (a candidate of
 * the step is one).  Each of `levels` halvings draws the separation at the midpoint of the
 * interval from the Brownian bridge (eq. midPGauss: mean the end points' average, variance
 * tau_h per coordinate for the half interval tau_h), conditioned on the encounter known to lie
 * in the interval: a proposal is accepted with q = 1 - (1 - p1)(1 - p2), p1 and p2 the encounter
 * probabilities (Sec. 2.2.1 in the radial form of Sec. 2.2.4: the closed form of Sec. 4.1 in 3D,
 * the expansion of Sec. 4.2 in 2D, evaluated at each half interval's tau) of the two halves;
 * the first half is kept with probability p1 / q.  lo[i] receives the index of the final
 * interval: the first contact lies in [lo, lo + 1) * dt / 2^levels.  attempts[i] (may be NULL)
 * receives the midpoint proposals drawn (at most 4096 per level).  A level whose 4096 proposals
 * are all rejected (an interval whose encounter probability is far below 1/4096) ends the
 * refinement: lo[i] is then the lower end of the interval reached, at the requested resolution,
 * and bit 31 of attempts[i] is set.  Draws: Philox
 * {i, level, step, 11 | attempt << 8} (midpoint normals) and {i, level, step, 12 | attempt << 8}
 * (acceptance and choice) with the handle's key.  xi, xf (3n doubles), lo (n uint64) and
 * attempts (n uint32) are DEVICE pointers owned by the caller.  Runs on the handle's stream and
 * returns when done.  SIM_EINVAL for NULL xi, xf or lo, n = 0, n > 2^32 or levels outside
 * [1, 52]; SIM_EUNSUPPORTED for a 2D handle with the exact functions (green2d) or an expansion
 * order other than 12; SIM_EDEVICE if a HIP call fails. */
int sim_eval_first_passage(sim_t *h, uint64_t n, const double *xi, const double *xf, int32_t levels, uint32_t step,
                           uint64_t *lo, uint32_t *attempts);

/* Draws the angle of the propagated pair (Sec. 3, Details: after the radius, the angle between
 * the separations before and after the step comes from J (G_ref - G_abs), J = 2 pi sin(Theta) r^2
 * in 3D and r in 2D) for n pairs: out[i] is the root, at u[i], of the distribution function of
 * cos Theta (3D handles) or of |theta| in [0, pi] (2D handles) given the radii.  R[i] is the new
 * and R0[i] the old separation in units of a (values below 1 count as 1), tau = D_eff dt / a^2
 * the handle's; a pair with R + R0 - 2 > 40 sqrt(tau) (no encounter reaches that far) or a NaN
 * radius gets NaN.  G_ref - G_abs is the series of eq. genericGF3D (Legendre polynomials,
 * half-integer orders) or eq. genericGF with eq. fRad (cos n theta, integer orders), reflecting
 * minus absorbing surface, with terms n <= min(160, 8 + ceil(sqrt(45 R R0 / tau))); each
 * coefficient is an integral over x by 16-point Gauss-Legendre panels of width at most
 * min(1, 2 pi / (R + R0 - 1)) on [0, sqrt(40 / tau)] (2D: 12 panels of ratio 4 on [4^-12, 1]
 * first, where Y_0 has its logarithm), the Bessel functions by the three-term recurrences of
 * Sec. 4.1 (eq. 3termBessel).  The cap of 160 terms keeps the truncation below 1e-15 for
 * R R0 / tau <= 500.  The coefficients sum terms of the size of the free Green's function down
 * to the image term, so the distribution function is accurate to about
 * 1e-14 e^{(R+R0-2)^2 / 4 tau}: to 1e-10 where the radial propagator puts nearly all its draws
 * ((R+R0-2)^2 / 4 tau below 9), and not at all beyond about 36.  The azimuth (3D) or the side
 * (2D) is uniform and left to the caller.
 * R, R0, u and out (n doubles each) are DEVICE pointers owned by the caller; u in (0, 1).
 * Returns when done; SIM_EINVAL for a NULL pointer, n = 0 or n > 2^32; SIM_EUNSUPPORTED for a
 * handle with tau < 2e-3 (the series would need more than its 160 terms); SIM_EDEVICE if a HIP
 * call fails.  Uses replica 0's parameters. */
int sim_eval_angle(sim_t *h, uint64_t n, const double *R, const double *R0, const double *u, double *out);

/* Releases all device memory of the handle; NULL is accepted. */
int sim_destroy(sim_t *h);

/* Human-readable description of the last error on h (thread-local if h is NULL). */
const char *sim_last_error(const sim_t *h);

#ifdef __cplusplus
}
#endif
#endif
