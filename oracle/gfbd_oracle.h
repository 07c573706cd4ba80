/*
 * FP64 CPU oracle for the coarse-grained Green's-function Brownian-dynamics
 * step of T. Pruestel and M. Meier-Schellersheim, "Coarse-Grained Stochastic
 * Particle-based Reaction-Diffusion Simulation Algorithm" (arXiv:1107.0270).
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the reference that the HIP path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant with the HIP library, and it never reads anything the HIP library
 * produced.
 *
 * Everything is evaluated in IEEE binary64.  Lengths are in units of the
 * encounter radius a (R = r/a) and time in units of a^2/D_eff
 * (tau = D_eff t / a^2, Sec. 4.1), exactly as the paper scales them.
 */
#ifndef GFBD_ORACLE_H
#define GFBD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- counter-based generator: Philox4x32-10 (Salmon et al., SC'11) ---- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01(uint32_t x); /* (x + 1/2) 2^-32, in (0, 1) */

/* ---- special functions ---- */
double orc_erfcx(double x);                            /* e^{x^2} erfc(x) */
void orc_ierfcx(double x, int kmax, double *out);       /* out[k+1] = e^{x^2} i^k erfc(x), k=-1..kmax */
double orc_i0e(double x);                               /* e^{-|x|} I_0(x) */
double orc_erfc_tail_inv(double yc, double u);          /* y >= yc with erfc(y) = u erfc(yc) */
void orc_asym_coeffs(double nu, int n, double *a);      /* a_k(nu), k = 0..n (Sec. 4.2) */

/* ---- 3D radial Green's functions, times a^3 (Sec. 4.1) ---- */
double orc_g3_free(double R, double R0, double tau);
double orc_g3_abs(double R, double R0, double tau);
double orc_g3_rad(double R, double R0, double tau, double hh);   /* hh = 0: reflecting */
double orc_penc3(double R, double R0, double tau);
double orc_preac3(double R, double R0, double tau, double hh);
double orc_loss3_abs(double R0, double tau);              /* 1 - S_abs(tau | R0) */
double orc_loss3_rad(double R0, double tau, double hh);   /* 1 - S_rad(tau | R0) */
double orc_prop3_density(double Rp, double R0, double tau); /* w_3 r^2 (g_ref - g_abs), per dR */

/* ---- 2D small-time expansions (Sec. 4.2) ---- */
void orc_gamma2(double R, double R0, double hh, int n, double *g_abs, double *g_ref, double *g_rad);
double orc_g2_bc(int kind, double R, double R0, double tau, double hh, int n); /* times a^2 */
double orc_g2_free(double R, double R0, double tau);                           /* times a^2 */
double orc_penc2(double R, double R0, double tau, int n);
double orc_preac2(double R, double R0, double tau, double hh, int n);
double orc_prop2_density(double Rp, double R0, double tau, int n);

/* ---- exact 2D radial functions (n = 0 term of eq. genericGF, by quadrature) ---- */
void orc_g2x(double R, double R0, double tau, double hh, double out[3]); /* a^2 g_abs, g_ref, g_rad */
void orc_m2x(double R, double R0, double tau, double out[2]);             /* int_1^R 2 pi R' g dR': abs, ref */
double orc_penc2x(double R, double R0, double tau);
double orc_preac2x(double R, double R0, double tau, double hh);
double orc_sample_prop2x(double R0, double tau, double u);                /* inversion, one uniform */
double orc_x2_switch(double tau);  /* R0 above which the exact 2D mode takes p_enc, p_reac from the expansions */
double orc_x2_prop_switch(double tau);  /* R0 above which it draws R'' from the expansion's propagator */
/* ---- radial propagator sampler (Sec. 3, Details; Sec. 2.2.2) ---- */
/* Draws R'' >= 1 from w_d r^{d-1}(g_ref - g_abs)(.|R0) by keyed rejection.
 * ctr[3] low byte is the tag; the attempt index is put in its upper 24 bits. */
double orc_sample_prop(int dim, double R0, double tau, int n_terms, const uint32_t ctr[4],
                       const uint32_t key[2], uint32_t *attempts, uint32_t *bound_hits);

/* ---- cut-off radius from the survival probability (Sec. 3, Details) ---- */
double orc_rcut(int dim, int bc, double a, double Deff, double dt, double kappa_a, double eps);

/* ---- the simulation step (Sec. 3) ---- */
enum { ORC_SP_A = 0, ORC_SP_B = 1, ORC_SP_C = 2, ORC_SP_FREE = 3, ORC_SP_RESERVED = 4 };
enum { ORC_BC_ABS = 0, ORC_BC_REF = 1, ORC_BC_RAD = 2 };

typedef struct {
    int32_t dim;        /* 2 or 3 */
    int32_t bc;         /* ORC_BC_* */
    int32_t store_f32;  /* 1: the state holds positions in binary32 */
    int32_t n_terms;    /* order of the 2D small-time expansion */
    double box[3];      /* periodic box edges, um */
    double dt;          /* s */
    double D[3];        /* diffusion constants of A, B, C, um^2/s */
    double sigma;       /* encounter radius a, um */
    double kappa_a;     /* intrinsic rate: um^3/s (3D) or um^2/s (2D) */
    double k_off;       /* C -> A + B rate, 1/s; 0 = irreversible */
    double eps_cut;     /* 1 - S(dt | r_cut) */
    double rcut;        /* > 0: use this cut-off instead of deriving it */
    uint64_t seed;
    uint32_t replica;
    int32_t exact2d;    /* 2D: 1 = exact radial functions by quadrature, 0 = small-time expansions */
    int32_t keep_dir;   /* 1: a propagated pair keeps the direction of its free end point (no angle draw) */
} orc_params;

typedef struct { uint32_t i, j; double R, R0, p; uint32_t draw; int32_t cand; } orc_pair;
typedef struct { uint32_t i, j; double p; } orc_pick;
/* draw: the reaction (matches) or geminate (decays) test's Philox word; cos_theta: the cosine
 * of the angle between a propagated pair's separations before and after, NaN if none drawn */
typedef struct { uint32_t i, j; int32_t reacted; uint32_t attempts, draw, pad; double Rpp, preac, cos_theta; } orc_match;
typedef struct { uint32_t c, j; int32_t decayed, recombined; uint32_t attempts, draw; double Rpp, preac; } orc_diss;

enum {
    ORC_ST_PAIRS = 0, ORC_ST_CAND, ORC_ST_OVERLAP, ORC_ST_R0CLAMP, ORC_ST_PICKS, ORC_ST_MATCHES,
    ORC_ST_REACT, ORC_ST_DECAY, ORC_ST_GEMINATE, ORC_ST_ATTEMPTS, ORC_ST_BOUND, ORC_ST_N
};

/* First-passage time by bisection (Appendix): the index lo of the interval
 * [lo, lo + 1) * dt / 2^levels that holds the first contact of a pair whose
 * separation (units of a) went from xi to xf over tau = D_eff dt / a^2 with at
 * least one encounter; dim 1 (half line x > 1), 2 or 3.  *attempts: midpoint
 * proposals drawn, bit 31 set if a level exhausted its proposals (the
 * refinement then stops at that level's interval). */
uint64_t orc_first_passage(int dim, const double *xi, const double *xf, double tau, int levels, int n_terms,
                           uint32_t c0, uint32_t step, const uint32_t key[2], uint32_t *attempts);

/* Angular propagator in 3D (Sec. 3, Details; eq. genericGF3D): the number of
 * Legendre terms, the half-integer Bessel functions J[k] = J_{k-1/2}(z),
 * Y[k] = Y_{k-1/2}(z) (k = 0 .. kmax), the coefficients w[0..N] of
 * G_ref - G_abs (kind 0) or of the free Green's function (kind 1), the
 * conditional distribution function of cos Theta given R, and one draw of
 * cos Theta by its inverse at u. */
int orc_angle3_terms(double R, double R0, double tau);
void orc_bessel_half(int kmax, double z, double *J, double *Y);
void orc_angle3_coef(int kind, double R, double R0, double tau, int N, double *w);
double orc_angle3_cdf(const double *w, int N, double c);
double orc_sample_angle3(double R, double R0, double tau, double u);

/* Angular propagator in 2D (Sec. 3, Details; eq. genericGF): integer-order
 * Bessel functions J[k] = J_{k-1}(z), Y[k] = Y_{k-1}(z), the coefficients
 * w[0..N] of G_ref - G_abs (kind 0) or of the free Green's function (kind 1),
 * the distribution function of |theta| in [0, pi] given R, and one draw. */
void orc_bessel_int(int kmax, double z, double *J, double *Y);
void orc_angle2_coef(int kind, double R, double R0, double tau, int N, double *w);
double orc_angle2_cdf(const double *w, int N, double t);
double orc_sample_angle2(double R, double R0, double tau, double u);

typedef struct orc_sim orc_sim;

orc_sim *orc_sim_create(const orc_params *p, uint64_t n, const int32_t *species, const double *pos,
                        const uint32_t *partner);
void orc_sim_destroy(orc_sim *s);
void orc_sim_step(orc_sim *s);
uint64_t orc_sim_cap(const orc_sim *s);
uint64_t orc_sim_stepno(const orc_sim *s);
void orc_sim_derived(const orc_sim *s, double out[6]); /* Deff, tau, hh, rcut, a, p_uni */
void orc_sim_state(const orc_sim *s, int32_t *species, double *pos, uint32_t *partner);
void orc_sim_moved(const orc_sim *s, double *pos_after_move);
void orc_sim_set_moved(orc_sim *s, const double *pos, const double *disp);
void orc_sim_moved_own(const orc_sim *s, double *pos);
void orc_sim_stats(const orc_sim *s, uint64_t out[ORC_ST_N]);
uint64_t orc_sim_n_pairs(const orc_sim *s);
uint64_t orc_sim_n_picks(const orc_sim *s);
uint64_t orc_sim_n_matches(const orc_sim *s);
uint64_t orc_sim_n_diss(const orc_sim *s);
void orc_sim_pairs(const orc_sim *s, orc_pair *out);
void orc_sim_picks(const orc_sim *s, orc_pick *out);
void orc_sim_matches(const orc_sim *s, orc_match *out);
void orc_sim_diss(const orc_sim *s, orc_diss *out);

#ifdef __cplusplus
}
#endif
#endif
