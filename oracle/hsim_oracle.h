/*
 * CPU oracle of the Heisenberg Metropolis hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library; only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header or table with the GPU library.
 *
 * Plain serial C, double precision, compiled without floating-point
 * contraction (-ffp-contract=off) so that every product and sum is rounded
 * separately in the order written.
 *
 * Model (paper, section "Classical spin Hamiltonian", Eqs. 1-3):
 *   H = - sum_<ij> J_ij S_i.S_j - B sum_i S_i.n_i - sum_i k_i (S_i.e_i)^2
 *       - sum_i kc_i (Sx^2 Sy^2 + Sy^2 Sz^2 + Sx^2 Sz^2)_i
 * with every unordered bond counted once and the anisotropy entering Eq. 1 with
 * a minus sign (k > 0 is an easy axis).  Spin i has length norm_i (1 unless
 * given); trial moves act on its direction.
 * Dynamics (paper, section "Monte Carlo Metropolis algorithm", Eq. 4): a trial
 * direction uniform on the sphere is accepted when dE <= 0 or u < exp(-dE/T),
 * k_B = 1; one attempt per site makes one Monte Carlo step (MCS).  Sites are
 * visited colour class by colour class of a greedy colouring (breadth-first
 * order), ascending site index inside a class.  After every MCS the energy, the magnetisation vector
 * and the number of accepted moves are recorded.
 */
#ifndef HSIM_ORACLE_H
#define HSIM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Lattice in user order.  Spins are stored [i][3]. */
typedef struct {
    int64_t n;
    const int64_t *row_ptr;  /* n+1 */
    const int32_t *col;      /* nnz */
    const double *J;         /* nnz, symmetric */
    const double *k;         /* n, or NULL for k = 0 */
    const double *axis;      /* 3n, or NULL for +z */
    const double *ndir;      /* 3n, or NULL for +z */
    const double *kc;        /* n cubic anisotropy constants (Eq. 3), or NULL for 0 */
    const double *norm;      /* n spin norms, or NULL for unit spins */
} or_lattice;

enum { OR_PROPOSAL_EXACT = 0, OR_PROPOSAL_F32MAP = 1 };
/* Update policies (paper, section "Monte Carlo Metropolis algorithm" and the
 * feature list of section "VEGAS software package"; the moves of Hinzke and
 * Nowak 1999): the trial direction of a site. */
enum {
    OR_POLICY_RANDOM = 0,     /* uniform on the sphere, independent of S */
    OR_POLICY_FLIP = 1,       /* S' = -S */
    OR_POLICY_SMALL_STEP = 2, /* uniform in the cap of half-angle theta around S */
    OR_POLICY_GAUSSIAN = 3,   /* S' = (S + sigma g) / |S + sigma g|, g standard normal */
    OR_POLICY_HN = 4,         /* random, flip or small step, one third each */
    OR_POLICY_ADAPTIVE = 5    /* Gaussian with a per-replica sigma tuned toward 50% acceptance */
};
#define OR_MAX_TYPES 8
enum { OR_INIT_GIVEN = 0, OR_INIT_COLD_Z = 1, OR_INIT_RANDOM = 2 };

typedef struct {
    uint64_t seed;           /* Philox key */
    uint32_t replica;        /* third counter word */
    int32_t n_steps;         /* T/B steps in this call */
    int32_t mcs_per_step;
    int32_t first_step;      /* absolute index of the first step (resume) */
    int32_t recompute_every; /* P: E reset to the full sum at in-step MCS m with m % P == 0 (0: step start only) */
    const double *T;         /* n_steps temperatures (0 = greedy, +inf = beta 0) */
    const double *B;         /* n_steps field intensities */
    int32_t proposal;        /* OR_PROPOSAL_* */
    int32_t init;            /* OR_INIT_*, applied to spins before the first step */
    const int64_t *order;    /* NULL, or a permutation: visiting order inside each class */
    const int32_t *colour;   /* NULL (computed here) or a colouring to validate and use */
    int32_t check_every_update; /* O(n) full-energy check of every accepted move */
    /* update policies per site type; n_types == 0: the random move everywhere */
    int32_t n_types;
    const int32_t *site_type;   /* n, values in [0, n_types) (NULL: type 0) */
    const int32_t *type_policy; /* n_types, OR_POLICY_* */
    const double *type_param;   /* n_types: half-angle theta (radians) for SMALL_STEP and HN,
                                   sigma for GAUSSIAN, starting sigma for ADAPTIVE */
    double sigma_min, sigma_max;/* bounds of the adaptive width */
    double *sigma;              /* in/out: the adaptive width (used when a type is ADAPTIVE) */
    double *sigma_trace;        /* NULL or n_steps*mcs_per_step: width used in each MCS */
} or_params;

typedef struct {
    double *spins;           /* 3n in/out */
    double *history;         /* n_steps*mcs_per_step*5: E, Mx, My, Mz, n_acc */
    uint8_t *accept;         /* NULL or (n_steps*mcs_per_step)*n, user order */
    double *e_full;          /* NULL or n_steps*mcs_per_step: full energy after each MCS */
    int64_t near_ties;       /* decisions with |u - p| <= 4 ulp(p) */
    double max_incr_err;     /* max |E_incr - E_full| / scale over all MCS */
    double max_update_err;   /* max |dE - (E_after - E_before)| / scale */
    int64_t n_decisions;
    /* per-type magnetisation after every MCS (NULL: not recorded):
     * n_steps*mcs_per_step*n_types*3, sites grouped by p->site_type */
    double *type_mag;
    /* spins at the end of every step (NULL: not recorded): n_steps*n*3 */
    double *snapshots;
    /* every decision's energy change and acceptance uniform (NULL: not
     * recorded): (n_steps*mcs_per_step)*n each, user order; lets a caller
     * find how far each decision was from its tie u = exp(-beta dE) */
    double *dE_trace;
    double *u_trace;
} or_outputs;

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw, SC'11). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_philox_batch(int64_t count, const uint32_t *ctr /*4*count*/, const uint32_t *key /*2*/, uint32_t *out);
/* Uniform maps of the random words: 53-bit and 23-bit odd-grid values in (0,1). */
double or_u53(uint32_t hi, uint32_t lo);
double or_u24(uint32_t w);
/* Exact (Marsaglia 1972) sphere point from counters {site, g, rep, 1..}.  Returns attempts used. */
int or_sphere_exact(uint64_t seed, uint32_t site, uint32_t g, uint32_t rep, double out[3]);
/* Single-call proposal of the FP32 production mode, evaluated in double; u_out gets the acceptance uniform. */
void or_sphere_f32map(uint64_t seed, uint32_t site, uint32_t g, uint32_t rep, double out[3], double *u_out);

/* Natural logarithm by a fixed sequence of correctly rounded operations
 * (binary exponent split, then the atanh series), so that any implementation
 * of the same steps gives the same bits.  x > 0 finite. */
double or_log(double x);
/* Trial direction of one site under a policy (both proposal maps).  s: the
 * current spin; param: theta or sigma; cos_theta: cos(param) for the cap
 * moves.  Returns the acceptance uniform; out gets the trial. */
double or_trial(int32_t proposal, int32_t policy, uint64_t seed, uint32_t site, uint32_t g,
                uint32_t rep, const double s[3], double param, double cos_theta, double out[3]);

/* 0 if valid, else a negative code: -1 argument, -2 structure, -3 values. */
int or_validate(const or_lattice *lat);
/* Greedy colouring in breadth-first order (components by lowest site index,
 * neighbours in CSR order), smallest colour unused by a coloured neighbour.
 * Returns the number of colours. */
int or_greedy_colour(const or_lattice *lat, int32_t *colour);
/* Number of links whose two ends share a colour. */
int64_t or_count_conflicts(const or_lattice *lat, const int32_t *colour);

/* Energy pieces of Eq. 1 for one configuration. */
double or_energy(const or_lattice *lat, double B, const double *spins,
                 double *e_ex, double *e_zee, double *e_ani, double *scale);
/* Bonds i < j in row-major CSR order; returns their number. */
int64_t or_bonds(const or_lattice *lat, int32_t *bond_ij /* 2*nb or NULL */, double *J_bond /* nb or NULL */);
/* Gradient of g*E: gS (3n), gJ per bond, gk (n), gB (scalar), all added to. */
void or_energy_grad(const or_lattice *lat, double B, const double *spins, double g,
                    double *gS, double *gJ_bond, double *gk, double *gB);

/* Run the colour-ordered sweep.  Returns 0 or a negative code. */
int or_run(const or_lattice *lat, const or_params *p, or_outputs *out);

#ifdef __cplusplus
}
#endif
#endif
