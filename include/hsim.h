/*
 * hsim — Metropolis Monte Carlo of the classical Heisenberg model on MI355X
 * (gfx950).  C-ABI of libhsim.so.
 *
 * Model (paper, section "Classical spin Hamiltonian", Eqs. 1-2), k_B = 1:
 *   E(S) = - sum_<ij> J_ij S_i.S_j  - B sum_i S_i.n_i  - sum_i k_i (S_i.e_i)^2
 * every unordered bond <ij> counted once; k_i > 0 is an easy axis e_i; the
 * field has one intensity B per temperature/field step and a fixed unit
 * direction n_i per site.
 * Dynamics (paper, section "Monte Carlo Metropolis algorithm", Eq. 4): a trial
 * direction uniform on the sphere, accepted when dE <= 0 or u < exp(-dE/T).
 * One attempt per site is one Monte Carlo step (MCS).  Sites are updated one
 * colour class of a greedy breadth-first colouring at a time (all sites of a
 * class in parallel), classes in ascending order.
 * Output (paper, section "VEGAS software package"): after every MCS of every
 * temperature/field step, the energy, the magnetisation vector and the number
 * of accepted moves of every replica, in double precision.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = 64-bit batch
 * seed (low word first), counter = {user site index, g, replica id, attempt}
 * with g = step * mcs_per_step + m (absolute step index).  A run therefore
 * does not depend on the internal site order, the layout, the launch mode or
 * on how a schedule is split into resumed runs.
 *
 * Conventions of every call:
 *  - Every function returns hsim_status: HSIM_OK (0) or a negative code; on
 *    failure hsim_last_error() gives a message (thread-local).  No C++
 *    exception crosses this interface.
 *  - Host arrays are read during the call and not retained.
 *  - Device buffers passed in (workspace, spins, history, traces, energy
 *    inputs and gradients) are owned by the caller, must stay allocated until
 *    the work queued on the given stream has finished, and are never freed by
 *    the library.  Plans and batches own their own device tables until
 *    destroyed.
 *  - Calls that take a hipStream_t only enqueue work and return.
 *  - Spin arrays at this interface are in user order, double precision, [i][3].
 */
#ifndef HSIM_H
#define HSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hsim_status;
#define HSIM_OK 0
#define HSIM_E_ARG (-1)          /* null pointer, bad size or bad enum */
#define HSIM_E_CSR (-2)          /* asymmetric, self loop, duplicate or out-of-range CSR */
#define HSIM_E_PARAM (-3)        /* non-finite value, axis norm off by > 1e-9, T < 0 */
#define HSIM_E_STATE (-4)        /* call order: e.g. run before bind */
#define HSIM_E_DEVICE (-5)       /* HIP runtime error (message in hsim_last_error) */
#define HSIM_E_UNSUPPORTED (-6)  /* combination not provided (e.g. FP64 in the replica layout) */
#define HSIM_E_TIMEOUT (-7)      /* a device barrier wait reached its cap */
#define HSIM_E_NUMERIC (-8)      /* NaN energy change seen on the device */

typedef struct hsim_plan_s *hsim_plan;   /* one lattice; opaque */
typedef struct hsim_batch_s *hsim_batch; /* replicas over one or more plans; opaque */

typedef enum { HSIM_FP32 = 0, HSIM_FP64_EXACT = 1 } hsim_precision;

/* Spin layouts.  SITE: one lane per site of one replica, spins [3][n] per
 * replica.  REPLICA: replicas sharing one lattice, one lane per replica of
 * one site, spins [n][3][R padded to 32 or a multiple of 64] (rows of all
 * replicas for one component of one site; [3][n][..] when the array is 2 GiB
 * or more); FP32 only.  BLOCK: each replica owned by one workgroup for the
 * whole run (spins staged in LDS when they fit).  AUTO: REPLICA for FP32
 * batches of at least 16 replicas on one lattice, else BLOCK when a replica
 * fits in LDS, else SITE. */
typedef enum {
    HSIM_LAYOUT_AUTO = 0, HSIM_LAYOUT_SITE = 1, HSIM_LAYOUT_REPLICA = 2, HSIM_LAYOUT_BLOCK = 3
} hsim_layout;

/* PLAIN: kernels enqueued one by one.  GRAPH: the same kernels captured once
 * into a hipGraph and replayed.  PERSISTENT: one launch that loops over MCS
 * and colours with device-wide barriers (replica layout).  AUTO: the mode
 * hsim_autotune chose for the batch, GRAPH before any autotuning.  The BLOCK
 * layout always runs as one launch.  Every mode gives the same spins, and
 * the same history within one layout. */
typedef enum {
    HSIM_LAUNCH_PLAIN = 0, HSIM_LAUNCH_PERSISTENT = 1, HSIM_LAUNCH_GRAPH = 2, HSIM_LAUNCH_AUTO = 3
} hsim_launch;

enum { HSIM_INIT_GIVEN = 0, HSIM_INIT_COLD_Z = 1, HSIM_INIT_RANDOM = 2 };

/* run_flags */
#define HSIM_RUN_TRACE_ACCEPTS 0x1u   /* write the accept bitmap to d_trace */
/* Failure-path checks (for tests of error handling; the run's results are
 * meaningless and every kernel still exits normally):
 *   DEBUG_NAN_FIELD: the run's field intensities are staged as NaN, so every
 *     energy change is NaN and the device reports HSIM_E_NUMERIC through
 *     hsim_batch_status;
 *   DEBUG_WAIT_CAP: persistent launches bound every device barrier wait by a
 *     single polling round, so a wait gives up, releases every later wait and
 *     hsim_batch_status reports HSIM_E_TIMEOUT. */
#define HSIM_RUN_DEBUG_NAN_FIELD 0x2u
#define HSIM_RUN_DEBUG_WAIT_CAP 0x4u

/* ------------------------------------------------------------------ plans */
/* Ingest one lattice (paper, section "Material building": sites, exchange
 * links with their constants, a field axis per site; anisotropy file: a
 * constant and an axis per site).
 *   n_sites >= 0 (a lattice without sites is allowed: its replicas record
 *     zero energy, magnetisation and acceptance);
 *   row_ptr [n+1] int64, col [nnz] int32: both directions of every link,
 *     J [nnz]: the constant of each entry; J must be symmetric.
 *   k [n] (NULL: 0), axis [3n] unit (NULL: +z), field_dir [3n] unit (NULL: +z).
 * Validates (HSIM_E_CSR / HSIM_E_PARAM), colours the graph greedily in
 * breadth-first order (components by lowest site index, neighbours in CSR
 * order, smallest colour unused by a coloured neighbour), sorts sites by
 * (colour, user index) and keeps every row's CSR entry order.  Host work
 * only; device tables are uploaded on first use.  flags: reserved, pass 0. */
hsim_status hsim_plan_create(hsim_plan *out, int64_t n_sites, const int64_t *row_ptr,
                             const int32_t *col, const double *J, const double *k,
                             const double *axis, const double *field_dir, uint32_t flags);

typedef struct {
    int64_t n_sites, nnz, n_bonds;
    int32_t n_colours;
    int32_t max_degree;
    int64_t colour_size[64];  /* sizes of the first 64 classes */
    double mean_degree;
    int32_t uniform_anisotropy; /* 1 if k and axis are the same at every site */
    int32_t uniform_field_dir;  /* 1 if n is the same at every site */
} hsim_plan_info_t;

hsim_status hsim_plan_info(hsim_plan plan, hsim_plan_info_t *out);
/* Colour of every site, user order [n]. */
hsim_status hsim_plan_colouring(hsim_plan plan, int32_t *colour_out);
/* Bonds i < j in row-major CSR order (the order of every per-bond array):
 * bond_ij_out [2*n_bonds] (may be NULL), *n_bonds_out (may be NULL). */
hsim_status hsim_plan_bonds(hsim_plan plan, int32_t *bond_ij_out, int64_t *n_bonds_out);
/* Half rows of the energy forward (Eq. 1 counts every bond once): each bond
 * is given to the one of its ends that a closed-walk (Euler) orientation
 * makes it leave, so a site of degree d holds at most ceil(d/2) bonds.
 * *width_out: slots per site (half the padded row width; 0 when a site's
 * degree exceeds 8 and the energy calls walk the CSR instead).
 * col_out, bond_out [width][n] slot-major, user order, host memory (may be
 * NULL): the far end and the bond id of each bond the site holds, in CSR
 * order; empty slots name the site itself with bond id -1. */
hsim_status hsim_plan_half_rows(hsim_plan plan, int32_t *width_out, int32_t *col_out,
                                int32_t *bond_out);
/* Site types (paper, section "Material building": every site belongs to a
 * magnetic phase, and each phase may use its own update policy).
 *   site_type [n] user order, values 0..7; NULL: type 0 everywhere.
 * Set the types before creating the batches that use the plan; a batch
 * picks them up at its next hsim_batch_bind or hsim_batch_set_policies.
 * HSIM_E_PARAM for a value outside 0..7. */
hsim_status hsim_plan_set_types(hsim_plan plan, const int32_t *site_type);
/* Per-site terms beyond Eqs. 1-2 (paper, Eq. 3 and the spin norm of the
 * material file, section "Material building"):
 *   k_cubic [n] user order (NULL: 0): cubic anisotropy, entering the energy
 *     as -k_cubic (Sx^2 Sy^2 + Sy^2 Sz^2 + Sx^2 Sz^2) (the same sign
 *     convention as the uniaxial term);
 *   spin_norm [n] user order (NULL: 1): the length of each spin.  Cold and
 *     random starts get the length; trial moves change the direction only.
 * Also counted by hsim_energy_forward / hsim_energy_backward (dE/dS includes
 * the cubic term).  Set before hsim_batch_bind.  With either term, PERSISTENT
 * launches run as PLAIN launches.  HSIM_E_PARAM for a non-finite constant or
 * a norm that is not positive and finite. */
hsim_status hsim_plan_set_site_terms(hsim_plan plan, const double *k_cubic,
                                     const double *spin_norm);
void hsim_plan_destroy(hsim_plan plan);

/* ---------------------------------------------------------------- batches */
/* n_rep replicas; replica r runs on lattice plan_of_rep[r] and draws its
 * random words with counter word 2 = replica_id[r] (NULL: r).  Plans must
 * outlive the batch. */
hsim_status hsim_batch_create(hsim_batch *out, int32_t n_rep, const hsim_plan *plan_of_rep,
                              uint64_t seed, const uint32_t *replica_id,
                              hsim_precision precision, hsim_layout layout);

typedef struct {
    int32_t layout;           /* resolved hsim_layout */
    int32_t n_rep, n_phases;  /* replicas, colour phases per MCS (max over lattices) */
    int64_t total_sites;      /* sum of lattice sizes over replicas */
    int32_t lds_resident;     /* BLOCK layout: spins held in LDS */
    int32_t reserved;
    /* REPLICA layout: sites per wave of a tile (4, 8 or 32) and the store
     * policy (0: every live lane writes its row back, 1: accepted moves
     * only); the launch mode and persistent grid AUTO uses (-1 / 0: not
     * tuned). */
    int32_t sites_per_wave, masked_store, tuned_launch, persistent_grid;
} hsim_batch_info_t;
hsim_status hsim_batch_info(hsim_batch b, hsim_batch_info_t *out);

/* The replica layout's tile shape and store policy, the knobs hsim_autotune
 * chooses, set by hand: sites_per_wave 4, 8 or 32 (HSIM_E_ARG otherwise),
 * masked_store 0 or 1.  Neither changes any spin: every site's update is
 * the same computation; the history's sums are grouped by tiles, so their
 * last bits may differ.  HSIM_E_UNSUPPORTED outside the replica layout.  May
 * be called while bound (the workspace covers every shape); a new shape
 * waits for the device before it replaces the tile order table. */
hsim_status hsim_batch_set_shape(hsim_batch b, int32_t sites_per_wave, int32_t masked_store);
/* The replica layout's dispatch order of each colour's tiles inside an
 * XCD's range (section "Monte Carlo Metropolis algorithm": the order of the
 * updates inside a colour class is free).  plane_sites > 1: tiles are
 * started in order of (tile mod p, tile / p), p = plane_sites / tile sites,
 * so that tiles one plane of the class apart, which read the same neighbour
 * rows, run together; 0: in order; -1 (the default): plane_sites derived
 * from the lattice's neighbour offsets and used only when a colour has more
 * tiles per XCD than the XCD runs at once.  Changes no result, spins or
 * history (records are kept per tile).  HSIM_E_ARG for 1 or below -1,
 * HSIM_E_UNSUPPORTED outside the replica layout.  On a bound batch it waits
 * for the device before it replaces the order table (as hsim_batch_set_shape
 * does when the shape changes). */
hsim_status hsim_batch_set_order(hsim_batch b, int32_t plane_sites);

/* Device bytes the caller must provide for a history of n_steps steps of
 * mcs_per_step MCS.  History layout: double [n_rep][n_steps][mcs_per_step][5]
 * = {E, Mx, My, Mz, accepted}.  Spins: the internal layout of the batch. */
hsim_status hsim_batch_sizes(hsim_batch b, int32_t n_steps, int32_t mcs_per_step,
                             size_t *workspace_bytes, size_t *spin_bytes,
                             size_t *history_bytes);
/* Attach caller-owned device buffers (sizes from hsim_batch_sizes, at least
 * 16-byte aligned, else HSIM_E_ARG).  Must precede init/run; may be called
 * again to re-attach (this clears the device status and resets the adaptive
 * widths). */
hsim_status hsim_batch_bind(hsim_batch b, int32_t n_steps, int32_t mcs_per_step,
                            void *d_workspace, void *d_spins, void *d_history);
/* Initial state (paper, section "File Formats": initial-state file).
 * GIVEN: host_spins [n_rep][n_r][3] user order, concatenated over replicas;
 * COLD_Z: all +z; RANDOM: exact sphere point from counter
 * {site, 0xFFFFFFFF, replica id, 1..} (the same map as the FP64 trial move),
 * rounded to single precision in FP32 mode. */
hsim_status hsim_batch_init_spins(hsim_batch b, int32_t mode, const double *host_spins,
                                  void *stream);
/* Run steps [first_step, first_step + n_steps) of the bound history.
 *   T, B: host arrays [n_rep][n_steps] (temperature >= 0, +inf allowed; field
 *     intensity); copied before return.
 *   recompute_every P: the energy carried between MCS is reset to a double
 *     precision full sum at every in-step MCS m with m % P == 0 (0: only at
 *     step start).
 *   d_trace: NULL, or with HSIM_RUN_TRACE_ACCEPTS a zeroed uint32 bitmap
 *     [n_rep][n_steps*mcs_per_step][ceil(n/32)] receiving bit (site % 32) of
 *     word site/32 for every accepted move (site = user index; every layout,
 *     in the replica layout only without update policies, cubic terms or
 *     spin norms: HSIM_E_UNSUPPORTED otherwise; a traced persistent request
 *     runs as plain launches).
 * Spins carry over between steps and between calls. */
hsim_status hsim_batch_run(hsim_batch b, int32_t first_step, int32_t n_steps, const double *T,
                           const double *B, int32_t recompute_every, hsim_launch launch,
                           uint32_t run_flags, uint32_t *d_trace, void *stream);
/* Update policies (paper, section "Monte Carlo Metropolis algorithm" and the
 * feature list: random, spin flip, small step, Gaussian and the adaptive
 * move, one policy per magnetic phase), one per site type:
 *   policy [n_types]: HSIM_POLICY_*; param [n_types]: the cap half-angle in
 *     radians, (0, pi], for SMALL_STEP and HN; the width sigma > 0 for
 *     GAUSSIAN; the starting width for ADAPTIVE (the first adaptive type's
 *     value; all adaptive types of a replica share one width).
 *   sigma_min, sigma_max: bounds of the adaptive width (0 < min <= max).
 * The adaptive width of a replica is scaled after every MCS by
 * 0.5 / (1 - a), a the acceptance of its adaptive sites in that MCS, then
 * clamped to the bounds; it carries over between runs and is reset to the
 * starting value by this call and by hsim_batch_bind.  n_types = 0 restores
 * the random move everywhere.  Every site type of the batch's plans must be
 * below n_types (HSIM_E_PARAM).  With policies set, PERSISTENT launches run
 * as PLAIN launches. */
enum {
    HSIM_POLICY_RANDOM = 0, HSIM_POLICY_FLIP = 1, HSIM_POLICY_SMALL_STEP = 2,
    HSIM_POLICY_GAUSSIAN = 3, HSIM_POLICY_HN = 4, HSIM_POLICY_ADAPTIVE = 5
};
hsim_status hsim_batch_set_policies(hsim_batch b, int32_t n_types, const int32_t *policy,
                                    const double *param, double sigma_min, double sigma_max);
/* Optional outputs of later runs (paper, feature list of section "VEGAS
 * software package": the statistics of each magnetic phase, and the final
 * state of every temperature/field step), caller-owned device buffers:
 *   d_type_mag: NULL, or double [n_rep][n_steps][mcs][n_types][3] of the
 *     bound history's shape: the magnetisation of every site type
 *     (hsim_plan_set_types; all sites type 0 without it) after every MCS;
 *     every site type must be below n_types (1..8);
 *   d_snapshots: NULL, or double [n_rep][n_steps][n_max][3], n_max the
 *     largest lattice of the batch: every replica's spins in user order at
 *     the end of every step.
 * The library keeps a small scratch for the per-type sums.  With outputs
 * bound, PERSISTENT launches run as PLAIN launches. */
hsim_status hsim_batch_bind_outputs(hsim_batch b, int32_t n_types, double *d_type_mag,
                                    double *d_snapshots);
/* Current adaptive width of every replica, host double [n_rep] (synchronous;
 * the batch must be bound). */
hsim_status hsim_batch_sigma(hsim_batch b, double *sigma_out);
/* Launch timing of the colour phases (the dominant kernels).  With every > 0,
 * plain-launch runs record a HIP event pair around each colour-phase launch
 * of every `every`-th MCS, on the run's stream; 0 switches it off.  GRAPH
 * and AUTO runs of a batch with timing on are enqueued as plain launches. */
hsim_status hsim_batch_time_phases(hsim_batch b, int32_t every);
/* Waits for the recorded events and returns their total: summed launch
 * duration in ms, number of timed launches, and attempted spin updates those
 * launches processed; then clears the record. */
hsim_status hsim_batch_phase_times(hsim_batch b, double *total_ms, int64_t *launches,
                                   int64_t *updates);
/* Replica rep's spins in user order, double [n][3], into device memory
 * (nothing is written for a lattice without sites; d_out may then be NULL). */
hsim_status hsim_batch_spins_to_user(hsim_batch b, int32_t rep, double *d_out, void *stream);
/* Device status word after the stream has been synchronised: 0, or
 * HSIM_E_NUMERIC / HSIM_E_TIMEOUT.  Clears it. */
hsim_status hsim_batch_status(hsim_batch b, int32_t *device_status_out);
/* Time the choices available for this batch on one step of trial_mcs MCS
 * at each replica's first bound temperature and field and keep the fastest
 * for HSIM_LAUNCH_AUTO.  In the replica layout first the tile shape (4, 8 or
 * 32 sites per wave) and the store policy with plain launches, then, for
 * that shape, graph launches and persistent grids of 1, 2, 4 and 8 blocks
 * per CU; in the site layout plain and graph launches.  A choice replaces
 * the current one only when it is more than 2% faster.  The trials use scratch
 * buffers the call allocates and frees; afterwards the batch's spins,
 * binding, adaptive widths, optional outputs, phase timing and device status
 * are as before the call.  Synchronises the stream.  The choice never
 * changes spin trajectories (see hsim_batch_set_shape for the history).
 * The block layout has nothing to choose (the call returns at once).  With
 * cache_path (NULL: no file) a choice recorded for the same GPU, ROCm
 * runtime and driver versions, layout, replica count, precision, update
 * policies and lattice (a hash of its rows, constants, axes and field
 * directions) is reused; a new choice is appended to the file. */
hsim_status hsim_autotune(hsim_batch b, const char *cache_path, int32_t trial_mcs,
                          void *stream);
/* The spin layout for a batch that hsim_batch_create would build from these
 * arguments, chosen by timing the MCS (section "Monte Carlo Metropolis
 * algorithm") in each candidate layout: every layout the batch
 * can use (SITE; REPLICA for FP32 batches on one shared lattice; BLOCK when
 * a replica's spins fit in LDS, or when it is the static choice) runs as a
 * fresh batch of its own, one warm-up step and one timed step of trial_mcs
 * MCS from a cold start, with the launch mode HSIM_LAUNCH_AUTO gives a batch
 * that was not tuned.  T, B: host arrays [n_rep], the temperature (>= 0,
 * +inf allowed) and field intensity of each replica.  *layout_out receives
 * the static HSIM_LAYOUT_AUTO choice unless another layout was more than 2%
 * faster.  Layouts give the same spins (the history can differ in rounding),
 * so the choice only changes speed.  Allocates and frees its scratch batches
 * and buffers and synchronises the stream; HSIM_E_ARG for a bad argument,
 * HSIM_E_PARAM for a negative or NaN temperature or a non-finite field. */
hsim_status hsim_choose_layout(int32_t n_rep, const hsim_plan *plan_of_rep, uint64_t seed,
                               const uint32_t *replica_id, hsim_precision precision, const double *T,
                               const double *B, int32_t trial_mcs, int32_t *layout_out, void *stream);
void hsim_batch_destroy(hsim_batch b);

/* ------------------------------------------------- energy and its gradient */
/* Uploads the plan's energy tables (user-order rows, padded to 6 or 8 slots
 * when every row fits) and allocates its fixed energy scratch: the partial
 * records of one pass of up to 2048 configurations, at most about 128 MiB
 * (more only when a single group of 32 configurations needs it).
 * Synchronous and allocating; idempotent.  An energy call on a plan that was
 * not prepared does this first; after it, energy calls only enqueue work,
 * allocate nothing and may be captured in graphs.  Batches larger than a
 * pass run as several passes over the same scratch. */
hsim_status hsim_energy_prepare(hsim_plan plan);
/* Eq. 1 for `batch` configurations of one lattice, precision HSIM_FP32
 * (float inputs, double accumulation) or HSIM_FP64_EXACT (double inputs).
 *   d_spins [batch][3][n] user order; d_J_bond [n_bonds] in hsim_plan_bonds
 *   order; d_k [n]; d_axis [3][n]; B scalar; d_field_dir [3][n] (NULL: +z).
 *   d_E [batch] double receives the energies. */
hsim_status hsim_energy_forward(hsim_plan plan, int32_t batch, hsim_precision precision,
                                const void *d_spins, const void *d_J_bond, const void *d_k,
                                const void *d_axis, double B, const void *d_field_dir,
                                double *d_E, void *stream);
/* For callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * hsim_energy_forward with the same arguments and results, whose partial
 * records live in a fixed array the library keeps on each GPU (8 MiB per
 * device, held until the process ends) instead of the plan's scratch.  It
 * calls no allocating routine.  The plan must have been prepared
 * (hsim_energy_prepare, HSIM_E_STATE otherwise); lattices of more than
 * 8,388,608 sites are rejected with HSIM_E_ARG.  Batches of any size run in
 * passes over the array.  Every call on one GPU shares that array: calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * ordered by the caller. */
hsim_status hsim_energy_forward_noalloc(hsim_plan plan, int32_t batch, hsim_precision precision,
                                        const void *d_spins, const void *d_J_bond,
                                        const void *d_k, const void *d_axis, double B,
                                        const void *d_field_dir, double *d_E, void *stream);
/* Vector-Jacobian product of the energies with upstream d_gE [batch]:
 *   d_gS [batch][3][n]   = gE_b (-sum_j J_ij S_j - B n_i - 2 k_i (S_i.e_i) e_i)
 *   d_gJ_bond [n_bonds]  = sum_b gE_b (-S_i.S_j)
 *   d_gk [n]             = sum_b gE_b (-(S_i.e_i)^2)
 *   d_gB [1] (double)    = sum_b gE_b (-sum_i S_i.n_i)
 * Any output may be NULL.  Outputs are overwritten (not accumulated); gS, gJ
 * and gk have the precision of the inputs.  With the cubic term of
 * hsim_plan_set_site_terms, dE/dS includes it.
 * Both energy calls use the plan's fixed device scratch (hsim_energy_prepare);
 * two energy calls on one plan must not run concurrently on different
 * streams. */
hsim_status hsim_energy_backward(hsim_plan plan, int32_t batch, hsim_precision precision,
                                 const void *d_spins, const void *d_J_bond, const void *d_k,
                                 const void *d_axis, double B, const void *d_field_dir,
                                 const double *d_gE, void *d_gS, void *d_gJ_bond, void *d_gk,
                                 double *d_gB, void *stream);
/* Fluctuation estimate of d<O>/d(theta) from n samples of the equilibrium
 * chain at inverse temperature beta:
 *   d<O>/dtheta = <dO/dtheta> - beta (<O dE/dtheta> - <O><dE/dtheta>)
 * d_O, d_dE [n] double, d_dO [n] double or NULL (0); d_out [2] double receives
 * the estimate and the covariance term. */
hsim_status hsim_fluct_estimate(int64_t n, double beta, const double *d_O, const double *d_dE,
                                const double *d_dO, double *d_out, void *stream);

/* Upstream weights that turn one hsim_energy_backward call into the
 * fluctuation estimate of the derivatives of a thermal average with respect
 * to every per-bond constant, every anisotropy constant and the field
 * intensity at once (paper, section "Thermal averages": response functions
 * as fluctuations of the equilibrium chain):
 *   d<O>/dtheta = <dO/dtheta> - beta (<O dE/dtheta> - <O><dE/dtheta>)
 *              = sum_k w_k dE_k/dtheta,   w_k = (c - beta (O_k - <O>)) / n
 * for samples k = 0..n-1 drawn at inverse temperature beta, with c = 1 when
 * O is the energy itself (its own derivative is dE/dtheta) and c = 0 when O
 * does not depend on the parameters (e.g. a magnetisation).
 *   d_O [n] double (device): the observable of each sample;
 *   d_w [n] double (device): receives the weights (may not alias d_O).
 * The mean <O> is summed in a fixed order.  HSIM_E_ARG for n < 1 or NULL
 * buffers, HSIM_E_PARAM for a negative or non-finite beta or non-finite c. */
hsim_status hsim_fluct_weights(int64_t n, double beta, const double *d_O, double c, double *d_w,
                               void *stream);
/* Layout conversion for the energy calls: site-major double spins
 * d_in [n_cfg][n_sites][3] (the layout of hsim_batch_spins_to_user and of
 * the step-end snapshots) into d_out [n_cfg][3][n_sites] of the given
 * precision (float for HSIM_FP32, rounded to nearest; double for
 * HSIM_FP64_EXACT), both device memory, caller-owned. */
hsim_status hsim_spins_planar(int64_t n_cfg, int64_t n_sites, const double *d_in,
                              hsim_precision precision, void *d_out, void *stream);

/* ------------------------------------------------- analysis of the history */
/* A series is the history of one replica at one step, MCS m0 .. mcs-1 of a
 * history d_history [n_rep][n_steps][mcs][5] (device, as written by
 * hsim_batch_run).  Results are per site (k_B = 1), with |M| the length of
 * the magnetisation vector and <.> the (weighted) mean over the series:
 *   [0] e = <E>/N            [1] m_abs = <|M|>/N     [2] m2 = <|M|^2>/N^2
 *   [3] m4 = <|M|^4>/N^4     [4] cv = beta^2 <(E-<E>)^2>/N
 *   [5] chi = beta <(|M|-<|M|>)^2>/N                 [6] u4 = 1 - m4/(3 m2^2)
 *   [7] v1 = -<(|M|-<|M|>)(E-<E>)>/<|M|>             [8] v2 = the same with |M|^2
 * (paper, sections "Thermal averages" and "Critical exponents": M, chi and
 * the specific heat, and the cumulants of the magnetisation used for
 * finite-size scaling; v_j = d ln<|M|^j>/d beta).  Every sum is taken in a
 * fixed order.  All calls return after their kernels have finished on
 * `stream`; they allocate small device tables of their own. */
#define HSIM_THERMAL_FIELDS 9
/* Thermal summary of every series, evaluated at n_eval inverse temperatures
 * by single-histogram reweighting (paper, section "Histogram and multiple
 * histogram methods"; weights exp(-(beta' - beta) E_m)):
 *   beta [n_rep][n_steps] (host): the sampling inverse temperatures;
 *   beta_eval [n_rep][n_steps][n_eval] (host; NULL with n_eval = 1: beta);
 *   d_out [n_rep][n_steps][n_eval][9] (device). */
hsim_status hsim_analysis_thermal(const double *d_history, int32_t n_rep, int32_t n_steps,
                                  int32_t mcs, int32_t m0, int64_t n_sites, const double *beta,
                                  int32_t n_eval, const double *beta_eval, double *d_out,
                                  void *stream);
/* Integrated autocorrelation time of E (observable 0) or |M| (1) of every
 * series (paper, section "Dynamic behavior"): tau = 1/2 + sum_{t=1..W} rho(t)
 * with Sokal's window, W the first lag with W >= c tau (at most the half
 * length).  d_tau [n_rep][n_steps] double, d_window (NULL or int32, same
 * shape). */
hsim_status hsim_analysis_tau(const double *d_history, int32_t n_rep, int32_t n_steps,
                              int32_t mcs, int32_t m0, int32_t observable, double c,
                              double *d_tau, int32_t *d_window, void *stream);
/* Multiple-histogram method (paper, section "Histogram and multiple
 * histogram methods"; Ferrenberg and Swendsen 1989) over K series
 * series [K][2] = (replica, step) (host) sampled at beta_k [K] (host): the
 * free energies f_k (f_0 = 0) from the self-consistent equations, iterated
 * in log space until max |f_new - f| < tol or max_iter iterations
 * (f_out [K] host, *iters_out), then the thermal summary at beta_eval [n_eval]
 * (host) into d_out [n_eval][9] (device). */
hsim_status hsim_analysis_multihist(const double *d_history, int32_t n_rep, int32_t n_steps,
                                    int32_t mcs, int32_t m0, int64_t n_sites, int32_t K,
                                    const int32_t *series, const double *beta_k, int32_t n_eval,
                                    const double *beta_eval, int32_t max_iter, double tol,
                                    double *f_out, int32_t *iters_out, double *d_out,
                                    void *stream);

const char *hsim_last_error(void);
const char *hsim_version(void);

#ifdef __cplusplus
}
#endif
#endif
