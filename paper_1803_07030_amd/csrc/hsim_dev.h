// Device-visible structures of libhsim and the launchers the host code calls.
// Shared by the host orchestration (plan.cpp, batch.cpp) and the kernels
// (*.hip); nothing here is visible at the C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsim {

constexpr int kMaxColours = 32;     // colour classes per lattice
constexpr int kSiteBlock = 256;     // threads per block of the site-lane kernels
constexpr int kFinThreads = 512;    // threads per block of the site-lane finish launch
#ifndef HSIM_REP_WAVES
#define HSIM_REP_WAVES 4
#endif
#ifndef HSIM_REP_SITES_PER_WAVE
#define HSIM_REP_SITES_PER_WAVE 32
#endif
constexpr int kRepWaves = HSIM_REP_WAVES;                    // waves per replica-lane block
constexpr int kRepSitesPerWave = HSIM_REP_SITES_PER_WAVE;    // sites per wave of a tile
constexpr int kRepThreads = kRepWaves * 64;
#ifndef HSIM_REP_SITES_PER_STEP
#define HSIM_REP_SITES_PER_STEP 1
#endif
// sites whose loads a wave issues together (64-lane groups); divides the
// sites per wave
constexpr int kRepSitesPerStep = HSIM_REP_SITES_PER_STEP;
static_assert(kRepSitesPerWave % kRepSitesPerStep == 0 && kRepSitesPerWave % 4 == 0,
              "sites per wave must be a multiple of the sites per step and of 4");
constexpr int kMaxPersistentBlocks = 4096;   // barrier flags reserved in the workspace
constexpr int kXBarLines = 48;   // the flag region's last lines: per-XCD barrier words (3 x 16)
constexpr int kRepTile = kRepWaves * kRepSitesPerWave;   // sites per replica-lane tile (at most)
// tile shapes (sites per wave) the replica layout may use
constexpr int kRepTileShapes[3] = {4, 8, kRepSitesPerWave};
constexpr int kRecSite = 8;         // doubles per site-lane partial record
constexpr int kRecFields = 7;       // dE, Mx, My, Mz, n_acc, E_full, adaptive accepts
constexpr int kChunks = 64;         // replica layout: chunks of the per-MCS record sum

// How the anisotropy and field-direction terms are read.
enum KMode : int { K_NONE = 0, K_UNIFORM = 1, K_SITE = 2 };
enum FMode : int { F_UNIFORM = 0, F_SITE = 1 };

// One replica: its lattice (internal colour-sorted order) and its spins.
struct RepDesc {
    const int32_t *rp;        // n+1 CSR row offsets
    const int32_t *ci;        // nnz internal column indices
    const void *J;            // nnz constants (float or double)
    const uint32_t *orig;     // n user index of each internal site
    const void *k;            // n (K_SITE)
    const void *ax;           // [3][n] (K_SITE), stride n
    const void *nd;           // [3][n] (F_SITE), stride n
    void *spins;              // [3][n_pad] of this replica (site and block layouts)
    const int32_t *type;      // n site types (internal order), NULL: type 0 everywhere
    const void *kc;           // n cubic constants (float or double), NULL: none
    const void *mu;           // n spin norms (float or double), NULL: unit spins
    const double *mu_d;       // n spin norms in double (initial states), NULL: unit
    const int32_t *ellT_col;  // [ell_w][n] padded rows, slot-major (NULL: use the CSR)
    const void *ellT_J;       // [ell_w][n] (float or double)
    double k0, e0[3], n0[3];  // uniform values (K_UNIFORM / F_UNIFORM)
    int64_t user_off;         // offset of this replica in replica-concatenated user arrays
    int32_t n, n_pad;
    uint32_t rep_id;
    int32_t ncol, ell_w;
    int32_t cls_off[kMaxColours + 1];
};

// A block's share of one colour phase of one replica: internal sites [begin, end).
struct Tile {
    int32_t rep, begin, end, colour;
    int32_t nsl;   // padded-row slots that any site of the tile uses (its largest degree)
};

// Update policy of every site type.
enum : int32_t { POL_RANDOM = 0, POL_FLIP = 1, POL_SMALL_STEP = 2, POL_GAUSSIAN = 3, POL_HN = 4,
                 POL_ADAPTIVE = 5 };
constexpr int kMaxTypes = 8;
struct Policies {
    int32_t n_types;            // 0: the random move everywhere
    int32_t adaptive;           // some type uses the adaptive move
    int32_t pol[kMaxTypes];
    double param[kMaxTypes];    // half-angle theta (small step, Hinzke-Nowak) or sigma (Gaussian)
    double cos_t[kMaxTypes];    // cos theta
    double sigma_min, sigma_max;
};

// Run-control word block at the start of the workspace.
struct Ctl {
    uint32_t g;          // first MCS of the current launch sequence
    uint32_t status;     // HSIM_E_* bits seen on the device
    uint32_t bar_arrive; // persistent-launch barrier
    uint32_t pad[61];
};

// Constants of one run, passed by value to every kernel of the run.
struct RunArgs {
    Ctl *ctl;
    const double *beta;   // [R][S_hist]
    const double *bfield; // [R][S_hist]
    double *ecarry;       // [R]
    double *partials;     // records (replica layout: [rec_win][tiles][6][Rp])
    double *chunks;       // replica layout: chunk sums [rec_win][64][6][Rp]
    double *carry;        // replica layout: per-MCS totals [rec_win][6][Rp]
    double *history;      // [R][S_hist][M][5]
    uint32_t *trace;      // NULL or [R][n_mcs_run][words]
    uint64_t seed;
    uint32_t g0;          // first g of the run
    int32_t M;            // MCS per step
    int32_t S_hist;       // steps in the bound history
    int32_t P;            // recompute period (0: step start only)
    int32_t n_mcs_run;    // MCS in this run
    int32_t trace_words;  // words per replica per MCS
    int32_t R;
    int32_t rec_win;      // replica layout: MCS per record window (>= 2)
    Policies pol;
    double *sigma;        // [R] adaptive width (when pol.adaptive)
    const double *n_ad;   // [R] sites under the adaptive move per replica
    double *sig_part;     // replica layout: [kChunks][Rp] partial adaptive accepts
    // optional outputs (NULL: off)
    double *type_mag;     // [R][S_hist][M][tm_types][3] magnetisation per site type
    double *tm_part;      // per-type partial sums
    int32_t tm_types;
    double *snapshots;    // [R][S_hist][snap_n][3] spins at each step end, user order
    int32_t snap_n;
};

struct RepLaneArgs {
    const int32_t *rp, *ci;
    const float *J;
    const int32_t *type;        // [n] site types (internal order), NULL: type 0
    const float *kc, *mu;       // [n] cubic constants / spin norms, NULL: none / unit
    const double *mu_d;         // [n] spin norms in double (initial states)
    const int32_t *ell_col;     // [n][maxd] padded rows, site-major
    const float *ell_J;
    const uint32_t *orig;
    const float *k, *ax, *nd;   // per-site (K_SITE / F_SITE)
    float *spins;               // row of Rp floats per (component c, site i) at c*cs + i*ss
    const uint32_t *rep_id;     // [Rp]
    int64_t cs;                 // component stride (floats)
    float k0, e0x, e0y, e0z, n0x, n0y, n0z;
    int32_t n, Rp, R;
    int32_t ss;                 // site stride (floats): Rp or 3*Rp
    int32_t spw;                // sites per wave of a tile: a multiple of 4, at most kRepSitesPerWave
    int32_t masked_store;       // 1: only accepted moves are stored; 0: every live lane writes its row
    int32_t ncol, ell_w;        // ell_w: padded row width (6 or 8), 0 = CSR walk
    int32_t cls_off[kMaxColours + 1];
    int32_t tile_off[kMaxColours + 1];   // first tile of each colour
    // dispatch order: slot u of colour c (after the XCD split) runs tile
    // tord[tile_off[c] + u] of the class; NULL: tile u
    const int32_t *tord;
};

// XCD-aware bijection of [0, nt): blocks are dispatched round-robin over the
// 8 XCDs, so block b runs on XCD b % 8; give each XCD a contiguous range of
// tiles, so that a tile and the tiles holding its neighbours share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nt)
{
    const int q = nt >> 3, rm = nt & 7, x = b & 7, k = b >> 3;
    return x * q + min(x, rm) + k;
}

// ------------------------------------------------------------- launchers
// All return hipError_t of the launch.  Template choices are resolved inside.
hipError_t launch_ctl_set(hipStream_t st, Ctl *ctl, uint32_t g);
hipError_t launch_fill_u32(hipStream_t st, uint32_t *p, uint32_t v, int64_t n);
// Schedule values carried in kernel arguments (for runs recorded into a
// caller's graph): entries k0 .. k0+cnt-1 of the flat (replica, step) order of
// a run, each a (beta, field) pair, written to beta/bfield [R][S_hist].
constexpr int kPutPairs = 112;
struct PutPairs {
    double v[2 * kPutPairs];
};
hipError_t launch_put_schedule(hipStream_t st, double *beta, double *bfield, int S_hist,
                               int first_step, int n_steps, int k0, int cnt, const PutPairs &vals);

hipError_t launch_init_spins(hipStream_t st, bool f64, const RepDesc *reps, int R,
                             int max_n, int mode, const double *given, const int64_t *given_off,
                             uint64_t seed);
hipError_t launch_init_spins_rep(hipStream_t st, const RepLaneArgs &a, int mode,
                                 const double *given, uint64_t seed);
hipError_t launch_to_user(hipStream_t st, bool f64, const RepDesc *reps, int rep, int n,
                          double *out);
hipError_t launch_to_user_rep(hipStream_t st, const RepLaneArgs &a, int rep, double *out);

hipError_t launch_site_phase(hipStream_t st, bool f64, int kmode, int fmode, bool trace, int ellw,
                             const RepDesc *reps, const Tile *tiles, int tile_off, int ntiles,
                             int t_off, const RunArgs &ra);
hipError_t launch_site_efull(hipStream_t st, bool f64, int kmode, int fmode, const RepDesc *reps,
                             const Tile *tiles, int tile_off, int ntiles, int t_off, const RunArgs &ra);
// Colour classes c_tail .. ncol_max-1 (one block per replica) plus the
// per-MCS history of every replica (the same results as a phase launch per
// class).
hipError_t launch_site_finish(hipStream_t st, bool f64, int kmode, int fmode, bool trace, int ellw,
                              const RepDesc *reps, const int32_t *rep_tiles, const int32_t *rlist,
                              int nrep, int ncol_max, int c_tail, int t_off, const RunArgs &ra);
hipError_t launch_ctl_advance(hipStream_t st, Ctl *ctl, uint32_t n);
hipError_t launch_block_sweep(hipStream_t st, bool f64, int kmode, int fmode, bool trace,
                              int ellw, bool lds, int threads, size_t lds_bytes, const RepDesc *reps,
                              const RunArgs &ra);
int block_sweep_max_lds(bool f64);

hipError_t launch_rep_phase(hipStream_t st, int kmode, int fmode, int colour, int t_off,
                            const RepLaneArgs &a, int ntiles, const RunArgs &ra);
hipError_t launch_rep_efull(hipStream_t st, int kmode, int fmode, const RepLaneArgs &a,
                            int ntiles, int t_off, const RunArgs &ra);
// Adaptive widths after MCS t_off of the current sequence (policies with the
// adaptive move).
hipError_t launch_rep_sigma(hipStream_t st, const RepLaneArgs &a, int ntiles, int t_off,
                            const RunArgs &ra);
// Reduction of the record window holding MCS t_first .. t_first + count - 1
// of the current sequence (count <= rec_win); advance > 0 closes the sequence.
hipError_t launch_rep_reduce(hipStream_t st, const RepLaneArgs &a, int ntiles, int t_first,
                             int count, int advance, const RunArgs &ra);
// Optional outputs (output_kernels.hip).
int type_part_blocks(bool replica_layout, int max_n);
hipError_t launch_type_mag_site(hipStream_t st, bool f64, const RepDesc *reps, int R, int max_n,
                                int t_off, const RunArgs &ra);
hipError_t launch_type_mag_rep(hipStream_t st, const RepLaneArgs &a, int t_off, const RunArgs &ra);
hipError_t launch_snapshot_site(hipStream_t st, bool f64, const RepDesc *reps, int R, int max_n,
                                int t_off, bool check, const RunArgs &ra);
hipError_t launch_snapshot_rep(hipStream_t st, const RepLaneArgs &a, int t_off, bool check,
                               const RunArgs &ra);
hipError_t launch_rep_persistent(hipStream_t st, int kmode, int fmode, const RepLaneArgs &a,
                                 int ntiles, int grid, const RunArgs &ra, uint32_t *flags,
                                 uint32_t spin_cap);
int rep_persistent_blocks_per_cu(int kmode, int fmode, int lane_w, int ell_w);

// energy
struct EnergyArgs {
    const int64_t *rp;      // user-order CSR (n+1)
    const int32_t *ci;      // nnz
    const int32_t *bond;    // nnz: bond id of each entry
    const int32_t *fwd_entry; // nb: the CSR entry of each bond at its lower end
    const int32_t *ecol;    // [ell_w][n] padded rows, slot-major (padding: the site itself)
    const int32_t *ebond;   // [ell_w][n] bond id of each slot (-1 past the row)
    const int32_t *hcol;    // [ell_w/2][n] half rows: the bonds each site leaves (forward)
    const int32_t *hbond;   // [ell_w/2][n] their bond ids (-1 past the row)
    int64_t n, nnz, nb;
    int batch;
    const void *S, *Jb, *k, *ax, *nd;
    const void *kc;         // NULL, or [n] cubic constants of the plan (user order)
    double B;
};
// Scratch of the energy calls: partial records of one pass of at most
// pass_cfg configurations (groups of 32), in doubles from the scratch start.
constexpr int kEnergyMaxGroups = 64;
struct EnergyLayout {
    int ntile, ell_w, groups, pass_cfg;
    int64_t off_partE, off_partB, off_partK, off_partJ, off_accK, off_accJ, off_pB, off_accB;
    int64_t doubles;
};
// Layout for a plan of n sites and nb bonds in a scratch of about
// cap_doubles, with at least min_groups groups per pass (0: groups = 0 when
// not even one fits); forward_only: the forward's records alone.
EnergyLayout energy_layout(int64_t n, int64_t nb, int ell_w, int64_t cap_doubles, bool forward_only,
                           int min_groups);
hipError_t launch_energy_forward(hipStream_t st, bool f64, const EnergyArgs &a,
                                 const EnergyLayout &L, double *scratch, double *E);
// The fixed device array of the allocation-free forward (8 MiB per GPU) and
// its address on the current device (resolved on first use per device).
constexpr int64_t kStaticEnergyScratchDoubles = (int64_t)1 << 20;
constexpr int kMaxDevices = 64;
hipError_t static_energy_scratch(double **out);
hipError_t launch_energy_backward(hipStream_t st, bool f64, const EnergyArgs &a, const double *gE,
                                  void *gS, void *gJ, void *gk, double *gB, const EnergyLayout &L,
                                  double *scratch);
hipError_t launch_fluct(hipStream_t st, int64_t n, double beta, const double *O,
                        const double *dE, const double *dO, double *out);
hipError_t launch_fluct_weights(hipStream_t st, int64_t n, double beta, const double *O, double c,
                                double *w);
hipError_t launch_spins_planar(hipStream_t st, bool f64, int64_t n_cfg, int64_t n,
                               const double *in, void *out);

}  // namespace hsim
