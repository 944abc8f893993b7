// Host-side objects behind the C-ABI: plans (one lattice each) and batches
// (replicas over plans, their tiles and launch state).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hsim.h"
#include "hsim_dev.h"

namespace hsim {

// Error carrying an hsim_status code; caught at the C-ABI boundary.
struct Error : std::runtime_error {
    hsim_status code;
    Error(hsim_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

inline void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess)
        throw Error(HSIM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Device allocation owned by a plan or batch.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T *upload(const std::vector<T> &v)
    {
        release();
        bytes = v.size() * sizeof(T);
        if (bytes == 0) bytes = sizeof(T);
        hip_check(hipMalloc(&p, bytes), "hipMalloc");
        if (!v.empty()) hip_check(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
        return (T *)p;
    }
    void *alloc(size_t b)
    {
        release();
        bytes = b ? b : 16;
        hip_check(hipMalloc(&p, bytes), "hipMalloc");
        return p;
    }
};

}  // namespace hsim

struct hsim_plan_s {
    int64_t n = 0, nnz = 0, nb = 0;
    uint64_t hash = 0;                    // of the lattice as given (autotuner cache key)
    int32_t ncol = 0, maxdeg = 0;
    std::vector<int32_t> colour;          // user order
    std::vector<int32_t> perm;            // internal -> user
    std::vector<int32_t> inv;             // user -> internal
    std::vector<int32_t> cls_off;         // ncol+1
    // internal CSR (colour-sorted rows, each row's entry order kept)
    std::vector<int32_t> rp, ci;
    std::vector<double> Jd;
    std::vector<float> Jf;
    // per-site parameters, internal order, [n] and [3][n]
    std::vector<double> kd, axd, ndd;
    std::vector<float> kf, axf, ndf;
    int kmode = 0, fmode = 0;
    double k0 = 0.0, e0[3] = {0, 0, 1}, n0[3] = {0, 0, 1};
    // padded rows (ELL) of the internal CSR when every row has <= 8 entries:
    // slot s of site i holds (col, J), or (i, 0) past the row's end;
    // site-major [n][ell_w] and slot-major [ell_w][n] copies
    int ell_w = 0;
    std::vector<int32_t> ell_col, ellT_col;
    std::vector<float> ell_Jf, ellT_Jf;
    std::vector<double> ellT_Jd;
    // site types (internal order; empty: type 0 everywhere)
    std::vector<int32_t> type;
    // cubic constants and spin norms (internal order; empty: none / unit),
    // and the cubic constants in user order for the energy API
    std::vector<double> kcd, mud, ukcd;
    std::vector<float> kcf, muf, ukcf;
    // user-order CSR for the energy and its gradient
    std::vector<int64_t> urp;
    std::vector<int32_t> uci, ubond, fwd_entry, bond_ij;

    // device copies (uploaded on first use)
    bool sweep_on_device = false, energy_on_device = false;
    hsim::DevBuf d_rp, d_ci, d_Jf, d_Jd, d_orig, d_kf, d_kd, d_axf, d_axd, d_ndf, d_ndd;
    hsim::DevBuf d_ell_col, d_ell_J, d_ellT_col, d_ellT_Jf, d_ellT_Jd, d_type;
    hsim::DevBuf d_kcf, d_kcd, d_muf, d_mud, d_ukcf, d_ukcd;
    void upload_terms();
    hsim::DevBuf d_urp, d_uci, d_ubond, d_fwd;
    // energy calls: padded rows of the user-order CSR (width 6 or 8 when
    // every row fits, else 0: CSR walk), slot-major [e_w][n]; the fixed
    // scratch and its pass layout, set up once by prepare_energy()
    int e_w = 0;
    std::vector<int32_t> uell_col, uell_bond;
    // the forward's half rows: every bond once, at the end an Euler
    // orientation makes it leave (at most ceil(deg/2) per site), slot-major
    // [h_w][n] with h_w = e_w / 2
    int h_w = 0;
    std::vector<int32_t> uhalf_col, uhalf_bond;
    hsim::DevBuf d_uell_col, d_uell_bond, d_uhalf_col, d_uhalf_bond, d_escratch;
    hsim::EnergyLayout elayout{};
    bool energy_ready = false;

    void upload_sweep();
    void upload_energy();
    void prepare_energy();
};

struct hsim_batch_s {
    int32_t R = 0;
    std::vector<hsim_plan> plans;
    std::vector<uint32_t> rep_id;
    uint64_t seed = 0;
    bool f64 = false;
    int layout = HSIM_LAYOUT_SITE;
    int kmode = 0, fmode = 0;
    int ncol_max = 0;
    int ellw = 0;                     // common padded row width of the plans (0: CSR walk)
    int64_t total_sites = 0;
    bool lds = false;
    int block_threads = 256;
    size_t lds_bytes = 0;

    // site and block layouts
    std::vector<hsim::RepDesc> reps;
    std::vector<hsim::Tile> tiles;
    std::vector<int32_t> rep_tiles;   // [R][ncol_max][2]
    int32_t c_tail = 0;               // colours >= c_tail run in the per-replica finish launch
    // site layout: the replicas with trailing classes (group 1) and the
    // others (group 0); tiles are group-major, then colour, then replica.
    // With two groups each runs its launch sequence on a stream of its own,
    // so one group's latency-bound finish overlaps the other's phases.
    int ngroups = 1;
    std::vector<int32_t> gtile_off[2];   // [ncol_max+1] first tile of colour c in group g
    std::vector<int64_t> gunits[2];      // [ncol_max] updates of colour c in group g
    std::vector<int32_t> grp_reps[2];
    hsim::DevBuf d_grp_reps[2];
    hipStream_t gstream[2] = {nullptr, nullptr};
    hipEvent_t gfork = nullptr, gjoin[2] = {nullptr, nullptr};
    std::vector<int64_t> spin_off;    // elements, per replica
    int64_t spin_elems = 0;
    // replica layout
    int32_t Rp = 0;
    int32_t rep_ntiles = 0;
    // update policies per site type, the adaptive sites per replica and the
    // starting adaptive width
    hsim::Policies pol{};
    std::vector<double> nad;
    hsim::DevBuf d_nad;
    double sigma0 = 1.0;
    size_t off_sigma = 0;
    // optional outputs (caller-owned device buffers) and their scratch
    double *type_mag = nullptr, *snapshots = nullptr;
    int32_t tm_types = 0;
    hsim::DevBuf d_tm_part;
    void reset_sigma();             // every replica's adaptive width to sigma0
    int32_t rec_win = 2;              // replica layout: MCS per record window
    // replica layout: bytes of the record window, its chunk sums and totals,
    // and the partial adaptive-accept sums
    size_t rep_rec_bytes() const
    {
        return ((size_t)rec_win * ((size_t)rep_ntiles * hsim::kRecFields + (size_t)hsim::kChunks * 6 + 6) +
                (size_t)hsim::kChunks) * Rp * 8;
    }
    hsim::RepLaneArgs la{};
    // replica layout: dispatch order of each colour's tiles (see rep_order):
    // order_mode -1 derives the plane stride from the lattice and uses it on
    // lattices too large to have every tile of a colour in flight, 0 keeps
    // the tiles in order, > 1 is the plane stride in sites
    int32_t order_mode = -1;
    int64_t plane_sites = -1;    // derived once (0: none found)
    std::vector<int32_t> tord;
    hsim::DevBuf d_tord;

    hsim::DevBuf d_reps, d_tiles, d_rep_tiles, d_rep_id;
    bool tables_on_device = false;

    // binding
    bool bound = false;
    int32_t S_hist = 0, M = 0;
    char *ws = nullptr;
    void *spins = nullptr;
    double *history = nullptr;
    size_t off_ecarry = 0, off_beta = 0, off_bfield = 0, off_part = 0, ws_bytes = 0;
    std::vector<double> h_beta, h_bfield;   // [R][S_hist]
    double *h_stage = nullptr;              // pinned staging of beta and bfield
    hipEvent_t stage_done = nullptr;

    // GRAPH launches: the instantiated graph of one recompute period, kept
    // across calls while the captured arguments stay the same; captured on a
    // private stream (nothing runs there) and replayed on the caller's
    hipGraph_t g_graph = nullptr;
    hipGraphExec_t g_exec = nullptr;
    hipStream_t g_cap = nullptr;
    hipEvent_t g_done = nullptr;          // recorded after the last enqueued replay
    std::vector<unsigned char> g_key;
    void drop_graph();                    // waits for enqueued replays, then frees

    // tuning
    int tuned_launch = -1;
    int persistent_grid = 0;
    // sampled launch timing of the colour phases: event pairs and the updates
    // each timed launch processed
    int time_every = 0;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<int64_t> ev_units;
    int64_t phase_updates(int colour) const;

    ~hsim_batch_s();
    void upload_tables();
    hsim::RunArgs run_args(uint32_t g0, int n_mcs, int P, uint32_t *trace);
};
