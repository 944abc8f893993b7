// Batches: replicas over plans, their spin layout, tiles and workspace, and
// the launch sequence of a run (paper, section "Monte Carlo Metropolis
// algorithm": MCS after MCS, every site once per MCS; section "VEGAS software
// package": history after every MCS of every temperature/field step).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <limits>
#include <memory>
#include <sstream>

#include "hsim_host.h"

using hsim::Error;
using hsim::hip_check;

// Replica layout: the three component rows of a site side by side
// ([n][3][Rp]; 1 to 2% faster colour phases on SC 64^3 than [3][n][Rp]);
// 0 selects the planar layout.
#ifndef HSIM_REP_INTERLEAVED
#define HSIM_REP_INTERLEAVED 1
#endif

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
int64_t pad64(int64_t n) { return (n + 63) / 64 * 64; }

int device_lds_limit()
{
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return 160 * 1024 - 1024;
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 160 * 1024 - 1024;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 64 * 1024 - 1024;
    return v - 1024;
}

int device_cus()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return v;
}

}  // namespace

void hsim_batch_s::drop_graph()
{
    if (g_exec) {
        if (g_done) (void)hipEventSynchronize(g_done);
        (void)hipGraphExecDestroy(g_exec);
    }
    if (g_graph) (void)hipGraphDestroy(g_graph);
    g_exec = nullptr;
    g_graph = nullptr;
    g_key.clear();
}

hsim_batch_s::~hsim_batch_s()
{
    drop_graph();
    for (int g = 0; g < 2; ++g) {
        if (gstream[g]) (void)hipStreamSynchronize(gstream[g]);
        if (gjoin[g]) (void)hipEventDestroy(gjoin[g]);
        if (gstream[g]) (void)hipStreamDestroy(gstream[g]);
    }
    if (gfork) (void)hipEventDestroy(gfork);
    if (g_done) (void)hipEventDestroy(g_done);
    if (g_cap) (void)hipStreamDestroy(g_cap);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (stage_done) {
        (void)hipEventSynchronize(stage_done);
        (void)hipEventDestroy(stage_done);
    }
    if (h_stage) (void)hipHostFree(h_stage);
}

namespace {

// Replica layout: blocks of the largest colour phase for tiles of
// kRepWaves x spw sites (times the lane columns of a tile).
int64_t rep_phase_blocks(hsim_batch b, int spw)
{
    hsim_plan P = b->plans[0];
    const int cols = b->Rp % 64 == 0 ? b->Rp / 64 : 1;   // lane columns per tile
    int64_t mx = 0;
    for (int c = 0; c < P->ncol; ++c) {
        const int64_t sz = P->cls_off[c + 1] - P->cls_off[c];
        mx = std::max<int64_t>(mx, (sz + hsim::kRepWaves * spw - 1) / (hsim::kRepWaves * spw));
    }
    return mx * cols;
}

// Tiles of kRepWaves x spw sites per colour class and the record window that
// goes with them: records of up to 64 MCS, about 256 MiB at most (2 at least).
struct RepTiling {
    int32_t tile_off[hsim::kMaxColours + 1];
    int32_t ntiles, rec_win;
};
RepTiling rep_tiling(hsim_batch b, int spw)
{
    hsim_plan P = b->plans[0];
    RepTiling t{};
    const int tile = hsim::kRepWaves * spw;
    t.tile_off[0] = 0;
    for (int c = 0; c < P->ncol; ++c) {
        const int sz = P->cls_off[c + 1] - P->cls_off[c];
        t.tile_off[c + 1] = t.tile_off[c] + (sz + tile - 1) / tile;
    }
    t.ntiles = t.tile_off[P->ncol];
    const size_t per_mcs = (size_t)t.ntiles * hsim::kRecFields * b->Rp * 8;
    t.rec_win = (int32_t)std::max<size_t>(2, std::min<size_t>(64, (256u << 20) / std::max<size_t>(per_mcs, 1)));
    return t;
}

}  // namespace

// Distance, in sites of a colour class, at which two sites of the class share
// a neighbour a plane apart: the 95th percentile of the class-position
// offsets between neighbours (a periodic wrap is rare, the largest regular
// offset common).  On a simple-cubic L^3 lattice it is L^2 / 2, the sites of
// one class in one plane.
int64_t derive_plane_sites(hsim_plan P)
{
    if (P->ncol < 2 || P->n == 0) return 0;
    std::vector<int32_t> cls(P->n);
    for (int c = 0; c < P->ncol; ++c)
        for (int32_t t = P->cls_off[c]; t < P->cls_off[c + 1]; ++t) cls[t] = c;
    const int32_t n0 = P->cls_off[1];
    const int32_t step = std::max<int32_t>(1, n0 / 65536);
    std::vector<int64_t> d;
    for (int32_t t = 0; t < n0; t += step)
        for (int32_t p = P->rp[t]; p < P->rp[t + 1]; ++p) {
            const int32_t j = P->ci[p];
            d.push_back(std::llabs((int64_t)(j - P->cls_off[cls[j]]) - (int64_t)t));
        }
    if (d.empty()) return 0;
    const size_t k = d.size() * 95 / 100;
    std::nth_element(d.begin(), d.begin() + k, d.end());
    return d[k];
}

// Dispatch order of the replica layout's tiles inside each XCD's range:
// ordered by (tile mod pt, tile / pt), pt = tiles per plane of the class, so
// that tiles one plane apart, which read the same neighbour rows, start
// together instead of a plane of traffic apart.  Results do not depend on it
// (records are kept per tile).  Used when a colour has more tiles per XCD
// than the XCD runs at once (8 blocks per CU).
void rep_order(hsim_batch b)
{
    b->tord.clear();
    int64_t ps = 0;
    if (b->order_mode > 1) ps = b->order_mode;
    else if (b->order_mode < 0) {
        if (b->plane_sites < 0) b->plane_sites = derive_plane_sites(b->plans[0]);
        int max_nt = 0;
        for (int c = 0; c < b->plans[0]->ncol; ++c)
            max_nt = std::max(max_nt, b->la.tile_off[c + 1] - b->la.tile_off[c]);
        const int cus = device_cus() > 0 ? device_cus() : 256;
        if (max_nt / 8 > cus) ps = b->plane_sites;
    }
    const int64_t tile_sites = (int64_t)hsim::kRepWaves * b->la.spw;
    const int pt = (int)((ps + tile_sites / 2) / tile_sites);
    if (pt >= 2) {
        const int C = b->plans[0]->ncol;
        b->tord.resize((size_t)b->rep_ntiles);
        for (int c = 0; c < C; ++c) {
            const int t0 = b->la.tile_off[c], nt = b->la.tile_off[c + 1] - t0;
            const int q = nt >> 3, rm = nt & 7;   // the XCD ranges of xcd_tile
            for (int x = 0; x < 8; ++x) {
                const int s = x * q + std::min(x, rm), len = q + (x < rm ? 1 : 0);
                std::vector<int32_t> r(len);
                for (int k = 0; k < len; ++k) r[k] = s + k;
                std::stable_sort(r.begin(), r.end(), [pt](int32_t u, int32_t v) {
                    return std::make_pair(u % pt, u / pt) < std::make_pair(v % pt, v / pt);
                });
                for (int k = 0; k < len; ++k) b->tord[(size_t)t0 + s + k] = r[k];
            }
        }
    }
    if (b->tables_on_device) {
        // launches already enqueued may still read the old table
        if (b->d_tord.p) hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
        if (b->tord.empty()) {
            b->la.tord = nullptr;
            b->d_tord.release();
        } else {
            b->d_tord.upload(b->tord);
            b->la.tord = (const int32_t *)b->d_tord.p;
        }
    }
}

// The replica layout's tile shape; the workspace is sized for every shape
// the autotuner may pick, so a bound batch can switch.
void set_rep_tiles(hsim_batch b, int spw)
{
    const RepTiling t = rep_tiling(b, spw);
    b->la.spw = spw;
    for (int c = 0; c <= hsim::kMaxColours; ++c) b->la.tile_off[c] = c <= b->plans[0]->ncol ? t.tile_off[c] : 0;
    b->rep_ntiles = t.ntiles;
    b->rec_win = t.rec_win;
    b->drop_graph();   // waits for replays that read the old order table
    rep_order(b);
}

void batch_set_order_impl(hsim_batch b, int32_t plane_sites)
{
    if (!b) throw Error(HSIM_E_ARG, "set_order: NULL batch");
    if (b->layout != HSIM_LAYOUT_REPLICA) throw Error(HSIM_E_UNSUPPORTED, "set_order: replica layout only");
    if (plane_sites < -1 || plane_sites == 1) throw Error(HSIM_E_ARG, "set_order: bad plane stride");
    b->order_mode = plane_sites;
    b->drop_graph();   // waits for replays that read the old order table
    rep_order(b);
}

void batch_set_shape_impl(hsim_batch b, int32_t spw, int32_t masked)
{
    if (!b) throw Error(HSIM_E_ARG, "set_shape: NULL batch");
    if (b->layout != HSIM_LAYOUT_REPLICA) throw Error(HSIM_E_UNSUPPORTED, "set_shape: replica layout only");
    bool ok = false;
    for (int c : hsim::kRepTileShapes) ok |= c == spw;
    if (!ok || (masked != 0 && masked != 1)) throw Error(HSIM_E_ARG, "set_shape: bad shape");
    if (spw != b->la.spw) set_rep_tiles(b, spw);
    if (masked != b->la.masked_store) {
        b->la.masked_store = masked;
        b->drop_graph();
    }
}

size_t rep_rec_bytes_max(hsim_batch b)
{
    size_t mx = 0;
    for (int spw : hsim::kRepTileShapes) {
        const RepTiling t = rep_tiling(b, spw);
        const size_t bytes = ((size_t)t.rec_win * ((size_t)t.ntiles * hsim::kRecFields +
                                                   (size_t)hsim::kChunks * 6 + 6) +
                              (size_t)hsim::kChunks) * b->Rp * 8;
        mx = std::max(mx, bytes);
    }
    return mx;
}

hsim_batch batch_create_impl(int32_t R, const hsim_plan *plans, uint64_t seed,
                             const uint32_t *rep_id, hsim_precision prec, hsim_layout layout)
{
    if (R < 1 || !plans) throw Error(HSIM_E_ARG, "batch needs at least one replica");
    if (prec != HSIM_FP32 && prec != HSIM_FP64_EXACT) throw Error(HSIM_E_ARG, "bad precision");
    if (layout < HSIM_LAYOUT_AUTO || layout > HSIM_LAYOUT_BLOCK) throw Error(HSIM_E_ARG, "bad layout");
    for (int r = 0; r < R; ++r)
        if (!plans[r]) throw Error(HSIM_E_ARG, "NULL plan");
    auto *b = new hsim_batch_s();
    try {
        b->R = R;
        b->plans.assign(plans, plans + R);
        b->rep_id.resize(R);
        for (int r = 0; r < R; ++r) b->rep_id[r] = rep_id ? rep_id[r] : (uint32_t)r;
        b->seed = seed;
        b->f64 = prec == HSIM_FP64_EXACT;
        const size_t elem = b->f64 ? 8 : 4;
        bool shared = true;
        int64_t max_n = 0, max_cls = 0;
        for (int r = 0; r < R; ++r) {
            hsim_plan P = plans[r];
            shared = shared && P == plans[0];
            b->kmode = std::max(b->kmode, P->kmode);
            b->fmode = std::max(b->fmode, P->fmode);
            b->ncol_max = std::max(b->ncol_max, P->ncol);
            b->total_sites += P->n;
            max_n = std::max(max_n, P->n);
            for (int c = 0; c < P->ncol; ++c)
                max_cls = std::max<int64_t>(max_cls, P->cls_off[c + 1] - P->cls_off[c]);
        }
        if (b->total_sites > (int64_t)INT32_MAX) throw Error(HSIM_E_UNSUPPORTED, "batch too large");
        b->ellw = plans[0]->ell_w;
        for (int r = 1; r < R; ++r)
            if (plans[r]->ell_w != b->ellw) b->ellw = 0;
        const int64_t lds_limit = device_lds_limit();
        const bool fits_lds = 3 * pad64(max_n) * (int64_t)elem <= lds_limit;
        int lay = layout;
        // replica layout: one spin plane (n x Rp floats) must stay below 2 GiB
        const int64_t rp_pad = R > 32 ? (R + 63) / 64 * 64 : 32;
        const bool plane_ok = max_n * rp_pad * 4 < ((int64_t)1 << 31);
        if (lay == HSIM_LAYOUT_REPLICA && (b->f64 || !shared || !plane_ok))
            throw Error(HSIM_E_UNSUPPORTED,
                        "replica layout needs FP32, one shared lattice and a spin plane below 2 GiB");
        if (lay == HSIM_LAYOUT_AUTO) {
            if (!b->f64 && shared && R >= 16 && plane_ok) lay = HSIM_LAYOUT_REPLICA;
            else if (fits_lds) lay = HSIM_LAYOUT_BLOCK;
            else lay = HSIM_LAYOUT_SITE;
        }
        b->layout = lay;
        if (lay == HSIM_LAYOUT_REPLICA) {
            b->Rp = R > 32 ? (int32_t)((R + 63) / 64 * 64) : 32;
            // sites per wave of a tile: the full kRepSitesPerWave while the
            // largest colour phase has at least 2 blocks per CU; else 8, or 4
            // when 8 still gives fewer than 4 blocks per CU, so that small
            // lattices fill the GPU.  Measured on SC L^3 x 64 replicas (us per
            // phase): L = 56: 45.8 (32), 54.8 (16); L = 48: 37.4 (32), 34.0
            // (16), 28.1 (8); L = 32: 17.6 (16), 12.6 (8), 11.9 (4); 16 sites
            // per wave was never the best and is not used.  hsim_autotune
            // may pick another of these shapes.
            const int cus = device_cus() > 0 ? device_cus() : 256;
            int spw = hsim::kRepSitesPerWave;
            if (rep_phase_blocks(b, spw) < 2 * (int64_t)cus)
                for (int cand : {8, 4})
                    if (cand < spw && cand % hsim::kRepSitesPerStep == 0) {
                        spw = cand;
                        if (rep_phase_blocks(b, cand) >= 4 * (int64_t)cus) break;
                    }
            set_rep_tiles(b, spw);
        } else {
            b->spin_off.resize(R);
            int64_t off = 0;
            for (int r = 0; r < R; ++r) {
                b->spin_off[r] = off;
                off += 3 * pad64(plans[r]->n);
            }
            b->spin_elems = off;
            if (lay == HSIM_LAYOUT_SITE) {
                const int C = b->ncol_max;
                // trailing colour classes beyond the first two with fewer than
                // two tiles per CU run inside the per-replica finish launch
                // instead of a launch each (the extra colours of odd-size
                // films: a few tiles per film, latency-bound as phases)
                std::vector<int64_t> ct(C, 0);
                for (int r = 0; r < R; ++r)
                    for (int c = 0; c < plans[r]->ncol; ++c)
                        ct[c] += (plans[r]->cls_off[c + 1] - plans[r]->cls_off[c] + hsim::kSiteBlock - 1) /
                                 hsim::kSiteBlock;
                const int cus = device_cus() > 0 ? device_cus() : 256;
                b->c_tail = C;
                while (b->c_tail > 2 && ct[b->c_tail - 1] < 2 * cus) --b->c_tail;
                // two groups when both are non-empty
                for (int r = 0; r < R; ++r) b->grp_reps[plans[r]->ncol > b->c_tail ? 1 : 0].push_back(r);
                b->ngroups = (!b->grp_reps[0].empty() && !b->grp_reps[1].empty()) ? 2 : 1;
                if (b->ngroups == 1) {
                    b->grp_reps[0].clear();
                    b->grp_reps[1].clear();
                    for (int r = 0; r < R; ++r) b->grp_reps[0].push_back(r);
                }
                b->rep_tiles.assign((size_t)R * C * 2, 0);
                for (int g = 0; g < b->ngroups; ++g) {
                    b->gtile_off[g].assign(C + 1, 0);
                    b->gunits[g].assign(C, 0);
                    for (int c = 0; c < C; ++c) {
                        b->gtile_off[g][c] = (int32_t)b->tiles.size();
                        for (int r : b->grp_reps[g]) {
                            hsim_plan P = plans[r];
                            const int32_t t0 = (int32_t)b->tiles.size();
                            if (c < P->ncol) {
                                b->gunits[g][c] += P->cls_off[c + 1] - P->cls_off[c];
                                for (int32_t s = P->cls_off[c]; s < P->cls_off[c + 1]; s += hsim::kSiteBlock) {
                                    const int32_t e = std::min(s + hsim::kSiteBlock, P->cls_off[c + 1]);
                                    int32_t nsl = 0;   // slots past every row's end are padding
                                    for (int32_t t = s; t < e; ++t) nsl = std::max(nsl, P->rp[t + 1] - P->rp[t]);
                                    b->tiles.push_back({r, s, e, c, nsl});
                                }
                            }
                            b->rep_tiles[((size_t)r * C + c) * 2] = t0;
                            b->rep_tiles[((size_t)r * C + c) * 2 + 1] = (int32_t)b->tiles.size();
                        }
                    }
                    b->gtile_off[g][C] = (int32_t)b->tiles.size();
                }
                if (b->tiles.size() > (size_t)INT32_MAX / 2) throw Error(HSIM_E_UNSUPPORTED, "too many tiles");
            } else {
                b->lds = fits_lds;
                b->lds_bytes = (size_t)(3 * pad64(max_n)) * elem;
                int64_t th = std::max<int64_t>(64, (max_cls + 63) / 64 * 64);
                b->block_threads = (int)std::min<int64_t>(th, 1024);
            }
        }
    } catch (...) {
        delete b;
        throw;
    }
    return b;
}

void batch_sizes_impl(hsim_batch b, int32_t S, int32_t M, size_t *ws, size_t *sp, size_t *hist)
{
    if (!b || S < 1 || M < 1) throw Error(HSIM_E_ARG, "sizes: bad argument");
    if ((uint64_t)S * (uint64_t)M >= 0xFFFFFFFFull) throw Error(HSIM_E_ARG, "steps*mcs too large");
    size_t off = align_up(sizeof(hsim::Ctl));
    off += align_up((size_t)b->R * 8);                 // ecarry
    off += 2 * align_up((size_t)b->R * S * 8);         // beta, bfield
    off += align_up((size_t)b->R * 8);                 // adaptive widths
    size_t part = 0;
    if (b->layout == HSIM_LAYOUT_SITE) part = b->tiles.size() * hsim::kRecSite * 8;
    else if (b->layout == HSIM_LAYOUT_REPLICA)
        part = rep_rec_bytes_max(b) +
               (size_t)hsim::kMaxPersistentBlocks * 128;   // barrier flags, one 128-byte line each
    off += align_up(std::max<size_t>(part, 8));
    if (ws) *ws = off;
    const size_t elem = b->f64 ? 8 : 4;
    if (sp) {
        if (b->layout == HSIM_LAYOUT_REPLICA) *sp = (size_t)3 * b->plans[0]->n * b->Rp * 4;
        else *sp = (size_t)b->spin_elems * elem;
        if (*sp == 0) *sp = 16;
    }
    if (hist) *hist = (size_t)b->R * S * M * 5 * 8;
}

void hsim_batch_s::upload_tables()
{
    const size_t elem = f64 ? 8 : 4;
    if (nad.size() != (size_t)R) nad.assign((size_t)R, 0.0);
    d_nad.upload(nad);
    for (auto P : plans) P->upload_sweep();
    if (layout == HSIM_LAYOUT_REPLICA) {
        hsim_plan P = plans[0];
        std::vector<uint32_t> ids(Rp, 0);
        for (int r = 0; r < R; ++r) ids[r] = rep_id[r];
        d_rep_id.upload(ids);
        la.rp = (const int32_t *)P->d_rp.p;
        la.ci = (const int32_t *)P->d_ci.p;
        la.J = (const float *)P->d_Jf.p;
        la.type = (const int32_t *)P->d_type.p;
        la.kc = (const float *)P->d_kcf.p;
        la.mu = (const float *)P->d_muf.p;
        la.mu_d = (const double *)P->d_mud.p;
        la.ell_col = (const int32_t *)P->d_ell_col.p;
        la.ell_J = (const float *)P->d_ell_J.p;
        la.orig = (const uint32_t *)P->d_orig.p;
        la.k = (const float *)P->d_kf.p;
        la.ax = (const float *)P->d_axf.p;
        la.nd = (const float *)P->d_ndf.p;
        la.spins = (float *)spins;
        la.rep_id = (const uint32_t *)d_rep_id.p;
        la.k0 = (float)P->k0;
        la.e0x = (float)P->e0[0];
        la.e0y = (float)P->e0[1];
        la.e0z = (float)P->e0[2];
        la.n0x = (float)P->n0[0];
        la.n0y = (float)P->n0[1];
        la.n0z = (float)P->n0[2];
        la.n = (int32_t)P->n;
        la.Rp = Rp;
        la.R = R;
        // spin rows: component c of site i at c*cs + i*ss (interleaved while
        // the whole array stays below 2 GiB, so byte offsets fit 32 bits)
        const bool inter = HSIM_REP_INTERLEAVED && 3 * (int64_t)P->n * Rp * 4 < ((int64_t)1 << 31);
        la.ss = inter ? 3 * Rp : Rp;
        la.cs = inter ? (int64_t)Rp : (int64_t)P->n * Rp;
        la.ncol = P->ncol;
        la.ell_w = P->ell_w;
        for (int c = 0; c <= P->ncol; ++c) la.cls_off[c] = P->cls_off[c];
        if (tord.empty()) la.tord = nullptr;
        else {
            d_tord.upload(tord);
            la.tord = (const int32_t *)d_tord.p;
        }
    } else {
        reps.assign(R, hsim::RepDesc{});
        int64_t uoff = 0;
        for (int r = 0; r < R; ++r) {
            hsim_plan P = plans[r];
            hsim::RepDesc &d = reps[r];
            d.rp = (const int32_t *)P->d_rp.p;
            d.ci = (const int32_t *)P->d_ci.p;
            d.J = f64 ? P->d_Jd.p : P->d_Jf.p;
            d.orig = (const uint32_t *)P->d_orig.p;
            d.k = f64 ? P->d_kd.p : P->d_kf.p;
            d.ax = f64 ? P->d_axd.p : P->d_axf.p;
            d.nd = f64 ? P->d_ndd.p : P->d_ndf.p;
            d.spins = (char *)spins + spin_off[r] * elem;
            d.ell_w = P->ell_w;
            d.type = (const int32_t *)P->d_type.p;
            d.kc = f64 ? P->d_kcd.p : P->d_kcf.p;
            d.mu = f64 ? P->d_mud.p : P->d_muf.p;
            d.mu_d = (const double *)P->d_mud.p;
            d.ellT_col = (const int32_t *)P->d_ellT_col.p;
            d.ellT_J = f64 ? P->d_ellT_Jd.p : P->d_ellT_Jf.p;
            d.k0 = P->k0;
            for (int c = 0; c < 3; ++c) {
                d.e0[c] = P->e0[c];
                d.n0[c] = P->n0[c];
            }
            d.user_off = uoff;
            uoff += P->n;
            d.n = (int32_t)P->n;
            d.n_pad = (int32_t)pad64(P->n);
            d.rep_id = rep_id[r];
            d.ncol = P->ncol;
            for (int c = 0; c <= P->ncol; ++c) d.cls_off[c] = P->cls_off[c];
        }
        d_reps.upload(reps);
        if (layout == HSIM_LAYOUT_SITE) {
            d_tiles.upload(tiles);
            d_rep_tiles.upload(rep_tiles);
            for (int g = 0; g < ngroups; ++g) d_grp_reps[g].upload(grp_reps[g]);
        }
    }
    tables_on_device = true;
}

void batch_bind_impl(hsim_batch b, int32_t S, int32_t M, void *ws, void *spins, void *hist)
{
    if (!b || !ws || !spins || !hist) throw Error(HSIM_E_ARG, "bind: NULL buffer");
    b->drop_graph();
    size_t wsb = 0;
    batch_sizes_impl(b, S, M, &wsb, nullptr, nullptr);
    if (((uintptr_t)ws | (uintptr_t)spins | (uintptr_t)hist) % 16)
        throw Error(HSIM_E_ARG, "bind: buffers must be 16-byte aligned");
    b->S_hist = S;
    b->M = M;
    b->ws = (char *)ws;
    b->spins = spins;
    b->history = (double *)hist;
    b->ws_bytes = wsb;
    size_t off = align_up(sizeof(hsim::Ctl));
    b->off_ecarry = off;
    off += align_up((size_t)b->R * 8);
    b->off_beta = off;
    off += align_up((size_t)b->R * S * 8);
    b->off_bfield = off;
    off += align_up((size_t)b->R * S * 8);
    b->off_sigma = off;
    off += align_up((size_t)b->R * 8);
    b->off_part = off;
    b->h_beta.assign((size_t)b->R * S, 0.0);
    b->h_bfield.assign((size_t)b->R * S, 0.0);
    if (b->stage_done) {
        hip_check(hipEventSynchronize(b->stage_done), "hipEventSynchronize");
    } else {
        hip_check(hipEventCreateWithFlags(&b->stage_done, hipEventDisableTiming), "hipEventCreate");
    }
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    b->h_stage = nullptr;
    hip_check(hipHostMalloc((void **)&b->h_stage, 2 * (size_t)b->R * S * 8, hipHostMallocDefault),
              "hipHostMalloc");
    b->upload_tables();
    // clear the control block once (outside any graph)
    hip_check(hipMemset(ws, 0, align_up(sizeof(hsim::Ctl))), "hipMemset");
    b->bound = true;
    b->reset_sigma();
}

void hsim_batch_s::reset_sigma()
{
    if (!bound) return;
    std::vector<double> s0((size_t)R, sigma0);
    hip_check(hipMemcpy(ws + off_sigma, s0.data(), (size_t)R * 8, hipMemcpyHostToDevice), "hipMemcpy");
}

// Update policy per site type.  n_types == 0: the random move everywhere.
void batch_set_policies_impl(hsim_batch b, int32_t nt, const int32_t *policy, const double *param,
                             double smin, double smax)
{
    if (!b || nt < 0 || nt > hsim::kMaxTypes || (nt > 0 && (!policy || !param)))
        throw Error(HSIM_E_ARG, "set_policies: bad argument");
    hsim::Policies P{};
    P.n_types = nt;
    double s0 = 1.0;
    for (int t = 0; t < nt; ++t) {
        const int pol = policy[t];
        const double prm = param[t];
        if (pol < hsim::POL_RANDOM || pol > hsim::POL_ADAPTIVE)
            throw Error(HSIM_E_ARG, "set_policies: unknown policy");
        if ((pol == hsim::POL_SMALL_STEP || pol == hsim::POL_HN) && !(prm > 0.0 && prm <= M_PI))
            throw Error(HSIM_E_PARAM, "cap half-angle must be in (0, pi]");
        if ((pol == hsim::POL_GAUSSIAN || pol == hsim::POL_ADAPTIVE) && !(prm > 0.0 && std::isfinite(prm)))
            throw Error(HSIM_E_PARAM, "Gaussian width must be positive and finite");
        P.pol[t] = pol;
        P.param[t] = prm;
        P.cos_t[t] = std::cos(prm);
        if (pol == hsim::POL_ADAPTIVE && !P.adaptive) {
            P.adaptive = 1;
            s0 = prm;
        }
    }
    if (P.adaptive && !(smin > 0.0 && smax >= smin && std::isfinite(smax)))
        throw Error(HSIM_E_PARAM, "adaptive width bounds must satisfy 0 < min <= max");
    b->drop_graph();
    P.sigma_min = smin;
    P.sigma_max = smax;
    std::vector<double> nad((size_t)b->R, 0.0);
    for (int r = 0; r < b->R; ++r) {
        hsim_plan pl = b->plans[r];
        if (nt > 0)
            for (int64_t k = 0; k < pl->n; ++k) {
                const int ty = pl->type.empty() ? 0 : pl->type[k];
                if (ty >= nt) throw Error(HSIM_E_PARAM, "a site type has no policy");
                if (P.pol[ty] == hsim::POL_ADAPTIVE) nad[r] += 1.0;
            }
    }
    b->pol = P;
    b->nad.swap(nad);
    b->sigma0 = s0;
    if (b->bound) {
        b->upload_tables();
        b->reset_sigma();
    }
}

// Optional outputs: per-type magnetisation [R][S][M][n_types][3] and step-end
// spins [R][S][n_max][3] (device buffers of the caller; NULL: off).
void batch_bind_outputs_impl(hsim_batch b, int32_t n_types, double *type_mag, double *snapshots)
{
    if (!b) throw Error(HSIM_E_ARG, "bind_outputs: NULL batch");
    if (type_mag && (n_types < 1 || n_types > hsim::kMaxTypes))
        throw Error(HSIM_E_ARG, "bind_outputs: n_types must be 1..8");
    if (type_mag)
        for (auto p : b->plans)
            for (int32_t t : p->type)
                if (t >= n_types) throw Error(HSIM_E_PARAM, "a site type is beyond n_types");
    b->drop_graph();
    b->type_mag = type_mag;
    b->snapshots = snapshots;
    b->tm_types = type_mag ? n_types : 0;
    b->d_tm_part.release();
    if (type_mag) {
        int64_t mn = 0;
        for (auto p : b->plans) mn = std::max(mn, p->n);
        const int nblk = hsim::type_part_blocks(b->layout == HSIM_LAYOUT_REPLICA, (int)mn);
        b->d_tm_part.alloc((size_t)b->R * nblk * n_types * 3 * 8);
    }
}

void batch_sigma_impl(hsim_batch b, double *out)
{
    if (!b || !out) throw Error(HSIM_E_ARG, "sigma: NULL argument");
    if (!b->bound) throw Error(HSIM_E_STATE, "sigma before bind");
    hip_check(hipMemcpy(out, b->ws + b->off_sigma, (size_t)b->R * 8, hipMemcpyDeviceToHost), "hipMemcpy");
}

hsim::RunArgs hsim_batch_s::run_args(uint32_t g0, int n_mcs, int P, uint32_t *trace)
{
    hsim::RunArgs a{};
    a.ctl = (hsim::Ctl *)ws;
    a.beta = (const double *)(ws + off_beta);
    a.bfield = (const double *)(ws + off_bfield);
    a.ecarry = (double *)(ws + off_ecarry);
    a.partials = (double *)(ws + off_part);
    if (layout == HSIM_LAYOUT_REPLICA) {
        a.chunks = a.partials + (size_t)rec_win * rep_ntiles * hsim::kRecFields * Rp;
        a.carry = a.chunks + (size_t)rec_win * hsim::kChunks * 6 * Rp;
        a.sig_part = a.carry + (size_t)rec_win * 6 * Rp;
    }
    a.rec_win = rec_win;
    a.pol = pol;
    a.type_mag = type_mag;
    a.tm_part = (double *)d_tm_part.p;
    a.tm_types = tm_types;
    a.snapshots = snapshots;
    {
        int64_t mn = 0;
        for (auto p : plans) mn = std::max(mn, p->n);
        a.snap_n = (int32_t)mn;
    }
    a.sigma = (double *)(ws + off_sigma);
    a.n_ad = (const double *)d_nad.p;
    a.history = history;
    a.trace = trace;
    a.seed = seed;
    a.g0 = g0;
    a.M = M;
    a.S_hist = S_hist;
    a.P = P;
    a.n_mcs_run = n_mcs;
    int64_t maxn = 0;
    for (auto p : plans) maxn = std::max(maxn, p->n);
    a.trace_words = (int32_t)((maxn + 31) / 32);
    a.R = R;
    return a;
}

void batch_init_impl(hsim_batch b, int32_t mode, const double *host, hipStream_t st)
{
    if (!b) throw Error(HSIM_E_ARG, "init: NULL batch");
    if (!b->bound) throw Error(HSIM_E_STATE, "init before bind");
    if (mode != HSIM_INIT_GIVEN && mode != HSIM_INIT_COLD_Z && mode != HSIM_INIT_RANDOM)
        throw Error(HSIM_E_ARG, "bad init mode");
    hsim::DevBuf given;
    if (mode == HSIM_INIT_GIVEN) {
        if (!host) throw Error(HSIM_E_ARG, "init: GIVEN needs host spins");
        const size_t cnt = (size_t)b->total_sites * 3;
        for (size_t t = 0; t < cnt; ++t)
            if (!std::isfinite(host[t])) throw Error(HSIM_E_PARAM, "non-finite initial spin");
        given.alloc(cnt * 8);
        hip_check(hipMemcpy(given.p, host, cnt * 8, hipMemcpyHostToDevice), "hipMemcpy");
    }
    if (b->total_sites == 0) return;   // lattices without sites: nothing to set
    if (b->layout == HSIM_LAYOUT_REPLICA) {
        hip_check(hsim::launch_init_spins_rep(st, b->la, mode, (const double *)given.p, b->seed),
                  "init launch");
    } else {
        int64_t maxn = 1;
        for (auto p : b->plans) maxn = std::max(maxn, p->n);
        hip_check(hsim::launch_init_spins(st, b->f64, (const hsim::RepDesc *)b->d_reps.p, b->R,
                                          (int)maxn, mode, (const double *)given.p, nullptr, b->seed),
                  "init launch");
    }
    if (given.p) hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
}

int64_t hsim_batch_s::phase_updates(int colour) const
{
    int64_t u = 0;
    if (layout == HSIM_LAYOUT_REPLICA) {
        const hsim_plan P = plans[0];
        if (colour < P->ncol) u = (int64_t)(P->cls_off[colour + 1] - P->cls_off[colour]) * R;
    } else {
        for (auto P : plans)
            if (colour < P->ncol) u += P->cls_off[colour + 1] - P->cls_off[colour];
    }
    return u;
}

namespace {

// Event pair around one colour-phase launch when this MCS is sampled.
struct PhaseTimer {
    hsim_batch b;
    hipStream_t st;
    hipEvent_t e1 = nullptr;
    int64_t units = 0;
    PhaseTimer(hsim_batch b_, hipStream_t st_, bool on, int colour, int64_t units_ = -1)
        : b(b_), st(st_)
    {
        if (!on) return;
        if (b->ev_used + 2 > b->ev_pool.size()) {
            for (int k = 0; k < 64; ++k) {
                hipEvent_t e;
                // timing only: no cache write-back/invalidate around the kernel
                hip_check(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreate");
                b->ev_pool.push_back(e);
            }
        }
        hipEvent_t e0 = b->ev_pool[b->ev_used++];
        e1 = b->ev_pool[b->ev_used++];
        units = units_ >= 0 ? units_ : b->phase_updates(colour);
        hip_check(hipEventRecord(e0, st), "hipEventRecord");
    }
    ~PhaseTimer() noexcept(false)
    {
        if (!e1) return;
        hip_check(hipEventRecord(e1, st), "hipEventRecord");
        b->ev_units.push_back(units);
    }
};

// Site layout: MCS t_off = 0..count-1 of a launch sequence starting at
// ctl->g (efull, colour phases, per-MCS reduction), then ctl->g moves on.
// Optional outputs after MCS t of a sequence: per-type magnetisation; the
// spins at a step end, which the host knows from the sequence's first MCS gb
// (plain launches) or the device checks (dev_check: captured graphs).
void enqueue_outputs(hsim_batch b, const hsim::RunArgs &ra, int t, uint32_t gb, bool dev_check,
                     hipStream_t st)
{
    const bool rep = b->layout == HSIM_LAYOUT_REPLICA;
    const auto *reps = (const hsim::RepDesc *)b->d_reps.p;
    if (b->type_mag) {
        if (rep) hip_check(hsim::launch_type_mag_rep(st, b->la, t, ra), "type launch");
        else hip_check(hsim::launch_type_mag_site(st, b->f64, reps, b->R, ra.snap_n, t, ra), "type launch");
    }
    if (b->snapshots && (dev_check || (gb + (uint32_t)t + 1) % (uint32_t)ra.M == 0)) {
        if (rep) hip_check(hsim::launch_snapshot_rep(st, b->la, t, dev_check, ra), "snapshot launch");
        else hip_check(hsim::launch_snapshot_site(st, b->f64, reps, b->R, ra.snap_n, t, dev_check, ra),
                       "snapshot launch");
    }
}

// Site layout, one group's MCS t of a sequence: the energy recompute when
// due, the colour phases below c_tail, the finish launch (trailing classes
// and history) of the group's replicas.
template <typename F>
void enqueue_site_mcs(hsim_batch b, const hsim::RunArgs &ra, int g, int t, F efull_mask, hipStream_t st)
{
    const auto *reps = (const hsim::RepDesc *)b->d_reps.p;
    const auto *tiles = (const hsim::Tile *)b->d_tiles.p;
    const std::vector<int32_t> &to = b->gtile_off[g];
    const int C = b->ncol_max;
    if (efull_mask(t))
        hip_check(hsim::launch_site_efull(st, b->f64, b->kmode, b->fmode, reps, tiles, to[0], to[C] - to[0],
                                          t, ra),
                  "efull launch");
    const bool timed = b->time_every > 0 && t % b->time_every == 0;
    for (int c = 0; c < b->c_tail; ++c) {
        PhaseTimer pt(b, st, timed && to[c + 1] > to[c], c, b->gunits[g][c]);
        hip_check(hsim::launch_site_phase(st, b->f64, b->kmode, b->fmode, ra.trace != nullptr, b->ellw, reps,
                                          tiles, to[c], to[c + 1] - to[c], t, ra),
                  "phase launch");
    }
    hip_check(hsim::launch_site_finish(st, b->f64, b->kmode, b->fmode, ra.trace != nullptr, b->ellw, reps,
                                       (const int32_t *)b->d_rep_tiles.p,
                                       b->ngroups > 1 ? (const int32_t *)b->d_grp_reps[g].p : nullptr,
                                       (int)b->grp_reps[g].size(), b->ncol_max, b->c_tail, t, ra),
              "finish launch");
}

// Site layout: MCS t_off = 0..count-1 of a launch sequence starting at
// ctl->g, then ctl->g moves on.  With two groups and no per-MCS outputs the
// groups run their sequences on the batch's two streams, forked from st and
// joined back into it (also inside a capture, where the fork and join become
// graph edges); otherwise both groups' launches go to st, MCS by MCS.
// Optional outputs after MCS t of a sequence: per-type magnetisation; the
// spins at a step end, which the host knows from the sequence's first MCS gb
// (plain launches) or the device checks (dev_check: captured graphs).
template <typename F>
void enqueue_site_sequence(hsim_batch b, const hsim::RunArgs &ra, int count, F efull_mask,
                           hipStream_t st, uint32_t gb, bool dev_check, bool split)
{
    if (count <= 0) return;
    if (split && b->ngroups > 1) {
        if (!b->gfork) {
            hip_check(hipEventCreateWithFlags(&b->gfork, hipEventDisableTiming), "hipEventCreate");
            for (int g = 0; g < 2; ++g) {
                hip_check(hipEventCreateWithFlags(&b->gjoin[g], hipEventDisableTiming), "hipEventCreate");
                hip_check(hipStreamCreateWithFlags(&b->gstream[g], hipStreamNonBlocking), "hipStreamCreate");
            }
        }
        hip_check(hipEventRecord(b->gfork, st), "hipEventRecord");
        for (int g = 0; g < 2; ++g) {
            hip_check(hipStreamWaitEvent(b->gstream[g], b->gfork, 0), "hipStreamWaitEvent");
            for (int t = 0; t < count; ++t) enqueue_site_mcs(b, ra, g, t, efull_mask, b->gstream[g]);
            hip_check(hipEventRecord(b->gjoin[g], b->gstream[g]), "hipEventRecord");
            hip_check(hipStreamWaitEvent(st, b->gjoin[g], 0), "hipStreamWaitEvent");
        }
    } else {
        for (int t = 0; t < count; ++t) {
            for (int g = 0; g < b->ngroups; ++g) enqueue_site_mcs(b, ra, g, t, efull_mask, st);
            enqueue_outputs(b, ra, t, gb, dev_check, st);
        }
    }
    hip_check(hsim::launch_ctl_advance(st, ra.ctl, (uint32_t)count), "control launch");
}

// Replica layout: MCS t_off = 0..count-1 of a launch sequence starting at
// ctl->g.  Records of MCS t go to slot t % rec_win; each full window (and the
// last, partial one) is reduced by its own two launches, the last of which
// also moves ctl->g on.  efull_mask(t): whether MCS t may need the energy
// recompute.
template <typename F>
void enqueue_rep_sequence(hsim_batch b, const hsim::RunArgs &ra, int count, F efull_mask,
                          hipStream_t st, uint32_t gb, bool dev_check)
{
    const int W = b->rec_win;
    for (int t = 0; t < count; ++t) {
        if (efull_mask(t))
            hip_check(hsim::launch_rep_efull(st, b->kmode, b->fmode, b->la, b->rep_ntiles, t, ra),
                      "efull launch");
        const bool timed = b->time_every > 0 && t % b->time_every == 0;
        for (int c = 0; c < b->la.ncol; ++c) {
            PhaseTimer pt(b, st, timed, c);
            hip_check(hsim::launch_rep_phase(st, b->kmode, b->fmode, c, t, b->la, b->rep_ntiles, ra),
                      "phase launch");
        }
        if (ra.pol.adaptive)
            hip_check(hsim::launch_rep_sigma(st, b->la, b->rep_ntiles, t, ra), "sigma launch");
        enqueue_outputs(b, ra, t, gb, dev_check, st);
        if ((t + 1) % W == 0 || t == count - 1) {
            const int first = t - t % W;
            hip_check(hsim::launch_rep_reduce(st, b->la, b->rep_ntiles, first, t - first + 1,
                                              t == count - 1 ? count : 0, ra),
                      "reduce launch");
        }
    }
}

bool due(uint32_t g, int M, int P)
{
    const uint32_t m = g % (uint32_t)M;
    return m == 0 || (P > 0 && m % (uint32_t)P == 0);
}

// Whether the site layout's groups may run on the batch's own streams: two
// groups, no per-MCS outputs (they read every replica after each MCS), and st
// not recording into a caller's graph (the library's own capture, in
// run_graph, forks and joins its streams inside the capture).
bool split_ok(hsim_batch b, hipStream_t st, bool own_capture)
{
    if (b->ngroups < 2 || b->type_mag || b->snapshots) return false;
    if (own_capture || st == nullptr) return true;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hip_check(hipStreamIsCapturing(st, &cs), "hipStreamIsCapturing");
    return cs == hipStreamCaptureStatusNone;
}

void run_plain(hsim_batch b, const hsim::RunArgs &ra, hipStream_t st, int from, int to)
{
    // ctl->g is at g0 + from here
    const uint32_t gb = ra.g0 + (uint32_t)from;
    auto mask = [&](int t) { return due(gb + (uint32_t)t, ra.M, ra.P); };
    if (b->layout == HSIM_LAYOUT_REPLICA) enqueue_rep_sequence(b, ra, to - from, mask, st, gb, false);
    else enqueue_site_sequence(b, ra, to - from, mask, st, gb, false, split_ok(b, st, false));
}

// Whether work enqueued on st is being recorded into a caller's graph.
bool capturing(hipStream_t st)
{
    if (st == nullptr) return false;   // the legacy stream cannot be captured
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hip_check(hipStreamIsCapturing(st, &cs), "hipStreamIsCapturing");
    return cs != hipStreamCaptureStatusNone;
}

// GRAPH mode: one recompute period (U MCS) captured once and replayed; the
// instantiated graph stays on the batch while its captured arguments stay the
// same (rebinding, new policies or outputs drop it).  Nothing synchronises:
// the capture runs on a private stream where nothing executes, and the
// replays are enqueued on the caller's stream.
void run_graph(hsim_batch b, const hsim::RunArgs &ra, hipStream_t st)
{
    const int total = ra.n_mcs_run;
    if (capturing(st)) {   // inside a caller's capture: plain launches become its nodes
        run_plain(b, ra, st, 0, total);
        return;
    }
    int U;
    bool efull_each;
    if (ra.P > 0 && ra.M % ra.P == 0 && ra.P <= 512) {
        U = ra.P;
        efull_each = false;
    } else {
        U = std::min(ra.M, 64);
        efull_each = true;
    }
    const int reps = total / U;
    if (reps < 2) {
        run_plain(b, ra, st, 0, total);
        return;
    }
    // the first MCS and the run length index only the accept trace; without
    // it they are left out of the captured arguments, so later calls reuse
    // the graph
    hsim::RunArgs rc = ra;
    if (!rc.trace) {
        rc.g0 = 0;
        rc.n_mcs_run = 0;
    }
    std::vector<unsigned char> key(sizeof rc + sizeof b->la + 2 * sizeof(int));
    const int fe = efull_each ? 1 : 0;
    std::memcpy(key.data(), &rc, sizeof rc);
    std::memcpy(key.data() + sizeof rc, &b->la, sizeof b->la);
    std::memcpy(key.data() + sizeof rc + sizeof b->la, &U, sizeof U);
    std::memcpy(key.data() + sizeof rc + sizeof b->la + sizeof U, &fe, sizeof fe);
    if (!b->g_exec || key != b->g_key) {
        b->drop_graph();
        if (!b->g_cap) hip_check(hipStreamCreateWithFlags(&b->g_cap, hipStreamNonBlocking), "hipStreamCreate");
        if (!b->g_done) hip_check(hipEventCreateWithFlags(&b->g_done, hipEventDisableTiming), "hipEventCreate");
        hipGraph_t graph = nullptr;
        hip_check(hipStreamBeginCapture(b->g_cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        try {
            auto mask = [&](int t) { return efull_each || t == 0; };
            if (b->layout == HSIM_LAYOUT_REPLICA) enqueue_rep_sequence(b, rc, U, mask, b->g_cap, 0, true);
            else enqueue_site_sequence(b, rc, U, mask, b->g_cap, 0, true, split_ok(b, b->g_cap, true));
        } catch (...) {
            (void)hipStreamEndCapture(b->g_cap, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        hip_check(hipStreamEndCapture(b->g_cap, &graph), "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            hip_check(e, "hipGraphInstantiate");
        }
        b->g_graph = graph;
        b->g_exec = exec;
        b->g_key.swap(key);
    }
    for (int k = 0; k < reps; ++k) hip_check(hipGraphLaunch(b->g_exec, st), "hipGraphLaunch");
    hip_check(hipEventRecord(b->g_done, st), "hipEventRecord");
    run_plain(b, ra, st, reps * U, total);
}

bool run_persistent(hsim_batch b, const hsim::RunArgs &ra, hipStream_t st, uint32_t spin_cap)
{
    const int bpc = hsim::rep_persistent_blocks_per_cu(b->kmode, b->fmode, b->Rp % 64 == 0 ? 64 : 32, b->la.ell_w);
    const int cus = device_cus();
    if (bpc <= 0 || cus <= 0) return false;
    const int groups = b->Rp / (b->Rp % 64 == 0 ? 64 : 32);
    int grid = b->persistent_grid > 0 ? b->persistent_grid : bpc * cus;
    grid = std::min(grid, bpc * cus);   // every block must be resident at once
    int max_phase_tiles = 1;            // more blocks than tiles of a phase would only wait
    for (int c = 0; c < b->la.ncol; ++c)
        max_phase_tiles = std::max(max_phase_tiles, b->la.tile_off[c + 1] - b->la.tile_off[c]);
    grid = std::min(grid, max_phase_tiles * groups);
    grid = std::min(grid, hsim::kMaxPersistentBlocks - hsim::kXBarLines);
    // barrier flags follow the record window
    auto *flags = (uint32_t *)(b->ws + b->off_part + rep_rec_bytes_max(b));
    hip_check(hsim::launch_rep_persistent(st, b->kmode, b->fmode, b->la, b->rep_ntiles, grid, ra,
                                          flags, spin_cap),
              "persistent launch");
    return true;
}

}  // namespace

void batch_run_impl(hsim_batch b, int32_t first_step, int32_t n_steps, const double *T,
                    const double *B, int32_t P, hsim_launch launch, uint32_t flags,
                    uint32_t *trace, hipStream_t st)
{
    if (!b) throw Error(HSIM_E_ARG, "run: NULL batch");
    if (!b->bound) throw Error(HSIM_E_STATE, "run before bind");
    if (first_step < 0 || n_steps < 0 || first_step + n_steps > b->S_hist)
        throw Error(HSIM_E_ARG, "run: steps outside the bound history");
    if (n_steps > 0 && (!T || !B)) throw Error(HSIM_E_ARG, "run: NULL schedule");
    if (P < 0) throw Error(HSIM_E_ARG, "run: negative recompute period");
    if (launch < HSIM_LAUNCH_PLAIN || launch > HSIM_LAUNCH_AUTO) throw Error(HSIM_E_ARG, "bad launch mode");
    const bool want_trace = (flags & HSIM_RUN_TRACE_ACCEPTS) != 0;
    if (want_trace && !trace) throw Error(HSIM_E_ARG, "run: trace requested without a buffer");
    if (want_trace && b->layout == HSIM_LAYOUT_REPLICA) {
        bool xt = b->pol.n_types > 0;
        for (auto p : b->plans) xt |= !p->kcd.empty() || !p->mud.empty();
        if (xt)
            throw Error(HSIM_E_UNSUPPORTED,
                        "accept trace in the replica layout: not with update policies, cubic terms or spin norms");
    }
    for (int r = 0; r < b->R; ++r)
        for (int s = 0; s < n_steps; ++s) {
            const double t = T[(size_t)r * n_steps + s], f = B[(size_t)r * n_steps + s];
            if (!(t >= 0.0)) throw Error(HSIM_E_PARAM, "temperature must be >= 0");
            if (!std::isfinite(f)) throw Error(HSIM_E_PARAM, "non-finite field");
            const size_t k = (size_t)r * b->S_hist + first_step + s;
            b->h_beta[k] = t > 0.0 ? 1.0 / t : std::numeric_limits<double>::infinity();
            b->h_bfield[k] = (flags & HSIM_RUN_DEBUG_NAN_FIELD)
                                 ? std::numeric_limits<double>::quiet_NaN() : f;
        }
    if (n_steps == 0) return;
    const bool cap = capturing(st);
    if (!cap) {
        const size_t half = (size_t)b->R * b->S_hist;
        hip_check(hipEventSynchronize(b->stage_done), "hipEventSynchronize");
        std::memcpy(b->h_stage, b->h_beta.data(), half * 8);
        std::memcpy(b->h_stage + half, b->h_bfield.data(), half * 8);
        hip_check(hipMemcpyAsync(b->ws + b->off_beta, b->h_stage, half * 8, hipMemcpyHostToDevice, st),
                  "hipMemcpyAsync");
        hip_check(hipMemcpyAsync(b->ws + b->off_bfield, b->h_stage + half, half * 8,
                                 hipMemcpyHostToDevice, st),
                  "hipMemcpyAsync");
        hip_check(hipEventRecord(b->stage_done, st), "hipEventRecord");
    } else {
        // recorded into a caller's graph: this run's schedule travels in the
        // arguments of small kernels, so every replay writes the same values
        // and no host buffer has to outlive the graph
        const int cnt_all = b->R * n_steps;
        for (int k0 = 0; k0 < cnt_all; k0 += hsim::kPutPairs) {
            const int cnt = std::min(hsim::kPutPairs, cnt_all - k0);
            hsim::PutPairs v{};
            for (int j = 0; j < cnt; ++j) {
                const int k = k0 + j, r = k / n_steps, s = k % n_steps;
                const size_t off = (size_t)r * b->S_hist + first_step + s;
                v.v[2 * j] = b->h_beta[off];
                v.v[2 * j + 1] = b->h_bfield[off];
            }
            hip_check(hsim::launch_put_schedule(st, (double *)(b->ws + b->off_beta),
                                                (double *)(b->ws + b->off_bfield), b->S_hist,
                                                first_step, n_steps, k0, cnt, v),
                      "schedule launch");
        }
    }

    const uint32_t g0 = (uint32_t)first_step * (uint32_t)b->M;
    const int n_mcs = n_steps * b->M;
    if (b->total_sites == 0) {
        // lattices without sites: every record of the run is E = M = accepted = 0
        // (and every per-type magnetisation)
        const size_t rows = (size_t)n_steps * b->M;
        for (int r = 0; r < b->R; ++r) {
            const size_t row0 = ((size_t)r * b->S_hist + first_step) * b->M;
            // a fill kernel, not a memset: callers may capture runs in graphs
            hip_check(hsim::launch_fill_u32(st, (uint32_t *)(b->history + row0 * 5), 0u,
                                            (int64_t)(rows * 5 * 2)),
                      "fill launch");
            if (b->type_mag)
                hip_check(hsim::launch_fill_u32(st, (uint32_t *)(b->type_mag + row0 * b->tm_types * 3), 0u,
                                                (int64_t)(rows * b->tm_types * 3 * 2)),
                          "fill launch");
        }
        return;
    }
    const hsim::RunArgs ra = b->run_args(g0, n_mcs, P, want_trace ? trace : nullptr);
    hip_check(hsim::launch_ctl_set(st, ra.ctl, g0), "control launch");

    if (b->layout == HSIM_LAYOUT_BLOCK) {
        hip_check(hsim::launch_block_sweep(st, b->f64, b->kmode, b->fmode, want_trace, b->ellw, b->lds,
                                           b->block_threads, b->lds_bytes,
                                           (const hsim::RepDesc *)b->d_reps.p, ra),
                  "block sweep launch");
        return;
    }
    int mode = launch;
    if (mode == HSIM_LAUNCH_AUTO) {
        if (b->tuned_launch >= 0) mode = b->tuned_launch;
        else mode = HSIM_LAUNCH_GRAPH;
    }
    // the persistent kernel runs the random move of the plain model without
    // optional outputs: with update policies, cubic constants, spin norms,
    // outputs bound or an accept trace the same sweep runs as plain launches
    bool xt = false;
    for (auto p : b->plans) xt |= !p->kcd.empty() || !p->mud.empty();
    if (mode == HSIM_LAUNCH_PERSISTENT &&
        (b->pol.n_types > 0 || xt || b->type_mag || b->snapshots || want_trace))
        mode = HSIM_LAUNCH_PLAIN;
    if (mode == HSIM_LAUNCH_PERSISTENT) {
        if (b->layout != HSIM_LAYOUT_REPLICA)
            throw Error(HSIM_E_UNSUPPORTED, "persistent launch needs the replica layout");
        if (!run_persistent(b, ra, st, (flags & HSIM_RUN_DEBUG_WAIT_CAP) ? 1u : 1u << 24))
            throw Error(HSIM_E_UNSUPPORTED, "persistent launch cannot be made co-resident");
        return;
    }
    if (cap) {
        // recorded into a caller's graph: plain launches without the sampled
        // phase timer (its events would become graph nodes)
        const int every = b->time_every;
        b->time_every = 0;
        try {
            run_plain(b, ra, st, 0, n_mcs);
        } catch (...) {
            b->time_every = every;
            throw;
        }
        b->time_every = every;
        return;
    }
    if (mode == HSIM_LAUNCH_GRAPH && b->time_every == 0) run_graph(b, ra, st);
    else run_plain(b, ra, st, 0, n_mcs);
}

void batch_to_user_impl(hsim_batch b, int32_t rep, double *out, hipStream_t st)
{
    if (!b || rep < 0 || rep >= b->R) throw Error(HSIM_E_ARG, "spins_to_user: bad argument");
    if (!b->bound) throw Error(HSIM_E_STATE, "spins_to_user before bind");
    if (b->plans[rep]->n == 0) return;
    if (!out) throw Error(HSIM_E_ARG, "spins_to_user: NULL out");
    if (b->layout == HSIM_LAYOUT_REPLICA)
        hip_check(hsim::launch_to_user_rep(st, b->la, rep, out), "to_user launch");
    else
        hip_check(hsim::launch_to_user(st, b->f64, (const hsim::RepDesc *)b->d_reps.p, rep,
                                       (int)b->plans[rep]->n, out),
                  "to_user launch");
}

int32_t batch_status_impl(hsim_batch b)
{
    if (!b || !b->bound) throw Error(HSIM_E_STATE, "status before bind");
    uint32_t s = 0;
    auto *ctl = (hsim::Ctl *)b->ws;
    hip_check(hipMemcpy(&s, &ctl->status, 4, hipMemcpyDeviceToHost), "hipMemcpy");
    const uint32_t z = 0;
    hip_check(hipMemcpy(&ctl->status, &z, 4, hipMemcpyHostToDevice), "hipMemcpy");
    if (s & 2u) return HSIM_E_TIMEOUT;
    if (s & 1u) return HSIM_E_NUMERIC;
    return 0;
}

// ---------------------------------------------------------------- autotune
// Times the launch modes (and persistent grid sizes) available for this
// batch on trial_mcs MCS of a scratch binding, restores the spins, and keeps
// the fastest choice for HSIM_LAUNCH_AUTO.  Every candidate runs the same
// per-site update and the same reduction order, so the choice changes
// neither spins nor history.

namespace {

std::string tune_key(hsim_batch b)
{
    int dev = 0, rt = 0, drv = 0;
    hipDeviceProp_t prop{};
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&prop, dev);
    (void)hipRuntimeGetVersion(&rt);
    (void)hipDriverGetVersion(&drv);
    std::ostringstream k;
    k << prop.gcnArchName << ":" << prop.multiProcessorCount << ":rt" << rt << ":drv" << drv
      << ":L" << b->layout << ":R" << b->R << ":P" << (b->f64 ? 64 : 32) << ":pol";
    const unsigned char *pb = (const unsigned char *)&b->pol;
    uint64_t ph = 1469598103934665603ull;
    for (size_t q = 0; q < sizeof b->pol; ++q) {
        ph ^= pb[q];
        ph *= 1099511628211ull;
    }
    k << std::hex << ph << std::dec;
    for (auto p : b->plans) {
        k << ":" << std::hex << p->hash << std::dec << "/" << (p->kcd.empty() ? 0 : 1)
          << (p->mud.empty() ? 0 : 1) << (p->type.empty() ? 0 : 1);
        if (b->layout == HSIM_LAYOUT_REPLICA) break;
    }
    return k.str();
}

}  // namespace

void autotune_impl(hsim_batch b, const char *cache_path, int32_t trial_mcs, hipStream_t st)
{
    if (!b) throw Error(HSIM_E_ARG, "autotune: NULL batch");
    if (!b->bound) throw Error(HSIM_E_STATE, "autotune before bind");
    if (trial_mcs < 1) throw Error(HSIM_E_ARG, "autotune: trial_mcs must be >= 1");
    if (b->layout == HSIM_LAYOUT_BLOCK) return;   // a single launch: nothing to choose
    const std::string key = tune_key(b);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k;
            int mode = 0, grid = 0, spw = 0, masked = 0;
            if (!(ls >> k >> mode >> grid >> spw >> masked) || k != key) continue;
            bool ok_spw = false;
            for (int c : hsim::kRepTileShapes) ok_spw |= c == spw;
            if (b->layout == HSIM_LAYOUT_REPLICA && ok_spw) {
                set_rep_tiles(b, spw);
                b->la.masked_store = masked ? 1 : 0;
            }
            b->tuned_launch = mode;
            b->persistent_grid = grid;
            return;
        }
    }
    // scratch binding: one step of trial_mcs MCS
    size_t wsb = 0, spb = 0, hb = 0;
    batch_sizes_impl(b, 1, trial_mcs, &wsb, &spb, &hb);
    hsim::DevBuf ws, hist, saved;
    ws.alloc(wsb);
    hist.alloc(hb);
    saved.alloc(spb);
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    hip_check(hipMemcpy(saved.p, b->spins, spb, hipMemcpyDeviceToDevice), "hipMemcpy");
    // keep the caller's binding, adaptive widths, outputs and phase timing to
    // restore them afterwards; the trial runs write none of the caller's outputs
    std::vector<double> sig0((size_t)b->R);
    hip_check(hipMemcpy(sig0.data(), b->ws + b->off_sigma, (size_t)b->R * 8, hipMemcpyDeviceToHost),
              "hipMemcpy");
    hsim::Ctl ctl0{};   // status flags of the caller's earlier runs
    hip_check(hipMemcpy(&ctl0, b->ws, sizeof(hsim::Ctl), hipMemcpyDeviceToHost), "hipMemcpy");
    double *tm0 = b->type_mag, *snap0 = b->snapshots;
    const int32_t every0 = b->time_every;
    b->type_mag = nullptr;
    b->snapshots = nullptr;
    b->time_every = 0;
    const int32_t S0 = b->S_hist, M0 = b->M;
    char *ws0 = b->ws;
    void *sp0 = b->spins;
    double *h0 = b->history;
    const std::vector<double> beta0 = b->h_beta, bf0 = b->h_bfield;
    std::vector<double> T(b->R), B(b->R);
    for (int r = 0; r < b->R; ++r) {
        const double be = beta0.empty() ? 1.0 : beta0[(size_t)r * S0];
        T[r] = (be > 0.0 && std::isfinite(be)) ? 1.0 / be : 1.0;
        B[r] = bf0.empty() ? 0.0 : bf0[(size_t)r * S0];
    }
    // replica layout: first the tile shape and store policy with plain
    // launches, then the launch mode for the chosen shape
    struct Cand { int mode, grid, spw, masked; };
    const int spw0 = b->la.spw, masked0 = b->la.masked_store;
    std::vector<Cand> shapes = {{HSIM_LAUNCH_PLAIN, 0, spw0, masked0}};
    if (b->layout == HSIM_LAYOUT_REPLICA)
        for (int spw : hsim::kRepTileShapes)
            for (int m : {0, 1})
                if (spw != spw0 || m != masked0) shapes.push_back({HSIM_LAUNCH_PLAIN, 0, spw, m});
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    Cand win = shapes[0];
    std::string err;
    // recompute period of the trials: half the trial, so that a graph launch
    // is captured once and replayed twice, as in a run of many MCS
    const int32_t p_trial = std::max(1, trial_mcs / 2);
    auto time_cand = [&](const Cand &c) -> float {
        if (b->layout == HSIM_LAYOUT_REPLICA && (c.spw != b->la.spw)) set_rep_tiles(b, c.spw);
        b->la.masked_store = c.masked;
        b->persistent_grid = c.grid;
        float ms_best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            hip_check(hipMemcpyAsync(b->spins, saved.p, spb, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
            hip_check(hipEventRecord(e0, st), "hipEventRecord");
            batch_run_impl(b, 0, 1, T.data(), B.data(), p_trial, (hsim_launch)c.mode, 0, nullptr, st);
            hip_check(hipEventRecord(e1, st), "hipEventRecord");
            hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.0f;
            hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            ms_best = std::min(ms_best, ms);
        }
        if (batch_status_impl(b) != 0) return 1e30f;   // a timed-out barrier disqualifies
        return ms_best;
    };
    try {
        batch_bind_impl(b, 1, trial_mcs, ws.p, b->spins, hist.p);
        // another choice must beat the current one by more than timing noise
        float best = time_cand(shapes[0]);
        for (size_t q = 1; q < shapes.size(); ++q) {
            const float ms = time_cand(shapes[q]);
            if (ms < 0.98f * best) {
                best = ms;
                win = shapes[q];
            }
        }
        std::vector<Cand> modes = {{HSIM_LAUNCH_GRAPH, 0, win.spw, win.masked}};
        if (b->layout == HSIM_LAYOUT_REPLICA) {
            const int bpc = hsim::rep_persistent_blocks_per_cu(b->kmode, b->fmode, b->Rp % 64 == 0 ? 64 : 32, b->la.ell_w);
            const int cus = device_cus();
            for (int f : {1, 2, 4, 8})
                if (bpc >= f && cus > 0) modes.push_back({HSIM_LAUNCH_PERSISTENT, f * cus, win.spw, win.masked});
        }
        const float plain_ms = best;
        for (const Cand &c : modes) {
            const float ms = time_cand(c);
            if (ms < best && ms < 0.98f * plain_ms) {
                best = ms;
                win = c;
            }
        }
    } catch (const std::exception &e) {
        err = e.what();
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the chosen tile shape and store policy (the original ones after an error)
    if (b->layout == HSIM_LAYOUT_REPLICA) {
        const int spw = err.empty() ? win.spw : spw0, masked = err.empty() ? win.masked : masked0;
        if (spw != b->la.spw) set_rep_tiles(b, spw);
        b->la.masked_store = masked;
    }
    // restore spins, the caller's binding, widths, outputs and timing
    b->type_mag = tm0;
    b->snapshots = snap0;
    b->time_every = every0;
    hip_check(hipMemcpy(sp0, saved.p, spb, hipMemcpyDeviceToDevice), "hipMemcpy");
    batch_bind_impl(b, S0, M0, ws0, sp0, h0);
    hip_check(hipMemcpy(b->ws + b->off_sigma, sig0.data(), (size_t)b->R * 8, hipMemcpyHostToDevice),
              "hipMemcpy");
    hip_check(hipMemcpy(b->ws, &ctl0, sizeof(hsim::Ctl), hipMemcpyHostToDevice), "hipMemcpy");
    b->h_beta = beta0;
    b->h_bfield = bf0;
    if (!err.empty()) throw Error(HSIM_E_DEVICE, "autotune: " + err);
    b->tuned_launch = win.mode;
    b->persistent_grid = win.grid;
    if (cache_path) {
        std::ofstream out(cache_path, std::ios::app);
        out << key << " " << win.mode << " " << win.grid << " " << win.spw << " " << win.masked << "\n";
    }
}

// ------------------------------------------------------------ layout choice
// Times every layout these replicas can use, each as a fresh batch of its
// own: one warm-up step and one timed step of trial_mcs MCS from a cold start
// at the given temperatures and fields, with the launch mode a fresh batch
// runs under HSIM_LAUNCH_AUTO.  Candidates: SITE; REPLICA when the batch
// allows it (FP32, one shared lattice); BLOCK when a replica's spins fit in
// LDS.  The static choice of HSIM_LAYOUT_AUTO is kept unless another layout
// is more than 2% faster.
int32_t choose_layout_impl(int32_t R, const hsim_plan *plans, uint64_t seed, const uint32_t *rep_id,
                           hsim_precision prec, const double *T, const double *B, int32_t trial_mcs,
                           hipStream_t st)
{
    if (R < 1 || !plans || !T || !B) throw Error(HSIM_E_ARG, "choose_layout: bad argument");
    if (trial_mcs < 1) throw Error(HSIM_E_ARG, "choose_layout: trial_mcs must be >= 1");
    for (int r = 0; r < R; ++r)
        if (!(T[r] >= 0.0) || std::isnan(B[r]) || std::isinf(B[r]))
            throw Error(HSIM_E_PARAM, "choose_layout: temperatures >= 0 and finite fields");
    struct Del { void operator()(hsim_batch b) const { delete b; } };
    int32_t auto_layout;
    {
        std::unique_ptr<hsim_batch_s, Del> b(batch_create_impl(R, plans, seed, rep_id, prec, HSIM_LAYOUT_AUTO));
        auto_layout = b->layout;
    }
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    std::string err;
    std::vector<std::pair<int32_t, float>> times;
    try {
        for (int32_t lay : {(int32_t)HSIM_LAYOUT_SITE, (int32_t)HSIM_LAYOUT_REPLICA, (int32_t)HSIM_LAYOUT_BLOCK}) {
            std::unique_ptr<hsim_batch_s, Del> b;
            try {
                b.reset(batch_create_impl(R, plans, seed, rep_id, prec, (hsim_layout)lay));
            } catch (const Error &e) {
                if (e.code == HSIM_E_UNSUPPORTED) continue;   // not a layout for this batch
                throw;
            }
            if (lay == HSIM_LAYOUT_BLOCK && !b->lds && lay != auto_layout) continue;
            size_t wsb = 0, spb = 0, hb = 0;
            batch_sizes_impl(b.get(), 2, trial_mcs, &wsb, &spb, &hb);
            hsim::DevBuf ws, sp, hist;
            ws.alloc(wsb);
            sp.alloc(spb);
            hist.alloc(hb);
            batch_bind_impl(b.get(), 2, trial_mcs, ws.p, sp.p, hist.p);
            batch_init_impl(b.get(), HSIM_INIT_COLD_Z, nullptr, st);
            // step 0 warms up (and captures a graph where the mode uses one);
            // T and B are [n_rep][1] for a run of one step
            batch_run_impl(b.get(), 0, 1, T, B, 0, HSIM_LAUNCH_AUTO, 0, nullptr, st);
            hip_check(hipEventRecord(e0, st), "hipEventRecord");
            batch_run_impl(b.get(), 1, 1, T, B, 0, HSIM_LAUNCH_AUTO, 0, nullptr, st);
            hip_check(hipEventRecord(e1, st), "hipEventRecord");
            hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.0f;
            hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            if (batch_status_impl(b.get()) != 0) throw Error(HSIM_E_DEVICE, "choose_layout: a trial run failed");
            hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
            times.push_back({lay, ms});
        }
    } catch (const std::exception &e) {
        err = e.what();
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!err.empty()) throw Error(HSIM_E_DEVICE, "choose_layout: " + err);
    // the static choice is always among the trials: it is creatable, and the
    // block layout is tried whenever it is the static choice
    float base = 0.0f;
    for (auto &t : times)
        if (t.first == auto_layout) base = t.second;
    int32_t win = auto_layout;
    float best = base;
    for (auto &t : times)
        if (t.second < 0.98f * base && t.second < best) {
            win = t.first;
            best = t.second;
        }
    return win;
}

// ------------------------------------------------------------ launch timing
void batch_time_phases_impl(hsim_batch b, int32_t every)
{
    if (!b || every < 0) throw Error(HSIM_E_ARG, "time_phases: bad argument");
    b->time_every = every;
}

void batch_phase_times_impl(hsim_batch b, double *total_ms, int64_t *launches, int64_t *updates)
{
    if (!b) throw Error(HSIM_E_ARG, "phase_times: NULL batch");
    double sum = 0.0;
    int64_t upd = 0;
    const size_t pairs = b->ev_units.size();
    for (size_t k = 0; k < pairs; ++k) {
        hip_check(hipEventSynchronize(b->ev_pool[2 * k + 1]), "hipEventSynchronize");
        float ms = 0.0f;
        hip_check(hipEventElapsedTime(&ms, b->ev_pool[2 * k], b->ev_pool[2 * k + 1]),
                  "hipEventElapsedTime");
        sum += ms;
        upd += b->ev_units[k];
    }
    if (total_ms) *total_ms = sum;
    if (launches) *launches = (int64_t)pairs;
    if (updates) *updates = upd;
    b->ev_units.clear();
    b->ev_used = 0;
}
