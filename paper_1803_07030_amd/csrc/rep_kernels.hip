// Replica-lane sweep: replicas that share one lattice are updated together,
// one lane per replica of one site.  Spins are rows of Rp floats (Rp =
// replicas padded to the lane-group width W), component c of site i at
// spins + c*cs + i*ss (planar [3][n][Rp] or interleaved [n][3][Rp]), so every
// neighbour read of a wave is a contiguous 4*W-byte row and the CSR row of a site (offsets, columns,
// constants) is read once for W replicas.
//
// Paper: Eq. 1-2 (energy), Eq. 4 (acceptance), section "Monte Carlo
// Metropolis algorithm" (one attempt per site per MCS); history per MCS
// (section "VEGAS software package").  Replicas are independent chains, each
// with its own temperature and field schedule.
//
// A tile is kRepWaves * spw consecutive sites of one colour class (spw =
// kRepSitesPerWave, or fewer for small lattices); wave w of the tile's block
// takes spw of them in order (kRepSitesPerStep at a time with 64-lane
// groups, two at a time with 32-lane groups).  Each XCD takes a contiguous
// range of a colour's tiles; inside it an optional order table starts tiles
// one plane of the class apart together (large lattices).
// Per-MCS history: every tile writes one record per replica; records are
// summed in 64 fixed chunks of tiles, and the chunks in order, the same way in
// every launch mode.  Plain and graph launches keep the records of a window of
// MCS and reduce the window in two launches of its own, so no sweep launch
// waits on a reduction.
#include "hsim_dev.h"
#include "update.h"

namespace hsim {

namespace {

// LDS of a replica-lane block: the tile sums ([kRepWaves][64][5]) and, reused,
// the history reductions (chunk quarters [4][6][32], final eighths [8][6][32]).
constexpr int kRedDoubles = kRepWaves * 64 * 6 > 8 * 6 * 32 ? kRepWaves * 64 * 6 : 8 * 6 * 32;

__device__ __forceinline__ bool rep_recompute_due(uint32_t m, int P)
{
    return m == 0 || (P > 0 && (m % (uint32_t)P) == 0);
}

// History accumulators of one lane without branches: energy change and count
// of accepted moves, and the final spin of every live site.
__device__ __forceinline__ void accumulate(double (&acc)[6], bool ok, bool live, float dE, float x,
                                           float y, float z)
{
    acc[0] += ok ? (double)dE : 0.0;
    acc[4] += ok ? 1.0 : 0.0;
    acc[1] += live ? (double)x : 0.0;
    acc[2] += live ? (double)y : 0.0;
    acc[3] += live ? (double)z : 0.0;
}

// Per-site parameters; UNI: the site index is wave-uniform (scalar loads).
template <int KM, int FM, bool UNI = false>
struct RepSite {
    float k, ex, ey, ez, nx, ny, nz;
    template <typename T>
    __device__ __forceinline__ static T ld(const T *p, int64_t i)
    {
        if constexpr (UNI) return ((const __attribute__((address_space(4))) T *)p)[i];
        else return p[i];
    }
    __device__ __forceinline__ RepSite(const RepLaneArgs &a, int i)
    {
        if (KM == K_SITE) {
            k = ld(a.k, i);
            ex = ld(a.ax, i);
            ey = ld(a.ax, (int64_t)a.n + i);
            ez = ld(a.ax, 2 * (int64_t)a.n + i);
        } else {
            k = (KM == K_UNIFORM) ? a.k0 : 0.0f;
            ex = a.e0x;
            ey = a.e0y;
            ez = a.e0z;
        }
        if (FM == F_SITE) {
            nx = ld(a.nd, i);
            ny = ld(a.nd, (int64_t)a.n + i);
            nz = ld(a.nd, 2 * (int64_t)a.n + i);
        } else {
            nx = a.n0x;
            ny = a.n0y;
            nz = a.n0z;
        }
    }
};

// Kernel variants: bit 0 (VAR_POL) update policies, bit 1 (VAR_XT) cubic
// anisotropy and / or spin norms, bit 2 (VAR_TRACE) the accept bitmap (alone:
// a traced run of the plain model).
constexpr int VAR_POL = 1, VAR_XT = 2, VAR_TRACE = 4;

// Accept bitmap of a traced run: bit (user site % 32) of word user site / 32
// of row (replica, MCS of the run).
__device__ __forceinline__ void rep_trace(const RunArgs &ra, int r, uint32_t g, uint32_t orig)
{
    atomicOr(&ra.trace[((size_t)r * ra.n_mcs_run + (g - ra.g0)) * ra.trace_words + (orig >> 5)],
             1u << (orig & 31));
}

// Trial of site i for one lane: the random move, or (VAR_POL) the move of the
// site's type, with the lane's replica width for the adaptive move; ad tells
// whether the move is adaptive (its accepts steer the width).  With VAR_XT
// and spin norms the move acts on the direction and the trial gets the
// site's length mu back.
template <int VAR>
__device__ __forceinline__ Trial32 rep_trial(const RepLaneArgs &a, const RunArgs &ra, int i,
                                             uint32_t orig, uint32_t g, uint32_t rid, float sx,
                                             float sy, float sz, float sigma, float mu, bool &ad)
{
    const uint4 w = draw(ra.seed, orig, g, rid, 0);
    ad = false;
    Trial32 t;
    if constexpr (!(VAR & VAR_POL)) {
        t = trial32(w);
    } else {
        const SitePol pl = pick_policy(ra.pol.pol, ra.pol.param, ra.pol.cos_t, a.type ? a.type[i] : 0);
        ad = pl.pol == POL_ADAPTIVE;
        if (pl.pol == POL_RANDOM) {
            t = trial32(w);
        } else {
            const float inv = (VAR & VAR_XT) ? 1.0f / mu : 1.0f;
            t = trial32_policy(pl.pol, w, sx * inv, sy * inv, sz * inv, ad ? sigma : (float)pl.param,
                               (float)(1.0 - pl.cos_t), ra.seed, orig, g, rid);
        }
    }
    if constexpr ((VAR & VAR_XT) != 0) {
        t.x *= mu;
        t.y *= mu;
        t.z *= mu;
    }
    return t;
}

// Per-site extra terms of a lane's update (VAR_XT): spin length and cubic
// constant (0 / 1 when the plan has none).
template <bool UNI>
struct RepXt {
    float mu = 1.0f, kc = 0.0f;
    __device__ __forceinline__ RepXt() {}
    __device__ __forceinline__ RepXt(const RepLaneArgs &a, int i)
    {
        if (a.mu) mu = UNI ? ((const __attribute__((address_space(4))) float *)a.mu)[i] : a.mu[i];
        if (a.kc) kc = UNI ? ((const __attribute__((address_space(4))) float *)a.kc)[i] : a.kc[i];
    }
};

// Update site i for replica lane r (spin column r of the rows),
// generic CSR row walk (rows of any degree).
template <int KM, int FM, int VAR>
__device__ __forceinline__ void rep_site_update(const RepLaneArgs &a, int i, int r, uint32_t g,
                                                float beta, float b, uint32_t rid, bool active,
                                                float sigma, const RunArgs &ra, double (&acc)[6])
{
    const size_t plane = (size_t)a.cs;
    float *S = a.spins + r;
    const int32_t rb = a.rp[i], re = a.rp[i + 1];
    float hx = 0.0f, hy = 0.0f, hz = 0.0f;
    for (int32_t p = rb; p < re; ++p) {
        const size_t o = (size_t)a.ci[p] * a.ss;
        const float Jp = a.J[p];
        hx = fmaf(Jp, S[o], hx);
        hy = fmaf(Jp, S[plane + o], hy);
        hz = fmaf(Jp, S[2 * plane + o], hz);
    }
    const RepSite<KM, FM> sp(a, i);
    hx = fmaf(b, sp.nx, hx);
    hy = fmaf(b, sp.ny, hy);
    hz = fmaf(b, sp.nz, hz);
    const size_t oi = (size_t)i * a.ss;
    const float sx = S[oi], sy = S[plane + oi], sz = S[2 * plane + oi];
    bool ad;
    const RepXt<false> xt = (VAR & VAR_XT) ? RepXt<false>(a, i) : RepXt<false>();
    const Trial32 t = rep_trial<VAR>(a, ra, i, a.orig[i], g, rid, sx, sy, sz, sigma, xt.mu, ad);
    float dE = (KM == K_NONE) ? delta_e32_iso(sx, sy, sz, t, hx, hy, hz)
                              : delta_e32(sx, sy, sz, t, hx, hy, hz, sp.k, sp.ex, sp.ey, sp.ez);
    if constexpr ((VAR & VAR_XT) != 0)
        dE = fmaf(-xt.kc, cubic32(t.x, t.y, t.z) - cubic32(sx, sy, sz), dE);
    const bool ok = accept32(dE, beta, t.u) && active;
    acc[5] += (ok && ad) ? 1.0 : 0.0;
    if (active && dE != dE) atomicOr(&ra.ctl->status, 1u);
    if (ok) {
        S[oi] = t.x;
        S[plane + oi] = t.y;
        S[2 * plane + oi] = t.z;
        if constexpr ((VAR & VAR_TRACE) != 0) rep_trace(ra, r, g, a.orig[i]);
    }
    accumulate(acc, ok, active, dE, ok ? t.x : sx, ok ? t.y : sy, ok ? t.z : sz);
}

// Read-only lattice tables seen through the constant address space: with a
// wave-uniform index the compiler loads them with scalar loads.
template <typename T>
__device__ __forceinline__ T cload(const T *p, int64_t i)
{
    return ((const __attribute__((address_space(4))) T *)p)[i];
}

// Fixed-width rows: the plan pads every row to MAXD slots (ell_col, ell_J,
// site-major); a slot past the row's end holds the site itself with constant
// 0, which leaves the fused multiply-add chain of the field unchanged
// (h + 0*S == h), so the padded walk gives the same bits as the CSR walk.
// Buffer resources over the rows of the three spin components (raw buffers
// from each component's first row to its last; the host keeps that extent
// below 2 GiB so that byte offsets fit the 32-bit offset fields).
struct SpinPlanes {
    __amdgpu_buffer_rsrc_t x, y, z;
    __device__ __forceinline__ SpinPlanes(const RepLaneArgs &a)
    {
        const int bytes = (int)(((int64_t)(a.n - 1) * a.ss + a.Rp) * 4);
        x = __builtin_amdgcn_make_buffer_rsrc(a.spins, 0, bytes, 0x00020000);
        y = __builtin_amdgcn_make_buffer_rsrc(a.spins + a.cs, 0, bytes, 0x00020000);
        z = __builtin_amdgcn_make_buffer_rsrc(a.spins + 2 * a.cs, 0, bytes, 0x00020000);
    }
};

__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t rs, int32_t lane_b, int32_t row_b)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, lane_b, row_b, 0));
}

// Spin rows are stored with the SC1 cache-policy bit (device scope): the
// colour phases ran 3.4% faster than with default stores (59.1 against
// 61.2 us on SC 64^3 x 64 replicas; NT, SC0|SC1 and NT|SC1 were no better or
// slower).  The bit changes how the stores travel through the caches, not
// what memory holds at the end of the launch.
constexpr int kSpinStorePolicy = 16;

__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t rs, int32_t lane_b, int32_t row_b,
                                       float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, lane_b, row_b,
                                          kSpinStorePolicy);
}

// kRepSitesPerStep sites of one 64-lane group at once, rows padded to MAXD:
// all loads of the step are issued before any store (sites of one colour
// class are never neighbours); the own rows are written back whole.  Row entries are wave-uniform scalar loads;
// spin rows go through the buffer descriptors with the row in soffset.
template <int KM, int FM, int MAXD, int VAR>
__device__ __forceinline__ void rep_step_uniform(const RepLaneArgs &a, const SpinPlanes &sp3,
                                                 int i0, int ce, int r, uint32_t g, float beta,
                                                 float b, uint32_t rid, bool active, float sigma,
                                                 const RunArgs &ra, double (&acc)[6])
{
    constexpr int NS = kRepSitesPerStep;
    const int32_t lane_b = r * 4;        // byte offset of this replica inside a row
    float hx[NS], hy[NS], hz[NS], sx[NS], sy[NS], sz[NS];
    int ic[NS];
    bool valid[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        valid[u] = i0 + u < ce;
        ic[u] = valid[u] ? i0 + u : ce - 1;
        hx[u] = 0.0f;
        hy[u] = 0.0f;
        hz[u] = 0.0f;
#pragma unroll
        for (int sl = 0; sl < MAXD; ++sl) {
            const int32_t ob = cload(a.ell_col, ic[u] * MAXD + sl) * a.ss * 4;   // row byte offset
            const float Jp = cload(a.ell_J, ic[u] * MAXD + sl);
            hx[u] = fmaf(Jp, bload(sp3.x, lane_b, ob), hx[u]);
            hy[u] = fmaf(Jp, bload(sp3.y, lane_b, ob), hy[u]);
            hz[u] = fmaf(Jp, bload(sp3.z, lane_b, ob), hz[u]);
        }
        const int32_t oi = ic[u] * a.ss * 4;
        sx[u] = bload(sp3.x, lane_b, oi);
        sy[u] = bload(sp3.y, lane_b, oi);
        sz[u] = bload(sp3.z, lane_b, oi);
    }
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const int i = ic[u];
        const RepSite<KM, FM, true> sp(a, i);
        const float fx = fmaf(b, sp.nx, hx[u]);
        const float fy = fmaf(b, sp.ny, hy[u]);
        const float fz = fmaf(b, sp.nz, hz[u]);
        bool ad;
        const RepXt<true> xt = (VAR & VAR_XT) ? RepXt<true>(a, i) : RepXt<true>();
        const Trial32 t = rep_trial<VAR>(a, ra, i, cload(a.orig, i), g, rid, sx[u], sy[u], sz[u],
                                         sigma, xt.mu, ad);
        float dE = (KM == K_NONE) ? delta_e32_iso(sx[u], sy[u], sz[u], t, fx, fy, fz)
                                  : delta_e32(sx[u], sy[u], sz[u], t, fx, fy, fz, sp.k, sp.ex,
                                              sp.ey, sp.ez);
        if constexpr ((VAR & VAR_XT) != 0)
            dE = fmaf(-xt.kc, cubic32(t.x, t.y, t.z) - cubic32(sx[u], sy[u], sz[u]), dE);
        const bool live = active && valid[u];
        const bool ok = accept32(dE, beta, t.u) && live;
        acc[5] += (ok && ad) ? 1.0 : 0.0;
        if (live && dE != dE) atomicOr(&ra.ctl->status, 1u);
        const int32_t oi = i * a.ss * 4;
        // every live lane stores (the old value when rejected): whole rows
        // reach memory faster than rows with holes while the spin set stays
        // in the last-level cache; masked_store keeps the accepted moves
        // only (fewer bytes once the rows stream from HBM).  Same values.
        if (live && (ok || !a.masked_store)) {
            bstore(sp3.x, lane_b, oi, ok ? t.x : sx[u]);
            bstore(sp3.y, lane_b, oi, ok ? t.y : sy[u]);
            bstore(sp3.z, lane_b, oi, ok ? t.z : sz[u]);
        }
        if constexpr ((VAR & VAR_TRACE) != 0)
            if (ok) rep_trace(ra, r, g, cload(a.orig, i));
        accumulate(acc, ok, live, dE, ok ? t.x : sx[u], ok ? t.y : sy[u], ok ? t.z : sz[u]);
    }
}

// Two sites of one lane group at once: all loads of both sites are issued
// before either stores (sites of one colour class are never neighbours).
template <int KM, int FM, int MAXD, int VAR>
__device__ __forceinline__ void rep_pair_update(const RepLaneArgs &a, int i0, int ce, int r,
                                                uint32_t g, float beta, float b, uint32_t rid,
                                                bool active, float sigma, const RunArgs &ra,
                                                double (&acc)[6])
{
    const size_t plane = (size_t)a.cs;
    float *S = a.spins + r;
    float hx[2], hy[2], hz[2], sx[2], sy[2], sz[2];
    int ic[2];
    bool valid[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        valid[u] = i0 + u < ce;
        ic[u] = valid[u] ? i0 + u : ce - 1;
        hx[u] = 0.0f;
        hy[u] = 0.0f;
        hz[u] = 0.0f;
#pragma unroll
        for (int sl = 0; sl < MAXD; ++sl) {
            const size_t o = (size_t)a.ell_col[ic[u] * MAXD + sl] * a.ss;
            const float Jp = valid[u] ? a.ell_J[ic[u] * MAXD + sl] : 0.0f;
            hx[u] = fmaf(Jp, S[o], hx[u]);
            hy[u] = fmaf(Jp, S[plane + o], hy[u]);
            hz[u] = fmaf(Jp, S[2 * plane + o], hz[u]);
        }
        const size_t oi = (size_t)ic[u] * a.ss;
        sx[u] = S[oi];
        sy[u] = S[plane + oi];
        sz[u] = S[2 * plane + oi];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = ic[u];
        const RepSite<KM, FM> sp(a, i);
        const float fx = fmaf(b, sp.nx, hx[u]);
        const float fy = fmaf(b, sp.ny, hy[u]);
        const float fz = fmaf(b, sp.nz, hz[u]);
        bool ad;
        const RepXt<false> xt = (VAR & VAR_XT) ? RepXt<false>(a, i) : RepXt<false>();
        const Trial32 t = rep_trial<VAR>(a, ra, i, a.orig[i], g, rid, sx[u], sy[u], sz[u], sigma,
                                         xt.mu, ad);
        float dE = (KM == K_NONE) ? delta_e32_iso(sx[u], sy[u], sz[u], t, fx, fy, fz)
                                  : delta_e32(sx[u], sy[u], sz[u], t, fx, fy, fz, sp.k, sp.ex,
                                              sp.ey, sp.ez);
        if constexpr ((VAR & VAR_XT) != 0)
            dE = fmaf(-xt.kc, cubic32(t.x, t.y, t.z) - cubic32(sx[u], sy[u], sz[u]), dE);
        const bool live = active && valid[u];
        const bool ok = accept32(dE, beta, t.u) && live;
        acc[5] += (ok && ad) ? 1.0 : 0.0;
        if (live && dE != dE) atomicOr(&ra.ctl->status, 1u);
        const size_t oi = (size_t)i * a.ss;
        if (ok) {
            S[oi] = t.x;
            S[plane + oi] = t.y;
            S[2 * plane + oi] = t.z;
            if constexpr ((VAR & VAR_TRACE) != 0) rep_trace(ra, r, g, a.orig[i]);
        }
        accumulate(acc, ok, live, dE, ok ? t.x : sx[u], ok ? t.y : sy[u], ok ? t.z : sz[u]);
    }
}

template <int KM, int FM>
__device__ __forceinline__ double rep_site_energy(const RepLaneArgs &a, int i, int r, double b)
{
    const size_t plane = (size_t)a.cs;
    const float *S = a.spins + r;
    double hx = 0.0, hy = 0.0, hz = 0.0;
    for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
        const size_t o = (size_t)a.ci[p] * a.ss;
        const double Jp = (double)a.J[p];
        hx += Jp * (double)S[o];
        hy += Jp * (double)S[plane + o];
        hz += Jp * (double)S[2 * plane + o];
    }
    const RepSite<KM, FM> sp(a, i);
    const size_t oi = (size_t)i * a.ss;
    const double sx = S[oi], sy = S[plane + oi], sz = S[2 * plane + oi];
    const double an = sx * (double)sp.ex + sy * (double)sp.ey + sz * (double)sp.ez;
    const double zn = sx * (double)sp.nx + sy * (double)sp.ny + sz * (double)sp.nz;
    double e = -0.5 * (sx * hx + sy * hy + sz * hz) - b * zn - (double)sp.k * an * an;
    if (a.kc) e -= (double)a.kc[i] * cubic64(sx, sy, sz);
    return e;
}

// The same energy through the padded rows (row entries in CSR order, then
// zero-J padding; 64-lane groups): scalar row loads, buffer spin loads.
template <int KM, int FM, int MAXD>
__device__ __forceinline__ double rep_site_energy_ell(const RepLaneArgs &a, const SpinPlanes &sp3,
                                                      int i, int32_t lane_b, double b)
{
    double hx = 0.0, hy = 0.0, hz = 0.0;
#pragma unroll
    for (int sl = 0; sl < MAXD; ++sl) {
        const int32_t ob = cload(a.ell_col, i * MAXD + sl) * a.ss * 4;
        const double Jp = (double)cload(a.ell_J, i * MAXD + sl);
        hx += Jp * (double)bload(sp3.x, lane_b, ob);
        hy += Jp * (double)bload(sp3.y, lane_b, ob);
        hz += Jp * (double)bload(sp3.z, lane_b, ob);
    }
    const RepSite<KM, FM, true> sp(a, i);
    const int32_t oi = i * a.ss * 4;
    const double sx = bload(sp3.x, lane_b, oi), sy = bload(sp3.y, lane_b, oi),
                 sz = bload(sp3.z, lane_b, oi);
    const double an = sx * (double)sp.ex + sy * (double)sp.ey + sz * (double)sp.ez;
    const double zn = sx * (double)sp.nx + sy * (double)sp.ny + sz * (double)sp.nz;
    double e = -0.5 * (sx * hx + sy * hy + sz * hz) - b * zn - (double)sp.k * an * an;
    if (a.kc) e -= (double)cload(a.kc, i) * cubic64(sx, sy, sz);
    return e;
}

// Lane geometry for lane-group width W: replica column and sub-group.
template <int W>
struct Lanes {
    int lane, w, sub, rl, r;
    __device__ __forceinline__ Lanes(int group)
    {
        lane = threadIdx.x & 63;
        w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
        sub = (W == 64) ? 0 : lane / W;
        rl = lane % W;
        r = rl + W * group;
    }
};

// One tile of one colour phase: the body shared by the per-phase kernel and
// the persistent kernel.  red: LDS [kRepWaves][64][NQ].  MAXD > 0: rows padded
// to MAXD entries; MAXD == 0: generic row walk.  VAR: VAR_POL update
// policies (the tile also records its accepted adaptive moves, field 6),
// VAR_XT cubic anisotropy and spin norms.
template <int KM, int FM, int W, int MAXD, int VAR = 0>
__device__ __forceinline__ void rep_tile(const RepLaneArgs &a, int colour, int tile, int group,
                                         uint32_t g, const RunArgs &ra, double *part,
                                         double *red)
{
    const int SPL = a.spw * W / 64;   // sites per lane group (even for W = 32)
    constexpr bool POL = (VAR & VAR_POL) != 0;
    constexpr int NQ = POL ? 6 : 5;
    const Lanes<W> L(group);
    const int ce = a.cls_off[colour + 1];
    const int wbase = a.cls_off[colour] + tile * (kRepWaves * a.spw) + L.w * a.spw;
    const int base = wbase + L.sub * SPL;
    const bool active = L.r < a.R;
    const uint32_t s_abs = g / (uint32_t)ra.M;
    float beta = 0.0f, b = 0.0f, sigma = 0.0f;
    uint32_t rid = 0;
    if (active) {
        const size_t sidx = (size_t)L.r * ra.S_hist + s_abs;
        beta = (float)ra.beta[sidx];
        b = (float)ra.bfield[sidx];
        rid = a.rep_id[L.r];
        if (POL && ra.pol.adaptive) sigma = (float)ra.sigma[L.r];
    }
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (MAXD > 0) {
        const SpinPlanes sp3(a);
        for (int j = 0; j < SPL && base + j < ce; j += (W == 64 ? kRepSitesPerStep : 2)) {
            if constexpr (W == 64)
                rep_step_uniform<KM, FM, MAXD, VAR>(a, sp3, base + j, ce, L.r, g, beta, b, rid,
                                                    active, sigma, ra, acc);
            else
                rep_pair_update<KM, FM, MAXD, VAR>(a, base + j, ce, L.r, g, beta, b, rid, active,
                                                   sigma, ra, acc);
        }
    } else {
        for (int j = 0; j < SPL; ++j) {
            const int i = base + j;
            if (i >= ce) break;
            rep_site_update<KM, FM, VAR>(a, i, L.r, g, beta, b, rid, active, sigma, ra, acc);
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) red[(L.w * 64 + L.lane) * NQ + q] = acc[q];
    __syncthreads();
    if (threadIdx.x < W) {
        double v[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = 0.0;
        for (int ww = 0; ww < kRepWaves; ++ww)
            for (int sb = 0; sb < 64 / W; ++sb)
#pragma unroll
                for (int q = 0; q < NQ; ++q) v[q] += red[(ww * 64 + sb * W + (int)threadIdx.x) * NQ + q];
        const int rr = (int)threadIdx.x + W * group;
        const int tg = a.tile_off[colour] + tile;
#pragma unroll
        for (int q = 0; q < 5; ++q) part[((size_t)tg * kRecFields + q) * a.Rp + rr] = v[q];
        if constexpr (POL) part[((size_t)tg * kRecFields + 6) * a.Rp + rr] = v[5];
    }
    __syncthreads();
}

// Energy records of one tile (field 5).
template <int KM, int FM, int W, int MAXD>
__device__ __forceinline__ void rep_tile_energy(const RepLaneArgs &a, int tg, int group,
                                                uint32_t g, const RunArgs &ra, double *part,
                                                double *red)
{
    const int SPL = a.spw * W / 64;
    const Lanes<W> L(group);
    int colour = 0;
    while (colour + 1 < a.ncol && a.tile_off[colour + 1] <= tg) ++colour;
    const int tile = tg - a.tile_off[colour];
    const int ce = a.cls_off[colour + 1];
    const int base = a.cls_off[colour] + tile * (kRepWaves * a.spw) + L.w * a.spw + L.sub * SPL;
    double e = 0.0;
    if (L.r < a.R) {
        const double b = ra.bfield[(size_t)L.r * ra.S_hist + g / (uint32_t)ra.M];
        if constexpr (MAXD > 0 && W == 64) {
            const SpinPlanes sp3(a);
            for (int j = 0; j < SPL; ++j) {
                const int i = base + j;
                if (i >= ce) break;
                e += rep_site_energy_ell<KM, FM, MAXD>(a, sp3, i, L.r * 4, b);
            }
        } else {
            for (int j = 0; j < SPL; ++j) {
                const int i = base + j;
                if (i >= ce) break;
                e += rep_site_energy<KM, FM>(a, i, L.r, b);
            }
        }
    }
    red[(L.w * 64 + L.lane) * 5] = e;
    __syncthreads();
    if (threadIdx.x < W) {
        double v = 0.0;
        for (int ww = 0; ww < kRepWaves; ++ww)
            for (int sb = 0; sb < 64 / W; ++sb) v += red[(ww * 64 + sb * W + (int)threadIdx.x) * 5];
        part[((size_t)tg * kRecFields + 5) * a.Rp + (int)threadIdx.x + W * group] = v;
    }
    __syncthreads();
}

// Chunk k of the tile records, per (field, replica): the chunk's tiles are
// cut into four fixed quarters, each summed in order by one thread, and the
// quarters added in order, so one load latency covers a quarter.  Replicas
// are handled 32 at a time through buf (LDS, >= 4 * 6 * 32 doubles).
__device__ __forceinline__ void rep_chunk_sum(const RepLaneArgs &a, int ntiles, int k,
                                              const double *part, double *chunk, double *buf)
{
    constexpr int G = 32;
    const int tb = (int)((int64_t)ntiles * k / kChunks), te = (int)((int64_t)ntiles * (k + 1) / kChunks);
    const size_t stride = (size_t)kRecFields * a.Rp;
    for (int r0 = 0; r0 < a.Rp; r0 += G) {
        for (int e = threadIdx.x; e < 4 * 6 * G; e += blockDim.x) {
            const int s = e / (6 * G), q = (e / G) % 6, rr = r0 + e % G;
            const int t0 = tb + (te - tb) * s / 4, t1 = tb + (te - tb) * (s + 1) / 4;
            double v = 0.0;
            if (rr < a.Rp) {
                const double *p = part + (size_t)q * a.Rp + rr;
                int t = t0;
                for (; t + 8 <= t1; t += 8) {
                    double x[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) x[u] = p[(size_t)(t + u) * stride];
#pragma unroll
                    for (int u = 0; u < 8; ++u) v += x[u];
                }
                for (; t < t1; ++t) v += p[(size_t)t * stride];
            }
            buf[e] = v;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 6 * G; e += blockDim.x) {
            const int q = e / G, rr = r0 + e % G;
            if (rr < a.Rp)
                chunk[((size_t)k * 6 + q) * a.Rp + rr] =
                    ((buf[e] + buf[6 * G + e]) + buf[12 * G + e]) + buf[18 * G + e];
        }
        __syncthreads();
    }
}

// Final sum over the chunks: eight fixed groups of eight chunks, each summed
// in order by one thread, then the groups in order.  v (LDS or global,
// [6][Rp]) receives the six totals of every replica.  buf: LDS, >= 8 * 6 * 32
// doubles.
__device__ __forceinline__ void rep_final_sums(const RepLaneArgs &a, const double *chunk,
                                               double *buf, double *v)
{
    constexpr int G = 32;
    const size_t stride = (size_t)6 * a.Rp;
    for (int r0 = 0; r0 < a.Rp; r0 += G) {
        for (int e = threadIdx.x; e < 8 * 6 * G; e += blockDim.x) {
            const int s = e / (6 * G), q = (e / G) % 6, rr = r0 + e % G;
            double x = 0.0;
            if (rr < a.Rp) {
                const double *p = chunk + (size_t)q * a.Rp + rr;   // chunk layout [k][6][Rp]
                double y[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) y[u] = p[(size_t)(8 * s + u) * stride];
#pragma unroll
                for (int u = 0; u < 8; ++u) x += y[u];
            }
            buf[e] = x;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 6 * G; e += blockDim.x) {
            const int q = e / G, rl = e % G, rr = r0 + rl;
            if (rr >= a.Rp) continue;
            double t = 0.0;
            for (int s = 0; s < 8; ++s) t += buf[(s * 6 + q) * G + rl];
            v[(size_t)q * a.Rp + rr] = t;
        }
        __syncthreads();
    }
}

// History record of MCS g from its six totals v ([6][Rp]) and the carried
// energy: at a recompute the energy restarts from the full energy (field 5),
// otherwise from the carried value; the energy change of g (field 0) is added.
__device__ __forceinline__ void rep_write_history(const RepLaneArgs &a, uint32_t g,
                                                  const RunArgs &ra, const double *v)
{
    const uint32_t s_abs = g / (uint32_t)ra.M, m = g % (uint32_t)ra.M;
    const bool due = rep_recompute_due(m, ra.P);
    for (int rr = threadIdx.x; rr < a.R; rr += blockDim.x) {
        const double E = (due ? v[5 * (size_t)a.Rp + rr] : ra.ecarry[rr]) + v[rr];
        ra.ecarry[rr] = E;
        double *h = ra.history + (((size_t)rr * ra.S_hist + s_abs) * ra.M + m) * 5;
        h[0] = E;
#pragma unroll
        for (int q = 1; q < 5; ++q) h[q] = v[(size_t)q * a.Rp + rr];
    }
}

// Both steps in one block (persistent kernel).  v: global [6][Rp].
__device__ __forceinline__ void rep_final(const RepLaneArgs &a, uint32_t g, const RunArgs &ra,
                                          const double *chunk, double *v, double *buf)
{
    rep_final_sums(a, chunk, buf, v);
    rep_write_history(a, g, ra, v);
    __syncthreads();
}

}  // namespace

// MCS numbering of the per-phase launches: g = ctl->g + t_off, where ctl->g
// is the first MCS of the current launch sequence (a captured graph replays
// one such sequence) and t_off the launch's position in it.  The tile records
// of MCS t_off go to slot t_off % rec_win of the record window; one reduction
// per window of rec_win MCS sums them (the persistent kernel uses slots 0, 1).
__device__ __forceinline__ double *rep_slot(const RunArgs &ra, const RepLaneArgs &a, int ntiles,
                                            int slot)
{
    return ra.partials + (size_t)slot * ntiles * kRecFields * a.Rp;
}

__device__ __forceinline__ double *rep_chunk_slot(const RunArgs &ra, const RepLaneArgs &a, int slot)
{
    return ra.chunks + (size_t)slot * kChunks * 6 * a.Rp;
}

// Per-phase kernel: grid (tiles of the colour, replica groups).
template <int KM, int FM, int W, int MAXD, int VAR>
__global__ __launch_bounds__(kRepThreads) void k_rep_phase(RepLaneArgs a, int colour, int t_off,
                                                           int ntiles, RunArgs ra)
{
    __shared__ double red[kRedDoubles];
    const uint32_t g = ra.ctl->g + (uint32_t)t_off;
    const int nt = a.tile_off[colour + 1] - a.tile_off[colour];
    const int u = xcd_tile(blockIdx.x, nt);
    rep_tile<KM, FM, W, MAXD, VAR>(a, colour, a.tord ? a.tord[a.tile_off[colour] + u] : u, blockIdx.y, g,
                                   ra, rep_slot(ra, a, ntiles, t_off % ra.rec_win), red);
}

// Adaptive widths after MCS t_off of the sequence: the accepted adaptive
// moves of every replica (record field 6 of all tiles of the MCS) are summed
// in kChunks fixed chunks of tiles, one per block, each in tile order; the
// last block to finish adds the chunks in order and steers every width.
__global__ __launch_bounds__(256) void k_rep_sigma(RepLaneArgs a, int ntiles, int t_off, RunArgs ra)
{
    __shared__ int last;
    const double *rec = rep_slot(ra, a, ntiles, t_off % ra.rec_win);
    const int k = blockIdx.x;
    const int tb = (int)((int64_t)ntiles * k / kChunks), te = (int)((int64_t)ntiles * (k + 1) / kChunks);
    for (int r = threadIdx.x; r < a.R; r += blockDim.x) {
        double v = 0.0;
        for (int tg = tb; tg < te; ++tg) v += rec[((size_t)tg * kRecFields + 6) * a.Rp + r];
        ra.sig_part[(size_t)k * a.Rp + r] = v;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = (atomicAdd(&ra.ctl->pad[2], 1u) == kChunks - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    for (int r = threadIdx.x; r < a.R; r += blockDim.x) {
        double n = 0.0;
        for (int q = 0; q < kChunks; ++q) n += ra.sig_part[(size_t)q * a.Rp + r];
        ra.sigma[r] = adapted_sigma(ra.sigma[r], n, ra.n_ad[r], ra.pol.sigma_min, ra.pol.sigma_max);
    }
    if (threadIdx.x == 0) ra.ctl->pad[2] = 0;
}

template <int KM, int FM, int W, int MAXD>
__global__ __launch_bounds__(kRepThreads) void k_rep_efull(RepLaneArgs a, int t_off, int ntiles,
                                                           RunArgs ra)
{
    __shared__ double red[kRedDoubles];
    const uint32_t g = ra.ctl->g + (uint32_t)t_off;
    if (!rep_recompute_due(g % (uint32_t)ra.M, ra.P)) return;
    rep_tile_energy<KM, FM, W, MAXD>(a, blockIdx.x, blockIdx.y, g, ra,
                               rep_slot(ra, a, ntiles, t_off % ra.rec_win), red);
}

// Reduction of a window of MCS t_first .. t_first + count - 1 of the current
// sequence, step 1: chunk k (blockIdx.x) of MCS t_first + blockIdx.y.
__global__ __launch_bounds__(1024) void k_rep_chunks(RepLaneArgs a, int ntiles, int t_first,
                                                     RunArgs ra)
{
    __shared__ double buf[4 * 6 * 32];
    const int slot = (t_first + (int)blockIdx.y) % ra.rec_win;
    rep_chunk_sum(a, ntiles, blockIdx.x, rep_slot(ra, a, ntiles, slot), rep_chunk_slot(ra, a, slot),
                  buf);
}

// Step 2: block j adds the chunks of MCS t_first + j and writes the fields
// that need no carry (M, accepted); the last block to finish runs the energy
// carry through the window in MCS order and, with advance > 0, moves ctl->g
// on by advance (end of the sequence).
__global__ __launch_bounds__(256) void k_rep_finals(RepLaneArgs a, int t_first, int count,
                                                    int advance, RunArgs ra)
{
    constexpr int kStage = 16;          // MCS of the window staged in LDS at a time
    __shared__ double buf[8 * 6 * 32];
    __shared__ double stage[kStage * 2 * 64];
    __shared__ int last;
    const uint32_t g0 = ra.ctl->g;
    {
        const int t = t_first + (int)blockIdx.x;
        const int slot = t % ra.rec_win;
        double *v = ra.carry + (size_t)slot * 6 * a.Rp;
        rep_final_sums(a, rep_chunk_slot(ra, a, slot), buf, v);
        const uint32_t g = g0 + (uint32_t)t;
        const uint32_t s_abs = g / (uint32_t)ra.M, m = g % (uint32_t)ra.M;
        for (int rr = threadIdx.x; rr < a.R; rr += blockDim.x) {
            double *h = ra.history + (((size_t)rr * ra.S_hist + s_abs) * ra.M + m) * 5;
#pragma unroll
            for (int q = 1; q < 5; ++q) h[q] = v[(size_t)q * a.Rp + rr];
        }
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = (atomicAdd(&ra.ctl->pad[1], 1u) == (uint32_t)count - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    // carry: replicas 64 at a time, the window kStage MCS at a time through LDS
    for (int r0 = 0; r0 < a.R; r0 += 64) {
        const int nr = min(64, a.R - r0);
        double E = threadIdx.x < nr ? ra.ecarry[r0 + threadIdx.x] : 0.0;
        for (int j0 = 0; j0 < count; j0 += kStage) {
            const int nj = min(kStage, count - j0);
            __syncthreads();
            for (int e = threadIdx.x; e < nj * 2 * 64; e += blockDim.x) {
                const int j = e / 128, f = (e / 64) % 2, rl = e % 64;
                const int slot = (t_first + j0 + j) % ra.rec_win;
                stage[e] = rl < nr ? ra.carry[((size_t)slot * 6 + (f ? 5 : 0)) * a.Rp + r0 + rl] : 0.0;
            }
            __syncthreads();
            if ((int)threadIdx.x < nr) {
                const int rr = r0 + threadIdx.x;
                for (int j = 0; j < nj; ++j) {
                    const uint32_t g = g0 + (uint32_t)(t_first + j0 + j);
                    const uint32_t s_abs = g / (uint32_t)ra.M, m = g % (uint32_t)ra.M;
                    const double de = stage[(j * 2) * 64 + threadIdx.x];
                    const double ef = stage[(j * 2 + 1) * 64 + threadIdx.x];
                    E = (rep_recompute_due(m, ra.P) ? ef : E) + de;
                    ra.history[(((size_t)rr * ra.S_hist + s_abs) * ra.M + m) * 5] = E;
                }
            }
        }
        if ((int)threadIdx.x < nr) ra.ecarry[r0 + threadIdx.x] = E;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ra.ctl->pad[1] = 0;
        if (advance > 0) ra.ctl->g = g0 + (uint32_t)advance;
    }
}

// ------------------------------------------------------------- persistent
// One launch for the whole run.  Registration barrier (once per launch; the
// run's barriers are xcd_barrier below), without a contended counter: every block publishes the barrier's epoch in its own 128-byte flag
// (after a release fence); block 0 waits for all flags, then publishes the
// epoch in one generation word, which the other blocks wait for (then an
// acquire fence).  All polls are relaxed loads; every wait is bounded (cap
// sleeps) and a timeout, once flagged, releases every later wait at once, so
// the grid always drains.
__device__ __forceinline__ bool barrier_wait(const uint32_t *w, uint32_t epoch, Ctl *ctl,
                                             uint32_t cap)
{
    uint32_t n = 0;
    while (__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
        __builtin_amdgcn_s_sleep(1);
        if (++n > cap ||
            (__hip_atomic_load(&ctl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2u)) {
            atomicOr(&ctl->status, 2u);
            return false;
        }
    }
    return true;
}

__device__ __forceinline__ void grid_barrier(Ctl *ctl, uint32_t *flags, uint32_t &epoch,
                                             uint32_t cap)
{
    __syncthreads();
    ++epoch;
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&flags[blockIdx.x * 32], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (blockIdx.x == 0) {
        // each thread watches up to kFlagsPerThread flags, all loaded in one
        // round trip per poll
        constexpr int kFlagsPerThread = kMaxPersistentBlocks / kRepThreads;
        uint32_t n = 0;
        for (;;) {
            bool all = true;
#pragma unroll
            for (int u = 0; u < kFlagsPerThread; ++u) {
                const int j = threadIdx.x + u * kRepThreads;
                if (j < (int)gridDim.x &&
                    __hip_atomic_load(&flags[j * 32], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch)
                    all = false;
            }
            if (all) break;
            __builtin_amdgcn_s_sleep(1);
            if (++n > cap ||
                (__hip_atomic_load(&ctl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2u)) {
                atomicOr(&ctl->status, 2u);
                break;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            __hip_atomic_store(&ctl->bar_arrive, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (threadIdx.x == 0) {
        barrier_wait(&ctl->bar_arrive, epoch, ctl, cap);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// The blocks' barrier for the rest of the run, after a registration pass.
// A release at agent scope writes back the L2 of the XCD that executes it,
// whichever block of that XCD asks; with one release per block, the XCD's L2
// would be written back once per resident block at every barrier.  Here one
// leader block per XCD writes back on behalf of the XCD's blocks:
//   1. every wave waits for its own stores (they are then in its XCD's L2);
//      a non-leader block adds one to its XCD's arrival counter;
//   2. the leader waits for the XCD's other blocks, writes the L2 back
//      (agent release) and publishes the epoch in the XCD's line;
//   3. the master (leader of the lowest XCD with blocks) waits for every
//      XCD's line and publishes the epoch in the control word;
//   4. every block waits for it and acquires at agent scope (this
//      invalidates its CU's L1 and its XCD's L2: an invalidation at
//      workgroup scope does not reach the L1 outside split-workgroup mode,
//      and without it other CUs' stores were seen stale).
// The XCD comes from the hardware register HW_REG_XCC_ID, so nothing rests
// on how blocks are dealt to XCDs.  Every wait is bounded as in grid_barrier.
struct XBar {
    uint32_t *arr, *pub;         // per-XCD lines, 32 words apart
    int x, slot, rank, nxcd;     // this block's XCD, its place there, the XCD's rank among used ones
    uint32_t nx, present;        // blocks on this XCD; mask of XCDs with blocks
    bool leader, master;
};

__device__ __forceinline__ uint32_t hw_xcc_id()
{
    // hardware register 20 (XCC_ID), bits 3:0
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15u;
}

// Registration: each block takes a place on its XCD, then one full barrier
// makes every count final.  Returns the state every later barrier uses.
__device__ XBar xbar_register(Ctl *ctl, uint32_t *flags, uint32_t &epoch, uint32_t cap)
{
    __shared__ int sh[2];
    uint32_t *reg = flags + (size_t)(kMaxPersistentBlocks - kXBarLines) * 32;
    XBar xb;
    xb.arr = reg + 16 * 32;
    xb.pub = reg + 32 * 32;
    if (threadIdx.x == 0) {
        const uint32_t x = hw_xcc_id();
        sh[0] = (int)x;
        sh[1] = (int)__hip_atomic_fetch_add(&reg[x * 32], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    grid_barrier(ctl, flags, epoch, cap);
    xb.x = sh[0];
    xb.slot = sh[1];
    xb.present = 0;
    xb.rank = 0;
    xb.nx = 1;
    int first = -1;
    for (int y = 0; y < 16; ++y) {
        const uint32_t c = __hip_atomic_load(&reg[y * 32], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (c == 0) continue;
        xb.present |= 1u << y;
        if (first < 0) first = y;
        if (y < xb.x) ++xb.rank;
        if (y == xb.x) xb.nx = c;
    }
    xb.nxcd = __popc(xb.present);
    xb.leader = xb.slot == 0;
    xb.master = xb.leader && xb.x == first;
    return xb;
}

__device__ __forceinline__ void xcd_barrier(Ctl *ctl, const XBar &xb, uint32_t &epoch, uint32_t cap)
{
    __builtin_amdgcn_s_waitcnt(0);   // this wave's stores are acknowledged by its L2
    __syncthreads();
    ++epoch;
    if (threadIdx.x == 0) {
        const int l = xb.x * 32;
        if (!xb.leader) {
            __hip_atomic_fetch_add(&xb.arr[l], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // epoch 1 was the registration barrier: (epoch - 1) of these so far
            barrier_wait(&xb.arr[l], (epoch - 1) * (xb.nx - 1), ctl, cap);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(&xb.pub[l], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (xb.master) {
                for (int y = 0; y < 16; ++y)
                    if ((xb.present >> y) & 1u) barrier_wait(&xb.pub[y * 32], epoch, ctl, cap);
                __hip_atomic_store(&ctl->bar_arrive, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        barrier_wait(&ctl->bar_arrive, epoch, ctl, cap);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __builtin_amdgcn_s_waitcnt(0);   // done before any wave of the block loads
    }
    __syncthreads();
}

// Work items [0, NT) of one phase split into contiguous ranges, one per XCD
// in use (by rank); the blocks of an XCD stride through its range by their
// place on it.
struct XcdRange {
    int u, end, step;
    __device__ __forceinline__ XcdRange(int NT, const XBar &xb)
    {
        const int q = NT / xb.nxcd, rm = NT % xb.nxcd, x = xb.rank;
        const int start = x * q + min(x, rm);
        end = start + q + (x < rm ? 1 : 0);
        step = (int)xb.nx;
        u = start + xb.slot;
    }
};

template <int KM, int FM, int W, int MAXD>
__global__ __launch_bounds__(kRepThreads) void k_rep_persistent(RepLaneArgs a, int ntiles,
                                                                RunArgs ra, uint32_t *flags,
                                                                uint32_t cap)
{
    __shared__ double red[kRedDoubles];   // tile sums, reused by the reductions
    uint32_t epoch = 0;
    const XBar xb = xbar_register(ra.ctl, flags, epoch, cap);
    const int groups = (a.Rp + W - 1) / W;
    for (int t = 0; t < ra.n_mcs_run; ++t) {
        const uint32_t g = ra.g0 + (uint32_t)t;
        double *part = rep_slot(ra, a, ntiles, t & 1);
        double *chk = rep_chunk_slot(ra, a, t & 1);
        if (rep_recompute_due(g % (uint32_t)ra.M, ra.P)) {
            for (int u = blockIdx.x; u < ntiles * groups; u += gridDim.x)
                rep_tile_energy<KM, FM, W, MAXD>(a, u % ntiles, u / ntiles, g, ra, part, red);
            // the energy reads spins that colour 0 is about to change
            xcd_barrier(ra.ctl, xb, epoch, cap);
        }
        for (int c = 0; c < a.ncol; ++c) {
            const int nt = a.tile_off[c + 1] - a.tile_off[c];
            for (XcdRange it(nt * groups, xb); it.u < it.end; it.u += it.step) {
                const int u = it.u % nt;
                rep_tile<KM, FM, W, MAXD>(a, c, a.tord ? a.tord[a.tile_off[c] + u] : u, it.u / nt, g, ra,
                                          part, red);
            }
            xcd_barrier(ra.ctl, xb, epoch, cap);
            // the chunk sums of the previous MCS are complete once colour 0
            // of this one is: the last block adds them and writes its history
            if (c == 0 && t > 0 && blockIdx.x == gridDim.x - 1)
                rep_final(a, g - 1, ra, rep_chunk_slot(ra, a, (t - 1) & 1),
                          ra.carry + (size_t)((t - 1) & 1) * 6 * a.Rp, red);
        }
        for (int k = blockIdx.x; k < kChunks; k += gridDim.x) rep_chunk_sum(a, ntiles, k, part, chk, red);
    }
    xcd_barrier(ra.ctl, xb, epoch, cap);
    if (blockIdx.x == gridDim.x - 1 && ra.n_mcs_run > 0) {
        const int t = ra.n_mcs_run - 1;
        rep_final(a, ra.g0 + (uint32_t)t, ra, rep_chunk_slot(ra, a, t & 1),
                  ra.carry + (size_t)(t & 1) * 6 * a.Rp, red);
        if (threadIdx.x == 0) ra.ctl->g = ra.g0 + (uint32_t)ra.n_mcs_run;
    }
}

// ------------------------------------------------------------ init / copy
__global__ void k_init_spins_rep(RepLaneArgs a, int mode, const double *given, uint64_t seed)
{
    const int i = blockIdx.x;
    const size_t plane = (size_t)a.cs;
    for (int r = threadIdx.x; r < a.Rp; r += blockDim.x) {
        double x = 0.0, y = 0.0, z = 1.0;
        if (r < a.R) {
            const uint32_t o = a.orig[i];
            if (mode == 2) {
                sphere64(seed, o, 0xFFFFFFFFu, a.rep_id[r], x, y, z);
            } else if (mode == 0) {
                const double *gv = given + 3 * ((size_t)r * a.n + o);
                x = gv[0];
                y = gv[1];
                z = gv[2];
            }
            if (mode != 0 && a.mu_d) {   // cold and random starts: spins of length mu
                const double mu = a.mu_d[i];
                x = mu * x;
                y = mu * y;
                z = mu * z;
            }
        }
        const size_t oi = (size_t)i * a.ss + r;
        a.spins[oi] = (float)x;
        a.spins[plane + oi] = (float)y;
        a.spins[2 * plane + oi] = (float)z;
    }
}

__global__ void k_to_user_rep(RepLaneArgs a, int rep, double *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const size_t plane = (size_t)a.cs, oi = (size_t)i * a.ss + rep;
    const uint32_t o = a.orig[i];
    out[3 * (size_t)o] = a.spins[oi];
    out[3 * (size_t)o + 1] = a.spins[plane + oi];
    out[3 * (size_t)o + 2] = a.spins[2 * plane + oi];
}

hipError_t launch_init_spins_rep(hipStream_t st, const RepLaneArgs &a, int mode,
                                 const double *given, uint64_t seed)
{
    hipLaunchKernelGGL(k_init_spins_rep, dim3((unsigned)a.n), dim3(64), 0, st, a, mode, given, seed);
    return hipGetLastError();
}

hipError_t launch_to_user_rep(hipStream_t st, const RepLaneArgs &a, int rep, double *out)
{
    hipLaunchKernelGGL(k_to_user_rep, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a,
                       rep, out);
    return hipGetLastError();
}

#define HSIM_DISPATCH_KF2(KM_, FM_, ...)                                                         \
    do {                                                                                          \
        if ((KM_) == K_NONE && (FM_) == F_UNIFORM) { constexpr int KM = K_NONE, FM = F_UNIFORM; __VA_ARGS__; } \
        else if ((KM_) == K_NONE) { constexpr int KM = K_NONE, FM = F_SITE; __VA_ARGS__; }        \
        else if ((KM_) == K_UNIFORM && (FM_) == F_UNIFORM) { constexpr int KM = K_UNIFORM, FM = F_UNIFORM; __VA_ARGS__; } \
        else if ((KM_) == K_UNIFORM) { constexpr int KM = K_UNIFORM, FM = F_SITE; __VA_ARGS__; }  \
        else if ((FM_) == F_UNIFORM) { constexpr int KM = K_SITE, FM = F_UNIFORM; __VA_ARGS__; }  \
        else { constexpr int KM = K_SITE, FM = F_SITE; __VA_ARGS__; }                             \
    } while (0)
#define HSIM_DISPATCH_KFW(KM_, FM_, W_, ...)                                                     \
    do {                                                                                          \
        if ((W_) == 64) { constexpr int W = 64; HSIM_DISPATCH_KF2(KM_, FM_, __VA_ARGS__); }       \
        else { constexpr int W = 32; HSIM_DISPATCH_KF2(KM_, FM_, __VA_ARGS__); }                  \
    } while (0)

static int lane_width(const RepLaneArgs &a) { return a.Rp % 64 == 0 ? 64 : 32; }

// Rows padded to 6 or 8 slots use the fixed-width pair updates (the plan
// pads to 6 when every row has at most 6 entries, else to 8); wider rows the
// generic row walk.
#define HSIM_DISPATCH_D(ELLW_, ...)                                                             \
    do {                                                                                         \
        if ((ELLW_) == 6) { constexpr int MAXD = 6; __VA_ARGS__; }                               \
        else if ((ELLW_) == 8) { constexpr int MAXD = 8; __VA_ARGS__; }                          \
        else { constexpr int MAXD = 0; __VA_ARGS__; }                                            \
    } while (0)

hipError_t launch_rep_phase(hipStream_t st, int kmode, int fmode, int colour, int t_off,
                            const RepLaneArgs &a, int ntiles, const RunArgs &ra)
{
    const int nt = a.tile_off[colour + 1] - a.tile_off[colour];
    if (nt <= 0) return hipSuccess;
    const int Wd = lane_width(a);
    dim3 grid((unsigned)nt, (unsigned)(a.Rp / Wd));
    dim3 blk(kRepThreads);
    HSIM_DISPATCH_KFW(kmode, fmode, Wd, HSIM_DISPATCH_D(a.ell_w, {
        const int var = (ra.pol.n_types > 0 ? VAR_POL : 0) | (a.kc || a.mu ? VAR_XT : 0) |
                        (ra.trace ? VAR_TRACE : 0);
        if ((var & VAR_TRACE) && var != VAR_TRACE) return hipErrorInvalidValue;
        if (var == VAR_TRACE)
            hipLaunchKernelGGL((k_rep_phase<KM, FM, W, MAXD, VAR_TRACE>), grid, blk, 0, st, a,
                               colour, t_off, ntiles, ra);
        else if (var == 0)
            hipLaunchKernelGGL((k_rep_phase<KM, FM, W, MAXD, 0>), grid, blk, 0, st, a, colour,
                               t_off, ntiles, ra);
        else if (var == VAR_POL)
            hipLaunchKernelGGL((k_rep_phase<KM, FM, W, MAXD, VAR_POL>), grid, blk, 0, st, a, colour,
                               t_off, ntiles, ra);
        else if (var == VAR_XT)
            hipLaunchKernelGGL((k_rep_phase<KM, FM, W, MAXD, VAR_XT>), grid, blk, 0, st, a, colour,
                               t_off, ntiles, ra);
        else
            hipLaunchKernelGGL((k_rep_phase<KM, FM, W, MAXD, VAR_POL | VAR_XT>), grid, blk, 0, st,
                               a, colour, t_off, ntiles, ra);
    }));
    return hipGetLastError();
}

hipError_t launch_rep_sigma(hipStream_t st, const RepLaneArgs &a, int ntiles, int t_off,
                            const RunArgs &ra)
{
    hipLaunchKernelGGL(k_rep_sigma, dim3(kChunks), dim3(256), 0, st, a, ntiles, t_off, ra);
    return hipGetLastError();
}

hipError_t launch_rep_efull(hipStream_t st, int kmode, int fmode, const RepLaneArgs &a,
                            int ntiles, int t_off, const RunArgs &ra)
{
    const int Wd = lane_width(a);
    dim3 grid((unsigned)ntiles, (unsigned)(a.Rp / Wd)), blk(kRepThreads);
    HSIM_DISPATCH_KFW(kmode, fmode, Wd, HSIM_DISPATCH_D(a.ell_w, {
        hipLaunchKernelGGL((k_rep_efull<KM, FM, W, MAXD>), grid, blk, 0, st, a, t_off, ntiles, ra);
    }));
    return hipGetLastError();
}

hipError_t launch_rep_reduce(hipStream_t st, const RepLaneArgs &a, int ntiles, int t_first,
                             int count, int advance, const RunArgs &ra)
{
    if (count < 1 || count > ra.rec_win) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rep_chunks, dim3(kChunks, (unsigned)count), dim3(1024), 0, st, a, ntiles,
                       t_first, ra);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rep_finals, dim3((unsigned)count), dim3(256), 0, st, a, t_first, count,
                       advance, ra);
    return hipGetLastError();
}

hipError_t launch_rep_persistent(hipStream_t st, int kmode, int fmode, const RepLaneArgs &a,
                                 int ntiles, int grid, const RunArgs &ra, uint32_t *flags,
                                 uint32_t spin_cap)
{
    if (grid > kMaxPersistentBlocks - kXBarLines || ra.rec_win < 2) return hipErrorInvalidValue;
    hipError_t e = launch_fill_u32(st, flags, 0u, (int64_t)grid * 32);
    if (e != hipSuccess) return e;
    e = launch_fill_u32(st, flags + (size_t)(kMaxPersistentBlocks - kXBarLines) * 32, 0u,
                        (int64_t)kXBarLines * 32);
    if (e != hipSuccess) return e;
    const int Wd = lane_width(a);
    HSIM_DISPATCH_KFW(kmode, fmode, Wd, HSIM_DISPATCH_D(a.ell_w, {
        hipLaunchKernelGGL((k_rep_persistent<KM, FM, W, MAXD>), dim3((unsigned)grid),
                           dim3(kRepThreads), 0, st, a, ntiles, ra, flags, spin_cap);
    }));
    return hipGetLastError();
}

int rep_persistent_blocks_per_cu(int kmode, int fmode, int lane_w, int ell_w)
{
    int nb = 0;
    HSIM_DISPATCH_KFW(kmode, fmode, lane_w, HSIM_DISPATCH_D(ell_w, {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rep_persistent<KM, FM, W, MAXD>, kRepThreads, 0) != hipSuccess)
            nb = 0;
    }));
    return nb;
}

}  // namespace hsim
