// Replica-lane sweep: replicas that share one lattice are updated together,
// one lane per replica of one site.  Spins are [3][n][Rp] (Rp = replicas
// padded to the lane-group width W), so every neighbour read of a wave is a
// contiguous 4*W-byte row and the CSR row of a site (offsets, columns,
// constants) is read once for W replicas.
//
// Paper: Eq. 1-2 (energy), Eq. 4 (acceptance), section "Monte Carlo
// Metropolis algorithm" (one attempt per site per MCS); history per MCS
// (section "VEGAS software package").  Replicas are independent chains, each
// with its own temperature and field schedule.
//
// A tile is kRepTile consecutive sites of one colour class; wave w of the
// tile's block takes 32 of them, in order.  Per-MCS history: every tile writes
// one record per replica; records are summed in 64 fixed chunks of tiles, and
// the chunks in order, the same way in every launch mode.
#include "hsim_dev.h"
#include "update.h"

namespace hsim {

namespace {

constexpr int kChunks = 64;

__device__ __forceinline__ bool rep_recompute_due(uint32_t m, int P)
{
    return m == 0 || (P > 0 && (m % (uint32_t)P) == 0);
}

template <int KM, int FM>
struct RepSite {
    float k, ex, ey, ez, nx, ny, nz;
    __device__ __forceinline__ RepSite(const RepLaneArgs &a, int i)
    {
        if (KM == K_SITE) {
            k = a.k[i];
            ex = a.ax[i];
            ey = a.ax[a.n + i];
            ez = a.ax[2 * a.n + i];
        } else {
            k = (KM == K_UNIFORM) ? a.k0 : 0.0f;
            ex = a.e0x;
            ey = a.e0y;
            ez = a.e0z;
        }
        if (FM == F_SITE) {
            nx = a.nd[i];
            ny = a.nd[a.n + i];
            nz = a.nd[2 * a.n + i];
        } else {
            nx = a.n0x;
            ny = a.n0y;
            nz = a.n0z;
        }
    }
};

// Update site i for replica lane r (spin column r of the [3][n][Rp] array).
template <int KM, int FM>
__device__ __forceinline__ void rep_site_update(const RepLaneArgs &a, int i, int r, uint32_t g,
                                                float beta, float b, uint32_t rid, bool active,
                                                const RunArgs &ra, double (&acc)[5])
{
    const size_t plane = (size_t)a.n * a.Rp;
    float *S = a.spins + r;
    const int32_t rb = a.rp[i], re = a.rp[i + 1];
    float hx = 0.0f, hy = 0.0f, hz = 0.0f;
    for (int32_t p = rb; p < re; ++p) {
        const size_t o = (size_t)a.ci[p] * a.Rp;
        const float Jp = a.J[p];
        hx = fmaf(Jp, S[o], hx);
        hy = fmaf(Jp, S[plane + o], hy);
        hz = fmaf(Jp, S[2 * plane + o], hz);
    }
    const RepSite<KM, FM> sp(a, i);
    hx = fmaf(b, sp.nx, hx);
    hy = fmaf(b, sp.ny, hy);
    hz = fmaf(b, sp.nz, hz);
    const size_t oi = (size_t)i * a.Rp;
    const float sx = S[oi], sy = S[plane + oi], sz = S[2 * plane + oi];
    const Trial32 t = trial32(draw(ra.seed, a.orig[i], g, rid, 0));
    const float dE = (KM == K_NONE) ? delta_e32_iso(sx, sy, sz, t, hx, hy, hz)
                                    : delta_e32(sx, sy, sz, t, hx, hy, hz, sp.k, sp.ex, sp.ey, sp.ez);
    const bool ok = accept32(dE, beta, t.u) && active;
    if (active && dE != dE) atomicOr(&ra.ctl->status, 1u);
    if (ok) {
        S[oi] = t.x;
        S[plane + oi] = t.y;
        S[2 * plane + oi] = t.z;
        acc[0] += (double)dE;
        acc[4] += 1.0;
        acc[1] += (double)t.x;
        acc[2] += (double)t.y;
        acc[3] += (double)t.z;
    } else if (active) {
        acc[1] += (double)sx;
        acc[2] += (double)sy;
        acc[3] += (double)sz;
    }
}

template <int KM, int FM>
__device__ __forceinline__ double rep_site_energy(const RepLaneArgs &a, int i, int r, double b)
{
    const size_t plane = (size_t)a.n * a.Rp;
    const float *S = a.spins + r;
    double hx = 0.0, hy = 0.0, hz = 0.0;
    for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
        const size_t o = (size_t)a.ci[p] * a.Rp;
        const double Jp = (double)a.J[p];
        hx += Jp * (double)S[o];
        hy += Jp * (double)S[plane + o];
        hz += Jp * (double)S[2 * plane + o];
    }
    const RepSite<KM, FM> sp(a, i);
    const size_t oi = (size_t)i * a.Rp;
    const double sx = S[oi], sy = S[plane + oi], sz = S[2 * plane + oi];
    const double an = sx * (double)sp.ex + sy * (double)sp.ey + sz * (double)sp.ez;
    const double zn = sx * (double)sp.nx + sy * (double)sp.ny + sz * (double)sp.nz;
    return -0.5 * (sx * hx + sy * hy + sz * hz) - b * zn - (double)sp.k * an * an;
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
// the persistent kernel.  red: LDS [kRepWaves][64][5].
template <int KM, int FM, int W>
__device__ __forceinline__ void rep_tile(const RepLaneArgs &a, int colour, int tile, int group,
                                         uint32_t g, const RunArgs &ra, double *part,
                                         double *red)
{
    constexpr int SPL = kRepSitesPerWave * W / 64;   // sites per lane group
    const Lanes<W> L(group);
    const int ce = a.cls_off[colour + 1];
    const int base = a.cls_off[colour] + tile * kRepTile + L.w * kRepSitesPerWave + L.sub * SPL;
    const bool active = L.r < a.R;
    const uint32_t s_abs = g / (uint32_t)ra.M;
    float beta = 0.0f, b = 0.0f;
    uint32_t rid = 0;
    if (active) {
        const size_t sidx = (size_t)L.r * ra.S_hist + s_abs;
        beta = (float)ra.beta[sidx];
        b = (float)ra.bfield[sidx];
        rid = a.rep_id[L.r];
    }
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j < SPL; ++j) {
        const int i = base + j;
        if (i >= ce) break;
        rep_site_update<KM, FM>(a, i, L.r, g, beta, b, rid, active, ra, acc);
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) red[(L.w * 64 + L.lane) * 5 + q] = acc[q];
    __syncthreads();
    if (threadIdx.x < W) {
        double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int ww = 0; ww < kRepWaves; ++ww)
            for (int sb = 0; sb < 64 / W; ++sb)
#pragma unroll
                for (int q = 0; q < 5; ++q) v[q] += red[(ww * 64 + sb * W + (int)threadIdx.x) * 5 + q];
        const int rr = (int)threadIdx.x + W * group;
        const int tg = a.tile_off[colour] + tile;
#pragma unroll
        for (int q = 0; q < 5; ++q) part[((size_t)tg * kRecFields + q) * a.Rp + rr] = v[q];
    }
    __syncthreads();
}

// Energy records of one tile (field 5).
template <int KM, int FM, int W>
__device__ __forceinline__ void rep_tile_energy(const RepLaneArgs &a, int tg, int group,
                                                uint32_t g, const RunArgs &ra, double *part,
                                                double *red)
{
    constexpr int SPL = kRepSitesPerWave * W / 64;
    const Lanes<W> L(group);
    int colour = 0;
    while (colour + 1 < a.ncol && a.tile_off[colour + 1] <= tg) ++colour;
    const int tile = tg - a.tile_off[colour];
    const int ce = a.cls_off[colour + 1];
    const int base = a.cls_off[colour] + tile * kRepTile + L.w * kRepSitesPerWave + L.sub * SPL;
    double e = 0.0;
    if (L.r < a.R) {
        const double b = ra.bfield[(size_t)L.r * ra.S_hist + g / (uint32_t)ra.M];
        for (int j = 0; j < SPL; ++j) {
            const int i = base + j;
            if (i >= ce) break;
            e += rep_site_energy<KM, FM>(a, i, L.r, b);
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

// Chunk k of the tile records: sequential sum over its tiles, per replica.
__device__ __forceinline__ void rep_chunk_sum(const RepLaneArgs &a, int ntiles, int k, int rr,
                                              const double *part, double *chunk)
{
    const int tb = (int)((int64_t)ntiles * k / kChunks), te = (int)((int64_t)ntiles * (k + 1) / kChunks);
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int t = tb; t < te; ++t)
#pragma unroll
        for (int q = 0; q < 6; ++q) v[q] += part[((size_t)t * kRecFields + q) * a.Rp + rr];
#pragma unroll
    for (int q = 0; q < 6; ++q) chunk[((size_t)k * 6 + q) * a.Rp + rr] = v[q];
}

// Final sum over chunks in order; writes history and the carried energy.
__device__ __forceinline__ void rep_final(const RepLaneArgs &a, int rr, uint32_t g,
                                          const RunArgs &ra, const double *chunk)
{
    if (rr >= a.R) return;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < kChunks; ++k)
#pragma unroll
        for (int q = 0; q < 6; ++q) v[q] += chunk[((size_t)k * 6 + q) * a.Rp + rr];
    const uint32_t s_abs = g / (uint32_t)ra.M, m = g % (uint32_t)ra.M;
    const double E = (rep_recompute_due(m, ra.P) ? v[5] : ra.ecarry[rr]) + v[0];
    ra.ecarry[rr] = E;
    double *h = ra.history + (((size_t)rr * ra.S_hist + s_abs) * ra.M + m) * 5;
    h[0] = E;
    h[1] = v[1];
    h[2] = v[2];
    h[3] = v[3];
    h[4] = v[4];
}

}  // namespace

// Per-phase kernel: grid (tiles of the colour, replica groups).
template <int KM, int FM, int W>
__global__ __launch_bounds__(256) void k_rep_phase(RepLaneArgs a, int colour, RunArgs ra)
{
    __shared__ double red[kRepWaves * 64 * 5];
    rep_tile<KM, FM, W>(a, colour, blockIdx.x, blockIdx.y, ra.ctl->g, ra, ra.partials, red);
}

template <int KM, int FM, int W>
__global__ __launch_bounds__(256) void k_rep_efull(RepLaneArgs a, RunArgs ra)
{
    __shared__ double red[kRepWaves * 64 * 5];
    const uint32_t g = ra.ctl->g;
    if (!rep_recompute_due(g % (uint32_t)ra.M, ra.P)) return;
    rep_tile_energy<KM, FM, W>(a, blockIdx.x, blockIdx.y, g, ra, ra.partials, red);
}

// Reduction: block k (k < 64) sums chunk k for all replicas; the last block to
// finish adds the chunks in order, writes the history and advances g.
__global__ __launch_bounds__(256) void k_rep_reduce(RepLaneArgs a, int ntiles, RunArgs ra,
                                                    double *chunk)
{
    __shared__ int last;
    const uint32_t g = ra.ctl->g;
    for (int rr = threadIdx.x; rr < a.Rp; rr += blockDim.x)
        rep_chunk_sum(a, ntiles, blockIdx.x, rr, ra.partials, chunk);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = (atomicAdd(&ra.ctl->pad[0], 1u) == gridDim.x - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    for (int rr = threadIdx.x; rr < a.Rp; rr += blockDim.x) rep_final(a, rr, g, ra, chunk);
    __syncthreads();
    if (threadIdx.x == 0) {
        ra.ctl->pad[0] = 0;
        ra.ctl->g = g + 1;
    }
}

// ------------------------------------------------------------- persistent
// One launch for the whole run.  Device-wide barrier: a monotone arrival
// counter; every wait is bounded (spin_cap sleeps) and any timeout, once
// flagged, releases every later wait at once, so the grid always drains.
__device__ __forceinline__ void grid_barrier(Ctl *ctl, uint32_t &epoch, uint32_t cap)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        ++epoch;
        const uint32_t target = epoch * gridDim.x;
        __threadfence();
        __hip_atomic_fetch_add(&ctl->bar_arrive, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t n = 0;
        while (__hip_atomic_load(&ctl->bar_arrive, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++n > cap ||
                (__hip_atomic_load(&ctl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2u)) {
                atomicOr(&ctl->status, 2u);
                break;
            }
        }
        __threadfence();
    }
    __syncthreads();
}

template <int KM, int FM, int W>
__global__ __launch_bounds__(256) void k_rep_persistent(RepLaneArgs a, int ntiles, RunArgs ra,
                                                        double *chunk, uint32_t cap)
{
    __shared__ double red[kRepWaves * 64 * 5];
    uint32_t epoch = 0;
    const int groups = (a.Rp + W - 1) / W;
    for (int t = 0; t < ra.n_mcs_run; ++t) {
        const uint32_t g = ra.g0 + (uint32_t)t;
        double *part = ra.partials + (size_t)(t & 1) * ntiles * kRecFields * a.Rp;
        double *chk = chunk + (size_t)(t & 1) * kChunks * 6 * a.Rp;
        if (rep_recompute_due(g % (uint32_t)ra.M, ra.P)) {
            for (int u = blockIdx.x; u < ntiles * groups; u += gridDim.x)
                rep_tile_energy<KM, FM, W>(a, u % ntiles, u / ntiles, g, ra, part, red);
            // the energy reads spins that colour 0 is about to change
            grid_barrier(ra.ctl, epoch, cap);
        }
        for (int c = 0; c < a.ncol; ++c) {
            const int nt = a.tile_off[c + 1] - a.tile_off[c];
            for (int u = blockIdx.x; u < nt * groups; u += gridDim.x)
                rep_tile<KM, FM, W>(a, c, u % nt, u / nt, g, ra, part, red);
            grid_barrier(ra.ctl, epoch, cap);
            // the chunk sums of the previous MCS are complete once colour 0
            // of this one is: add them in order and write its history
            if (c == 0 && t > 0 && blockIdx.x == 0)
                for (int rr = threadIdx.x; rr < a.Rp; rr += blockDim.x)
                    rep_final(a, rr, g - 1, ra, chunk + (size_t)((t - 1) & 1) * kChunks * 6 * a.Rp);
        }
        for (int k = blockIdx.x; k < kChunks; k += gridDim.x)
            for (int rr = threadIdx.x; rr < a.Rp; rr += blockDim.x)
                rep_chunk_sum(a, ntiles, k, rr, part, chk);
    }
    grid_barrier(ra.ctl, epoch, cap);
    if (blockIdx.x == 0 && ra.n_mcs_run > 0) {
        const int t = ra.n_mcs_run - 1;
        for (int rr = threadIdx.x; rr < a.Rp; rr += blockDim.x)
            rep_final(a, rr, ra.g0 + (uint32_t)t, ra, chunk + (size_t)(t & 1) * kChunks * 6 * a.Rp);
        __syncthreads();
        if (threadIdx.x == 0) ra.ctl->g = ra.g0 + (uint32_t)ra.n_mcs_run;
    }
}

// ------------------------------------------------------------ init / copy
__global__ void k_init_spins_rep(RepLaneArgs a, int mode, const double *given, uint64_t seed)
{
    const int i = blockIdx.x;
    const size_t plane = (size_t)a.n * a.Rp;
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
        }
        const size_t oi = (size_t)i * a.Rp + r;
        a.spins[oi] = (float)x;
        a.spins[plane + oi] = (float)y;
        a.spins[2 * plane + oi] = (float)z;
    }
}

__global__ void k_to_user_rep(RepLaneArgs a, int rep, double *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const size_t plane = (size_t)a.n * a.Rp, oi = (size_t)i * a.Rp + rep;
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

hipError_t launch_rep_phase(hipStream_t st, int kmode, int fmode, int colour,
                            const RepLaneArgs &a, const RunArgs &ra)
{
    const int nt = a.tile_off[colour + 1] - a.tile_off[colour];
    if (nt <= 0) return hipSuccess;
    const int Wd = lane_width(a);
    dim3 grid((unsigned)nt, (unsigned)(a.Rp / Wd)), blk(256);
    HSIM_DISPATCH_KFW(kmode, fmode, Wd, {
        hipLaunchKernelGGL((k_rep_phase<KM, FM, W>), grid, blk, 0, st, a, colour, ra);
    });
    return hipGetLastError();
}

hipError_t launch_rep_efull(hipStream_t st, int kmode, int fmode, const RepLaneArgs &a,
                            int ntiles, const RunArgs &ra)
{
    const int Wd = lane_width(a);
    dim3 grid((unsigned)ntiles, (unsigned)(a.Rp / Wd)), blk(256);
    HSIM_DISPATCH_KFW(kmode, fmode, Wd, {
        hipLaunchKernelGGL((k_rep_efull<KM, FM, W>), grid, blk, 0, st, a, ra);
    });
    return hipGetLastError();
}

hipError_t launch_rep_reduce(hipStream_t st, const RepLaneArgs &a, int ntiles, const RunArgs &ra)
{
    // chunk sums live right after the tile records (two parities) in the workspace
    double *chunk = ra.partials + (size_t)2 * ntiles * kRecFields * a.Rp;
    hipLaunchKernelGGL(k_rep_reduce, dim3(kChunks), dim3(256), 0, st, a, ntiles, ra, chunk);
    return hipGetLastError();
}

hipError_t launch_rep_persistent(hipStream_t st, int kmode, int fmode, const RepLaneArgs &a,
                                 int ntiles, int grid, const RunArgs &ra, uint32_t spin_cap)
{
    double *chunk = ra.partials + (size_t)2 * ntiles * kRecFields * a.Rp;
    const int Wd = lane_width(a);
    HSIM_DISPATCH_KFW(kmode, fmode, Wd, {
        hipLaunchKernelGGL((k_rep_persistent<KM, FM, W>), dim3((unsigned)grid), dim3(256), 0, st,
                           a, ntiles, ra, chunk, spin_cap);
    });
    return hipGetLastError();
}

int rep_persistent_blocks_per_cu(int kmode, int fmode, int lane_w)
{
    int nb = 0;
    HSIM_DISPATCH_KFW(kmode, fmode, lane_w, {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rep_persistent<KM, FM, W>, 256, 0) != hipSuccess)
            nb = 0;
    });
    return nb;
}

}  // namespace hsim
