// Sweep kernels of the colour-ordered Metropolis Monte Carlo (gfx950, wave64,
// no MFMA: the update is a sparse gather, not a dense contraction).
//
// Paper: Eq. 1-2 (energy), Eq. 4 (acceptance), one attempt per site per MCS
// (section "Monte Carlo Metropolis algorithm"); history of E and M after every
// MCS of every temperature/field step (section "VEGAS software package").
//
// All sites of one colour class have no link between them, so one class is
// updated in parallel; classes follow each other, separated by a kernel
// boundary (site-lane and replica-lane phases), a workgroup barrier (block
// layout) or a device-wide barrier (persistent launch).
//
// History sums are deterministic: each tile (a block's share of a class)
// reduces its sites in a fixed order (wave butterfly, then waves in order) and
// the per-MCS reduction adds tile records in table order.
#include "hsim_dev.h"
#include "update.h"

namespace hsim {

namespace {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum NV values over the block; the result is valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) lds[w * NV + q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int ww = 1; ww < nw; ++ww)
#pragma unroll
            for (int q = 0; q < NV; ++q) v[q] += lds[ww * NV + q];
    }
    __syncthreads();
}

__device__ __forceinline__ bool recompute_due(uint32_t m, int P)
{
    return m == 0 || (P > 0 && (m % (uint32_t)P) == 0);
}

__device__ __forceinline__ void adapt_sigma(const RunArgs &ra, int r, double n_acc)
{
    ra.sigma[r] = adapted_sigma(ra.sigma[r], n_acc, ra.n_ad[r], ra.pol.sigma_min, ra.pol.sigma_max);
}

template <typename T>
__device__ __forceinline__ T as_t(double v)
{
    return (T)v;
}

// Site parameters: anisotropy constant and axis, field direction.
template <typename T, int KM, int FM>
struct SiteParams {
    T k, ex, ey, ez, nx, ny, nz;
    __device__ __forceinline__ SiteParams(const RepDesc &rd, int i)
    {
        if (KM == K_SITE) {
            const T *kk = (const T *)rd.k;
            const T *ax = (const T *)rd.ax;
            k = kk[i];
            ex = ax[i];
            ey = ax[rd.n + i];
            ez = ax[2 * rd.n + i];
        } else {
            k = (KM == K_UNIFORM) ? as_t<T>(rd.k0) : T(0);
            ex = as_t<T>(rd.e0[0]);
            ey = as_t<T>(rd.e0[1]);
            ez = as_t<T>(rd.e0[2]);
        }
        if (FM == F_SITE) {
            const T *nd = (const T *)rd.nd;
            nx = nd[i];
            ny = nd[rd.n + i];
            nz = nd[2 * rd.n + i];
        } else {
            nx = as_t<T>(rd.n0[0]);
            ny = as_t<T>(rd.n0[1]);
            nz = as_t<T>(rd.n0[2]);
        }
    }
};

// One site's update in the site-lane / block layouts.  S points at the
// replica's spins [3][n_pad] (global or LDS).  Returns the accumulators.
// Exchange field of site i: the CSR row walk (MAXD == 0) or the padded row of
// MAXD slots (slot-major copy, coalesced across the lanes of a wave).  A
// padding slot holds the site itself with constant 0 and leaves every sum
// unchanged, so both walks give the same bits.  Slots from nsl on are padding
// for every site of the block's tile (the same in every lane; the surface
// layers of a film, one neighbour short, leave their last slot empty): they
// are read at the tile's first site, ts, whose entry there is padding too
// (itself, constant 0), so every lane reads one cached line instead of the
// tile's stretch of the slot, and the sum is unchanged (h + 0 * S_ts == h for
// the finite, never negative-zero partial sums h).
template <typename T, int MAXD>
__device__ __forceinline__ void exchange_field(const RepDesc &rd, const T *S, int i, T &hx, T &hy,
                                               T &hz, int nsl = MAXD, int ts = 0)
{
    const int np = rd.n_pad;
    hx = T(0);
    hy = T(0);
    hz = T(0);
    if constexpr (MAXD > 0) {
        const T *EJ = (const T *)rd.ellT_J;
#pragma unroll
        for (int sl = 0; sl < MAXD; ++sl) {
            const int src = sl < nsl ? i : ts;
            const int32_t j = rd.ellT_col[sl * rd.n + src];
            const T Jp = EJ[sl * rd.n + src];
            if constexpr (sizeof(T) == 4) {
                hx = fmaf(Jp, S[j], hx);
                hy = fmaf(Jp, S[np + j], hy);
                hz = fmaf(Jp, S[2 * np + j], hz);
            } else {
                hx = hx + Jp * S[j];
                hy = hy + Jp * S[np + j];
                hz = hz + Jp * S[2 * np + j];
            }
        }
    } else {
        const T *J = (const T *)rd.J;
        for (int32_t p = rd.rp[i]; p < rd.rp[i + 1]; ++p) {
            const int32_t j = rd.ci[p];
            const T Jp = J[p];
            if constexpr (sizeof(T) == 4) {
                hx = fmaf(Jp, S[j], hx);
                hy = fmaf(Jp, S[np + j], hy);
                hz = fmaf(Jp, S[2 * np + j], hz);
            } else {
                hx = hx + Jp * S[j];
                hy = hy + Jp * S[np + j];
                hz = hz + Jp * S[2 * np + j];
            }
        }
    }
}

// sigma: the replica's adaptive width; ad counts accepted adaptive moves.
template <typename T, int KM, int FM, bool TRACE, int MAXD>
__device__ __forceinline__ void site_update(const RepDesc &rd, T *S, int i, uint32_t g,
                                            const RunArgs &ra, int rep, T beta, T b,
                                            double sigma, double (&acc)[5], double &ad,
                                            int nsl = MAXD, int ts = 0, bool given = false,
                                            double gu = 0.0, double gx = 0.0, double gy = 0.0,
                                            double gz = 0.0)
{
    const int np = rd.n_pad;
    const SiteParams<T, KM, FM> sp(rd, i);
    const T sx = S[i], sy = S[np + i], sz = S[2 * np + i];
    const uint32_t orig = rd.orig[i];
    bool acc_move;
    T nx, ny, nz, dE;
    T hx, hy, hz;
    exchange_field<T, MAXD>(rd, S, i, hx, hy, hz, nsl, ts);
    SitePol pl{POL_RANDOM, 0.0, 1.0};
    if (ra.pol.n_types > 0) {
        pl = pick_policy(ra.pol.pol, ra.pol.param, ra.pol.cos_t, rd.type ? rd.type[i] : 0);
        if (pl.pol == POL_ADAPTIVE) pl.param = sigma;
    }
    if constexpr (sizeof(T) == 4) {
        hx = fmaf(b, sp.nx, hx);
        hy = fmaf(b, sp.ny, hy);
        hz = fmaf(b, sp.nz, hz);
        const uint4 w0 = draw(ra.seed, orig, g, rd.rep_id, 0);
        const float mu = rd.mu ? ((const float *)rd.mu)[i] : 1.0f;
        const float inv = rd.mu ? 1.0f / mu : 1.0f;
        Trial32 t = pl.pol == POL_RANDOM
                        ? trial32(w0)
                        : trial32_policy(pl.pol, w0, sx * inv, sy * inv, sz * inv, (float)pl.param,
                                         (float)(1.0 - pl.cos_t), ra.seed, orig, g, rd.rep_id);
        if (rd.mu) {
            t.x *= mu;
            t.y *= mu;
            t.z *= mu;
        }
        dE = (KM == K_NONE) ? delta_e32_iso(sx, sy, sz, t, hx, hy, hz)
                            : delta_e32(sx, sy, sz, t, hx, hy, hz, sp.k, sp.ex, sp.ey, sp.ez);
        if (rd.kc)
            dE = fmaf(-((const float *)rd.kc)[i], cubic32(t.x, t.y, t.z) - cubic32(sx, sy, sz), dE);
        acc_move = accept32(dE, beta, t.u);
        nx = t.x;
        ny = t.y;
        nz = t.z;
    } else {
        hx = hx + b * sp.nx;
        hy = hy + b * sp.ny;
        hz = hz + b * sp.nz;
        double dd;
        if (rd.kc || rd.mu)
            acc_move = update64_general(pl.pol, pl.param, pl.cos_t, ra.seed, orig, g, rd.rep_id, sx,
                                        sy, sz, hx, hy, hz, sp.k, sp.ex, sp.ey, sp.ez, rd.kc != nullptr,
                                        rd.kc ? ((const double *)rd.kc)[i] : 0.0, rd.mu != nullptr,
                                        rd.mu ? ((const double *)rd.mu)[i] : 1.0, beta, nx, ny, nz, dd);
        else if (pl.pol == POL_RANDOM && given) {
            // update64 with its acceptance word and trial point drawn ahead
            // (draw_ahead64): the same operations in the same order
            nx = gx;
            ny = gy;
            nz = gz;
            const double dSx = nx - sx, dSy = ny - sy, dSz = nz - sz;
            const double q = (dSx * hx + dSy * hy) + dSz * hz;
            const double a1 = dot64(nx, ny, nz, sp.ex, sp.ey, sp.ez);
            const double a0 = dot64(sx, sy, sz, sp.ex, sp.ey, sp.ez);
            dd = -q - sp.k * (a1 * a1 - a0 * a0);
            acc_move = dd <= 0.0 || gu < exp(-beta * dd);
        } else if (pl.pol == POL_RANDOM)
            acc_move = update64(ra.seed, orig, g, rd.rep_id, sx, sy, sz, hx, hy, hz, sp.k, sp.ex,
                                sp.ey, sp.ez, beta, nx, ny, nz, dd);
        else
            acc_move = update64_policy(pl.pol, pl.param, pl.cos_t, ra.seed, orig, g, rd.rep_id, sx,
                                       sy, sz, hx, hy, hz, sp.k, sp.ex, sp.ey, sp.ez, beta, nx, ny,
                                       nz, dd);
        dE = dd;
    }
    ad += (pl.pol == POL_ADAPTIVE && acc_move) ? 1.0 : 0.0;
    if (dE != dE) atomicOr(&ra.ctl->status, 1u);
    if (acc_move) {
        S[i] = nx;
        S[np + i] = ny;
        S[2 * np + i] = nz;
        if (TRACE)
            atomicOr(&ra.trace[((size_t)rep * ra.n_mcs_run + (g - ra.g0)) * ra.trace_words +
                               (orig >> 5)],
                     1u << (orig & 31));
    }
    // branch-free accumulation of the history sums
    acc[0] += acc_move ? (double)dE : 0.0;
    acc[4] += acc_move ? 1.0 : 0.0;
    acc[1] += (double)(acc_move ? nx : sx);
    acc[2] += (double)(acc_move ? ny : sy);
    acc[3] += (double)(acc_move ? nz : sz);
}

// Site energy in double precision, each bond counted half at either end:
//   e_i = -1/2 S_i.sum_j J_ij S_j - B S_i.n_i - k_i (S_i.e_i)^2
template <typename T, int KM, int FM>
__device__ __forceinline__ double site_energy(const RepDesc &rd, const T *S, int i, double b)
{
    const int np = rd.n_pad;
    const T *J = (const T *)rd.J;
    double hx = 0.0, hy = 0.0, hz = 0.0;
    for (int32_t p = rd.rp[i]; p < rd.rp[i + 1]; ++p) {
        const int32_t j = rd.ci[p];
        const double Jp = (double)J[p];
        hx += Jp * (double)S[j];
        hy += Jp * (double)S[np + j];
        hz += Jp * (double)S[2 * np + j];
    }
    const SiteParams<T, KM, FM> sp(rd, i);
    const double sx = S[i], sy = S[np + i], sz = S[2 * np + i];
    const double a = sx * (double)sp.ex + sy * (double)sp.ey + sz * (double)sp.ez;
    const double zn = sx * (double)sp.nx + sy * (double)sp.ny + sz * (double)sp.nz;
    double e = -0.5 * (sx * hx + sy * hy + sz * hz) - b * zn - (double)sp.k * a * a;
    if (rd.kc) e -= (double)((const T *)rd.kc)[i] * cubic64(sx, sy, sz);
    return e;
}

}  // namespace

// ------------------------------------------------------------------ control
__global__ void k_ctl_set(Ctl *ctl, uint32_t g)
{
    if (threadIdx.x == 0) {
        ctl->g = g;
        ctl->bar_arrive = 0;
        ctl->pad[0] = 0;
        ctl->pad[1] = 0;
        ctl->pad[2] = 0;
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_ctl_set(hipStream_t st, Ctl *ctl, uint32_t g)
{
    hipLaunchKernelGGL(k_ctl_set, dim3(1), dim3(64), 0, st, ctl, g);
    return hipGetLastError();
}

hipError_t launch_fill_u32(hipStream_t st, uint32_t *p, uint32_t v, int64_t n)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

__global__ void k_put_schedule(double *beta, double *bfield, int S_hist, int first_step,
                               int n_steps, int k0, int cnt, PutPairs vals)
{
    const int j = threadIdx.x;
    if (j >= cnt) return;
    const int k = k0 + j, r = k / n_steps, s = k - r * n_steps;
    const size_t off = (size_t)r * S_hist + first_step + s;
    beta[off] = vals.v[2 * j];
    bfield[off] = vals.v[2 * j + 1];
}

hipError_t launch_put_schedule(hipStream_t st, double *beta, double *bfield, int S_hist,
                               int first_step, int n_steps, int k0, int cnt, const PutPairs &vals)
{
    hipLaunchKernelGGL(k_put_schedule, dim3(1), dim3(kPutPairs), 0, st, beta, bfield, S_hist,
                       first_step, n_steps, k0, cnt, vals);
    return hipGetLastError();
}

// ------------------------------------------------------------ initial state
template <typename T>
__global__ void k_init_spins(const RepDesc *reps, int mode, const double *given, uint64_t seed)
{
    const RepDesc &rd = reps[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rd.n) return;
    T *S = (T *)rd.spins;
    const uint32_t orig = rd.orig[i];
    double x = 0.0, y = 0.0, z = 1.0;
    if (mode == 2) {
        sphere64(seed, orig, 0xFFFFFFFFu, rd.rep_id, x, y, z);
    } else if (mode == 0) {
        const double *gv = given + 3 * ((size_t)rd.user_off + orig);
        x = gv[0];
        y = gv[1];
        z = gv[2];
    }
    if (mode != 0 && rd.mu_d) {    // cold and random starts: spins of length mu
        const double mu = rd.mu_d[i];
        x = mu * x;
        y = mu * y;
        z = mu * z;
    }
    S[i] = (T)x;
    S[rd.n_pad + i] = (T)y;
    S[2 * rd.n_pad + i] = (T)z;
}

hipError_t launch_init_spins(hipStream_t st, bool f64, const RepDesc *reps, int R, int max_n,
                             int mode, const double *given, const int64_t *, uint64_t seed)
{
    dim3 grid((unsigned)((max_n + 255) / 256), (unsigned)R);
    if (f64)
        hipLaunchKernelGGL(k_init_spins<double>, grid, dim3(256), 0, st, reps, mode, given, seed);
    else
        hipLaunchKernelGGL(k_init_spins<float>, grid, dim3(256), 0, st, reps, mode, given, seed);
    return hipGetLastError();
}

template <typename T>
__global__ void k_to_user(const RepDesc *reps, int rep, double *out)
{
    const RepDesc &rd = reps[rep];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rd.n) return;
    const T *S = (const T *)rd.spins;
    const uint32_t o = rd.orig[i];
    out[3 * (size_t)o] = (double)S[i];
    out[3 * (size_t)o + 1] = (double)S[rd.n_pad + i];
    out[3 * (size_t)o + 2] = (double)S[2 * rd.n_pad + i];
}

hipError_t launch_to_user(hipStream_t st, bool f64, const RepDesc *reps, int rep, int n,
                          double *out)
{
    dim3 grid((unsigned)((n + 255) / 256));
    if (f64)
        hipLaunchKernelGGL(k_to_user<double>, grid, dim3(256), 0, st, reps, rep, out);
    else
        hipLaunchKernelGGL(k_to_user<float>, grid, dim3(256), 0, st, reps, rep, out);
    return hipGetLastError();
}

// ------------------------------------------------------- site-lane phases
// MCS numbering of the site-lane launches: g = ctl->g + t_off, where ctl->g is
// the first MCS of the current launch sequence (a captured graph replays one
// sequence; k_ctl_advance moves ctl->g on at its end).
template <typename T, int KM, int FM, bool TRACE, int MAXD>
__global__ __launch_bounds__(kSiteBlock) void k_site_phase(const RepDesc *__restrict__ reps,
                                                           const Tile *__restrict__ tiles,
                                                           int tile_off, int t_off, RunArgs ra)
{
    __shared__ double red[(kSiteBlock / 64) * 6];
    const int tl = tile_off + xcd_tile((int)blockIdx.x, (int)gridDim.x);   // this block's tile
    const Tile t = tiles[tl];
    const RepDesc &rd = reps[t.rep];
    const uint32_t g = ra.ctl->g + (uint32_t)t_off;
    const uint32_t s_abs = g / (uint32_t)ra.M;
    const size_t sidx = (size_t)t.rep * ra.S_hist + s_abs;
    const T beta = (T)ra.beta[sidx];
    const T b = (T)ra.bfield[sidx];
    const double sigma = ra.pol.adaptive ? ra.sigma[t.rep] : 0.0;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double ad = 0.0;
    const int i = t.begin + (int)threadIdx.x;
    if (i < t.end)
        site_update<T, KM, FM, TRACE, MAXD>(rd, (T *)rd.spins, i, g, ra, t.rep, beta, b, sigma,
                                            acc, ad, t.nsl, t.begin);
    double v[6] = {acc[0], acc[1], acc[2], acc[3], acc[4], ad};
    block_sum<6>(v, red);
    if (threadIdx.x == 0) {
        double *rec = ra.partials + (size_t)tl * kRecSite;
#pragma unroll
        for (int q = 0; q < 5; ++q) rec[q] = v[q];
        rec[6] = v[5];
    }
}

template <typename T, int KM, int FM>
__global__ __launch_bounds__(kSiteBlock) void k_site_efull(const RepDesc *__restrict__ reps,
                                                           const Tile *__restrict__ tiles,
                                                           int tile_off, int t_off, RunArgs ra)
{
    __shared__ double red[(kSiteBlock / 64)];
    const uint32_t g = ra.ctl->g + (uint32_t)t_off;
    if (!recompute_due(g % (uint32_t)ra.M, ra.P)) return;
    const int tl = tile_off + xcd_tile((int)blockIdx.x, (int)gridDim.x);   // this block's tile
    const Tile t = tiles[tl];
    const RepDesc &rd = reps[t.rep];
    const uint32_t s_abs = g / (uint32_t)ra.M;
    const double b = ra.bfield[(size_t)t.rep * ra.S_hist + s_abs];
    double e[1] = {0.0};
    const int i = t.begin + (int)threadIdx.x;
    if (i < t.end) e[0] = site_energy<T, KM, FM>(rd, (const T *)rd.spins, i, b);
    block_sum<1>(e, red);
    if (threadIdx.x == 0) ra.partials[(size_t)tl * kRecSite + 5] = e[0];
}

__global__ void k_ctl_advance(Ctl *ctl, uint32_t n)
{
    if (threadIdx.x == 0) ctl->g += n;
}

hipError_t launch_ctl_advance(hipStream_t st, Ctl *ctl, uint32_t n)
{
    hipLaunchKernelGGL(k_ctl_advance, dim3(1), dim3(64), 0, st, ctl, n);
    return hipGetLastError();
}

#define HSIM_DISPATCH_KF(KM_, FM_, ...)                                                         \
    do {                                                                                         \
        if ((KM_) == K_NONE && (FM_) == F_UNIFORM) { constexpr int KM = K_NONE, FM = F_UNIFORM; __VA_ARGS__; } \
        else if ((KM_) == K_NONE) { constexpr int KM = K_NONE, FM = F_SITE; __VA_ARGS__; }       \
        else if ((KM_) == K_UNIFORM && (FM_) == F_UNIFORM) { constexpr int KM = K_UNIFORM, FM = F_UNIFORM; __VA_ARGS__; } \
        else if ((KM_) == K_UNIFORM) { constexpr int KM = K_UNIFORM, FM = F_SITE; __VA_ARGS__; } \
        else if ((FM_) == F_UNIFORM) { constexpr int KM = K_SITE, FM = F_UNIFORM; __VA_ARGS__; } \
        else { constexpr int KM = K_SITE, FM = F_SITE; __VA_ARGS__; }                            \
    } while (0)

#define HSIM_DISPATCH_W(ELLW_, ...)                                                             \
    do {                                                                                         \
        if ((ELLW_) == 6) { constexpr int MAXD = 6; __VA_ARGS__; }                               \
        else if ((ELLW_) == 8) { constexpr int MAXD = 8; __VA_ARGS__; }                          \
        else { constexpr int MAXD = 0; __VA_ARGS__; }                                            \
    } while (0)

hipError_t launch_site_phase(hipStream_t st, bool f64, int kmode, int fmode, bool trace, int ellw,
                             const RepDesc *reps, const Tile *tiles, int tile_off, int ntiles,
                             int t_off, const RunArgs &ra)
{
    if (ntiles <= 0) return hipSuccess;
    dim3 grid((unsigned)ntiles), blk(kSiteBlock);
    HSIM_DISPATCH_KF(kmode, fmode, HSIM_DISPATCH_W(ellw, {
        if (f64) {
            if (trace) hipLaunchKernelGGL((k_site_phase<double, KM, FM, true, MAXD>), grid, blk, 0, st, reps, tiles, tile_off, t_off, ra);
            else hipLaunchKernelGGL((k_site_phase<double, KM, FM, false, MAXD>), grid, blk, 0, st, reps, tiles, tile_off, t_off, ra);
        } else {
            if (trace) hipLaunchKernelGGL((k_site_phase<float, KM, FM, true, MAXD>), grid, blk, 0, st, reps, tiles, tile_off, t_off, ra);
            else hipLaunchKernelGGL((k_site_phase<float, KM, FM, false, MAXD>), grid, blk, 0, st, reps, tiles, tile_off, t_off, ra);
        }
    }));
    return hipGetLastError();
}

hipError_t launch_site_efull(hipStream_t st, bool f64, int kmode, int fmode, const RepDesc *reps,
                             const Tile *tiles, int tile_off, int ntiles, int t_off, const RunArgs &ra)
{
    if (ntiles <= 0) return hipSuccess;
    dim3 grid((unsigned)ntiles), blk(kSiteBlock);
    HSIM_DISPATCH_KF(kmode, fmode, {
        if (f64) hipLaunchKernelGGL((k_site_efull<double, KM, FM>), grid, blk, 0, st, reps, tiles, tile_off, t_off, ra);
        else hipLaunchKernelGGL((k_site_efull<float, KM, FM>), grid, blk, 0, st, reps, tiles, tile_off, t_off, ra);
    });
    return hipGetLastError();
}

// The colour classes c_tail .. ncol-1 of every replica (of the list rlist, or
// all) and then its per-MCS history, in one launch of one block of
// kFinThreads threads per replica
// (512: 1024 would spill the double-precision state and measured no faster
// in single precision on the films).
// Small trailing classes (the extra colours of odd-size films: a few hundred
// sites per film) would otherwise cost a launch each, every one a single
// dependent step of latency.  The block sweeps such a class with a stride of
// its size (a block barrier between classes orders them) and keeps the
// sums in registers; then every thread adds, at a stride of the block, the
// records of the replica's phase-launched tiles (and, when the energy is
// recomputed, every tile's recompute partial), and one block sum gives the
// MCS totals.  The grouping of the additions depends only on the tables, so
// plain and graph launches give identical history.
template <typename T, int KM, int FM, bool TRACE, int MAXD>
__global__ __launch_bounds__(kFinThreads) void k_site_finish(const RepDesc *__restrict__ reps,
                                                    const int32_t *__restrict__ rep_tiles,
                                                    const int32_t *__restrict__ rlist, int ncol_max,
                                                    int c_tail, int t_off, RunArgs ra)
{
    __shared__ double red[(kFinThreads / 64) * 7];
    const int r = rlist ? rlist[blockIdx.x] : (int)blockIdx.x;
    const RepDesc &rd = reps[r];
    const uint32_t g = ra.ctl->g + (uint32_t)t_off;
    const uint32_t s_abs = g / (uint32_t)ra.M, m = g % (uint32_t)ra.M;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double ad = 0.0;
    if (c_tail < rd.ncol) {
        const size_t sidx = (size_t)r * ra.S_hist + s_abs;
        const T beta = (T)ra.beta[sidx];
        const T b = (T)ra.bfield[sidx];
        const double sigma = ra.pol.adaptive ? ra.sigma[r] : 0.0;
        for (int c = c_tail; c < rd.ncol; ++c) {
            const int ce = rd.cls_off[c + 1];
            for (int i = rd.cls_off[c] + (int)threadIdx.x; i < ce; i += kFinThreads)
                site_update<T, KM, FM, TRACE, MAXD>(rd, (T *)rd.spins, i, g, ra, r, beta, b, sigma, acc,
                                                    ad);
            __syncthreads();   // this class's stores are seen by the next class's reads
        }
    }
    const bool rec_due = recompute_due(m, ra.P);
    double v[7] = {acc[0], acc[1], acc[2], acc[3], acc[4], 0.0, ad};
    for (int c = 0; c < ncol_max; ++c) {
        const int tb = rep_tiles[(r * ncol_max + c) * 2], te = rep_tiles[(r * ncol_max + c) * 2 + 1];
        if (c < c_tail) {
            for (int tt = tb + (int)threadIdx.x; tt < te; tt += kFinThreads) {
                const double *rec = ra.partials + (size_t)tt * kRecSite;
#pragma unroll
                for (int q = 0; q < 7; ++q) v[q] += rec[q];
            }
        } else if (rec_due) {
            for (int tt = tb + (int)threadIdx.x; tt < te; tt += kFinThreads)
                v[5] += ra.partials[(size_t)tt * kRecSite + 5];
        }
    }
    block_sum<7>(v, red);
    if (threadIdx.x != 0) return;
    if (ra.pol.adaptive) adapt_sigma(ra, r, v[6]);
    const double E = (rec_due ? v[5] : ra.ecarry[r]) + v[0];
    ra.ecarry[r] = E;
    double *h = ra.history + (((size_t)r * ra.S_hist + s_abs) * ra.M + m) * 5;
    h[0] = E;
    h[1] = v[1];
    h[2] = v[2];
    h[3] = v[3];
    h[4] = v[4];
}

hipError_t launch_site_finish(hipStream_t st, bool f64, int kmode, int fmode, bool trace, int ellw,
                              const RepDesc *reps, const int32_t *rep_tiles, const int32_t *rlist,
                              int nrep, int ncol_max, int c_tail, int t_off, const RunArgs &ra)
{
    if (nrep <= 0) return hipSuccess;
    const dim3 grid((unsigned)nrep), blk(kFinThreads);
    HSIM_DISPATCH_KF(kmode, fmode, HSIM_DISPATCH_W(ellw, {
        if (f64) {
            if (trace) hipLaunchKernelGGL((k_site_finish<double, KM, FM, true, MAXD>), grid, blk, 0, st, reps, rep_tiles, rlist, ncol_max, c_tail, t_off, ra);
            else hipLaunchKernelGGL((k_site_finish<double, KM, FM, false, MAXD>), grid, blk, 0, st, reps, rep_tiles, rlist, ncol_max, c_tail, t_off, ra);
        } else {
            if (trace) hipLaunchKernelGGL((k_site_finish<float, KM, FM, true, MAXD>), grid, blk, 0, st, reps, rep_tiles, rlist, ncol_max, c_tail, t_off, ra);
            else hipLaunchKernelGGL((k_site_finish<float, KM, FM, false, MAXD>), grid, blk, 0, st, reps, rep_tiles, rlist, ncol_max, c_tail, t_off, ra);
        }
    }));
    return hipGetLastError();
}

// --------------------------------------------------------- block layout
// The acceptance word and the trial point of a double-precision random move
// depend on the counters only (site, MCS, replica, attempt), not on the
// state: update64's attempt 0 and Marsaglia's map on attempts 1, 2, ...
// (sphere64).  Both sites' first two draws are formed together, four
// independent Philox chains, so their latencies overlap; a rejected first
// point continues from attempt 2 as sphere64 does.
__device__ __forceinline__ void draw_ahead64(uint64_t seed, const uint32_t (&o)[2], uint32_t g,
                                             uint32_t rep, double (&u)[2], double (&x)[2],
                                             double (&y)[2], double (&z)[2])
{
    uint4 w0[2], w1[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        w0[c] = draw(seed, o[c], g, rep, 0);
        w1[c] = draw(seed, o[c], g, rep, 1);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        u[c] = u53(w0[c].x, w0[c].y);
        uint4 w = w1[c];
        x[c] = 0.0;
        y[c] = 0.0;
        z[c] = 1.0;
        for (uint32_t t = 1; t <= 32; ++t) {
            if (t > 1) w = draw(seed, o[c], g, rep, t);
            const double v1 = 2.0 * u53(w.x, w.y) - 1.0;
            const double v2 = 2.0 * u53(w.z, w.w) - 1.0;
            const double s = v1 * v1 + v2 * v2;
            if (s < 1.0) {
                const double f = 2.0 * sqrt(1.0 - s);
                x[c] = v1 * f;
                y[c] = v2 * f;
                z[c] = 1.0 - 2.0 * s;
                break;
            }
        }
    }
}

// One workgroup owns one replica for the whole run: colour classes are
// separated by workgroup barriers, spins live in LDS when they fit, and the
// per-MCS history is written directly.
// NT: the largest block it is launched with.  The double-precision kernel
// needs more than the 128 VGPRs a block of 1024 threads leaves each lane, so
// blocks of up to 256 threads (classes of up to 256 sites) with spins in LDS
// use an instantiation bounded at 256.
template <typename T, int KM, int FM, bool TRACE, bool LDS, int MAXD, int NT = 1024>
__global__ __launch_bounds__(NT) void k_block_sweep(const RepDesc *__restrict__ reps, RunArgs ra)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[16 * 6];
    const int rep = blockIdx.x;
    const RepDesc &rd = reps[rep];
    const int np = rd.n_pad, n = rd.n;
    T *G = (T *)rd.spins;
    T *S = LDS ? (T *)smem : G;
    if (LDS) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            S[i] = G[i];
            S[np + i] = G[np + i];
            S[2 * np + i] = G[2 * np + i];
        }
        __syncthreads();
    }
    // Double precision, random moves, no cubic term or spin lengths, at most
    // two classes of at most one site per thread: the draws of both of a
    // thread's sites are made ahead of the phases.  Only in the kernel
    // bounded at 256 threads: under the 1024-thread bound the extra live
    // values spill (143 VGPRs against 43) and cost more than they save.
    bool ahead = NT <= 256 && sizeof(T) == 8 && ra.pol.n_types == 0 && !rd.kc && !rd.mu && rd.ncol <= 2;
    for (int c = 0; c < rd.ncol; ++c)
        ahead = ahead && rd.cls_off[c + 1] - rd.cls_off[c] <= (int)blockDim.x;
    uint32_t ao[2] = {0u, 0u};
    if (ahead)
        for (int c = 0; c < rd.ncol; ++c) {
            // a thread past its class's end draws for the class's last site
            // and never uses the result
            const int lo = rd.cls_off[c], hi = rd.cls_off[c + 1];
            ao[c] = hi > lo ? rd.orig[min(lo + (int)threadIdx.x, hi - 1)] : 0u;
        }
    double E = 0.0;
    for (int t = 0; t < ra.n_mcs_run; ++t) {
        const uint32_t g = ra.g0 + (uint32_t)t;
        double au[2], ax[2], ay[2], az[2];
        if (ahead) draw_ahead64(ra.seed, ao, g, rd.rep_id, au, ax, ay, az);
        const uint32_t s_abs = g / (uint32_t)ra.M, m = g % (uint32_t)ra.M;
        const size_t sidx = (size_t)rep * ra.S_hist + s_abs;
        const double bd = ra.bfield[sidx];
        if (recompute_due(m, ra.P)) {
            double e[1] = {0.0};
            for (int i = threadIdx.x; i < n; i += blockDim.x)
                e[0] += site_energy<T, KM, FM>(rd, S, i, bd);
            block_sum<1>(e, red);
            E = e[0];
        }
        const T beta = (T)ra.beta[sidx];
        const T b = (T)bd;
        const double sigma = ra.pol.adaptive ? ra.sigma[rep] : 0.0;
        double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        double ad = 0.0;
        for (int c = 0; c < rd.ncol; ++c) {
            const int ce = rd.cls_off[c + 1];
            for (int i = rd.cls_off[c] + threadIdx.x; i < ce; i += blockDim.x)
                site_update<T, KM, FM, TRACE, MAXD>(rd, S, i, g, ra, rep, beta, b, sigma, acc, ad, MAXD, 0,
                                                    ahead, c ? au[1] : au[0], c ? ax[1] : ax[0],
                                                    c ? ay[1] : ay[0], c ? az[1] : az[0]);
            __syncthreads();
        }
        double v[6] = {acc[0], acc[1], acc[2], acc[3], acc[4], ad};
        block_sum<6>(v, red);
        if (threadIdx.x == 0) {
            E = E + v[0];
            double *h = ra.history + (sidx * ra.M + m) * 5;
            h[0] = E;
            h[1] = v[1];
            h[2] = v[2];
            h[3] = v[3];
            h[4] = v[4];
            if (ra.pol.adaptive) adapt_sigma(ra, rep, v[5]);
        }
        __syncthreads();
        // optional outputs: magnetisation per site type, spins at a step end
        if (ra.type_mag) {
            for (int t = 0; t < ra.tm_types; ++t) {
                double q[3] = {0.0, 0.0, 0.0};
                for (int i = threadIdx.x; i < n; i += blockDim.x) {
                    if ((rd.type ? rd.type[i] : 0) != t) continue;
                    q[0] += (double)S[i];
                    q[1] += (double)S[np + i];
                    q[2] += (double)S[2 * np + i];
                }
                block_sum<3>(q, red);
                if (threadIdx.x == 0)
                    for (int c = 0; c < 3; ++c)
                        ra.type_mag[((sidx * ra.M + m) * ra.tm_types + t) * 3 + c] = q[c];
            }
        }
        if (ra.snapshots && m + 1 == (uint32_t)ra.M)
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                double *o = ra.snapshots + (sidx * ra.snap_n + rd.orig[i]) * 3;
                o[0] = (double)S[i];
                o[1] = (double)S[np + i];
                o[2] = (double)S[2 * np + i];
            }
    }
    if (threadIdx.x == 0) ra.ecarry[rep] = E;
    if (LDS) {
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            G[i] = S[i];
            G[np + i] = S[np + i];
            G[2 * np + i] = S[2 * np + i];
        }
    }
}

int block_sweep_max_lds(bool)
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    return v - 1024;   // static reduction scratch
}

hipError_t launch_block_sweep(hipStream_t st, bool f64, int kmode, int fmode, bool trace,
                              int ellw, bool lds, int threads, size_t lds_bytes,
                              const RepDesc *reps, const RunArgs &ra)
{
    dim3 grid((unsigned)ra.R), blk((unsigned)threads);
    const size_t sh = lds ? lds_bytes : 0;
#define HSIM_BLK(T_, TR_, L_, NT_)                                                             \
    do {                                                                                       \
        auto kfn = k_block_sweep<T_, KM, FM, TR_, L_, MAXD, NT_>;                                    \
        if (sh > 65536)                                                                        \
            (void)hipFuncSetAttribute((const void *)kfn,                                       \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);    \
        hipLaunchKernelGGL(kfn, grid, blk, sh, st, reps, ra);                                  \
    } while (0)
    HSIM_DISPATCH_KF(kmode, fmode, HSIM_DISPATCH_W(ellw, {
        if (f64 && threads <= 256 && lds) {
            if (trace) HSIM_BLK(double, true, true, 256);
            else HSIM_BLK(double, false, true, 256);
        } else if (f64) {
            if (trace) { if (lds) HSIM_BLK(double, true, true, 1024); else HSIM_BLK(double, true, false, 1024); }
            else { if (lds) HSIM_BLK(double, false, true, 1024); else HSIM_BLK(double, false, false, 1024); }
        } else {
            if (trace) { if (lds) HSIM_BLK(float, true, true, 1024); else HSIM_BLK(float, true, false, 1024); }
            else { if (lds) HSIM_BLK(float, false, true, 1024); else HSIM_BLK(float, false, false, 1024); }
        }
    }));
#undef HSIM_BLK
    return hipGetLastError();
}

}  // namespace hsim
