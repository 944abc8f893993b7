// Energy of Eq. 1 (paper, section "Classical spin Hamiltonian") for a batch of
// configurations of one lattice, its vector-Jacobian product with respect to
// the spins, the per-bond exchange constants, the per-site anisotropy
// constants and the field intensity, and the fluctuation estimator that turns
// sampled derivatives into derivatives of thermal averages.
//
// Layout (user order): spins [batch][3][n]; per-bond constants in the plan's
// bond order; anisotropy axes and field directions [3][n].
//
// A sparse gather: every site reads its neighbours in each configuration.
// Work items are (group of kEG configurations, tile of kEBlock sites); items
// are dealt to the 8 XCDs in contiguous ranges (group-major), so the tiles
// holding a tile's neighbours are processed by the same XCD at about the same
// time and the neighbour reads hit its L2.  Rows of at most 8 entries are
// read as padded rows (slot-major, padding = the site itself with constant
// 0, which leaves every sum unchanged), so each configuration's gathers are
// issued together without branches; kEU configurations are in flight at
// once.  The forward, which needs every bond once, reads half rows (the
// bonds each site leaves under the plan's Euler orientation) and counts each
// bond term whole, and stages each step's own spins of its tile in LDS, so
// that neighbours inside the tile are read there instead of gathered; the
// backward reads full rows, since dE/dS needs every neighbour, and on rows
// of 6 stages its tile the same way.  The lattice
// tables of a site are read once per group.  Sums over
// sites and configurations are double precision in a fixed order: lanes by
// recursive halving, waves in order, tiles lane-strided then butterfly,
// groups and passes in order.  Batches larger than the plan's pass size run
// in passes over a fixed scratch (no allocation per call).
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "hsim_dev.h"

namespace hsim {

namespace {

constexpr int kEBlock = 256;   // sites per tile, one per thread
constexpr int kEG = 32;        // configurations per work item
constexpr int kEU = 2;         // configurations whose loads are in flight together

__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block sum of one double, valid in thread 0.
__device__ __forceinline__ double bsum(double v, double *lds)
{
    v = wsum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += lds[k];
    __syncthreads();
    return t;
}

// Wave sums of U values per lane by recursive halving: at each step a lane
// keeps the half of its values selected by its lane bit and adds its
// partner's copy of that half; once one value is left, a butterfly.  Lane l
// ends with the wave sum of value halving_index<U>(l), the same in every lane
// of its group of 64/U.
template <int U>
__device__ __forceinline__ double halving_sum(double (&v)[U], int ln)
{
    int cnt = U;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        if (cnt > 1) {
            const int h = cnt / 2;
            const bool up = (ln & m) != 0;
#pragma unroll
            for (int k = 0; k < U / 2; ++k)
                if (k < h) {
                    const double send = up ? v[k] : v[k + h];
                    const double keep = up ? v[k + h] : v[k];
                    v[k] = keep + __shfl_xor(send, m, 64);
                }
            cnt = h;
        } else {
            v[0] += __shfl_xor(v[0], m, 64);
        }
    }
    return v[0];
}

template <int U>
__device__ __forceinline__ int halving_index(int ln)
{
    int idx = 0, cnt = U;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        if (cnt > 1) {
            const int h = cnt / 2;
            if (ln & m) idx += h;
            cnt = h;
        }
    return idx;
}

// Lattice data of one site, read once and used for every configuration of
// a batch chunk: up to kMaxNb neighbours (column, constant) in registers,
// longer rows walked in the CSR for each configuration.
constexpr int kMaxNb = 8;
template <typename T>
struct SiteTables {
    int64_t rb = 0;
    int deg = 0;
    int32_t col[kMaxNb];
    T J[kMaxNb];
    T k, ex, ey, ez, nx, ny, nz, kc;
    __device__ __forceinline__ SiteTables(const EnergyArgs &a, int64_t i)
    {
        const T *Jb = (const T *)a.Jb;
        rb = a.rp[i];
        deg = (int)(a.rp[i + 1] - rb);
#pragma unroll
        for (int q = 0; q < kMaxNb; ++q) {
            col[q] = q < deg ? a.ci[rb + q] : 0;
            J[q] = q < deg ? Jb[a.bond[rb + q]] : T(0);
        }
        const T *kk = (const T *)a.k, *ax = (const T *)a.ax, *nd = (const T *)a.nd;
        k = kk ? kk[i] : T(0);
        ex = ax ? ax[i] : T(0);
        ey = ax ? ax[a.n + i] : T(0);
        ez = ax ? ax[2 * a.n + i] : T(1);
        nx = nd ? nd[i] : T(0);
        ny = nd ? nd[a.n + i] : T(0);
        nz = nd ? nd[2 * a.n + i] : T(1);
        kc = a.kc ? ((const T *)a.kc)[i] : T(0);
    }
    // exchange field of configuration S at site i, entries in CSR order
    __device__ __forceinline__ void field(const EnergyArgs &a, const T *S, T &hx, T &hy, T &hz) const
    {
        const T *Jb = (const T *)a.Jb;
        hx = T(0);
        hy = T(0);
        hz = T(0);
        if (deg <= kMaxNb) {
#pragma unroll
            for (int q = 0; q < kMaxNb; ++q)
                if (q < deg) {
                    const int64_t j = col[q];
                    hx += J[q] * S[j];
                    hy += J[q] * S[a.n + j];
                    hz += J[q] * S[2 * a.n + j];
                }
        } else {
            for (int64_t p = rb; p < rb + deg; ++p) {
                const int64_t j = a.ci[p];
                const T Jp = Jb[a.bond[p]];
                hx += Jp * S[j];
                hy += Jp * S[a.n + j];
                hz += Jp * S[2 * a.n + j];
            }
        }
    }
};

}  // namespace

// Padded rows of width W: one work item per block (XCD-aware order), each
// thread one site and the kEG configurations of the item, kEU at a time.
// STAGE: each step's own spins of the tile also go to LDS, and neighbours
// inside the tile are read there.
template <typename T, bool BWD, int W, bool HALF, bool STAGE>
__device__ __forceinline__ void energy_ell(const EnergyArgs &a, int ntile, int items,
                                           const double *__restrict__ gE, T *gS, double *partE,
                                           double *partB, double *partK, double *partJ)
{
    static_assert(!(HALF && BWD), "half rows serve the forward only");
    static_assert(!HALF || STAGE, "the half-row forward stages its tile");
    const int u_item = xcd_tile((int)blockIdx.x, items);
    const int grp = u_item / ntile, tile = u_item - grp * ntile;
    constexpr int kW = kEBlock / 64;
    __shared__ double ew[kEG][kW], zw[BWD ? kEG : 1][kW];
    const int64_t i = (int64_t)tile * kEBlock + threadIdx.x;
    const bool live = i < a.n;
    const int64_t ii = live ? i : 0;
    const T *Jb = (const T *)a.Jb;
    int32_t col[W];
    T J[W];
    int32_t bid[W];
    const int32_t *tcol = HALF ? a.hcol : a.ecol, *tbond = HALF ? a.hbond : a.ebond;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        col[q] = tcol[(size_t)q * a.n + ii];
        bid[q] = tbond[(size_t)q * a.n + ii];
        const T jv = Jb[bid[q] >= 0 ? bid[q] : 0];
        J[q] = bid[q] >= 0 ? jv : T(0);
    }
    const T *kk = (const T *)a.k, *ax = (const T *)a.ax, *nd = (const T *)a.nd;
    const T k = kk ? kk[ii] : T(0);
    const T ex = ax ? ax[ii] : T(0), ey = ax ? ax[a.n + ii] : T(0), ez = ax ? ax[2 * a.n + ii] : T(1);
    const T nx = nd ? nd[ii] : T(0), ny = nd ? nd[a.n + ii] : T(0), nz = nd ? nd[2 * a.n + ii] : T(1);
    const T kc = a.kc ? ((const T *)a.kc)[ii] : T(0);
    // Staged: the tile's own spins also go to LDS (two buffers, alternate
    // steps), and a neighbour inside the tile is read there; only the others
    // are gathered from memory.  loc: the neighbour's place in the tile, or -1.
    __shared__ T sh_own[STAGE ? 2 : 1][kEU][3][STAGE ? kEBlock : 1];
    int loc[W];
#pragma unroll
    for (int q = 0; q < W; ++q) {
        const int64_t d = (int64_t)col[q] - (int64_t)tile * kEBlock;
        loc[q] = STAGE && d >= 0 && d < kEBlock ? (int)d : -1;
    }
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int b0 = grp * kEG;
    const int nc = min(kEG, a.batch - b0);
    const bool params = BWD && (partK || partJ);
    // dE/dk and dE/dJ of the group, summed over its configurations in the
    // spins' precision (at most kEG terms), then handed on in double
    T gk = T(0), gj[W];
#pragma unroll
    for (int q = 0; q < W; ++q) gj[q] = T(0);
#pragma unroll 1
    for (int c0 = 0; c0 < nc; c0 += kEU) {
        double ev[kEU], zv[kEU];
        T own[kEU][3], nb[kEU][W][3];
        // the step's weights dL/dE, read before the spins: the index is the
        // same in every lane, so these are scalar loads
        double gw[BWD ? kEU : 1];
#pragma unroll
        for (int u = 0; u < (BWD ? kEU : 0); ++u) gw[u] = gE[min(b0 + c0 + u, a.batch - 1)];
#pragma unroll
        for (int u = 0; u < kEU; ++u) {
            const int b = min(b0 + c0 + u, a.batch - 1);
            const T *S = (const T *)a.S + (size_t)b * 3 * a.n;
            own[u][0] = S[ii];
            own[u][1] = S[a.n + ii];
            own[u][2] = S[2 * a.n + ii];
#pragma unroll
            for (int q = 0; q < W; ++q) {
                if (loc[q] >= 0) continue;
                nb[u][q][0] = S[col[q]];
                nb[u][q][1] = S[a.n + col[q]];
                nb[u][q][2] = S[2 * a.n + col[q]];
            }
        }
        if constexpr (STAGE) {
            // a thread of a site past the end holds site 0's spins: no row
            // names that slot
            const int p = (c0 / kEU) & 1;
#pragma unroll
            for (int u = 0; u < kEU; ++u)
#pragma unroll
                for (int d = 0; d < 3; ++d) sh_own[p][u][d][threadIdx.x] = own[u][d];
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kEU; ++u)
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    if (loc[q] < 0) continue;
#pragma unroll
                    for (int d = 0; d < 3; ++d) nb[u][q][d] = sh_own[p][u][d][loc[q]];
                }
        }
        // dE/dS of the step's configurations, stored after the last of them
        // is formed: with a store issued between two configurations, the
        // waits for the second one's loads (on the one counter of
        // outstanding vector-memory operations) also waited for the store
        T go[BWD ? kEU : 1][3];
#pragma unroll
        for (int u = 0; u < kEU; ++u) {
            const int c = c0 + u, b = b0 + c;
            const bool ok = live && c < nc;
            // exchange field, entries in CSR order (padding adds 0 * S_i)
            T thx = T(0), thy = T(0), thz = T(0);
#pragma unroll
            for (int q = 0; q < W; ++q) {
                thx = fma(J[q], nb[u][q][0], thx);
                thy = fma(J[q], nb[u][q][1], thy);
                thz = fma(J[q], nb[u][q][2], thz);
            }
            const T tsx = own[u][0], tsy = own[u][1], tsz = own[u][2];
            if constexpr (!BWD) {
                // full rows count every bond from both ends (half each); half
                // rows count it once, at the end it leaves.  A site's terms in
                // the spins' precision (fused multiply-adds), the sums over
                // sites in double.
                constexpr T kBond = HALF ? T(1) : T(0.5);
                const T dot = fma(tsx, thx, fma(tsy, thy, tsz * thz));
                const T an_t = fma(tsx, ex, fma(tsy, ey, tsz * ez));
                const T zn_t = fma(tsx, nx, fma(tsy, ny, tsz * nz));
                T e = fma(-k * an_t, an_t, fma(-(T)a.B, zn_t, -kBond * dot));
                // cubic term of Eq. 3, -kc (Sx^2 Sy^2 + Sy^2 Sz^2 + Sx^2 Sz^2)
                if (a.kc) {
                    const T x2 = tsx * tsx, y2 = tsy * tsy, z2 = tsz * tsz;
                    e = fma(-kc, fma(x2, y2, fma(y2, z2, x2 * z2)), e);
                }
                ev[u] = ok ? (double)e : 0.0;
            }
            if constexpr (BWD) {
                const double sx = tsx, sy = tsy, sz = tsz;
                zv[u] = ok ? sx * (double)nx + sy * (double)ny + sz * (double)nz : 0.0;
            }
            if (BWD) {
                const double gb = ok ? gw[BWD ? u : 0] : 0.0;
                const T g = (T)gb;
                const T B = (T)a.B;
                const T an_t = fma(tsx, ex, fma(tsy, ey, tsz * ez));
                const T two_ka = T(2) * k * an_t;
                T cx = T(0), cy = T(0), cz = T(0);
                if (a.kc) {
                    const T kc2 = T(2) * kc;
                    const T x2 = tsx * tsx, y2 = tsy * tsy, z2 = tsz * tsz;
                    cx = kc2 * tsx * (y2 + z2);
                    cy = kc2 * tsy * (x2 + z2);
                    cz = kc2 * tsz * (x2 + y2);
                }
                go[BWD ? u : 0][0] = -g * (fma(two_ka, ex, fma(B, nx, thx)) + cx);
                go[BWD ? u : 0][1] = -g * (fma(two_ka, ey, fma(B, ny, thy)) + cy);
                go[BWD ? u : 0][2] = -g * (fma(two_ka, ez, fma(B, nz, thz)) + cz);
                if (params) {
                    gk = fma(-g, an_t * an_t, gk);
                    // bonds whose lower end is i (padding: col == i, skipped)
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        const T d = fma(tsx, nb[u][q][0], fma(tsy, nb[u][q][1], tsz * nb[u][q][2]));
                        gj[q] = col[q] > i ? fma(-g, d, gj[q]) : gj[q];
                    }
                }
            }
        }
        if constexpr (BWD) {
            // every value is formed here (an empty asm takes them in
            // registers, so their arithmetic cannot sink below the stores),
            // and nothing moves past the scheduling barrier
#pragma unroll
            for (int u = 0; u < kEU; ++u)
                asm volatile("" : "+v"(go[u][0]), "+v"(go[u][1]), "+v"(go[u][2]));
            __builtin_amdgcn_sched_barrier(0);
            if (gS && live) {
#pragma unroll
                for (int u = 0; u < kEU; ++u) {
                    if (c0 + u >= nc) continue;
                    // non-temporal: dE/dS is not read again by this kernel
                    T *o = gS + (size_t)(b0 + c0 + u) * 3 * a.n;
                    __builtin_nontemporal_store(go[u][0], &o[i]);
                    __builtin_nontemporal_store(go[u][1], &o[a.n + i]);
                    __builtin_nontemporal_store(go[u][2], &o[2 * a.n + i]);
                }
            }
        }
        const int cw = c0 + halving_index<kEU>(ln);
        const bool wr = (ln & (64 / kEU - 1)) == 0 && cw < nc;
        if constexpr (!BWD) {
            const double es = halving_sum<kEU>(ev, ln);
            if (wr) ew[cw][wv] = es;
        } else {
            const double zs = halving_sum<kEU>(zv, ln);
            if (wr) zw[cw][wv] = zs;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nc) {
        const int c = threadIdx.x, b = b0 + c;
        const size_t t = (size_t)b * ntile + tile;
        double et = 0.0, zt = 0.0;
        for (int q = 0; q < kW; ++q) {
            if (!BWD) et += ew[c][q];
            if (BWD) zt += zw[c][q];
        }
        if (!BWD && partE) partE[t] = et;
        if (BWD) partB[t] = -gE[b] * zt;
    }
    if (!params || !live) return;
    if (partK) partK[(size_t)grp * a.n + i] = (double)gk;
    if (!partJ) return;
#pragma unroll
    for (int q = 0; q < W; ++q)
        if (col[q] > i) partJ[(size_t)grp * a.nb + bid[q]] = (double)gj[q];
}

template <typename T, bool BWD, int W, bool HALF = false, bool STAGE = HALF>
__global__ __launch_bounds__(kEBlock) void k_energy_ell(EnergyArgs a, int ntile, int items,
                                                        const double *__restrict__ gE, T *gS, double *partE,
                                                        double *partB, double *partK, double *partJ)
{
    energy_ell<T, BWD, W, HALF, STAGE>(a, ntile, items, gE, gS, partE, partB, partK, partJ);
}

// The single-precision backward on rows of 6, staged: its rows, group sums
// and LDS addressing take 123 VGPRs when the compiler is held to four waves
// per SIMD (129, i.e. three waves, otherwise); staging pays only at four.
// The double-precision backward on rows of 6 is staged at two waves either
// way (190 VGPRs unstaged, 197 staged) and needs no limit; under this one it
// would spill.
template <typename T, int W>
__global__ __launch_bounds__(kEBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_energy_ell_bwd_staged(
    EnergyArgs a, int ntile, int items, const double *__restrict__ gE, T *gS, double *partE, double *partB,
    double *partK, double *partJ)
{
    energy_ell<T, true, W, false, true>(a, ntile, items, gE, gS, partE, partB, partK, partJ);
}

// Rows longer than the padded width (any degree): grid (site tiles, chunks of
// kEG configurations), each thread one site walking its CSR row for every
// configuration of the chunk.  Forward: E partial per (configuration, tile).
// Backward (BWD): also dE/dS of every site, the dE/dB partial and the chunk's
// dE/dk, dE/dJ partials (per site, per bond).
template <typename T, bool BWD>
__global__ __launch_bounds__(kEBlock) void k_energy_csr(EnergyArgs a, const double *gE, T *gS,
                                                         double *partE, double *partB,
                                                         double *partK, double *partJ)
{
    // wave sums of every configuration of the chunk, added in wave order
    // after the loop (one barrier per chunk instead of two per configuration)
    constexpr int kW = kEBlock / 64;
    __shared__ double ew[kEG][kW], zw[BWD ? kEG : 1][kW];
    const int64_t i = (int64_t)blockIdx.x * kEBlock + threadIdx.x;
    const bool live = i < a.n;
    const SiteTables<T> st(a, live ? i : 0);
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int b0 = (int)blockIdx.y * kEG;
    // backward, parameter gradients of the chunk: dE/dk_i and dE/dJ of the
    // bonds whose lower end is i (rows up to kMaxNb entries here; longer rows
    // below), summed over the chunk's configurations in order
    const bool params = BWD && (partK || partJ);
    double gk = 0.0, gj[kMaxNb];
#pragma unroll
    for (int q = 0; q < kMaxNb; ++q) gj[q] = 0.0;
    for (int c = 0; c < kEG; ++c) {
        const int b = b0 + c;
        if (b >= a.batch) break;   // uniform over the block
        double e = 0.0, zn = 0.0;
        if (live) {
            const T *S = (const T *)a.S + (size_t)b * 3 * a.n;
            const T tsx = S[i], tsy = S[a.n + i], tsz = S[2 * a.n + i];
            T thx, thy, thz;
            st.field(a, S, thx, thy, thz);
            const double sx = tsx, sy = tsy, sz = tsz;
            const double an = sx * (double)st.ex + sy * (double)st.ey + sz * (double)st.ez;
            zn = sx * (double)st.nx + sy * (double)st.ny + sz * (double)st.nz;
            e = -0.5 * (sx * (double)thx + sy * (double)thy + sz * (double)thz) - a.B * zn -
                (double)st.k * an * an;
            // cubic term of Eq. 3, -kc (Sx^2 Sy^2 + Sy^2 Sz^2 + Sx^2 Sz^2)
            if (a.kc) e -= (double)st.kc * ((sx * sx * (sy * sy) + sy * sy * (sz * sz)) + sx * sx * (sz * sz));
            if (BWD) {
                const T g = (T)gE[b];
                const T B = (T)a.B;
                const T an_t = tsx * st.ex + tsy * st.ey + tsz * st.ez;
                const T two_ka = T(2) * st.k * an_t;
                T *o = gS + (size_t)b * 3 * a.n;
                T cx = T(0), cy = T(0), cz = T(0);
                if (a.kc) {
                    const T kc2 = T(2) * st.kc;
                    const T x2 = tsx * tsx, y2 = tsy * tsy, z2 = tsz * tsz;
                    cx = kc2 * tsx * (y2 + z2);
                    cy = kc2 * tsy * (x2 + z2);
                    cz = kc2 * tsz * (x2 + y2);
                }
                if (gS) {
                    o[i] = g * (-thx - B * st.nx - two_ka * st.ex - cx);
                    o[a.n + i] = g * (-thy - B * st.ny - two_ka * st.ey - cy);
                    o[2 * a.n + i] = g * (-thz - B * st.nz - two_ka * st.ez - cz);
                }
                if (params) {
                    const double gb = gE[b];
                    gk += gb * -(an * an);
                    if (st.deg <= kMaxNb) {
#pragma unroll
                        for (int q = 0; q < kMaxNb; ++q)
                            if (q < st.deg && st.col[q] > i) {
                                const int64_t j = st.col[q];
                                const double d = sx * (double)S[j] + sy * (double)S[a.n + j] +
                                                 sz * (double)S[2 * a.n + j];
                                gj[q] += gb * -d;
                            }
                    }
                }
            }
        }
        e = wsum(e);
        if (ln == 0) ew[c][wv] = e;
        if (BWD) {
            zn = wsum(zn);
            if (ln == 0) zw[c][wv] = zn;
        }
    }
    __syncthreads();
    const int nc = min(kEG, a.batch - b0);
    if ((int)threadIdx.x < nc) {
        const int c = threadIdx.x, b = b0 + c;
        const size_t t = (size_t)b * gridDim.x + blockIdx.x;
        double et = 0.0, zt = 0.0;
        for (int k = 0; k < kW; ++k) {
            et += ew[c][k];
            if (BWD) zt += zw[c][k];
        }
        if (partE) partE[t] = et;
        if (BWD) partB[t] = -gE[b] * zt;
    }
    if (!params || !live) return;
    const size_t ch = blockIdx.y;   // this chunk's partial records
    if (partK) partK[ch * a.n + i] = gk;
    if (!partJ) return;
    if (st.deg <= kMaxNb) {
#pragma unroll
        for (int q = 0; q < kMaxNb; ++q)
            if (q < st.deg && st.col[q] > i) partJ[ch * a.nb + a.bond[st.rb + q]] = gj[q];
    } else {
        const int b1 = min(a.batch, b0 + kEG);
        for (int64_t p = st.rb; p < st.rb + st.deg; ++p) {
            const int64_t j = a.ci[p];
            if (j <= i) continue;
            double v = 0.0;
            for (int b = b0; b < b1; ++b) {
                const T *S = (const T *)a.S + (size_t)b * 3 * a.n;
                const double d = (double)S[i] * (double)S[j] + (double)S[a.n + i] * (double)S[a.n + j] +
                                 (double)S[2 * a.n + i] * (double)S[2 * a.n + j];
                v += gE[b] * -d;
            }
            partJ[ch * a.nb + a.bond[p]] = v;
        }
    }
}

// Per-configuration sums of tile partials: one wave per configuration,
// lanes over tiles lane-strided in order, then a butterfly.
__global__ __launch_bounds__(256) void k_energy_tiles(int cnt, int ntile, const double *part,
                                                      double *out)
{
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6), ln = threadIdx.x & 63;
    if (b >= cnt) return;
    double v = 0.0;
    for (int t = ln; t < ntile; t += 64) v += part[(size_t)b * ntile + t];
    v = wsum(v);
    if (ln == 0) out[b] = v;
}

// Sum of column t of part [ngroups][stride] in group order; the loads of
// eight groups are issued together, the additions stay in order.
__device__ __forceinline__ double group_sum(const double *part, int ngroups, int64_t stride, int64_t t)
{
    double v = 0.0;
    int g = 0;
    for (; g + 8 <= ngroups; g += 8) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = part[(size_t)(g + u) * stride + t];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += x[u];
    }
    for (; g < ngroups; ++g) v += part[(size_t)g * stride + t];
    return v;
}

// dE/dk and dE/dJ of a pass: the groups' partials summed in order, added to
// the sums of the earlier passes (first: start them); the last pass writes
// the outputs in the inputs' precision.
template <typename T>
__global__ __launch_bounds__(256) void k_energy_params(int64_t n, int64_t nb, int ngroups,
                                                       const double *partK, const double *partJ,
                                                       double *accK, double *accJ, int first,
                                                       int last, T *gk, T *gJ)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gJ && t < nb) {
        double v = group_sum(partJ, ngroups, nb, t);
        if (!first) v = accJ[t] + v;
        if (last) gJ[t] = (T)v;
        else accJ[t] = v;
    }
    if (gk && t < n) {
        double v = group_sum(partK, ngroups, n, t);
        if (!first) v = accK[t] + v;
        if (last) gk[t] = (T)v;
        else accK[t] = v;
    }
}

// dE/dB of a pass: its configurations' sums in a fixed order (thread t takes
// t, t + 256, ...; then the block sum), added to the earlier passes'.
__global__ __launch_bounds__(256) void k_energy_gB(int cnt, const double *pB, double *accB,
                                                   int first, int last, double *gB)
{
    __shared__ double red[4];
    double v = 0.0;
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) v += pB[t];
    v = bsum(v, red);
    if (threadIdx.x == 0) {
        if (!first) v = accB[0] + v;
        if (last) gB[0] = v;
        else accB[0] = v;
    }
}

EnergyLayout energy_layout(int64_t n, int64_t nb, int ell_w, int64_t cap_doubles, bool forward_only,
                           int min_groups)
{
    EnergyLayout L{};
    L.ntile = (int)((n + kEBlock - 1) / kEBlock);
    L.ell_w = ell_w;
    // groups per pass: the partial records of a pass fit the scratch
    const int64_t per_group = forward_only ? (int64_t)kEG * L.ntile
                                           : 2 * (int64_t)kEG * L.ntile + n + nb + kEG;
    const int64_t fixed = forward_only ? 0 : n + nb + 8;
    int64_t g = (cap_doubles - fixed) / std::max<int64_t>(per_group, 1);
    g = std::min<int64_t>(g, kEnergyMaxGroups);
    L.groups = (int)std::max<int64_t>(g, min_groups);
    L.pass_cfg = L.groups * kEG;
    auto al = [](int64_t x) { return (x + 31) / 32 * 32; };   // 256-byte aligned blocks
    int64_t off = 0;
    L.off_partE = off;
    off += al((int64_t)L.pass_cfg * L.ntile);
    if (!forward_only) {
        L.off_partB = off;
        off += al((int64_t)L.pass_cfg * L.ntile);
        L.off_partK = off;
        off += al((int64_t)L.groups * n);
        L.off_partJ = off;
        off += al((int64_t)L.groups * nb);
        L.off_accK = off;
        off += al(n);
        L.off_accJ = off;
        off += al(nb);
        L.off_pB = off;
        off += al(L.pass_cfg);
        L.off_accB = off;
        off += 32;
    }
    L.doubles = off;
    return L;
}

namespace {

template <typename T, bool BWD>
hipError_t launch_site_kernel(hipStream_t st, const EnergyArgs &a, const EnergyLayout &L,
                              const double *gE, T *gS, double *partE, double *partB,
                              double *partK, double *partJ)
{
    const int ngroups = (a.batch + kEG - 1) / kEG;
    if (!BWD && a.hcol && (L.ell_w == 6 || L.ell_w == 8)) {
        // the forward needs every bond once: half rows of width ell_w / 2
        const int items = ngroups * L.ntile;
        if (L.ell_w == 6)
            hipLaunchKernelGGL((k_energy_ell<T, false, 3, true>), dim3((unsigned)items), dim3(kEBlock), 0,
                               st, a, L.ntile, items, gE, gS, partE, partB, partK, partJ);
        else
            hipLaunchKernelGGL((k_energy_ell<T, false, 4, true>), dim3((unsigned)items), dim3(kEBlock), 0,
                               st, a, L.ntile, items, gE, gS, partE, partB, partK, partJ);
    } else if (L.ell_w == 6 || L.ell_w == 8) {
        const int items = ngroups * L.ntile;
        if constexpr (BWD && std::is_same<T, float>::value) {
            if (L.ell_w == 6) {
                hipLaunchKernelGGL((k_energy_ell_bwd_staged<T, 6>), dim3((unsigned)items), dim3(kEBlock), 0,
                                   st, a, L.ntile, items, gE, gS, partE, partB, partK, partJ);
                return hipGetLastError();
            }
        }
        if (L.ell_w == 6)
            hipLaunchKernelGGL((k_energy_ell<T, BWD, 6, false, BWD>), dim3((unsigned)items), dim3(kEBlock), 0, st, a,
                               L.ntile, items, gE, gS, partE, partB, partK, partJ);
        else
            hipLaunchKernelGGL((k_energy_ell<T, BWD, 8>), dim3((unsigned)items), dim3(kEBlock), 0, st, a,
                               L.ntile, items, gE, gS, partE, partB, partK, partJ);
    } else {
        hipLaunchKernelGGL((k_energy_csr<T, BWD>), dim3((unsigned)L.ntile, (unsigned)ngroups),
                           dim3(kEBlock), 0, st, a, gE, gS, partE, partB, partK, partJ);
    }
    return hipGetLastError();
}

// The pass [b0, b0 + cnt) of the batch: the arguments with the spins (and
// their gradients) moved to the pass's first configuration.
EnergyArgs pass_args(const EnergyArgs &a, bool f64, int b0, int cnt)
{
    EnergyArgs p = a;
    const size_t es = f64 ? 8 : 4;
    p.S = (const char *)a.S + (size_t)b0 * 3 * a.n * es;
    p.batch = cnt;
    return p;
}

}  // namespace

hipError_t launch_energy_forward(hipStream_t st, bool f64, const EnergyArgs &a,
                                 const EnergyLayout &L, double *scratch, double *E)
{
    if (L.pass_cfg < 1) return hipErrorInvalidValue;
    for (int b0 = 0; b0 < a.batch; b0 += L.pass_cfg) {
        const int cnt = std::min(L.pass_cfg, a.batch - b0);
        const EnergyArgs p = pass_args(a, f64, b0, cnt);
        double *partE = scratch + L.off_partE;
        hipError_t e = f64 ? launch_site_kernel<double, false>(st, p, L, nullptr, nullptr, partE, nullptr, nullptr, nullptr)
                           : launch_site_kernel<float, false>(st, p, L, nullptr, nullptr, partE, nullptr, nullptr, nullptr);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_energy_tiles, dim3((unsigned)((cnt + 3) / 4)), dim3(256), 0, st, cnt,
                           L.ntile, (const double *)partE, E + b0);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_energy_backward(hipStream_t st, bool f64, const EnergyArgs &a, const double *gE,
                                  void *gS, void *gJ, void *gk, double *gB, const EnergyLayout &L,
                                  double *scratch)
{
    if (L.pass_cfg < 1) return hipErrorInvalidValue;
    double *partB = scratch + L.off_partB, *partK = scratch + L.off_partK;
    double *partJ = scratch + L.off_partJ, *accK = scratch + L.off_accK, *accJ = scratch + L.off_accJ;
    double *pB = scratch + L.off_pB, *accB = scratch + L.off_accB;
    const size_t es = f64 ? 8 : 4;
    const int64_t m = std::max<int64_t>(std::max<int64_t>(a.n, a.nb), 1);
    for (int b0 = 0; b0 < a.batch; b0 += L.pass_cfg) {
        const int cnt = std::min(L.pass_cfg, a.batch - b0);
        const int first = b0 == 0, last = b0 + cnt >= a.batch;
        const EnergyArgs p = pass_args(a, f64, b0, cnt);
        void *gSp = gS ? (char *)gS + (size_t)b0 * 3 * a.n * es : nullptr;
        double *pk = gk ? partK : nullptr, *pj = gJ ? partJ : nullptr;
        hipError_t e = f64 ? launch_site_kernel<double, true>(st, p, L, gE + b0, (double *)gSp, nullptr, partB, pk, pj)
                           : launch_site_kernel<float, true>(st, p, L, gE + b0, (float *)gSp, nullptr, partB, pk, pj);
        if (e != hipSuccess) return e;
        if (gJ || gk) {
            const int ng = (cnt + kEG - 1) / kEG;
            const dim3 g3((unsigned)((m + 255) / 256));
            if (f64)
                hipLaunchKernelGGL((k_energy_params<double>), g3, dim3(256), 0, st, a.n, a.nb, ng,
                                   (const double *)partK, (const double *)partJ, accK, accJ, first,
                                   last, (double *)gk, (double *)gJ);
            else
                hipLaunchKernelGGL((k_energy_params<float>), g3, dim3(256), 0, st, a.n, a.nb, ng,
                                   (const double *)partK, (const double *)partJ, accK, accJ, first,
                                   last, (float *)gk, (float *)gJ);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (gB) {
            hipLaunchKernelGGL(k_energy_tiles, dim3((unsigned)((cnt + 3) / 4)), dim3(256), 0, st, cnt,
                               L.ntile, (const double *)partB, pB);
            hipLaunchKernelGGL(k_energy_gB, dim3(1), dim3(256), 0, st, cnt, (const double *)pB, accB,
                               first, last, gB);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// ------------------------------------------------ forward without allocation
// Partial records of hsim_energy_forward_noalloc: a fixed device array that
// lives as long as the process, one copy per GPU.  In host code the array's
// name only stands for the symbol; its device address comes from
// hipGetSymbolAddress, resolved once per device (with that device current)
// and cached.
static __device__ __align__(256) double scratch[kStaticEnergyScratchDoubles];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_energy_scratch(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// d<O>/dtheta = <dO> - beta (<O dE> - <O><dE>): one block, fixed-order sums.
__global__ __launch_bounds__(1024) void k_fluct(int64_t n, double beta, const double *O,
                                                const double *dE, const double *dO, double *out)
{
    __shared__ double red[16];
    double so = 0.0, se = 0.0, sd = 0.0;
    for (int64_t t = threadIdx.x; t < n; t += blockDim.x) {
        so += O[t];
        se += dE[t];
        if (dO) sd += dO[t];
    }
    const double mo = bsum(so, red) / (double)n;
    const double me = bsum(se, red) / (double)n;
    const double md = bsum(sd, red) / (double)n;
    __shared__ double mean[2];
    if (threadIdx.x == 0) {
        mean[0] = mo;
        mean[1] = me;
    }
    __syncthreads();
    double sc = 0.0;
    for (int64_t t = threadIdx.x; t < n; t += blockDim.x) sc += (O[t] - mean[0]) * (dE[t] - mean[1]);
    const double cov = bsum(sc, red) / (double)n;
    if (threadIdx.x == 0) {
        out[0] = md - beta * cov;
        out[1] = cov;
    }
}

hipError_t launch_fluct(hipStream_t st, int64_t n, double beta, const double *O, const double *dE,
                        const double *dO, double *out)
{
    hipLaunchKernelGGL(k_fluct, dim3(1), dim3(1024), 0, st, n, beta, O, dE, dO, out);
    return hipGetLastError();
}

// Upstream weights of the fluctuation estimator: w_k = (c - beta (O_k - <O>)) / n
// (one block; the mean in a fixed order).
__global__ __launch_bounds__(1024) void k_fluct_weights(int64_t n, double beta, const double *O,
                                                        double c, double *w)
{
    __shared__ double red[16];
    __shared__ double mean;
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < n; t += blockDim.x) s += O[t];
    s = bsum(s, red);
    if (threadIdx.x == 0) mean = s / (double)n;
    __syncthreads();
    const double m = mean, inv = 1.0 / (double)n;
    for (int64_t t = threadIdx.x; t < n; t += blockDim.x) w[t] = (c - beta * (O[t] - m)) * inv;
}

hipError_t launch_fluct_weights(hipStream_t st, int64_t n, double beta, const double *O, double c,
                                double *w)
{
    hipLaunchKernelGGL(k_fluct_weights, dim3(1), dim3(1024), 0, st, n, beta, O, c, w);
    return hipGetLastError();
}

// Site-major double spins [cfg][n][3] -> planar [cfg][3][n] of type T.
template <typename T>
__global__ __launch_bounds__(256) void k_spins_planar(int64_t total, int64_t n, const double *in,
                                                      T *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // cfg * n + i
    if (t >= total) return;
    const int64_t c = t / n, i = t - c * n;
    const double *s = in + 3 * t;
    T *o = out + 3 * c * n + i;
    o[0] = (T)s[0];
    o[n] = (T)s[1];
    o[2 * n] = (T)s[2];
}

hipError_t launch_spins_planar(hipStream_t st, bool f64, int64_t n_cfg, int64_t n,
                               const double *in, void *out)
{
    const int64_t total = n_cfg * n;
    if (total == 0) return hipSuccess;
    const dim3 grid((unsigned)((total + 255) / 256));
    if (f64) hipLaunchKernelGGL(k_spins_planar<double>, grid, dim3(256), 0, st, total, n, in, (double *)out);
    else hipLaunchKernelGGL(k_spins_planar<float>, grid, dim3(256), 0, st, total, n, in, (float *)out);
    return hipGetLastError();
}

}  // namespace hsim
