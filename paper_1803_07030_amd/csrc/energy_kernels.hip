// Energy of Eq. 1 (paper, section "Classical spin Hamiltonian") for a batch of
// configurations of one lattice, its vector-Jacobian product with respect to
// the spins, the per-bond exchange constants, the per-site anisotropy
// constants and the field intensity, and the fluctuation estimator that turns
// sampled derivatives into derivatives of thermal averages.
//
// Layout (user order): spins [batch][3][n]; per-bond constants in the plan's
// bond order; anisotropy axes and field directions [3][n].
//
// The work is a sparse gather (each site reads its neighbours), so it is
// bandwidth-bound: spins stream from HBM once per pass while the lattice
// tables (a few MB) stay in L2.  Sums over sites and configurations are done
// in double precision in a fixed order (wave butterfly, waves in order,
// tiles in order, batch chunks in order).
#include "hsim_dev.h"

namespace hsim {

namespace {

constexpr int kEBlock = 256;

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

// grid (site tiles, batch chunks of kECfg configurations).  Forward: E
// partial per (configuration, tile).  Backward (BWD): also dE/dS of every
// site and the dE/dB partial.  The lattice tables of a site are read once
// per chunk.
constexpr int kECfg = 32;
template <typename T, bool BWD>
__global__ __launch_bounds__(kEBlock) void k_energy_site(EnergyArgs a, const double *gE, T *gS,
                                                         double *partE, double *partB,
                                                         double *partK, double *partJ)
{
    // wave sums of every configuration of the chunk, added in wave order
    // after the loop (one barrier per chunk instead of two per configuration)
    constexpr int kW = kEBlock / 64;
    __shared__ double ew[kECfg][kW], zw[BWD ? kECfg : 1][kW];
    const int64_t i = (int64_t)blockIdx.x * kEBlock + threadIdx.x;
    const bool live = i < a.n;
    const SiteTables<T> st(a, live ? i : 0);
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int b0 = (int)blockIdx.y * kECfg;
    // backward, parameter gradients of the chunk: dE/dk_i and dE/dJ of the
    // bonds whose lower end is i (rows up to kMaxNb entries here; longer rows
    // below), summed over the chunk's configurations in order
    const bool params = BWD && (partK || partJ);
    double gk = 0.0, gj[kMaxNb];
#pragma unroll
    for (int q = 0; q < kMaxNb; ++q) gj[q] = 0.0;
    for (int c = 0; c < kECfg; ++c) {
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
    const int nc = min(kECfg, a.batch - b0);
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
            if (q < st.deg && st.col[q] > i) partJ[ch * a.nnz + st.rb + q] = gj[q];
    } else {
        const int b1 = min(a.batch, b0 + kECfg);
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
            partJ[ch * a.nnz + p] = v;
        }
    }
}

// Sums in order: E[b] over tiles; gJ over chunks (at each bond's lower-end
// entry); gk over chunks; gB over (config, tile) records.
template <typename T>
__global__ __launch_bounds__(256) void k_energy_finish(EnergyArgs a, int ntile, int nchunk,
                                                       const double *partE, double *E,
                                                       const double *partK, const double *partJ,
                                                       const int32_t *fwd_entry, T *gJ, T *gk,
                                                       const double *partB, double *partBc)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (E && t < a.batch) {
        double v = 0.0;
        for (int k = 0; k < ntile; ++k) v += partE[(size_t)t * ntile + k];
        E[t] = v;
    }
    if (gJ && t < a.nb) {
        const int64_t p = fwd_entry[t];
        double v = 0.0;
        for (int c = 0; c < nchunk; ++c) v += partJ[(size_t)c * a.nnz + p];
        gJ[t] = (T)v;
    }
    if (gk && t < a.n) {
        double v = 0.0;
        for (int c = 0; c < nchunk; ++c) v += partK[(size_t)c * a.n + t];
        gk[t] = (T)v;
    }
    if (partBc && t < a.batch) {
        double v = 0.0;
        for (int k = 0; k < ntile; ++k) v += partB[(size_t)t * ntile + k];
        partBc[t] = v;
    }
}

// dE/dB: the per-configuration sums in a fixed order (thread t takes
// configurations t, t + 256, ... in order; then the block sum).
__global__ __launch_bounds__(256) void k_energy_gB(int batch, const double *partBc, double *gB)
{
    __shared__ double red[4];
    double v = 0.0;
    for (int t = threadIdx.x; t < batch; t += blockDim.x) v += partBc[t];
    v = bsum(v, red);
    if (threadIdx.x == 0) gB[0] = v;
}

int64_t energy_scratch_doubles(int64_t n, int64_t nnz, int batch, int)
{
    const int64_t ntile = (n + kEBlock - 1) / kEBlock;
    const int64_t nchunk = (batch + kECfg - 1) / kECfg;
    // partE, partB: batch*ntile each; partK: nchunk*n; partJ: nchunk*nnz; partBc: batch
    return 2 * (int64_t)batch * ntile + nchunk * n + nchunk * nnz + batch;
}

hipError_t launch_energy_forward(hipStream_t st, bool f64, const EnergyArgs &a, double *scratch,
                                 int, double *E)
{
    const int ntile = (int)((a.n + kEBlock - 1) / kEBlock);
    dim3 grid((unsigned)ntile, (unsigned)((a.batch + kECfg - 1) / kECfg));
    double *partE = scratch;
    if (f64)
        hipLaunchKernelGGL((k_energy_site<double, false>), grid, dim3(kEBlock), 0, st, a,
                           (const double *)nullptr, (double *)nullptr, partE, (double *)nullptr,
                           (double *)nullptr, (double *)nullptr);
    else
        hipLaunchKernelGGL((k_energy_site<float, false>), grid, dim3(kEBlock), 0, st, a,
                           (const double *)nullptr, (float *)nullptr, partE, (double *)nullptr,
                           (double *)nullptr, (double *)nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 g2((unsigned)((a.batch + 255) / 256));
    if (f64)
        hipLaunchKernelGGL((k_energy_finish<double>), g2, dim3(256), 0, st, a, ntile, 0, partE, E,
                           (const double *)nullptr, (const double *)nullptr,
                           (const int32_t *)nullptr, (double *)nullptr, (double *)nullptr,
                           (const double *)nullptr, (double *)nullptr);
    else
        hipLaunchKernelGGL((k_energy_finish<float>), g2, dim3(256), 0, st, a, ntile, 0, partE, E,
                           (const double *)nullptr, (const double *)nullptr,
                           (const int32_t *)nullptr, (float *)nullptr, (float *)nullptr,
                           (const double *)nullptr, (double *)nullptr);
    return hipGetLastError();
}

hipError_t launch_energy_backward(hipStream_t st, bool f64, const EnergyArgs &a, const double *gE,
                                  void *gS, void *gJ, void *gk, double *gB, double *scratch,
                                  int)
{
    const int ntile = (int)((a.n + kEBlock - 1) / kEBlock);
    const int nchunk = (a.batch + kECfg - 1) / kECfg;
    double *partE = scratch;
    double *partB = partE + (size_t)a.batch * ntile;
    double *partK = partB + (size_t)a.batch * ntile;
    double *partJ = partK + (size_t)nchunk * a.n;
    double *partBc = partJ + (size_t)nchunk * a.nnz;
    const int32_t *fwd = a.fwd_entry;
    dim3 grid((unsigned)ntile, (unsigned)nchunk);
    // one pass: dE/dS, the dE/dB partials and the dE/dk, dE/dJ chunk partials
    double *pk = gk ? partK : nullptr, *pj = gJ ? partJ : nullptr;
    if (f64)
        hipLaunchKernelGGL((k_energy_site<double, true>), grid, dim3(kEBlock), 0, st, a, gE,
                           (double *)gS, (double *)nullptr, partB, pk, pj);
    else
        hipLaunchKernelGGL((k_energy_site<float, true>), grid, dim3(kEBlock), 0, st, a, gE,
                           (float *)gS, (double *)nullptr, partB, pk, pj);
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
    int64_t m = a.nb;
    if (a.n > m) m = a.n;
    if (a.batch > m) m = a.batch;
    if (m < 1) m = 1;
    dim3 g3((unsigned)((m + 255) / 256));
    double *bc = gB ? partBc : nullptr;
    if (f64)
        hipLaunchKernelGGL((k_energy_finish<double>), g3, dim3(256), 0, st, a, ntile, nchunk,
                           (const double *)nullptr, (double *)nullptr, partK, partJ, fwd,
                           (double *)gJ, (double *)gk, (const double *)partB, bc);
    else
        hipLaunchKernelGGL((k_energy_finish<float>), g3, dim3(256), 0, st, a, ntile, nchunk,
                           (const double *)nullptr, (double *)nullptr, partK, partJ, fwd,
                           (float *)gJ, (float *)gk, (const double *)partB, bc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !gB) return e;
    hipLaunchKernelGGL(k_energy_gB, dim3(1), dim3(256), 0, st, a.batch, (const double *)partBc, gB);
    return hipGetLastError();
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

}  // namespace hsim
