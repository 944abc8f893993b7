// Optional per-run outputs: the magnetisation of every site type after
// every MCS (each magnetic phase gets statistics of its own) and the spins at
// the end of every temperature/field step (the final states stored per
// step), both from the paper's feature list (section "VEGAS software
// package").
//
// Per-type sums are deterministic: a fixed chunk of sites per block, a fixed
// tree inside the block, and the chunks added in order.
#include "hsim_dev.h"

namespace hsim {

namespace {

constexpr int kOT = 256;        // threads of the per-type blocks
constexpr int kOChunk = 2048;   // sites per block (site and block layouts)

__device__ void tree3(double (&v)[3], double *lds)
{
    // sum of v over the block in a fixed tree, result in thread 0's v
#pragma unroll
    for (int c = 0; c < 3; ++c) lds[c * kOT + threadIdx.x] = v[c];
    __syncthreads();
    for (int s = kOT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int c = 0; c < 3; ++c) lds[c * kOT + threadIdx.x] += lds[c * kOT + threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = lds[c * kOT];
    __syncthreads();
}

// Site and block layouts, step 1: chunk b = blockIdx.x of replica r =
// blockIdx.y; for every type, the chunk's sum -> part[r][b][t][3].
template <typename T>
__global__ __launch_bounds__(kOT) void k_type_part_site(const RepDesc *reps, int nblk, RunArgs ra)
{
    __shared__ double lds[3 * kOT];
    const int r = blockIdx.y, b = blockIdx.x;
    const RepDesc &rd = reps[r];
    const T *S = (const T *)rd.spins;
    const int i0 = b * kOChunk, i1 = min(rd.n, i0 + kOChunk);
    for (int t = 0; t < ra.tm_types; ++t) {
        double v[3] = {0.0, 0.0, 0.0};
        for (int i = i0 + (int)threadIdx.x; i < i1; i += kOT) {
            if ((rd.type ? rd.type[i] : 0) != t) continue;
            v[0] += (double)S[i];
            v[1] += (double)S[rd.n_pad + i];
            v[2] += (double)S[2 * rd.n_pad + i];
        }
        tree3(v, lds);
        if (threadIdx.x == 0)
#pragma unroll
            for (int c = 0; c < 3; ++c) ra.tm_part[(((size_t)r * nblk + b) * ra.tm_types + t) * 3 + c] = v[c];
    }
}

// Replica layout, step 1: chunk b of 64 sites per block, lanes = replicas
// (Rp columns, 64 at a time), four site slices summed in order.
__global__ __launch_bounds__(kOT) void k_type_part_rep(RepLaneArgs a, int nblk, RunArgs ra)
{
    __shared__ double lds[4 * 64 * 3];
    const int b = blockIdx.x;
    const int lane = threadIdx.x & 63, slice = threadIdx.x >> 6;
    const size_t plane = (size_t)a.cs;
    const int i0 = b * 64, i1 = min(a.n, i0 + 64);
    for (int r0 = 0; r0 < a.R; r0 += 64) {
        const int r = r0 + lane;
        for (int t = 0; t < ra.tm_types; ++t) {
            double v[3] = {0.0, 0.0, 0.0};
            if (r < a.R)
                for (int i = i0 + slice; i < i1; i += 4) {
                    if ((a.type ? a.type[i] : 0) != t) continue;
                    const size_t o = (size_t)i * a.ss + r;
                    v[0] += (double)a.spins[o];
                    v[1] += (double)a.spins[plane + o];
                    v[2] += (double)a.spins[2 * plane + o];
                }
#pragma unroll
            for (int c = 0; c < 3; ++c) lds[(slice * 64 + lane) * 3 + c] = v[c];
            __syncthreads();
            if (slice == 0 && r < a.R)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double s = ((lds[lane * 3 + c] + lds[(64 + lane) * 3 + c]) +
                                      lds[(128 + lane) * 3 + c]) + lds[(192 + lane) * 3 + c];
                    ra.tm_part[(((size_t)r * nblk + b) * ra.tm_types + t) * 3 + c] = s;
                }
            __syncthreads();
        }
    }
}

// Step 2: per replica (blockIdx.x) and (type, component) (threads), the
// chunks in order, into type_mag[r][s][m][t][3] of MCS ctl->g + t_off.
__global__ void k_type_final(int nblk, int t_off, RunArgs ra)
{
    const int r = blockIdx.x;
    const uint32_t g = ra.ctl->g + (uint32_t)t_off;
    const uint32_t s_abs = g / (uint32_t)ra.M, m = g % (uint32_t)ra.M;
    for (int q = threadIdx.x; q < ra.tm_types * 3; q += blockDim.x) {
        double v = 0.0;
        for (int b = 0; b < nblk; ++b) v += ra.tm_part[((size_t)r * nblk + b) * ra.tm_types * 3 + q];
        ra.type_mag[(((size_t)r * ra.S_hist + s_abs) * ra.M + m) * ra.tm_types * 3 + q] = v;
    }
}

// Spins of every replica at the end of step g / M, user order, double, into
// snapshots[r][s][n_max][3].  check: copy only if MCS ctl->g + t_off ends a step.
template <typename T>
__global__ void k_snapshot_site(const RepDesc *reps, int t_off, int check, RunArgs ra)
{
    const uint32_t g = ra.ctl->g + (uint32_t)t_off;
    if (check && (g + 1) % (uint32_t)ra.M != 0) return;
    const RepDesc &rd = reps[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rd.n) return;
    const T *S = (const T *)rd.spins;
    double *o = ra.snapshots + (((size_t)blockIdx.y * ra.S_hist + g / (uint32_t)ra.M) * ra.snap_n +
                                rd.orig[i]) * 3;
    o[0] = (double)S[i];
    o[1] = (double)S[rd.n_pad + i];
    o[2] = (double)S[2 * rd.n_pad + i];
}

__global__ void k_snapshot_rep(RepLaneArgs a, int t_off, int check, RunArgs ra)
{
    const uint32_t g = ra.ctl->g + (uint32_t)t_off;
    if (check && (g + 1) % (uint32_t)ra.M != 0) return;
    const int i = blockIdx.x;
    const size_t plane = (size_t)a.cs;
    for (int r = threadIdx.x; r < a.R; r += blockDim.x) {
        const size_t src = (size_t)i * a.ss + r;
        double *o = ra.snapshots + (((size_t)r * ra.S_hist + g / (uint32_t)ra.M) * ra.snap_n +
                                    a.orig[i]) * 3;
        o[0] = (double)a.spins[src];
        o[1] = (double)a.spins[plane + src];
        o[2] = (double)a.spins[2 * plane + src];
    }
}

}  // namespace

int type_part_blocks(bool replica_layout, int max_n)
{
    return replica_layout ? (max_n + 63) / 64 : (max_n + kOChunk - 1) / kOChunk;
}

hipError_t launch_type_mag_site(hipStream_t st, bool f64, const RepDesc *reps, int R, int max_n,
                                int t_off, const RunArgs &ra)
{
    const int nblk = type_part_blocks(false, max_n);
    if (f64)
        hipLaunchKernelGGL(k_type_part_site<double>, dim3((unsigned)nblk, (unsigned)R), dim3(kOT), 0,
                           st, reps, nblk, ra);
    else
        hipLaunchKernelGGL(k_type_part_site<float>, dim3((unsigned)nblk, (unsigned)R), dim3(kOT), 0,
                           st, reps, nblk, ra);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_type_final, dim3((unsigned)R), dim3(64), 0, st, nblk, t_off, ra);
    return hipGetLastError();
}

hipError_t launch_type_mag_rep(hipStream_t st, const RepLaneArgs &a, int t_off, const RunArgs &ra)
{
    const int nblk = type_part_blocks(true, a.n);
    hipLaunchKernelGGL(k_type_part_rep, dim3((unsigned)nblk), dim3(kOT), 0, st, a, nblk, ra);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_type_final, dim3((unsigned)a.R), dim3(64), 0, st, nblk, t_off, ra);
    return hipGetLastError();
}

hipError_t launch_snapshot_site(hipStream_t st, bool f64, const RepDesc *reps, int R, int max_n,
                                int t_off, bool check, const RunArgs &ra)
{
    dim3 grid((unsigned)((max_n + 255) / 256), (unsigned)R);
    if (f64)
        hipLaunchKernelGGL(k_snapshot_site<double>, grid, dim3(256), 0, st, reps, t_off, check ? 1 : 0, ra);
    else
        hipLaunchKernelGGL(k_snapshot_site<float>, grid, dim3(256), 0, st, reps, t_off, check ? 1 : 0, ra);
    return hipGetLastError();
}

hipError_t launch_snapshot_rep(hipStream_t st, const RepLaneArgs &a, int t_off, bool check,
                               const RunArgs &ra)
{
    hipLaunchKernelGGL(k_snapshot_rep, dim3((unsigned)a.n), dim3(64), 0, st, a, t_off, check ? 1 : 0, ra);
    return hipGetLastError();
}

}  // namespace hsim
