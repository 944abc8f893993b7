// Analysis of the per-MCS history on the GPU (double precision).
//
// Paper: thermal averages of M, chi and the specific heat ("Thermal
// averages"); cumulants of the magnetisation for finite-size scaling
// ("Critical exponents"); equilibrium correlation times ("Dynamic
// behavior"); single and multiple histogram reweighting ("Histogram and
// multiple histogram methods").
//
// A series is the history of one replica at one temperature/field step,
// history[r][s][m][5] = (E, Mx, My, Mz, accepted), MCS m0 .. M-1.  Every sum
// is taken in a fixed order (strided per thread, then a fixed tree), so the
// results are reproducible run to run.
#include <cmath>
#include <vector>

#include "hsim_host.h"

namespace hsim {

namespace {

constexpr int kAT = 256;   // threads per analysis block

// Block-wide sum (fixed order: per-thread values, then a halving tree);
// every thread gets the result.
__device__ double block_sum(double v, double *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = kAT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

__device__ double block_max(double v, double *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = kAT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

// Sample k of a set of series: series t = k / n, MCS m0 + k % n.
struct Samples {
    const double *hist;
    const int32_t *rs;     // [K][2] (replica, step)
    int32_t S, M, m0, n;   // steps, MCS per step, first MCS, samples per series
    __device__ const double *rec(int64_t k) const
    {
        const int t = (int)(k / n), m = m0 + (int)(k % n);
        return hist + (((size_t)rs[2 * t] * S + rs[2 * t + 1]) * M + m) * 5;
    }
    __device__ double E(int64_t k) const { return rec(k)[0]; }
    __device__ double A(int64_t k) const
    {
        const double *h = rec(k);
        return sqrt((h[1] * h[1] + h[2] * h[2]) + h[3] * h[3]);
    }
};

// Thermal summary of samples [k0, k0 + count) with log-weights
// logw(k) (weights shifted by their maximum); out[9] =
// (e, m_abs, m2, m4, cv, chi, u4, v1, v2) for N sites at beta.
template <typename LW>
__device__ void thermal_block(const Samples &sm, int64_t k0, int64_t count, LW logw, double N,
                              double beta, double *lds, double *out)
{
    double mx = -INFINITY;
    for (int64_t k = threadIdx.x; k < count; k += kAT) mx = fmax(mx, logw(k0 + k));
    mx = block_max(mx, lds);
    double sw = 0, sE = 0, sA = 0, sA2 = 0, sA4 = 0;
    for (int64_t k = threadIdx.x; k < count; k += kAT) {
        const double w = exp(logw(k0 + k) - mx);
        const double e = sm.E(k0 + k), a = sm.A(k0 + k), a2 = a * a;
        sw += w;
        sE += w * e;
        sA += w * a;
        sA2 += w * a2;
        sA4 += w * (a2 * a2);
    }
    const double W = block_sum(sw, lds);
    const double mE = block_sum(sE, lds) / W, mA = block_sum(sA, lds) / W;
    const double mA2 = block_sum(sA2, lds) / W, mA4 = block_sum(sA4, lds) / W;
    double vE = 0, vA = 0, c1 = 0, c2 = 0;
    for (int64_t k = threadIdx.x; k < count; k += kAT) {
        const double w = exp(logw(k0 + k) - mx);
        const double a = sm.A(k0 + k);
        const double dE = sm.E(k0 + k) - mE, dA = a - mA, dA2 = a * a - mA2;
        vE += w * (dE * dE);
        vA += w * (dA * dA);
        c1 += w * (dA * dE);
        c2 += w * (dA2 * dE);
    }
    vE = block_sum(vE, lds) / W;
    vA = block_sum(vA, lds) / W;
    c1 = block_sum(c1, lds) / W;
    c2 = block_sum(c2, lds) / W;
    if (threadIdx.x == 0) {
        const double m2 = mA2 / (N * N), m4 = mA4 / (N * N * N * N);
        out[0] = mE / N;
        out[1] = mA / N;
        out[2] = m2;
        out[3] = m4;
        out[4] = beta * beta * vE / N;
        out[5] = beta * vA / N;
        out[6] = m2 > 0 ? 1.0 - m4 / (3.0 * m2 * m2) : 0.0;
        out[7] = mA > 0 ? -c1 / mA : 0.0;
        out[8] = mA2 > 0 ? -c2 / mA2 : 0.0;
    }
}

// grid (series, n_eval): series t at its sampling beta0[t], evaluated at
// beta_eval[t][j] with weights exp(-(beta - beta0) E).
__global__ __launch_bounds__(kAT) void k_thermal(Samples sm, double N, const double *beta0,
                                                 const double *beta_eval, int n_eval, double *out)
{
    __shared__ double lds[kAT];
    const int t = blockIdx.x, j = blockIdx.y;
    const double b0 = beta0[t], b = beta_eval[(size_t)t * n_eval + j];
    const double db = b - b0;
    auto logw = [&](int64_t k) { return db == 0.0 ? 0.0 : -db * sm.E(k); };
    thermal_block(sm, (int64_t)t * sm.n, sm.n, logw, N, b, lds, out + ((size_t)t * n_eval + j) * 9);
}

// Integrated autocorrelation time of series t (observable 0: E, 1: |M|)
// with the automatic window of Sokal: lags are evaluated 256 at a time, each
// as one ordered sum, and thread 0 walks them until lag >= c tau.
__global__ __launch_bounds__(kAT) void k_tau(Samples sm, int obs, double c, double *tau_out,
                                             int32_t *win_out)
{
    __shared__ double lds[kAT];
    __shared__ double rho[kAT];
    __shared__ int done;
    const int t = blockIdx.x;
    const int64_t k0 = (int64_t)t * sm.n;
    const int n = sm.n;
    auto x = [&](int m) { return obs == 0 ? sm.E(k0 + m) : sm.A(k0 + m); };
    double s = 0.0;
    for (int m = threadIdx.x; m < n; m += kAT) s += x(m);
    const double mean = block_sum(s, lds) / n;
    double q = 0.0;
    for (int m = threadIdx.x; m < n; m += kAT) {
        const double d = x(m) - mean;
        q += d * d;
    }
    const double c0 = block_sum(q, lds) / n;
    double tau = 0.5;
    int win = n / 2;
    if (threadIdx.x == 0) done = c0 > 0.0 ? 0 : 1;
    __syncthreads();
    for (int base = 1; base <= n / 2 && !done; base += kAT) {
        const int lag = base + (int)threadIdx.x;
        double r = 0.0;
        if (lag <= n / 2) {
            for (int m = 0; m + lag < n; ++m) r += (x(m) - mean) * (x(m + lag) - mean);
            r = r / (n - lag) / c0;
        }
        rho[threadIdx.x] = r;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int u = 0; u < kAT && base + u <= n / 2; ++u) {
                tau += rho[u];
                if (base + u >= c * tau) {
                    win = base + u;
                    done = 1;
                    break;
                }
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        tau_out[t] = c0 > 0.0 ? tau : 0.5;
        if (win_out) win_out[t] = c0 > 0.0 ? win : 0;
    }
}

// Multiple histogram, per sample: ln D = ln sum_j n_j exp(f_j - beta_j E),
// shifted by the largest exponent.
__global__ void k_mh_logd(Samples sm, int K, const double *beta_k, const double *f,
                          double *logd)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)K * sm.n) return;
    const double e = sm.E(k), ln_n = log((double)sm.n);
    double mx = -INFINITY;
    for (int j = 0; j < K; ++j) mx = fmax(mx, ln_n + f[j] - beta_k[j] * e);
    double s = 0.0;
    for (int j = 0; j < K; ++j) s += exp(ln_n + f[j] - beta_k[j] * e - mx);
    logd[k] = mx + log(s);
}

// f_k = -ln sum_i exp(-beta_k E_i - ln D_i), one block per k.
__global__ __launch_bounds__(kAT) void k_mh_f(Samples sm, int K, const double *beta_k,
                                              const double *logd, double *f_new)
{
    __shared__ double lds[kAT];
    const int k = blockIdx.x;
    const int64_t tot = (int64_t)K * sm.n;
    const double b = beta_k[k];
    double mx = -INFINITY;
    for (int64_t i = threadIdx.x; i < tot; i += kAT) mx = fmax(mx, -b * sm.E(i) - logd[i]);
    mx = block_max(mx, lds);
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < tot; i += kAT) s += exp(-b * sm.E(i) - logd[i] - mx);
    s = block_sum(s, lds);
    if (threadIdx.x == 0) f_new[k] = -(mx + log(s));
}

// Thermal summary at beta_eval[j] from all samples of the K series with
// weights exp(-beta E - ln D).
__global__ __launch_bounds__(kAT) void k_mh_thermal(Samples sm, int K, double N, const double *logd,
                                                    const double *beta_eval, double *out)
{
    __shared__ double lds[kAT];
    const int j = blockIdx.x;
    const double b = beta_eval[j];
    auto logw = [&](int64_t k) { return -b * sm.E(k) - logd[k]; };
    thermal_block(sm, 0, (int64_t)K * sm.n, logw, N, b, lds, out + (size_t)j * 9);
}

void check_hist(const double *h, int32_t R, int32_t S, int32_t M, int32_t m0)
{
    if (!h || R < 1 || S < 1 || M < 1 || m0 < 0 || M - m0 < 2)
        throw Error(HSIM_E_ARG, "analysis: bad history shape or first MCS");
}

}  // namespace

void analysis_thermal_impl(const double *d_hist, int32_t R, int32_t S, int32_t M, int32_t m0,
                           int64_t n_sites, const double *beta, int32_t n_eval,
                           const double *beta_eval, double *d_out, hipStream_t st)
{
    check_hist(d_hist, R, S, M, m0);
    if (n_sites < 1 || !beta || n_eval < 1 || !d_out || (n_eval > 1 && !beta_eval))
        throw Error(HSIM_E_ARG, "analysis_thermal: bad argument");
    const int T = R * S;
    std::vector<int32_t> rs(2 * (size_t)T);
    std::vector<double> be((size_t)T * n_eval);
    for (int t = 0; t < T; ++t) {
        rs[2 * t] = t / S;
        rs[2 * t + 1] = t % S;
        if (!std::isfinite(beta[t]) || beta[t] < 0) throw Error(HSIM_E_PARAM, "beta must be finite and >= 0");
        for (int j = 0; j < n_eval; ++j) {
            const double b = beta_eval ? beta_eval[(size_t)t * n_eval + j] : beta[t];
            if (!std::isfinite(b) || b < 0) throw Error(HSIM_E_PARAM, "beta must be finite and >= 0");
            be[(size_t)t * n_eval + j] = b;
        }
    }
    DevBuf d_rs, d_b0, d_be;
    d_rs.upload(rs);
    d_b0.upload(std::vector<double>(beta, beta + T));
    d_be.upload(be);
    Samples sm{d_hist, (const int32_t *)d_rs.p, S, M, m0, M - m0};
    hipLaunchKernelGGL(k_thermal, dim3((unsigned)T, (unsigned)n_eval), dim3(kAT), 0, st, sm,
                       (double)n_sites, (const double *)d_b0.p, (const double *)d_be.p, n_eval,
                       d_out);
    hip_check(hipGetLastError(), "thermal launch");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");   // before the tables are freed
}

void analysis_tau_impl(const double *d_hist, int32_t R, int32_t S, int32_t M, int32_t m0,
                       int32_t obs, double c, double *d_tau, int32_t *d_win, hipStream_t st)
{
    check_hist(d_hist, R, S, M, m0);
    if ((obs != 0 && obs != 1) || !(c > 0.0) || !d_tau) throw Error(HSIM_E_ARG, "analysis_tau: bad argument");
    const int T = R * S;
    std::vector<int32_t> rs(2 * (size_t)T);
    for (int t = 0; t < T; ++t) {
        rs[2 * t] = t / S;
        rs[2 * t + 1] = t % S;
    }
    DevBuf d_rs;
    d_rs.upload(rs);
    Samples sm{d_hist, (const int32_t *)d_rs.p, S, M, m0, M - m0};
    hipLaunchKernelGGL(k_tau, dim3((unsigned)T), dim3(kAT), 0, st, sm, obs, c, d_tau, d_win);
    hip_check(hipGetLastError(), "tau launch");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
}

void analysis_multihist_impl(const double *d_hist, int32_t R, int32_t S, int32_t M, int32_t m0,
                             int64_t n_sites, int32_t K, const int32_t *series,
                             const double *beta_k, int32_t n_eval, const double *beta_eval,
                             int32_t max_iter, double tol, double *f_out, int32_t *iters_out,
                             double *d_out, hipStream_t st)
{
    check_hist(d_hist, R, S, M, m0);
    if (n_sites < 1 || K < 1 || !series || !beta_k || n_eval < 0 || (n_eval > 0 && (!beta_eval || !d_out)) ||
        max_iter < 1 || !(tol > 0.0) || !f_out)
        throw Error(HSIM_E_ARG, "analysis_multihist: bad argument");
    std::vector<int32_t> rs(series, series + 2 * (size_t)K);
    for (int k = 0; k < K; ++k) {
        if (rs[2 * k] < 0 || rs[2 * k] >= R || rs[2 * k + 1] < 0 || rs[2 * k + 1] >= S)
            throw Error(HSIM_E_ARG, "analysis_multihist: series outside the history");
        if (!std::isfinite(beta_k[k]) || beta_k[k] < 0) throw Error(HSIM_E_PARAM, "beta must be finite and >= 0");
    }
    for (int j = 0; j < n_eval; ++j)
        if (!std::isfinite(beta_eval[j]) || beta_eval[j] < 0) throw Error(HSIM_E_PARAM, "beta must be finite and >= 0");
    const int n = M - m0;
    const int64_t tot = (int64_t)K * n;
    DevBuf d_rs, d_bk, d_f, d_fn, d_logd, d_be;
    d_rs.upload(rs);
    d_bk.upload(std::vector<double>(beta_k, beta_k + K));
    std::vector<double> f((size_t)K, 0.0), fn((size_t)K);
    d_f.upload(f);
    d_fn.alloc((size_t)K * 8);
    d_logd.alloc((size_t)tot * 8);
    Samples sm{d_hist, (const int32_t *)d_rs.p, S, M, m0, n};
    const unsigned gl = (unsigned)((tot + 255) / 256);
    int it = 0;
    while (it < max_iter) {
        ++it;
        hipLaunchKernelGGL(k_mh_logd, dim3(gl), dim3(256), 0, st, sm, K, (const double *)d_bk.p,
                           (const double *)d_f.p, (double *)d_logd.p);
        hipLaunchKernelGGL(k_mh_f, dim3((unsigned)K), dim3(kAT), 0, st, sm, K, (const double *)d_bk.p,
                           (const double *)d_logd.p, (double *)d_fn.p);
        hip_check(hipGetLastError(), "multihist launch");
        hip_check(hipMemcpyAsync(fn.data(), d_fn.p, (size_t)K * 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        double dmax = 0.0;
        const double f0 = fn[0];
        for (int k = 0; k < K; ++k) {
            fn[k] = fn[k] - f0;
            dmax = std::max(dmax, std::fabs(fn[k] - f[k]));
        }
        f = fn;
        hip_check(hipMemcpyAsync(d_f.p, f.data(), (size_t)K * 8, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
        if (dmax < tol) break;
    }
    hipLaunchKernelGGL(k_mh_logd, dim3(gl), dim3(256), 0, st, sm, K, (const double *)d_bk.p,
                       (const double *)d_f.p, (double *)d_logd.p);
    if (n_eval > 0) {
        d_be.upload(std::vector<double>(beta_eval, beta_eval + n_eval));
        hipLaunchKernelGGL(k_mh_thermal, dim3((unsigned)n_eval), dim3(kAT), 0, st, sm, K,
                           (double)n_sites, (const double *)d_logd.p, (const double *)d_be.p, d_out);
    }
    hip_check(hipGetLastError(), "multihist launch");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    for (int k = 0; k < K; ++k) f_out[k] = f[k];
    if (iters_out) *iters_out = it;
}

}  // namespace hsim
