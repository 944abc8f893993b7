// Per-site Metropolis update of the classical Heisenberg model on gfx950:
// random words, trial moves, energy change and acceptance.
//
// Every sweep kernel (site-lane, replica-lane, block-resident, persistent)
// calls these functions, so a site's update is the same instruction sequence
// whatever the layout or launch shape, and spin trajectories do not depend on
// those choices.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hsim_dev.h"

namespace hsim {

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
// 32x32->64-bit products (multipliers 0xD2511F53 on word 0 and 0xCD9E8D57 on
// word 2); the high halves are xored with the other two words and the round
// key, which advances by the Weyl increments 0x9E3779B9 / 0xBB67AE85.
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t t0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t t2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = t0;
        c2 = t2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Words for counter {site, g, replica id, attempt} under the 64-bit seed.
__device__ __forceinline__ uint4 draw(uint64_t seed, uint32_t site, uint32_t g, uint32_t rep,
                                      uint32_t attempt)
{
    return philox4x32_10(site, g, rep, attempt, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// (2k+1) 2^-24 with k the top 23 bits of w: exact in float, inside (0, 1).
__device__ __forceinline__ float u24f(uint32_t w)
{
    return (float)(((w >> 9) << 1) | 1u) * 0x1p-24f;
}

// (2k+1) 2^-53 with k = (hi << 20) | (lo >> 12): exact in double, inside (0, 1).
__device__ __forceinline__ double u53(uint32_t hi, uint32_t lo)
{
    const uint64_t k = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return (double)((k << 1) | 1u) * 0x1p-53;
}

// ------------------------------------------------------------ single precision
struct Trial32 {
    float x, y, z, u;
};

// One call of the generator per update: z = 2 u24(w0) - 1 is uniform on
// (-1, 1) (so the point is uniform on the sphere, Archimedes), the azimuth is
// u24(w1) turns, evaluated by the hardware sine/cosine (which take turns),
// and u24(w2) is the acceptance uniform.
__device__ __forceinline__ Trial32 trial32(uint4 w)
{
    const float z = fmaf(2.0f, u24f(w.x), -1.0f);
    const float turns = u24f(w.y);
    const float r = __builtin_amdgcn_sqrtf(fmaxf(fmaf(-z, z, 1.0f), 0.0f));
    Trial32 t;
    t.x = r * __builtin_amdgcn_cosf(turns);
    t.y = r * __builtin_amdgcn_sinf(turns);
    t.z = z;
    t.u = u24f(w.z);
    return t;
}

// Energy change of S -> S' at a site with local field h (exchange plus
// Zeeman) and uniaxial term -k (S.e)^2:
//   dE = -(S' - S).h - k ((S'.e)^2 - (S.e)^2)
__device__ __forceinline__ float delta_e32(float sx, float sy, float sz, const Trial32 &t,
                                           float hx, float hy, float hz, float k, float ex,
                                           float ey, float ez)
{
    const float dx = t.x - sx, dy = t.y - sy, dz = t.z - sz;
    const float q = fmaf(dz, hz, fmaf(dy, hy, dx * hx));
    const float a1 = fmaf(t.z, ez, fmaf(t.y, ey, t.x * ex));
    const float a0 = fmaf(sz, ez, fmaf(sy, ey, sx * ex));
    return fmaf(-k, (a1 - a0) * (a1 + a0), -q);
}

__device__ __forceinline__ float delta_e32_iso(float sx, float sy, float sz, const Trial32 &t,
                                               float hx, float hy, float hz)
{
    const float dx = t.x - sx, dy = t.y - sy, dz = t.z - sz;
    return -fmaf(dz, hz, fmaf(dy, hy, dx * hx));
}

// Cubic anisotropy function of Eq. 3: Sx^2 Sy^2 + Sy^2 Sz^2 + Sx^2 Sz^2.
__device__ __forceinline__ float cubic32(float x, float y, float z)
{
    const float a = x * x, b = y * y, c = z * z;
    return fmaf(a, c, fmaf(b, c, a * b));
}

// Metropolis rule (Eq. 4, k_B = 1): accept if dE <= 0 or u < exp(-beta dE).
__device__ __forceinline__ bool accept32(float dE, float beta, float u)
{
    const float p = __builtin_amdgcn_exp2f(-(beta * dE) * 1.44269504088896341f);
    return dE <= 0.0f || u < p;
}

// ------------------------------------------------------------ update policies
// Trial moves of the update policies (the moves of Hinzke and Nowak 1999 that
// the paper's "Monte Carlo Metropolis algorithm" section names, plus the
// adaptive Gaussian move): random, spin flip, small step (uniform in the cap
// of half-angle theta around S), Gaussian (S + sigma g normalised), the
// Hinzke-Nowak combination (random, flip or small step, one third each, by
// the fourth word of attempt 0) and adaptive (Gaussian with the replica's
// current width).  Policy ids: POL_* (hsim_dev.h).

// Policy of a site from its type: selects over the (at most NT) table
// entries with constant indices, so the table stays in kernel arguments.
struct SitePol {
    int pol;
    double param, cos_t;
};

template <int NT>
__device__ __forceinline__ SitePol pick_policy(const int32_t (&pol)[NT], const double (&param)[NT],
                                               const double (&cos_t)[NT], int type)
{
    SitePol r{pol[0], param[0], cos_t[0]};
#pragma unroll
    for (int k = 1; k < NT; ++k)
        if (type == k) {
            r.pol = pol[k];
            r.param = param[k];
            r.cos_t = cos_t[k];
        }
    return r;
}

// Adaptive width after an MCS in which n_acc of the n adaptive-move attempts
// of a replica were accepted: scaled by 0.5 / (1 - a), a = n_acc / n, then
// kept in [smin, smax]; unchanged when the replica has no adaptive site.
__device__ __forceinline__ double adapted_sigma(double sigma, double n_acc, double n, double smin,
                                                double smax)
{
    if (!(n > 0.0)) return sigma;
    const double a = n_acc / n;
    const double sg = sigma * (0.5 / (1.0 - a));
    return fmin(smax, fmax(smin, sg));
}

// Part of the Hinzke-Nowak combination: floor(3 w / 2^32).
__device__ __forceinline__ int hn_part(uint32_t w)
{
    return (int)(((uint64_t)w * 3u) >> 32);
}

// Single precision (u_k = u24 of word k of attempt 0):
//   flip: -S, acceptance u2;
//   small step: cos of the angle to S c = 1 - u0 (1 - cos theta), azimuth u1
//     turns in the basis below, acceptance u2;
//   Gaussian: normals (r0 cos 2pi u1, r0 sin 2pi u1, r1 cos 2pi u3) with
//     r0 = sqrt(-2 ln u0), r1 = sqrt(-2 ln u2); acceptance u24 of word 0 of
//     attempt 1.
// Small-step and Gaussian trials are normalised.
__device__ __forceinline__ void onb32(float nx, float ny, float nz, float (&b1)[3], float (&b2)[3])
{
    // Duff et al., "Building an orthonormal basis, revisited" (JCGT 2017)
    const float sign = copysignf(1.0f, nz);
    const float a = -1.0f / (sign + nz);
    const float b = nx * ny * a;
    b1[0] = 1.0f + sign * nx * nx * a;
    b1[1] = sign * b;
    b1[2] = -sign * nx;
    b2[0] = b;
    b2[1] = sign + ny * ny * a;
    b2[2] = -ny;
}

__device__ __forceinline__ void normalise32(float &x, float &y, float &z, float sx, float sy,
                                            float sz)
{
    const float nn = fmaf(z, z, fmaf(y, y, x * x));
    if (nn > 0.0f) {
        const float r = __builtin_amdgcn_rsqf(nn);
        x *= r;
        y *= r;
        z *= r;
    } else {
        x = sx;
        y = sy;
        z = sz;
    }
}

// omc: 1 - cos theta (rounded once from double).  The cap point uses
// sin = sqrt(d (2 - d)) with d = 1 - c, free of the cancellation in 1 - c^2.
__device__ __forceinline__ Trial32 trial32_policy(int pol, uint4 w, float sx, float sy, float sz,
                                                  float param, float omc, uint64_t seed,
                                                  uint32_t site, uint32_t g, uint32_t rep)
{
    if (pol == POL_HN) {
        const int part = hn_part(w.w);
        pol = part == 0 ? POL_RANDOM : (part == 1 ? POL_FLIP : POL_SMALL_STEP);
    }
    if (pol == POL_RANDOM) return trial32(w);
    Trial32 t;
    if (pol == POL_FLIP) {
        t.x = -sx;
        t.y = -sy;
        t.z = -sz;
        t.u = u24f(w.z);
        return t;
    }
    if (pol == POL_SMALL_STEP) {
        const float d = u24f(w.x) * omc;
        const float c = 1.0f - d;
        const float turns = u24f(w.y);
        const float cp = __builtin_amdgcn_cosf(turns), sp = __builtin_amdgcn_sinf(turns);
        float b1[3], b2[3];
        onb32(sx, sy, sz, b1, b2);
        const float st = __builtin_amdgcn_sqrtf(fmaxf(d * (2.0f - d), 0.0f));
        t.x = fmaf(c, sx, st * fmaf(cp, b1[0], sp * b2[0]));
        t.y = fmaf(c, sy, st * fmaf(cp, b1[1], sp * b2[1]));
        t.z = fmaf(c, sz, st * fmaf(cp, b1[2], sp * b2[2]));
        normalise32(t.x, t.y, t.z, sx, sy, sz);
        t.u = u24f(w.z);
        return t;
    }
    // Gaussian / adaptive: -2 ln u = -2 ln 2 log2 u
    const float r0 = __builtin_amdgcn_sqrtf(-1.38629436111989061f * __builtin_amdgcn_logf(u24f(w.x)));
    const float r1 = __builtin_amdgcn_sqrtf(-1.38629436111989061f * __builtin_amdgcn_logf(u24f(w.z)));
    const float t1 = u24f(w.y), t3 = u24f(w.w);
    t.x = fmaf(param, r0 * __builtin_amdgcn_cosf(t1), sx);
    t.y = fmaf(param, r0 * __builtin_amdgcn_sinf(t1), sy);
    t.z = fmaf(param, r1 * __builtin_amdgcn_cosf(t3), sz);
    normalise32(t.x, t.y, t.z, sx, sy, sz);
    t.u = u24f(draw(seed, site, g, rep, 1).x);
    return t;
}

// ------------------------------------------------------------ double precision
// The validation mode follows a fixed operation order with no contraction
// (the library is built with -ffp-contract=off), so that it reproduces a
// serial double-precision evaluation of the same rules.
#pragma clang fp contract(off)

// Marsaglia (1972): from attempt t's words, v1 = 2 u53(w0,w1) - 1 and
// v2 = 2 u53(w2,w3) - 1; reject s = v1^2 + v2^2 >= 1; the point is
// (2 v1 sqrt(1-s), 2 v2 sqrt(1-s), 1 - 2s).  Attempts 1..32, then +z.
__device__ inline void sphere64(uint64_t seed, uint32_t site, uint32_t g, uint32_t rep, double &x,
                                double &y, double &z)
{
    for (uint32_t t = 1; t <= 32; ++t) {
        const uint4 w = draw(seed, site, g, rep, t);
        const double v1 = 2.0 * u53(w.x, w.y) - 1.0;
        const double v2 = 2.0 * u53(w.z, w.w) - 1.0;
        const double s = v1 * v1 + v2 * v2;
        if (s < 1.0) {
            const double f = 2.0 * sqrt(1.0 - s);
            x = v1 * f;
            y = v2 * f;
            z = 1.0 - 2.0 * s;
            return;
        }
    }
    x = 0.0;
    y = 0.0;
    z = 1.0;
}

__device__ inline double dot64(double ax, double ay, double az, double bx, double by, double bz)
{
    return (ax * bx + ay * by) + az * bz;
}

// Full validation-mode update.  h already includes the Zeeman term.
// Returns true if the move is accepted; (nx, ny, nz) is the proposal.
__device__ inline bool update64(uint64_t seed, uint32_t site, uint32_t g, uint32_t rep, double sx,
                                double sy, double sz, double hx, double hy, double hz, double k,
                                double ex, double ey, double ez, double beta, double &nx,
                                double &ny, double &nz, double &dE)
{
    const uint4 w0 = draw(seed, site, g, rep, 0);
    const double u = u53(w0.x, w0.y);
    sphere64(seed, site, g, rep, nx, ny, nz);
    const double dSx = nx - sx, dSy = ny - sy, dSz = nz - sz;
    const double q = (dSx * hx + dSy * hy) + dSz * hz;
    const double a1 = dot64(nx, ny, nz, ex, ey, ez);
    const double a0 = dot64(sx, sy, sz, ex, ey, ez);
    dE = -q - k * (a1 * a1 - a0 * a0);
    if (dE <= 0.0) return true;
    return u < exp(-beta * dE);
}

// Natural logarithm from correctly rounded operations only, so that it is
// reproducible bit for bit: x = m 2^e with m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(t), t = (m-1)/(m+1), summed as 2t (1 + t^2/3 + ... + t^22/23)
// in Horner form; ln x = e ln 2 + ln m.  x > 0 finite.
__device__ inline double log_exact(double x)
{
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752440) {
        m = m * 2.0;
        e = e - 1;
    }
    const double t = (m - 1.0) / (m + 1.0);
    const double t2 = t * t;
    double p = 1.0 / 23.0;
    for (int k = 10; k >= 0; --k) p = p * t2 + 1.0 / (double)(2 * k + 1);
    return (double)e * 0x1.62e42fefa39efp-1 + 2.0 * t * p;
}

// Duff et al. (JCGT 2017) basis perpendicular to the unit vector n.
__device__ inline void onb64(double nx, double ny, double nz, double (&b1)[3], double (&b2)[3])
{
    const double sign = copysign(1.0, nz);
    const double a = -1.0 / (sign + nz);
    const double b = nx * ny * a;
    b1[0] = 1.0 + sign * nx * nx * a;
    b1[1] = sign * b;
    b1[2] = -sign * nx;
    b2[0] = b;
    b2[1] = sign + ny * ny * a;
    b2[2] = -ny;
}

__device__ inline void normalise64(double &x, double &y, double &z, double sx, double sy, double sz)
{
    const double nn = sqrt((x * x + y * y) + z * z);
    if (nn > 0.0) {
        x = x / nn;
        y = y / nn;
        z = z / nn;
    } else {
        x = sx;
        y = sy;
        z = sz;
    }
}

// A point (v1, v2) uniform in the unit disk minus its centre from attempts
// att, att+1, ... (v = 2 u53 - 1 per word pair); att moves past the accepted
// attempt.  False after 64 rejections.
__device__ inline bool disk64(uint64_t seed, uint32_t site, uint32_t g, uint32_t rep, uint32_t &att,
                              double &v1, double &v2, double &s)
{
    for (int tries = 0; tries < 64; ++tries) {
        const uint4 w = draw(seed, site, g, rep, att++);
        const double a = 2.0 * u53(w.x, w.y) - 1.0;
        const double b = 2.0 * u53(w.z, w.w) - 1.0;
        const double q = a * a + b * b;
        if (q < 1.0 && q > 0.0) {
            v1 = a;
            v2 = b;
            s = q;
            return true;
        }
    }
    return false;
}

// Validation-mode trial of a policy: acceptance uniform u53(w0, w1) of
// attempt 0 (returned); random: Marsaglia, attempts 1..32; flip: -S; small
// step: c = 1 - u53(attempt 1: w0, w1) (1 - cos theta), azimuth from the first
// disk point of attempts 2.., normalised; Gaussian: polar-method normals
// (v f with f = sqrt(-2 ln s / s)) from disk points of attempts 1.., two of the
// first point and one of the second, normalised; Hinzke-Nowak: part from w3.
__device__ inline double trial64_policy(int pol, uint64_t seed, uint32_t site, uint32_t g,
                                        uint32_t rep, double sx, double sy, double sz,
                                        double param, double cos_t, double &nx, double &ny,
                                        double &nz)
{
    const uint4 w0 = draw(seed, site, g, rep, 0);
    const double u = u53(w0.x, w0.y);
    if (pol == POL_HN) {
        const int part = hn_part(w0.w);
        pol = part == 0 ? POL_RANDOM : (part == 1 ? POL_FLIP : POL_SMALL_STEP);
    }
    if (pol == POL_RANDOM) {
        sphere64(seed, site, g, rep, nx, ny, nz);
    } else if (pol == POL_FLIP) {
        nx = -sx;
        ny = -sy;
        nz = -sz;
    } else if (pol == POL_SMALL_STEP) {
        const uint4 w1 = draw(seed, site, g, rep, 1);
        const double c = 1.0 - u53(w1.x, w1.y) * (1.0 - cos_t);
        uint32_t att = 2;
        double v1, v2, q, cp = 1.0, sp = 0.0;
        if (disk64(seed, site, g, rep, att, v1, v2, q)) {
            const double r = sqrt(q);
            cp = v1 / r;
            sp = v2 / r;
        }
        double b1[3], b2[3];
        onb64(sx, sy, sz, b1, b2);
        const double st2 = 1.0 - c * c;
        const double st = sqrt(st2 > 0.0 ? st2 : 0.0);
        nx = c * sx + st * (cp * b1[0] + sp * b2[0]);
        ny = c * sy + st * (cp * b1[1] + sp * b2[1]);
        nz = c * sz + st * (cp * b1[2] + sp * b2[2]);
        normalise64(nx, ny, nz, sx, sy, sz);
    } else {
        double n0 = 0.0, n1 = 0.0, n2 = 0.0;
        uint32_t att = 1;
        double v1, v2, q;
        if (disk64(seed, site, g, rep, att, v1, v2, q)) {
            const double f = sqrt(-2.0 * log_exact(q) / q);
            n0 = v1 * f;
            n1 = v2 * f;
            if (disk64(seed, site, g, rep, att, v1, v2, q)) {
                const double f2 = sqrt(-2.0 * log_exact(q) / q);
                n2 = v1 * f2;
            }
        }
        nx = sx + param * n0;
        ny = sy + param * n1;
        nz = sz + param * n2;
        normalise64(nx, ny, nz, sx, sy, sz);
    }
    return u;
}

// Eq. 3's function in the validation mode, in the order
// (a b + b c) + a c with a = Sx^2, b = Sy^2, c = Sz^2.
__device__ inline double cubic64(double x, double y, double z)
{
    const double a = x * x, b = y * y, c = z * z;
    return (a * b + b * c) + a * c;
}

// Validation-mode update under a policy (random: identical to update64).
__device__ inline bool update64_policy(int pol, double param, double cos_t, uint64_t seed,
                                       uint32_t site, uint32_t g, uint32_t rep, double sx,
                                       double sy, double sz, double hx, double hy, double hz,
                                       double k, double ex, double ey, double ez, double beta,
                                       double &nx, double &ny, double &nz, double &dE)
{
    const double u = trial64_policy(pol, seed, site, g, rep, sx, sy, sz, param, cos_t, nx, ny, nz);
    const double dSx = nx - sx, dSy = ny - sy, dSz = nz - sz;
    const double q = (dSx * hx + dSy * hy) + dSz * hz;
    const double a1 = dot64(nx, ny, nz, ex, ey, ez);
    const double a0 = dot64(sx, sy, sz, ex, ey, ez);
    dE = -q - k * (a1 * a1 - a0 * a0);
    if (dE <= 0.0) return true;
    return u < exp(-beta * dE);
}

// Validation-mode update of a spin of length mu (has_mu) with a cubic term
// kc (has_kc): the trial acts on the direction S / mu and gets the length
// back, and dE gains -kc (f(S') - f(S)).  Without either term it is
// update64 / update64_policy.
__device__ inline bool update64_general(int pol, double param, double cos_t, uint64_t seed,
                                        uint32_t site, uint32_t g, uint32_t rep, double sx,
                                        double sy, double sz, double hx, double hy, double hz,
                                        double k, double ex, double ey, double ez, bool has_kc,
                                        double kc, bool has_mu, double mu, double beta, double &nx,
                                        double &ny, double &nz, double &dE)
{
    double dx = sx, dy = sy, dz = sz;
    if (has_mu) {
        dx = sx / mu;
        dy = sy / mu;
        dz = sz / mu;
    }
    double u;
    if (pol == POL_RANDOM) {
        const uint4 w0 = draw(seed, site, g, rep, 0);
        u = u53(w0.x, w0.y);
        sphere64(seed, site, g, rep, nx, ny, nz);
    } else {
        u = trial64_policy(pol, seed, site, g, rep, dx, dy, dz, param, cos_t, nx, ny, nz);
    }
    if (has_mu) {
        nx = mu * nx;
        ny = mu * ny;
        nz = mu * nz;
    }
    const double dSx = nx - sx, dSy = ny - sy, dSz = nz - sz;
    const double q = (dSx * hx + dSy * hy) + dSz * hz;
    const double a1 = dot64(nx, ny, nz, ex, ey, ez);
    const double a0 = dot64(sx, sy, sz, ex, ey, ez);
    dE = -q - k * (a1 * a1 - a0 * a0);
    if (has_kc) dE = dE - kc * (cubic64(nx, ny, nz) - cubic64(sx, sy, sz));
    if (dE <= 0.0) return true;
    return u < exp(-beta * dE);
}


}  // namespace hsim
