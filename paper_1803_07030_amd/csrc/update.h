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

// Metropolis rule (Eq. 4, k_B = 1): accept if dE <= 0 or u < exp(-beta dE).
__device__ __forceinline__ bool accept32(float dE, float beta, float u)
{
    const float p = __builtin_amdgcn_exp2f(-(beta * dE) * 1.44269504088896341f);
    return dE <= 0.0f || u < p;
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


}  // namespace hsim
