/*
 * CPU oracle of the Heisenberg Metropolis hot path.  TEST INFRASTRUCTURE ONLY:
 * loaded by the tests, the smoke check and the CPU-baseline leg of the
 * benchmark, never by the GPU library, with which it shares no code.
 *
 * Plain, serial, double precision; built with -O2 -ffp-contract=off so that
 * every operation below is rounded separately, in the order written.
 * The numeric contract that the GPU path reproduces independently (counter
 * layout of the random words, uniform maps, proposal maps, operation order)
 * is stated next to each function.
 */
#include "hsim_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11).  Each round multiplies words 0 and 2 of the
 * counter by the two round multipliers, takes the 64-bit products apart, and
 * mixes the high halves with the other two words and the round key; the key
 * is advanced by the two Weyl constants between rounds. */
#define OR_TWO_PI 6.283185307179586476925286766559
#define OR_PHILOX_M0 0xD2511F53u
#define OR_PHILOX_M1 0xCD9E8D57u
#define OR_PHILOX_W0 0x9E3779B9u
#define OR_PHILOX_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)OR_PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)OR_PHILOX_M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += OR_PHILOX_W0;
        k1 += OR_PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void or_philox_batch(int64_t count, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    for (int64_t t = 0; t < count; ++t) or_philox4x32_10(ctr + 4 * t, key, out + 4 * t);
}

static void words(uint64_t seed, uint32_t site, uint32_t g, uint32_t rep, uint32_t attempt,
                  uint32_t w[4])
{
    /* key = 64-bit seed, low word first; counter = {site, g, replica, attempt} */
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {site, g, rep, attempt};
    or_philox4x32_10(ctr, key, w);
}

/* u = (2k+1) 2^-53 with k the 52-bit number (hi << 20) | (lo >> 12): exact, in (0,1). */
double or_u53(uint32_t hi, uint32_t lo)
{
    uint64_t k = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return (double)(2 * k + 1) * 0x1p-53;
}

/* u = (2k+1) 2^-24 with k = w >> 9 (23 bits): exact in single precision, in (0,1). */
double or_u24(uint32_t w)
{
    uint32_t k = w >> 9;
    return (double)(2 * k + 1) * 0x1p-24;
}

/* Marsaglia (1972): v1, v2 uniform in (-1,1) from attempt t's four words;
 * reject s = v1^2 + v2^2 >= 1; the point is (2 v1 sqrt(1-s), 2 v2 sqrt(1-s), 1-2s).
 * Attempts 1..32; after 32 rejections (probability below 1e-21) the point is +z. */
int or_sphere_exact(uint64_t seed, uint32_t site, uint32_t g, uint32_t rep, double out[3])
{
    for (uint32_t t = 1; t <= 32; ++t) {
        uint32_t w[4];
        words(seed, site, g, rep, t, w);
        double v1 = 2.0 * or_u53(w[0], w[1]) - 1.0;
        double v2 = 2.0 * or_u53(w[2], w[3]) - 1.0;
        double s = v1 * v1 + v2 * v2;
        if (s < 1.0) {
            double f = 2.0 * sqrt(1.0 - s);
            out[0] = v1 * f;
            out[1] = v2 * f;
            out[2] = 1.0 - 2.0 * s;
            return (int)t;
        }
    }
    out[0] = 0.0; out[1] = 0.0; out[2] = 1.0;
    return 33;
}

/* Single-call proposal of the production (single-precision) mode: with words
 * (w0, w1, w2) of attempt 0, z = 2 u24(w0) - 1, phi = u24(w1) turns,
 * point (r cos 2 pi phi, r sin 2 pi phi, z) with r = sqrt(1 - z^2); the
 * acceptance uniform is u24(w2).  Evaluated here in double. */
void or_sphere_f32map(uint64_t seed, uint32_t site, uint32_t g, uint32_t rep, double out[3],
                      double *u_out)
{
    uint32_t w[4];
    words(seed, site, g, rep, 0, w);
    double z = 2.0 * or_u24(w[0]) - 1.0;
    double phi = or_u24(w[1]);
    double r2 = 1.0 - z * z;
    double r = sqrt(r2 > 0.0 ? r2 : 0.0);
    double ang = OR_TWO_PI * phi;
    out[0] = r * cos(ang);
    out[1] = r * sin(ang);
    out[2] = z;
    if (u_out) *u_out = or_u24(w[2]);
}

/* ---------------------------------------------------------------------- */
/* Natural logarithm from correctly rounded operations only: x = m 2^e with m
 * in [sqrt(1/2), sqrt(2)) (exact), ln m = 2 atanh(t) with t = (m-1)/(m+1),
 * |t| < 0.172, summed as 2t (1 + t^2/3 + ... + t^22/23) in Horner form (the
 * next term is below 2^-60 of the sum); ln x = e ln 2 + ln m. */
double or_log(double x)
{
    int e;
    double m = frexp(x, &e);                 /* m in [0.5, 1) */
    if (m < 0.70710678118654752440) {
        m = m * 2.0;
        e = e - 1;
    }
    double t = (m - 1.0) / (m + 1.0);
    double t2 = t * t;
    double p = 1.0 / 23.0;
    for (int k = 10; k >= 0; --k) p = p * t2 + 1.0 / (double)(2 * k + 1);
    return (double)e * 0x1.62e42fefa39efp-1 + 2.0 * t * p;
}

/* Orthonormal pair perpendicular to the unit vector n (Duff, Burgess,
 * Christensen, Hery, Kensler, Liani and Villemin, "Building an orthonormal
 * basis, revisited", JCGT 2017), products taken left to right. */
static void onb(const double n[3], double b1[3], double b2[3])
{
    double sign = copysign(1.0, n[2]);
    double a = -1.0 / (sign + n[2]);
    double b = n[0] * n[1] * a;
    b1[0] = 1.0 + sign * n[0] * n[0] * a;
    b1[1] = sign * b;
    b1[2] = -sign * n[0];
    b2[0] = b;
    b2[1] = sign + n[1] * n[1] * a;
    b2[2] = -n[1];
}

/* v / |v|, or s unchanged when |v| is 0. */
static void normalise(const double v[3], const double s[3], double out[3])
{
    double nn = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    if (nn > 0.0) {
        out[0] = v[0] / nn;
        out[1] = v[1] / nn;
        out[2] = v[2] / nn;
    } else {
        out[0] = s[0];
        out[1] = s[1];
        out[2] = s[2];
    }
}

/* Point of the cap around s: polar cosine c, azimuth (cphi, sphi) in the
 * basis of onb(s), then normalised. */
static void cap_point(const double s[3], double c, double cphi, double sphi, double out[3])
{
    double b1[3], b2[3], v[3];
    onb(s, b1, b2);
    double st2 = 1.0 - c * c;
    double st = sqrt(st2 > 0.0 ? st2 : 0.0);
    for (int k = 0; k < 3; ++k) v[k] = c * s[k] + st * (cphi * b1[k] + sphi * b2[k]);
    normalise(v, s, out);
}

/* Exact mode: a point (v1, v2) uniform in the unit disk minus its centre,
 * from the words of attempts t = *att, *att+1, ... (v = 2 u53 - 1 per pair of
 * words); *att is advanced past the accepted attempt.  Returns 0 after 64
 * rejections (probability below 1e-40). */
static int disk_point(uint64_t seed, uint32_t site, uint32_t g, uint32_t rep, uint32_t *att,
                      double *v1, double *v2, double *s)
{
    for (int tries = 0; tries < 64; ++tries) {
        uint32_t w[4];
        words(seed, site, g, rep, (*att)++, w);
        double a = 2.0 * or_u53(w[0], w[1]) - 1.0;
        double b = 2.0 * or_u53(w[2], w[3]) - 1.0;
        double q = a * a + b * b;
        if (q < 1.0 && q > 0.0) {
            *v1 = a;
            *v2 = b;
            *s = q;
            return 1;
        }
    }
    return 0;
}

/* Trial of one site.
 *   Exact mode (double precision, correctly rounded operations and or_log):
 *     acceptance uniform u53(w0, w1) of attempt 0 for every policy;
 *     random: Marsaglia from attempts 1..32 (or_sphere_exact);
 *     flip: -s;
 *     small step: c = 1 - u53(attempt 1: w0, w1) (1 - cos theta); azimuth
 *       from the first disk point of attempts 2.., (v1, v2)/sqrt(s);
 *     Gaussian (and adaptive): three normals by the polar method (Marsaglia
 *       and Bray 1964) from disk points of attempts 1..: f = sqrt(-2 ln s / s),
 *       (v1 f, v2 f) from the first point, v1 f from the second;
 *     Hinzke-Nowak: part k = (3 w3) >> 32 of attempt 0 picks random (0), flip
 *       (1) or small step (2).
 *   Single-precision map (evaluated here in double; u_k = u24 of word k):
 *     random: z = 2 u0 - 1, phi = u1 turns, acceptance u2 (attempt 0);
 *     flip: acceptance u2;
 *     small step: c = 1 - u0 (1 - cos theta), phi = u1 turns, acceptance u2;
 *     Gaussian: r0 = sqrt(-2 ln u0), r1 = sqrt(-2 ln u2), normals
 *       (r0 cos 2pi u1, r0 sin 2pi u1, r1 cos 2pi u3); acceptance u24(w0) of
 *       attempt 1;
 *     Hinzke-Nowak: part from w3 as above, then random or small step on
 *       (u0, u1), acceptance u2.
 *   Small step, Gaussian and adaptive trials are normalised. */
double or_trial(int32_t proposal, int32_t policy, uint64_t seed, uint32_t site, uint32_t g,
                uint32_t rep, const double s[3], double param, double cos_theta, double out[3])
{
    uint32_t w[4];
    words(seed, site, g, rep, 0, w);
    int pol = policy;
    if (pol == OR_POLICY_HN) {
        uint32_t part = (uint32_t)(((uint64_t)w[3] * 3u) >> 32);
        pol = part == 0 ? OR_POLICY_RANDOM : (part == 1 ? OR_POLICY_FLIP : OR_POLICY_SMALL_STEP);
    }
    if (proposal == OR_PROPOSAL_EXACT) {
        double u = or_u53(w[0], w[1]);
        if (pol == OR_POLICY_RANDOM) {
            or_sphere_exact(seed, site, g, rep, out);
        } else if (pol == OR_POLICY_FLIP) {
            out[0] = -s[0];
            out[1] = -s[1];
            out[2] = -s[2];
        } else if (pol == OR_POLICY_SMALL_STEP) {
            uint32_t w1[4];
            words(seed, site, g, rep, 1, w1);
            double c = 1.0 - or_u53(w1[0], w1[1]) * (1.0 - cos_theta);
            uint32_t att = 2;
            double v1, v2, q, cphi = 1.0, sphi = 0.0;
            if (disk_point(seed, site, g, rep, &att, &v1, &v2, &q)) {
                double r = sqrt(q);
                cphi = v1 / r;
                sphi = v2 / r;
            }
            cap_point(s, c, cphi, sphi, out);
        } else {   /* Gaussian, adaptive */
            double n3[3] = {0.0, 0.0, 0.0};
            uint32_t att = 1;
            double v1, v2, q;
            if (disk_point(seed, site, g, rep, &att, &v1, &v2, &q)) {
                double f = sqrt(-2.0 * or_log(q) / q);
                n3[0] = v1 * f;
                n3[1] = v2 * f;
                if (disk_point(seed, site, g, rep, &att, &v1, &v2, &q)) {
                    double f2 = sqrt(-2.0 * or_log(q) / q);
                    n3[2] = v1 * f2;
                }
            }
            double v[3];
            for (int k = 0; k < 3; ++k) v[k] = s[k] + param * n3[k];
            normalise(v, s, out);
        }
        return u;
    }
    double u0 = or_u24(w[0]), u1 = or_u24(w[1]), u2 = or_u24(w[2]), u3 = or_u24(w[3]);
    if (pol == OR_POLICY_RANDOM) {
        double z = 2.0 * u0 - 1.0;
        double r2 = 1.0 - z * z;
        double r = sqrt(r2 > 0.0 ? r2 : 0.0);
        out[0] = r * cos(OR_TWO_PI * u1);
        out[1] = r * sin(OR_TWO_PI * u1);
        out[2] = z;
        return u2;
    }
    if (pol == OR_POLICY_FLIP) {
        out[0] = -s[0];
        out[1] = -s[1];
        out[2] = -s[2];
        return u2;
    }
    if (pol == OR_POLICY_SMALL_STEP) {
        double c = 1.0 - u0 * (1.0 - cos_theta);
        cap_point(s, c, cos(OR_TWO_PI * u1), sin(OR_TWO_PI * u1), out);
        return u2;
    }
    double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
    double n3[3] = {r0 * cos(OR_TWO_PI * u1), r0 * sin(OR_TWO_PI * u1), r1 * cos(OR_TWO_PI * u3)};
    double v[3];
    for (int k = 0; k < 3; ++k) v[k] = s[k] + param * n3[k];
    normalise(v, s, out);
    uint32_t wa[4];
    words(seed, site, g, rep, 1, wa);
    return or_u24(wa[0]);
}

/* ---------------------------------------------------------------------- */
static double dot3(const double *a, const double *b)
{
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

static const double ZHAT[3] = {0.0, 0.0, 1.0};

static const double *axis_of(const or_lattice *lat, int64_t i)
{
    return lat->axis ? lat->axis + 3 * i : ZHAT;
}
static const double *ndir_of(const or_lattice *lat, int64_t i)
{
    return lat->ndir ? lat->ndir + 3 * i : ZHAT;
}
static double k_of(const or_lattice *lat, int64_t i)
{
    return lat->k ? lat->k[i] : 0.0;
}
static double kc_of(const or_lattice *lat, int64_t i)
{
    return lat->kc ? lat->kc[i] : 0.0;
}
static double norm_of(const or_lattice *lat, int64_t i)
{
    return lat->norm ? lat->norm[i] : 1.0;
}

/* Cubic anisotropy function of Eq. 3: Sx^2 Sy^2 + Sy^2 Sz^2 + Sx^2 Sz^2. */
static double cubic_f(const double *s)
{
    double a = s[0] * s[0], b = s[1] * s[1], c = s[2] * s[2];
    return (a * b + b * c) + a * c;
}

int or_validate(const or_lattice *lat)
{
    if (!lat || lat->n < 0 || !lat->row_ptr) return -1;
    int64_t n = lat->n;
    if (lat->row_ptr[0] != 0) return -2;
    for (int64_t i = 0; i < n; ++i)
        if (lat->row_ptr[i + 1] < lat->row_ptr[i]) return -2;
    int64_t nnz = lat->row_ptr[n];
    if (nnz > 0 && (!lat->col || !lat->J)) return -1;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = lat->row_ptr[i]; p < lat->row_ptr[i + 1]; ++p) {
            int64_t j = lat->col[p];
            if (j < 0 || j >= n || j == i) return -2;
            if (!isfinite(lat->J[p])) return -3;
            for (int64_t q = lat->row_ptr[i]; q < p; ++q)
                if (lat->col[q] == lat->col[p]) return -2;       /* duplicate link */
            int found = 0;                                        /* reverse entry with equal J */
            for (int64_t q = lat->row_ptr[j]; q < lat->row_ptr[j + 1]; ++q)
                if (lat->col[q] == i) { found = (lat->J[q] == lat->J[p]) ? 1 : -1; break; }
            if (found == 0) return -2;
            if (found < 0) return -3;
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(k_of(lat, i)) || !isfinite(kc_of(lat, i))) return -3;
        if (!(norm_of(lat, i) > 0.0) || !isfinite(norm_of(lat, i))) return -3;
        const double *e = axis_of(lat, i), *m = ndir_of(lat, i);
        if (!(fabs(sqrt(dot3(e, e)) - 1.0) <= 1e-9)) return -3;
        if (!(fabs(sqrt(dot3(m, m)) - 1.0) <= 1e-9)) return -3;
    }
    return 0;
}

/* Greedy colouring in breadth-first order: components are taken in ascending
 * order of their lowest site index, each is searched breadth-first from that
 * site with neighbours queued in CSR order, and every site receives the
 * smallest colour not carried by an already coloured neighbour.  On a
 * connected bipartite graph this yields the two sides of the bipartition. */
int or_greedy_colour(const or_lattice *lat, int32_t *colour)
{
    int64_t n = lat->n;
    int64_t maxdeg = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t d = lat->row_ptr[i + 1] - lat->row_ptr[i];
        if (d > maxdeg) maxdeg = d;
    }
    int64_t *seen = (int64_t *)malloc(sizeof(int64_t) * (size_t)(maxdeg + 2));
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t c = 0; c < maxdeg + 2; ++c) seen[c] = -1;
    for (int64_t i = 0; i < n; ++i) colour[i] = -1;
    int32_t ncol = 0;
    int64_t head = 0, tail = 0;
    for (int64_t root = 0; root < n; ++root) {
        if (colour[root] >= 0) continue;
        colour[root] = -2;                       /* queued */
        queue[tail++] = root;
        while (head < tail) {
            int64_t i = queue[head++];
            for (int64_t p = lat->row_ptr[i]; p < lat->row_ptr[i + 1]; ++p) {
                int64_t j = lat->col[p];
                if (colour[j] >= 0) seen[colour[j]] = i;
                else if (colour[j] == -1) { colour[j] = -2; queue[tail++] = j; }
            }
            int32_t c = 0;
            while (seen[c] == i) ++c;
            colour[i] = c;
            if (c + 1 > ncol) ncol = c + 1;
        }
    }
    free(queue);
    free(seen);
    return ncol;
}

int64_t or_count_conflicts(const or_lattice *lat, const int32_t *colour)
{
    int64_t bad = 0;
    for (int64_t i = 0; i < lat->n; ++i)
        for (int64_t p = lat->row_ptr[i]; p < lat->row_ptr[i + 1]; ++p)
            if (lat->col[p] > i && colour[lat->col[p]] == colour[i]) ++bad;
    return bad;
}

/* Eq. 1 with each unordered bond once (taken at its lower-indexed end). */
double or_energy(const or_lattice *lat, double B, const double *S,
                 double *e_ex, double *e_zee, double *e_ani, double *scale)
{
    double ex = 0.0, zsum = 0.0, an = 0.0, sc = 0.0, zabs = 0.0;
    for (int64_t i = 0; i < lat->n; ++i) {
        const double *si = S + 3 * i;
        for (int64_t p = lat->row_ptr[i]; p < lat->row_ptr[i + 1]; ++p) {
            int64_t j = lat->col[p];
            if (j > i) {
                double t = lat->J[p] * dot3(si, S + 3 * j);
                ex = ex - t;
                sc = sc + fabs(t);
            }
        }
        double zn = dot3(si, ndir_of(lat, i));
        zsum = zsum + zn;
        zabs = zabs + fabs(zn);
        double a = dot3(si, axis_of(lat, i));
        double ta = k_of(lat, i) * (a * a);
        an = an - ta;
        sc = sc + fabs(ta);
        if (lat->kc) {
            double tc = lat->kc[i] * cubic_f(si);
            an = an - tc;
            sc = sc + fabs(tc);
        }
    }
    double zee = -(B * zsum);
    sc = sc + fabs(B) * zabs;
    if (e_ex) *e_ex = ex;
    if (e_zee) *e_zee = zee;
    if (e_ani) *e_ani = an;
    if (scale) *scale = sc;
    return (ex + zee) + an;
}

int64_t or_bonds(const or_lattice *lat, int32_t *bond_ij, double *J_bond)
{
    int64_t b = 0;
    for (int64_t i = 0; i < lat->n; ++i)
        for (int64_t p = lat->row_ptr[i]; p < lat->row_ptr[i + 1]; ++p)
            if (lat->col[p] > i) {
                if (bond_ij) { bond_ij[2 * b] = (int32_t)i; bond_ij[2 * b + 1] = lat->col[p]; }
                if (J_bond) J_bond[b] = lat->J[p];
                ++b;
            }
    return b;
}

/* Derivatives of E = -sum_b J_b S_i.S_j - B sum_i S_i.n_i - sum_i k_i (S_i.e_i)^2:
 *   dE/dS_i = -sum_j J_ij S_j - B n_i - 2 k_i (S_i.e_i) e_i
 *   dE/dJ_b = -S_i.S_j,  dE/dk_i = -(S_i.e_i)^2,  dE/dB = -sum_i S_i.n_i
 * each scaled by g and added to the outputs. */
void or_energy_grad(const or_lattice *lat, double B, const double *S, double g,
                    double *gS, double *gJ_bond, double *gk, double *gB)
{
    int64_t b = 0;
    double zsum = 0.0;
    for (int64_t i = 0; i < lat->n; ++i) {
        const double *si = S + 3 * i;
        double h[3] = {0.0, 0.0, 0.0};
        for (int64_t p = lat->row_ptr[i]; p < lat->row_ptr[i + 1]; ++p) {
            const double *sj = S + 3 * lat->col[p];
            h[0] = h[0] + lat->J[p] * sj[0];
            h[1] = h[1] + lat->J[p] * sj[1];
            h[2] = h[2] + lat->J[p] * sj[2];
            if (lat->col[p] > i) {
                if (gJ_bond) gJ_bond[b] += g * -dot3(si, sj);
                ++b;
            }
        }
        const double *e = axis_of(lat, i), *m = ndir_of(lat, i);
        double a = dot3(si, e);
        double ki = k_of(lat, i);
        if (gS) {
            for (int c = 0; c < 3; ++c)
                gS[3 * i + c] += g * (-h[c] - B * m[c] - 2.0 * ki * a * e[c]);
            if (lat->kc) {
                /* d/dS of -kc (Sx^2 Sy^2 + Sy^2 Sz^2 + Sx^2 Sz^2) */
                double x2 = si[0] * si[0], y2 = si[1] * si[1], z2 = si[2] * si[2];
                double kci = lat->kc[i];
                gS[3 * i + 0] += g * (-2.0 * kci * si[0] * (y2 + z2));
                gS[3 * i + 1] += g * (-2.0 * kci * si[1] * (x2 + z2));
                gS[3 * i + 2] += g * (-2.0 * kci * si[2] * (x2 + y2));
            }
        }
        if (gk) gk[i] += g * -(a * a);
        zsum = zsum + dot3(si, m);
    }
    if (gB) *gB += g * -zsum;
}

/* ---------------------------------------------------------------------- */
typedef struct { int32_t colour; int64_t rank; int64_t site; } visit_t;

static int visit_cmp(const void *a, const void *b)
{
    const visit_t *x = (const visit_t *)a, *y = (const visit_t *)b;
    if (x->colour != y->colour) return x->colour < y->colour ? -1 : 1;
    if (x->rank != y->rank) return x->rank < y->rank ? -1 : 1;
    return 0;
}

int or_run(const or_lattice *lat, const or_params *p, or_outputs *out)
{
    int rc = or_validate(lat);
    if (rc) return rc;
    if (!p || !out || !out->spins || !out->history || p->n_steps < 0 || p->mcs_per_step < 0 ||
        p->recompute_every < 0 || (p->n_steps > 0 && (!p->T || !p->B)))
        return -1;
    int64_t n = lat->n;
    int64_t M = p->mcs_per_step;
    /* g = step * M + m must stay below 0xFFFFFFFF, which the random start uses */
    if (((int64_t)p->first_step + p->n_steps) * M >= (int64_t)0xFFFFFFFF || p->first_step < 0)
        return -1;
    for (int32_t s = 0; s < p->n_steps; ++s)
        if (!(p->T[s] >= 0.0) || !isfinite(p->B[s])) return -3;
    /* update policies per site type */
    int has_adaptive = 0;
    double cos_t[OR_MAX_TYPES];
    if (p->n_types < 0 || p->n_types > OR_MAX_TYPES) return -1;
    if (p->n_types > 0) {
        if (!p->type_policy || !p->type_param) return -1;
        for (int32_t t = 0; t < p->n_types; ++t) {
            int32_t pol = p->type_policy[t];
            double prm = p->type_param[t];
            if (pol < OR_POLICY_RANDOM || pol > OR_POLICY_ADAPTIVE) return -1;
            if ((pol == OR_POLICY_SMALL_STEP || pol == OR_POLICY_HN) &&
                !(prm > 0.0 && prm <= 3.14159265358979323846))
                return -3;
            if ((pol == OR_POLICY_GAUSSIAN || pol == OR_POLICY_ADAPTIVE) && !(prm > 0.0 && isfinite(prm)))
                return -3;
            cos_t[t] = cos(prm);
            if (pol == OR_POLICY_ADAPTIVE) has_adaptive = 1;
        }
        if (p->site_type)
            for (int64_t i = 0; i < lat->n; ++i)
                if (p->site_type[i] < 0 || p->site_type[i] >= p->n_types) return -1;
        if (has_adaptive && (!p->sigma || !(*p->sigma > 0.0) || !isfinite(*p->sigma) ||
                             !(p->sigma_min > 0.0) || !(p->sigma_max >= p->sigma_min) ||
                             !isfinite(p->sigma_max)))
            return -3;
    }

    int32_t *colour = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    if (p->colour) {
        memcpy(colour, p->colour, sizeof(int32_t) * (size_t)n);
        if (or_count_conflicts(lat, colour) != 0) { free(colour); return -2; }
    } else {
        or_greedy_colour(lat, colour);
    }
    /* sweep order: colour classes ascending; inside a class ascending site
     * index, or the order given by p->order */
    visit_t *vis = (visit_t *)malloc(sizeof(visit_t) * (size_t)(n + 1));
    for (int64_t i = 0; i < n; ++i) { vis[i].colour = colour[i]; vis[i].rank = i; vis[i].site = i; }
    if (p->order)
        for (int64_t t = 0; t < n; ++t) vis[p->order[t]].rank = t;
    qsort(vis, (size_t)n, sizeof(visit_t), visit_cmp);

    double *S = out->spins;
    if (p->init == OR_INIT_COLD_Z) {
        for (int64_t i = 0; i < n; ++i) { S[3 * i] = 0.0; S[3 * i + 1] = 0.0; S[3 * i + 2] = norm_of(lat, i); }
    } else if (p->init == OR_INIT_RANDOM) {
        for (int64_t i = 0; i < n; ++i) {
            or_sphere_exact(p->seed, (uint32_t)i, 0xFFFFFFFFu, p->replica, S + 3 * i);
            if (lat->norm)
                for (int c = 0; c < 3; ++c) S[3 * i + c] = lat->norm[i] * S[3 * i + c];
        }
    }

    out->near_ties = 0;
    out->max_incr_err = 0.0;
    out->max_update_err = 0.0;
    out->n_decisions = 0;

    for (int32_t s = 0; s < p->n_steps; ++s) {
        double T = p->T[s];
        double beta = (T > 0.0) ? 1.0 / T : INFINITY;
        double b = p->B[s];
        double E = 0.0;
        for (int64_t m = 0; m < M; ++m) {
            if (m == 0 || (p->recompute_every > 0 && m % p->recompute_every == 0))
                E = or_energy(lat, b, S, NULL, NULL, NULL, NULL);
            uint32_t g = (uint32_t)(((int64_t)p->first_step + s) * M + m);
            int64_t rec = (int64_t)s * M + m;
            double dEsum = 0.0;
            int64_t nacc = 0;
            int64_t n_ad = 0, acc_ad = 0;     /* adaptive-policy sites: attempts, accepts */
            double sigma = has_adaptive ? *p->sigma : 0.0;
            if (p->sigma_trace) p->sigma_trace[rec] = sigma;
            for (int64_t t = 0; t < n; ++t) {
                int64_t i = vis[t].site;
                double *si = S + 3 * i;
                double hx = 0.0, hy = 0.0, hz = 0.0;
                for (int64_t q = lat->row_ptr[i]; q < lat->row_ptr[i + 1]; ++q) {
                    const double *sj = S + 3 * lat->col[q];
                    double Jq = lat->J[q];
                    hx = hx + Jq * sj[0];
                    hy = hy + Jq * sj[1];
                    hz = hz + Jq * sj[2];
                }
                const double *nd = ndir_of(lat, i);
                hx = hx + b * nd[0];
                hy = hy + b * nd[1];
                hz = hz + b * nd[2];

                double sn[3], u;
                int32_t ty = (p->n_types > 0 && p->site_type) ? p->site_type[i] : 0;
                int32_t pol = p->n_types > 0 ? p->type_policy[ty] : OR_POLICY_RANDOM;
                /* trial moves act on the direction; the trial gets the norm back */
                const double mu = norm_of(lat, i);
                double dir[3] = {si[0], si[1], si[2]};
                if (lat->norm)
                    for (int c = 0; c < 3; ++c) dir[c] = si[c] / mu;
                if (pol != OR_POLICY_RANDOM) {
                    double prm = pol == OR_POLICY_ADAPTIVE ? sigma : p->type_param[ty];
                    u = or_trial(p->proposal, pol, p->seed, (uint32_t)i, g, p->replica, dir, prm,
                                 cos_t[ty], sn);
                } else if (p->proposal == OR_PROPOSAL_EXACT) {
                    uint32_t w[4];
                    words(p->seed, (uint32_t)i, g, p->replica, 0, w);
                    u = or_u53(w[0], w[1]);
                    or_sphere_exact(p->seed, (uint32_t)i, g, p->replica, sn);
                } else {
                    or_sphere_f32map(p->seed, (uint32_t)i, g, p->replica, sn, &u);
                }
                if (lat->norm)
                    for (int c = 0; c < 3; ++c) sn[c] = mu * sn[c];
                double dSx = sn[0] - si[0], dSy = sn[1] - si[1], dSz = sn[2] - si[2];
                double q = dSx * hx + dSy * hy + dSz * hz;
                const double *e = axis_of(lat, i);
                double a1 = dot3(sn, e);
                double a0 = dot3(si, e);
                double dE = -q - k_of(lat, i) * (a1 * a1 - a0 * a0);
                if (lat->kc) dE = dE - lat->kc[i] * (cubic_f(sn) - cubic_f(si));

                int acc;
                if (dE <= 0.0) {
                    acc = 1;
                } else {
                    double pr = exp(-beta * dE);
                    acc = u < pr;
                    double ulp = nextafter(pr, INFINITY) - pr;
                    if (fabs(u - pr) <= 4.0 * ulp) out->near_ties++;
                }
                out->n_decisions++;
                if (out->dE_trace) out->dE_trace[rec * n + i] = dE;
                if (out->u_trace) out->u_trace[rec * n + i] = u;
                if (pol == OR_POLICY_ADAPTIVE) {
                    n_ad++;
                    acc_ad += acc;
                }
                if (out->accept) out->accept[rec * n + i] = (uint8_t)acc;
                if (acc) {
                    if (p->check_every_update) {
                        double sc, e0 = or_energy(lat, b, S, NULL, NULL, NULL, &sc);
                        si[0] = sn[0]; si[1] = sn[1]; si[2] = sn[2];
                        double e1 = or_energy(lat, b, S, NULL, NULL, NULL, NULL);
                        double err = fabs(dE - (e1 - e0)) / (sc > 0.0 ? sc : 1.0);
                        if (err > out->max_update_err) out->max_update_err = err;
                    } else {
                        si[0] = sn[0]; si[1] = sn[1]; si[2] = sn[2];
                    }
                    dEsum = dEsum + dE;
                    nacc++;
                }
            }
            E = E + dEsum;
            /* adaptive width for the next MCS: scaled by 0.5 / (1 - a), a the
             * acceptance of the adaptive sites in this MCS, kept in bounds */
            if (has_adaptive && n_ad > 0) {
                double a = (double)acc_ad / (double)n_ad;
                double sg = sigma * (0.5 / (1.0 - a));
                *p->sigma = fmin(p->sigma_max, fmax(p->sigma_min, sg));
            }
            double Mx = 0.0, My = 0.0, Mz = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                Mx = Mx + S[3 * i];
                My = My + S[3 * i + 1];
                Mz = Mz + S[3 * i + 2];
            }
            double *h = out->history + 5 * rec;
            h[0] = E; h[1] = Mx; h[2] = My; h[3] = Mz; h[4] = (double)nacc;
            /* magnetisation of every site type ("the statistics of each
             * magnetic phase"), sites in index order within a type */
            if (out->type_mag) {
                int32_t nt = p->n_types > 0 ? p->n_types : 1;
                double *tm = out->type_mag + (size_t)rec * nt * 3;
                for (int32_t t = 0; t < nt; ++t) {
                    double x = 0.0, y = 0.0, z = 0.0;
                    for (int64_t i = 0; i < n; ++i) {
                        int32_t ty = (p->n_types > 0 && p->site_type) ? p->site_type[i] : 0;
                        if (ty != t) continue;
                        x = x + S[3 * i];
                        y = y + S[3 * i + 1];
                        z = z + S[3 * i + 2];
                    }
                    tm[3 * t] = x; tm[3 * t + 1] = y; tm[3 * t + 2] = z;
                }
            }
            /* final state of the step: every spin after the step's last MCS
             * (section "VEGAS software package", its list of stored results) */
            if (out->snapshots && m == M - 1)
                memcpy(out->snapshots + (size_t)s * n * 3, S, sizeof(double) * 3 * (size_t)n);
            if (out->e_full) {
                double sc, ef = or_energy(lat, b, S, NULL, NULL, NULL, &sc);
                out->e_full[rec] = ef;
                double err = fabs(E - ef) / (sc > 0.0 ? sc : 1.0);
                if (err > out->max_incr_err) out->max_incr_err = err;
            }
        }
    }
    free(vis);
    free(colour);
    return 0;
}
