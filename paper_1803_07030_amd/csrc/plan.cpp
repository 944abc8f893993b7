// Lattice ingest (host): validation, greedy breadth-first colouring,
// colour-sorted permutation, internal CSR, bond tables; and the energy /
// gradient entry points, which work on one plan.
//
// Paper: the material file of section "Material building" (sites, exchange
// links with constants, a field axis per site) and the anisotropy file of
// section "File Formats" (a constant and an axis per site) become CSR arrays
// with per-entry constants and per-site parameters.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>

#include "hsim_host.h"

using hsim::Error;

namespace {

double norm3(const double *v) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

void validate(int64_t n, const int64_t *rp, const int32_t *col, const double *J, const double *k,
              const double *axis, const double *fd)
{
    if (n < 0 || n > INT32_MAX - 64) throw Error(HSIM_E_ARG, "n_sites out of range");
    if (!rp) throw Error(HSIM_E_ARG, "row_ptr is NULL");
    if (rp[0] != 0) throw Error(HSIM_E_CSR, "row_ptr[0] != 0");
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) throw Error(HSIM_E_CSR, "row_ptr not non-decreasing");
    const int64_t nnz = rp[n];
    if (nnz > INT32_MAX) throw Error(HSIM_E_ARG, "too many CSR entries");
    if (nnz > 0 && (!col || !J)) throw Error(HSIM_E_ARG, "col or J is NULL");
    // in range, no self loop, finite constants
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (col[p] < 0 || col[p] >= n) throw Error(HSIM_E_CSR, "column index out of range");
            if (col[p] == i) throw Error(HSIM_E_CSR, "self loop");
            if (!std::isfinite(J[p])) throw Error(HSIM_E_PARAM, "non-finite exchange constant");
        }
    // no duplicate link in a row; every entry has its reverse with an equal constant
    std::vector<int64_t> mark(n, -1);
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (mark[col[p]] == i) throw Error(HSIM_E_CSR, "duplicate link");
            mark[col[p]] = i;
        }
    }
    // every entry (i -> j) has its reverse (j -> i) with an equal constant
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            const int64_t j = col[p];
            int64_t q = rp[j];
            while (q < rp[j + 1] && col[q] != i) ++q;
            if (q == rp[j + 1]) throw Error(HSIM_E_CSR, "link without its reverse entry");
            if (J[q] != J[p]) throw Error(HSIM_E_PARAM, "exchange constants not symmetric");
        }
    for (int64_t i = 0; i < n; ++i) {
        if (k && !std::isfinite(k[i])) throw Error(HSIM_E_PARAM, "non-finite anisotropy constant");
        if (axis && !(std::fabs(norm3(axis + 3 * i) - 1.0) <= 1e-9))
            throw Error(HSIM_E_PARAM, "anisotropy axis is not a unit vector");
        if (fd && !(std::fabs(norm3(fd + 3 * i) - 1.0) <= 1e-9))
            throw Error(HSIM_E_PARAM, "field direction is not a unit vector");
    }
}

// Greedy colouring in breadth-first order: components by lowest site index,
// neighbours queued in CSR order, each site takes the smallest colour not
// carried by an already coloured neighbour.
int32_t bfs_greedy(int64_t n, const int64_t *rp, const int32_t *col, std::vector<int32_t> &c,
                   int32_t &maxdeg)
{
    maxdeg = 0;
    for (int64_t i = 0; i < n; ++i) maxdeg = std::max<int32_t>(maxdeg, (int32_t)(rp[i + 1] - rp[i]));
    c.assign(n, -1);
    std::vector<int64_t> used(maxdeg + 2, -1), queue;
    queue.reserve(n);
    int32_t ncol = 0;
    size_t head = 0;
    for (int64_t root = 0; root < n; ++root) {
        if (c[root] != -1) continue;
        c[root] = -2;
        queue.push_back(root);
        while (head < queue.size()) {
            const int64_t i = queue[head++];
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                const int32_t j = col[p];
                if (c[j] >= 0) used[c[j]] = i;
                else if (c[j] == -1) {
                    c[j] = -2;
                    queue.push_back(j);
                }
            }
            int32_t k = 0;
            while (used[k] == i) ++k;
            c[i] = k;
            ncol = std::max(ncol, k + 1);
        }
    }
    return ncol;
}

}  // namespace

// Half rows for the energy forward, where each bond is needed once.  Every
// bond is given a direction by closed walks: odd-degree sites of a component
// are joined to one extra vertex (there is an even number of them), so every
// degree is even; a walk that takes unused edges from a vertex can only stop
// where it started, so along each walk every vertex is left as often as it
// is entered, and a site of degree d leaves at most ceil(d / 2) of its bonds.
// A site's row lists the bonds it leaves, in CSR order.
void half_rows(hsim_plan P, const int64_t *rp, const int32_t *col)
{
    const int64_t n = P->n;
    // adjacency: CSR entries, then one virtual edge per odd site (to vertex n)
    std::vector<int64_t> odd;
    for (int64_t i = 0; i < n; ++i)
        if ((rp[i + 1] - rp[i]) & 1) odd.push_back(i);
    const int64_t nb = P->nb, ne = nb + (int64_t)odd.size();
    std::vector<int64_t> vodd(n, -1);
    for (size_t k = 0; k < odd.size(); ++k) vodd[odd[k]] = (int64_t)k;
    // per vertex: CSR entries (target, edge) and, for odd sites, the virtual edge
    auto deg_of = [&](int64_t v) -> int64_t {
        return v == n ? (int64_t)odd.size() : (rp[v + 1] - rp[v]) + (vodd[v] >= 0 ? 1 : 0);
    };
    auto entry = [&](int64_t v, int64_t q, int64_t &to, int64_t &edge) {
        if (v == n) {
            to = odd[q];
            edge = nb + q;
        } else if (q < rp[v + 1] - rp[v]) {
            to = col[rp[v] + q];
            edge = P->ubond[rp[v] + q];
        } else {
            to = n;
            edge = nb + vodd[v];
        }
    };
    std::vector<uint8_t> used(ne, 0);
    std::vector<int64_t> next(n + 1, 0);
    std::vector<uint8_t> leaves(nb, 0);   // 1: the bond leaves its lower end
    for (int64_t s = 0; s <= n; ++s) {
        for (;;) {
            // a closed walk from s over unused edges
            int64_t v = s;
            bool moved = false;
            for (;;) {
                int64_t to = -1, edge = -1;
                const int64_t d = deg_of(v);
                while (next[v] < d) {
                    entry(v, next[v]++, to, edge);
                    if (!used[edge]) break;
                    edge = -1;
                }
                if (edge < 0) break;
                used[edge] = 1;
                if (edge < nb) leaves[edge] = v < to ? 1 : 0;
                v = to;
                moved = true;
            }
            if (!moved || v != s) break;
        }
    }
    std::vector<int32_t> outn(n, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            const int32_t b = P->ubond[p];
            if ((col[p] > i) == (leaves[b] != 0)) ++outn[i];
        }
    int32_t hw = 0;
    for (int64_t i = 0; i < n; ++i) hw = std::max(hw, outn[i]);
    if (hw > P->e_w / 2) throw Error(HSIM_E_UNSUPPORTED, "internal: bond orientation left a site unbalanced");
    P->h_w = P->e_w / 2;
    const int W = P->h_w;
    P->uhalf_col.assign((size_t)W * n, 0);
    P->uhalf_bond.assign((size_t)W * n, -1);
    for (int64_t i = 0; i < n; ++i) {
        int q = 0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            const int32_t b = P->ubond[p];
            if ((col[p] > i) != (leaves[b] != 0)) continue;
            P->uhalf_col[(size_t)q * n + i] = col[p];
            P->uhalf_bond[(size_t)q * n + i] = b;
            ++q;
        }
        for (; q < W; ++q) P->uhalf_col[(size_t)q * n + i] = (int32_t)i;
    }
}

hsim_plan plan_create_impl(int64_t n, const int64_t *rp, const int32_t *col, const double *J,
                           const double *k, const double *axis, const double *fd)
{
    validate(n, rp, col, J, k, axis, fd);
    auto *P = new hsim_plan_s();
    try {
        // FNV-1a over the lattice as given (the autotuner's cache key)
        uint64_t h = 1469598103934665603ull;
        auto mix = [&h](const void *p, size_t bytes) {
            const unsigned char *c = (const unsigned char *)p;
            for (size_t q = 0; q < bytes; ++q) {
                h ^= c[q];
                h *= 1099511628211ull;
            }
        };
        mix(&n, sizeof n);
        mix(rp, (size_t)(n + 1) * sizeof(int64_t));
        mix(col, (size_t)rp[n] * sizeof(int32_t));
        mix(J, (size_t)rp[n] * sizeof(double));
        const double none = 0.0;
        mix(k ? (const void *)k : &none, k ? (size_t)n * 8 : 8);
        mix(axis ? (const void *)axis : &none, axis ? (size_t)n * 24 : 8);
        mix(fd ? (const void *)fd : &none, fd ? (size_t)n * 24 : 8);
        P->hash = h;
        P->n = n;
        P->nnz = rp[n];
        P->nb = P->nnz / 2;
        P->ncol = bfs_greedy(n, rp, col, P->colour, P->maxdeg);
        if (P->ncol > hsim::kMaxColours)
            throw Error(HSIM_E_UNSUPPORTED, "lattice needs more than 32 colours");
        // colour-sorted order, user index inside a class
        P->perm.resize(n);
        std::iota(P->perm.begin(), P->perm.end(), 0);
        std::stable_sort(P->perm.begin(), P->perm.end(),
                         [&](int32_t a, int32_t b) { return P->colour[a] < P->colour[b]; });
        P->inv.resize(n);
        for (int64_t t = 0; t < n; ++t) P->inv[P->perm[t]] = (int32_t)t;
        P->cls_off.assign(P->ncol + 1, 0);
        for (int64_t i = 0; i < n; ++i) P->cls_off[P->colour[i] + 1]++;
        for (int c = 0; c < P->ncol; ++c) P->cls_off[c + 1] += P->cls_off[c];
        // internal CSR
        P->rp.resize(n + 1);
        P->ci.resize(P->nnz);
        P->Jd.resize(P->nnz);
        P->rp[0] = 0;
        for (int64_t t = 0; t < n; ++t) {
            const int64_t i = P->perm[t];
            int32_t q = P->rp[t];
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p, ++q) {
                P->ci[q] = P->inv[col[p]];
                P->Jd[q] = J[p];
            }
            P->rp[t + 1] = q;
        }
        P->Jf.assign(P->Jd.begin(), P->Jd.end());
        // padded rows for the fixed-width kernels
        if (P->maxdeg <= 8) {
            const int W = P->maxdeg <= 6 ? 6 : 8;
            P->ell_w = W;
            P->ell_col.assign((size_t)n * W, 0);
            P->ell_Jf.assign((size_t)n * W, 0.0f);
            P->ellT_col.assign((size_t)n * W, 0);
            P->ellT_Jf.assign((size_t)n * W, 0.0f);
            P->ellT_Jd.assign((size_t)n * W, 0.0);
            for (int64_t t = 0; t < n; ++t)
                for (int sl = 0; sl < W; ++sl) {
                    const int32_t p = P->rp[t] + sl;
                    const bool in = p < P->rp[t + 1];
                    const int32_t c = in ? P->ci[p] : (int32_t)t;
                    const double J = in ? P->Jd[p] : 0.0;
                    P->ell_col[t * W + sl] = c;
                    P->ell_Jf[t * W + sl] = (float)J;
                    P->ellT_col[(size_t)sl * n + t] = c;
                    P->ellT_Jf[(size_t)sl * n + t] = (float)J;
                    P->ellT_Jd[(size_t)sl * n + t] = J;
                }
        }
        // per-site parameters, internal order
        P->kd.resize(n);
        P->axd.resize(3 * n);
        P->ndd.resize(3 * n);
        for (int64_t t = 0; t < n; ++t) {
            const int64_t i = P->perm[t];
            P->kd[t] = k ? k[i] : 0.0;
            for (int c = 0; c < 3; ++c) {
                P->axd[c * n + t] = axis ? axis[3 * i + c] : (c == 2 ? 1.0 : 0.0);
                P->ndd[c * n + t] = fd ? fd[3 * i + c] : (c == 2 ? 1.0 : 0.0);
            }
        }
        P->kf.assign(P->kd.begin(), P->kd.end());
        P->axf.assign(P->axd.begin(), P->axd.end());
        P->ndf.assign(P->ndd.begin(), P->ndd.end());
        bool kzero = true, kuni = true, nuni = true;
        for (int64_t t = 0; t < n; ++t) {
            if (P->kd[t] != 0.0) kzero = false;
            if (P->kd[t] != P->kd[0]) kuni = false;
            for (int c = 0; c < 3; ++c) {
                if (P->axd[c * n + t] != P->axd[c * n]) kuni = false;
                if (P->ndd[c * n + t] != P->ndd[c * n]) nuni = false;
            }
        }
        P->kmode = kzero ? hsim::K_NONE : (kuni ? hsim::K_UNIFORM : hsim::K_SITE);
        P->fmode = nuni ? hsim::F_UNIFORM : hsim::F_SITE;
        if (n > 0) {
            P->k0 = P->kd[0];
            for (int c = 0; c < 3; ++c) {
                P->e0[c] = P->kmode == hsim::K_NONE ? (c == 2 ? 1.0 : 0.0) : P->axd[c * n];
                P->n0[c] = P->ndd[c * n];
            }
        }
        // user-order CSR with bond ids (bond b = b-th entry with col > row)
        P->urp.assign(rp, rp + n + 1);
        P->uci.assign(col, col + P->nnz);
        P->ubond.assign(P->nnz, -1);
        P->fwd_entry.clear();
        P->bond_ij.clear();
        for (int64_t i = 0; i < n; ++i)
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
                if (col[p] > i) {
                    P->ubond[p] = (int32_t)P->fwd_entry.size();
                    P->fwd_entry.push_back((int32_t)p);
                    P->bond_ij.push_back((int32_t)i);
                    P->bond_ij.push_back(col[p]);
                }
        // the reverse entry of a bond gets the same id
        for (int64_t i = 0; i < n; ++i)
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                const int64_t j = col[p];
                if (j >= i) continue;
                int64_t q = rp[j];
                while (col[q] != i) ++q;   // exists: validated above
                P->ubond[p] = P->ubond[q];
            }
        P->nb = (int64_t)P->fwd_entry.size();
        // padded rows for the energy calls (slot-major; padding: the site
        // itself with bond id -1, i.e. constant 0)
        int64_t md = 0;
        for (int64_t i = 0; i < n; ++i) md = std::max<int64_t>(md, rp[i + 1] - rp[i]);
        P->e_w = md <= 6 ? 6 : (md <= 8 ? 8 : 0);
        if (P->e_w > 0 && n > 0) {
            const int W = P->e_w;
            P->uell_col.assign((size_t)W * n, 0);
            P->uell_bond.assign((size_t)W * n, -1);
            for (int64_t i = 0; i < n; ++i)
                for (int q = 0; q < W; ++q) {
                    const int64_t p = rp[i] + q;
                    const bool in = p < rp[i + 1];
                    P->uell_col[(size_t)q * n + i] = in ? col[p] : (int32_t)i;
                    P->uell_bond[(size_t)q * n + i] = in ? P->ubond[p] : -1;
                }
            half_rows(P, rp, col);
        }
    } catch (...) {
        delete P;
        throw;
    }
    return P;
}

void hsim_plan_s::upload_sweep()
{
    if (sweep_on_device) return;
    std::vector<uint32_t> orig(perm.begin(), perm.end());
    d_rp.upload(rp);
    d_ci.upload(ci);
    d_Jf.upload(Jf);
    d_Jd.upload(Jd);
    d_orig.upload(orig);
    d_kf.upload(kf);
    d_kd.upload(kd);
    d_axf.upload(axf);
    d_axd.upload(axd);
    d_ndf.upload(ndf);
    d_ndd.upload(ndd);
    if (ell_w > 0) {
        d_ell_col.upload(ell_col);
        d_ell_J.upload(ell_Jf);
        d_ellT_col.upload(ellT_col);
        d_ellT_Jf.upload(ellT_Jf);
        d_ellT_Jd.upload(ellT_Jd);
    }
    if (!type.empty()) d_type.upload(type);
    sweep_on_device = true;
    upload_terms();
}

// Device copies of the cubic constants and spin norms (idempotent).
void hsim_plan_s::upload_terms()
{
    if (!kcd.empty() && !d_kcd.p) {
        d_kcd.upload(kcd);
        d_kcf.upload(kcf);
        d_ukcd.upload(ukcd);
        d_ukcf.upload(ukcf);
    }
    if (!mud.empty() && !d_mud.p) {
        d_mud.upload(mud);
        d_muf.upload(muf);
    }
}

// Cubic constants (Eq. 3) and spin norms, user order; NULL, all-zero
// constants or all-unit norms mean none.
void plan_set_site_terms_impl(hsim_plan P, const double *k_cubic, const double *spin_norm)
{
    if (!P) throw Error(HSIM_E_ARG, "set_site_terms: NULL plan");
    const int64_t n = P->n;
    bool any_kc = false, any_mu = false;
    for (int64_t u = 0; u < n; ++u) {
        if (k_cubic) {
            if (!std::isfinite(k_cubic[u])) throw Error(HSIM_E_PARAM, "non-finite cubic constant");
            any_kc |= k_cubic[u] != 0.0;
        }
        if (spin_norm) {
            if (!(spin_norm[u] > 0.0) || !std::isfinite(spin_norm[u]))
                throw Error(HSIM_E_PARAM, "spin norms must be positive and finite");
            any_mu |= spin_norm[u] != 1.0;
        }
    }
    P->kcd.clear(); P->kcf.clear(); P->ukcd.clear(); P->ukcf.clear();
    P->mud.clear(); P->muf.clear();
    P->d_kcd.release(); P->d_kcf.release(); P->d_ukcd.release(); P->d_ukcf.release();
    P->d_mud.release(); P->d_muf.release();
    if (any_kc) {
        P->ukcd.assign(k_cubic, k_cubic + n);
        P->ukcf.resize(n);
        P->kcd.resize(n);
        P->kcf.resize(n);
        for (int64_t u = 0; u < n; ++u) P->ukcf[u] = (float)k_cubic[u];
        for (int64_t k = 0; k < n; ++k) {
            P->kcd[k] = k_cubic[P->perm[k]];
            P->kcf[k] = (float)P->kcd[k];
        }
    }
    if (any_mu) {
        P->mud.resize(n);
        P->muf.resize(n);
        for (int64_t k = 0; k < n; ++k) {
            P->mud[k] = spin_norm[P->perm[k]];
            P->muf[k] = (float)P->mud[k];
        }
    }
    if (P->sweep_on_device || P->energy_ready) P->upload_terms();
}

// Site types (user order, values 0 .. kMaxTypes-1) kept in internal order;
// NULL clears them.
void plan_set_types_impl(hsim_plan P, const int32_t *user_type)
{
    if (!P) throw Error(HSIM_E_ARG, "set_types: NULL plan");
    if (!user_type) {
        P->type.clear();
        P->d_type.release();
        return;
    }
    std::vector<int32_t> t(P->n);
    for (int64_t k = 0; k < P->n; ++k) {
        const int32_t v = user_type[P->perm[k]];
        if (v < 0 || v >= hsim::kMaxTypes) throw Error(HSIM_E_PARAM, "site type outside 0..7");
        t[k] = v;
    }
    P->type.swap(t);
    if (P->sweep_on_device) P->d_type.upload(P->type);
}

void hsim_plan_s::upload_energy()
{
    if (energy_on_device) return;
    d_urp.upload(urp);
    d_uci.upload(uci);
    d_ubond.upload(ubond);
    d_fwd.upload(fwd_entry);
    if (e_w > 0) {
        d_uell_col.upload(uell_col);
        d_uell_bond.upload(uell_bond);
        d_uhalf_col.upload(uhalf_col);
        d_uhalf_bond.upload(uhalf_bond);
    }
    energy_on_device = true;
}

// Energy tables on the device and the fixed scratch: at most about
// kEnergyScratchDoubles, at least one group of configurations per pass.
constexpr int64_t kEnergyScratchDoubles = (int64_t)16 << 20;   // 128 MiB
void hsim_plan_s::prepare_energy()
{
    if (energy_ready) return;
    upload_energy();
    upload_terms();
    elayout = hsim::energy_layout(n, nb, e_w, kEnergyScratchDoubles, false, 1);
    d_escratch.alloc((size_t)elayout.doubles * sizeof(double));
    energy_ready = true;
}

// ----------------------------------------------------------------- energy
namespace {

hsim::EnergyArgs energy_args(hsim_plan P, int32_t batch, const void *S, const void *Jb,
                             const void *k, const void *ax, double B, const void *nd, bool f64)
{
    hsim::EnergyArgs a{};
    a.rp = (const int64_t *)P->d_urp.p;
    a.ci = (const int32_t *)P->d_uci.p;
    a.bond = (const int32_t *)P->d_ubond.p;
    a.fwd_entry = (const int32_t *)P->d_fwd.p;
    a.ecol = (const int32_t *)P->d_uell_col.p;
    a.ebond = (const int32_t *)P->d_uell_bond.p;
    a.hcol = (const int32_t *)P->d_uhalf_col.p;
    a.hbond = (const int32_t *)P->d_uhalf_bond.p;
    a.n = P->n;
    a.nnz = P->nnz;
    a.nb = P->nb;
    a.batch = batch;
    a.S = S;
    // the padded-row kernels read Jb[0] for empty slots (and discard it);
    // without bonds the caller may pass no array, so point them at a table
    // of the plan that holds at least one element
    a.Jb = P->nb > 0 ? Jb : P->d_uell_bond.p;
    a.k = k;
    a.ax = ax;
    a.nd = nd;
    a.kc = P->ukcd.empty() ? nullptr : (f64 ? P->d_ukcd.p : P->d_ukcf.p);
    a.B = B;
    return a;
}

}  // namespace

void energy_forward_impl(hsim_plan P, int32_t batch, hsim_precision prec, const void *S,
                         const void *Jb, const void *k, const void *ax, double B, const void *nd,
                         double *E, hipStream_t st)
{
    if (!P || batch < 0 || !E || (P->n > 0 && batch > 0 && !S) || (P->nb > 0 && !Jb))
        throw Error(HSIM_E_ARG, "energy_forward: bad argument");
    if (prec != HSIM_FP32 && prec != HSIM_FP64_EXACT) throw Error(HSIM_E_ARG, "bad precision");
    if (!std::isfinite(B)) throw Error(HSIM_E_PARAM, "non-finite field");
    if (batch == 0) return;
    if (P->n == 0) {   // no sites: every energy is 0
        // a fill kernel, not a memset: callers may capture these calls in graphs
        hsim::hip_check(hsim::launch_fill_u32(st, (uint32_t *)E, 0u, (int64_t)batch * 2), "fill launch");
        return;
    }
    P->prepare_energy();
    const hsim::EnergyArgs a = energy_args(P, batch, S, Jb, k, ax, B, nd, prec == HSIM_FP64_EXACT);
    hsim::hip_check(hsim::launch_energy_forward(st, prec == HSIM_FP64_EXACT, a, P->elayout,
                                                (double *)P->d_escratch.p, E),
                    "energy forward launch");
}

void energy_backward_impl(hsim_plan P, int32_t batch, hsim_precision prec, const void *S,
                          const void *Jb, const void *k, const void *ax, double B,
                          const void *nd, const double *gE, void *gS, void *gJ, void *gk,
                          double *gB, hipStream_t st)
{
    if (!P || batch < 0 || (batch > 0 && !gE) || (P->n > 0 && batch > 0 && !S) ||
        (P->nb > 0 && !Jb))
        throw Error(HSIM_E_ARG, "energy_backward: bad argument");
    if (prec != HSIM_FP32 && prec != HSIM_FP64_EXACT) throw Error(HSIM_E_ARG, "bad precision");
    if (!std::isfinite(B)) throw Error(HSIM_E_PARAM, "non-finite field");
    if (batch == 0) return;
    if (P->n == 0) {   // no sites, no bonds: the field gradient is 0, the rest empty
        if (gB) hsim::hip_check(hsim::launch_fill_u32(st, (uint32_t *)gB, 0u, 2), "fill launch");
        return;
    }
    P->prepare_energy();
    const hsim::EnergyArgs a = energy_args(P, batch, S, Jb, k, ax, B, nd, prec == HSIM_FP64_EXACT);
    hsim::hip_check(hsim::launch_energy_backward(st, prec == HSIM_FP64_EXACT, a, gE, gS, gJ, gk, gB,
                                                 P->elayout, (double *)P->d_escratch.p),
                    "energy backward launch");
}

void energy_prepare_impl(hsim_plan P)
{
    if (!P) throw Error(HSIM_E_ARG, "energy_prepare: NULL plan");
    if (P->n > 0) P->prepare_energy();
}

// Forward with its partial records in the library's fixed device array: no
// allocation.  The plan's energy tables must already be on the device.
void energy_forward_noalloc_impl(hsim_plan P, int32_t batch, hsim_precision prec, const void *S,
                                 const void *Jb, const void *k, const void *ax, double B,
                                 const void *nd, double *E, hipStream_t st)
{
    if (!P || batch < 0 || !E || (P->n > 0 && batch > 0 && !S) || (P->nb > 0 && !Jb))
        throw Error(HSIM_E_ARG, "energy_forward_noalloc: bad argument");
    if (prec != HSIM_FP32 && prec != HSIM_FP64_EXACT) throw Error(HSIM_E_ARG, "bad precision");
    if (!std::isfinite(B)) throw Error(HSIM_E_PARAM, "non-finite field");
    const hsim::EnergyLayout L =
        hsim::energy_layout(P->n, P->nb, P->e_w, hsim::kStaticEnergyScratchDoubles, true, 0);
    if (P->n > 0 && L.groups < 1)
        throw Error(HSIM_E_ARG, "energy_forward_noalloc: the lattice is too large for the fixed "
                                "scratch (at most " +
                                    std::to_string(hsim::kStaticEnergyScratchDoubles / 32 * 256) +
                                    " sites)");
    if (batch == 0) return;
    if (P->n == 0) {
        hsim::hip_check(hsim::launch_fill_u32(st, (uint32_t *)E, 0u, (int64_t)batch * 2), "fill launch");
        return;
    }
    if (!P->energy_ready)
        throw Error(HSIM_E_STATE, "energy_forward_noalloc: call hsim_energy_prepare on the plan first");
    double *scr = nullptr;
    hsim::hip_check(hsim::static_energy_scratch(&scr), "hipGetSymbolAddress");
    const hsim::EnergyArgs a = energy_args(P, batch, S, Jb, k, ax, B, nd, prec == HSIM_FP64_EXACT);
    hsim::hip_check(hsim::launch_energy_forward(st, prec == HSIM_FP64_EXACT, a, L, scr, E),
                    "energy forward launch");
}
