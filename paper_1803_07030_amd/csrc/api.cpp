// extern "C" entry points of libhsim.so (declared in include/hsim.h).  Each
// one validates its arguments, runs the C++ implementation and turns any
// error into an hsim_status plus a thread-local message: no exception leaves
// the library.
#include <cstring>
#include <string>

#include "hsim_host.h"

hsim_plan plan_create_impl(int64_t, const int64_t *, const int32_t *, const double *,
                           const double *, const double *, const double *);
void energy_prepare_impl(hsim_plan);
void energy_forward_noalloc_impl(hsim_plan, int32_t, hsim_precision, const void *, const void *,
                                 const void *, const void *, double, const void *, double *,
                                 hipStream_t);
void energy_forward_impl(hsim_plan, int32_t, hsim_precision, const void *, const void *,
                         const void *, const void *, double, const void *, double *, hipStream_t);
void energy_backward_impl(hsim_plan, int32_t, hsim_precision, const void *, const void *,
                          const void *, const void *, double, const void *, const double *, void *,
                          void *, void *, double *, hipStream_t);
hsim_batch batch_create_impl(int32_t, const hsim_plan *, uint64_t, const uint32_t *,
                             hsim_precision, hsim_layout);
void batch_set_shape_impl(hsim_batch, int32_t, int32_t);
void batch_set_order_impl(hsim_batch, int32_t);
void batch_sizes_impl(hsim_batch, int32_t, int32_t, size_t *, size_t *, size_t *);
void batch_bind_impl(hsim_batch, int32_t, int32_t, void *, void *, void *);
void batch_init_impl(hsim_batch, int32_t, const double *, hipStream_t);
void batch_run_impl(hsim_batch, int32_t, int32_t, const double *, const double *, int32_t,
                    hsim_launch, uint32_t, uint32_t *, hipStream_t);
void batch_to_user_impl(hsim_batch, int32_t, double *, hipStream_t);
int32_t batch_status_impl(hsim_batch);
void autotune_impl(hsim_batch, const char *, int32_t, hipStream_t);
int32_t choose_layout_impl(int32_t, const hsim_plan *, uint64_t, const uint32_t *, hsim_precision,
                           const double *, const double *, int32_t, hipStream_t);
void batch_time_phases_impl(hsim_batch, int32_t);
void plan_set_types_impl(hsim_plan, const int32_t *);
void plan_set_site_terms_impl(hsim_plan, const double *, const double *);
void batch_set_policies_impl(hsim_batch, int32_t, const int32_t *, const double *, double, double);
void batch_sigma_impl(hsim_batch, double *);
void batch_bind_outputs_impl(hsim_batch, int32_t, double *, double *);
namespace hsim {
void analysis_thermal_impl(const double *, int32_t, int32_t, int32_t, int32_t, int64_t,
                           const double *, int32_t, const double *, double *, hipStream_t);
void analysis_tau_impl(const double *, int32_t, int32_t, int32_t, int32_t, int32_t, double,
                       double *, int32_t *, hipStream_t);
void analysis_multihist_impl(const double *, int32_t, int32_t, int32_t, int32_t, int64_t, int32_t,
                             const int32_t *, const double *, int32_t, const double *, int32_t,
                             double, double *, int32_t *, double *, hipStream_t);
}  // namespace hsim
void batch_phase_times_impl(hsim_batch, double *, int64_t *, int64_t *);

namespace {

thread_local std::string g_last_error;

template <typename F>
hsim_status guarded(F &&f)
{
    try {
        f();
        g_last_error.clear();
        return HSIM_OK;
    } catch (const hsim::Error &e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host out of memory";
        return HSIM_E_DEVICE;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return HSIM_E_DEVICE;
    } catch (...) {
        g_last_error = "unknown error";
        return HSIM_E_DEVICE;
    }
}

hipStream_t S(void *s) { return (hipStream_t)s; }

}  // namespace

extern "C" {

hsim_status hsim_plan_create(hsim_plan *out, int64_t n, const int64_t *row_ptr, const int32_t *col,
                             const double *J, const double *k, const double *axis,
                             const double *field_dir, uint32_t flags)
{
    return guarded([&] {
        if (!out) throw hsim::Error(HSIM_E_ARG, "plan_create: NULL out");
        if (flags != 0) throw hsim::Error(HSIM_E_ARG, "plan_create: flags must be 0");
        *out = nullptr;
        *out = plan_create_impl(n, row_ptr, col, J, k, axis, field_dir);
    });
}

hsim_status hsim_plan_info(hsim_plan p, hsim_plan_info_t *out)
{
    return guarded([&] {
        if (!p || !out) throw hsim::Error(HSIM_E_ARG, "plan_info: NULL argument");
        std::memset(out, 0, sizeof(*out));
        out->n_sites = p->n;
        out->nnz = p->nnz;
        out->n_bonds = p->nb;
        out->n_colours = p->ncol;
        out->max_degree = p->maxdeg;
        for (int c = 0; c < p->ncol && c < 64; ++c) out->colour_size[c] = p->cls_off[c + 1] - p->cls_off[c];
        out->mean_degree = p->n > 0 ? (double)p->nnz / (double)p->n : 0.0;
        out->uniform_anisotropy = p->kmode != hsim::K_SITE;
        out->uniform_field_dir = p->fmode == hsim::F_UNIFORM;
    });
}

hsim_status hsim_plan_colouring(hsim_plan p, int32_t *colour_out)
{
    return guarded([&] {
        if (!p || (!colour_out && p->n > 0)) throw hsim::Error(HSIM_E_ARG, "plan_colouring: NULL argument");
        if (p->n > 0) std::memcpy(colour_out, p->colour.data(), p->n * sizeof(int32_t));
    });
}

hsim_status hsim_plan_bonds(hsim_plan p, int32_t *bond_ij_out, int64_t *n_bonds_out)
{
    return guarded([&] {
        if (!p) throw hsim::Error(HSIM_E_ARG, "plan_bonds: NULL plan");
        if (n_bonds_out) *n_bonds_out = p->nb;
        if (bond_ij_out && p->nb > 0)
            std::memcpy(bond_ij_out, p->bond_ij.data(), 2 * p->nb * sizeof(int32_t));
    });
}

hsim_status hsim_plan_half_rows(hsim_plan p, int32_t *width_out, int32_t *col_out, int32_t *bond_out)
{
    return guarded([&] {
        if (!p) throw hsim::Error(HSIM_E_ARG, "plan_half_rows: NULL plan");
        if (width_out) *width_out = p->h_w;
        const size_t cnt = (size_t)p->h_w * (size_t)p->n;
        if (col_out && cnt > 0) std::memcpy(col_out, p->uhalf_col.data(), cnt * sizeof(int32_t));
        if (bond_out && cnt > 0) std::memcpy(bond_out, p->uhalf_bond.data(), cnt * sizeof(int32_t));
    });
}

hsim_status hsim_plan_set_types(hsim_plan p, const int32_t *site_type)
{
    return guarded([&] { plan_set_types_impl(p, site_type); });
}

hsim_status hsim_plan_set_site_terms(hsim_plan p, const double *k_cubic, const double *spin_norm)
{
    return guarded([&] { plan_set_site_terms_impl(p, k_cubic, spin_norm); });
}

void hsim_plan_destroy(hsim_plan p) { delete p; }

hsim_status hsim_batch_create(hsim_batch *out, int32_t n_rep, const hsim_plan *plans, uint64_t seed,
                              const uint32_t *replica_id, hsim_precision precision,
                              hsim_layout layout)
{
    return guarded([&] {
        if (!out) throw hsim::Error(HSIM_E_ARG, "batch_create: NULL out");
        *out = nullptr;
        *out = batch_create_impl(n_rep, plans, seed, replica_id, precision, layout);
    });
}

hsim_status hsim_batch_info(hsim_batch b, hsim_batch_info_t *out)
{
    return guarded([&] {
        if (!b || !out) throw hsim::Error(HSIM_E_ARG, "batch_info: NULL argument");
        std::memset(out, 0, sizeof(*out));
        out->layout = b->layout;
        out->n_rep = b->R;
        out->n_phases = b->ncol_max;
        out->total_sites = b->total_sites;
        out->lds_resident = b->layout == HSIM_LAYOUT_BLOCK && b->lds;
        out->sites_per_wave = b->layout == HSIM_LAYOUT_REPLICA ? b->la.spw : 0;
        out->masked_store = b->layout == HSIM_LAYOUT_REPLICA ? b->la.masked_store : 0;
        out->tuned_launch = b->tuned_launch;
        out->persistent_grid = b->persistent_grid;
    });
}

hsim_status hsim_batch_set_shape(hsim_batch b, int32_t spw, int32_t masked)
{
    return guarded([&] { batch_set_shape_impl(b, spw, masked); });
}

hsim_status hsim_batch_set_order(hsim_batch b, int32_t plane_sites)
{
    return guarded([&] { batch_set_order_impl(b, plane_sites); });
}

hsim_status hsim_batch_sizes(hsim_batch b, int32_t n_steps, int32_t mcs, size_t *ws, size_t *sp,
                             size_t *hist)
{
    return guarded([&] { batch_sizes_impl(b, n_steps, mcs, ws, sp, hist); });
}

hsim_status hsim_batch_bind(hsim_batch b, int32_t n_steps, int32_t mcs, void *ws, void *sp, void *hist)
{
    return guarded([&] { batch_bind_impl(b, n_steps, mcs, ws, sp, hist); });
}

hsim_status hsim_batch_init_spins(hsim_batch b, int32_t mode, const double *host, void *stream)
{
    return guarded([&] { batch_init_impl(b, mode, host, S(stream)); });
}

hsim_status hsim_batch_run(hsim_batch b, int32_t first_step, int32_t n_steps, const double *T,
                           const double *B, int32_t recompute_every, hsim_launch launch,
                           uint32_t run_flags, uint32_t *d_trace, void *stream)
{
    return guarded([&] {
        batch_run_impl(b, first_step, n_steps, T, B, recompute_every, launch, run_flags, d_trace,
                       S(stream));
    });
}

hsim_status hsim_batch_set_policies(hsim_batch b, int32_t n_types, const int32_t *policy,
                                    const double *param, double sigma_min, double sigma_max)
{
    return guarded([&] { batch_set_policies_impl(b, n_types, policy, param, sigma_min, sigma_max); });
}

hsim_status hsim_batch_bind_outputs(hsim_batch b, int32_t n_types, double *d_type_mag,
                                    double *d_snapshots)
{
    return guarded([&] { batch_bind_outputs_impl(b, n_types, d_type_mag, d_snapshots); });
}

hsim_status hsim_batch_sigma(hsim_batch b, double *sigma_out)
{
    return guarded([&] { batch_sigma_impl(b, sigma_out); });
}

hsim_status hsim_batch_time_phases(hsim_batch b, int32_t every)
{
    return guarded([&] { batch_time_phases_impl(b, every); });
}

hsim_status hsim_batch_phase_times(hsim_batch b, double *total_ms, int64_t *launches, int64_t *updates)
{
    return guarded([&] { batch_phase_times_impl(b, total_ms, launches, updates); });
}

hsim_status hsim_batch_spins_to_user(hsim_batch b, int32_t rep, double *d_out, void *stream)
{
    return guarded([&] { batch_to_user_impl(b, rep, d_out, S(stream)); });
}

hsim_status hsim_batch_status(hsim_batch b, int32_t *out)
{
    return guarded([&] {
        if (!out) throw hsim::Error(HSIM_E_ARG, "batch_status: NULL out");
        *out = batch_status_impl(b);
    });
}

hsim_status hsim_autotune(hsim_batch b, const char *cache_path, int32_t trial_mcs, void *stream)
{
    return guarded([&] { autotune_impl(b, cache_path, trial_mcs, S(stream)); });
}

hsim_status hsim_choose_layout(int32_t n_rep, const hsim_plan *plan_of_rep, uint64_t seed,
                               const uint32_t *replica_id, hsim_precision precision, const double *T,
                               const double *B, int32_t trial_mcs, int32_t *layout_out, void *stream)
{
    return guarded([&] {
        if (!layout_out) throw hsim::Error(HSIM_E_ARG, "choose_layout: NULL layout_out");
        *layout_out = choose_layout_impl(n_rep, plan_of_rep, seed, replica_id, precision, T, B, trial_mcs,
                                         S(stream));
    });
}

void hsim_batch_destroy(hsim_batch b) { delete b; }

hsim_status hsim_energy_prepare(hsim_plan plan)
{
    return guarded([&] { energy_prepare_impl(plan); });
}

hsim_status hsim_energy_forward(hsim_plan plan, int32_t batch, hsim_precision precision,
                                const void *d_spins, const void *d_J_bond, const void *d_k,
                                const void *d_axis, double B, const void *d_field_dir,
                                double *d_E, void *stream)
{
    return guarded([&] {
        energy_forward_impl(plan, batch, precision, d_spins, d_J_bond, d_k, d_axis, B,
                            d_field_dir, d_E, S(stream));
    });
}

hsim_status hsim_energy_forward_noalloc(hsim_plan plan, int32_t batch, hsim_precision precision,
                                        const void *d_spins, const void *d_J_bond, const void *d_k,
                                        const void *d_axis, double B, const void *d_field_dir,
                                        double *d_E, void *stream)
{
    return guarded([&] {
        energy_forward_noalloc_impl(plan, batch, precision, d_spins, d_J_bond, d_k, d_axis, B,
                                    d_field_dir, d_E, S(stream));
    });
}

hsim_status hsim_energy_backward(hsim_plan plan, int32_t batch, hsim_precision precision,
                                 const void *d_spins, const void *d_J_bond, const void *d_k,
                                 const void *d_axis, double B, const void *d_field_dir,
                                 const double *d_gE, void *d_gS, void *d_gJ_bond, void *d_gk,
                                 double *d_gB, void *stream)
{
    return guarded([&] {
        energy_backward_impl(plan, batch, precision, d_spins, d_J_bond, d_k, d_axis, B,
                             d_field_dir, d_gE, d_gS, d_gJ_bond, d_gk, d_gB, S(stream));
    });
}

hsim_status hsim_fluct_estimate(int64_t n, double beta, const double *d_O, const double *d_dE,
                                const double *d_dO, double *d_out, void *stream)
{
    return guarded([&] {
        if (n < 1 || !d_O || !d_dE || !d_out) throw hsim::Error(HSIM_E_ARG, "fluct_estimate: bad argument");
        if (!std::isfinite(beta) || beta < 0) throw hsim::Error(HSIM_E_PARAM, "beta must be finite and >= 0");
        hsim::hip_check(hsim::launch_fluct(S(stream), n, beta, d_O, d_dE, d_dO, d_out), "fluct launch");
    });
}

hsim_status hsim_fluct_weights(int64_t n, double beta, const double *d_O, double c, double *d_w,
                               void *stream)
{
    return guarded([&] {
        if (n < 1 || !d_O || !d_w) throw hsim::Error(HSIM_E_ARG, "fluct_weights: bad argument");
        if (!std::isfinite(beta) || beta < 0) throw hsim::Error(HSIM_E_PARAM, "beta must be finite and >= 0");
        if (!std::isfinite(c)) throw hsim::Error(HSIM_E_PARAM, "c must be finite");
        hsim::hip_check(hsim::launch_fluct_weights(S(stream), n, beta, d_O, c, d_w), "fluct weights launch");
    });
}

hsim_status hsim_spins_planar(int64_t n_cfg, int64_t n_sites, const double *d_in,
                              hsim_precision precision, void *d_out, void *stream)
{
    return guarded([&] {
        if (n_cfg < 0 || n_sites < 0 || (n_cfg * n_sites > 0 && (!d_in || !d_out)))
            throw hsim::Error(HSIM_E_ARG, "spins_planar: bad argument");
        if (precision != HSIM_FP32 && precision != HSIM_FP64_EXACT)
            throw hsim::Error(HSIM_E_ARG, "bad precision");
        hsim::hip_check(hsim::launch_spins_planar(S(stream), precision == HSIM_FP64_EXACT, n_cfg,
                                                  n_sites, d_in, d_out),
                        "spins planar launch");
    });
}

hsim_status hsim_analysis_thermal(const double *d_history, int32_t n_rep, int32_t n_steps,
                                  int32_t mcs, int32_t m0, int64_t n_sites, const double *beta,
                                  int32_t n_eval, const double *beta_eval, double *d_out,
                                  void *stream)
{
    return guarded([&] {
        hsim::analysis_thermal_impl(d_history, n_rep, n_steps, mcs, m0, n_sites, beta, n_eval,
                                    beta_eval, d_out, S(stream));
    });
}

hsim_status hsim_analysis_tau(const double *d_history, int32_t n_rep, int32_t n_steps,
                              int32_t mcs, int32_t m0, int32_t observable, double c,
                              double *d_tau, int32_t *d_window, void *stream)
{
    return guarded([&] {
        hsim::analysis_tau_impl(d_history, n_rep, n_steps, mcs, m0, observable, c, d_tau, d_window,
                                S(stream));
    });
}

hsim_status hsim_analysis_multihist(const double *d_history, int32_t n_rep, int32_t n_steps,
                                    int32_t mcs, int32_t m0, int64_t n_sites, int32_t K,
                                    const int32_t *series, const double *beta_k, int32_t n_eval,
                                    const double *beta_eval, int32_t max_iter, double tol,
                                    double *f_out, int32_t *iters_out, double *d_out, void *stream)
{
    return guarded([&] {
        hsim::analysis_multihist_impl(d_history, n_rep, n_steps, mcs, m0, n_sites, K, series,
                                      beta_k, n_eval, beta_eval, max_iter, tol, f_out, iters_out,
                                      d_out, S(stream));
    });
}

const char *hsim_last_error(void) { return g_last_error.c_str(); }

const char *hsim_version(void) { return "hsim 0.1 (gfx950)"; }

}  // extern "C"
