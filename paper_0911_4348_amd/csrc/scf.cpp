// Self-consistent second-Born ground state (paper Sec. 2.3): FE-DVR setup,
// HF, then Sigma_2B / energy / Dyson step until the energy settles.
//
// Loop (k = 0, 1, ...): Sigma_c = Sigma_2B[G_k]; E_k = E_GM[G_k, Sigma_c];
// stop if k >= 1 and |E_k - E_(k-1)| < tol; else G_(k+1) = Dyson step of G_k.
// The mixed form runs this loop in float32 (Sigma_2B optionally on bf16
// matrix cores) and then continues in float64 from the float32 fixed point
// until the float64 energy settles; energies, the HF step and the chemical
// potential are always float64.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <vector>

#include "common.h"

using namespace negf;

namespace {

struct Iterate {
    int k;
    double E, N;
};

template <class T>
int scf_phase(negf_ctx* ctx, const negf_tau_grid_t* tg, int n, int sigma, const double* h, const double* V64,
              const T* Vt, const double* eps, const double* C, double mu, const double* Sigma0, T* G, T* Sc,
              double alpha, int symmetrize, int conv_algo, int sig_dtype, double tol, int limit, bool fixed,
              int dtype_tag, double e_nn, int* steps_done, double* E_last, double* N_last, bool* converged,
              negf_iter_log_t* log, int log_cap, int* log_n, int step_offset, hipStream_t st) {
    const int n_tau = tg->n_tau;
    const int dt = sizeof(T) == 8 ? NEGF_F64 : NEGF_F32;
    double E_prev = NAN;
    int k = 0;
    *converged = false;
    while (true) {
        auto t0 = std::chrono::steady_clock::now();
        NEGF_TRY(negf_sigma2b(ctx, n, n_tau, sigma, Vt, G, Sc, sig_dtype, st));
        double E = 0, N = 0;
        NEGF_TRY(energy_run<T>(ctx, tg, n, sigma, h, V64, G, Sc, &E, &N, st));
        E += e_nn;
        if (!std::isfinite(E) || !std::isfinite(N)) {
            set_error("energy or particle number not finite at step %d", step_offset + k);
            *E_last = E;
            *N_last = N;
            *steps_done = k;
            return NEGF_ENAN;
        }
        const double dE = std::isnan(E_prev) ? NAN : E - E_prev;
        bool stop = false;
        if (!fixed && k >= 1 && std::fabs(dE) < tol) {
            *converged = true;
            stop = true;
        }
        if (k >= limit) stop = true;
        if (!stop) NEGF_TRY(dyson_run<T>(ctx, tg, n, sigma, h, V64, eps, C, mu, Sigma0, G, Sc, alpha, symmetrize,
                                         conv_algo, G, st));
        HIP_TRY(hipStreamSynchronize(st));
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (log && *log_n < log_cap) log[(*log_n)++] = negf_iter_log_t{step_offset + k, dtype_tag, E, dE, N, ms};
        *E_last = E;
        *N_last = N;
        if (stop) break;
        E_prev = E;
        ++k;
    }
    *steps_done = k;
    (void)dt;
    return NEGF_OK;
}

}  // namespace

extern "C" int negf_scf(negf_ctx* ctx, const negf_system_t* sys, const negf_opts_t* o, const double* G_guess,
                        double* G_out, double* E_out, double* N_out, int* iters, negf_iter_log_t* log, int log_cap,
                        double* hf_E, double* hf_mu, void* stream) {
    NEGF_REQUIRE(ctx && sys && o, "NULL argument");
    NEGF_REQUIRE(o->alpha > 0 && o->alpha <= 1, "alpha must be in (0, 1]");
    NEGF_REQUIRE(o->tol > 0, "tol must be positive");
    NEGF_REQUIRE(o->max_iter >= 1 || o->fixed_iters > 0, "max_iter must be >= 1");
    NEGF_REQUIRE(o->dtype == NEGF_F64 || o->dtype == NEGF_F32 || o->dtype == NEGF_BF16, "bad dtype");
    NEGF_REQUIRE(o->conv_algo >= NEGF_CONV_AUTO && o->conv_algo <= NEGF_CONV_DIRECT, "bad conv_algo");
    NEGF_REQUIRE(sys->sigma == 1 || sys->sigma == 2, "sigma must be 1 or 2");
    NEGF_REQUIRE(sys->beta > 0 && std::isfinite(sys->beta), "beta must be positive");
    NEGF_REQUIRE(log_cap >= 0, "log_cap < 0");
    int n = 0, n_tau = 0;
    NEGF_TRY(negf_fedvr_size(sys->grid.n_e, sys->grid.n_g, &n));
    NEGF_REQUIRE(n <= 4096, "n_b too large");
    NEGF_REQUIRE(sys->n_elec > 0 && sys->n_elec < (double)sys->sigma * n, "n_elec out of range");
    NEGF_TRY(negf_tau_count(sys->tau_kind, sys->M, sys->u, sys->p, &n_tau));
    std::vector<double> tau(n_tau);
    NEGF_TRY(negf_tau_grid(sys->tau_kind, sys->beta, sys->M, sys->u, sys->p, tau.data()));
    negf_tau_grid_t tg{sys->tau_kind, n_tau, sys->tau_kind == NEGF_TAU_POWER ? sys->u : 0, sys->beta, tau.data()};
    NEGF_TRY(check_tau_grid(&tg));
    if (o->conv_algo == NEGF_CONV_FFT) {
        const int M = n_tau - 1;
        NEGF_REQUIRE(sys->tau_kind == NEGF_TAU_UNIFORM && (M & (M - 1)) == 0 && M <= 8192,
                     "the Fourier route needs a uniform grid with a power-of-two M <= 8192");
    }
    const long nn = (long)n * n;
    std::vector<double> T((size_t)nn), v(n), V((size_t)nn), h((size_t)nn);
    NEGF_TRY(fedvr_build(&sys->grid, &sys->pot, nullptr, nullptr, T.data(), v.data(), V.data()));
    for (long e = 0; e < nn; ++e) h[e] = T[e] + ((e / n) == (e % n) ? v[e / n] : 0.0);
    NEGF_TRY(bind_device(ctx));
    hipStream_t st = (hipStream_t)stream;

    void *dT, *dv, *dV, *dh;
    NEGF_TRY(upload(ctx, "scf_T", T.data(), sizeof(double) * nn, st, &dT));
    NEGF_TRY(upload(ctx, "scf_v", v.data(), sizeof(double) * n, st, &dv));
    NEGF_TRY(upload(ctx, "scf_V", V.data(), sizeof(double) * nn, st, &dV));
    NEGF_TRY(upload(ctx, "scf_h", h.data(), sizeof(double) * nn, st, &dh));
    double *eps, *C, *rho, *Sig0;
    NEGF_TRY(scratch_t(ctx, "scf_eps", n, &eps));
    NEGF_TRY(scratch_t(ctx, "scf_C", nn, &C));
    NEGF_TRY(scratch_t(ctx, "scf_rho", nn, &rho));
    NEGF_TRY(scratch_t(ctx, "scf_Sig0", nn, &Sig0));
    double mu = 0, Ehf = 0;
    int hf_it = 0;
    const double hf_tol = o->hf_tol > 0 ? o->hf_tol : 1e-13;
    const int hf_max = o->hf_max_iter > 0 ? o->hf_max_iter : 1000;
    NEGF_TRY(hf_run(ctx, n, (double*)dT, (double*)dv, (double*)dV, sys->n_elec, sys->sigma, sys->beta, hf_tol, hf_max,
                    eps, C, rho, Sig0, &mu, &Ehf, &hf_it, st));
    if (hf_E) *hf_E = Ehf + sys->e_nn;
    if (hf_mu) *hf_mu = mu;

    double *G, *Sc;
    NEGF_TRY(scratch_t(ctx, "scf_G", nn * n_tau, &G));
    NEGF_TRY(scratch_t(ctx, "scf_Sc", nn * n_tau, &Sc));
    if (G_guess) HIP_TRY(hipMemcpyAsync(G, G_guess, sizeof(double) * nn * n_tau, hipMemcpyDeviceToDevice, st));
    else NEGF_TRY(g0_build<double>(ctx, n, n_tau, tau.data(), sys->beta, eps, C, mu, G, st));

    const bool fixed = o->fixed_iters > 0;
    const int limit = fixed ? o->fixed_iters : o->max_iter;
    int log_n = 0, steps = 0, total = 0;
    double E = 0, N = 0;
    bool conv = false;
    int rc = NEGF_OK;
    if (o->dtype == NEGF_F64) {
        rc = scf_phase<double>(ctx, &tg, n, sys->sigma, (double*)dh, (double*)dV, (double*)dV, eps, C, mu, Sig0, G, Sc,
                               o->alpha, o->symmetrize, o->conv_algo, NEGF_F64, o->tol, limit, fixed, NEGF_F64,
                               sys->e_nn, &steps, &E, &N, &conv, log, log_cap, &log_n, 0, st);
        total = steps;
    } else {
        float *Gf, *Scf, *Vf;
        NEGF_TRY(scratch_t(ctx, "scf_Gf", nn * n_tau, &Gf));
        NEGF_TRY(scratch_t(ctx, "scf_Scf", nn * n_tau, &Scf));
        NEGF_TRY(scratch_t(ctx, "scf_Vf", nn, &Vf));
        NEGF_TRY(to_f32(G, Gf, nn * n_tau, st));
        NEGF_TRY(to_f32((double*)dV, Vf, nn, st));
        rc = scf_phase<float>(ctx, &tg, n, sys->sigma, (double*)dh, (double*)dV, Vf, eps, C, mu, Sig0, Gf, Scf, o->alpha,
                              o->symmetrize, o->conv_algo, o->dtype, o->tol, limit, fixed, o->dtype, sys->e_nn, &steps,
                              &E, &N, &conv, log, log_cap, &log_n, 0, st);
        total = steps;
        if (rc == NEGF_OK && !fixed) {
            // float64 refinement starting from the low-precision fixed point
            NEGF_TRY((convert<double, float>(Gf, G, nn * n_tau, st)));
            const double rt = o->refine_tol > 0 ? o->refine_tol : o->tol;
            int s2 = 0;
            rc = scf_phase<double>(ctx, &tg, n, sys->sigma, (double*)dh, (double*)dV, (double*)dV, eps, C, mu, Sig0, G,
                                   Sc, o->alpha, o->symmetrize, o->conv_algo, NEGF_F64, rt,
                                   o->max_iter > steps ? o->max_iter - steps : 1, false, NEGF_F64, sys->e_nn, &s2, &E,
                                   &N, &conv, log, log_cap, &log_n, steps, st);
            total = steps + s2;
        } else if (rc == NEGF_OK) {
            NEGF_TRY((convert<double, float>(Gf, G, nn * n_tau, st)));
        }
    }
    if (G_out) HIP_TRY(hipMemcpyAsync(G_out, G, sizeof(double) * nn * n_tau, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (E_out) *E_out = E;
    if (N_out) *N_out = N;
    if (iters) *iters = total;
    if (rc != NEGF_OK) return rc;
    if (!fixed && !conv) {
        set_error("SCF not converged after %d steps", total);
        return NEGF_ENOCONV;
    }
    return NEGF_OK;
}
