// Self-consistent second-Born ground state (paper Sec. 2.3): FE-DVR setup,
// HF, then Sigma_2B / energy / Dyson step until the energy settles, for one
// system or a batch of systems of different sizes on one tau grid.
//
// Loop (k = 0, 1, ...), per system: Sigma_c = Sigma_2B[G_k]; E_k = E_GM[G_k,
// Sigma_c]; stop if k >= 1 and |E_k - E_(k-1)| < tol; else G_(k+1) = Dyson step
// of G_k. The mixed form runs this loop in float32 (Sigma_2B optionally on bf16
// matrix cores) and then continues in float64 from the float32 fixed point
// until the float64 energy settles; energies, the HF step and the chemical
// potential are always float64.
//
// Batch execution: one iteration of all unfinished systems is two stream
// segments, (a) Sigma_2B of every system in one persistent kernel launch per
// arithmetic mode plus every energy, (b) every Dyson step. A batch of one system
// with n_b <= 240 runs its float64 Sigma_2B through the single-system tiles
// instead (the direct-to-LDS tile), which the persistent kernel does not have. The energies are
// read back between them (the only host synchronisation per iteration). Each
// segment is recorded once as a HIP graph and replayed while the set of
// unfinished systems does not change; a new set is first run directly (it may
// grow scratch buffers) and recorded at its second iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "common.h"

using namespace negf;

extern "C" int negf_mlp_guess(negf_ctx* ctx, const float* params, double out_scale, int n_b, const double* x,
                              const double* v, int n_c, const double* Xc, const double* Zc, int n_tau,
                              const double* tau, double beta, const double* G0, double* G_out, int dtype,
                              void* stream);

namespace {

enum { PH_LOW = 0, PH_F64 = 1, PH_DONE = 2 };

// out[0] = trace of the n x n matrix A
__global__ __launch_bounds__(256) void k_trace(int n, const double* __restrict__ A, double* out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += A[(long)i * n + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

struct Sys {
    int b;                   // index in the caller's arrays
    int n;
    long nn;
    double *T, *v, *V, *h, *x;          // device, float64
    double *eps, *C, *rho, *Sig0;       // HF state
    double mu = 0, Ehf = 0;
    int hf_it = 0;
    double* G = nullptr;     // float64 iterate
    double* Sc = nullptr;
    float *Gf = nullptr, *Scf = nullptr, *Vf = nullptr;
    int phase = PH_F64;
    int k = 0;               // Sigma/energy evaluations done in this phase, minus one
    int limit = 0;
    int steps_low = 0;
    double E_prev = NAN, E = 0, N = 0;
    bool conv = false;
    bool nan = false;
    bool hf_ok = true;       // HF converged; otherwise the system is not iterated
    bool learned = false;    // started from the learned guess
    bool restarted = false;  // learned start abandoned for G0 after a non-finite energy
    int wasted = 0;          // steps spent before such a restart
    int log_n = 0;
    double alpha = 0.3;      // mixing of this system (halved by each guard restart)
    int backoffs = 0;        // guard restarts so far
    double dh[4] = {0, 0, 0, 0};   // last energy changes of the current run, newest first
    int nd = 0;
};

constexpr double kNGuard = 0.5;    // relative particle-number drift that restarts a run
constexpr int kMaxBackoff = 3;

// The guard's runaway test: E or N not finite, N off by more than kNGuard, or
// the energy change growing three times in a row.
bool runaway(double E, double N, double n_elec, const double* dh, int nd) {
    if (!std::isfinite(E) || !std::isfinite(N)) return true;
    if (std::fabs(N - n_elec) > kNGuard * n_elec) return true;
    return nd >= 4 && std::fabs(dh[0]) > std::fabs(dh[1]) && std::fabs(dh[1]) > std::fabs(dh[2]) &&
           std::fabs(dh[2]) > std::fabs(dh[3]);
}

// The stopping test on the last energy changes (dh[0] newest, nd of them).
bool stop_test(int rule, const double* dh, int nd, double tol) {
    if (nd < 1) return false;
    if (rule == NEGF_STOP_DELTA) return std::fabs(dh[0]) < tol;
    if (dh[0] == 0.0) return true;
    if (nd < 3 || dh[1] == 0.0 || dh[2] == 0.0) return false;
    const double rho = std::max(std::fabs(dh[0] / dh[1]), std::fabs(dh[1] / dh[2]));
    return rho < 1.0 && std::fabs(dh[0]) * rho / (1.0 - rho) < tol;
}

struct GraphSlot {
    std::string key;
    hipGraphExec_t exec = nullptr;
    void drop() {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
    }
};

// Run `body` on stream st: directly, or recorded into slot's graph and replayed.
template <class F>
int run_segment(GraphSlot& slot, const std::string& key, bool graphs, GraphSlot& other, hipStream_t st, F body) {
    if (!graphs) return body();
    if (key != slot.key) {
        // new set of systems: run directly once (scratch may grow, which
        // invalidates every recorded graph)
        slot.drop();
        other.drop();
        slot.key = key;
        return body();
    }
    if (!slot.exec) {
        HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
        const int rc = body();
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(st, &g);
        if (rc != NEGF_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) {
            set_error("graph capture failed: %s", hipGetErrorString(e));
            return NEGF_EHIP;
        }
        const hipError_t e2 = hipGraphInstantiate(&slot.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) {
            slot.exec = nullptr;
            set_error("graph instantiation failed: %s", hipGetErrorString(e2));
            return NEGF_EHIP;
        }
    }
    HIP_TRY(hipGraphLaunch(slot.exec, st));
    return NEGF_OK;
}

int validate(const negf_system_t* s, int* n, int* n_tau) {
    NEGF_REQUIRE(s->sigma == 1 || s->sigma == 2, "sigma must be 1 or 2");
    NEGF_REQUIRE(s->beta > 0 && std::isfinite(s->beta), "beta must be positive");
    NEGF_TRY(negf_fedvr_size(s->grid.n_e, s->grid.n_g, n));
    NEGF_REQUIRE(*n <= 4096, "n_b too large");
    NEGF_REQUIRE(s->n_elec > 0 && s->n_elec < (double)s->sigma * *n, "n_elec out of range");
    NEGF_TRY(negf_tau_count(s->tau_kind, s->M, s->u, s->p, n_tau));
    return NEGF_OK;
}

}  // namespace

extern "C" int negf_scf_batched(negf_ctx* ctx, int batch, const negf_system_t* systems, const negf_opts_t* o,
                                double* const* G_guess, double* const* G_out, double* E_out, double* N_out,
                                int* iters, int* status, negf_iter_log_t* log, int log_cap, int* log_n,
                                double* hf_E, double* hf_mu, void* stream) {
    NEGF_REQUIRE(ctx && systems && o, "NULL argument");
    NEGF_REQUIRE(batch >= 1 && batch <= 4096, "batch = %d out of range [1, 4096]", batch);
    NEGF_REQUIRE(o->alpha > 0 && o->alpha <= 1, "alpha must be in (0, 1]");
    NEGF_REQUIRE(o->tol > 0, "tol must be positive");
    NEGF_REQUIRE(o->max_iter >= 1 || o->fixed_iters > 0, "max_iter must be >= 1");
    NEGF_REQUIRE(o->dtype == NEGF_F64 || o->dtype == NEGF_F32 || o->dtype == NEGF_BF16, "bad dtype");
    NEGF_REQUIRE(o->conv_algo >= NEGF_CONV_AUTO && o->conv_algo <= NEGF_CONV_DIRECT, "bad conv_algo");
    NEGF_REQUIRE(log_cap >= 0, "log_cap < 0");
    NEGF_REQUIRE(!o->guess_params || !G_guess, "give either G_guess or guess_params, not both");
    NEGF_REQUIRE(o->stop_rule == NEGF_STOP_DELTA || o->stop_rule == NEGF_STOP_CONTRACTION, "bad stop_rule %d",
                 o->stop_rule);
    const negf_system_t& s0 = systems[0];
    int n_tau = 0;
    std::vector<int> nb(batch);
    for (int b = 0; b < batch; ++b) {
        const negf_system_t& s = systems[b];
        int nt = 0;
        NEGF_TRY(validate(&s, &nb[b], &nt));
        NEGF_REQUIRE(s.tau_kind == s0.tau_kind && s.beta == s0.beta && s.M == s0.M && s.u == s0.u && s.p == s0.p,
                     "system %d: every system of a batch must use the same tau grid", b);
        if (o->guess_params) NEGF_REQUIRE(s.pot.n_c <= 3, "the learned guess takes at most 3 nuclei");
        n_tau = nt;
    }
    std::vector<double> tau(n_tau);
    NEGF_TRY(negf_tau_grid(s0.tau_kind, s0.beta, s0.M, s0.u, s0.p, tau.data()));
    negf_tau_grid_t tg{s0.tau_kind, n_tau, s0.tau_kind == NEGF_TAU_POWER ? s0.u : 0, s0.beta, tau.data()};
    NEGF_TRY(check_tau_grid(&tg));
    if (o->conv_algo == NEGF_CONV_FFT) {
        const int M = n_tau - 1;
        NEGF_REQUIRE(s0.tau_kind == NEGF_TAU_UNIFORM && (M & (M - 1)) == 0 && M <= 8192,
                     "the Fourier route needs a uniform grid with a power-of-two M <= 8192");
    }
    NEGF_TRY(bind_device(ctx));
    if (!ctx->work_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->work_stream, hipStreamNonBlocking));
    hipStream_t st = ctx->work_stream;
    {
        hipEvent_t ev;
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(ev, (hipStream_t)stream));
        HIP_TRY(hipStreamWaitEvent(st, ev, 0));
        (void)hipEventDestroy(ev);
    }

    // ---------------- setup: systems by decreasing n_b, matrices stacked in that order
    std::vector<int> order(batch);
    for (int b = 0; b < batch; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return nb[a] > nb[c]; });
    std::vector<Sys> S(batch);
    long tot_nn = 0, tot_n = 0, tot_g = 0;
    for (int r = 0; r < batch; ++r) {
        S[r].b = order[r];
        S[r].n = nb[order[r]];
        S[r].nn = (long)S[r].n * S[r].n;
        tot_nn += S[r].nn;
        tot_n += S[r].n;
        if (!(G_out && G_out[order[r]])) tot_g += S[r].nn * n_tau;
    }
    std::vector<double> hT(tot_nn), hv(tot_n), hV(tot_nn), hh(tot_nn), hx(tot_n);
    {
        long om = 0, ov = 0;
        for (int r = 0; r < batch; ++r) {
            const negf_system_t& s = systems[S[r].b];
            const int n = S[r].n;
            NEGF_TRY(fedvr_build(&s.grid, &s.pot, hx.data() + ov, nullptr, hT.data() + om, hv.data() + ov,
                                 hV.data() + om));
            for (long e = 0; e < S[r].nn; ++e)
                hh[om + e] = hT[om + e] + ((e / n) == (e % n) ? hv[ov + e / n] : 0.0);
            om += S[r].nn;
            ov += n;
        }
    }
    void *dT, *dv, *dV, *dh, *dx, *dtau;
    NEGF_TRY(upload(ctx, "scf_T", hT.data(), sizeof(double) * tot_nn, st, &dT));
    NEGF_TRY(upload(ctx, "scf_v", hv.data(), sizeof(double) * tot_n, st, &dv));
    NEGF_TRY(upload(ctx, "scf_V", hV.data(), sizeof(double) * tot_nn, st, &dV));
    NEGF_TRY(upload(ctx, "scf_h", hh.data(), sizeof(double) * tot_nn, st, &dh));
    NEGF_TRY(upload(ctx, "scf_x", hx.data(), sizeof(double) * tot_n, st, &dx));
    NEGF_TRY(upload_cached(ctx, "scf_tau", tau.data(), sizeof(double) * n_tau, st, &dtau));
    double *eps, *C, *rho, *Sig0, *Sc, *Gint = nullptr;
    NEGF_TRY(scratch_t(ctx, "scf_eps", tot_n, &eps));
    NEGF_TRY(scratch_t(ctx, "scf_C", tot_nn, &C));
    NEGF_TRY(scratch_t(ctx, "scf_rho", tot_nn, &rho));
    NEGF_TRY(scratch_t(ctx, "scf_Sig0", tot_nn, &Sig0));
    NEGF_TRY(scratch_t(ctx, "scf_Sc", tot_nn * n_tau, &Sc));
    if (tot_g) NEGF_TRY(scratch_t(ctx, "scf_G", tot_g, &Gint));
    const bool low = o->dtype != NEGF_F64;
    float *Gf = nullptr, *Scf = nullptr, *Vf = nullptr;
    if (low) {
        NEGF_TRY(scratch_t(ctx, "scf_Gf", tot_nn * n_tau, &Gf));
        NEGF_TRY(scratch_t(ctx, "scf_Scf", tot_nn * n_tau, &Scf));
        NEGF_TRY(scratch_t(ctx, "scf_Vf", tot_nn, &Vf));
    }
    {
        long om = 0, ov = 0, og = 0;
        for (int r = 0; r < batch; ++r) {
            Sys& y = S[r];
            y.T = (double*)dT + om;
            y.V = (double*)dV + om;
            y.h = (double*)dh + om;
            y.v = (double*)dv + ov;
            y.x = (double*)dx + ov;
            y.eps = eps + ov;
            y.C = C + om;
            y.rho = rho + om;
            y.Sig0 = Sig0 + om;
            y.Sc = Sc + om * n_tau;
            if (G_out && G_out[y.b]) {
                y.G = G_out[y.b];
            } else {
                y.G = Gint + og;
                og += y.nn * n_tau;
            }
            if (low) {
                y.Gf = Gf + om * n_tau;
                y.Scf = Scf + om * n_tau;
                y.Vf = Vf + om;
            }
            om += y.nn;
            ov += y.n;
        }
    }

    // ---------------- HF, one batched solve per group of equal n_b
    const double hf_tol = o->hf_tol > 0 ? o->hf_tol : 1e-13;
    const int hf_max = o->hf_max_iter > 0 ? o->hf_max_iter : 1000;
    for (int r0 = 0; r0 < batch;) {
        int r1 = r0;
        while (r1 < batch && S[r1].n == S[r0].n && systems[S[r1].b].n_elec == systems[S[r0].b].n_elec &&
               systems[S[r1].b].sigma == systems[S[r0].b].sigma)
            ++r1;
        const int B = r1 - r0;
        std::vector<double> mu(B), E(B);
        std::vector<int> it(B), ok(B, 1);
        const negf_system_t& sg = systems[S[r0].b];
        const int hrc = hf_run_batched(ctx, B, S[r0].n, S[r0].T, S[r0].v, S[r0].V, sg.n_elec, sg.sigma, sg.beta,
                                       hf_tol, hf_max, S[r0].eps, S[r0].C, S[r0].rho, S[r0].Sig0, mu.data(),
                                       E.data(), it.data(), st, ok.data());
        if (hrc != NEGF_ENOCONV) NEGF_TRY(hrc);
        for (int r = r0; r < r1; ++r) {
            S[r].mu = mu[r - r0];
            S[r].Ehf = E[r - r0];
            S[r].hf_it = it[r - r0];
            S[r].hf_ok = ok[r - r0] != 0;
            if (hf_E) hf_E[S[r].b] = S[r].Ehf + systems[S[r].b].e_nn;
            if (hf_mu) hf_mu[S[r].b] = S[r].mu;
        }
        r0 = r1;
    }

    // ---------------- starting G
    double* dtr;
    NEGF_TRY(scratch_t(ctx, "scf_trace", 1, &dtr));
    for (Sys& y : S) {
        const negf_system_t& s = systems[y.b];
        if (G_guess && G_guess[y.b]) {
            HIP_TRY(hipMemcpyAsync(y.G, G_guess[y.b], sizeof(double) * y.nn * n_tau, hipMemcpyDeviceToDevice, st));
        } else {
            NEGF_TRY(g0_build<double>(ctx, y.n, n_tau, tau.data(), s.beta, y.eps, y.C, y.mu, y.G, st));
            if (o->guess_params) {
                NEGF_TRY(negf_mlp_guess(ctx, o->guess_params, o->guess_scale, y.n, y.x, y.v, s.pot.n_c, s.pot.X,
                                        s.pot.Z, n_tau, (const double*)dtau, s.beta, y.G, y.G, NEGF_BF16, st));
                // the learned start must hold the right number of electrons,
                // N = -sigma Tr G(beta^-), to within 2%; otherwise start from G0
                hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, st, y.n, y.G + (long)(n_tau - 1) * y.nn, dtr);
                LAUNCH_CHECK();
                double tr = 0.0;
                HIP_TRY(hipMemcpyAsync(&tr, dtr, sizeof(double), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                const double N = -s.sigma * tr;
                if (std::isfinite(N) && std::fabs(N - s.n_elec) <= 0.02 * s.n_elec) y.learned = true;
                else NEGF_TRY(g0_build<double>(ctx, y.n, n_tau, tau.data(), s.beta, y.eps, y.C, y.mu, y.G, st));
            }
        }
        if (low) {
            NEGF_TRY(to_f32(y.G, y.Gf, y.nn * n_tau, st));
            NEGF_TRY(to_f32(y.V, y.Vf, y.nn, st));
        }
    }

    // ---------------- iteration
    const bool fixed = o->fixed_iters > 0;
    int n_hf_fail = 0;
    for (Sys& y : S) {
        y.phase = !y.hf_ok ? PH_DONE : (low ? PH_LOW : PH_F64);
        y.limit = fixed ? o->fixed_iters : o->max_iter;
        y.alpha = o->alpha;
        n_hf_fail += !y.hf_ok;
    }
    if (n_hf_fail) set_error("HF not converged for %d system(s); those were not iterated", n_hf_fail);
    // One system whose direct-to-LDS float64 tile fits its LDS (n_b <= 240, the
    // limit of Sigma-2B configuration 11) runs its float64 Sigma_2B through the
    // single-system tiles; everything else through the persistent kernel.
    const bool single_f64 = batch == 1 && S[0].n <= 240;
    if (o->tune) {
        // tile autotuner for each arithmetic mode over the whole batch (first 16 slice pairs)
        for (int pass = 0; pass < (low ? 2 : 1); ++pass) {
            const int dt = pass == 0 ? o->dtype : NEGF_F64;
            // a single system's float64 Sigma-2B does not use the persistent kernel
            if (single_f64 && dt == NEGF_F64) continue;
            std::vector<int> n(batch), sg(batch);
            std::vector<const void*> Vp(batch), Gp(batch);
            std::vector<void*> Sp(batch);
            for (int r = 0; r < batch; ++r) {
                n[r] = S[r].n;
                sg[r] = systems[S[r].b].sigma;
                const bool f = dt != NEGF_F64;
                Vp[r] = f ? (const void*)S[r].Vf : (const void*)S[r].V;
                Gp[r] = f ? (const void*)S[r].Gf : (const void*)S[r].G;
                Sp[r] = f ? (void*)S[r].Scf : (void*)S[r].Sc;
            }
            S2BBatch probe;
            NEGF_TRY(s2b_batch_prepare(ctx, "probe", dt, batch, n.data(), n_tau, sg.data(), Vp.data(), Gp.data(),
                                       Sp.data(), 16, &probe, st));
            if (!ctx->filled.count(probe.key))
                NEGF_TRY(s2b_batch_tune(ctx, dt, batch, n.data(), n_tau, sg.data(), Vp.data(), Gp.data(), Sp.data(),
                                        16, nullptr, nullptr, st));
        }
    }

    double* dEN;
    NEGF_TRY(scratch_t(ctx, "scf_EN", 2 * (size_t)batch, &dEN));
    std::vector<double> hEN(2 * (size_t)batch);
    const bool graphs = !o->no_graph;
    GraphSlot gS, gD;
    S2BBatch plan_lo, plan_hi;
    std::string plan_key;
    int rc = NEGF_OK;
    auto t_prev = std::chrono::steady_clock::now();
    while (true) {
        std::vector<int> act_lo, act_hi;
        for (int r = 0; r < batch; ++r) {
            if (S[r].phase == PH_LOW) act_lo.push_back(r);
            else if (S[r].phase == PH_F64) act_hi.push_back(r);
        }
        if (act_lo.empty() && act_hi.empty()) break;
        std::string keyS = "S";
        for (int r : act_lo) keyS += " l" + std::to_string(r);
        for (int r : act_hi) keyS += " h" + std::to_string(r);
        if (keyS != plan_key) {
            // work lists of the persistent Sigma-2B launches (uploads: outside any graph)
            auto prep = [&](const std::vector<int>& rs, int dt, const char* tag, S2BBatch* pl) -> int {
                *pl = S2BBatch();
                if (rs.empty()) return NEGF_OK;
                const int B = (int)rs.size();
                std::vector<int> n(B), sg(B);
                std::vector<const void*> Vp(B), Gp(B);
                std::vector<void*> Sp(B);
                for (int i = 0; i < B; ++i) {
                    const Sys& y = S[rs[i]];
                    n[i] = y.n;
                    sg[i] = systems[y.b].sigma;
                    const bool f = dt != NEGF_F64;
                    Vp[i] = f ? (const void*)y.Vf : (const void*)y.V;
                    Gp[i] = f ? (const void*)y.Gf : (const void*)y.G;
                    Sp[i] = f ? (void*)y.Scf : (void*)y.Sc;
                }
                return s2b_batch_prepare(ctx, tag, dt, B, n.data(), n_tau, sg.data(), Vp.data(), Gp.data(),
                                         Sp.data(), 0, pl, st);
            };
            NEGF_TRY(prep(act_lo, o->dtype, "lo", &plan_lo));
            if (!single_f64) NEGF_TRY(prep(act_hi, NEGF_F64, "hi", &plan_hi));
            plan_key = keyS;
            gS.drop();
            gD.drop();
            gS.key.clear();
            gD.key.clear();
        }
        // (a) Sigma_2B of every unfinished system, then every energy
        NEGF_TRY(run_segment(gS, keyS, graphs, gD, st, [&]() -> int {
            if (!act_lo.empty()) NEGF_TRY(s2b_batch_launch(plan_lo, st));
            if (!act_hi.empty()) {
                if (single_f64) {
                    // one system: the float64 tile of negf_sigma2b (direct-to-LDS)
                    const Sys& y = S[act_hi[0]];
                    NEGF_TRY(sigma2b_run_f64_single(ctx, y.n, n_tau, systems[y.b].sigma, y.V, y.G, y.Sc, st));
                } else {
                    NEGF_TRY(s2b_batch_launch(plan_hi, st));
                }
            }
            for (int r : act_lo) {
                const Sys& y = S[r];
                NEGF_TRY(energy_launch<float>(ctx, &tg, y.n, systems[y.b].sigma, y.h, y.V, y.Gf, y.Scf,
                                              dEN + 2 * r, st));
            }
            for (int r : act_hi) {
                const Sys& y = S[r];
                NEGF_TRY(energy_launch<double>(ctx, &tg, y.n, systems[y.b].sigma, y.h, y.V, y.G, y.Sc,
                                               dEN + 2 * r, st));
            }
            return NEGF_OK;
        }));
        HIP_TRY(hipMemcpyAsync(hEN.data(), dEN, sizeof(double) * 2 * batch, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const auto t_now = std::chrono::steady_clock::now();
        const double ms = std::chrono::duration<double, std::milli>(t_now - t_prev).count();
        t_prev = t_now;

        // stopping rule per system
        std::vector<int> dy_lo, dy_hi;
        double max_dE = 0.0;
        for (int r = 0; r < batch; ++r) {
            Sys& y = S[r];
            if (y.phase == PH_DONE) continue;
            const double E = hEN[2 * r] + systems[y.b].e_nn, N = hEN[2 * r + 1];
            y.E = E;
            y.N = N;
            const int step = y.wasted + (y.phase == PH_F64 ? y.steps_low : 0) + y.k;
            const double dE = std::isnan(y.E_prev) ? NAN : E - y.E_prev;
            if (y.k >= 1) {
                for (int h = 3; h > 0; --h) y.dh[h] = y.dh[h - 1];
                y.dh[0] = dE;
                y.nd = std::min(y.nd + 1, 4);
            }
            if (o->guard && y.backoffs < kMaxBackoff && runaway(E, N, systems[y.b].n_elec, y.dh, y.nd)) {
                // particle-number guard: restart from G0 with half the mixing
                if (log && log_n && y.log_n < log_cap)
                    log[(size_t)y.b * log_cap + y.log_n++] =
                        negf_iter_log_t{step, y.phase == PH_LOW ? o->dtype : NEGF_F64, E, NAN, N, ms};
                y.wasted = step + 1;
                y.backoffs++;
                y.alpha *= 0.5;
                NEGF_TRY(g0_build<double>(ctx, y.n, n_tau, tau.data(), systems[y.b].beta, y.eps, y.C, y.mu, y.G, st));
                if (low) NEGF_TRY(to_f32(y.G, y.Gf, y.nn * n_tau, st));
                y.phase = low ? PH_LOW : PH_F64;
                y.k = 0;
                y.steps_low = 0;
                y.E_prev = NAN;
                y.nd = 0;
                y.limit = fixed ? o->fixed_iters : o->max_iter;
                continue;
            }
            if (!o->guard && (!std::isfinite(E) || !std::isfinite(N)) && y.learned && !y.restarted) {
                // the learned start left the basin of the iteration: restart from G0
                y.wasted = step + 1;
                y.restarted = true;
                NEGF_TRY(g0_build<double>(ctx, y.n, n_tau, tau.data(), systems[y.b].beta, y.eps, y.C, y.mu, y.G, st));
                if (low) NEGF_TRY(to_f32(y.G, y.Gf, y.nn * n_tau, st));
                y.phase = low ? PH_LOW : PH_F64;
                y.k = 0;
                y.steps_low = 0;
                y.E_prev = NAN;
                y.limit = fixed ? o->fixed_iters : o->max_iter;
                continue;
            }
            if (!std::isfinite(E) || !std::isfinite(N)) {
                // this system stops; the others go on
                set_error("energy or particle number not finite at step %d (system %d)", step, y.b);
                rc = NEGF_ENAN;
                y.nan = true;
                y.phase = PH_DONE;
                continue;
            }
            if (std::isfinite(dE)) max_dE = std::max(max_dE, std::fabs(dE));
            // a fixed-count run ignores the tolerance; the float64 refinement of
            // the mixed form has its own
            const double tol = (low && y.phase == PH_F64 && o->refine_tol > 0) ? o->refine_tol : o->tol;
            bool stop = false;
            // the low-precision loop of the mixed form also ends on |dE| < tol/10:
            // at the float32 noise the ratios of successive changes stop
            // measuring the contraction, and the float64 refinement that
            // follows applies the chosen rule
            const bool hit = stop_test(o->stop_rule, y.dh, y.nd, tol) ||
                             (y.phase == PH_LOW && stop_test(NEGF_STOP_DELTA, y.dh, y.nd, 0.1 * tol));
            if (!fixed && y.k >= 1 && hit) {
                y.conv = true;
                stop = true;
            }
            if (y.k >= y.limit) stop = true;
            if (log && log_n && y.log_n < log_cap)
                log[(size_t)y.b * log_cap + y.log_n++] =
                    negf_iter_log_t{step, y.phase == PH_LOW ? o->dtype : NEGF_F64, E, dE, N, ms};
            if (!stop) {
                y.E_prev = E;
                ++y.k;
                (y.phase == PH_LOW ? dy_lo : dy_hi).push_back(r);
                continue;
            }
            if (y.phase == PH_LOW) {
                y.steps_low = y.k;
                NEGF_TRY((convert<double, float>(y.Gf, y.G, y.nn * n_tau, st)));
                if (fixed) {
                    y.phase = PH_DONE;
                } else {
                    y.phase = PH_F64;
                    y.k = 0;
                    y.E_prev = NAN;
                    y.nd = 0;
                    y.conv = false;
                    y.limit = o->max_iter > y.steps_low ? o->max_iter - y.steps_low : 1;
                }
            } else {
                y.phase = PH_DONE;
            }
        }
        if (o->progress) {
            std::fprintf(stderr, "negf_scf: iteration done in %.0f ms, %d of %d systems going on, max |dE| %.2e\n", ms,
                         (int)(dy_lo.size() + dy_hi.size()), batch, max_dE);
            std::fflush(stderr);
        }
        // (b) Dyson step of every system that goes on
        if (!dy_lo.empty() || !dy_hi.empty()) {
            // the mixing of each system is part of the recorded segment
            std::string keyD = "D";
            for (int r : dy_lo) keyD += " l" + std::to_string(r) + "a" + std::to_string(S[r].backoffs);
            for (int r : dy_hi) keyD += " h" + std::to_string(r) + "a" + std::to_string(S[r].backoffs);
            NEGF_TRY(run_segment(gD, keyD, graphs, gS, st, [&]() -> int {
                for (int r : dy_lo) {
                    const Sys& y = S[r];
                    NEGF_TRY(dyson_run<float>(ctx, &tg, y.n, systems[y.b].sigma, y.h, y.V, y.eps, y.C, y.mu, y.Sig0,
                                              y.Gf, y.Scf, y.alpha, o->symmetrize, o->conv_algo, y.Gf, st));
                }
                for (int r : dy_hi) {
                    const Sys& y = S[r];
                    NEGF_TRY(dyson_run<double>(ctx, &tg, y.n, systems[y.b].sigma, y.h, y.V, y.eps, y.C, y.mu,
                                               y.Sig0, y.G, y.Sc, y.alpha, o->symmetrize, o->conv_algo, y.G, st));
                }
                return NEGF_OK;
            }));
        }
    }
    gS.drop();
    gD.drop();
    HIP_TRY(hipStreamSynchronize(st));
    int n_unconv = 0;
    for (const Sys& y : S) {
        if (E_out) E_out[y.b] = y.E;
        if (N_out) N_out[y.b] = y.N;
        if (iters) iters[y.b] = y.wasted + y.steps_low + y.k;
        if (log_n) log_n[y.b] = y.log_n;
        if (status)
            status[y.b] = y.nan ? NEGF_ENAN : ((!y.hf_ok || (!fixed && !y.conv)) ? NEGF_ENOCONV : NEGF_OK);
        if ((!fixed && !y.conv && !y.nan) || !y.hf_ok) ++n_unconv;
    }
    if (rc != NEGF_OK) return rc;
    if (n_unconv) {
        if (n_hf_fail) set_error("HF not converged for %d and SCF for %d of %d system(s)", n_hf_fail,
                                 n_unconv - n_hf_fail, batch);
        else set_error("SCF not converged for %d of %d system(s)", n_unconv, batch);
        return NEGF_ENOCONV;
    }
    return NEGF_OK;
}

extern "C" int negf_scf(negf_ctx* ctx, const negf_system_t* sys, const negf_opts_t* o, const double* G_guess,
                        double* G_out, double* E_out, double* N_out, int* iters, negf_iter_log_t* log, int log_cap,
                        double* hf_E, double* hf_mu, void* stream) {
    NEGF_REQUIRE(sys, "NULL argument");
    double* guess = const_cast<double*>(G_guess);
    int ln = 0;
    return negf_scf_batched(ctx, 1, sys, o, G_guess ? &guess : nullptr, G_out ? &G_out : nullptr, E_out, N_out,
                            iters, nullptr, log, log_cap, log ? &ln : nullptr, hf_E, hf_mu, stream);
}
