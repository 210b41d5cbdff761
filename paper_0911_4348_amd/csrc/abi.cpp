// C-ABI entry points: error reporting, context, host-side FE-DVR setup and
// tau grids, argument validation, and dispatch to the device code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "negf_measure.h"

namespace {
thread_local std::string g_err;
}

namespace negf {

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}

int bind_device(negf_ctx* c) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != c->device) HIP_TRY(hipSetDevice(c->device));
    return NEGF_OK;
}

int scratch(negf_ctx* c, const char* name, size_t bytes, void** out) {
    Buf& b = c->bufs[name];
    if (bytes == 0) bytes = 1;
    if (b.cap < bytes) {
        if (b.p) {
            // the stream may still use the old buffer; wait before freeing it
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(b.p));
            c->total -= b.cap;
            b.p = nullptr;
            b.cap = 0;
        }
        size_t cap = (bytes + 255) & ~size_t(255);
        hipError_t e = hipMalloc(&b.p, cap);
        if (e != hipSuccess) {
            set_error("scratch '%s': hipMalloc(%zu) failed: %s", name, cap, hipGetErrorString(e));
            b.p = nullptr;
            return NEGF_ENOMEM;
        }
        b.cap = cap;
        c->total += cap;
    }
    *out = b.p;
    return NEGF_OK;
}

int upload(negf_ctx* c, const char* name, const void* host, size_t bytes, hipStream_t st, void** out) {
    NEGF_TRY(scratch(c, name, bytes, out));
    HIP_TRY(hipMemcpyAsync(*out, host, bytes, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return NEGF_OK;
}

int upload_cached(negf_ctx* c, const char* name, const void* host, size_t bytes, hipStream_t st, void** out) {
    auto& prev = c->host_copy[name];
    const char* h = static_cast<const char*>(host);
    auto bi = c->bufs.find(name);
    if (bi != c->bufs.end() && bi->second.p && prev.size() == bytes && std::memcmp(prev.data(), h, bytes) == 0) {
        *out = bi->second.p;
        return NEGF_OK;
    }
    NEGF_TRY(upload(c, name, host, bytes, st, out));
    prev.assign(h, h + bytes);
    return NEGF_OK;
}

int check_tau_grid(const negf_tau_grid_t* tg) {
    NEGF_REQUIRE(tg != nullptr, "tau grid is NULL");
    NEGF_REQUIRE(tg->tau != nullptr, "tau grid points are NULL");
    NEGF_REQUIRE(tg->n_tau >= 3, "n_tau = %d < 3", tg->n_tau);
    NEGF_REQUIRE(tg->beta > 0 && std::isfinite(tg->beta), "beta must be positive");
    NEGF_REQUIRE(tg->kind == NEGF_TAU_UNIFORM || tg->kind == NEGF_TAU_POWER, "bad tau kind %d", tg->kind);
    const int n = tg->n_tau;
    NEGF_REQUIRE(tg->tau[0] == 0.0 && tg->tau[n - 1] == tg->beta, "tau grid must run from 0 to beta");
    for (int q = 1; q < n; ++q)
        NEGF_REQUIRE(tg->tau[q] > tg->tau[q - 1], "tau grid not increasing at %d", q);
    for (int q = 0; q < n; ++q)
        NEGF_REQUIRE(std::fabs(tg->tau[q] + tg->tau[n - 1 - q] - tg->beta) <= 1e-12 * tg->beta,
                     "tau grid not symmetric under tau -> beta - tau at %d", q);
    if (tg->kind == NEGF_TAU_POWER) {
        NEGF_REQUIRE(tg->block >= 4 && (n - 1) % tg->block == 0,
                     "power mesh needs block (u) >= 4 dividing n_tau - 1");
    }
    return NEGF_OK;
}

}  // namespace negf

using namespace negf;

// ============================================================== error / version
extern "C" const char* negf_last_error(void) { return g_err.c_str(); }
extern "C" int negf_version(void) { return 1; }

// ============================================================== context
extern "C" int negf_ctx_create(int device, negf_ctx** out) {
    NEGF_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        set_error("no HIP device available");
        return NEGF_ENODEV;
    }
    if (device < 0 || device >= n) {
        set_error("device %d out of range (%d devices)", device, n);
        return NEGF_ENODEV;
    }
    // address of this device's copy of the allocation-free Sigma-2B array
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    HIP_TRY(hipSetDevice(device));
    const int irc = s2b_noalloc_init(device);
    (void)hipSetDevice(cur);
    NEGF_TRY(irc);
    negf_ctx* c = new negf_ctx();
    c->device = device;
    *out = c;
    return NEGF_OK;
}

extern "C" int negf_ctx_destroy(negf_ctx* c) {
    if (!c) return NEGF_OK;
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : c->bufs)
        if (kv.second.p) (void)hipFree(kv.second.p);
    if (c->work_stream) (void)hipStreamDestroy(c->work_stream);
    if (cur >= 0) (void)hipSetDevice(cur);
    delete c;
    return NEGF_OK;
}

extern "C" int negf_ctx_scratch_bytes(const negf_ctx* c, size_t* bytes) {
    NEGF_REQUIRE(c && bytes, "NULL argument");
    *bytes = c->total;
    return NEGF_OK;
}

// ============================================================== FE-DVR (host, float64)
namespace {

// Legendre P_N and its first derivative at x by the three-term recurrence.
void legendre(int N, double x, double* P, double* dP) {
    double p0 = 1.0, p1 = x;
    if (N == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int k = 2; k <= N; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    *P = p1;
    // derivative from (1 - x^2) P_N' = N (P_(N-1) - x P_N), valid for |x| < 1
    *dP = (std::fabs(x) < 1.0) ? N * (p0 - x * p1) / (1.0 - x * x) : 0.5 * N * (N + 1) * (x > 0 ? 1.0 : (N % 2 ? 1.0 : -1.0));
}

// Generalized Gauss-Lobatto nodes on [-1, 1]: endpoints and the zeros of P_N',
// found by Newton's method from Chebyshev-Lobatto starting points, with
// P_N'' taken from Legendre's equation.
void gll(int N, std::vector<double>& x, std::vector<double>& w, std::vector<double>& D) {
    x.assign(N + 1, 0.0);
    w.assign(N + 1, 0.0);
    x[0] = -1.0;
    x[N] = 1.0;
    for (int j = 1; j < N; ++j) {
        double z = -std::cos(M_PI * j / N);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(N, z, &P, &dP);
            double d2P = (2.0 * z * dP - N * (N + 1.0) * P) / (1.0 - z * z);
            double dz = dP / d2P;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        x[j] = z;
    }
    std::vector<double> PN(N + 1);
    for (int m = 0; m <= N; ++m) {
        double P, dP;
        legendre(N, x[m], &P, &dP);
        PN[m] = P;
        w[m] = 2.0 / (N * (N + 1.0) * P * P);
    }
    // derivative of the Lagrange basis at the nodes (closed form for GLL points)
    D.assign((N + 1) * (N + 1), 0.0);
    for (int m = 0; m <= N; ++m)
        for (int b = 0; b <= N; ++b)
            if (m != b) D[m * (N + 1) + b] = PN[m] / (PN[b] * (x[m] - x[b]));
    D[0] = -N * (N + 1.0) / 4.0;
    D[N * (N + 1) + N] = N * (N + 1.0) / 4.0;
}

}  // namespace

extern "C" int negf_fedvr_size(int n_e, int n_g, int* n_b) {
    NEGF_REQUIRE(n_b != nullptr, "n_b is NULL");
    NEGF_REQUIRE(n_e >= 1 && n_g >= 2, "need n_e >= 1 and n_g >= 2 (got %d, %d)", n_e, n_g);
    NEGF_REQUIRE((long)n_e * n_g - 1 <= 65536, "basis too large");
    *n_b = n_e * n_g - 1;
    return NEGF_OK;
}

extern "C" int fedvr_build(const negf_grid_t* g, const negf_potential_t* pot, double* x_out,
                           double* W_out, double* T_out, double* v_out, double* V_out) {
    NEGF_REQUIRE(g && pot, "grid or potential is NULL");
    int n_b = 0;
    NEGF_TRY(negf_fedvr_size(g->n_e, g->n_g, &n_b));
    NEGF_REQUIRE(g->bounds != nullptr, "bounds is NULL");
    for (int e = 0; e < g->n_e; ++e)
        NEGF_REQUIRE(g->bounds[e + 1] > g->bounds[e] && std::isfinite(g->bounds[e + 1]),
                     "element bounds must increase (element %d)", e);
    NEGF_REQUIRE(pot->n_c >= 0 && pot->n_c <= 64, "n_c out of range");
    NEGF_REQUIRE(pot->n_c == 0 || (pot->X && pot->Z), "centres/charges NULL");
    NEGF_REQUIRE(pot->soft > 0 && pot->ee_soft > 0, "softening must be positive");
    NEGF_REQUIRE(pot->omega >= 0 && std::isfinite(pot->omega), "omega must be finite and >= 0");
    const int N = g->n_g, n_e = g->n_e;
    std::vector<double> xr, wr, D;
    gll(N, xr, wr, D);

    // global index of local node m in element e (Eq. basis): interior nodes,
    // then the bridge shared with element e+1; the outer end nodes are dropped.
    auto gidx = [&](int e, int m) -> int {
        if (m == 0) return e == 0 ? -1 : e * N - 1;
        if (m == N) return e == n_e - 1 ? -1 : e * N + N - 1;
        return e * N + m - 1;
    };
    std::vector<double> x(n_b, 0.0), W(n_b, 0.0);
    for (int e = 0; e < n_e; ++e) {
        double a = g->bounds[e], b = g->bounds[e + 1], h = b - a;
        for (int m = 0; m <= N; ++m) {
            int k = gidx(e, m);
            if (k < 0) continue;
            W[k] += 0.5 * wr[m] * h;                                   // Eq. wim
            if (m == N) x[k] = b;                                      // bridge node = boundary
            else if (m > 0) x[k] = 0.5 * (h * xr[m] + (b + a));        // Eq. xim
        }
    }
    if (x_out) std::memcpy(x_out, x.data(), sizeof(double) * n_b);
    if (W_out) std::memcpy(W_out, W.data(), sizeof(double) * n_b);
    if (T_out) {
        std::vector<double> T((size_t)n_b * n_b, 0.0);
        for (int e = 0; e < n_e; ++e) {
            double h = g->bounds[e + 1] - g->bounds[e];
            for (int a = 0; a <= N; ++a) {
                int ka = gidx(e, a);
                if (ka < 0) continue;
                for (int b = 0; b <= N; ++b) {
                    int kb = gidx(e, b);
                    if (kb < 0) continue;
                    // t~_ab = sum_m f_a'(x_m) f_b'(x_m) w_m on the element (Eq. tmat)
                    double t = 0.0;
                    for (int m = 0; m <= N; ++m) t += wr[m] * D[m * (N + 1) + a] * D[m * (N + 1) + b];
                    t *= 2.0 / h;
                    T[(size_t)ka * n_b + kb] += 0.5 * t / std::sqrt(W[ka] * W[kb]);
                }
            }
        }
        std::memcpy(T_out, T.data(), sizeof(double) * T.size());
    }
    if (v_out) {
        for (int k = 0; k < n_b; ++k) {
            double s = 0.0;
            for (int c = 0; c < pot->n_c; ++c) {
                double d = x[k] - pot->X[c];
                s -= pot->Z[c] / std::sqrt(d * d + pot->soft);
            }
            s += 0.5 * pot->omega * pot->omega * x[k] * x[k];          // harmonic confinement
            v_out[k] = s;                                              // Eq. vmat
        }
    }
    if (V_out) {
        for (int a = 0; a < n_b; ++a)
            for (int b = 0; b < n_b; ++b) {
                double d = x[a] - x[b];
                V_out[(size_t)a * n_b + b] = pot->ee_scale / std::sqrt(d * d + pot->ee_soft);
            }
    }
    return NEGF_OK;
}

// ============================================================== density (host)
extern "C" int negf_density_at(const negf_grid_t* g, const double* rho, int sigma, int n_x, const double* xs,
                               double* n_out) {
    NEGF_REQUIRE(g && rho && (n_x == 0 || (xs && n_out)), "NULL argument");
    NEGF_REQUIRE(sigma == 1 || sigma == 2, "sigma must be 1 or 2");
    NEGF_REQUIRE(n_x >= 0, "n_x < 0");
    int n_b = 0;
    NEGF_TRY(negf_fedvr_size(g->n_e, g->n_g, &n_b));
    NEGF_REQUIRE(g->bounds != nullptr, "bounds is NULL");
    for (int e = 0; e < g->n_e; ++e)
        NEGF_REQUIRE(g->bounds[e + 1] > g->bounds[e] && std::isfinite(g->bounds[e + 1]),
                     "element bounds must increase (element %d)", e);
    const int N = g->n_g, n_e = g->n_e;
    std::vector<double> xr, wr, D;
    gll(N, xr, wr, D);
    auto gidx = [&](int e, int m) -> int {
        if (m == 0) return e == 0 ? -1 : e * N - 1;
        if (m == N) return e == n_e - 1 ? -1 : e * N + N - 1;
        return e * N + m - 1;
    };
    std::vector<double> W(n_b, 0.0);
    for (int e = 0; e < n_e; ++e)
        for (int m = 0; m <= N; ++m) {
            const int k = gidx(e, m);
            if (k >= 0) W[k] += 0.5 * wr[m] * (g->bounds[e + 1] - g->bounds[e]);
        }
    std::vector<double> xe(N + 1), chi(N + 1);
    std::vector<int> id(N + 1);
    for (int p = 0; p < n_x; ++p) {
        const double x = xs[p];
        if (!(x >= g->bounds[0] && x <= g->bounds[n_e])) {     // outside the box (Dirichlet)
            n_out[p] = 0.0;
            continue;
        }
        int e = (int)(std::upper_bound(g->bounds, g->bounds + n_e + 1, x) - g->bounds) - 1;
        e = std::min(std::max(e, 0), n_e - 1);
        const double a = g->bounds[e], b = g->bounds[e + 1], h = b - a;
        for (int m = 0; m <= N; ++m) xe[m] = 0.5 * (h * xr[m] + (b + a));
        for (int m = 0; m <= N; ++m) {
            // Lobatto shape function f_m(x) (Sec. 2.1) over the basis normalisation
            double f = 1.0;
            for (int j = 0; j <= N; ++j)
                if (j != m) f *= (x - xe[j]) / (xe[m] - xe[j]);
            id[m] = gidx(e, m);
            chi[m] = id[m] >= 0 ? f / std::sqrt(W[id[m]]) : 0.0;
        }
        double s = 0.0;
        for (int m = 0; m <= N; ++m) {
            if (id[m] < 0) continue;
            for (int k = 0; k <= N; ++k)
                if (id[k] >= 0) s += chi[m] * chi[k] * rho[(size_t)id[m] * n_b + id[k]];
        }
        n_out[p] = sigma * s;
    }
    return NEGF_OK;
}

// ============================================================== tau grids
extern "C" int negf_tau_count(int kind, int M, int u, int p, int* n_tau) {
    NEGF_REQUIRE(n_tau != nullptr, "n_tau is NULL");
    if (kind == NEGF_TAU_UNIFORM) {
        NEGF_REQUIRE(M >= 2 && M % 2 == 0 && M <= (1 << 20), "uniform grid needs even M >= 2 (got %d)", M);
        *n_tau = M + 1;
    } else if (kind == NEGF_TAU_POWER) {
        NEGF_REQUIRE(u >= 4 && p >= 1 && p <= 40 && (long)u * p <= (1 << 19), "power mesh needs u >= 4, 1 <= p <= 40");
        *n_tau = 2 * u * p + 1;
    } else {
        NEGF_REQUIRE(false, "bad tau kind %d", kind);
    }
    return NEGF_OK;
}

extern "C" int negf_tau_grid(int kind, double beta, int M, int u, int p, double* tau) {
    int n = 0;
    NEGF_TRY(negf_tau_count(kind, M, u, p, &n));
    NEGF_REQUIRE(tau != nullptr, "tau is NULL");
    NEGF_REQUIRE(beta > 0 && std::isfinite(beta), "beta must be positive");
    const int half = (n - 1) / 2;
    if (kind == NEGF_TAU_UNIFORM) {
        for (int q = 0; q <= half; ++q) tau[q] = beta * q / M;
    } else {
        // breakpoints beta/2^p, beta/2^(p-1), ..., beta/2 with u steps in each interval
        tau[0] = 0.0;
        int q = 1;
        double lo = 0.0;
        for (int k = 0; k < p; ++k) {
            double hi = beta / std::ldexp(1.0, p - k);
            for (int j = 1; j <= u; ++j) tau[q++] = lo + (hi - lo) * j / u;
            lo = hi;
        }
        tau[half] = 0.5 * beta;
    }
    for (int q = half + 1; q < n; ++q) tau[q] = beta - tau[n - 1 - q];
    return NEGF_OK;
}

// ============================================================== HF / G0
extern "C" int negf_hf(negf_ctx* ctx, int n_b, const double* T, const double* v, const double* V,
                       double n_elec, int sigma, double beta, double tol, int max_iter,
                       double* eps, double* C, double* rho, double* Sigma0, double* mu,
                       double* E_hf, int* iters, void* stream) {
    NEGF_REQUIRE(ctx, "ctx is NULL");
    NEGF_REQUIRE(n_b >= 1 && n_b <= 4096, "n_b = %d out of range [1, 4096]", n_b);
    NEGF_REQUIRE(T && v && V && eps && C && rho && Sigma0, "NULL device buffer");
    NEGF_REQUIRE(sigma == 1 || sigma == 2, "sigma must be 1 or 2");
    NEGF_REQUIRE(n_elec > 0 && n_elec < (double)sigma * n_b, "n_elec must be in (0, sigma n_b)");
    NEGF_REQUIRE(beta > 0 && std::isfinite(beta), "beta must be positive");
    NEGF_REQUIRE(tol > 0, "tol must be positive");
    NEGF_REQUIRE(max_iter >= 1, "max_iter must be >= 1");
    NEGF_TRY(bind_device(ctx));
    return hf_run(ctx, n_b, T, v, V, n_elec, sigma, beta, tol, max_iter, eps, C, rho, Sigma0,
                  mu, E_hf, iters, (hipStream_t)stream);
}

extern "C" int negf_hf_batched(negf_ctx* ctx, int batch, int n_b, const double* T, const double* v,
                               const double* V, double n_elec, int sigma, double beta, double tol, int max_iter,
                               double* eps, double* C, double* rho, double* Sigma0, double* mu, double* E_hf,
                               int* iters, void* stream) {
    NEGF_REQUIRE(ctx, "ctx is NULL");
    NEGF_REQUIRE(batch >= 1 && batch <= 65535, "batch = %d out of range [1, 65535]", batch);
    NEGF_REQUIRE(n_b >= 1 && n_b <= 4096, "n_b = %d out of range [1, 4096]", n_b);
    NEGF_REQUIRE(T && v && V && eps && C && rho && Sigma0, "NULL device buffer");
    NEGF_REQUIRE(sigma == 1 || sigma == 2, "sigma must be 1 or 2");
    NEGF_REQUIRE(n_elec > 0 && n_elec < (double)sigma * n_b, "n_elec must be in (0, sigma n_b)");
    NEGF_REQUIRE(beta > 0 && std::isfinite(beta), "beta must be positive");
    NEGF_REQUIRE(tol > 0, "tol must be positive");
    NEGF_REQUIRE(max_iter >= 1, "max_iter must be >= 1");
    NEGF_TRY(bind_device(ctx));
    return hf_run_batched(ctx, batch, n_b, T, v, V, n_elec, sigma, beta, tol, max_iter, eps, C, rho, Sigma0, mu,
                          E_hf, iters, (hipStream_t)stream);
}

extern "C" int negf_g0_build(negf_ctx* ctx, int n_b, int n_tau, const double* tau, double beta,
                             const double* eps, const double* C, double mu, void* G0, int dtype,
                             void* stream) {
    NEGF_REQUIRE(ctx, "ctx is NULL");
    NEGF_REQUIRE(n_b >= 1 && n_b <= 4096, "n_b out of range");
    NEGF_REQUIRE(n_tau >= 2, "n_tau < 2");
    NEGF_REQUIRE(tau && eps && C && G0, "NULL argument");
    NEGF_REQUIRE(beta > 0, "beta must be positive");
    NEGF_REQUIRE(dtype == NEGF_F64 || dtype == NEGF_F32, "dtype must be NEGF_F64 or NEGF_F32");
    NEGF_TRY(bind_device(ctx));
    if (dtype == NEGF_F64)
        return g0_build<double>(ctx, n_b, n_tau, tau, beta, eps, C, mu, (double*)G0, (hipStream_t)stream);
    return g0_build<float>(ctx, n_b, n_tau, tau, beta, eps, C, mu, (float*)G0, (hipStream_t)stream);
}

// ============================================================== Sigma 2B
extern "C" int negf_sigma2b(negf_ctx* ctx, int n_b, int n_tau, int sigma, const void* V,
                            const void* G, void* Sc, int dtype, void* stream) {
    NEGF_REQUIRE(ctx, "ctx is NULL");
    NEGF_REQUIRE(n_b >= 1 && n_b <= 4096, "n_b = %d out of range [1, 4096]", n_b);
    NEGF_REQUIRE(n_tau >= 2 && n_tau <= (1 << 20), "n_tau = %d out of range", n_tau);
    NEGF_REQUIRE(sigma == 1 || sigma == 2, "sigma must be 1 or 2");
    NEGF_REQUIRE(V && G && Sc, "NULL buffer");
    NEGF_REQUIRE(G != Sc, "Sigma_c must not alias G");
    NEGF_REQUIRE(dtype == NEGF_F64 || dtype == NEGF_F32 || dtype == NEGF_BF16, "bad dtype %d", dtype);
    NEGF_REQUIRE(dtype != NEGF_BF16 || n_tau <= 65535, "n_tau = %d exceeds 65535 slices for NEGF_BF16", n_tau);
    NEGF_TRY(bind_device(ctx));
    hipStream_t st = (hipStream_t)stream;
    if (dtype == NEGF_F64)
        return sigma2b_run<double>(ctx, n_b, n_tau, sigma, (const double*)V, (const double*)G,
                                   (double*)Sc, false, st);
    return sigma2b_run<float>(ctx, n_b, n_tau, sigma, (const float*)V, (const float*)G,
                              (float*)Sc, dtype == NEGF_BF16, st);
}

extern "C" int negf_density(negf_ctx* ctx, int n_b, int n_tau, int sigma, const double* W, const void* G, int dtype,
                            double* n, void* stream) {
    NEGF_REQUIRE(ctx, "ctx is NULL");
    NEGF_REQUIRE(n_b >= 1 && n_b <= 65536, "n_b = %d out of range", n_b);
    NEGF_REQUIRE(n_tau >= 2, "n_tau = %d < 2", n_tau);
    NEGF_REQUIRE(sigma == 1 || sigma == 2, "sigma must be 1 or 2");
    NEGF_REQUIRE(W && G && n, "NULL buffer");
    NEGF_REQUIRE(dtype == NEGF_F64 || dtype == NEGF_F32, "dtype must be NEGF_F64 or NEGF_F32");
    NEGF_TRY(bind_device(ctx));
    if (dtype == NEGF_F64) return density_run<double>(n_b, n_tau, sigma, W, (const double*)G, n, (hipStream_t)stream);
    return density_run<float>(n_b, n_tau, sigma, W, (const float*)G, n, (hipStream_t)stream);
}

extern "C" int negf_sigma2b_noalloc(negf_ctx* ctx, int n_b, int n_tau, int sigma, const void* V, const void* G,
                                    void* Sc, int dtype, void* stream) {
    NEGF_REQUIRE(ctx, "ctx is NULL");
    NEGF_REQUIRE(n_b >= 1 && n_b <= 4096, "n_b = %d out of range [1, 4096]", n_b);
    NEGF_REQUIRE(n_tau >= 2 && n_tau <= NEGF_SIGMA2B_NOALLOC_MAX_TAU,
                 "n_tau = %d out of range [2, %d] for the allocation-free entry", n_tau, NEGF_SIGMA2B_NOALLOC_MAX_TAU);
    NEGF_REQUIRE(sigma == 1 || sigma == 2, "sigma must be 1 or 2");
    NEGF_REQUIRE(V && G && Sc, "NULL buffer");
    NEGF_REQUIRE(G != Sc, "Sigma_c must not alias G");
    NEGF_REQUIRE(dtype == NEGF_F64 || dtype == NEGF_F32,
                 "dtype %d: the allocation-free entry takes NEGF_F64 or NEGF_F32 (bf16 needs a slice copy)", dtype);
    NEGF_TRY(bind_device(ctx));
    hipStream_t st = (hipStream_t)stream;
    if (dtype == NEGF_F64)
        return sigma2b_run_noalloc<double>(ctx, n_b, n_tau, sigma, (const double*)V, (const double*)G, (double*)Sc,
                                           st);
    return sigma2b_run_noalloc<float>(ctx, n_b, n_tau, sigma, (const float*)V, (const float*)G, (float*)Sc, st);
}

extern "C" int negf_sigma2b_tune(negf_ctx* ctx, int n_b, int n_tau, int sigma, const void* V, const void* G,
                                 void* Sc, int dtype, int* best, double* ms, void* stream) {
    NEGF_REQUIRE(ctx, "ctx is NULL");
    NEGF_REQUIRE(n_b >= 1 && n_b <= 4096, "n_b = %d out of range [1, 4096]", n_b);
    NEGF_REQUIRE(n_tau >= 2 && n_tau <= (1 << 20), "n_tau = %d out of range", n_tau);
    NEGF_REQUIRE(sigma == 1 || sigma == 2, "sigma must be 1 or 2");
    NEGF_REQUIRE(V && G && Sc, "NULL buffer");
    NEGF_REQUIRE(G != Sc, "Sigma_c must not alias G");
    NEGF_REQUIRE(dtype == NEGF_F64 || dtype == NEGF_F32 || dtype == NEGF_BF16, "bad dtype %d", dtype);
    NEGF_REQUIRE(dtype != NEGF_BF16 || n_tau <= 65535, "n_tau = %d exceeds 65535 slices for NEGF_BF16", n_tau);
    NEGF_TRY(bind_device(ctx));
    hipStream_t st = (hipStream_t)stream;
    if (dtype == NEGF_F64)
        return sigma2b_tune<double>(ctx, n_b, n_tau, sigma, (const double*)V, (const double*)G, (double*)Sc, false,
                                    best, ms, st);
    return sigma2b_tune<float>(ctx, n_b, n_tau, sigma, (const float*)V, (const float*)G, (float*)Sc,
                               dtype == NEGF_BF16, best, ms, st);
}

namespace {
int check_s2b_batch(negf_ctx* ctx, int batch, const int* n_b, int n_tau, const int* sigma, const void* const* V,
                    const void* const* G, void* const* Sc, int dtype) {
    NEGF_REQUIRE(ctx, "ctx is NULL");
    NEGF_REQUIRE(batch >= 1 && batch <= 65535, "batch = %d out of range [1, 65535]", batch);
    NEGF_REQUIRE(n_b && sigma && V && G && Sc, "NULL argument array");
    NEGF_REQUIRE(n_tau >= 2 && n_tau <= (1 << 20), "n_tau = %d out of range", n_tau);
    NEGF_REQUIRE(dtype == NEGF_F64 || dtype == NEGF_F32 || dtype == NEGF_BF16, "bad dtype %d", dtype);
    NEGF_REQUIRE(dtype != NEGF_BF16 || n_tau <= 65535, "n_tau = %d exceeds 65535 slices for NEGF_BF16", n_tau);
    for (int b = 0; b < batch; ++b) {
        NEGF_REQUIRE(n_b[b] >= 1 && n_b[b] <= 4096, "n_b[%d] = %d out of range [1, 4096]", b, n_b[b]);
        NEGF_REQUIRE(sigma[b] == 1 || sigma[b] == 2, "sigma[%d] must be 1 or 2", b);
        NEGF_REQUIRE(V[b] && G[b] && Sc[b], "NULL buffer for system %d", b);
        NEGF_REQUIRE(G[b] != Sc[b], "Sigma_c must not alias G (system %d)", b);
    }
    return NEGF_OK;
}
}  // namespace

extern "C" int negf_sigma2b_batched(negf_ctx* ctx, int batch, const int* n_b, int n_tau, const int* sigma,
                                    const void* const* V, const void* const* G, void* const* Sc, int dtype,
                                    void* stream) {
    NEGF_TRY(check_s2b_batch(ctx, batch, n_b, n_tau, sigma, V, G, Sc, dtype));
    NEGF_TRY(bind_device(ctx));
    hipStream_t st = (hipStream_t)stream;
    S2BBatch pl;
    NEGF_TRY(s2b_batch_prepare(ctx, "abi", dtype, batch, n_b, n_tau, sigma, V, G, Sc, 0, &pl, st));
    return s2b_batch_launch(pl, st);
}

extern "C" int negf_sigma2b_batched_tune(negf_ctx* ctx, int batch, const int* n_b, int n_tau, const int* sigma,
                                         const void* const* V, const void* const* G, void* const* Sc, int dtype,
                                         int pair_lim, int* best, double* ms, void* stream) {
    NEGF_TRY(check_s2b_batch(ctx, batch, n_b, n_tau, sigma, V, G, Sc, dtype));
    NEGF_REQUIRE(pair_lim >= 0, "pair_lim < 0");
    NEGF_TRY(bind_device(ctx));
    return s2b_batch_tune(ctx, dtype, batch, n_b, n_tau, sigma, V, G, Sc, pair_lim, best, ms, (hipStream_t)stream);
}

extern "C" int negf_sigma2b_batched_set_config(negf_ctx* ctx, int batch, const int* n_b, int dtype, int cfg) {
    NEGF_REQUIRE(ctx && n_b, "NULL argument");
    NEGF_REQUIRE(batch >= 1 && batch <= 65535, "batch = %d out of range [1, 65535]", batch);
    NEGF_REQUIRE(dtype == NEGF_F64 || dtype == NEGF_F32 || dtype == NEGF_BF16, "bad dtype %d", dtype);
    NEGF_REQUIRE(cfg >= 0 && cfg < 11, "tile configuration %d out of range [0, 11)", cfg);
    for (int b = 0; b < batch; ++b) NEGF_REQUIRE(n_b[b] >= 1 && n_b[b] <= 4096, "n_b[%d] out of range", b);
    std::vector<int> ns(n_b, n_b + batch);
    std::sort(ns.begin(), ns.end());
    std::string key = "s2bB_" + std::to_string(dtype == NEGF_F64 ? 0 : (dtype == NEGF_BF16 ? 2 : 1));
    for (int v : ns) key += "_" + std::to_string(v);
    ctx->filled[key] = cfg;
    return NEGF_OK;
}

extern "C" int negf_sigma2b_set_config(negf_ctx* ctx, int n_b, int dtype, int cfg) {
    NEGF_REQUIRE(ctx, "ctx is NULL");
    NEGF_REQUIRE(n_b >= 1 && n_b <= 4096, "n_b = %d out of range [1, 4096]", n_b);
    NEGF_REQUIRE(dtype == NEGF_F64 || dtype == NEGF_F32 || dtype == NEGF_BF16, "bad dtype %d", dtype);
    return sigma2b_set_cfg(ctx, dtype, n_b, cfg);
}

extern "C" int negf_matrix_rate(negf_ctx* ctx, int dtype, double* tflops, double* clock_ghz, void* stream) {
    NEGF_REQUIRE(ctx, "ctx is NULL");
    NEGF_REQUIRE(tflops && clock_ghz, "NULL output");
    NEGF_REQUIRE(dtype == NEGF_F64 || dtype == NEGF_F32 || dtype == NEGF_BF16, "bad dtype %d", dtype);
    NEGF_TRY(bind_device(ctx));
    return matrix_rate(ctx, dtype, tflops, clock_ghz, (hipStream_t)stream);
}

extern "C" int negf_f64_issue_probe(negf_ctx* ctx, int n_mfma, int n_fma, double* ms, double* mfma_tflops,
                                    double* fma_tflops, void* stream) {
    NEGF_REQUIRE(ctx, "ctx is NULL");
    NEGF_REQUIRE(ms && mfma_tflops && fma_tflops, "NULL output");
    NEGF_REQUIRE(n_mfma >= 0 && n_fma >= 0 && n_mfma + n_fma > 0, "bad chain counts (%d, %d)", n_mfma, n_fma);
    NEGF_TRY(bind_device(ctx));
    return issue_probe_f64(ctx, n_mfma, n_fma, ms, mfma_tflops, fma_tflops, (hipStream_t)stream);
}

// ============================================================== Dyson / energy
namespace {
int check_dyson_common(negf_ctx* ctx, const negf_tau_grid_t* tg, int n_b, int sigma, int dtype) {
    NEGF_REQUIRE(ctx, "ctx is NULL");
    NEGF_TRY(check_tau_grid(tg));
    NEGF_REQUIRE(n_b >= 1 && n_b <= 4096, "n_b = %d out of range [1, 4096]", n_b);
    NEGF_REQUIRE(sigma == 1 || sigma == 2, "sigma must be 1 or 2");
    NEGF_REQUIRE(dtype == NEGF_F64 || dtype == NEGF_F32, "dtype must be NEGF_F64 or NEGF_F32");
    return NEGF_OK;
}
}  // namespace

extern "C" int negf_dyson_step(negf_ctx* ctx, const negf_tau_grid_t* tg, int n_b, int sigma,
                               const double* h, const double* V, const double* eps,
                               const double* C, double mu, const double* Sigma0, const void* G_in,
                               const void* Sc, double alpha, int symmetrize, int conv_algo,
                               int dtype, void* G_out, double* E_out, double* N_out, void* stream) {
    NEGF_TRY(check_dyson_common(ctx, tg, n_b, sigma, dtype));
    NEGF_REQUIRE(h && V && eps && C && Sigma0 && G_in && Sc && G_out, "NULL buffer");
    NEGF_REQUIRE(G_out != Sc, "G_out must not alias Sigma_c");
    NEGF_REQUIRE(alpha > 0 && alpha <= 1, "alpha must be in (0, 1]");
    NEGF_REQUIRE(conv_algo == NEGF_CONV_AUTO || conv_algo == NEGF_CONV_FFT || conv_algo == NEGF_CONV_DIRECT,
                 "bad conv_algo");
    if (conv_algo == NEGF_CONV_FFT) {
        const int M = tg->n_tau - 1;
        NEGF_REQUIRE(tg->kind == NEGF_TAU_UNIFORM, "the Fourier route needs a uniform grid");
        NEGF_REQUIRE((M & (M - 1)) == 0 && M >= 2 && M <= 8192, "the Fourier route needs n_tau - 1 a power of two <= 8192");
    }
    NEGF_TRY(bind_device(ctx));
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if (dtype == NEGF_F64) {
        if (E_out || N_out) {
            double E, N;
            NEGF_TRY(energy_run<double>(ctx, tg, n_b, sigma, h, V, (const double*)G_in, (const double*)Sc, &E, &N, st));
            if (E_out) *E_out = E;
            if (N_out) *N_out = N;
            if (!std::isfinite(E) || !std::isfinite(N)) {
                rc = dyson_run<double>(ctx, tg, n_b, sigma, h, V, eps, C, mu, Sigma0, (const double*)G_in,
                                       (const double*)Sc, alpha, symmetrize, conv_algo, (double*)G_out, st);
                set_error("energy or particle number not finite");
                return rc == NEGF_OK ? NEGF_ENAN : rc;
            }
        }
        return dyson_run<double>(ctx, tg, n_b, sigma, h, V, eps, C, mu, Sigma0, (const double*)G_in,
                                 (const double*)Sc, alpha, symmetrize, conv_algo, (double*)G_out, st);
    }
    if (E_out || N_out) {
        double E, N;
        NEGF_TRY(energy_run<float>(ctx, tg, n_b, sigma, h, V, (const float*)G_in, (const float*)Sc, &E, &N, st));
        if (E_out) *E_out = E;
        if (N_out) *N_out = N;
        if (!std::isfinite(E) || !std::isfinite(N)) {
            rc = dyson_run<float>(ctx, tg, n_b, sigma, h, V, eps, C, mu, Sigma0, (const float*)G_in,
                                  (const float*)Sc, alpha, symmetrize, conv_algo, (float*)G_out, st);
            set_error("energy or particle number not finite");
            return rc == NEGF_OK ? NEGF_ENAN : rc;
        }
    }
    return dyson_run<float>(ctx, tg, n_b, sigma, h, V, eps, C, mu, Sigma0, (const float*)G_in,
                            (const float*)Sc, alpha, symmetrize, conv_algo, (float*)G_out, st);
}

extern "C" int negf_energy(negf_ctx* ctx, const negf_tau_grid_t* tg, int n_b, int sigma,
                           const double* h, const double* V, const void* G, const void* Sc,
                           int dtype, double* E_out, double* N_out, void* stream) {
    NEGF_TRY(check_dyson_common(ctx, tg, n_b, sigma, dtype));
    NEGF_REQUIRE(h && V && G && Sc, "NULL buffer");
    NEGF_TRY(bind_device(ctx));
    double E = 0, N = 0;
    hipStream_t st = (hipStream_t)stream;
    if (dtype == NEGF_F64)
        NEGF_TRY(energy_run<double>(ctx, tg, n_b, sigma, h, V, (const double*)G, (const double*)Sc, &E, &N, st));
    else
        NEGF_TRY(energy_run<float>(ctx, tg, n_b, sigma, h, V, (const float*)G, (const float*)Sc, &E, &N, st));
    if (E_out) *E_out = E;
    if (N_out) *N_out = N;
    if (!std::isfinite(E) || !std::isfinite(N)) {
        set_error("energy or particle number not finite");
        return NEGF_ENAN;
    }
    return NEGF_OK;
}
