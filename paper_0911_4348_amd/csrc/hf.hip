// Hartree-Fock ground state on the GPU in float64 (paper Sec. 2.3, Eqs.
// sigmahf, hamhf, hfgf) and the HF Green's function on the tau grid.
//
//   Sigma^HF_ij = delta_ij sigma sum_k V_ik rho_kk - V_ij rho_ij
//   F = h + Sigma^HF[rho];  F C = C diag(eps);  sum_k f(eps_k - mu) = N / sigma
//   rho = C diag(f) C^T;    E = sigma (Tr[h rho] + Tr[Sigma^HF[rho] rho] / 2)
//   G0(tau) = -C diag((1 - f_k) e^(-tau xi_k)) C^T,  xi = eps - mu
//
// The eigensolver is a two-sided cyclic Jacobi method with round-robin pair
// ordering, run by one workgroup per matrix; from the second HF iteration on
// it starts from the previous eigenvectors (F is then nearly diagonal in that
// basis and a few sweeps suffice).
#include <cmath>
#include <vector>

#include "common.h"
#include "mfma.h"

namespace negf {
namespace {

constexpr int JAC_THREADS = 1024;

__device__ __forceinline__ double fermi_d(double x, double beta) {
    if (x > 0) {
        const double e = exp(-beta * x);
        return e / (1.0 + e);
    }
    return 1.0 / (1.0 + exp(beta * x));
}

// Block-wide sum (deterministic order) for blockDim.x = NT, NT a multiple of 64.
template <int NT>
__device__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int k = 0; k < NT / 64; ++k) s += red[k];
        red[NT / 64] = s;
    }
    __syncthreads();
    return red[NT / 64];
}

// Cyclic Jacobi on the symmetric n x n matrix A (overwritten; its diagonal ends
// up holding the eigenvalues); Vv accumulates the rotations (on entry the
// basis to rotate, e.g. the identity). Pairs of one round are disjoint, so
// their rotations are applied together: first to rows, then to columns.
__global__ __launch_bounds__(JAC_THREADS) void k_jacobi(int n, double* A, double* Vv, int max_sweeps,
                                                        double rel_tol, int* sweeps_out) {
    extern __shared__ double jsm[];
    const int nn = n + (n & 1);          // even number of players (one dummy if n is odd)
    const int npair = nn / 2;
    double* cs = jsm;                    // [npair]
    double* sn = cs + npair;             // [npair]
    int* P = reinterpret_cast<int*>(sn + npair);    // [npair]
    int* Q = P + npair;                  // [npair]
    double* red = reinterpret_cast<double*>(Q + npair);   // 2 npair ints keep 8-byte alignment
    const int tid = threadIdx.x;
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        // convergence test: off-diagonal norm against the whole norm
        double off = 0.0, all = 0.0;
        for (long e = tid; e < (long)n * n; e += JAC_THREADS) {
            const double a = A[e];
            const long r = e / n, c = e % n;
            all += a * a;
            if (r != c) off += a * a;
        }
        off = block_sum<JAC_THREADS>(off, red);
        all = block_sum<JAC_THREADS>(all, red);
        if (off <= rel_tol * rel_tol * all) break;
        for (int round = 0; round < nn - 1; ++round) {
            // players: position 0 fixed, the others rotate by `round`
            for (int s = tid; s < npair; s += JAC_THREADS) {
                auto player = [&](int pos) { return pos == 0 ? 0 : ((pos - 1 + round) % (nn - 1)) + 1; };
                int p = player(s), q = player(nn - 1 - s);
                if (p > q) { int t = p; p = q; q = t; }
                double c = 1.0, sv = 0.0;
                if (q < n) {
                    const double apq = A[(long)p * n + q];
                    if (apq != 0.0) {
                        const double app = A[(long)p * n + p], aqq = A[(long)q * n + q];
                        const double theta = (aqq - app) / (2.0 * apq);
                        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        sv = t * c;
                    }
                } else {
                    p = q = -1;
                }
                cs[s] = c;
                sn[s] = sv;
                P[s] = p;
                Q[s] = q;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (long e = tid; e < (long)npair * n; e += JAC_THREADS) {
                const int s = (int)(e / n), j = (int)(e % n);
                const int p = P[s], q = Q[s];
                if (p < 0 || sn[s] == 0.0) continue;
                const double c = cs[s], sv = sn[s];
                const double ap = A[(long)p * n + j], aq = A[(long)q * n + j];
                A[(long)p * n + j] = c * ap - sv * aq;
                A[(long)q * n + j] = sv * ap + c * aq;
            }
            __syncthreads();
            // columns: A <- A J, Vv <- Vv J
            for (long e = tid; e < (long)npair * n; e += JAC_THREADS) {
                const int s = (int)(e / n), i = (int)(e % n);
                const int p = P[s], q = Q[s];
                if (p < 0 || sn[s] == 0.0) continue;
                const double c = cs[s], sv = sn[s];
                const double ap = A[(long)i * n + p], aq = A[(long)i * n + q];
                A[(long)i * n + p] = c * ap - sv * aq;
                A[(long)i * n + q] = sv * ap + c * aq;
                const double vp = Vv[(long)i * n + p], vq = Vv[(long)i * n + q];
                Vv[(long)i * n + p] = c * vp - sv * vq;
                Vv[(long)i * n + q] = sv * vp + c * vq;
            }
            __syncthreads();
            for (int s = tid; s < npair; s += JAC_THREADS) {
                const int p = P[s], q = Q[s];
                if (p >= 0 && sn[s] != 0.0) {
                    A[(long)p * n + q] = 0.0;
                    A[(long)q * n + p] = 0.0;
                }
            }
            __syncthreads();
        }
    }
    if (tid == 0 && sweeps_out) *sweeps_out = sweep;
}

// eps = sorted diagonal of A; C = the matching columns of Vv (ascending order,
// ties by index).
__global__ void k_sort_eig(int n, const double* A, const double* Vv, double* eps, double* C) {
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const double ek = A[(long)k * n + k];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double ej = A[(long)j * n + j];
            if (ej < ek || (ej == ek && j < k)) ++rank;
        }
        eps[rank] = ek;
        for (int i = 0; i < n; ++i) C[(long)i * n + rank] = Vv[(long)i * n + k];
    }
}

// Chemical potential by bisection (one workgroup). For integer N/sigma = n_occ
// the excess is sum_{k >= n_occ} f(eps_k - mu) - sum_{k < n_occ} f(mu - eps_k),
// each term accurate even deep in the gap. Also writes f_k.
__global__ __launch_bounds__(256) void k_mu_bisect(int n, const double* eps, double n_spin, double beta,
                                                   double* mu_out, double* f_out) {
    __shared__ double red[256 / 64 + 1];
    const int n_occ = (int)floor(n_spin + 0.5);
    const bool integer = fabs(n_spin - n_occ) < 1e-12 && n_occ >= 0 && n_occ <= n;
    double lo = eps[0] - 50.0 / beta, hi = eps[n - 1] + 50.0 / beta;
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double s = 0.0;
        for (int k = threadIdx.x; k < n; k += 256) {
            if (integer) s += (k >= n_occ) ? fermi_d(eps[k] - mid, beta) : -fermi_d(mid - eps[k], beta);
            else s += fermi_d(eps[k] - mid, beta);
        }
        s = block_sum<256>(s, red);
        const double g = integer ? s : s - n_spin;
        if (g > 0.0) hi = mid;
        else lo = mid;
    }
    const double mu = 0.5 * (lo + hi);
    if (threadIdx.x == 0) *mu_out = mu;
    for (int k = threadIdx.x; k < n; k += 256) f_out[k] = fermi_d(eps[k] - mu, beta);
}

// F = h + Sigma^HF[rho], h = T + diag(v)
__global__ void k_fock(int n, const double* T, const double* v, const double* V, const double* rho,
                       int sigma, double* F, double* Sig) {
    const long nn = (long)n * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e % n);
        double s = -V[e] * rho[e];
        if (i == j) {
            double h = 0.0;
            for (int k = 0; k < n; ++k) h += V[(long)i * n + k] * rho[(long)k * n + k];
            s += sigma * h;
        }
        Sig[e] = s;
        F[e] = T[e] + (i == j ? v[i] : 0.0) + s;
    }
}

// h = T + diag(v)
__global__ void k_core(int n, const double* T, const double* v, double* h) {
    const long nn = (long)n * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e % n);
        h[e] = T[e] + (i == j ? v[i] : 0.0);
    }
}

__global__ void k_identity(int n, double* I) {
    const long nn = (long)n * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x)
        I[e] = (e / n == e % n) ? 1.0 : 0.0;
}

// out[0] = sigma (Tr[h rho] + Tr[Sigma^HF[rho] rho]/2), out[1] = max |rho - rho_old|
__global__ __launch_bounds__(256) void k_hf_energy(int n, const double* T, const double* v, const double* V,
                                                   const double* rho, const double* rho_old, int sigma,
                                                   double* out) {
    __shared__ double red[256 / 64 + 1];
    __shared__ double mred[256];
    double e1 = 0.0, e2 = 0.0, dm = 0.0;
    const long nn = (long)n * n;
    for (long e = threadIdx.x; e < nn; e += 256) {
        const int i = (int)(e / n), j = (int)(e % n);
        const double rji = rho[(long)j * n + i];
        const double h = T[e] + (i == j ? v[i] : 0.0);
        e1 += h * rji;
        // Tr[Sigma^HF rho] = sigma sum_i rho_ii sum_k V_ik rho_kk - sum_ij V_ij rho_ij rho_ji
        e2 += sigma * rho[(long)i * n + i] * V[e] * rho[(long)j * n + j] - V[e] * rho[e] * rji;
        if (rho_old) dm = fmax(dm, fabs(rho[e] - rho_old[e]));
    }
    e1 = block_sum<256>(e1, red);
    e2 = block_sum<256>(e2, red);
    mred[threadIdx.x] = dm;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) mred[threadIdx.x] = fmax(mred[threadIdx.x], mred[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sigma * (e1 + 0.5 * e2);
        out[1] = mred[0];
    }
}

// g[q][k] = (1 - f_k) e^(-tau_q xi_k) in the form with non-positive exponents
__global__ void k_g0_table(int n, int n_tau, const double* tau, double beta, const double* eps, double mu,
                           double* g) {
    const long tot = (long)n * n_tau;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        const int q = (int)(e / n), k = (int)(e % n);
        const double xi = eps[k] - mu, t = tau[q];
        g[e] = xi >= 0 ? exp(-t * xi) / (1.0 + exp(-beta * xi)) : exp((beta - t) * xi) / (1.0 + exp(beta * xi));
    }
}

template <class T>
__global__ void k_g0_scale(long tot, const double* g, T* gs) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x)
        gs[e] = (T)g[e];
}

inline unsigned grid_for(long total) {
    long b = (total + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

// ============================================================== HF driver
int hf_run(negf_ctx* ctx, int n, const double* T, const double* v, const double* V, double n_elec,
           int sigma, double beta, double tol, int max_iter, double* eps, double* C, double* rho,
           double* Sigma0, double* mu_out, double* E_out, int* iters_out, hipStream_t st) {
    const long nn = (long)n * n;
    double *A, *Vv, *F, *Cp, *tmp, *f, *rho_old, *dmu, *dres;
    int* dsw;
    NEGF_TRY(scratch_t(ctx, "hf_A", nn, &A));
    NEGF_TRY(scratch_t(ctx, "hf_V", nn, &Vv));
    NEGF_TRY(scratch_t(ctx, "hf_F", nn, &F));
    NEGF_TRY(scratch_t(ctx, "hf_Cp", nn, &Cp));
    NEGF_TRY(scratch_t(ctx, "hf_tmp", nn, &tmp));
    NEGF_TRY(scratch_t(ctx, "hf_f", n, &f));
    NEGF_TRY(scratch_t(ctx, "hf_rho_old", nn, &rho_old));
    NEGF_TRY(scratch_t(ctx, "hf_small", 8, &dmu));
    dres = dmu + 2;
    NEGF_TRY(scratch_t(ctx, "hf_sw", 4, &dsw));

    const int npair = (n + 1) / 2;
    const size_t jsm = sizeof(double) * 2 * npair + sizeof(int) * 2 * npair +
                       sizeof(double) * (JAC_THREADS / 64 + 2);
    const double n_spin = n_elec / sigma;

    // eigen-decomposition of a symmetric matrix M into (eps, C); warm start from Cprev if given
    auto eig = [&](const double* Mx, const double* Cprev) -> int {
        if (Cprev) {
            // A = Cprev^T M Cprev, Vv = Cprev
            NEGF_TRY(gemm<double>(st, true, false, n, n, n, 1.0, Cprev, n, 0, Mx, n, 0, 0.0, nullptr, 0, 0,
                                  tmp, n, 0, 1));
            NEGF_TRY(gemm<double>(st, false, false, n, n, n, 1.0, tmp, n, 0, Cprev, n, 0, 0.0, nullptr, 0, 0,
                                  A, n, 0, 1));
            HIP_TRY(hipMemcpyAsync(Vv, Cprev, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
        } else {
            HIP_TRY(hipMemcpyAsync(A, Mx, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
            hipLaunchKernelGGL(k_identity, dim3(grid_for(nn)), dim3(256), 0, st, n, Vv);
            LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(JAC_THREADS), jsm, st, n, A, Vv, 60, 1e-15, dsw);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sort_eig, dim3(1), dim3(256), 0, st, n, A, Vv, eps, C);
        LAUNCH_CHECK();
        return NEGF_OK;
    };
    auto density = [&]() -> int {
        hipLaunchKernelGGL(k_mu_bisect, dim3(1), dim3(256), 0, st, n, eps, n_spin, beta, dmu, f);
        LAUNCH_CHECK();
        // rho = C diag(f) C^T
        return gemm<double>(st, false, true, n, n, n, 1.0, C, n, 0, C, n, 0, 0.0, nullptr, 0, 0, rho, n, 0,
                            1, f, 0);
    };

    // start: core Hamiltonian
    hipLaunchKernelGGL(k_core, dim3(grid_for(nn)), dim3(256), 0, st, n, T, v, F);
    LAUNCH_CHECK();
    NEGF_TRY(eig(F, nullptr));
    NEGF_TRY(density());
    double E_old = INFINITY, E = 0.0, dm = 0.0;
    int it = 0;
    bool conv = false;
    for (it = 1; it <= max_iter; ++it) {
        hipLaunchKernelGGL(k_fock, dim3(grid_for(nn)), dim3(256), 0, st, n, T, v, V, rho, sigma, F, Sigma0);
        LAUNCH_CHECK();
        HIP_TRY(hipMemcpyAsync(Cp, C, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(rho_old, rho, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
        NEGF_TRY(eig(F, Cp));
        NEGF_TRY(density());
        hipLaunchKernelGGL(k_hf_energy, dim3(1), dim3(256), 0, st, n, T, v, V, rho, rho_old, sigma, dres);
        LAUNCH_CHECK();
        double hres[2];
        HIP_TRY(hipMemcpyAsync(hres, dres, sizeof(hres), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        E = hres[0];
        dm = hres[1];
        if (!std::isfinite(E)) {
            set_error("HF energy not finite at iteration %d", it);
            return NEGF_ENAN;
        }
        if (std::fabs(E - E_old) < tol && dm < 10.0 * tol) {
            conv = true;
            break;
        }
        E_old = E;
    }
    if (it > max_iter) it = max_iter;
    double hmu = 0.0;
    HIP_TRY(hipMemcpyAsync(&hmu, dmu, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (mu_out) *mu_out = hmu;
    if (E_out) *E_out = E;
    if (iters_out) *iters_out = it;
    if (!conv) {
        set_error("HF not converged after %d iterations (|dE| tol %g)", max_iter, tol);
        return NEGF_ENOCONV;
    }
    return NEGF_OK;
}

template <class T>
int g0_build(negf_ctx* ctx, int n, int n_tau, const double* tau_host, double beta, const double* eps,
             const double* C, double mu, T* G0, hipStream_t st) {
    double *dtau, *g;
    NEGF_TRY(scratch_t(ctx, "g0_tau", n_tau, &dtau));
    NEGF_TRY(scratch_t(ctx, "g0_tab", (size_t)n * n_tau, &g));
    HIP_TRY(hipMemcpyAsync(dtau, tau_host, sizeof(double) * n_tau, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_g0_table, dim3(grid_for((long)n * n_tau)), dim3(256), 0, st, n, n_tau, dtau, beta,
                       eps, mu, g);
    LAUNCH_CHECK();
    const long nn = (long)n * n;
    if (sizeof(T) == 8) {
        // G0[q] = -C diag(g_q) C^T
        NEGF_TRY(gemm<double>(st, false, true, n, n, n, -1.0, C, n, 0, C, n, 0, 0.0, nullptr, 0, 0,
                              (double*)G0, n, nn, n_tau, g, n));
    } else {
        float *Cf, *gf;
        NEGF_TRY(scratch_t(ctx, "g0_Cf", nn, &Cf));
        NEGF_TRY(scratch_t(ctx, "g0_tabf", (size_t)n * n_tau, &gf));
        NEGF_TRY(to_f32(C, Cf, nn, st));
        hipLaunchKernelGGL((k_g0_scale<float>), dim3(grid_for((long)n * n_tau)), dim3(256), 0, st,
                           (long)n * n_tau, g, gf);
        LAUNCH_CHECK();
        NEGF_TRY(gemm<float>(st, false, true, n, n, n, -1.0f, Cf, n, 0, Cf, n, 0, 0.0f, nullptr, 0, 0,
                             (float*)G0, n, nn, n_tau, gf, n));
    }
    return NEGF_OK;
}

template int g0_build<double>(negf_ctx*, int, int, const double*, double, const double*, const double*,
                              double, double*, hipStream_t);
template int g0_build<float>(negf_ctx*, int, int, const double*, double, const double*, const double*,
                             double, float*, hipStream_t);

}  // namespace negf
