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
#include <algorithm>
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

// Cyclic Jacobi on a batch of symmetric n x n matrices, one workgroup per
// matrix (blockIdx.x = system; systems with active[b] == 0 are skipped).
// A (overwritten; its diagonal ends up holding the eigenvalues) and Vt, the
// transpose of the accumulated rotation (on entry the transpose of the basis
// to rotate, e.g. the identity). The n/2 pairs of one round are disjoint, so
// A <- J^T A J touches each 2 x 2 block (pair s1, pair s2) independently: one
// thread per block reads its four entries, applies the row and the column
// rotation, and writes them back; Vt <- J^T Vt updates rows of Vt.
__global__ __launch_bounds__(JAC_THREADS) void k_jacobi(int n, long stride, double* Ab, double* Vtb, int max_sweeps,
                                                        double rel_tol, const int* active) {
    if (active && !active[blockIdx.x]) return;
    double* A = Ab + blockIdx.x * stride;
    double* Vt = Vtb + blockIdx.x * stride;
    extern __shared__ double jsm[];
    const int nn = n + (n & 1);          // even number of players (one dummy if n is odd)
    const int npair = nn / 2;
    double* cs = jsm;                    // [npair]
    double* sn = cs + npair;             // [npair]
    int* P = reinterpret_cast<int*>(sn + npair);    // [npair]
    int* Q = P + npair;                  // [npair]
    double* red = reinterpret_cast<double*>(Q + npair);   // 2 npair ints keep 8-byte alignment
    const int tid = threadIdx.x;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        double off = 0.0, all = 0.0;
        for (long e = tid; e < (long)n * n; e += JAC_THREADS) {
            const double a = A[e];
            all += a * a;
            if (e / n != e % n) off += a * a;
        }
        off = block_sum<JAC_THREADS>(off, red);
        all = block_sum<JAC_THREADS>(all, red);
        if (off <= rel_tol * rel_tol * all) break;
        for (int round = 0; round < nn - 1; ++round) {
            for (int s = tid; s < npair; s += JAC_THREADS) {
                // players: position 0 fixed, the others rotate by `round`
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
                }
                cs[s] = c;
                sn[s] = sv;
                P[s] = p;
                Q[s] = q;                 // q == n marks the dummy partner
            }
            __syncthreads();
            for (long e = tid; e < (long)npair * npair; e += JAC_THREADS) {
                const int s1 = (int)(e / npair), s2 = (int)(e % npair);
                const int p1 = P[s1], q1 = Q[s1], p2 = P[s2], q2 = Q[s2];
                const double c1 = cs[s1], t1 = sn[s1], c2 = cs[s2], t2 = sn[s2];
                const bool r1 = q1 < n, r2 = q2 < n;
                const double a = A[(long)p1 * n + p2];
                const double b = r2 ? A[(long)p1 * n + q2] : 0.0;
                const double c = r1 ? A[(long)q1 * n + p2] : 0.0;
                const double d = (r1 && r2) ? A[(long)q1 * n + q2] : 0.0;
                // rows: (p, q) <- (c p - s q, s p + c q)
                const double ra = c1 * a - t1 * c, rb = c1 * b - t1 * d;
                const double rc = t1 * a + c1 * c, rd = t1 * b + c1 * d;
                // columns likewise
                double na = c2 * ra - t2 * rb, nb = t2 * ra + c2 * rb;
                double nc = c2 * rc - t2 * rd, nd = t2 * rc + c2 * rd;
                if (s1 == s2 && t1 != 0.0) { nb = 0.0; nc = 0.0; }
                A[(long)p1 * n + p2] = na;
                if (r2) A[(long)p1 * n + q2] = nb;
                if (r1) A[(long)q1 * n + p2] = nc;
                if (r1 && r2) A[(long)q1 * n + q2] = nd;
            }
            for (long e = tid; e < (long)npair * n; e += JAC_THREADS) {
                const int s = (int)(e / n), i = (int)(e % n);
                const int p = P[s], q = Q[s];
                const double sv = sn[s];
                if (q >= n || sv == 0.0) continue;
                const double c = cs[s];
                const double vp = Vt[(long)p * n + i], vq = Vt[(long)q * n + i];
                Vt[(long)p * n + i] = c * vp - sv * vq;
                Vt[(long)q * n + i] = sv * vp + c * vq;
            }
            __syncthreads();
        }
    }
}

// eps = sorted diagonal of A; C[i][rank(k)] = Vt[k][i] (ascending order, ties by index).
__global__ void k_sort_eig(int n, long stride, const double* Ab, const double* Vtb, double* epsb, double* Cb,
                           const int* active) {
    if (active && !active[blockIdx.x]) return;
    const double* A = Ab + blockIdx.x * stride;
    const double* Vt = Vtb + blockIdx.x * stride;
    double* eps = epsb + (long)blockIdx.x * n;
    double* C = Cb + blockIdx.x * stride;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const double ek = A[(long)k * n + k];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double ej = A[(long)j * n + j];
            if (ej < ek || (ej == ek && j < k)) ++rank;
        }
        eps[rank] = ek;
        for (int i = 0; i < n; ++i) C[(long)i * n + rank] = Vt[(long)k * n + i];
    }
}

// Chemical potential by bisection (one workgroup per system). For integer
// N/sigma = n_occ the excess is sum_{k >= n_occ} f(eps_k - mu) - sum_{k < n_occ}
// f(mu - eps_k), each term accurate even deep in the gap. Also writes f_k.
__global__ __launch_bounds__(256) void k_mu_bisect(int n, const double* epsb, double n_spin, double beta,
                                                   double* mub, double* fb, const int* active) {
    if (active && !active[blockIdx.x]) return;
    const double* eps = epsb + (long)blockIdx.x * n;
    double* f_out = fb + (long)blockIdx.x * n;
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
    if (threadIdx.x == 0) mub[blockIdx.x] = mu;
    for (int k = threadIdx.x; k < n; k += 256) f_out[k] = fermi_d(eps[k] - mu, beta);
}

// F = h + Sigma^HF[rho], h = T + diag(v); grid.y = system
__global__ void k_fock(int n, long stride, const double* Tb, const double* vb, const double* Vb, const double* rhob,
                       int sigma, double* Fb, double* Sigb, const int* active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const double *T = Tb + b * stride, *V = Vb + b * stride, *rho = rhob + b * stride, *v = vb + (long)b * n;
    double *F = Fb + b * stride, *Sig = Sigb + b * stride;
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

// h = T + diag(v); grid.y = system
__global__ void k_core(int n, long stride, const double* Tb, const double* vb, double* hb) {
    const int b = blockIdx.y;
    const double *T = Tb + b * stride, *v = vb + (long)b * n;
    double* h = hb + b * stride;
    const long nn = (long)n * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e % n);
        h[e] = T[e] + (i == j ? v[i] : 0.0);
    }
}

// I (or I^T, the same) per system; grid.y = system
__global__ void k_identity(int n, long stride, double* Ib) {
    double* I = Ib + blockIdx.y * stride;
    const long nn = (long)n * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x)
        I[e] = (e / n == e % n) ? 1.0 : 0.0;
}

// out[2b] = sigma (Tr[h rho] + Tr[Sigma^HF[rho] rho]/2), out[2b+1] = max |rho - rho_old|
__global__ __launch_bounds__(256) void k_hf_energy(int n, long stride, const double* Tb, const double* vb,
                                                   const double* Vb, const double* rhob, const double* rho_oldb,
                                                   int sigma, double* out) {
    const int b = blockIdx.x;
    const double *T = Tb + b * stride, *V = Vb + b * stride, *rho = rhob + b * stride, *v = vb + (long)b * n;
    const double* rho_old = rho_oldb ? rho_oldb + b * stride : nullptr;
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
        out[2 * b] = sigma * (e1 + 0.5 * e2);
        out[2 * b + 1] = mred[0];
    }
}

// Pulay (DIIS) error of a Fock matrix F built from rho: E = F rho - rho F,
// which vanishes at self-consistency (rho is a function of F). With P = F rho,
// rho F = P^T for symmetric F and rho, so E = P - P^T; grid.y = system.
__global__ void k_comm_err(int n, long stride, const double* Pb, double* Eb, const int* active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const double* P = Pb + b * stride;
    double* E = Eb + b * stride;
    const long nn = (long)n * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e % n);
        E[e] = P[e] - P[(long)j * n + i];
    }
}

// DIIS history [M][B][nn]: dots[b M + k] = <E_slot, E_k> for k < nh; grid (nh, B).
__global__ __launch_bounds__(256) void k_diis_dots(long nn, int B, int M, const double* Eh, int slot, double* dots,
                                                   const int* active) {
    const int k = blockIdx.x, b = blockIdx.y;
    if (active && !active[b]) return;
    const double* En = Eh + ((long)slot * B + b) * nn;
    const double* Ek = Eh + ((long)k * B + b) * nn;
    __shared__ double red[256 / 64 + 1];
    double s = 0.0;
    for (long e = threadIdx.x; e < nn; e += 256) s += En[e] * Ek[e];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) dots[(long)b * M + k] = s;
}

// F[b] = sum over k < nh of c[b M + k] Fh[k][b]; grid.y = system.
__global__ void k_diis_combine(long nn, int B, int M, int nh, const double* Fh, const double* c, double* Fb,
                               const int* active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    double* F = Fb + b * nn;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int k = 0; k < nh; ++k) v += c[(long)b * M + k] * Fh[((long)k * B + b) * nn + e];
        F[e] = v;
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

// out[b] = in[b]^T for B square n x n matrices
__global__ void k_transpose(int n, long stride, const double* in, double* out) {
    const double* a = in + blockIdx.y * stride;
    double* o = out + blockIdx.y * stride;
    const long nn = (long)n * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x)
        o[(e % n) * n + e / n] = a[e];
}

// Pulay coefficients over q history entries (indices idx[0..q), Gram matrix
// gram[i * M + j] = <E_i, E_j>): minimise |sum c_k E_k| subject to sum c_k = 1,
// i.e. [G 1; 1^T 0] [c; l] = [0; 1], by Gaussian elimination with partial
// pivoting on the Gram matrix scaled by its largest diagonal entry. Returns
// false if the system is singular to working precision.
bool diis_solve(int q, const int* idx, const double* gram, int M, double* c) {
    double a[8][9];
    const int m = q + 1;
    double scale = 0.0;
    for (int i = 0; i < q; ++i) scale = std::max(scale, std::fabs(gram[idx[i] * M + idx[i]]));
    if (!(scale > 0.0) || !std::isfinite(scale)) return false;
    for (int i = 0; i < q; ++i) {
        for (int j = 0; j < q; ++j) a[i][j] = gram[idx[i] * M + idx[j]] / scale;
        a[i][q] = 1.0;
        a[i][m] = 0.0;
    }
    for (int j = 0; j < q; ++j) a[q][j] = 1.0;
    a[q][q] = 0.0;
    a[q][m] = 1.0;
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int r = col + 1; r < m; ++r)
            if (std::fabs(a[r][col]) > std::fabs(a[piv][col])) piv = r;
        if (std::fabs(a[piv][col]) < 1e-14) return false;
        if (piv != col)
            for (int k = 0; k <= m; ++k) std::swap(a[piv][k], a[col][k]);
        for (int r = col + 1; r < m; ++r) {
            const double f = a[r][col] / a[col][col];
            for (int k = col; k <= m; ++k) a[r][k] -= f * a[col][k];
        }
    }
    double x[8];
    for (int r = m - 1; r >= 0; --r) {
        double v = a[r][m];
        for (int k = r + 1; k < m; ++k) v -= a[r][k] * x[k];
        x[r] = v / a[r][r];
    }
    for (int i = 0; i < q; ++i) {
        if (!std::isfinite(x[i])) return false;
        c[i] = x[i];
    }
    return true;
}

int transpose_batched(const double* in, double* out, int n, int B, hipStream_t st) {
    const long nn = (long)n * n;
    const unsigned g = grid_for(nn) > 256 ? 256 : grid_for(nn);
    hipLaunchKernelGGL(k_transpose, dim3(g, B), dim3(256), 0, st, n, nn, in, out);
    LAUNCH_CHECK();
    return NEGF_OK;
}

}  // namespace

// ============================================================== HF driver
// B systems of the same size n, stored with stride n*n (vectors with stride n),
// iterated in lockstep; a system stops changing once its own test passes.
int hf_run_batched(negf_ctx* ctx, int B, int n, const double* T, const double* v, const double* V, double n_elec,
                   int sigma, double beta, double tol, int max_iter, double* eps, double* C, double* rho,
                   double* Sigma0, double* mu_out, double* E_out, int* iters_out, hipStream_t st,
                   int* converged) {
    const long nn = (long)n * n;
    double *A, *Vt, *F, *Cp, *tmp, *f, *rho_old, *dmu, *dres;
    int* dact;
    NEGF_TRY(scratch_t(ctx, "hf_A", nn * B, &A));
    NEGF_TRY(scratch_t(ctx, "hf_Vt", nn * B, &Vt));
    NEGF_TRY(scratch_t(ctx, "hf_F", nn * B, &F));
    NEGF_TRY(scratch_t(ctx, "hf_Cp", nn * B, &Cp));
    NEGF_TRY(scratch_t(ctx, "hf_tmp", nn * B, &tmp));
    NEGF_TRY(scratch_t(ctx, "hf_f", (size_t)n * B, &f));
    NEGF_TRY(scratch_t(ctx, "hf_rho_old", nn * B, &rho_old));
    NEGF_TRY(scratch_t(ctx, "hf_mu", B, &dmu));
    NEGF_TRY(scratch_t(ctx, "hf_res", 2 * B, &dres));
    NEGF_TRY(scratch_t(ctx, "hf_act", B, &dact));
    // Pulay (DIIS) extrapolation of the Fock matrix over the last DIIS_M
    // iterations: same fixed point as the plain iteration, fewer iterations.
    // A system uses it while its last density change exceeds DIIS_OFF; the
    // iterations after that are plain, so the returned eigenpairs are those of
    // h + Sigma0 exactly as in the plain iteration.
    constexpr int DIIS_M = 6;
    constexpr double DIIS_OFF = 1e-9;
    double *Fh, *Eh, *ddots, *dcoef;
    NEGF_TRY(scratch_t(ctx, "hf_diis_F", (size_t)DIIS_M * nn * B, &Fh));
    NEGF_TRY(scratch_t(ctx, "hf_diis_E", (size_t)DIIS_M * nn * B, &Eh));
    NEGF_TRY(scratch_t(ctx, "hf_diis_dots", (size_t)DIIS_M * B, &ddots));
    NEGF_TRY(scratch_t(ctx, "hf_diis_c", (size_t)DIIS_M * B, &dcoef));
    std::vector<double> gram((size_t)B * DIIS_M * DIIS_M, 0.0), hdots((size_t)DIIS_M * B), hcoef((size_t)DIIS_M * B);
    std::vector<int> act(B, 1), its(B, max_iter);
    std::vector<double> E(B, 0.0), E_old(B, INFINITY), hres(2 * B), dlast(B, INFINITY);
    HIP_TRY(hipMemcpyAsync(dact, act.data(), sizeof(int) * B, hipMemcpyHostToDevice, st));

    const int npair = (n + 1) / 2;
    const size_t jsm = sizeof(double) * 2 * npair + sizeof(int) * 2 * npair + sizeof(double) * (JAC_THREADS / 64 + 2);
    const double n_spin = n_elec / sigma;
    const dim3 g2(grid_for(nn) > 256 ? 256 : grid_for(nn), B);

    // eigen-decomposition of the symmetric Mx (per system) into (eps, C); warm start from Cprev
    // Jacobi tolerance on the relative off-diagonal norm: loose while the density
    // still changes (an exact eigenbasis of a Fock matrix that is itself far from
    // converged buys nothing), 1e-4 x the last density change once it is small,
    // never tighter than 1e-15; the iterations that decide convergence run tight
    double jac_tol = 1e-8;
    auto eig = [&](const double* Mx, const double* Cprev) -> int {
        if (Cprev) {
            // A = Cprev^T M Cprev, Vt = Cprev^T
            NEGF_TRY(gemm<double>(st, true, false, n, n, n, 1.0, Cprev, n, nn, Mx, n, nn, 0.0, nullptr, 0, 0, tmp, n,
                                  nn, B));
            NEGF_TRY(gemm<double>(st, false, false, n, n, n, 1.0, tmp, n, nn, Cprev, n, nn, 0.0, nullptr, 0, 0, A, n,
                                  nn, B));
            NEGF_TRY(transpose_batched(Cprev, Vt, n, B, st));
        } else {
            HIP_TRY(hipMemcpyAsync(A, Mx, sizeof(double) * nn * B, hipMemcpyDeviceToDevice, st));
            hipLaunchKernelGGL(k_identity, g2, dim3(256), 0, st, n, nn, Vt);
            LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_jacobi, dim3(B), dim3(JAC_THREADS), jsm, st, n, nn, A, Vt, 60, jac_tol, dact);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sort_eig, dim3(B), dim3(256), 0, st, n, nn, A, Vt, eps, C, dact);
        LAUNCH_CHECK();
        return NEGF_OK;
    };
    auto density = [&]() -> int {
        hipLaunchKernelGGL(k_mu_bisect, dim3(B), dim3(256), 0, st, n, eps, n_spin, beta, dmu, f, dact);
        LAUNCH_CHECK();
        // rho = C diag(f) C^T
        return gemm<double>(st, false, true, n, n, n, 1.0, C, n, nn, C, n, nn, 0.0, nullptr, 0, 0, rho, n, nn, B, f, n);
    };

    hipLaunchKernelGGL(k_core, g2, dim3(256), 0, st, n, nn, T, v, F);
    LAUNCH_CHECK();
    NEGF_TRY(eig(F, nullptr));
    NEGF_TRY(density());
    int it = 0, n_active = B;
    for (it = 1; it <= max_iter && n_active > 0; ++it) {
        hipLaunchKernelGGL(k_fock, g2, dim3(256), 0, st, n, nn, T, v, V, rho, sigma, F, Sigma0, dact);
        LAUNCH_CHECK();
        {
            // DIIS: store F and its error F rho - rho F in slot (it - 1) mod DIIS_M,
            // form the new row of each system's Gram matrix, then replace F by the
            // combination of the stored ones whose error combination is smallest
            const int slot = (it - 1) % DIIS_M, nh = std::min(it, DIIS_M);
            double* Fs = Fh + (long)slot * B * nn;
            double* Es = Eh + (long)slot * B * nn;
            HIP_TRY(hipMemcpyAsync(Fs, F, sizeof(double) * nn * B, hipMemcpyDeviceToDevice, st));
            NEGF_TRY(gemm<double>(st, false, false, n, n, n, 1.0, F, n, nn, rho, n, nn, 0.0, nullptr, 0, 0, tmp, n, nn,
                                  B));
            hipLaunchKernelGGL(k_comm_err, g2, dim3(256), 0, st, n, nn, tmp, Es, dact);
            LAUNCH_CHECK();
            hipLaunchKernelGGL(k_diis_dots, dim3(nh, B), dim3(256), 0, st, nn, B, DIIS_M, Eh, slot, ddots, dact);
            LAUNCH_CHECK();
            HIP_TRY(hipMemcpyAsync(hdots.data(), ddots, sizeof(double) * DIIS_M * B, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            bool any = false;                          // some system extrapolates
            for (int b = 0; b < B; ++b) {
                double* gb = gram.data() + (size_t)b * DIIS_M * DIIS_M;
                double* cb = hcoef.data() + (size_t)b * DIIS_M;
                std::fill(cb, cb + DIIS_M, 0.0);
                cb[slot] = 1.0;
                if (!act[b]) continue;
                for (int k = 0; k < nh; ++k) gb[slot * DIIS_M + k] = gb[k * DIIS_M + slot] = hdots[(size_t)b * DIIS_M + k];
                if (!(dlast[b] > DIIS_OFF)) continue;
                // the newest q entries; fewer if the Gram system is singular
                for (int q = nh; q >= 2; --q) {
                    int idx[DIIS_M];
                    double cq[DIIS_M];
                    for (int t = 0; t < q; ++t) idx[t] = (slot - t + DIIS_M) % DIIS_M;
                    if (diis_solve(q, idx, gb, DIIS_M, cq)) {
                        cb[slot] = 0.0;
                        for (int t = 0; t < q; ++t) cb[idx[t]] = cq[t];
                        any = true;
                        break;
                    }
                }
            }
            if (any) {
                HIP_TRY(hipMemcpyAsync(dcoef, hcoef.data(), sizeof(double) * DIIS_M * B, hipMemcpyHostToDevice, st));
                hipLaunchKernelGGL(k_diis_combine, g2, dim3(256), 0, st, nn, B, DIIS_M, nh, Fh, dcoef, F, dact);
                LAUNCH_CHECK();
            }
        }
        HIP_TRY(hipMemcpyAsync(Cp, C, sizeof(double) * nn * B, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(rho_old, rho, sizeof(double) * nn * B, hipMemcpyDeviceToDevice, st));
        NEGF_TRY(eig(F, Cp));
        NEGF_TRY(density());
        hipLaunchKernelGGL(k_hf_energy, dim3(B), dim3(256), 0, st, n, nn, T, v, V, rho, rho_old, sigma, dres);
        LAUNCH_CHECK();
        HIP_TRY(hipMemcpyAsync(hres.data(), dres, sizeof(double) * 2 * B, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        bool changed = false;
        double d_min = INFINITY;                   // smallest density change among active systems
        for (int b = 0; b < B; ++b)
            if (act[b]) d_min = std::min(d_min, hres[2 * b + 1]);
        if (std::isfinite(d_min)) jac_tol = std::max(1e-15, std::min(1e-8, 1e-4 * d_min));
        for (int b = 0; b < B; ++b) {
            if (!act[b]) continue;
            dlast[b] = hres[2 * b + 1];
            E[b] = hres[2 * b];
            if (!std::isfinite(E[b])) {
                set_error("HF energy not finite at iteration %d (system %d)", it, b);
                return NEGF_ENAN;
            }
            if (std::fabs(E[b] - E_old[b]) < tol && hres[2 * b + 1] < 10.0 * tol) {
                act[b] = 0;
                its[b] = it;
                --n_active;
                changed = true;
            }
            E_old[b] = E[b];
        }
        if (changed) HIP_TRY(hipMemcpyAsync(dact, act.data(), sizeof(int) * B, hipMemcpyHostToDevice, st));
    }
    std::vector<double> hmu(B);
    HIP_TRY(hipMemcpyAsync(hmu.data(), dmu, sizeof(double) * B, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int b = 0; b < B; ++b) {
        if (mu_out) mu_out[b] = hmu[b];
        if (E_out) E_out[b] = E[b];
        if (iters_out) iters_out[b] = its[b];
        if (converged) converged[b] = act[b] ? 0 : 1;
    }
    if (n_active > 0) {
        set_error("HF not converged after %d iterations for %d system(s) (|dE| tol %g)", max_iter, n_active, tol);
        return NEGF_ENOCONV;
    }
    return NEGF_OK;
}

int hf_run(negf_ctx* ctx, int n, const double* T, const double* v, const double* V, double n_elec, int sigma,
           double beta, double tol, int max_iter, double* eps, double* C, double* rho, double* Sigma0, double* mu_out,
           double* E_out, int* iters_out, hipStream_t st) {
    return hf_run_batched(ctx, 1, n, T, v, V, n_elec, sigma, beta, tol, max_iter, eps, C, rho, Sigma0, mu_out, E_out,
                          iters_out, st);
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
