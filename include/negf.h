/*
 * negf.h -- C ABI of the MI355X FE-DVR second-Born ground-state library.
 *
 * The method: Balzer, Bauch, Bonitz, "Finite elements and the discrete
 * variable representation in nonequilibrium Green's function calculations.
 * Atomic and molecular models". Sec. 2.1-2.2 build the FE-DVR basis and the
 * one- and two-body matrices; Sec. 2.3 gives the HF and second-Born
 * self-energies (Eqs. sigmahf, sigma2ndb), the HF Green's function (Eqs.
 * hamhf, hfgf) and the Matsubara Dyson equation (Eq. deq).
 *
 * Conventions shared by every call
 *   - Status: every call returns NEGF_OK (0) or a negative NEGF_E* code; on
 *     error negf_last_error() returns a message (thread-local, valid until the
 *     next call on the same thread). No C++ exception crosses the ABI.
 *   - Arguments are validated on the host before any device work; an invalid
 *     argument returns NEGF_EINVAL and launches nothing.
 *   - Ownership: the caller owns every buffer passed in. The library never
 *     frees caller memory. Scratch memory belongs to a negf_ctx and lives until
 *     negf_ctx_destroy.
 *   - Device pointers ("dev") must be device memory of the context's GPU; host
 *     pointers ("host") ordinary host memory.
 *   - stream: a hipStream_t (NULL = the default stream). Calls that only write
 *     device outputs are stream-ordered and asynchronous; calls that return
 *     host scalars synchronise the stream before returning.
 *   - Layouts are row-major. An n_b x n_b matrix A has A[i*n_b + j]. A
 *     tau-resolved tensor is [n_tau][n_b][n_b]; slot 0 holds the value at
 *     tau = 0^+ and slot n_tau-1 the value at tau = beta^-.
 *   - One spin channel is stored; sigma (1 or 2) is the spin degeneracy.
 *     G(tau) = -<T psi(tau) psi^dagger(0)> on [0, beta]; the density matrix is
 *     rho = -G(beta^-) and the particle number N = -sigma Tr G(beta^-).
 *   - Tau grids are symmetric under tau -> beta - tau (slot q pairs with slot
 *     n_tau-1-q); the uniform grid and the power mesh both are.
 *   - The second-Born kernels use G_q^T = G_q: every slice of G must be
 *     symmetric (the Dyson iteration keeps it so).
 */
#ifndef NEGF_H
#define NEGF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define NEGF_OK        0
#define NEGF_EINVAL   -1   /* invalid argument (checked before any device work) */
#define NEGF_ENODEV   -2   /* no usable GPU / wrong device */
#define NEGF_EHIP     -3   /* a HIP runtime call failed */
#define NEGF_ENAN     -4   /* NaN/Inf appeared in an energy or particle number */
#define NEGF_ENOCONV  -5   /* iteration limit reached before the tolerance */
#define NEGF_ENOMEM   -6   /* device allocation failed */

/* ------------------------------------------------------------------ enums */
#define NEGF_F64   0       /* storage and arithmetic in float64 */
#define NEGF_F32   1       /* storage and arithmetic in float32 */
#define NEGF_BF16  2       /* float32 storage; dense products on bf16 MFMA, float32 accumulation */

#define NEGF_TAU_UNIFORM 0 /* M intervals, M+1 points */
#define NEGF_TAU_POWER   1 /* power mesh, 2 u p + 1 points */

#define NEGF_CONV_AUTO   0 /* Fourier route on uniform grids, direct quadrature otherwise */
#define NEGF_CONV_FFT    1 /* antiperiodic DFT route; uniform grids only */
#define NEGF_CONV_DIRECT 2 /* direct split-trapezoid quadrature (any grid) */

const char* negf_last_error(void);
int negf_version(void);

/* ------------------------------------------------------------------ context */
typedef struct negf_ctx negf_ctx;

/* Create a context bound to GPU `device` (scratch buffers, Fourier tables, tuned
 * tile choices, the SCF driver's own stream). *out receives the handle. A context
 * is used by one host thread at a time; calls on it are ordered on the caller's
 * stream. Errors: NEGF_EINVAL (out NULL), NEGF_ENODEV. */
int negf_ctx_create(int device, negf_ctx** out);
/* Release the context's device scratch. NULL is accepted. */
int negf_ctx_destroy(negf_ctx* ctx);
/* Bytes of device scratch currently held by the context. */
int negf_ctx_scratch_bytes(const negf_ctx* ctx, size_t* bytes);

/* ------------------------------------------------------------------ grid */
/* Basis size of n_e elements with n_g basis functions each: n_b = n_e n_g - 1
 * (Sec. 2.1, Eq. basisdim). n_g is the number of generalized Gauss-Lobatto
 * points per element minus one. Errors: NEGF_EINVAL if n_e < 1 or n_g < 2. */
int negf_fedvr_size(int n_e, int n_g, int* n_b);

typedef struct {
    int n_e;                 /* number of finite elements */
    int n_g;                 /* basis functions per element (GLL points - 1) */
    const double* bounds;    /* host, n_e+1 strictly increasing element boundaries */
} negf_grid_t;

typedef struct {
    int n_c;                 /* number of nuclei (0..64) */
    const double* X;         /* host, n_c positions */
    const double* Z;         /* host, n_c charges */
    double soft;             /* v(x) = -sum Z_c / sqrt((x - X_c)^2 + soft) */
    double ee_soft;          /* V(x,x') = ee_scale / sqrt((x - x')^2 + ee_soft) */
    double ee_scale;
    double omega;            /* harmonic confinement: v(x) += omega^2 x^2 / 2 (0: none) */
} negf_potential_t;

/* FE-DVR setup (Sec. 2.1-2.2): GLL nodes and weights per element (Eqs. xim,
 * wim), bridge/element basis with Dirichlet ends (Eq. basis), kinetic matrix
 * (Eq. tmat), diagonal potential (Eq. vmat) and the diagonal-pair interaction
 * kernel V_ab = u(|x_a - x_b|) (Eqs. umat1, umatred).
 * Outputs (host, float64): x[n_b] nodes, W[n_b] summed GLL weights,
 * T[n_b*n_b], v[n_b], V[n_b*n_b]. Any output may be NULL to skip it.
 * Errors: NEGF_EINVAL for bad sizes, non-increasing bounds, soft <= 0. */
int fedvr_build(const negf_grid_t* grid, const negf_potential_t* pot,
                double* x, double* W, double* T, double* v, double* V);

/* Number of stored tau points: M+1 (uniform, M >= 2 even) or 2 u p + 1
 * (power mesh, u >= 4, p >= 1). */
int negf_tau_count(int kind, int M, int u, int p, int* n_tau);
/* Tau points (host, n_tau doubles). Uniform: beta q / M. Power mesh (Sec. 3.1,
 * the cited power mesh): breakpoints 0, beta/2^p, ..., beta/2, each interval
 * split into u equal steps, mirrored about beta/2. Both grids are built as
 * their first half plus its mirror beta - tau, so they are exactly symmetric. */
int negf_tau_grid(int kind, double beta, int M, int u, int p, double* tau);

/* ------------------------------------------------------------------ HF */
/* Self-consistent Hartree-Fock ground state on the GPU in float64 (Sec. 2.3,
 * Eqs. sigmahf, hamhf): F = h + Sigma^HF[rho], F = C diag(eps) C^T by a
 * cyclic Jacobi eigensolver, mu by bisection so that sum_k f(eps_k - mu) =
 * n_elec/sigma, rho = C f C^T; repeated until |dE| < tol and
 * max|d rho| < 10 tol, at most max_iter times. Start: rho of h = T + diag(v).
 * Inputs (dev, float64): T[n_b*n_b], v[n_b], V[n_b*n_b].
 * Outputs (dev, float64): eps[n_b] ascending, C[n_b*n_b] (column k is the
 * eigenvector of eps_k), rho[n_b*n_b], Sigma0[n_b*n_b] = F - h of the last
 * diagonalised F; (host) *mu, *E_hf = sigma(Tr[h rho] + Tr[Sigma^HF[rho] rho]/2),
 * *iters. Synchronises the stream.
 * Errors: NEGF_EINVAL; NEGF_ENOCONV (outputs valid, last iterate); NEGF_ENAN. */
int negf_hf(negf_ctx* ctx, int n_b, const double* T, const double* v, const double* V,
            double n_elec, int sigma, double beta, double tol, int max_iter,
            double* eps, double* C, double* rho, double* Sigma0,
            double* mu, double* E_hf, int* iters, void* stream);

/* The same HF iteration for `batch` systems of equal size n_b at once (one
 * Jacobi workgroup per system), e.g. a family of potentials on one grid.
 * Device arrays are stacked with stride n_b*n_b (matrices) or n_b (vectors):
 * T, v, V, eps, C, rho, Sigma0. Host arrays mu[batch], E_hf[batch],
 * iters[batch] (each may be NULL). Every system keeps iterating until its own
 * stopping rule holds; a converged system is frozen while the others go on,
 * so each result equals what negf_hf returns for that system alone up to
 * rounding. Errors: as negf_hf; NEGF_ENOCONV if any system did not converge
 * (all outputs valid). Synchronises the stream. */
int negf_hf_batched(negf_ctx* ctx, int batch, int n_b, const double* T, const double* v,
                    const double* V, double n_elec, int sigma, double beta, double tol,
                    int max_iter, double* eps, double* C, double* rho, double* Sigma0,
                    double* mu, double* E_hf, int* iters, void* stream);

/* HF Green's function on the tau grid (Eq. hfgf moved to tau > 0):
 * G0(tau_q) = -C diag((1 - f_k) e^(-tau_q xi_k)) C^T, xi = eps - mu, evaluated
 * with non-positive exponents only.
 * tau (host, n_tau); eps, C (dev, float64); G0 (dev, [n_tau][n_b][n_b],
 * float64 or float32 by dtype NEGF_F64 / NEGF_F32). */
int negf_g0_build(negf_ctx* ctx, int n_b, int n_tau, const double* tau, double beta,
                  const double* eps, const double* C, double mu, void* G0, int dtype,
                  void* stream);

/* ------------------------------------------------------------------ density */
/* One-electron density at the DVR nodes (Sec. 2.3: from the equal-time Green's
 * function; Fig. 3b): n(x_a) = -sigma G_aa(beta^-) / W_a, the only basis
 * function non-zero at x_a being chi_a(x_a) = 1/sqrt(W_a).
 * W (dev, float64, n_b) summed GLL weights from fedvr_build; G (dev, dtype
 * NEGF_F64 or NEGF_F32, [n_tau][n_b][n_b]), only its last slice is read;
 * n (dev, float64, n_b) output. Stream-ordered, no synchronisation.
 * Errors: NEGF_EINVAL. */
int negf_density(negf_ctx* ctx, int n_b, int n_tau, int sigma, const double* W, const void* G, int dtype,
                 double* n, void* stream);

/* The density n(x) = sigma sum_ab chi_a(x) chi_b(x) rho_ab at arbitrary points
 * of the box, from the per-spin density matrix rho = -G(beta^-) (host, float64,
 * n_b*n_b) through the Lobatto shape functions of the element holding x
 * (Sec. 2.1, Eq. basis). x (host, n_x) points; n_out (host, n_x); points
 * outside [bounds[0], bounds[n_e]] give 0 (Dirichlet ends). Host computation.
 * Errors: NEGF_EINVAL. */
int negf_density_at(const negf_grid_t* grid, const double* rho, int sigma, int n_x, const double* x,
                    double* n_out);

/* ------------------------------------------------------------------ Sigma 2B */
/* Second-Born correlation self-energy for every tau slice (Sec. 2.3,
 * Eq. sigma2ndb with the interaction lines at equal times):
 *   Sigma_c,ij(tau) = sum_kl V_ik V_jl [sigma G_ij G_kl Gb_lk - G_il Gb_lk G_kj],
 *   Gb = G(beta - tau) = slot n_tau-1-q.
 * The slices q and n_tau-1-q are computed together (they share their
 * intermediate products). Cost: about n_b^4 + 10 n_b^3 flops per slice.
 * V (dev, float64 for NEGF_F64, float32 otherwise) [n_b*n_b], symmetric.
 * G (dev) [n_tau][n_b][n_b], every slice symmetric; Sigma_c (dev, same shape);
 * G and Sigma_c are float64 for NEGF_F64 and float32 for NEGF_F32 / NEGF_BF16.
 * For NEGF_F32 and NEGF_BF16 each slice is scaled by a power of two (so its
 * largest entry lies in [1/2, 1)) and the result unscaled, so no slice
 * underflows before the output. NEGF_BF16 keeps a bf16 copy of the scaled
 * slices in context scratch (n_tau * n_b * 8*ceil(n_b/8) * 2 bytes), written
 * once per call, and takes at most 65535 slices. Sigma_c must not alias G.
 * Errors: NEGF_EINVAL (n_b < 1, n_tau < 2, sigma not 1 or 2, bad dtype, NULL
 * pointers, NEGF_BF16 with n_tau > 65535). */
int negf_sigma2b(negf_ctx* ctx, int n_b, int n_tau, int sigma, const void* V,
                 const void* G, void* Sigma_c, int dtype, void* stream);

/* Largest n_tau accepted by negf_sigma2b_noalloc. */
#define NEGF_SIGMA2B_NOALLOC_MAX_TAU 65536

/* negf_sigma2b for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops that forbid hipMalloc): the same kernels and
 * the same tile configuration as negf_sigma2b, so the same results, but no
 * allocation of any kind. The per-slice exponents of NEGF_F32 go to a fixed
 * device array of NEGF_SIGMA2B_NOALLOC_MAX_TAU ints (256 KiB) that the library
 * holds on every GPU it runs on until the process ends; negf_ctx_create takes
 * its address for the context's device. NEGF_F64 needs no scratch. Every call
 * on one GPU shares that array and overwrites it completely before use, so
 * calls that overlap on one GPU (different streams, different host threads)
 * race and must not be issued. Arguments as for negf_sigma2b; the context's
 * tuned configuration (negf_sigma2b_tune / _set_config) is used if present.
 * Errors: as negf_sigma2b, plus NEGF_EINVAL for n_tau above the limit and for
 * NEGF_BF16 (its slice copy is too large for a fixed array). */
int negf_sigma2b_noalloc(negf_ctx* ctx, int n_b, int n_tau, int sigma, const void* V,
                         const void* G, void* Sigma_c, int dtype, void* stream);

/* Autotuner for negf_sigma2b: times each of its tile configurations (values of i
 * per workgroup x column-chunk width) on the given input and stores the fastest
 * for (dtype, n_b) in the context; later negf_sigma2b calls with that dtype and
 * n_b use it. Arguments as for negf_sigma2b (Sigma_c is overwritten). *best
 * (host, nullable) receives the chosen index, ms (host, nullable, 13 entries) the
 * measured times (-1 for a configuration that does not fit or does not exist
 * for this dtype). Synchronises. */
int negf_sigma2b_tune(negf_ctx* ctx, int n_b, int n_tau, int sigma, const void* V,
                      const void* G, void* Sigma_c, int dtype, int* best, double* ms, void* stream);

/* Pin the negf_sigma2b tile configuration for (dtype, n_b) in this context:
 * 0..3 = (8 or 4 values of i per workgroup) x (208- or 112-column chunks) with
 * single-buffered k-panels; 4, 5 = 8 x 112 and 8 x 208 with double-buffered
 * k-panels; 6, 7 (NEGF_F32 and NEGF_BF16 only) = 4 waves with two values of i
 * each x 112- or 64-column chunks; 8, 9, 10 (NEGF_F64 only) = float64 vector-ALU
 * tiles: 8 waves x 40 x 40 blocks of M^(i), 4 waves with two values of i each x
 * 40 x 40 or 32 x 32 blocks; 11, 12 (NEGF_F64 only) = 208-column chunks whose
 * k-panels are staged by direct global-to-LDS loads, double-buffered, from
 * zero-padded copies of G and V kept in context scratch (n_tau * np^2 + np^2
 * doubles, np = n_b rounded up to 16): 11 with 8 values of i and k-panels of
 * 16 (one workgroup per compute unit; n_b <= 240), 12 with 4 values of i and
 * k-panels of 4 (75 KB of LDS at n_b <= 208, two workgroups per compute unit).
 * With an odd n_tau, 11 and 12 split the middle slice (tau = beta/2) over up to
 * 8 parts of its rows l and add the parts in a second kernel; the parts take
 * 2 * 8 * ceil(n_b/IB) * IB * np more doubles of context scratch (IB = 8 or 4).
 * The float64 matrix-core tiles (0-5, 11, 12) run on the four-block 4x4x4
 * float64 MFMA shape. */
int negf_sigma2b_set_config(negf_ctx* ctx, int n_b, int dtype, int cfg);

/* negf_matrix_rate and negf_f64_issue_probe, measurement helpers outside the
 * method, are declared in negf_measure.h. */

/* Sigma-2B (as negf_sigma2b) for `batch` systems of any sizes n_b[b] on one
 * tau grid of n_tau points, in a single persistent kernel launch: work items
 * (system, slice pair, block of rows i) are dealt to per-XCD queues in order of
 * decreasing n_b, each queue an equal share of the flops, and idle workgroups
 * steal from the other queues. n_b, sigma (host, batch ints); V, G, Sigma_c
 * (host arrays of batch device pointers, layouts and element types as
 * negf_sigma2b for `dtype`). Uses the configuration stored by
 * negf_sigma2b_batched_tune for this dtype and multiset of n_b, else the
 * default. Uploads the work list, so it synchronises the stream once.
 * Errors: NEGF_EINVAL (as negf_sigma2b, per system; n_b beyond the LDS budget
 * of the configuration). */
int negf_sigma2b_batched(negf_ctx* ctx, int batch, const int* n_b, int n_tau, const int* sigma,
                         const void* const* V, const void* const* G, void* const* Sigma_c,
                         int dtype, void* stream);

/* Pin the negf_sigma2b_batched tile configuration (0..10, as negf_sigma2b_set_config)
 * for this dtype and multiset of n_b (host, batch ints). */
int negf_sigma2b_batched_set_config(negf_ctx* ctx, int batch, const int* n_b, int dtype, int cfg);

/* Autotuner for negf_sigma2b_batched: times each tile configuration on the
 * first pair_lim slice pairs of every system (0: all pairs), keeps the fastest
 * for this dtype and multiset of n_b. Sigma_c is overwritten (partly). *best,
 * ms[13] (host, nullable) as for negf_sigma2b_tune (configurations 11 and 12 do
 * not exist in the persistent kernel: -1). Synchronises. */
int negf_sigma2b_batched_tune(negf_ctx* ctx, int batch, const int* n_b, int n_tau, const int* sigma,
                              const void* const* V, const void* const* G, void* const* Sigma_c,
                              int dtype, int pair_lim, int* best, double* ms, void* stream);

/* ------------------------------------------------------------------ Dyson */
typedef struct {
    int kind;                /* NEGF_TAU_UNIFORM or NEGF_TAU_POWER */
    int n_tau;               /* number of points */
    int block;               /* power mesh: u (steps per uniform block); 0 for uniform */
    double beta;
    const double* tau;       /* host, n_tau points as from negf_tau_grid */
} negf_tau_grid_t;

/* One step of the Matsubara Dyson equation (Sec. 2.3, Eq. deq) with linear
 * mixing, plus the total energy of the incoming G:
 *   rho = -G(beta^-), St = Sigma^HF[rho] - Sigma0,
 *   I1 = St G + Q[Sigma_c, G],  I2 = Q[G0, I1],  G_new = G0 + I2,
 *   G_out = (1 - alpha) G_in + alpha G_new, then G_out = (G_out + G_out^T)/2
 *   slice by slice if symmetrize.
 * Q is the split trapezoid rule: the tau-bar integral is split at tau_p and
 * each part uses the trapezoid rule on the grid points it covers, with the
 * antiperiodic continuation A(s - beta) = -A(s). G0 enters through its
 * eigen-decomposition (eps, C, mu) exactly; on the power mesh Sigma_c between
 * grid points is 4-point Lagrange-interpolated within its uniform block.
 * conv_algo picks the route for Q[Sigma_c, G] (both give the same sums on
 * uniform grids; NEGF_CONV_FFT needs a uniform grid with n_tau - 1 a power of two).
 * Energy (Galitskii-Migdal, computed in float64 whatever dtype):
 *   E = sigma(Tr[h rho] + Tr[Sigma^HF[rho] rho]/2)
 *       - sigma/2 sum_q w_q Tr[Sigma_c(beta - tau_q) G(tau_q)],
 *   w = trapezoid weights; N = -sigma Tr G(beta^-).
 * Inputs (dev): h = T + diag(v), V, Sigma0, C [n_b*n_b] float64; eps [n_b]
 * float64; G_in, Sigma_c [n_tau][n_b][n_b] in dtype (NEGF_F64 or NEGF_F32).
 * Outputs: G_out (dev, dtype; may alias G_in); *E_out, *N_out (host; either may be
 * NULL). Synchronises the stream when E_out or N_out is non-NULL.
 * Errors: NEGF_EINVAL, NEGF_ENAN (E or N not finite; G_out still written). */
int negf_dyson_step(negf_ctx* ctx, const negf_tau_grid_t* tg, int n_b, int sigma,
                    const double* h, const double* V, const double* eps, const double* C,
                    double mu, const double* Sigma0, const void* G_in, const void* Sigma_c,
                    double alpha, int symmetrize, int conv_algo, int dtype, void* G_out,
                    double* E_out, double* N_out, void* stream);

/* Galitskii-Migdal energy and particle number of (G, Sigma_c) alone, the same
 * formulas as in negf_dyson_step (paper Sec. 2.3): float64 products and
 * compensated (Neumaier) float64 sums in a fixed order, in every dtype.
 * Synchronises. */
int negf_energy(negf_ctx* ctx, const negf_tau_grid_t* tg, int n_b, int sigma,
                const double* h, const double* V, const void* G, const void* Sigma_c,
                int dtype, double* E_out, double* N_out, void* stream);

/* ------------------------------------------------------------------ SCF */
typedef struct {
    negf_grid_t grid;
    negf_potential_t pot;
    double n_elec;           /* electrons (both spins) */
    int sigma;               /* spin degeneracy, 1 or 2 */
    double beta;             /* inverse temperature */
    int tau_kind;            /* NEGF_TAU_UNIFORM / NEGF_TAU_POWER */
    int M;                   /* uniform: intervals */
    int u, p;                /* power mesh */
    double e_nn;             /* constant added once to the total energy */
} negf_system_t;

typedef struct {
    double alpha;            /* linear mixing, (0, 1] */
    double tol;              /* stop when |E_k - E_(k-1)| < tol (Ha) */
    int max_iter;            /* limit on Dyson steps */
    int fixed_iters;         /* > 0: run exactly this many Dyson steps, ignore tol */
    int dtype;               /* NEGF_F64, or NEGF_F32 / NEGF_BF16 for the mixed form */
    int conv_algo;           /* NEGF_CONV_* */
    int symmetrize;          /* 1: symmetrise every iterate */
    double refine_tol;       /* mixed form: after the low-precision loop, float64
                                steps until |dE| < refine_tol (<= 0: tol) */
    double hf_tol;           /* HF stopping rule (<= 0: 1e-13) */
    int hf_max_iter;         /* (<= 0: 1000) */
    const float* guess_params;   /* dev, nullable: start from the learned guess of this
                                    network (negf_mlp_guess on G0, bf16 inference) instead
                                    of G0; a guess whose electron count is off by more than
                                    2%, or whose iteration turns non-finite, is replaced by G0 */
    double guess_scale;      /* its output scale */
    int tune;                /* 1: run the batch tile autotuner first (once per batch shape) */
    int no_graph;            /* 1: launch every iteration directly (no HIP graphs) */
    int progress;            /* 1: one line per iteration on stderr (systems left, max |dE|, ms) */
    int stop_rule;           /* NEGF_STOP_DELTA (0): |E_k - E_(k-1)| < tol;
                                NEGF_STOP_CONTRACTION (1): |d_k| rho / (1 - rho) < tol,
                                d_k = E_k - E_(k-1), rho = max(|d_k / d_(k-1)|,
                                |d_(k-1) / d_(k-2)|) < 1, k >= 3 (or d_k = 0): a bound
                                on |E_k - E_inf| for a geometric tail. The
                                low-precision loop of the mixed form, whose
                                energy changes reach the float32 noise, also
                                ends when |E_k - E_(k-1)| < tol/10; the float64
                                refinement applies the chosen rule alone. */
    int guard;               /* 1: runaway guard (Sec. 3.1, stable N): if E_k or N_k is not
                                finite, |N_k - n_elec| > n_elec / 2, or |dE| grew three
                                times in a row, restart from G0 with alpha halved, at
                                most 3 times per system (steps before a restart count
                                in iters) */
} negf_opts_t;

#define NEGF_STOP_DELTA       0
#define NEGF_STOP_CONTRACTION 1

typedef struct {
    int iter;                /* Dyson steps done before this energy */
    int dtype;               /* arithmetic of the step that produced G_iter */
    double E, dE, N;         /* energy of G_iter, change, particle number */
    double ms;               /* wall time of the iteration (sigma + energy + step) */
} negf_iter_log_t;

/* Whole self-consistent second-Born ground state (Sec. 2.3): fedvr_build,
 * negf_hf, G = G0 (or G_guess), then for k = 0, 1, ...:
 *   Sigma_c = Sigma_2B[G_k]; E_k = E_GM[G_k]; stop if k >= 1 and the
 *   stopping rule holds (opts.stop_rule: |E_k - E_(k-1)| < tol, or the
 *   contraction-aware bound); else G_(k+1) = Dyson step of G_k.
 * Mixed form (dtype F32/BF16): the loop runs in float32 until tol, then
 * float64 steps continue from that G until refine_tol.
 * G_guess (dev, float64, [n_tau][n_b][n_b], nullable) replaces G0 as the start.
 * G_out (dev, float64, nullable) receives the final G; *E_out, *N_out, *iters
 * (host, nullable) the final energy, particle number and number of Dyson steps
 * (all precisions). log (host, nullable) receives up to log_cap records.
 * HF results (host, nullable): hf_E, hf_mu.
 * Errors: NEGF_EINVAL, NEGF_ENOCONV (outputs hold the last iterate), NEGF_ENAN,
 * NEGF_ENOMEM. */
int negf_scf(negf_ctx* ctx, const negf_system_t* sys, const negf_opts_t* opts,
             const double* G_guess, double* G_out, double* E_out, double* N_out,
             int* iters, negf_iter_log_t* log, int log_cap, double* hf_E, double* hf_mu,
             void* stream);

/* The same self-consistent loop for `batch` systems (any n_b, one tau grid:
 * equal tau_kind, beta, M, u, p) at once. HF runs batched over systems of equal
 * n_b. Every iteration evaluates Sigma_2B of all unfinished systems in one
 * persistent kernel launch per arithmetic mode (negf_sigma2b_batched), then
 * their energies, then their Dyson steps; the two segments are recorded as HIP
 * graphs and replayed while the set of unfinished systems is unchanged. Each
 * system stops by its own rule, so its result equals negf_scf on it alone (to
 * rounding: the tile configuration may differ). A batch of one system (what
 * negf_scf runs) with n_b <= 240 evaluates its float64 Sigma_2B with
 * negf_sigma2b's tiles instead: the configuration tuned for (NEGF_F64, n_b) in
 * the context, else configuration 11 (the autotuner then skips float64).
 * systems (host, batch). G_guess, G_out (host arrays of batch device pointers,
 * each float64 [n_tau][n_b][n_b]; the arrays and their entries nullable).
 * E_out, N_out, iters, hf_E, hf_mu, log_n (host, batch entries, nullable);
 * status (host, batch ints, nullable): NEGF_OK, NEGF_ENOCONV, or NEGF_ENAN for a
 * system whose energy became non-finite (it stops there; the others go on).
 * log (host, nullable): batch x log_cap records, system b from b*log_cap; the
 * record's ms is the wall time of the whole batch iteration.
 * Errors: as negf_scf; NEGF_ENAN if any system failed so, else NEGF_ENOCONV if
 * any did not converge (all outputs valid in both cases). Runs on a
 * stream of its own that first waits for `stream`; returns after it finished. */
int negf_scf_batched(negf_ctx* ctx, int batch, const negf_system_t* systems,
                     const negf_opts_t* opts, double* const* G_guess, double* const* G_out,
                     double* E_out, double* N_out, int* iters, int* status, negf_iter_log_t* log,
                     int log_cap, int* log_n, double* hf_E, double* hf_mu, void* stream);

/* ------------------------------------------------------------------ learned initial guess */
/* A tau-resolved float32 MLP predicts dG_ij(tau) = G(tau) - G0(tau) of the converged
 * second-Born G from per-sample features; the guess is G_init = G0 + (dG + dG^T)/2.
 * (Not in the paper: a production pattern around the method; the plain HF start remains
 * the fallback.) Features of a sample (i, j, tau): x_i/10, x_j/10, v(x_i), v(x_j),
 * Chebyshev T_0..T_15(2 tau/beta - 1), Z_1..Z_3, X_1/10..X_3/10 (nuclei zero-padded):
 * 26 numbers. Network 26 -> 256 -> 256 -> 256 -> 1, tanh on the hidden layers; its
 * output is multiplied by a fixed envelope (negf_mlp_envelope) that follows the
 * decay of the correction away from the nuclei;
 * parameters are one float32 array in the order W1 (26 x 256, row-major, input-major),
 * b1, W2 (256 x 256), b2, W3, b3, W4 (256 x 1), b4. */
int negf_mlp_param_count(int* count);

/* Feature rows F[n_samples][26] (dev, float32) for the samples (ii[s], jj[s], qq[s])
 * (dev int32: basis indices and tau index). x, v (dev, float64, n_b), tau (dev,
 * float64, n_tau); Xc, Zc (host, n_c <= 3). Errors: NEGF_EINVAL. */
int negf_mlp_features(negf_ctx* ctx, int n_b, const double* x, const double* v, int n_c,
                      const double* Xc, const double* Zc, int n_tau, const double* tau, double beta,
                      int n_samples, const int* ii, const int* jj, const int* qq, float* F, void* stream);

/* Envelope of the learned correction at the samples (dev, float32):
 * e(i, j) = (1 + (d_i + d_j)/5)^(-3/2), d_i = distance of node x_i to the nearest of
 * the n_c nuclei Xc (host; n_c = 0: d = 0); tau and beta are accepted for the
 * signature's sake and do not enter. x, tau dev. */
int negf_mlp_envelope(negf_ctx* ctx, const double* x, int n_c, const double* Xc, const double* tau,
                      double beta, int n_samples, const int* ii, const int* jj, const int* qq,
                      float* env, void* stream);

/* Training targets t[s] = (G[qq][ii][jj] - G0[qq][ii][jj]) / (out_scale e(ii, jj, tau_qq))
 * (dev), e the envelope of negf_mlp_envelope. */
int negf_mlp_targets(negf_ctx* ctx, int n_b, const double* G, const double* G0, double out_scale,
                     const double* x, int n_c, const double* Xc, int n_tau, const double* tau,
                     double beta, int n_samples, const int* ii, const int* jj, const int* qq,
                     float* t, void* stream);

/* Network output y[s] (dev, float32) for feature rows F (dev). */
int negf_mlp_forward(negf_ctx* ctx, const float* params, int n_samples, const float* F, float* y,
                     void* stream);

/* One training step on a mini-batch: forward, mean-squared error against target,
 * backward, and (lr > 0) one Adam update (beta1 0.9, beta2 0.999, eps 1e-8, bias
 * corrections for `step`, counted from 1) of params with moments m, v (all dev,
 * float32, param_count entries). grad_out (dev, nullable) receives the gradient of
 * the loss; *loss (host, nullable) the loss before the update (synchronises). */
int negf_mlp_train_step(negf_ctx* ctx, float* params, float* m, float* v, int step, double lr,
                        int n_samples, const float* F, const float* target, float* grad_out,
                        double* loss, void* stream);

/* Inference on the whole grid: for every q and i <= j, G_out[q][i][j] = G_out[q][j][i]
 * = (G0[q][i][j] + G0[q][j][i])/2 + out_scale e(i, j, tau_q) y(i, j, tau_q), e the
 * envelope of negf_mlp_envelope. dtype NEGF_F32: the network in float32 (as trained);
 * NEGF_BF16: weights and activations rounded to bf16 on the matrix cores with float32
 * accumulation (about 4x faster; output perturbed by ~1e-2 relative). x, v, tau
 * (dev, float64);
 * G0, G_out (dev, float64 [n_tau][n_b][n_b]; may alias). */
int negf_mlp_guess(negf_ctx* ctx, const float* params, double out_scale, int n_b, const double* x,
                   const double* v, int n_c, const double* Xc, const double* Zc, int n_tau,
                   const double* tau, double beta, const double* G0, double* G_out, int dtype,
                   void* stream);

#ifdef __cplusplus
}
#endif
#endif /* NEGF_H */
