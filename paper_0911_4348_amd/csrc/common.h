// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <vector>
#include <string>

#include "negf.h"

namespace negf {

void set_error(const char* fmt, ...);

struct Buf {
    void* p = nullptr;
    size_t cap = 0;
};

}  // namespace negf

struct negf_ctx {
    int device = 0;
    std::map<std::string, negf::Buf> bufs;   // named, grow-only scratch
    std::map<std::string, int> filled;       // constant tables already uploaded
    std::map<std::string, std::vector<char>> host_copy;   // contents of cached uploads
    size_t total = 0;
    hipStream_t work_stream = nullptr;        // stream of the SCF driver (graph capture needs one)
};

namespace negf {

// Named scratch buffer of at least `bytes`, grown with hipMalloc when needed.
int scratch(negf_ctx* c, const char* name, size_t bytes, void** out);
template <class T>
inline int scratch_t(negf_ctx* c, const char* name, size_t count, T** out) {
    void* p = nullptr;
    int rc = scratch(c, name, count * sizeof(T), &p);
    *out = static_cast<T*>(p);
    return rc;
}
int bind_device(negf_ctx* c);
// Copy a small host table into named scratch and wait for the copy.
int upload(negf_ctx* c, const char* name, const void* host, size_t bytes, hipStream_t st, void** out);
// As upload, but skipped (no copy, no wait) when the buffer already holds these bytes.
int upload_cached(negf_ctx* c, const char* name, const void* host, size_t bytes, hipStream_t st, void** out);

// ---------------------------------------------------------------- GEMM
// C[b] = alpha * op(A[b]) diag(s[b]) op(B[b]) + beta * Cin[b] for b < batch.
// op(A) is M x K, op(B) is K x N; ta/tb select the transposed storage.
// Strides are in elements; a batch stride of 0 shares the operand. colscale
// (nullable) scales column k of op(A) by s[b*sS + k]. Cin may equal C.
template <class T>
int gemm(hipStream_t st, bool ta, bool tb, int M, int N, int K, T alpha,
         const T* A, long lda, long sA, const T* B, long ldb, long sB,
         T beta, const T* Cin, long ldci, long sCi, T* C, long ldc, long sC,
         int batch, const T* colscale = nullptr, long sS = 0);
// Batched complex product of n x n matrices in planar form: Cr + i Ci =
// (Ar + i Ai)(Br + i Bi), matrix b of each array at offset b * stride.
template <class T>
int cgemm(hipStream_t st, int n, const T* Ar, const T* Ai, const T* Br, const T* Bi, T* Cr, T* Ci, long stride,
          int batch);

// ---------------------------------------------------------------- HF pieces
// Work list of the persistent Sigma-2B kernel for a batch of systems.
struct S2BBatch {
    int mode = 0, cfg = -1, n_cu = 0;
    int n_inst = 0, n_tau = 0, max_n = 0;
    long n_items = 0;
    std::vector<long> cuts;              // 9 item offsets: the per-XCD queues
    void* d_inst = nullptr;              // device descriptors (systems by decreasing n_b)
    int* heads = nullptr;                // 8 queue counters
    std::vector<int> n_sorted;
    std::vector<const void*> G_sorted;
    std::vector<int*> ex_sorted;
    std::vector<void*> gh_sorted;        // bf16 copies of the slices (bf16 mode)
    std::string key;                     // tuner cache key (mode and multiset of n_b)
};
int s2b_batch_prepare(negf_ctx* ctx, const char* tag, int dtype, int batch, const int* n, int n_tau,
                      const int* sigma, const void* const* V, const void* const* G, void* const* Sc, int pair_lim,
                      S2BBatch* plan, hipStream_t st);
int s2b_batch_launch(const S2BBatch& plan, hipStream_t st);
// Sustained rate (TFLOP/s) of the dtype's MFMA shape and the shader clock (GHz)
// it ran at, from a kernel of independent MFMA chains; synchronises.
int matrix_rate(negf_ctx* ctx, int dtype, double* tflops, double* ghz, hipStream_t st);
int issue_probe_f64(negf_ctx* ctx, int n_mfma, int n_fma, double* ms, double* tf_mfma, double* tf_fma,
                    hipStream_t st);
int s2b_batch_tune(negf_ctx* ctx, int dtype, int batch, const int* n, int n_tau, const int* sigma,
                   const void* const* V, const void* const* G, void* const* Sc, int pair_lim, int* best, double* ms,
                   hipStream_t st);
int hf_run_batched(negf_ctx* ctx, int B, int n_b, const double* T, const double* v, const double* V,
                   double n_elec, int sigma, double beta, double tol, int max_iter, double* eps, double* C,
                   double* rho, double* Sigma0, double* mu, double* E_hf, int* iters, hipStream_t st,
                   int* converged = nullptr);
int hf_run(negf_ctx* ctx, int n_b, const double* T, const double* v, const double* V,
           double n_elec, int sigma, double beta, double tol, int max_iter,
           double* eps, double* C, double* rho, double* Sigma0, double* mu, double* E_hf,
           int* iters, hipStream_t st);
template <class T>
int g0_build(negf_ctx* ctx, int n_b, int n_tau, const double* tau_host, double beta,
             const double* eps, const double* C, double mu, T* G0, hipStream_t st);

// ---------------------------------------------------------------- Sigma 2B
template <class T>
int sigma2b_run(negf_ctx* ctx, int n_b, int n_tau, int sigma, const T* V, const T* G,
                T* Sc, bool bf16, hipStream_t st);
int sigma2b_set_cfg(negf_ctx* ctx, int dtype, int n_b, int cfg);
// Float64 Sigma-2B of one system in the tuned configuration, else the fastest
// one measured at n_b = 199 where it fits (the direct-to-LDS tile).
int sigma2b_run_f64_single(negf_ctx* ctx, int n_b, int n_tau, int sigma, const double* V, const double* G,
                           double* Sc, hipStream_t st);
// Allocation-free form (float64 / float32): the float32 slice exponents go to a
// fixed per-device array whose address s2b_noalloc_init (device current) records.
int s2b_noalloc_init(int device);
template <class T>
int sigma2b_run_noalloc(negf_ctx* ctx, int n_b, int n_tau, int sigma, const T* V, const T* G, T* Sc,
                        hipStream_t st);
template <class T>
int sigma2b_tune(negf_ctx* ctx, int n_b, int n_tau, int sigma, const T* V, const T* G, T* Sc,
                 bool bf16, int* best, double* ms, hipStream_t st);

// ---------------------------------------------------------------- Dyson
template <class T>
int dyson_run(negf_ctx* ctx, const negf_tau_grid_t* tg, int n_b, int sigma, const double* h,
              const double* V, const double* eps, const double* C, double mu,
              const double* Sigma0, const T* G_in, const T* Sc, double alpha, int symmetrize,
              int conv_algo, T* G_out, hipStream_t st);
template <class T>
int energy_launch(negf_ctx* ctx, const negf_tau_grid_t* tg, int n_b, int sigma, const double* h,
                  const double* V, const T* G, const T* Sc, double* out, hipStream_t st);
template <class T>
int energy_run(negf_ctx* ctx, const negf_tau_grid_t* tg, int n_b, int sigma, const double* h,
               const double* V, const T* G, const T* Sc, double* E, double* N, hipStream_t st);

template <class T>
int density_run(int n_b, int n_tau, int sigma, const double* W, const T* G, double* out, hipStream_t st);

// ---------------------------------------------------------------- small kernels
template <class Tout, class Tin>
int convert(const Tin* in, Tout* out, size_t n, hipStream_t st);
int to_f32(const double* in, float* out, size_t n, hipStream_t st);

// ---------------------------------------------------------------- validation
int check_tau_grid(const negf_tau_grid_t* tg);

}  // namespace negf

#define NEGF_REQUIRE(cond, ...)               \
    do {                                      \
        if (!(cond)) {                        \
            negf::set_error(__VA_ARGS__);     \
            return NEGF_EINVAL;               \
        }                                     \
    } while (0)

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            negf::set_error("%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
            return NEGF_EHIP;                                                           \
        }                                                                               \
    } while (0)

#define NEGF_TRY(expr)          \
    do {                        \
        int rc_ = (expr);       \
        if (rc_ != NEGF_OK)     \
            return rc_;         \
    } while (0)

#define LAUNCH_CHECK()                                                                  \
    do {                                                                                \
        hipError_t e_ = hipGetLastError();                                              \
        if (e_ != hipSuccess) {                                                         \
            negf::set_error("kernel launch: %s (%s:%d)", hipGetErrorString(e_), __FILE__, __LINE__); \
            return NEGF_EHIP;                                                           \
        }                                                                               \
    } while (0)
