// Batched dense matrix product on the matrix cores (float64 and float32).
//
// C[b] = alpha * op(A[b]) diag(s[b]) op(B[b]) + beta * Cin[b]
//
// Workgroup tile 64 x 64, k-panel 16, four waves each owning a 32 x 32
// quadrant (2 x 2 MFMA tiles). Panels are staged in LDS k-major so that each
// lane's operand fetch for one MFMA is a row of 16 consecutive elements, in two
// buffers (the next panel is loaded while the current one is multiplied).
#include <type_traits>

#include "common.h"
#include "mfma.h"

namespace negf {
namespace {

constexpr int GB_M = 64, GB_N = 64, GB_K = 16, GB_PAD = 2;

// Workgroups are dealt to the 8 XCDs round-robin by linear index; renumber them
// so that each XCD receives a contiguous range of logical blocks, which puts
// all tiles of one matrix of the batch on one XCD (its operands are then read
// from HBM once into that XCD's L2, not once per XCD).
__device__ __forceinline__ long gemm_xcd_remap(long b, long nb) {
    const long x = b & 7, k = b >> 3;
    const long base = nb >> 3, rem = nb & 7;
    return x * base + (x < rem ? x : rem) + k;
}

template <class T, bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, T alpha, const T* __restrict__ A,
                                              long lda, long sA, const T* __restrict__ B, long ldb,
                                              long sB, T beta, const T* Cin, long ldci, long sCi,
                                              T* C, long ldc, long sC, const T* __restrict__ S,
                                              long sS) {
    // two LDS buffers: the loads of k-panel p + 1 are in flight while the
    // matrix cores work on panel p, and one barrier per panel remains
    __shared__ T As[2][GB_K][GB_M + GB_PAD];
    __shared__ T Bs[2][GB_K][GB_N + GB_PAD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const long nbx = gridDim.x, nby = gridDim.y;
    const long lb = gemm_xcd_remap(blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z), nbx * nby * gridDim.z);
    const long b = lb / (nbx * nby);
    const int m0 = (int)((lb / nbx) % nby) * GB_M, n0 = (int)(lb % nbx) * GB_N;
    A += b * sA;
    B += b * sB;
    if (S) S += b * sS;
    typename Mma<T>::acc_t acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = Mma<T>::zero();

    T ra[4], rb[4];
    auto load = [&](int k0) {
        // A panel: op(A)(m, k) for m in [m0, m0+64), k in [k0, k0+16)
        if (!TA) {
            const int m = m0 + (tid >> 2), kb = k0 + (tid & 3) * 4;
            for (int e = 0; e < 4; ++e) {
                const int k = kb + e;
                ra[e] = (m < M && k < K) ? A[(long)m * lda + k] : T(0);
                if (S && k < K) ra[e] *= S[k];
            }
        } else {
            const int k = k0 + (tid >> 4), mb = m0 + (tid & 15) * 4;
            for (int e = 0; e < 4; ++e) {
                const int m = mb + e;
                ra[e] = (m < M && k < K) ? A[(long)k * lda + m] : T(0);
                if (S && k < K) ra[e] *= S[k];
            }
        }
        if (!TB) {
            const int k = k0 + (tid >> 4), nb = n0 + (tid & 15) * 4;
            for (int e = 0; e < 4; ++e) {
                const int n = nb + e;
                rb[e] = (n < N && k < K) ? B[(long)k * ldb + n] : T(0);
            }
        } else {
            const int n = n0 + (tid >> 2), kb = k0 + (tid & 3) * 4;
            for (int e = 0; e < 4; ++e) {
                const int k = kb + e;
                rb[e] = (n < N && k < K) ? B[(long)n * ldb + k] : T(0);
            }
        }
    };
    auto store = [&](int buf) {
        if (!TA) {
            for (int e = 0; e < 4; ++e) As[buf][(tid & 3) * 4 + e][tid >> 2] = ra[e];
        } else {
            for (int e = 0; e < 4; ++e) As[buf][tid >> 4][(tid & 15) * 4 + e] = ra[e];
        }
        if (!TB) {
            for (int e = 0; e < 4; ++e) Bs[buf][tid >> 4][(tid & 15) * 4 + e] = rb[e];
        } else {
            for (int e = 0; e < 4; ++e) Bs[buf][(tid & 3) * 4 + e][tid >> 2] = rb[e];
        }
    };
    // 16 x 16 blocks of this wave's quadrant that hold some row < M and some
    // column < N (wave-uniform): blocks wholly in the padding of the last tile
    // row or column are not multiplied
    const int wm = __builtin_amdgcn_readfirstlane(m0 + wr * 32), wn = __builtin_amdgcn_readfirstlane(n0 + wc * 32);
    const int nmi = wm >= M ? 0 : (wm + 16 >= M ? 1 : 2), nni = wn >= N ? 0 : (wn + 16 >= N ? 1 : 2);
    auto panel = [&](int buf, auto mi_t, auto ni_t) {
        constexpr int MI = decltype(mi_t)::value, NI = decltype(ni_t)::value;
#pragma unroll
        for (int ks = 0; ks < GB_K / 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            AFrag<T> a[MI];
            T bf[NI];
#pragma unroll
            for (int i = 0; i < MI; ++i) a[i].load(lane, [&](int m) { return As[buf][kk][wr * 32 + 16 * i + m]; });
#pragma unroll
            for (int j = 0; j < NI; ++j) bf[j] = Bs[buf][kk][wc * 32 + 16 * j + (lane & 15)];
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
                for (int j = 0; j < NI; ++j) acc[i][j] = a[i].mma(bf[j], acc[i][j]);
        }
    };
    typedef std::integral_constant<int, 1> C1;
    typedef std::integral_constant<int, 2> C2;
    load(0);
    store(0);
    __syncthreads();
    for (int k0 = 0, buf = 0; k0 < K; k0 += GB_K, buf ^= 1) {
        const bool more = k0 + GB_K < K;
        if (more) load(k0 + GB_K);
        if (nmi == 2 && nni == 2) panel(buf, C2(), C2());
        else if (nmi == 2 && nni == 1) panel(buf, C2(), C1());
        else if (nmi == 1 && nni == 2) panel(buf, C1(), C2());
        else if (nmi == 1 && nni == 1) panel(buf, C1(), C1());
        // the other buffer was last read before the previous barrier
        if (more) store(buf ^ 1);
        __syncthreads();
    }
    C += b * sC;
    if (Cin) Cin += b * sCi;
    for (int mi = 0; mi < 2; ++mi)
        for (int ni = 0; ni < 2; ++ni)
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wr * 32 + mi * 16 + Mma<T>::row(lane, r);
                const int col = n0 + wc * 32 + ni * 16 + (lane & 15);
                if (row < M && col < N) {
                    T v = alpha * acc[mi][ni][r];
                    if (beta != T(0)) v += beta * Cin[(long)row * ldci + col];
                    C[(long)row * ldc + col] = v;
                }
            }
}

// Batched complex product C = A B of n x n matrices in planar form (real and
// imaginary parts in separate arrays, matrix b at offset b * stride):
//   Cr = Ar Br - Ai Bi,  Ci = Ar Bi + Ai Br,
// each part accumulated in one chain over k. The tile layout, staging and
// XCD order are those of k_gemm; every operand tile is read once for both
// parts (four real products would read each operand twice and write, reread
// and rewrite the outputs).
template <class T>
__global__ __launch_bounds__(256) void k_cgemm(int n, const T* __restrict__ Ar, const T* __restrict__ Ai,
                                               const T* __restrict__ Br, const T* __restrict__ Bi,
                                               T* __restrict__ Cr, T* __restrict__ Ci, long stride) {
    __shared__ T Asr[2][GB_K][GB_M + GB_PAD], Asi[2][GB_K][GB_M + GB_PAD];
    __shared__ T Bsr[2][GB_K][GB_N + GB_PAD], Bsi[2][GB_K][GB_N + GB_PAD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const long nbx = gridDim.x, nby = gridDim.y;
    const long lb = gemm_xcd_remap(blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z), nbx * nby * gridDim.z);
    const long b = lb / (nbx * nby);
    const int m0 = (int)((lb / nbx) % nby) * GB_M, n0 = (int)(lb % nbx) * GB_N;
    const long off = b * stride;
    typename Mma<T>::acc_t cr[2][2], ci[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) cr[i][j] = ci[i][j] = Mma<T>::zero();
    T rar[4], rai[4], rbr[4], rbi[4];
    auto load = [&](int k0) {
        {
            const int m = m0 + (tid >> 2), kb = k0 + (tid & 3) * 4;
            for (int e = 0; e < 4; ++e) {
                const int k = kb + e;
                const bool in = m < n && k < n;
                rar[e] = in ? Ar[off + (long)m * n + k] : T(0);
                rai[e] = in ? Ai[off + (long)m * n + k] : T(0);
            }
        }
        {
            const int k = k0 + (tid >> 4), nb = n0 + (tid & 15) * 4;
            for (int e = 0; e < 4; ++e) {
                const int c = nb + e;
                const bool in = c < n && k < n;
                rbr[e] = in ? Br[off + (long)k * n + c] : T(0);
                rbi[e] = in ? Bi[off + (long)k * n + c] : T(0);
            }
        }
    };
    auto store = [&](int buf) {
        for (int e = 0; e < 4; ++e) {
            Asr[buf][(tid & 3) * 4 + e][tid >> 2] = rar[e];
            Asi[buf][(tid & 3) * 4 + e][tid >> 2] = rai[e];
            Bsr[buf][tid >> 4][(tid & 15) * 4 + e] = rbr[e];
            Bsi[buf][tid >> 4][(tid & 15) * 4 + e] = rbi[e];
        }
    };
    // as in k_gemm: 16 x 16 blocks wholly in the padding are not multiplied
    const int wm = __builtin_amdgcn_readfirstlane(m0 + wr * 32), wn = __builtin_amdgcn_readfirstlane(n0 + wc * 32);
    const int nmi = wm >= n ? 0 : (wm + 16 >= n ? 1 : 2), nni = wn >= n ? 0 : (wn + 16 >= n ? 1 : 2);
    auto panel = [&](int buf, auto mi_t, auto ni_t) {
        constexpr int MI = decltype(mi_t)::value, NI = decltype(ni_t)::value;
#pragma unroll
        for (int ks = 0; ks < GB_K / 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            AFrag<T> ar[MI], ai[MI], nai[MI];
            T br[NI], bi[NI];
#pragma unroll
            for (int h = 0; h < MI; ++h) {
                ar[h].load(lane, [&](int m) { return Asr[buf][kk][wr * 32 + 16 * h + m]; });
                ai[h].load(lane, [&](int m) { return Asi[buf][kk][wr * 32 + 16 * h + m]; });
                nai[h] = ai[h].neg();
            }
#pragma unroll
            for (int h = 0; h < NI; ++h) {
                br[h] = Bsr[buf][kk][wc * 32 + 16 * h + (lane & 15)];
                bi[h] = Bsi[buf][kk][wc * 32 + 16 * h + (lane & 15)];
            }
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
                for (int j = 0; j < NI; ++j) {
                    cr[i][j] = ar[i].mma(br[j], cr[i][j]);
                    cr[i][j] = nai[i].mma(bi[j], cr[i][j]);
                    ci[i][j] = ar[i].mma(bi[j], ci[i][j]);
                    ci[i][j] = ai[i].mma(br[j], ci[i][j]);
                }
        }
    };
    typedef std::integral_constant<int, 1> C1;
    typedef std::integral_constant<int, 2> C2;
    load(0);
    store(0);
    __syncthreads();
    for (int k0 = 0, buf = 0; k0 < n; k0 += GB_K, buf ^= 1) {
        const bool more = k0 + GB_K < n;
        if (more) load(k0 + GB_K);
        if (nmi == 2 && nni == 2) panel(buf, C2(), C2());
        else if (nmi == 2 && nni == 1) panel(buf, C2(), C1());
        else if (nmi == 1 && nni == 2) panel(buf, C1(), C2());
        else if (nmi == 1 && nni == 1) panel(buf, C1(), C1());
        if (more) store(buf ^ 1);
        __syncthreads();
    }
    for (int mi = 0; mi < 2; ++mi)
        for (int ni = 0; ni < 2; ++ni)
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wr * 32 + mi * 16 + Mma<T>::row(lane, r);
                const int col = n0 + wc * 32 + ni * 16 + (lane & 15);
                if (row < n && col < n) {
                    Cr[off + (long)row * n + col] = cr[mi][ni][r];
                    Ci[off + (long)row * n + col] = ci[mi][ni][r];
                }
            }
}

}  // namespace

template <class T>
int cgemm(hipStream_t st, int n, const T* Ar, const T* Ai, const T* Br, const T* Bi, T* Cr, T* Ci, long stride,
          int batch) {
    if (n <= 0 || batch <= 0) return NEGF_OK;
    for (int b0 = 0; b0 < batch; b0 += 65535) {
        const int nb = batch - b0 < 65535 ? batch - b0 : 65535;
        const long o = (long)b0 * stride;
        dim3 grid((n + GB_N - 1) / GB_N, (n + GB_M - 1) / GB_M, nb);
        hipLaunchKernelGGL((k_cgemm<T>), grid, dim3(256), 0, st, n, Ar + o, Ai + o, Br + o, Bi + o, Cr + o, Ci + o,
                           stride);
        LAUNCH_CHECK();
    }
    return NEGF_OK;
}
template int cgemm<double>(hipStream_t, int, const double*, const double*, const double*, const double*, double*,
                           double*, long, int);
template int cgemm<float>(hipStream_t, int, const float*, const float*, const float*, const float*, float*, float*,
                          long, int);

template <class T>
int gemm(hipStream_t st, bool ta, bool tb, int M, int N, int K, T alpha, const T* A, long lda,
         long sA, const T* B, long ldb, long sB, T beta, const T* Cin, long ldci, long sCi, T* C,
         long ldc, long sC, int batch, const T* S, long sS) {
    if (M <= 0 || N <= 0 || batch <= 0) return NEGF_OK;
    if (batch > 65535) {
        // split very large batches over several launches
        for (int b0 = 0; b0 < batch; b0 += 65535) {
            int nb = batch - b0 < 65535 ? batch - b0 : 65535;
            NEGF_TRY(gemm<T>(st, ta, tb, M, N, K, alpha, A + (long)b0 * sA, lda, sA, B + (long)b0 * sB,
                             ldb, sB, beta, Cin ? Cin + (long)b0 * sCi : nullptr, ldci, sCi,
                             C + (long)b0 * sC, ldc, sC, nb, S ? S + (long)b0 * sS : nullptr, sS));
        }
        return NEGF_OK;
    }
    dim3 grid((N + GB_N - 1) / GB_N, (M + GB_M - 1) / GB_M, batch);
    if (beta != T(0) && Cin == nullptr) {
        set_error("gemm: beta != 0 needs Cin");
        return NEGF_EINVAL;
    }
#define NEGF_GEMM_LAUNCH(TA_, TB_)                                                               \
    hipLaunchKernelGGL((k_gemm<T, TA_, TB_>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, sA, B, \
                       ldb, sB, beta, Cin, ldci, sCi, C, ldc, sC, S, sS)
    if (!ta && !tb) NEGF_GEMM_LAUNCH(false, false);
    else if (!ta && tb) NEGF_GEMM_LAUNCH(false, true);
    else if (ta && !tb) NEGF_GEMM_LAUNCH(true, false);
    else NEGF_GEMM_LAUNCH(true, true);
#undef NEGF_GEMM_LAUNCH
    LAUNCH_CHECK();
    return NEGF_OK;
}

template int gemm<double>(hipStream_t, bool, bool, int, int, int, double, const double*, long, long,
                          const double*, long, long, double, const double*, long, long, double*,
                          long, long, int, const double*, long);
template int gemm<float>(hipStream_t, bool, bool, int, int, int, float, const float*, long, long,
                         const float*, long, long, float, const float*, long, long, float*, long,
                         long, int, const float*, long);

// ---------------------------------------------------------------- conversions
namespace {
template <class To, class Ti>
__global__ void k_convert(const Ti* __restrict__ in, To* __restrict__ out, size_t n) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) out[i] = (To)in[i];
}
}  // namespace

template <class Tout, class Tin>
int convert(const Tin* in, Tout* out, size_t n, hipStream_t st) {
    if (n == 0) return NEGF_OK;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL((k_convert<Tout, Tin>), dim3((unsigned)blocks), dim3(256), 0, st, in, out, n);
    LAUNCH_CHECK();
    return NEGF_OK;
}
template int convert<float, double>(const double*, float*, size_t, hipStream_t);
template int convert<double, float>(const float*, double*, size_t, hipStream_t);

int to_f32(const double* in, float* out, size_t n, hipStream_t st) { return convert<float, double>(in, out, n, st); }

}  // namespace negf
