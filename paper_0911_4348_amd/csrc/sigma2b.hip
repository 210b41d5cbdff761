// Second-Born correlation self-energy on the Matsubara grid (paper Sec. 2.3,
// Eq. sigma2ndb, with both interaction lines between points at equal times):
//
//   Sigma_c,ij(tau) = sum_kl V_ik V_jl [sigma G_ij G_kl Gb_lk - G_il Gb_lk G_kj],
//   Gb = G(beta - tau).
//
// Slices q and q' = n_tau-1-q are done together. With symmetric slices:
//   direct  D = V (G o Gb) V          -> Sigma_c[q] += sigma G o D, Sigma_c[q'] += sigma Gb o D
//   exchange M^(i) = Gb diag(V_i,:) G  (one n_b x n_b x n_b product per i)
//            X_ij  = sum_l G_il  V_jl M^(i)_lj   -> Sigma_c[q]  -= X
//            X'_il = sum_j Gb_ij V_lj M^(i)_lj   -> Sigma_c[q'] -= X'
// The exchange products never reach memory: a workgroup owns one slice pair
// and IB values of i (one per wave), streams l-tiles of 16 rows of M^(i)
// through the matrix cores with the operand A[l][k] = Gb_lk V_ik formed while
// staging, and reduces each finished tile into X and X' in registers and LDS.
#include "common.h"
#include "mfma.h"

namespace negf {
namespace {

constexpr int SX_BK = 16;   // k-panel
constexpr int SX_JB = 13;   // 16-wide column blocks per chunk (208 columns)
constexpr int SX_PAD = 1;

template <class T, int IB>
__global__ __launch_bounds__(IB * 64) void k_sigma2b_exchange(int n, int n_tau, int n_iblk,
                                                               const T* __restrict__ V,
                                                               const T* __restrict__ G,
                                                               T* __restrict__ Sc) {
    extern __shared__ unsigned char smem_raw[];
    T* Gs = reinterpret_cast<T*>(smem_raw);                       // [SX_BK][SX_JB*16 + SX_PAD]
    constexpr int GS_LD = SX_JB * 16 + SX_PAD;
    T* Ab = Gs + SX_BK * GS_LD;                                   // [16][SX_BK + 1]
    T* Vk = Ab + 16 * (SX_BK + 1);                                // [IB][SX_BK]
    T* XPs = Vk + IB * SX_BK;                                     // [IB][np]
    const int np = (n + 15) & ~15;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int pair = blockIdx.x / n_iblk, iblk = blockIdx.x % n_iblk;
    const int q = pair, qb = n_tau - 1 - pair;
    const bool middle = (q == qb);
    const long nn = (long)n * n;
    const T* Gq = G + (long)q * nn;
    const T* Gb = G + (long)qb * nn;
    const int i = iblk * IB + w;
    const bool iok = i < n;
    const int lc = lane & 15;

    for (int e = tid; e < IB * np; e += IB * 64) XPs[e] = T(0);

    for (int j0 = 0; j0 < np; j0 += SX_JB * 16) {
        const int njb = min(SX_JB, (np - j0) >> 4);
        T gbi[SX_JB], xcol[SX_JB];
#pragma unroll
        for (int jb = 0; jb < SX_JB; ++jb) {
            const int j = j0 + jb * 16 + lc;
            gbi[jb] = (iok && jb < njb && j < n) ? Gb[(long)i * n + j] : T(0);
            xcol[jb] = T(0);
        }
        for (int l0 = 0; l0 < n; l0 += 16) {
            typename Mma<T>::acc_t acc[SX_JB];
#pragma unroll
            for (int jb = 0; jb < SX_JB; ++jb) acc[jb] = Mma<T>::zero();
            for (int k0 = 0; k0 < n; k0 += SX_BK) {
                __syncthreads();
                for (int e = tid; e < SX_BK * njb * 16; e += IB * 64) {
                    const int kk = e / (njb * 16), jj = e % (njb * 16);
                    const int k = k0 + kk, j = j0 + jj;
                    Gs[kk * GS_LD + jj] = (k < n && j < n) ? Gq[(long)k * n + j] : T(0);
                }
                for (int e = tid; e < 16 * SX_BK; e += IB * 64) {
                    const int ll = e / SX_BK, kk = e % SX_BK;
                    const int l = l0 + ll, k = k0 + kk;
                    Ab[ll * (SX_BK + 1) + kk] = (l < n && k < n) ? Gb[(long)l * n + k] : T(0);
                }
                for (int e = tid; e < IB * SX_BK; e += IB * 64) {
                    const int ww = e / SX_BK, kk = e % SX_BK;
                    const int ii = iblk * IB + ww, k = k0 + kk;
                    Vk[e] = (ii < n && k < n) ? V[(long)ii * n + k] : T(0);
                }
                __syncthreads();
#pragma unroll
                for (int ks = 0; ks < SX_BK / 4; ++ks) {
                    const int kk = ks * 4 + (lane >> 4);
                    const T a = Ab[lc * (SX_BK + 1) + kk] * Vk[w * SX_BK + kk];
#pragma unroll
                    for (int jb = 0; jb < SX_JB; ++jb)
                        if (jb < njb) acc[jb] = Mma<T>::mma(a, Gs[kk * GS_LD + jb * 16 + lc], acc[jb]);
                }
            }
            // epilogue of the (l-tile, column chunk): V rows l0..l0+15 into Gs
            __syncthreads();
            for (int e = tid; e < 16 * njb * 16; e += IB * 64) {
                const int ll = e / (njb * 16), jj = e % (njb * 16);
                const int l = l0 + ll, j = j0 + jj;
                Gs[ll * GS_LD + jj] = (l < n && j < n) ? V[(long)l * n + j] : T(0);
            }
            __syncthreads();
            T gil[4], xp[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int l = l0 + Mma<T>::row(lane, r);
                gil[r] = (iok && l < n) ? Gq[(long)i * n + l] : T(0);
                xp[r] = T(0);
            }
#pragma unroll
            for (int jb = 0; jb < SX_JB; ++jb) {
                if (jb < njb) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const T vm = Gs[Mma<T>::row(lane, r) * GS_LD + jb * 16 + lc] * acc[jb][r];
                        xp[r] += gbi[jb] * vm;
                        xcol[jb] += gil[r] * vm;
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const T s = sum16(xp[r]);
                const int l = l0 + Mma<T>::row(lane, r);
                if (lc == 0 && l < np) XPs[w * np + l] += s;
            }
        }
#pragma unroll
        for (int jb = 0; jb < SX_JB; ++jb) {
            const T s = sum4x16(xcol[jb]);
            const int j = j0 + jb * 16 + lc;
            if (iok && jb < njb && (lane >> 4) == 0 && j < n) Sc[(long)q * nn + (long)i * n + j] = -s;
        }
    }
    __syncthreads();
    if (!middle && iok)
        for (int l = lane; l < n; l += 64) Sc[(long)qb * nn + (long)i * n + l] = -XPs[w * np + l];
}

// W[t] = G[t] o G[n_tau-1-t]
template <class T>
__global__ void k_pair_hadamard(int n, int n_tau, int n_pairs, const T* __restrict__ G, T* __restrict__ W) {
    const long nn = (long)n * n;
    const long total = nn * n_pairs;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const long t = e / nn, r = e % nn;
        W[e] = G[t * nn + r] * G[(n_tau - 1 - t) * nn + r];
    }
}

// Sigma_c[q] += sigma G[q] o D[t], Sigma_c[q'] += sigma G[q'] o D[t]
template <class T>
__global__ void k_direct_epilogue(int n, int n_tau, int n_pairs, T sigma, const T* __restrict__ G,
                                  const T* __restrict__ D, T* __restrict__ Sc) {
    const long nn = (long)n * n;
    const long total = nn * n_pairs;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const long t = e / nn, r = e % nn;
        const long qb = n_tau - 1 - t;
        const T d = D[e];
        Sc[t * nn + r] += sigma * G[t * nn + r] * d;
        if (qb != t) Sc[qb * nn + r] += sigma * G[qb * nn + r] * d;
    }
}

inline unsigned grid_for(long total) {
    long b = (total + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

template <class T>
int sigma2b_run(negf_ctx* ctx, int n, int n_tau, int sigma, const T* V, const T* G, T* Sc,
                bool bf16, hipStream_t st) {
    if (bf16) {
        set_error("bf16 exchange path not available");
        return NEGF_EINVAL;
    }
    const int n_pairs = (n_tau + 1) / 2;
    constexpr int IB = 8;
    const int n_iblk = (n + IB - 1) / IB;
    const int np = (n + 15) & ~15;
    const size_t smem = sizeof(T) * ((size_t)SX_BK * (SX_JB * 16 + SX_PAD) + 16 * (SX_BK + 1) +
                                     IB * SX_BK + (size_t)IB * np);
    if (smem > 160 * 1024) {
        set_error("n_b = %d too large for the exchange kernel's LDS budget", n);
        return NEGF_EINVAL;
    }
    const long blocks = (long)n_pairs * n_iblk;
    if (blocks > 0x7fffffffL) {
        set_error("too many workgroups");
        return NEGF_EINVAL;
    }
    static bool attr_set[2] = {false, false};
    const int ti = sizeof(T) == 8 ? 0 : 1;
    if (!attr_set[ti]) {
        HIP_TRY(hipFuncSetAttribute((const void*)k_sigma2b_exchange<T, IB>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        attr_set[ti] = true;
    }
    hipLaunchKernelGGL((k_sigma2b_exchange<T, IB>), dim3((unsigned)blocks), dim3(IB * 64), smem, st,
                       n, n_tau, n_iblk, V, G, Sc);
    LAUNCH_CHECK();

    // direct term
    const long nn = (long)n * n;
    T *W = nullptr, *T1 = nullptr;
    NEGF_TRY(scratch_t(ctx, "s2b_w", (size_t)nn * n_pairs, &W));
    NEGF_TRY(scratch_t(ctx, "s2b_t1", (size_t)nn * n_pairs, &T1));
    hipLaunchKernelGGL((k_pair_hadamard<T>), dim3(grid_for(nn * n_pairs)), dim3(256), 0, st, n, n_tau,
                       n_pairs, G, W);
    LAUNCH_CHECK();
    NEGF_TRY(gemm<T>(st, false, false, n, n, n, T(1), V, n, 0, W, n, nn, T(0), nullptr, 0, 0, T1, n, nn,
                     n_pairs));
    NEGF_TRY(gemm<T>(st, false, false, n, n, n, T(1), T1, n, nn, V, n, 0, T(0), nullptr, 0, 0, W, n, nn,
                     n_pairs));
    hipLaunchKernelGGL((k_direct_epilogue<T>), dim3(grid_for(nn * n_pairs)), dim3(256), 0, st, n, n_tau,
                       n_pairs, T(sigma), G, W, Sc);
    LAUNCH_CHECK();
    return NEGF_OK;
}

template int sigma2b_run<double>(negf_ctx*, int, int, int, const double*, const double*, double*, bool, hipStream_t);
template int sigma2b_run<float>(negf_ctx*, int, int, int, const float*, const float*, float*, bool, hipStream_t);

}  // namespace negf
