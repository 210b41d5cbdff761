// Learned initial guess: a tau-resolved 4-layer MLP (float32) that predicts
// dG_ij(tau) = G(tau) - G0(tau) from per-sample features; the guess is
// G_init = G0 + (dG + dG^T)/2. Training and inference run in these kernels.
// The network output y is scaled by a fixed envelope that follows the decay of
// the correction away from the nuclei: dG = s e(i, j) y with
//   e = (1 + (d_i + d_j)/L)^(-3/2),
// d_i the distance of node i to the nearest nucleus, L = 5 a.u.; the network's
// residual error far from the nuclei is damped by the same factor.
//
// Features per sample (i, j, tau): x_i/s, x_j/s, v_i, v_j, T_0..T_15(2 tau/beta - 1),
// Z_1..Z_3, X_1/s..X_3/s (s = 10, nuclei zero-padded). Network 26 -> 256 -> 256 ->
// 256 -> 1 with tanh hidden activations; parameters flat as W1 (26 x 256), b1,
// W2, b2, W3, b3, W4 (256 x 1), b4. Hidden layers use the float32 matrix cores
// with the bias and tanh fused into the product's epilogue.
#include <cmath>
#include <vector>

#include "common.h"
#include "mfma.h"

namespace negf {
namespace {

constexpr int N_CHEB = 16, N_CENT = 3, D_IN = 4 + N_CHEB + 2 * N_CENT, HID = 256;
constexpr float X_SCALE = 10.0f;
constexpr long OFF_W1 = 0, OFF_B1 = OFF_W1 + D_IN * HID, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
               OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID * HID, OFF_W4 = OFF_B3 + HID, OFF_B4 = OFF_W4 + HID,
               N_PARAMS = OFF_B4 + 1;

inline unsigned grid_for(long total) {
    long b = (total + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

constexpr double ENV_L = 5.0;

struct NucTab {
    float Z[N_CENT];
    float X[N_CENT];
    int n;
};

__device__ __forceinline__ double envelope(double xi, double xj, double tau, double beta, const NucTab& nt) {
    double di = 0.0, dj = 0.0;
    if (nt.n > 0) {
        di = dj = 1e300;
        for (int c = 0; c < nt.n; ++c) {
            di = fmin(di, fabs(xi - (double)nt.X[c]));
            dj = fmin(dj, fabs(xj - (double)nt.X[c]));
        }
    }
    (void)tau;
    (void)beta;
    const double u = 1.0 + (di + dj) / ENV_L;
    return 1.0 / (u * sqrt(u));
}

__device__ __forceinline__ void feature_row(float* f, float xi, float xj, float vi, float vj, float t,
                                            const NucTab& nt) {
    f[0] = xi / X_SCALE;
    f[1] = xj / X_SCALE;
    f[2] = vi;
    f[3] = vj;
    float tm2 = 1.f, tm1 = t;
    f[4] = 1.f;
    f[5] = t;
    for (int k = 2; k < N_CHEB; ++k) {
        const float tk = 2.f * t * tm1 - tm2;
        f[4 + k] = tk;
        tm2 = tm1;
        tm1 = tk;
    }
    for (int c = 0; c < N_CENT; ++c) {
        f[4 + N_CHEB + c] = nt.Z[c];
        f[4 + N_CHEB + N_CENT + c] = nt.X[c] / X_SCALE;
    }
}

// Features for explicit samples (ii, jj, qq).
__global__ void k_features(int S, const double* __restrict__ x, const double* __restrict__ v,
                           const double* __restrict__ tau, double beta, const int* __restrict__ ii,
                           const int* __restrict__ jj, const int* __restrict__ qq, NucTab nt, float* __restrict__ F) {
    for (long s = blockIdx.x * (long)blockDim.x + threadIdx.x; s < S; s += (long)gridDim.x * blockDim.x) {
        const int i = ii[s], j = jj[s], q = qq[s];
        feature_row(F + s * D_IN, (float)x[i], (float)x[j], (float)v[i], (float)v[j],
                    (float)(2.0 * tau[q] / beta - 1.0), nt);
    }
}

// Features for a contiguous range of the full (q, i <= j) grid: sample s of the
// range is global index g = g0 + s, q = g / P, pair r = g % P with (i, j) the
// r-th upper-triangle pair in row-major order.
__device__ __forceinline__ void pair_of(int n, long r, int* pi, int* pj) {
    // rows i hold n - i pairs; invert the running count
    int i = 0;
    long base = 0;
    // closed form start, then correct
    double nn = n + 0.5;
    double est = nn - sqrt(nn * nn - 2.0 * (double)r);
    i = (int)est;
    if (i < 0) i = 0;
    if (i > n - 1) i = n - 1;
    base = (long)i * n - (long)i * (i - 1) / 2;
    while (i > 0 && base > r) {
        --i;
        base = (long)i * n - (long)i * (i - 1) / 2;
    }
    while (i < n - 1 && base + (n - i) <= r) {
        base += n - i;
        ++i;
    }
    *pi = i;
    *pj = i + (int)(r - base);
}

__global__ void k_features_grid(int n, long g0, long S, const double* __restrict__ x, const double* __restrict__ v,
                                const double* __restrict__ tau, double beta, NucTab nt, float* __restrict__ F) {
    const long P = (long)n * (n + 1) / 2;
    for (long s = blockIdx.x * (long)blockDim.x + threadIdx.x; s < S; s += (long)gridDim.x * blockDim.x) {
        const long g = g0 + s;
        const int q = (int)(g / P);
        int i, j;
        pair_of(n, g % P, &i, &j);
        feature_row(F + s * D_IN, (float)x[i], (float)x[j], (float)v[i], (float)v[j],
                    (float)(2.0 * tau[q] / beta - 1.0), nt);
    }
}

// C[S][N] = act(A[S][K] W[K][N] + b), act = tanh or identity, float32 MFMA.
template <bool TANH>
__global__ __launch_bounds__(256) void k_dense(int S, int K, int N, const float* __restrict__ A,
                                               const float* __restrict__ Wt, const float* __restrict__ b,
                                               float* __restrict__ C) {
    __shared__ float As[16][66];
    __shared__ float Bs[16][66];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    fv4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) acc[a][c] = fv4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        float ra[4], rb[4];
        {
            const int m = m0 + (tid >> 2), kb = k0 + (tid & 3) * 4;
            for (int e = 0; e < 4; ++e) ra[e] = (m < S && kb + e < K) ? A[(long)m * K + kb + e] : 0.f;
            const int k = k0 + (tid >> 4), nb = n0 + (tid & 15) * 4;
            for (int e = 0; e < 4; ++e) rb[e] = (k < K && nb + e < N) ? Wt[(long)k * N + nb + e] : 0.f;
        }
        __syncthreads();
        for (int e = 0; e < 4; ++e) As[(tid & 3) * 4 + e][tid >> 2] = ra[e];
        for (int e = 0; e < 4; ++e) Bs[tid >> 4][(tid & 15) * 4 + e] = rb[e];
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            const float a0 = As[kk][wr * 32 + (lane & 15)], a1 = As[kk][wr * 32 + 16 + (lane & 15)];
            const float b0 = Bs[kk][wc * 32 + (lane & 15)], b1 = Bs[kk][wc * 32 + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
    for (int mi = 0; mi < 2; ++mi)
        for (int ni = 0; ni < 2; ++ni)
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wr * 32 + mi * 16 + Mma<float>::row(lane, r);
                const int col = n0 + wc * 32 + ni * 16 + (lane & 15);
                if (row < S && col < N) {
                    float z = acc[mi][ni][r] + b[col];
                    C[(long)row * N + col] = TANH ? tanhf(z) : z;
                }
            }
}

// y[s] = a3[s] . W4 + b4 (one wave per sample block)
__global__ void k_out(int S, const float* __restrict__ a3, const float* __restrict__ W4, const float* __restrict__ b4,
                      float* __restrict__ y) {
    const int lane = threadIdx.x & 63;
    for (long s = (blockIdx.x * (long)blockDim.x + threadIdx.x) >> 6; s < S; s += ((long)gridDim.x * blockDim.x) >> 6) {
        float acc = 0.f;
        for (int k = lane; k < HID; k += 64) acc += a3[s * HID + k] * W4[k];
        acc = wave_sum(acc);
        if (lane == 0) y[s] = acc + b4[0];
    }
}

// dy = 2 (y - t) / S and per-block partial losses
__global__ __launch_bounds__(256) void k_mse(int S, const float* __restrict__ y, const float* __restrict__ t,
                                             float* __restrict__ dy, double* __restrict__ part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (long s = blockIdx.x * (long)blockDim.x + threadIdx.x; s < S; s += (long)gridDim.x * blockDim.x) {
        const float r = y[s] - t[s];
        dy[s] = 2.f * r / (float)S;
        acc += (double)r * r;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// d3[s][k] = dy[s] W4[k] (1 - a3^2)
__global__ void k_back_out(int S, const float* dy, const float* W4, const float* a3, float* d3) {
    const long tot = (long)S * HID;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        const long s = e / HID;
        const int k = (int)(e % HID);
        const float a = a3[e];
        d3[e] = dy[s] * W4[k] * (1.f - a * a);
    }
}

// d *= (1 - a^2)
__global__ void k_tanh_grad(long tot, const float* a, float* d) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        const float v = a[e];
        d[e] *= (1.f - v * v);
    }
}

// Column reductions over the samples, in a fixed order (deterministic):
// g[c] = sum_s D[s][c] * (w ? w[s] : 1) for c < N. Block (64 columns x 16 row
// groups); each thread sums every 16th row of its column in double, then the 16
// partial sums are added in order.
__global__ __launch_bounds__(1024) void k_colsum(int S, int N, const float* __restrict__ D,
                                                 const float* __restrict__ w, float* __restrict__ g) {
    __shared__ double part[16][65];
    const int cx = threadIdx.x & 63, ry = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + cx;
    double acc = 0.0;
    if (c < N) {
        for (int s = ry; s < S; s += 16) acc += (double)D[(long)s * N + c] * (w ? (double)w[s] : 1.0);
    }
    part[ry][cx] = acc;
    __syncthreads();
    if (ry == 0 && c < N) {
        double t = 0.0;
        for (int r = 0; r < 16; ++r) t += part[r][cx];
        g[c] = (float)t;
    }
}

// g[c] = sum_k P[k][c] over nsplit partial products (fixed order)
__global__ void k_sum_partials(long count, int nsplit, const float* __restrict__ P, float* __restrict__ g) {
    for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < count; c += (long)gridDim.x * blockDim.x) {
        float t = 0.f;
        for (int k = 0; k < nsplit; ++k) t += P[(long)k * count + c];
        g[c] = t;
    }
}

__global__ void k_adam(long n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const float gg = g[e];
        const float mm = b1 * m[e] + (1.f - b1) * gg;
        const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
        m[e] = mm;
        v[e] = vv;
        p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
}

// targets t[s] = (G[q][i][j] - G0[q][i][j]) / scale
__global__ void k_targets(int S, int n, const double* G, const double* G0, double scale, const double* x,
                          const double* tau, double beta, NucTab nt, const int* ii, const int* jj, const int* qq,
                          float* t) {
    const long nn = (long)n * n;
    for (long s = blockIdx.x * (long)blockDim.x + threadIdx.x; s < S; s += (long)gridDim.x * blockDim.x) {
        const int i = ii[s], j = jj[s], q = qq[s];
        const long e = (long)q * nn + (long)i * n + j;
        t[s] = (float)((G[e] - G0[e]) / (scale * envelope(x[i], x[j], tau[q], beta, nt)));
    }
}

__global__ void k_envelope(int S, const double* x, const double* tau, double beta, NucTab nt, const int* ii,
                           const int* jj, const int* qq, float* env) {
    for (long s = blockIdx.x * (long)blockDim.x + threadIdx.x; s < S; s += (long)gridDim.x * blockDim.x)
        env[s] = (float)envelope(x[ii[s]], x[jj[s]], tau[qq[s]], beta, nt);
}

// G_out[q][i][j] = G_out[q][j][i] = G0[q][i][j] + scale y  for the range's samples
__global__ void k_scatter_guess(int n, long g0, long S, const float* y, double scale, const double* x,
                                const double* tau, double beta, NucTab nt, const double* G0, double* Gout) {
    const long P = (long)n * (n + 1) / 2, nn = (long)n * n;
    for (long s = blockIdx.x * (long)blockDim.x + threadIdx.x; s < S; s += (long)gridDim.x * blockDim.x) {
        const long g = g0 + s;
        const int q = (int)(g / P);
        int i, j;
        pair_of(n, g % P, &i, &j);
        const double d = scale * envelope(x[i], x[j], tau[q], beta, nt) * (double)y[s];
        const long a = (long)q * nn + (long)i * n + j, b = (long)q * nn + (long)j * n + i;
        // symmetric average of the two G0 entries keeps the guess exactly symmetric
        const double base = 0.5 * (G0[a] + G0[b]);
        Gout[a] = base + d;
        Gout[b] = base + d;
    }
}

NucTab make_nuc(int n_c, const double* X, const double* Z) {
    NucTab t{};
    t.n = n_c < N_CENT ? n_c : N_CENT;
    for (int c = 0; c < N_CENT; ++c) {
        t.Z[c] = c < n_c ? (float)Z[c] : 0.f;
        t.X[c] = c < n_c ? (float)X[c] : 0.f;
    }
    return t;
}

// ---------------------------------------------------------------- bf16 inference
// Inference-only path on the bf16 matrix cores (float32 accumulation): weights
// transposed to [N][K] bf16 once per call, activations kept in bf16 between
// layers, bias and tanh fused. Layer 1's K = 26 is zero-padded to 32.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int K1P = 32;

// WtT[n][k] = bf16(W[k][n]) for k < K (zero for K <= k < KP)
__global__ void k_weights_bf16(int K, int KP, int N, const float* __restrict__ W, __bf16* __restrict__ WtT) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)N * KP; e += (long)gridDim.x * blockDim.x) {
        const int n = (int)(e / KP), k = (int)(e % KP);
        WtT[e] = (__bf16)(k < K ? W[(long)k * N + n] : 0.f);
    }
}

// Features of a grid range (as k_features_grid) in bf16, rows padded to K1P.
__global__ void k_features_grid_bf16(int n, long g0, long S, const double* __restrict__ x,
                                     const double* __restrict__ v, const double* __restrict__ tau, double beta,
                                     NucTab nt, __bf16* __restrict__ F) {
    const long P = (long)n * (n + 1) / 2;
    for (long s = blockIdx.x * (long)blockDim.x + threadIdx.x; s < S; s += (long)gridDim.x * blockDim.x) {
        const long g = g0 + s;
        const int q = (int)(g / P);
        int i, j;
        pair_of(n, g % P, &i, &j);
        float f[D_IN];
        feature_row(f, (float)x[i], (float)x[j], (float)v[i], (float)v[j], (float)(2.0 * tau[q] / beta - 1.0), nt);
        __bf16* o = F + s * K1P;
        for (int k = 0; k < K1P; ++k) o[k] = (__bf16)(k < D_IN ? f[k] : 0.f);
    }
}

// C[S][HID] = tanh(A[S][K] W + b): block = 4 waves x 16 rows, each wave all HID
// columns (16 tiles of 16); A rows and WtT rows are read as 16-byte fragments.
__global__ __launch_bounds__(256) void k_dense_bf16(int S, int K, const __bf16* __restrict__ A,
                                                    const __bf16* __restrict__ WtT, const float* __restrict__ b,
                                                    __bf16* __restrict__ C) {
    constexpr int NT = HID / 16;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lc = lane & 15, lg = lane >> 4;
    const long r0 = (long)blockIdx.x * 64 + w * 16;
    fv4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = fv4{0.f, 0.f, 0.f, 0.f};
    const long ra = r0 + lc;
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 a;
        if (ra < S) a = *reinterpret_cast<const bf16x8*>(A + ra * K + k0 + lg * 8);
        else
            for (int e = 0; e < 8; ++e) a[e] = (__bf16)0.f;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const bf16x8 bb = *reinterpret_cast<const bf16x8*>(WtT + (long)(t * 16 + lc) * K + k0 + lg * 8);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long row = r0 + 4 * lg + r;
            const int col = t * 16 + lc;
            if (row < S) C[row * HID + col] = (__bf16)tanhf(acc[t][r] + b[col]);
        }
}

__global__ void k_out_bf16(int S, const __bf16* __restrict__ a3, const float* __restrict__ W4,
                           const float* __restrict__ b4, float* __restrict__ y) {
    const int lane = threadIdx.x & 63;
    for (long s = (blockIdx.x * (long)blockDim.x + threadIdx.x) >> 6; s < S; s += ((long)gridDim.x * blockDim.x) >> 6) {
        float acc = 0.f;
        for (int k = lane; k < HID; k += 64) acc += (float)a3[s * HID + k] * W4[k];
        acc = wave_sum(acc);
        if (lane == 0) y[s] = acc + b4[0];
    }
}

int forward(negf_ctx* ctx, int S, const float* F, const float* p, float** a1, float** a2, float** a3, float* y,
            hipStream_t st) {
    NEGF_TRY(scratch_t(ctx, "mlp_a1", (size_t)S * HID, a1));
    NEGF_TRY(scratch_t(ctx, "mlp_a2", (size_t)S * HID, a2));
    NEGF_TRY(scratch_t(ctx, "mlp_a3", (size_t)S * HID, a3));
    dim3 g(HID / 64, (S + 63) / 64);
    hipLaunchKernelGGL((k_dense<true>), g, dim3(256), 0, st, S, D_IN, HID, F, p + OFF_W1, p + OFF_B1, *a1);
    LAUNCH_CHECK();
    hipLaunchKernelGGL((k_dense<true>), g, dim3(256), 0, st, S, HID, HID, *a1, p + OFF_W2, p + OFF_B2, *a2);
    LAUNCH_CHECK();
    hipLaunchKernelGGL((k_dense<true>), g, dim3(256), 0, st, S, HID, HID, *a2, p + OFF_W3, p + OFF_B3, *a3);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_out, dim3(grid_for((long)S * 64)), dim3(256), 0, st, S, *a3, p + OFF_W4, p + OFF_B4, y);
    LAUNCH_CHECK();
    return NEGF_OK;
}

}  // namespace
}  // namespace negf

using namespace negf;

extern "C" int negf_mlp_param_count(int* count) {
    NEGF_REQUIRE(count, "count is NULL");
    *count = (int)N_PARAMS;
    return NEGF_OK;
}

extern "C" int negf_mlp_features(negf_ctx* ctx, int n_b, const double* x, const double* v, int n_c,
                                 const double* Xc, const double* Zc, int n_tau, const double* tau, double beta,
                                 int n_samples, const int* ii, const int* jj, const int* qq, float* F, void* stream) {
    NEGF_REQUIRE(ctx && x && v && tau && ii && jj && qq && F, "NULL argument");
    NEGF_REQUIRE(n_b >= 1 && n_tau >= 2 && n_samples >= 1 && beta > 0, "bad sizes");
    NEGF_REQUIRE(n_c >= 0 && n_c <= N_CENT && (n_c == 0 || (Xc && Zc)), "n_c must be 0..3");
    NEGF_TRY(bind_device(ctx));
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_features, dim3(grid_for(n_samples)), dim3(256), 0, st, n_samples, x, v, tau, beta, ii, jj, qq,
                       make_nuc(n_c, Xc, Zc), F);
    LAUNCH_CHECK();
    return NEGF_OK;
}

extern "C" int negf_mlp_targets(negf_ctx* ctx, int n_b, const double* G, const double* G0, double out_scale,
                                const double* x, int n_c, const double* Xc, int n_tau, const double* tau, double beta,
                                int n_samples, const int* ii, const int* jj, const int* qq, float* t, void* stream) {
    NEGF_REQUIRE(ctx && G && G0 && x && tau && ii && jj && qq && t, "NULL argument");
    NEGF_REQUIRE(n_b >= 1 && n_samples >= 1 && out_scale > 0 && n_tau >= 2 && beta > 0, "bad sizes");
    NEGF_REQUIRE(n_c >= 0 && n_c <= N_CENT && (n_c == 0 || Xc), "n_c must be 0..3");
    NEGF_TRY(bind_device(ctx));
    std::vector<double> zz(N_CENT, 0.0);
    hipLaunchKernelGGL(k_targets, dim3(grid_for(n_samples)), dim3(256), 0, (hipStream_t)stream, n_samples, n_b, G, G0,
                       out_scale, x, tau, beta, make_nuc(n_c, Xc, zz.data()), ii, jj, qq, t);
    LAUNCH_CHECK();
    return NEGF_OK;
}

extern "C" int negf_mlp_envelope(negf_ctx* ctx, const double* x, int n_c, const double* Xc, const double* tau,
                                 double beta, int n_samples, const int* ii, const int* jj, const int* qq, float* env,
                                 void* stream) {
    NEGF_REQUIRE(ctx && x && tau && ii && jj && qq && env, "NULL argument");
    NEGF_REQUIRE(n_samples >= 1 && beta > 0, "bad sizes");
    NEGF_REQUIRE(n_c >= 0 && n_c <= N_CENT && (n_c == 0 || Xc), "n_c must be 0..3");
    NEGF_TRY(bind_device(ctx));
    std::vector<double> zz(N_CENT, 0.0);
    hipLaunchKernelGGL(k_envelope, dim3(grid_for(n_samples)), dim3(256), 0, (hipStream_t)stream, n_samples, x, tau,
                       beta, make_nuc(n_c, Xc, zz.data()), ii, jj, qq, env);
    LAUNCH_CHECK();
    return NEGF_OK;
}

extern "C" int negf_mlp_forward(negf_ctx* ctx, const float* params, int n_samples, const float* F, float* y,
                                void* stream) {
    NEGF_REQUIRE(ctx && params && F && y, "NULL argument");
    NEGF_REQUIRE(n_samples >= 1 && n_samples <= (1 << 26), "n_samples out of range");
    NEGF_TRY(bind_device(ctx));
    float *a1, *a2, *a3;
    return forward(ctx, n_samples, F, params, &a1, &a2, &a3, y, (hipStream_t)stream);
}

extern "C" int negf_mlp_train_step(negf_ctx* ctx, float* params, float* m, float* v, int step, double lr,
                                   int n_samples, const float* F, const float* target, float* grad_out,
                                   double* loss, void* stream) {
    NEGF_REQUIRE(ctx && params && m && v && F && target, "NULL argument");
    NEGF_REQUIRE(n_samples >= 1 && n_samples <= (1 << 24), "n_samples out of range");
    NEGF_REQUIRE(step >= 1 && lr >= 0, "step must be >= 1, lr >= 0");
    NEGF_TRY(bind_device(ctx));
    hipStream_t st = (hipStream_t)stream;
    const int S = n_samples;
    float *a1, *a2, *a3, *y, *dy, *d3, *d2, *g;
    double* part;
    NEGF_TRY(scratch_t(ctx, "mlp_y", S, &y));
    NEGF_TRY(scratch_t(ctx, "mlp_dy", S, &dy));
    NEGF_TRY(scratch_t(ctx, "mlp_d3", (size_t)S * HID, &d3));
    NEGF_TRY(scratch_t(ctx, "mlp_d2", (size_t)S * HID, &d2));
    NEGF_TRY(scratch_t(ctx, "mlp_g", N_PARAMS, &g));
    const int nblk = 256;
    NEGF_TRY(scratch_t(ctx, "mlp_part", nblk, &part));
    NEGF_TRY(forward(ctx, S, F, params, &a1, &a2, &a3, y, st));
    hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, st, S, y, target, dy, part);
    LAUNCH_CHECK();
    // weight gradients A^T D over the samples, split into NS sample ranges
    // (batched products into partial buffers, then a fixed-order sum)
    constexpr int NS = 16;
    float* wpart;
    NEGF_TRY(scratch_t(ctx, "mlp_wpart", (size_t)(NS + 1) * HID * HID, &wpart));
    auto wgrad = [&](const float* A, int K, const float* Dm, float* out) -> int {
        const int c = S / NS, r = S - NS * c;
        int np = 0;
        if (c > 0) {
            NEGF_TRY(gemm<float>(st, true, false, K, HID, c, 1.f, A, K, (long)c * K, Dm, HID, (long)c * HID, 0.f,
                                 nullptr, 0, 0, wpart, HID, (long)K * HID, NS));
            np = NS;
        }
        if (r > 0) {
            NEGF_TRY(gemm<float>(st, true, false, K, HID, r, 1.f, A + (long)NS * c * K, K, 0,
                                 Dm + (long)NS * c * HID, HID, 0, 0.f, nullptr, 0, 0, wpart + (long)np * K * HID,
                                 HID, 0, 1));
            ++np;
        }
        hipLaunchKernelGGL(k_sum_partials, dim3(grid_for((long)K * HID)), dim3(256), 0, st, (long)K * HID, np, wpart,
                           out);
        LAUNCH_CHECK();
        return NEGF_OK;
    };
    const unsigned cb = (HID + 63) / 64;
    // output layer: gW4 = a3^T dy, gb4 = sum dy
    hipLaunchKernelGGL(k_colsum, dim3(cb), dim3(1024), 0, st, S, HID, a3, dy, g + OFF_W4);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(1024), 0, st, S, 1, dy, nullptr, g + OFF_B4);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_back_out, dim3(grid_for((long)S * HID)), dim3(256), 0, st, S, dy, params + OFF_W4, a3, d3);
    LAUNCH_CHECK();
    // layer 3: gW3 = a2^T d3, gb3 = colsum d3, d2 = (d3 W3^T) o (1 - a2^2)
    NEGF_TRY(wgrad(a2, HID, d3, g + OFF_W3));
    hipLaunchKernelGGL(k_colsum, dim3(cb), dim3(1024), 0, st, S, HID, d3, nullptr, g + OFF_B3);
    LAUNCH_CHECK();
    NEGF_TRY(gemm<float>(st, false, true, S, HID, HID, 1.f, d3, HID, 0, params + OFF_W3, HID, 0, 0.f, nullptr, 0, 0, d2,
                         HID, 0, 1));
    hipLaunchKernelGGL(k_tanh_grad, dim3(grid_for((long)S * HID)), dim3(256), 0, st, (long)S * HID, a2, d2);
    LAUNCH_CHECK();
    // layer 2: gW2 = a1^T d2, gb2, d1 = (d2 W2^T) o (1 - a1^2)   (d1 reuses d3)
    NEGF_TRY(wgrad(a1, HID, d2, g + OFF_W2));
    hipLaunchKernelGGL(k_colsum, dim3(cb), dim3(1024), 0, st, S, HID, d2, nullptr, g + OFF_B2);
    LAUNCH_CHECK();
    NEGF_TRY(gemm<float>(st, false, true, S, HID, HID, 1.f, d2, HID, 0, params + OFF_W2, HID, 0, 0.f, nullptr, 0, 0, d3,
                         HID, 0, 1));
    hipLaunchKernelGGL(k_tanh_grad, dim3(grid_for((long)S * HID)), dim3(256), 0, st, (long)S * HID, a1, d3);
    LAUNCH_CHECK();
    // layer 1: gW1 = F^T d1, gb1
    NEGF_TRY(wgrad(F, D_IN, d3, g + OFF_W1));
    hipLaunchKernelGGL(k_colsum, dim3(cb), dim3(1024), 0, st, S, HID, d3, nullptr, g + OFF_B1);
    LAUNCH_CHECK();
    if (grad_out) HIP_TRY(hipMemcpyAsync(grad_out, g, sizeof(float) * N_PARAMS, hipMemcpyDeviceToDevice, st));
    if (lr > 0) {
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
        hipLaunchKernelGGL(k_adam, dim3(grid_for(N_PARAMS)), dim3(256), 0, st, N_PARAMS, params, g, m, v, (float)lr, b1,
                           b2, 1e-8f, c1, c2);
        LAUNCH_CHECK();
    }
    if (loss) {
        std::vector<double> hp(nblk);
        HIP_TRY(hipMemcpyAsync(hp.data(), part, sizeof(double) * nblk, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        double s = 0.0;
        for (int k = 0; k < nblk; ++k) s += hp[k];
        *loss = s / S;
    }
    return NEGF_OK;
}

extern "C" int negf_mlp_guess(negf_ctx* ctx, const float* params, double out_scale, int n_b, const double* x,
                              const double* v, int n_c, const double* Xc, const double* Zc, int n_tau,
                              const double* tau, double beta, const double* G0, double* G_out, int dtype,
                              void* stream) {
    NEGF_REQUIRE(ctx && params && x && v && tau && G0 && G_out, "NULL argument");
    NEGF_REQUIRE(n_b >= 1 && n_tau >= 2 && beta > 0 && out_scale > 0, "bad sizes");
    NEGF_REQUIRE(n_c >= 0 && n_c <= N_CENT && (n_c == 0 || (Xc && Zc)), "n_c must be 0..3");
    NEGF_REQUIRE(dtype == NEGF_F32 || dtype == NEGF_BF16, "dtype must be NEGF_F32 or NEGF_BF16");
    NEGF_TRY(bind_device(ctx));
    hipStream_t st = (hipStream_t)stream;
    const long P = (long)n_b * (n_b + 1) / 2;
    const long total = P * n_tau;
    const long CH = 1L << 20;
    float* y;
    NEGF_TRY(scratch_t(ctx, "mlp_yg", (size_t)CH, &y));
    const NucTab nt = make_nuc(n_c, Xc, Zc);
    if (dtype == NEGF_BF16) {
        __bf16 *W1, *W2, *W3, *Fb, *h1, *h2;
        NEGF_TRY(scratch_t(ctx, "mlpb_W1", (size_t)HID * K1P, &W1));
        NEGF_TRY(scratch_t(ctx, "mlpb_W2", (size_t)HID * HID, &W2));
        NEGF_TRY(scratch_t(ctx, "mlpb_W3", (size_t)HID * HID, &W3));
        NEGF_TRY(scratch_t(ctx, "mlpb_F", (size_t)CH * K1P, &Fb));
        NEGF_TRY(scratch_t(ctx, "mlpb_h1", (size_t)CH * HID, &h1));
        NEGF_TRY(scratch_t(ctx, "mlpb_h2", (size_t)CH * HID, &h2));
        hipLaunchKernelGGL(k_weights_bf16, dim3(grid_for((long)HID * K1P)), dim3(256), 0, st, D_IN, K1P, HID,
                           params + OFF_W1, W1);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_weights_bf16, dim3(grid_for((long)HID * HID)), dim3(256), 0, st, HID, HID, HID,
                           params + OFF_W2, W2);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_weights_bf16, dim3(grid_for((long)HID * HID)), dim3(256), 0, st, HID, HID, HID,
                           params + OFF_W3, W3);
        LAUNCH_CHECK();
        for (long g0 = 0; g0 < total; g0 += CH) {
            const long S = total - g0 < CH ? total - g0 : CH;
            const unsigned nb = (unsigned)((S + 63) / 64);
            hipLaunchKernelGGL(k_features_grid_bf16, dim3(grid_for(S)), dim3(256), 0, st, n_b, g0, S, x, v, tau,
                               beta, nt, Fb);
            LAUNCH_CHECK();
            hipLaunchKernelGGL(k_dense_bf16, dim3(nb), dim3(256), 0, st, (int)S, K1P, Fb, W1, params + OFF_B1, h1);
            LAUNCH_CHECK();
            hipLaunchKernelGGL(k_dense_bf16, dim3(nb), dim3(256), 0, st, (int)S, HID, h1, W2, params + OFF_B2, h2);
            LAUNCH_CHECK();
            hipLaunchKernelGGL(k_dense_bf16, dim3(nb), dim3(256), 0, st, (int)S, HID, h2, W3, params + OFF_B3, h1);
            LAUNCH_CHECK();
            hipLaunchKernelGGL(k_out_bf16, dim3(grid_for(S * 64)), dim3(256), 0, st, (int)S, h1, params + OFF_W4,
                               params + OFF_B4, y);
            LAUNCH_CHECK();
            hipLaunchKernelGGL(k_scatter_guess, dim3(grid_for(S)), dim3(256), 0, st, n_b, g0, S, y, out_scale, x, tau,
                               beta, nt, G0, G_out);
            LAUNCH_CHECK();
        }
        return NEGF_OK;
    }
    float* F;
    NEGF_TRY(scratch_t(ctx, "mlp_F", (size_t)CH * D_IN, &F));
    for (long g0 = 0; g0 < total; g0 += CH) {
        const long S = total - g0 < CH ? total - g0 : CH;
        hipLaunchKernelGGL(k_features_grid, dim3(grid_for(S)), dim3(256), 0, st, n_b, g0, S, x, v, tau, beta, nt, F);
        LAUNCH_CHECK();
        float *a1, *a2, *a3;
        NEGF_TRY(forward(ctx, (int)S, F, params, &a1, &a2, &a3, y, st));
        hipLaunchKernelGGL(k_scatter_guess, dim3(grid_for(S)), dim3(256), 0, st, n_b, g0, S, y, out_scale, x, tau, beta,
                           nt, G0, G_out);
        LAUNCH_CHECK();
    }
    return NEGF_OK;
}
