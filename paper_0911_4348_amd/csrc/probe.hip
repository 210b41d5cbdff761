// Measurement helper, not part of the method: sustained matrix-core rate of the
// MFMA shapes the Sigma-2B kernels issue, measured on the device at hand, a
// ceiling for the roofline comparison beside the datasheet figure. Every wave
// runs 8 independent accumulator chains of one MFMA shape with register
// operands (no memory traffic in the loop), 8 waves per SIMD on every compute
// unit. Each wave also reads the core-clock counter
// (s_memtime) and the fixed-rate counter (s_memrealtime) around its loop, which
// gives the shader clock the loop ran at.
#include <algorithm>
#include <vector>

#include "common.h"

namespace negf {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kChains = 8;
constexpr int kWavesPerBlock = 4;
constexpr int kBlocksPerCU = 8;

template <int MODE>
struct Shape;
// float64: the four-block 4x4x4 shape the float64 Sigma-2B tiles issue
template <>
struct Shape<NEGF_F64> {
    typedef double acc_t;
    static constexpr double flops = 2.0 * 4 * 4 * 4 * 4;
    static __device__ __forceinline__ acc_t zero() { return 0.0; }
    static __device__ __forceinline__ double first(acc_t c) { return c; }
    static __device__ __forceinline__ acc_t step(acc_t c, int t) {
        const double a = t * 1e-3, b = 1.0 + t * 1e-4;
        return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct Shape<NEGF_F32> {
    typedef f4 acc_t;
    static constexpr double flops = 2.0 * 16 * 16 * 4;
    static __device__ __forceinline__ acc_t zero() { return acc_t{0, 0, 0, 0}; }
    static __device__ __forceinline__ double first(acc_t c) { return (double)c[0] + (double)c[3]; }
    static __device__ __forceinline__ acc_t step(acc_t c, int t) {
        const float a = t * 1e-3f, b = 1.0f + t * 1e-4f;
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct Shape<NEGF_BF16> {
    typedef f4 acc_t;
    static constexpr double flops = 2.0 * 16 * 16 * 32;
    static __device__ __forceinline__ acc_t zero() { return acc_t{0, 0, 0, 0}; }
    static __device__ __forceinline__ double first(acc_t c) { return (double)c[0] + (double)c[3]; }
    static __device__ __forceinline__ acc_t step(acc_t c, int t) {
        bf8 a, b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            a[e] = (__bf16)(t * 1e-3f);
            b[e] = (__bf16)1.0f;
        }
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

// out: one value per thread (keeps the chains live); tm: 4 counters per wave.
template <int MODE>
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_matrix_rate(int iters, double* __restrict__ out,
                                                                     unsigned long long* __restrict__ tm) {
    typedef typename Shape<MODE>::acc_t acc_t;
    const int t = threadIdx.x;
    acc_t acc[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) acc[j] = Shape<MODE>::zero();
    const unsigned long long c0 = __builtin_amdgcn_s_memtime();
    const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int j = 0; j < kChains; ++j) acc[j] = Shape<MODE>::step(acc[j], t);
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += Shape<MODE>::first(acc[j]);
    const unsigned long long c1 = __builtin_amdgcn_s_memtime();
    const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
    out[(long)blockIdx.x * blockDim.x + t] = s;
    if ((t & 63) == 0) {
        const long wv = (long)blockIdx.x * kWavesPerBlock + (t >> 6);
        tm[wv * 4 + 0] = c0;
        tm[wv * 4 + 1] = c1;
        tm[wv * 4 + 2] = r0;
        tm[wv * 4 + 3] = r1;
    }
}

template <int MODE>
int run(negf_ctx* ctx, int iters, double* tflops, double* ghz, hipStream_t st) {
    int dev = 0, n_cu = 0, wall_khz = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev));
    if (n_cu <= 0 || wall_khz <= 0) {
        set_error("device reports %d compute units, wall clock %d kHz", n_cu, wall_khz);
        return NEGF_ENODEV;
    }
    const int blocks = n_cu * kBlocksPerCU;
    const long n_waves = (long)blocks * kWavesPerBlock;
    double* out = nullptr;
    unsigned long long* tm = nullptr;
    NEGF_TRY(scratch_t(ctx, "probe_out", (size_t)blocks * 64 * kWavesPerBlock, &out));
    NEGF_TRY(scratch_t(ctx, "probe_tm", (size_t)n_waves * 4, &tm));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best_ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {   // the first launch warms the clocks up
        HIP_TRY(hipEventRecord(e0, st));
        hipLaunchKernelGGL(k_matrix_rate<MODE>, dim3(blocks), dim3(64 * kWavesPerBlock), 0, st, iters, out, tm);
        LAUNCH_CHECK();
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (rep == 0 || ms < best_ms) best_ms = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::vector<unsigned long long> h((size_t)n_waves * 4);
    HIP_TRY(hipMemcpy(h.data(), tm, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    std::vector<double> f;
    f.reserve(n_waves);
    for (long w = 0; w < n_waves; ++w) {
        const double dc = (double)(h[w * 4 + 1] - h[w * 4 + 0]);
        const double dr = (double)(h[w * 4 + 3] - h[w * 4 + 2]);
        if (dr > 0) f.push_back(dc / (dr / (wall_khz * 1e3)) * 1e-9);
    }
    std::sort(f.begin(), f.end());
    *ghz = f.empty() ? 0.0 : f[f.size() / 2];
    const double flop = (double)n_waves * iters * kChains * Shape<MODE>::flops;
    *tflops = best_ms > 0.f ? flop / (best_ms * 1e-3) * 1e-12 : 0.0;
    return NEGF_OK;
}

// Float64 issue probe: NM independent chains of the four-block 4x4x4 float64
// MFMA and NV independent chains of the float64 vector FMA per wave, one
// instruction of each chain per iteration, register operands only. Comparing
// the time of a mixed loop with those of its two parts shows whether the two
// kinds of operation run side by side on a SIMD.
template <int NM, int NV>
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_issue_mix(int iters, double* __restrict__ out) {
    const int t = threadIdx.x;
    double acc[NM > 0 ? NM : 1], x[NV > 0 ? NV : 1];
#pragma unroll
    for (int j = 0; j < NM; ++j) acc[j] = 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j) x[j] = 1.0 + j * 1e-3 + t * 1e-6;
    const double a = t * 1e-3, b = 1.0 + t * 1e-4, y = 0.999999, z = 1e-7;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < (NM > NV ? NM : NV); ++j) {
            if (j < NM) acc[j] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, acc[j], 0, 0, 0);
            if (j < NV) x[j] = __builtin_fma(x[j], y, z);
        }
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NM; ++j) s += acc[j];
#pragma unroll
    for (int j = 0; j < NV; ++j) s += x[j];
    out[(long)blockIdx.x * blockDim.x + t] = s;
}

template <int NM, int NV>
int issue_run(negf_ctx* ctx, int iters, double* ms, double* tf_mfma, double* tf_fma, hipStream_t st) {
    int dev = 0, n_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    if (n_cu <= 0) {
        set_error("device reports %d compute units", n_cu);
        return NEGF_ENODEV;
    }
    const int blocks = n_cu * kBlocksPerCU;
    double* out = nullptr;
    NEGF_TRY(scratch_t(ctx, "probe_out", (size_t)blocks * 64 * kWavesPerBlock, &out));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best_ms = 0.f;
    for (int rep = 0; rep < 3; ++rep) {
        HIP_TRY(hipEventRecord(e0, st));
        hipLaunchKernelGGL((k_issue_mix<NM, NV>), dim3(blocks), dim3(64 * kWavesPerBlock), 0, st, iters, out);
        LAUNCH_CHECK();
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        if (rep == 0 || t < best_ms) best_ms = t;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const double waves = (double)blocks * kWavesPerBlock, sec = best_ms * 1e-3;
    *ms = best_ms;
    *tf_mfma = sec > 0 ? waves * iters * NM * Shape<NEGF_F64>::flops / sec * 1e-12 : 0.0;
    *tf_fma = sec > 0 ? waves * iters * NV * 2.0 * 64 / sec * 1e-12 : 0.0;
    return NEGF_OK;
}

}  // namespace

int issue_probe_f64(negf_ctx* ctx, int n_mfma, int n_fma, double* ms, double* tf_mfma, double* tf_fma,
                    hipStream_t st) {
    constexpr int it = 20000;
#define NEGF_ISSUE(NM, NV) \
    if (n_mfma == NM && n_fma == NV) return issue_run<NM, NV>(ctx, it, ms, tf_mfma, tf_fma, st)
    NEGF_ISSUE(8, 0);
    NEGF_ISSUE(0, 8);
    NEGF_ISSUE(0, 32);
    NEGF_ISSUE(8, 2);
    NEGF_ISSUE(8, 4);
    NEGF_ISSUE(8, 8);
    NEGF_ISSUE(8, 16);
    NEGF_ISSUE(8, 32);
#undef NEGF_ISSUE
    set_error("issue probe: (%d MFMA, %d FMA chains) is not one of the built combinations", n_mfma, n_fma);
    return NEGF_EINVAL;
}

int matrix_rate(negf_ctx* ctx, int dtype, double* tflops, double* ghz, hipStream_t st) {
    switch (dtype) {
        case NEGF_F64: return run<NEGF_F64>(ctx, 16000, tflops, ghz, st);
        case NEGF_F32: return run<NEGF_F32>(ctx, 8000, tflops, ghz, st);
        default: return run<NEGF_BF16>(ctx, 4000, tflops, ghz, st);
    }
}

}  // namespace negf
