// CDNA4 matrix-core (MFMA) wrappers used by the dense products.
//
// 16x16x4 shapes, one operand element per lane:
//   A[i][k] sits in lane i + 16 k, B[k][j] in lane j + 16 k (i, j < 16, k < 4).
// Result element D[i][j] sits in lane j + 16 (i % 4), register i / 4 for the
// float64 instruction, and in lane j + 16 (i / 4), register i % 4 for the
// float32 one; row() returns i for a (lane, register) pair.
#pragma once

#include <hip/hip_runtime.h>

namespace negf {

typedef double dv4 __attribute__((ext_vector_type(4)));
typedef float fv4 __attribute__((ext_vector_type(4)));

template <class T>
struct Mma;

template <>
struct Mma<double> {
    typedef dv4 acc_t;
    static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};

template <>
struct Mma<float> {
    typedef fv4 acc_t;
    static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Sum over the 16 lanes that share lane / 16 (lane bits 0-3).
template <class T>
__device__ __forceinline__ T sum16(T v) {
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    return v;
}

// Sum over the 4 lanes that share lane % 16 (lane bits 4-5).
template <class T>
__device__ __forceinline__ T sum4x16(T v) {
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// Full 64-lane sum.
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace negf
