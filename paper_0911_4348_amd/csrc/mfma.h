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

// A operand of one 16 x 16 x 4 product, and the product itself, in the form
// each dtype runs fastest on gfx950. float32: the 16x16x4 shape, one value per
// lane, A[lane % 16][lane / 16]. float64: four four-block 4x4x4 products (rows
// 4r .. 4r+3 of the tile), which sustain about 1.5x the rate of the 16x16x4
// shape; with the same A rows in all four blocks, block b holds columns
// 4b .. 4b+3, so B and the result keep the 16x16x4 lanes and registers, and A
// needs A[4r + lane % 4][lane / 16] for r < 4. load(row) returns A[row][lane / 16].
template <class T>
struct AFrag;

template <>
struct AFrag<double> {
    double v[4];
    template <class F>
    __device__ __forceinline__ void load(int lane, F row) {
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = row(4 * r + (lane & 3));
    }
    __device__ __forceinline__ dv4 mma(double b, dv4 c) const {
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] = __builtin_amdgcn_mfma_f64_4x4x4f64(v[r], b, c[r], 0, 0, 0);
        return c;
    }
    __device__ __forceinline__ AFrag neg() const {
        AFrag o;
#pragma unroll
        for (int r = 0; r < 4; ++r) o.v[r] = -v[r];
        return o;
    }
};

template <>
struct AFrag<float> {
    float v;
    template <class F>
    __device__ __forceinline__ void load(int lane, F row) { v = row(lane & 15); }
    __device__ __forceinline__ fv4 mma(float b, fv4 c) const { return Mma<float>::mma(v, b, c); }
    __device__ __forceinline__ AFrag neg() const { return AFrag{-v}; }
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
