/* Measurement helpers of the FE-DVR second-Born library (libnegf.so): not part
 * of the method. They measure the sustained rate of the matrix-core operation
 * the Sigma-2B kernels issue, so that a benchmark can quote a measured ceiling
 * beside the datasheet peak, and whether float64 vector FMAs add throughput
 * beside it. Types and error codes are those of negf.h. */
#ifndef NEGF_MEASURE_H
#define NEGF_MEASURE_H

#include "negf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Sustained rate of the matrix-core operation the Sigma-2B kernels issue for
 * `dtype` (NEGF_F64: four-block 4x4x4 float64, NEGF_F32: 16x16x4 float32, NEGF_BF16:
 * 16x16x32 bf16 with float32 accumulation), measured on the context's GPU: a
 * kernel of 8 independent accumulator chains per wave with register operands,
 * 8 waves per SIMD on every compute unit, run twice (the faster run counts).
 * host out: tflops (TFLOP/s), clock_ghz (median shader clock of the waves,
 * from the core-clock and fixed-rate counters). A measured ceiling to quote
 * beside the datasheet peak; not part of the method. Uses context scratch
 * (a few MB). Synchronises. */
int negf_matrix_rate(negf_ctx* ctx, int dtype, double* tflops, double* clock_ghz, void* stream);

/* Float64 issue probe: whether float64 vector FMAs run beside the four-block
 * 4x4x4 float64 MFMA. Every wave runs n_mfma independent MFMA accumulator
 * chains and n_fma independent vector-FMA chains, one instruction of each chain
 * per loop iteration (20000 iterations), register operands only, 8 waves per
 * SIMD on every compute unit; best of 3 launches. Built combinations (n_mfma,
 * n_fma): (8, 0), (0, 8), (0, 32), (8, 2), (8, 4), (8, 8), (8, 16), (8, 32);
 * others return NEGF_EINVAL. host out: ms (kernel time), mfma_tflops and
 * fma_tflops (the two kinds' flop rates over that time). If a mixed loop takes
 * the sum of its parts' times, the two share the SIMD's issue. Not part of the
 * method. Uses context scratch (a few MB). Synchronises. */
int negf_f64_issue_probe(negf_ctx* ctx, int n_mfma, int n_fma, double* ms, double* mfma_tflops,
                         double* fma_tflops, void* stream);

#ifdef __cplusplus
}
#endif

#endif
