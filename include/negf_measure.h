/* Measurement helper of the FE-DVR second-Born library (libnegf.so): not part of
 * the method. It measures the sustained rate of the matrix-core operation the
 * Sigma-2B kernels issue, so that a benchmark can quote a measured ceiling
 * beside the datasheet peak. Types and error codes are those of negf.h. */
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

#ifdef __cplusplus
}
#endif

#endif
