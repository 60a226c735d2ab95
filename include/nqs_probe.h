/*
 * nqs_probe.h -- microbenchmarks of the rates this device achieves, used to
 * put the roofline figures of the method's kernels next to measured ceilings.
 * Measurement support only: no step of the method goes through these calls.
 */
#ifndef NQS_PROBE_H
#define NQS_PROBE_H

#include <stdint.h>

#include "nqs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NQS_PROBE_FMA_F32 = 0,        /* v_fma_f32 (packed FP32 is not used by this library) */
    NQS_PROBE_LOG_F32 = 1,        /* v_log_f32 (log2) */
    NQS_PROBE_EXP_F32 = 2,        /* v_exp_f32 (exp2) */
    NQS_PROBE_MFMA_BF16_K16 = 3,  /* v_mfma_f32_16x16x16_bf16 */
    NQS_PROBE_MFMA_BF16_K32 = 4,  /* v_mfma_f32_16x16x32_bf16 */
    NQS_PROBE_MFMA_F32 = 5,       /* v_mfma_f32_16x16x4_f32 */
    NQS_PROBE_MFMA_F64 = 6,       /* v_mfma_f64_16x16x4_f64 */
    NQS_PROBE_HBM_READ = 7,       /* read `size` bytes of src */
    NQS_PROBE_HBM_COPY = 8,       /* copy `size` bytes from src to dst */
    NQS_PROBE_MUL_F32 = 9,        /* v_mul_f32 */
    NQS_PROBE_XOR_U32 = 10,       /* v_xor_b32 (each of the eight values takes the xor of its neighbour) */
    NQS_PROBE_DPP_ADD_F32 = 11,   /* v_add_f32 with a row_shr:1 DPP source */
    NQS_PROBE_MULHI_U32 = 12,     /* v_mul_hi_u32 */
    NQS_PROBE_FMA_F32_W1 = 13,    /* v_fma_f32, one block of 256 threads per CU (one wave per SIMD) */
    NQS_PROBE_FMA_F32_W2 = 14,    /* v_fma_f32, two blocks per CU (two waves per SIMD) */
    NQS_PROBE_FMA_F32_DEP = 15,   /* one dependent v_fma_f32 chain per thread, one wave per SIMD (latency) */
    NQS_PROBE_LDS_READ = 16,      /* ds_read_b128 from consecutive 16-byte words, one block of 512 threads per CU */
    NQS_PROBE_MFMA_BF16_32 = 17,  /* v_mfma_f32_32x32x16_bf16, operands in registers, one block of 512 per CU */
    NQS_PROBE_MFMA_BF16_32_LDS = 18,  /* the same, each product's B operand read from LDS (ds_read_b128) */
    NQS_PROBE_MFMA_BF16_32_LDS_JIT = 19   /* as 18 with the reads where the compiler schedules them */
} nqs_probe_kind;

/* One launch of probe `kind` on `stream` (asynchronous; the caller times it).
 * Compute probes: `size` = loop iterations per thread (1 .. 2^24), the grid is
 * 8 blocks of 256 threads per compute unit (1 or 2 for the _W1 / _W2 / _DEP
 * kinds), `dst` = device scratch of at least (CUs x 8 x 256) floats, `src`
 * unused; every vector probe keeps eight independent chains per thread except
 * _DEP (one); the LDS and 32x32 kinds run one block of 512 threads per
 * compute unit (two waves per SIMD) with one accumulator chain per wave, the
 * LDS kinds over a 32 x 512 tile of 16-bit values with rows padded by 8 (one
 * read per product for _LDS, issued two products ahead; for _LDS_JIT where
 * the compiler puts it); *work = operations of the launch per lane (an FMA or a matrix
 * product element counts 2; a multiply, log, exp, DPP add or integer
 * instruction 1; bytes read for LDS_READ).
 * Memory probes: `size` = bytes, a positive multiple of 16; `src` a device
 * buffer of that size; `dst` for the copy a second one, for the read a
 * scratch of at least (CUs x 16 x 256) floats; all 16-byte aligned; *work =
 * bytes moved (read, or read + written).  *work is a host pointer.  NQS_EINVAL on a
 * bad kind, size or pointer. */
nqs_status nqs_probe_rate(int32_t kind, int64_t size, const void *src, void *dst, double *work, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NQS_PROBE_H */
