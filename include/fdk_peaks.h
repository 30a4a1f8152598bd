/*
 * fdk_peaks.h -- microbenchmarks of the three ceilings the back-projector is
 * held against (the GPU counterpart of the paper's roofline analysis,
 * Sections 4.3-4.4: achieved throughput against the bandwidth of the memory
 * level the update reads from and against the arithmetic issue rate).
 *
 * Each call enqueues ONE kernel on `stream` (a hipStream_t) and returns; the
 * caller times it (HIP events on the same stream) and divides the work the
 * call reports by the elapsed time.  The kernels compute nothing of the
 * back-projection: they read or combine values only so that the compiler
 * keeps every load and every FMA, and write to `sink` (device memory, one
 * word, contents unspecified) only under a condition that the data never
 * meets.  Conventions and errors as in fdk.h.
 */
#ifndef FDK_PEAKS_H
#define FDK_PEAKS_H

#include <stdint.h>

#include "fdk.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * fdk_peak_hbm_read -- stream `bytes` of device memory at `buf` once, with
 * 16-byte loads (four in flight per thread) from `blocks` blocks of 256
 * threads striding over the buffer.  buf must be 16-byte aligned and bytes a
 * positive multiple of 16, else FDK_E_INVALID.  Work: `bytes` read from HBM
 * (buffers far larger than the last-level cache).
 */
fdk_status fdk_peak_hbm_read(const void* buf, int64_t bytes, int32_t blocks, uint32_t* sink,
                             void* stream);

/* Access patterns of fdk_peak_lds_read. */
typedef enum {
    FDK_LDS_B32 = 0,        /* ds_read_b32, 64 consecutive words per wave (no bank conflict) */
    FDK_LDS_READ2_B32 = 1,  /* ds_read2_b32, two runs of 64 consecutive words, 36 words apart */
    FDK_LDS_B64 = 2,        /* ds_read_b64, 64 consecutive 8-byte words per wave */
    FDK_LDS_B128 = 3,       /* ds_read_b128, 64 consecutive 16-byte words per wave */
    FDK_LDS_TAPS_F16 = 4,   /* the back-projector's binary16 taps: per update, the pair words
                               of rows floor(v) and floor(v) + 1 (36-word rows) at the columns
                               of a 16 x 16 voxel tile seen at 1.6 detector pixels per voxel
                               (view at 30 degrees), v advancing 1.6 rows per slice */
    FDK_LDS_TAPS_F32 = 5,   /* the same with float32 taps: per update, words (c, c + 1) of
                               rows floor(v) and floor(v) + 1 (72-word rows) */
    FDK_LDS_B64_ASM = 6,    /* ds_read_b64 at 8-byte aligned addresses, issued four at a time
                               by an assembly block that waits for them */
    FDK_LDS_B64_ASM_DWORD = 7 /* the same at addresses 4 mod 8 (dword aligned) */
} fdk_lds_pattern;

/*
 * fdk_peak_lds_read -- `blocks` blocks of 256 threads fill 32 KiB of LDS, then
 * each thread issues iters x 16 LDS read instructions of the given pattern
 * (fdk_lds_pattern).  *bytes_out (host) receives the bytes the launch reads
 * from LDS (lanes x bytes per lane per instruction), the work to divide by the
 * kernel time.  iters >= 1, blocks >= 1.
 */
fdk_status fdk_peak_lds_read(int32_t pattern, int32_t blocks, int32_t iters, uint32_t* sink,
                             int64_t* bytes_out, void* stream);

/*
 * fdk_peak_valu_fma -- `blocks` blocks of 256 threads, each thread running 8
 * independent chains of iters x 16 float32 FMAs (v_fma_f32, not packed).
 * *ops_out (host) receives the lane-operations of the launch (threads x 8 x
 * 16 x iters): the VALU issue rate the back-projector's instruction counts
 * are compared with.  iters >= 1, blocks >= 1.
 */
fdk_status fdk_peak_valu_fma(int32_t blocks, int32_t iters, float* sink, int64_t* ops_out,
                             void* stream);

/* Instructions of fdk_peak_valu_op: the VALU instructions of the
 * back-projector's hot loop. */
typedef enum {
    FDK_OP_FMA_F32 = 0,      /* v_fma_f32 (VOP3), float32 */
    FDK_OP_FMAC_F32 = 1,     /* v_fmac_f32 (VOP2), float32, accumulator in place */
    FDK_OP_SUB_F32 = 2,      /* v_sub_f32 */
    FDK_OP_FRACT_F32 = 3,    /* v_fract_f32 */
    FDK_OP_CVT_I32_F32 = 4,  /* v_cvt_i32_f32 */
    FDK_OP_MAD_U32_U24 = 5,  /* v_mad_u32_u24 (24-bit integer multiply-add) */
    FDK_OP_FMA_MIX_F32 = 6,  /* v_fma_mix_f32 with one binary16 operand (FP32 arithmetic) */
    FDK_OP_CVT_F32_F16 = 7,  /* v_cvt_f32_f16 */
    FDK_OP_DOT2_F32_F16 = 8, /* v_dot2_f32_f16 */
    FDK_OP_PK_FMA_F16 = 9,   /* v_pk_fma_f16 (two binary16 lanes) */
    FDK_OP_ADD_U32 = 10,     /* v_add_u32 */
    FDK_OP_FLOOR_F32 = 11    /* v_floor_f32 */
} fdk_valu_op;

/*
 * fdk_peak_valu_op -- the issue rate of one VALU instruction: `blocks` blocks
 * of 256 threads, each thread running 8 independent chains of iters x 16
 * instructions `op` (fdk_valu_op), written as inline assembly so that exactly
 * that instruction is issued.  *ops_out (host) receives the lane-operations
 * (threads x 8 x 16 x iters).  iters >= 1, blocks >= 1, else FDK_E_INVALID.
 */
fdk_status fdk_peak_valu_op(int32_t op, int32_t blocks, int32_t iters, float* sink,
                            int64_t* ops_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FDK_PEAKS_H */
