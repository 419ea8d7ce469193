/*
 * bsm_peaks.h - measured rooflines of the GPU the library runs on.
 *
 * The roofline fractions of the BSM kernels are quoted against the
 * published MI355X figures (32-bit vector lane operations: 256 CUs x 2.4 GHz
 * x 64 per CU and clock, the unpacked rate behind the 78.6 TFLOP/s fp64
 * vector figure; dense int8 matrix ops 5.0 POP/s; dense fp4 matrix ops
 * 10.1 POP/s; HBM3E 8 TB/s).  This call
 * measures what the same units reach on the device at hand, with kernels
 * that do nothing but that work, so that a fraction can also be read
 * against an attainable ceiling.  It is a measurement utility beside the
 * matching calls of bsm.h and shares their status codes and
 * bsm_last_error().
 */
#ifndef BSM_PEAKS_H
#define BSM_PEAKS_H

#include <stddef.h>

#include "bsm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bsm_peaks {
    /* 32-bit integer vector-ALU lane operations per second (one per lane
       per instruction) of the kinds the describe and cost kernels issue
       most: v_perm_b32, v_bcnt_u32_b32, v_alignbit_b32, v_pk_sub_u16,
       v_msad_u8, v_max_u32, v_and_or_b32, v_bitop3_b32, in equal shares. */
    double valu_int32_ops;
    /* The same for plain v_add_u32 / v_xor_b32, which issue faster. */
    double valu_addxor_ops;
    /* Dense int8 matrix operations per second: v_mfma_i32_32x32x32_i8,
       two operations per multiply-add (32 x 32 x 32 x 2 per instruction). */
    double mfma_i8_ops;
    /* Dense fp4 (e2m1) matrix operations per second at unit scale:
       v_mfma_scale_f32_32x32x64_f8f6f4, 32 x 32 x 64 x 2 per instruction,
       the product the matrix-core cost kernels issue. */
    double mfma_fp4_ops;
    /* HBM bytes per second of a streaming read (16-byte loads) of a buffer
       of hbm_bytes, far larger than the L2 and last-level caches. */
    double hbm_read_bps;
    /* HBM bytes per second of a streaming copy of hbm_bytes / 2 bytes,
       counting the bytes read plus the bytes written. */
    double hbm_copy_bps;
    /* Compute units of the device (hipDeviceProp_t::multiProcessorCount). */
    int compute_units;
} bsm_peaks;

/* Runs each probe `reps` times (>= 1) on device `device` and reports the
   best rate of each.  hbm_bytes (a multiple of 64 KiB, at least 256 MiB)
   is the size of the buffer the HBM probes stream; the call allocates that
   much device memory for its duration and frees it before returning.  The
   call synchronizes the device.  Host pointer `out` is written on success.
   Errors: BSM_EINVAL (bad argument), BSM_ENOMEM (allocation failed),
   BSM_EDEVICE (HIP error). */
bsm_status bsm_measure_peaks(int device, size_t hbm_bytes, int reps, bsm_peaks *out);

#ifdef __cplusplus
}
#endif

#endif /* BSM_PEAKS_H */
