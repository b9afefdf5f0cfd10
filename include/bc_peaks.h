/*
 * bc_peaks.h -- microbenchmarks of the device rates the enumeration kernel
 * is measured against (the denominators of its roofline): LDS read
 * bandwidth and 32-bit integer VALU issue rate, summed over every CU.
 * Not part of the counting path; built as libbc_peaks.so.
 *
 * Each call runs on the current device and the null stream, times one
 * launch with HIP events (after one untimed warm-up launch) and returns 0,
 * or a hipError_t value on failure (outputs unwritten).  Both allocate a
 * small result sink with hipMalloc and free it before returning.
 */
#ifndef BC_PEAKS_H
#define BC_PEAKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* LDS reads: 32 blocks per CU of 256 threads, each thread reading 16 bytes
 * (ds_read_b128, conflict-free) 16 times per step for `iters` steps.
 * *bytes_per_s = bytes read / launch time; *ms = launch time. */
int bc_peak_lds(uint32_t iters, double *bytes_per_s, double *ms);

/* Integer VALU: 64 blocks per CU of 256 threads, each lane issuing 16
 * independent v_and_b32 / v_bcnt_u32_b32 per step for `iters` steps.
 * *ops_per_s = lane-instructions / launch time; *ms = launch time. */
int bc_peak_valu_int(uint32_t iters, double *ops_per_s, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* BC_PEAKS_H */
