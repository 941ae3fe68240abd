/*
 * adg_peaks.h -- measured device peaks for the roofline of the MI355X
 * (gfx950) library's kernels: FP64 vector FMA rate, FP64 matrix-core (MFMA)
 * rate and device-to-device copy bandwidth, measured on the device at hand so
 * that they can be reported beside the published figures (FP64 vector and
 * matrix 78.6 TFLOP/s, HBM3E 8 TB/s).  Not part of the method: a measuring
 * aid.  Conventions (ownership, streams, errors) as in adg.h.
 */
#ifndef ADG_PEAKS_H
#define ADG_PEAKS_H

#include <stddef.h>

#include "adg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Size in bytes of the device buffer the compute loops write their results
 * to (so that no work is optimised away). */
int adg_peaks_sink_bytes(size_t* bytes);

/* Runs, on the given stream, a loop of independent FP64 fused multiply-adds
 * on every SIMD, a loop of independent v_mfma_f64_16x16x4 instructions
 * (2048 flops each) on every SIMD, and, if copy_bytes > 0, a stream copy of
 * copy_bytes bytes from src to dst; each once untimed, then three timed
 * launches (device events), keeping the fastest.  sink: device buffer of
 * adg_peaks_sink_bytes bytes; src, dst: device buffers of copy_bytes bytes,
 * 16-byte aligned, copy_bytes a multiple of 16 (unused when copy_bytes is
 * 0).  out (host) = (FP64 vector TFLOP/s, FP64 MFMA TFLOP/s, copy GB/s
 * counting the bytes read and written; NaN when copy_bytes is 0).
 * Synchronises the stream.  EINVAL on null or misaligned arguments. */
int adg_measure_peaks(void* sink, const void* src, void* dst, size_t copy_bytes, double* out, void* stream);

/* Whether FP64 matrix cores add to the FP64 vector rate: chains of
 * v_mfma_f64_4x4x4 (512 flops each) on every wave; chains of vector FMAs on
 * every wave; then half the waves of each workgroup on each.  out (host,
 * 5 doubles) = (MFMA TFLOP/s alone, FMA TFLOP/s alone, combined TFLOP/s of
 * the half-and-half run, its MFMA part, its FMA part): a combined rate near
 * the larger single rate means the two share the FP64 units, near their sum
 * that they add.  sink as for adg_measure_peaks.  Synchronises the stream. */
int adg_measure_fp64_sharing(void* sink, double* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* ADG_PEAKS_H */
