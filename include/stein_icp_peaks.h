/*
 * stein_icp_peaks.h -- device ceilings measured on the device itself.
 *
 * Not part of the method: these calls time what the hardware sustains for
 * the three kinds of work the Stein-ICP kernels do, so that a kernel's
 * roofline fraction can be read against a measured ceiling as well as the
 * published one:
 *  - a streaming copy (HBM bandwidth; the published figure is 8 TB/s),
 *  - FP32 fused multiply-adds on the vector ALUs, unpacked (the library is
 *    built without packed FP32 instructions; the published 157.3 TFLOP/s
 *    counts packed ones),
 *  - dense 32x32x16 FP16 and BF16 matrix-core products, the instruction
 *    shape of the nearest-neighbour screens (published: 2.5 PFLOP/s).
 * The work of a call (bytes or floating-point operations) comes from
 * stein_icp_peak_work; the caller times the call on its stream.
 *
 * Conventions as in stein_icp.h: device pointers owned by the caller,
 * hip_stream a hipStream_t (NULL = default stream), the calls only enqueue,
 * negative status on failure with stein_icp_last_error() describing it.
 */
#ifndef STEIN_ICP_PEAKS_H
#define STEIN_ICP_PEAKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* in: n float4 (16-byte aligned); out: n float4; out = in. Work: 32 n
 * bytes (read and written once). */
#define STEIN_ICP_PEAK_COPY 0
/* out: n floats, one per thread (n a positive multiple of 256); thread i
 * runs sixteen independent chains a_k <- fmaf(a_k, b, c), iters times, from
 * a_k = i + k, and writes the sum of the sixteen. Work: 32 n iters flops. */
#define STEIN_ICP_PEAK_FMA32 1
/* in: 128 uint4 A and B fragments (lane l of a wavefront reads in[l] as A
 * and in[64 + l] as B, eight FP16 or BF16 values each); out: n floats, one
 * per lane (n a positive multiple of 256). Every wavefront runs iters trips
 * of four independent v_mfma_f32_32x32x16 products accumulating into four
 * 32x32 FP32 tiles from zero, and lane l writes the sum of its 64 tile
 * values. Work: 4 x 32768 iters flops per wavefront. */
#define STEIN_ICP_PEAK_MFMA_F16 2
#define STEIN_ICP_PEAK_MFMA_BF16 3

/* Enqueue one probe of `kind` (above) on `hip_stream`. n >= 1 (a multiple
 * of 256 for the arithmetic kinds), 1 <= iters <= 2^24; b and c feed FMA32
 * only. Returns STEIN_ICP_E_INVALID for a bad kind or size, before any
 * launch. */
int stein_icp_peak_probe(int kind, const void *in, void *out, int64_t n, int32_t iters, float b, float c,
                         void *hip_stream);

/* Work of one probe call with these arguments: bytes for COPY, floating-
 * point operations otherwise; negative for a bad kind. */
double stein_icp_peak_work(int kind, int64_t n, int32_t iters);

/* Properties of the current device: compute units, LDS bytes per compute
 * unit, wavefront width, peak engine clock (kHz) and the architecture name
 * (NUL-terminated, truncated to arch_len bytes). Blocking. */
int stein_icp_device_info(int32_t *compute_units, int32_t *lds_bytes_per_cu, int32_t *wave_size,
                          int32_t *clock_khz, char *arch, int32_t arch_len);

#ifdef __cplusplus
}
#endif

#endif /* STEIN_ICP_PEAKS_H */
