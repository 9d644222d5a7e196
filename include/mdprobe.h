/* mdprobe.h - measurement probe shipped beside libmdlj (libmdprobe.so).  It is
 * not part of the MD path: it measures the FP32 FMA rate that kernels built
 * like this library's (gfx950, packed FP32 instructions disabled) can reach,
 * the ceiling quoted beside the published FP32 peak in the roofline of the
 * force kernels. */
#ifndef MDPROBE_H
#define MDPROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Launch workgroups x 256 threads, each running 8 independent chains of
 * iters dependent FP32 fused multiply-adds, on the HIP stream `stream`
 * (NULL: the default stream).  out: DEVICE float[workgroups * 256], written
 * (the chains' sums, so that the work is not elided); owned by the caller.
 * Returns 0, -1 for a non-positive count or NULL out, -2 if the launch
 * failed.  Asynchronous: time it with events on the same stream. */
int mdprobe_fma_f32(int32_t workgroups, int32_t iters, float *out, void *stream);

/* Floating-point operations of one such launch (an FMA counts two). */
int64_t mdprobe_fma_f32_flops(int32_t workgroups, int32_t iters);

#ifdef __cplusplus
}
#endif

#endif
