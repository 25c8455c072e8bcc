/*
 * fdbb_probe.h -- streaming probes that measure what HBM delivers on the
 * device at hand (read-only, write-only, copy), and give the plain copy
 * kernel against which hardware byte counters are calibrated.  They are not
 * building blocks of the method; they bound them: every building block is a
 * pure streaming pass, so these rates are its practical ceiling.
 *
 * Accesses are 16 bytes per lane; stores are streaming stores with the nt
 * and sc1 cache-policy bits, as in the fused kernel.
 *
 * Pointers are device pointers, 16-byte aligned; `bytes` is a multiple of
 * 16.  Calls enqueue one kernel on `stream` (hipStream_t as void*, NULL for
 * the default stream) and return at once.  Return values are fdbb_status
 * codes (fdbb.h): FDBB_EINVAL for NULL, misaligned or negative arguments,
 * FDBB_EHIP for a launch error.
 */
#ifndef FDBB_PROBE_H
#define FDBB_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* dst[0 .. bytes) = src[0 .. bytes): reads and writes `bytes` each. */
int fdbb_probe_copy(const void *src, void *dst, int64_t bytes, int grid, void *stream);

/* Fill dst[0 .. bytes) with a 64-bit pattern; writes `bytes`. */
int fdbb_probe_write(void *dst, int64_t bytes, uint64_t pattern, int grid, void *stream);

/* Read src[0 .. bytes) and store one 64-bit xor per workgroup to sink[] (the
 * caller provides at least `grid` elements); reads `bytes`. */
int fdbb_probe_read(const void *src, int64_t bytes, uint64_t *sink, int grid, void *stream);

/* The 3D fused pass's stores without its loads or arithmetic: constant
 * values written in the fused kernel's output layout and store order
 * (flux tensor F, 15 fields of n; Riemann invariants R, 7 fields of n;
 * Jacobian blocks A, 3 x n blocks of 25 doubles; all with ld = n), with its
 * tiling (128 threads per workgroup, 4 points per thread, each wave storing
 * its 256 points' F and R chunk by chunk, then its blocks one direction at a
 * time), and its store flavour (nt + sc1).  Writes 776 bytes per point.
 * n must be a positive multiple of 512
 * (FDBB_EINVAL otherwise); the arrays are FP64 and 16-byte aligned. */
int fdbb_probe_fused_stores(double *F, double *R, double *A, int64_t n, void *stream);

/* The power x^y = exp(y log x) that the building blocks take for the
 * entropy p / rho^gamma and for rho from the entropy, evaluated on the
 * device for out[i] = x[i]^y[i], i < n, with the same device functions:
 * fp32_form = 0 selects the library's exp and log (the FP64-storage
 * kernels, relative error below 1e-14 for |y log x| < 40), nonzero the
 * base-2 form of the FP32-storage kernels (FP64 exponent split and scaling,
 * hardware FP32 log2 and exp2 of the reduced arguments; relative error
 * below 6e-7 for |y| <= 3).  Zero, negative and non-finite x give what
 * exp(y log x) gives in IEEE arithmetic.  Exposed so the accuracy of the
 * shared power can be checked apart from the building blocks.  Unlike the
 * streaming probes, accesses are 8 bytes per lane with regular stores; the
 * arrays are FP64 device arrays of n elements, 8-byte aligned (FDBB_EINVAL
 * for NULL, misaligned pointers or n < 0; n = 0 launches nothing). */
int fdbb_probe_pow(const double *x, const double *y, double *out, int64_t n, int fp32_form, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FDBB_PROBE_H */
